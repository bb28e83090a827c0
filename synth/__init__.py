"""Seeded synthetic inputs for CLAMP reconstructions.

This package simulates the acquisition that CLAMP inverts (paper Sec. II-B and
Sec. V-B): a faceted reflectivity scene, fully developed speckle per look and
circular-pupil measurements with complex white noise.  It is shared by the
test oracle and by the GPU path as their common input source, and it holds
none of the reconstruction's arithmetic (no adjoint, no gradient, no MM
update, no consensus step).
"""

from .scenes import (  # noqa: F401
    CONFIGS,
    batch_specs,
    SceneSpec,
    facet_scene,
    measure_looks,
    make_problem,
    noise_variance,
    seed_sequence,
    synth_pupil,
)
