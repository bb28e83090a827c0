"""The constants the paper fixes (tests/golden/paper_constants.json, each
entry with its section) against the oracle's and the GPU drivers' own
definitions: agent weights (Sec. III-A), the Mann parameter and the range
zero-padding factors (Sec. V), the learning-rate decay (Sec. III-C)."""

import inspect
import json
import os

import numpy as np
import pytest

import oracle
from oracle import mace

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_constants.json")


@pytest.fixture(scope="module")
def paper():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("looks", [1, 4, 16, 32])
def test_agent_weights(paper, looks):
    """1/(2L) per forward agent, 1/2 for the prior agent: both the oracle's
    and the drivers' weights, which sum to one."""
    from paper_2406_13651_amd import agent_weights
    want = np.array([1.0 / (2 * looks)] * looks + [paper["agent_weights"]["prior_agent"]])
    np.testing.assert_allclose(mace.agent_weights(looks, True), want, rtol=0, atol=1e-15)
    np.testing.assert_allclose(agent_weights(looks, True), want, rtol=0, atol=1e-15)
    assert abs(want.sum() - 1.0) < 1e-15


def test_mann_parameter_defaults(paper):
    from paper_2406_13651_amd import ClampGPU
    rho = paper["mann_rho"]["value"]
    assert inspect.signature(oracle.clamp_iteration).parameters["rho"].default == rho
    assert inspect.signature(oracle.clamp_run).parameters["rho"].default == rho
    assert inspect.signature(ClampGPU.__init__).parameters["rho"].default == rho


def test_learning_rate_decay_defaults(paper):
    from paper_2406_13651_amd import learned
    d = paper["learning_rate_decay"]
    sig = inspect.signature(learned.train).parameters
    assert sig["decay"].default == d["factor"] and sig["decay_every"].default == d["every_batches"]


def test_default_sigma2_in_the_papers_range(paper):
    import bench
    lo, hi = paper["forward_sigma2_range"]["low"], paper["forward_sigma2_range"]["high"]
    assert lo <= bench.parser().parse_args([]).sigma2 <= hi


def test_zero_padding_factors_of_the_padded_workload(paper):
    import bench
    qs = sorted({q for _, q, allpass in bench.PADDED_CASES if not allpass})
    assert qs == paper["zero_padding_q"]["values"]


def test_paper_timing_configuration_of_the_bench(paper):
    """The paper workload of bench.py runs the configuration the paper times
    (Sec. III-D, Sec. V-A, Sec. V-B) and quotes its bound."""
    import bench
    t = paper["timing_configuration"]
    c = bench.PAPER_CONFIG
    assert [c["n"]] * 3 == t["image"] and c["looks"] == t["looks"]
    assert c["n"] / c["range_box"] == t["q"]
    assert bench.PAPER_SECONDS_PER_ITERATION == t["seconds_per_iteration_below"]
