"""Host logic of the learned form's fallback, on the CPU with a stand-in
reconstruction object (no GPU)."""

import math

import numpy as np

import torch

from paper_2406_13651_amd import learned as Lm


class Fake:
    """Stand-in with the interface run_with_fallback uses: a scripted
    consensus error per iteration and a wbar that records the iteration."""

    def __init__(self, errs, tag):
        self.errs = errs
        self.tag = tag
        self.k = 0
        self.fault = torch.zeros(1, dtype=torch.int32)
        self.wbar = torch.zeros(4)

    def init(self, y):
        self.k = 0

    def iterate(self):
        self.k += 1
        self.wbar = torch.full((4,), float(self.tag * 1000 + self.k))

    def run(self, iters):
        for _ in range(iters):
            self.iterate()

    def conv_err(self):
        return self.errs[min(self.k, len(self.errs)) - 1]


def test_rising_consensus_error_falls_back():
    errs = [1.0 / (k + 1) for k in range(10)] + [0.1 * (1.5 ** k) for k in range(40)]
    out, info = Lm.run_with_fallback(lambda: Fake(errs, 1), lambda: Fake(errs, 2), None, 50, check_every=5,
                                     patience=3)
    assert info["fallback"] and info["reason"] == "consensus error rising"
    assert float(out[0]) == 2050.0  # the forward-only stand-in ran all 50 iterations


def test_decreasing_error_keeps_learned_result():
    errs = [1.0 / (k + 1) for k in range(50)]
    out, info = Lm.run_with_fallback(lambda: Fake(errs, 1), lambda: Fake(errs, 2), None, 50)
    assert not info["fallback"]
    assert float(out[0]) == 1050.0


def test_non_finite_error_falls_back():
    errs = [0.5, 0.4, 0.3, 0.2, math.nan] * 10
    out, info = Lm.run_with_fallback(lambda: Fake(errs, 1), lambda: Fake(errs, 2), None, 20)
    assert info["fallback"] and info["reason"] == "fault"


def test_nrmse_is_scale_free():
    r = torch.rand(3, 4, 5) + 0.1
    assert Lm.nrmse(7.0 * r, r) < 1e-6  # float32 rounding of 7 r
    noisy = r + 0.01 * torch.randn(3, 4, 5)
    assert abs(Lm.nrmse(3.0 * noisy, r) - Lm.nrmse(noisy, r)) < 1e-6


def test_unet_initial_parameters_follow_the_library_layout():
    """unet_init_params lays out the flat vector in the order of the C
    interface (the oracle's flatten order): gamma 1, beta 0, zero biases and
    a zero output layer where that order puts them."""
    from oracle import unet as U
    from paper_2406_13651_amd import _clamp as C
    from paper_2406_13651_amd.learned import unet_init_params
    p = unet_init_params(0)
    assert p.size == C.UNET_PARAMS == U.param_count()
    q = U.unflatten(p.astype(np.float64))
    for i in range(U.CONVS):
        assert np.all(q["gamma"][i] == 1.0) and np.all(q["beta"][i] == 0.0)
        assert np.std(q["conv"][i]) > 0.0
    for j in range(U.LEVELS):
        assert np.all(q["up_b"][j] == 0.0) and np.std(q["up_w"][j]) > 0.0
    assert np.all(q["final_w"] == 0.0) and np.all(q["final_b"] == 0.0)
