"""Pins for the oracle's mixed-noise loss and amplitude regularisers (CPU).

The paper implements MLE with mixed noise statistics and L1 / TV
regularisation of the amplitude (Section "Universal Ptychography Algorithm
based on Automatic Differentiation" and the reconstruction section); the
exact forms are readings.  Pinned here: hand-computed values, the
constant-amplitude and step-edge closed forms of the TV term, the large
read-noise limit, and central differences of the whole loss.
"""
import math

import numpy as np
import pytest

from oracle import model as om

from test_oracle_model import _fd_check, _perturbed_measurement, crandn, tiny_problem


def test_mixed_loss_hand_values():
    # I' = 3, measured 1, v = 1: (2^2)/4 + ln 4 ; d = 2*2/4 - (2/4)^2 + 1/4
    ell, d = om.pointwise_loss(np.array([3.0]), np.array([1.0]), om.LOSS_MIXED, 0.0, 1.0)
    assert abs(ell[0] - (1.0 + math.log(4.0))) < 1e-15
    assert abs(d[0] - 1.0) < 1e-15
    # at a match only the log term is left
    ell, d = om.pointwise_loss(np.array([5.0]), np.array([5.0]), om.LOSS_MIXED, 0.0, 3.0)
    assert abs(ell[0] - math.log(8.0)) < 1e-15 and abs(d[0] - 1.0 / 8.0) < 1e-15


def test_mixed_loss_large_read_noise_is_gaussian():
    # v >> I': the derivative tends to 2 (I' - measured) / v (a Gaussian of variance v)
    I, m, v = np.array([10.0, 3.0]), np.array([7.0, 4.0]), 1e8
    _, d = om.pointwise_loss(I, m, om.LOSS_MIXED, 0.0, v)
    assert np.allclose(d * v, 2.0 * (I - m) + 1.0, rtol=0, atol=1e-5)


def test_mixed_loss_derivative_by_differences():
    rng = np.random.default_rng(2)
    I = rng.uniform(0.1, 20, 50)
    m = rng.poisson(I).astype(float)
    h = 1e-6
    lp, _ = om.pointwise_loss(I + h, m, om.LOSS_MIXED, 0.0, 2.5)
    lm, _ = om.pointwise_loss(I - h, m, om.LOSS_MIXED, 0.0, 2.5)
    _, d = om.pointwise_loss(I, m, om.LOSS_MIXED, 0.0, 2.5)
    assert np.allclose((lp - lm) / (2 * h), d, rtol=1e-7, atol=1e-9)


def test_regulariser_constant_amplitude():
    rng = np.random.default_rng(3)
    O = 0.8 * np.exp(1j * rng.uniform(-3, 3, (2, 5, 7)))
    v, g = om.regulariser(O, 0.3, 0.5, 1e-2)
    assert abs(v - (0.3 * 0.8 * 70 + 0.5 * 1e-2 * 70)) < 1e-12
    # the TV term is flat; the L1 term pulls along the phase of O
    assert np.allclose(g, 0.3 * O / 0.8, atol=1e-12)


def test_regulariser_step_edge():
    H, W, x0, d = 6, 9, 4, 1e-3
    O = np.where(np.arange(W)[None, :] < x0, 1.0, 2.0) * np.ones((H, W)) * np.exp(0.3j)
    v, g = om.regulariser(O, 0.0, 1.0, d)
    assert abs(v - (H * math.sqrt(1.0 + d * d) + (H * W - H) * d)) < 1e-12
    # dTV/da at the two pixels of the edge: -1/t on the left, +1/t on the right
    t = math.sqrt(1.0 + d * d)
    ga = np.real(g * np.exp(-0.3j))
    assert np.allclose(ga[:, x0 - 1], -1.0 / t) and np.allclose(ga[:, x0], 1.0 / t)
    assert np.allclose(np.delete(ga, [x0 - 1, x0], axis=1), 0.0, atol=1e-12)


def test_regulariser_gradient_by_differences():
    rng = np.random.default_rng(4)
    O = crandn(rng, 2, 6, 8)
    v0, g = om.regulariser(O, 0.2, 0.7, 0.05)
    for _ in range(3):
        dv = crandn(rng, *O.shape)
        h = 1e-6
        fd = (om.regulariser(O + h * dv, 0.2, 0.7, 0.05)[0] -
              om.regulariser(O - h * dv, 0.2, 0.7, 0.05)[0]) / (2 * h)
        assert abs(fd - np.real(np.vdot(g, dv))) <= 1e-7 * max(abs(fd), 1.0)


@pytest.mark.parametrize("kind", [om.LOSS_MIXED, om.LOSS_AMPLITUDE])
def test_whole_loss_with_regulariser_by_differences(kind):
    pr = tiny_problem(seed=31, L=2, M=2, Ns=2, with_sigma=True, with_bg=True)
    meas = _perturbed_measurement(pr)
    kw = dict(kind=kind, eps=1e-3, scale=0.4, sigma=pr["sigma"], background=pr["bg"],
              noise_var=2.0, l1=0.05, tv=0.2, tv_eps=0.01)
    base = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, **kw)
    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(2):
        v = crandn(rng, *pr["obj"].shape)
        fd, an = _fd_check(lambda o: om.loss_grad(o, pr["prb"], pr["pos"], pr["pads"], meas,
                                                  **kw)["loss"], base["g_object"], pr["obj"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)
        v = crandn(rng, *pr["prb"].shape)
        fd, an = _fd_check(lambda p: om.loss_grad(pr["obj"], p, pr["pos"], pr["pads"], meas,
                                                  **kw)["loss"], base["g_probe"], pr["prb"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)
    # the regulariser is part of the loss once, not per position
    a = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, positions=[0, 1], **kw)
    b = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas,
                     positions=list(range(2, pr["pos"].shape[0])), **kw)
    rv, _ = om.regulariser(pr["obj"], 0.05, 0.2, 0.01)
    assert abs(a["loss"] + b["loss"] + rv - base["loss"]) <= 1e-12 * abs(base["loss"])
