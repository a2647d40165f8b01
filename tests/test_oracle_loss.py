"""Closed-form values of the per-pixel losses and their derivatives."""
import numpy as np
import pytest

from oracle import model as om


def test_amplitude_loss_closed_form():
    ell, d = om.pointwise_loss(np.array([4.0]), np.array([1.0]), om.LOSS_AMPLITUDE, 0.0)
    assert ell[0] == pytest.approx(1.0)          # (2 - 1)^2
    assert d[0] == pytest.approx(0.5)            # 1 - 1/2


def test_poisson_loss_closed_form():
    ell, d = om.pointwise_loss(np.array([np.e]), np.array([2.0]), om.LOSS_POISSON, 0.0)
    assert ell[0] == pytest.approx(np.e - 2.0)   # I - Î ln I with ln e = 1
    assert d[0] == pytest.approx(1.0 - 2.0 / np.e)


def test_gaussian_loss_closed_form():
    ell, d = om.pointwise_loss(np.array([3.0]), np.array([1.0]), om.LOSS_GAUSSIAN, 0.0)
    assert ell[0] == pytest.approx(4.0)
    assert d[0] == pytest.approx(4.0)


@pytest.mark.parametrize("kind", [om.LOSS_AMPLITUDE, om.LOSS_POISSON, om.LOSS_GAUSSIAN, om.LOSS_VJP])
def test_loss_derivative_matches_difference(kind):
    I = np.array([0.01, 0.7, 3.0, 250.0])
    meas = np.array([0.0, 1.0, 2.0, 260.0])
    h = 1e-6 * np.maximum(I, 1e-2)
    lp, _ = om.pointwise_loss(I + h, meas, kind, 1e-3)
    lm, _ = om.pointwise_loss(I - h, meas, kind, 1e-3)
    _, d = om.pointwise_loss(I, meas, kind, 1e-3)
    assert np.allclose((lp - lm) / (2 * h), d, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("kind", [om.LOSS_AMPLITUDE, om.LOSS_POISSON])
def test_loss_derivative_vanishes_at_match(kind):
    x = np.array([0.0, 1.0, 17.0])
    _, d = om.pointwise_loss(x, x, kind, 1e-6)
    assert np.all(d == 0.0)
