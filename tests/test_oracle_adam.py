"""Pins of the oracle's Adam step (the paper's optimiser, Section "Universal
Ptychography Algorithm based on Automatic Differentiation").

* A three-step table with non-zero starting moments, derived by hand in
  exact rational arithmetic (tests/golden/adam_three_steps.txt): it fixes
  the moment recursions (beta * previous moment), the bias corrections at
  t = 1, 2, 3, the square root and the sign of the step.
* Constant gradient from zero moments: the bias-corrected moments equal g and
  g^2 exactly at every t (geometric series), so every step is
  lr g / (|g| + eps) -- a closed form that a dropped bias correction or a
  dropped beta * m term breaks from t = 2 on.
* With eps = 0 the step is invariant under g -> c g, m -> c m, v -> c^2 v
  (c > 0), which fails without the square root.
* Complex variables are updated as independent real and imaginary parts.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adam_three_steps.txt")


def _table():
    rows = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].strip()
        if line:
            rows.append([float(Fraction(x)) for x in line.split()])
    return np.array(rows)


def test_three_steps_from_a_resumed_state_match_the_hand_derived_table():
    tab = _table()
    assert tab.shape == (3, 9)
    x = np.array([1.0, 1.0])
    m = np.array([1.0, -1.0])
    v = np.array([4.0, 4.0])
    for row in tab:
        t = int(row[0])
        g = np.array([row[1], row[5]])
        x, m, v = oracle.adam_step(x, g, m, v, t, lr=1.0, beta1=0.5, beta2=0.75, eps=0.0)
        np.testing.assert_allclose(m, [row[2], row[6]], rtol=1e-15, atol=0)
        np.testing.assert_allclose(v, [row[3], row[7]], rtol=1e-15, atol=0)
        np.testing.assert_allclose(x, [row[4], row[8]], rtol=1e-14, atol=0)


@pytest.mark.parametrize("beta1,beta2", [(0.9, 0.999), (0.5, 0.75), (0.0, 0.9)])
def test_constant_gradient_steps_are_lr_sign_g(beta1, beta2):
    rng = np.random.default_rng(3)
    g = rng.normal(size=50) * 10.0 ** rng.uniform(-3, 3, 50)
    x = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 0.01, 1e-8
    for t in range(1, 8):
        x1, m, v = oracle.adam_step(x, g, m, v, t, lr, beta1, beta2, eps)
        np.testing.assert_allclose(x - x1, lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
        x = x1


def test_step_is_invariant_to_the_gradient_scale_without_eps():
    rng = np.random.default_rng(5)
    x = rng.normal(size=40)
    g = rng.normal(size=40)
    m = rng.normal(size=40)
    v = rng.uniform(0.1, 2.0, 40)
    a = oracle.adam_step(x, g, m, v, 4, 0.1, eps=0.0)[0]
    for c in (1e-3, 7.0, 1e4):
        b = oracle.adam_step(x, c * g, c * m, c * c * v, 4, 0.1, eps=0.0)[0]
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-15)


def test_complex_variable_is_its_real_and_imaginary_parts():
    rng = np.random.default_rng(7)
    z = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    gz = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    m = rng.normal(size=24)
    v = rng.uniform(0.1, 1.0, 24)
    zn, mn, vn = oracle.adam_step(z, gz, m, v, 2, 0.05)
    xr = np.stack([z.real, z.imag], -1).ravel()
    gr = np.stack([gz.real, gz.imag], -1).ravel()
    xn, mr, vr = oracle.adam_step(xr, gr, m, v, 2, 0.05)
    assert zn.shape == z.shape and np.iscomplexobj(zn)
    np.testing.assert_array_equal(np.stack([zn.real, zn.imag], -1).ravel(), xn)
    np.testing.assert_array_equal(mn, mr)
    np.testing.assert_array_equal(vn, vr)


def test_adam_rejects_mismatched_state_and_step_zero():
    with pytest.raises(ValueError):
        oracle.adam_step(np.zeros(3), np.zeros(3), np.zeros(2), np.zeros(3), 1, 0.1)
    with pytest.raises(ValueError):
        oracle.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3), 0, 0.1)
