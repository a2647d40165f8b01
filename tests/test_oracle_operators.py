"""Pins for the oracle's linear operators (CPU only).

Each operator is checked against something other than its own code:
explicit DFT double sums, closed-form shifts, numpy.roll, Parseval and the
adjoint identity <A x, y> = <x, A^H y>.
"""
import numpy as np
import pytest

from oracle import model as om

RNG = np.random.default_rng(1234)


def crandn(*shape):
    return RNG.normal(size=shape) + 1j * RNG.normal(size=shape)


def brute_propagate(psi, nl):
    """Explicit double sum: Psi[a,b] = 1/nl sum_{y,x} psi e^{-2 pi i (u_a y + u_b x)/nl}."""
    N = psi.shape[0]
    out = np.zeros((N, N), dtype=np.complex128)
    for a in range(N):
        ua = a - N // 2
        for b in range(N):
            ub = b - N // 2
            acc = 0j
            for y in range(N):
                for x in range(N):
                    acc += psi[y, x] * np.exp(-2j * np.pi * (ua * y + ub * x) / nl)
            out[a, b] = acc / nl
    return out


@pytest.mark.parametrize("N,nl", [(4, 4), (4, 5), (4, 7), (6, 6), (6, 7), (6, 11),
                                  (8, 8), (8, 9), (8, 11)])
def test_propagate_matches_double_sum(N, nl):
    psi = crandn(N, N)
    ref = brute_propagate(psi, nl)
    got = om.propagate(psi, nl)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_propagate_plane_wave_lands_on_centre_bin():
    # A constant field of N x N ones with nl = N puts all its energy at DC,
    # which is stored at index (N/2, N/2); the value is N^2 / N = N.
    N = 8
    out = om.propagate(np.ones((N, N)), N)
    assert abs(out[N // 2, N // 2] - N) < 1e-12
    out[N // 2, N // 2] = 0
    assert np.max(np.abs(out)) < 1e-12


def test_propagate_textbook_special_case():
    # nl = N: the operator is the centred unitary 2D DFT.
    N = 16
    psi = crandn(N, N)
    ref = np.fft.fftshift(np.fft.fft2(psi, norm="ortho"))
    assert np.allclose(om.propagate(psi, N), ref, atol=1e-12)


@pytest.mark.parametrize("N,nl", [(8, 8), (8, 13), (16, 21)])
def test_parseval(N, nl):
    psi = crandn(N, N)
    out = om.propagate(psi, nl)
    e_in = np.sum(np.abs(psi) ** 2)
    e_out = np.sum(np.abs(out) ** 2)
    if nl == N:
        assert abs(e_out - e_in) <= 1e-12 * e_in
    else:
        # Only N of nl bins per axis are kept: the kept energy cannot exceed
        # the total, which equals the input energy on the full grid.
        z = np.zeros((nl, nl), complex)
        z[:N, :N] = psi
        full = np.fft.fft2(z, norm="ortho")
        assert abs(np.sum(np.abs(full) ** 2) - e_in) <= 1e-12 * e_in
        assert e_out <= e_in * (1 + 1e-12)


@pytest.mark.parametrize("N,nl", [(8, 8), (8, 11), (12, 15)])
def test_propagate_adjoint_identity(N, nl):
    x = crandn(N, N)
    y = crandn(N, N)
    lhs = np.vdot(y, om.propagate(x, nl))
    rhs = np.vdot(om.propagate_adjoint(y, nl), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_shift_zero_is_identity():
    A = crandn(8, 8)
    assert np.allclose(om.shift_patch(A, (0.0, 0.0)), A, atol=1e-14)


def test_integer_shift_is_roll():
    # result(r) = A(r + delta): a shift by +1 row is numpy.roll by -1.
    A = crandn(8, 8)
    assert np.allclose(om.shift_patch(A, (1.0, 0.0)), np.roll(A, -1, axis=0), atol=1e-13)
    assert np.allclose(om.shift_patch(A, (0.0, -2.0)), np.roll(A, 2, axis=1), atol=1e-13)


def test_subpixel_shift_of_smooth_bump_is_translation():
    # A wide Gaussian is band-limited to machine precision, so its Fourier
    # shift equals the analytic Gaussian evaluated at r + delta.
    N = 64
    y, x = np.mgrid[0:N, 0:N].astype(float)
    c, s = 31.0, 3.0
    A = np.exp(-((y - c) ** 2 + (x - c) ** 2) / (2 * s * s))
    d = (0.3, -0.45)
    ref = np.exp(-((y + d[0] - c) ** 2 + (x + d[1] - c) ** 2) / (2 * s * s))
    assert np.max(np.abs(om.shift_patch(A, d) - ref)) < 1e-12


def test_shift_of_single_fourier_mode():
    # A(r) = exp(2 pi i j r / N) with signed frequency nu = fftfreq(N)[j]
    # becomes A(r) * exp(2 pi i nu delta); the Nyquist bin has nu = -1/2.
    N = 8
    r = np.arange(N)
    for j in range(N):
        nu = np.fft.fftfreq(N)[j]
        A = np.exp(2j * np.pi * j * r / N)[:, None] * np.ones((1, N))
        d = 0.37
        out = om.shift_patch(A, (d, 0.0))
        assert np.allclose(out, A * np.exp(2j * np.pi * nu * d), atol=1e-13)


def test_shift_adjoint_identity_and_unitarity():
    x = crandn(10, 10)
    y = crandn(10, 10)
    d = (0.21, -0.33)
    lhs = np.vdot(y, om.shift_patch(x, d))
    rhs = np.vdot(om.shift_patch_adjoint(y, d), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    assert np.allclose(om.shift_patch_adjoint(om.shift_patch(x, d), d), x, atol=1e-13)


def test_resample_adjoint_identity():
    N = 12
    idx = RNG.integers(0, N * N, size=(N * N, 4)).astype(np.int32)
    w = RNG.uniform(0, 1, size=(N * N, 4)).astype(np.float32)
    x = RNG.normal(size=(N, N))
    y = RNG.normal(size=(N, N))
    lhs = np.sum(y * om.resample(x, idx, w))
    rhs = np.sum(om.resample_adjoint(y, idx, w) * x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_resample_identity_table():
    N = 6
    idx = np.repeat(np.arange(N * N, dtype=np.int32)[:, None], 4, 1)
    w = np.full((N * N, 4), 0.25, np.float32)
    x = RNG.normal(size=(N, N))
    assert np.allclose(om.resample(x, idx, w), x)


def test_split_positions_rounding_in_float32():
    # The largest float32 below 0.5 plus 0.5 rounds to 1.0 in float32.
    s = np.array([[np.nextafter(np.float32(0.5), np.float32(0)), 2.5]], np.float32)
    p, d = om.split_positions(s)
    assert p.tolist() == [[1, 3]]
    assert np.all(d >= -0.5 - 1e-7) and np.all(d < 0.5)
    s = np.array([[10.49, -3.2]], np.float32)
    p, d = om.split_positions(s)
    assert p.tolist() == [[10, -3]]
    assert np.allclose(d, [[np.float64(np.float32(10.49)) - 10, np.float64(np.float32(-3.2)) + 3]])
