"""Pins for the oracle's exact-ratio propagator (CPU only).

With an exact sampling ratio alpha = N lambda_l / lambda_min the propagator of
Eq. 1 is the scaled DFT that the chirp z-transform evaluates (section
"Benchmarking with state-of-art open-source ptychography algorithm").  These
tests tie the oracle's matrix form to results fixed elsewhere: the
zero-padded FFT at integer ratios (numpy's FFT, a different code path),
closed forms for point sources and discrete plane waves (geometric series),
continuity in alpha, the adjoint identity, and central finite differences of
the loss through the whole model.
"""
import numpy as np
import pytest

from oracle import model as om

from test_oracle_model import _fd_check, _perturbed_measurement, crandn, tiny_problem


def _rand(N, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))


@pytest.mark.parametrize("N,nl", [(4, 4), (4, 7), (6, 11), (8, 13), (8, 8)])
def test_integer_ratio_is_the_zero_padded_dft(N, nl):
    psi = _rand(N, nl)
    a = om.propagate(psi, float(nl))
    b = om.propagate(psi, int(nl))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))
    g = _rand(N, nl + 1)
    a = om.propagate_adjoint(g, float(nl))
    b = om.propagate_adjoint(g, int(nl))
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


@pytest.mark.parametrize("N,alpha", [(6, 7.3), (8, 11.77), (16, 23.456)])
def test_point_source_closed_form(N, alpha):
    r0, s0 = 2, N - 3
    psi = np.zeros((N, N), complex)
    psi[r0, s0] = 1.0
    u = np.arange(N) - N // 2
    ref = np.exp(-2j * np.pi * (u[:, None] * r0 + u[None, :] * s0) / alpha) / alpha
    got = om.propagate(psi, alpha)
    assert np.max(np.abs(got - ref)) <= 1e-14


@pytest.mark.parametrize("N,alpha,ky,kx", [(8, 10.5, 1.3, -2.7), (12, 17.25, -3.1, 0.45)])
def test_discrete_plane_wave_geometric_series(N, alpha, ky, kx):
    r = np.arange(N)
    psi = np.exp(2j * np.pi * (ky * r[:, None] + kx * r[None, :]) / alpha)
    u = np.arange(N) - N // 2

    def geo(d):
        q = np.exp(2j * np.pi * d / alpha)
        return (1 - q ** N) / (1 - q)

    ref = np.outer(geo(ky - u), geo(kx - u)) / alpha
    got = om.propagate(psi, alpha)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_continuous_in_the_ratio():
    # the scaled DFT is smooth in alpha and meets the padded DFT at integers
    N, nl = 8, 11
    psi = _rand(N, 5)
    b = om.propagate(psi, nl)
    for h in (1e-6, -1e-6):
        a = om.propagate(psi, nl + h)
        assert 0 < np.max(np.abs(a - b)) <= 1e-4 * np.max(np.abs(b))


@pytest.mark.parametrize("N,alpha", [(8, 9.6), (12, 16.9)])
def test_adjoint_identity(N, alpha):
    x, y = _rand(N, 1), _rand(N, 2)
    lhs = np.vdot(y, om.propagate(x, alpha))
    rhs = np.vdot(om.propagate_adjoint(y, alpha), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_ratio_below_the_window_is_rejected():
    with pytest.raises(ValueError):
        om.propagate(_rand(8), 7.5)


def test_forward_brute_force_with_ratios():
    from test_oracle_model import brute_forward
    pr = tiny_problem(seed=4, L=2, M=2, Ns=1, N=4, pads=(4.0, 5.63), H=9, W=9, K=2,
                      with_sigma=True)
    ref = brute_forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"], pr["sigma"], None, None)
    got = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"], sigma=pr["sigma"])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("kind", [om.LOSS_AMPLITUDE, om.LOSS_POISSON])
def test_gradients_match_central_differences_with_ratios(kind):
    pr = tiny_problem(seed=17, L=2, M=2, pads=(9.41, 12.66), with_sigma=True)
    meas = _perturbed_measurement(pr)
    kw = dict(kind=kind, eps=1e-3, scale=0.5, sigma=pr["sigma"])
    base = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, **kw)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(2):
        v = crandn(rng, *pr["obj"].shape)
        fd, an = _fd_check(lambda o: om.loss_grad(o, pr["prb"], pr["pos"], pr["pads"], meas,
                                                  **kw)["loss"], base["g_object"], pr["obj"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("object", fd, an)
        v = crandn(rng, *pr["prb"].shape)
        fd, an = _fd_check(lambda p: om.loss_grad(pr["obj"], p, pr["pos"], pr["pads"], meas,
                                                  **kw)["loss"], base["g_probe"], pr["prb"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("probe", fd, an)
    v = rng.normal(size=pr["sigma"].shape)
    fd, an = _fd_check(lambda s: om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas,
                                              **{**kw, "sigma": s})["loss"],
                       base["g_sigma"], pr["sigma"], v, h)
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("sigma", fd, an)
    # position derivative, differentiated in float64 through the shift
    N = pr["prb"].shape[-1]
    p, d = om.split_positions(pr["pos"])
    for k in range(2):
        def loss_at(delta):
            tot = 0.0
            I = np.zeros((N, N))
            for l in range(2):
                A = pr["obj"][l, 0, p[k, 0]:p[k, 0] + N, p[k, 1]:p[k, 1] + N]
                Os = om.shift_patch(A, delta)
                for m in range(2):
                    I += np.abs(om.propagate(pr["sigma"][k] * pr["prb"][l, m] * Os,
                                             pr["pads"][l])) ** 2
            ell, _ = om.pointwise_loss(I, meas[k], kind, 1e-3)
            tot += float(np.sum(ell)) * 0.5
            return tot
        for ax in range(2):
            e = np.zeros(2)
            e[ax] = h
            fd = (loss_at(d[k] + e) - loss_at(d[k] - e)) / (2 * h)
            assert abs(fd - base["g_pos"][k, ax]) <= 1e-6 * max(abs(fd), 1e-3), (k, ax)


def test_zero_gradient_at_noiseless_truth_with_ratios():
    pr = tiny_problem(seed=19, pads=(8.0, 10.37))
    meas = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"])
    r = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas)
    assert abs(r["loss"]) <= 1e-12 * np.sum(meas)
    for key in ("g_object", "g_probe", "g_pos"):
        assert np.max(np.abs(r[key])) < 1e-9, key


def test_ratio_gradient_matches_central_differences():
    # dL/d alpha_l: the propagation-distance gradient of the exact-ratio model
    for kind in (om.LOSS_AMPLITUDE, om.LOSS_POISSON):
        pr = tiny_problem(seed=23, L=2, M=2, pads=(9.41, 12.66), with_sigma=True,
                          with_bg=True, with_table=True)
        meas = _perturbed_measurement(pr)
        kw = dict(kind=kind, eps=1e-3, scale=0.7, sigma=pr["sigma"], background=pr["bg"],
                  resample_table=pr["table"])
        base = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, **kw)
        h = 1e-5
        for l in range(2):
            up, dn = list(pr["pads"]), list(pr["pads"])
            up[l] += h
            dn[l] -= h
            fd = (om.loss_grad(pr["obj"], pr["prb"], pr["pos"], tuple(up), meas, **kw)["loss"] -
                  om.loss_grad(pr["obj"], pr["prb"], pr["pos"], tuple(dn), meas, **kw)["loss"]) / (2 * h)
            an = base["g_ratio"][l]
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (kind, l, fd, an)


def test_ratio_gradient_is_zero_for_padded_wavelengths_and_at_truth():
    pr = tiny_problem(seed=25, pads=(8, 10.37))
    meas = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"])
    r = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas)
    assert r["g_ratio"][0] == 0.0
    assert abs(r["g_ratio"][1]) < 1e-9
    pr2 = tiny_problem(seed=25, pads=(8, 10.37))
    meas2 = _perturbed_measurement(pr2)
    r2 = om.loss_grad(pr2["obj"], pr2["prb"], pr2["pos"], pr2["pads"], meas2)
    assert r2["g_ratio"][0] == 0.0 and abs(r2["g_ratio"][1]) > 1e-6


def test_ratio_derivative_of_the_propagator_matches_differences():
    N, a = 8, 11.3
    psi = _rand(N, 9)
    h = 1e-6
    fd = (om.propagate(psi, a + h) - om.propagate(psi, a - h)) / (2 * h)
    an = om.propagate_dalpha(psi, a)
    assert np.max(np.abs(fd - an)) <= 1e-7 * np.max(np.abs(an))
