"""Pins for the oracle's forward model, loss and gradient (CPU only)."""
import numpy as np
import pytest

from oracle import model as om


def crandn(rng, *shape):
    return rng.normal(size=shape) + 1j * rng.normal(size=shape)


def tiny_problem(seed=0, L=2, M=2, Ns=1, N=8, pads=(8, 11), H=20, W=22, K=5,
                 with_sigma=False, with_bg=False, with_table=False):
    rng = np.random.default_rng(seed)
    obj = (0.6 + 0.4 * rng.uniform(size=(L, Ns, H, W))) * np.exp(1j * rng.uniform(-3, 3, (L, Ns, H, W)))
    prb = crandn(rng, L, M, N, N)
    pos = np.stack([rng.uniform(0.6, H - N - 0.6, K), rng.uniform(0.6, W - N - 0.6, K)], 1)
    # keep the sub-pixel part away from the rounding boundary so that
    # finite differences never change the integer window corner
    p, d = om.split_positions(pos.astype(np.float32))
    d = np.clip(d, -0.4, 0.4)
    pos = (p + d).astype(np.float32)
    sigma = rng.uniform(0.7, 1.3, K) if with_sigma else None
    bg = rng.uniform(0, 0.5, (N, N)) if with_bg else None
    table = None
    if with_table:
        idx = rng.integers(0, N * N, size=(N * N, 4)).astype(np.int32)
        w = rng.uniform(0, 0.5, size=(N * N, 4)).astype(np.float32)
        table = (idx, w)
    return dict(obj=obj, prb=prb, pos=pos, pads=pads[:L], sigma=sigma, bg=bg, table=table, rng=rng)


# --------------------------------------------------------------- brute force
def brute_forward(obj, prb, pos, pads, sigma, bg, table):
    """Eq. 1 written as explicit sums (tiny sizes only)."""
    L, Ns, H, W = obj.shape
    M, N = prb.shape[1], prb.shape[-1]
    K = pos.shape[0]
    nu = np.array([j / N if j < N / 2 else (j - N) / N for j in range(N)])
    out = np.zeros((K, N, N))
    for k in range(K):
        s = pos[k].astype(np.float32)
        p = [int(np.floor(np.float32(s[i]) + np.float32(0.5))) for i in range(2)]
        dl = [float(s[i]) - p[i] for i in range(2)]
        sig = 1.0 if sigma is None else sigma[k]
        I = np.zeros((N, N))
        for l in range(L):
            nl = pads[l]
            for n in range(Ns):
                A = obj[l, n, p[0]:p[0] + N, p[1]:p[1] + N]
                # Fourier coefficients, then evaluation at r + delta
                c = np.zeros((N, N), complex)
                for a in range(N):
                    for b in range(N):
                        c[a, b] = sum(A[y, x] * np.exp(-2j * np.pi * (a * y + b * x) / N)
                                      for y in range(N) for x in range(N)) / (N * N)
                Os = np.zeros((N, N), complex)
                for y in range(N):
                    for x in range(N):
                        Os[y, x] = sum(c[a, b] * np.exp(2j * np.pi * (nu[a] * (y + dl[0]) + nu[b] * (x + dl[1])))
                                       for a in range(N) for b in range(N))
                for m in range(M):
                    psi = sig * prb[l, m] * Os
                    for ia in range(N):
                        for ib in range(N):
                            u, v = ia - N // 2, ib - N // 2
                            acc = sum(psi[y, x] * np.exp(-2j * np.pi * (u * y + v * x) / nl)
                                      for y in range(N) for x in range(N)) / nl
                            I[ia, ib] += abs(acc) ** 2
        if bg is not None:
            I = I + bg
        if table is not None:
            idx, w = table
            flat = I.ravel()
            J = np.zeros(N * N)
            for a in range(N * N):
                for t in range(4):
                    J[a] += float(w[a, t]) * flat[idx[a, t]]
            I = J.reshape(N, N)
        out[k] = I
    return out


def test_forward_matches_brute_force_eq1():
    pr = tiny_problem(seed=3, L=2, M=2, Ns=2, N=4, pads=(4, 6), H=9, W=9, K=3,
                      with_sigma=True, with_bg=True, with_table=True)
    ref = brute_forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"], pr["sigma"], pr["bg"], pr["table"])
    got = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"], sigma=pr["sigma"],
                     background=pr["bg"], resample_table=pr["table"])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_forward_rejects_window_outside_object():
    pr = tiny_problem()
    pos = pr["pos"].copy()
    pos[0] = (-1.0, 0.0)
    with pytest.raises(ValueError):
        om.forward(pr["obj"], pr["prb"], pos, pr["pads"])


# ----------------------------------------------------- truth, invariants, FD
@pytest.mark.parametrize("kind", [om.LOSS_AMPLITUDE, om.LOSS_GAUSSIAN, om.LOSS_POISSON])
def test_zero_gradient_at_noiseless_truth(kind):
    pr = tiny_problem(seed=5, with_sigma=True, with_bg=True)
    meas = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"], sigma=pr["sigma"], background=pr["bg"])
    r = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, kind=kind,
                     sigma=pr["sigma"], background=pr["bg"])
    if kind != om.LOSS_POISSON:
        assert abs(r["loss"]) <= 1e-12 * np.sum(meas)
    for key in ("g_object", "g_probe", "g_pos", "g_sigma", "g_background"):
        assert np.max(np.abs(r[key])) < 1e-9, key


def _perturbed_measurement(pr, seed=11):
    meas = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"], sigma=pr["sigma"],
                      background=pr["bg"], resample_table=pr["table"])
    rng = np.random.default_rng(seed)
    return rng.poisson(meas * 1.3 + 0.2).astype(np.float64)


def _fd_check(fun, grad, x, direction, h):
    lp = fun(x + h * direction)
    lm = fun(x - h * direction)
    fd = (lp - lm) / (2 * h)
    an = float(np.real(np.vdot(grad, direction)))
    return fd, an


@pytest.mark.parametrize("kind", [om.LOSS_AMPLITUDE, om.LOSS_GAUSSIAN, om.LOSS_POISSON])
@pytest.mark.parametrize("extras", [False, True])
def test_gradients_match_central_differences(kind, extras):
    pr = tiny_problem(seed=7, L=2, M=2, Ns=2 if extras else 1, with_sigma=extras,
                      with_bg=extras, with_table=extras)
    meas = _perturbed_measurement(pr)
    mask = None
    if extras:
        mask = (pr["rng"].uniform(size=meas.shape[1:]) > 0.2).astype(np.uint8)
    kw = dict(kind=kind, eps=1e-3, scale=0.37, sigma=pr["sigma"], background=pr["bg"],
              mask=mask, resample_table=pr["table"])
    base = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, **kw)
    rng = np.random.default_rng(99)
    h = 1e-6

    def L_obj(o):
        return om.loss_grad(o, pr["prb"], pr["pos"], pr["pads"], meas, **kw)["loss"]

    def L_prb(p):
        return om.loss_grad(pr["obj"], p, pr["pos"], pr["pads"], meas, **kw)["loss"]

    def L_pos(s):
        return om.loss_grad(pr["obj"], pr["prb"], s, pr["pads"], meas, **kw)["loss"]

    for _ in range(3):
        v = crandn(rng, *pr["obj"].shape)
        fd, an = _fd_check(L_obj, base["g_object"], pr["obj"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("object", fd, an)
        v = crandn(rng, *pr["prb"].shape)
        fd, an = _fd_check(L_prb, base["g_probe"], pr["prb"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("probe", fd, an)
    # positions: float32 inputs, so difference in float64 through the same
    # split (p fixed, delta varies): perturb delta directly via float64 pos.
    for k in range(pr["pos"].shape[0]):
        for ax in range(2):
            e = np.zeros(pr["pos"].shape)
            e[k, ax] = 1.0
            sp = pr["pos"].astype(np.float64)
            hh = 1e-4
            # split_positions casts to float32, so step in float32-safe sizes
            lp = L_pos(sp + hh * e)
            lm = L_pos(sp - hh * e)
            dp = (np.float32(sp[k, ax] + hh) - np.float32(sp[k, ax] - hh))
            fd = (lp - lm) / float(dp)
            an = base["g_pos"][k, ax]
            assert abs(fd - an) <= 2e-3 * max(abs(an), 1e-2), ("pos", k, ax, fd, an)
    if extras:
        def L_sig(sv):
            return om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas,
                                **{**kw, "sigma": sv})["loss"]
        v = rng.normal(size=pr["sigma"].shape)
        fd, an = _fd_check(L_sig, base["g_sigma"], pr["sigma"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("sigma", fd, an)

        def L_bg(b):
            return om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas,
                                **{**kw, "background": b})["loss"]
        v = rng.normal(size=pr["bg"].shape)
        fd, an = _fd_check(L_bg, base["g_background"], pr["bg"], v, h)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), ("background", fd, an)


def test_position_gradient_matches_fd_in_float64_delta():
    # Tighter check of the Fourier phase-ramp derivative: differentiate the
    # shift itself in float64 (independent of float32 position storage).
    pr = tiny_problem(seed=8, L=1, M=1, K=1)
    meas = _perturbed_measurement(pr)
    N = pr["prb"].shape[-1]
    p, d = om.split_positions(pr["pos"])
    obj = pr["obj"][0, 0]
    A = obj[p[0, 0]:p[0, 0] + N, p[0, 1]:p[0, 1] + N]

    def loss_at(delta):
        Os = om.shift_patch(A, delta)
        Psi = om.propagate(pr["prb"][0, 0] * Os, pr["pads"][0])
        ell, _ = om.pointwise_loss(np.abs(Psi) ** 2, meas[0], om.LOSS_AMPLITUDE, 1e-6)
        return float(np.sum(ell))

    r = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas)
    h = 1e-6
    for ax in range(2):
        e = np.zeros(2)
        e[ax] = h
        fd = (loss_at(d[0] + e) - loss_at(d[0] - e)) / (2 * h)
        assert abs(fd - r["g_pos"][0, ax]) <= 1e-6 * max(abs(fd), 1e-3)


def test_unitary_mode_mixing_invariance_and_covariance():
    pr = tiny_problem(seed=12, L=2, M=3)
    meas = _perturbed_measurement(pr)
    rng = np.random.default_rng(5)
    U = [np.linalg.qr(crandn(rng, 3, 3))[0] for _ in range(2)]
    prb2 = np.stack([np.tensordot(U[l], pr["prb"][l], axes=(1, 0)) for l in range(2)])
    I1 = om.forward(pr["obj"], pr["prb"], pr["pos"], pr["pads"])
    I2 = om.forward(pr["obj"], prb2, pr["pos"], pr["pads"])
    assert np.max(np.abs(I1 - I2)) <= 1e-12 * np.max(I1)
    g1 = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas)["g_probe"]
    g2 = om.loss_grad(pr["obj"], prb2, pr["pos"], pr["pads"], meas)["g_probe"]
    g1m = np.stack([np.tensordot(U[l], g1[l], axes=(1, 0)) for l in range(2)])
    assert np.max(np.abs(g2 - g1m)) <= 1e-11 * np.max(np.abs(g2))


def test_gauge_identities():
    pr = tiny_problem(seed=13, L=2, M=2, Ns=1, with_sigma=True)
    meas = _perturbed_measurement(pr)
    r = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, sigma=pr["sigma"])
    gO, gP = r["g_object"], r["g_probe"]
    for l in range(2):
        ip_o = np.vdot(gO[l], pr["obj"][l])
        ip_p = sum(np.vdot(gP[l, m], pr["prb"][l, m]) for m in range(2))
        scale = np.sum(np.abs(gO[l]) * np.abs(pr["obj"][l]))
        # global phase of O_l: Im <G_O, O> = 0 ; scale trade-off between O_l and P_l
        assert abs(ip_o.imag) <= 1e-11 * scale
        assert abs(ip_o.real - ip_p.real) <= 1e-11 * scale
        # global phase of each probe mode: Im <G_P, P> = 0
        for m in range(2):
            assert abs(np.vdot(gP[l, m], pr["prb"][l, m]).imag) <= 1e-11 * scale
    tot_p = sum(np.vdot(gP[l, m], pr["prb"][l, m]).real for l in range(2) for m in range(2))
    assert abs(np.dot(pr["sigma"], r["g_sigma"]) - tot_p) <= 1e-10 * abs(tot_p)


def test_loss_is_sum_over_position_subsets():
    pr = tiny_problem(seed=21, K=6)
    meas = _perturbed_measurement(pr)
    full = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas)
    a = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, positions=[0, 2, 4])
    b = om.loss_grad(pr["obj"], pr["prb"], pr["pos"], pr["pads"], meas, positions=[1, 3, 5])
    assert abs(a["loss"] + b["loss"] - full["loss"]) <= 1e-12 * abs(full["loss"])
    for key in ("g_object", "g_probe", "g_pos", "g_background"):
        assert np.allclose(a[key] + b[key], full[key], rtol=0, atol=1e-12 * np.max(np.abs(full[key])))
