"""GPU parity beyond the basic cases: the reflection (tilt-table) workload,
the large multiplexed shapes, the VJP mode, the Adam step, the autograd
wrappers with finite differences, and the full-size four-wavelength workload
at the benchmark's launch configuration."""
import numpy as np
import pytest

import oracle
import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def test_c5_tilt_table_positions_full_shapes():
    case = U.make_case(synth.get_workload("C5"), K=3)
    assert case["table"] is not None and case["mask"] is not None
    prob = U.to_problem(case, DEV)
    fwd = U.gpu_forward(prob)
    ref = U.oracle_forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                           case["pos"], case["pads"], table=case["table"])
    U.check_array("C5(K=3) forward", fwd, ref, 1e-5)
    got = U.gpu_grads(prob)
    print("C5(K=3) grads", U.compare(got, U.oracle_grads(case)))


def test_c3_shapes_reduced_positions():
    # 16 positions at the full N / L / M of the large multiplexed workload,
    # several chunks per call
    case = U.make_case(synth.get_workload("C3"), K=16, workers=U.default_workers())
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, chunk=5)
    print("C3(K=16) grads", U.compare(got, U.oracle_grads(case, workers=U.default_workers())))


def test_vjp_mode_matches_oracle():
    case = U.make_case(synth.reduced(synth.get_workload("C1"), K=10, name="C1v"))
    rng = np.random.default_rng(4)
    case["meas"] = rng.normal(size=case["meas"].shape).astype(np.float32)  # upstream dL/dI'
    prob = U.to_problem(case, DEV)
    got = U.gpu_grads(prob, kind=3)
    print("VJP", U.compare(got, U.oracle_grads(case, kind=3)))


def test_adam_step_updates_state():
    from paper_2311_14780_amd import binding as B
    case = U.make_case(synth.reduced(synth.get_workload("C1"), K=16, name="C1a"))
    prob = U.to_problem(case, DEV)
    o0, p0, s0 = prob.object.clone(), prob.probe.clone(), prob.pos.clone()
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV))
    z = lambda x: torch.zeros(x.numel() * (2 if x.is_complex() else 1), device=DEV)
    adam = dict(m_object=z(o0), v_object=z(o0), m_probe=z(p0), v_probe=z(p0), m_pos=z(s0),
                v_pos=z(s0), lr_object=1e-3, lr_probe=2e-3, lr_pos=1e-2, t=1)
    ws = B.workspace([prob], 2)
    B.ptycho_step([prob], [g], [adam], workspace=ws)
    torch.cuda.synchronize()
    # the gradient is the oracle's at the state before the update
    ref = U.oracle_grads(case)
    errs = U.compare({"loss": float(g["loss"].item()), "g_object": g["g_object"].cpu().numpy(),
                      "g_probe": g["g_probe"].cpu().numpy(), "g_pos": g["g_pos"].cpu().numpy()}, ref)
    print("step grads", errs)

    def adam1(x0, grad, lr):
        x0 = np.asarray(x0, np.float64).ravel()
        gr = np.asarray(grad, np.float64).ravel()
        m = 0.1 * gr
        v = 0.001 * gr * gr
        return x0 - lr * (m / 0.1) / (np.sqrt(v / 0.001) + 1e-8)

    for x0, x1, gg, lr in ((o0, prob.object, g["g_object"], 1e-3), (p0, prob.probe, g["g_probe"], 2e-3),
                           (s0, prob.pos, g["g_pos"], 1e-2)):
        r0 = torch.view_as_real(x0).cpu().numpy() if x0.is_complex() else x0.cpu().numpy()
        rg = torch.view_as_real(gg).cpu().numpy() if gg.is_complex() else gg.cpu().numpy()
        r1 = torch.view_as_real(x1).cpu().numpy() if x1.is_complex() else x1.cpu().numpy()
        want = adam1(r0, rg, lr)
        d_got = r1.ravel().astype(np.float64) - r0.ravel()
        d_want = want - r0.ravel()
        assert U.rel_l2(d_got, d_want) <= 1e-3
    # the Adam state holds the first moments
    assert torch.allclose(adam["m_pos"], 0.1 * g["g_pos"].reshape(-1), rtol=1e-6, atol=0)


def test_adam_step_updates_sigma_and_background():
    # the power coefficients and the common background are variables too
    from paper_2311_14780_amd import binding as B
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=10, name="C1sb")
    case = U.make_case(w, with_sigma=True, with_bg=True, with_mask=True, pads=(80, 64))
    prob = U.to_problem(case, DEV)
    sg0, bg0 = prob.sigma.clone(), prob.background.clone()
    g = dict(loss=torch.zeros(1, device=DEV), g_sigma=torch.zeros(prob.K, device=DEV),
             g_background=torch.zeros(prob.N, prob.N, device=DEV))
    z = lambda x: torch.zeros(x.numel(), device=DEV)
    adam = dict(m_sigma=z(sg0), v_sigma=z(sg0), m_background=z(bg0), v_background=z(bg0),
                lr_sigma=5e-3, lr_background=2e-2, t=1)
    ws = B.workspace([prob], 2)
    B.ptycho_step([prob], [g], [adam], kind=1, workspace=ws)
    torch.cuda.synchronize()
    ref = U.oracle_grads(case, kind=1)
    got = {"loss": float(g["loss"].item()), "g_sigma": g["g_sigma"].cpu().numpy(),
           "g_background": g["g_background"].cpu().numpy()}
    print("sigma/background grads", U.compare(got, ref, keys=("g_sigma", "g_background")))
    for x0, x1, gg, lr in ((sg0, prob.sigma, g["g_sigma"], 5e-3),
                           (bg0, prob.background, g["g_background"], 2e-2)):
        gr = gg.cpu().numpy().astype(np.float64).ravel()
        want = -lr * gr / (np.abs(gr) + 1e-8)  # first Adam step: -lr sign(g)
        d_got = (x1.cpu().numpy().astype(np.float64) - x0.cpu().numpy()).ravel()
        assert U.rel_l2(d_got, want) <= 1e-4
    # object, probe and positions were left alone (zero learning rates)
    assert torch.equal(prob.object, torch.from_numpy(case["obj"]).to(DEV))


def test_autograd_loss_matches_direct_call_and_differences():
    from paper_2311_14780_amd import autograd as A
    case = U.make_case(synth.reduced(synth.get_workload("C1"), K=8, name="C1g"))
    prob = U.to_problem(case, DEV)
    obj = prob.object.clone().requires_grad_(True)
    prb = prob.probe.clone().requires_grad_(True)
    pos = prob.pos.clone().requires_grad_(True)
    loss = A.ptycho_loss(obj, prb, pos, prob.pads, prob.measured, scale=1.0 / prob.K)
    (2.0 * loss).backward()
    direct = U.gpu_grads(prob, scale=1.0 / prob.K)
    assert np.array_equal(obj.grad.cpu().numpy(), 2.0 * direct["g_object"])
    assert np.array_equal(prb.grad.cpu().numpy(), 2.0 * direct["g_probe"])
    assert np.array_equal(pos.grad.cpu().numpy(), 2.0 * direct["g_pos"])
    # Central differences of the float32 loss along random sparse directions
    # (32 random object pixels and 32 random probe pixels, complex normal
    # weights scaled to the local magnitude): dense random directions have a
    # tiny directional derivative next to their curvature, which float32
    # differences cannot resolve.  Richardson extrapolation removes the h^2
    # term; the tolerance adds the float32 noise of the loss (1e-6 L / h).
    rng = np.random.default_rng(6)
    go = direct["g_object"]
    gp = direct["g_probe"]
    L0 = prob.K * direct["loss"]
    ob_np = obj.detach().cpu().numpy()
    pr_np = prb.detach().cpu().numpy()
    support = np.flatnonzero(np.abs(pr_np) > 0.05 * np.abs(pr_np).max())
    fails = []
    for trial in range(64):
        vo = np.zeros(ob_np.size, np.complex128)
        vp = np.zeros(pr_np.size, np.complex128)
        # object pixels inside some window, probe pixels inside the support
        io = rng.choice(np.flatnonzero(np.abs(go.ravel()) > 0), 32, replace=False)
        ip = rng.choice(support, 32, replace=False)
        vo[io] = (rng.normal(size=32) + 1j * rng.normal(size=32)) * np.abs(ob_np.ravel()[io])
        vp[ip] = (rng.normal(size=32) + 1j * rng.normal(size=32)) * np.abs(pr_np.ravel()[ip])
        an = prob.K * float(np.sum(go.ravel().real * vo.real + go.ravel().imag * vo.imag)
                            + np.sum(gp.ravel().real * vp.real + gp.ravel().imag * vp.imag))
        vo_t = torch.from_numpy(vo.reshape(ob_np.shape).astype(np.complex64)).to(DEV)
        vp_t = torch.from_numpy(vp.reshape(pr_np.shape).astype(np.complex64)).to(DEV)
        h = 1e-2

        def central(hh):
            with torch.no_grad():
                lp = A.ptycho_loss(obj + hh * vo_t, prb + hh * vp_t, pos, prob.pads, prob.measured).double().item()
                lm = A.ptycho_loss(obj - hh * vo_t, prb - hh * vp_t, pos, prob.pads, prob.measured).double().item()
            return (lp - lm) / (2.0 * hh)

        fd = (4.0 * central(h / 2) - central(h)) / 3.0
        if abs(fd - an) > 1e-2 * abs(an) + 1e-6 * abs(L0) / h:
            fails.append((trial, fd, an))
    assert not fails, fails


def test_forward_autograd_is_the_vjp():
    from paper_2311_14780_amd import autograd as A
    case = U.make_case(synth.reduced(synth.get_workload("C1"), K=6, name="C1f"))
    prob = U.to_problem(case, DEV)
    obj = prob.object.clone().requires_grad_(True)
    prb = prob.probe.clone().requires_grad_(True)
    pos = prob.pos.clone().requires_grad_(True)
    I = A.ptycho_forward(obj, prb, pos, prob.pads)
    u = torch.from_numpy(np.random.default_rng(8).normal(size=tuple(I.shape)).astype(np.float32)).to(DEV)
    (I * u).sum().backward()
    case["meas"] = u.cpu().numpy()
    ref = U.oracle_grads(case, kind=3)
    got = {"loss": float((I.detach() * u).sum().item()), "g_object": obj.grad.cpu().numpy(),
           "g_probe": prb.grad.cpu().numpy(), "g_pos": pos.grad.cpu().numpy()}
    print("forward VJP", U.compare(got, ref, tol_loss=1e-5))


def test_forward_autograd_background_and_distance():
    # the VJP of the forward model through the background and the exact ratios
    from paper_2311_14780_amd import autograd as A
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=6, name="C1fv")
    ratios = synth.ratios_for(w.N, w.harmonics, w.ref_harmonic)
    case = U.make_case(w, pads=ratios, with_bg=True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    obj = t(case["obj"]).requires_grad_()
    bg = t(case["bg"]).requires_grad_()
    ratio = torch.tensor(ratios, dtype=torch.float64, requires_grad=True)
    I = A.ptycho_forward(obj, t(case["prb"]), t(case["pos"]), (0, 0), background=bg, ratio=ratio)
    u = torch.from_numpy(np.random.default_rng(9).normal(size=tuple(I.shape)).astype(np.float32)).to(DEV)
    (I * u).sum().backward()
    case["meas"] = u.cpu().numpy()
    ref = U.oracle_grads(case, kind=3)
    got = {"loss": float((I.detach() * u).sum().item()), "g_object": obj.grad.cpu().numpy(),
           "g_background": bg.grad.cpu().numpy(), "g_ratio": ratio.grad.numpy()}
    print("forward VJP bg/ratio", U.compare(got, ref))


def test_c2_full_size_at_bench_configuration():
    """All 400 positions of the four-wavelength workload in one chunk (the
    benchmark's launch configuration); the oracle runs over position blocks
    in worker processes and its parts add up exactly."""
    w = synth.get_workload("C2")
    nw = U.default_workers()
    case = U.make_case(w, workers=nw)
    prob = U.to_problem(case, DEV)
    fwd = U.gpu_forward(prob)
    sample = [0, 57, 199, 311, 399]
    ref_i = oracle.forward(case["obj"].astype(np.complex128), case["prb"].astype(np.complex128),
                           case["pos"][sample], case["pads"])
    U.check_array("C2 full forward (sampled positions)", fwd[sample], ref_i, 1e-5)
    got = U.gpu_grads(prob)
    ref = U.oracle_grads(case, workers=nw)
    print("C2 full grads", U.compare(got, ref))


def test_autograd_background_distance_and_regularisers():
    # torch autograd through the library: background and the exact ratios
    # (alpha proportional to the propagation distance) as differentiable inputs
    from paper_2311_14780_amd import autograd as A
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=8, name="C1-ag")
    ratios = synth.ratios_for(w.N, w.harmonics, w.ref_harmonic)
    case = U.make_case(w, pads=ratios, with_bg=True)
    reg = dict(l1=0.01, tv=0.2, tv_eps=0.05)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    obj = t(case["obj"]).requires_grad_()
    prb = t(case["prb"]).requires_grad_()
    pos = t(case["pos"])
    bg = t(case["bg"]).requires_grad_()
    ratio = torch.tensor(ratios, dtype=torch.float64, requires_grad=True)
    loss = A.ptycho_loss(obj, prb, pos, (0, 0), t(case["meas"]), background=bg, ratio=ratio,
                         kind=1, **reg)
    loss.backward()
    ref = U.oracle_grads(case, kind=1, **reg)
    got = {"loss": float(loss.item()), "g_object": obj.grad.cpu().numpy(),
           "g_probe": prb.grad.cpu().numpy(), "g_background": bg.grad.cpu().numpy(),
           "g_ratio": ratio.grad.numpy()}
    assert ratio.grad.dtype == torch.float64
    print("autograd bg/ratio/reg", U.compare(got, ref))
