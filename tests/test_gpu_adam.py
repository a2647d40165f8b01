"""Three consecutive fused steps (loss + gradient + Adam, ``ptycho_step``)
against the FP64 oracle's Adam step (the paper's optimiser, Section
"Universal Ptychography Algorithm based on Automatic Differentiation").

Every step t = 1, 2, 3 is checked in two parts:
* the gradient the step used is the oracle's gradient at the state before
  the step (relative L2 and max-abs/max-ref 1e-4; per position 1e-3);
* the new variables and moments are oracle.adam_step applied to the state,
  moments and gradient before the step.  Both sides then do the same
  arithmetic on the same inputs, FP32 against FP64: the moments agree to a
  few float32 roundings (2^-20 relative), and each variable to a few
  roundings of its own magnitude plus 1e-5 of its step.
From t = 2 on the moments are non-zero, so the beta * m and beta * v terms
and the bias corrections at t > 1 are exercised.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import parity_util as U

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"

VARS = ("object", "probe", "pos", "sigma", "background")
# the background stays well above zero (it starts in [0, 2], moves by at most
# 3 lr): the Poisson loss needs I' + eps > 0 on every pixel
LR = dict(object=2e-3, probe=1e-3, pos=1e-2, sigma=2e-3, background=1e-3)


def _real(t):
    t = t.detach()
    return (torch.view_as_real(t) if t.is_complex() else t).double().cpu().numpy().ravel()


def test_three_fused_adam_steps_match_the_oracle():
    from paper_2311_14780_amd import binding as B
    w = synth.reduced(synth.get_workload("C1"), L=2, M=2, harmonics=(19, 23),
                      mode_weights=(0.75, 0.25), K=12, name="C1-adam3")
    case = U.make_case(w, with_sigma=True, with_bg=True, with_mask=True, pads=(80, 64))
    case["bg"] = (case["bg"] + 0.5).astype(np.float32)
    prob = U.to_problem(case, DEV)
    var = dict(object=prob.object, probe=prob.probe, pos=prob.pos, sigma=prob.sigma,
               background=prob.background)
    n = {k: v.numel() * (2 if v.is_complex() else 1) for k, v in var.items()}
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV),
             g_sigma=torch.zeros(prob.K, device=DEV),
             g_background=torch.zeros(prob.N, prob.N, device=DEV))
    adam = {"t": 0, "beta1": 0.9, "beta2": 0.999, "eps": 1e-8}
    for k in VARS:
        adam["m_" + k] = torch.zeros(n[k], device=DEV)
        adam["v_" + k] = torch.zeros(n[k], device=DEV)
        adam["lr_" + k] = LR[k]
    ws = B.workspace([prob], 2)
    for t in (1, 2, 3):
        x0 = {k: var[k].detach().clone() for k in VARS}
        m0 = {k: adam["m_" + k].clone() for k in VARS}
        v0 = {k: adam["v_" + k].clone() for k in VARS}
        adam["t"] = t
        B.ptycho_step([prob], [g], [adam], kind=1, workspace=ws)
        torch.cuda.synchronize()
        assert B.ptycho_status(ws, 0) == B.PTYCHO_OK
        # the gradient of the state before the step, against the oracle
        st = dict(case, obj=x0["object"].cpu().numpy(), prb=x0["probe"].cpu().numpy(),
                  pos=x0["pos"].cpu().numpy(), sigma=x0["sigma"].cpu().numpy(),
                  bg=x0["background"].cpu().numpy())
        got = {"loss": float(g["loss"].item())}
        got.update({"g_" + k: g["g_" + k].cpu().numpy() for k in VARS})
        print(f"t={t}", end=" ")
        U.compare(got, U.oracle_grads(st, kind=1))
        # the update: oracle Adam on the device's state, moments and gradient,
        # with the hyper-parameters as the device holds them (float32)
        b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
        lr_of = lambda k: float(np.float32(LR[k]))
        for k in VARS:
            xk, gk, mk, vk = _real(x0[k]), _real(g["g_" + k]), _real(m0[k]), _real(v0[k])
            xr, mr, vr = oracle.adam_step(xk, gk, mk, vk, t, lr_of(k), b1, b2,
                                          float(np.float32(1e-8)))
            mg, vg, xg = _real(adam["m_" + k]), _real(adam["v_" + k]), _real(var[k])
            # a few float32 roundings of the two terms of each recursion
            dm = 2.0 ** -22 * (np.abs(b1 * mk) + np.abs((1 - b1) * gk))
            dv = 2.0 ** -22 * (np.abs(b2 * vk) + np.abs((1 - b2) * gk * gk))
            assert np.all(np.abs(mg - mr) <= dm + 1e-38), (t, k, "m")
            assert np.all(np.abs(vg - vr) <= dv + 1e-38), (t, k, "v")
            # the step carries the device's rounding of m and v, its own few
            # roundings, and the final rounding of x
            den = np.sqrt(vr / (1 - b2 ** t)) + 1e-8
            step = np.abs(xr - xk)
            tol = (2.0 ** -22 * np.maximum(np.abs(xr), np.abs(xk)) + 2.0 ** -20 * step
                   + lr_of(k) / (1 - b1 ** t) * dm / den + step * dv / np.maximum(vr, 1e-38) + 1e-38)
            bad = np.abs(xg - xr) > tol
            assert not bad.any(), (t, k, int(bad.sum()), float(np.max(np.abs(xg - xr) - tol)))
            if t > 1:
                assert np.any(mr != 0) and np.any(m0[k].cpu().numpy() != 0), k
        print(f"t={t}: variables and moments match oracle.adam_step", flush=True)


def test_step_with_a_window_outside_leaves_the_state_unchanged():
    # a window that leaves the object: the call reports PTYCHO_ERANGE, and the
    # Adam step of that job changes neither its variables nor its moments
    from paper_2311_14780_amd import binding as B
    w = synth.reduced(synth.get_workload("C1"), K=6, name="C1-erange-step")
    case = U.make_case(w)
    prob = U.to_problem(case, DEV)
    pos = prob.pos.clone()
    pos[3, 1] = 250.0  # window [250, 314) leaves the 256-px object
    prob.pos = pos
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(prob.K, 2, device=DEV))
    gen = torch.Generator(device=DEV).manual_seed(5)
    r = lambda x: torch.rand(x.numel() * (2 if x.is_complex() else 1), device=DEV, generator=gen)
    adam = dict(m_object=r(prob.object), v_object=r(prob.object), m_probe=r(prob.probe),
                v_probe=r(prob.probe), m_pos=r(prob.pos), v_pos=r(prob.pos),
                lr_object=1e-2, lr_probe=1e-2, lr_pos=1e-1, t=2)
    before = [t.clone() for t in (prob.object, prob.probe, prob.pos, adam["m_object"],
                                  adam["v_object"], adam["m_probe"], adam["v_probe"],
                                  adam["m_pos"], adam["v_pos"])]
    ws = B.workspace([prob], 2)
    B.ptycho_step([prob], [g], [adam], workspace=ws)
    torch.cuda.synchronize()
    assert B.ptycho_status(ws, 0) == B.PTYCHO_ERANGE
    assert np.isnan(float(g["loss"].item()))
    after = (prob.object, prob.probe, prob.pos, adam["m_object"], adam["v_object"],
             adam["m_probe"], adam["v_probe"], adam["m_pos"], adam["v_pos"])
    for a, b in zip(before, after):
        assert torch.equal(a, b)
