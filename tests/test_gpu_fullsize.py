"""Parity at the full sizes of the large multiplexed workload (5 wavelengths
x 8 modes, 512^2 probe, 3072^2 object, 2500 positions), the reflection
workload (3 wavelengths x 4 modes, 384^2 probe, 900 positions, tilt table)
and the benchmark workload (4 wavelengths x 3 modes, 256^2 probe, 400
positions) with the exact-ratio propagator.

The whole scan runs on the device; the FP64 oracle, which cannot evaluate
2500 positions in a test, checks what it can compute position by position:
the predicted patterns and the position and sigma gradients of sampled
positions (each depends on its own position only), and the object gradient
element by element on a 16 x 64 tile that only a few windows overlap (the
oracle sums those windows on a crop of the object).  The probe gradient, a
sum over every window, and the object gradient as a whole are checked
through identities that hold at any size: a global phase of the object leaves the loss unchanged
(Im<G_O, O> = 0), and so does scaling the object up and every probe mode of
the same wavelength down (Re<G_O, O> = sum_m Re<G_P, P> per wavelength).
The device workspace is chunked (several position chunks per call); results
do not depend on the chunk size (bitwise, tested elsewhere).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import parity_util as U

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _case(name, sigma_seed, exact_ratio=False):
    w = synth.get_workload(name)
    truth = synth.make_truth(w)
    if exact_ratio:
        truth["pads"] = truth["ratios"]
    start = synth.make_start(truth, w)
    rng = np.random.default_rng(sigma_seed)
    sigma = rng.uniform(0.8, 1.2, w.K).astype(np.float32)
    return dict(w=w, obj=start["object"][:, 0].astype(np.complex64),
                prb=start["probe"].astype(np.complex64), pos=start["pos"].copy(),
                pads=tuple(truth["pads"]), meas=synth.synthetic_counts(w.K, w.N, w.photons, w.seed),
                sigma=sigma, bg=None, mask=truth["mask"], table=truth["resample"])


def _run(case, ks, ws_gb):
    from paper_2311_14780_amd import binding as B
    w = case["w"]
    print(f"{w.name}: K={w.K} L={w.L} M={w.M} N={w.N} object {w.H}x{w.W} pads {case['pads']}",
          flush=True)
    prob = U.to_problem(case, DEV)
    # forward over the whole scan
    out = torch.empty(w.K, w.N, w.N, device=DEV)
    B.ptycho_forward([prob], [out], torch.empty(int(ws_gb * 2**30), dtype=torch.uint8, device=DEV))
    torch.cuda.synchronize()
    I_gpu = out[ks].cpu().numpy()
    del out
    g = dict(loss=torch.zeros(1, device=DEV), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(w.K, 2, device=DEV),
             g_sigma=torch.zeros(w.K, device=DEV))
    ws = torch.empty(int(ws_gb * 2**30), dtype=torch.uint8, device=DEV)
    B.ptycho_loss_grad([prob], [g], workspace=ws)
    torch.cuda.synchronize()
    assert B.ptycho_status(ws, 0) == B.PTYCHO_OK
    got = {k: v.cpu().numpy() for k, v in g.items()}
    print(f"{w.name}: device loss {float(got['loss'][0]):.6e}", flush=True)
    return I_gpu, got


def _check(case, ks, I_gpu, got):
    obj = case["obj"].astype(np.complex128)
    prb = case["prb"].astype(np.complex128)
    # patterns of the sampled positions
    I_ref = oracle.forward(obj, prb, case["pos"][ks], case["pads"], sigma=case["sigma"][ks],
                           resample_table=case["table"])
    U.check_array(case["w"].name + " intensity (sampled positions)", I_gpu, I_ref, 1e-5)
    # position and sigma gradients of the sampled positions
    gp, gs = [], []
    for k in ks:
        r = oracle.loss_grad(obj, prb, case["pos"], case["pads"], case["meas"], sigma=case["sigma"],
                             mask=case["mask"], resample_table=case["table"], positions=[k])
        gp.append(r["g_pos"][k])
        gs.append(r["g_sigma"][k])
    e_pos = U.rel_l2(got["g_pos"][ks], np.array(gp))
    e_sig = U.rel_l2(got["g_sigma"][ks], np.array(gs))
    pp = max(U.per_position_rel(got["g_pos"][ks], np.array(gp)),
             U.per_position_rel(got["g_sigma"][ks], np.array(gs)))
    # the object gradient, element by element, on a tile that a few windows
    # overlap (it depends on those windows only)
    w = case["w"]
    ty, tx, hit = U.sparse_object_tile(case["pos"], w.N, w.H, w.W)
    ref_tile = U.oracle_object_tile(case, ty, tx, hit, workers=min(len(hit), U.default_workers()))
    got_tile = got["g_object"][..., ty:ty + 16, tx:tx + 64]
    print(f"{w.name}: object tile ({ty}, {tx}) over windows {list(hit)}", flush=True)
    U.check_array(w.name + " g_object tile", got_tile, ref_tile, 1e-4)
    # gauge identities of the object and probe gradients (every window)
    go = got["g_object"].astype(np.complex128)
    gpr = got["g_probe"].astype(np.complex128)
    L = obj.shape[0]
    worst_phase, worst_scale = 0.0, 0.0
    for l in range(L):
        inner_o = np.vdot(obj[l], go[l])  # <O, G> = sum conj(O) G
        norm_o = float(np.sum(np.abs(obj[l]) * np.abs(go[l])))
        inner_p = sum(np.vdot(prb[l, m], gpr[l, m]) for m in range(prb.shape[1]))
        norm_p = float(np.sum(np.abs(prb[l]) * np.abs(gpr[l])))
        worst_phase = max(worst_phase, abs(inner_o.imag) / norm_o)
        worst_scale = max(worst_scale, abs(inner_o.real - inner_p.real) / (norm_o + norm_p))
    errs = dict(g_pos=e_pos, g_sigma=e_sig, per_position=pp, phase_identity=worst_phase,
                scale_identity=worst_scale)
    print(case["w"].name, errs, flush=True)
    assert e_pos <= 1e-4 and e_sig <= 1e-4 and pp <= 1e-3, errs
    assert worst_phase <= 1e-4 and worst_scale <= 1e-4, errs


def test_large_multiplexed_workload_full_size():
    case = _case("C3", 31)
    ks = [0, 1249, 2499]
    I_gpu, got = _run(case, ks, ws_gb=24)
    _check(case, ks, I_gpu, got)


def test_reflection_workload_full_size():
    case = _case("C5", 51)
    ks = [0, 451, 899]
    I_gpu, got = _run(case, ks, ws_gb=8)
    _check(case, ks, I_gpu, got)


def test_benchmark_workload_exact_ratios_full_size():
    case = _case("C2", 21, exact_ratio=True)
    assert all(isinstance(a, float) for a in case["pads"])
    ks = [0, 199, 399]
    I_gpu, got = _run(case, ks, ws_gb=2)
    _check(case, ks, I_gpu, got)


def test_reflection_workload_exact_ratios_full_size():
    # N = 384, Bluestein length 768, tilt table, 900 positions
    case = _case("C5", 52, exact_ratio=True)
    ks = [0, 450, 899]
    I_gpu, got = _run(case, ks, ws_gb=8)
    _check(case, ks, I_gpu, got)
