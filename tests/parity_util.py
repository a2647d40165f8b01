"""Shared helpers of the GPU parity tests: seeded inputs (from synth), the
FP64 oracle side, and the device side through the C ABI binding."""
from __future__ import annotations

import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import oracle
import synth


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def _oracle_forward_part(args):
    obj, prb, pos, pads, sigma, bg, table = args
    return oracle.forward(obj, prb, pos, pads, sigma=sigma, background=bg, resample_table=table)


def oracle_forward(obj, prb, pos, pads, sigma=None, bg=None, table=None, workers=1):
    """oracle.forward, optionally split over position blocks in processes."""
    K = len(pos)
    if workers <= 1 or K < 2 * workers:
        return oracle.forward(obj, prb, pos, pads, sigma=sigma, background=bg, resample_table=table)
    parts = np.array_split(np.arange(K), workers)
    args = [(obj, prb, pos[p], pads, None if sigma is None else sigma[p], bg, table) for p in parts]
    with ProcessPoolExecutor(workers) as ex:
        outs = list(ex.map(_oracle_forward_part, args))
    return np.concatenate(outs, 0)


def _oracle_grad_part(args):
    kw, positions = args
    return oracle.loss_grad(positions=list(positions), **kw)


def oracle_loss_grad(workers=1, **kw):
    """oracle.loss_grad summed over position blocks computed in processes
    (the loss is a sum over positions, so the parts add up exactly)."""
    K = len(kw["pos"])
    if workers <= 1 or K < 2 * workers:
        return oracle.loss_grad(**kw)
    parts = np.array_split(np.arange(K), workers)
    with ProcessPoolExecutor(workers) as ex:
        outs = list(ex.map(_oracle_grad_part, [(kw, p) for p in parts]))
    res = dict(outs[0])
    for o in outs[1:]:
        res["loss"] += o["loss"]
        for key in ("g_object", "g_probe", "g_pos", "g_sigma", "g_background", "g_ratio"):
            res[key] = res[key] + o[key]
    if kw.get("l1") or kw.get("tv"):  # the regulariser belongs to no position
        rv, rg = oracle.regulariser(kw["obj"], kw.get("l1", 0.0), kw.get("tv", 0.0),
                                    kw.get("tv_eps", 1e-3))
        res["loss"] += rv
        res["g_object"] = res["g_object"] + rg
    return res


def default_workers() -> int:
    return max(1, min(16, (os.cpu_count() or 1)))


def make_case(w, K=None, with_sigma=False, with_bg=False, with_mask=False, seed_offset=0,
              workers=1, pads=None):
    """Truth, perturbed start and oracle-simulated counts for workload w
    (``pads`` overrides the per-wavelength DFT sizes on both sides)."""
    if K is not None:
        w = synth.reduced(w, K=K)
    truth = synth.make_truth(w)
    if pads is not None:
        truth["pads"] = tuple(pads)
    start = synth.make_start(truth, w)
    K = w.K
    rng = np.random.default_rng(w.seed + 77 + seed_offset)
    sigma = rng.uniform(0.8, 1.2, K).astype(np.float32) if with_sigma else None
    bg = rng.uniform(0.0, 2.0, (w.N, w.N)).astype(np.float32) if with_bg else None
    mask = truth["mask"]
    if with_mask and mask is None:
        mask = (rng.uniform(size=(w.N, w.N)) > 0.1).astype(np.uint8)
    table = truth["resample"]
    I = oracle_forward(truth["object"], truth["probe"], truth["pos"], truth["pads"],
                       sigma=sigma, bg=bg, table=table, workers=workers)
    meas = synth.sample_counts(I, w.seed + seed_offset)
    # the model and the GPU both consume the float32 / complex64 inputs
    obj = start["object"]  # [L][Ns][H][W]; one sample mode is passed as [L][H][W]
    obj = (obj[:, 0] if obj.shape[1] == 1 else obj).astype(np.complex64)
    prb = start["probe"].astype(np.complex64)
    return dict(w=w, obj=obj, prb=prb, pos=start["pos"].copy(), pads=tuple(truth["pads"]),
                meas=meas, sigma=sigma, bg=bg, mask=mask, table=table, truth=truth)


def oracle_grads(case, kind=0, eps=1e-6, scale=1.0, workers=1, **extra):
    """``extra``: noise_var, l1, tv, tv_eps of oracle.loss_grad."""
    return oracle_loss_grad(
        workers=workers, obj=case["obj"].astype(np.complex128), probe=case["prb"].astype(np.complex128),
        pos=case["pos"], pads=case["pads"], measured=case["meas"], kind=kind, eps=eps,
        scale=scale, sigma=case["sigma"], background=case["bg"], mask=case["mask"],
        resample_table=case["table"], **extra)


def to_problem(case, device):
    import torch
    from paper_2311_14780_amd import binding as B
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(device)
    res = None
    if case["table"] is not None:
        res = B.resample_tables(case["table"][0], case["table"][1], device)
    return B.Problem(object=t(case["obj"]), probe=t(case["prb"]), pos=t(case["pos"]),
                     pads=case["pads"], measured=t(case["meas"]), sigma=t(case["sigma"]),
                     background=t(case["bg"]), mask=t(case["mask"]), resample=res)


def gpu_grads(prob, kind=0, eps=1e-6, scale=1.0, chunk=0,
              want=("object", "probe", "pos", "sigma", "background"), stream=None, **reg):
    import torch
    from paper_2311_14780_amd import binding as B
    dev = prob.object.device
    g = dict(loss=torch.zeros(1, device=dev))
    if "object" in want:
        g["g_object"] = torch.zeros_like(prob.object)
    if "probe" in want:
        g["g_probe"] = torch.zeros_like(prob.probe)
    if "pos" in want:
        g["g_pos"] = torch.zeros(prob.K, 2, device=dev)
    if "sigma" in want:
        g["g_sigma"] = torch.zeros(prob.K, device=dev)
    if "background" in want:
        g["g_background"] = torch.zeros(prob.N, prob.N, device=dev)
    if "ratio" in want:
        g["g_ratio"] = torch.zeros(prob.L, device=dev)
    ws = B.workspace([prob], 1, chunk)
    B.ptycho_loss_grad([prob], [g], kind=kind, eps=eps, scale=scale, workspace=ws, stream=stream,
                       **reg)
    torch.cuda.synchronize()
    out = {k: v.cpu().numpy() for k, v in g.items()}
    out["loss"] = float(out["loss"][0])
    out["_ws"] = ws
    return out


def gpu_forward(prob, chunk=0):
    import torch
    from paper_2311_14780_amd import binding as B
    out = torch.empty(prob.K, prob.N, prob.N, device=prob.object.device)
    ws = B.workspace([prob], 0, chunk)
    B.ptycho_forward([prob], [out], ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def compare(got, ref, tol_grad=1e-4, tol_loss=1e-5,
            keys=("g_object", "g_probe", "g_pos", "g_sigma", "g_background", "g_ratio")):
    """Relative L2 errors per output; raises with all of them on failure."""
    errs = {"loss": abs(got["loss"] - ref["loss"]) / max(abs(ref["loss"]), 1e-30)}
    for k in keys:
        if k in got:
            r = ref[k]
            if k == "g_object" and r.ndim == 4 and np.asarray(got[k]).ndim == 3:
                r = r[:, 0]
            errs[k] = rel_l2(got[k], r)
    bad = {k: v for k, v in errs.items() if v > (tol_loss if k == "loss" else tol_grad)}
    assert not bad, f"parity failed: {errs}"
    return errs
