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


def max_rel(a, b) -> float:
    """Element-wise bound: max |a - b| / max |b| (one localised error -- a
    wrong crop edge row, a Nyquist-bin slip, a dim-pixel error -- shows here
    even where the relative L2 norm of the whole array hides it)."""
    a = np.asarray(a)
    b = np.asarray(b)
    mb = float(np.max(np.abs(b))) if b.size else 0.0
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0)) if b.size else 0.0


# Floor of the per-position bound, as a fraction of the rms over positions:
# a position whose derivative is a near-cancelling sum of N^2 terms carries
# the FP32 error of those terms, not of the (small) result.
PER_POSITION_FLOOR = 0.1


def per_position_rel(a, b) -> float:
    """Per-position bound for [K] / [K][2] arrays (position and power
    gradients): max_k |a_k - b_k| / max(|b_k|, floor * rms_k |b_k|)."""
    a = np.asarray(a, np.float64).reshape(len(b), -1)
    b = np.asarray(b, np.float64).reshape(len(b), -1)
    if b.size == 0:
        return 0.0
    rms = float(np.sqrt(np.mean(b * b)))
    den = np.maximum(np.abs(b), PER_POSITION_FLOOR * rms)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(a - b) / den))


def check_array(name, got, ref, tol, log=None) -> dict:
    """Relative L2 and element-wise (max-abs / max-ref) bounds of one array,
    both at ``tol``; printed, and returned as a dict."""
    e = {"rel_l2": rel_l2(got, ref), "max_rel": max_rel(got, ref)}
    print(f"PARITY {name}: rel_l2 {e['rel_l2']:.3e} max_abs/max_ref {e['max_rel']:.3e} (tol {tol:g})",
          flush=True)
    if log is not None:
        log[name] = e
    assert e["rel_l2"] <= tol and e["max_rel"] <= tol, f"{name}: {e} above {tol}"
    return e


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


PER_POSITION_KEYS = ("g_pos", "g_sigma")


def compare(got, ref, tol_grad=1e-4, tol_loss=1e-5,
            keys=("g_object", "g_probe", "g_pos", "g_sigma", "g_background", "g_ratio"),
            tol_pp=None):
    """Every output against the oracle, three bounds per gradient array:
    relative L2 <= tol_grad, max|got - ref| <= tol_grad * max|ref|, and for
    the per-position arrays (g_pos, g_sigma) max_k |d_k| / max(|ref_k|,
    0.1 rms) <= tol_pp (default 10 tol_grad).  The loss is bounded
    relatively by tol_loss.  Prints every figure; raises with all of them
    on failure."""
    tol_pp = 10.0 * tol_grad if tol_pp is None else tol_pp
    assert np.isfinite(ref["loss"]) and np.isfinite(got["loss"]), (got["loss"], ref["loss"])
    errs = {"loss": abs(got["loss"] - ref["loss"]) / max(abs(ref["loss"]), 1e-30)}
    bad = {}
    if errs["loss"] > tol_loss:
        bad["loss"] = errs["loss"]
    for k in keys:
        if k in got:
            r = ref[k]
            if k == "g_object" and r.ndim == 4 and np.asarray(got[k]).ndim == 3:
                r = r[:, 0]
            g = np.asarray(got[k])
            errs[k] = rel_l2(g, r)
            errs[k + ":max"] = max_rel(g, r)
            if errs[k] > tol_grad:
                bad[k] = errs[k]
            if errs[k + ":max"] > tol_grad:
                bad[k + ":max"] = errs[k + ":max"]
            if k in PER_POSITION_KEYS:
                errs[k + ":pp"] = per_position_rel(g, r)
                if errs[k + ":pp"] > tol_pp:
                    bad[k + ":pp"] = errs[k + ":pp"]
    print("PARITY " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    assert not bad, f"parity failed: {bad} (all: {errs})"
    return errs


def sparse_object_tile(pos, N, H, W, th=16, tw=64, lo=3, hi=6):
    """A th x tw tile of the object that between lo and hi windows overlap
    (the most such windows; ties: the first tile in raster order), and the
    ascending indices of those windows.  At full size the oracle cannot
    sum every window, but the object gradient on such a tile depends on
    these windows only."""
    p, _ = oracle.split_positions(pos)
    best = None
    for ty in range(0, H - th + 1, th):
        for tx in range(0, W - tw + 1, tw):
            hit = np.flatnonzero(~((p[:, 0] >= ty + th) | (p[:, 0] + N <= ty) |
                                   (p[:, 1] >= tx + tw) | (p[:, 1] + N <= tx)))
            if lo <= len(hit) <= hi and (best is None or len(hit) > len(best[2])):
                best = (ty, tx, hit)
    assert best is not None, "no tile with the requested overlap"
    return best


def _tile_part(args):
    kw, positions = args
    return oracle.loss_grad(positions=list(positions), **kw)["g_object"]


def oracle_object_tile(case, ty, tx, hit, th=16, tw=64, kind=0, eps=1e-6, scale=1.0,
                       workers=1):
    """Oracle object gradient on the tile [ty, ty+th) x [tx, tx+tw) of every
    slot, summed over the windows ``hit`` (those that overlap it).  The
    object is cropped to the windows' bounding box and the positions are
    shifted by the integer corner of the crop: a float32 position minus an
    integer is exact, so the windows, sub-pixel shifts and the arithmetic
    are those of the full-size problem."""
    p, _ = oracle.split_positions(case["pos"])
    N = case["w"].N
    # the crop holds the windows and the tile (part of which no window covers)
    y0, x0 = min(int(p[hit, 0].min()), ty), min(int(p[hit, 1].min()), tx)
    y1, x1 = max(int(p[hit, 0].max()) + N, ty + th), max(int(p[hit, 1].max()) + N, tx + tw)
    obj = np.asarray(case["obj"])
    crop = obj[..., y0:y1, x0:x1].astype(np.complex128)
    pos = (case["pos"][hit] - np.array([y0, x0], np.float32)).astype(np.float32)
    assert np.array_equal(oracle.split_positions(pos)[0] + np.array([y0, x0]), p[hit])
    sig = None if case["sigma"] is None else case["sigma"][hit]
    kw = dict(obj=crop, probe=case["prb"].astype(np.complex128), pos=pos, pads=case["pads"],
              measured=case["meas"][hit], kind=kind, eps=eps, scale=scale, sigma=sig,
              background=case["bg"], mask=case["mask"], resample_table=case["table"])
    K = len(hit)
    if workers <= 1 or K < 2:
        g = oracle.loss_grad(**kw)["g_object"]
    else:
        parts = np.array_split(np.arange(K), min(workers, K))
        with ProcessPoolExecutor(len(parts)) as ex:
            g = sum(ex.map(_tile_part, [(kw, q) for q in parts]))
    return g[..., ty - y0:ty - y0 + th, tx - x0:tx - x0 + tw]
