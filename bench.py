#!/usr/bin/env python3
"""Throughput of the ptychography loss + gradient iteration on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload C3] [--extra C2]

One step is one pass of the whole hot path over the workload: positions ->
object patches -> sub-pixel Fourier shift -> probe modes -> per-wavelength
padded DFT -> incoherent sum -> loss -> hand-written adjoint -> object,
probe, position and power-coefficient gradients -> Adam update of object,
probe and positions (``ptycho_step``).  All inputs are seeded synthetic data
resident in HBM before the timed region starts; the measured patterns are
Poisson draws from the model's own forward pass of the ground truth.

Prints one JSON line.  The headline workload is the largest single-GPU
configuration (C3: 5 wavelengths x 8 probe modes, 512 x 512 probe, 3072 x 3072
object per wavelength, 2500 positions); ``extra`` holds the same figures for
the four-wavelength 256 x 256 workload (C2), the reflection workload with the
tilt table (C5) and the single-wavelength 64 x 64 case (C1, whose
``ms_per_step`` is the latency of one loss + gradient + Adam step).  ``value`` is pattern-modes per
second (one pattern-mode is one (position, wavelength, probe mode)
propagation, forward and adjoint).
``roofline`` reports the kernel class with the largest GPU time: algorithmic
HBM bytes per launch / average launch duration (HIP events on the launch
stream, over the timed region) against the 8 TB/s HBM3E peak.
``roofline.traffic`` is the measured HBM traffic per launch of that kernel
(rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by a plain-copy
calibration; committed under profiles/), reported only while the kernel
sources are the ones that were measured, else null.  ``roofline.valu_issue_frac``
is the same kernel's VALU issue rate against the chip's (SQ_INSTS_VALU per
launch from a committed counter pass / launch duration, against 1024 SIMDs x
clock / 4 cycles per wave64 instruction), under the same source condition.
``cpu_baseline`` times the FP64 oracle on a bounded sample of positions.
``serving`` runs a reduced serving stream (continuous batching against
first-come first-served sequential execution); ``--serving-jobs 64
--serving-iters 50`` is the full stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pattern-modes/s for loss+gradient iteration (%HBM roofline); serving p50/p99"


def alg_bytes(kernel: str, K: int, L: int, M: int, N: int, H: int, W: int) -> float:
    """Algorithmic HBM bytes of one step attributed to a kernel class.

    Per (position, wavelength): object gather 8N^2, object-gradient
    contribution 8N^2, forward shift transpose 16N^2 (write + read), adjoint
    shift transpose 16N^2; per (position, wavelength, mode): column-pass
    output written and read 16N^2, detector-pass output written and read
    16N^2; per position: measured pattern 4N^2; state: probe and object read
    plus gradient write 16 L (M N^2 + H W); Adam: 28 bytes per real
    coordinate of object, probe and positions.
    """
    n2 = float(N) * N
    kl, klm = K * L, K * L * M
    table = {
        "row_fwd": kl * 16 * n2,                               # gather + X write
        "col_fwd": kl * 8 * n2 + klm * 8 * n2 + L * M * 8 * n2,  # X read + Y write + probe read
        "det": klm * 16 * n2 + K * 4 * n2,                     # Y read + Z write + measured
        "col_adj": klm * 8 * n2 + kl * 8 * n2 + L * M * 8 * n2,  # Z read + GX write + probe read
        "row_adj": kl * 8 * n2,                                # GX read
        "obj_gather": kl * 8 * n2 + L * 16.0 * H * W,          # contribution + object r/w
        "probe_reduce": L * M * 8 * n2,                        # probe gradient write
        "adam": 28.0 * (2 * L * H * W + 2 * L * M * n2 + 2 * K),
    }
    return table.get(kernel, 0.0)


def step_alg_bytes(K, L, M, N, H, W) -> float:
    return sum(alg_bytes(k, K, L, M, N, H, W) for k in
               ("row_fwd", "col_fwd", "det", "col_adj", "row_adj", "obj_gather", "probe_reduce", "adam"))


def kernel_source_sha256() -> str:
    csrc = os.path.join(ROOT, "paper_2311_14780_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read()
                   for f in ("kernels.hip", "fft.hpp", "kernels.hpp"))
    return hashlib.sha256(src).hexdigest()


def _profile_entry(workload: str, kind: str, kernel: str):
    """Per-launch figures of a kernel class from a committed counter summary
    (profiles/<workload>_step_<kind>.json), if the kernel sources still hash
    to the measured ones; else None."""
    path = os.path.join(ROOT, "profiles", f"{workload}_step_{kind}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if kernel_source_sha256() != d.get("source_sha256"):
        return None
    return d["kernels"].get(kernel)


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE passes), or None."""
    k = _profile_entry(workload, "hbm_traffic", kernel)
    if not k:
        return None
    return float(k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"])


# VALU issue limit: 256 CUs x 4 SIMDs issue one wave64 VALU instruction each
# per 4 cycles (16 lanes per SIMD; packed FP32 is not used).
SIMDS = 1024
CYCLES_PER_WAVE64_VALU = 4


def valu_issue(workload: str, kernel: str, avg_launch_us: float):
    """VALU issue fraction of a kernel class: SQ_INSTS_VALU per launch (a
    committed counter pass) / (1024 SIMDs x clock / 4 x launch duration),
    with the clock measured in the same pass (GRBM_GUI_ACTIVE per XCD over
    the kernel's duration); None without a summary for these sources."""
    k = _profile_entry(workload, "valu_counters", kernel)
    if not k:
        return None
    clk = float(k["clock_hz"])
    peak = SIMDS * clk / CYCLES_PER_WAVE64_VALU  # wave64 VALU instructions per second
    insts = float(k["sq_insts_valu_per_launch"])
    return dict(valu_insts_per_launch=insts, clock_GHz=round(clk / 1e9, 3),
                issue_rate=round(insts / (avg_launch_us * 1e-6), 1), peak_rate=round(peak, 1),
                frac=round(insts / (avg_launch_us * 1e-6) / peak, 4))


def build_inputs(w, device, exact_ratio: bool = False):
    import torch
    import synth
    from paper_2311_14780_amd import binding as B
    truth = synth.make_truth(w)
    if exact_ratio:
        # the exact wavelength ratios (floats) select the exact-ratio propagator
        truth["pads"] = truth["ratios"]
    start = synth.make_start(truth, w)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    res = None
    if truth["resample"] is not None:
        res = B.resample_tables(truth["resample"][0], truth["resample"][1], device)
    mask = None if truth["mask"] is None else t(truth["mask"])
    # simulate the measurement with the model itself on the ground truth
    tprob = B.Problem(object=t(truth["object"][:, 0].astype(np.complex64)),
                      probe=t(truth["probe"].astype(np.complex64)), pos=t(truth["pos"]),
                      pads=truth["pads"], mask=mask, resample=res)
    I = torch.empty(w.K, w.N, w.N, device=device)
    ws = B.workspace([tprob], 0, 64)
    B.ptycho_forward([tprob], [I], ws)
    torch.cuda.synchronize()
    meas = synth.sample_counts(I.cpu().numpy(), w.seed)
    del ws, tprob, I
    prob = B.Problem(object=t(start["object"][:, 0].astype(np.complex64)),
                     probe=t(start["probe"].astype(np.complex64)), pos=t(start["pos"]),
                     pads=start["pads"], measured=t(meas), mask=mask, resample=res)
    return truth, start, prob


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


_POOL_DATA = None


def _pool_init(data):
    """Initializer of the all-cores baseline's workers: the inputs, once."""
    global _POOL_DATA
    _POOL_DATA = data


def _oracle_positions(ks):
    """Worker of the all-cores baseline: loss + gradients of some positions."""
    import oracle
    obj, prb, pos, pads, meas, mask, table = _POOL_DATA
    for k in ks:
        oracle.loss_grad(obj, prb, pos, pads, meas, mask=mask, resample_table=table, positions=[k])
    return len(ks)


def cpu_baseline_pool(w, truth, start, workers: int, per_worker: int = 16,
                      timeout_s: float = 600.0):
    """The same oracle over a pool of processes (one BLAS thread each) on the
    host's cores: ``per_worker`` positions per worker, wall time of the pool.
    The pool is terminated if it has not finished within ``timeout_s``."""
    import oracle
    import synth
    import multiprocessing as mp
    n = workers * per_worker
    obj = start["object"].astype(np.complex64).astype(np.complex128)
    prb = start["probe"].astype(np.complex64).astype(np.complex128)
    I = oracle.forward(truth["object"], truth["probe"], truth["pos"][:n], truth["pads"],
                       resample_table=truth["resample"])
    meas = synth.sample_counts(I, w.seed)
    common = (obj, prb, start["pos"][:n], start["pads"], meas, truth["mask"], truth["resample"])
    parts = [list(range(i, n, workers)) for i in range(workers)]
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"  # inherited by the workers
    pool = mp.get_context("spawn").Pool(workers, initializer=_pool_init, initargs=(common,))
    try:
        pool.map_async(_oracle_positions, [[0]] * workers, chunksize=1).get(timeout_s)  # warm-up
        t0 = time.perf_counter()
        done = sum(pool.map_async(_oracle_positions, parts, chunksize=1).get(timeout_s))
        elapsed = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
    pm = done * w.L * w.M * w.Ns
    return dict(value=pm / elapsed, unit="pattern-modes/s", cores=workers, kind="oracle",
                sample=(f"{done} of {w.K} positions of {w.name}, {workers} processes of one "
                        f"thread, {elapsed:.1f} s wall; {cpu_model()}"))


def graph_timing(B, prob, g, ws, steps: int, warmup: int) -> dict:
    """Loss + gradient call (no Adam: a captured step would replay its Adam
    step number) eager and replayed from a captured HIP graph, ms per call."""
    import torch
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    call = lambda: B.ptycho_loss_grad([prob], [g], kind=B.LOSS_AMPLITUDE, eps=1e-6, scale=1.0,
                                      workspace=ws, stream=s)
    with torch.cuda.stream(s):
        for _ in range(max(warmup, 1)):
            call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(s):
        for _ in range(steps):
            call()
    torch.cuda.synchronize()
    eager = (time.perf_counter() - t0) * 1e3 / steps
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        call()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    replay = (time.perf_counter() - t0) * 1e3 / steps
    del graph
    return {"eager_ms_per_call": round(eager, 4), "graph_ms_per_call": round(replay, 4),
            "note": "loss + gradient call, eager vs replayed from one captured graph"}


def copy_bandwidth(mib: int = 1024, reps: int = 5) -> float:
    """Measured device-to-device copy bandwidth (GB/s, read + write bytes)."""
    import torch
    a = torch.empty(mib * 2**18, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2.0 * mib * 2**20 / sec / 1e9


def cpu_baseline(w, truth, start, budget_s: float = 20.0, max_positions: int = 256):
    """FP64 oracle loss + gradient of the workload's first positions, one
    position at a time until the time budget is spent (at least two).  Each
    position's measured pattern is drawn from the oracle's forward model of
    the truth before its timed call; only the loss + gradient is timed."""
    import oracle
    import synth
    obj = start["object"].astype(np.complex64).astype(np.complex128)
    prb = start["probe"].astype(np.complex64).astype(np.complex128)
    exact = any(oracle.is_ratio(p) for p in start["pads"])
    elapsed, done = 0.0, 0
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):  # one core: the matrix products of the exact ratio too
        while done < min(max_positions, w.K) and (elapsed < budget_s or done < 2):
            k = done
            I = oracle.forward(truth["object"], truth["probe"], truth["pos"][k:k + 1],
                               truth["pads"], resample_table=truth["resample"])
            meas = synth.sample_counts(I, w.seed + k)
            t0 = time.perf_counter()
            oracle.loss_grad(obj, prb, start["pos"][k:k + 1], start["pads"], meas,
                             mask=truth["mask"], resample_table=truth["resample"])
            elapsed += time.perf_counter() - t0
            done += 1
    pm = done * w.L * w.M * w.Ns
    prop = ("exact-ratio scaled DFT as matrix products" if exact
            else "zero-padded DFT by pocketfft")
    return dict(value=pm / elapsed, unit="pattern-modes/s", cores=1, kind="oracle",
                sample=(f"{done} of {w.K} positions of {w.name} at full N/L/M "
                        f"({pm} pattern-modes), amplitude loss + object/probe/position/sigma "
                        f"gradients, FP64 NumPy ({prop}), one thread, {elapsed:.1f} s; host has "
                        f"{os.cpu_count()} logical CPUs, {cpu_model()}"))


def copy_calibration(mib: int) -> int:
    """Three plain device-to-device copies of ``mib`` MiB: each reads and
    writes exactly ``mib`` MiB, which fixes the scale of the HBM byte
    counters for the kernels of a step."""
    import torch
    a = torch.ones(mib * 2**18, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "copies": 3}), flush=True)
    return 0


def time_workload(B, w, dev, args, czt: bool, label: str, plain: bool = False) -> dict:
    """Times ``args.steps`` fused steps (loss + gradients + Adam) of workload
    ``w`` after ``args.warmup`` warm-up steps; returns the figures of the
    JSON line (value, ms per step, step and dominant-kernel rooflines,
    per-class kernel times) and the inputs (for the CPU baseline).  With
    ``plain`` the step time comes from a second timed loop without any
    profiling event (small workloads, whose steps the events would lengthen
    noticeably); the kernel figures still come from the bracketed loop."""
    import torch
    print(f"[{label}] building inputs of {w.name}", file=sys.stderr, flush=True)
    truth, start, prob = build_inputs(w, dev, exact_ratio=czt)
    K, L, M, N, H, W = w.K, w.L, w.M, w.N, w.H, w.W
    g = dict(loss=torch.zeros(1, device=dev), g_object=torch.zeros_like(prob.object),
             g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(K, 2, device=dev),
             g_sigma=torch.zeros(K, device=dev))
    zeros = lambda x: torch.zeros(x.numel() * (2 if x.is_complex() else 1), device=dev)
    adam = dict(m_object=zeros(prob.object), v_object=zeros(prob.object),
                m_probe=zeros(prob.probe), v_probe=zeros(prob.probe),
                m_pos=zeros(prob.pos), v_pos=zeros(prob.pos),
                lr_object=1e-3, lr_probe=1e-3, lr_pos=5e-3, t=0)
    ws = B.workspace([prob], 2)
    stream = torch.cuda.current_stream()

    def step():
        adam["t"] += 1
        B.ptycho_step([prob], [g], [adam], kind=B.LOSS_AMPLITUDE, eps=1e-6, scale=1.0,
                      workspace=ws, stream=stream)

    # Kernel timing: with two or more warm-up steps, every launch of the
    # warm-up steps after the first is bracketed with HIP events (the
    # per-class breakdown), and in the timed region only the launches of the
    # class with the most time, whose figures the roofline object reports.
    # With fewer warm-up steps every launch of the timed region is bracketed.
    timing = not args.no_kernel_timing
    split = timing and args.warmup >= 2
    kern_warm, n_warm = {}, 0
    print(f"[{label}] {args.warmup} warm-up steps", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        if split and i == 1:
            torch.cuda.synchronize()
            B.ptycho_profile(True)
        step()
    torch.cuda.synchronize()
    if split:
        kern_warm, n_warm = B.ptycho_profile_read(), args.warmup - 1
        B.ptycho_profile(False)
    # the dominant class among the hot-path kernels (those with algorithmic
    # bytes), not the bookkeeping launches (tables, status, zeroing)
    hot = [k for k in kern_warm if alg_bytes(k, 1, 1, 1, 1, 1, 1) > 0]
    dom_warm = max(hot, key=lambda k: kern_warm[k][0]) if hot else None
    if timing:
        B.ptycho_profile(True)
        if dom_warm is not None:
            B.ptycho_profile_classes([dom_warm])
    print(f"[{label}] {args.steps} timed steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {}
    if timing:
        kern = B.ptycho_profile_read()
        B.ptycho_profile(False)
    if plain and timing:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    status = B.ptycho_status(ws, 0)
    if status != 0:
        raise RuntimeError(f"device status {status}: a window left the object")
    ms = (t1 - t0) * 1e3 / args.steps
    pm = K * L * M * w.Ns
    value = pm / (ms * 1e-3)
    b_step = step_alg_bytes(K, L, M, N, H, W)

    roof = None
    kern_out = {}
    if kern:
        # per-class figures: the timed region's where it bracketed the class,
        # else those of the profiled warm-up steps
        for src, nsteps in ((kern_warm, n_warm), (kern, args.steps)):
            for name, (tot, n) in src.items():
                if n:
                    kern_out[name] = dict(ms_per_step=tot / nsteps, launches_per_step=n / nsteps,
                                          avg_launch_us=1e3 * tot / n,
                                          timed_region=src is kern)
        hot_out = [k for k in kern_out if alg_bytes(k, 1, 1, 1, 1, 1, 1) > 0] or list(kern_out)
        dom = dom_warm or max(hot_out, key=lambda k: kern_out[k]["ms_per_step"])
        d = kern_out[dom]
        per_launch = alg_bytes(dom, K, L, M, N, H, W) / d["launches_per_step"]
        achieved = per_launch / (d["avg_launch_us"] * 1e-6) / 1e9
        traffic = None if czt else measured_traffic(w.name, dom)
        roof = dict(kernel=dom, bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=None if traffic is None else round(traffic / 1e9, 4),
                    traffic_unit="GB per launch",
                    alg_bytes_per_launch=per_launch, avg_launch_us=round(d["avg_launch_us"], 2))
        vi = None if czt else valu_issue(w.name, dom, d["avg_launch_us"])
        roof["valu_issue_frac"] = None if vi is None else vi["frac"]
        roof["valu_issue"] = vi
        for name, d in kern_out.items():
            b = alg_bytes(name, K, L, M, N, H, W)
            if b:
                d["alg_GBps"] = round(b / (d["ms_per_step"] * 1e-3) / 1e9, 1)
            if not czt:
                v = valu_issue(w.name, name, d["avg_launch_us"])
                if v is not None:
                    d["valu_issue_frac"] = v["frac"]
    graph = None
    if args.graph:
        graph = graph_timing(B, prob, g, ws, args.steps, args.warmup)
    pads = [round(p, 4) if isinstance(p, float) else int(p) for p in prob.pads]
    prop = ("exact-ratio propagator (scaled DFT by Bluestein's method, FFT length 2N), ratios "
            if czt else "zero-padded DFT, pads ")
    del g, adam, ws, prob
    torch.cuda.empty_cache()
    print(f"[{label}] {w.name}: {ms:.3f} ms per step", file=sys.stderr, flush=True)
    return dict(
        value=round(value, 1), ms_per_step=round(ms, 4),
        config={"workload": (f"{w.name}: {L} wavelengths (harmonics {'/'.join(map(str, w.harmonics))}) "
                             f"x {M} probe modes, probe {N}x{N}, object {H}x{W} per wavelength, "
                             f"{K} positions ({w.scan}), {prop}{'/'.join(map(str, pads))}, "
                             f"{w.photons:.0e} photons/pattern; step = loss + gradients + Adam"),
                "K": K, "L": L, "M": M, "N": N, "H": H, "W": W, "pads": pads,
                "propagator": "exact-ratio" if czt else "zero-padded DFT",
                "parallelism": "single GPU"},
        step_roofline={"alg_bytes_per_step": b_step,
                       "achieved_GBps": round(b_step / (ms * 1e-3) / 1e9, 1),
                       "frac": round(b_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        roofline=roof, graph=graph, kernels=kern_out,
        kernel_timing=(None if not timing else
                       "HIP events around the dominant class's launches in the timed region; "
                       "other classes from the bracketed warm-up steps" if split else
                       "HIP events around every launch of the timed region"),
        _truth=truth, _start=start)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C3",
                    help="workload of the headline line (default C3, the largest "
                         "single-GPU configuration)")
    ap.add_argument("--extra", default="C2,C5,C1",
                    help="comma-separated workloads also timed and reported under 'extra' "
                         "(default C2, C5 and C1, whose ms_per_step is the latency of the "
                         "small single-wavelength case; empty for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-jobs", type=int, default=16)
    ap.add_argument("--serving-iters", type=int, default=5)
    ap.add_argument("--propagator", choices=("pad", "czt"), default="pad",
                    help="pad: zero-padded DFT at the smooth pad sizes; czt: exact-ratio "
                         "propagator (scaled DFT by Bluestein's method)")
    ap.add_argument("--graph", action="store_true",
                    help="also time the loss + gradient call replayed from a captured HIP graph "
                         "(launch overhead of small workloads); reported as graph_ms_per_call")
    ap.add_argument("--cpu-pool", type=int, default=0, metavar="WORKERS",
                    help="only time the oracle over a pool of WORKERS processes on the host "
                         "(no GPU use) and print it as one JSON line")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three plain device copies of MIB MiB (the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args(argv)
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.cpu_pool:
        import synth
        w = synth.get_workload(args.workload)
        truth = synth.make_truth(w)
        if args.propagator == "czt":
            truth["pads"] = truth["ratios"]
        start = synth.make_start(truth, w)
        print(json.dumps({"cpu_baseline_pool": cpu_baseline_pool(w, truth, start, args.cpu_pool),
                          "workload": w.name, "propagator": args.propagator}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU position-sharded design is not built)", file=sys.stderr)
        return 2

    import torch
    import synth
    from paper_2311_14780_amd import binding as B

    dev = torch.device("cuda:0")
    czt = args.propagator == "czt"
    w = synth.get_workload(args.workload)
    main_run = time_workload(B, w, dev, args, czt, "main")
    truth, start = main_run.pop("_truth"), main_run.pop("_start")
    cpu = None
    if not args.no_cpu_baseline:
        print("[main] CPU baseline (oracle, one thread)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, truth, start)
    del truth, start
    extra = {}
    for name in [x for x in args.extra.split(",") if x and x != args.workload]:
        r = time_workload(B, synth.get_workload(name), dev, args, czt, "extra", plain=True)
        r.pop("_truth"), r.pop("_start")
        extra[name] = r
    copy_gbps = copy_bandwidth()
    serving = None
    if not args.no_serving:
        from paper_2311_14780_amd import serving as S
        torch.cuda.empty_cache()
        serving = S.run_stream(args.serving_jobs, args.serving_iters,
                               log=lambda m: print(m, file=sys.stderr, flush=True))
    out = {
        "metric": METRIC, "value": main_run["value"], "unit": "pattern-modes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": main_run["config"],
        "step_roofline": main_run["step_roofline"],
        "roofline": main_run["roofline"],
        "cpu_baseline": cpu,
        "graph": main_run["graph"],
        "context": {"device_copy_GBps": round(copy_gbps, 1),
                    "note": "torch device-to-device copy of 1 GiB, read + write bytes"},
        "extra": extra or None,
        "serving": serving,
        "kernels": main_run["kernels"],
        "kernel_timing": main_run["kernel_timing"],
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
