"""Continuous-batching serving loop for ptychographic reconstruction jobs.

A job is one reconstruction: a scan of K positions at L wavelengths with M
probe modes and an N x N probe window, and a number of Adam iterations of
the loss + gradient (ptycho_step).  Its object, probe, position and Adam
state stay in device memory from admission to completion.

Scheduling (``Scheduler.run``):

* Requests arrive over time (``JobRequest.arrival``, seconds after the start
  of the run).  Waiting requests are admitted strictly in arrival order
  while the sum of the device footprints of the admitted jobs stays within
  the budget; a request that could never fit is rejected.
* Every tick runs ONE iteration of every admitted job in a single fused
  ``ptycho_step`` call: the library groups the jobs by window size, and the
  patterns of all jobs in a group share the same batched FFT launches.
* A job leaves as soon as its iterations are done (or its loss stops being
  finite, or it is cancelled), and the memory it frees admits the next
  arrivals at the following tick.  New work thus joins the device while
  other jobs are mid-flight: continuous batching, not a queue.

``mode="sequential"`` is the baseline: first-come first-served, one job at
a time, each job running all its iterations alone.

The scheduler talks to an executor (``TorchExecutor`` on the GPU; tests use
a fake) and to a clock, so its policy is testable without a GPU.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Optional, Sequence

import numpy as np


@dataclass
class JobRequest:
    job_id: int
    arrival: float            # seconds after the start of the run
    iters: int                # Adam iterations to run
    K: int
    L: int
    M: int
    N: int
    H: int
    W: int
    pads: tuple
    payload: object = None    # executor-specific job data (host arrays)
    lr: tuple = (1e-3, 1e-3, 5e-3)  # object, probe, positions

    @property
    def pattern_modes(self) -> int:
        return self.K * self.L * self.M

    @property
    def work(self) -> int:
        """Pattern-pixels per iteration, K L M N^2: the unit of the tick cap."""
        return self.K * self.L * self.M * self.N * self.N


@dataclass
class JobRecord:
    job_id: int
    arrival: float
    status: str = "waiting"   # waiting | running | done | failed | cancelled | rejected
    admitted_at: float = math.nan
    finished_at: float = math.nan
    iters_done: int = 0
    iter_latency: list = field(default_factory=list)   # device seconds of each iteration's call
    iter_wall: list = field(default_factory=list)      # wall seconds from the previous
                                                       # completion (or admission) to this one
    losses: list = field(default_factory=list)
    reason: str = ""


@dataclass
class ServeReport:
    mode: str
    records: dict             # job_id -> JobRecord
    makespan: float           # first arrival to last completion (s)
    pattern_modes: int        # sum over completed iterations of K L M
    ticks: int
    max_active: int           # most jobs resident at once
    peak_bytes: int
    max_fused: int = 0        # most jobs in one fused call

    def _lat(self):
        return np.array([x for r in self.records.values() for x in r.iter_latency])

    def _wall(self, first: bool = True):
        return np.array([x for r in self.records.values() for x in r.iter_wall[0 if first else 1:]])

    def summary(self) -> dict:
        it = self._lat()
        wall = self._wall()
        gap = self._wall(first=False)  # between consecutive iterations only
        done = [r for r in self.records.values() if r.status == "done"]
        jl = np.array([r.finished_at - r.arrival for r in done])
        q = lambda a, p: float(np.percentile(a, p)) if a.size else math.nan
        return {
            "mode": self.mode,
            "jobs_done": len(done),
            "jobs_failed": sum(r.status == "failed" for r in self.records.values()),
            "jobs_rejected": sum(r.status == "rejected" for r in self.records.values()),
            "makespan_s": round(self.makespan, 4),
            "pattern_modes_per_s": round(self.pattern_modes / self.makespan, 1)
            if self.makespan > 0 else math.nan,
            "iter_latency_p50_ms": round(1e3 * q(it, 50), 3),
            "iter_latency_p99_ms": round(1e3 * q(it, 99), 3),
            "iter_wall_p50_ms": round(1e3 * q(wall, 50), 3),
            "iter_wall_p99_ms": round(1e3 * q(wall, 99), 3),
            "iter_gap_p50_ms": round(1e3 * q(gap, 50), 3),
            "iter_gap_p99_ms": round(1e3 * q(gap, 99), 3),
            "job_latency_p50_s": round(q(jl, 50), 4),
            "job_latency_p99_s": round(q(jl, 99), 4),
            "ticks": self.ticks,
            "max_resident_jobs": self.max_active,
            "max_fused_jobs": self.max_fused,
            "peak_state_bytes": int(self.peak_bytes),
        }


class Executor:
    """Interface between the scheduler and the device.

    ``launch`` enqueues one fused iteration and returns a ticket at once;
    ``collect`` waits for it and returns (losses, seconds of device time).
    An executor that only implements the blocking ``step`` gets both for
    free (the work then runs inside ``launch``)."""

    def footprint(self, req: JobRequest) -> int:
        """Device bytes held by the job while admitted."""
        raise NotImplementedError

    def fits(self, reqs: Sequence[JobRequest]) -> bool:
        """Whether these jobs can run together in one fused call."""
        return True

    def admit(self, req: JobRequest):
        """Start making the job resident; returns a handle."""
        raise NotImplementedError

    def ready(self, handle) -> bool:
        """Whether the job's data has reached the device."""
        return True

    def wait(self, handles: Sequence) -> None:
        """Block until at least one of these jobs is ready."""

    def step(self, handles: Sequence) -> list:
        """One fused iteration of every job, blocking; returns the losses."""
        raise NotImplementedError

    def launch(self, handles: Sequence):
        t0 = time.perf_counter()
        losses = self.step(handles)
        return losses, time.perf_counter() - t0

    def collect(self, ticket):
        return ticket

    def release(self, handle) -> None:
        raise NotImplementedError


POLICIES = ("hybrid", "srpt", "fifo")


class Scheduler:
    """Continuous batching over an executor.

    Each tick fuses the ready admitted jobs chosen by ``policy``:

    * ``"hybrid"`` (default): the job that arrived first always runs, and
      the others fill up to ``tick_cap`` pattern-pixels of extra work,
      shortest remaining work first.  The oldest job thus progresses as
      under first-come first-served while short jobs ride along.  With
      ``work_ratio`` set, a job rides along only if its work per iteration
      is within that factor of the oldest job's, and the extra work of a
      call is at most the oldest job's own: a call then takes at most about
      twice the time of each of its jobs alone, so no job's iteration waits
      for a much larger one (the iteration-latency bound), while the others
      keep their arrival order for the next calls.
    * ``"srpt"``: shortest remaining work first, ``tick_cap`` in total.
    * ``"fifo"``: arrival order, ``tick_cap`` in total.

    Up to ``depth`` ticks are in flight: the next fused call is enqueued
    before the losses of the previous one are read, so the device does not
    idle while the host books results and admits jobs.  A non-finite loss
    is therefore noticed one tick late; the job is then retired as failed.
    """

    def __init__(self, executor: Executor, budget_bytes: int,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep,
                 on_tick: Optional[Callable[["Scheduler", int], None]] = None,
                 log: Optional[Callable[[str], None]] = None,
                 tick_cap: Optional[int] = None, policy: str = "hybrid", depth: int = 1,
                 work_ratio: Optional[float] = None):
        if policy not in POLICIES:
            raise ValueError(policy)
        if depth < 1:
            raise ValueError("depth must be at least 1")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.tick_cap = tick_cap   # pattern-pixels per fused call (None: no cap)
        if work_ratio is not None and not work_ratio >= 1.0:
            raise ValueError("work_ratio must be at least 1")
        self.work_ratio = work_ratio  # hybrid: riders within this factor of the head's work
        self.policy = policy
        self.depth = depth
        self.clock = clock
        self.sleep = sleep
        self.on_tick = on_tick
        self.log = log
        self._cancel: set = set()

    def cancel(self, job_id: int) -> None:
        """Cancel a waiting or running job (honoured at the next tick)."""
        self._cancel.add(job_id)

    def _select(self, cand, launched):
        cap = self.tick_cap
        rem = lambda r: (r.iters - launched[r.job_id]) * r.work
        if self.policy == "hybrid":
            cand = sorted(cand, key=lambda rh: (rh[0].arrival, rh[0].job_id))
            head, rest = cand[0], sorted(cand[1:], key=lambda rh: (rem(rh[0]), rh[0].arrival))
            sel, extra = [head], 0
            ratio = self.work_ratio
            hw = head[0].work
            if ratio is not None:
                cap = hw if cap is None else min(cap, hw)
            for r, h in rest:
                if ratio is not None and not (hw / ratio <= r.work <= hw * ratio):
                    continue
                if cap is None or extra + r.work <= cap:
                    sel.append((r, h))
                    extra += r.work
            return sel
        if self.policy == "srpt":
            cand = sorted(cand, key=lambda rh: (rem(rh[0]), rh[0].arrival, rh[0].job_id))
        else:
            cand = sorted(cand, key=lambda rh: (rh[0].arrival, rh[0].job_id))
        sel, work = [], 0
        for r, h in cand:
            if sel and cap is not None and work + r.work > cap:
                continue
            sel.append((r, h))
            work += r.work
        return sel

    def run(self, requests: Sequence[JobRequest], mode: str = "batch") -> ServeReport:
        if mode not in ("batch", "sequential"):
            raise ValueError(mode)
        pending = sorted(requests, key=lambda r: (r.arrival, r.job_id))
        recs = {r.job_id: JobRecord(r.job_id, r.arrival) for r in pending}
        foot = {r.job_id: int(self.ex.footprint(r)) for r in pending}
        # admitted jobs: job_id -> [request, handle, launched, in flight, stop status]
        active: dict = {}
        inflight = deque()         # (ticket, job ids)
        last_done: dict = {}       # job_id -> time of its last completed iteration
        used = peak = ticks = max_active = max_fused = pm = 0
        t0 = self.clock()
        now = lambda: self.clock() - t0
        self._cancel = set(self._cancel)

        def settle(jid):
            """Retire a job whose work is over once nothing of it is in flight."""
            nonlocal used
            req, h, launched, nfl, stop = active[jid]
            rec = recs[jid]
            if nfl:
                return
            status = stop or ("done" if rec.iters_done >= req.iters else None)
            if status is None:
                return
            rec.status = status
            if status == "failed":
                rec.reason = "non-finite loss (or a window left the object)"
            rec.finished_at = now()
            self.ex.release(h)
            used -= foot[jid]
            del active[jid]

        while pending or active:
            # cancellations, of waiting and of admitted jobs
            if self._cancel:
                keep = []
                for r in pending:
                    if r.job_id in self._cancel:
                        recs[r.job_id].status = "cancelled"
                        recs[r.job_id].finished_at = now()
                    else:
                        keep.append(r)
                pending = keep
                for jid in list(active):
                    if jid in self._cancel and not active[jid][4]:
                        active[jid][4] = "cancelled"
                        settle(jid)
            # admission, strictly in arrival order
            t = now()
            while pending and pending[0].arrival <= t:
                r = pending[0]
                if foot[r.job_id] > self.budget or not self.ex.fits([r]):
                    recs[r.job_id].status = "rejected"
                    recs[r.job_id].reason = "larger than the memory budget"
                    recs[r.job_id].finished_at = t
                    pending.pop(0)
                    continue
                if mode == "sequential" and active:
                    break
                if used + foot[r.job_id] > self.budget:
                    break
                if not self.ex.fits([a[0] for a in active.values()] + [r]):
                    break
                pending.pop(0)
                h = self.ex.admit(r)
                used += foot[r.job_id]
                peak = max(peak, used)
                recs[r.job_id].status = "running"
                recs[r.job_id].admitted_at = now()
                last_done[r.job_id] = recs[r.job_id].admitted_at
                active[r.job_id] = [r, h, 0, 0, None]
            max_active = max(max_active, len(active))
            # enqueue a tick if there is room in the pipeline
            if len(inflight) < self.depth:
                cand = [(a[0], a[1]) for a in active.values()
                        if not a[4] and a[2] < a[0].iters and self.ex.ready(a[1])]
                if cand:
                    sel = self._select(cand, {j: a[2] for j, a in active.items()})
                    ticket = self.ex.launch([h for _, h in sel])
                    for r, _ in sel:
                        active[r.job_id][2] += 1
                        active[r.job_id][3] += 1
                    inflight.append((ticket, [r.job_id for r, _ in sel]))
                    max_fused = max(max_fused, len(sel))
                    continue
            if inflight:
                ticket, jids = inflight.popleft()
                losses, dt = self.ex.collect(ticket)
                # device seconds of each job's call (one figure: a single call)
                dts = list(dt) if isinstance(dt, (list, tuple)) else [dt] * len(jids)
                ticks += 1
                t_done = now()
                for jid, lo, dt in zip(jids, losses, dts):
                    a = active[jid]
                    rec = recs[jid]
                    a[3] -= 1
                    rec.iter_latency.append(dt)
                    rec.iter_wall.append(t_done - last_done[jid])
                    last_done[jid] = t_done
                    rec.losses.append(float(lo))
                    rec.iters_done += 1
                    pm += a[0].pattern_modes
                    if not math.isfinite(lo) and not a[4]:
                        a[4] = "failed"
                for jid in jids:
                    settle(jid)
                if self.log and ticks % 100 == 0:
                    self.log(f"tick {ticks}: t={now():.2f}s active={len(active)} waiting={len(pending)} "
                             f"done={sum(x.status == 'done' for x in recs.values())}")
                if self.on_tick:
                    self.on_tick(self, ticks)
                continue
            if active:
                # nothing to launch and nothing in flight: data still arriving
                self.ex.wait([a[1] for a in active.values()])
                continue
            if pending:
                wait = pending[0].arrival - now()
                if wait > 0:
                    self.sleep(wait)
        ends = [r.finished_at for r in recs.values() if not math.isnan(r.finished_at)]
        starts = [r.arrival for r in recs.values()]
        makespan = (max(ends) - min(starts)) if ends else 0.0
        return ServeReport(mode, recs, makespan, pm, ticks, max_active, peak, max_fused)


# ---------------------------------------------------------------- GPU side

def state_bytes(K: int, L: int, M: int, N: int, H: int, W: int) -> int:
    """Device bytes of one job's resident state: object, probe and positions
    with their gradients and two Adam moments each, the measured patterns
    and the loss scalar."""
    obj = 8 * L * H * W
    prb = 8 * L * M * N * N
    pos = 8 * K
    return 4 * (obj + prb + pos) + 4 * K * N * N + 4


class TorchExecutor(Executor):
    """Runs jobs through the C ABI on one device.

    ``workspace_bytes`` of device memory is allocated once and shared by
    every fused call; the library splits each call into as many position
    chunks as that workspace requires.  A request's payload is a dict of
    host arrays: ``object`` complex64 [L][H][W], ``probe`` complex64
    [L][M][N][N], ``pos`` float32 [K][2], ``measured`` float32 [K][N][N].
    """

    def __init__(self, device, workspace_bytes: int, keep_final: bool = False,
                 fuse_work: Optional[int] = None):
        import torch
        from . import binding as B
        self.torch = torch
        self.B = B
        self.device = torch.device(device)
        # pattern-pixels up to which a tick's jobs share one call (None: all)
        self.fuse_work = fuse_work
        self.ws = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.device)
        # job data is copied in on its own stream while other jobs compute
        self.copy_stream = torch.cuda.Stream(device=self.device)
        self.keep_final = keep_final
        self.final = {}  # job_id -> (object, probe, pos) on release, if keep_final

    def footprint(self, req: JobRequest) -> int:
        return state_bytes(req.K, req.L, req.M, req.N, req.H, req.W)

    def fits(self, reqs) -> bool:
        # the smallest workspace (one position per chunk) must fit
        need = self.B.workspace_bytes_for_shapes(
            [(r.K, r.L, r.M, r.N, r.H, r.W, tuple(r.pads)) for r in reqs], which=2, chunk=1)
        return need <= self.ws.numel()

    def _upload(self, a):
        # Allocated on the copy stream: a block taken from the compute
        # stream's pool could still be read by work in flight there (the
        # ticks are pipelined).  Recorded on the compute stream, so that
        # after release the block is not reused before that stream is done.
        torch = self.torch
        src = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
        with torch.cuda.stream(self.copy_stream):
            dst = torch.empty(src.shape, dtype=src.dtype, device=self.device)
            dst.copy_(src, non_blocking=True)  # asynchronous when src is pinned
        dst.record_stream(torch.cuda.current_stream(self.device))
        return dst

    def admit(self, req: JobRequest):
        torch = self.torch
        d = req.payload
        dev = self.device
        prob = self.B.Problem(object=self._upload(d["object"]), probe=self._upload(d["probe"]),
                              pos=self._upload(d["pos"]), pads=tuple(req.pads),
                              measured=self._upload(d["measured"]))
        ev = torch.cuda.Event()
        ev.record(self.copy_stream)
        z = lambda x: torch.zeros(x.numel() * (2 if x.is_complex() else 1), device=dev)
        g = dict(loss=torch.zeros(1, device=dev), g_object=torch.zeros_like(prob.object),
                 g_probe=torch.zeros_like(prob.probe), g_pos=torch.zeros(req.K, 2, device=dev))
        adam = dict(m_object=z(prob.object), v_object=z(prob.object), m_probe=z(prob.probe),
                    v_probe=z(prob.probe), m_pos=z(prob.pos), v_pos=z(prob.pos),
                    lr_object=req.lr[0], lr_probe=req.lr[1], lr_pos=req.lr[2], t=0)
        return {"req": req, "prob": prob, "g": g, "adam": adam, "ev": ev, "waited": False}

    def ready(self, handle) -> bool:
        return handle["waited"] or handle["ev"].query()

    def wait(self, handles) -> None:
        for h in handles:
            if not self.ready(h):
                h["ev"].synchronize()
                return

    def calls_of(self, handles) -> list:
        """The tick's jobs split into calls: consecutive jobs share a call
        while its work stays within ``fuse_work`` pattern-pixels; a larger
        job gets a call of its own."""
        return split_calls([h["req"].work for h in handles], self.fuse_work)

    def launch(self, handles):
        torch = self.torch
        main = torch.cuda.current_stream(self.device)
        for h in handles:
            if not h["waited"]:
                main.wait_event(h["ev"])  # the job's data is in place
                h["waited"] = True
            h["adam"]["t"] += 1
        timed = []  # (start, end, number of jobs) per call, in job order
        for idx in self.calls_of(handles):
            hs = [handles[i] for i in idx]
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(main)
            self.B.ptycho_step([h["prob"] for h in hs], [h["g"] for h in hs],
                               [h["adam"] for h in hs], workspace=self.ws, stream=main)
            end.record(main)
            timed.append((start, end, len(hs)))
        # snapshot of this iteration's losses (the next call overwrites them)
        snap = torch.cat([h["g"]["loss"] for h in handles])
        host = torch.empty(len(handles), dtype=snap.dtype, pin_memory=True)
        host.copy_(snap, non_blocking=True)
        done = torch.cuda.Event()
        done.record(main)
        return (timed, done, host)

    def collect(self, ticket):
        timed, done, host = ticket
        done.synchronize()
        dts = []
        for start, end, n in timed:
            dts += [start.elapsed_time(end) * 1e-3] * n
        return [float(x) for x in host], dts

    def step(self, handles) -> list:
        return self.collect(self.launch(handles))[0]

    def release(self, handle) -> None:
        if self.keep_final and handle:
            p = handle["prob"]
            self.final[handle["req"].job_id] = (p.object.clone(), p.probe.clone(), p.pos.clone())
        handle.clear()


# ------------------------------------------------------------ job data

def _host_job(w):
    """Seeded host data of one serving job: the ground truth and the start
    state (complex64 / float32).  Runs in a worker process."""
    import synth
    truth = synth.make_truth(w)
    start = synth.make_start(truth, w)
    c64 = lambda a: np.ascontiguousarray(a[:, 0] if a.ndim == 4 else a).astype(np.complex64)
    return dict(t_object=c64(truth["object"]), t_probe=truth["probe"].astype(np.complex64),
                t_pos=truth["pos"].astype(np.float32), object=c64(start["object"]),
                probe=start["probe"].astype(np.complex64), pos=start["pos"].astype(np.float32),
                pads=tuple(truth["pads"]))


def host_jobs(workloads, workers: int = 0) -> list:
    """Host data of every workload, made in a pool of spawned processes."""
    import os
    from concurrent.futures import ProcessPoolExecutor
    import multiprocessing as mp
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1, len(workloads))
    if workers <= 1:
        return [_host_job(w) for w in workloads]
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as pool:
        return list(pool.map(_host_job, workloads))


def build_requests(workloads, hosts, arrivals, iters: int, device, chunk: int = 64,
                   pinned: bool = True) -> list:
    """Requests with measured patterns: the library's forward model on the
    ground truth, Poisson-sampled on the device with a per-job seed.  The
    payload is kept in page-locked host memory (when ``pinned``), so that
    admission copies run asynchronously."""
    import torch
    from . import binding as B
    reqs = []
    for j, (w, hd, t_arr) in enumerate(zip(workloads, hosts, arrivals)):
        dev = torch.device(device)
        tprob = B.Problem(object=torch.from_numpy(hd["t_object"]).to(dev),
                          probe=torch.from_numpy(hd["t_probe"]).to(dev),
                          pos=torch.from_numpy(hd["t_pos"]).to(dev), pads=hd["pads"])
        I = torch.empty(w.K, w.N, w.N, device=dev)
        ws = B.workspace([tprob], 0, chunk)
        B.ptycho_forward([tprob], [I], ws)
        gen = torch.Generator(device=dev)
        gen.manual_seed(w.seed + 2000)
        meas_dev = torch.poisson(I.clamp_min(0.0), generator=gen)
        del tprob, I, ws
        pin = lambda t: torch.empty(t.shape, dtype=t.dtype, pin_memory=pinned).copy_(t)
        payload = dict(object=pin(torch.from_numpy(hd["object"])),
                       probe=pin(torch.from_numpy(hd["probe"])),
                       pos=pin(torch.from_numpy(hd["pos"])), measured=pin(meas_dev))
        del meas_dev
        reqs.append(JobRequest(job_id=j, arrival=float(t_arr), iters=iters, K=w.K, L=w.L, M=w.M,
                               N=w.N, H=w.H, W=w.W, pads=hd["pads"], payload=payload))
    return reqs


def measure_service_times(executor: TorchExecutor, reqs, reps: int = 1) -> list:
    """Seconds per iteration of each job run alone (after one warm-up)."""
    out = []
    for r in reqs:
        h = executor.admit(r)
        executor.step([h])
        t0 = time.perf_counter()
        for _ in range(reps):
            executor.step([h])
        out.append((time.perf_counter() - t0) / reps)
        executor.release(h)
    return out


# Default extra work per tick of the hybrid policy: one 256^2 x 4800-pattern-
# mode iteration.  On the 64-job stream below it keeps the job-latency p99 at
# that of first-come first-served execution (twice as much shortens the
# median further but lengthens the p99).
DEFAULT_TICK_CAP = 4800 * 256 * 256
# Default fusion window of the hybrid policy: none (every rider within the cap).
DEFAULT_WORK_RATIO = None
# Calls of fewer pattern-pixels than this are dominated by their ~25 kernel
# launches (a 64^2 x 100-position single-mode step takes 0.12 ms against
# about 0.01 ms of work at the rate of a saturated step), so jobs below it
# share one call; larger jobs fill the GPU alone and run in calls of their
# own, each taking its own time.
DEFAULT_FUSE_WORK = 8 << 20


def split_calls(works, fuse_work: Optional[int]) -> list:
    """Indices of each call: consecutive jobs share a call while its summed
    work stays within ``fuse_work`` (None: one call for all)."""
    if fuse_work is None:
        return [list(range(len(works)))]
    calls, cur, acc = [], [], 0
    for i, w in enumerate(works):
        if cur and acc + w > fuse_work:
            calls.append(cur)
            cur, acc = [], 0
        cur.append(i)
        acc += w
    if cur:
        calls.append(cur)
    return calls


def run_stream(n_jobs: int = 64, iters: int = 50, seed: int = 4, load: float = 2.0,
               budget_bytes: Optional[int] = None, workspace_bytes: int = 8 << 30,
               device="cuda:0", log=print, tick_cap: Optional[int] = DEFAULT_TICK_CAP,
               policy: str = "hybrid", depth: int = 2, exact_fraction: float = 0.0,
               work_ratio: Optional[float] = DEFAULT_WORK_RATIO,
               fuse_work: Optional[int] = DEFAULT_FUSE_WORK) -> dict:
    """The serving stream end to end: job mix, data, service-time probe,
    Poisson arrivals at ``load`` times the sequential service rate, then the
    continuous-batching run and the first-come first-served sequential run
    over the same arrivals."""
    import torch
    import synth.serving as SS
    wl = SS.serving_jobs(n_jobs, seed, exact_fraction=exact_fraction)
    t0 = time.perf_counter()
    hosts = host_jobs(wl)
    log(f"host data of {n_jobs} jobs: {time.perf_counter() - t0:.1f} s")
    ex = TorchExecutor(device, workspace_bytes, fuse_work=fuse_work)
    reqs = build_requests(wl, hosts, np.zeros(n_jobs), iters, device)
    del hosts
    log(f"measured patterns: {time.perf_counter() - t0:.1f} s")
    svc = measure_service_times(ex, reqs)
    seq_service = iters * float(np.sum(svc))
    for n in sorted({r.N for r in reqs}):
        sel = [(r, t) for r, t in zip(reqs, svc) if r.N == n]
        log(f"alone, N={n}: {len(sel)} jobs, "
            f"{sum(r.pattern_modes for r, _ in sel) / sum(t for _, t in sel):.0f} pattern-modes/s")
    gap = seq_service / n_jobs / load
    arr = SS.poisson_arrivals(n_jobs, gap, seed)
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    log(f"service time alone: {seq_service:.2f} s; mean arrival gap {gap * 1e3:.1f} ms")
    if budget_bytes is None:
        free, _ = torch.cuda.mem_get_info(torch.device(device))
        budget_bytes = int(0.9 * free)
    out = {"jobs": n_jobs, "iters": iters, "seed": seed, "offered_load": load,
           "mean_arrival_gap_s": round(gap, 5), "budget_bytes": int(budget_bytes),
           "workspace_bytes": int(workspace_bytes), "tick_cap_pattern_pixels": tick_cap,
           "policy": policy, "pipeline_depth": depth, "work_ratio": work_ratio,
           "fuse_work_pattern_pixels": fuse_work,
           "exact_ratio_jobs": int(sum(w.exact_ratio for w in wl)),
           "pattern_modes_total": int(iters * sum(r.pattern_modes for r in reqs))}
    for mode in ("batch", "sequential"):
        sch = Scheduler(ex, budget_bytes, log=log, tick_cap=tick_cap, policy=policy, depth=depth,
                        work_ratio=work_ratio)
        rep = sch.run(reqs, mode)
        out[mode] = rep.summary()
        log(f"{mode}: {json_line(out[mode])}")
    return out


def json_line(d) -> str:
    import json
    return json.dumps(d)


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="serving stream: continuous batching vs sequential")
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--iters", type=int, default=50)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--load", type=float, default=2.0)
    ap.add_argument("--budget-gb", type=float, default=0.0, help="0: 0.9 x free device memory")
    ap.add_argument("--workspace-gb", type=float, default=8.0)
    ap.add_argument("--tick-cap", type=float, default=DEFAULT_TICK_CAP,
                    help="pattern-pixels (K L M N^2) per fused call; 0: no cap")
    ap.add_argument("--policy", default="hybrid", choices=POLICIES)
    ap.add_argument("--depth", type=int, default=2, help="fused calls in flight")
    ap.add_argument("--exact-fraction", type=float, default=0.0,
                    help="fraction of jobs using the exact-ratio propagator")
    ap.add_argument("--work-ratio", type=float, default=DEFAULT_WORK_RATIO or 0.0,
                    help="hybrid policy: riders within this factor of the oldest job's work "
                         "per iteration (0: no bound)")
    ap.add_argument("--fuse-work", type=float, default=DEFAULT_FUSE_WORK,
                    help="pattern-pixels up to which a tick's jobs share one call; larger "
                         "jobs run in calls of their own (0: one call per tick)")
    a = ap.parse_args()
    res = run_stream(a.jobs, a.iters, a.seed, a.load,
                     None if a.budget_gb <= 0 else int(a.budget_gb * 1e9),
                     int(a.workspace_gb * (1 << 30)),
                     log=lambda s: print(s, flush=True),
                     tick_cap=int(a.tick_cap) if a.tick_cap > 0 else None, policy=a.policy,
                     depth=a.depth, exact_fraction=a.exact_fraction,
                     work_ratio=a.work_ratio if a.work_ratio > 0 else None,
                     fuse_work=int(a.fuse_work) if a.fuse_work > 0 else None)
    print(json.dumps(res), flush=True)
