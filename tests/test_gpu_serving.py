"""Serving on the GPU: every job's result is the same alone and in the
continuous-batching mix."""
import numpy as np
import pytest
import torch

import synth.serving as SS

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


class TickClock:
    """Virtual time: one unit per fused call, so arrivals are in ticks."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


def _requests(iters):
    from paper_2311_14780_amd import serving as S
    # jobs 2 and 4 use the exact-ratio propagator (their own launch groups
    # inside the same fused calls)
    specs = [(128, 2, 3, 14, False), (256, 1, 2, 6, False), (128, 3, 1, 9, True),
             (128, 1, 4, 11, False), (256, 2, 1, 5, True)]
    wl = [SS.serving_workload(j, N, L, M, K, 900 + j, x) for j, (N, L, M, K, x) in enumerate(specs)]
    hosts = S.host_jobs(wl, workers=1)
    # arrivals in ticks: two at once, then one joining each of the next ticks
    return S.build_requests(wl, hosts, [0.0, 0.0, 1.0, 2.5, 4.0], iters, DEV)


def test_each_job_is_the_same_alone_and_in_the_mix():
    from paper_2311_14780_amd import serving as S
    iters = 5
    reqs = _requests(iters)
    for r in reqs:
        print("job", r.job_id, "N", r.N, "L", r.L, "M", r.M, "K", r.K, "pads", r.pads, flush=True)
    # a small workspace forces several position chunks per fused call
    ex = S.TorchExecutor(DEV, 32 << 20, keep_final=True)

    class Ticking(S.Executor):
        def __init__(self, inner, clock):
            self.inner, self.clock = inner, clock

        def footprint(self, r):
            return self.inner.footprint(r)

        def fits(self, rs):
            return self.inner.fits(rs)

        def admit(self, r):
            return self.inner.admit(r)

        def release(self, h):
            self.inner.release(h)

        def step(self, hs):
            out = self.inner.step(hs)
            self.clock.t += 1.0
            return out

    clk = TickClock()
    sch = S.Scheduler(Ticking(ex, clk), budget_bytes=1 << 40, clock=clk, sleep=clk.sleep)
    rep = sch.run(reqs, "batch")
    mixed = dict(ex.final)
    rec = rep.records
    assert all(r.status == "done" and r.iters_done == iters for r in rec.values())
    assert rep.max_fused >= 3
    # a job joined while another was mid-flight
    assert rec[3].admitted_at > rec[0].admitted_at and rec[3].admitted_at < rec[0].finished_at
    for r in reqs:
        ex.final.clear()
        clk2 = TickClock()
        alone = S.Scheduler(Ticking(ex, clk2), 1 << 40, clock=clk2, sleep=clk2.sleep).run(
            [S.JobRequest(**{**r.__dict__, "arrival": 0.0})], "batch")
        a = ex.final[r.job_id]
        m = mixed[r.job_id]
        assert alone.records[r.job_id].losses == rec[r.job_id].losses, r.job_id
        for name, x, y in zip(("object", "probe", "pos"), a, m):
            assert torch.equal(x, y), (r.job_id, name)
        # the state moved: Adam steps were taken
        assert not torch.equal(m[2], torch.as_tensor(r.payload["pos"]).to(DEV))


def test_sequential_and_batched_runs_agree():
    from paper_2311_14780_amd import serving as S
    reqs = _requests(3)
    for r in reqs:
        r.arrival = 0.0
    ex = S.TorchExecutor(DEV, 256 << 20, keep_final=True)
    seq_rep = S.Scheduler(ex, 1 << 40).run(reqs, "sequential")
    seq = dict(ex.final)
    # pipelined ticks (two fused calls in flight, losses read one tick late),
    # asynchronous admission copies, a cap on the work riding with the head
    for policy, cap in (("hybrid", 2 * 20 * 128 * 128), ("srpt", None), ("fifo", 200 * 128 * 128)):
        ex.final.clear()
        rep = S.Scheduler(ex, 1 << 40, tick_cap=cap, policy=policy, depth=2).run(reqs, "batch")
        assert rep.max_fused >= 2, policy
        for j, a in seq.items():
            assert rep.records[j].losses == seq_rep.records[j].losses, (policy, j)
            for x, y in zip(a, ex.final[j]):
                assert torch.equal(x, y), (policy, j)


def test_ticks_split_into_calls_agree_with_sequential():
    """Jobs above the fusion threshold run in calls of their own within a
    tick (each timed on its own); the states are those of sequential runs."""
    from paper_2311_14780_amd import serving as S
    reqs = _requests(3)
    for r in reqs:
        r.arrival = 0.0
    ex = S.TorchExecutor(DEV, 256 << 20, keep_final=True)
    seq_rep = S.Scheduler(ex, 1 << 40).run(reqs, "sequential")
    seq = dict(ex.final)
    # threshold: jobs 1 and 2 (adjacent) fit one call, job 0 does not join them
    fuse = reqs[1].work + reqs[2].work
    assert reqs[0].work + reqs[1].work > fuse
    split = S.TorchExecutor(DEV, 256 << 20, keep_final=True, fuse_work=fuse)
    calls = split.calls_of([{"req": r} for r in reqs])
    print("calls of one tick over all jobs:", calls, flush=True)
    assert [1, 2] in calls and 1 < len(calls) < len(reqs)
    rep = S.Scheduler(split, 1 << 40, tick_cap=None, policy="hybrid", depth=2).run(reqs, "batch")
    assert rep.max_fused == len(reqs)
    for j, a in seq.items():
        assert rep.records[j].losses == seq_rep.records[j].losses, j
        for x, y in zip(a, split.final[j]):
            assert torch.equal(x, y), j
    # each job's iteration latency is its own call's device time
    lat = {j: r.iter_latency[0] for j, r in rep.records.items()}
    assert len(set(lat.values())) > 1, lat


def test_jobs_admitted_mid_flight_with_pipelined_ticks():
    """Real clock, two fused calls in flight, job data copied in on its own
    stream while earlier jobs compute: nothing fails and every job ends in
    the state it reaches alone."""
    from paper_2311_14780_amd import serving as S
    reqs = _requests(12)
    ex = S.TorchExecutor(DEV, 64 << 20, keep_final=True)
    alone = {}
    for r in reqs:
        ex.final.clear()
        S.Scheduler(ex, 1 << 40).run([S.JobRequest(**{**r.__dict__, "arrival": 0.0})])
        alone[r.job_id] = ex.final[r.job_id]
    # a fraction of a millisecond apart (an iteration of these jobs takes
    # about 0.2 ms): later jobs arrive while ticks are in flight
    for i, r in enumerate(reqs):
        r.arrival = 0.0004 * i
    ex.final.clear()
    rep = S.Scheduler(ex, 1 << 40, policy="hybrid", tick_cap=None, depth=2).run(reqs)
    assert all(x.status == "done" for x in rep.records.values()), \
        {j: (x.status, x.losses) for j, x in rep.records.items()}
    assert rep.max_fused >= 2
    for j, a in alone.items():
        for x, y in zip(a, ex.final[j]):
            assert torch.equal(x, y), j
