"""Serving scheduler policy on the CPU: a fake executor with a cost model and
a virtual clock stand in for the device."""
import math

import numpy as np
import pytest

from paper_2311_14780_amd.serving import Executor, JobRequest, Scheduler


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor(Executor):
    """Cost of a fused call: a fixed launch overhead plus the work of every
    job in it.  ``nan_at`` = {job_id: iteration} makes that iteration's loss
    NaN."""

    def __init__(self, clock, overhead=1.0, nan_at=None, max_jobs=None):
        self.clock = clock
        self.overhead = overhead
        self.nan_at = nan_at or {}
        self.max_jobs = max_jobs
        self.calls = []          # job ids of every fused call
        self.resident = set()
        self.iters = {}

    def footprint(self, req):
        return req.payload["fp"]

    def fits(self, reqs):
        return self.max_jobs is None or len(reqs) <= self.max_jobs

    def admit(self, req):
        assert req.job_id not in self.resident
        self.resident.add(req.job_id)
        self.iters[req.job_id] = 0
        return req

    def step(self, handles):
        self.calls.append([h.job_id for h in handles])
        self.clock.t += self.overhead + sum(h.payload["work"] for h in handles)
        out = []
        for h in handles:
            self.iters[h.job_id] += 1
            bad = self.nan_at.get(h.job_id) == self.iters[h.job_id]
            out.append(math.nan if bad else 1.0 / self.iters[h.job_id])
        return out

    def release(self, h):
        self.resident.remove(h.job_id)


def req(i, arrival, fp, work=1.0, iters=5):
    return JobRequest(job_id=i, arrival=arrival, iters=iters, K=10, L=1, M=1, N=128, H=256,
                      W=256, pads=(128,), payload={"fp": fp, "work": work})


def run(reqs, budget, mode="batch", sched=None, **kw):
    clk = Clock()
    ex = FakeExecutor(clk, **kw)
    sch = Scheduler(ex, budget, clock=clk, sleep=clk.sleep, **(sched or {}))
    return sch, ex, sch.run(reqs, mode)


def test_admission_respects_the_memory_budget():
    reqs = [req(0, 0.0, 4), req(1, 0.0, 4), req(2, 0.0, 4)]
    _, ex, rep = run(reqs, budget=10)
    # the third job waits until one of the first two has left
    assert ex.calls[0] == [0, 1]
    assert all(len(c) <= 2 for c in ex.calls)
    assert rep.peak_bytes <= 10
    r = rep.records
    assert r[2].admitted_at >= min(r[0].finished_at, r[1].finished_at)
    assert all(x.status == "done" and x.iters_done == 5 for x in r.values())


def test_arrivals_join_while_others_run():
    # job 1 arrives mid-flight and shares fused calls with job 0
    reqs = [req(0, 0.0, 1, iters=10), req(1, 3.5, 1, iters=3)]
    _, ex, rep = run(reqs, budget=10)
    r = rep.records
    assert r[0].admitted_at < r[1].admitted_at < r[0].finished_at
    assert any(sorted(c) == [0, 1] for c in ex.calls)
    assert r[1].finished_at < r[0].finished_at  # the short job is not queued behind job 0


def test_admission_is_first_come_first_served():
    # the big head-of-line job blocks the small one behind it
    reqs = [req(0, 0.0, 6), req(1, 0.1, 6), req(2, 0.2, 1)]
    _, ex, rep = run(reqs, budget=10)
    order = sorted(rep.records.values(), key=lambda x: x.admitted_at)
    assert [x.job_id for x in order] == [0, 1, 2]
    assert rep.records[2].admitted_at >= rep.records[0].finished_at


def test_failed_job_is_isolated():
    reqs = [req(0, 0.0, 1), req(1, 0.0, 1), req(2, 0.0, 1)]
    _, ex, rep = run(reqs, budget=10, nan_at={1: 3})
    r = rep.records
    assert r[1].status == "failed" and r[1].iters_done == 3
    assert r[0].status == r[2].status == "done"
    assert r[0].iters_done == r[2].iters_done == 5
    assert not ex.resident  # every job's memory was given back


def test_cancellation_frees_memory_for_waiting_jobs():
    reqs = [req(0, 0.0, 8, iters=100), req(1, 0.0, 8)]
    clk = Clock()
    ex = FakeExecutor(clk)

    def on_tick(sch, tick):
        if tick == 2:
            sch.cancel(0)

    sch = Scheduler(ex, 10, clock=clk, sleep=clk.sleep, on_tick=on_tick)
    rep = sch.run(reqs)
    r = rep.records
    assert r[0].status == "cancelled" and r[0].iters_done == 2
    assert r[1].status == "done" and r[1].admitted_at >= r[0].finished_at
    assert not ex.resident


def test_oversized_job_is_rejected_and_others_run():
    reqs = [req(0, 0.0, 50), req(1, 0.0, 2)]
    _, ex, rep = run(reqs, budget=10)
    assert rep.records[0].status == "rejected"
    assert rep.records[1].status == "done"


def test_sequential_mode_runs_one_job_at_a_time():
    reqs = [req(i, 0.1 * i, 1) for i in range(4)]
    _, ex, rep = run(reqs, budget=100, mode="sequential")
    assert all(len(c) == 1 for c in ex.calls)
    fin = [rep.records[i].finished_at for i in range(4)]
    assert fin == sorted(fin)


def test_batching_beats_sequential_when_calls_have_overhead():
    rng = np.random.default_rng(0)
    reqs = [req(i, float(a), 1, work=float(w), iters=20)
            for i, (a, w) in enumerate(zip(np.cumsum(rng.exponential(2.0, 12)), rng.uniform(0.2, 2.0, 12)))]
    _, _, b = run(reqs, budget=100)
    _, _, s = run(reqs, budget=100, mode="sequential")
    sb, ss = b.summary(), s.summary()
    assert sb["jobs_done"] == ss["jobs_done"] == 12
    assert b.pattern_modes == s.pattern_modes
    assert sb["makespan_s"] < ss["makespan_s"]
    assert sb["job_latency_p50_s"] < ss["job_latency_p50_s"]


def test_fits_limits_the_fused_set():
    reqs = [req(i, 0.0, 1) for i in range(5)]
    _, ex, rep = run(reqs, budget=100, max_jobs=2)
    assert max(len(c) for c in ex.calls) == 2
    assert all(x.status == "done" for x in rep.records.values())


def test_idle_gaps_are_waited_out():
    reqs = [req(0, 0.0, 1, iters=1), req(1, 100.0, 1, iters=1)]
    _, ex, rep = run(reqs, budget=10)
    assert rep.records[1].admitted_at >= 100.0
    assert rep.ticks == 2


def test_tick_cap_bounds_the_fused_work():
    # every request is K L M N^2 = 10 * 128^2 pattern-pixels per iteration
    reqs = [req(i, 0.0, 1) for i in range(6)]
    _, ex, rep = run(reqs, budget=100, sched=dict(tick_cap=25 * 128 * 128, policy="srpt"))
    assert max(len(c) for c in ex.calls) == 2
    assert all(x.status == "done" and x.iters_done == 5 for x in rep.records.values())


def test_a_job_larger_than_the_cap_still_runs():
    reqs = [req(0, 0.0, 1)]
    _, ex, rep = run(reqs, budget=100, sched=dict(tick_cap=3 * 128 * 128))
    assert rep.records[0].status == "done"


def test_shortest_remaining_work_goes_first():
    # one slot per tick: the short job that arrives later overtakes the long one
    reqs = [req(0, 0.0, 1, iters=50), req(1, 0.5, 1, iters=3)]
    _, ex, rep = run(reqs, budget=100, sched=dict(tick_cap=10 * 128 * 128, policy="srpt"))
    r = rep.records
    assert r[1].finished_at < r[0].finished_at
    _, ex2, rep2 = run(reqs, budget=100, sched=dict(tick_cap=10 * 128 * 128, policy="fifo"))
    assert rep2.records[1].finished_at > rep2.records[0].finished_at


class SlowCopies(FakeExecutor):
    """Jobs become ready a fixed time after admission (asynchronous copies)."""

    def __init__(self, clock, delay, **kw):
        super().__init__(clock, **kw)
        self.delay = delay
        self.t_ready = {}

    def admit(self, r):
        self.t_ready[r.job_id] = self.clock.t + self.delay
        return super().admit(r)

    def ready(self, h):
        return self.clock.t >= self.t_ready[h.job_id]

    def wait(self, hs):
        self.clock.t = max(self.clock.t, min(self.t_ready[h.job_id] for h in hs))


def test_jobs_run_once_their_data_has_arrived():
    clk = Clock()
    ex = SlowCopies(clk, delay=2.5)
    reqs = [req(0, 0.0, 1, iters=10), req(1, 1.0, 1, iters=2)]
    rep = Scheduler(ex, 100, clock=clk, sleep=clk.sleep).run(reqs)
    # job 0 waited for its copy; job 1 was admitted while job 0 ran and
    # joined the fused calls only once its own copy had landed
    assert ex.calls[0] == [0]
    first_with_1 = next(i for i, c in enumerate(ex.calls) if 1 in c)
    assert first_with_1 > 0
    assert all(x.status == "done" for x in rep.records.values())


def test_hybrid_keeps_the_oldest_job_moving():
    # a long job at the head and short ones behind it: the head runs in every
    # tick, the short ones ride along within the extra-work cap
    reqs = [req(0, 0.0, 1, iters=30)] + [req(i, 0.5 * i, 1, iters=4) for i in range(1, 6)]
    _, ex, rep = run(reqs, budget=100, sched=dict(tick_cap=2 * 10 * 128 * 128))
    head_ticks = [c for c in ex.calls if 0 in c]
    assert len(head_ticks) == 30
    assert all(c[0] == 0 for c in ex.calls[:30])
    assert max(len(c) for c in ex.calls) == 3
    r = rep.records
    assert all(r[i].finished_at < r[0].finished_at for i in range(1, 6))


def test_pipelined_ticks_give_the_same_schedule_outcome():
    reqs = [req(i, 0.3 * i, 2, iters=6) for i in range(6)]
    outs = []
    for depth in (1, 2, 3):
        _, ex, rep = run(reqs, budget=6, sched=dict(depth=depth))
        outs.append({j: (x.status, x.iters_done, x.losses) for j, x in rep.records.items()})
        assert rep.peak_bytes <= 6
    assert outs[0] == outs[1] == outs[2]


def test_failure_is_noticed_one_tick_late_when_pipelined():
    reqs = [req(0, 0.0, 1, iters=8), req(1, 0.0, 1, iters=8)]
    _, ex, rep = run(reqs, budget=10, nan_at={1: 3}, sched=dict(depth=2))
    r = rep.records
    assert r[1].status == "failed" and 3 <= r[1].iters_done <= 4
    assert r[0].status == "done" and r[0].iters_done == 8
    assert not ex.resident


def reqk(i, arrival, K, iters=3, fp=1):
    # work per iteration K L M N^2 (scheduler) and the fake executor's cost agree up to a scale
    return JobRequest(job_id=i, arrival=arrival, iters=iters, K=K, L=1, M=1, N=128, H=256,
                      W=256, pads=(128,), payload={"fp": fp, "work": K / 100.0})


def test_work_ratio_keeps_much_smaller_jobs_out_of_a_large_jobs_call():
    # head: 1000 positions; a 900-position job rides along (within 2x, fits the
    # head's own work as extra), a 100-position job does not
    reqs = [reqk(0, 0.0, 1000), reqk(1, 0.0, 900), reqk(2, 0.0, 100)]
    _, ex, rep = run(reqs, budget=10, sched=dict(work_ratio=2.0))
    assert ex.calls[0] == [0, 1]
    assert all(not (0 in c and 2 in c) for c in ex.calls)
    assert all(r.status == "done" for r in rep.records.values())
    # without the bound the small job rides along with the head
    _, ex2, _ = run(reqs, budget=10)
    assert 2 in ex2.calls[0]


def test_work_ratio_caps_the_extra_work_at_the_heads_own():
    # three equal jobs: only one rider per call (extra work <= the head's)
    reqs = [reqk(i, 0.0, 500) for i in range(3)]
    _, ex, _ = run(reqs, budget=10, sched=dict(work_ratio=4.0))
    assert all(len(c) <= 2 for c in ex.calls)


def test_wall_latency_counts_the_ticks_a_job_waits():
    # job 1 waits out job 0's calls while it is kept out of them
    reqs = [reqk(0, 0.0, 1000, iters=2), reqk(1, 0.0, 100, iters=2)]
    _, ex, rep = run(reqs, budget=10, sched=dict(work_ratio=2.0), overhead=0.0)
    r0, r1 = rep.records[0], rep.records[1]
    assert [c for c in ex.calls] == [[0], [0], [1], [1]]
    # (iter_latency holds the executor's own timing: here the fake's host time)
    np.testing.assert_allclose(r0.iter_wall, [10.0, 10.0])
    # job 1's first iteration completes 21 s after its admission (it waited 20 s)
    np.testing.assert_allclose(r1.iter_wall, [21.0, 1.0])
    s = rep.summary()
    assert s["iter_wall_p99_ms"] >= 1e3 * 20.0


def test_work_ratio_below_one_is_rejected():
    with pytest.raises(ValueError):
        Scheduler(None, 1, work_ratio=0.5)


def test_split_calls_groups_consecutive_small_jobs():
    from paper_2311_14780_amd.serving import split_calls
    assert split_calls([5, 1, 1, 1, 9, 2], None) == [[0, 1, 2, 3, 4, 5]]
    # small jobs share a call up to the threshold; a larger job runs alone
    assert split_calls([1, 1, 1, 9, 2, 2], 3) == [[0, 1, 2], [3], [4], [5]]
    assert split_calls([2, 2, 1], 4) == [[0, 1], [2]]
    assert split_calls([], 4) == []


class SplitExecutor(FakeExecutor):
    """Reports each job's own device time, as an executor that runs the
    jobs of a tick in calls of their own does."""

    def launch(self, handles):
        losses = self.step(handles)
        return losses, [h.payload["work"] for h in handles]


def test_per_job_device_times_are_recorded_per_job():
    clk = Clock()
    ex = SplitExecutor(clk, overhead=0.0)
    reqs = [req(0, 0.0, 1, work=4.0, iters=2), req(1, 0.0, 1, work=1.0, iters=2)]
    rep = Scheduler(ex, 10, clock=clk, sleep=clk.sleep).run(reqs, "batch")
    assert ex.calls[0] == [0, 1]
    assert rep.records[0].iter_latency == [4.0, 4.0]
    assert rep.records[1].iter_latency == [1.0, 1.0]
