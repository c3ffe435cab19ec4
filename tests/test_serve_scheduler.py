"""The serving loop's admission and ordering logic, on the CPU, with a
scripted executor and a simulated clock (no GPU)."""
import pytest

from paper_1907_10526_amd import serve


class FakeExecutor:
    """A grouped step costs a fixed launch overhead plus each job's work
    divided by the parallelism the device still had free; a single-job step
    pays the overhead every time."""

    def __init__(self, clock, overhead=2e-3, unit=1e-9, width=4.0):
        self.clock, self.overhead, self.unit, self.width = clock, overhead, unit, width
        self.live = {}
        self.log = []
        self.step_iters = []    # iterations of each logged step

    def work(self, spec):
        return spec.n * spec.n * spec.n_views * 3 * self.unit

    def prepare(self, spec):
        self.live[spec.job_id] = spec
        self.log.append(("prepare", spec.job_id, self.clock.now()))
        return spec.job_id

    def iteration_costs(self, handles, iters):
        """Device time of each iteration of a step: iteration k runs the jobs
        with more than k iterations."""
        counts = _counts(handles, iters)
        out = []
        for k in range(max(counts)):
            hs = [h for h, c in zip(handles, counts) if c > k]
            tot = sum(self.work(self.live[h]) for h in hs)
            big = max(self.work(self.live[h]) for h in hs)
            out.append(max(tot / self.width, big))
        return out

    def step(self, handles, iters=1):
        for t in self.iteration_costs(handles, iters):
            self.clock.advance(self.overhead + t)
        self.log.append(("step", tuple(handles), self.clock.now()))
        self.step_iters.append(_counts(handles, iters))

    def run_job(self, h, iters):
        for _ in range(iters):
            self.clock.advance(self.overhead + self.work(self.live[h]))

    def result(self, h):
        return h

    def release(self, h):
        self.live.pop(h)
        self.log.append(("release", h, self.clock.now()))


def _counts(handles, iters):
    return [iters] * len(handles) if isinstance(iters, int) else list(iters)


def _trace(count=40, rate=50.0, seed=5, iters=20):
    return serve.make_trace(count, rate, seed, iters=iters)


def test_trace_is_seeded_and_follows_recipe():
    a, b = _trace(), _trace()
    assert [(s.arrival, s.n, s.n_views) for s in a] == [(s.arrival, s.n, s.n_views) for s in b]
    for s in a:
        assert s.n in (256, 512, 1024) and s.n_views in (180, 360, 720, 1440)
        assert s.n_det == 2 * s.n and 2 * s.n <= s.dsc <= 4 * s.n and s.dsd == pytest.approx(1.5 * s.dsc)
    gaps = [y.arrival - x.arrival for x, y in zip(a, a[1:])]
    assert all(g > 0 for g in gaps)


def test_all_jobs_complete_in_fifo_admission_order():
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    trace = _trace()
    res = serve.Server(ex, hbm_budget=1 << 30, clock=clock).run(trace)
    assert sorted(res.latency) == [s.job_id for s in trace]
    assert res.order == [s.job_id for s in sorted(trace, key=lambda s: s.arrival)]
    for s in trace:
        assert res.admitted[s.job_id] >= s.arrival
        assert res.latency[s.job_id] > 0
    assert not ex.live


def test_budget_limits_concurrency():
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    trace = _trace(count=30)
    budget = 3 * max(serve.job_device_bytes(s) for s in trace)
    res = serve.Server(ex, hbm_budget=budget, clock=clock).run(trace)
    assert res.peak_bytes <= budget
    # replay the log: the live set never exceeds the budget
    live, used = set(), 0
    sizes = {s.job_id: serve.job_device_bytes(s) for s in trace}
    for kind, x, _ in ex.log:
        if kind == "prepare":
            live.add(x)
            used += sizes[x]
            assert used <= budget
        elif kind == "release":
            live.discard(x)
            used -= sizes[x]


def test_job_larger_than_budget_runs_alone():
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    trace = _trace(count=6)
    small = min(serve.job_device_bytes(s) for s in trace)
    res = serve.Server(ex, hbm_budget=small, clock=clock).run(trace)
    assert res.peak_active == 1
    assert len(res.latency) == 6


def test_slot_limit():
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    res = serve.Server(ex, hbm_budget=1 << 40, max_active=2, clock=clock).run(_trace(count=20))
    assert res.peak_active <= 2


def test_batching_beats_plain_under_load():
    trace = _trace(count=60, rate=100.0, iters=10)
    c1 = serve.SimClock()
    batched = serve.Server(FakeExecutor(c1), hbm_budget=1 << 40, clock=c1).run(trace)
    c2 = serve.SimClock()
    plain = serve.run_plain(FakeExecutor(c2), trace, clock=c2)
    sb, sp = serve.latency_stats(batched), serve.latency_stats(plain)
    assert sb["p99_s"] < sp["p99_s"]
    assert sb["makespan_s"] < sp["makespan_s"]


def test_late_arrivals_join_running_batch():
    """A job arriving while others run is admitted between steps, before the
    earlier jobs finish (continuous batching, not a queue)."""
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    first = serve.JobSpec(0, 0.0, 512, 720, 1024, 1500.0, 2250.0, iters=30)
    late = serve.JobSpec(1, 0.05, 256, 180, 512, 700.0, 1050.0, iters=5)
    res = serve.Server(ex, hbm_budget=1 << 40, clock=clock).run([first, late])
    assert res.admitted[1] < res.finished[0]
    assert res.finished[1] < res.finished[0]


def test_step_plan_follows_priority_and_budget():
    """Each step takes jobs in order of remaining device time less the aging
    credit of their time in the system, as many iterations each as the work
    budget holds (the first job at least one); no job runs past its last
    iteration, and a step with more than one job stays within the budget."""
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    trace = _trace(count=30, rate=200.0, iters=8)
    big = max(serve.job_iteration_work(s) for s in trace)
    srv = serve.Server(ex, hbm_budget=1 << 40, step_work=big, clock=clock)
    res = srv.run(trace)
    assert len(res.latency) == 30
    done = {}
    for (kind, handles, _), counts in zip([e for e in ex.log if e[0] == "step"], ex.step_iters):
        assert all(c >= 1 for c in counts) and all(c <= srv.max_iters for c in counts)
        work = 0.0
        for h, c in zip(handles, counts):
            done[h] = done.get(h, 0) + c
            assert done[h] <= trace[h].iters
            work += c * serve.job_iteration_work(trace[h])
        assert len(handles) == 1 or work <= big
    assert all(done[s.job_id] == s.iters for s in trace)


def test_plan_order():
    """Shortest remaining first; waiting raises a job's priority; with a
    large aging weight the order is arrival order."""
    srv = serve.Server(None, step_work=1e30, rate=1e9, aging=1.0, max_iters=1)
    big = serve.JobSpec(0, 0.0, 1024, 1440, 2048, 3000.0, 4500.0, iters=20)
    small = serve.JobSpec(1, 0.5, 256, 180, 512, 700.0, 1050.0, iters=20)
    a_big = serve._Active(big, "big", 0, 0.0)
    a_small = serve._Active(small, "small", 0, 0.5)
    order = lambda now, s=srv: [a.handle for a, _ in s.plan([a_big, a_small], now)]
    assert order(0.5) == ["small", "big"]
    # the big job's remaining time: 20 x 9.06e9 entries at 1e9/s = 181 s;
    # a small job that arrives 190 s after it no longer overtakes it
    late = serve._Active(serve.JobSpec(2, 190.0, 256, 180, 512, 700.0, 1050.0, iters=20),
                         "late", 0, 190.0)
    assert [a.handle for a, _ in srv.plan([a_big, late], 200.0)] == ["big", "late"]
    fifo = serve.Server(None, step_work=1e30, rate=1e9, aging=1e9, max_iters=1)
    assert order(0.5, fifo) == ["big", "small"]
    # the budget: the first job always goes, a later one only if it fits
    tight = serve.Server(None, step_work=1.0, rate=1e9, aging=1.0, max_iters=4)
    plan = tight.plan([a_big, a_small], 0.5)
    assert [(a.handle, k) for a, k in plan] == [("small", 1)]
    roomy = serve.Server(None, step_work=3.5 * serve.job_iteration_work(small), rate=1e9,
                         aging=1.0, max_iters=8)
    assert [(a.handle, k) for a, k in roomy.plan([a_small], 0.5)] == [("small", 3)]


def test_small_job_overtakes_a_large_one():
    """A small job arriving while a large one runs finishes long before the
    large one (shortest remaining first), which still completes."""
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    big = serve.JobSpec(0, 0.0, 1024, 1440, 2048, 3000.0, 4500.0, iters=20)
    small = serve.JobSpec(1, 0.05, 256, 180, 512, 700.0, 1050.0, iters=20)
    # (rate: the fake device's entries per second, so that remaining times
    # and waiting times are on one clock)
    rate = serve.job_iteration_work(big) / ex.work(big)
    res = serve.Server(ex, hbm_budget=1 << 40, clock=clock, rate=rate).run([big, small])
    assert res.finished[1] < res.finished[0]
    c2 = serve.SimClock()
    plain = serve.run_plain(FakeExecutor(c2), [big, small], clock=c2)
    assert res.latency[1] < 0.5 * plain.latency[1]


class SaturatingExecutor(FakeExecutor):
    """A step costs the launch overhead plus its total work at the device's
    full rate, but never less than the time of `sat` work: a step with little
    work leaves the device partly idle."""

    def __init__(self, clock, sat=0.02, **kw):
        super().__init__(clock, **kw)
        self.sat = sat

    def step(self, handles, iters=1):
        counts = _counts(handles, iters)
        for k in range(max(counts)):
            tot = sum(self.work(self.live[h]) for h, c in zip(handles, counts) if c > k)
            self.clock.advance(self.overhead + max(tot, self.sat) / self.width)
        self.log.append(("step", tuple(handles), self.clock.now()))


def test_work_budget_improves_median_over_unbounded_batching():
    """Once a step's work fills the device, taking every admitted job into
    each step only stretches the older jobs: with the same throughput, the
    bounded step finishes jobs earlier."""
    trace = _trace(count=80, rate=150.0, iters=10)
    sat = max(SaturatingExecutor(None).work(s) for s in trace)
    runs = {}
    big = max(serve.job_iteration_work(s) for s in trace)
    for name, budget in (("unbounded", 1e30), ("bounded", 2.0 * big)):
        c = serve.SimClock()
        runs[name] = serve.Server(SaturatingExecutor(c, sat=sat), hbm_budget=1 << 40,
                                  step_work=budget, clock=c).run(trace)
    a, b = serve.latency_stats(runs["unbounded"]), serve.latency_stats(runs["bounded"])
    assert b["p50_s"] < a["p50_s"]
    assert b["makespan_s"] <= a["makespan_s"] * 1.05


class AsyncFakeExecutor(FakeExecutor):
    """launch() queues a step on a simulated device timeline and costs the
    host only `host` seconds; wait() advances the clock to the step's end;
    release() synchronises with the device (as destroying a geometry does)."""

    def __init__(self, clock, host=1e-3, **kw):
        super().__init__(clock, **kw)
        self.host = host
        self.busy_until = 0.0

    def launch(self, handles, iters=1):
        self.clock.advance(self.host)
        start = max(self.busy_until, self.clock.now())
        self.busy_until = start + sum(self.iteration_costs(handles, iters))
        self.log.append(("step", tuple(handles), self.busy_until))
        self.step_iters.append(_counts(handles, iters))
        return self.busy_until

    def wait(self, token):
        self.clock.wait_until(token)

    def release(self, h):
        self.clock.wait_until(self.busy_until)
        super().release(h)


class SyncFakeExecutor(FakeExecutor):
    """The same costs without overlap: host launch cost plus device time."""

    def __init__(self, clock, host=1e-3, **kw):
        super().__init__(clock, overhead=host, **kw)


def test_pipelined_loop_is_complete_and_within_budget():
    clock = serve.SimClock()
    ex = AsyncFakeExecutor(clock)
    trace = _trace(count=40, rate=80.0, iters=6)
    budget = 4 * max(serve.job_device_bytes(s) for s in trace)
    res = serve.Server(ex, hbm_budget=budget, clock=clock).run(trace)
    assert sorted(res.latency) == [s.job_id for s in trace]
    assert not ex.live
    steps = {}
    live, used = set(), 0
    sizes = {s.job_id: serve.job_device_bytes(s) for s in trace}
    step_iters = iter(ex.step_iters)
    for kind, x, t in ex.log:
        if kind == "prepare":
            live.add(x)
            used += sizes[x]
            assert used <= budget
        elif kind == "release":
            live.discard(x)
            used -= sizes[x]
        else:
            for h, n_it in zip(x, next(step_iters)):
                assert h in live
                steps[h] = steps.get(h, 0) + n_it
    assert all(steps[s.job_id] == s.iters for s in trace)
    for s in trace:        # a job completes no earlier than its last step ends
        last = max(t for kind, x, t in ex.log if kind == "step" and s.job_id in x)
        assert res.finished[s.job_id] >= last - 1e-12


def test_pipelining_overlaps_host_and_device():
    """Steps of a few milliseconds with a host cost of 1 ms per launch: the
    pipelined loop hides the host cost behind the device."""
    trace = _trace(count=60, rate=200.0, iters=8)
    kw = dict(host=1e-3, unit=2e-12)
    c1 = serve.SimClock()
    pipe = serve.Server(AsyncFakeExecutor(c1, **kw), hbm_budget=1 << 40, step_work=2e9,
                        clock=c1).run(trace)
    c2 = serve.SimClock()
    sync = serve.Server(SyncFakeExecutor(c2, **kw), hbm_budget=1 << 40, step_work=2e9,
                        clock=c2).run(trace)
    assert pipe.makespan < sync.makespan
    assert serve.latency_stats(pipe)["mean_s"] < serve.latency_stats(sync)["mean_s"]


def test_lone_jobs_take_several_iterations_per_step():
    """A job alone takes as many iterations per step as the work budget
    holds (at most max_iters), so a small job needs few host round trips."""
    clock = serve.SimClock()
    ex = FakeExecutor(clock)
    trace = _trace(count=12, rate=5.0, iters=10)
    res = serve.Server(ex, hbm_budget=1 << 40, clock=clock, max_iters=4).run(trace)
    assert len(res.latency) == 12
    counts = [c for cs in ex.step_iters for c in cs]
    assert max(counts) == 4 and min(counts) >= 1
    clock = serve.SimClock()
    ex1 = FakeExecutor(clock)
    serve.Server(ex1, hbm_budget=1 << 40, clock=clock, max_iters=1).run(trace)
    assert {c for cs in ex1.step_iters for c in cs} == {1}
