"""Serving reconstruction jobs with continuous batching.

A job is a SIRT reconstruction (the iterative family the projector serves,
Sec. I): a fan-beam geometry, a sinogram and a number of iterations.  Jobs
arrive over time with different image sizes, view counts and detector counts.

``Server.run`` is the request loop:

* arrived jobs wait in a FIFO queue and are admitted while the device-memory
  budget and the slot limit allow (admission by free HBM);
* an admitted job keeps its geometry tables, iterate, sinogram and scratch on
  the device until it finishes;
* every step advances admitted jobs by SIRT iterations in grouped launches
  (``fp_sirt_step_multi``: the padded copies and forward residuals of up to
  12 jobs of different geometries in one launch each, then each job's back
  update), so jobs that arrive while others run join at the next step and
  their work overlaps on the device (continuous batching).  A job large enough
  to fill the device by itself runs its iterations with the single-job kernels
  instead, in the same stream;
* a step fills a work budget with jobs in order of their remaining device
  time less `aging` times the time they have spent in the system (shortest
  remaining first, so a small job that arrives while a large one runs does
  not wait for all of it, while a job's priority rises as it waits, so none
  starves): one iteration each while the budget holds (the first job
  always), several for a job that ends up alone;
* finished jobs leave and free their memory for the queue.

``run_plain`` is the comparison path: one job at a time, in arrival order,
with ``fp_sirt_step``.

The scheduler only talks to an executor (``prepare``, ``step`` or ``launch``
and ``wait``, ``run_job``, ``result``, ``release``; a step takes the jobs'
handles and an iteration count per job)
and a clock, so its admission and ordering logic can be tested on the CPU
with a scripted executor and a simulated clock.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

__all__ = ["JobSpec", "make_trace", "job_device_bytes", "job_iteration_work", "RealClock", "SimClock", "Server",
           "run_plain", "latency_stats", "GpuExecutor"]


@dataclass
class JobSpec:
    job_id: int
    arrival: float          # seconds after the start of the trace
    n: int                  # image side (n x n, pixel size 1)
    n_views: int            # views uniformly over [0, 2 pi)
    n_det: int              # detector cells of width det_width
    dsc: float              # source-to-centre distance
    dsd: float              # source-to-detector distance
    iters: int = 20
    det_width: float = 1.0
    seed: int = 0           # seed of the job's data

    def geometry_kwargs(self) -> dict:
        ang = 2.0 * np.pi * np.arange(self.n_views, dtype=np.float64) / self.n_views
        return dict(nx=self.n, ny=self.n, pixel=1.0, dsc=self.dsc, dsd=self.dsd, angles=ang,
                    n_det=self.n_det, det_width=self.det_width)


def make_trace(count: int, rate: float, seed: int, sizes=(256, 512, 1024),
               views=(180, 360, 720, 1440), iters: int = 20) -> list:
    """Seeded Poisson arrivals (exponential gaps, mean 1/rate) of jobs with
    image side from `sizes`, views from `views`, detectors = 2 x side,
    source-centre U[2, 4] x side and magnification 1.5."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(sizes))
        nv = int(rng.choice(views))
        dsc = float(rng.uniform(2.0, 4.0)) * n
        out.append(JobSpec(job_id=k, arrival=t, n=n, n_views=nv, n_det=2 * n, dsc=dsc,
                           dsd=1.5 * dsc, iters=iters, seed=int(rng.integers(0, 2 ** 31))))
    return out


def job_iteration_work(spec: JobSpec) -> float:
    """Matrix entries one SIRT iteration of the job evaluates (a forward and a
    back projection, about 3 non-zero cells per pixel and view)."""
    return 2.0 * 3.0 * spec.n * spec.n * spec.n_views


def _view_groups(tiles: int, views: int, cus: int) -> int:
    """View groups the library's back projection splits `views` into over
    `tiles` tiles (about 8 work-groups per compute unit, at most 32, at
    least 8 views per group)."""
    g = max(1, min(-(-8 * cus // tiles), 32))
    while g > 1 and views // g < 8:
        g -= 1
    return g


def job_scratch_bytes(spec: JobSpec, cus: int = 256) -> int:
    """Device scratch one SIRT step of the job takes from the library's
    buffers: the padded image copies and the back projection's partial sums,
    in the octant form (views a multiple of 8 over 2 pi from angle 0: views
    0 .. nv/8 with eight sums per pixel), the quarter-turn form (a multiple
    of 4: nv/4 views, four sums) or the plain one.  Equal to
    fp_sirt_scratch_bytes for the job's geometry."""
    n, nv = spec.n, spec.n_views
    tiles = math.ceil(n / 16) * math.ceil(n / 32)
    copies = 4 * n * 2 * (n + 32)          # row-major and transposed padded copies
    if nv % 8 == 0:
        partial = 4 * _view_groups(tiles, nv // 8 + 1, cus) * 8 * n * n
    elif nv % 4 == 0:
        partial = 4 * _view_groups(tiles, nv // 4, cus) * 4 * n * n
    else:
        g = _view_groups(tiles, nv, cus)
        partial = 4 * g * n * n if g > 1 else 0
    return -(-copies // 256) * 256 + partial


def job_device_bytes(spec: JobSpec, cus: int = 256) -> int:
    """Upper estimate of the device memory a job holds while admitted: the
    FP32 per-ray tables (11 per ray), per-view and per-tile tables, the SIRT
    weights, iterate, sinogram, residual and its share of the launch scratch
    (job_scratch_bytes)."""
    rays = spec.n_views * spec.n_det
    pix = spec.n * spec.n
    tiles = math.ceil(spec.n / 16) * math.ceil(spec.n / 32)
    tables = 4 * 11 * rays + 16 * spec.n_views + 16 * spec.n_views * tiles
    weights = 4 * (rays + pix)
    buffers = 4 * (pix + 2 * rays)
    return tables + weights + buffers + job_scratch_bytes(spec, cus) + 16 * 4096


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait_until(self, t: float) -> None:
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


class SimClock:
    """Simulated time: advances only when told to (scripted executors)."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def advance(self, dt: float) -> None:
        self.t += dt

    def wait_until(self, t: float) -> None:
        self.t = max(self.t, t)


@dataclass
class _Active:
    spec: JobSpec
    handle: object
    nbytes: int
    admitted: float
    done_iters: int = 0


@dataclass
class ServeResult:
    latency: dict = field(default_factory=dict)     # job_id -> completion - arrival
    admitted: dict = field(default_factory=dict)    # job_id -> admission time
    finished: dict = field(default_factory=dict)    # job_id -> completion time
    order: list = field(default_factory=list)       # job ids in admission order
    steps: int = 0
    peak_active: int = 0
    peak_bytes: int = 0
    makespan: float = 0.0
    outputs: dict = field(default_factory=dict)     # job_id -> final iterate (if kept)
    batch_sizes: list = field(default_factory=list) # jobs per step


class Server:
    """Continuous-batching request loop over an executor.

    hbm_budget: bytes the admitted jobs may hold together (a job larger than
    the budget is admitted alone when nothing else runs); max_active: slot
    limit; step_work: matrix entries one step may evaluate (its first job
    always goes); aging, rate, max_iters: the step plan (``plan``);
    keep_outputs: True, False or the job ids whose final iterates ``run``
    returns.  With an executor that reports ``available_bytes()`` (the
    device's free memory), a job is admitted only while its estimate also
    fits that less `reserve` bytes; finished jobs whose memory the executor
    still holds are flushed first.

    With an executor that can launch a step without waiting for it
    (``launch`` returning a token and ``wait`` on a token), the loop keeps
    ``depth`` steps in flight: it launches step k + 1 before waiting for step
    k, so the device never idles while the host schedules, and a job's
    completion time is when the wait on its last step returns.  A finished
    job (its last step waited for) is released when its memory is needed for
    admission or when nothing is in flight; the executor may defer the
    device-side frees.
    """

    def __init__(self, executor, hbm_budget: int = 2 << 30, max_active: int = 64,
                 step_work: float = 4e9, clock=None, keep_outputs: bool = False,
                 depth: int = 2, reserve: int = 256 << 20, aging: float = 3.0,
                 rate: float = 2e12, max_iters: int = 8):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.reserve = int(reserve)
        self.max_active = int(max_active)
        self.step_work = float(step_work)
        self.clock = clock or RealClock()
        self.keep_outputs = keep_outputs
        self.depth = max(1, int(depth))
        self.aging = float(aging)
        self.rate = float(rate)
        self.max_iters = max(1, int(max_iters))

    def plan(self, active, now):
        """Jobs and iteration counts of the next step.  Jobs are taken in
        order of remaining device time (remaining work / `rate`) less `aging`
        times their time in the system, one iteration each while the step's
        work budget holds (the first job always; a later one that does not
        fit is passed over for the next), so small jobs share the device; a
        job that ends up alone gets more iterations (up to `max_iters` and
        its remaining ones) while the budget still holds.  Returns
        [(job, iterations)] in that order."""
        def key(a):
            rem = (a.spec.iters - a.done_iters) * job_iteration_work(a.spec)
            return (rem / self.rate - self.aging * (now - a.spec.arrival), a.spec.arrival)
        order = sorted(active, key=key)
        counts, left = {}, self.step_work
        for a in order:
            w = job_iteration_work(a.spec)
            if counts and w > left:
                continue
            counts[id(a)] = 1
            left -= w
            if left <= 0:
                break
        plan = [a for a in order if id(a) in counts]
        if len(plan) == 1 and left > 0:
            # a job alone: more of its iterations in the step (fewer host
            # round trips); several jobs keep one iteration each, so that
            # every iteration of the step still shares the device
            a = plan[0]
            w = job_iteration_work(a.spec)
            extra = min(a.spec.iters - a.done_iters, self.max_iters) - 1
            counts[id(a)] += max(0, min(extra, int(left // w)))
        return [(a, counts[id(a)]) for a in plan]

    def run(self, trace) -> ServeResult:
        res = ServeResult()
        pending = deque(sorted(trace, key=lambda s: (s.arrival, s.job_id)))
        waiting = deque()
        active: list = []          # admitted jobs with iterations left to launch
        inflight = deque()         # (token, jobs whose last iteration it holds)
        done = []                  # finished jobs not yet released
        used = 0
        clock = self.clock
        pipelined = hasattr(self.ex, "launch") and hasattr(self.ex, "wait")

        def release_done():
            nonlocal used
            for a in done:
                if self._keep(a.spec.job_id):
                    res.outputs[a.spec.job_id] = self.ex.result(a.handle)
                self.ex.release(a.handle)
                used -= a.nbytes
            done.clear()

        def retire(token, finishing):
            if pipelined:
                self.ex.wait(token)
            t = clock.now()
            for a in finishing:
                res.finished[a.spec.job_id] = t
                res.latency[a.spec.job_id] = t - a.spec.arrival
                done.append(a)

        while pending or waiting or active or inflight or done:
            now = clock.now()
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admission by free device memory, FIFO (no overtaking)
            while waiting and len(active) < self.max_active:
                spec = waiting[0]
                need = job_device_bytes(spec)
                fits = used + need <= self.budget and self._device_fits(need)
                if (active or inflight or done) and not fits:
                    if done:                      # free finished jobs first
                        release_done()
                        continue
                    break
                waiting.popleft()
                handle = self.ex.prepare(spec)
                active.append(_Active(spec, handle, need, clock.now()))
                used += need
                res.admitted[spec.job_id] = clock.now()
                res.order.append(spec.job_id)
            res.peak_active = max(res.peak_active, len(active))
            res.peak_bytes = max(res.peak_bytes, used)
            if active:
                plan = self.plan(active, clock.now())
                handles = [a.handle for a, _ in plan]
                iters = [k for _, k in plan]
                fn = self.ex.launch if pipelined else self.ex.step
                token = fn(handles, iters)
                res.steps += 1
                res.batch_sizes.append(len(plan))
                finishing = []
                for a, k in plan:
                    a.done_iters += k
                    if a.done_iters >= a.spec.iters:
                        finishing.append(a)
                if finishing:
                    fin = {id(a) for a in finishing}
                    active = [a for a in active if id(a) not in fin]
                inflight.append((token, finishing))
                while len(inflight) > (self.depth - 1 if pipelined else 0):
                    retire(*inflight.popleft())
                continue
            # nothing left to launch: drain, free, then wait for arrivals
            while inflight:
                retire(*inflight.popleft())
            release_done()
            if pending and not waiting:
                clock.wait_until(pending[0].arrival)
        res.makespan = clock.now()
        if hasattr(self.ex, "flush"):
            self.ex.flush()
        return res

    def _keep(self, job_id) -> bool:
        """keep_outputs: True (every job), a collection of job ids, or False."""
        k = self.keep_outputs
        return bool(k) if isinstance(k, bool) else job_id in k

    def _device_fits(self, need: int) -> bool:
        """Whether `need` more bytes fit the device's free memory (always true
        for an executor that does not report it); memory of released jobs the
        executor still holds is given back first."""
        if not hasattr(self.ex, "available_bytes"):
            return True
        if self.ex.available_bytes() - self.reserve >= need:
            return True
        if hasattr(self.ex, "flush"):
            self.ex.flush()
        return self.ex.available_bytes() - self.reserve >= need


def run_plain(executor, trace, clock=None, keep_outputs: bool = False) -> ServeResult:
    """The plain path: one job at a time in arrival order, each run to the end
    with single-job SIRT steps."""
    clock = clock or RealClock()
    res = ServeResult()
    for spec in sorted(trace, key=lambda s: (s.arrival, s.job_id)):
        clock.wait_until(spec.arrival)
        h = executor.prepare(spec)
        res.admitted[spec.job_id] = clock.now()
        res.order.append(spec.job_id)
        executor.run_job(h, spec.iters)
        res.steps += spec.iters
        t = clock.now()
        res.finished[spec.job_id] = t
        res.latency[spec.job_id] = t - spec.arrival
        if keep_outputs:
            res.outputs[spec.job_id] = executor.result(h)
        executor.release(h)
    res.peak_active = 1
    res.makespan = clock.now()
    if hasattr(executor, "flush"):
        executor.flush()
    return res


def latency_stats(res: ServeResult) -> dict:
    lat = np.array(sorted(res.latency.values()))
    n = len(lat)
    return {"jobs": n, "p50_s": float(np.percentile(lat, 50)) if n else None,
            "p99_s": float(np.percentile(lat, 99)) if n else None,
            "mean_s": float(lat.mean()) if n else None,
            "makespan_s": res.makespan, "throughput_jobs_per_s": n / res.makespan if res.makespan else None,
            "steps": res.steps, "peak_active": res.peak_active,
            "mean_batch": float(np.mean(res.batch_sizes)) if res.batch_sizes else 1.0}


class GpuExecutor:
    """Executor on one GPU through the C ABI: each job gets its own geometry,
    an iterate starting at zero, a seeded sinogram U[0, 4] and a residual
    buffer, all on the device.

    SIRT steps run on a stream of their own, so preparing a job (building
    its geometry tables and weights on the default stream, which waits for
    its own copies) overlaps the steps already queued.  A step runs the jobs
    whose forward projection has at least `solo_blocks` work-groups of 256
    rays with the single-job kernels, which also split the back projection
    over view groups, and groups the others in ``fp_sirt_step_multi``
    launches.  Released jobs are destroyed `free_batch` at a time (one by one
    by default: destroying a geometry does not wait; the library recycles its
    memory once the job's queued work is done)."""

    def __init__(self, device="cuda", solo_blocks: int | None = None, free_batch: int = 1,
                 keep_inputs: bool = False):
        import torch

        from . import fanproj
        self.torch = torch
        self.fp = fanproj
        self.device = torch.device(device)
        self.keep_inputs = keep_inputs
        self.inputs = {}         # job_id -> host copy of the job's sinogram (keep_inputs)
        if solo_blocks is None:
            solo_blocks = 8 * torch.cuda.get_device_properties(self.device).multi_processor_count
        self.solo_blocks = int(solo_blocks)
        self.stream = torch.cuda.Stream(device=self.device)
        self.free_batch = max(1, int(free_batch))
        self._released = []

    def _queue(self, handles) -> None:
        grouped = []
        for h in handles:
            g, x, y, w = h
            if len(handles) == 1 or g.n_views * -(-g.n_det // 256) >= self.solo_blocks:
                g.sirt_step(x, y, 1.0, w)
            else:
                grouped.append(h)
        if grouped:
            self.fp.fp_sirt_step_multi([(g.handle, x, y, w, 1.0) for g, x, y, w in grouped])

    def prepare(self, spec: JobSpec):
        torch = self.torch
        g = self.fp.Geometry(**spec.geometry_kwargs())
        gen = torch.Generator(device=self.device).manual_seed(spec.seed)
        y = torch.rand((g.n_views, g.n_det), generator=gen, device=self.device) * 4.0
        x = torch.zeros((g.ny, g.nx), device=self.device)
        w = torch.empty_like(y)
        self.fp.fp_sirt_prepare(g.handle)
        k = self.keep_inputs
        if (bool(k) if isinstance(k, bool) else spec.job_id in k):
            self.inputs[spec.job_id] = y.cpu().numpy()
        # the step stream sees the prepared data; the tensors stay allocated
        # until its work on them is done
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        for t in (x, y, w):
            t.record_stream(self.stream)
        return (g, x, y, w)

    def step(self, handles, iters=1) -> None:
        self.launch(handles, iters).synchronize()

    def launch(self, handles, iters=1):
        """Queue SIRT iterations of the jobs (`iters`: one count for all, or
        one per job: iteration k runs the jobs with more than k); returns an
        event recorded after them."""
        counts = [iters] * len(handles) if isinstance(iters, int) else list(iters)
        with self.torch.cuda.stream(self.stream):
            for k in range(max(counts, default=0)):
                self._queue([h for h, c in zip(handles, counts) if c > k])
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        return ev

    def wait(self, token) -> None:
        token.synchronize()

    def run_job(self, h, iters: int) -> None:
        g, x, y, w = h
        with self.torch.cuda.stream(self.stream):
            for _ in range(iters):
                g.sirt_step(x, y, 1.0, w)
        self.stream.synchronize()

    def result(self, h):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return h[1].detach().clone()

    def available_bytes(self) -> int:
        """Free device memory: the device's own free bytes plus what torch's
        caching allocator holds unused."""
        torch = self.torch
        free, _ = torch.cuda.mem_get_info(self.device)
        cached = torch.cuda.memory_reserved(self.device) - torch.cuda.memory_allocated(self.device)
        return int(free + cached)

    def release(self, h) -> None:
        self._released.append(h)
        if len(self._released) >= self.free_batch:
            self.flush()

    def flush(self) -> None:
        """Destroy the released jobs' geometries."""
        for g, *_ in self._released:
            g.close()
        self._released.clear()
