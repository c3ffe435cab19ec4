"""Throughput of one CNSF projection pair (forward + back) on one MI355X.

One step = fp_forward of one 512 x 512 FP32 image into 720 views x 1024
cells (flat-detector fan beam, source-centre 1000, source-detector 1500,
cell width 1) followed by fp_back of one 720 x 1024 sinogram.  Inputs are
resident in HBM before timing starts.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 flops of one matrix entry given the per-ray constants:
# offset 1, s' 2, L 3, tau' 1, tau'/2 1, 12 argument adds, 8 max, 8 signed
# square-accumulate FMAs (16), normalisation (reciprocal + multiply) 2,
# accumulate FMA 2.
FLOPS_PER_ENTRY = 48
FLOPS_ACCUMULATE = 2


def flops_per_entry(views_per_evaluation: int) -> float:
    """Algorithmic flops per non-zero entry when one evaluation of the entry
    (everything but its accumulate FMA) serves `views_per_evaluation` views:
    8 in the octant form of the back projection, where views v + k V/4 and
    their reflections across the image diagonal share the entries of view v
    on the turned and reflected image, 4 in the quarter-turn form (turns
    only), 1 in the plain form."""
    return (FLOPS_PER_ENTRY - FLOPS_ACCUMULATE) / views_per_evaluation + FLOPS_ACCUMULATE
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2 (packed / dual issue) x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3
# The same without packed FP32 instructions (one FP32 FMA per lane per cycle),
# which the library's build keeps out of the generated code: the ceiling of
# the code that runs.
PEAK_FP32_UNPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of each entry point at this workload (quarter-turn
# forward, octant back), from rocprofv3 FETCH_SIZE and WRITE_SIZE runs of this script, each
# scaled by what the same counter reads for a 256 MiB device copy in the same
# run (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0); the summary and commands are in
# profiles/.  Valid only for the kernel sources they were taken on: `traffic`
# is reported as null once the hash of those sources differs.
TRAFFIC = {
    "sources_sha256": "fed6574cb584bdd4f516dacc82fb68acba1aeef39159fc10eac6871937679fec",
    # entry-point brackets: padded copies + quarter-turn forward walk; octant
    # back + its finalize
    "bytes_per_launch": {"forward": 29727232, "back": 113501920},
    # VALU instruction utilisation of each entry point's main kernel, from the
    # same profile's SQ_INSTS_VALU: wave-instructions per CU per cycle over
    # the kernel's duration in the kernel trace of this script's default run,
    # at 2.4 GHz (one FP32 FMA wave64 instruction per CU per cycle is the
    # unpacked FP32 peak; other instructions can issue faster, so this is
    # not bounded by 1)
    "valu_utilization": {"forward": 0.77, "back": 0.66},
    "profile": "profiles/cnsf_symmetric_pair_512x720x1024.md",
}
TRAFFIC_SOURCES = ["kernels.h", "fanproj_internal.h", "forward.hip", "back_launch.h",
                   "back_flat_f32.hip"]


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1907_10526_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def time_pairs(geom, imgs, steps):
    """Average milliseconds of one forward + back of `imgs` on `geom`."""
    import torch
    sino = geom.forward(imgs)
    back = geom.back(sino)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        geom.forward(imgs, out=sino)
        geom.back(sino, out=back)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps, sino, back


def batched_pairs(geom, img, nb, steps):
    """Context beside the batch-1 headline: the same pair on nb images at once
    (the kernels evaluate each entry once for all images of a batch).
    Returns the record and the last images, sinograms and back projections
    (the back projection of each image's own forward sinogram)."""
    import torch
    imgs = torch.stack([torch.roll(img, shifts=3 * b, dims=1) for b in range(nb)])
    ms, sino, back = time_pairs(geom, imgs, steps)
    rec = {"images": nb, "steps": steps, "ms_per_batch": ms, "pairs_per_s": nb / (ms * 1e-3)}
    return rec, (imgs.cpu().numpy(), sino.cpu().numpy(), back.cpu().numpy())


def batch_rel_l2(og, outputs, seed=17):
    """rel-L2 of a batch's results against the FP64 oracle on sampled rays and
    pixels of every image (part of the CPU-baseline leg)."""
    imgs, y, z = outputs
    nb, nv, nd = y.shape
    rng = np.random.default_rng(seed)
    got_f, ref_f, got_b, ref_b = [], [], [], []
    for b in range(nb):
        x = imgs[b].astype(np.float64)
        for _ in range(6):
            v, m = int(rng.integers(0, nv)), int(rng.integers(nd // 4, 3 * nd // 4))
            got_f.append(y[b, v, m])
            ref_f.append(og.forward_ray(x, v, m))
        yb = y[b].astype(np.float64)
        for _ in range(2):
            i, j = int(rng.integers(0, z.shape[2])), int(rng.integers(0, z.shape[1]))
            got_b.append(z[b, j, i])
            ref_b.append(og.back_pixel(yb, i, j))

    def rel(a, r):
        return float(np.linalg.norm(np.subtract(a, r)) / np.linalg.norm(r))
    return {"forward": rel(got_f, ref_f), "back": rel(got_b, ref_b),
            "sample": f"{len(got_f)} rays and {len(got_b)} pixels over the {nb} images"}


def other_form_pairs(scan, img, steps, form):
    """Context: the pair in another form.  "plain": the same views listed in
    reverse order, which the library does not recognise as quarter turns
    (every view evaluated on its own); "quarter-turn": the views shifted by
    half a view step, a scan the quarter turns leave unchanged but the
    diagonal reflection does not (each entry evaluated for four views)."""
    from paper_1907_10526_amd import fanproj
    kw = scan.kwargs()
    ang = kw["angles"]
    if form == "plain":
        kw["angles"], vpe = ang[::-1].copy(), 1
        what = "views in reverse order: every view evaluated on its own"
    else:
        kw["angles"], vpe = ang + 0.5 * (ang[1] - ang[0]), 4
        what = "views shifted by half a step: each entry evaluated for four views"
    g = fanproj.Geometry(**kw)
    try:
        assert g.symmetry() == vpe
        ms, _, _ = time_pairs(g, img, steps)
    finally:
        g.close()
    return {"ms_per_pair": ms, "pairs_per_s": 1e3 / ms, "steps": steps, "what": what}


def sirt_steps(geom, img, steps):
    """Context: the SIRT step (fp_sirt_step: forward residual and back update,
    one image) on the workload's geometry, from zero on the image's own
    sinogram; the first call builds the weights and is not timed."""
    import torch
    y = geom.forward(img)
    x = torch.zeros_like(img)
    work = torch.empty_like(y)
    geom.sirt_step(x, y, 1.0, work)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        geom.sirt_step(x, y, 1.0, work)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    return {"ms": ms, "steps_per_s": 1e3 / ms, "steps": steps}


def large_scan(steps):
    """Context: the 2048^2 x 1440-view x 2048-cell scan (source-centre 4000,
    source-detector 6000, cell width 1; views uniform over 2 pi, symmetry
    order 8): geometry creation, one forward + back pair and one SIRT step of
    one image.  Returns the record and the inputs and outputs that the
    CPU-baseline leg samples against the oracle."""
    import torch
    from paper_1907_10526_amd import fanproj, phantoms, workloads
    scan = workloads.LARGE
    torch.cuda.synchronize()
    t = time.perf_counter()
    g = fanproj.Geometry(**scan.kwargs())
    torch.cuda.synchronize()
    t_geom = time.perf_counter() - t
    try:
        img_np = workloads.phantom(scan)
        img = torch.from_numpy(img_np).cuda()
        ms_pair, y, _ = time_pairs(g, img, steps)
        sino_np = phantoms.uniform((scan.n_views, scan.n_det), 14, 0.0, 1.0)
        z = g.back(torch.from_numpy(sino_np).cuda())
        # SIRT steps from zero on the image's own sinogram (the first call
        # builds the row and column weights and is not timed)
        x = torch.zeros_like(img)
        work = torch.empty_like(y)
        g.sirt_step(x, y, 1.0, work)
        stream = torch.cuda.current_stream()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            g.sirt_step(x, y, 1.0, work)
        stop.record(stream)
        torch.cuda.synchronize()
        ms_sirt = start.elapsed_time(stop) / steps
        nnz = g.count_nonzero()
        sym = g.symmetry()
        data = (img_np, y.cpu().numpy(), sino_np, z.cpu().numpy())
    finally:
        g.close()
    rec = {"workload": "2048x2048 image (pixel 1), 1440 views over 2pi, 2048 flat-detector cells "
                       "of width 1, source-centre 4000, source-detector 6000, 20 seeded ellipses",
           "symmetry": sym, "geometry_create_ms": 1e3 * t_geom, "steps": steps,
           "ms_per_pair": ms_pair, "pairs_per_s": 1e3 / ms_pair, "sirt_step_ms": ms_sirt,
           "entries_per_projection": nnz,
           "algorithmic_tflops_pair": 2 * FLOPS_PER_ENTRY * nnz / (ms_pair * 1e-3) / 1e12}
    return rec, data


def large_rel_l2(data, seed=19):
    """rel-L2 of the large scan's forward and back projections against the
    FP64 oracle on sampled rays and pixels (part of the CPU-baseline leg)."""
    import oracle
    from paper_1907_10526_amd import workloads
    img, y, sino, z = data
    og = oracle.Geometry(**workloads.LARGE.kwargs())
    nv, nd = y.shape
    rng = np.random.default_rng(seed)
    x = img.astype(np.float64)
    got_f, ref_f = [], []
    for _ in range(12):
        v, m = int(rng.integers(0, nv)), int(rng.integers(nd // 4, 3 * nd // 4))
        got_f.append(y[v, m])
        ref_f.append(og.forward_ray(x, v, m))
    s64 = sino.astype(np.float64)
    got_b, ref_b = [], []
    for _ in range(16):
        i, j = int(rng.integers(0, z.shape[1])), int(rng.integers(0, z.shape[0]))
        got_b.append(z[j, i])
        ref_b.append(og.back_pixel(s64, i, j))

    def rel(a, r):
        return float(np.linalg.norm(np.subtract(a, r)) / np.linalg.norm(r))
    return {"forward": rel(got_f, ref_f), "back": rel(got_b, ref_b),
            "sample": f"{len(got_f)} rays of the phantom's sinogram, {len(got_b)} pixels of the "
                      "back projection of a U[0, 1] sinogram"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-batch8", action="store_true",
                   help="skip the context measurements: the 8-image batch, the other forms "
                        "and the large scan (profiled runs)")
    p.add_argument("--cpu-sample-views", type=int, default=720,
                   help="views of the workload the FP64 oracle is timed on")
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="repeat the oracle sample until this much time has passed (at most 8 passes)")
    p.add_argument("--serve-jobs", type=int, default=1000,
                   help="jobs in the served-vs-plain comparison (0 skips it)")
    p.add_argument("--serve-rates", type=float, nargs="*", default=[50.0],
                   help="arrival rates (jobs/s) of served-vs-plain traces (the served-stream "
                        "workload's 50/s by default)")
    p.add_argument("--serve-loads", type=float, nargs="*", default=[0.9],
                   help="further traces at these fractions of the plain path's measured "
                        "capacity (jobs/s with every job queued at once): near capacity")
    p.add_argument("--serve-budget-gib", type=float, default=2.0,
                   help="device-memory budget of the serving loop")
    p.add_argument("--serve-step-work", type=float, default=4e9,
                   help="matrix entries one serving step may evaluate (the oldest job always goes)")
    p.add_argument("--plain-form", action="store_true",
                   help="list the workload's views in reverse order, so that the library "
                        "evaluates every view on its own (profiles of the plain form)")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run one device-to-device copy of this many MiB before timing, as a "
                        "known-size reference for hardware byte counters")
    return p.parse_args()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(scan, img, sino, y_gpu_rows, z_gpu_part, n_views_sample, min_seconds):
    """The FP64 oracle (as it is, OpenMP on the host cores) on a bounded sample:
    forward rows and back-projection partial sums over the first
    `n_views_sample` views, repeated until `min_seconds` of CPU time have
    passed (at most 8 times).  Returns the baseline record and the rel-L2 of
    the GPU against it on that sample."""
    import oracle
    og = oracle.Geometry(**scan.kwargs())
    k = n_views_sample
    img64 = img.astype(np.float64)
    sino64 = sino.astype(np.float64)
    t_fwd = t_back = 0.0
    reps = 0
    while reps < 8 and (reps == 0 or t_fwd + t_back < min_seconds):
        t0 = time.perf_counter()
        y_ref = og.forward_views(img64, 0, k)[:k]
        t1 = time.perf_counter()
        z_ref = og.back_views(sino64, 0, k)
        t2 = time.perf_counter()
        t_fwd += t1 - t0
        t_back += t2 - t1
        reps += 1
    frac = k / scan.n_views
    secs = (t_fwd + t_back) / reps / frac  # seconds per full pair
    rec = {"value": 1.0 / secs, "unit": "pairs/s", "cores": oracle.threads(), "kind": "oracle",
           "seconds_per_pair": secs, "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
           "sample": f"forward rows and back partial sums of views 0..{k - 1} of {scan.n_views}, "
                     f"{reps} times ({t_fwd:.1f} s + {t_back:.1f} s in all, FP64), "
                     f"scaled by {scan.n_views}/{k} per pass"}
    # one core, on a smaller sample of the same workload
    k1 = max(1, min(24, k))
    n_all = oracle.threads()
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        og.forward_views(img64, 0, k1)
        og.back_views(sino64, 0, k1)
        t1 = time.perf_counter()
    finally:
        oracle.set_threads(n_all)
    rec["single_core"] = {"value": (k1 / scan.n_views) / (t1 - t0), "unit": "pairs/s", "cores": 1,
                          "seconds_per_pair": (t1 - t0) * scan.n_views / k1,
                          "sample": f"forward rows and back partial sums of views 0..{k1 - 1} "
                                    f"({t1 - t0:.1f} s, FP64), scaled by {scan.n_views}/{k1}"}
    rel = {
        "forward": float(np.linalg.norm(y_gpu_rows - y_ref) / np.linalg.norm(y_ref)),
        "back": float(np.linalg.norm(z_gpu_part - z_ref) / np.linalg.norm(z_ref)),
        "sample_views": k,
    }
    return rec, rel


def serving(args):
    """Served (continuous batching) vs plain (one job at a time) on the same
    seeded arrival traces: SIRT jobs of 256/512/1024-pixel images, 180-1440
    views, 2 x side cells, 20 iterations each.  The rates are --serve-rates
    (50/s: the served-stream workload), then the fractions --serve-loads of
    the plain path's capacity, measured first on 300 jobs of the same mix
    queued at once (seed 6).  Returns the
    record and, for the first rate, the final iterates and sinograms of the
    first two 256 x 256, 180-view jobs (for the oracle check of the
    CPU-baseline leg)."""
    from paper_1907_10526_amd import serve
    budget = int(args.serve_budget_gib * (1 << 30))
    out = {"trace": f"{args.serve_jobs} jobs, Poisson arrivals (seed 5), image side "
                    "{256,512,1024}, views {180,360,720,1440}, cells 2 x side, source-centre "
                    "U[2,4] x side, magnification 1.5, 20 SIRT iterations, sinograms U[0, 4]",
           "hbm_budget_bytes": budget, "step_work_entries": args.serve_step_work, "rates": {}}
    rates = [(f"{r:g}/s", r) for r in (args.serve_rates or [])]
    if args.serve_loads:
        t0 = time.perf_counter()
        cal = serve.latency_stats(serve.run_plain(serve.GpuExecutor(),
                                                  serve.make_trace(300, 1e6, seed=6)))
        cap = cal["throughput_jobs_per_s"]
        out["plain_capacity_jobs_per_s"] = cap
        rates += [(f"{load:g} x capacity ({load * cap:.1f}/s)", load * cap)
                  for load in args.serve_loads]
        print(f"serving: plain capacity {cap:.1f} jobs/s ({time.perf_counter() - t0:.1f} s)",
              file=sys.stderr, flush=True)
    kept = None
    for k, (key, rate) in enumerate(rates):
        trace = serve.make_trace(args.serve_jobs, rate, seed=5)
        check = [s.job_id for s in trace if s.n == 256 and s.n_views == 180][:2] if k == 0 else []
        ex = serve.GpuExecutor(keep_inputs=set(check))
        t0 = time.perf_counter()
        batched = serve.Server(ex, hbm_budget=budget, step_work=args.serve_step_work,
                               keep_outputs=set(check)).run(trace)
        print(f"serving {rate:.1f}/s: batched loop done in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        plain = serve.run_plain(ex, trace)
        print(f"serving {rate:.1f}/s: plain path done in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
        bs, ps = serve.latency_stats(batched), serve.latency_stats(plain)
        out["rates"][key] = {
            "rate_jobs_per_s": rate, "batched": bs, "plain": ps,
            "p50_batched_vs_plain": bs["p50_s"] / ps["p50_s"],
            "p99_batched_vs_plain": bs["p99_s"] / ps["p99_s"]}
        if check:
            kept = [(trace[j], ex.inputs[j], batched.outputs[j].cpu().numpy()) for j in check]
    return out, kept


def served_rel_l2(kept):
    """rel-L2 of served jobs' final iterates against the FP64 oracle's SIRT on
    the same data (part of the CPU-baseline leg)."""
    import oracle
    errs = []
    for spec, y, x in kept:
        og = oracle.Geometry(**spec.geometry_kwargs())
        ref = og.sirt(y.astype(np.float64), spec.iters)
        errs.append(float(np.linalg.norm(x.astype(np.float64) - ref) / np.linalg.norm(ref)))
    return {"jobs": [spec.job_id for spec, _, _ in kept], "rel_l2": errs,
            "worst": max(errs) if errs else None,
            "what": f"{len(kept)} served 256 x 256, 180-view jobs of the first trace, "
                    f"{kept[0][0].iters if kept else 0} SIRT iterations"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the projector is not sharded "
                                   "across GPUs (use --gpus 1)"}))
        sys.exit(2)

    import torch
    from paper_1907_10526_amd import fanproj, phantoms, workloads

    scan = workloads.MEDIUM
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    kw = scan.kwargs()
    if args.plain_form:
        # the same views listed in reverse order: every view evaluated on its
        # own (the oracle comparisons below index views in the usual order,
        # so that leg is skipped)
        kw["angles"] = kw["angles"][::-1].copy()
        args.no_cpu_baseline = True
    fanproj.Geometry(**kw).close()   # first call pays one-time runtime set-up
    t_geom = time.perf_counter()
    geom = fanproj.Geometry(**kw)
    t_geom = time.perf_counter() - t_geom
    img_np = workloads.phantom(scan)
    img = torch.from_numpy(img_np).to(dev)
    sino = torch.empty((scan.n_views, scan.n_det), dtype=torch.float32, device=dev)
    back = torch.empty((scan.n, scan.n), dtype=torch.float32, device=dev)
    nnz = geom.count_nonzero()
    stream = torch.cuda.current_stream()
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        geom.forward(img, out=sino)
        geom.back(sino, out=back)
    torch.cuda.synchronize()

    K = args.steps
    # Per-entry-point HIP events on every fifth step of the timed region (at
    # least 5 steps): each event record costs the stream a few microseconds
    # (measured: 15 us per pair with three on every step), so recording them
    # on every step would understate the throughput they sit in.
    every = max(1, min(5, K // 5))
    sampled = list(range(every - 1, K, every))   # (not the first step after the sync)
    ev = {k: [torch.cuda.Event(enable_timing=True) for _ in range(3)] for k in sampled}
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    start.record(stream)
    for k in range(K):
        e = ev.get(k)
        if e:
            e[0].record(stream)
        geom.forward(img, out=sino)
        if e:
            e[1].record(stream)
        geom.back(sino, out=back)
        if e:
            e[2].record(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = start.elapsed_time(stop)
    fwd_ms = np.array([e[0].elapsed_time(e[1]) for e in ev.values()])
    bck_ms = np.array([e[1].elapsed_time(e[2]) for e in ev.values()])
    step_ms = fwd_ms + bck_ms
    ms_per_step = total_ms / K

    # Roofline of the dominant entry point.  `achieved` counts the method's
    # algorithmic work, FLOPS_PER_ENTRY (48) flops per non-zero entry of the
    # matrix, as for the plain form.  The symmetric forms evaluate each entry
    # once for several views (the back projection uses the scan's whole
    # symmetry, 8 with the diagonal reflection; the forward its quarter
    # turns), so they execute fewer flops for the same work: `executed`
    # counts those, (48 - 2) / views + 2 per non-zero entry.  The algorithmic
    # rate of a symmetric form can therefore exceed the FP32 peak.
    sym = geom.symmetry()
    vpe = {"forward": min(sym, 4), "back": sym}
    kernels = {"forward": float(fwd_ms.mean()), "back": float(bck_ms.mean())}
    dom = max(kernels, key=kernels.get)
    flops = FLOPS_PER_ENTRY * nnz                                      # per launch
    ex_flops = {k: flops_per_entry(v) * nnz for k, v in vpe.items()}   # per launch
    rate = lambda f, ms: f / (ms * 1e-3) / 1e12
    achieved = rate(flops, kernels[dom])
    traffic = valu = None
    if TRAFFIC["sources_sha256"] and TRAFFIC["sources_sha256"] == kernel_sources_sha256():
        traffic = TRAFFIC["bytes_per_launch"].get(dom)
        valu = TRAFFIC["valu_utilization"].get(dom)
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "traffic_unit": "bytes per launch", "traffic_profile": TRAFFIC["profile"],
                "valu_utilization": valu,
                "flops_per_entry": FLOPS_PER_ENTRY, "entries_per_launch": nnz,
                "flops_per_launch": flops,
                "form": {8: "quarter-turn forward, octant back", 4: "quarter-turn"}.get(sym, "plain"),
                "avg_ms": {k: round(v, 5) for k, v in kernels.items()},
                "executed": {
                    "views_per_entry_evaluation": vpe[dom],
                    "flops_per_entry": flops_per_entry(vpe[dom]),
                    "achieved": rate(ex_flops[dom], kernels[dom]),
                    "frac": rate(ex_flops[dom], kernels[dom]) / PEAK_FP32_TFLOPS,
                    "frac_of_unpacked_fp32": rate(ex_flops[dom], kernels[dom]) / PEAK_FP32_UNPACKED_TFLOPS},
                "by_kernel": {k: {"views_per_entry_evaluation": vpe[k],
                                  "algorithmic_tflops": rate(flops, v),
                                  "executed_frac": rate(ex_flops[k], v) / PEAK_FP32_TFLOPS}
                              for k, v in kernels.items()}}

    out = {
        "metric": "projection pairs (A+A\u1d40)/sec at 512\u00b2\u00d7720 views; p99 job latency; "
                  "rel-L2 vs FP64",
        "value": K / (total_ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fan-beam CNSF forward+back, 512x512 image (pixel 1), 720 views over "
                               "2pi, 1024 flat-detector cells of width 1, source-centre 1000, "
                               "source-detector 1500, 20 seeded ellipses, batch 1" +
                               (", views in reverse order (plain form)" if args.plain_form else "")},
        "p50_ms": float(np.percentile(step_ms, 50)),
        "p99_ms": float(np.percentile(step_ms, 99)),
        "event_sampled_steps": len(sampled),
        "wall_s": t_wall,
        "geometry_create_ms": 1e3 * t_geom,
        "roofline": roofline,
    }

    batch_out = large_out = None
    if not args.no_batch8:
        out["batch8"], batch_out = batched_pairs(geom, img, 8, max(2, K // 5))
        out["plain_form"] = other_form_pairs(scan, img, max(5, K // 2), "plain")
        out["quarter_form"] = other_form_pairs(scan, img, max(5, K // 2), "quarter-turn")
        out["large"], large_out = large_scan(max(3, K // 10))
        out["sirt_step"] = sirt_steps(geom, img, max(5, K // 10))

    kept = None
    if args.serve_jobs > 0:
        out["serving"], kept = serving(args)

    if not args.no_cpu_baseline:
        k = max(1, min(args.cpu_sample_views, scan.n_views))
        sino_in = phantoms.uniform((scan.n_views, scan.n_det), 13, 0.0, 1.0)
        y_rows = geom.forward(img)[:k].cpu().numpy()
        part = np.zeros_like(sino_in)
        part[:k] = sino_in[:k]
        z_part = geom.back(torch.from_numpy(part).to(dev)).cpu().numpy()
        rec, rel = cpu_baseline(scan, img_np, sino_in, y_rows, z_part, k, args.cpu_seconds)
        out["cpu_baseline"] = rec
        out["rel_l2_vs_fp64"] = rel
        if kept:
            out["serving"]["rel_l2_vs_fp64"] = served_rel_l2(kept)
        if batch_out is not None:
            import oracle
            out["batch8"]["rel_l2_vs_fp64"] = batch_rel_l2(oracle.Geometry(**scan.kwargs()),
                                                           batch_out)
        if large_out is not None:
            out["large"]["rel_l2_vs_fp64"] = large_rel_l2(large_out)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)
    geom.close()


if __name__ == "__main__":
    main()
