"""Continuous-batching serving on the GPU: every job's result is the same
alone and in the mix (to FP32 summation order), and the loop respects its
device-memory budget."""
import pytest

from paper_1907_10526_amd import serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    return torch


@pytest.mark.parametrize("solo_blocks", [None, 300])
def test_results_alone_equal_results_in_the_mix(torch_cuda, solo_blocks):
    """solo_blocks=300 sends the larger jobs of the mix to the single-job
    kernels and groups the rest; by default all of these jobs are grouped."""
    torch = torch_cuda
    trace = serve.make_trace(10, rate=200.0, seed=11, sizes=(64, 128, 256), views=(90, 180, 360),
                             iters=6)
    ex = serve.GpuExecutor(solo_blocks=solo_blocks)
    budget = 3 * max(serve.job_device_bytes(s) for s in trace)
    mixed = serve.Server(ex, hbm_budget=budget, keep_outputs=True).run(trace)
    assert mixed.peak_active >= 2 and mixed.peak_bytes <= budget
    alone = serve.run_plain(ex, trace, keep_outputs=True)
    for s in trace:
        a, b = mixed.outputs[s.job_id].double(), alone.outputs[s.job_id].double()
        err = float((a - b).norm() / b.norm())
        assert err <= 1e-5, (s.job_id, s.n, s.n_views, err)
    st = serve.latency_stats(mixed)
    print("mixed", st, "plain", serve.latency_stats(alone), flush=True)


def test_served_jobs_match_the_oracle(torch_cuda, oracle_mod):
    """Every job of a served mix (quarter-turn and plain geometries, several
    jobs per grouped step) ends within the SIRT bar of the FP64 oracle's own
    SIRT on the job's data."""
    import numpy as np
    trace = serve.make_trace(8, rate=20000.0, seed=21, sizes=(32, 48, 64), views=(24, 30, 40),
                             iters=10)
    assert {s.n_views % 4 for s in trace} == {0, 2}
    ex = serve.GpuExecutor(keep_inputs=True)
    res = serve.Server(ex, hbm_budget=1 << 30, keep_outputs=True).run(trace)
    assert res.peak_active >= 2 and max(res.batch_sizes) >= 2
    worst = 0.0
    for s in trace:
        og = oracle_mod.Geometry(**s.geometry_kwargs())
        ref = og.sirt(ex.inputs[s.job_id].astype(np.float64), s.iters)
        got = res.outputs[s.job_id].cpu().numpy().astype(np.float64)
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        worst = max(worst, err)
        assert err <= 1e-4, (s.job_id, s.n, s.n_views, err)
    print(f"served jobs vs oracle SIRT-{trace[0].iters}: worst rel-L2 {worst:.3e}", flush=True)


@pytest.mark.parametrize("n,views", [(256, 180), (512, 1440), (1024, 720), (256, 90)])
def test_admission_estimate_bounds_device_memory(torch_cuda, n, views):
    """job_device_bytes bounds what an admitted job holds: its geometry's
    tables and weights, its iterate, sinogram and residual, and the scratch
    of one SIRT step (job_scratch_bytes, equal to the library's own figure)."""
    torch = torch_cuda
    spec = serve.JobSpec(job_id=0, arrival=0.0, n=n, n_views=views, n_det=2 * n, dsc=3.0 * n,
                         dsd=4.5 * n)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    ex = serve.GpuExecutor()
    g, x, y, w = ex.prepare(spec)
    scratch = g.sirt_scratch_bytes(1)
    assert serve.job_scratch_bytes(spec, cus) == scratch
    held = g.device_bytes() + 4 * (x.numel() + y.numel() + w.numel()) + scratch
    est = serve.job_device_bytes(spec, cus)
    print(f"{n}^2 x {views}: estimate {est} bytes, held {held} bytes "
          f"(symmetry order {g.symmetry()})", flush=True)
    assert est >= held
    ex.release((g, x, y, w))
    ex.flush()
