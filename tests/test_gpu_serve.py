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
