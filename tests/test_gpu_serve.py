"""Serving loop (continuous batching): requests arriving while others run are
admitted into batch slots as slots and device memory free up, their rounds
overlap with the others' on the device, and each result is bit for bit the
same as the same request propagated alone (its class's plan, the same step).
Run once with room for every class and once with a memory budget that holds a
single batch, so that requests wait and batches are released and re-created."""
import numpy as np
import pytest

from paper_1708_05324_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05324_amd import gmmpa
    gmmpa.load_library()
    return torch


@pytest.mark.parametrize("tight,max_groups,length_scale", [(False, 3, 0.002), (True, 3, 0.002), (False, 7, 5e-4)],
                         ids=["room", "tight", "to_28_modes"])
def test_served_results_equal_alone(torch_gpu, tight, max_groups, length_scale):
    """The third stream reaches 28 modes: classes of 21 and 28 modes run on the
    wide rank-r route beside classes of the other routes."""
    from paper_1708_05324_amd import gmmpa, serve
    torch = torch_gpu
    reqs = synth.request_stream(seed=9, count=10, rate=3000.0, max_groups=max_groups, length_scale=length_scale)
    srv = serve.Server(precision="bf16x3", slots=2, keep_fields=True)
    srv.prepare(reqs)
    if tight:   # room for the largest single batch only
        srv.budget_bytes = max(srv._estimate((r.groups, r.nt)) for r in reqs) + (1 << 20)
    out, summary = srv.run(reqs, realtime=True)
    print(f"[tight={tight}] {summary}", flush=True)
    assert sorted(out) == [r.idx for r in reqs]
    assert summary["not_ok"] == 0
    if tight:   # admission kept the batches alive within the budget
        assert summary["peak_device_bytes"] <= srv.budget_bytes
    for r in reqs:
        s = out[r.idx]
        w = srv.template((r.groups, r.nt))
        plan = gmmpa.plan_from_workload(w, precision="bf16x3", tol=serve.TOL["bf16x3"], max_iter=30)
        A0 = torch.from_numpy(r.A0).to(device="cuda", dtype=torch.complex64)
        alone = plan.propagate(A0, r.L, serve.step_for(r, w), srv.M)
        got, ref = s.field.cpu().numpy(), alone.field.cpu().numpy()
        assert s.admitted >= s.arrival - 1e-9 and s.completed >= s.admitted
        assert np.array_equal(got, ref), r.idx
        assert s.stats["iterations"] == alone.stats["iterations"]
        assert s.stats["small_steps"] == alone.stats["small_steps"]
        plan.close()
    srv.close()
