"""GPU tests of the C-ABI boundary options: device-resident inputs and
outputs (memory_kind = PDHCG_MEM_DEVICE, torch CUDA tensors), the caller's
device allocator (torch's caching allocator through dev_alloc / dev_free),
and the dual slack s = Q x + c - A^T y computed on the device.

Device and host memory kinds run the same kernels on the same data, so
their results must agree bit for bit; s is checked against its definition
evaluated on the CPU at the returned point."""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from parity_util import edge_cone_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _slack_cpu(p, x, y):
    q = np.zeros(p.n)
    if p.P is not None:
        q += p.P @ x
    if p.R is not None:
        D = p.D if p.D is not None else np.eye(p.R.shape[0])
        q += p.R.T @ (D @ (p.R @ x))
    return q + p.c - p.A.T @ y


def _host(t):
    return t.cpu().numpy() if hasattr(t, "cpu") else t


@pytest.mark.parametrize("make,kw", [(lambda: synth.tiny_mixed(4), {}),
                                     (lambda: synth.mixed_cone_scaled(seed=3, scale=0.02), {"interleave": 1}),
                                     (lambda: synth.tiny_qp(2), {"grid_dim": 1}),
                                     (lambda: synth.bounded_qp(seed=3), {})],
                         ids=["mixed", "interleaved", "one_workgroup", "bounded"])
def test_device_memory_matches_host(make, kw):
    p = make()
    print(f"[device io] {p.name} {kw}", flush=True)
    gh = G.solve(p, want_s=True, **kw)
    gd = G.solve(p, want_s=True, memory_kind="device", **kw)
    for key in ("x", "y", "s"):
        assert isinstance(gd[key], torch.Tensor) and gd[key].is_cuda, key
        assert np.array_equal(_host(gd[key]), gh[key]), key
    for key in ("status", "iterations", "inner_iterations", "restarts", "primal_obj", "dual_obj"):
        assert gd[key] == gh[key], key
    s = _slack_cpu(p, gh["x"], gh["y"])
    np.testing.assert_allclose(gh["s"], s, rtol=1e-9, atol=1e-11 * max(1.0, np.abs(s).max()))


def test_device_warm_start_matches_host():
    p = synth.tiny_mixed(5)
    g0 = G.solve(p, tol=1e-4)
    x0, y0 = g0["x"] * 1.01, g0["y"] * 0.99
    gh = G.solve(p, x0=x0, y0=y0)
    gd = G.solve(p, x0=torch.from_numpy(x0).cuda(), y0=torch.from_numpy(y0).cuda(), memory_kind="device")
    assert gd["iterations"] == gh["iterations"]
    assert np.array_equal(_host(gd["x"]), gh["x"])
    assert np.array_equal(_host(gd["y"]), gh["y"])


def test_torch_allocator():
    """The handle's device memory comes from torch's caching allocator: it
    shows in torch's accounting while the handle lives and goes back at
    pdhcg_free; results equal those of hipMalloc'd buffers."""
    p = synth.mixed_cone_scaled(seed=4, scale=0.05)
    ref = G.solve(p, want_s=True)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    h = G.setup(p, allocator="torch")
    during = torch.cuda.memory_allocated()
    try:
        g = h.solve(want_s=True)
    finally:
        h.free()
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated()
    print(f"[torch allocator] before {before} during {during} after {after}", flush=True)
    assert during - before > 8 * p.A.nnz            # at least A's values and columns
    assert after == before
    for key in ("x", "y", "s"):
        assert np.array_equal(g[key], ref[key]), key


def test_batch_device_memory_and_allocator():
    ps = [synth.tiny_mixed(4), edge_cone_problem(2), synth.tiny_qp(1),
          synth.portfolio(1_000_100, n_assets=120)]
    # autotune off: the autotuner times candidate lane mappings, and two
    # setups may pick different ones (different rounding)
    rh = G.setup_batch(ps, autotune=0).solve(want_s=True)
    h = G.setup_batch(ps, memory_kind="device", allocator="torch", autotune=0)
    try:
        x0s = [torch.from_numpy(r["x"]).cuda() if i % 2 == 0 else None for i, r in enumerate(rh)]
        rd = h.solve(want_s=True)
        rw = h.solve(x0s=x0s, want_s=True)
    finally:
        h.free()
    for i, p in enumerate(ps):
        for key in ("x", "y", "s"):
            assert np.array_equal(_host(rd[i][key]), rh[i][key]), (i, key)
        s = _slack_cpu(p, rh[i]["x"], rh[i]["y"])
        np.testing.assert_allclose(rh[i]["s"], s, rtol=1e-9, atol=1e-11 * max(1.0, np.abs(s).max()))
        assert rw[i]["status"] == "OPTIMAL"
        if i % 2 == 0:           # device warm start: the primal solution, scaled on the device
            assert rw[i]["rel_primal"] <= 1e-6
