"""The allocation-free projection entry point (pdhcg_project_cones_noalloc)
against pdhcg_project_cones, on device tensors, two calls in a row (the
second with fewer blocks, so stale flags of the first call would show), for
SOC and RSOC with a metric (per-block flags in the static array matter),
EXP with a metric and POW: outputs bit-identical (same kernel, same
flags)."""
import numpy as np
import pytest

import paper_2608_09159_amd as G

pytestmark = pytest.mark.gpu


def _case(rng, kind, count, dim):
    r = rng.standard_normal((count, dim)) * 10.0 ** rng.uniform(-2, 2, (count, 1))
    m = 10.0 ** rng.uniform(-1, 1, (count, dim))
    m[::3] = m[::3, :1]               # every third block has a constant metric
    al = rng.uniform(0.05, 0.95, count) if kind == "pow" else None
    return r, m, al


@pytest.mark.parametrize("kind,dim", [("soc", 20), ("rsoc", 10), ("exp", 3), ("pow", 3)])
def test_noalloc_projection_matches(kind, dim):
    import torch
    rng = np.random.default_rng(7)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    for count in (20000, 7000):
        r, m, al = _case(rng, kind, count, dim)
        # the constant-metric pattern of the second call differs from the first
        if count == 7000:
            m[1::3] = m[1::3, :1]
        ref = G.project_cones(kind, r, m, al)
        rt = torch.from_numpy(r).to(dev)
        mt = torch.from_numpy(m).to(dev)
        at = torch.from_numpy(al).to(dev) if al is not None else None
        out = torch.full_like(rt, float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            G.project_cones_noalloc(kind, rt, out, mt, at, stream=stream)
        stream.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), (kind, count, float(np.nanmax(np.abs(got - ref))))


def test_noalloc_rejects_oversize():
    import torch
    r = torch.zeros((1, 3), dtype=torch.float64, device="cuda:0")
    lib = G.load()
    rc = lib.pdhcg_project_cones_noalloc(2, 3, (1 << 22) + 1, None, r.data_ptr(), None, r.data_ptr(), None)
    assert rc == -1
