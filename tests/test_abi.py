"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/pdhcg.h, reports the paper's defaults, and rejects invalid
problems during host-side validation (no device work is issued)."""
import ctypes as C
import json
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2608_09159_amd as G
from instances import Problem, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(G.lib_path()):
        from paper_2608_09159_amd import build
        build.build()
    return G.load()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "pdhcg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(pdhcg_\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 9
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(names) == set(G.EXPORTS)


def test_struct_sizes_match_header_layout(lib):
    # pdhcg_settings is filled by the library; a layout mismatch would garble
    # the fields read back here
    s = G.default_settings()
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "practical_defaults.json")))
    assert s.ruiz_iters == gold["ruiz_iters"] and s.pc_alpha == gold["pc_alpha"]
    assert (s.eps_in0, s.gamma_in, s.eps_min) == (gold["eps_in0"], gold["gamma_in"], gold["eps_min"])
    assert (s.beta_s, s.beta_n, s.beta_a) == (gold["beta_s"], gold["beta_n"], gold["beta_a"])
    assert (s.pid_beta_i, s.pid_kp, s.pid_ki, s.pid_kd) == (
        gold["pid_beta_i"], gold["pid_kp"], gold["pid_ki"], gold["pid_kd"])
    assert s.rho == gold["rho"] and s.inner == 0 and s.bound_objective == 1
    assert s.tol == 1e-6 and s.check_every == 64 and s.j_max == 500 and s.power_iters == 128
    assert s.host_poll == 512 and s.verbose == 0


def test_strerror(lib):
    assert lib.pdhcg_strerror(-3) == b"invalid CSR structure"
    assert lib.pdhcg_strerror(1) == b"optimal"
    assert b"gfx950" in lib.pdhcg_version()


def _setup_rc(prob, **kw):
    m = G._Marshalled(prob)
    s = G.default_settings(**kw)
    h = C.c_void_p()
    rc = G.load().pdhcg_setup(C.byref(m.pc), 1, C.byref(s), C.byref(h))
    assert h.value is None
    return rc


def test_rejects_bad_cones(lib):
    p = synth.tiny_nonneg_qp(0)
    bad = Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=p.P, cones=[("nonneg", 0, p.n - 1, 0.0)])
    assert _setup_rc(bad) == -4
    bad = Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=p.P,
                  cones=[("nonneg", 0, 5, 0.0), ("exp", 5, 3, 0.0), ("soc", 8, 0, 0.0)])
    assert _setup_rc(bad) == -4
    bad = Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=p.P,
                  cones=[("pow", 0, 3, 1.5), ("nonneg", 3, p.n - 3, 0.0)])
    assert _setup_rc(bad) == -4


def test_rejects_nonsymmetric_P(lib):
    p = synth.tiny_nonneg_qp(0)
    P = p.P.toarray()
    P[0, 1] += 1.0
    bad = Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=sp.csr_matrix(P), cones=p.cones)
    assert _setup_rc(bad) == -5


def test_rejects_bad_csr(lib):
    p = synth.tiny_nonneg_qp(0)
    m = G._Marshalled(p)
    m.keep[1][0] = p.n + 3            # column index out of range
    s = G.default_settings()
    h = C.c_void_p()
    assert G.load().pdhcg_setup(C.byref(m.pc), 1, C.byref(s), C.byref(h)) == -3


def test_rejects_bad_settings(lib):
    p = synth.tiny_nonneg_qp(0)
    assert _setup_rc(p, tol=0.0) == -1
    assert _setup_rc(p, rho=0.3) == -1
    assert _setup_rc(p, lanes_at=3) == -1
    assert _setup_rc(p, cone_scaling=2) == -1
    assert _setup_rc(p, memory_kind=2) == -1
    assert _setup_rc(p, interleave=3) == -1
    assert _setup_rc(p, interleave=-2) == -1
    # an allocator needs both callbacks
    s = G.default_settings()
    s.dev_alloc = G.TORCH_ALLOC
    m = G._Marshalled(p)
    h = C.c_void_p()
    assert G.load().pdhcg_setup(C.byref(m.pc), 1, C.byref(s), C.byref(h)) == -1


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        G.load(str(tmp_path / "nope.so"))


def test_batch_rejects_invalid_member(lib):
    """A batch is validated instance by instance on the host before any
    device work; one bad member fails the whole setup."""
    good = synth.portfolio(1_000_000, n_assets=60)
    p = synth.tiny_nonneg_qp(0)
    bad = Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=p.P, cones=[("nonneg", 0, p.n - 1, 0.0)])
    ms = [G._Marshalled(q) for q in (good, bad, good)]
    arr = (G.ProblemC * 3)(*[m.pc for m in ms])
    h = C.c_void_p()
    rc = G.load().pdhcg_setup(arr, 3, C.byref(G.default_settings()), C.byref(h))
    assert rc == -4 and h.value is None


def test_batch_binding_needs_two_problems(lib):
    with pytest.raises(ValueError):
        G.setup_batch([synth.tiny_qp(0)])


def test_defaults_of_execution_settings(lib):
    s = G.default_settings()
    assert s.autotune == 1 and s.tune_iters == 64 and s.time_kernels == 0
    assert s.cone_scaling == 0                             # cone-preserving block scaling
    assert s.interleave == G.ORDER["auto"] == 0            # degree order where it applies
    assert s.memory_kind == 0 and not s.dev_alloc and not s.dev_free and not s.alloc_ctx


def test_setup_rejects_invalid_bounds():
    """Host validation of the implementation form: NaN or crossed row
    bounds, a lower endpoint of +inf, and a box block without bounds are
    PDHCG_E_ARG before any device work."""
    import math
    from instances import synth
    base = synth.bounded_qp(0)

    def setup_rc(p):
        m = G._Marshalled(p)
        h = C.c_void_p()
        return G.load().pdhcg_setup(C.byref(m.pc), 1, C.byref(G.default_settings()), C.byref(h))

    for field, idx, val in (("row_lo", 3, math.nan), ("row_lo", 1, 1e9), ("row_lo", 4, math.inf),
                            ("x_lo", 0, 5.0), ("x_hi", 1, -math.inf)):
        p = synth.bounded_qp(0)
        arr = getattr(p, field).copy()
        arr[idx] = val
        setattr(p, field, arr)
        if field == "row_lo" and val == 1e9:
            p.row_hi[idx] = 0.0
        assert setup_rc(p) == -1, (field, idx, val)
    p = synth.bounded_qp(0)
    p.x_lo = p.x_hi = None
    assert setup_rc(p) == -1
    p = synth.bounded_qp(0)
    p.row_hi = None
    assert setup_rc(p) == -1
