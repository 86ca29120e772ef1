"""CPU checks of the host setup's device coordinate order (settings.interleave,
PDHCG_ORDER_*): the library's host code (host_setup.cpp, compiled here with
g++ and a small probe) against the order recomputed from its stated rule
(parity_util.degree_order_rule), on the large sparse QP family (power-law
column degrees, slack columns, sparse P) at n = 2e5; and every array the
setup computes compared byte for byte between 1 and 8 host threads."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from instances import synth
from parity_util import degree_order_rule

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2608_09159_amd", "csrc")
CODES = {"free": 0, "nonneg": 1}      # PDHCG_CONE_FREE, PDHCG_CONE_NONNEG

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("probe") / "host_order_probe")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(HERE, "host_order_probe.cpp"), os.path.join(CSRC, "host_setup.cpp"),
                    "-o", exe], check=True)
    return exe


@pytest.fixture(scope="module")
def problem(tmp_path_factory):
    p = synth.large_sparse_qp(seed=3, n=200_000, m=100_000)
    d = tmp_path_factory.mktemp("problem")
    A, P = p.A, p.P
    A.indptr.astype(np.int64).tofile(d / "A_ptr"); A.indices.astype(np.int32).tofile(d / "A_col")
    A.data.astype(np.float64).tofile(d / "A_val")
    P.indptr.astype(np.int64).tofile(d / "P_ptr"); P.indices.astype(np.int32).tofile(d / "P_col")
    P.data.astype(np.float64).tofile(d / "P_val")
    p.b.tofile(d / "b"); p.c.tofile(d / "c")
    np.array([CODES[k] for k, _, _, _ in p.cones], dtype=np.int32).tofile(d / "cone_type")
    np.array([st for _, st, _, _ in p.cones], dtype=np.int32).tofile(d / "cone_start")
    np.array([dim for _, _, dim, _ in p.cones], dtype=np.int32).tofile(d / "cone_dim")
    return p, str(d)


OUTPUTS = ("perm", "A_out_ptr", "A_out_col", "A_out_val", "AT_out_ptr", "AT_out_col", "AT_out_val",
           "P_out_ptr", "P_out_col", "P_out_val", "Sx_out", "Sy_out", "b_out", "c_out", "qdiag_out", "nu_out")


def _run(probe, d, order, threads=None):
    env = dict(os.environ)
    if threads is not None:
        env["PDHCG_HOST_THREADS"] = str(threads)
    out = subprocess.run([probe, d, str(order)], check=True, capture_output=True, text=True,
                         env=env).stdout.split()
    perm = np.fromfile(os.path.join(d, "perm"), dtype=np.int32)
    ptr = np.fromfile(os.path.join(d, "A_out_ptr"), dtype=np.int64)
    col = np.fromfile(os.path.join(d, "A_out_col"), dtype=np.int32)
    return int(out[0]), int(out[1]), perm, ptr, col


def test_degree_order_follows_its_rule(probe, problem):
    p, d = problem
    rc, head, perm, ptr, col = _run(probe, d, 2)            # PDHCG_ORDER_DEGREE
    assert rc == 0
    want, want_head = degree_order_rule(p)
    print(f"[host order] n={p.n} head {head} rows", flush=True)
    assert head == want_head and head > 0
    assert np.array_equal(perm, want.astype(np.int32))
    # A's columns renumbered by the order, each row still sorted
    inv = np.empty(p.n, dtype=np.int64)
    inv[want] = np.arange(p.n)
    assert np.array_equal(ptr, p.A.indptr)
    for l in range(0, p.m, 997):
        got = col[ptr[l]:ptr[l + 1]]
        assert np.array_equal(got, np.sort(inv[p.A.indices[p.A.indptr[l]:p.A.indptr[l + 1]]])), l


def test_caller_and_auto_orders_keep_small_problems_in_place(probe, problem):
    p, d = problem
    for order in (-1, 0):                                    # CALLER; AUTO below n = 2^20
        rc, head, perm, ptr, col = _run(probe, d, order)
        assert rc == 0 and head == 0 and perm.size == 0
        assert np.array_equal(col, p.A.indices)


@pytest.mark.parametrize("order", [2, -1])
def test_setup_is_bit_identical_for_any_thread_count(probe, problem, order):
    """The host setup's threaded loops (scaling maxima, powers, renumbering,
    transpose) give the same bytes on 1 thread and on 8."""
    p, d = problem
    got = {}
    for threads in (1, 8):
        assert _run(probe, d, order, threads)[0] == 0
        got[threads] = {f: open(os.path.join(d, f), "rb").read() for f in OUTPUTS}
    for f in OUTPUTS:
        assert got[1][f] == got[8][f], f
    assert len(got[1]["AT_out_col"]) == 4 * p.A.nnz
