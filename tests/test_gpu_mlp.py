"""GPU parity of the warm-start network kernels (BF16 matrix-core GEMMs with
FP32 accumulation, fused bias/ReLU/mask epilogues, MSE gradient, bias
gradients, Adam) against the FP64 reference oracle/mlp.py.

* Exact regime: inputs and weights are small multiples of powers of two, so
  every forward FP32 accumulation is exact (checked on the reference) and
  both sides round the same values to BF16: forward outputs and the loss
  agree bit for bit, which fixes the MFMA operand and result layouts and the
  split-K path; gradients (transposed GEMM variants) within their bound.
* General data: outputs and gradients agree within the FP32-accumulation
  bound K 2^-24 sum|terms| per product, widened by one BF16 step of an
  intermediate activation (a rounding of a hidden value may fall on the
  other side of a BF16 boundary).
* Adam: one step agrees with the reference to FP32 precision wherever the
  gradients agree bit for bit (elsewhere within one step); training a small
  network reduces its loss.
* Full size (51,000 -> 512 -> 512 -> 56,500, batch 256): loss and sampled
  gradient entries of the first and last layer against the reference.
"""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from oracle import mlp as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _exact_case(rng, dims, B):
    Ws = [rng.integers(-2, 3, (a, b)).astype(np.float32) / 8 for a, b in zip(dims[:-1], dims[1:])]
    bs = [rng.integers(-2, 3, b).astype(np.float32) / 4 for b in dims[1:]]
    X = rng.integers(-2, 3, (B, dims[0])).astype(np.float32)
    Y = rng.integers(-8, 9, (B, dims[-1])).astype(np.float32) / 4
    return Ws, bs, X, Y


def _net(dims, B, Ws, bs):
    net = G.MLP(dims, B)
    for l, (W, b) in enumerate(zip(Ws, bs)):
        net.set_params(l, W, b)
    return net


def _exact_precondition(ref, X):
    """Every forward product's |partial sums| stay below 2^24 units of its
    granularity (inputs integers, weights multiples of 1/8, biases of 1/4,
    so layer l's products are multiples of 8^-l), hence FP32 accumulation is
    exact in any order."""
    _, hs = ref.forward(X)
    for l in range(ref.layers):
        terms = np.abs(hs[l]) @ np.abs(M.bf16_round(ref.W[l])) + np.abs(ref.b[l])
        assert terms.max() < 2.0 ** 24 * 8.0 ** -(l + 1), (l, terms.max())


@pytest.mark.parametrize("dims,B", [([40, 72, 24, 32], 16),     # every tile has a ragged edge
                                    ([96, 128, 64, 64], 64),    # whole tiles
                                    ([300, 130, 70, 4], 8)])    # long K (split-K), tiny batch
def test_exact_regime(dims, B):
    """Forward outputs and loss bit-identical (every forward sum is exact);
    gradients within the FP32 accumulation bound plus one BF16 step of the
    backward signals (their FP32 sums need not be exact)."""
    rng = np.random.default_rng(sum(dims) + B)
    Ws, bs, X, Y = _exact_case(rng, dims, B)
    ref = M.MLP(Ws, bs)
    _exact_precondition(ref, X)
    net = _net(dims, B, Ws, bs)
    try:
        yh = net.forward(_dev(X)).cpu().numpy().astype(np.float64)
        loss = net.train_step(_dev(X), _dev(Y), update=False)
        grads = [net.grads(l) for l in range(len(Ws))]
    finally:
        net.free()
    ryh, _ = ref.forward(X)
    np.testing.assert_array_equal(yh, ryh)
    rloss, rdW, rdb, dzs, hs = ref.gradients(X, Y, signals=True)
    assert loss == pytest.approx(rloss, rel=1e-12)
    L = len(Ws)
    for l in range(L):
        scale = np.abs(hs[l]).T @ np.abs(dzs[l])
        err = np.abs(grads[l][0] - rdW[l])
        assert np.all(err <= 2.0 ** -7 * scale + B * 2.0 ** -24 * scale), l
        bscale = np.abs(dzs[l]).sum(axis=0)
        assert np.all(np.abs(grads[l][1] - rdb[l]) <= 2.0 ** -7 * bscale + B * 2.0 ** -24 * bscale), l
        same = float(np.mean(grads[l][0] == rdW[l]))
        print(f"[mlp exact] layer {l}: {same:.4f} of dW entries bit-identical", flush=True)


def _bound_forward(ref, X):
    """Per-output bound: FP32 accumulation of the last product plus one BF16
    step (2^-8 relative) of every hidden activation propagated through the
    later layers' absolute weights."""
    h = np.abs(M.bf16_round(X))
    err = np.zeros_like(h)
    for l in range(ref.layers):
        Wa = np.abs(M.bf16_round(ref.W[l]))
        terms = h @ Wa + np.abs(ref.b[l])
        err = err @ Wa + h.shape[1] * 2.0 ** -24 * terms
        _, hs = ref.forward(X)
        if l < ref.layers - 1:
            h = np.abs(hs[l + 1])
            err = err + 2.0 ** -8 * h + 2.0 ** -8 * err
    return err


def test_general_data_within_bounds():
    rng = np.random.default_rng(5)
    dims, B = [257, 96, 80, 131], 33
    Ws = [(rng.standard_normal((a, b)) / np.sqrt(a)).astype(np.float32) for a, b in zip(dims[:-1], dims[1:])]
    bs = [(0.1 * rng.standard_normal(b)).astype(np.float32) for b in dims[1:]]
    X = rng.standard_normal((B, dims[0])).astype(np.float32)
    Y = rng.standard_normal((B, dims[-1])).astype(np.float32)
    net = _net(dims, B, Ws, bs)
    try:
        yh = net.forward(_dev(X)).cpu().numpy().astype(np.float64)
        loss = net.train_step(_dev(X), _dev(Y), update=False)
        dW0, _ = net.grads(0)
        dWL, dbL = net.grads(len(Ws) - 1)
    finally:
        net.free()
    ref = M.MLP(Ws, bs)
    ryh, hs = ref.forward(X)
    bound = _bound_forward(ref, X)
    assert np.all(np.abs(yh - ryh) <= bound + 1e-30), float(np.max(np.abs(yh - ryh) / (bound + 1e-30)))
    rloss, rdW, rdb = ref.gradients(X, Y)
    assert loss == pytest.approx(rloss, rel=1e-3)
    # last layer: dW = H^T dZ with dZ one BF16 rounding away
    scale = np.abs(hs[-1]).T @ np.abs(M.bf16_round(2 * (ryh - Y) / Y.size))
    assert np.all(np.abs(dWL - rdW[-1]) <= 2.0 ** -7 * scale + 1e-12)
    assert np.abs(dbL - rdb[-1]).max() <= 2.0 ** -7 * np.abs(rdb[-1]).max() + 1e-9
    rel0 = np.linalg.norm(dW0 - rdW[0]) / np.linalg.norm(rdW[0])
    print(f"[mlp] first-layer gradient relative error {rel0:.2e}", flush=True)
    assert rel0 <= 2e-2


def test_adam_step_matches_reference():
    """One Adam step from exact-regime data.  Where the library's gradient
    equals the reference's bit for bit, the updated weights agree to FP32
    rounding; elsewhere (a gradient within rounding of zero can flip the
    normalised step m / sqrt(v)) the difference is at most one step, lr."""
    rng = np.random.default_rng(6)
    dims, B = [300, 130, 70, 4], 8
    Ws, bs, X, Y = _exact_case(rng, dims, B)
    lr = 1e-3
    net = _net(dims, B, Ws, bs)
    try:
        net.train_step(_dev(X), _dev(Y), update=False)
        gW = [net.grads(l) for l in range(len(Ws))]
        net.set_params(0, Ws[0], bs[0])          # resets the step count
        net.train_step(_dev(X), _dev(Y), lr=lr)
        got = [net.get_params(l) for l in range(len(Ws))]
    finally:
        net.free()
    ref = M.MLP(Ws, bs)
    _, dW, db = ref.gradients(X, Y)
    opt = M.Adam([w.shape for w in Ws] + [b.shape for b in bs], lr=lr)
    new = opt.step(ref.W + ref.b, dW + db)
    L = len(Ws)
    for l in range(L):
        for k, (g, r, p) in enumerate(((gW[l][0], dW[l], new[l]), (gW[l][1], db[l], new[L + l]))):
            same = g.astype(np.float64) == r
            diff = np.abs(got[l][k] - p)
            tight = 2e-7 * np.abs(p) + 1e-6 * lr
            assert np.all(diff[same] <= tight[same]), (l, k)
            assert np.all(diff <= lr * (1 + 1e-6) + tight), (l, k)
        print(f"[mlp adam] layer {l}: {np.mean(gW[l][0] == dW[l]):.4f} of gradients bit-identical",
              flush=True)


def test_training_reduces_loss():
    rng = np.random.default_rng(8)
    dims, B = [64, 48, 48, 32], 64
    X = rng.standard_normal((B, dims[0])).astype(np.float32)
    T = (np.tanh(X[:, :32]) * 0.5).astype(np.float32)
    Ws = [(rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32) for a, b in zip(dims[:-1], dims[1:])]
    bs = [np.zeros(b, np.float32) for b in dims[1:]]
    net = _net(dims, B, Ws, bs)
    try:
        losses = [net.train_step(_dev(X), _dev(T), lr=3e-3) for _ in range(200)]
    finally:
        net.free()
    print(f"[mlp train] loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.2 * losses[0]


def test_full_size_step():
    """The warm-start network at its full size on one batch of 256."""
    dims, B = [51000, 512, 512, 56500], 256
    rng = np.random.default_rng(7)
    Ws = [(rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32)
          for a, b in zip(dims[:-1], dims[1:])]
    bs = [np.zeros(b, np.float32) for b in dims[1:]]
    X = rng.standard_normal((B, dims[0])).astype(np.float32)
    Y = rng.standard_normal((B, dims[-1])).astype(np.float32)
    net = _net(dims, B, Ws, bs)
    try:
        loss = net.train_step(_dev(X), _dev(Y), update=False)
        dW0, db0 = net.grads(0)
        dW2, db2 = net.grads(2)
    finally:
        net.free()
    ref = M.MLP(Ws, bs)
    rloss, rdW, rdb = ref.gradients(X, Y)
    print(f"[mlp full] loss gpu {loss:.6f} ref {rloss:.6f}", flush=True)
    assert loss == pytest.approx(rloss, rel=1e-3)
    for g, r in ((dW0, rdW[0]), (dW2, rdW[2]), (db0, rdb[0]), (db2, rdb[2])):
        rel = np.linalg.norm(g - r) / np.linalg.norm(r)
        assert rel <= 2e-2, rel
