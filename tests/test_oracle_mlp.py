"""Pins for the warm-start network reference (oracle/mlp.py): BF16 rounding
against its bit-level definition, the chain-rule gradients against central
finite differences of the loss, and Adam's first step against its closed
form."""
import struct

import numpy as np

from oracle import mlp as M


def _bf16_by_hand(x):
    """Round-to-nearest-even of an FP32 to BF16 through its bit pattern."""
    (bits,) = struct.unpack("<I", struct.pack("<f", np.float32(x)))
    keep = bits >> 16
    rest = bits & 0xFFFF
    if rest > 0x8000 or (rest == 0x8000 and (keep & 1)):
        keep += 1
    (val,) = struct.unpack("<f", struct.pack("<I", (keep << 16) & 0xFFFFFFFF))
    return val


def test_bf16_round_matches_definition():
    rng = np.random.default_rng(0)
    xs = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.uniform(-20, 20, 2000),
                         [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 255.5, 256.5, 3.0e38]])
    got = M.bf16_round(xs)
    for x, g in zip(xs, got):
        assert g == _bf16_by_hand(x), (x, g)
    # values with 8 significant bits are fixed points
    exact = np.array([1.0, 1.5, -0.375, 2.0 ** -100, 96.0])
    np.testing.assert_array_equal(M.bf16_round(exact), exact)


def _net(rng, dims):
    Ws = [rng.standard_normal((a, b)) / np.sqrt(a) for a, b in zip(dims[:-1], dims[1:])]
    bs = [0.1 * rng.standard_normal(b) for b in dims[1:]]
    return M.MLP(Ws, bs)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    dims = [7, 9, 6, 5]
    net = _net(rng, dims)
    X = rng.standard_normal((4, dims[0]))
    Y = rng.standard_normal((4, dims[-1]))
    loss, dWs, dbs = net.gradients(X, Y, rounding=False)
    assert loss == net.loss(X, Y, rounding=False)
    h = 1e-6
    for l in range(net.layers):
        for (i, j) in [(0, 0), (dims[l] - 1, dims[l + 1] - 1), (2, 3)]:
            w0 = net.W[l][i, j]
            net.W[l][i, j] = w0 + h
            fp = net.loss(X, Y, rounding=False)
            net.W[l][i, j] = w0 - h
            fm = net.loss(X, Y, rounding=False)
            net.W[l][i, j] = w0
            fd = (fp - fm) / (2 * h)
            assert abs(fd - dWs[l][i, j]) <= 1e-7 * max(1.0, abs(fd)), (l, i, j, fd, dWs[l][i, j])
        for j in [0, dims[l + 1] - 1]:
            b0 = net.b[l][j]
            net.b[l][j] = b0 + h
            fp = net.loss(X, Y, rounding=False)
            net.b[l][j] = b0 - h
            fm = net.loss(X, Y, rounding=False)
            net.b[l][j] = b0
            fd = (fp - fm) / (2 * h)
            assert abs(fd - dbs[l][j]) <= 1e-7 * max(1.0, abs(fd)), (l, j)


def test_rounded_forward_uses_bf16_operands():
    """With operands already BF16 and small integer data, the rounded forward
    equals the exact forward (every product and sum is representable)."""
    rng = np.random.default_rng(2)
    dims = [6, 5, 4]
    Ws = [rng.integers(-2, 3, (a, b)).astype(float) / 8 for a, b in zip(dims[:-1], dims[1:])]
    bs = [rng.integers(-2, 3, b).astype(float) / 4 for b in dims[1:]]
    net = M.MLP(Ws, bs)
    X = rng.integers(-2, 3, (3, dims[0])).astype(float)
    a, _ = net.forward(X, rounding=True)
    b, _ = net.forward(X, rounding=False)
    np.testing.assert_array_equal(a, b)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = [rng.standard_normal((3, 4))]
    g = [rng.standard_normal((3, 4))]
    g[0][1, 2] = 0.0
    opt = M.Adam([x.shape for x in p], lr=1e-3)
    q = opt.step(p, g)
    d = q[0] - p[0]
    # first step: mhat = g, vhat = g^2, update = -lr g / (|g| + eps)
    expect = -1e-3 * g[0] / (np.abs(g[0]) + 1e-8)
    np.testing.assert_allclose(d, expect, rtol=1e-12, atol=1e-18)
    assert d[1, 2] == 0.0
