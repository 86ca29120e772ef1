"""FP64 reference of the warm-start network: a ReLU multilayer perceptron
whose matrix products take BF16 operands.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The paper has no
learned component; this network is project-defined (a learned warm start for
the PDHG solve), so the definitions below are the reference, written out:

* layers l = 1..L with weights W_l (d_{l-1} x d_l) and biases b_l (d_l);
  Z_l = H_{l-1} W_l + b_l,  H_l = relu(Z_l) for l < L,  output Yhat = Z_L;
* every operand of a matrix product is BF16: the input X, the weights W_l,
  the hidden activations H_l and the backward signals dZ_l are rounded to
  the nearest BF16 (ties to even) of their FP32 value; products and sums are
  exact here (FP64), and an FP32 value is first rounded from FP64 to FP32;
* loss: mean squared error (1 / (B d_L)) sum (Yhat - Y)^2 over the batch B;
* gradients: dZ_L = 2 (Yhat - Y) / (B d_L); dW_l = H_{l-1}^T dZ_l;
  db_l = sum over the batch of dZ_l; dZ_{l-1} = (dZ_l W_l^T) * [H_{l-1} > 0];
* Adam (Kingma and Ba, 2015) on FP32 master weights: m = b1 m + (1-b1) g,
  v = b2 v + (1-b2) g^2, W -= lr mhat / (sqrt(vhat) + eps) with
  mhat = m / (1 - b1^t), vhat = v / (1 - b2^t).

Pins (tests/test_oracle_mlp.py): gradients against central finite
differences of the FP64 loss (the BF16 roundings switched off), BF16 rounding
against the bit-level definition, Adam's first step against its closed form
(|update| = lr on every coordinate with a nonzero gradient).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Nearest BF16 value (ties to even) of the FP32 rounding of `a`,
    returned as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = rounded.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out[nan] = np.nan
    return out


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


class MLP:
    """Weights W[l] (d_{l-1} x d_l) and biases b[l], FP64 copies of the FP32
    master values."""

    def __init__(self, Ws, bs):
        self.W = [np.array(w, dtype=np.float64) for w in Ws]
        self.b = [np.array(b, dtype=np.float64) for b in bs]

    @property
    def layers(self):
        return len(self.W)

    def forward(self, X, rounding=True):
        """Returns (Yhat, hs) with hs[l] the BF16 activations H_l (hs[0] = X
        rounded)."""
        rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
        h = rnd(X)
        hs = [h]
        for l in range(self.layers):
            z = h @ rnd(self.W[l]) + self.b[l]
            if l < self.layers - 1:
                h = rnd(f32(np.maximum(z, 0.0)) if rounding else np.maximum(z, 0.0))
                hs.append(h)
            else:
                return (f32(z) if rounding else z), hs

    def loss(self, X, Y, rounding=True):
        yh, _ = self.forward(X, rounding)
        return float(np.mean((yh - np.asarray(Y, dtype=np.float64)) ** 2))

    def gradients(self, X, Y, rounding=True, signals=False):
        """(loss, dW list, db list) by the chain rule of the module docstring;
        with signals=True also the backward signals dZ_l and activations."""
        rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
        Y = np.asarray(Y, dtype=np.float64)
        yh, hs = self.forward(X, rounding)
        B, dL = yh.shape
        loss = float(np.mean((yh - Y) ** 2))
        dz = 2.0 * (yh - (f32(Y) if rounding else Y)) / (B * dL)
        dz = rnd(f32(dz) if rounding else dz)
        dWs = [None] * self.layers
        dbs = [None] * self.layers
        dzs = [None] * self.layers
        for l in range(self.layers - 1, -1, -1):
            dzs[l] = dz
            dWs[l] = hs[l].T @ dz
            dbs[l] = dz.sum(axis=0)
            if l > 0:
                dh = dz @ rnd(self.W[l]).T
                g = dh * (hs[l] > 0)
                dz = rnd(f32(g) if rounding else g)
        if signals:
            return loss, dWs, dbs, dzs, hs
        return loss, dWs, dbs


class Adam:
    def __init__(self, shapes, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros(s) for s in shapes]
        self.v = [np.zeros(s) for s in shapes]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            out.append(p - self.lr * (self.m[i] / c1) / (np.sqrt(self.v[i] / c2) + self.eps))
        return out
