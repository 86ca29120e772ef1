"""Learned warm start for a parametric family of problems.

The paper has no learned component; this is the library's own production
pattern.  For a family of problems that differ only in their parameters, a
network maps the parameters to the solver's primal-dual solution; its
prediction seeds pdhcg_solve, which still runs to the same tolerance, so the
plain cold-started method remains the fallback and sets the accuracy.

Family: the quasilinear Fisher market in exponential-cone form on a fixed
valuation graph (buyers x goods, edges E).  An instance is (u on E, budgets
w).  Features: standardised (log u, log w).  Targets: the standardised
unscaled primal-dual solution (x*, y*) of the solver at the tolerance.

Training runs on the GPU through the library's network kernels
(pdhcg_mlp_*: BF16 matrix-core GEMMs, FP32 master weights, Adam); labels come
from batched solves (pdhcg_solve_batch).  This module only moves data and
drives those calls.
"""
from __future__ import annotations

import time

import numpy as np

from . import MLP, setup, setup_batch


class Standardizer:
    """Per-column affine map to zero mean and unit standard deviation
    (columns with a tiny spread keep unit scale)."""

    def __init__(self, A):
        A = np.asarray(A, dtype=np.float64)
        self.mean = A.mean(axis=0)
        sd = A.std(axis=0)
        self.std = np.where(sd > 1e-8 * max(float(sd.max(initial=0.0)), 1e-300), sd, 1.0)

    def apply(self, A):
        return ((np.asarray(A, dtype=np.float64) - self.mean) / self.std).astype(np.float32)

    def invert(self, Z):
        return np.asarray(Z, dtype=np.float64) * self.std + self.mean


class FisherFamily:
    """Fisher markets on one valuation graph (instances.synth.fisher).
    spread=None: independent lognormal valuations and budgets per instance;
    spread=s: lognormal perturbations of one base market (smooth solution
    map)."""

    def __init__(self, n_buyers=1000, n_goods=500, density=0.1, graph_seed=0, spread=None):
        from instances import synth
        self._synth = synth
        self.n_buyers, self.n_goods, self.density, self.spread = n_buyers, n_goods, density, spread
        self.graph = synth.fisher_graph(n_buyers, n_goods, density, graph_seed)

    def instance(self, seed):
        return self._synth.fisher(seed=seed, n_buyers=self.n_buyers, n_goods=self.n_goods,
                                  density=self.density, graph=self.graph, spread=self.spread)

    @staticmethod
    def features(prob):
        return np.concatenate([np.log(prob.meta["u"]), np.log(prob.meta["w"])])


def solve_family(probs, chunk=256, x0s=None, y0s=None, log=None, **settings):
    """Batched solves of `probs` (pdhcg_solve_batch, `chunk` instances per
    launch); returns the list of result dicts.  log(msg), when given, hears
    of every launch."""
    out = []
    for s in range(0, len(probs), chunk):
        if log and s > 0:
            log(f"solved {s} of {len(probs)}")
        part = probs[s:s + chunk]
        xs = None if x0s is None else x0s[s:s + chunk]
        ys = None if y0s is None else y0s[s:s + chunk]
        if len(part) == 1:
            h = setup(part[0], **settings)
            try:
                out.append(h.solve(xs[0] if xs else None, ys[0] if ys else None))
            finally:
                h.free()
            continue
        h = setup_batch(part, **settings)
        try:
            out.extend(h.solve(xs, ys))
        finally:
            h.free()
    return out


class WarmStartModel:
    """Network plus the feature and target standardisations."""

    def __init__(self, feat_std, targ_std, n, hidden=(512, 512), max_batch=256, stream=None):
        self.fs, self.ts, self.n = feat_std, targ_std, n
        self.dims = [feat_std.mean.size, *hidden, targ_std.mean.size]
        self.max_batch = max_batch
        self.net = MLP(self.dims, max_batch, stream)

    def init_params(self, seed=0):
        """He-normal weights, zero biases (drawn on the host from `seed`)."""
        rng = np.random.default_rng(seed)
        for l, (a, b) in enumerate(zip(self.dims[:-1], self.dims[1:])):
            W = (rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).astype(np.float32)
            self.net.set_params(l, W, np.zeros(b, np.float32))

    def train(self, F, T, epochs=30, batch=256, lr=1e-3, seed=0, log=None):
        """F: raw features (N x d_in), T: raw targets (N x d_out).  Returns
        the mean loss of every epoch and the GEMM FLOP count."""
        import torch
        Xd = torch.from_numpy(self.fs.apply(F)).cuda()
        Yd = torch.from_numpy(self.ts.apply(T)).cuda()
        N = Xd.shape[0]
        rng = np.random.default_rng(seed)
        hist = []
        nb = 0
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(N)).cuda()
            tot = 0.0
            cnt = 0
            for s in range(0, N - batch + 1 if N >= batch else 1, batch):
                idx = perm[s:s + batch]
                xb = Xd.index_select(0, idx).contiguous()
                yb = Yd.index_select(0, idx).contiguous()
                tot += self.net.train_step(xb, yb, lr=lr) * xb.shape[0]
                cnt += xb.shape[0]
                nb += xb.shape[0]
            hist.append(tot / max(cnt, 1))
            if log:
                log(f"epoch {ep + 1}/{epochs}: loss {hist[-1]:.5f}")
        flops = 6.0 * nb * sum(a * b for a, b in zip(self.dims[:-1], self.dims[1:]))
        return hist, flops

    def predict(self, F):
        """Raw features (k x d_in) -> list of (x0, y0) in the original space."""
        import torch
        F = np.atleast_2d(F)
        X = torch.from_numpy(self.fs.apply(F)).cuda()
        out = []
        for s in range(0, X.shape[0], self.max_batch):
            Z = self.net.forward(X[s:s + self.max_batch].contiguous()).cpu().numpy()
            P = self.ts.invert(Z)
            out.extend((p[:self.n], p[self.n:]) for p in P)
        return out

    def free(self):
        self.net.free()


def build_and_train(family, train_seeds, tol=1e-6, epochs=30, batch=256, lr=1e-3, hidden=(512, 512),
                    seed=0, log=None):
    """Label `train_seeds` with the solver, fit the standardisations and train
    the network.  Returns (model, info)."""
    t0 = time.perf_counter()
    probs = [family.instance(s) for s in train_seeds]
    res = solve_family(probs, tol=tol, log=log)
    t_label = time.perf_counter() - t0
    F = np.stack([family.features(p) for p in probs])
    T = np.stack([np.concatenate([r["x"], r["y"]]) for r in res])
    model = WarmStartModel(Standardizer(F), Standardizer(T), probs[0].n, hidden, batch)
    model.init_params(seed)
    t0 = time.perf_counter()
    hist, flops = model.train(F, T, epochs=epochs, batch=batch, lr=lr, seed=seed, log=log)
    import torch
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    info = dict(train_instances=len(probs), label_s=t_label, train_s=t_train, loss=hist,
                train_tflops=flops / t_train / 1e12,
                label_statuses={s: sum(r["status"] == s for r in res) for s in {r["status"] for r in res}},
                label_iterations_median=float(np.median([r["iterations"] for r in res])))
    return model, info


def evaluate(model, family, seeds, tol=1e-6, timed=None, log=None):
    """Cold and warm solves of the held-out `seeds`.  Iterations for all of
    them (batched solves); wall time, network inference included, for the
    first `timed` seeds with single solves."""
    probs = [family.instance(s) for s in seeds]
    F = np.stack([family.features(p) for p in probs])
    preds = model.predict(F)
    cold = solve_family(probs, tol=tol, log=log)
    warm = solve_family(probs, tol=tol, x0s=[p[0] for p in preds], y0s=[p[1] for p in preds], log=log)
    ic = np.array([r["iterations"] for r in cold], float)
    iw = np.array([r["iterations"] for r in warm], float)
    out = dict(instances=len(probs),
               cold_iterations_median=float(np.median(ic)), cold_iterations_p90=float(np.percentile(ic, 90)),
               warm_iterations_median=float(np.median(iw)), warm_iterations_p90=float(np.percentile(iw, 90)),
               frac_warm_more_iterations=float(np.mean(iw > ic)),
               statuses_cold={s: sum(r["status"] == s for r in cold) for s in {r["status"] for r in cold}},
               statuses_warm={s: sum(r["status"] == s for r in warm) for s in {r["status"] for r in warm}})
    if timed:
        import torch
        tc, tw = [], []
        for p, f in zip(probs[:timed], F[:timed]):
            h = setup(p, tol=tol)
            try:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h.solve()
                tc.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
                x0, y0 = model.predict(f[None, :])[0]
                h.solve(x0, y0)
                tw.append(time.perf_counter() - t0)
            finally:
                h.free()
        tc, tw = np.array(tc), np.array(tw)
        out.update(timed_instances=len(tc), cold_time_median_s=float(np.median(tc)),
                   cold_time_p90_s=float(np.percentile(tc, 90)), warm_time_median_s=float(np.median(tw)),
                   warm_time_p90_s=float(np.percentile(tw, 90)), frac_warm_slower=float(np.mean(tw > tc)),
                   speedup_median=float(np.median(tc) / np.median(tw)))
    return out
