"""Learned surrogate of the cell problem with FFT fallback.

For one fixed microstructure (like the paper's surrogate, Sec. 3: trained
per microstructure, evaluated with macroscopic inputs only), a network maps
the macroscopic inputs of one load increment to the effective outputs:

  inputs (32):  E^{n+1} (6, Mandel), theta^{n+1}, log10 dt,
                summary of the macroscopic history: E^n (6), <sigma>^n (6),
                E^{n-1} (6), theta^n, <D_diss>^n, int <D_diss> dt, grad theta (3)
  outputs (10): <sigma>^{n+1} (6, Mandel), <q> (3), <D_diss>^{n+1}

Every summary entry is macroscopic and observable, so a two-scale code can
roll the summary forward from the surrogate's own outputs. Training data come
from the batched FFT solver; two independently seeded networks are trained,
and their disagreement on the stress decides, row by row, whether the mean
prediction is accepted or the FFT solver is asked instead.

Error measure: per increment, |<sigma>_net - <sigma>_FFT| / max_t |<sigma>_FFT|
over the history (the normalization of the paper's error measure, Sec. 5.4).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import hom
from . import workloads as W

N_IN = 32
N_OUT = 10
SQ2 = math.sqrt(2.0)
MANDEL_W = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


def microstructure(n=32, seed=5):
    """The fixed 32^3 RSA sphere microstructure (radius n/8, fraction 0.20)."""
    img, rec = W.rsa_spheres(n, seed, (n / 8.0, n / 8.0), 0.20)
    return img, rec


def histories(count, seed, steps=5):
    """Proportional strain / temperature histories (see workloads.batch_problem):
    returns strain [count, steps, 6] (tensor components), theta [count, steps],
    dt [count], grad [count, 3]."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(count, 6))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    amp = rng.uniform(0.0, 0.015, size=count)
    e_full = amp[:, None] * d / MANDEL_W[None, :]
    dT = rng.uniform(0.0, 80.0, size=count)
    dt = np.exp(rng.uniform(math.log(0.006), math.log(6.0), size=count))
    grad = rng.normal(size=(count, 3))
    k = np.arange(1, steps + 1) / steps
    strain = e_full[:, None, :] * k[None, :, None]
    theta = 293.15 + dT[:, None] * k[None, :]
    return dict(strain=strain, theta=theta, dt=dt, grad=grad)


def solve_histories(img, hist, chunk=1000, precision=hom.FP32, tol=1e-6, predictor=1):
    """Run every history through the batched FFT solver (with the predictor
    start unless predictor = 0). Returns stress [count, steps, 6] (Mandel),
    flux [count, steps, 3], dissipation [count, steps], elapsed seconds and
    the number of point updates."""
    count, steps = hist["theta"].shape
    laws = [W.pa66(), W.e_glass()]
    stress = np.zeros((count, steps, 6))
    flux = np.zeros((count, steps, 3))
    diss = np.zeros((count, steps))
    status = np.zeros((count, steps), dtype=int)
    elapsed = 0.0
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        b = hom.Batch([img] * (c1 - c0), laws, scheme=hom.SCHEME_NEWTON_CG, precision=precision, tol=tol,
                      predictor=predictor)
        for k in range(steps):
            t0 = time.perf_counter()
            res = b.solve_increment(hist["strain"][c0:c1, k], hist["theta"][c0:c1, k], hist["grad"][c0:c1],
                                    hist["dt"][c0:c1])
            elapsed += time.perf_counter() - t0
            for i, r in enumerate(res):
                stress[c0 + i, k] = np.asarray(r["stress"]) * MANDEL_W
                flux[c0 + i, k] = r["heat_flux"]
                diss[c0 + i, k] = r["dissipation"]
                status[c0 + i, k] = r["status"]
        b.close()
    return dict(stress=stress, flux=flux, dissipation=diss, status=status, seconds=elapsed,
                updates=count * steps)


def features(hist, sol):
    """Rows (history, increment): inputs X [rows, 32], targets Y [rows, 10],
    per-row stress normalization max_t |<sigma>| of the history, history id."""
    strain = hist["strain"] * MANDEL_W[None, None, :]
    theta, dt, grad = hist["theta"], hist["dt"], hist["grad"]
    count, steps = theta.shape
    X = np.zeros((count, steps, N_IN))
    Y = np.zeros((count, steps, N_OUT))
    # layout: 0-5 E^{n+1}, 6 theta^{n+1}, 7 log10 dt, 8-13 E^n, 14-19 <sigma>^n,
    # 20-25 E^{n-1}, 26 theta^n, 27 <D_diss>^n, 28 int <D_diss> dt, 29-31 grad theta
    for k in range(steps):
        X[:, k, 0:6] = strain[:, k]
        X[:, k, 6] = theta[:, k]
        X[:, k, 7] = np.log10(dt)
        X[:, k, 26] = 293.15
        if k >= 1:
            X[:, k, 8:14] = strain[:, k - 1]
            X[:, k, 14:20] = sol["stress"][:, k - 1]
            X[:, k, 26] = theta[:, k - 1]
            X[:, k, 27] = sol["dissipation"][:, k - 1]
            X[:, k, 28] = (sol["dissipation"][:, :k] * dt[:, None]).sum(axis=1)
        if k >= 2:
            X[:, k, 20:26] = strain[:, k - 2]
        X[:, k, 29:32] = grad
        Y[:, k, 0:6] = sol["stress"][:, k]
        Y[:, k, 6:9] = sol["flux"][:, k]
        Y[:, k, 9] = sol["dissipation"][:, k]
    denom = np.linalg.norm(sol["stress"], axis=2).max(axis=1)
    hid = np.repeat(np.arange(count), steps)
    return (X.reshape(-1, N_IN).astype(np.float32), Y.reshape(-1, N_OUT).astype(np.float32),
            np.repeat(denom, steps), hid)


def stress_errors(y_pred, y_true, denom):
    return np.linalg.norm(y_pred[:, :6] - y_true[:, :6], axis=1) / np.maximum(denom, 1e-12)


class Surrogate:
    """Independently seeded networks (eight by default) with a calibrated
    acceptance threshold on their spread."""

    def __init__(self, seeds=tuple(range(8))):
        self.nets = [hom.MLP(N_IN, N_OUT, seed=s) for s in seeds]
        self.threshold = None
        self.floor = 1.0  # MPa: stress scale below which the spread is taken absolute

    # gate inputs of the polynomial skip: log10 dt, theta^{n+1}, theta^n
    GATES = (7, 6, 26)

    def fit(self, X, Y, denom=None, epochs=150, batch=256, lr=2e-3, seed=0):
        """Least-squares gated polynomial skip (fixed, fitted by the library),
        networks trained on the residual. With denom (each row's error
        normalization, max_t |<sigma>| of its history) the rows are weighted by
        1 / denom^2, so the loss is the squared relative error that decides
        acceptance (denominators below `floor` count as `floor`). Returns
        the per-epoch losses."""
        lw = np.ones(N_OUT, dtype=np.float32)
        lw[:6] = 4.0          # the stress is the accuracy target
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        rw = None
        if denom is not None:
            rw = (1.0 / np.maximum(np.asarray(denom, dtype=np.float64), self.floor) ** 2).astype(np.float32)
        # the networks are independent: one host thread each (the library
        # releases the interpreter and trains each network on its own stream)
        from concurrent.futures import ThreadPoolExecutor

        def one(i):
            net = self.nets[i]
            net.fit_skip(X, Y, self.GATES, lw, rw)
            return net.train(X, Y, epochs=epochs, batch=batch, lr=lr, seed=seed + 17 * i, row_weight=rw)

        with ThreadPoolExecutor(max_workers=len(self.nets)) as pool:
            losses = list(pool.map(one, range(len(self.nets))))
        # the method without the network: same skip, network output held at zero
        self.skip_net = hom.MLP(N_IN, N_OUT, seed=0)
        self.skip_net.fit_skip(X, Y, self.GATES, lw, rw)
        self.skip_net.set_params(np.zeros(self.skip_net.param_count, dtype=np.float32))
        return losses

    def skip_only(self, X):
        """Prediction of the fixed skip alone (the method without the network)."""
        return self.skip_net.forward(np.ascontiguousarray(X, dtype=np.float32))

    def infer(self, X_dev):
        """Device tensor [n, 32] -> (y, spread, accept) device tensors."""
        thr = self.threshold if self.threshold is not None else 0.0
        return hom.mlp_ensemble_infer(self.nets, X_dev, thr, self.floor)

    def calibrate(self, X, Y, denom, target=1e-3, quantile=1.0):
        """Largest spread threshold under which the accepted validation rows all
        (or the given quantile of them) meet the target error."""
        import torch

        xd = torch.as_tensor(X, device="cuda")
        self.threshold = 0.0
        y, spread, _ = self.infer(xd)
        torch.cuda.synchronize()
        y, spread = y.cpu().numpy(), spread.cpu().numpy()
        err = stress_errors(y, Y, denom)
        order = np.argsort(spread)
        ok = err[order] <= target
        if quantile >= 1.0:
            bad = np.nonzero(~ok)[0]
            cut = bad[0] if bad.size else len(ok)
        else:
            run = np.cumsum(~ok) / np.arange(1, len(ok) + 1)
            good = np.nonzero(run <= 1.0 - quantile)[0]
            cut = good[-1] + 1 if good.size else 0
        self.threshold = float(spread[order[cut - 1]]) if cut > 0 else 0.0
        return dict(threshold=self.threshold, accepted=cut / len(ok), rows=len(ok),
                    median_error=float(np.median(err)), p99_error=float(np.quantile(err, 0.99)))
