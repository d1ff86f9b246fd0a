"""Learned initial guess for the all-at-once CN solve: training data from
plain solves, training on the GPU, and the initial guess at solve time.

GMRES reduces the residual it starts from (Sec. 4, eq. (4.1)), so an initial
guess close to the solution saves iterations.  The network (cn_warmstart.h)
maps the features of a local-volatility put -- sigma(x) at 64 equispaced
points of [-3, 3] and (r, T, K) -- to the solution on a coarse 128 x 64
space-time grid; the coarse values are interpolated to the fine grid with
the initial condition and the Dirichlet data, and the solve starts from
there (use_x0 = 2: an instance whose guess does not reduce the residual
below ||b|| starts from zero instead, so the plain method remains the
fallback, and the true residual decides convergence either way).

Every arithmetic step runs in the library's kernels: the solves that make
the training targets, the restriction to the coarse grid, the network's
forward and backward passes and Adam, the interpolation.  This module only
orders the calls, draws the seeded inputs and moves mini-batches.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import List, Optional

import numpy as np
import torch

from . import binding as B
from . import workloads as W

N_IN = W.WS_FEATURE_POINTS + 3
N_OUT = B.COARSE_X * B.COARSE_T
WIDTH = 512


@dataclass
class FamilyBatch:
    """Device inputs of `count` warm-start instances of one shape."""
    params: np.ndarray        # (count, 5): a1, a2, r, T, K
    nx: int
    nt: int
    probs: List[dict]         # per-instance operator rows for cn_batch_create
    u0: torch.Tensor          # packed initial conditions (count * nx)
    f: torch.Tensor           # packed forcing (count * nt * nx)
    gl: torch.Tensor          # Dirichlet data (count * nt), left
    gr: torch.Tensor          # right
    features: torch.Tensor    # (count, N_IN) float32

    @property
    def count(self):
        return self.params.shape[0]


def family_batch(params: np.ndarray, nx: int = W.WS_NX, nt: int = W.WS_NT,
                 m_max: int = 20, dev: Optional[torch.device] = None) -> FamilyBatch:
    dev = dev or torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev)
    count = params.shape[0]
    probs, u0s, fcols, gls, grs = [], [], [], [], []
    for p in params:
        (sigma, lo, di, up, u0, f_col, x, h), gl, gr = W.config4_rows(p, nx, nt)
        probs.append(dict(a_lo=T(lo), a_di=T(di), a_up=T(up), nt=nt, T=float(p[3]),
                          alpha=0.01, m_max=m_max))
        u0s.append(u0)
        fcols.append(f_col)
        gls.append(gl)
        grs.append(gr)
    # forcing: only the first spatial entry of every level is non-zero
    f = torch.zeros((count, nt, nx), dtype=torch.float64, device=dev)
    f[:, :, 0] = T(np.stack(fcols))
    feats = torch.as_tensor(W.config4_features(params), dtype=torch.float32, device=dev)
    return FamilyBatch(params, nx, nt, probs, T(np.concatenate(u0s)), f.reshape(-1),
                       T(np.concatenate(gls)), T(np.concatenate(grs)), feats.contiguous())


def solve_family(fb: FamilyBatch, x0=None, m: int = 20, rtol: float = 1e-8,
                 pc_prec: str = "fp32", warm: bool = False, err_tol: float = 0.0):
    """Batched solve of the family batch; returns (x, total, per-instance,
    seconds of the solve call).  warm: x0 holds the initial guess (fallback
    start); err_tol > 0: error-controlled stopping."""
    bat = B.Batch(fb.probs, pc_prec=pc_prec)
    b = torch.empty(fb.count * fb.nx * fb.nt, dtype=torch.float64, device=fb.u0.device)
    bat.rhs(fb.u0, fb.f, b)
    x = x0 if x0 is not None else torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot, per = bat.solve(b, x, m=m, rtol=rtol, use_x0=2 if warm else 0, err_tol=err_tol)
    sec = time.perf_counter() - t0
    bat.close()
    return x, tot, per, sec


def generate(params: np.ndarray, chunk: int = 128, nx: int = W.WS_NX, nt: int = W.WS_NT,
             log=None):
    """Training pairs from plain (zero-start) solves: features (count, N_IN)
    and coarse restrictions of the solutions (count, N_OUT), float32, on the
    GPU."""
    dev = torch.device("cuda:0")
    count = params.shape[0]
    X = torch.empty((count, N_IN), dtype=torch.float32, device=dev)
    Y = torch.empty((count, N_OUT), dtype=torch.float32, device=dev)
    ones = torch.ones(chunk, dtype=torch.float64, device=dev)
    worst = 0.0
    for c0 in range(0, count, chunk):
        fb = family_batch(params[c0:c0 + chunk], nx, nt, dev=dev)
        x, tot, per, sec = solve_family(fb)
        if tot.status != B.CN_OK:
            raise RuntimeError(f"training solve {c0}: relres {tot.relres_true:.2e}")
        worst = max(worst, tot.relres_true)
        B.ws_restrict(x, fb.count, nx, nt, ones[:fb.count], Y[c0:c0 + fb.count])
        X[c0:c0 + fb.count] = fb.features
        if log:
            log(f"[warmstart] data {c0 + fb.count}/{count}: {tot.iters} iters, "
                f"{sec * 1e3:.1f} ms solve")
        del fb, x
    return X, Y, worst


def init_params(seed: int, n_in: int = N_IN, width: int = WIDTH, n_out: int = N_OUT):
    """He-uniform weights, zero biases, in the flat layout of cn_warmstart.h."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((n_in, width), (width, width), (width, width), (width, n_out)):
        lim = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, size=fo * fi))
        parts.append(np.zeros(fo))
    # the output layer starts small: predictions start at the target mean
    parts[-2] *= 0.1
    return np.concatenate(parts).astype(np.float32)


def normalization(X: torch.Tensor, Y: torch.Tensor):
    """Per-column mean and spread of the features and targets (float32);
    spreads are floored so that near-constant columns are not amplified."""
    def stats(A, rel_floor):
        mu = A.double().mean(dim=0)
        sd = A.double().std(dim=0)
        sd = torch.clamp(sd, min=max(rel_floor * float(sd.max()), 1e-12))
        return mu.float().contiguous(), sd.float().contiguous()
    in_mu, in_sd = stats(X, 1e-3)
    out_mu, out_sd = stats(Y, 1e-2)
    return in_mu, in_sd, out_mu, out_sd


def train(X: torch.Tensor, Y: torch.Tensor, epochs: int = 200, batch: int = 256,
          lr: float = 1e-3, lr_min: float = 1e-5, seed: int = 0, width: int = WIDTH, log=None):
    """Adam on the mean-squared standardised error; cosine learning-rate
    decay from lr to lr_min.  Returns the network and the per-epoch mean
    losses."""
    dev = X.device
    count = X.shape[0]
    net = B.Mlp(N_IN, width, N_OUT, batch)
    net.set_params(torch.as_tensor(init_params(seed, width=width), device=dev))
    net.set_normalization(*normalization(X, Y))
    rng = np.random.default_rng(seed + 1)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    nb = count // batch
    history = []
    for ep in range(epochs):
        perm = torch.as_tensor(rng.permutation(count), device=dev)
        Xs, Ys = X[perm], Y[perm]
        acc = torch.zeros(1, dtype=torch.float32, device=dev)
        lr_ep = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * ep / max(1, epochs - 1)))
        for i in range(nb):
            net.loss_grad(Xs[i * batch:(i + 1) * batch], Ys[i * batch:(i + 1) * batch],
                          loss=loss)
            net.adam_step(float(lr_ep))
            acc += loss
        history.append(float(acc) / nb)
        if log and (ep % 20 == 0 or ep == epochs - 1):
            log(f"[warmstart] epoch {ep}: loss {history[-1]:.3e} (lr {lr_ep:.2e})")
    return net, history


def initial_guess(net: B.Mlp, fb: FamilyBatch, coarse: Optional[torch.Tensor] = None,
                  x0: Optional[torch.Tensor] = None):
    """x0 for every instance of the family batch: network forward pass on the
    features, then interpolation to the fine grid (one library call)."""
    dev = fb.u0.device
    if coarse is None:
        coarse = torch.empty((fb.count, N_OUT), dtype=torch.float32, device=dev)
    if x0 is None:
        x0 = torch.empty(fb.count * fb.nx * fb.nt, dtype=torch.float64, device=dev)
    scale = torch.ones(fb.count, dtype=torch.float64, device=dev)
    net.predict(fb.features, fb.nx, fb.nt, fb.u0, fb.gl, fb.gr, scale, coarse, x0)
    return x0, coarse
