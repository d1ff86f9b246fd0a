"""CPU oracle of the learned initial guess (test infrastructure only).

Plain float64 definitions of what the warm-start kernels compute, for the
tests and the benchmark's CPU leg; nothing in the library path imports this
module.  The initial guess serves the residual bound of Sec. 4, eq. (4.1):
GMRES on the preconditioned system reduces the initial residual, so the
iteration count falls with a better u_0.

  * the network n_in -> w -> w -> w -> n_out with ReLU after the hidden
    layers, on standardised inputs and targets; forward pass, mean-squared
    error and its gradient by the chain rule written out layer by layer,
    optionally with every matrix-product operand rounded to bfloat16 (the
    operand precision of the matrix cores; sums stay float64);
  * Adam with bias-corrected moments;
  * restriction of a fine space-time solution to the 128 x 64 coarse grid
    and bilinear interpolation back, the latter by two passes of np.interp
    (space on each coarse level, then time) over the coarse grid extended by
    the Dirichlet data and the initial condition.

Pinned by tests/test_mlp_oracle_pins.py: gradients against central finite
differences of the loss, Adam against its closed form under a constant
gradient, interpolation against bilinear functions (reproduced exactly) and
restriction of an interpolant (returns the coarse values).
"""
from __future__ import annotations

import numpy as np

CX, CT = 128, 64          # coarse grid: points in space, levels in time
X_MIN, X_MAX = -3.0, 3.0  # space interval of the problem family

# --------------------------------------------------------------------------
# the network
# --------------------------------------------------------------------------


def param_shapes(n_in: int, w: int, n_out: int):
    return [(w, n_in), (w,), (w, w), (w,), (w, w), (w,), (n_out, w), (n_out,)]


def unflatten(p: np.ndarray, n_in: int, w: int, n_out: int):
    out, o = [], 0
    for s in param_shapes(n_in, w, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(p[o:o + k], dtype=np.float64).reshape(s))
        o += k
    assert o == p.size, "flat parameter array has the wrong length"
    return out


def num_params(n_in: int, w: int, n_out: int) -> int:
    return sum(int(np.prod(s)) for s in param_shapes(n_in, w, n_out))


def bf16(a):
    """Round to bfloat16 (8 significant bits, nearest-even) and back, by
    torch's CPU conversion: the operand precision of the matrix-core
    products."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


def _ident(a):
    return a


def forward(p, X, n_in, w, n_out, in_mu=None, in_sd=None, rnd=None):
    """Standardised output z and the activations (xn, h1, h2, h3).
    rnd (optional) rounds every operand of a matrix product (e.g. bf16);
    biases, activations and sums stay in float64."""
    r = rnd or _ident
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(p, n_in, w, n_out)
    X = np.asarray(X, dtype=np.float64)
    mu = np.zeros(n_in) if in_mu is None else np.asarray(in_mu, dtype=np.float64)
    sd = np.ones(n_in) if in_sd is None else np.asarray(in_sd, dtype=np.float64)
    xn = (X - mu) / sd
    h1 = np.maximum(r(xn) @ r(W1).T + b1, 0.0)
    h2 = np.maximum(r(h1) @ r(W2).T + b2, 0.0)
    h3 = np.maximum(r(h2) @ r(W3).T + b3, 0.0)
    z = r(h3) @ r(W4).T + b4
    return z, (xn, h1, h2, h3)


def predict(p, X, n_in, w, n_out, in_mu=None, in_sd=None, out_mu=None, out_sd=None,
            rnd=None):
    """De-standardised prediction y = out_mu + out_sd * z."""
    z, _ = forward(p, X, n_in, w, n_out, in_mu, in_sd, rnd)
    mu = 0.0 if out_mu is None else np.asarray(out_mu, dtype=np.float64)
    sd = 1.0 if out_sd is None else np.asarray(out_sd, dtype=np.float64)
    return mu + sd * z


def loss(p, X, Yt, n_in, w, n_out, in_mu=None, in_sd=None, out_mu=None, out_sd=None):
    z, _ = forward(p, X, n_in, w, n_out, in_mu, in_sd)
    t = _std_target(Yt, out_mu, out_sd)
    return float(np.mean((z - t) ** 2))


def _std_target(Yt, out_mu, out_sd):
    t = np.asarray(Yt, dtype=np.float64)
    if out_mu is not None:
        t = t - np.asarray(out_mu, dtype=np.float64)
    if out_sd is not None:
        t = t / np.asarray(out_sd, dtype=np.float64)
    return t


def loss_grad(p, X, Yt, n_in, w, n_out, in_mu=None, in_sd=None, out_mu=None, out_sd=None,
              rnd=None):
    """Loss (mean over all entries of the squared standardised error) and its
    gradient with respect to the flat parameters, by back-propagation.
    rnd: as in forward, applied to every operand of every product."""
    r = rnd or _ident
    W1, b1, W2, b2, W3, b3, W4, b4 = unflatten(p, n_in, w, n_out)
    z, (xn, h1, h2, h3) = forward(p, X, n_in, w, n_out, in_mu, in_sd, rnd)
    t = _std_target(Yt, out_mu, out_sd)
    d = z - t
    L = float(np.mean(d ** 2))
    dz = 2.0 * d / d.size
    gW4 = r(dz).T @ r(h3)
    gb4 = dz.sum(axis=0)
    d3 = (r(dz) @ r(W4)) * (h3 > 0)
    gW3 = r(d3).T @ r(h2)
    gb3 = d3.sum(axis=0)
    d2 = (r(d3) @ r(W3)) * (h2 > 0)
    gW2 = r(d2).T @ r(h1)
    gb2 = d2.sum(axis=0)
    d1 = (r(d2) @ r(W2)) * (h1 > 0)
    gW1 = r(d1).T @ r(xn)
    gb1 = d1.sum(axis=0)
    g = np.concatenate([a.reshape(-1) for a in (gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4)])
    return L, g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015): moments, bias correction, step.
    Returns new (p, m, v); `step` is the 1-based index of this update."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# --------------------------------------------------------------------------
# coarse grid <-> fine grid
# --------------------------------------------------------------------------


def coarse_positions(nx: int, nt: int, T: float):
    """Space positions of the 128 coarse nodes (cell centres of 128 equal
    cells of [x_min, x_max]) and times of the 64 coarse levels (q+1) T/64,
    with the fine index of each (interior node i sits at x_min + (i+1) h,
    row k of the all-at-once layout at t = (k+1) T/nt)."""
    assert (nx + 1) % CX == 0 and (nx + 1) // CX >= 2 and nt % CT == 0
    H = (X_MAX - X_MIN) / CX
    xc = X_MIN + (np.arange(CX) + 0.5) * H
    tc = (np.arange(CT) + 1.0) * T / CT
    h = (X_MAX - X_MIN) / (nx + 1)
    ic = np.rint((xc - X_MIN) / h).astype(np.int64) - 1
    kc = np.rint(tc / (T / nt)).astype(np.int64) - 1
    return xc, tc, ic, kc


def restrict(x, nx: int, nt: int, inv_scale: float = 1.0):
    """coarse[q, c] = float32(inv_scale * u(t_q, x_c)) for one instance."""
    xc, tc, ic, kc = coarse_positions(nx, nt, 1.0)
    U = np.asarray(x, dtype=np.float64).reshape(nt, nx)
    return (U[np.ix_(kc, ic)] * inv_scale).astype(np.float32)


def interpolate(coarse, nx: int, nt: int, u0, gl, gr, scale: float = 1.0):
    """Fine initial guess (nt*nx values) from one instance's coarse values.

    Space first: on every coarse level the values at [x_min, coarse nodes,
    x_max] (Dirichlet data of that level, scale * coarse, Dirichlet data)
    are interpolated linearly to the fine nodes.  Then time: every fine
    level is interpolated linearly between the levels [0, coarse levels],
    level 0 being the initial condition at the fine nodes."""
    T = 1.0
    xc, tc, ic, kc = coarse_positions(nx, nt, T)
    h = (X_MAX - X_MIN) / (nx + 1)
    xf = X_MIN + (np.arange(nx) + 1.0) * h
    C = np.asarray(coarse, dtype=np.float64).reshape(CT, CX) * scale
    gl = np.asarray(gl, dtype=np.float64)
    gr = np.asarray(gr, dtype=np.float64)
    xs = np.concatenate([[X_MIN], xc, [X_MAX]])
    rows = np.empty((CT + 1, nx))
    rows[0] = np.asarray(u0, dtype=np.float64)
    for q in range(CT):
        ys = np.concatenate([[gl[kc[q]]], C[q], [gr[kc[q]]]])
        rows[q + 1] = np.interp(xf, xs, ys)
    ts = np.concatenate([[0.0], tc])
    tf = (np.arange(nt) + 1.0) * T / nt
    out = np.empty((nt, nx))
    for i in range(nx):
        out[:, i] = np.interp(tf, ts, rows[:, i])
    return out.reshape(-1)
