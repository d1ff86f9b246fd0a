"""Seeded synthetic option-pricing workloads (inputs only).

This module produces the *inputs* of the all-at-once Crank-Nicolson solve:
the spatial operator A (three diagonals, the paper's A ~ L of eq. (1.1)),
the initial condition u^0 and the boundary forcing f^{k+1/2}.  It contains
none of the method's arithmetic (no all-at-once assembly, no right-hand side
b, no preconditioner, no Krylov step): both the CPU oracle and the GPU path
take what it returns as their input.

Problem family: 1D Black-Scholes in log-price x = ln S and time-to-maturity t,
    u_t = a(x) u_xx + b(x) u_x - r u,   a = sigma(x)^2/2,  b = r - sigma(x)^2/2,
an instance of the drift-diffusion-reaction operators of eq. (1.2) (first
case), discretised by second-order central differences on the interior nodes
x_i = x_min + i h, i = 1..N_x, h = (x_max - x_min)/(N_x + 1).  The European
put payoff max(K - e^x, 0) is the initial condition; Dirichlet data are the
discounted put asymptotics g_L(t) = K e^{-rt} - e^{x_min} (an exact solution
of the PDE) and g_R(t) = 0.  The source term of eq. (2.1) is the boundary
contribution evaluated at the midpoint t_{k+1/2} (Sec. 2.1): only its first
entry is non-zero, f_1 = A_{1,0} g_L(t_{k+1/2}).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

X_MIN = -3.0
X_MAX = 3.0


@dataclass
class Instance:
    """One pricing instance: operator, data and solver settings."""
    nx: int
    nt: int
    T: float
    r: float
    K: float
    alpha: float
    sigma: np.ndarray            # sigma(x_i) at the interior nodes, length nx
    a_lo: np.ndarray             # A_{i,i-1} (entry 0 unused), length nx
    a_di: np.ndarray             # A_{i,i}
    a_up: np.ndarray             # A_{i,i+1} (entry nx-1 unused)
    u0: np.ndarray               # initial condition, length nx
    f: np.ndarray                # f^{k+1/2}, shape (nt, nx)
    x: np.ndarray                # interior nodes
    h: float
    m: int = 20                  # GMRES restart length
    rtol: float = 1e-8
    pc_prec: str = "fp64"        # "fp64" or "fp32"
    name: str = ""
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.nx * self.nt


def grid(nx: int, x_min: float = X_MIN, x_max: float = X_MAX):
    h = (x_max - x_min) / (nx + 1)
    x = x_min + h * np.arange(1, nx + 1, dtype=np.float64)
    return x, h


def bs_operator(sigma: np.ndarray, r: float, h: float):
    """Central-difference Black-Scholes operator rows (lower, diagonal, upper)."""
    a = 0.5 * sigma ** 2
    b = r - 0.5 * sigma ** 2
    peclet = np.abs(b) * h / a
    if np.any(peclet >= 2.0):
        raise ValueError(f"cell Peclet number {peclet.max():.3f} >= 2")
    lo = a / h ** 2 - b / (2 * h)
    di = -2.0 * a / h ** 2 - r
    up = a / h ** 2 + b / (2 * h)
    lo = lo.copy()
    up = up.copy()
    lo[0] = 0.0       # couples to the left boundary node (moved into f)
    up[-1] = 0.0      # couples to the right boundary node (g_R = 0)
    return lo, di, up


def left_boundary(t, K: float, r: float, x_min: float = X_MIN):
    return K * np.exp(-r * np.asarray(t, dtype=np.float64)) - np.exp(x_min)


def family_rows(nx: int, nt: int, T: float, r: float, K: float,
                sigma_fn: Callable[[np.ndarray], np.ndarray]):
    """Operator rows, initial condition and the one non-zero column of the
    forcing of one put instance: (sigma, lo, di, up, u0, f_col, x, h), with
    f^{k+1/2} = f_col[k] e_1."""
    x, h = grid(nx)
    sigma = np.asarray(sigma_fn(x), dtype=np.float64)
    if sigma.min() < 0.02:
        raise ValueError("sigma below 0.02")
    a = 0.5 * sigma ** 2
    b = r - 0.5 * sigma ** 2
    lo, di, up = bs_operator(sigma, r, h)
    a10 = a[0] / h ** 2 - b[0] / (2 * h)        # A_{1,0}: coupling to x_0
    u0 = np.maximum(K - np.exp(x), 0.0)
    tau = T / nt
    th = (np.arange(nt, dtype=np.float64) + 0.5) * tau
    f_col = a10 * left_boundary(th, K, r)
    return sigma, lo, di, up, u0, f_col, x, h


def make_instance(nx: int, nt: int, T: float, r: float, K: float,
                  sigma_fn: Callable[[np.ndarray], np.ndarray], alpha: float,
                  m: int = 20, rtol: float = 1e-8, pc_prec: str = "fp64",
                  name: str = "", params: Optional[dict] = None) -> Instance:
    sigma, lo, di, up, u0, f_col, x, h = family_rows(nx, nt, T, r, K, sigma_fn)
    f = np.zeros((nt, nx), dtype=np.float64)
    f[:, 0] = f_col
    return Instance(nx=nx, nt=nt, T=T, r=r, K=K, alpha=alpha, sigma=sigma,
                    a_lo=lo, a_di=di, a_up=up, u0=u0, f=f, x=x, h=h, m=m,
                    rtol=rtol, pc_prec=pc_prec, name=name, params=params or {})


# ---------------------------------------------------------------------------
# volatility families
# ---------------------------------------------------------------------------

def local_vol_amplitudes(rng: np.random.Generator):
    """sigma(x) = 0.2 + a1 tanh x + a2 sin 3x with a1, a2 drawn within +-20%."""
    a1 = 0.1 * rng.uniform(0.8, 1.2)
    a2 = 0.05 * rng.uniform(0.8, 1.2)
    return a1, a2


def local_vol(a1: float, a2: float):
    return lambda x: 0.2 + a1 * np.tanh(x) + a2 * np.sin(3.0 * x)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def config1(nx: int = 127, nt: int = 64) -> Instance:
    """Constant volatility put: sigma 0.3, r 0.05, K 1, T 1, alpha 0.01."""
    return make_instance(nx, nt, T=1.0, r=0.05, K=1.0,
                         sigma_fn=lambda x: np.full_like(x, 0.3), alpha=0.01,
                         m=20, rtol=1e-12, pc_prec="fp64",
                         name=f"bs-const-{nx}x{nt}")


def config2(alpha: float = 0.01, pc_prec: str = "fp64", nx: int = 4095,
            nt: int = 1024, seed: int = 2) -> Instance:
    """Local volatility put, r 0.03, K 1, T 2, flexible GMRES(30), rtol 1e-8."""
    rng = np.random.default_rng(seed)
    a1, a2 = local_vol_amplitudes(rng)
    return make_instance(nx, nt, T=2.0, r=0.03, K=1.0,
                         sigma_fn=local_vol(a1, a2), alpha=alpha, m=30,
                         rtol=1e-8, pc_prec=pc_prec,
                         name=f"bs-localvol-{nx}x{nt}",
                         params={"a1": a1, "a2": a2, "seed": seed})


BATCH_NX = (255, 511, 1023, 2047)
BATCH_NT = (64, 128, 256, 512)


def config3(count: int = 512, seed: int = 3, nx_choices=BATCH_NX,
            nt_choices=BATCH_NT) -> List[Instance]:
    """Uneven batch of constant-volatility puts (FP32 preconditioner)."""
    rng = np.random.default_rng(seed)
    out = []
    for q in range(count):
        sigma = rng.uniform(0.1, 0.5)
        r = rng.uniform(0.0, 0.08)
        K = rng.uniform(0.8, 1.2)
        T = rng.uniform(0.25, 2.0)
        nx = int(rng.choice(nx_choices))
        nt = int(rng.choice(nt_choices))
        out.append(make_instance(nx, nt, T=T, r=r, K=K,
                                 sigma_fn=(lambda s: (lambda x: np.full_like(x, s)))(sigma),
                                 alpha=0.01, m=20, rtol=1e-8, pc_prec="fp32",
                                 name=f"batch-{q}",
                                 params={"sigma": sigma}))
    return out


WS_NX = 2047
WS_NT = 512
WS_FEATURE_POINTS = 64


def config4_params(count: int, seed: int):
    """Per-instance (a1, a2, r, T, K) for the warm-start family."""
    rng = np.random.default_rng(seed)
    p = np.empty((count, 5), dtype=np.float64)
    for q in range(count):
        a1, a2 = local_vol_amplitudes(rng)
        p[q] = (a1, a2, rng.uniform(0.0, 0.08), rng.uniform(0.25, 2.0),
                rng.uniform(0.8, 1.2))
    return p


def config4_instance(p, nx: int = WS_NX, nt: int = WS_NT) -> Instance:
    a1, a2, r, T, K = (float(v) for v in p)
    return make_instance(nx, nt, T=T, r=r, K=K, sigma_fn=local_vol(a1, a2),
                         alpha=0.01, m=20, rtol=1e-8, pc_prec="fp32",
                         name="ws", params={"a1": a1, "a2": a2})


def config4_rows(p, nx: int = WS_NX, nt: int = WS_NT):
    """family_rows of one warm-start instance plus its Dirichlet data at the
    fine levels t_{k+1} (left: discounted put asymptote, right: 0)."""
    a1, a2, r, T, K = (float(v) for v in p)
    rows = family_rows(nx, nt, T=T, r=r, K=K, sigma_fn=local_vol(a1, a2))
    tk = (np.arange(nt, dtype=np.float64) + 1.0) * (T / nt)
    return rows, left_boundary(tk, K, r), np.zeros(nt)


def config4_features(params: np.ndarray) -> np.ndarray:
    """sigma at 64 equispaced points of [-3, 3] followed by (r, T, K)."""
    xs = np.linspace(X_MIN, X_MAX, WS_FEATURE_POINTS)
    out = np.empty((params.shape[0], WS_FEATURE_POINTS + 3), dtype=np.float64)
    for q, (a1, a2, r, T, K) in enumerate(params):
        out[q, :WS_FEATURE_POINTS] = local_vol(a1, a2)(xs)
        out[q, WS_FEATURE_POINTS:] = (r, T, K)
    return out


def config5(nx: int = 65535, nt: int = 4096, seed: int = 5) -> Instance:
    """Production-size local volatility put, FP32 preconditioner, GMRES(20)."""
    rng = np.random.default_rng(seed)
    a1, a2 = local_vol_amplitudes(rng)
    return make_instance(nx, nt, T=2.0, r=0.03, K=1.0,
                         sigma_fn=local_vol(a1, a2), alpha=0.01, m=20,
                         rtol=1e-8, pc_prec="fp32",
                         name=f"bs-localvol-{nx}x{nt}",
                         params={"a1": a1, "a2": a2, "seed": seed})


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


# ---------------------------------------------------------------------------
# 2D drift-diffusion operators on a tensor grid (synthetic stand-ins for the
# 2D operators of Sec. 5; none of the paper's model parameters are used)
# ---------------------------------------------------------------------------

# stencil entry q of grid point i multiplies the unknown at (iy + dy, ix + dx),
# q = 3 (dy + 1) + (dx + 1); unknown i = iy N_x + ix (x fastest)
STENCIL_OFFSETS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


@dataclass
class Instance2D:
    nx: int
    ny: int
    nt: int
    T: float
    alpha: float
    st: np.ndarray        # (9, N_x N_y) stencil coefficients of A
    u0: np.ndarray        # (N_x N_y,) initial condition
    f: np.ndarray         # (N_t, N_x N_y) source blocks f^{k+1/2}
    name: str = ""

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nt

    @property
    def npts(self) -> int:
        return self.nx * self.ny


def drift_diffusion_2d_stencil(nx: int, ny: int, a, b, c, d, e, r):
    """Nine-point central-difference stencil of
        A u = a u_xx + b u_yy + c u_xy + d u_x + e u_y - r u
    on the interior nodes of the unit square (h_x = 1/(N_x+1),
    h_y = 1/(N_y+1)), homogeneous Dirichlet data outside; a..r are functions
    of (x, y) evaluated at the nodes (or constants)."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    X, Y = np.meshgrid(np.arange(1, nx + 1) * hx, np.arange(1, ny + 1) * hy)
    ev = lambda g: np.broadcast_to(np.asarray(g(X, Y) if callable(g) else g, dtype=np.float64),
                                   X.shape).reshape(-1)
    A_, B_, C_, D_, E_, R_ = (ev(g) for g in (a, b, c, d, e, r))
    st = np.zeros((9, nx * ny))
    q = {o: k for k, o in enumerate(STENCIL_OFFSETS)}
    st[q[(0, -1)]] = A_ / hx ** 2 - D_ / (2 * hx)
    st[q[(0, 1)]] = A_ / hx ** 2 + D_ / (2 * hx)
    st[q[(-1, 0)]] = B_ / hy ** 2 - E_ / (2 * hy)
    st[q[(1, 0)]] = B_ / hy ** 2 + E_ / (2 * hy)
    st[q[(0, 0)]] = -2 * A_ / hx ** 2 - 2 * B_ / hy ** 2 - R_
    cm = C_ / (4 * hx * hy)
    st[q[(1, 1)]] = cm
    st[q[(-1, -1)]] = cm
    st[q[(1, -1)]] = -cm
    st[q[(-1, 1)]] = -cm
    return st


def drift_diffusion_2d(nx: int, ny: int, nt: int, T: float = 0.5, alpha: float = 0.01,
                       seed: int = 21, mixed: float = 0.0) -> Instance2D:
    """Seeded variable-coefficient drift-diffusion-reaction operator (not
    separable: every coefficient depends on x and y), a smooth bump as the
    initial condition and a small smooth source.  `mixed` scales a mixed
    derivative term c = mixed sqrt(a b).  The cell Peclet numbers stay below
    1, so with mixed = 0 the stencil is an M-matrix pattern (weakly
    diagonally dominant rows)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.8, 1.2, size=8)
    a = lambda x, y: 0.20 * p[0] * (1.0 + 0.3 * np.sin(np.pi * x) * np.cos(np.pi * y))
    b = lambda x, y: 0.10 * p[1] * (1.0 + 0.3 * np.cos(2 * np.pi * x * y))
    d = lambda x, y: 0.3 * p[2] * np.cos(np.pi * y) * (1.0 - x)
    e = lambda x, y: 0.2 * p[3] * np.sin(np.pi * x) - 0.1 * p[4]
    r = 0.05 * p[5]
    c = lambda x, y: mixed * np.sqrt(a(x, y) * b(x, y))
    st = drift_diffusion_2d_stencil(nx, ny, a, b, c, d, e, r)
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    X, Y = np.meshgrid(np.arange(1, nx + 1) * hx, np.arange(1, ny + 1) * hy)
    u0 = (np.exp(-40 * ((X - 0.4 * p[6]) ** 2 + (Y - 0.5) ** 2))).reshape(-1)
    tk = (np.arange(nt) + 0.5) * (T / nt)
    f = 0.1 * p[7] * np.outer(np.exp(-tk), (np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1))
    return Instance2D(nx, ny, nt, T, alpha, st, u0, f, name=f"dd2d-{nx}x{ny}x{nt}")
