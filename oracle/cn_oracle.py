"""CPU FP64 oracle for the all-at-once Crank-Nicolson system and its
alpha-circulant preconditioned GMRES solve.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
reference that the GPU path is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never calls it and shares no code with it.

Everything is float64 / complex128 and follows the paper's definitions
directly:
  * eq. (2.1)/(2.2) and Sec. 3.2: the CN scheme, the all-at-once matrix
    M = B1 (x) I - B2 (x) A~ with A~ = tau A, and b = xi + tau f;
  * eq. (3.1): the preconditioner P_alpha = C1 (x) I - C2 (x) A~;
  * Sec. 3.1 and eq. (3.2): its three-step inverse, with the DFT along time
    written as direct O(N_t^2) sums (never an FFT), all N_t shifted systems
    solved (no conjugate-pair halving), each by a plain Thomas elimination;
  * Sec. 4, P_alpha = M - alpha R: the dense form used on tiny sizes;
  * block forward substitution (Sec. 2.2): the exact M^{-1} b;
  * right-preconditioned restarted GMRES(m) with modified Gram-Schmidt
    (Sec. 5 uses right preconditioning, zero start, relative residual stop).

Sign reading of the eigenvalue formula: the DFT matrix is built with
omega = exp(-2 pi i / N_t) and D_l = diag(sqrt(N_t) F Lambda_alpha C_l(:,1)),
which gives lambda_{1,j} = 1 - alpha^{1/N_t} omega^j and
lambda_{2,j} = (1 + alpha^{1/N_t} omega^j)/2 for the j-th forward DFT mode.
The printed eigenvalue formula has exp(+2(k-1) pi i/N_t), the same set in the
opposite order; the oracle derives the eigenvalues from the diagonalisation
itself (lambda = unnormalised DFT of Lambda_alpha C_l(:,1)), so it pairs each
eigenvalue with the mode it belongs to.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# The all-at-once system (Sec. 2.2, eq. (2.2); block form of Sec. 3.2)
# ---------------------------------------------------------------------------

def tridiag_dense(lo, di, up):
    """Dense matrix with rows (lo[i], di[i], up[i]); lo[0], up[-1] unused."""
    n = len(di)
    A = np.diag(np.asarray(di, dtype=np.float64))
    if n > 1:
        A += np.diag(np.asarray(lo[1:], dtype=np.float64), -1)
        A += np.diag(np.asarray(up[:-1], dtype=np.float64), 1)
    return A


def tridiag_mul(lo, di, up, x):
    """y = A x for a tridiagonal A given by rows; x may be (..., nx)."""
    y = di * x
    y[..., 1:] += lo[1:] * x[..., :-1]
    y[..., :-1] += up[:-1] * x[..., 1:]
    return y


def aao_matrix_dense(lo, di, up, T, nt):
    """M = B1 (x) I_s - B2 (x) A~, B1 = tridiag(-1,1,0), B2 = tridiag(1,1,0)/2
    (eq. (2.2)); A~ = tau A with tau = T/N_t."""
    tau = T / nt
    At = tau * tridiag_dense(lo, di, up)
    nx = At.shape[0]
    B1 = np.eye(nt) - np.eye(nt, k=-1)
    B2 = 0.5 * (np.eye(nt) + np.eye(nt, k=-1))
    return np.kron(B1, np.eye(nx)) - np.kron(B2, At)


def aao_matvec(lo, di, up, T, nt, u, d=None):
    """y = M u using the block-bidiagonal form of Sec. 3.2:
    y^1 = Q1 u^1, y^k = Q1 u^k - Q2 u^{k-1}, Q1 = I - A~/2, Q2 = I + A~/2.
    Vector layout: u = [u^1; ...; u^{N_t}], space fastest (eq. (2.2)).
    With time weights d (length N_t) the matrix is B1 (x) I - (D B2) (x) A~
    (the time-dependent-coefficient form of Sec. 5.2)."""
    nx = len(di)
    tau = T / nt
    U = np.asarray(u, dtype=np.float64).reshape(nt, nx)
    Y = np.empty_like(U)
    for k in range(nt):
        s = U[k].copy()
        diff = U[k].copy()
        if k > 0:
            s += U[k - 1]
            diff -= U[k - 1]
        w = 1.0 if d is None else d[k]
        Y[k] = diff - 0.5 * w * tau * tridiag_mul(lo, di, up, s)
    return Y.reshape(-1)


def aao_rhs(lo, di, up, T, nt, u0, f, d=None):
    """b = xi + tau f with xi = [(I + A~/2) u^0; 0; ...; 0] (eq. (2.2));
    f = [f^{1/2}; ...; f^{N_t-1/2}] of shape (N_t, N_x)."""
    nx = len(di)
    tau = T / nt
    w0 = 1.0 if d is None else d[0]
    b = tau * np.asarray(f, dtype=np.float64).reshape(nt, nx).copy()
    b[0] += u0 + 0.5 * w0 * tau * tridiag_mul(lo, di, up, np.asarray(u0, dtype=np.float64))
    return b.reshape(-1)


def sequential_cn(lo, di, up, T, nt, u0, f, d=None):
    """Exact M^{-1} b by block forward substitution (Sec. 2.2), i.e. CN time
    stepping (eq. (2.1)): (I - A~/2) u^{k+1} = (I + A~/2) u^k + tau f^{k+1/2}.
    Each step is solved by a plain Thomas elimination."""
    nx = len(di)
    tau = T / nt
    F = np.asarray(f, dtype=np.float64).reshape(nt, nx)
    u = np.asarray(u0, dtype=np.float64).copy()
    out = np.empty((nt, nx))
    for k in range(nt):
        w = 1.0 if d is None else d[k]
        rhs = u + 0.5 * w * tau * tridiag_mul(lo, di, up, u) + tau * F[k]
        u = thomas(-0.5 * w * tau * lo, 1.0 - 0.5 * w * tau * di,
                   -0.5 * w * tau * up, rhs)
        out[k] = u
    return out.reshape(-1)


def sequential_cn_banded(lo, di, up, T, nt, u0, f_col=None, f=None):
    """sequential_cn for production sizes: the same CN steps with every
    tridiagonal solve done by LAPACK's banded solver (scipy.linalg.solve_banded)
    instead of the Python-loop Thomas elimination.  The forcing is either
    dense (f, nt x nx) or only in the first spatial entry of every level
    (f_col, nt values).  Constant weights only."""
    from scipy.linalg import solve_banded
    nx = len(di)
    tau = T / nt
    lo = np.asarray(lo, dtype=np.float64)
    di = np.asarray(di, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    ab = np.zeros((3, nx))
    ab[0, 1:] = -0.5 * tau * up[:-1]
    ab[1, :] = 1.0 - 0.5 * tau * di
    ab[2, :-1] = -0.5 * tau * lo[1:]
    u = np.asarray(u0, dtype=np.float64).copy()
    out = np.empty((nt, nx))
    for k in range(nt):
        rhs = u + 0.5 * tau * tridiag_mul(lo, di, up, u)
        if f is not None:
            rhs += tau * np.asarray(f[k], dtype=np.float64)
        elif f_col is not None:
            rhs[0] += tau * f_col[k]
        u = solve_banded((1, 1), ab, rhs, overwrite_b=True, check_finite=False)
        out[k] = u
    return out.reshape(-1)


def thomas(lo, di, up, rhs):
    """Plain Thomas elimination (no pivoting) for one tridiagonal system with
    rows (lo[i], di[i], up[i]); works for real or complex data.  rhs may carry
    trailing batch dimensions after the first axis."""
    n = len(di)
    dt = np.result_type(lo, di, up, rhs)
    c = np.zeros(n, dtype=dt)
    d = np.zeros(np.shape(rhs), dtype=dt)
    piv = di[0]
    c[0] = up[0] / piv if n > 1 else 0.0
    d[0] = rhs[0] / piv
    for i in range(1, n):
        piv = di[i] - lo[i] * c[i - 1]
        if i < n - 1:
            c[i] = up[i] / piv
        d[i] = (rhs[i] - lo[i] * d[i - 1]) / piv
    x = np.zeros_like(d)
    x[n - 1] = d[n - 1]
    for i in range(n - 2, -1, -1):
        x[i] = d[i] - c[i] * x[i + 1]
    return x


def thomas_batched(lo, di, up, rhs):
    """Thomas elimination for a batch of systems sharing nothing but the
    size: lo, di, up, rhs have shape (batch, n).  Same recurrence as thomas(),
    vectorised over the batch axis."""
    n = di.shape[1]
    c = np.zeros_like(di)
    d = np.zeros_like(rhs)
    piv = di[:, 0]
    if n > 1:
        c[:, 0] = up[:, 0] / piv
    d[:, 0] = rhs[:, 0] / piv
    for i in range(1, n):
        piv = di[:, i] - lo[:, i] * c[:, i - 1]
        if i < n - 1:
            c[:, i] = up[:, i] / piv
        d[:, i] = (rhs[:, i] - lo[:, i] * d[:, i - 1]) / piv
    x = np.zeros_like(d)
    x[:, n - 1] = d[:, n - 1]
    for i in range(n - 2, -1, -1):
        x[:, i] = d[:, i] - c[:, i] * x[:, i + 1]
    return x


# ---------------------------------------------------------------------------
# The preconditioner (Sec. 3.1)
# ---------------------------------------------------------------------------

def alpha_circulants(alpha, nt):
    """C1^(alpha), C2^(alpha) of Sec. 3.1 (dense, N_t x N_t)."""
    C1 = np.eye(nt) - np.eye(nt, k=-1)
    C2 = 0.5 * (np.eye(nt) + np.eye(nt, k=-1))
    C1[0, nt - 1] += -alpha
    C2[0, nt - 1] += 0.5 * alpha
    return C1, C2


def pc_matrix_dense(lo, di, up, T, nt, alpha):
    """P_alpha = C1 (x) I_s - C2 (x) A~ (eq. (3.1))."""
    tau = T / nt
    At = tau * tridiag_dense(lo, di, up)
    C1, C2 = alpha_circulants(alpha, nt)
    nx = At.shape[0]
    return np.kron(C1, np.eye(nx)) - np.kron(C2, At)


def pc_matvec(lo, di, up, T, nt, alpha, z):
    """y = P_alpha z block by block (eq. (3.1)): y^k = z^k - z^{k-1} -
    (A~/2)(z^k + z^{k-1}), where for the first block the previous block is
    alpha z^{N_t} (the wrap-around entries of C1, C2).  Vectorised over the
    time levels, for full-size residual checks of the preconditioner."""
    nx = len(di)
    tau = T / nt
    Z = np.asarray(z, dtype=np.float64).reshape(nt, nx)
    Zp = np.roll(Z, 1, axis=0)
    Zp[0] *= alpha
    S = Z + Zp
    Y = Z - Zp
    Y -= 0.5 * tau * tridiag_mul(np.asarray(lo), np.asarray(di), np.asarray(up), S)
    return Y.reshape(-1)


def coupling_matrix_dense(lo, di, up, T, nt):
    """R of Sec. 4: Q2 in block (1, N_t), zero elsewhere, so that
    P_alpha = M - alpha R."""
    tau = T / nt
    At = tau * tridiag_dense(lo, di, up)
    nx = At.shape[0]
    R = np.zeros((nt * nx, nt * nx))
    R[:nx, (nt - 1) * nx:] = np.eye(nx) + 0.5 * At
    return R


def dft_matrix(nt):
    """Unnormalised DFT matrix [omega^{jm}], omega = exp(-2 pi i/N_t)
    (Sec. 3.1; the unitary F of the paper is this divided by sqrt(N_t))."""
    j = np.arange(nt)
    return np.exp(-2j * np.pi * np.outer(j, j) / nt)


def alpha_weights(alpha, nt):
    """Diagonal of Lambda_alpha: alpha^{m/N_t}, m = 0..N_t-1 (Sec. 3.1)."""
    return alpha ** (np.arange(nt) / nt)


def pc_eigenvalues(alpha, nt):
    """lambda_{l,j} = (sqrt(N_t) F Lambda_alpha C_l(:,1))_j, l = 1, 2 (Sec. 3.1),
    evaluated with the same direct DFT sums as step (a)."""
    C1, C2 = alpha_circulants(alpha, nt)
    W = dft_matrix(nt)
    lam = alpha_weights(alpha, nt)
    return W @ (lam * C1[:, 0]), W @ (lam * C2[:, 0])


def pc_apply(lo, di, up, T, nt, alpha, v, dbar=1.0):
    """z = P_alpha^{-1} v by the three steps of eq. (3.2).

    step (a): z1 = (V_alpha^{-1} (x) I) v, V_alpha^{-1} = F Lambda_alpha;
    step (b): (lambda_{1,j} I - lambda_{2,j} A~) z2_j = z1_j, every j;
    step (c): z = (V_alpha (x) I) z2, V_alpha = Lambda_alpha^{-1} F^*.
    The two unitary normalisations 1/sqrt(N_t) are combined into a single
    1/N_t on step (c).  dbar scales C2 (the averaged weight of Sec. 5.2)."""
    nx = len(di)
    tau = T / nt
    V = np.asarray(v, dtype=np.float64).reshape(nt, nx)
    lam = alpha_weights(alpha, nt)
    W = dft_matrix(nt)
    # step (a): direct DFT sums along time of the alpha-weighted blocks
    Z1 = W @ (lam[:, None] * V)
    # step (b): N_t complex shifted tridiagonal systems along space
    l1, l2 = pc_eigenvalues(alpha, nt)
    l2 = dbar * l2
    At_lo, At_di, At_up = tau * lo, tau * di, tau * up
    Z2 = np.empty_like(Z1)
    lo_b = -np.outer(l2, At_lo)
    di_b = l1[:, None] - np.outer(l2, At_di)
    up_b = -np.outer(l2, At_up)
    Z2[:] = thomas_batched(lo_b, di_b, up_b, Z1)
    # step (c): inverse DFT sums, 1/N_t, undo the alpha weights
    Zc = (W.conj() @ Z2) / nt
    Zc = Zc / lam[:, None]
    scale = max(np.abs(Zc).max(), 1e-300)
    if np.abs(Zc.imag).max() > 1e-10 * scale:
        raise AssertionError("preconditioned vector is not real")
    return Zc.real.reshape(-1)


# ---------------------------------------------------------------------------
# GMRES (Sec. 5: right-preconditioned restarted GMRES, zero start,
# relative-residual stopping rule)
# ---------------------------------------------------------------------------

class GmresResult:
    def __init__(self, x, iters, restarts, relres, history, converged, H=None,
                 V=None, Z=None):
        self.x = x
        self.iters = iters
        self.restarts = restarts
        self.relres = relres
        self.history = history
        self.converged = converged
        self.H = H
        self.V = V
        self.Z = Z


def gmres_right(matvec, precond, b, x0=None, m=20, rtol=1e-8, max_iters=1000,
                keep_basis=False):
    """Restarted right-preconditioned (flexible form) GMRES(m).

    Arnoldi by modified Gram-Schmidt on M P^{-1}; the preconditioned vectors
    z_j = P^{-1} v_j are stored so the update is x += Z y (identical to
    x += P^{-1} V y for a fixed P).  The cycle ends when the least-squares
    residual estimate reaches rtol ||b||, the restart length is reached or the
    iteration budget is spent; the true residual ||b - M x|| / ||b|| is then
    recomputed and decides convergence."""
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return GmresResult(np.zeros(n), 0, 0, 0.0, [0.0], True)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    relres = beta / bnorm
    history = [relres]
    iters = 0
    restarts = 0
    last = None
    while relres > rtol and iters < max_iters:
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        V[0] = r / beta
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            iters += 1
            # residual estimate from the small least-squares problem
            e1 = np.zeros(k + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
            est = np.linalg.norm(e1 - H[:k + 1, :k] @ y)
            history.append(est / bnorm)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            if H[j + 1, j] == 0.0 or est <= rtol * bnorm or iters >= max_iters:
                break
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        relres = beta / bnorm
        last = (H[:k + 1, :k], V[:k + 1], Z[:k])
        if relres > rtol and iters < max_iters:
            restarts += 1
    res = GmresResult(x, iters, restarts, relres, history, relres <= rtol)
    if keep_basis and last is not None:
        res.H, res.V, res.Z = last
    return res


def cn_gmres_solve(lo, di, up, T, nt, alpha, b, x0=None, m=20, rtol=1e-8,
                   max_iters=1000, keep_basis=False):
    """Right-preconditioned GMRES(m) on M u = b with P_alpha (Sec. 5 setup)."""
    mv = lambda u: aao_matvec(lo, di, up, T, nt, u)
    pc = lambda v: pc_apply(lo, di, up, T, nt, alpha, v)
    return gmres_right(mv, pc, b, x0=x0, m=m, rtol=rtol, max_iters=max_iters,
                       keep_basis=keep_basis)


# ---------------------------------------------------------------------------
# Spectra (Sec. 3.2) -- dense, tiny sizes only
# ---------------------------------------------------------------------------

def preconditioned_spectrum(lo, di, up, T, nt, alpha):
    """Eigenvalues of P_alpha^{-1} M (dense)."""
    import scipy.linalg
    M = aao_matrix_dense(lo, di, up, T, nt)
    P = pc_matrix_dense(lo, di, up, T, nt, alpha)
    return scipy.linalg.eigvals(np.linalg.solve(P, M))
