"""CPU FP64 oracle for the all-at-once Crank-Nicolson system of a 2D spatial
operator and the three-step inverse of its alpha-circulant preconditioner.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never calls it and shares no code with it.

The spatial operator of the paper's 2D experiments (Sec. 5, eq. (5.1) and
the SABR operator after it) is a sparse N_x N_y x N_x N_y matrix A; the
all-at-once matrix (eq. (2.2)) and the preconditioner (eq. (3.1)) are built
from A~ = tau A exactly as in one dimension, and step (b) of eq. (3.2)
becomes one complex-shifted sparse solve (lambda_{1,j} I - lambda_{2,j} A~)
per frequency j.

Grid and stencil convention (shared with the GPU path only as an input
format): grid point (iy, ix), 0 <= ix < N_x, 0 <= iy < N_y, is unknown
i = iy N_x + ix (x fastest).  A is given as nine coefficient arrays
st[q, i], q = 3 (dy + 1) + (dx + 1) for dy, dx in {-1, 0, 1}: row i of A
has st[q, i] in the column of grid point (iy + dy, ix + dx), and entries
whose neighbour lies outside the grid are ignored (homogeneous Dirichlet
data outside the grid).

Everything is float64 / complex128; the time DFT is written as direct
O(N_t^2) sums and each shifted system is solved by a sparse direct solver
(SuperLU through scipy), never by the GPU path's band factorisation.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import cn_oracle as O1

OFFSETS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# ---------------------------------------------------------------------------
# the spatial operator
# ---------------------------------------------------------------------------

def stencil_matrix(st, nx, ny):
    """Sparse A (CSR) from the nine coefficient arrays (see the module
    docstring), written out point by point."""
    st = np.asarray(st, dtype=np.float64).reshape(9, nx * ny)
    rows, cols, vals = [], [], []
    for iy in range(ny):
        for ix in range(nx):
            i = iy * nx + ix
            for q, (dy, dx) in enumerate(OFFSETS):
                jy, jx = iy + dy, ix + dx
                if 0 <= jy < ny and 0 <= jx < nx and st[q, i] != 0.0:
                    rows.append(i)
                    cols.append(jy * nx + jx)
                    vals.append(st[q, i])
    n = nx * ny
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


# ---------------------------------------------------------------------------
# the all-at-once system (eq. (2.2), block form of Sec. 3.2)
# ---------------------------------------------------------------------------

def aao_matrix_dense(A, T, nt):
    """M = B1 (x) I - B2 (x) A~ (eq. (2.2)), dense; A dense or sparse."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    tau = T / nt
    n = A.shape[0]
    B1 = np.eye(nt) - np.eye(nt, k=-1)
    B2 = 0.5 * (np.eye(nt) + np.eye(nt, k=-1))
    return np.kron(B1, np.eye(n)) - np.kron(B2, tau * A)


def aao_matvec(A, T, nt, u):
    """y = M u block by block: y^k = (u^k - u^{k-1}) - (A~/2)(u^k + u^{k-1}),
    u^0 := 0 (Sec. 3.2)."""
    tau = T / nt
    n = A.shape[0]
    U = np.asarray(u, dtype=np.float64).reshape(nt, n)
    Up = np.vstack([np.zeros((1, n)), U[:-1]])
    return ((U - Up) - 0.5 * tau * (A @ (U + Up).T).T).reshape(-1)


def aao_rhs(A, T, nt, u0, f):
    """b = xi + tau f, xi = [(I + A~/2) u^0; 0; ...] (eq. (2.2)); f has the
    N_t source blocks f^{k+1/2}."""
    tau = T / nt
    n = A.shape[0]
    b = tau * np.asarray(f, dtype=np.float64).reshape(nt, n).copy()
    u0 = np.asarray(u0, dtype=np.float64)
    b[0] += u0 + 0.5 * tau * (A @ u0)
    return b.reshape(-1)


def sequential_cn(A, T, nt, u0, f):
    """Exact M^{-1} b by block forward substitution, i.e. CN time stepping
    (eq. (2.1)): (I - A~/2) u^{k+1} = (I + A~/2) u^k + tau f^{k+1/2}, with
    one sparse LU of (I - A~/2)."""
    tau = T / nt
    n = A.shape[0]
    I = sp.identity(n, format="csc")
    lu = spla.splu((I - 0.5 * tau * A).tocsc())
    F = np.asarray(f, dtype=np.float64).reshape(nt, n)
    u = np.asarray(u0, dtype=np.float64).copy()
    out = np.empty((nt, n))
    for k in range(nt):
        u = lu.solve(u + 0.5 * tau * (A @ u) + tau * F[k])
        out[k] = u
    return out.reshape(-1)


# ---------------------------------------------------------------------------
# the preconditioner (eq. (3.1)) and its three-step inverse (eq. (3.2))
# ---------------------------------------------------------------------------

def pc_matrix_dense(A, T, nt, alpha):
    """P_alpha = C1 (x) I - C2 (x) A~ (eq. (3.1)), dense."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    tau = T / nt
    C1, C2 = O1.alpha_circulants(alpha, nt)
    n = A.shape[0]
    return np.kron(C1, np.eye(n)) - np.kron(C2, tau * A)


def coupling_matrix_dense(A, T, nt):
    """R of Sec. 4 (P_alpha = M - alpha R): I + A~/2 in block (1, N_t)."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    tau = T / nt
    n = A.shape[0]
    R = np.zeros((nt * n, nt * n))
    R[:n, (nt - 1) * n:] = np.eye(n) + 0.5 * tau * A
    return R


def pc_apply(A, T, nt, alpha, v):
    """z = P_alpha^{-1} v by the three steps of eq. (3.2):
    (a) alpha-weighting and direct DFT sums along time;
    (b) for every frequency j (all N_t of them, no conjugate-pair halving)
        the sparse shifted solve (lambda_{1,j} I - lambda_{2,j} A~) z2_j = z1_j;
    (c) inverse DFT sums, 1/N_t, and the inverse weights."""
    tau = T / nt
    n = A.shape[0]
    V = np.asarray(v, dtype=np.float64).reshape(nt, n)
    lam = O1.alpha_weights(alpha, nt)
    W = O1.dft_matrix(nt)
    Z1 = W @ (lam[:, None] * V)
    l1, l2 = O1.pc_eigenvalues(alpha, nt)
    I = sp.identity(n, format="csc", dtype=np.complex128)
    At = (tau * A).tocsc().astype(np.complex128)
    Z2 = np.empty_like(Z1)
    for j in range(nt):
        Z2[j] = spla.spsolve(l1[j] * I - l2[j] * At, Z1[j])
    Zc = (W.conj() @ Z2) / nt / lam[:, None]
    scale = max(np.abs(Zc).max(), 1e-300)
    if np.abs(Zc.imag).max() > 1e-10 * scale:
        raise AssertionError("preconditioned vector is not real")
    return Zc.real.reshape(-1)


def pc_matvec(A, T, nt, alpha, z):
    """y = P_alpha z block by block (eq. (3.1)): as M, with alpha z^{N_t} in
    place of the (zero) block before the first."""
    tau = T / nt
    n = A.shape[0]
    Z = np.asarray(z, dtype=np.float64).reshape(nt, n)
    Zp = np.roll(Z, 1, axis=0)
    Zp[0] *= alpha
    return ((Z - Zp) - 0.5 * tau * (A @ (Z + Zp).T).T).reshape(-1)


def preconditioned_spectrum(A, T, nt, alpha):
    """Eigenvalues of P_alpha^{-1} M (dense, tiny sizes)."""
    import scipy.linalg
    M = aao_matrix_dense(A, T, nt)
    P = pc_matrix_dense(A, T, nt, alpha)
    return scipy.linalg.eigvals(np.linalg.solve(P, M))
