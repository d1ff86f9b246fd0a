"""Pins of the 2D oracle (oracle/cn2d_oracle.py) against what the paper and
the mathematics fix, independently of the oracle's own formulas:

* the stencil assembly against the Kronecker form of the same central
  differences (Sec. 5's operators are sums of such terms);
* the block forms of M and P_alpha against their dense Kronecker forms
  (eqs. (2.2), (3.1)), P_alpha = M - alpha R (Sec. 4), and the three-step
  apply (eq. (3.2)) against a dense solve with P_alpha;
* Lemma 3.1 for a separable constant-coefficient operator, whose
  eigenvalues are sums of the textbook 1D Toeplitz eigenvalues;
* Thm 3.1's annulus for a variable-coefficient operator;
* CN time stepping as the exact inverse of M, and its second-order
  convergence to the closed-form solution of an anisotropic heat equation;
* planted mistakes (x and y swapped in the stencil, a conjugated shift in
  step (b)) trip the pins.
"""
import numpy as np
import pytest

from oracle import cn2d_oracle as O2
from paper_2401_16113_amd import workloads as W


def kron_operator(nx, ny, a, b, c, d, e, r):
    """The same central differences as Kronecker products of 1D matrices
    (constant coefficients), x fastest: A = a I(x)T2x + b T2y(x)I +
    c D1y(x)D1x + d I(x)D1x + e D1y(x)I - r I."""
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    T2 = lambda m, h: (np.eye(m, k=-1) - 2 * np.eye(m) + np.eye(m, k=1)) / h ** 2
    D1 = lambda m, h: (np.eye(m, k=1) - np.eye(m, k=-1)) / (2 * h)
    Ix, Iy = np.eye(nx), np.eye(ny)
    return (a * np.kron(Iy, T2(nx, hx)) + b * np.kron(T2(ny, hy), Ix)
            + c * np.kron(D1(ny, hy), D1(nx, hx)) + d * np.kron(Iy, D1(nx, hx))
            + e * np.kron(D1(ny, hy), Ix) - r * np.eye(nx * ny))


def const_stencil(nx, ny, a=0.7, b=0.3, c=0.2, d=0.5, e=-0.4, r=0.1):
    return W.drift_diffusion_2d_stencil(nx, ny, a, b, c, d, e, r)


@pytest.mark.parametrize("nx,ny", [(5, 4), (7, 3), (1, 6), (6, 1)])
def test_stencil_assembly_equals_kronecker_form(nx, ny):
    A = O2.stencil_matrix(const_stencil(nx, ny), nx, ny).toarray()
    K = kron_operator(nx, ny, 0.7, 0.3, 0.2, 0.5, -0.4, 0.1)
    assert np.max(np.abs(A - K)) <= 1e-12 * np.max(np.abs(K))


def test_planted_swapped_axes_are_caught(monkeypatch):
    swapped = [(dx, dy) for dy, dx in O2.OFFSETS]
    monkeypatch.setattr(O2, "OFFSETS", swapped)
    nx, ny = 5, 4
    A = O2.stencil_matrix(const_stencil(nx, ny), nx, ny).toarray()
    K = kron_operator(nx, ny, 0.7, 0.3, 0.2, 0.5, -0.4, 0.1)
    assert np.max(np.abs(A - K)) > 1e-3 * np.max(np.abs(K))


def small_instance(nx=4, ny=3, nt=4, mixed=0.0, seed=21):
    inst = W.drift_diffusion_2d(nx, ny, nt, mixed=mixed, seed=seed)
    return inst, O2.stencil_matrix(inst.st, nx, ny)


@pytest.mark.parametrize("mixed", [0.0, 0.3])
def test_block_forms_equal_dense_forms(mixed):
    inst, A = small_instance(mixed=mixed)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(inst.n)
    M = O2.aao_matrix_dense(A, inst.T, inst.nt)
    assert np.allclose(O2.aao_matvec(A, inst.T, inst.nt, u), M @ u, rtol=0, atol=1e-12)
    P = O2.pc_matrix_dense(A, inst.T, inst.nt, 0.05)
    assert np.allclose(O2.pc_matvec(A, inst.T, inst.nt, 0.05, u), P @ u, rtol=0, atol=1e-12)
    R = O2.coupling_matrix_dense(A, inst.T, inst.nt)
    assert np.max(np.abs(P - (M - 0.05 * R))) <= 1e-14


@pytest.mark.parametrize("mixed,alpha", [(0.0, 0.01), (0.3, 0.05), (0.0, 0.5)])
def test_pc_apply_inverts_dense_preconditioner(mixed, alpha):
    inst, A = small_instance(nx=5, ny=4, nt=8, mixed=mixed)
    v = np.random.default_rng(2).standard_normal(inst.n)
    z = O2.pc_apply(A, inst.T, inst.nt, alpha, v)
    P = O2.pc_matrix_dense(A, inst.T, inst.nt, alpha)
    ref = np.linalg.solve(P, v)
    assert np.max(np.abs(z - ref)) <= 1e-11 * np.max(np.abs(ref))


def test_planted_conjugated_shift_is_caught(monkeypatch):
    real_eig = O2.O1.pc_eigenvalues
    monkeypatch.setattr(O2.O1, "pc_eigenvalues",
                        lambda a, nt: tuple(np.conj(x) for x in real_eig(a, nt)))
    inst, A = small_instance(nx=5, ny=4, nt=8)
    v = np.random.default_rng(2).standard_normal(inst.n)
    P = O2.pc_matrix_dense(A, inst.T, inst.nt, 0.05)
    ref = np.linalg.solve(P, v)
    try:
        z = O2.pc_apply(A, inst.T, inst.nt, 0.05, v)
    except AssertionError:
        return  # the non-real result is itself caught
    assert np.max(np.abs(z - ref)) > 1e-6 * np.max(np.abs(ref))


def R_cn(z):
    return (1 + z / 2) / (1 - z / 2)


@pytest.mark.parametrize("nx,ny,nt,alpha", [(4, 3, 4, 0.05), (3, 5, 6, 0.01)])
def test_spectrum_separable_closed_form(nx, ny, nt, alpha):
    """Lemma 3.1: (N_t-1) N_x N_y eigenvalues of P_alpha^{-1} M equal 1; the
    others are 1/(1 - alpha R(tau mu)^{N_t}) over the eigenvalues mu of A,
    which for a u_xx + b u_yy - r u are the sums
    -r - (4a/hx^2) sin^2(i pi/(2(N_x+1))) - (4b/hy^2) sin^2(l pi/(2(N_y+1)))."""
    a, b, r, T = 0.7, 0.3, 0.1, 0.5
    st = W.drift_diffusion_2d_stencil(nx, ny, a, b, 0.0, 0.0, 0.0, r)
    A = O2.stencil_matrix(st, nx, ny)
    ev = O2.preconditioned_spectrum(A, T, nt, alpha)
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    sx = np.sin(np.arange(1, nx + 1) * np.pi / (2 * (nx + 1))) ** 2
    sy = np.sin(np.arange(1, ny + 1) * np.pi / (2 * (ny + 1))) ** 2
    mu = (-r - 4 * a / hx ** 2 * sx[None, :] - 4 * b / hy ** 2 * sy[:, None]).reshape(-1)
    closed = 1.0 / (1.0 - alpha * R_cn(T / nt * mu) ** nt)
    # the expected multiset: (N_t - 1) N_x N_y ones and the closed forms (a
    # closed form may itself be 1 to rounding, when R(tau mu) is tiny)
    expected = np.concatenate([np.ones((nt - 1) * nx * ny), closed])
    left = list(ev)
    for cval in sorted(expected, key=lambda z: (z.real, z.imag)):
        k = int(np.argmin([abs(x - cval) for x in left]))
        assert abs(left[k] - cval) <= 1e-8 * max(1.0, abs(cval))
        left.pop(k)


@pytest.mark.parametrize("alpha", [0.01, 0.05, 0.3])
def test_spectrum_annulus_variable_coefficients(alpha):
    """Thm 3.1: every eigenvalue of P_alpha^{-1} M lies in the annulus
    1/(1+alpha) <= |z| <= 1/(1-alpha) when Re lambda(A) <= 0."""
    inst, A = small_instance(nx=5, ny=4, nt=6)
    assert np.max(np.linalg.eigvals(A.toarray()).real) <= 0
    ev = O2.preconditioned_spectrum(A, inst.T, inst.nt, alpha)
    assert np.all(np.abs(ev) >= 1 / (1 + alpha) - 1e-10)
    assert np.all(np.abs(ev) <= 1 / (1 - alpha) + 1e-10)


@pytest.mark.parametrize("mixed", [0.0, 0.3])
def test_sequential_cn_is_exact_inverse(mixed):
    inst, A = small_instance(nx=5, ny=4, nt=6, mixed=mixed)
    b = O2.aao_rhs(A, inst.T, inst.nt, inst.u0, inst.f)
    u = O2.sequential_cn(A, inst.T, inst.nt, inst.u0, inst.f)
    M = O2.aao_matrix_dense(A, inst.T, inst.nt)
    ref = np.linalg.solve(M, b)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_cn_second_order_anisotropic_heat():
    """u_t = a u_xx + b u_yy on the unit square, u0 = sin(pi x) sin(2 pi y):
    u(T) = exp(-(a + 4b) pi^2 T) u0.  The CN solution's error at T falls by
    about 4 when h and tau are halved (O(h^2 + tau^2)); the mode's y
    frequency differs from its x frequency, so swapping the axes (or a or b)
    changes the decay rate and is caught."""
    a, b, T = 0.2, 0.1, 0.25
    errs = []
    for m in (15, 31, 63):
        nx = ny = m
        nt = m + 1
        st = W.drift_diffusion_2d_stencil(nx, ny, a, b, 0.0, 0.0, 0.0, 0.0)
        A = O2.stencil_matrix(st, nx, ny)
        h = 1.0 / (m + 1)
        X, Y = np.meshgrid(np.arange(1, m + 1) * h, np.arange(1, m + 1) * h)
        u0 = (np.sin(np.pi * X) * np.sin(2 * np.pi * Y)).reshape(-1)
        u = O2.sequential_cn(A, T, nt, u0, np.zeros((nt, m * m)))
        exact = np.exp(-(a + 4 * b) * np.pi ** 2 * T) * u0
        errs.append(np.max(np.abs(u.reshape(nt, -1)[-1] - exact)))
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(3.6 <= q <= 4.4 for q in ratios), (errs, ratios)
