"""2D spatial operators (Sec. 5's setting): the all-at-once matvec, the
right-hand side and the preconditioner apply of cn_aao2d.h against the 2D
oracle, element by element, over tile counts with ragged tails, both band
widths of the substitution kernel (half-bandwidth N_x + 1 up to 64 and up to
128), a single grid row, N_t = 1 and a mixed-derivative operator."""
import numpy as np
import pytest
import torch

from oracle import cn2d_oracle as O2
from oracle import cn_oracle as O1
from paper_2401_16113_amd import binding as B
from paper_2401_16113_amd import workloads as W
from gpu_helpers import T, banner, rel_inf

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps

# (nx, ny, nt, mixed): 16-point transform tiles with ragged tails (851 and
# 4161 points), half-bandwidths 1 (one grid row), 6, 64 and 128
CASES = [(1, 1, 1, 0.0), (5, 4, 8, 0.0), (37, 23, 64, 0.0), (40, 1, 32, 0.0),
         (63, 63, 64, 0.0), (127, 33, 16, 0.0), (31, 17, 128, 0.2), (9, 7, 1024, 0.0)]


def setup(nx, ny, nt, mixed):
    inst = W.drift_diffusion_2d(nx, ny, nt, mixed=mixed)
    A = O2.stencil_matrix(inst.st, nx, ny)
    s = B.Solver2D(T(inst.st.reshape(-1)), nx, ny, nt, inst.T, inst.alpha)
    return inst, A, s


@pytest.mark.parametrize("nx,ny,nt,mixed", CASES)
def test_matvec_and_rhs_match_oracle(nx, ny, nt, mixed):
    banner(f"2d matvec/rhs {nx}x{ny}x{nt} mixed={mixed}")
    inst, A, s = setup(nx, ny, nt, mixed)
    x = W.random_vector(inst.n, 3)
    y = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.matvec(T(x), y)
    assert rel_inf(y.cpu().numpy(), O2.aao_matvec(A, inst.T, nt, x)) <= 1e-13
    b = torch.empty_like(y)
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    assert rel_inf(b.cpu().numpy(), O2.aao_rhs(A, inst.T, nt, inst.u0, inst.f)) <= 1e-13
    s.close()


def pc_tol(inst, A):
    """As for the 1D apply: 2 N_t eps / alpha for the transforms and the
    shifted systems' conditioning, 1 + tau ||A||_inf / mu_0 with
    mu_0 = 2 (1 - alpha^{1/N_t}) / (1 + alpha^{1/N_t}), times eps."""
    q = inst.alpha ** (1.0 / inst.nt)
    mu0 = 2.0 * (1.0 - q) / (1.0 + q)
    norm = inst.T / inst.nt * abs(A).sum(axis=1).max()
    return max(2.0 * inst.nt * EPS64 / inst.alpha, 1e-14) + EPS64 * (1.0 + norm / mu0)


@pytest.mark.parametrize("nx,ny,nt,mixed", CASES)
def test_pc_apply_matches_oracle(nx, ny, nt, mixed):
    banner(f"2d pc_apply {nx}x{ny}x{nt} mixed={mixed}")
    inst, A, s = setup(nx, ny, nt, mixed)
    v = W.random_vector(inst.n, 4)
    z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.pc_apply(T(v), z)
    ref = O2.pc_apply(A, inst.T, nt, inst.alpha, v)
    err = rel_inf(z.cpu().numpy(), ref)
    tol = pc_tol(inst, A)
    print(f"  error {err:.2e} (bar {tol:.2e})", flush=True)
    assert err <= tol
    # in place, and a second call gives the same bits
    z2 = T(v)
    s.pc_apply(z2, z2)
    assert torch.equal(z2, z)
    s.close()


def test_pc_apply_inverts_preconditioner_matrix():
    """P_alpha z = v through the oracle's block form of eq. (3.1)."""
    inst, A, s = setup(63, 63, 64, 0.0)
    v = W.random_vector(inst.n, 5)
    z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.pc_apply(T(v), z)
    res = O2.pc_matvec(A, inst.T, inst.nt, inst.alpha, z.cpu().numpy()) - v
    assert np.abs(res).max() <= pc_tol(inst, A) * np.abs(v).max()
    s.close()


def test_create_rejects_bad_problems():
    inst = W.drift_diffusion_2d(8, 8, 8)
    st = T(inst.st.reshape(-1))
    for kw in (dict(nx=128, ny=2), dict(nx=100, ny=100), dict(nx=8, ny=8, nt=12),
               dict(nx=8, ny=8, nt=2048), dict(nx=8, ny=8, alpha=1.0)):
        args = dict(nx=8, ny=8, nt=8, T=0.5, alpha=0.01)
        args.update(kw)
        with pytest.raises(B.CnError) as ei:
            B.Solver2D(st, **args)
        assert ei.value.status == B.CN_EINVAL


@pytest.mark.parametrize("nx,ny,nt,mixed", [(31, 17, 32, 0.0), (63, 63, 64, 0.0), (37, 23, 128, 0.2)])
def test_gmres_solve_matches_cn_time_stepping(nx, ny, nt, mixed):
    """Flexible GMRES(20) with P_alpha on the 2D system to relres 1e-10
    against the oracle's CN time stepping (the exact M^{-1} b), and its
    iteration count against the oracle's right-preconditioned GMRES."""
    banner(f"2d gmres {nx}x{ny}x{nt} mixed={mixed}")
    inst = W.drift_diffusion_2d(nx, ny, nt, mixed=mixed)
    A = O2.stencil_matrix(inst.st, nx, ny)
    s = B.Solver2D(T(inst.st.reshape(-1)), nx, ny, nt, inst.T, inst.alpha, m_max=20)
    b = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    x = torch.full_like(b, 3.0)      # ignored: zero start
    r = s.solve(b, x, m=20, rtol=1e-10)
    u = O2.sequential_cn(A, inst.T, nt, inst.u0, inst.f)
    err = rel_inf(x.cpu().numpy(), u)
    bh = O2.aao_rhs(A, inst.T, nt, inst.u0, inst.f)
    ref = O1.gmres_right(lambda v: O2.aao_matvec(A, inst.T, nt, v),
                         lambda v: O2.pc_apply(A, inst.T, nt, inst.alpha, v), bh, m=20, rtol=1e-10)
    print(f"  iterations {r.iters} (oracle {ref.iters}), relres {r.relres_true:.2e}, "
          f"error {err:.2e}", flush=True)
    assert r.status == B.CN_OK and r.relres_true <= 1e-10
    assert err <= 1e-8
    assert abs(r.iters - ref.iters) <= 1
    # restarts (m = 2) and a warm start from the solution
    x2 = torch.empty_like(b)
    r2 = s.solve(b, x2, m=2, rtol=1e-10)
    assert r2.status == B.CN_OK and r2.restarts >= 1
    assert rel_inf(x2.cpu().numpy(), u) <= 1e-8
    r3 = s.solve(b, x, m=20, rtol=1e-8, use_x0=True)
    assert r3.status == B.CN_OK and r3.iters == 0
    # b = 0: x = 0 whatever the guess
    z0 = torch.zeros_like(b)
    r4 = s.solve(z0, x, m=20, rtol=1e-8, use_x0=True)
    assert r4.status == B.CN_OK and r4.iters == 0 and float(x.abs().max()) == 0.0
    s.close()
