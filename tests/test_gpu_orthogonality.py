"""Orthogonality of the Arnoldi basis built by the one-pass Gram-Schmidt step.

The update forms v_{j+1} = w - Q c with c = h1 + (I - G) h1, h1 = Q^T w and G
the Gram matrix of the stored, normalised basis Q (equal to CGS2 in exact
arithmetic).  With E = G - I, the new vector satisfies
    Q^T v_{j+1} = E^2 h1 + delta,   |delta| <~ (j+2) eps (||w|| + |Q| |c|),
so its normalised dots are bounded by about (j+2) eps kappa_j + ||E||^2, with
kappa_j = ||w_j|| / ||v_{j+1}|| the cancellation of step j (the column norm
of the least-squares factor over h_{j+1,j}).  Two-pass CGS2 removes the eps
kappa_j term; this scheme keeps it.  The tests read the stored basis back,
form Q^T Q independently, and check (i) the Gram matrix the solver records
equals it, (ii) every entry of Q^T Q - I is within the bound above, (iii)
the least-squares residual estimate tracks the true residual, and (iv) the
iteration count matches the oracle's modified Gram-Schmidt GMRES."""
import numpy as np
import pytest
import torch

from oracle import cn_oracle as O
from paper_2401_16113_amd import workloads as W

from gpu_helpers import T, banner, dev, solver

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


def basis_check(s, inst, res, rtol):
    assert res.restarts == 0 and res.iters >= 1
    k = res.iters
    gram, rfac, scale = s.cycle(k)
    vs = []
    for q in range(k + 1):
        out = torch.empty(inst.n, dtype=torch.float64, device=dev())
        s.basis(q, out)
        nrm = float(torch.linalg.vector_norm(out))
        if q >= 1:
            # the recorded scale is that of the stored vector
            assert abs(float(scale[q]) * nrm - 1.0) <= 1e-12
        vs.append(out / nrm)
    Q = torch.stack(vs)
    Gt = (Q @ Q.T).cpu().numpy()
    # (i) the recorded Gram matrix is that of the stored basis
    rec_err = float(np.max(np.abs(gram - Gt)))
    # (ii) per new vector v_{j+1}: its dots against the earlier basis
    worst = 0.0
    e_prev = 0.0
    for j in range(k):
        kappa = float(np.linalg.norm(rfac[j, :j + 1])) * float(scale[j + 1])
        bound = 4.0 * (j + 2) * EPS * max(kappa, 1.0) + (j + 1) * e_prev ** 2
        dots = np.abs(Gt[j + 1, :j + 1])
        worst = max(worst, float(np.max(dots) / bound))
        e_prev = max(e_prev, float(np.max(dots)))
    off = float(np.max(np.abs(Gt - np.eye(k + 1))))
    print(f"  k={k} max|QtQ-I|={off:.2e} recorded-vs-recomputed={rec_err:.2e} "
          f"worst dot/bound={worst:.2f} est={res.relres_est:.2e} true={res.relres_true:.2e}")
    assert rec_err <= 1e-13
    assert worst <= 1.0
    # (iii) the estimate tracks the true residual
    assert res.relres_true <= rtol
    assert abs(res.relres_est - res.relres_true) <= 0.25 * res.relres_true + 64 * EPS
    return k, off


@pytest.mark.parametrize("alpha", [0.01, 0.3, 0.9])
def test_basis_orthogonality_constant_volatility(alpha):
    """127 x 64 workload, float64 preconditioner, GMRES(30) to 1e-13 in one
    cycle (alpha up to 0.9 for longer cycles)."""
    inst = W.config1()
    banner(f"orthogonality 127x64 alpha={alpha}")
    rtol = 1e-13
    s = solver(inst, pc_prec="fp64", m_max=30, alpha=alpha)
    b = torch.empty(inst.n, dtype=torch.float64, device=dev())
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    x = torch.empty_like(b)
    res = s.solve(b, x, m=30, rtol=rtol, max_iters=30)
    k, off = basis_check(s, inst, res, rtol)
    # (iv) the same iteration count as the oracle's MGS GMRES (within one)
    args = (inst.a_lo, inst.a_di, inst.a_up, inst.T, inst.nt)
    bh = O.aao_rhs(*args, inst.u0, inst.f)
    ref = O.cn_gmres_solve(*args, alpha, bh, m=30, rtol=rtol, max_iters=30)
    assert abs(res.iters - ref.iters) <= 1, (res.iters, ref.iters)
    s.close()


def test_basis_orthogonality_local_volatility_fp32():
    """4095 x 1024 local-volatility workload, alpha = 0.05, float32
    preconditioner (flexible GMRES), GMRES(30) to 1e-8."""
    inst = W.config2(alpha=0.05, pc_prec="fp32")
    banner("orthogonality 4095x1024 alpha=0.05 fp32")
    rtol = 1e-8
    s = solver(inst, pc_prec="fp32", m_max=30)
    b = torch.empty(inst.n, dtype=torch.float64, device=dev())
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    x = torch.empty_like(b)
    res = s.solve(b, x, m=30, rtol=rtol)
    basis_check(s, inst, res, rtol)
    s.close()
