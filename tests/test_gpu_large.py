"""Production shape: N_x = 65535, N_t = 4096 (2.7e8 unknowns, a 47 GB
Krylov basis), float32 preconditioner inside float64 flexible GMRES(20),
alpha = 0.01, with error-controlled stopping.  Checked at full size against the oracle's CN time stepping
(block forward substitution, Sec. 2.2, with banded solves), and the
preconditioner apply through the operator that defines it (eq. (3.1)):
P_alpha z must give back v."""
import numpy as np
import pytest
import torch

from oracle import cn_oracle as O
from paper_2401_16113_amd import binding as B
from paper_2401_16113_amd import workloads as W
from gpu_helpers import T, banner, rel_inf, solver

pytestmark = pytest.mark.gpu


def test_production_shape_solve_and_preconditioner():
    banner("production shape 65535x4096 fp32 preconditioner")
    inst = W.config5()
    args = (inst.a_lo, inst.a_di, inst.a_up, inst.T, inst.nt)
    s = solver(inst)
    b = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    x = torch.empty_like(b)
    r = s.solve(b, x, m=20, rtol=1e-8, err_tol=5e-8)
    print(f"iterations {r.iters}, relres {r.relres_true:.3e}, error estimate {r.err_est:.3e}, "
          f"{r.seconds * 1e3:.2f} ms", flush=True)
    assert r.status == B.CN_OK and r.relres_true <= 1e-8 and 0.0 <= r.err_est <= 5e-8
    assert r.iters <= 12
    u = O.sequential_cn_banded(*args, inst.u0, f_col=inst.f[:, 0])
    err = rel_inf(x.cpu().numpy(), u)
    print(f"error vs CN time stepping {err:.3e}", flush=True)
    assert err <= 1e-7
    assert 0.8 <= r.err_est / err <= 1.25
    del u
    # z = P^{-1} b in float32 arithmetic: its residual in the defining
    # operator is bounded like the apply's error, 0.1 N_t eps32 / alpha
    z = torch.empty_like(b)
    s.pc_apply(b, z)
    bh = b.cpu().numpy()
    res = np.linalg.norm(O.pc_matvec(*args, inst.alpha, z.cpu().numpy()) - bh) / np.linalg.norm(bh)
    print(f"preconditioner residual {res:.3e}", flush=True)
    assert res <= 0.1 * inst.nt * np.finfo(np.float32).eps / inst.alpha
    s.close()
