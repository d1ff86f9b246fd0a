"""The allocation-free preconditioner apply (cn_pc_apply_noalloc) against the
handle's apply (cn_pc_apply, same transform variant) and against the oracle,
on two calls in a row (the second on a smaller problem, which reuses the
library's fixed work array), in float64 and float32."""
import numpy as np
import pytest
import torch

from oracle import cn_oracle as O
from paper_2401_16113_amd import binding as B
from paper_2401_16113_amd import workloads as W

from gpu_helpers import T, banner, rel_inf, solver
from test_gpu_parity import oracle_args, pc_tol_wide, localvol

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_apply_matches_handle_apply(prec, monkeypatch):
    monkeypatch.setenv("CN_AUTOTUNE", "0")   # the handle takes the default variant too
    for (nx, nt, seed) in ((4095, 1024, 11), (1000, 128, 12)):
        banner(f"no-alloc apply {prec} {nx}x{nt}")
        inst = localvol(nx, nt, seed=seed)
        v = W.random_vector(inst.n, seed)
        vt = T(v)
        z_ref = torch.empty_like(vt)
        s = solver(inst, pc_prec=prec)
        s.pc_apply(vt, z_ref)
        z = torch.full_like(vt, np.nan)
        B.pc_apply_noalloc(T(inst.a_lo), T(inst.a_di), T(inst.a_up), inst.nt, inst.T,
                           inst.alpha, vt, z, pc_prec=prec)
        torch.cuda.synchronize()
        zh, zr = z.cpu().numpy(), z_ref.cpu().numpy()
        tol = pc_tol_wide(inst, prec)
        ref = O.pc_apply(*oracle_args(inst), inst.alpha, v)
        d_handle = rel_inf(zh, zr)
        d_oracle = rel_inf(zh, ref)
        print(f"  vs handle apply {d_handle:.2e}, vs oracle {d_oracle:.2e} (bar {tol:.2e})")
        assert np.all(np.isfinite(zh))
        assert d_handle <= tol and d_oracle <= tol
        s.close()


def test_noalloc_rejects_oversized_and_invalid():
    inst = localvol(4095, 8192)      # about 0.4 GB of work arrays: over the fixed size
    v = torch.zeros(inst.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CnError) as ei:
        B.pc_apply_noalloc(T(inst.a_lo), T(inst.a_di), T(inst.a_up), inst.nt, inst.T,
                           inst.alpha, v, v)
    assert ei.value.status == B.CN_EINVAL and "scratch" in str(ei.value)
    with pytest.raises(B.CnError) as ei:
        B.pc_apply_noalloc(T(inst.a_lo), T(inst.a_di), T(inst.a_up), inst.nt, inst.T,
                           1.0, v, v)
    assert ei.value.status == B.CN_EINVAL
