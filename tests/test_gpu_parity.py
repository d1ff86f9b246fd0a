"""GPU path vs the CPU oracle, element by element, through the C ABI.

Tolerances (relative infinity norm, normalised by max|reference|):
  * matvec, right-hand side: the same few float64 operations in a different
    order -> 1e-13.
  * preconditioner, float64: rounding of the length-N_t transforms
    (~log2(N_t) eps) and of the tile/interface elimination, amplified by the
    alpha unscaling alpha^{-k/N_t} <= 1/alpha (the roundoff caveat of Sec. 4)
    and by the conditioning of the shifted systems -> 2e-11 for alpha >= 0.01,
    2e-10 for alpha = 0.001.
  * preconditioner, float32: the same with eps_32 -> 5e-4 (alpha >= 0.01),
    5e-3 (alpha = 0.001).  Only its quality as a preconditioner matters: the
    flexible GMRES solution is held to the float64 bar below.
  * GMRES, float64 preconditioner, rtol 1e-12: 1e-9 against the exact M^{-1} b.
  * GMRES, float32 preconditioner or rtol 1e-8: 1e-7 (error ~10x relres).
"""
import numpy as np
import pytest
import torch

from oracle import cn_oracle as O
from paper_2401_16113_amd import binding as B
from paper_2401_16113_amd import workloads as W
from gpu_helpers import T, banner, rel_inf, solver

pytestmark = pytest.mark.gpu


def oracle_args(inst):
    return (inst.a_lo, inst.a_di, inst.a_up, inst.T, inst.nt)


_EXACT = {}


def exact(inst):
    """Block forward substitution (exact M^{-1} b), cached per workload."""
    key = (inst.name, inst.nx, inst.nt, inst.T, inst.r, inst.K, tuple(sorted(inst.params.items())))
    if key not in _EXACT:
        _EXACT[key] = O.sequential_cn(*oracle_args(inst), inst.u0, inst.f)
    return _EXACT[key]


def localvol(nx, nt, seed=7, alpha=0.01, T_=2.0):
    rng = np.random.default_rng(seed)
    a1, a2 = W.local_vol_amplitudes(rng)
    return W.make_instance(nx, nt, T=T_, r=0.03, K=1.0, sigma_fn=W.local_vol(a1, a2),
                           alpha=alpha, m=20, rtol=1e-8)


EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


def pc_tol(alpha, prec, nt):
    """Rounding of the three steps of eq. (3.2) grows like N_t/alpha: step (a)
    weights level k by alpha^(k/N_t); the lowest shifted system has
    |lambda_{1,0}| ~ |ln alpha|/N_t, so its solution is up to N_t/|ln alpha|
    times its right-hand side and carries the transform's rounding at that
    size; step (c) multiplies late levels by up to 1/alpha.  The error is
    C N_t eps/alpha with C = 2 (float64) and 0.1 (float32, where the float32
    stages round relative to a float64 input); measured C stays below 0.3
    and 0.01 on every shape tested."""
    if prec == "fp64":
        return max(2.0 * nt * EPS64 / alpha, 1e-14)
    return max(0.1 * nt * EPS32 / alpha, 1e-5)


def shifted_condition(inst):
    """Condition estimate of the worst shifted system of step (b) (Sec. 3.1):
    the lowest mode solves (mu_0 I - A~) with mu_0 = lambda_{1,0}/lambda_{2,0}
    = 2 (1 - alpha^{1/N_t}) / (1 + alpha^{1/N_t}), so kappa ~ 1 + ||A~|| / mu_0.
    It grows like N_x^2 N_t; on wide grids it, not N_t/alpha, sets the
    rounding floor of both the kernels and the oracle."""
    q = inst.alpha ** (1.0 / inst.nt)
    mu0 = 2.0 * (1.0 - q) / (1.0 + q)
    tau = inst.T / inst.nt
    norm = tau * np.max(np.abs(inst.a_lo) + np.abs(inst.a_di) + np.abs(inst.a_up))
    return 1.0 + norm / mu0


def pc_tol_wide(inst, prec):
    """pc_tol plus the shifted systems' conditioning times the precision."""
    eps = EPS64 if prec == "fp64" else EPS32
    return pc_tol(inst.alpha, prec, inst.nt) + eps * shifted_condition(inst)


# ---------------------------------------------------------------------------
# matvec and right-hand side
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,nt", [(1, 1), (7, 1), (5, 4), (127, 64), (300, 16), (1000, 128),
                                   (4095, 1024)])
def test_matvec_matches_oracle(nx, nt):
    banner(f"matvec nx={nx} nt={nt}")
    inst = localvol(nx, nt) if nx >= 255 else W.config1(nx=nx, nt=nt)
    s = solver(inst)
    x = W.random_vector(inst.n, 1)
    y = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.matvec(T(x), y)
    ref = O.aao_matvec(*oracle_args(inst), x)
    assert rel_inf(y.cpu().numpy(), ref) <= 1e-13


@pytest.mark.parametrize("nx,nt", [(1, 1), (127, 64), (4095, 1024)])
def test_rhs_matches_oracle(nx, nt):
    banner(f"rhs nx={nx} nt={nt}")
    inst = localvol(nx, nt) if nx >= 255 else W.config1(nx=nx, nt=nt)
    s = solver(inst)
    b = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    ref = O.aao_rhs(*oracle_args(inst), inst.u0, inst.f)
    assert rel_inf(b.cpu().numpy(), ref) <= 1e-13


# ---------------------------------------------------------------------------
# preconditioner
# ---------------------------------------------------------------------------

PC_CASES = [
    # (nx, nt): single tile, ragged last tile, exact multiple, tiny time axes
    (1, 1), (5, 1), (5, 2), (3, 4), (16, 8), (37, 8), (33, 16), (64, 32), (127, 64),
    (300, 128), (513, 256), (1000, 512), (200, 2048), (100, 4096), (50, 8192),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,nt", PC_CASES)
def test_pc_apply_matches_oracle(nx, nt, prec):
    banner(f"pc_apply {prec} nx={nx} nt={nt}")
    inst = localvol(nx, nt) if nx >= 255 else W.config1(nx=nx, nt=nt)
    s = solver(inst, pc_prec=prec)
    v = W.random_vector(inst.n, nx + nt)
    z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.pc_apply(T(v), z)
    ref = O.pc_apply(*oracle_args(inst), inst.alpha, v)
    err = rel_inf(z.cpu().numpy(), ref)
    print(f"  err={err:.3e} tiles={s.query()}")
    assert err <= pc_tol(inst.alpha, prec, nt)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("alpha", [0.001, 0.01, 0.05])
def test_pc_apply_localvol_workload_size(alpha, prec):
    """The 4095 x 1024 local-volatility workload, every element."""
    banner(f"pc_apply {prec} 4095x1024 alpha={alpha}")
    inst = W.config2(alpha=alpha, pc_prec=prec)
    s = solver(inst)
    v = W.random_vector(inst.n, 3)
    z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.pc_apply(T(v), z)
    ref = O.pc_apply(*oracle_args(inst), alpha, v)
    err = rel_inf(z.cpu().numpy(), ref)
    print(f"  err={err:.3e}")
    assert err <= pc_tol(alpha, prec, inst.nt)


def test_pc_apply_in_place_and_deterministic():
    banner("pc_apply in place / determinism")
    inst = localvol(1000, 256)
    s = solver(inst)
    v = T(W.random_vector(inst.n, 9))
    z1 = torch.empty_like(v)
    z2 = torch.empty_like(v)
    s.pc_apply(v, z1)
    s.pc_apply(v, z2)
    assert torch.equal(z1, z2)
    w = v.clone()
    s.pc_apply(w, w)
    assert torch.equal(w, z1)


# ---------------------------------------------------------------------------
# GMRES solves
# ---------------------------------------------------------------------------

def gpu_solve(inst, prec, rtol, m=None, alpha=None, x0=None, max_iters=1000):
    s = solver(inst, pc_prec=prec, alpha=alpha)
    b = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    x = T(x0) if x0 is not None else torch.empty_like(b)
    res = s.solve(b, x, m=m or inst.m, rtol=rtol, max_iters=max_iters, use_x0=x0 is not None)
    return res, x.cpu().numpy(), s, b


def test_gmres_config1_fp64_parity():
    """Constant-volatility workload (127 x 64), GMRES(20) to 1e-12: <= 1e-9."""
    banner("gmres config1 fp64")
    inst = W.config1()
    res, x, _, _ = gpu_solve(inst, "fp64", 1e-12, m=20)
    u = exact(inst)
    orc = O.cn_gmres_solve(*oracle_args(inst), inst.alpha,
                           O.aao_rhs(*oracle_args(inst), inst.u0, inst.f), m=20, rtol=1e-12)
    err = rel_inf(x, u)
    print(f"  iters={res.iters} (oracle {orc.iters}) relres={res.relres_true:.2e} err={err:.2e}")
    assert res.status == B.CN_OK and res.relres_true <= 1e-12
    assert err <= 1e-9
    assert rel_inf(x, orc.x) <= 1e-9
    assert abs(res.iters - orc.iters) <= 1


@pytest.mark.parametrize("alpha", [0.001, 0.01, 0.05])
def test_gmres_config2_fp64_tight(alpha):
    banner(f"gmres config2 fp64 alpha={alpha} rtol=1e-12")
    inst = W.config2(alpha=alpha)
    res, x, _, _ = gpu_solve(inst, "fp64", 1e-12, m=30)
    u = exact(inst)
    err = rel_inf(x, u)
    print(f"  iters={res.iters} relres={res.relres_true:.2e} err={err:.2e}")
    assert res.status == B.CN_OK
    assert err <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("alpha", [0.001, 0.01, 0.05])
def test_gmres_config2_rtol_1e8(alpha, prec):
    """Flexible GMRES(30) to relres 1e-8: error <= 1e-7 for both precisions."""
    banner(f"gmres config2 {prec} alpha={alpha} rtol=1e-8")
    inst = W.config2(alpha=alpha, pc_prec=prec)
    res, x, _, _ = gpu_solve(inst, prec, 1e-8, m=30)
    u = exact(inst)
    err = rel_inf(x, u)
    print(f"  iters={res.iters} relres={res.relres_true:.2e} err={err:.2e} t={res.seconds*1e3:.2f}ms")
    assert res.status == B.CN_OK and res.relres_true <= 1e-8
    assert err <= 1e-7


def test_gmres_deterministic():
    banner("gmres determinism")
    inst = localvol(1000, 256)
    r1, x1, _, _ = gpu_solve(inst, "fp32", 1e-10)
    r2, x2, _, _ = gpu_solve(inst, "fp32", 1e-10)
    assert r1.iters == r2.iters and np.array_equal(x1, x2)


def test_gmres_restarts_and_budget():
    banner("gmres restarts / budget")
    inst = localvol(255, 64)
    u = exact(inst)
    res, x, _, _ = gpu_solve(inst, "fp64", 1e-11, m=2)
    assert res.status == B.CN_OK and res.restarts >= 1
    assert rel_inf(x, u) <= 1e-8
    res, x, _, _ = gpu_solve(inst, "fp64", 1e-14, m=20, max_iters=1)
    assert res.status == B.CN_NOT_CONVERGED and res.iters == 1


def test_gmres_warm_exact_start_and_zero_rhs():
    banner("gmres exact x0 / zero b")
    inst = localvol(255, 64)
    u = exact(inst)
    res, x, _, _ = gpu_solve(inst, "fp64", 1e-8, x0=u)
    assert res.status == B.CN_OK and res.iters == 0
    s = solver(inst)
    b = torch.zeros(inst.n, dtype=torch.float64, device="cuda")
    xx = torch.full_like(b, 3.0)
    r = s.solve(b, xx, m=5, rtol=1e-8)
    assert r.status == B.CN_OK and r.iters == 0 and torch.count_nonzero(xx) == 0


@pytest.mark.parametrize("nx,nt", [(1, 1), (1, 8), (9, 1), (40, 2)])
def test_gmres_degenerate_shapes(nx, nt):
    banner(f"gmres degenerate nx={nx} nt={nt}")
    inst = W.config1(nx=max(nx, 1), nt=nt)
    res, x, _, _ = gpu_solve(inst, "fp64", 1e-12, m=10)
    u = exact(inst)
    assert res.status == B.CN_OK and rel_inf(x, u) <= 1e-9


def test_time_dependent_weights():
    """L(t) = d(t) L (Sec. 5.2): matvec and rhs with D~ B2, preconditioner
    with the mean weight times C2."""
    banner("time-dependent weights")
    inst = localvol(255, 64)
    th = (np.arange(inst.nt) + 0.5) * inst.T / inst.nt
    d = np.exp(-0.05 * th)
    s = solver(inst, d_half=d)
    x = W.random_vector(inst.n, 4)
    y = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.matvec(T(x), y)
    assert rel_inf(y.cpu().numpy(), O.aao_matvec(*oracle_args(inst), x, d=d)) <= 1e-13
    b = torch.empty_like(y)
    s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
    assert rel_inf(b.cpu().numpy(), O.aao_rhs(*oracle_args(inst), inst.u0, inst.f, d=d)) <= 1e-13
    xx = torch.empty_like(b)
    r = s.solve(b, xx, m=20, rtol=1e-12)
    u = O.sequential_cn(*oracle_args(inst), inst.u0, inst.f, d=d)
    assert r.status == B.CN_OK and rel_inf(xx.cpu().numpy(), u) <= 1e-9
    v = W.random_vector(inst.n, 5)
    z = torch.empty_like(b)
    s.pc_apply(T(v), z)
    ref = O.pc_apply(*oracle_args(inst), inst.alpha, v, dbar=float(np.mean(d)))
    assert rel_inf(z.cpu().numpy(), ref) <= pc_tol(inst.alpha, "fp64", inst.nt)


# ---------------------------------------------------------------------------
# error paths on the device side
# ---------------------------------------------------------------------------

def test_alpha_one_singular_operator():
    """Remark 2: alpha = 1 with a singular A makes P_1 singular."""
    banner("alpha=1 singular")
    nx = 20
    z = np.zeros(nx)
    with pytest.raises(B.CnError) as ei:
        B.Solver(T(z), T(z), T(z), 8, 1.0, 1.0, m_max=5, flags=B.CN_FLAG_ALLOW_ALPHA_ONE)
    assert ei.value.status == B.CN_ESINGULAR
    # the same operator is fine for alpha < 1 (lambda_{1,j} != 0)
    s = B.Solver(T(z), T(z), T(z), 8, 1.0, 0.5, m_max=5)
    s.close()


def test_alpha_one_nonsingular_comparator():
    """P_1 (alpha = 1) is a valid preconditioner for nonsingular A."""
    banner("alpha=1 comparator")
    inst = W.config1(nx=63, nt=32)
    s = solver(inst, alpha=1.0, flags=B.CN_FLAG_ALLOW_ALPHA_ONE)
    v = W.random_vector(inst.n, 2)
    zz = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.pc_apply(T(v), zz)
    ref = O.pc_apply(*oracle_args(inst), 1.0, v)
    # P_1's lowest shifted system is -A~ alone (lambda_{1,0} = 0): cond ~ 1/(tau r)
    assert rel_inf(zz.cpu().numpy(), ref) <= 1e-11


def test_aliasing_rejected():
    banner("aliasing")
    inst = W.config1(nx=31, nt=8)
    s = solver(inst)
    x = torch.zeros(inst.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.CnError):
        s.matvec(x, x)
    with pytest.raises(B.CnError):
        s.solve(x, x)
    with pytest.raises(B.CnError):
        s.solve(x, torch.empty_like(x), m=inst.m + 1)


# ---------------------------------------------------------------------------
# every compiled (tile width, workgroup size) variant of the transform kernels
# ---------------------------------------------------------------------------

# (tile columns, threads, inverse-transform workgroups per tile,
#  forward transform by frequency parity: 2)
VARIANTS = [(16, 256, 1, 1), (16, 512, 1, 1), (16, 1024, 1, 1), (8, 256, 1, 1), (8, 512, 1, 1),
            (8, 1024, 1, 1), (4, 256, 1, 1), (4, 512, 1, 1), (16, 256, 2, 1), (16, 512, 2, 1),
            (8, 256, 2, 1), (8, 512, 2, 1), (8, 512, 1, 2)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,nt", [(300, 64), (1000, 512), (257, 1024), (255, 4096)])
def test_pc_apply_every_variant(nx, nt, prec, monkeypatch):
    """The autotuner may pick any compiled variant: each one must match,
    in the standalone apply (row-major output) and inside a solve (Z stored
    blocked by the columns one inverse-transform workgroup writes)."""
    inst = localvol(nx, nt) if nx >= 255 else W.config1(nx=nx, nt=nt)
    v = W.random_vector(inst.n, 11)
    ref = O.pc_apply(*oracle_args(inst), inst.alpha, v)
    u = O.sequential_cn(*oracle_args(inst), inst.u0, inst.f)
    ran = 0
    for bcols, thr, split, fsplit in VARIANTS:
        monkeypatch.setenv("CN_PC_TILE", f"{bcols},{thr},{split},{fsplit}")
        try:
            s = solver(inst, pc_prec=prec)
        except B.CnError as e:
            assert e.status == B.CN_EINVAL and "not a compiled variant" in str(e)
            continue
        banner(f"pc_apply variant {prec} B={bcols} T={thr} S={split} F={fsplit} nx={nx} nt={nt}")
        q = s.query()
        assert (q["tile_cols"], q["threads"], q["inverse_split"], q["forward_split"]) == \
            (bcols, thr, split, fsplit)
        z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
        s.pc_apply(T(v), z)
        err = rel_inf(z.cpu().numpy(), ref)
        assert err <= pc_tol(inst.alpha, prec, nt), (bcols, thr, split, fsplit, err)
        b = torch.empty(inst.n, dtype=torch.float64, device="cuda")
        s.rhs(T(inst.u0), T(inst.f.reshape(-1)), b)
        x = torch.empty_like(b)
        r = s.solve(b, x, m=20, rtol=1e-10)
        assert r.status == B.CN_OK and r.relres_true <= 1e-10
        assert rel_inf(x.cpu().numpy(), u) <= 1e-8, (bcols, thr, split, fsplit)
        s.close()
        ran += 1
    assert ran >= 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,nt,tile", [(16383, 64, "16,256"), (16383, 64, "8,256"),
                                        (16383, 128, "4,256"), (65535, 128, "4,256")])
def test_interface_solve_variants(nx, nt, tile, prec, monkeypatch):
    """Wide instances select the interface-solve layouts with 4 and 16
    wavefronts per frequency line, separators held in registers or streamed
    (1023, 2047, 4095 and 16383 separators).  Every element against the
    oracle for N_x = 16383 (bound: pc_tol plus precision times the shifted
    systems' condition number, which reaches ~1e6 on this grid); the widest
    through the defining operator of eq. (3.1) (P_alpha z = v)."""
    monkeypatch.setenv("CN_PC_TILE", tile)
    inst = localvol(nx, nt)
    banner(f"interface solve {prec} nx={nx} tile={tile}")
    s = solver(inst, pc_prec=prec)
    v = W.random_vector(inst.n, 21)
    z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
    s.pc_apply(T(v), z)
    zh = z.cpu().numpy()
    if nx <= 16383:
        ref = O.pc_apply(*oracle_args(inst), inst.alpha, v)
        err = rel_inf(zh, ref)
    else:
        # residual in the defining operator; a backward-stable solve keeps it
        # below eps ||mu I - A~|| ||y||, i.e. eps kappa ||r|| when a random
        # right-hand side excites the lowest modes: same bound
        err = np.linalg.norm(O.pc_matvec(*oracle_args(inst), inst.alpha, zh) - v) / np.linalg.norm(v)
    tol = pc_tol_wide(inst, prec)
    print(f"  err={err:.3e} bound={tol:.3e} kappa={shifted_condition(inst):.3e} "
          f"tiles={s.query()}")
    assert err <= tol
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_interface_solve_variant_matches_oracle(prec, monkeypatch):
    """Each layout of the interface solve (1, 4, 8 or 16 wavefronts per line;
    2..8 separators per lane in registers, or streamed; the strided layout
    with block scans, rho' in registers or in scratch; the rounds layout of
    8 separators per lane in two rounds) forced on the same 255-separator
    system, every element against the oracle."""
    monkeypatch.setenv("CN_PC_TILE", "16,256")
    inst = localvol(4095, 64)
    v = W.random_vector(inst.n, 23)
    ref = O.pc_apply(*oracle_args(inst), inst.alpha, v)
    for cls in (36, 40, 129, 130, 132, 136, 257, 258, 260, 264, 513, 514, 516, 512,
                4097, 4098, 4100, 4104, 4112, 8194):
        monkeypatch.setenv("CN_K2_CLASS", str(cls))
        banner(f"interface variant {cls} {prec}")
        s = solver(inst, pc_prec=prec)
        assert s.query()["tiles"] == 256
        z = torch.empty(inst.n, dtype=torch.float64, device="cuda")
        s.pc_apply(T(v), z)
        err = rel_inf(z.cpu().numpy(), ref)
        assert err <= pc_tol_wide(inst, prec), (cls, err)
        s.close()
