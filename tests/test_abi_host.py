"""C ABI checks that need no GPU: the library loads, exports every entry
point include/cn_aao.h declares, and rejects invalid arguments before any
device work."""
import ctypes
import os
import re

import pytest

from paper_2401_16113_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(cn_[a-z0-9_]+)\s*\(", txt))
    return names


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert {"cn_aao_create", "cn_matvec", "cn_pc_apply", "cn_gmres_solve"} <= names
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for s in (B.CN_OK, B.CN_NOT_CONVERGED, B.CN_EINVAL, B.CN_ENOMEM, B.CN_EHIP, B.CN_ESINGULAR):
        assert lib.cn_status_string(s)
    assert b"singular" in lib.cn_status_string(B.CN_ESINGULAR)


def _create(lib, **kw):
    base = dict(nx=16, nt=8, m_max=10, flags=0, T=1.0, alpha=0.01, a_lo=1, a_di=1, a_up=1,
                d_half=None, pc_prec=0, stream=None)
    base.update(kw)
    p = B.CnProblem(**{k: v for k, v in base.items()})
    h = ctypes.c_void_p(1234)
    st = lib.cn_aao_create(ctypes.byref(p), ctypes.byref(h))
    return st, h, lib.cn_last_error().decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(nx=0), "nx"),
    (dict(nt=3), "power of two"),
    (dict(nt=16384), "power of two"),
    (dict(nt=0), "power of two"),
    (dict(m_max=0), "m_max"),
    (dict(m_max=65), "m_max"),
    (dict(T=0.0), "T must"),
    (dict(T=float("nan")), "T must"),
    (dict(alpha=0.0), "alpha"),
    (dict(alpha=1.0), "alpha"),
    (dict(alpha=1.5), "alpha"),
    (dict(alpha=float("nan")), "alpha"),
    (dict(pc_prec=7), "pc_prec"),
    (dict(a_lo=None), "device pointers"),
])
def test_create_rejects_invalid_problem(lib, kw, msg):
    st, h, err = _create(lib, **kw)
    assert st == B.CN_EINVAL
    assert h.value is None
    assert msg in err


def test_null_arguments(lib):
    h = ctypes.c_void_p()
    assert lib.cn_aao_create(None, ctypes.byref(h)) == B.CN_EINVAL
    assert lib.cn_aao_destroy(None) == B.CN_EINVAL
    assert lib.cn_matvec(None, None, None) == B.CN_EINVAL
    assert lib.cn_pc_apply(None, None, None) == B.CN_EINVAL
    assert lib.cn_rhs(None, None, None, None) == B.CN_EINVAL
    assert lib.cn_gmres_solve(None, None, None, None, None) == B.CN_EINVAL
    assert lib.cn_aao_query(None, None, None, None, None, None) == B.CN_EINVAL


def test_mlp_create_rejects_bad_sizes(lib):
    h = ctypes.c_void_p(1234)
    for args in ((0, 8, 4, 4), (4, 0, 4, 4), (4, 8, 0, 4), (4, 8, 4, 0)):
        assert lib.cn_mlp_create(*args, None, ctypes.byref(h)) == B.CN_EINVAL
        assert h.value is None
    assert lib.cn_mlp_create(4, 8, 4, 4, None, None) == B.CN_EINVAL
    assert lib.cn_mlp_destroy(None) == B.CN_EINVAL
    assert lib.cn_mlp_adam_step(None, 1e-3, 0.9, 0.999, 1e-8) == B.CN_EINVAL


def test_ws_grid_calls_reject_bad_arguments(lib):
    p = ctypes.c_void_p(4096)
    # NULL pointers
    assert lib.cn_ws_restrict(None, 1, 255, 64, p, p, None) == B.CN_EINVAL
    assert lib.cn_ws_interpolate(p, 1, 255, 64, p, p, None, p, p, None) == B.CN_EINVAL
    # incompatible grids are refused before any device work
    for nx, nt in ((127, 64), (256, 64), (255, 60), (255, 0)):
        assert lib.cn_ws_restrict(p, 1, nx, nt, p, p, None) == B.CN_EINVAL
        assert b"multiple" in lib.cn_ws_last_error()
    assert lib.cn_ws_restrict(p, 0, 255, 64, p, p, None) == B.CN_EINVAL


def test_gmres_info_layout():
    # six 32-bit fields then four doubles, as include/cn_aao.h declares
    assert ctypes.sizeof(B.CnGmresInfo) == 56
    assert B.CnGmresInfo.relres_true.offset == 24
    assert B.CnGmresInfo.err_est.offset == 48
    # four 32-bit fields then rtol and err_tol
    assert ctypes.sizeof(B.CnGmresOpts) == 32
    assert B.CnGmresOpts.rtol.offset == 16 and B.CnGmresOpts.err_tol.offset == 24


def test_cn2d_create_rejects_bad_arguments(lib):
    """Validation of cn2d_create happens before any device call."""
    vp = ctypes.c_void_p
    h = vp()
    good = dict(nx=8, ny=8, nt=8, m_max=0, T=0.5, alpha=0.01, stencil=4096, stream=None)
    assert lib.cn2d_create(None, ctypes.byref(h)) == B.CN_EINVAL
    for bad in (dict(nx=0), dict(nx=128), dict(ny=0), dict(nx=100, ny=100), dict(nt=12),
                dict(nt=2048), dict(T=0.0), dict(alpha=1.0), dict(alpha=0.0), dict(m_max=65),
                dict(stencil=None)):
        args = dict(good)
        args.update(bad)
        prob = B.Cn2dProblem(**args)
        assert lib.cn2d_create(ctypes.byref(prob), ctypes.byref(h)) == B.CN_EINVAL
        assert h.value is None
    assert lib.cn2d_destroy(None) == B.CN_EINVAL
    assert lib.cn2d_pc_apply(None, None, None) == B.CN_EINVAL
