"""ctypes binding of libcn_aao (include/cn_aao.h).

Argument marshalling only: tensors are passed as device pointers, every step
runs in the library's HIP kernels.  Loading fails loudly when the library has
not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcn_aao.so")

CN_OK = 0
CN_NOT_CONVERGED = 1
CN_EINVAL = -1
CN_ENOMEM = -2
CN_EHIP = -3
CN_ESINGULAR = -4

CN_PC_FP64 = 0
CN_SOLVE_NO_GRAPHS = 1
CN_SOLVE_ITERATION_GRAPHS = 2
CN_PC_FP32 = 1
CN_FLAG_ALLOW_ALPHA_ONE = 1


class CnProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("nt", ctypes.c_int32), ("m_max", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("T", ctypes.c_double), ("alpha", ctypes.c_double),
        ("a_lo", ctypes.c_void_p), ("a_di", ctypes.c_void_p), ("a_up", ctypes.c_void_p),
        ("d_half", ctypes.c_void_p), ("pc_prec", ctypes.c_int), ("stream", ctypes.c_void_p),
    ]


class Cn2dProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nt", ctypes.c_int32),
        ("m_max", ctypes.c_int32), ("T", ctypes.c_double), ("alpha", ctypes.c_double),
        ("stencil", ctypes.c_void_p), ("stream", ctypes.c_void_p),
    ]


class CnGmresOpts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("err_tol", ctypes.c_double)]


class CnGmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("matvecs", ctypes.c_int32), ("pc_applies", ctypes.c_int32),
                ("x0_rejected", ctypes.c_int32), ("err_passes", ctypes.c_int32),
                ("relres_true", ctypes.c_double), ("relres_est", ctypes.c_double),
                ("seconds", ctypes.c_double), ("err_est", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load():
    """Load libcn_aao.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sig = {
        "cn_aao_create": (ctypes.c_int, [ctypes.POINTER(CnProblem), ctypes.POINTER(vp)]),
        "cn_aao_destroy": (ctypes.c_int, [vp]),
        "cn_aao_query": (ctypes.c_int, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32)]),
        "cn_aao_cycle": (ctypes.c_int, [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                        ctypes.POINTER(dbl)]),
        "cn_aao_basis": (ctypes.c_int, [vp, i32, vp]),
        "cn_pc_apply_noalloc": (ctypes.c_int, [ctypes.POINTER(CnProblem), vp, vp]),
        "cn_rhs": (ctypes.c_int, [vp, vp, vp, vp]),
        "cn_matvec": (ctypes.c_int, [vp, vp, vp]),
        "cn_pc_apply": (ctypes.c_int, [vp, vp, vp]),
        "cn_gmres_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(CnGmresOpts),
                                          ctypes.POINTER(CnGmresInfo)]),
        "cn_profile_step": (ctypes.c_int, [vp, i32, i32, ctypes.POINTER(dbl),
                                           ctypes.POINTER(dbl)]),
        "cn_batch_create": (ctypes.c_int, [ctypes.POINTER(CnProblem), i32, ctypes.POINTER(vp)]),
        "cn_batch_destroy": (ctypes.c_int, [vp]),
        "cn_batch_offsets": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64)]),
        "cn_batch_rhs": (ctypes.c_int, [vp, vp, vp, vp]),
        "cn_batch_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(CnGmresOpts),
                                          ctypes.POINTER(CnGmresInfo),
                                          ctypes.POINTER(CnGmresInfo)]),
        "cn_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "cn_last_error": (ctypes.c_char_p, []),
        # learned initial guess (cn_warmstart.h)
        "cn_mlp_create": (ctypes.c_int, [i32, i32, i32, i32, vp, ctypes.POINTER(vp)]),
        "cn_mlp_destroy": (ctypes.c_int, [vp]),
        "cn_mlp_num_params": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int64)]),
        "cn_mlp_set_params": (ctypes.c_int, [vp, vp]),
        "cn_mlp_get_params": (ctypes.c_int, [vp, vp]),
        "cn_mlp_set_normalization": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "cn_mlp_forward": (ctypes.c_int, [vp, vp, i32, vp]),
        "cn_mlp_loss_grad": (ctypes.c_int, [vp, vp, vp, i32, vp, vp]),
        "cn_mlp_adam_step": (ctypes.c_int, [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float]),
        "cn_ws_restrict": (ctypes.c_int, [vp, i32, i32, i32, vp, vp, vp]),
        "cn_ws_interpolate": (ctypes.c_int, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "cn_ws_predict": (ctypes.c_int, [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "cn_ws_predict_batch": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "cn_ws_last_error": (ctypes.c_char_p, []),
        "cn2d_create": (ctypes.c_int, [ctypes.POINTER(Cn2dProblem), ctypes.POINTER(vp)]),
        "cn2d_destroy": (ctypes.c_int, [vp]),
        "cn2d_matvec": (ctypes.c_int, [vp, vp, vp]),
        "cn2d_rhs": (ctypes.c_int, [vp, vp, vp, vp]),
        "cn2d_pc_apply": (ctypes.c_int, [vp, vp, vp]),
        "cn2d_gmres_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(CnGmresOpts),
                                            ctypes.POINTER(CnGmresInfo)]),
        "cn2d_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class CnError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        last = (lib.cn_ws_last_error if where.startswith(("cn_mlp", "cn_ws"))
                else lib.cn2d_last_error if where.startswith("cn2d") else lib.cn_last_error)
        msg = last().decode()
        super().__init__(f"{where}: {lib.cn_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.device.type != "cuda":
        raise ValueError("tensor must live on the GPU")
    dtype = torch.float64 if dtype is None else dtype
    if t.dtype != dtype:
        raise TypeError(f"tensor must be {dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(status: int, where: str, ok=(CN_OK,)):
    if status not in ok:
        raise CnError(status, where)
    return status


@dataclass
class SolveResult:
    status: int
    iters: int
    restarts: int
    matvecs: int
    pc_applies: int
    relres_true: float
    relres_est: float
    seconds: float
    x0_rejected: int = 0
    err_est: float = -1.0  # error estimate of error-controlled stopping (-1: off)
    err_passes: int = 0    # continuation solves error-controlled stopping took


class Solver:
    """One all-at-once CN problem on one GPU (wraps a cn_aao handle).

    a_lo, a_di, a_up: float64 CUDA tensors of length nx holding the rows of A
    (not tau A).  d_half: optional float64 CUDA tensor of length nt."""

    def __init__(self, a_lo, a_di, a_up, nt: int, T: float, alpha: float, m_max: int = 30,
                 pc_prec: str = "fp64", d_half=None, flags: int = 0, stream=None):
        lib = load()
        self._lib = lib
        nx = int(a_lo.numel())
        if stream is None:
            stream = torch.cuda.current_stream(a_lo.device)
        self.stream = stream
        prob = CnProblem(nx=nx, nt=int(nt), m_max=int(m_max), flags=int(flags), T=float(T),
                         alpha=float(alpha), a_lo=_ptr(a_lo), a_di=_ptr(a_di), a_up=_ptr(a_up),
                         d_half=_ptr(d_half), pc_prec=CN_PC_FP32 if pc_prec == "fp32" else CN_PC_FP64,
                         stream=ctypes.c_void_p(stream.cuda_stream))
        h = ctypes.c_void_p()
        _check(lib.cn_aao_create(ctypes.byref(prob), ctypes.byref(h)), "cn_aao_create")
        self._h = h
        self.nx, self.nt = nx, int(nt)
        self.n = nx * int(nt)
        self.m_max = int(m_max)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cn_aao_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self):
        b, p, t, sp, fs = (ctypes.c_int32() for _ in range(5))
        _check(self._lib.cn_aao_query(self._h, ctypes.byref(b), ctypes.byref(p), ctypes.byref(t),
                                      ctypes.byref(sp), ctypes.byref(fs)), "cn_aao_query")
        return {"tile_cols": b.value, "tiles": p.value, "threads": t.value,
                "inverse_split": sp.value, "forward_split": fs.value}

    def cycle(self, k: int):
        """The Arnoldi record of the last cycle, which ran k inner
        iterations: the Gram matrix of the normalised basis ((k+1) x (k+1)),
        the triangular factor's columns (k x (k+1), column j in row j) and
        the basis scales 1/||v_q|| (entry 0 excepted, see cn_aao.h)."""
        import numpy as np
        kk = int(k)
        g = (ctypes.c_double * ((kk + 1) * (kk + 1)))()
        r = (ctypes.c_double * max(1, kk * (kk + 1)))()
        sc = (ctypes.c_double * (kk + 1))()
        _check(self._lib.cn_aao_cycle(self._h, kk, g, r, sc), "cn_aao_cycle")
        gram = np.array(g[:]).reshape(kk + 1, kk + 1)
        rfac = np.array(r[:kk * (kk + 1)]).reshape(kk, kk + 1)
        return gram, rfac, np.array(sc[:])

    def basis(self, q: int, out):
        """Copy the stored (unnormalised) basis vector q into out."""
        _check(self._lib.cn_aao_basis(self._h, int(q), _ptr(out)), "cn_aao_basis")
        return out

    def rhs(self, u0, f, out):
        _check(self._lib.cn_rhs(self._h, _ptr(u0), _ptr(f), _ptr(out)), "cn_rhs")
        return out

    def matvec(self, x, out):
        _check(self._lib.cn_matvec(self._h, _ptr(x), _ptr(out)), "cn_matvec")
        return out

    def pc_apply(self, v, out):
        _check(self._lib.cn_pc_apply(self._h, _ptr(v), _ptr(out)), "cn_pc_apply")
        return out

    KERNELS = ("pc_forward", "pc_reduced", "pc_inverse", "matvec_dots", "cgs_update")

    def profile_step(self, j: int, reps: int = 20):
        """Average launch time (ms) and algorithmic bytes of the kernels of
        inner iteration j (after a solve with more than j iterations): the
        preconditioner apply (pc_forward, pc_reduced, pc_inverse) and the two
        streaming Krylov kernels (matvec with the basis dots, Gram-Schmidt
        update)."""
        n = len(self.KERNELS)
        ms = (ctypes.c_double * n)()
        by = (ctypes.c_double * n)()
        _check(self._lib.cn_profile_step(self._h, int(j), int(reps), ms, by), "cn_profile_step")
        return {k: {"ms": ms[i], "bytes": by[i]} for i, k in enumerate(self.KERNELS) if ms[i] > 0}

    def solve(self, b, x, m: int = 20, rtol: float = 1e-8, max_iters: int = 1000,
              use_x0: bool = False, allow_not_converged: bool = True,
              err_tol: float = 0.0) -> SolveResult:
        """err_tol > 0: error-controlled stopping (the estimated relative
        max-norm error must also fall below err_tol)."""
        opts = CnGmresOpts(m=int(m), max_iters=int(max_iters), use_x0=int(use_x0),
                           flags=0, rtol=float(rtol), err_tol=float(err_tol))
        info = CnGmresInfo()
        ok = (CN_OK, CN_NOT_CONVERGED) if allow_not_converged else (CN_OK,)
        st = _check(self._lib.cn_gmres_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(opts),
                                             ctypes.byref(info)), "cn_gmres_solve", ok)
        return SolveResult(st, info.iters, info.restarts, info.matvecs, info.pc_applies,
                           info.relres_true, info.relres_est, info.seconds, info.x0_rejected,
                           info.err_est, info.err_passes)


class Batch:
    """Many independent problems of uneven size solved together (wraps a
    cn_batch handle).  `problems`: list of dicts with keys a_lo, a_di, a_up
    (float64 CUDA tensors of length nx), nt, T, alpha and optionally m_max,
    d_half.  Packed vectors hold the instances back to back (see offsets)."""

    def __init__(self, problems, pc_prec: str = "fp32", stream=None):
        lib = load()
        self._lib = lib
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._keep = []
        arr = (CnProblem * len(problems))()
        for i, pr in enumerate(problems):
            self._keep.append(pr)
            arr[i] = CnProblem(nx=int(pr["a_lo"].numel()), nt=int(pr["nt"]),
                               m_max=int(pr.get("m_max", 20)), flags=int(pr.get("flags", 0)),
                               T=float(pr["T"]), alpha=float(pr["alpha"]),
                               a_lo=_ptr(pr["a_lo"]), a_di=_ptr(pr["a_di"]),
                               a_up=_ptr(pr["a_up"]), d_half=_ptr(pr.get("d_half")),
                               pc_prec=CN_PC_FP32 if pc_prec == "fp32" else CN_PC_FP64,
                               stream=ctypes.c_void_p(stream.cuda_stream))
        h = ctypes.c_void_p()
        _check(lib.cn_batch_create(arr, len(problems), ctypes.byref(h)), "cn_batch_create")
        self._h = h
        self.count = len(problems)
        off = (ctypes.c_int64 * (self.count + 1))()
        soff = (ctypes.c_int64 * (self.count + 1))()
        _check(lib.cn_batch_offsets(h, off, soff), "cn_batch_offsets")
        self.offsets = list(off)
        self.space_offsets = list(soff)
        self.n = self.offsets[-1]

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cn_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rhs(self, u0, f, out):
        _check(self._lib.cn_batch_rhs(self._h, _ptr(u0), _ptr(f), _ptr(out)), "cn_batch_rhs")
        return out

    def solve(self, b, x, m: int = 20, rtol: float = 1e-8, max_iters: int = 1000,
              use_x0: int = 0, graphs: bool = True, err_tol: float = 0.0,
              cycle_graphs: bool = True):
        """use_x0: 0 zero start, 1 x holds the guess, 2 guess with fallback
        to zero; graphs: launch each inner iteration as a captured graph;
        cycle_graphs: the first iterations of a cycle as one graph (as many
        as the last solve's first cycle took); err_tol > 0: error-controlled
        stopping per instance."""
        flags = (0 if graphs else CN_SOLVE_NO_GRAPHS) | (0 if cycle_graphs else CN_SOLVE_ITERATION_GRAPHS)
        opts = CnGmresOpts(m=int(m), max_iters=int(max_iters), use_x0=int(use_x0),
                           flags=flags, rtol=float(rtol), err_tol=float(err_tol))
        infos = (CnGmresInfo * self.count)()
        total = CnGmresInfo()
        st = _check(self._lib.cn_batch_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(opts), infos,
                                             ctypes.byref(total)), "cn_batch_solve",
                    (CN_OK, CN_NOT_CONVERGED))
        per = [SolveResult(CN_OK if i.relres_true <= rtol and (err_tol <= 0 or i.err_est <= err_tol)
                           else CN_NOT_CONVERGED, i.iters,
                           i.restarts, i.matvecs, i.pc_applies, i.relres_true, i.relres_est,
                           i.seconds, i.x0_rejected, i.err_est, i.err_passes) for i in infos]
        tot = SolveResult(st, total.iters, total.restarts, total.matvecs, total.pc_applies,
                          total.relres_true, total.relres_est, total.seconds, total.x0_rejected,
                          total.err_est, total.err_passes)
        return tot, per


# ---------------------------------------------------------------------------
# learned initial guess
# ---------------------------------------------------------------------------
COARSE_X, COARSE_T = 128, 64


def _f32(t):
    return _ptr(t, torch.float32)


class Mlp:
    """The warm-start network (wraps a cn_mlp handle): n_in -> w -> w -> w ->
    n_out with ReLU, bf16 matrix-core products with float32 accumulation,
    float32 masters and Adam.  Tensors: float32, contiguous, on the GPU."""

    def __init__(self, n_in: int, width: int, n_out: int, max_batch: int, stream=None):
        self._lib = load()
        self.n_in, self.width, self.n_out, self.max_batch = n_in, width, n_out, max_batch
        h = ctypes.c_void_p()
        s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        _check(self._lib.cn_mlp_create(n_in, width, n_out, max_batch, s, ctypes.byref(h)),
               "cn_mlp_create")
        self._h = h
        n = ctypes.c_int64()
        _check(self._lib.cn_mlp_num_params(self._h, ctypes.byref(n)), "cn_mlp_num_params")
        self.num_params = n.value

    def close(self):
        if self._h:
            _check(self._lib.cn_mlp_destroy(self._h), "cn_mlp_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        _check(self._lib.cn_mlp_set_params(self._h, _f32(p)), "cn_mlp_set_params")

    def get_params(self, out):
        _check(self._lib.cn_mlp_get_params(self._h, _f32(out)), "cn_mlp_get_params")
        return out

    def set_normalization(self, in_mean, in_scale, out_mean, out_scale):
        _check(self._lib.cn_mlp_set_normalization(self._h, _f32(in_mean), _f32(in_scale),
                                                  _f32(out_mean), _f32(out_scale)),
               "cn_mlp_set_normalization")

    def forward(self, X, Y):
        _check(self._lib.cn_mlp_forward(self._h, _f32(X), int(X.shape[0]), _f32(Y)),
               "cn_mlp_forward")
        return Y

    def loss_grad(self, X, Yt, grads=None, loss=None):
        _check(self._lib.cn_mlp_loss_grad(self._h, _f32(X), _f32(Yt), int(X.shape[0]),
                                          _f32(grads), _f32(loss)), "cn_mlp_loss_grad")

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _check(self._lib.cn_mlp_adam_step(self._h, lr, beta1, beta2, eps), "cn_mlp_adam_step")

    def predict(self, features, nx: int, nt: int, u0, gl, gr, scale, coarse, x0):
        """Forward pass + interpolation to the fine grid (cn_ws_predict)."""
        _check(self._lib.cn_ws_predict(self._h, _f32(features), int(features.shape[0]), nx, nt,
                                       _ptr(u0), _ptr(gl), _ptr(gr), _ptr(scale), _f32(coarse),
                                       _ptr(x0)), "cn_ws_predict")
        return x0

    def predict_batch(self, features, batch, u0, gl, gr, scale, coarse, x0):
        """Forward pass + interpolation of every instance of an uneven batch
        to its own grid (cn_ws_predict_batch)."""
        _check(self._lib.cn_ws_predict_batch(self._h, _f32(features), batch._h, _ptr(u0),
                                             _ptr(gl), _ptr(gr), _ptr(scale), _f32(coarse),
                                             _ptr(x0)), "cn_ws_predict_batch")
        return x0


def pc_apply_noalloc(a_lo, a_di, a_up, nt: int, T: float, alpha: float, v, out,
                     pc_prec: str = "fp64", d_half=None, stream=None):
    """z = P_alpha^{-1} v without a handle and without allocation
    (cn_pc_apply_noalloc): the work arrays live in the library's fixed
    per-GPU array."""
    lib = load()
    if stream is None:
        stream = torch.cuda.current_stream(a_lo.device)
    prob = CnProblem(nx=int(a_lo.numel()), nt=int(nt), m_max=1, flags=0, T=float(T),
                     alpha=float(alpha), a_lo=_ptr(a_lo), a_di=_ptr(a_di), a_up=_ptr(a_up),
                     d_half=_ptr(d_half), pc_prec=CN_PC_FP32 if pc_prec == "fp32" else CN_PC_FP64,
                     stream=ctypes.c_void_p(stream.cuda_stream))
    _check(lib.cn_pc_apply_noalloc(ctypes.byref(prob), _ptr(v), _ptr(out)), "cn_pc_apply_noalloc")
    return out


def ws_restrict(x, count: int, nx: int, nt: int, inv_scale, coarse, stream=None):
    lib = load()
    s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(lib.cn_ws_restrict(_ptr(x), count, nx, nt, _ptr(inv_scale), _f32(coarse), s),
           "cn_ws_restrict")
    return coarse


def ws_interpolate(coarse, count: int, nx: int, nt: int, u0, gl, gr, scale, x0, stream=None):
    lib = load()
    s = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
    _check(lib.cn_ws_interpolate(_f32(coarse), count, nx, nt, _ptr(u0), _ptr(gl), _ptr(gr),
                                 _ptr(scale), _ptr(x0), s), "cn_ws_interpolate")
    return x0


class Solver2D:
    """All-at-once CN system of a 2D nine-point stencil operator and its
    alpha-circulant preconditioner (wraps a cn2d handle, cn_aao2d.h).
    stencil: float64 CUDA tensor of 9 * nx * ny coefficients (entry q of grid
    point i = iy nx + ix multiplies the unknown at (iy + q//3 - 1,
    ix + q%3 - 1))."""

    def __init__(self, stencil, nx: int, ny: int, nt: int, T: float, alpha: float,
                 m_max: int = 0, stream=None):
        lib = load()
        self._lib = lib
        if stream is None:
            stream = torch.cuda.current_stream(stencil.device)
        self._keep = stencil
        prob = Cn2dProblem(nx=int(nx), ny=int(ny), nt=int(nt), m_max=int(m_max), T=float(T),
                           alpha=float(alpha), stencil=_ptr(stencil),
                           stream=ctypes.c_void_p(stream.cuda_stream))
        h = ctypes.c_void_p()
        _check(lib.cn2d_create(ctypes.byref(prob), ctypes.byref(h)), "cn2d_create")
        self._h = h
        self.nx, self.ny, self.nt = int(nx), int(ny), int(nt)
        self.n = self.nx * self.ny * self.nt

    def matvec(self, x, y):
        _check(self._lib.cn2d_matvec(self._h, _ptr(x), _ptr(y)), "cn2d_matvec")
        return y

    def rhs(self, u0, f, b):
        _check(self._lib.cn2d_rhs(self._h, _ptr(u0), _ptr(f), _ptr(b)), "cn2d_rhs")
        return b

    def pc_apply(self, v, z):
        _check(self._lib.cn2d_pc_apply(self._h, _ptr(v), _ptr(z)), "cn2d_pc_apply")
        return z

    def solve(self, b, x, m: int = 20, rtol: float = 1e-8, max_iters: int = 1000,
              use_x0: bool = False) -> SolveResult:
        """Flexible GMRES(m) with P_alpha (cn2d_gmres_solve)."""
        opts = CnGmresOpts(m=int(m), max_iters=int(max_iters), use_x0=int(use_x0), flags=0,
                           rtol=float(rtol), err_tol=0.0)
        info = CnGmresInfo()
        st = _check(self._lib.cn2d_gmres_solve(self._h, _ptr(b), _ptr(x), ctypes.byref(opts),
                                               ctypes.byref(info)), "cn2d_gmres_solve",
                    (CN_OK, CN_NOT_CONVERGED))
        return SolveResult(st, info.iters, info.restarts, info.matvecs, info.pc_applies,
                           info.relres_true, info.relres_est, info.seconds)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cn2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
