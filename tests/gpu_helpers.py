"""Shared helpers of the GPU tests: move a workload to the device and build
a solver handle through the C ABI."""
import numpy as np
import torch

from paper_2401_16113_amd import binding as B


def dev():
    return torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=dev())


def solver(inst, pc_prec=None, m_max=None, alpha=None, d_half=None, flags=0):
    return B.Solver(T(inst.a_lo), T(inst.a_di), T(inst.a_up), inst.nt, inst.T,
                    inst.alpha if alpha is None else alpha,
                    m_max=inst.m if m_max is None else m_max,
                    pc_prec=inst.pc_prec if pc_prec is None else pc_prec,
                    d_half=None if d_half is None else T(d_half), flags=flags)


def rel_inf(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def banner(msg):
    print(f"\n[gpu-case] {msg}", flush=True)


def batch(insts, pc_prec="fp32", m_max=20):
    probs = [dict(a_lo=T(i.a_lo), a_di=T(i.a_di), a_up=T(i.a_up), nt=i.nt, T=i.T,
                  alpha=i.alpha, m_max=m_max) for i in insts]
    return B.Batch(probs, pc_prec=pc_prec)


def packed(insts, attr):
    if attr == "u0":
        return T(np.concatenate([i.u0 for i in insts]))
    return T(np.concatenate([i.f.reshape(-1) for i in insts]))
