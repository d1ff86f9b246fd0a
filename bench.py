#!/usr/bin/env python
"""Throughput of the alpha-circulant preconditioned all-at-once CN solve.

Metric: space-time unknowns per second to relative residual 1e-8 on one
MI355X.  Workload: the local-volatility Black-Scholes put with
N_x = 4095, N_t = 1024 (4,193,280 unknowns), T = 2, r = 0.03,
sigma(x) = 0.2 + a1 tanh x + a2 sin 3x (seeded amplitudes), alpha = 0.01,
flexible GMRES(30), zero initial guess.  One step = one whole solve (every
kernel of the hot path) with b and x resident in HBM.

Two forms are timed on the same workload:
  plain_fp64 -- float64 preconditioner (the method as stated),
  fp32_pc    -- float32 preconditioner inside float64 flexible GMRES.
`value` is the fp32_pc form (both reach relres <= 1e-8; accuracy against the
exact CN solution is reported by the cpu_baseline leg).

Also reported: the roofline position of the dominant kernel (HIP-event
timing of each kernel of one inner iteration, algorithmic bytes per launch
against the 8 TB/s HBM peak) and the CPU oracle timed on the host.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
RTOL = 1e-8
M = 30
# sources whose change invalidates stored hardware-counter traffic figures
KERNEL_SOURCES = ["paper_2401_16113_amd/csrc/cn_device.hpp",
                  "paper_2401_16113_amd/csrc/cn_pc_kernels.hpp",
                  "paper_2401_16113_amd/csrc/cn_pc.hip",
                  "paper_2401_16113_amd/csrc/cn_krylov.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_localvol_4095x1024_fp32pc.txt")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy of known size), or None when the
    summary is missing or the kernel sources changed since it was taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_hash") != kernel_source_hash():
            return None
        v = kv.get(f"traffic_bytes[{kernel}]")
        return float(v) if v is not None else None
    except OSError:
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_variant(B, W, inst, prec, steps, warmup, dev, torch):
    import numpy as np
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    s = B.Solver(t(inst.a_lo), t(inst.a_di), t(inst.a_up), inst.nt, inst.T, inst.alpha,
                 m_max=M, pc_prec=prec)
    b = torch.empty(inst.n, dtype=torch.float64, device=dev)
    s.rhs(t(inst.u0), t(inst.f.reshape(-1)), b)
    x = torch.empty_like(b)
    for _ in range(warmup):
        s.solve(b, x, m=M, rtol=RTOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [s.solve(b, x, m=M, rtol=RTOL) for _ in range(steps)]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    last = res[-1]
    if last.status != B.CN_OK or last.relres_true > RTOL:
        raise RuntimeError(f"{prec}: solve did not reach relres {RTOL}: {last}")
    ms = el / steps * 1e3
    prof = s.profile_step(j=min(1, last.iters - 1), reps=20)
    out = {
        "pc_variant": s.query(),
        "ms_per_solve": ms,
        "unknowns_per_s": inst.n / (ms * 1e-3),
        "iters": last.iters,
        "relres": last.relres_true,
        "device_ms_per_solve": statistics.median(r.seconds for r in res) * 1e3,
        "kernels_step1": {k: {"us": v["ms"] * 1e3, "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
                          for k, v in prof.items()},
    }
    x_host = x.cpu().numpy()
    s.close()
    return out, prof, x_host


def cpu_baseline(inst, x_gpu):
    import numpy as np
    from oracle import cn_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max((p.get("num_threads", 1) for p in threadpool_info()), default=1)
    except Exception:
        cores = len(os.sched_getaffinity(0))
    args = (inst.a_lo, inst.a_di, inst.a_up, inst.T, inst.nt)
    b = O.aao_rhs(*args, inst.u0, inst.f)
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        r = O.cn_gmres_solve(*args, inst.alpha, b, m=M, rtol=RTOL)
        times.append(time.perf_counter() - t0)
    sec = statistics.median(times)
    u = O.sequential_cn(*args, inst.u0, inst.f)
    scale = np.max(np.abs(u))
    errs = {k: float(np.max(np.abs(v - u)) / scale) for k, v in x_gpu.items()}
    return {
        "value": inst.n / sec, "unit": "unknowns/s", "cores": int(cores), "kind": "oracle",
        "sample": (f"whole solve of the same {inst.nx}x{inst.nt} workload by the FP64 oracle "
                   f"(right-preconditioned GMRES({M}), direct O(N_t^2) DFT sums), median of 3 "
                   f"runs, {sec:.2f} s each, {r.iters} iterations"),
        "gpu_err_vs_exact_cn": errs,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=0.01)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run 256 MiB device copies (hardware-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_16113_amd import binding as B
    from paper_2401_16113_amd import workloads as W

    dev = torch.device("cuda:0")
    inst = W.config2(alpha=args.alpha)
    variants, profs, xs = {}, {}, {}
    for prec in ("fp64", "fp32"):
        log(f"[bench] {prec} preconditioner: {args.warmup} warm-up + {args.steps} timed solves")
        v, p, x = run_variant(B, W, inst, prec, args.steps, args.warmup, dev, torch)
        variants["plain_fp64" if prec == "fp64" else "fp32_pc"] = v
        profs[prec], xs[prec] = p, x
        log(f"[bench] {prec}: {v['ms_per_solve']:.3f} ms/solve, {v['iters']} iters, "
            f"relres {v['relres']:.2e}")
    prim = variants["fp32_pc"]
    prof = profs["fp32"]
    dom = max(prof, key=lambda k: prof[k]["ms"])
    ach = prof[dom]["bytes"] / (prof[dom]["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(dom),
            "avg_launch_us": round(prof[dom]["ms"] * 1e3, 2),
            "algorithmic_bytes": prof[dom]["bytes"]}
    out = {
        "metric": "space-time unknowns/s to rel.res 1e-8",
        "value": prim["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (f32 preconditioner)",
        "data": "synthetic",
        "config": {"workload": f"local-vol Black-Scholes put, N_x={inst.nx}, N_t={inst.nt}, "
                               f"alpha={inst.alpha}, flexible GMRES({M}), rtol {RTOL}",
                   "unknowns": inst.n, "form": "fp32_pc"},
        "variants": variants,
        "roofline": roof,
    }
    if args.calibrate_copy:
        log("[bench] calibration: 5 device copies of 256 MiB")
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        log("[bench] cpu_baseline: oracle solve on the host")
        out["cpu_baseline"] = cpu_baseline(inst, {"plain_fp64": xs["fp64"], "fp32_pc": xs["fp32"]})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
