#!/usr/bin/env python
"""Throughput of the alpha-circulant preconditioned all-at-once CN solve.

Metric: space-time unknowns per second to relative residual 1e-8 on one
MI355X, plain method against batched + float32 preconditioner + learned
initial guess.  Headline workload: the local-volatility Black-Scholes put
with N_x = 4095, N_t = 1024 (4,193,280 unknowns), T = 2, r = 0.03,
sigma(x) = 0.2 + a1 tanh x + a2 sin 3x (seeded amplitudes), alpha = 0.01,
flexible GMRES(30), zero initial guess.  One step = one whole solve (every
kernel of the hot path) with b and x resident in HBM.  `value` is the plain
method (float64 preconditioner); the float32-preconditioner form and the
alpha sweep (0.001, 0.01, 0.05, both precisions) are timed the same way.

`roofline` is the preconditioner apply (K1 + K2 + K3 of one inner
iteration, HIP-event timing on the solver's stream) at the algorithmic
48 B (float64) per unknown against the 8 TB/s HBM peak; the longest single
launch of that iteration is reported beside it.  The production
forms on their own workloads ("forms"):
  constant_vol -- the 127 x 64 constant-volatility put, float64, GMRES(20)
                  to 1e-12 (latency-bound);
  batch_uneven -- 512 uneven constant-volatility puts (N_x in 255..2047,
                  N_t in 64..512) in one batched solve, float32 preconditioner;
  warm_start   -- held-out local-volatility puts, N_x = 2047, N_t = 512:
                  plain (float64 preconditioner, one instance at a time, zero
                  start) against batched + float32 preconditioner, from zero
                  and from the learned initial guess (network trained here on
                  20000 plain solves; inference and interpolation inside the
                  timed region);
  drift_diffusion_2d -- a 2D variable-coefficient operator with a mixed
                  derivative, 127 x 63 grid, 256 steps, float64, GMRES(20);
  production   -- the 65535 x 4096 local-volatility put (2.7e8 unknowns),
                  float32 preconditioner, GMRES(20), with per-kernel rates.
The cpu_baseline leg times the CPU oracle on the host and reports every
form's error against the exact CN solution (the oracle's time stepping).
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
# error-controlled stopping of the batched and warm-start forms: estimated
# relative max-norm error at most half the 1e-7 accuracy bar
ERR_TOL = 5e-8
M = 30
# sources whose change invalidates stored hardware-counter traffic figures
KERNEL_SOURCES = ["paper_2401_16113_amd/csrc/cn_device.hpp",
                  "paper_2401_16113_amd/csrc/cn_internal.hpp",
                  "paper_2401_16113_amd/csrc/cn_pc_kernels.hpp",
                  "paper_2401_16113_amd/csrc/cn_pc_reduced.hpp",
                  "paper_2401_16113_amd/csrc/cn_pc.hip",
                  "paper_2401_16113_amd/csrc/cn_krylov.hip"]
# hardware-counter traffic of the headline's float64 apply and of the
# production form's float32 apply (variant 8 x 512, two inverse workgroups)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_localvol_4095x1024_fp64pc.txt")
TRAFFIC_FILE_PROD = os.path.join(ROOT, "profiles", "traffic_localvol_65535x4096_fp32pc.txt")
TRAFFIC_PROD_VARIANT = {"tile_cols": 8, "threads": 512, "inverse_split": 1, "forward_split": 2}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, path=None):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy of known size), or None when the
    summary is missing or the kernel sources changed since it was taken."""
    try:
        kv = {}
        with open(path or TRAFFIC_FILE) as fh:
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


PC_KERNELS = ("pc_forward", "pc_reduced", "pc_inverse")
# algorithmic bytes per unknown of one preconditioner apply (float64 input
# and output: v read once, the half spectrum written, read, written and read
# once in the preconditioner's precision, z written once)
PC_BYTES = {"fp64": 48, "fp32": 28}


def apply_roofline(us, n, prec):
    """Rate of one preconditioner apply at the algorithmic bytes per unknown."""
    by = PC_BYTES[prec] * n
    ach = by / (us * 1e-6) / 1e9
    return {"us": round(us, 2), "algorithmic_bytes": by, "bytes_per_unknown": PC_BYTES[prec],
            "GBps": round(ach, 1), "frac_of_peak": round(ach / HBM_PEAK_GBS, 4)}


def stored_traffic_sum(kernels, path=None):
    vals = [stored_traffic(k, path) for k in kernels]
    return None if any(v is None for v in vals) else float(sum(vals))


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


def timed(fn, reps, torch):
    """Median wall time of fn() over reps calls (fn synchronises)."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), out


def form_constant_vol(B, W, torch, reps):
    """The 127 x 64 constant-volatility put: float64, GMRES(20) to 1e-12."""
    import numpy as np
    dev = torch.device("cuda:0")
    inst = W.config1()
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    s = B.Solver(t(inst.a_lo), t(inst.a_di), t(inst.a_up), inst.nt, inst.T, inst.alpha,
                 m_max=20, pc_prec="fp64")
    b = torch.empty(inst.n, dtype=torch.float64, device=dev)
    s.rhs(t(inst.u0), t(inst.f.reshape(-1)), b)
    x = torch.empty_like(b)
    for _ in range(3):
        s.solve(b, x, m=20, rtol=inst.rtol)
    sec, r = timed(lambda: s.solve(b, x, m=20, rtol=inst.rtol), reps, torch)
    if r.status != B.CN_OK:
        raise RuntimeError(f"constant-volatility solve did not converge: {r}")
    out = {"nx": inst.nx, "nt": inst.nt, "unknowns": inst.n, "rtol": inst.rtol,
           "ms_per_solve": sec * 1e3, "device_ms_per_solve": r.seconds * 1e3,
           "unknowns_per_s": inst.n / sec, "iters": r.iters, "relres": r.relres_true}
    x_host = x.cpu().numpy()
    s.close()
    return out, (inst, x_host)


def form_drift_diffusion_2d(B, W, torch, reps):
    """A 2D operator (Sec. 5's setting): seeded variable-coefficient
    drift-diffusion with a mixed derivative on a 127 x 63 grid, 256 steps
    (2,048,256 unknowns), float64, flexible GMRES(20) to 1e-8.  Reports the
    set-up (the band factors of the 129 shifted systems), one preconditioner
    apply and the whole solve."""
    import numpy as np
    dev = torch.device("cuda:0")
    inst = W.drift_diffusion_2d(127, 63, 256, T=0.5, alpha=0.01, seed=21, mixed=0.2)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = B.Solver2D(t(inst.st.reshape(-1)), inst.nx, inst.ny, inst.nt, inst.T, inst.alpha,
                   m_max=20)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    n = inst.nx * inst.ny * inst.nt
    b = torch.empty(n, dtype=torch.float64, device=dev)
    s.rhs(t(inst.u0), t(inst.f.reshape(-1)), b)
    x = torch.empty_like(b)
    z = torch.empty_like(b)
    for _ in range(2):
        s.solve(b, x, m=20, rtol=RTOL)
        s.pc_apply(b, z)
    sec_pc, _ = timed(lambda: s.pc_apply(b, z), 10, torch)
    sec, r = timed(lambda: s.solve(b, x, m=20, rtol=RTOL), reps, torch)
    if r.status != B.CN_OK:
        raise RuntimeError(f"2D solve did not converge: {r}")
    out = {"nx": inst.nx, "ny": inst.ny, "nt": inst.nt, "unknowns": n, "mixed_derivative": 0.2,
           "create_s": create_s, "pc_apply_ms": sec_pc * 1e3, "ms_per_solve": sec * 1e3,
           "unknowns_per_s": n / sec, "iters": r.iters, "relres": r.relres_true}
    x_host = x.cpu().numpy()
    s.close()
    return out, (inst, x_host)


def form_batch_uneven(B, W, torch, reps):
    import numpy as np
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    insts = W.config3()
    probs = [dict(a_lo=t(i.a_lo), a_di=t(i.a_di), a_up=t(i.a_up), nt=i.nt, T=i.T,
                  alpha=i.alpha, m_max=20) for i in insts]
    t0 = time.perf_counter()
    bat = B.Batch(probs, pc_prec="fp32")
    create_s = time.perf_counter() - t0
    b = torch.empty(bat.n, dtype=torch.float64, device=dev)
    bat.rhs(t(np.concatenate([i.u0 for i in insts])),
            t(np.concatenate([i.f.reshape(-1) for i in insts])), b)
    x = torch.empty_like(b)
    bat.solve(b, x, m=20, rtol=RTOL, err_tol=ERR_TOL)
    sec, (tot, per) = timed(lambda: bat.solve(b, x, m=20, rtol=RTOL, err_tol=ERR_TOL), reps, torch)
    if tot.status != B.CN_OK:
        raise RuntimeError(f"uneven batch did not converge: {tot}")
    sec_ng, _ = timed(lambda: bat.solve(b, x, m=20, rtol=RTOL, graphs=False, err_tol=ERR_TOL),
                      reps, torch)
    sec_rr, (tot_rr, _) = timed(lambda: bat.solve(b, x, m=20, rtol=RTOL), reps, torch)
    out = {"instances": len(insts), "unknowns": int(bat.n), "ms_per_solve": sec * 1e3,
           "ms_per_solve_without_graphs": sec_ng * 1e3,
           "unknowns_per_s": bat.n / sec, "max_iters": tot.iters,
           "mean_iters": sum(r.iters for r in per) / len(per),
           "max_relres": tot.relres_true, "max_err_est": tot.err_est,
           "err_tol": ERR_TOL, "create_s": create_s,
           "residual_only": {"ms_per_solve": sec_rr * 1e3, "max_iters": tot_rr.iters}}
    # the reported solution is the error-controlled one
    bat.solve(b, x, m=20, rtol=RTOL, err_tol=ERR_TOL)
    x_host = x.cpu().numpy()
    bat.close()
    return out, (insts, x_host)


def form_warm_start(B, W, torch, n_train, n_held, epochs, reps):
    import numpy as np
    from paper_2401_16113_amd import warmstart as WS
    dev = torch.device("cuda:0")
    chunk = 128
    t0 = time.perf_counter()
    X, Y, worst = WS.generate(W.config4_params(n_train, seed=4), chunk=chunk,
                              log=log if n_train > 4096 else None)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, hist = WS.train(X, Y, epochs=epochs, batch=128, lr=2e-3, seed=0, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del X, Y
    held = W.config4_params(n_held, seed=40)
    acc = {k: {"sec": 0.0, "iters": [], "relres": 0.0} for k in
           ("plain_fp64", "batched_fp32", "batched_fp32_warm", "perfect_coarse")}
    rejected, unknowns, dev_plain = 0, 0, 0.0
    sample = {}   # solutions of the first chunk, per form (error against the oracle)
    for c0 in range(0, n_held, chunk):
        fb = WS.family_batch(held[c0:c0 + chunk])
        n1 = fb.nx * fb.nt
        unknowns += fb.count * n1
        bat = B.Batch(fb.probs, pc_prec="fp32")
        b = torch.empty(bat.n, dtype=torch.float64, device=dev)
        bat.rhs(fb.u0, fb.f, b)
        x = torch.zeros_like(b)
        bat.solve(b, x, m=20, rtol=RTOL, err_tol=ERR_TOL)
        sec, (tot, per) = timed(lambda: bat.solve(b, x, m=20, rtol=RTOL, err_tol=ERR_TOL), reps,
                                torch)
        a = acc["batched_fp32"]
        a["sec"] += sec
        a["iters"] += [r.iters for r in per]
        a["relres"] = max(a["relres"], tot.relres_true)
        a["err_est"] = max(a.get("err_est", 0.0), tot.err_est)
        x_ref = x.clone()
        coarse = torch.empty((fb.count, WS.N_OUT), dtype=torch.float32, device=dev)
        xw = torch.empty_like(b)

        def warm():
            WS.initial_guess(net, fb, coarse=coarse, x0=xw)
            return bat.solve(b, xw, m=20, rtol=RTOL, use_x0=2, err_tol=ERR_TOL)
        warm()
        sec, (tot, per) = timed(warm, reps, torch)
        a = acc["batched_fp32_warm"]
        a["sec"] += sec
        a["iters"] += [r.iters for r in per]
        a["relres"] = max(a["relres"], tot.relres_true)
        a["err_est"] = max(a.get("err_est", 0.0), tot.err_est)
        rejected += sum(r.x0_rejected for r in per)
        # ceiling: the restriction of the converged solution as the guess
        ones = torch.ones(fb.count, dtype=torch.float64, device=dev)
        B.ws_restrict(x_ref, fb.count, fb.nx, fb.nt, ones, coarse)
        xp = torch.empty_like(b)
        B.ws_interpolate(coarse, fb.count, fb.nx, fb.nt, fb.u0, fb.gl, fb.gr, ones, xp)
        tot, per = bat.solve(b, xp, m=20, rtol=RTOL, use_x0=2, err_tol=ERR_TOL)
        a = acc["perfect_coarse"]
        a["iters"] += [r.iters for r in per]
        a["relres"] = max(a["relres"], tot.relres_true)
        a["err_est"] = max(a.get("err_est", 0.0), tot.err_est)
        bat.close()
        if c0 == 0:
            sample = {"params": held[:fb.count], "batched_fp32": x_ref.cpu().numpy(),
                      "batched_fp32_warm": xw.cpu().numpy(), "plain_fp64": np.empty(fb.count * n1)}
        # plain: float64 preconditioner, one instance at a time, zero start
        a = acc["plain_fp64"]
        for q, pr in enumerate(fb.probs):
            s = B.Solver(pr["a_lo"], pr["a_di"], pr["a_up"], fb.nt, pr["T"], 0.01, m_max=20,
                         pc_prec="fp64")
            bq = b[q * n1:(q + 1) * n1]
            xq = torch.zeros_like(bq)
            s.solve(bq, xq, m=20, rtol=RTOL, err_tol=ERR_TOL)
            sec, r = timed(lambda: s.solve(bq, xq, m=20, rtol=RTOL, err_tol=ERR_TOL), 1, torch)
            a["sec"] += sec
            a["iters"].append(r.iters)
            a["relres"] = max(a["relres"], r.relres_true)
            a["err_est"] = max(a.get("err_est", 0.0), r.err_est)
            dev_plain += r.seconds
            if c0 == 0:
                sample["plain_fp64"][q * n1:(q + 1) * n1] = xq.cpu().numpy()
            s.close()
        del fb, bat, b, x, x_ref, xw, xp
    out = {"train_instances": n_train, "heldout_instances": n_held, "nx": W.WS_NX,
           "nt": W.WS_NT, "unknowns": unknowns, "data_gen_s": gen_s, "train_s": train_s,
           "epochs": epochs, "final_loss": hist[-1], "worst_training_relres": worst,
           "rejected_guesses": rejected}
    for k, a in acc.items():
        it = a["iters"]
        e = {"mean_iters": sum(it) / len(it), "max_iters": max(it), "max_relres": a["relres"],
             "max_err_est": a.get("err_est"), "err_tol": ERR_TOL}
        if a["sec"] > 0:
            e["ms_per_instance"] = a["sec"] / n_held * 1e3
            e["unknowns_per_s"] = unknowns / a["sec"]
        out[k] = e
    out["speedup_vs_plain"] = {k: out[k]["unknowns_per_s"] / out["plain_fp64"]["unknowns_per_s"]
                               for k in ("batched_fp32", "batched_fp32_warm")}
    net.close()
    return out, sample


def form_production(B, W, torch, reps):
    """The production shape (2.7e8 unknowns) with the float32 preconditioner:
    whole-solve throughput and the per-kernel rates of inner iteration 1."""
    import numpy as np
    dev = torch.device("cuda:0")
    inst = W.config5()
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    s = B.Solver(t(inst.a_lo), t(inst.a_di), t(inst.a_up), inst.nt, inst.T, inst.alpha,
                 m_max=20, pc_prec="fp32")
    b = torch.empty(inst.n, dtype=torch.float64, device=dev)
    s.rhs(t(inst.u0), t(inst.f.reshape(-1)), b)
    # the forcing is the left boundary column only: keep that for the oracle
    f_col = inst.f[:, 0].copy()
    del inst.f
    x = torch.empty_like(b)
    s.solve(b, x, m=20, rtol=RTOL)
    sec, r = timed(lambda: s.solve(b, x, m=20, rtol=RTOL), reps, torch)
    if r.status != B.CN_OK:
        raise RuntimeError(f"production shape did not converge: {r}")
    prof = s.profile_step(j=1, reps=5)
    pc_us = sum(prof[k]["ms"] for k in PC_KERNELS) * 1e3
    out = {"nx": inst.nx, "nt": inst.nt, "unknowns": inst.n, "pc_variant": s.query(),
           "ms_per_solve": sec * 1e3, "unknowns_per_s": inst.n / sec, "iters": r.iters,
           "relres": r.relres_true,
           "kernels_step1": {k: {"us": v["ms"] * 1e3, "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9}
                             for k, v in prof.items()},
           "pc_apply": apply_roofline(pc_us, inst.n, "fp32")}
    q = out["pc_variant"]
    same = all(q.get(k) == v for k, v in TRAFFIC_PROD_VARIANT.items())
    out["pc_apply"]["traffic"] = stored_traffic_sum(PC_KERNELS, TRAFFIC_FILE_PROD) if same else None
    x_host = x.cpu().numpy()
    s.close()
    return out, (inst, f_col, x_host)


def rel_err(x, u):
    import numpy as np
    return float(np.max(np.abs(x - u)) / np.max(np.abs(u)))


def cpu_baseline(inst, x_gpu, checks):
    """The oracle on the host: its whole solve of the headline workload
    (timed) and the exact CN solution of every timed form (time stepping,
    Sec. 2.2), against which each form's GPU result is compared (relative
    max-norm over all space-time nodes)."""
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
    t0 = time.perf_counter()
    u = O.sequential_cn_banded(*args, inst.u0, f=inst.f)
    sec_cn = time.perf_counter() - t0
    errs = {k: rel_err(v, u) for k, v in x_gpu.items()}
    extra = {}
    if "constant_vol" in checks:
        ci, xc = checks["constant_vol"]
        uc = O.sequential_cn(ci.a_lo, ci.a_di, ci.a_up, ci.T, ci.nt, ci.u0, ci.f)
        extra["constant_vol"] = rel_err(xc, uc)
    if "batch_uneven" in checks:
        insts, xb = checks["batch_uneven"]
        worst, off = 0.0, 0
        for i in insts:
            ui = O.sequential_cn_banded(i.a_lo, i.a_di, i.a_up, i.T, i.nt, i.u0, f=i.f)
            worst = max(worst, rel_err(xb[off:off + i.n], ui))
            off += i.n
        extra["batch_uneven_max_over_instances"] = worst
    if "warm_start" in checks:
        from paper_2401_16113_amd import workloads as W
        smp = checks["warm_start"]
        params = smp["params"]
        n1 = W.WS_NX * W.WS_NT
        ws = {k: 0.0 for k in ("plain_fp64", "batched_fp32", "batched_fp32_warm")}
        for q, p in enumerate(params):
            (_, lo, di, up, u0, f_col, _, _), _, _ = W.config4_rows(p)
            uq = O.sequential_cn_banded(lo, di, up, float(p[3]), W.WS_NT, u0, f_col=f_col)
            for k in ws:
                ws[k] = max(ws[k], rel_err(smp[k][q * n1:(q + 1) * n1], uq))
        extra["warm_start_sample"] = {"instances": int(len(params)), **ws}
    if "drift_diffusion_2d" in checks:
        from oracle import cn2d_oracle as O2
        di, xd = checks["drift_diffusion_2d"]
        A2 = O2.stencil_matrix(di.st, di.nx, di.ny)
        extra["drift_diffusion_2d"] = rel_err(xd, O2.sequential_cn(A2, di.T, di.nt, di.u0, di.f))
    if "production" in checks:
        pi, f_col, xp = checks["production"]
        up_ = O.sequential_cn_banded(pi.a_lo, pi.a_di, pi.a_up, pi.T, pi.nt, pi.u0, f_col=f_col)
        extra["production"] = rel_err(xp, up_)
        del up_
    cpu = ""
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": inst.n / sec, "unit": "unknowns/s", "cores": int(cores), "kind": "oracle",
        "sample": (f"whole solve of the same {inst.nx}x{inst.nt} workload by the FP64 oracle "
                   f"(right-preconditioned GMRES({M}), direct O(N_t^2) DFT sums), median of 3 "
                   f"runs, {sec:.2f} s each, {r.iters} iterations"),
        "cpu_model": cpu, "host_cores": len(os.sched_getaffinity(0)),
        "sequential_cn_unknowns_per_s": inst.n / sec_cn,
        "gpu_err_vs_exact_cn": errs,
        "forms_err_vs_exact_cn": extra,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the constant-volatility, batch, warm-start and production forms")
    ap.add_argument("--forms", default="",
                    help="comma-separated subset of the forms to run (constant_vol, batch_uneven, "
                         "warm_start, drift_diffusion_2d, production); default all")
    ap.add_argument("--ws-train", type=int, default=20000,
                    help="training instances of the warm-start network")
    ap.add_argument("--ws-heldout", type=int, default=1024,
                    help="held-out instances of the warm-start comparison")
    ap.add_argument("--ws-epochs", type=int, default=60)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run 256 MiB device copies (hardware-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2401_16113_amd import binding as B
    from paper_2401_16113_amd import workloads as W

    dev = torch.device("cuda:0")
    # headline workload and the alpha sweep, both preconditioner precisions
    variants, profs, xs = {}, {}, {}
    sweep = {}
    for alpha in (0.01, 0.001, 0.05):
        inst_a = W.config2(alpha=alpha)
        for prec in ("fp64", "fp32"):
            head = alpha == 0.01
            steps = args.steps if head else max(3, args.steps // 4)
            log(f"[bench] alpha {alpha} {prec} preconditioner: {args.warmup} warm-up + "
                f"{steps} timed solves")
            v, p, x = run_variant(B, W, inst_a, prec, steps, args.warmup, dev, torch)
            key = "plain_fp64" if prec == "fp64" else "fp32_pc"
            if head:
                variants[key], profs[prec] = v, p
            sweep.setdefault(f"alpha={alpha}", {})[key] = {
                k: v[k] for k in ("ms_per_solve", "unknowns_per_s", "iters", "relres")}
            xs[f"alpha={alpha} {key}"] = x
            log(f"[bench] {prec}: {v['ms_per_solve']:.3f} ms/solve, {v['iters']} iters, "
                f"relres {v['relres']:.2e}")
    inst = W.config2(alpha=0.01)
    prim = variants["plain_fp64"]
    # roofline: the preconditioner apply of the headline form, with the longest
    # single launch beside it
    prof = profs["fp64"]
    pc_us = sum(prof[k]["ms"] for k in PC_KERNELS) * 1e3
    ap_ = apply_roofline(pc_us, inst.n, "fp64")
    dom = max(prof, key=lambda k: prof[k]["ms"])
    dach = prof[dom]["bytes"] / (prof[dom]["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": "preconditioner apply (pc_forward + pc_reduced + "
                                      "pc_inverse), float64",
            "achieved": ap_["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ap_["frac_of_peak"], "traffic": stored_traffic_sum(PC_KERNELS),
            "avg_launch_us": ap_["us"], "algorithmic_bytes": ap_["algorithmic_bytes"],
            "bytes_per_unknown": ap_["bytes_per_unknown"],
            "per_kernel_us": {k: round(prof[k]["ms"] * 1e3, 2) for k in PC_KERNELS},
            "longest_launch": {"kernel": dom, "avg_launch_us": round(prof[dom]["ms"] * 1e3, 2),
                               "algorithmic_bytes": prof[dom]["bytes"],
                               "achieved": round(dach, 1),
                               "frac": round(dach / HBM_PEAK_GBS, 4),
                               "traffic": stored_traffic(dom)}}
    out = {
        "metric": "space-time unknowns/s to rel.res 1e-8: plain vs batched+FP32-PC+warm-start",
        "value": prim["unknowns_per_s"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"local-vol Black-Scholes put, N_x={inst.nx}, N_t={inst.nt}, "
                               f"alpha={inst.alpha}, flexible GMRES({M}), rtol {RTOL}",
                   "unknowns": inst.n, "form": "plain_fp64",
                   "batched_warm_form": "forms.warm_start (held-out 2047x512 local-vol puts: "
                                        "plain_fp64 vs batched_fp32 vs batched_fp32_warm)"},
        "variants": variants,
        "alpha_sweep": sweep,
        "roofline": roof,
    }
    checks = {}
    if not args.no_forms:
        forms = {}
        want = set(args.forms.split(",")) if args.forms else None
        run = lambda name: want is None or name in want
        if run("constant_vol"):
            log("[bench] form: constant volatility 127x64")
            forms["constant_vol"], checks["constant_vol"] = form_constant_vol(B, W, torch, reps=20)
        if run("batch_uneven"):
            log("[bench] form: uneven batch of 512 instances")
            forms["batch_uneven"], checks["batch_uneven"] = form_batch_uneven(B, W, torch, reps=5)
            log(f"[bench] batch: {forms['batch_uneven']['ms_per_solve']:.2f} ms, "
                f"{forms['batch_uneven']['unknowns_per_s']:.3e} unknowns/s")
        if run("warm_start"):
            log(f"[bench] form: warm start ({args.ws_train} training solves, "
                f"{args.ws_heldout} held-out)")
            forms["warm_start"], checks["warm_start"] = form_warm_start(
                B, W, torch, args.ws_train, args.ws_heldout, args.ws_epochs, reps=3)
            ws = forms["warm_start"]
            log(f"[bench] warm start: plain {ws['plain_fp64']['unknowns_per_s']:.3e}, batched "
                f"{ws['batched_fp32']['unknowns_per_s']:.3e}, batched+warm "
                f"{ws['batched_fp32_warm']['unknowns_per_s']:.3e} unknowns/s; iterations "
                f"{ws['plain_fp64']['mean_iters']:.2f} / {ws['batched_fp32']['mean_iters']:.2f} / "
                f"{ws['batched_fp32_warm']['mean_iters']:.2f}")
            out["batched_fp32_warm_vs_plain"] = ws["speedup_vs_plain"]["batched_fp32_warm"]
        if run("drift_diffusion_2d"):
            log("[bench] form: 2D drift-diffusion 127x63x256")
            forms["drift_diffusion_2d"], checks["drift_diffusion_2d"] = form_drift_diffusion_2d(
                B, W, torch, reps=5)
            d2 = forms["drift_diffusion_2d"]
            log(f"[bench] 2D: {d2['ms_per_solve']:.2f} ms, {d2['unknowns_per_s']:.3e} unknowns/s, "
                f"{d2['iters']} iters, apply {d2['pc_apply_ms']:.3f} ms, set-up {d2['create_s']:.2f} s")
        if run("production"):
            log("[bench] form: production shape 65535x4096")
            forms["production"], checks["production"] = form_production(B, W, torch, reps=3)
            pr = forms["production"]
            log(f"[bench] production: {pr['ms_per_solve']:.2f} ms, {pr['unknowns_per_s']:.3e} "
                f"unknowns/s, {pr['iters']} iters, preconditioner apply "
                f"{pr['pc_apply']['GBps']:.0f} GB/s")
        out["forms"] = forms
    if args.calibrate_copy:
        log("[bench] calibration: 5 device copies of 256 MiB")
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 8
    if not args.no_cpu_baseline:
        log("[bench] cpu_baseline: oracle solve on the host, errors of every form")
        out["cpu_baseline"] = cpu_baseline(inst, xs, checks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
