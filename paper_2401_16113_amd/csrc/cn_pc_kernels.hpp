// Transform kernels of the alpha-circulant preconditioner (included by the
// per-precision translation units cn_pc_f64.hip and cn_pc_f32.hip).
//
//  K1 (k_pc_forward): one workgroup per tile of B spatial columns.  Loads the
//     B x N_t tile, applies the alpha weights Lambda_alpha (step (a)), runs a
//     length-N_t complex Stockham FFT in LDS on pairs of real columns (two
//     real transforms per complex one; only the N_t/2+1 non-redundant modes
//     are used, Remark 1), then for every frequency j solves the shifted
//     system (lambda_{1,j} I - lambda_{2,j} A~) restricted to the tile's
//     interior columns (step (b), local part) and writes the tile image plus
//     two partial right-hand sides of the separator systems per (j, tile).
//  K3 (k_pc_inverse): per tile, adds the separator contributions to the local
//     solution, runs the inverse FFT, multiplies by Lambda_alpha^{-1}/N_t
//     (step (c)) and writes z.
#pragma once
#include <type_traits>

#include "cn_internal.hpp"
#include "cn_pc_reduced.hpp"

namespace cn {

// ---------------------------------------------------------------------------
// K1
// ---------------------------------------------------------------------------
template <typename R, int LOG2N, int BB, int TT>
__device__ __forceinline__ void pc_forward_tile(
    int p, const CN_G double* __restrict__ v, const CN_G double* scp, const CN_G int* stop,
    const CN_G double* __restrict__ lo,
    const CN_G double* __restrict__ di, const CN_G double* __restrict__ up,
    const CN_G double* __restrict__ wfw, const Cx<R>* __restrict__ tw,
    const CN_G Cx<double>* __restrict__ mu, const CN_G Cx<double>* __restrict__ il2,
    CN_G Cx<R>* __restrict__ spec, CN_G Cx<R>* __restrict__ iface, int nx, int vp, int P) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  __shared__ Cx<R> lds[Cfg::LDS_ELEMS];
  __shared__ Cx<R> ltw[Cfg::TWN];
  __shared__ R co[3 * B];
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  // step (a): alpha-weighted tile, columns (2s, 2s+1) packed as one complex
  // sequence.  The stop flag and the basis scale are uniform scalar loads,
  // issued first (they do not wait behind vector loads); then every vector
  // load of the phase (weights, tile, twiddles, operator rows) is issued
  // before any is consumed, in the order they are used.
  R* ldsr = reinterpret_cast<R*>(lds);
  {
    const int stopped = stop != nullptr ? *stop : 0;
    const double sc = scp != nullptr ? *scp : 1.0;
    // the alpha weights of the thread's levels: B divides T, so its levels
    // are k = tid/B + q T/B and w_q = alpha^{k/N_t} = w_0 rho^q with
    // rho = alpha^{(T/B)/N_t}, formed by recurrence (rounding <= LPT eps
    // relative) instead of one table load per element
    static_assert(T % B == 0, "the workgroup size must be a multiple of the tile width");
    const double w0 = wfw[min(tid / B, N - 1)];
    const double rho = wfw[T / B < N ? T / B : 0];
    constexpr int LPT = (N * B + T - 1) / T;
    double xv[LPT];
    {
      // element (k, b) of the tile at byte offset (k vp + b) 8 from column
      // i0; thread tid reads column b = tid mod B (unconditionally: columns
      // past the grid's edge re-read its last column and are masked when
      // staged) at levels tid/B + q T/B, a uniform step of (T/B) vp 8 bytes
      // per q.  Offsets stay below N_t vp 8 bytes (below 2^32: checked at
      // set-up).
      const BufRd vb(v + i0);
      const unsigned vo = ((unsigned)(tid / B) * (unsigned)vp + (unsigned)min(tid % B, ncols - 1)) * 8u;
      const unsigned step = (unsigned)(T / B) * (unsigned)vp * 8u;
#pragma unroll
      for (int q = 0; q < LPT; ++q) {
        const int e = tid + q * T;
        if ((N * B) % T == 0 || e < N * B) xv[q] = vb.f64(vo, (unsigned)q * step);
      }
    }
    TwStage<R, Cfg::TWN, T, Cfg::TWPT> tws;
    if constexpr (Cfg::TWL) tws.fetch(gp(tw));
    double cov = 0.0;
    if (tid < 3 * B) {
      const int b = min(tid / 3, ncols - 1), c = tid % 3;
      cov = c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]);
    }
    // a stopped cycle's loads are simply dropped
    if (stopped) return;
    if (tid < 3 * B) co[tid] = tid / 3 < ncols ? (R)cov : R(0);
    double w = w0 * sc;
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      if ((N * B) % T == 0 || e < N * B) {
        const int k = e / B, b = e % B;
        const R val = (R)(xv[q] * w);
        ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] = b < ncols ? val : R(0);
      }
      w *= rho;
    }
    if constexpr (Cfg::TWL) tws.store(ltw);
  }
  __syncthreads();
  fft_tile<Cfg, R, LOG2N, false>(lds, ltw, tw, threadIdx.x);

  // the shifts of the thread's frequencies (task u: t = tid + u T; t = 0
  // solves the real modes 0 and N/2, held as (.x, .y)).  With several tasks
  // per thread they are requested together after the FFT (one latency for
  // all of them); with one task, at the task (earlier placement cost the
  // 16-column, 1024-thread variants register spills).
  constexpr int NTK = Cfg::NTK;
  auto shifts = [&](int t, Cx<double>& m, Cx<double>& s2) {
    if (t == 0) {
      const int h = N >= 2 ? N / 2 : 0;
      m = Cx<double>{mu[0].x, mu[h].x};
      s2 = Cx<double>{il2[0].x, il2[h].x};
    } else if (Cfg::TASKS % T == 0 || t < Cfg::TASKS) {
      m = gld(mu + t);
      s2 = gld(il2 + t);
    }
  };
  Cx<double> tmd[NTK], tsd[NTK];
  if constexpr (NTK > 1) {
#pragma unroll
    for (int u = 0; u < NTK; ++u) shifts(tid + u * T, tmd[u], tsd[u]);
  }

  // step (b), tile-local part.  Per frequency the tile leaves two partial
  // right-hand sides of the separator systems: d + lo y_last for its own
  // separator (its last column) and up y_first for the separator left of it.
  const bool has_sep = p < P - 1;
  const int nb = has_sep ? B - 1 : ncols;
  const R lsep = has_sep ? co[3 * (B - 1)] : R(0);
  const R uprev = p > 0 ? (R)up[i0 - 1] : R(0);
  CN_G Cx<R>* ifc = iface + (size_t)p * 2;
#pragma unroll
  for (int u = 0; u < NTK; ++u) {
    const int t = tid + u * T;
    if (Cfg::TASKS % T != 0 && t >= Cfg::TASKS) break;
    if constexpr (NTK == 1) shifts(t, tmd[u], tsd[u]);
    if (t == 0) {
      // j = 0 and j = N/2: real modes, real shifts
      const int nreal = N >= 2 ? 2 : 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nreal) break;
        const int j = h == 0 ? 0 : N / 2;
        const R m = (R)(h == 0 ? tmd[u].x : tmd[u].y), s2 = (R)(h == 0 ? tsd[u].x : tsd[u].y);
        R d[B];
#pragma unroll
        for (int c = 0; c < NSEQ; ++c) {
          const Cx<R> z = lds[lidx<N>(c, j)];
          d[2 * c] = z.x * s2;
          d[2 * c + 1] = z.y * s2;
        }
        const R sepv = d[B - 1];
        tile_solve<R, R, B>(d, m, co, nb);
        R ylast = d[0];
#pragma unroll
        for (int b = 1; b < B; ++b)
          if (b == nb - 1) ylast = d[b];
#pragma unroll
        for (int c = 0; c < NSEQ; ++c) lds[lidx<N>(c, j)] = Cx<R>{d[2 * c], d[2 * c + 1]};
        CN_G Cx<R>* f = ifc + (size_t)j * P * 2;
        gst(f, Cx<R>{has_sep ? sepv + lsep * ylast : R(0), R(0)});
        gst(f + 1, Cx<R>{uprev * d[0], R(0)});
      }
    } else {
      const int j = t;
      const Cx<R> m{(R)tmd[u].x, (R)tmd[u].y}, s2{(R)tsd[u].x, (R)tsd[u].y};
      Cx<R> d[B];
#pragma unroll
      for (int c = 0; c < NSEQ; ++c) {
        const Cx<R> z = lds[lidx<N>(c, j)];
        const Cx<R> zc = conj(lds[lidx<N>(c, N - j)]);
        const Cx<R> sum = z + zc, dif = z - zc;
        // X_{2c} = (Z_j + conj Z_{N-j})/2, X_{2c+1} = (Z_j - conj Z_{N-j})/(2i)
        d[2 * c] = (R(0.5) * sum) * s2;
        d[2 * c + 1] = Cx<R>{R(0.5) * dif.y, R(-0.5) * dif.x} * s2;
      }
      const Cx<R> sepv = d[B - 1];
      tile_solve<R, Cx<R>, B>(d, m, co, nb);
      Cx<R> ylast = d[0];
#pragma unroll
      for (int b = 1; b < B; ++b)
        if (b == nb - 1) ylast = d[b];
#pragma unroll
      for (int c = 0; c < NSEQ; ++c) {
        lds[lidx<N>(c, j)] = d[2 * c];
        lds[lidx<N>(c, N - j)] = d[2 * c + 1];
      }
      CN_G Cx<R>* f = ifc + (size_t)j * P * 2;
      gst(f, has_sep ? sepv + lsep * ylast : Cx<R>{R(0), R(0)});
      gst(f + 1, uprev * d[0]);
    }
  }
  __syncthreads();
  CN_G Cx<R>* img = spec + (size_t)p * NSEQ * N;
  {
    constexpr int SPT = (NSEQ * N + T - 1) / T;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSEQ * N) % T == 0 || e < NSEQ * N) gst(img + e, lds[lidx<N>(e / N, e % N)]);
    }
  }
}

// v_ovr: input vector instead of V_j; pitch: its row pitch (0: the internal
// pitch of V)
template <typename R, int LOG2N, int BB, int TT>
__global__ __launch_bounds__(TT) void k_pc_forward(const InstDesc* __restrict__ D,
                                                   const int2* __restrict__ items, int nitems,
                                                   int nitems_pad, int jv,
                                                   const double* __restrict__ v_ovr, int pitch) {
  const int itx = xcd_tile(blockIdx.x, nitems_pad);
  if (itx >= nitems) return;
  const int2 wi = work_item(items, itx);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  // inside a solve: input V_j scaled by 1/||v_j||, skipped once the cycle stopped
  const bool in_solve = v_ovr == nullptr;
  const double* v = in_solve ? d.V + (size_t)jv * d.vstride : v_ovr;
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  const Cx<R>* tw = Cfg::TWMODE == 3
                        ? (std::is_same<R, double>::value ? (const Cx<R>*)pl.tw2 : (const Cx<R>*)pl.tw2_f)
                        : (std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f);
  pc_forward_tile<R, LOG2N, BB, TT>(wi.y, gp(v), in_solve ? gp(d.st->vscale + jv) : nullptr,
                                    in_solve ? gp(&d.st->sum.done) : nullptr, gp(pl.lo), gp(pl.di),
                                    gp(pl.up), gp(pl.wfw), tw, gp((const Cx<double>*)pl.mu),
                                    gp((const Cx<double>*)pl.il2), gp((Cx<R>*)pl.spec),
                                    gp((Cx<R>*)pl.iface), pl.nx, pitch > 0 ? pitch : d.ldx, pl.P);
}

// ---------------------------------------------------------------------------
// K1 by frequency parity (float32, half the LDS)
// ---------------------------------------------------------------------------
// One radix-2 step of a decimation in frequency: with y the weighted tile
// sequence, a_k = y_k + y_{k+N/2} and b_k = (y_k - y_{k+N/2}) w_N^k for
// k < N/2, the even frequencies are Y_{2m} = DFT_{N/2}(a)_m and the odd ones
// Y_{2m+1} = DFT_{N/2}(b)_m.  A conjugate pair (j, N - j) has one parity, so
// the workgroup transforms a in LDS, solves the step-(b) systems of the even
// frequencies and stores them while b waits in registers, then does the same
// for b and the odd frequencies.  The tile is read once; LDS holds half of
// it, so two workgroups (two tiles) share a CU and one's loads overlap the
// other's transforms.  Sequence c of tile p keeps position j of the length-N
// layout at (p NSEQ + c) N + (j mod 2) N/2 + floor(j/2) of the tile image;
// the interface right-hand sides are written per frequency as in K1.
template <typename R, int LOG2N, int BB, int TT>
__device__ __forceinline__ void pc_forward_pair(
    int p, const CN_G double* __restrict__ v, const CN_G double* scp, const CN_G int* stop,
    const CN_G double* __restrict__ lo, const CN_G double* __restrict__ di,
    const CN_G double* __restrict__ up, const CN_G double* __restrict__ wfw,
    const CN_G Cx<R>* __restrict__ tw2, const CN_G Cx<double>* __restrict__ mu,
    const CN_G Cx<double>* __restrict__ il2, CN_G Cx<R>* __restrict__ spec,
    CN_G Cx<R>* __restrict__ iface, int nx, int vp, int P) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  using CfgH = PcCfg<R, LOG2N - 1, BB, TT>;
  constexpr int N = Cfg::N, NH = N / 2, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  constexpr int TWN = Split2<N>::SIZE;
  static_assert(T % B == 0 && NH % (T / B) == 0, "levels k and k + N/2 must share a thread");
  // thread tid reads column b = tid mod B at levels k = tid/B + q T/B;
  // level k + N/2 is q + LPH, so each thread pairs its own loads.  The tile
  // is read in RND rounds of LPR pairs (2 LPR loads in flight).
  constexpr int LPH = NH * B / T;
  constexpr int RND = LPH >= 16 ? 2 : 1;
  constexpr int LPR = LPH / RND;
  __shared__ Cx<R> lds[CfgH::LDS_ELEMS];
  __shared__ Cx<R> ltw[TWN];
  __shared__ R co[3 * B];
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  R* ldsr = reinterpret_cast<R*>(lds);
  R bv[LPH];  // this thread's entries of b (column tid mod B)
  {
    // weights as in K1: w_q = w_0 rho^q; level k + N/2 has w_q alpha^{1/2}
    const int stopped = stop != nullptr ? *stop : 0;
    const double sc = scp != nullptr ? *scp : 1.0;
    const double w0 = wfw[tid / B];
    const double rho = wfw[T / B];
    const double ah = wfw[NH];
    const BufRd vb(v + i0);
    const int b = tid % B;
    const unsigned vo = ((unsigned)(tid / B) * (unsigned)vp + (unsigned)min(b, ncols - 1)) * 8u;
    const unsigned step = (unsigned)(T / B) * (unsigned)vp * 8u;
    const unsigned hstep = (unsigned)NH * (unsigned)vp * 8u;
    TwStage<R, TWN, T, (TWN + T - 1) / T> tws;
    double w = w0 * sc;
    const bool live = b < ncols;
    const int slot = b & 1, sq = b >> 1;
#pragma unroll
    for (int r = 0; r < RND; ++r) {
      double xl[LPR], xh[LPR];
#pragma unroll
      for (int q = 0; q < LPR; ++q) {
        const unsigned o = (unsigned)(r * LPR + q) * step;
        xl[q] = vb.f64(vo, o);
        xh[q] = vb.f64(vo, o + hstep);
      }
      if (r == 0) {
        tws.fetch(tw2);
        double cov = 0.0;
        if (tid < 3 * B) {
          const int bb = min(tid / 3, ncols - 1), c = tid % 3;
          cov = c == 0 ? lo[i0 + bb] : (c == 1 ? di[i0 + bb] : up[i0 + bb]);
        }
        // a stopped cycle's loads are simply dropped
        if (stopped) return;
        if (tid < 3 * B) co[tid] = tid / 3 < ncols ? (R)cov : R(0);
      }
#pragma unroll
      for (int q = 0; q < LPR; ++q) {
        const int k = tid / B + (r * LPR + q) * (T / B);
        const double yl = xl[q] * w, yh = xh[q] * (w * ah);
        ldsr[2 * lidx<NH>(sq, k) + slot] = live ? (R)(yl + yh) : R(0);
        R bq = live ? (R)(yl - yh) : R(0);
        // formed here: sunk to its use after the even half, it would keep
        // the float64 inputs live instead (twice the registers, spilled)
        asm volatile("" : "+v"(bq));
        bv[r * LPR + q] = bq;
        w *= rho;
      }
      // the next round's loads stay behind this one's use (hoisted, they
      // would need twice the registers)
      __builtin_amdgcn_sched_barrier(0);
    }
    tws.store(ltw);
  }
  __syncthreads();

  constexpr int TASKS = N / 4;  // per parity
  constexpr int NTK = (TASKS + T - 1) / T;
  const bool has_sep = p < P - 1;
  const int nb = has_sep ? B - 1 : ncols;
  const R lsep = has_sep ? co[3 * (B - 1)] : R(0);
  const R uprev = p > 0 ? (R)up[i0 - 1] : R(0);
  CN_G Cx<R>* ifc = iface + (size_t)p * 2;
#pragma unroll 1
  for (int hf = 0; hf < 2; ++hf) {
    const bool odd = hf != 0;
    if (odd) {
      // b replaces a in LDS (its w_N^k factor is applied by the first pass)
#pragma unroll
      for (int q = 0; q < LPH; ++q) {
        const int t = phase_tid<T>();
        const int k = t / B + q * (T / B);
        ldsr[2 * lidx<NH>((t % B) >> 1, k) + (t & 1)] = bv[q];
      }
      __syncthreads();
    }
    fft_half<R, LOG2N, NSEQ, T, CfgH::MAXLOG>(lds, ltw, phase_tid<T>(), odd);
    // Task t < N/4: even half, t = 0 the real modes 0 and N/2 (positions 0
    // and N/4), else j = 2t at positions t and N/2 - t; odd half, j = 2t + 1
    // at positions t and N/2 - 1 - t.
    const int tid2 = phase_tid<T>();
    Cx<double> tmd[NTK], tsd[NTK];
#pragma unroll
    for (int u = 0; u < NTK; ++u) {
      const int t = tid2 + u * T;
      const int tt = (TASKS % T == 0 || t < TASKS) ? t : 0;
      const int j = 2 * tt + hf;
      const Cx<double> ma = gld(mu + j), mb = gld(mu + NH);
      const Cx<double> sa = gld(il2 + j), sb = gld(il2 + NH);
      const bool real = !odd && t == 0;
      tmd[u] = real ? Cx<double>{ma.x, mb.x} : ma;
      tsd[u] = real ? Cx<double>{sa.x, sb.x} : sa;
    }
#pragma unroll
    for (int u = 0; u < NTK; ++u) {
      const int t = tid2 + u * T;
      if (TASKS % T != 0 && t >= TASKS) break;
      if (!odd && t == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = h == 0 ? 0 : NH, pos = h == 0 ? 0 : NH / 2;
          const R m = (R)(h == 0 ? tmd[u].x : tmd[u].y), s2 = (R)(h == 0 ? tsd[u].x : tsd[u].y);
          R d[B];
#pragma unroll
          for (int c = 0; c < NSEQ; ++c) {
            const Cx<R> z = lds[lidx<NH>(c, pos)];
            d[2 * c] = z.x * s2;
            d[2 * c + 1] = z.y * s2;
          }
          const R sepv = d[B - 1];
          tile_solve<R, R, B>(d, m, co, nb);
          R ylast = d[0];
#pragma unroll
          for (int bb = 1; bb < B; ++bb)
            if (bb == nb - 1) ylast = d[bb];
#pragma unroll
          for (int c = 0; c < NSEQ; ++c) lds[lidx<NH>(c, pos)] = Cx<R>{d[2 * c], d[2 * c + 1]};
          CN_G Cx<R>* f = ifc + (size_t)j * P * 2;
          gst(f, Cx<R>{has_sep ? sepv + lsep * ylast : R(0), R(0)});
          gst(f + 1, Cx<R>{uprev * d[0], R(0)});
        }
      } else {
        const int j = 2 * t + hf;
        const int pa = t, pb = NH - hf - t;
        const Cx<R> m{(R)tmd[u].x, (R)tmd[u].y}, s2{(R)tsd[u].x, (R)tsd[u].y};
        Cx<R> d[B];
#pragma unroll
        for (int c = 0; c < NSEQ; ++c) {
          const Cx<R> z = lds[lidx<NH>(c, pa)];
          const Cx<R> zc = conj(lds[lidx<NH>(c, pb)]);
          const Cx<R> sum = z + zc, dif = z - zc;
          d[2 * c] = (R(0.5) * sum) * s2;
          d[2 * c + 1] = Cx<R>{R(0.5) * dif.y, R(-0.5) * dif.x} * s2;
        }
        const Cx<R> sepv = d[B - 1];
        tile_solve<R, Cx<R>, B>(d, m, co, nb);
        Cx<R> ylast = d[0];
#pragma unroll
        for (int bb = 1; bb < B; ++bb)
          if (bb == nb - 1) ylast = d[bb];
#pragma unroll
        for (int c = 0; c < NSEQ; ++c) {
          lds[lidx<NH>(c, pa)] = d[2 * c];
          lds[lidx<NH>(c, pb)] = d[2 * c + 1];
        }
        CN_G Cx<R>* f = ifc + (size_t)j * P * 2;
        gst(f, has_sep ? sepv + lsep * ylast : Cx<R>{R(0), R(0)});
        gst(f + 1, uprev * d[0]);
      }
    }
    __syncthreads();
    {
      const int tid3 = phase_tid<T>();
      CN_G Cx<R>* img = spec + (size_t)p * NSEQ * N + (size_t)hf * NH;
      constexpr int SPT = (NSEQ * NH + T - 1) / T;
#pragma unroll
      for (int q = 0; q < SPT; ++q) {
        const int e = tid3 + q * T;
        if ((NSEQ * NH) % T == 0 || e < NSEQ * NH) {
          const int c = e / NH, m = e % NH;
          gst(img + (size_t)c * N + m, lds[lidx<NH>(c, m)]);
        }
      }
    }
    // the odd half overwrites the LDS the stores above read
    __syncthreads();
  }
}

// At most 128 registers, so that two workgroups fit a CU.
template <typename R, int LOG2N, int BB, int TT>
__global__ __launch_bounds__(TT) __attribute__((amdgpu_waves_per_eu(4)))
void k_pc_forward_pair(const InstDesc* __restrict__ D, const int2* __restrict__ items, int nitems,
                       int nitems_pad, int jv, const double* __restrict__ v_ovr, int pitch) {
  const int itx = xcd_tile(blockIdx.x, nitems_pad);
  if (itx >= nitems) return;
  const int2 wi = work_item(items, itx);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  const bool in_solve = v_ovr == nullptr;
  const double* v = in_solve ? d.V + (size_t)jv * d.vstride : v_ovr;
  const Cx<R>* tw2 = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw2 : (const Cx<R>*)pl.tw2_f;
  pc_forward_pair<R, LOG2N, BB, TT>(
      wi.y, gp(v), in_solve ? gp(d.st->vscale + jv) : nullptr,
      in_solve ? gp(&d.st->sum.done) : nullptr, gp(pl.lo), gp(pl.di), gp(pl.up), gp(pl.wfw),
      gp(tw2), gp((const Cx<double>*)pl.mu), gp((const Cx<double>*)pl.il2),
      gp((Cx<R>*)pl.spec), gp((Cx<R>*)pl.iface), pl.nx, pitch > 0 ? pitch : d.ldx, pl.P);
}

// ---------------------------------------------------------------------------
// K3
// ---------------------------------------------------------------------------
// Workgroup hf of the SPL that serve tile p inverts the tile's sequences
// [hf NSEQ/SPL, (hf+1) NSEQ/SPL) (columns [hf B/SPL, (hf+1) B/SPL)); each
// forms the interface correction of the whole tile (it couples all B
// columns) and applies it to its own sequences.
template <typename R, int LOG2N, int BB, int TT, typename TZ, int SPL>
__device__ __forceinline__ void pc_inverse_tile(
    int p, int hf, const CN_G int* stop, const CN_G Cx<R>* __restrict__ spec,
    const CN_G Cx<R>* __restrict__ sep, const CN_G double* __restrict__ lo,
    const CN_G double* __restrict__ di, const CN_G double* __restrict__ up,
    const CN_G double* __restrict__ winv, const Cx<R>* __restrict__ tw,
    const CN_G Cx<double>* __restrict__ mu, CN_G TZ* __restrict__ z, int nx, int zp, int P,
    int NS) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;          // the tile (interface correction)
  using CfgF = PcCfg<R, LOG2N, BB / SPL, TT>;   // the part this workgroup inverts
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  constexpr int BF = CfgF::B, NSF = CfgF::NSEQ;
  __shared__ Cx<R> lds[CfgF::LDS_ELEMS];
  __shared__ Cx<R> ltw[CfgF::TWN];
  __shared__ R co[3 * B];
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  const CN_G Cx<R>* img = spec + ((size_t)p * NSEQ + (size_t)hf * NSF) * N;
  constexpr int NTK = Cfg::NTK;
  const Cx<R> zero{R(0), R(0)};
  Cx<R> slv[NTK], srv[NTK];
  Cx<double> tmd[NTK];
  // the stop flag first, as a uniform scalar load; then every vector load of
  // the phase is issued before any is consumed (see K1)
  const int stopped = stop != nullptr ? *stop : 0;
  // inverse weights alpha^{-k/N_t}/N_t of the thread's levels k = tid/BF +
  // q T/BF by recurrence, as in K1: w_q = w_0 rho^q, rho = alpha^{-(T/BF)/N_t}
  static_assert(T % BF == 0, "the workgroup size must be a multiple of the part width");
  double w = winv[min(tid / BF, N - 1)];
  const double rho = winv[T / BF < N ? T / BF : 0] * (double)N;
  {
    constexpr int SPT = (NSF * N + T - 1) / T;
    Cx<R> iv[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSF * N) % T == 0 || e < NSF * N) iv[q] = gld(img + e);
    }
    // the separator values of the thread's frequencies and their shifts are
    // requested with the image (task u: t = tid + u T; t = 0 solves the real
    // modes 0 and N/2, held as (.x, .y)); indices are clamped to the
    // separator array (at least one entry per line) and masked where the
    // tile has no such separator
    // Every thread loads its line and line N/2 (the same address across the
    // workgroup) and selects: a load whose value is assembled under the
    // lane-dependent t == 0 branch made the compiler wait there for every
    // load in flight, the tile image included.
    const int sli = max(p - 1, 0), sri = min(p, max(NS - 1, 0));
    const int h = N >= 2 ? N / 2 : 0;
    const size_t hr = (size_t)h * NS;
#pragma unroll
    for (int u = 0; u < NTK; ++u) {
      const int t = tid + u * T;
      const int tt = (Cfg::TASKS % T == 0 || t < Cfg::TASKS) ? t : 0;
      const Cx<R> la = gld(sep + (size_t)tt * NS + sli), lb = gld(sep + hr + sli);
      const Cx<R> ra = gld(sep + (size_t)tt * NS + sri), rb = gld(sep + hr + sri);
      const Cx<double> ma = gld(mu + tt), mb = gld(mu + h);
      const bool real = t == 0;
      slv[u] = real ? Cx<R>{la.x, lb.x} : la;
      srv[u] = real ? Cx<R>{ra.x, rb.x} : ra;
      tmd[u] = real ? Cx<double>{ma.x, mb.x} : ma;
    }
    TwStage<R, CfgF::TWN, T, CfgF::TWPT> tws;
    if constexpr (CfgF::TWL) tws.fetch(gp(tw));
    double cov = 0.0;
    if (tid < 3 * B) {
      const int b = min(tid / 3, ncols - 1), c = tid % 3;
      cov = c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]);
    }
    if (stopped) return;  // a stopped cycle's loads are simply dropped
    if (tid < 3 * B) co[tid] = tid / 3 < ncols ? (R)cov : R(0);
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSF * N) % T == 0 || e < NSF * N) lds[lidx<N>(e / N, e % N)] = iv[q];
    }
    if constexpr (CfgF::TWL) tws.store(ltw);
  }
  __syncthreads();
  const bool has_sep = p < P - 1;
  const bool has_left = p > 0;
  const int nb = has_sep ? B - 1 : ncols;
#pragma unroll
  for (int u = 0; u < NTK; ++u) {
    const int t = tid + u * T;
    if (Cfg::TASKS % T != 0 && t >= Cfg::TASKS) break;
    if (t == 0) {
      const int nreal = N >= 2 ? 2 : 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nreal) break;
        const int j = h == 0 ? 0 : N / 2;
        const R m = (R)(h == 0 ? tmd[u].x : tmd[u].y);
        const R sl = has_left ? (h == 0 ? slv[u].x : slv[u].y) : R(0);
        const R sr = has_sep ? (h == 0 ? srv[u].x : srv[u].y) : R(0);
        R d[B];
#pragma unroll
        for (int b = 0; b < B; ++b) d[b] = R(0);
        d[0] = co[0] * sl;
#pragma unroll
        for (int b = 0; b < B; ++b)
          if (b == nb - 1) d[b] = d[b] + co[3 * b + 2] * sr;
        tile_solve<R, R, B>(d, m, co, nb);
        // sequence c of the tile (columns 2c, 2c+1) is local sequence c - hf NSF
        // (the loop runs over the whole tile, so d is indexed by constants)
#pragma unroll
        for (int c = 0; c < NSEQ; ++c) {
          if (c / NSF != hf) continue;
          const int cl = c - hf * NSF;
          const Cx<R> yv = lds[lidx<N>(cl, j)];
          R xa = yv.x + d[2 * c], xb = yv.y + d[2 * c + 1];
          if (2 * c >= nb) xa = (2 * c == B - 1 && has_sep) ? sr : R(0);
          if (2 * c + 1 >= nb) xb = (2 * c + 1 == B - 1 && has_sep) ? sr : R(0);
          lds[lidx<N>(cl, j)] = Cx<R>{xa, xb};
        }
      }
    } else {
      const int j = t;
      const Cx<R> m{(R)tmd[u].x, (R)tmd[u].y};
      const Cx<R> sl = has_left ? slv[u] : zero, sr = has_sep ? srv[u] : zero;
      Cx<R> d[B];
#pragma unroll
      for (int b = 0; b < B; ++b) d[b] = zero;
      d[0] = co[0] * sl;
#pragma unroll
      for (int b = 0; b < B; ++b)
        if (b == nb - 1) d[b] = d[b] + co[3 * b + 2] * sr;
      tile_solve<R, Cx<R>, B>(d, m, co, nb);
#pragma unroll
      for (int c = 0; c < NSEQ; ++c) {
        if (c / NSF != hf) continue;
        const int cl = c - hf * NSF;
        Cx<R> xa = lds[lidx<N>(cl, j)] + d[2 * c];
        Cx<R> xb = lds[lidx<N>(cl, N - j)] + d[2 * c + 1];
        if (2 * c >= nb) xa = (2 * c == B - 1 && has_sep) ? sr : zero;
        if (2 * c + 1 >= nb) xb = (2 * c + 1 == B - 1 && has_sep) ? sr : zero;
        // Z'_j = X_{2c} + i X_{2c+1}; Z'_{N-j} = conj(X_{2c}) + i conj(X_{2c+1})
        lds[lidx<N>(cl, j)] = Cx<R>{xa.x - xb.y, xa.y + xb.x};
        lds[lidx<N>(cl, N - j)] = Cx<R>{xa.x + xb.y, xb.x - xa.y};
      }
    }
  }
  __syncthreads();
  fft_tile<CfgF, R, LOG2N, true>(lds, ltw, tw, threadIdx.x);
  const R* ldsr = reinterpret_cast<const R*>(lds);
  {
    constexpr int LPT = (N * BF + T - 1) / T;
    const int c0 = hf * BF;  // first column of the part within the tile
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      const int k = e / BF, b = e % BF;
      const double wq = w;
      w *= rho;
      if (((N * BF) % T == 0 || e < N * BF) && c0 + b < ncols) {
        const double val = (double)ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] * wq;
        // zp > 0: row-major with pitch zp; 0: tile-blocked (the tile's B x N_t
        // block is contiguous: element (k, c) at (p N_t + k) B + c; the SPL
        // parts of a tile fill the rows of one block, and the Krylov kernels
        // read blocks of the full tile width much faster than narrower ones)
        const size_t zi = zp > 0 ? (size_t)k * zp + i0 + c0 + b
                                 : ((size_t)p * N + k) * B + c0 + b;
        z[zi] = (TZ)val;
      }
    }
  }
}

// z_ovr: output vector instead of Z_j; pitch: its row pitch (row-major), or 0
// for the tile-blocked layout of Z.  SPL workgroups per tile item: nitems
// counts tiles, the grid covers SPL nitems parts (the parts of one tile are
// consecutive, so they share an XCD).
template <typename R, int LOG2N, int BB, int TT, typename TZ, int SPL>
__global__ __launch_bounds__(TT) void k_pc_inverse(const InstDesc* __restrict__ D,
                                                   const int2* __restrict__ items, int nitems,
                                                   int nitems_pad, int jv, TZ* __restrict__ z_ovr,
                                                   int pitch) {
  const int itx = xcd_tile(blockIdx.x, nitems_pad);
  if (itx >= nitems * SPL) return;
  const int2 wi = work_item(items, itx / SPL);
  const int hf = itx % SPL;
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  TZ* z = z_ovr != nullptr ? z_ovr : (TZ*)d.Z + (size_t)jv * d.vstride;
  using CfgF = PcCfg<R, LOG2N, BB / SPL, TT>;
  const Cx<R>* tw = CfgF::TWMODE == 3
                        ? (std::is_same<R, double>::value ? (const Cx<R>*)pl.tw2 : (const Cx<R>*)pl.tw2_f)
                        : (std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f);
  pc_inverse_tile<R, LOG2N, BB, TT, TZ, SPL>(wi.y, hf, z_ovr == nullptr ? gp(&d.st->sum.done) : nullptr,
                                        gp((const Cx<R>*)pl.spec), gp((const Cx<R>*)pl.sep),
                                        gp(pl.lo), gp(pl.di), gp(pl.up), gp(pl.winv), tw,
                                        gp((const Cx<double>*)pl.mu), gp(z), pl.nx,
                                        pitch > 0 ? pitch : (z_ovr == nullptr && d.zlog < 0 ? d.ldx : 0),
                                        pl.P, pl.NS);
}

// ---------------------------------------------------------------------------
// K3 by frequency parity (float32, half the LDS; reads the image of the
// parity K1)
// ---------------------------------------------------------------------------
// With a and b the length-N/2 inverse transforms of the corrected even and
// odd frequencies, x_k = a_k + w_N^{-k} b_k and x_{k+N/2} = a_k - w_N^{-k} b_k.
// The odd half of the image waits in registers while the even half is
// corrected and transformed, then a waits in registers while the odd half
// is; the interface correction of each frequency is formed once.
template <typename R, int LOG2N, int BB, int TT, typename TZ>
__device__ __forceinline__ void pc_inverse_pair(
    int p, const CN_G int* stop, const CN_G Cx<R>* __restrict__ spec,
    const CN_G Cx<R>* __restrict__ sep, const CN_G double* __restrict__ lo,
    const CN_G double* __restrict__ di, const CN_G double* __restrict__ up,
    const CN_G double* __restrict__ winv, const CN_G Cx<R>* __restrict__ tw2,
    const CN_G Cx<double>* __restrict__ mu, CN_G TZ* __restrict__ z, int nx, int zp, int P,
    int NS) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  using CfgH = PcCfg<R, LOG2N - 1, BB, TT>;
  constexpr int N = Cfg::N, NH = N / 2, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  constexpr int TWN = Split2<N>::SIZE;
  constexpr int EH = NSEQ * NH;  // complex entries of one half
  constexpr int EPT = EH / T;
  static_assert(EH % T == 0 && T % NSEQ == 0, "a half must spread evenly over the workgroup");
  constexpr int TASKS = N / 4;  // per parity
  constexpr int NTK = (TASKS + T - 1) / T;
  __shared__ Cx<R> lds[CfgH::LDS_ELEMS];
  __shared__ Cx<R> ltw[TWN];
  __shared__ R co[3 * B];
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  const CN_G Cx<R>* img = spec + (size_t)p * NSEQ * N;
  const int sli = max(p - 1, 0), sri = min(p, max(NS - 1, 0));
  const bool has_sep = p < P - 1;
  const bool has_left = p > 0;
  const int nb = has_sep ? B - 1 : ncols;
  const Cx<R> zero{R(0), R(0)};
  Cx<R> hold[EPT];  // the odd half of the image, later a
  {
    // element e of a half: sequence e / NH, position e mod NH (coalesced)
    const int stopped = stop != nullptr ? *stop : 0;
    Cx<R> ev[EPT];
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * T;
      const CN_G Cx<R>* g = img + (size_t)(e / NH) * N + e % NH;
      ev[q] = gld(g);
      hold[q] = gld(g + NH);
    }
    TwStage<R, TWN, T, (TWN + T - 1) / T> tws;
    tws.fetch(tw2);
    double cov = 0.0;
    if (tid < 3 * B) {
      const int b = min(tid / 3, ncols - 1), c = tid % 3;
      cov = c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]);
    }
    if (stopped) return;  // a stopped cycle's loads are simply dropped
    if (tid < 3 * B) co[tid] = tid / 3 < ncols ? (R)cov : R(0);
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * T;
      lds[lidx<NH>(e / NH, e % NH)] = ev[q];
    }
    tws.store(ltw);
  }
  __syncthreads();
#pragma unroll 1
  for (int hf = 0; hf < 2; ++hf) {
    const bool odd = hf != 0;
    const int tid2 = phase_tid<T>();
    // separator values and shifts of this parity's frequencies (task t:
    // j = 2t + hf; the even task 0 takes the real modes 0 and N/2, held as
    // (.x, .y)); every thread loads and selects, as in K3
    Cx<R> slv[NTK], srv[NTK];
    Cx<double> tmd[NTK];
    const size_t hr = (size_t)NH * NS;
#pragma unroll
    for (int u = 0; u < NTK; ++u) {
      const int t = tid2 + u * T;
      const int tt = (TASKS % T == 0 || t < TASKS) ? t : 0;
      const size_t jr = (size_t)(2 * tt + hf) * NS;
      const Cx<R> la = gld(sep + jr + sli), lb = gld(sep + hr + sli);
      const Cx<R> ra = gld(sep + jr + sri), rb = gld(sep + hr + sri);
      const Cx<double> ma = gld(mu + 2 * tt + hf), mb = gld(mu + NH);
      const bool real = !odd && t == 0;
      slv[u] = real ? Cx<R>{la.x, lb.x} : la;
      srv[u] = real ? Cx<R>{ra.x, rb.x} : ra;
      tmd[u] = real ? Cx<double>{ma.x, mb.x} : ma;
    }
#pragma unroll
    for (int u = 0; u < NTK; ++u) {
      const int t = tid2 + u * T;
      if (TASKS % T != 0 && t >= TASKS) break;
      if (!odd && t == 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int pos = h == 0 ? 0 : NH / 2;
          const R m = (R)(h == 0 ? tmd[u].x : tmd[u].y);
          const R sl = has_left ? (h == 0 ? slv[u].x : slv[u].y) : R(0);
          const R sr = has_sep ? (h == 0 ? srv[u].x : srv[u].y) : R(0);
          R d[B];
#pragma unroll
          for (int b = 0; b < B; ++b) d[b] = R(0);
          d[0] = co[0] * sl;
#pragma unroll
          for (int b = 0; b < B; ++b)
            if (b == nb - 1) d[b] = d[b] + co[3 * b + 2] * sr;
          tile_solve<R, R, B>(d, m, co, nb);
#pragma unroll
          for (int c = 0; c < NSEQ; ++c) {
            const Cx<R> yv = lds[lidx<NH>(c, pos)];
            R xa = yv.x + d[2 * c], xb = yv.y + d[2 * c + 1];
            if (2 * c >= nb) xa = (2 * c == B - 1 && has_sep) ? sr : R(0);
            if (2 * c + 1 >= nb) xb = (2 * c + 1 == B - 1 && has_sep) ? sr : R(0);
            lds[lidx<NH>(c, pos)] = Cx<R>{xa, xb};
          }
        }
      } else {
        const int pa = t, pb = NH - hf - t;
        const Cx<R> m{(R)tmd[u].x, (R)tmd[u].y};
        const Cx<R> sl = has_left ? slv[u] : zero, sr = has_sep ? srv[u] : zero;
        Cx<R> d[B];
#pragma unroll
        for (int b = 0; b < B; ++b) d[b] = zero;
        d[0] = co[0] * sl;
#pragma unroll
        for (int b = 0; b < B; ++b)
          if (b == nb - 1) d[b] = d[b] + co[3 * b + 2] * sr;
        tile_solve<R, Cx<R>, B>(d, m, co, nb);
#pragma unroll
        for (int c = 0; c < NSEQ; ++c) {
          Cx<R> xa = lds[lidx<NH>(c, pa)] + d[2 * c];
          Cx<R> xb = lds[lidx<NH>(c, pb)] + d[2 * c + 1];
          if (2 * c >= nb) xa = (2 * c == B - 1 && has_sep) ? sr : zero;
          if (2 * c + 1 >= nb) xb = (2 * c + 1 == B - 1 && has_sep) ? sr : zero;
          lds[lidx<NH>(c, pa)] = Cx<R>{xa.x - xb.y, xa.y + xb.x};
          lds[lidx<NH>(c, pb)] = Cx<R>{xa.x + xb.y, xb.x - xa.y};
        }
      }
    }
    __syncthreads();
    fft_run<R, LOG2N - 1, NSEQ, T, true, CfgH::MAXLOG, 0>(lds, TwTab2Half<R, N>{ltw},
                                                         phase_tid<T>());
    if (!odd) {
      // a, in the store's order (sequence fastest), to registers; then the
      // odd half of the image into LDS
      const int tid3 = phase_tid<T>();
      Cx<R> av[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid3 + q * T;
        av[q] = lds[lidx<NH>(e % NSEQ, e / NSEQ)];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int e = tid3 + q * T;
        lds[lidx<NH>(e / NH, e % NH)] = hold[q];
        hold[q] = av[q];
      }
      __syncthreads();
    }
  }
  // x_k = a_k + w^{-k} b_k, x_{k+N/2} = a_k - w^{-k} b_k, times
  // alpha^{-k/N_t}/N_t (by recurrence over the thread's levels k = tid/NSEQ +
  // q T/NSEQ, as in K3); columns 2c, 2c+1 of rows k and k + N/2
  {
    const int tid4 = phase_tid<T>();
    double w = winv[tid4 / NSEQ];
    const double rho = winv[T / NSEQ] * (double)N;
    const double wh = winv[NH] * (double)N;
    const TwTab2<R, N> twf{ltw};
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid4 + q * T;
      const int c = e % NSEQ, k = e / NSEQ;
      const Cx<R> bq = lds[lidx<NH>(c, k)];
      const Cx<R> wk = conj(twf(k));
      const Cx<R> tq = wk * bq;
      const Cx<R> xl = hold[q] + tq, xh = hold[q] - tq;
      const double wl = w, whi = w * wh;
      w *= rho;
      if (zp == 0 && 2 * c + 1 < ncols) {
        // tile-blocked: columns 2c, 2c+1 are adjacent (even offset), one
        // vector store per row
        typedef TZ tz2 __attribute__((ext_vector_type(2)));
        tz2 vl, vh;
        vl.x = (TZ)((double)xl.x * wl);
        vl.y = (TZ)((double)xl.y * wl);
        vh.x = (TZ)((double)xh.x * whi);
        vh.y = (TZ)((double)xh.y * whi);
        *(CN_G tz2*)(z + ((size_t)p * N + k) * B + 2 * c) = vl;
        *(CN_G tz2*)(z + ((size_t)p * N + k + NH) * B + 2 * c) = vh;
      } else {
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2) {
          const int col = 2 * c + s2;
          if (col < ncols) {
            const double vl = (double)(s2 == 0 ? xl.x : xl.y) * wl;
            const double vh = (double)(s2 == 0 ? xh.x : xh.y) * whi;
            const size_t zl = zp > 0 ? (size_t)k * zp + i0 + col : ((size_t)p * N + k) * B + col;
            const size_t zh = zp > 0 ? (size_t)(k + NH) * zp + i0 + col
                                     : ((size_t)p * N + k + NH) * B + col;
            z[zl] = (TZ)vl;
            z[zh] = (TZ)vh;
          }
        }
      }
    }
  }
}

template <typename R, int LOG2N, int BB, int TT, typename TZ>
__global__ __launch_bounds__(TT) __attribute__((amdgpu_waves_per_eu(4)))
void k_pc_inverse_pair(const InstDesc* __restrict__ D, const int2* __restrict__ items, int nitems,
                       int nitems_pad, int jv, TZ* __restrict__ z_ovr, int pitch) {
  const int itx = xcd_tile(blockIdx.x, nitems_pad);
  if (itx >= nitems) return;
  const int2 wi = work_item(items, itx);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  TZ* z = z_ovr != nullptr ? z_ovr : (TZ*)d.Z + (size_t)jv * d.vstride;
  const Cx<R>* tw2 = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw2 : (const Cx<R>*)pl.tw2_f;
  pc_inverse_pair<R, LOG2N, BB, TT, TZ>(
      wi.y, z_ovr == nullptr ? gp(&d.st->sum.done) : nullptr, gp((const Cx<R>*)pl.spec),
      gp((const Cx<R>*)pl.sep), gp(pl.lo), gp(pl.di), gp(pl.up), gp(pl.winv), gp(tw2),
      gp((const Cx<double>*)pl.mu), gp(z), pl.nx,
      pitch > 0 ? pitch : (z_ovr == nullptr && d.zlog < 0 ? d.ldx : 0), pl.P, pl.NS);
}

// ---------------------------------------------------------------------------
// launch one compiled (B, T) candidate; dispatch over candidates and log2(N_t)
// ---------------------------------------------------------------------------
static inline int pad8(int v) { return (v + 7) / 8 * 8; }

template <typename R, int L, int CI>
static hipError_t launch_fwd_c(const Launch& Lc, const Items& it, int j, const double* v,
                               int pitch, hipStream_t s) {
  using C = PcCand<R, L, CI>;
  if constexpr (!C::ok) {
    return hipErrorInvalidValue;
  } else {
    if (it.n <= 0) return hipSuccess;
    if constexpr (C::F == 2) {
      const int nwg = pad8(it.n);
      hipLaunchKernelGGL((k_pc_forward_pair<R, L, C::B, C::T>), dim3(nwg), dim3(C::T), 0, s, Lc.D,
                         it.it, it.n, nwg, j, v, pitch);
    } else {
      const int nwg = pad8(it.n);
      hipLaunchKernelGGL((k_pc_forward<R, L, C::B, C::T>), dim3(nwg), dim3(C::T), 0, s, Lc.D,
                         it.it, it.n, nwg, j, v, pitch);
    }
    return hipGetLastError();
  }
}

template <typename R, int L, int CI>
static hipError_t launch_inv_c(const Launch& Lc, const Items& it, int j, void* z, int zf,
                               int pitch, hipStream_t s) {
  using C = PcCand<R, L, CI>;
  if constexpr (!C::ok) {
    return hipErrorInvalidValue;
  } else {
    if (it.n <= 0) return hipSuccess;
    if constexpr (C::F == 2) {
      const int nwg = pad8(it.n);
      if (zf)
        hipLaunchKernelGGL((k_pc_inverse_pair<R, L, C::B, C::T, float>), dim3(nwg), dim3(C::T), 0,
                           s, Lc.D, it.it, it.n, nwg, j, (float*)z, pitch);
      else
        hipLaunchKernelGGL((k_pc_inverse_pair<R, L, C::B, C::T, double>), dim3(nwg), dim3(C::T),
                           0, s, Lc.D, it.it, it.n, nwg, j, (double*)z, pitch);
      return hipGetLastError();
    }
    const int nwg = pad8(it.n * C::S);
    if (zf)
      hipLaunchKernelGGL((k_pc_inverse<R, L, C::B, C::T, float, C::S>), dim3(nwg), dim3(C::T), 0,
                         s, Lc.D, it.it, it.n, nwg, j, (float*)z, pitch);
    else
      hipLaunchKernelGGL((k_pc_inverse<R, L, C::B, C::T, double, C::S>), dim3(nwg), dim3(C::T), 0,
                         s, Lc.D, it.it, it.n, nwg, j, (double*)z, pitch);
    return hipGetLastError();
  }
}

template <typename R, int L, int CI = 0>
static hipError_t fwd_cand(int ci, const Launch& Lc, const Items& it, int j, const double* v,
                           int pitch, hipStream_t s) {
  if constexpr (CI >= kNumCand) {
    return hipErrorInvalidValue;
  } else {
    if (ci == CI) return launch_fwd_c<R, L, CI>(Lc, it, j, v, pitch, s);
    return fwd_cand<R, L, CI + 1>(ci, Lc, it, j, v, pitch, s);
  }
}

template <typename R, int L, int CI = 0>
static hipError_t inv_cand(int ci, const Launch& Lc, const Items& it, int j, void* z, int zf,
                           int pitch, hipStream_t s) {
  if constexpr (CI >= kNumCand) {
    return hipErrorInvalidValue;
  } else {
    if (ci == CI) return launch_inv_c<R, L, CI>(Lc, it, j, z, zf, pitch, s);
    return inv_cand<R, L, CI + 1>(ci, Lc, it, j, z, zf, pitch, s);
  }
}

template <typename R, int L, int CI = 0>
static bool cand_info(int ci, int* B, int* T, int* S, int* FS) {
  if constexpr (CI >= kNumCand) {
    return false;
  } else {
    if (ci == CI) {
      *B = PcCand<R, L, CI>::B;
      *T = PcCand<R, L, CI>::T;
      *S = PcCand<R, L, CI>::S;
      *FS = PcCand<R, L, CI>::F;
      return PcCand<R, L, CI>::ok;
    }
    return cand_info<R, L, CI + 1>(ci, B, T, S, FS);
  }
}

#define CN_LOG2N_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13)

#define CN_DEFINE_PC_PRECISION(R, SUF)                                                        \
  hipError_t pc_forward_##SUF(int log2n, int cand, const Launch& Lc, const Items& it, int j,  \
                              const double* v, int pitch, hipStream_t s) {                    \
    switch (log2n) {                                                                          \
      CN_LOG2N_CASES(CN_FWD_CASE_##SUF)                                                       \
    }                                                                                         \
    return hipErrorInvalidValue;                                                              \
  }                                                                                           \
  hipError_t pc_inverse_##SUF(int log2n, int cand, const Launch& Lc, const Items& it, int j,  \
                              void* z, int zf, int pitch, hipStream_t s) {                    \
    switch (log2n) {                                                                          \
      CN_LOG2N_CASES(CN_INV_CASE_##SUF)                                                       \
    }                                                                                         \
    return hipErrorInvalidValue;                                                              \
  }                                                                                           \
  bool pc_candidate_##SUF(int log2n, int ci, int* B, int* T, int* S, int* FS) {               \
    switch (log2n) {                                                                          \
      CN_LOG2N_CASES(CN_INFO_CASE_##SUF)                                                      \
    }                                                                                         \
    return false;                                                                             \
  }

}  // namespace cn
