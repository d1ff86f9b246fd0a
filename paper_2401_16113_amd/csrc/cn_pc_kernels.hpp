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
    int p, const CN_G double* __restrict__ v, const double* scp, const int* stop,
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
  // sequence.  All of a thread's loads (tile, then twiddles) are issued
  // before any is consumed.
  R* ldsr = reinterpret_cast<R*>(lds);
  {
    constexpr int LPT = (N * B + T - 1) / T;
    double xv[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      const int k = e / B, b = e % B;
      xv[q] = ((N * B) % T == 0 || e < N * B) && b < ncols ? v[(size_t)k * vp + i0 + b] : 0.0;
    }
    // the stop flag and the basis scale are read with the tile in flight
    // (a stopped cycle's loads are simply dropped)
    if (stop != nullptr && *stop) return;
    const double sc = scp != nullptr ? *scp : 1.0;
    TwStage<R, Cfg::TWN, T, Cfg::TWPT> tws;
    if constexpr (Cfg::TWL) tws.fetch(gp(tw));
    if (tid < 3 * B) {
      const int b = tid / 3, c = tid % 3;
      R val = R(0);
      if (b < ncols) val = (R)(c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]));
      co[tid] = val;
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      if ((N * B) % T == 0 || e < N * B) {
        const int k = e / B, b = e % B;
        ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] = (R)(xv[q] * (wfw[k] * sc));
      }
    }
    if constexpr (Cfg::TWL) tws.store(ltw);
  }
  __syncthreads();
  fft_tile<Cfg, R, LOG2N, false>(lds, ltw, tw, threadIdx.x);

  // step (b), tile-local part.  Per frequency the tile leaves two partial
  // right-hand sides of the separator systems: d + lo y_last for its own
  // separator (its last column) and up y_first for the separator left of it.
  const bool has_sep = p < P - 1;
  const int nb = has_sep ? B - 1 : ncols;
  const R lsep = has_sep ? co[3 * (B - 1)] : R(0);
  const R uprev = p > 0 ? (R)up[i0 - 1] : R(0);
  CN_G Cx<R>* ifc = iface + (size_t)p * 2;
  for (int t = tid; t < Cfg::TASKS; t += T) {
    if (t == 0) {
      // j = 0 and j = N/2: real modes, real shifts
      const int nreal = N >= 2 ? 2 : 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nreal) break;
        const int j = h == 0 ? 0 : N / 2;
        const R m = (R)mu[j].x, s2 = (R)il2[j].x;
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
      const Cx<double> md = gld(mu + j), sd = gld(il2 + j);
      const Cx<R> m{(R)md.x, (R)md.y}, s2{(R)sd.x, (R)sd.y};
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
  const Cx<R>* tw = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f;
  pc_forward_tile<R, LOG2N, BB, TT>(wi.y, gp(v), in_solve ? d.st->vscale + jv : nullptr,
                                    in_solve ? &d.st->sum.done : nullptr, gp(pl.lo), gp(pl.di),
                                    gp(pl.up), gp(pl.wfw), tw, gp((const Cx<double>*)pl.mu),
                                    gp((const Cx<double>*)pl.il2), gp((Cx<R>*)pl.spec),
                                    gp((Cx<R>*)pl.iface), pl.nx, pitch > 0 ? pitch : d.ldx, pl.P);
}

// ---------------------------------------------------------------------------
// K3
// ---------------------------------------------------------------------------
template <typename R, int LOG2N, int BB, int TT, typename TZ>
__device__ __forceinline__ void pc_inverse_tile(
    int p, const int* stop, const CN_G Cx<R>* __restrict__ spec,
    const CN_G Cx<R>* __restrict__ sep, const CN_G double* __restrict__ lo,
    const CN_G double* __restrict__ di, const CN_G double* __restrict__ up,
    const CN_G double* __restrict__ winv, const Cx<R>* __restrict__ tw,
    const CN_G Cx<double>* __restrict__ mu, CN_G TZ* __restrict__ z, int nx, int zp, int P,
    int NS) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  __shared__ Cx<R> lds[Cfg::LDS_ELEMS];
  __shared__ Cx<R> ltw[Cfg::TWN];
  __shared__ R co[3 * B];
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  const CN_G Cx<R>* img = spec + (size_t)p * NSEQ * N;
  {
    constexpr int SPT = (NSEQ * N + T - 1) / T;
    Cx<R> iv[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSEQ * N) % T == 0 || e < NSEQ * N) iv[q] = gld(img + e);
    }
    if (stop != nullptr && *stop) return;  // read with the image in flight
    TwStage<R, Cfg::TWN, T, Cfg::TWPT> tws;
    if constexpr (Cfg::TWL) tws.fetch(gp(tw));
    if (tid < 3 * B) {
      const int b = tid / 3, c = tid % 3;
      R val = R(0);
      if (b < ncols) val = (R)(c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]));
      co[tid] = val;
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSEQ * N) % T == 0 || e < NSEQ * N) lds[lidx<N>(e / N, e % N)] = iv[q];
    }
    if constexpr (Cfg::TWL) tws.store(ltw);
  }
  __syncthreads();
  const bool has_sep = p < P - 1;
  const bool has_left = p > 0;
  const int nb = has_sep ? B - 1 : ncols;
  for (int t = tid; t < Cfg::TASKS; t += T) {
    if (t == 0) {
      const int nreal = N >= 2 ? 2 : 1;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (h >= nreal) break;
        const int j = h == 0 ? 0 : N / 2;
        const R m = (R)mu[j].x;
        const R sl = has_left ? sep[(size_t)j * NS + p - 1].x : R(0);
        const R sr = has_sep ? sep[(size_t)j * NS + p].x : R(0);
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
          const Cx<R> yv = lds[lidx<N>(c, j)];
          R xa = yv.x + d[2 * c], xb = yv.y + d[2 * c + 1];
          if (2 * c >= nb) xa = (2 * c == B - 1 && has_sep) ? sr : R(0);
          if (2 * c + 1 >= nb) xb = (2 * c + 1 == B - 1 && has_sep) ? sr : R(0);
          lds[lidx<N>(c, j)] = Cx<R>{xa, xb};
        }
      }
    } else {
      const int j = t;
      const Cx<double> md = gld(mu + j);
      const Cx<R> m{(R)md.x, (R)md.y};
      const Cx<R> zero{R(0), R(0)};
      const Cx<R> sl = has_left ? gld(sep + (size_t)j * NS + p - 1) : zero;
      const Cx<R> sr = has_sep ? gld(sep + (size_t)j * NS + p) : zero;
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
        Cx<R> xa = lds[lidx<N>(c, j)] + d[2 * c];
        Cx<R> xb = lds[lidx<N>(c, N - j)] + d[2 * c + 1];
        if (2 * c >= nb) xa = (2 * c == B - 1 && has_sep) ? sr : zero;
        if (2 * c + 1 >= nb) xb = (2 * c + 1 == B - 1 && has_sep) ? sr : zero;
        // Z'_j = X_{2c} + i X_{2c+1}; Z'_{N-j} = conj(X_{2c}) + i conj(X_{2c+1})
        lds[lidx<N>(c, j)] = Cx<R>{xa.x - xb.y, xa.y + xb.x};
        lds[lidx<N>(c, N - j)] = Cx<R>{xa.x + xb.y, xb.x - xa.y};
      }
    }
  }
  __syncthreads();
  fft_tile<Cfg, R, LOG2N, true>(lds, ltw, tw, threadIdx.x);
  const R* ldsr = reinterpret_cast<const R*>(lds);
  {
    constexpr int LPT = (N * B + T - 1) / T;
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      const int k = e / B, b = e % B;
      if (((N * B) % T == 0 || e < N * B) && b < ncols) {
        const double val = (double)ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] * winv[k];
        z[(size_t)k * zp + i0 + b] = (TZ)val;
      }
    }
  }
}

// z_ovr: output vector instead of Z_j; pitch: its row pitch (0: the internal
// pitch of Z)
template <typename R, int LOG2N, int BB, int TT, typename TZ>
__global__ __launch_bounds__(TT) void k_pc_inverse(const InstDesc* __restrict__ D,
                                                   const int2* __restrict__ items, int nitems,
                                                   int nitems_pad, int jv, TZ* __restrict__ z_ovr,
                                                   int pitch) {
  const int itx = xcd_tile(blockIdx.x, nitems_pad);
  if (itx >= nitems) return;
  const int2 wi = work_item(items, itx);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  TZ* z = z_ovr != nullptr ? z_ovr : (TZ*)d.Z + (size_t)jv * d.vstride;
  const Cx<R>* tw = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f;
  pc_inverse_tile<R, LOG2N, BB, TT, TZ>(wi.y, z_ovr == nullptr ? &d.st->sum.done : nullptr,
                                        gp((const Cx<R>*)pl.spec), gp((const Cx<R>*)pl.sep),
                                        gp(pl.lo), gp(pl.di), gp(pl.up), gp(pl.winv), tw,
                                        gp((const Cx<double>*)pl.mu), gp(z), pl.nx,
                                        pitch > 0 ? pitch : d.ldx, pl.P, pl.NS);
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
    const int nwg = pad8(it.n);
    hipLaunchKernelGGL((k_pc_forward<R, L, C::B, C::T>), dim3(nwg), dim3(C::T), 0, s, Lc.D, it.it,
                       it.n, nwg, j, v, pitch);
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
    const int nwg = pad8(it.n);
    if (zf)
      hipLaunchKernelGGL((k_pc_inverse<R, L, C::B, C::T, float>), dim3(nwg), dim3(C::T), 0, s,
                         Lc.D, it.it, it.n, nwg, j, (float*)z, pitch);
    else
      hipLaunchKernelGGL((k_pc_inverse<R, L, C::B, C::T, double>), dim3(nwg), dim3(C::T), 0, s,
                         Lc.D, it.it, it.n, nwg, j, (double*)z, pitch);
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
static bool cand_info(int ci, int* B, int* T) {
  if constexpr (CI >= kNumCand) {
    return false;
  } else {
    if (ci == CI) {
      *B = PcCand<R, L, CI>::B;
      *T = PcCand<R, L, CI>::T;
      return PcCand<R, L, CI>::ok;
    }
    return cand_info<R, L, CI + 1>(ci, B, T);
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
  bool pc_candidate_##SUF(int log2n, int ci, int* B, int* T) {                                \
    switch (log2n) {                                                                          \
      CN_LOG2N_CASES(CN_INFO_CASE_##SUF)                                                      \
    }                                                                                         \
    return false;                                                                             \
  }

}  // namespace cn
