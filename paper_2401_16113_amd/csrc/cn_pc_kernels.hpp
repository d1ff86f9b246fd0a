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
//     three interface values per (j, tile).
//  K3 (k_pc_inverse): per tile, adds the separator contributions to the local
//     solution, runs the inverse FFT, multiplies by Lambda_alpha^{-1}/N_t
//     (step (c)) and writes z.
//  k_pc_fused: K1, the interface solves and K3 in one launch for an instance
//     whose tiles are all resident at once (one workgroup per tile): the tile
//     image stays in LDS, and two grid-wide barriers order the interface
//     values, the separator solves and their use.
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

  // step (b), tile-local part
  const bool has_sep = p < P - 1;
  const int nb = has_sep ? B - 1 : ncols;
  CN_G Cx<R>* ifc = iface + (size_t)p * 3;
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
        CN_G Cx<R>* f = ifc + (size_t)j * P * 3;
        gst(f, Cx<R>{has_sep ? sepv : R(0), R(0)});
        gst(f + 1, Cx<R>{ylast, R(0)});
        gst(f + 2, Cx<R>{d[0], R(0)});
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
      CN_G Cx<R>* f = ifc + (size_t)j * P * 3;
      gst(f, has_sep ? sepv : Cx<R>{R(0), R(0)});
      gst(f + 1, ylast);
      gst(f + 2, d[0]);
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
// phases of the single-launch apply (K1 and K3 split at the interface solve;
// each phase derives its indices from its own phase_tid, so the long kernel
// does not keep them live across phases)
// ---------------------------------------------------------------------------
// Load the tile with the alpha weights (step (a)), columns (2s, 2s+1) packed as
// one complex sequence, plus the tile's operator rows and the twiddle table.
// All of a thread's loads (tile, then twiddles) are issued before any is
// consumed.  Returns false (uniformly) when the cycle has stopped.
template <typename R, int LOG2N, int BB, int TT>
__device__ __forceinline__ bool fwd_load(int p, const double* __restrict__ v, const double* scp,
                                         const int* stop, const double* __restrict__ lo,
                                         const double* __restrict__ di,
                                         const double* __restrict__ up,
                                         const double* __restrict__ wfw,
                                         const Cx<R>* __restrict__ tw, Cx<R>* __restrict__ lds,
                                         Cx<R>* __restrict__ ltw, R* __restrict__ co, int nx,
                                         int vp) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  constexpr int N = Cfg::N, B = Cfg::B, T = Cfg::T;
  const int tid = phase_tid<T>();
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  R* ldsr = reinterpret_cast<R*>(lds);
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
  if (stop != nullptr && *stop) return false;
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
  __syncthreads();
  return true;
}

// FFT of the loaded tile and the tile-local part of step (b); writes the
// three interface values of every (j, tile) (device-coherently when COH) and
// leaves the tile image in LDS.
template <typename R, int LOG2N, int BB, int TT, bool COH = false>
__device__ __forceinline__ void fwd_solve(int p, Cx<R>* __restrict__ lds,
                                          const Cx<R>* __restrict__ ltw, const R* __restrict__ co,
                                          const Cx<R>* __restrict__ tw,
                                          const Cx<double>* __restrict__ mu,
                                          const Cx<double>* __restrict__ il2, Cx<R>* iface,
                                          int nx, int P) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  const int tid = phase_tid<T>();
  const int ncols = min(B, nx - p * B);
  fft_tile<Cfg, R, LOG2N, false>(lds, ltw, tw, tid);

  const bool has_sep = p < P - 1;
  const int nb = has_sep ? B - 1 : ncols;
  Cx<R>* ifc = iface + (size_t)p * 3;
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
        Cx<R>* f = ifc + (size_t)j * P * 3;
        st_x<COH>(f, Cx<R>{has_sep ? sepv : R(0), R(0)});
        st_x<COH>(f + 1, Cx<R>{ylast, R(0)});
        st_x<COH>(f + 2, Cx<R>{d[0], R(0)});
      }
    } else {
      const int j = t;
      const Cx<double> md = mu[j], sd = il2[j];
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
      Cx<R>* f = ifc + (size_t)j * P * 3;
      st_x<COH>(f, has_sep ? sepv : Cx<R>{R(0), R(0)});
      st_x<COH>(f + 1, ylast);
      st_x<COH>(f + 2, d[0]);
    }
  }
  __syncthreads();
}

// Separator contributions (read device-coherently when COH), inverse FFT,
// Lambda_alpha^{-1}/N_t and the store of z.
template <typename R, int LOG2N, int BB, int TT, typename TZ, bool COH = false>
__device__ __forceinline__ void inv_finish(int p, Cx<R>* __restrict__ lds,
                                           const Cx<R>* __restrict__ ltw, const R* __restrict__ co,
                                           const Cx<R>* sep, const double* __restrict__ winv,
                                           const Cx<R>* __restrict__ tw,
                                           const Cx<double>* __restrict__ mu,
                                           TZ* __restrict__ z, int nx, int zp, int P, int NS) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  const int tid = phase_tid<T>();
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
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
        const R sl = has_left ? ld_x<COH>(sep + (size_t)j * NS + p - 1).x : R(0);
        const R sr = has_sep ? ld_x<COH>(sep + (size_t)j * NS + p).x : R(0);
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
      const Cx<double> md = mu[j];
      const Cx<R> m{(R)md.x, (R)md.y};
      const Cx<R> zero{R(0), R(0)};
      const Cx<R> sl = has_left ? ld_x<COH>(sep + (size_t)j * NS + p - 1) : zero;
      const Cx<R> sr = has_sep ? ld_x<COH>(sep + (size_t)j * NS + p) : zero;
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
  fft_tile<Cfg, R, LOG2N, true>(lds, ltw, tw, phase_tid<T>());
  const R* ldsr = reinterpret_cast<const R*>(lds);
  constexpr int LPT = (N * B + T - 1) / T;
  const int tz = phase_tid<T>();
#pragma unroll
  for (int q = 0; q < LPT; ++q) {
    const int e = tz + q * T;
    const int k = e / B, b = e % B;
    if (((N * B) % T == 0 || e < N * B) && b < ncols) {
      const double val = (double)ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] * winv[k];
      z[(size_t)k * zp + i0 + b] = (TZ)val;
    }
  }
}

// ---------------------------------------------------------------------------
// single-launch apply
// ---------------------------------------------------------------------------
// Grid-wide barrier for a launch whose workgroups are all resident (the host
// checks the occupancy before choosing this kernel).  *cnt counts arrivals
// and is never reset: a workgroup arriving as number `old` waits until the
// count reaches the next multiple of nwg (the host clears the counter when
// the grid size changes).  The data exchanged across the barrier is written
// and read with device-coherent accesses (st_dev / ld_dev), so the barrier
// only orders them: every wave waits for its own stores to complete before
// its workgroup arrives, and the counter accesses are device-scope atomics.
// (A release/acquire pair at device scope would write back or invalidate the
// whole L2 of an XCD once per workgroup.)  The wait is bounded: after
// max_polls polls (~2^22 by default, ~1 s) the workgroup gives up, raises *err
// and the caller abandons the apply, so a launch whose workgroups were not all
// resident still ends (max_polls = 0: every workgroup but the last to arrive
// gives up at once).
__device__ __forceinline__ bool grid_barrier(unsigned long long* cnt, unsigned nwg,
                                             unsigned max_polls, int* err) {
  __shared__ int pass;
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long old =
        __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long target = (old / nwg + 1) * nwg;
    int ok = 1;
    if (old + 1 < target) {
      if (max_polls == 0) {
        ok = 0;
      } else {
        unsigned polls = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          if (++polls > max_polls) {
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    if (!ok) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    pass = ok;
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  return pass != 0;
}

// One workgroup per tile (grid = P, all resident): K1 phases, barrier, the
// F interface lines (one wavefront per line, lines dealt over the grid's
// wavefronts), barrier, K3 phases on the image still in LDS.  Inside a solve
// (v_ovr null) the input is V_j scaled by 1/||v_j|| and the output Z_j; the
// launch returns at entry once the cycle has stopped (a flag no kernel of
// this launch writes, so every workgroup takes the same branch).  v_ovr and
// z_ovr may be the same vector (in-place apply): a tile's input is in LDS
// before any output is written.
template <typename R, int LOG2N, int BB, int TT, typename TZ>
__global__ __launch_bounds__(TT) void k_pc_fused(const InstDesc* __restrict__ D, int jv,
                                                 const double* v_ovr, int vpitch,
                                                 TZ* z_ovr, int zpitch,
                                                 unsigned long long* bar, unsigned max_polls,
                                                 int* err) {
  using Cfg = PcCfg<R, LOG2N, BB, TT>;
  __shared__ __align__(16) Cx<R> lds[Cfg::LDS_ELEMS];
  __shared__ __align__(16) Cx<R> ltw[Cfg::TWN];
  __shared__ __align__(16) R co[3 * BB];
  const InstDesc& d = D[0];
  const PcPlan& pl = d.pl;
  const int p = blockIdx.x;
  const bool in_solve = v_ovr == nullptr;
  const double* v = in_solve ? d.V + (size_t)jv * d.vstride : v_ovr;
  TZ* z = in_solve ? (TZ*)d.Z + (size_t)jv * d.vstride : z_ovr;
  const Cx<R>* tw = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f;
  Cx<R>* iface = (Cx<R>*)pl.iface;
  Cx<R>* sep = (Cx<R>*)pl.sep;
  if (!fwd_load<R, LOG2N, BB, TT>(p, v, in_solve ? d.st->vscale + jv : nullptr,
                                  in_solve ? &d.st->sum.done : nullptr, pl.lo, pl.di, pl.up,
                                  pl.wfw, tw, lds, ltw, co, pl.nx, vpitch > 0 ? vpitch : d.ldx))
    return;
  fwd_solve<R, LOG2N, BB, TT, true>(p, lds, ltw, co, tw, pl.mu, pl.il2, iface, pl.nx, pl.P);
  if (pl.NS > 0) {
    if (!grid_barrier(bar, gridDim.x, max_polls, err)) return;
    constexpr int NW = TT / 64;
    const int t2 = phase_tid<TT>();
    const int wave = t2 >> 6, lane = t2 & 63;
    for (int L = wave * pl.P + p; L < pl.F; L += pl.P * NW) {
      const size_t row = (size_t)L * pl.NS;
      reduced_line<R, 1, 4, true>(iface + (size_t)L * pl.P * 3, sep + row,
                            (const RedRec<R>*)pl.red + row, nullptr, pl.lo, pl.up, pl.NS, BB,
                            lane, nullptr, nullptr);
    }
    if (!grid_barrier(bar, gridDim.x, max_polls, err)) return;
  }
  inv_finish<R, LOG2N, BB, TT, TZ, true>(p, lds, ltw, co, sep, pl.winv, tw, pl.mu, z, pl.nx,
                                         zpitch > 0 ? zpitch : d.ldx, pl.P, pl.NS);
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

// Single-launch apply: compiled for the 16-column candidates (the fewest
// tiles, hence the widest instance whose tiles are all resident).
template <typename R, int L, int CI>
struct FusedCand {
  static constexpr bool ok = PcCand<R, L, CI>::ok && PcCand<R, L, CI>::B == 16;
};

template <typename R, int L, int CI>
static hipError_t launch_fused_c(const Launch& Lc, int P, int j, const double* v, int vpitch,
                                 void* z, int zf, int zpitch, unsigned long long* bar, unsigned polls,
                                 int* err, hipStream_t s) {
  using C = PcCand<R, L, CI>;
  if constexpr (!FusedCand<R, L, CI>::ok) {
    return hipErrorInvalidValue;
  } else {
    if (P <= 0) return hipSuccess;
    if (zf) {
      if constexpr (std::is_same<R, float>::value)
        hipLaunchKernelGGL((k_pc_fused<R, L, C::B, C::T, float>), dim3(P), dim3(C::T), 0, s, Lc.D,
                           j, v, vpitch, (float*)z, zpitch, bar, polls, err);
      else
        return hipErrorInvalidValue;
    } else {
      hipLaunchKernelGGL((k_pc_fused<R, L, C::B, C::T, double>), dim3(P), dim3(C::T), 0, s, Lc.D,
                         j, v, vpitch, (double*)z, zpitch, bar, polls, err);
    }
    return hipGetLastError();
  }
}

// Workgroups of the single-launch kernel the device holds at once (0: not
// compiled for this candidate).
template <typename R, int L, int CI>
static int fused_capacity_c(int zf) {
  using C = PcCand<R, L, CI>;
  if constexpr (!FusedCand<R, L, CI>::ok) {
    return 0;
  } else {
    int per_cu = 0;
    hipError_t e = hipSuccess;
    if constexpr (std::is_same<R, float>::value) {
      if (zf)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_pc_fused<R, L, C::B, C::T, float>, C::T, 0);
      else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, k_pc_fused<R, L, C::B, C::T, double>, C::T, 0);
    } else {
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, k_pc_fused<R, L, C::B, C::T, double>, C::T, 0);
    }
    int dev = 0, cus = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return e == hipSuccess ? per_cu * cus : 0;
  }
}

template <typename R, int L, int CI = 0>
static hipError_t fused_cand(int ci, const Launch& Lc, int P, int j, const double* v, int vpitch,
                             void* z, int zf, int zpitch, unsigned long long* bar, unsigned polls,
                             int* err, hipStream_t s) {
  if constexpr (CI >= kNumCand) {
    return hipErrorInvalidValue;
  } else {
    if (ci == CI) return launch_fused_c<R, L, CI>(Lc, P, j, v, vpitch, z, zf, zpitch, bar, polls, err, s);
    return fused_cand<R, L, CI + 1>(ci, Lc, P, j, v, vpitch, z, zf, zpitch, bar, polls, err, s);
  }
}

template <typename R, int L, int CI = 0>
static int fused_capacity(int ci, int zf) {
  if constexpr (CI >= kNumCand) {
    return 0;
  } else {
    if (ci == CI) return fused_capacity_c<R, L, CI>(zf);
    return fused_capacity<R, L, CI + 1>(ci, zf);
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
  } \
  hipError_t pc_fused_##SUF(int log2n, int cand, const Launch& Lc, int P, int j,               \
                            const double* v, int vpitch, void* z, int zf, int zpitch,         \
                            unsigned long long* bar, unsigned polls, int* err, hipStream_t s) {         \
    switch (log2n) {                                                                          \
      CN_LOG2N_CASES(CN_FUSED_CASE_##SUF)                                                     \
    }                                                                                         \
    return hipErrorInvalidValue;                                                              \
  }                                                                                           \
  int pc_fused_capacity_##SUF(int log2n, int cand, int zf) {                                  \
    switch (log2n) {                                                                          \
      CN_LOG2N_CASES(CN_FCAP_CASE_##SUF)                                                      \
    }                                                                                         \
    return 0;                                                                                 \
  }

}  // namespace cn
