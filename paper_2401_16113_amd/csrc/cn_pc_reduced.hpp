// Interface (separator) systems of the partitioned step-(b) solve: the
// per-frequency line solver.
#pragma once
#include "cn_internal.hpp"

namespace cn {

// ---------------------------------------------------------------------------
// K2: interface (separator) systems, one line (frequency j) per W wavefronts:
//   rho_s = d_s + lo_s y_last(s) + up_s y_first(s+1)           (s = 0..NS-1)
//   forward  rho'_s = a_s rho'_{s-1} + rho_s,       a_s  = -m_s
//   backward S_s    = ap_s S_{s+1} + inv_s rho'_s,  ap_s = -c_s inv_s
// Each recurrence is an affine scan: every lane composes the maps of its
// chunk of consecutive separators, a Hillis-Steele scan of the lane maps runs
// on cross-lane shuffles, the W wave aggregates are chained through LDS
// (W > 1), then every lane replays its chunk from the carried value.  With
// CH > 0 a lane loads its whole chunk (<= CH separators) up front and keeps
// rho' in registers; CH = 0 (very wide instances) streams through the rho'
// scratch array.  W = 1 packs four lines into a 256-thread workgroup.
// ---------------------------------------------------------------------------
constexpr int K2_THREADS = 256;
constexpr int K2_STRIDED = 4096;  // variant code offset of the strided layout

__device__ __forceinline__ Cx<double> shfl_up_c(Cx<double> v, int off) {
  return Cx<double>{__shfl_up(v.x, off, 64), __shfl_up(v.y, off, 64)};
}
__device__ __forceinline__ Cx<double> shfl_down_c(Cx<double> v, int off) {
  return Cx<double>{__shfl_down(v.x, off, 64), __shfl_down(v.y, off, 64)};
}

// Scan of the maps r -> A r + Bv held by the line's lanes in lane order (UP)
// or in reverse order; returns the value carried into the lane's chunk (the
// composed map of all preceding lanes applied to 0).
template <bool UP, int W>
__device__ __forceinline__ Cx<double> line_carry(Cx<double> A, Cx<double> Bv, int lane, int wave,
                                                 Cx<double>* sA, Cx<double>* sB) {
  const Cx<double> one{1.0, 0.0}, zero{0.0, 0.0};
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const Cx<double> pa = UP ? shfl_up_c(A, off) : shfl_down_c(A, off);
    const Cx<double> pb = UP ? shfl_up_c(Bv, off) : shfl_down_c(Bv, off);
    const bool has = UP ? lane >= off : lane + off < 64;
    if (has) {
      Bv = A * pb + Bv;
      A = A * pa;
    }
  }
  Cx<double> eA = UP ? shfl_up_c(A, 1) : shfl_down_c(A, 1);
  Cx<double> eB = UP ? shfl_up_c(Bv, 1) : shfl_down_c(Bv, 1);
  if (UP ? lane == 0 : lane == 63) {
    eA = one;
    eB = zero;
  }
  if constexpr (W == 1) {
    return eB;
  } else {
    __syncthreads();  // earlier readers of sA/sB are done
    if (UP ? lane == 63 : lane == 0) {
      sA[wave] = A;
      sB[wave] = Bv;
    }
    __syncthreads();
    Cx<double> c = zero;
    if (UP) {
      for (int u = 0; u < wave; ++u) c = sA[u] * c + sB[u];
    } else {
      for (int u = W - 1; u > wave; --u) c = sA[u] * c + sB[u];
    }
    return eA * c + eB;
  }
}

template <typename R>
__device__ __forceinline__ Cx<double> wide(Cx<R> v) {
  return Cx<double>{(double)v.x, (double)v.y};
}

// Factor record of separator s: {a_s, ap_s, inv_s} in the preconditioner's
// precision (the substitutions run in float64).
template <typename R>
struct RedRec {
  Cx<R> a, ap, inv;
};

template <typename R, int W, int CH>
__device__ __forceinline__ void reduced_line(
    const Cx<R>* __restrict__ f, Cx<R>* __restrict__ sep, const RedRec<R>* __restrict__ rec,
    Cx<double>* __restrict__ rtmp, const double* __restrict__ lo,
    const double* __restrict__ up, int NS, int B, int t, Cx<double>* sA, Cx<double>* sB) {
  const int lane = t & 63, wave = t >> 6;
  const int chunk = (NS + 64 * W - 1) / (64 * W);
  const int s0 = min(NS, t * chunk), s1 = min(NS, s0 + chunk);
  auto rho = [&](int s) -> Cx<double> {
    const int is = (s + 1) * B - 1;
    const Cx<R> d = f[(size_t)s * 3 + 0], yl = f[(size_t)s * 3 + 1], yf = f[(size_t)(s + 1) * 3 + 2];
    const double l = lo[is], u = up[is];
    return Cx<double>{(double)d.x + l * (double)yl.x + u * (double)yf.x,
                      (double)d.y + l * (double)yl.y + u * (double)yf.y};
  };
  const Cx<double> one{1.0, 0.0}, zero{0.0, 0.0};
  if constexpr (CH > 0) {
    // the forward operands of the lane's chunk are loaded up front
    // (independent loads, one memory latency), the backward ones once the
    // forward sweep is done (fewer live registers); padding entries are
    // identity maps
    Cx<R> a[CH];
    Cx<double> rh[CH];
    const Cx<R> onef{R(1), R(0)}, zerof{R(0), R(0)};
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int s = s0 + q;
      a[q] = s < s1 ? rec[s].a : onef;
      rh[q] = s < s1 ? rho(s) : zero;
    }
    Cx<double> A = one, Bv = zero;
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const Cx<double> aw = wide(a[q]);
      Bv = aw * Bv + rh[q];
      A = aw * A;
    }
    Cx<double> r = line_carry<true, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      r = wide(a[q]) * r + rh[q];
      rh[q] = r;  // rho'_s
    }
    Cx<R> ap[CH], iv[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int s = s0 + q;
      ap[q] = s < s1 ? rec[s].ap : onef;
      iv[q] = s < s1 ? rec[s].inv : zerof;
    }
    A = one;
    Bv = zero;
#pragma unroll
    for (int q = CH - 1; q >= 0; --q) {
      const Cx<double> apw = wide(ap[q]);
      Bv = apw * Bv + wide(iv[q]) * rh[q];
      A = apw * A;
    }
    Cx<double> S = line_carry<false, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll
    for (int q = CH - 1; q >= 0; --q) {
      S = wide(ap[q]) * S + wide(iv[q]) * rh[q];
      const int s = s0 + q;
      if (s < s1) sep[s] = Cx<R>{(R)S.x, (R)S.y};
    }
  } else {
    Cx<double> A = one, Bv = zero;
#pragma unroll 4
    for (int s = s0; s < s1; ++s) {
      const Cx<double> a = wide(rec[s].a);
      Bv = a * Bv + rho(s);
      A = a * A;
    }
    Cx<double> r = line_carry<true, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll 4
    for (int s = s0; s < s1; ++s) {
      r = wide(rec[s].a) * r + rho(s);
      rtmp[s] = r;
    }
    A = one;
    Bv = zero;
#pragma unroll 4
    for (int s = s1 - 1; s >= s0; --s) {
      const RedRec<R> q = rec[s];
      const Cx<double> ap = wide(q.ap);
      Bv = ap * Bv + wide(q.inv) * rtmp[s];
      A = ap * A;
    }
    Cx<double> S = line_carry<false, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll 4
    for (int s = s1 - 1; s >= s0; --s) {
      const RedRec<R> q = rec[s];
      S = wide(q.ap) * S + wide(q.inv) * rtmp[s];
      sep[s] = Cx<R>{(R)S.x, (R)S.y};
    }
  }
}

}  // namespace cn
