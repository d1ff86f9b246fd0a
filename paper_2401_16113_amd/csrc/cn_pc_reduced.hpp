// Interface (separator) systems of the partitioned step-(b) solve: the
// per-frequency line solver.
#pragma once
#include "cn_internal.hpp"

namespace cn {

// ---------------------------------------------------------------------------
// K2: interface (separator) systems, one line (frequency j) per W wavefronts.
// K1 leaves two partial right-hand sides per tile p: p1_p = d + lo y_last
// (its own separator) and p2_p = up y_first (the separator left of it), so
//   rho_s = p1_s + p2_{s+1}                                      (s = 0..NS-1)
//   forward  rho'_s = a_s rho'_{s-1} + rho_s,   rr_s = inv_s rho'_s
//   backward S_s    = ap_s S_{s+1} + rr_s
// with a_s = -m_s, ap_s = -c_s inv_s from the LU factors of the separator
// system (computed at set-up).  Each recurrence is an affine scan: every lane
// composes the maps of its chunk of consecutive separators, a Hillis-Steele
// scan of the lane maps runs on cross-lane shuffles, the W wave aggregates
// are chained through LDS (W > 1), then every lane replays its chunk from the
// carried value.  With CH > 0 a lane loads its whole chunk (<= CH
// separators) up front and keeps rr in registers; CH = 0 (very wide
// instances) streams through the rr scratch array.  W = 1 packs four lines
// into a 256-thread workgroup.
// ---------------------------------------------------------------------------
constexpr int K2_THREADS = 256;

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

// Forward factor record of separator s, {a_s, inv_s}; the backward one is
// ap_s alone.  Precision of the preconditioner (the substitutions run in
// float64).
template <typename R>
struct RedFwd {
  Cx<R> a, inv;
};
template <typename R>
__device__ __forceinline__ RedFwd<R> gld(const CN_G RedFwd<R>* p) {
  const CN_G Cx<R>* c = (const CN_G Cx<R>*)p;
  return RedFwd<R>{gld(c), gld(c + 1)};
}

// rho_s of one line from the partial right-hand sides f[2p], f[2p+1] of the tiles
template <typename R>
__device__ __forceinline__ Cx<double> line_rho(const CN_G Cx<R>* __restrict__ f, int s) {
  const Cx<R> p1 = gld(f + (size_t)2 * s), p2 = gld(f + (size_t)2 * s + 3);
  return Cx<double>{(double)p1.x + (double)p2.x, (double)p1.y + (double)p2.y};
}

template <typename R, int W, int CH>
__device__ __forceinline__ void reduced_line(const CN_G Cx<R>* __restrict__ f, CN_G Cx<R>* __restrict__ sep,
                                             const CN_G RedFwd<R>* __restrict__ rf,
                                             const CN_G Cx<R>* __restrict__ rb,
                                             CN_G Cx<double>* __restrict__ rtmp, int NS, int t,
                                             Cx<double>* sA, Cx<double>* sB) {
  const int lane = t & 63, wave = t >> 6;
  const int chunk = (NS + 64 * W - 1) / (64 * W);
  const int s0 = min(NS, t * chunk), s1 = min(NS, s0 + chunk);
  const Cx<double> one{1.0, 0.0}, zero{0.0, 0.0};
  if constexpr (CH > 0) {
    // every operand of the lane's chunk is requested up front (independent
    // loads, one memory latency); padding entries are identity maps
    Cx<R> a[CH], iv[CH], ap[CH];
    Cx<double> rh[CH];
    const Cx<R> onef{R(1), R(0)}, zerof{R(0), R(0)};
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int s = s0 + q;
      const RedFwd<R> r = s < s1 ? gld(rf + s) : RedFwd<R>{onef, zerof};
      a[q] = r.a;
      iv[q] = r.inv;
      rh[q] = s < s1 ? line_rho(f, s) : zero;
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) ap[q] = s0 + q < s1 ? gld(rb + s0 + q) : onef;
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
      rh[q] = wide(iv[q]) * r;  // rr_s
    }
    A = one;
    Bv = zero;
#pragma unroll
    for (int q = CH - 1; q >= 0; --q) {
      const Cx<double> apw = wide(ap[q]);
      Bv = apw * Bv + rh[q];
      A = apw * A;
    }
    Cx<double> S = line_carry<false, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll
    for (int q = CH - 1; q >= 0; --q) {
      S = wide(ap[q]) * S + rh[q];
      const int s = s0 + q;
      if (s < s1) gst(sep + s, Cx<R>{(R)S.x, (R)S.y});
    }
  } else {
    Cx<double> A = one, Bv = zero;
#pragma unroll 4
    for (int s = s0; s < s1; ++s) {
      const Cx<double> a = wide(gld(rf + s).a);
      Bv = a * Bv + line_rho(f, s);
      A = a * A;
    }
    Cx<double> r = line_carry<true, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll 4
    for (int s = s0; s < s1; ++s) {
      const RedFwd<R> q = gld(rf + s);
      r = wide(q.a) * r + line_rho(f, s);
      gst(rtmp + s, wide(q.inv) * r);
    }
    A = one;
    Bv = zero;
#pragma unroll 4
    for (int s = s1 - 1; s >= s0; --s) {
      const Cx<double> ap = wide(gld(rb + s));
      Bv = ap * Bv + gld(rtmp + s);
      A = ap * A;
    }
    Cx<double> S = line_carry<false, W>(A, Bv, lane, wave, sA, sB);
#pragma unroll 4
    for (int s = s1 - 1; s >= s0; --s) {
      S = wide(gld(rb + s)) * S + gld(rtmp + s);
      gst(sep + s, Cx<R>{(R)S.x, (R)S.y});
    }
  }
}

}  // namespace cn
