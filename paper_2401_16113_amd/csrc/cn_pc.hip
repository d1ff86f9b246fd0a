// The alpha-circulant preconditioner z = P_alpha^{-1} v (eq. (3.1)-(3.2)) on
// gfx950, as two streaming passes over the space-time vector (K1, K3 in
// cn_pc_kernels.hpp) plus a small interface solve (K2, here):
//
//  K1 (pc_forward): one workgroup per tile of B spatial columns.  Loads the
//     B x N_t tile, applies the alpha weights Lambda_alpha (step (a)), runs a
//     length-N_t complex Stockham FFT in LDS on pairs of real columns (two
//     real transforms per complex one; only the N_t/2+1 non-redundant modes
//     are used, Remark 1), then for every frequency j solves the shifted
//     system (lambda_{1,j} I - lambda_{2,j} A~) restricted to the tile's
//     interior columns (step (b), local part) and writes the tile image plus
//     two partial right-hand sides of the separator systems per (j, tile).
//  K2 (pc_reduced): for every j, the tridiagonal system of the separator
//     columns (one per tile boundary), factored once at set-up; solved by two
//     chunked affine scans.
//  K3 (pc_inverse): per tile, adds the separator contributions to the local
//     solution, runs the inverse FFT, multiplies by Lambda_alpha^{-1}/N_t
//     (step (c)) and writes z.
#include <math.h>

#include <algorithm>

#include <type_traits>

#include "cn_internal.hpp"
#include "cn_pc_reduced.hpp"

namespace cn {

// Strided layout for very wide grids: lane t of the line's L = 64 W lanes
// owns separators s = q L + t (q < CH), so every load and store is
// coalesced.  Each block q of L consecutive separators is scanned across
// the workgroup (shuffles within a wavefront, the W wavefront aggregates
// through LDS, double-buffered so one barrier per block suffices), and the
// value carried between blocks is the block's total map applied to the
// previous carry.
template <bool UP, int W>
__device__ __forceinline__ void block_affine(Cx<double>& A, Cx<double>& Bv, Cx<double>& At,
                                             Cx<double>& Bt, int lane, int wave, Cx<double>* sA,
                                             Cx<double>* sB) {
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
  // sA/sB[0..W): wavefront aggregates; [W..2W): their exclusive prefixes in
  // scan order; [2W]: the block total
  if (UP ? lane == 63 : lane == 0) {
    sA[wave] = A;
    sB[wave] = Bv;
  }
  __syncthreads();
  if (wave == 0) {
    // one wavefront scans the W aggregates (lane u holds aggregate u, in scan
    // order: reversed for the backward sweep)
    const int u = UP ? lane : W - 1 - lane;
    Cx<double> wa = lane < W ? sA[u] : one, wb = lane < W ? sB[u] : zero;
#pragma unroll
    for (int off = 1; off < W; off <<= 1) {
      const Cx<double> pa = shfl_up_c(wa, off), pb = shfl_up_c(wb, off);
      if (lane >= off) {
        wb = wa * pb + wb;
        wa = wa * pa;
      }
    }
    Cx<double> ea = shfl_up_c(wa, 1), eb = shfl_up_c(wb, 1);
    if (lane == 0) {
      ea = one;
      eb = zero;
    }
    if (lane < W) {
      sA[W + u] = ea;
      sB[W + u] = eb;
    }
    if (lane == W - 1) {
      sA[2 * W] = wa;
      sB[2 * W] = wb;
    }
  }
  __syncthreads();
  const Cx<double> pA = sA[W + wave], pB = sB[W + wave];
  At = sA[2 * W];
  Bt = sB[2 * W];
  Bv = A * pB + Bv;
  A = A * pA;
}

template <typename R, int W, int CH>
__device__ __forceinline__ void reduced_line_strided(
    const CN_G Cx<R>* __restrict__ f, CN_G Cx<R>* __restrict__ sep, const CN_G RedFwd<R>* __restrict__ rf,
    const CN_G Cx<R>* __restrict__ rb, CN_G Cx<double>* __restrict__ rtmp, int NS, int t,
    Cx<double> (*sA)[2 * W + 1], Cx<double> (*sB)[2 * W + 1]) {
  // rr of up to four blocks stays in registers; beyond, it goes through
  // the (coalesced) scratch array
  constexpr bool KEEP = CH <= 4;
  constexpr int L = 64 * W;
  const int lane = t & 63, wave = t >> 6;
  const Cx<double> zero{0.0, 0.0};
  const Cx<R> onef{R(1), R(0)}, zerof{R(0), R(0)};
  // operands of block q + 1 are loaded while block q is scanned
  auto fwd_ops = [&](int q, RedFwd<R>& r, Cx<double>& rho) {
    const int s = q * L + t;
    r = s < NS ? gld(rf + s) : RedFwd<R>{onef, zerof};
    rho = s < NS ? line_rho(f, s) : zero;
  };
  auto bwd_ops = [&](int q, Cx<R>& ap) {
    const int s = q * L + t;
    ap = s < NS ? gld(rb + s) : onef;
  };
  Cx<double> rh[KEEP ? CH : 1];
  RedFwd<R> rn;
  Cx<double> pn;
  fwd_ops(0, rn, pn);
  int buf = 0;
  Cx<double> carry = zero;
#pragma unroll
  for (int q = 0; q < CH; ++q) {
    const Cx<double> inv = wide(rn.inv);
    Cx<double> A = wide(rn.a), Bv = pn, At, Bt;
    if (q + 1 < CH) fwd_ops(q + 1, rn, pn);
    block_affine<true, W>(A, Bv, At, Bt, lane, wave, sA[buf], sB[buf]);
    buf ^= 1;
    const Cx<double> r = inv * (A * carry + Bv);  // rr_s = inv_s rho'_s
    if constexpr (KEEP) {
      rh[q] = r;
    } else {
      const int s = q * L + t;
      if (s < NS) gst(rtmp + s, r);
    }
    carry = At * carry + Bt;
  }
  Cx<R> apn;
  bwd_ops(CH - 1, apn);
  carry = zero;
#pragma unroll
  for (int q = CH - 1; q >= 0; --q) {
    Cx<double> rq;
    if constexpr (KEEP) {
      rq = rh[q];
    } else {
      const int s = q * L + t;
      rq = s < NS ? gld(rtmp + s) : zero;
    }
    Cx<double> A = wide(apn), Bv = rq, At, Bt;
    if (q > 0) bwd_ops(q - 1, apn);
    block_affine<false, W>(A, Bv, At, Bt, lane, wave, sA[buf], sB[buf]);
    buf ^= 1;
    const Cx<double> S = A * carry + Bv;
    carry = At * carry + Bt;
    const int s = q * L + t;
    if (s < NS) gst(sep + s, Cx<R>{(R)S.x, (R)S.y});
  }
}

// Block scan of the lanes' maps (in lane order, or reversed for the
// backward sweep) returning the exclusive prefix of the lane (the maps of
// the lanes before it) and the block total.  sA/sB: 2W+1 entries.
template <bool UP, int W>
__device__ __forceinline__ void block_affine_excl(Cx<double> A, Cx<double> Bv, Cx<double>& Ae,
                                                  Cx<double>& Be, Cx<double>& At, Cx<double>& Bt,
                                                  int lane, int wave, Cx<double>* sA,
                                                  Cx<double>* sB) {
  const Cx<double> one{1.0, 0.0}, zero{0.0, 0.0};
  Cx<double> Ai = A, Bi = Bv;
  block_affine<UP, W>(Ai, Bi, At, Bt, lane, wave, sA, sB);
  // exclusive = inclusive of the neighbour before it in scan order; the
  // first lane of a wavefront takes the wavefront's exclusive prefix
  Ae = UP ? shfl_up_c(Ai, 1) : shfl_down_c(Ai, 1);
  Be = UP ? shfl_up_c(Bi, 1) : shfl_down_c(Bi, 1);
  if (UP ? lane == 0 : lane == 63) {
    Ae = sA[W + wave];
    Be = sB[W + wave];
  }
  (void)one;
  (void)zero;
}

// Rounds layout for wide grids (4096 < NS <= 8192): L = 512 lanes, lane
// t of round r owns the CH = 8 consecutive separators from r L CH + t CH.
// All operands of a round are requested at once; each round needs one block
// scan per sweep, and the value carried between rounds is the round's total
// map applied to the previous carry.  rr stays in registers.
template <typename R, int RD>
__device__ __forceinline__ void reduced_line_rounds(
    const CN_G Cx<R>* __restrict__ f, CN_G Cx<R>* __restrict__ sep, const CN_G RedFwd<R>* __restrict__ rf,
    const CN_G Cx<R>* __restrict__ rb, int NS, int t, Cx<double> (*sA)[17], Cx<double> (*sB)[17]) {
  constexpr int W = 8, L = 64 * W, CH = 8;
  const int lane = t & 63, wave = t >> 6;
  const Cx<double> one{1.0, 0.0}, zero{0.0, 0.0};
  const Cx<R> onef{R(1), R(0)}, zerof{R(0), R(0)};
  Cx<double> rh[RD][CH];
  int buf = 0;
  Cx<double> carry = zero;
#pragma unroll
  for (int r = 0; r < RD; ++r) {
    const int s0 = r * L * CH + t * CH;
    // operands as loaded (rho_s = p1_s + p2_{s+1} is formed where used)
    RedFwd<R> q[CH];
    Cx<R> p1[CH], p2[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      // loaded from a clamped index and selected (a load under the s < NS
      // branch made the compiler wait there for every load in flight)
      const int s = s0 + c, sc = min(s, NS - 1);
      const RedFwd<R> qv = gld(rf + sc);
      const Cx<R> v1 = gld(f + (size_t)2 * sc), v2 = gld(f + (size_t)2 * sc + 3);
      q[c] = s < NS ? qv : RedFwd<R>{onef, zerof};
      p1[c] = s < NS ? v1 : zerof;
      p2[c] = s < NS ? v2 : zerof;
    }
    auto rho = [&](int c) {
      return Cx<double>{(double)p1[c].x + (double)p2[c].x, (double)p1[c].y + (double)p2[c].y};
    };
    Cx<double> A = one, Bv = zero;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const Cx<double> aw = wide(q[c].a);
      Bv = aw * Bv + rho(c);
      A = aw * A;
    }
    Cx<double> Ae, Be, At, Bt;
    block_affine_excl<true, W>(A, Bv, Ae, Be, At, Bt, lane, wave, sA[buf], sB[buf]);
    buf ^= 1;
    Cx<double> v = Ae * carry + Be;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      v = wide(q[c].a) * v + rho(c);
      rh[r][c] = wide(q[c].inv) * v;  // rr_s
    }
    carry = At * carry + Bt;
  }
  carry = zero;
#pragma unroll
  for (int r = RD - 1; r >= 0; --r) {
    const int s0 = r * L * CH + t * CH;
    Cx<R> ap[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const Cx<R> v = gld(rb + min(s0 + c, NS - 1));
      ap[c] = s0 + c < NS ? v : onef;
    }
    Cx<double> A = one, Bv = zero;
#pragma unroll
    for (int c = CH - 1; c >= 0; --c) {
      const Cx<double> aw = wide(ap[c]);
      Bv = aw * Bv + rh[r][c];
      A = aw * A;
    }
    Cx<double> Ae, Be, At, Bt;
    block_affine_excl<false, W>(A, Bv, Ae, Be, At, Bt, lane, wave, sA[buf], sB[buf]);
    buf ^= 1;
    Cx<double> S = Ae * carry + Be;
#pragma unroll
    for (int c = CH - 1; c >= 0; --c) {
      S = wide(ap[c]) * S + rh[r][c];
      const int s = s0 + c;
      if (s < NS) gst(sep + s, Cx<R>{(R)S.x, (R)S.y});
    }
    carry = At * carry + Bt;
  }
}

template <typename R, int RD>
__global__ __launch_bounds__(512) void k_pc_reduced_rounds(const InstDesc* __restrict__ D,
                                                           const int2* __restrict__ items,
                                                           int nitems, int standalone) {
  __shared__ Cx<double> sA[2][17], sB[2][17];
  const int item = blockIdx.x;
  if (item >= nitems) return;
  const int2 wi = work_item(items, item);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  if (!standalone && d.st->sum.done) return;
  const int j = wi.y;
  const size_t row = (size_t)j * pl.NS;
  reduced_line_rounds<R, RD>(gp((const Cx<R>*)pl.iface + (size_t)j * pl.P * 2),
                             gp((Cx<R>*)pl.sep + row), gp((const RedFwd<R>*)pl.recf + row),
                             gp((const Cx<R>*)pl.recb + row), pl.NS, threadIdx.x, sA, sB);
}

template <typename R, int W, int CH>
__global__ __launch_bounds__(64 * W) void k_pc_reduced_strided(
    const InstDesc* __restrict__ D, const int2* __restrict__ items, int nitems, int standalone) {
  __shared__ Cx<double> sA[2][2 * W + 1], sB[2][2 * W + 1];
  const int item = blockIdx.x;
  if (item >= nitems) return;
  const int2 wi = work_item(items, item);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  if (!standalone && d.st->sum.done) return;
  const int j = wi.y;
  const size_t row = (size_t)j * pl.NS;
  reduced_line_strided<R, W, CH>(gp((const Cx<R>*)pl.iface + (size_t)j * pl.P * 2),
                                 gp((Cx<R>*)pl.sep + row), gp((const RedFwd<R>*)pl.recf + row),
                                 gp((const Cx<R>*)pl.recb + row), gp(pl.red_tmp + row), pl.NS,
                                 threadIdx.x, sA, sB);
}

template <typename R, int W, int CH>
__global__ __launch_bounds__(W == 1 ? K2_THREADS : 64 * W) void k_pc_reduced(
    const InstDesc* __restrict__ D, const int2* __restrict__ items, int nitems, int standalone) {
  __shared__ Cx<double> sA[W], sB[W];
  // W == 1: four lines per workgroup, one per wavefront; else one line
  const int item = W == 1 ? blockIdx.x * (K2_THREADS / 64) + (threadIdx.x >> 6) : blockIdx.x;
  const int t = W == 1 ? (threadIdx.x & 63) : threadIdx.x;
  if (item >= nitems) return;  // uniform over the line
  const int2 wi = work_item(items, item);
  const InstDesc& d = D[wi.x];
  const PcPlan& pl = d.pl;
  if (!standalone && d.st->sum.done) return;
  const int j = wi.y;
  const size_t row = (size_t)j * pl.NS;
  reduced_line<R, W, CH>(gp((const Cx<R>*)pl.iface + (size_t)j * pl.P * 2),
                         gp((Cx<R>*)pl.sep + row), gp((const RedFwd<R>*)pl.recf + row),
                         gp((const Cx<R>*)pl.recb + row), gp(pl.red_tmp + row), pl.NS, t, sA,
                         sB);
}

// ---------------------------------------------------------------------------
// set-up: spikes of every (j, tile) and the LU factors of the separator systems
// ---------------------------------------------------------------------------
template <int B>
__global__ void k_setup_spikes(const double* __restrict__ lo, const double* __restrict__ di,
                               const double* __restrict__ up, const Cx<double>* __restrict__ mu,
                               int nx, int P, int F, Cx<double>* __restrict__ spk,
                               int* __restrict__ err) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= F * P) return;
  const int j = gid / P, t = gid % P;
  const int i0 = t * B;
  const int ncols = min(B, nx - i0);
  const int nb = t < P - 1 ? B - 1 : ncols;
  double co[3 * B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    co[3 * b] = b < ncols ? lo[i0 + b] : 0.0;
    co[3 * b + 1] = b < ncols ? di[i0 + b] : 0.0;
    co[3 * b + 2] = b < ncols ? up[i0 + b] : 0.0;
  }
  const Cx<double> m = mu[j];
  // pivots of the tile-interior elimination
  Cx<double> cp{0.0, 0.0};
  bool bad = false;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if (b < nb) {
      const double lb = b == 0 ? 0.0 : -co[3 * b];
      const Cx<double> piv = axpy_r(shift_sub(m, co[3 * b + 1]), lb, cp);
      const double mag = sqrt(piv.x * piv.x + piv.y * piv.y);
      const double scl = sqrt(m.x * m.x + m.y * m.y) + fabs(co[3 * b]) + fabs(co[3 * b + 1]) +
                         fabs(co[3 * b + 2]);
      if (!(mag > 1e-13 * scl) || !isfinite(mag)) bad = true;
      const Cx<double> q = crcp(piv);
      cp = (b < nb - 1) ? rmul(-co[3 * b + 2], q) : Cx<double>{0.0, 0.0};
    }
  }
  if (bad) atomicOr(err, 1);
  Cx<double> g[B], h[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    g[b] = Cx<double>{0.0, 0.0};
    h[b] = Cx<double>{0.0, 0.0};
  }
  g[0] = Cx<double>{co[0], 0.0};
#pragma unroll
  for (int b = 0; b < B; ++b)
    if (b == nb - 1) h[b] = Cx<double>{co[3 * b + 2], 0.0};
  tile_solve<double, Cx<double>, B>(g, m, co, nb);
  tile_solve<double, Cx<double>, B>(h, m, co, nb);
  Cx<double> gl = g[0], hl = h[0];
#pragma unroll
  for (int b = 1; b < B; ++b)
    if (b == nb - 1) {
      gl = g[b];
      hl = h[b];
    }
  Cx<double>* o = spk + (size_t)gid * 4;
  o[0] = g[0];
  o[1] = gl;
  o[2] = h[0];
  o[3] = hl;
}

__device__ inline Cx<double> cdiv(Cx<double> a, Cx<double> b) {
  const double s = 1.0 / (b.x * b.x + b.y * b.y);
  return Cx<double>{(a.x * b.x + a.y * b.y) * s, (a.y * b.x - a.x * b.y) * s};
}

template <typename R>
__global__ void k_setup_reduced(const double* __restrict__ lo, const double* __restrict__ di,
                                const double* __restrict__ up, const Cx<double>* __restrict__ mu,
                                const Cx<double>* __restrict__ spk, int P, int NS, int B, int F,
                                RedFwd<R>* __restrict__ rf, Cx<R>* __restrict__ rb,
                                int* __restrict__ err) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= F) return;
  const Cx<double> m = mu[j];
  const Cx<double>* sp = spk + (size_t)j * P * 4;
  Cx<double> beta_prev{1.0, 0.0}, cm_prev{0.0, 0.0};
  const size_t row = (size_t)j * NS;
  bool bad = false;
  for (int s = 0; s < NS; ++s) {
    const int is = (s + 1) * B - 1;
    const double lS = -lo[is], uS = -up[is];
    const Cx<double> dS{m.x - di[is], m.y};
    const Cx<double> glast = sp[(size_t)s * 4 + 1], hlast = sp[(size_t)s * 4 + 3];
    const Cx<double> gfirst = sp[(size_t)(s + 1) * 4 + 0], hfirst = sp[(size_t)(s + 1) * 4 + 2];
    const Cx<double> Am = lS * glast;
    const Cx<double> Bd = dS + lS * hlast + uS * gfirst;
    const Cx<double> Cm = (s < NS - 1) ? uS * hfirst : Cx<double>{0.0, 0.0};
    Cx<double> mlt{0.0, 0.0}, beta = Bd;
    if (s > 0) {
      mlt = cdiv(Am, beta_prev);
      beta = Bd - mlt * cm_prev;
    }
    const double mag = sqrt(beta.x * beta.x + beta.y * beta.y);
    const double scl = sqrt(Bd.x * Bd.x + Bd.y * Bd.y) + sqrt(Am.x * Am.x + Am.y * Am.y) +
                       sqrt(Cm.x * Cm.x + Cm.y * Cm.y);
    if (!(mag > 1e-13 * scl) || !isfinite(mag)) bad = true;
    const Cx<double> inv = cdiv(Cx<double>{1.0, 0.0}, beta);
    const Cx<double> capi = Cm * inv;
    rf[row + s] = RedFwd<R>{Cx<R>{(R)-mlt.x, (R)-mlt.y}, Cx<R>{(R)inv.x, (R)inv.y}};
    rb[row + s] = Cx<R>{(R)-capi.x, (R)-capi.y};
    beta_prev = beta;
    cm_prev = Cm;
  }
  if (bad) atomicOr(err, 2);
}

// ---------------------------------------------------------------------------
// launchers: the transform kernels live in cn_pc_f64.hip / cn_pc_f32.hip
// ---------------------------------------------------------------------------
hipError_t pc_forward_f64(int, int, const Launch&, const Items&, int, const double*, int,
                          hipStream_t);
hipError_t pc_forward_f32(int, int, const Launch&, const Items&, int, const double*, int,
                          hipStream_t);
hipError_t pc_inverse_f64(int, int, const Launch&, const Items&, int, void*, int, int,
                          hipStream_t);
hipError_t pc_inverse_f32(int, int, const Launch&, const Items&, int, void*, int, int,
                          hipStream_t);
bool pc_candidate_f64(int log2n, int ci, int* B, int* T, int* S, int* FS);
bool pc_candidate_f32(int log2n, int ci, int* B, int* T, int* S, int* FS);
bool pc_candidate(int prec, int log2n, int ci, int* B, int* T, int* S, int* FS) {
  int s = 1, f = 1;
  const bool ok = prec ? pc_candidate_f32(log2n, ci, B, T, &s, &f)
                       : pc_candidate_f64(log2n, ci, B, T, &s, &f);
  if (S != nullptr) *S = s;
  if (FS != nullptr) *FS = f;
  return ok;
}

hipError_t pc_forward(int prec, int log2n, int cand, const Launch& L, const Items& it, int j,
                      const double* v, int pitch, hipStream_t s) {
  return prec ? pc_forward_f32(log2n, cand, L, it, j, v, pitch, s)
              : pc_forward_f64(log2n, cand, L, it, j, v, pitch, s);
}

hipError_t pc_inverse(int prec, int log2n, int cand, const Launch& L, const Items& it, int j,
                      void* z, int zf, int pitch, hipStream_t s) {
  return prec ? pc_inverse_f32(log2n, cand, L, it, j, z, zf, pitch, s)
              : pc_inverse_f64(log2n, cand, L, it, j, z, zf, pitch, s);
}

// Interface-solve variant for separator systems of up to `ns` unknowns:
// 32 W + CH with W wavefronts per line and CH separators per lane held in
// registers (CH = 0: streamed), the fewest wavefronts that keep the chunk in
// registers without spilling: CH <= 8 (W = 1, 4, 8), CH <= 4 in 1024-thread
// workgroups (W = 16).
int k2_chunk_class(int ns, int prec) {
  (void)prec;
  for (int w : {1, 4, 8, 16}) {
    const int chunk = (ns + 64 * w - 1) / (64 * w);
    const int cmax = w == 16 ? 4 : 8;
    for (int c = 1; c <= cmax; c *= 2)
      if (chunk <= c) return 32 * w + c;
  }
  // two rounds of 4096 separators (K2_ROUNDS + 2), then strided blocks of 1024
  // separators (K2_STRIDED + CH), then streamed
  if (ns <= 2 * 4096) return K2_ROUNDS + 2;
  const int blocks = (ns + 1023) / 1024;
  for (int c = 4; c <= 16; c *= 2)
    if (blocks <= c) return K2_STRIDED + c;
  return 32 * 16;
}

hipError_t pc_reduced(int prec, const Launch& L, const Items& it, int chunk_class, int j,
                      int standalone, hipStream_t s) {
  (void)j;
  if (it.n <= 0) return hipSuccess;
  switch (chunk_class) {
#define K2(W, CH)                                                                              \
  case 32 * W + CH: {                                                                          \
    const dim3 grid(W == 1 ? (it.n + 3) / 4 : it.n), block(W == 1 ? K2_THREADS : 64 * W);    \
    if (prec)                                                                                  \
      hipLaunchKernelGGL((k_pc_reduced<float, W, CH>), grid, block, 0, s, L.D, it.it, it.n,   \
                         standalone);                                                          \
    else                                                                                       \
      hipLaunchKernelGGL((k_pc_reduced<double, W, CH>), grid, block, 0, s, L.D, it.it, it.n,  \
                         standalone);                                                          \
    break;                                                                                     \
  }
    K2(1, 1) K2(1, 2) K2(1, 4) K2(1, 8)
    K2(4, 1) K2(4, 2) K2(4, 4) K2(4, 8)
    K2(16, 1) K2(16, 2) K2(16, 4) K2(16, 0)
    K2(8, 1) K2(8, 2) K2(8, 4) K2(8, 8)
#define K2S(CH)                                                                                \
  case K2_STRIDED + CH:                                                                        \
    if (prec)                                                                                  \
      hipLaunchKernelGGL((k_pc_reduced_strided<float, 16, CH>), dim3(it.n), dim3(1024), 0, s, \
                         L.D, it.it, it.n, standalone);                                        \
    else                                                                                       \
      hipLaunchKernelGGL((k_pc_reduced_strided<double, 16, CH>), dim3(it.n), dim3(1024), 0,   \
                         s, L.D, it.it, it.n, standalone);                                     \
    break;
    K2S(1) K2S(2) K2S(4) K2S(8) K2S(16)
#undef K2S
#define K2R(RD)                                                                                \
  case K2_ROUNDS + RD:                                                                         \
    if (prec)                                                                                  \
      hipLaunchKernelGGL((k_pc_reduced_rounds<float, RD>), dim3(it.n), dim3(512), 0, s, L.D,  \
                         it.it, it.n, standalone);                                             \
    else                                                                                       \
      hipLaunchKernelGGL((k_pc_reduced_rounds<double, RD>), dim3(it.n), dim3(512), 0, s, L.D, \
                         it.it, it.n, standalone);                                             \
    break;
    K2R(2)
#undef K2R
#undef K2
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t pc_setup(PcPlan& pl, Cx<double>* spk, int* err, hipStream_t s) {
  const int n = pl.F * pl.P;
  const int thr = 128, blk = (n + thr - 1) / thr;
  switch (pl.B) {
#define SP(BB)                                                                                 \
  case BB:                                                                                     \
    hipLaunchKernelGGL((k_setup_spikes<BB>), dim3(blk), dim3(thr), 0, s, pl.lo, pl.di, pl.up, \
                       pl.mu, pl.nx, pl.P, pl.F, spk, err);                                   \
    break;
    SP(2) SP(4) SP(8) SP(16)
#undef SP
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && pl.NS > 0) {
    const int t2 = 64, b2 = (pl.F + t2 - 1) / t2;
    if (pl.prec)
      hipLaunchKernelGGL(k_setup_reduced<float>, dim3(b2), dim3(t2), 0, s, pl.lo, pl.di, pl.up,
                         pl.mu, spk, pl.P, pl.NS, pl.B, pl.F, (RedFwd<float>*)pl.recf,
                         (Cx<float>*)pl.recb, err);
    else
      hipLaunchKernelGGL(k_setup_reduced<double>, dim3(b2), dim3(t2), 0, s, pl.lo, pl.di, pl.up,
                         pl.mu, spk, pl.P, pl.NS, pl.B, pl.F, (RedFwd<double>*)pl.recf,
                         (Cx<double>*)pl.recb, err);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace cn
