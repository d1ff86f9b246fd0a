// Krylov kernels of the right-preconditioned GMRES(m) solve on gfx950:
//   * the all-at-once CN matvec (block form of Sec. 3.2), plain, as a
//     residual b - M x, and fused with the first Gram-Schmidt dot pass;
//   * the CGS2 update pass: both projections in one update of w (formed
//     again from z_j rather than stored by the matvec), the second
//     one's coefficients from the Gram matrix of the basis (kept up to date
//     by this pass itself: while it writes v_{j+1} it also forms the dots of
//     v_{j+1} with the basis), so the second projection needs no pass over
//     the basis of its own; the basis is stored unnormalised with a float64
//     scale per vector, so normalisation never costs a pass either;
//   * the Givens / least-squares update (one workgroup per instance);
//   * x += Z y and the right-hand side b = xi + tau f (eq. (2.2)).
// Every kernel serves a list of instances: work items (instance, block) index
// an array of instance descriptors, so a single solve and a batch of uneven
// solves share one code path and one launch per step.
// Reductions are deterministic: every workgroup writes its partial sums; a
// finishing kernel (one workgroup per instance) adds them in a fixed order
// and updates the solver state.  Stream order makes the partials visible,
// so no workgroup issues a device-scope fence (on a multi-XCD part such a
// fence writes back and invalidates the XCD's L2).
#include <math.h>

#include <type_traits>

#include "cn_internal.hpp"

namespace cn {


__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-reduce NV accumulators into partials[q*nblk + blk] (fixed order).
template <int NV, int THREADS = KT>
__device__ __forceinline__ void block_partials(const double (&acc)[NV], int nv, double* red,
                                               double* partials, int blk, int nblk) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    if (q < nv) {
      const double s = wave_sum(acc[q]);
      if (lane == 0) red[wv * NV + q] = s;
    }
  }
  __syncthreads();
  if (tid < nv) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < THREADS / 64; ++w) s += red[w * NV + tid];
    gp(partials)[(size_t)tid * nblk + blk] = s;
  }
}

// Sum partials[q*nblk + b] over b for q < nv into out[q]: wave w handles
// q = w, w + W, ... (W wavefronts); lane l adds b = l, l + 64, ... then the
// wave adds its lanes.  The order is fixed, so the result is bitwise
// reproducible -- and identical in every workgroup that computes it.
constexpr int FT = 1024;    // threads of a finishing kernel
constexpr int FCHUNK = 32;  // partials per lane loaded back to back
template <int THREADS = FT>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partials, int nblk,
                                                int nv, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = wv; q < nv; q += THREADS / 64) {
    const CN_G double* p = gp(partials + (size_t)q * nblk);
    double s = 0.0;
    for (int base = 0; base < nblk; base += 64 * FCHUNK) {
      double v[FCHUNK];
#pragma unroll
      for (int i = 0; i < FCHUNK; ++i) {
        const int b = base + lane + 64 * i;
        v[i] = b < nblk ? p[b] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < FCHUNK; ++i) s += v[i];
    }
    s = wave_sum(s);
    if (lane == 0) out[q] = s;
  }
  __syncthreads();
}

// Publish a summary to a host slot: fields first, then (after a system-scope
// fence) the sequence number the host polls for.
__device__ __forceinline__ void publish(GSummary* host, const GSummary& sm, int seq) {
  if (host == nullptr) return;
  host->bnorm = sm.bnorm;
  host->beta = sm.beta;
  host->est = sm.est;
  host->relres = sm.relres;
  host->k = sm.k;
  host->done = sm.done;
  host->breakdown = sm.breakdown;
  host->x0_rejected = sm.x0_rejected;
  host->err = sm.err;
  __threadfence_system();
  *(volatile int*)&host->seq = seq;
}

// ---------------------------------------------------------------------------
// matvec: y = M x (MODE 0, one instance: x = xo, y = yo),
//         r = b - M x into V_0 with ||r||^2, ||b||^2 (MODE 1: x = xo + off,
//         unread when bit 0 of x_zero is set; bit 1: only for instances whose
//         cycle has stopped; b = bo + off),
//         the dots of w = M z_j with V_0..V_j (MODE 2, the coefficients of the
//         first CGS2 projection; w itself is not stored: the update forms it
//         again from z_j, which moves fewer bytes than storing and re-reading it)
// Each thread marches down the time levels of one spatial column.
// ---------------------------------------------------------------------------
// One thread's column of the matvec, levels k0 .. k1-1 (see k_matvec).  The
// vectors are parameters so that __restrict__ holds (y is never one of the
// vectors read), which lets the loads of later levels be issued before the
// store of the current one.
// Neighbour z or x at a grid edge: loaded unconditionally from a valid address
// and dropped by a select when the vector is float32 (the conversion to
// float64 inside a lane-dependent branch made the compiler wait for every load
// in flight before leaving the branch, at every level), and behind the branch
// when it is float64 (no conversion; measured faster).
template <typename TX>
__device__ __forceinline__ double edge_load(const CN_G TX* p, size_t e, bool keep) {
  if constexpr (std::is_same<TX, float>::value) {
    const double v = (double)p[e];
    return keep ? v : 0.0;
  } else {
    return keep ? (double)p[e] : 0.0;
  }
}

// DW: the instance has time weights d_k (a compile-time choice, so that the
// level loop is one basic block and later levels' loads can be issued ahead)
template <typename TX, int MODE, int NV, int NA, bool DW>
__device__ __forceinline__ void matvec_column(const CN_G TX* __restrict__ x,
                                              const CN_G double* __restrict__ b,
                                              CN_G double* __restrict__ y,
                                              const CN_G double* __restrict__ V,
                                              const CN_G double* __restrict__ plo,
                                              const CN_G double* __restrict__ pdi,
                                              const CN_G double* __restrict__ pup,
                                              const CN_G double* __restrict__ dw, long long vstride,
                                              VecLayout xl, int px, int py, int nx, int nv, int i,
                                              int k0, int k1, double (&acc)[NA]) {
  const double lo = plo[i], di = pdi[i], up = pup[i];
  const bool hl = i > 0, hr = i < nx - 1;
  // x's columns i-1, i, i+1 (layout xl); b and y are row-major (pitches px, py);
  // at the grid's edges the missing neighbour's offset is 0 (a valid address,
  // see edge_load)
  const size_t xm = hl ? xl.col(i - 1) : 0, xc = xl.col(i), xp = hr ? xl.col(i + 1) : 0;
  const size_t xrow = (size_t)xl.row;
  double pm = 0.0, pc = 0.0, pp = 0.0;  // previous level at i-1, i, i+1
  // MODE 2 reads z_j, never null (no branch in the level loop)
  const bool have_x = MODE == 2 || x != nullptr;
  if (k0 > 0 && have_x) {
    const size_t o = (size_t)(k0 - 1) * xrow;
    pc = (double)x[o + xc];
    pm = edge_load(x, o + xm, hl);
    pp = edge_load(x, o + xp, hr);
  }
  size_t vo[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) vo[q] = (size_t)(q < nv ? q : nv - 1) * vstride;
  constexpr int UNR = NV <= 4 ? 4 : (NV <= 8 ? 2 : 1);
#pragma unroll UNR
  for (int k = k0; k < k1; ++k) {
    double cm = 0.0, cc = 0.0, cp = 0.0;
    const size_t off = (size_t)k * px, offy = (size_t)k * py, offx = (size_t)k * xrow;
    if (have_x) {
      cc = (double)x[offx + xc];
      cm = edge_load(x, offx + xm, hl);
      cp = edge_load(x, offx + xp, hr);
    }
    const double w = DW ? dw[k] : 1.0;
    // (M x)^k = (x^k - x^{k-1}) - (w/2) A~ (x^k + x^{k-1})
    const double sm = cm + pm, s0 = cc + pc, sp = cp + pp;
    const double ax = lo * sm + di * s0 + up * sp;
    double yv = (cc - pc) - 0.5 * w * ax;
    if (MODE == 1) {
      const double bv = b[off + i];
      yv = bv - yv;
      acc[0] += yv * yv;
      acc[1] += bv * bv;
    }
    if (MODE == 2) {
      // q >= nv re-reads v_{nv-1} (cache hits); those dots are never written
#pragma unroll
      for (int q = 0; q < NV; ++q) acc[q] += V[vo[q] + offy + i] * yv;
    } else {
      y[offy + i] = yv;
    }
    pm = cm;
    pc = cc;
    pp = cp;
  }
}

template <typename TX, int MODE, int NV>
__global__ __launch_bounds__(MVT) void k_matvec(const InstDesc* __restrict__ D,
                                               const int2* __restrict__ items, int j,
                                               const TX* __restrict__ xo,
                                               const double* __restrict__ bo,
                                               double* __restrict__ yo, int x_zero) {
  constexpr int NA = NV > 2 ? NV : 2;
  __shared__ double red[(MVT / 64) * NA];
  const int2 wi = work_item(items, blockIdx.x);
  const InstDesc& d = D[wi.x];
  if (MODE == 2 && d.st->sum.done) return;
  // MODE 1, bit 1 of x_zero: speculative residual, only for a stopped cycle
  if (MODE == 1 && (x_zero & 2) && !d.st->sum.done) return;
  const TX* __restrict__ x;
  const double* __restrict__ b = nullptr;
  double* __restrict__ y;
  if (MODE == 0) {
    x = xo;
    y = yo;
  } else if (MODE == 1) {
    x = (x_zero & 1) ? nullptr : xo + d.off;
    b = bo + d.off;
    y = d.V;
  } else {
    x = (const TX*)d.Z + (size_t)j * d.vstride;
    y = nullptr;
  }
  const int nv = j + 1;
  const int nx = d.nx;
  // row pitches: caller vectors use N_x, the basis ldx; Z_j (MODE 2) is
  // tile-blocked
  const int px = nx;                       // b (and x for MODE 0, 1)
  const int py = MODE == 0 ? nx : d.ldx;   // y (and the basis V)
  const VecLayout xl = MODE == 2 ? z_layout(d) : row_major(nx, d.nt);
  const int blk = wi.y;
  const int cb = blk % d.mv_cols, rb = blk / d.mv_cols;
  const int i = cb * MVT + threadIdx.x;
  const int k0 = rb * d.rows, k1 = min(d.nt, k0 + d.rows);
  double acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  if (i < nx) {
    if (d.dw != nullptr)
      matvec_column<TX, MODE, NV, NA, true>(gp(x), gp(b), gp(y), gp(d.V), gp(d.pl.lo),
                                            gp(d.pl.di), gp(d.pl.up), gp(d.dw), d.vstride, xl, px,
                                            py, nx, nv, i, k0, k1, acc);
    else
      matvec_column<TX, MODE, NV, NA, false>(gp(x), gp(b), gp(y), gp(d.V), gp(d.pl.lo),
                                             gp(d.pl.di), gp(d.pl.up), gp(d.dw), d.vstride, xl,
                                             px, py, nx, nv, i, k0, k1, acc);
  }
  if (MODE == 0) return;
  block_partials<NA, MVT>(acc, MODE == 1 ? 2 : nv, red, d.partials, blk, d.mv_grid);
}

// ---------------------------------------------------------------------------
// CGS2 update: v_{j+1} = w - V (c1 + c2), its norm and its Gram row
// ---------------------------------------------------------------------------
// Coefficients of both projections.  The first, h1_q = <q_q, w> for the
// normalised basis q_q = v_q / ||v_q||, from the matvec's partial dots: every
// workgroup reduces them itself (same order, same values), so no finishing
// kernel sits between the matvec and this pass.  The second projection of
// CGS2, h2 = Q^T (w - Q h1) = (I - Q^T Q) h1 in exact arithmetic, from the
// Gram matrix G = Q^T Q of the basis (unit diagonal, so h2_p = -sum_{q != p}
// G_pq h1_q).  The update forms v_{j+1} from w in one pass either way, so the
// dots against the once-projected vector would only add that vector's own
// rounding; the Gram matrix carries what the second pass corrects, the
// basis' loss of orthogonality.  c = (h1 + h2) / ||v_q|| are the coefficients
// of the stored (unnormalised) basis; block 0 of each instance keeps h1, h2
// for the Hessenberg column.
__device__ __forceinline__ void update_coeffs(const double* __restrict__ partials, int nblk,
                                              int nv, GState* st, bool keep, double* sh,
                                              double* sc) {
  reduce_partials<MVT>(partials, nblk, nv, sh);
  if (threadIdx.x < nv) sh[threadIdx.x] *= st->vscale[threadIdx.x];
  __syncthreads();
  if (threadIdx.x < nv) {
    const int p = threadIdx.x;
    const double* g = st->gram + (size_t)p * NVMAX;
    double h2 = 0.0;
    // every entry loaded (no branch around the loads), the diagonal skipped
    for (int q = 0; q < nv; ++q) {
      const double gq = g[q];
      if (q != p) h2 -= gq * sh[q];
    }
    const double h1 = sh[p], s = st->vscale[p];
    sc[p] = (h1 + h2) * s;
    if (keep) {
      st->h1[p] = h1;
      st->h2[p] = h2;
      st->c1[p] = h1 * s;
      st->c2[p] = h2 * s;
    }
  }
  __syncthreads();
}

// The update's column: at levels k0 .. k1-1 of column i, w = (M z_j) formed
// again from z_j as the matvec forms it (same expression, same bits),
// v_{j+1} = w - V c, with ||v_{j+1}||^2 into acc[0] and <v_q, v_{j+1}> into
// acc[1 + q].  The vectors are parameters so that __restrict__ holds
// (v_{j+1} is the basis buffer's next vector, disjoint from the vectors read).
// Vectors q >= nv re-read v_{nv-1} (cache hits) with coefficient 0; their
// dots are never written: no branch between the loads.
// Every thread of the workgroup calls this (act: the column exists) and
// coeffs() -- the coefficient reduction, with workgroup barriers -- runs
// after the column's first levels have been requested: the barriers wait for
// LDS only, so those loads are in flight during the reduction instead of
// starting after it.
template <typename TX, int NV, bool DW, typename Coeffs>
__device__ __forceinline__ void update_column(const CN_G TX* __restrict__ z,
                                              const CN_G double* __restrict__ V,
                                              CN_G double* __restrict__ vout,
                                              const CN_G double* __restrict__ plo,
                                              const CN_G double* __restrict__ pdi,
                                              const CN_G double* __restrict__ pup,
                                              const CN_G double* __restrict__ dw,
                                              long long vstride, VecLayout zl, int ldx, int nx,
                                              int nv, int i, bool act, int k0, int k1,
                                              Coeffs&& coeffs, double (&acc)[NV + 1]) {
  // levels in flight together: fewer for long bases (registers)
  constexpr int UNR = NV <= 4 ? 4 : (NV <= 8 ? 2 : 1);
  const bool hl = i > 0, hr = i < nx - 1;
  // basis offsets in registers for short bases, formed per load for long ones
  constexpr int NVO = NV <= 8 ? NV : 1;
  size_t vo[NVO];
#pragma unroll
  for (int q = 0; q < NVO; ++q) vo[q] = (size_t)(q < nv ? q : nv - 1) * vstride;
  auto voff = [&](int q) -> size_t {
    if constexpr (NV <= 8) return vo[q];
    else return (size_t)(q < nv ? q : nv - 1) * vstride;
  };
  double lo = 0.0, di = 0.0, up = 0.0;
  double pm = 0.0, pc = 0.0, pp = 0.0;  // z at the previous level, i-1, i, i+1
  // z's columns i-1, i, i+1 in its (tile-blocked) layout (edges: edge_load)
  const size_t zm = act && hl ? zl.col(i - 1) : 0, zc = act ? zl.col(i) : 0,
               zp = act && hr ? zl.col(i + 1) : 0;
  const size_t zrow = (size_t)zl.row;
  // the first PF levels, requested before the coefficients exist (few: the
  // registers they hold must not cost the kernel its second workgroup per CU)
  constexpr int PF = NV <= 4 ? 2 : 1;
  double fc[PF], fm[PF], fp[PF], fv[PF][NV], fw[PF];
  if (act) {
    lo = plo[i];
    di = pdi[i];
    up = pup[i];
    if (k0 > 0) {
      const size_t o = (size_t)(k0 - 1) * zrow;
      pc = (double)z[o + zc];
      pm = edge_load(z, o + zm, hl);
      pp = edge_load(z, o + zp, hr);
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      // levels past k1 re-read level k1-1 (in bounds, never used)
      const int k = min(k0 + u, k1 - 1);
      const size_t off = (size_t)k * ldx, oz = (size_t)k * zrow;
      fc[u] = (double)z[oz + zc];
      fm[u] = edge_load(z, oz + zm, hl);
      fp[u] = edge_load(z, oz + zp, hr);
#pragma unroll
      for (int q = 0; q < NV; ++q) fv[u][q] = V[voff(q) + off + i];
      fw[u] = DW ? dw[k] : 1.0;
    }
  }
  const double* c = coeffs();
  if (!act) return;
  // one level: (M z)^k = (z^k - z^{k-1}) - (w/2) A~ (z^k + z^{k-1}), then the
  // projections
  auto level = [&](int k, double cc, double cm, double cp, const double (&vq)[NV], double w) {
    const size_t off = (size_t)k * ldx;
    const double sm = cm + pm, s0 = cc + pc, sp = cp + pp;
    const double ax = lo * sm + di * s0 + up * sp;
    double v = (cc - pc) - 0.5 * w * ax;
#pragma unroll
    for (int q = 0; q < NV; ++q) v -= c[q] * vq[q];
    vout[off + i] = v;
    acc[0] += v * v;
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[1 + q] += vq[q] * v;
    pm = cm;
    pc = cc;
    pp = cp;
  };
#pragma unroll
  for (int u = 0; u < PF; ++u)
    if (k0 + u < k1) level(k0 + u, fc[u], fm[u], fp[u], fv[u], fw[u]);
#pragma unroll UNR
  for (int k = k0 + PF; k < k1; ++k) {
    const size_t off = (size_t)k * ldx, oz = (size_t)k * zrow;
    const double cc = (double)z[oz + zc];
    const double cm = edge_load(z, oz + zm, hl), cp = edge_load(z, oz + zp, hr);
    double vq[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) vq[q] = V[voff(q) + off + i];
    const double w = DW ? dw[k] : 1.0;
    level(k, cc, cm, cp, vq, w);
  }
}

// CGS2 update over the matvec's blocks (z_j in TX).  partials2 rows:
// 0 = ||v_{j+1}||^2, 1 + q = <v_q, v_{j+1}> (q <= j).  The pad columns of
// v_{j+1} (N_x <= i < ldx) are never written and stay zero.
template <typename TX, int NV>
__global__ __launch_bounds__(MVT) void k_cgs_update(const InstDesc* __restrict__ D,
                                                    const int2* __restrict__ items, int j) {
  constexpr int NA = NV + 1;
  __shared__ double red[(MVT / 64) * NA];
  __shared__ double sh[NVMAX], sc[NVMAX];
  const int2 wi = work_item(items, blockIdx.x);
  const InstDesc& d = D[wi.x];
  GState* st = d.st;
  if (st->sum.done) return;
  const int nv = j + 1;
  double acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  const int blk = wi.y;
  const int cb = blk % d.mv_cols, rb = blk / d.mv_cols;
  const int i = cb * MVT + threadIdx.x;
  const int k0 = rb * d.rows, k1 = min(d.nt, k0 + d.rows);
  auto coeffs = [&]() -> const double* {
    update_coeffs(d.partials, d.mv_grid, nv, st, wi.y == 0, sh, sc);
    // coefficients of vectors past the live count are zero
    if (threadIdx.x >= nv && threadIdx.x < NV) sc[threadIdx.x] = 0.0;
    __syncthreads();
    return sc;
  };
  // d.dw is the same for every thread of the workgroup (the coefficient
  // reduction's barriers are reached by all of them either way)
  if (d.dw != nullptr)
    update_column<TX, NV, true>(gp((const TX*)d.Z + (size_t)j * d.vstride), gp(d.V),
                                gp(d.V + (size_t)(j + 1) * d.vstride), gp(d.pl.lo), gp(d.pl.di),
                                gp(d.pl.up), gp(d.dw), d.vstride, z_layout(d), d.ldx, d.nx, nv,
                                i, i < d.nx, k0, k1, coeffs, acc);
  else
    update_column<TX, NV, false>(gp((const TX*)d.Z + (size_t)j * d.vstride), gp(d.V),
                                 gp(d.V + (size_t)(j + 1) * d.vstride), gp(d.pl.lo), gp(d.pl.di),
                                 gp(d.pl.up), gp(d.dw), d.vstride, z_layout(d), d.ldx, d.nx, nv,
                                 i, i < d.nx, k0, k1, coeffs, acc);
  block_partials<NA, MVT>(acc, nv + 1, red, d.partials2, blk, d.mv_grid);
}

// ---------------------------------------------------------------------------
// finishing kernels, one workgroup per instance (blockIdx.x):
// FIN 1: residual r = b - M x -> ||b||, beta, v_0 scale, g, relres, stop flag;
//        j = start mode: 0 restart, 1 first residual, 2 first residual with
//        fallback to x = 0 when ||r|| >= ||b|| (then beta = ||b||)
// FIN 4: ||v_{j+1}|| -> Hessenberg column, Givens rotation, residual estimate,
//        and the Gram row of v_{j+1}
// (the Gram-Schmidt coefficients in between are reduced by the pass that
// consumes them)
// FIN 1 and FIN 4 publish the summary to host slot `slot` of the instance.
// ---------------------------------------------------------------------------
// FIN 4, the Givens step of inner iteration j.  Everything the serial part
// reads from the solver state (the Gram-Schmidt coefficients, the rotations
// so far, g, the basis scales, the columns of R for the back substitution,
// the summary) is loaded by the workgroup's threads together, with the
// partial sums in flight, and handed over through LDS: the one thread that
// then forms the column, the rotation and (when the cycle stops) y = R^{-1} g
// waits for no memory (a dependent chain of state loads and a column held in
// private memory had made this kernel several memory latencies long).
__device__ __forceinline__ void givens_step(const InstDesc& d, GState* st, GSummary* host, int j,
                                            int stop_iter, double rtol, int seq, double* out) {
  constexpr int LDH = MMAX + 1;              // column pitch of R
  constexpr int HPT = (MMAX * LDH + FT - 1) / FT;
  __shared__ double s_h1[NVMAX], s_h2[NVMAX], s_vs[NVMAX], s_g[MMAX + 1];
  __shared__ double s_cs[MMAX], s_sn[MMAX], s_col[NVMAX], s_y[MMAX];
  __shared__ double s_R[MMAX * LDH];
  const int t = threadIdx.x;
  double r_h1 = 0.0, r_h2 = 0.0, r_vs = 0.0, r_g = 0.0, r_cs = 0.0, r_sn = 0.0, r_R[HPT];
  if (t <= j) {
    r_h1 = st->h1[t];
    r_h2 = st->h2[t];
    r_vs = st->vscale[t];
    r_g = st->g[t];
  }
  if (t < j) {
    r_cs = st->cs[t];
    r_sn = st->sn[t];
  }
  const int nR = j * LDH;  // columns 0 .. j-1 of R
#pragma unroll
  for (int c = 0; c < HPT; ++c) {
    const int e = t + c * FT;
    r_R[c] = e < nR ? st->H[e] : 0.0;
  }
  const GSummary sm0 = st->sum;
  // the partial sums are read before the stop flag is looked at (a stopped
  // cycle's are stale and go unused), so the two loads overlap
  reduce_partials(d.partials2, d.mv_grid, j + 2, out);
  if (sm0.done) {
    // the cycle already stopped: still tell a polling host so
    if (t == 0) publish(host, sm0, seq);
    return;
  }
  if (t <= j) {
    s_h1[t] = r_h1;
    s_h2[t] = r_h2;
    s_vs[t] = r_vs;
    s_g[t] = r_g;
  }
  if (t < j) {
    s_cs[t] = r_cs;
    s_sn[t] = r_sn;
  }
#pragma unroll
  for (int c = 0; c < HPT; ++c) {
    const int e = t + c * FT;
    if (e < nR) s_R[e] = r_R[c];
  }
  __syncthreads();
  if (t != 0) return;
  GSummary sm = sm0;
  const double hn = sqrt(out[0]);
  double* col = s_col;
  for (int q = 0; q <= j; ++q) col[q] = s_h1[q] + s_h2[q];
  col[j + 1] = hn;
  for (int q = 0; q < j; ++q) {
    const double t0 = s_cs[q] * col[q] + s_sn[q] * col[q + 1];
    const double t1 = -s_sn[q] * col[q] + s_cs[q] * col[q + 1];
    col[q] = t0;
    col[q + 1] = t1;
  }
  const double den = hypot(col[j], col[j + 1]);
  double cs = 1.0, sn = 0.0;
  if (den > 0.0) {
    cs = col[j] / den;
    sn = col[j + 1] / den;
  }
  st->cs[j] = cs;
  st->sn[j] = sn;
  col[j] = den;
  for (int q = 0; q <= j; ++q) st->H[j * LDH + q] = col[q];
  const double gj = s_g[j];
  const double gnew = cs * gj, gnext = -sn * gj;
  st->g[j] = gnew;
  st->g[j + 1] = gnext;
  s_g[j] = gnew;
  const double est = fabs(gnext);
  sm.est = sm.bnorm > 0.0 ? est / sm.bnorm : 0.0;
  const double sn1 = hn > 0.0 ? 1.0 / hn : 0.0;
  st->vscale[j + 1] = sn1;
  double* grow = st->gram + (size_t)(j + 1) * NVMAX;
  for (int q = 0; q <= j; ++q) {
    const double gq = out[1 + q] * s_vs[q] * sn1;
    grow[q] = gq;
    st->gram[(size_t)q * NVMAX + j + 1] = gq;
  }
  grow[j + 1] = 1.0;
  sm.k = j + 1;
  const bool brk = !(hn > 1e-300 * (sm.beta > 0.0 ? sm.beta : 1.0));
  sm.breakdown = brk ? 1 : 0;
  if (est <= rtol * d.ctl->rscale * sm.bnorm || brk || j + 1 >= stop_iter) {
    sm.done = 1;
    // the cycle stops here: y = R^{-1} g for the cycle end (column j of R is
    // the one just formed, the others were loaded above)
    for (int q = j; q >= 0; --q) {
      double s = s_g[q];
      for (int r = q + 1; r <= j; ++r) s -= (r == j ? col[q] : s_R[r * LDH + q]) * s_y[r];
      const double dd = q == j ? col[j] : s_R[q * LDH + q];
      const double yq = dd != 0.0 ? s / dd : 0.0;
      s_y[q] = yq;
      st->y[q] = yq;
    }
  }
  st->sum.est = sm.est;
  st->sum.k = sm.k;
  st->sum.breakdown = sm.breakdown;
  st->sum.done = sm.done;
  publish(host, sm, seq);
}

template <int FIN>
__global__ __launch_bounds__(FT) void k_finish(const InstDesc* __restrict__ D, int j,
                                               int stop_iter, double rtol, int slot, int seq) {
  static_assert(FIN == 1 || FIN == 4, "finishing kernels: cycle start and Givens step");
  __shared__ double out[NVMAX];
  const InstDesc& d = D[blockIdx.x];
  GState* st = d.st;
  GSummary* host = d.host != nullptr ? d.host + slot : nullptr;
  if constexpr (FIN == 4) {
    givens_step(d, st, host, j, stop_iter, rtol, seq, out);
    return;
  }
  // FIN 1 with stop_iter != 0: speculative cycle start, only after a stopped cycle
  if (stop_iter != 0 && !st->sum.done) return;
  reduce_partials(d.partials, d.mv_grid, 2, out);
  if (threadIdx.x != 0) return;
  GSummary& sm = st->sum;
  // start of a cycle: beta = ||r||, v_0 = r / beta (stored unnormalised)
  sm.bnorm = sqrt(out[1]);
  double beta = sqrt(out[0]);
  if (j >= 1) sm.x0_rejected = 0;
  if (j == 2 && beta >= sm.bnorm && sm.bnorm > 0.0) {
    sm.x0_rejected = 1;
    beta = sm.bnorm;
  }
  sm.beta = beta;
  st->vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
  st->gram[0] = 1.0;
  st->g[0] = beta;
  for (int q = 1; q <= MMAX; ++q) st->g[q] = 0.0;
  sm.relres = sm.bnorm > 0.0 ? beta / sm.bnorm : 0.0;
  sm.breakdown = 0;
  sm.k = 0;
  // rtol < 0: the residual of an error estimate; every instance it is asked
  // for goes on to the preconditioner (no stop threshold)
  if (rtol < 0.0)
    sm.done = (d.ctl->est_skip || beta == 0.0) ? 1 : 0;
  else
    sm.done = (sm.relres <= rtol * d.ctl->rscale || beta == 0.0) ? 1 : 0;
  publish(host, sm, seq);
}

// Fallback start: an instance whose initial guess was rejected by the first
// residual's finishing kernel gets v_0 = b and x = 0.
__global__ __launch_bounds__(KT) void k_fallback(const InstDesc* __restrict__ D,
                                                 const int2* __restrict__ items,
                                                 const double* __restrict__ bb,
                                                 double* __restrict__ xb) {
  const int2 wi = work_item(items, blockIdx.x);
  const InstDesc& d = D[wi.x];
  if (!d.st->sum.x0_rejected) return;
  const double* __restrict__ b = bb + d.off;
  double* __restrict__ x = xb + d.off;
  double* __restrict__ v = d.V;
  // rows of the caller layout (pitch N_x) into V_0 (pitch ldx)
  for (int k = wi.y; k < d.nt; k += d.st_grid) {
    for (int i = threadIdx.x; i < d.nx; i += KT) {
      v[(size_t)k * d.ldx + i] = b[(size_t)k * d.nx + i];
      x[(size_t)k * d.nx + i] = 0.0;
    }
  }
}

// End of a cycle, one thread per instance: solve R y = g (k x k upper
// triangular) and publish the cycle's summary (k, estimate) to host slot.
__global__ void k_cycle_finish(const InstDesc* __restrict__ D, int ninst, int slot, int seq,
                               int guard) {
  const int inst = blockIdx.x * blockDim.x + threadIdx.x;
  if (inst >= ninst) return;
  const InstDesc& d = D[inst];
  GState* st = d.st;
  if (guard && !st->sum.done) return;  // speculative: the cycle has not stopped
  publish(d.host != nullptr ? d.host + slot : nullptr, st->sum, seq);
  const int k = st->sum.k;
  for (int q = k - 1; q >= 0; --q) {
    double s = st->g[q];
    for (int r = q + 1; r < k; ++r) s -= st->H[r * (MMAX + 1) + q] * st->y[r];
    const double dd = st->H[q * (MMAX + 1) + q];
    st->y[q] = dd != 0.0 ? s / dd : 0.0;
  }
}

// End of a cycle that started from x = 0, in one pass (y = R^{-1} g was formed
// by the Givens kernel that stopped the cycle; block 0 publishes the cycle
// summary to host slot `slot`): x = Z y,
// and the true residual r = b - M x with the partial sums of ||r||^2 and
// ||b||^2 for FIN 1; r itself goes to V_0 only when store_r is set (a restart
// starts from it; a caller that skips it forms r again before restarting,
// which saves a vector's write whenever the cycle converges).  The matvec's blocks (MVT columns x `rows` levels),
// walked UR_R levels at a time: every thread forms x at its column for the
// UR_R levels with all loads in flight, the values go through LDS so that
// each residual sees its neighbours' x, and an extra wavefront forms the two
// halo columns of the block; the level above the block is formed again from
// Z.  Nothing is read from the x being written, which is why a cycle that
// started from a nonzero x takes k_update and the residual matvec instead.
// guard: speculative launch, returns unless the cycle has stopped.
constexpr int UR_T = MVT + 64;  // MVT columns + one wavefront for the 2 halo columns
constexpr int UR_R = 8;         // time levels per step

template <typename TZ, int KB>
__global__ __launch_bounds__(UR_T) void k_update_residual(const InstDesc* __restrict__ D,
                                                          const int2* __restrict__ items,
                                                          const double* __restrict__ bo,
                                                          double* __restrict__ xo, int guard,
                                                          int store_r, int slot, int seq) {
  __shared__ double red[(UR_T / 64) * 2];
  __shared__ double ys[KB];
  __shared__ double xs[UR_R + 1][MVT + 2];  // level above the step + its UR_R levels
  const int2 wi = work_item(items, blockIdx.x);
  const InstDesc& d = D[wi.x];
  const GState* st = d.st;
  if (guard && !st->sum.done) return;
  const int kk = st->sum.k;
  if (threadIdx.x == 0 && wi.y == 0)
    publish(d.host != nullptr ? d.host + slot : nullptr, st->sum, seq);
  if (threadIdx.x < KB) ys[threadIdx.x] = (int)threadIdx.x < kk ? st->y[threadIdx.x] : 0.0;
  __syncthreads();
  const CN_G TZ* __restrict__ Z = gp((const TZ*)d.Z);
  const long long zs = d.vstride;
  const VecLayout zl = z_layout(d);
  const CN_G double* __restrict__ b = gp(bo + d.off);
  CN_G double* __restrict__ x = gp(xo + d.off);
  CN_G double* __restrict__ v0 = gp(d.V);
  const int nx = d.nx, ldx = d.ldx;
  const int blk = wi.y;
  const int cb = blk % d.mv_cols, rb = blk / d.mv_cols;
  const int k0 = rb * d.rows, k1 = min(d.nt, k0 + d.rows);
  const int t = threadIdx.x, i0 = cb * MVT;
  // this thread's column and LDS slot: MVT own columns, then the halo columns
  // i0 - 1 and i0 + MVT; the rest of the last wavefront idles
  int col = -1, sl = -1;
  if (t < MVT) {
    col = i0 + t;
    sl = t + 1;
  } else if (t == MVT) {
    col = i0 - 1;
    sl = 0;
  } else if (t == MVT + 1) {
    col = i0 + MVT;
    sl = MVT + 1;
  }
  const bool valid = col >= 0 && col < nx;
  const bool own = t < MVT && col < nx;
  const size_t zcol = valid ? zl.col(col) : 0, zrow = (size_t)zl.row;
  double lo = 0.0, di = 0.0, up = 0.0;
  if (own) {
    lo = gp(d.pl.lo)[col];
    di = gp(d.pl.di)[col];
    up = gp(d.pl.up)[col];
  }
  // x at levels kc .. kc + nr - 1 of this thread's column, loads in flight together
  // (vectors q >= kk re-read vector kk - 1 -- cache hits -- with weight 0: no
  // branch between the loads of a batch)
  constexpr int QG = KB < 8 ? KB : 8;  // vectors per batch of loads
  // x at UR_R levels from kc, every load of a batch in flight together
  auto form = [&](int kc, double (&xr)[UR_R]) {
#pragma unroll
    for (int r = 0; r < UR_R; ++r) xr[r] = 0.0;
    if (!valid || kk == 0) return;
#pragma unroll 1
    for (int q0 = 0; q0 < KB; q0 += QG) {
      if (q0 < kk) {
        TZ zv[QG][UR_R];
#pragma unroll
        for (int g = 0; g < QG; ++g) {
          const int q = q0 + g;
          const size_t zq = (size_t)(q < kk ? q : kk - 1) * zs + zcol + (size_t)kc * zrow;
#pragma unroll
          for (int r = 0; r < UR_R; ++r) zv[g][r] = Z[zq + (size_t)r * zrow];
        }
#pragma unroll
        for (int g = 0; g < QG; ++g)
#pragma unroll
          for (int r = 0; r < UR_R; ++r) xr[r] += ys[q0 + g] * (double)zv[g][r];
      }
    }
  };
  // x at one level (short steps: the last of a block, or the blocks of one
  // or a few levels that small instances have)
  auto form1 = [&](int k) -> double {
    double xv = 0.0;
    if (!valid || kk == 0) return xv;
    const size_t zk = (size_t)k * zrow + zcol;
#pragma unroll 1
    for (int q0 = 0; q0 < KB; q0 += QG) {
      if (q0 < kk) {
        TZ zv[QG];
#pragma unroll
        for (int g = 0; g < QG; ++g) {
          const int q = q0 + g;
          zv[g] = Z[(size_t)(q < kk ? q : kk - 1) * zs + zk];
        }
#pragma unroll
        for (int g = 0; g < QG; ++g) xv += ys[q0 + g] * (double)zv[g];
      }
    }
    return xv;
  };
  // residual at level k from the x of levels k-1 (LDS row ra) and k (row ra+1)
  auto resid = [&](int k, int ra, double bv, double (&acc)[2]) {
    const double pm = xs[ra][sl - 1], pc = xs[ra][sl], pp = xs[ra][sl + 1];
    const double cm = xs[ra + 1][sl - 1], cc = xs[ra + 1][sl], cp = xs[ra + 1][sl + 1];
    const double w = d.dw != nullptr ? gp(d.dw)[k] : 1.0;
    const double ax = lo * (cm + pm) + di * (cc + pc) + up * (cp + pp);
    const double rv = bv - ((cc - pc) - 0.5 * w * ax);
    if (store_r) v0[(size_t)k * ldx + col] = rv;
    acc[0] += rv * rv;
    acc[1] += bv * bv;
  };
  if (sl >= 0) xs[0][sl] = k0 > 0 ? form1(k0 - 1) : 0.0;
  double acc[2] = {0.0, 0.0};
  for (int kc = k0; kc < k1; kc += UR_R) {
    const int nr = min(UR_R, k1 - kc);
    if (nr == UR_R) {
      double xr[UR_R], bv[UR_R];
      form(kc, xr);
      if (own) {
#pragma unroll
        for (int r = 0; r < UR_R; ++r) bv[r] = b[(size_t)(kc + r) * nx + col];
      }
      if (sl >= 0) {
#pragma unroll
        for (int r = 0; r < UR_R; ++r) xs[1 + r][sl] = xr[r];
      }
      if (own) {
#pragma unroll
        for (int r = 0; r < UR_R; ++r) x[(size_t)(kc + r) * nx + col] = xr[r];
      }
      __syncthreads();
      if (own) {
#pragma unroll
        for (int r = 0; r < UR_R; ++r) resid(kc + r, r, bv[r], acc);
      }
    } else {
      for (int r = 0; r < nr; ++r) {
        const double xv = form1(kc + r);
        if (sl >= 0) xs[1 + r][sl] = xv;
        if (own) x[(size_t)(kc + r) * nx + col] = xv;
      }
      __syncthreads();
      if (own) {
        for (int r = 0; r < nr; ++r) resid(kc + r, r, b[(size_t)(kc + r) * nx + col], acc);
      }
    }
    __syncthreads();
    // the last level of this step is the level above the next one
    if (sl >= 0) xs[0][sl] = xs[nr][sl];
  }
  block_partials<2, UR_T>(acc, 2, red, d.partials, blk, d.mv_grid);
}

// x += sum_q y_q z_q (x = sum_q y_q z_q when the initial guess was zero)
template <typename TZ>
__global__ __launch_bounds__(KT) void k_update(const InstDesc* __restrict__ D,
                                               const int2* __restrict__ items,
                                               double* __restrict__ xb, int x_zero) {
  const int2 wi = work_item(items, blockIdx.x);
  const InstDesc& d = D[wi.x];
  const GState* st = d.st;
  if ((x_zero & 2) && !st->sum.done) return;  // speculative: the cycle has not stopped
  const int k = st->sum.k;
  if (k == 0 && !(x_zero & 1)) return;
  const double* y = st->y;
  const TZ* __restrict__ Z = (const TZ*)d.Z;
  double* __restrict__ x = xb + d.off;
  const long long zstride = d.vstride;
  const VecLayout zl = z_layout(d);
  // rows of the caller layout (pitch N_x); Z is tile-blocked
  for (int row = wi.y; row < d.nt; row += d.st_grid) {
    for (int i = threadIdx.x; i < d.nx; i += KT) {
      const size_t e = (size_t)row * d.nx + i, ez = zl.col(i) + (size_t)row * zl.row;
      double s = (x_zero & 1) ? 0.0 : x[e];
      int q = 0;
      for (; q + 4 <= k; q += 4) {
        s += y[q] * (double)Z[(size_t)q * zstride + ez] +
             y[q + 1] * (double)Z[(size_t)(q + 1) * zstride + ez] +
             y[q + 2] * (double)Z[(size_t)(q + 2) * zstride + ez] +
             y[q + 3] * (double)Z[(size_t)(q + 3) * zstride + ez];
      }
      for (; q < k; ++q) s += y[q] * (double)Z[(size_t)q * zstride + ez];
      x[e] = s;
    }
  }
}

// Number of instances still iterating, published with a sequence number
// taken from a device counter (so the launch has no per-call arguments).
__global__ __launch_bounds__(256) void k_batch_summary(const InstDesc* __restrict__ D,
                                                       int ninst, int* __restrict__ counter,
                                                       GSummary* __restrict__ host) {
  __shared__ int s_active[256];
  __shared__ double s_est[256];
  int act = 0;
  double est = 0.0;
  for (int i = threadIdx.x; i < ninst; i += 256) {
    const GSummary& sm = D[i].st->sum;
    if (!sm.done) act += 1;
    est = fmax(est, sm.est);
  }
  s_active[threadIdx.x] = act;
  s_est[threadIdx.x] = est;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s_active[threadIdx.x] += s_active[threadIdx.x + off];
      s_est[threadIdx.x] = fmax(s_est[threadIdx.x], s_est[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int seq = *counter + 1;
    *counter = seq;
    GSummary sm{};
    sm.k = s_active[0];
    sm.est = s_est[0];
    sm.done = s_active[0] == 0 ? 1 : 0;
    publish(host, sm, seq);
  }
}

// Error estimate of a stopped solve (error-controlled stopping).  With
// V_0 = r = b - M x and Z_0 = P_alpha^{-1} r / ||r|| (the cycle start with no
// stop threshold, then the preconditioner of iteration 0), the error
// e = M^{-1} r is estimated by ||r|| Z_0: P_alpha differs from M only in the
// alpha-scaled wrap-around block (eq. (3.1)), so P_alpha^{-1} M = I + O(alpha)
// and the estimate is within a relative O(alpha) of e.  Each workgroup folds
// max |Z_0| and max |x| over its rows into the instance's state (bit patterns
// of non-negative float64 values order like unsigned integers).
template <typename TZ>
__global__ __launch_bounds__(KT) void k_err_parts(const InstDesc* __restrict__ D,
                                                  const int2* __restrict__ items,
                                                  const double* __restrict__ xb) {
  __shared__ double red[2][KT / 64];
  const int2 wi = work_item(items, blockIdx.x);
  const InstDesc& d = D[wi.x];
  GState* st = d.st;
  if (st->sum.done) return;  // r = 0: nothing was applied, the estimate is 0
  const TZ* __restrict__ Z = (const TZ*)d.Z;
  const double* __restrict__ x = xb + d.off;
  const VecLayout zl = z_layout(d);
  double mz = 0.0, mx = 0.0;
  for (int row = wi.y; row < d.nt; row += d.st_grid) {
    for (int i = threadIdx.x; i < d.nx; i += KT) {
      mz = fmax(mz, fabs((double)Z[zl.col(i) + (size_t)row * zl.row]));
      mx = fmax(mx, fabs(x[(size_t)row * d.nx + i]));
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    mz = fmax(mz, __shfl_xor(mz, off, 64));
    mx = fmax(mx, __shfl_xor(mx, off, 64));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = mz;
    red[1][wave] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < KT / 64; ++w) {
      mz = fmax(mz, red[0][w]);
      mx = fmax(mx, red[1][w]);
    }
    atomicMax(&st->emax[0], (unsigned long long)__double_as_longlong(mz));
    atomicMax(&st->emax[1], (unsigned long long)__double_as_longlong(mx));
  }
}

// err = ||r|| max|Z_0| / max|x| (0 when r = 0, -1 when not asked for) into
// the summary slot; clears the maxima for the next estimate
__global__ __launch_bounds__(64) void k_err_publish(const InstDesc* __restrict__ D, int slot,
                                                    int seq) {
  if (threadIdx.x != 0) return;
  const InstDesc& d = D[blockIdx.x];
  GState* st = d.st;
  GSummary& sm = st->sum;
  const double mz = __longlong_as_double((long long)st->emax[0]);
  const double mx = __longlong_as_double((long long)st->emax[1]);
  // skipped instances publish -1 (no new estimate)
  double err = d.ctl->est_skip ? -1.0 : 0.0;
  if (!sm.done) err = mx > 0.0 ? sm.beta * mz / mx : (mz > 0.0 ? INFINITY : 0.0);
  sm.err = err;
  st->emax[0] = 0ull;
  st->emax[1] = 0ull;
  publish(d.host != nullptr ? d.host + slot : nullptr, sm, seq);
}

// b = xi + tau f, xi = [(I + (d_0/2) A~) u0; 0; ...]
__global__ __launch_bounds__(KT) void k_rhs(const double* __restrict__ lo,
                                            const double* __restrict__ di,
                                            const double* __restrict__ up,
                                            const double* __restrict__ dw, double tau,
                                            const double* __restrict__ u0,
                                            const double* __restrict__ f, double* __restrict__ b,
                                            int nx, long long n) {
  const long long e = (long long)blockIdx.x * KT + threadIdx.x;
  if (e >= n) return;
  double v = tau * f[e];
  if (e < nx) {
    const int i = (int)e;
    const double w = dw != nullptr ? dw[0] : 1.0;
    double ax = di[i] * u0[i];
    if (i > 0) ax += lo[i] * u0[i - 1];
    if (i < nx - 1) ax += up[i] * u0[i + 1];
    v += u0[i] + 0.5 * w * ax;
  }
  b[e] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int nv_bucket(int nv) {
  int b = 1;
  while (b < nv) b <<= 1;
  return b;
}

int matvec_rows(int nx, int nt) {
  const int cb = (nx + MVT - 1) / MVT;
  int rb = MV_KGRID / cb;
  if (rb < 1) rb = 1;
  if (rb > nt) rb = nt;
  return (nt + rb - 1) / rb;
}

int stream_grid(long long n) {
  long long g = (n + KT * 4 - 1) / (KT * 4);
  if (g > KGRID) g = KGRID;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_matvec_plain(const Launch& L, const Items& mv, const double* x, double* y,
                               hipStream_t s) {
  hipLaunchKernelGGL((k_matvec<double, 0, 2>), dim3(mv.n), dim3(MVT), 0, s, L.D, mv.it, 0, x,
                     nullptr, y, 0);
  return hipGetLastError();
}

hipError_t launch_residual(const Launch& L, const Items& mv, const Items& stv,
                           const double* b_base, double* x_base, int x_zero, double rtol,
                           int slot, int seq, hipStream_t s, int start, bool guard) {
  hipLaunchKernelGGL((k_matvec<double, 1, 2>), dim3(mv.n), dim3(MVT), 0, s, L.D, mv.it, 0,
                     (const double*)x_base, b_base, nullptr, (x_zero ? 1 : 0) | (guard ? 2 : 0));
  hipLaunchKernelGGL((k_finish<1>), dim3(L.ninst), dim3(FT), 0, s, L.D, start, guard ? 1 : 0,
                     rtol, slot, seq);
  if (start == 2)
    hipLaunchKernelGGL(k_fallback, dim3(stv.n), dim3(KT), 0, s, L.D, stv.it, b_base, x_base);
  return hipGetLastError();
}

hipError_t launch_arnoldi(const Launch& L, const Items& mv, const Items& stv, int j, int stop_iter,
                          double rtol, int slot, int seq, hipStream_t s, int passes,
                          bool finish) {
  const int bk = nv_bucket(j + 1);
  switch (bk) {
#define AR(NVB)                                                                               \
  case NVB:                                                                                   \
    if (passes & 1) {                                                                         \
      if (L.zf)                                                                               \
        hipLaunchKernelGGL((k_matvec<float, 2, NVB>), dim3(mv.n), dim3(MVT), 0, s, L.D, mv.it,\
                           j, (const float*)nullptr, nullptr, nullptr, 0);                    \
      else                                                                                    \
        hipLaunchKernelGGL((k_matvec<double, 2, NVB>), dim3(mv.n), dim3(MVT), 0, s, L.D,      \
                           mv.it, j, (const double*)nullptr, nullptr, nullptr, 0);            \
    }                                                                                         \
    if (passes & 4) {                                                                         \
      if (L.zf)                                                                               \
        hipLaunchKernelGGL((k_cgs_update<float, NVB>), dim3(mv.n), dim3(MVT), 0, s, L.D,      \
                           mv.it, j);                                                         \
      else                                                                                    \
        hipLaunchKernelGGL((k_cgs_update<double, NVB>), dim3(mv.n), dim3(MVT), 0, s, L.D,     \
                           mv.it, j);                                                         \
      if (finish)                                                                             \
        hipLaunchKernelGGL((k_finish<4>), dim3(L.ninst), dim3(FT), 0, s, L.D, j, stop_iter,  \
                           rtol, slot, seq);                                                  \
    }                                                                                         \
    break;
    AR(1) AR(2) AR(4) AR(8) AR(16) AR(32) AR(64)
#undef AR
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cycle_end(const Launch& L, const Items& stv, double* x_base, int x_zero,
                            int slot, int seq, hipStream_t s, bool guard) {
  hipLaunchKernelGGL(k_cycle_finish, dim3((L.ninst + 63) / 64), dim3(64), 0, s, L.D, L.ninst,
                     slot, seq, guard ? 1 : 0);
  x_zero = (x_zero ? 1 : 0) | (guard ? 2 : 0);
  if (L.zf)
    hipLaunchKernelGGL((k_update<float>), dim3(stv.n), dim3(KT), 0, s, L.D, stv.it, x_base,
                       x_zero);
  else
    hipLaunchKernelGGL((k_update<double>), dim3(stv.n), dim3(KT), 0, s, L.D, stv.it, x_base,
                       x_zero);
  return hipGetLastError();
}

hipError_t launch_cycle_end_zero(const Launch& L, const Items& mv, int kmax,
                                 const double* b_base, double* x_base, double rtol, int slot_fin,
                                 int seq_fin, int slot_res, int seq_res, hipStream_t s,
                                 bool guard, bool store_r) {
  const int bk = nv_bucket(kmax < 1 ? 1 : kmax);
  switch (bk) {
#define UR(KB)                                                                                \
  case KB:                                                                                    \
    if (L.zf)                                                                                 \
      hipLaunchKernelGGL((k_update_residual<float, KB>), dim3(mv.n), dim3(UR_T), 0, s, L.D,   \
                         mv.it, b_base, x_base, guard ? 1 : 0, store_r ? 1 : 0, slot_fin,   \
                         seq_fin);                                                            \
    else                                                                                      \
      hipLaunchKernelGGL((k_update_residual<double, KB>), dim3(mv.n), dim3(UR_T), 0, s, L.D,  \
                         mv.it, b_base, x_base, guard ? 1 : 0, store_r ? 1 : 0, slot_fin,   \
                         seq_fin);                                                            \
    break;
    UR(1) UR(2) UR(4) UR(8) UR(16) UR(32) UR(64)
#undef UR
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL((k_finish<1>), dim3(L.ninst), dim3(FT), 0, s, L.D, 0, guard ? 1 : 0, rtol,
                     slot_res, seq_res);
  return hipGetLastError();
}

// Start of an error estimate from the residual the last cycle end of a batch
// left in V_0 (its norm beta and the scale of v_0 in the state): every
// instance asked for goes on to the preconditioner.
__global__ __launch_bounds__(256) void k_err_begin(const InstDesc* __restrict__ D, int ninst) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ninst) return;
  const InstDesc& d = D[i];
  GSummary& sm = d.st->sum;
  sm.done = (d.ctl->est_skip || sm.beta == 0.0 || sm.bnorm == 0.0) ? 1 : 0;
}

hipError_t launch_err_begin(const Launch& L, hipStream_t s) {
  hipLaunchKernelGGL(k_err_begin, dim3((L.ninst + 255) / 256), dim3(256), 0, s, L.D, L.ninst);
  return hipGetLastError();
}

hipError_t launch_err_estimate(const Launch& L, const Items& stv, const double* x_base, int slot,
                               int seq, hipStream_t s) {
  if (L.zf)
    hipLaunchKernelGGL((k_err_parts<float>), dim3(stv.n), dim3(KT), 0, s, L.D, stv.it, x_base);
  else
    hipLaunchKernelGGL((k_err_parts<double>), dim3(stv.n), dim3(KT), 0, s, L.D, stv.it, x_base);
  hipLaunchKernelGGL(k_err_publish, dim3(L.ninst), dim3(64), 0, s, L.D, slot, seq);
  return hipGetLastError();
}

hipError_t launch_batch_summary(const Launch& L, int* counter, GSummary* host, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_summary, dim3(1), dim3(256), 0, s, L.D, L.ninst, counter, host);
  return hipGetLastError();
}

hipError_t launch_rhs(const double* lo, const double* di, const double* up, const double* dw,
                      double tau, const double* u0, const double* f, double* b, int nx,
                      long long n, hipStream_t s) {
  const long long grid = (n + KT - 1) / KT;
  hipLaunchKernelGGL(k_rhs, dim3((unsigned)grid), dim3(KT), 0, s, lo, di, up, dw, tau, u0, f, b,
                     nx, n);
  return hipGetLastError();
}

}  // namespace cn
