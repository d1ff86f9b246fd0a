// Krylov kernels of the right-preconditioned GMRES(m) solve on gfx950:
//   * the all-at-once CN matvec (block form of Sec. 3.2), plain, as a
//     residual b - M x, and fused with the first Gram-Schmidt dot pass;
//   * the two remaining CGS2 passes (dots against the stored basis, update,
//     norm) -- the basis is stored unnormalised with a float64 scale per
//     vector, so normalisation never costs a pass;
//   * the Givens / least-squares update, done by the last workgroup of the
//     final pass (no host round-trip inside a cycle);
//   * x += Z y and the right-hand side b = xi + tau f (eq. (2.2)).
// Reductions are deterministic: every workgroup of a streaming pass writes
// its partial sums; a one-workgroup finishing kernel adds them in a fixed
// order and updates the solver state.  Stream order makes the partials
// visible, so no workgroup issues a device-scope fence (on a multi-XCD part
// such a fence writes back and invalidates the XCD's L2).
#include <math.h>

#include "cn_internal.hpp"

namespace cn {

constexpr int KT = 256;  // threads per workgroup of the streaming kernels

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-reduce NV accumulators into partials[q*nblk + blk] (fixed order).
template <int NV>
__device__ __forceinline__ void block_partials(const double (&acc)[NV], int nv, double* red,
                                               double* partials, int blk) {
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
    for (int w = 0; w < KT / 64; ++w) s += red[w * NV + tid];
    partials[(size_t)tid * gridDim.x + blk] = s;
  }
}

// Sum partials[q*nblk + b] over b for q < nv into out[q]: wave w handles
// q = w, w + 16, ...; lane l adds b = l, l + 64, ... then the wave adds its
// lanes.  The order is fixed, so the result is bitwise reproducible.
constexpr int FT = 1024;  // threads of a finishing kernel
constexpr int FCHUNK = 32;  // partials per lane loaded back to back
__device__ __forceinline__ void reduce_partials(const double* __restrict__ partials, int nblk,
                                                int nv, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q = wv; q < nv; q += FT / 64) {
    const double* p = partials + (size_t)q * nblk;
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

// Publish the summary to the host slot: fields first, then (after a
// system-scope fence) the sequence number the host polls for.
__device__ __forceinline__ void publish(GSummary* host, const GSummary& sm, int seq) {
  if (host == nullptr) return;
  host->bnorm = sm.bnorm;
  host->beta = sm.beta;
  host->est = sm.est;
  host->relres = sm.relres;
  host->k = sm.k;
  host->done = sm.done;
  host->breakdown = sm.breakdown;
  __threadfence_system();
  *(volatile int*)&host->seq = seq;
}

// ---------------------------------------------------------------------------
// matvec: y = M x (MODE 0), y = b - M x with norms (MODE 1),
//         y = M x with dots against V_0..V_{nv-1} (MODE 2, first CGS pass)
// ---------------------------------------------------------------------------
template <typename TX, int MODE, int NV>
__global__ __launch_bounds__(KT) void k_matvec(KArgs a, const TX* __restrict__ x,
                                               const double* __restrict__ b,
                                               double* __restrict__ y) {
  __shared__ double red[(KT / 64) * (NV > 2 ? NV : 2)];
  GState* st = a.st;
  if (MODE == 2 && st->sum.done) return;
  const int nx = a.nx;
  const int col_blocks = (nx + KT - 1) / KT;
  const int blk = blockIdx.x;
  const int cb = blk % col_blocks, rb = blk / col_blocks;
  const int i = cb * KT + threadIdx.x;
  const int k0 = rb * a.rows, k1 = min(a.nt, k0 + a.rows);
  double acc[NV > 2 ? NV : 2];
#pragma unroll
  for (int q = 0; q < (NV > 2 ? NV : 2); ++q) acc[q] = 0.0;
  if (i < nx) {
    const double lo = a.lo[i], di = a.di[i], up = a.up[i];
    const bool hl = i > 0, hr = i < nx - 1;
    double pm = 0.0, pc = 0.0, pp = 0.0;  // previous level at i-1, i, i+1
    if (k0 > 0 && x != nullptr) {
      const TX* xr = x + (size_t)(k0 - 1) * nx;
      pc = (double)xr[i];
      if (hl) pm = (double)xr[i - 1];
      if (hr) pp = (double)xr[i + 1];
    }
    for (int k = k0; k < k1; ++k) {
      double cm = 0.0, cc = 0.0, cp = 0.0;
      const size_t off = (size_t)k * nx;
      if (x != nullptr) {
        cc = (double)x[off + i];
        if (hl) cm = (double)x[off + i - 1];
        if (hr) cp = (double)x[off + i + 1];
      }
      const double w = a.dw != nullptr ? a.dw[k] : 1.0;
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
      y[off + i] = yv;
      if (MODE == 2) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
          if (q < a.nv) acc[q] += a.V[(size_t)q * a.vstride + off + i] * yv;
      }
      pm = cm;
      pc = cc;
      pp = cp;
    }
  }
  if (MODE == 0) return;
  const int nacc = MODE == 1 ? 2 : a.nv;
  block_partials<(NV > 2 ? NV : 2)>(acc, nacc, red, a.partials, blk);
}

// ---------------------------------------------------------------------------
// CGS2 second pass: h2 = V^T (w - V c1)
// ---------------------------------------------------------------------------
template <int NV>
__global__ __launch_bounds__(KT) void k_cgs_pass1(KArgs a, const double* __restrict__ w) {
  __shared__ double red[(KT / 64) * NV];
  GState* st = a.st;
  if (st->sum.done) return;
  double c[NV], acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    c[q] = q < a.nv ? st->c1[q] : 0.0;
    acc[q] = 0.0;
  }
  const long long stride = (long long)gridDim.x * KT;
  for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < a.n; e += stride) {
    double vq[NV];
    double wv = w[e];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      vq[q] = q < a.nv ? a.V[(size_t)q * a.vstride + e] : 0.0;
      wv -= c[q] * vq[q];
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] += vq[q] * wv;
  }
  block_partials<NV>(acc, a.nv, red, a.partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// CGS2 update: v_{j+1} = w - V (c1 + c2), its norm, the Hessenberg column,
// Givens rotations and the residual estimate (last workgroup).
// ---------------------------------------------------------------------------
template <int NV>
__global__ __launch_bounds__(KT) void k_cgs_pass2(KArgs a, const double* __restrict__ w,
                                                  double* __restrict__ vout) {
  __shared__ double red[(KT / 64) * 2];
  GState* st = a.st;
  if (st->sum.done) return;
  double c[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) c[q] = q < a.nv ? st->c1[q] + st->c2[q] : 0.0;
  double acc[2] = {0.0, 0.0};
  const long long stride = (long long)gridDim.x * KT;
  for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < a.n; e += stride) {
    double wv = w[e];
#pragma unroll
    for (int q = 0; q < NV; ++q)
      if (q < a.nv) wv -= c[q] * a.V[(size_t)q * a.vstride + e];
    vout[e] = wv;
    acc[0] += wv * wv;
  }
  block_partials<2>(acc, 1, red, a.partials, blockIdx.x);
}

// ---------------------------------------------------------------------------
// finishing kernels (one workgroup): fixed-order sums of the partials
// ---------------------------------------------------------------------------
// FIN 1: residual r = b - M x -> ||b||, beta, v_0 scale, g, relres, stop flag
// FIN 2: first Gram-Schmidt dots -> h1, c1
// FIN 3: second Gram-Schmidt dots -> h2, c2
// FIN 4: ||v_{j+1}|| -> Hessenberg column, Givens rotation, residual estimate
template <int FIN>
__global__ __launch_bounds__(FT) void k_finish(GState* __restrict__ st,
                                               const double* __restrict__ partials, int nblk,
                                               int nv, int j, int stop_iter, double rtol,
                                               GSummary* __restrict__ host, int seq) {
  __shared__ double out[NVMAX];
  if (FIN != 1 && st->sum.done) {
    // the cycle already stopped: still tell a polling host so
    if (FIN == 4 && threadIdx.x == 0) publish(host, st->sum, seq);
    return;
  }
  const int nq = FIN == 1 ? 2 : (FIN == 4 ? 1 : nv);
  reduce_partials(partials, nblk, nq, out);
  if (threadIdx.x != 0) return;
  GSummary& sm = st->sum;
  if (FIN == 1) {
    // start of a cycle: beta = ||r||, v_0 = r / beta (stored unnormalised)
    sm.bnorm = sqrt(out[1]);
    const double beta = sqrt(out[0]);
    sm.beta = beta;
    st->vscale[0] = beta > 0.0 ? 1.0 / beta : 0.0;
    st->g[0] = beta;
    for (int q = 1; q <= MMAX; ++q) st->g[q] = 0.0;
    sm.relres = sm.bnorm > 0.0 ? beta / sm.bnorm : 0.0;
    sm.breakdown = 0;
    sm.k = 0;
    sm.done = (sm.relres <= rtol || beta == 0.0) ? 1 : 0;
    publish(host, sm, seq);
  } else if (FIN == 2 || FIN == 3) {
    double* hh = FIN == 2 ? st->h1 : st->h2;
    double* cc = FIN == 2 ? st->c1 : st->c2;
    for (int q = 0; q < nv; ++q) {
      const double h = out[q] * st->vscale[q];
      hh[q] = h;
      cc[q] = h * st->vscale[q];
    }
  } else {
    const double hn = sqrt(out[0]);
    double col[MMAX + 1];
    for (int q = 0; q <= j; ++q) col[q] = st->h1[q] + st->h2[q];
    col[j + 1] = hn;
    for (int q = 0; q < j; ++q) {
      const double t0 = st->cs[q] * col[q] + st->sn[q] * col[q + 1];
      const double t1 = -st->sn[q] * col[q] + st->cs[q] * col[q + 1];
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
    for (int q = 0; q <= j; ++q) st->H[j * (MMAX + 1) + q] = col[q];
    const double gj = st->g[j];
    st->g[j] = cs * gj;
    st->g[j + 1] = -sn * gj;
    const double est = fabs(st->g[j + 1]);
    sm.est = sm.bnorm > 0.0 ? est / sm.bnorm : 0.0;
    st->vscale[j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    sm.k = j + 1;
    const bool brk = !(hn > 1e-300 * (sm.beta > 0.0 ? sm.beta : 1.0));
    sm.breakdown = brk ? 1 : 0;
    if (est <= rtol * sm.bnorm || brk || j + 1 >= stop_iter) sm.done = 1;
    publish(host, sm, seq);
  }
}

// End of a cycle: solve the k x k triangular system R y = g; copy the
// cycle's summary (k, estimate) to the host slot.
__global__ void k_cycle_finish(GState* st, GSummary* host, int seq) {
  if (threadIdx.x != 0) return;
  publish(host, st->sum, seq);
  const int k = st->sum.k;
  for (int q = k - 1; q >= 0; --q) {
    double s = st->g[q];
    for (int r = q + 1; r < k; ++r) s -= st->H[r * (MMAX + 1) + q] * st->y[r];
    const double d = st->H[q * (MMAX + 1) + q];
    st->y[q] = d != 0.0 ? s / d : 0.0;
  }
}

// x += sum_q y_q z_q
template <typename TZ>
__global__ __launch_bounds__(KT) void k_update(const GState* __restrict__ st,
                                               const TZ* __restrict__ Z, long long zstride,
                                               double* __restrict__ x, long long n,
                                               int x_zero) {
  const int k = st->sum.k;
  const double* y = st->y;
  const long long stride = (long long)gridDim.x * KT;
  for (long long e = (long long)blockIdx.x * KT + threadIdx.x; e < n; e += stride) {
    double s = x_zero ? 0.0 : x[e];
    int q = 0;
    for (; q + 4 <= k; q += 4) {
      s += y[q] * (double)Z[(size_t)q * zstride + e] +
           y[q + 1] * (double)Z[(size_t)(q + 1) * zstride + e] +
           y[q + 2] * (double)Z[(size_t)(q + 2) * zstride + e] +
           y[q + 3] * (double)Z[(size_t)(q + 3) * zstride + e];
    }
    for (; q < k; ++q) s += y[q] * (double)Z[(size_t)q * zstride + e];
    x[e] = s;
  }
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
  const int cb = (nx + KT - 1) / KT;
  int rb = KGRID / cb;
  if (rb < 1) rb = 1;
  if (rb > nt) rb = nt;
  return (nt + rb - 1) / rb;
}

int matvec_grid(int nx, int nt) {
  const int rows = matvec_rows(nx, nt);
  return ((nx + KT - 1) / KT) * ((nt + rows - 1) / rows);
}

int stream_grid(long long n) {
  long long g = (n + KT * 4 - 1) / (KT * 4);
  if (g > KGRID) g = KGRID;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_matvec(const KArgs& a, const void* x, int x_is_float, const double* b,
                         double* y, int mode, hipStream_t s, double rtol, GSummary* host,
                         int seq, bool finish) {
  const int grid = ((a.nx + KT - 1) / KT) * ((a.nt + a.rows - 1) / a.rows);
  if (mode == 0) {
    if (x_is_float)
      hipLaunchKernelGGL((k_matvec<float, 0, 2>), dim3(grid), dim3(KT), 0, s, a, (const float*)x, b, y);
    else
      hipLaunchKernelGGL((k_matvec<double, 0, 2>), dim3(grid), dim3(KT), 0, s, a, (const double*)x, b, y);
    return hipGetLastError();
  }
  if (mode == 1) {
    hipLaunchKernelGGL((k_matvec<double, 1, 2>), dim3(grid), dim3(KT), 0, s, a, (const double*)x, b, y);
    hipLaunchKernelGGL((k_finish<1>), dim3(1), dim3(FT), 0, s, a.st, a.partials, grid, 2, 0, 0,
                       rtol, host, seq);
    return hipGetLastError();
  }
  const int bk = nv_bucket(a.nv);
#define MV(NVB)                                                                                    \
  case NVB:                                                                                        \
    if (x_is_float)                                                                                \
      hipLaunchKernelGGL((k_matvec<float, 2, NVB>), dim3(grid), dim3(KT), 0, s, a, (const float*)x, b, y); \
    else                                                                                           \
      hipLaunchKernelGGL((k_matvec<double, 2, NVB>), dim3(grid), dim3(KT), 0, s, a, (const double*)x, b, y); \
    break;
  switch (bk) {
    MV(1) MV(2) MV(4) MV(8) MV(16) MV(32) MV(64)
    default:
      return hipErrorInvalidValue;
  }
#undef MV
  if (finish)
    hipLaunchKernelGGL((k_finish<2>), dim3(1), dim3(FT), 0, s, a.st, a.partials, grid, a.nv, 0,
                       0, rtol, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_cgs(const KArgs& a, const double* w, double* vout, int j, int stop_iter,
                      hipStream_t s, int passes, double rtol, GSummary* host, int seq,
                      bool finish) {
  const int grid = stream_grid(a.n);
  const int bk = nv_bucket(a.nv);
  if ((passes & 2) && vout == nullptr) return hipErrorInvalidValue;
  switch (bk) {
#define CG(NVB)                                                                            \
  case NVB:                                                                                \
    if (passes & 1) {                                                                      \
      hipLaunchKernelGGL((k_cgs_pass1<NVB>), dim3(grid), dim3(KT), 0, s, a, w);            \
      if (finish)                                                                          \
        hipLaunchKernelGGL((k_finish<3>), dim3(1), dim3(FT), 0, s, a.st, a.partials, grid, \
                           a.nv, j, stop_iter, rtol, nullptr, 0);                          \
    }                                                                                      \
    if (passes & 2) {                                                                      \
      hipLaunchKernelGGL((k_cgs_pass2<NVB>), dim3(grid), dim3(KT), 0, s, a, w, vout);      \
      if (finish)                                                                          \
        hipLaunchKernelGGL((k_finish<4>), dim3(1), dim3(FT), 0, s, a.st, a.partials, grid, \
                           a.nv, j, stop_iter, rtol, host, seq);                           \
    }                                                                                      \
    break;
    CG(1) CG(2) CG(4) CG(8) CG(16) CG(32) CG(64)
#undef CG
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finish_update(GState* st, const void* Z, int z_is_float, long long zstride,
                                double* x, long long n, int x_zero, GSummary* host, int seq,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_finish, dim3(1), dim3(64), 0, s, st, host, seq);
  const int grid = stream_grid(n);
  if (z_is_float)
    hipLaunchKernelGGL((k_update<float>), dim3(grid), dim3(KT), 0, s, st, (const float*)Z, zstride, x, n, x_zero);
  else
    hipLaunchKernelGGL((k_update<double>), dim3(grid), dim3(KT), 0, s, st, (const double*)Z, zstride, x, n, x_zero);
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
