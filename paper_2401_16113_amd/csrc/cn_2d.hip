// The all-at-once CN system and the alpha-circulant preconditioner for a
// 2D spatial operator (the setting of Sec. 5): a nine-point stencil A on an
// N_x x N_y grid, x fastest.
//
// Step (a) and (c) of eq. (3.2) run per tile of B consecutive grid points:
// the alpha-weighted levels of two points form one complex sequence, one
// LDS Stockham FFT per sequence, and the N_t/2 + 1 non-redundant modes of
// every point (Remark 1) go to a spectrum laid out by frequency,
// S[j][i].  Step (b) solves, per frequency, (mu_j I - A~) y = S[j] / lambda_2
// with the band LU factors computed once at creation (half-bandwidth
// N_x + 1 in the x-fastest ordering, no pivoting): one wavefront per
// frequency keeps the vector in LDS and runs the forward and backward
// substitutions one row at a time, each lane updating one entry of the band,
// with the next rows' band coefficients requested ahead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "cn_aao2d.h"
#include "cn_internal.hpp"

namespace cn_twod {
using namespace cn;

constexpr int kMaxNx = 127;
constexpr int kMaxPts = 8192;
constexpr int kMaxLog2N = 10;
constexpr int BANDT = 64;       // one wavefront per frequency line of the substitution
constexpr int FACT = 256;       // threads per frequency of the factorisation

__device__ __forceinline__ Cx<double> czero() { return Cx<double>{0.0, 0.0}; }

// y = M x (MODE 0) or b = xi + tau f (MODE 1, x = u0, aux = f) over every
// space-time element; half_tau = tau/2.  (M x)^k = (x^k - x^{k-1}) -
// (A~/2)(x^k + x^{k-1}) with x^{-1} = 0 (Sec. 3.2).
template <int MODE>
__global__ __launch_bounds__(256) void k2d_matvec(const double* __restrict__ st, int nx, int ny,
                                                  int nt, double tau, const double* __restrict__ x,
                                                  const double* __restrict__ aux,
                                                  double* __restrict__ y) {
  const int npts = nx * ny;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)nt * npts) return;
  const int k = (int)(e / npts), i = (int)(e % npts);
  const int iy = i / nx, ix = i % nx;
  if constexpr (MODE == 0) {
    const double* xk = x + (size_t)k * npts;
    const double* xp = k > 0 ? xk - npts : nullptr;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const int jy = iy + q / 3 - 1, jx = ix + q % 3 - 1;
      if (jy < 0 || jy >= ny || jx < 0 || jx >= nx) continue;
      const int m = jy * nx + jx;
      const double s = xk[m] + (xp != nullptr ? xp[m] : 0.0);
      acc += st[(size_t)q * npts + i] * s;
    }
    const double d = xk[i] - (xp != nullptr ? xp[i] : 0.0);
    y[e] = d - 0.5 * tau * acc;
  } else {
    double v = tau * aux[e];
    if (k == 0) {
      double acc = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const int jy = iy + q / 3 - 1, jx = ix + q % 3 - 1;
        if (jy < 0 || jy >= ny || jx < 0 || jx >= nx) continue;
        acc += st[(size_t)q * npts + i] * x[jy * nx + jx];
      }
      v += x[i] + 0.5 * tau * acc;
    }
    y[e] = v;
  }
}

// Step (a): tile of B grid points, alpha-weighted, time FFT, the N/2 + 1
// modes of every point to S[j][i].
template <int LOG2N>
__global__ __launch_bounds__((PcDefault<double, LOG2N>::T)) void k2d_forward(
    const double* __restrict__ v, int npts, const double* __restrict__ wfw,
    const Cx<double>* __restrict__ tw, Cx<double>* __restrict__ S) {
  using D = PcDefault<double, LOG2N>;
  using Cfg = PcCfg<double, LOG2N, D::B, D::T>;
  constexpr int N = Cfg::N, B = Cfg::B, T = Cfg::T, F = N / 2 + 1;
  __shared__ Cx<double> lds[Cfg::LDS_ELEMS];
  __shared__ Cx<double> ltw[Cfg::TWN];
  const int tid = threadIdx.x, i0 = blockIdx.x * B, ncols = min(B, npts - i0);
  TwStage<double, Cfg::TWN, T, Cfg::TWPT> tws;
  tws.fetch(gp(tw));
  double* ldsr = reinterpret_cast<double*>(lds);
  for (int e = tid; e < N * B; e += T) {
    const int k = e / B, b = e % B;
    ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] =
        b < ncols ? v[(size_t)k * npts + i0 + b] * wfw[k] : 0.0;
  }
  tws.store(ltw);
  __syncthreads();
  fft_tile<Cfg, double, LOG2N, false>(lds, ltw, tw, tid);
  __syncthreads();
  // X_{2c} = (Z_j + conj Z_{N-j})/2, X_{2c+1} = (Z_j - conj Z_{N-j})/(2i)
  for (int e = tid; e < F * B; e += T) {
    const int j = e / B, b = e % B;
    if (b >= ncols) continue;
    const Cx<double> z = lds[lidx<N>(b >> 1, j)];
    const Cx<double> zc = conj(lds[lidx<N>(b >> 1, (N - j) & (N - 1))]);
    const Cx<double> sum = z + zc, dif = z - zc;
    S[(size_t)j * npts + i0 + b] =
        (b & 1) ? Cx<double>{0.5 * dif.y, -0.5 * dif.x} : Cx<double>{0.5 * sum.x, 0.5 * sum.y};
  }
}

// Step (c): the modes of the tile's points back into complex sequences,
// inverse FFT, times alpha^{-k/N}/N.
template <int LOG2N>
__global__ __launch_bounds__((PcDefault<double, LOG2N>::T)) void k2d_inverse(
    const Cx<double>* __restrict__ S, int npts, const double* __restrict__ winv,
    const Cx<double>* __restrict__ tw, double* __restrict__ z) {
  using D = PcDefault<double, LOG2N>;
  using Cfg = PcCfg<double, LOG2N, D::B, D::T>;
  constexpr int N = Cfg::N, B = Cfg::B, T = Cfg::T, F = N / 2 + 1, NSEQ = Cfg::NSEQ;
  __shared__ Cx<double> lds[Cfg::LDS_ELEMS];
  __shared__ Cx<double> ltw[Cfg::TWN];
  const int tid = threadIdx.x, i0 = blockIdx.x * B, ncols = min(B, npts - i0);
  TwStage<double, Cfg::TWN, T, Cfg::TWPT> tws;
  tws.fetch(gp(tw));
  // Z'_j = X_{2c} + i X_{2c+1}, Z'_{N-j} = conj(X_{2c}) + i conj(X_{2c+1});
  // the modes j = 0 and N/2 are real
  for (int e = tid; e < F * NSEQ; e += T) {
    const int j = e / NSEQ, c = e % NSEQ;
    const Cx<double> xa = 2 * c < ncols ? S[(size_t)j * npts + i0 + 2 * c] : czero();
    const Cx<double> xb = 2 * c + 1 < ncols ? S[(size_t)j * npts + i0 + 2 * c + 1] : czero();
    if (j == 0 || 2 * j == N) {
      lds[lidx<N>(c, j)] = Cx<double>{xa.x, xb.x};
    } else {
      lds[lidx<N>(c, j)] = Cx<double>{xa.x - xb.y, xa.y + xb.x};
      lds[lidx<N>(c, N - j)] = Cx<double>{xa.x + xb.y, xb.x - xa.y};
    }
  }
  tws.store(ltw);
  __syncthreads();
  fft_tile<Cfg, double, LOG2N, true>(lds, ltw, tw, tid);
  __syncthreads();
  const double* ldsr = reinterpret_cast<const double*>(lds);
  for (int e = tid; e < N * B; e += T) {
    const int k = e / B, b = e % B;
    if (b < ncols) z[(size_t)k * npts + i0 + b] = ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] * winv[k];
  }
}

// Set-up, one workgroup per frequency j: the band of G = mu_j I - tau A in
// row storage G[i][c - i + p] (c in [i - p, i + p]), eliminated in place
// without pivoting, then split into column-ordered factors for the
// substitutions: Lc[k][t] = L[k+1+t][k], Uc[k][t] = U[k-1-t][k],
// dinv[k] = 1/U[k][k].  A pivot below 1e-12 of its row's scale (|mu| plus
// the row's absolute stencil sum) sets *err.
__global__ __launch_bounds__(FACT) void k2d_factor(const double* __restrict__ st, int nx, int ny,
                                                   double tau, const Cx<double>* __restrict__ mu,
                                                   int p, Cx<double>* __restrict__ Gall,
                                                   Cx<double>* __restrict__ Lc,
                                                   Cx<double>* __restrict__ Uc,
                                                   Cx<double>* __restrict__ dinv,
                                                   int* __restrict__ err) {
  const int npts = nx * ny, w = 2 * p + 1;
  const int j = blockIdx.x, tid = threadIdx.x;
  Cx<double>* G = Gall + (size_t)j * npts * w;
  const Cx<double> m = mu[j];
  for (size_t e = tid; e < (size_t)npts * w; e += FACT) G[e] = czero();
  __syncthreads();
  for (int i = tid; i < npts; i += FACT) {
    const int iy = i / nx, ix = i % nx;
    for (int q = 0; q < 9; ++q) {
      const int jy = iy + q / 3 - 1, jx = ix + q % 3 - 1;
      if (jy < 0 || jy >= ny || jx < 0 || jx >= nx) continue;
      const int c = jy * nx + jx;
      Cx<double>& g = G[(size_t)i * w + (c - i + p)];
      g.x -= tau * st[(size_t)q * npts + i];
    }
    Cx<double>& d = G[(size_t)i * w + p];
    d.x += m.x;
    d.y += m.y;
  }
  __syncthreads();
  __shared__ Cx<double> s_inv;
  for (int k = 0; k < npts; ++k) {
    if (tid == 0) {
      const Cx<double> piv = G[(size_t)k * w + p];
      // the scale of row k of mu I - tau A
      double scale = sqrt(m.x * m.x + m.y * m.y);
      for (int q = 0; q < 9; ++q) scale += tau * fabs(st[(size_t)q * npts + k]);
      const double mag = sqrt(piv.x * piv.x + piv.y * piv.y);
      if (!(mag > 1e-12 * scale) || !isfinite(mag)) atomicOr(err, 1);
      s_inv = crcp(piv);
    }
    __syncthreads();
    const Cx<double> inv = s_inv;
    // multipliers of the rows below (column k)
    for (int t = tid; t < p; t += FACT) {
      const int i = k + 1 + t;
      if (i < npts) {
        Cx<double>& l = G[(size_t)i * w + (p - 1 - t)];
        l = l * inv;
      }
    }
    __syncthreads();
    // rank-1 update of the trailing p x p window
    for (int e = tid; e < p * p; e += FACT) {
      const int a = e / p, b = e % p;
      const int i = k + 1 + a, c = k + 1 + b;
      if (i >= npts || c >= npts) continue;
      const Cx<double> l = G[(size_t)i * w + (p - 1 - a)];
      const Cx<double> u = G[(size_t)k * w + (p + 1 + b)];
      Cx<double>& g = G[(size_t)i * w + (b - a + p)];
      g = g - l * u;
    }
    __syncthreads();
  }
  Cx<double>* L = Lc + (size_t)j * npts * p;
  Cx<double>* U = Uc + (size_t)j * npts * p;
  for (size_t e = tid; e < (size_t)npts * p; e += FACT) {
    const int k = (int)(e / p), t = (int)(e % p);
    const int il = k + 1 + t, iu = k - 1 - t;
    L[e] = il < npts ? G[(size_t)il * w + (p - 1 - t)] : czero();
    U[e] = iu >= 0 ? G[(size_t)iu * w + (p + 1 + t)] : czero();
  }
  for (int k = tid; k < npts; k += FACT) dinv[(size_t)j * npts + k] = crcp(G[(size_t)k * w + p]);
}

// Step (b): one wavefront per frequency j, S[j] <- (1/lambda_2) (L U)^{-1} S[j].
// Blocked substitution: a step takes RB consecutive rows of a sweep.  Lane u
// of the wavefront (u < RB + p, in NCH chunks of 64 lanes) holds row k0 + u
// of the forward sweep (k0 - u of the backward one); for r = 0..RB-1 the
// final value of the step's row r is broadcast from lane r and every lane
// subtracts its coefficient times it.  The coefficient of (u, r) is entry
// u - r - 1 of the factor column of row r (stored by column, see
// k2d_factor; zero outside the band), so a chunk's lanes read consecutive
// entries.  The rows cost one LDS read and one write per step instead of per
// row; the coefficients of the next NB steps are in flight.
constexpr int RB = 8;  // rows per step

__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ Cx<double> lane_value(Cx<double> v, int lane) {
  return Cx<double>{lane_value(v.x, lane), lane_value(v.y, lane)};
}

template <int P64>
__global__ __launch_bounds__(BANDT) void k2d_band(const Cx<double>* __restrict__ Lc,
                                                  const Cx<double>* __restrict__ Uc,
                                                  const Cx<double>* __restrict__ dinv,
                                                  const Cx<double>* __restrict__ il2, int npts, int p,
                                                  Cx<double>* __restrict__ S) {
  constexpr int NCH = (RB + 64 * P64 + 63) / 64;  // lane chunks: RB + p rows
  constexpr int NB = P64 == 1 ? 3 : 2;            // steps of coefficients in flight
  extern __shared__ Cx<double> y[];
  const int j = blockIdx.x, t = threadIdx.x;
  Cx<double>* s = S + (size_t)j * npts;
  const Cx<double>* L = Lc + (size_t)j * npts * p;
  const Cx<double>* U = Uc + (size_t)j * npts * p;
  const Cx<double>* di = dinv + (size_t)j * npts;
  for (int i = t; i < npts; i += BANDT) y[i] = s[i];
  __syncthreads();
  // coefficient of lane u for the step row r whose factor column is col
  auto coef = [&](const Cx<double>* base, int col, int u, int r) -> Cx<double> {
    const int e = u - r - 1;
    return (col >= 0 && col < npts && e >= 0 && e < p) ? base[(size_t)col * p + e] : czero();
  };
  // forward: unit lower L, column k holds L[k+1+e][k]
  {
    Cx<double> cb[NB][RB][NCH];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < NCH; ++c) cb[q][r][c] = coef(L, q * RB + r, t + 64 * c, r);
    for (int kb = 0; kb < npts; kb += NB * RB) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k0 = kb + q * RB;
        if (k0 < npts) {
          Cx<double> yu[NCH];
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int u = t + 64 * c, i = k0 + u;
            yu[c] = (u < RB + p && i < npts) ? y[i] : czero();
          }
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            if (k0 + r < npts) {
              const Cx<double> yr = lane_value(yu[0], r);
#pragma unroll
              for (int c = 0; c < NCH; ++c) yu[c] = yu[c] - cb[q][r][c] * yr;
            }
          }
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int u = t + 64 * c, i = k0 + u;
            if (u < RB + p && i < npts) y[i] = yu[c];
          }
        }
        // the coefficients of the step NB ahead
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int c = 0; c < NCH; ++c) cb[q][r][c] = coef(L, k0 + NB * RB + r, t + 64 * c, r);
        __syncthreads();
      }
    }
  }
  // backward: row k scaled by 1/U[k][k]; column k holds U[k-1-e][k]
  {
    Cx<double> cb[NB][RB][NCH];
    Cx<double> db[NB];  // lane r < RB: 1/U of the step's row r
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int k0 = npts - 1 - q * RB;
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < NCH; ++c) cb[q][r][c] = coef(U, k0 - r, t + 64 * c, r);
      db[q] = (t < RB && k0 - t >= 0) ? di[k0 - t] : czero();
    }
    for (int kb = npts - 1; kb >= 0; kb -= NB * RB) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k0 = kb - q * RB;
        if (k0 >= 0) {
          Cx<double> yu[NCH];
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int u = t + 64 * c, i = k0 - u;
            yu[c] = (u < RB + p && i >= 0) ? y[i] : czero();
          }
#pragma unroll
          for (int r = 0; r < RB; ++r) {
            if (k0 - r >= 0) {
              if (t == r) yu[0] = yu[0] * db[q];
              const Cx<double> yr = lane_value(yu[0], r);
#pragma unroll
              for (int c = 0; c < NCH; ++c) yu[c] = yu[c] - cb[q][r][c] * yr;
            }
          }
#pragma unroll
          for (int c = 0; c < NCH; ++c) {
            const int u = t + 64 * c, i = k0 - u;
            if (u < RB + p && i >= 0) y[i] = yu[c];
          }
        }
        const int kn = k0 - NB * RB;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
          for (int c = 0; c < NCH; ++c) cb[q][r][c] = coef(U, kn - r, t + 64 * c, r);
        db[q] = (t < RB && kn - t >= 0) ? di[kn - t] : czero();
        __syncthreads();
      }
    }
  }
  const Cx<double> sc = il2[j];
  for (int i = t; i < npts; i += BANDT) s[i] = y[i] * sc;
}

// ---------------------------------------------------------------------------
// GMRES for the 2D system: right-preconditioned flexible GMRES(m) with
// classical Gram-Schmidt applied twice (two passes of dots and updates), the
// Hessenberg column, Givens rotations and y on the device (one thread); the
// host waits once per inner iteration for the residual estimate.
// ---------------------------------------------------------------------------
constexpr int KB = 256;     // threads per block of the streaming kernels
constexpr int NBLK = 512;   // blocks of a dot pass (partial sums per dot)

struct GmState {
  double H[(MMAX + 1) * MMAX];  // column j at H[j (MMAX+1)]
  double cs[MMAX], sn[MMAX];
  double g[MMAX + 1];
  double y[MMAX];
  double h[NVMAX], h2[NVMAX];   // the two Gram-Schmidt passes
  double nrm2, bsq;             // ||w||^2 after both passes, ||b||^2
  double bnorm, scale;          // ||b||, 1/||v|| of the vector being normalised
  double unit;                  // 1.0 (the coefficient of r = b - 1 * (M x))
};

struct GmSummary {
  double relres;  // ||r|| / ||b|| at a cycle start, or the estimate after an iteration
  double hnext;   // h_{j+1,j}
  double bnorm;   // ||b|| (cycle start)
};

// partials[q NBLK + blk] = <V_q, w> over the block's slice, q < gridDim.y
__global__ __launch_bounds__(KB) void k2d_dots(const double* __restrict__ V, long long stride,
                                               const double* __restrict__ w, long long n,
                                               double* __restrict__ part) {
  __shared__ double red[KB / 64];
  const int q = blockIdx.y, blk = blockIdx.x, t = threadIdx.x;
  const double* v = V + (size_t)q * stride;
  double acc = 0.0;
  for (long long i = (long long)blk * KB + t; i < n; i += (long long)NBLK * KB) acc += v[i] * w[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((t & 63) == 0) red[t >> 6] = acc;
  __syncthreads();
  if (t == 0) {
    double s = 0.0;
    for (int u = 0; u < KB / 64; ++u) s += red[u];
    part[(size_t)q * NBLK + blk] = s;
  }
}

// out[q] = sum of the NBLK partials of dot q, in a fixed order
__global__ __launch_bounds__(64) void k2d_sum(const double* __restrict__ part, int nv,
                                              double* __restrict__ out) {
  const int q = blockIdx.x * 64 + threadIdx.x;
  if (q >= nv) return;
  double s = 0.0;
  for (int b = 0; b < NBLK; ++b) s += part[(size_t)q * NBLK + b];
  out[q] = s;
}

// out = base + sign * sum_q c[q] V_q (c on the device; base may be out)
__global__ __launch_bounds__(KB) void k2d_combine(double* __restrict__ out, const double* base,
                                                  const double* __restrict__ V, long long stride,
                                                  int nv, const double* __restrict__ c,
                                                  double sign, long long n) {
  const long long i = (long long)blockIdx.x * KB + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int q = 0; q < nv; ++q) s += c[q] * V[(size_t)q * stride + i];
  out[i] = (base != nullptr ? base[i] : 0.0) + sign * s;
}

// v = w * (*scale)
__global__ __launch_bounds__(KB) void k2d_scale(double* __restrict__ v, const double* __restrict__ w,
                                                const double* __restrict__ scale, long long n) {
  const long long i = (long long)blockIdx.x * KB + threadIdx.x;
  if (i < n) v[i] = w[i] * *scale;
}

// cycle start: beta = sqrt(nrm2), g = beta e_1, scale = 1/beta, relres
__global__ void k2d_gm_start(GmState* st, GmSummary* sum) {
  if (threadIdx.x != 0) return;
  const double beta = sqrt(st->nrm2);
  st->bnorm = sqrt(st->bsq);
  for (int q = 0; q <= MMAX; ++q) st->g[q] = 0.0;
  st->g[0] = beta;
  st->scale = beta > 0.0 ? 1.0 / beta : 0.0;
  sum->relres = st->bnorm > 0.0 ? beta / st->bnorm : 0.0;
  sum->hnext = beta;
  sum->bnorm = st->bnorm;
}

// column j of the Hessenberg matrix (h + h2, ||w||), the earlier rotations
// applied to it, the new rotation, g and the residual estimate
__global__ void k2d_gm_column(GmState* st, int j, GmSummary* sum) {
  if (threadIdx.x != 0) return;
  double* col = st->H + (size_t)j * (MMAX + 1);
  for (int q = 0; q <= j; ++q) col[q] = st->h[q] + st->h2[q];
  const double hn = sqrt(st->nrm2);
  col[j + 1] = hn;
  for (int q = 0; q < j; ++q) {
    const double a = col[q], b = col[q + 1];
    col[q] = st->cs[q] * a + st->sn[q] * b;
    col[q + 1] = -st->sn[q] * a + st->cs[q] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double r = hypot(a, b);
  const double c = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? b / r : 0.0;
  st->cs[j] = c;
  st->sn[j] = sn;
  col[j] = r;
  col[j + 1] = 0.0;
  st->g[j + 1] = -sn * st->g[j];
  st->g[j] = c * st->g[j];
  st->scale = hn > 0.0 ? 1.0 / hn : 0.0;
  sum->relres = st->bnorm > 0.0 ? fabs(st->g[j + 1]) / st->bnorm : 0.0;
  sum->hnext = hn;
}

// y = R^{-1} g over the first k columns
__global__ void k2d_gm_y(GmState* st, int k) {
  if (threadIdx.x != 0) return;
  for (int q = k - 1; q >= 0; --q) {
    double s = st->g[q];
    for (int r = q + 1; r < k; ++r) s -= st->H[(size_t)r * (MMAX + 1) + q] * st->y[r];
    const double d = st->H[(size_t)q * (MMAX + 1) + q];
    st->y[q] = d != 0.0 ? s / d : 0.0;
  }
}

}  // namespace cn_twod

using namespace cn_twod;

static thread_local std::string g_err2d;

struct cn2d {
  int nx = 0, ny = 0, npts = 0, nt = 0, log2n = 0, F = 0, p = 0;
  double T = 0, tau = 0, alpha = 0;
  hipStream_t stream = nullptr;
  double *st = nullptr, *wfw = nullptr, *winv = nullptr;
  Cx<double> *tw = nullptr, *tw2 = nullptr, *mu = nullptr, *il2 = nullptr;
  Cx<double> *Lc = nullptr, *Uc = nullptr, *dinv = nullptr, *S = nullptr;
  // GMRES workspace (m_max > 0): basis V (m_max + 1 vectors), Z (m_max), w,
  // dot partials, the device state and the host-mapped summary
  int m_max = 0;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *part = nullptr;
  GmState* gs = nullptr;
  GmSummary* hsum = nullptr;
  GmSummary* hsum_dev = nullptr;
  std::vector<void*> allocs;
};

static cn_status fail2d(cn_status s, const std::string& msg) {
  g_err2d = msg;
  return s;
}

static void release2d(cn2d* h) {
  if (h == nullptr) return;
  (void)hipStreamSynchronize(h->stream);
  for (void* q : h->allocs) (void)hipFree(q);
  if (h->hsum != nullptr) (void)hipHostFree(h->hsum);
  delete h;
}

template <typename P>
static hipError_t alloc2d(cn2d* h, P** p, size_t bytes) {
  void* q = nullptr;
  const hipError_t e = hipMalloc(&q, bytes);
  if (e == hipSuccess) {
    h->allocs.push_back(q);
    *p = (P*)q;
  }
  return e;
}

// launch helpers over log2(N_t)
template <int L = 0>
static hipError_t launch_transform(bool inverse, int log2n, int tiles, const cn2d* h,
                                   const double* v, double* z) {
  if constexpr (L > kMaxLog2N) {
    return hipErrorInvalidValue;
  } else {
    if (log2n != L) return launch_transform<L + 1>(inverse, log2n, tiles, h, v, z);
    using Cfg = PcCfg<double, L, PcDefault<double, L>::B, PcDefault<double, L>::T>;
    const Cx<double>* tw = Cfg::TWMODE == 3 ? h->tw2 : h->tw;
    if (!inverse)
      hipLaunchKernelGGL(k2d_forward<L>, dim3(tiles), dim3(Cfg::T), 0, h->stream, v, h->npts,
                         h->wfw, tw, h->S);
    else
      hipLaunchKernelGGL(k2d_inverse<L>, dim3(tiles), dim3(Cfg::T), 0, h->stream, h->S, h->npts,
                         h->winv, tw, z);
    return hipGetLastError();
  }
}

template <int L = 0>
static int tile_points(int log2n) {
  if constexpr (L > kMaxLog2N) {
    return 0;
  } else {
    if (log2n == L) return PcDefault<double, L>::B;
    return tile_points<L + 1>(log2n);
  }
}

#define TRY2(x)                                                                     \
  do {                                                                              \
    const hipError_t e_ = (x);                                                      \
    if (e_ != hipSuccess) {                                                         \
      const cn_status s_ = fail2d(e_ == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP,  \
                                  std::string(#x) + ": " + hipGetErrorString(e_));  \
      release2d(h);                                                                 \
      return s_;                                                                    \
    }                                                                               \
  } while (0)

extern "C" {

const char* cn2d_last_error(void) { return g_err2d.c_str(); }

cn_status cn2d_create(const cn2d_problem* p, cn2d** out) {
  if (out == nullptr) return fail2d(CN_EINVAL, "out is NULL");
  *out = nullptr;
  if (p == nullptr || p->stencil == nullptr) return fail2d(CN_EINVAL, "problem or stencil is NULL");
  if (p->nx < 1 || p->nx > kMaxNx) return fail2d(CN_EINVAL, "nx must be in [1, 127]");
  if (p->ny < 1 || (long long)p->nx * p->ny > kMaxPts)
    return fail2d(CN_EINVAL, "ny must be >= 1 with nx * ny <= 8192");
  if (p->nt < 1 || p->nt > (1 << kMaxLog2N) || (p->nt & (p->nt - 1)) != 0)
    return fail2d(CN_EINVAL, "nt must be a power of two in [1, 1024]");
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail2d(CN_EINVAL, "T must be finite and > 0");
  if (!(p->alpha > 0.0 && p->alpha < 1.0)) return fail2d(CN_EINVAL, "alpha must satisfy 0 < alpha < 1");
  if (p->m_max < 0 || p->m_max > MMAX) return fail2d(CN_EINVAL, "m_max must be in [0, 64]");
  cn2d* h = new cn2d();
  h->nx = p->nx;
  h->ny = p->ny;
  h->npts = p->nx * p->ny;
  h->nt = p->nt;
  while ((1 << h->log2n) < h->nt) ++h->log2n;
  h->F = h->nt / 2 + 1;
  h->p = h->ny > 1 ? h->nx + 1 : 1;
  h->T = p->T;
  h->tau = p->T / p->nt;
  h->alpha = p->alpha;
  h->stream = (hipStream_t)p->stream;
  h->m_max = p->m_max;
  const int nt = h->nt, F = h->F, npts = h->npts, pb = h->p;
  const size_t nvec = (size_t)nt * npts;
  const size_t band = (size_t)F * npts * pb * sizeof(Cx<double>);
  const size_t gband = (size_t)F * npts * (2 * pb + 1) * sizeof(Cx<double>);
  {
    size_t freeb = 0, totalb = 0;
    TRY2(hipMemGetInfo(&freeb, &totalb));
    const size_t need = 2 * band + gband + 2 * (size_t)F * npts * sizeof(Cx<double>) +
                        (size_t)(2 * h->m_max + 2) * nvec * sizeof(double);
    if (need > freeb) {
      release2d(h);
      return fail2d(CN_ENOMEM, "band factors need " + std::to_string(need) + " bytes");
    }
  }
  // time tables (long double on the host): alpha^{+-k/N}, the DFT
  // twiddles, and the eigenvalues of the alpha-circulants derived from
  // their diagonalisation: lambda_1 = 1 - q w^j, lambda_2 = (1 + q w^j)/2,
  // q = alpha^{1/N}, w = exp(-2 pi i/N) (Sec. 3.1)
  const long double la = logl((long double)h->alpha), pi = acosl(-1.0L);
  std::vector<double> wfw(nt), winv(nt);
  std::vector<Cx<double>> tw(nt), mu(F), il2(F);
  for (int k = 0; k < nt; ++k) {
    wfw[k] = (double)expl(la * k / nt);
    winv[k] = (double)(expl(-la * k / nt) / nt);
    tw[k] = Cx<double>{(double)cosl(2 * pi * k / nt), (double)-sinl(2 * pi * k / nt)};
  }
  const int wsl = std::min(nt, 64), wsh = nt / wsl;
  std::vector<Cx<double>> tw2(wsl + wsh);
  for (int e = 0; e < wsl + wsh; ++e) tw2[e] = tw[e < wsl ? e : (e - wsl) * wsl];
  const long double q = expl(la / nt);
  for (int j = 0; j < F; ++j) {
    const long double wr = j == 0 ? 1.0L : (2 * j == nt ? -1.0L : cosl(2 * pi * j / nt));
    const long double wi = (j == 0 || 2 * j == nt) ? 0.0L : -sinl(2 * pi * j / nt);
    const long double l1r = 1 - q * wr, l1i = -q * wi;
    const long double l2r = (1 + q * wr) / 2, l2i = q * wi / 2;
    const long double d2 = l2r * l2r + l2i * l2i;
    mu[j] = Cx<double>{(double)((l1r * l2r + l1i * l2i) / d2), (double)((l1i * l2r - l1r * l2i) / d2)};
    il2[j] = Cx<double>{(double)(l2r / d2), (double)(-l2i / d2)};
  }
  TRY2(alloc2d(h, &h->st, (size_t)9 * npts * sizeof(double)));
  TRY2(hipMemcpyAsync(h->st, p->stencil, (size_t)9 * npts * sizeof(double), hipMemcpyDeviceToDevice,
                      h->stream));
  TRY2(alloc2d(h, &h->wfw, nt * sizeof(double)));
  TRY2(alloc2d(h, &h->winv, nt * sizeof(double)));
  TRY2(alloc2d(h, &h->tw, nt * sizeof(Cx<double>)));
  TRY2(alloc2d(h, &h->tw2, tw2.size() * sizeof(Cx<double>)));
  TRY2(alloc2d(h, &h->mu, F * sizeof(Cx<double>)));
  TRY2(alloc2d(h, &h->il2, F * sizeof(Cx<double>)));
  TRY2(hipMemcpy(h->wfw, wfw.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  TRY2(hipMemcpy(h->winv, winv.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  TRY2(hipMemcpy(h->tw, tw.data(), nt * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY2(hipMemcpy(h->tw2, tw2.data(), tw2.size() * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY2(hipMemcpy(h->mu, mu.data(), F * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY2(hipMemcpy(h->il2, il2.data(), F * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY2(alloc2d(h, &h->Lc, band));
  TRY2(alloc2d(h, &h->Uc, band));
  TRY2(alloc2d(h, &h->dinv, (size_t)F * npts * sizeof(Cx<double>)));
  TRY2(alloc2d(h, &h->S, (size_t)F * npts * sizeof(Cx<double>)));
  if (h->m_max > 0) {
    TRY2(alloc2d(h, &h->V, (size_t)(h->m_max + 1) * nvec * sizeof(double)));
    TRY2(alloc2d(h, &h->Z, (size_t)h->m_max * nvec * sizeof(double)));
    TRY2(alloc2d(h, &h->w, nvec * sizeof(double)));
    TRY2(alloc2d(h, &h->part, (size_t)NVMAX * NBLK * sizeof(double)));
    TRY2(alloc2d(h, &h->gs, sizeof(GmState)));
    {
      GmState g0{};
      g0.unit = 1.0;
      TRY2(hipMemcpy(h->gs, &g0, sizeof(GmState), hipMemcpyHostToDevice));
    }
    TRY2(hipHostMalloc((void**)&h->hsum, sizeof(GmSummary), hipHostMallocCoherent | hipHostMallocMapped));
    TRY2(hipHostGetDevicePointer((void**)&h->hsum_dev, h->hsum, 0));
  }
  // the band of every frequency during the factorisation (freed after)
  Cx<double>* G = nullptr;
  int* err = nullptr;
  TRY2(hipMalloc((void**)&G, gband));
  hipError_t e = hipMalloc((void**)&err, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(err, 0, sizeof(int), h->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k2d_factor, dim3(F), dim3(FACT), 0, h->stream, h->st, h->nx, h->ny, h->tau,
                       h->mu, pb, G, h->Lc, h->Uc, h->dinv, err);
    e = hipGetLastError();
  }
  int herr = 0;
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) e = hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost);
  (void)hipFree(G);
  if (err != nullptr) (void)hipFree(err);
  if (e != hipSuccess) {
    release2d(h);
    return fail2d(CN_EHIP, std::string("factorisation: ") + hipGetErrorString(e));
  }
  if (herr != 0) {
    release2d(h);
    return fail2d(CN_ESINGULAR, "a shifted system has a vanishing pivot (not diagonally dominant?)");
  }
  // the substitution keeps one frequency's vector in LDS: allow the largest
  // (the attribute is per kernel, shared by every handle)
  const int lds_max = kMaxPts * (int)sizeof(Cx<double>);
  e = hipFuncSetAttribute((const void*)k2d_band<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k2d_band<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
  if (e != hipSuccess) {
    release2d(h);
    return fail2d(CN_EHIP, std::string("LDS size: ") + hipGetErrorString(e));
  }
  *out = h;
  return CN_OK;
}

cn_status cn2d_destroy(cn2d* h) {
  if (h == nullptr) return fail2d(CN_EINVAL, "handle is NULL");
  release2d(h);
  return CN_OK;
}

cn_status cn2d_matvec(cn2d* h, const double* x, double* y) {
  if (h == nullptr || x == nullptr || y == nullptr) return fail2d(CN_EINVAL, "NULL argument");
  const long long n = (long long)h->nt * h->npts;
  if (x < y + n && y < x + n) return fail2d(CN_EINVAL, "x and y overlap");
  hipLaunchKernelGGL(k2d_matvec<0>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     h->st, h->nx, h->ny, h->nt, h->tau, x, nullptr, y);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CN_OK : fail2d(CN_EHIP, hipGetErrorString(e));
}

cn_status cn2d_rhs(cn2d* h, const double* u0, const double* f, double* b) {
  if (h == nullptr || u0 == nullptr || f == nullptr || b == nullptr)
    return fail2d(CN_EINVAL, "NULL argument");
  const long long n = (long long)h->nt * h->npts;
  hipLaunchKernelGGL(k2d_matvec<1>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream,
                     h->st, h->nx, h->ny, h->nt, h->tau, u0, f, b);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CN_OK : fail2d(CN_EHIP, hipGetErrorString(e));
}

cn_status cn2d_pc_apply(cn2d* h, const double* v, double* z) {
  if (h == nullptr || v == nullptr || z == nullptr) return fail2d(CN_EINVAL, "NULL argument");
  const int B = tile_points(h->log2n);
  const int tiles = (h->npts + B - 1) / B;
  hipError_t e = launch_transform(false, h->log2n, tiles, h, v, nullptr);
  if (e == hipSuccess) {
    const size_t lds = (size_t)h->npts * sizeof(Cx<double>);
    if (h->p <= BANDT)
      hipLaunchKernelGGL(k2d_band<1>, dim3(h->F), dim3(BANDT), lds, h->stream, h->Lc, h->Uc, h->dinv,
                         h->il2, h->npts, h->p, h->S);
    else
      hipLaunchKernelGGL(k2d_band<2>, dim3(h->F), dim3(BANDT), lds, h->stream, h->Lc, h->Uc, h->dinv,
                         h->il2, h->npts, h->p, h->S);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_transform(true, h->log2n, tiles, h, nullptr, z);
  return e == hipSuccess ? CN_OK : fail2d(CN_EHIP, hipGetErrorString(e));
}

}  // extern "C"

// dots of V_0..V_{nv-1} with w into out[0..nv) (device)
static hipError_t dots2d(cn2d* h, const double* V, int nv, const double* w, double* out) {
  const long long n = (long long)h->nt * h->npts;
  hipLaunchKernelGGL(k2d_dots, dim3(NBLK, nv), dim3(KB), 0, h->stream, V, n, w, n, h->part);
  hipLaunchKernelGGL(k2d_sum, dim3((nv + 63) / 64), dim3(64), 0, h->stream, h->part, nv, out);
  return hipGetLastError();
}

static hipError_t combine2d(cn2d* h, double* out, const double* base, const double* V, int nv,
                            const double* c, double sign) {
  const long long n = (long long)h->nt * h->npts;
  hipLaunchKernelGGL(k2d_combine, dim3((unsigned)((n + KB - 1) / KB)), dim3(KB), 0, h->stream, out,
                     base, V, n, nv, c, sign, n);
  return hipGetLastError();
}

// r = b - M x into V_0 (x = 0: r = b), ||r||^2 and the cycle start
static hipError_t restart2d(cn2d* h, const double* b, const double* x, bool x_zero) {
  const long long n = (long long)h->nt * h->npts;
  hipError_t e = hipSuccess;
  if (x_zero) {
    e = hipMemcpyAsync(h->V, b, n * sizeof(double), hipMemcpyDeviceToDevice, h->stream);
  } else {
    hipLaunchKernelGGL(k2d_matvec<0>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, h->st,
                       h->nx, h->ny, h->nt, h->tau, x, nullptr, h->w);
    e = hipGetLastError();
    // V_0 = b - w
    if (e == hipSuccess) e = combine2d(h, h->V, b, h->w, 1, &h->gs->unit, -1.0);
  }
  if (e == hipSuccess) e = dots2d(h, h->V, 1, h->V, &h->gs->nrm2);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k2d_gm_start, dim3(1), dim3(1), 0, h->stream, h->gs, h->hsum_dev);
    e = hipGetLastError();
  }
  return e;
}

extern "C" cn_status cn2d_gmres_solve(cn2d* h, const double* b, double* x, const cn_gmres_opts* opts,
                                      cn_gmres_info* info) {
  if (h == nullptr || b == nullptr || x == nullptr || opts == nullptr)
    return fail2d(CN_EINVAL, "NULL argument");
  if (h->m_max < 1) return fail2d(CN_EINVAL, "the handle has no solver workspace (m_max = 0)");
  if (opts->m < 1 || opts->m > h->m_max) return fail2d(CN_EINVAL, "opts->m must be in [1, m_max]");
  if (opts->max_iters < 1) return fail2d(CN_EINVAL, "opts->max_iters must be >= 1");
  if (opts->use_x0 < 0 || opts->use_x0 > 1) return fail2d(CN_EINVAL, "opts->use_x0 must be 0 or 1");
  if (opts->flags != 0 || opts->err_tol != 0.0)
    return fail2d(CN_EINVAL, "flags and err_tol are not supported for 2D operators");
  if (!(opts->rtol >= 0.0) || !std::isfinite(opts->rtol))
    return fail2d(CN_EINVAL, "opts->rtol must be finite and >= 0");
  const long long n = (long long)h->nt * h->npts;
  if (b < x + n && x < b + n) return fail2d(CN_EINVAL, "b and x overlap");
  const auto wall0 = std::chrono::steady_clock::now();
  hipStream_t s = h->stream;
  GmState* gs = h->gs;
  const double rtol = opts->rtol;
  cn_gmres_info in{};
  in.err_est = -1.0;
#define CK(expr)                                                        \
  do {                                                                  \
    const hipError_t e_ = (expr);                                       \
    if (e_ != hipSuccess) return fail2d(CN_EHIP, hipGetErrorString(e_)); \
  } while (0)
  CK(dots2d(h, b, 1, b, &gs->bsq));
  bool x_zero = opts->use_x0 == 0;
  if (x_zero) CK(hipMemsetAsync(x, 0, n * sizeof(double), s));
  CK(restart2d(h, b, x, x_zero));
  in.matvecs = x_zero ? 0 : 1;
  CK(hipStreamSynchronize(s));
  double relres = h->hsum->relres;
  if (h->hsum->bnorm == 0.0) {
    // b = 0: the solution is x = 0, whatever the guess
    if (!x_zero) CK(hipMemsetAsync(x, 0, n * sizeof(double), s));
    CK(hipStreamSynchronize(s));
    relres = 0.0;
  }
  int done = 0;
  while (!(relres <= rtol) && done < opts->max_iters) {
    hipLaunchKernelGGL(k2d_scale, dim3((unsigned)((n + KB - 1) / KB)), dim3(KB), 0, s, h->V, h->V,
                       &gs->scale, n);
    CK(hipGetLastError());
    const int m_eff = std::min(opts->m, opts->max_iters - done);
    int k = 0;
    for (int j = 0; j < m_eff; ++j) {
      double* vj = h->V + (size_t)j * n;
      double* zj = h->Z + (size_t)j * n;
      const cn_status ps = cn2d_pc_apply(h, vj, zj);
      if (ps != CN_OK) return ps;
      hipLaunchKernelGGL(k2d_matvec<0>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h->st,
                         h->nx, h->ny, h->nt, h->tau, zj, nullptr, h->w);
      CK(hipGetLastError());
      // two passes of classical Gram-Schmidt against V_0..V_j
      CK(dots2d(h, h->V, j + 1, h->w, gs->h));
      CK(combine2d(h, h->w, h->w, h->V, j + 1, gs->h, -1.0));
      CK(dots2d(h, h->V, j + 1, h->w, gs->h2));
      CK(combine2d(h, h->w, h->w, h->V, j + 1, gs->h2, -1.0));
      CK(dots2d(h, h->w, 1, h->w, &gs->nrm2));
      hipLaunchKernelGGL(k2d_gm_column, dim3(1), dim3(1), 0, s, gs, j, h->hsum_dev);
      CK(hipGetLastError());
      hipLaunchKernelGGL(k2d_scale, dim3((unsigned)((n + KB - 1) / KB)), dim3(KB), 0, s,
                         h->V + (size_t)(j + 1) * n, h->w, &gs->scale, n);
      CK(hipGetLastError());
      CK(hipStreamSynchronize(s));
      k = j + 1;
      ++in.iters;
      ++in.pc_applies;
      ++in.matvecs;
      in.relres_est = h->hsum->relres;
      if (in.relres_est <= rtol || h->hsum->hnext == 0.0) break;
    }
    done += k;
    // x += Z y, then the true residual
    hipLaunchKernelGGL(k2d_gm_y, dim3(1), dim3(1), 0, s, gs, k);
    CK(hipGetLastError());
    CK(combine2d(h, x, x, h->Z, k, gs->y, 1.0));
    CK(restart2d(h, b, x, false));
    ++in.matvecs;
    CK(hipStreamSynchronize(s));
    relres = h->hsum->relres;
    if (!(relres <= rtol)) ++in.restarts;
  }
#undef CK
  in.relres_true = relres;
  in.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  if (info != nullptr) *info = in;
  return relres <= rtol ? CN_OK : CN_NOT_CONVERGED;
}
