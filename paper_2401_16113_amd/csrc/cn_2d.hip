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
constexpr int PF = 8;           // rows of band coefficients requested ahead
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
// Row k of a sweep needs entry k final, which the row before wrote; the
// sweeps therefore run row by row, each lane updating band entries t,
// t + 64, ...; coefficient rows are requested PF rows ahead.  P64: the
// half-bandwidth in units of 64 lanes (1 or 2).
template <int P64>
__global__ __launch_bounds__(BANDT) void k2d_band(const Cx<double>* __restrict__ Lc,
                                                  const Cx<double>* __restrict__ Uc,
                                                  const Cx<double>* __restrict__ dinv,
                                                  const Cx<double>* __restrict__ il2, int npts, int p,
                                                  Cx<double>* __restrict__ S) {
  extern __shared__ Cx<double> y[];
  const int j = blockIdx.x, t = threadIdx.x;
  Cx<double>* s = S + (size_t)j * npts;
  const Cx<double>* L = Lc + (size_t)j * npts * p;
  const Cx<double>* U = Uc + (size_t)j * npts * p;
  const Cx<double>* di = dinv + (size_t)j * npts;
  for (int i = t; i < npts; i += BANDT) y[i] = s[i];
  __syncthreads();
  auto coef = [&](const Cx<double>* base, int k, int r) -> Cx<double> {
    const int tt = t + r * BANDT;
    return (k >= 0 && k < npts && tt < p) ? base[(size_t)k * p + tt] : czero();
  };
  // forward: y[k+1+t] -= L[k+1+t][k] y[k]
  {
    Cx<double> cb[PF][P64];
#pragma unroll
    for (int q = 0; q < PF; ++q)
#pragma unroll
      for (int r = 0; r < P64; ++r) cb[q][r] = coef(L, q, r);
    for (int k0 = 0; k0 < npts; k0 += PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int k = k0 + q;
        Cx<double> c[P64];
#pragma unroll
        for (int r = 0; r < P64; ++r) {
          c[r] = cb[q][r];
          cb[q][r] = coef(L, k + PF, r);
        }
        if (k < npts) {
          const Cx<double> yk = y[k];
#pragma unroll
          for (int r = 0; r < P64; ++r) {
            const int i = k + 1 + t + r * BANDT;
            if (t + r * BANDT < p && i < npts) y[i] = y[i] - c[r] * yk;
          }
        }
        __syncthreads();
      }
    }
  }
  // backward: y[k] *= 1/U[k][k]; y[k-1-t] -= U[k-1-t][k] y[k]
  {
    Cx<double> cb[PF][P64];
    Cx<double> db[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int k = npts - 1 - q;
#pragma unroll
      for (int r = 0; r < P64; ++r) cb[q][r] = coef(U, k, r);
      db[q] = k >= 0 ? di[k] : czero();
    }
    for (int k0 = npts - 1; k0 >= 0; k0 -= PF) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int k = k0 - q;
        Cx<double> c[P64];
#pragma unroll
        for (int r = 0; r < P64; ++r) {
          c[r] = cb[q][r];
          cb[q][r] = coef(U, k - PF, r);
        }
        const Cx<double> dk = db[q];
        db[q] = k - PF >= 0 ? di[k - PF] : czero();
        if (k >= 0) {
          const Cx<double> yk = y[k] * dk;
          __syncthreads();  // every lane has read y[k] before lane 0 rewrites it
          if (t == 0) y[k] = yk;
#pragma unroll
          for (int r = 0; r < P64; ++r) {
            const int i = k - 1 - t - r * BANDT;
            if (t + r * BANDT < p && i >= 0) y[i] = y[i] - c[r] * yk;
          }
        }
        __syncthreads();
      }
    }
  }
  const Cx<double> sc = il2[j];
  for (int i = t; i < npts; i += BANDT) s[i] = y[i] * sc;
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
  if (p->flags != 0) return fail2d(CN_EINVAL, "flags must be 0");
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
  const int nt = h->nt, F = h->F, npts = h->npts, pb = h->p;
  const size_t band = (size_t)F * npts * pb * sizeof(Cx<double>);
  const size_t gband = (size_t)F * npts * (2 * pb + 1) * sizeof(Cx<double>);
  {
    size_t freeb = 0, totalb = 0;
    TRY2(hipMemGetInfo(&freeb, &totalb));
    const size_t need = 2 * band + gband + 2 * (size_t)F * npts * sizeof(Cx<double>);
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
