// The alpha-circulant preconditioner z = P_alpha^{-1} v (eq. (3.1)-(3.2)) on
// gfx950, as two streaming passes over the space-time vector plus a small
// interface solve:
//
//  K1 (pc_forward): one workgroup per tile of B spatial columns.  Loads the
//     B x N_t tile, applies the alpha weights Lambda_alpha (step (a)), runs a
//     length-N_t complex Stockham FFT in LDS on pairs of real columns (two
//     real transforms per complex one; only the N_t/2+1 non-redundant modes
//     are used, Remark 1), then for every frequency j solves the shifted
//     system (lambda_{1,j} I - lambda_{2,j} A~) restricted to the tile's
//     interior columns (step (b), local part) and writes the tile image plus
//     three interface values per (j, tile).
//  K2 (pc_reduced): for every j, the tridiagonal system of the separator
//     columns (one per tile boundary), factored once at set-up; solved by two
//     chunked affine scans.
//  K3 (pc_inverse): per tile, adds the separator contributions to the local
//     solution, runs the inverse FFT, multiplies by Lambda_alpha^{-1}/N_t
//     (step (c)) and writes z.
#include <math.h>

#include "cn_internal.hpp"

namespace cn {

// ---------------------------------------------------------------------------
// K1
// ---------------------------------------------------------------------------
template <typename R, int LOG2N>
__global__ __launch_bounds__((PcCfg<R, LOG2N>::T)) void k_pc_forward(
    const double* __restrict__ v, const double* __restrict__ scale,
    const int* __restrict__ done, const double* __restrict__ lo,
    const double* __restrict__ di, const double* __restrict__ up,
    const double* __restrict__ wfw, const Cx<R>* __restrict__ tw,
    const Cx<double>* __restrict__ mu, const Cx<double>* __restrict__ il2,
    Cx<R>* __restrict__ spec, Cx<R>* __restrict__ iface, int nx, int P, int nwg_pad) {
  using Cfg = PcCfg<R, LOG2N>;
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  __shared__ Cx<R> lds[Cfg::LDS_ELEMS];
  __shared__ R co[3 * B];
  if (done != nullptr && *done) return;
  const int p = xcd_tile(blockIdx.x, nwg_pad);
  if (p >= P) return;
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  const double sc = scale != nullptr ? *scale : 1.0;
  if (tid < 3 * B) {
    const int b = tid / 3, c = tid % 3;
    R val = R(0);
    if (b < ncols) val = (R)(c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]));
    co[tid] = val;
  }
  // step (a): alpha-weighted tile, columns (2s, 2s+1) packed as one complex
  // sequence.  All of a thread's loads are issued before any is consumed.
  R* ldsr = reinterpret_cast<R*>(lds);
  {
    constexpr int LPT = (N * B + T - 1) / T;
    double xv[LPT];
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      const int k = e / B, b = e % B;
      xv[q] = ((N * B) % T == 0 || e < N * B) && b < ncols ? v[(size_t)k * nx + i0 + b] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      if ((N * B) % T == 0 || e < N * B) {
        const int k = e / B, b = e % B;
        ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] = (R)(xv[q] * (wfw[k] * sc));
      }
    }
  }
  __syncthreads();
  fft_run<R, LOG2N, NSEQ, T, false, Cfg::MAXLOG, 0>(lds, tw);

  // step (b), tile-local part
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
        f[0] = Cx<R>{has_sep ? sepv : R(0), R(0)};
        f[1] = Cx<R>{ylast, R(0)};
        f[2] = Cx<R>{d[0], R(0)};
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
      f[0] = has_sep ? sepv : Cx<R>{R(0), R(0)};
      f[1] = ylast;
      f[2] = d[0];
    }
  }
  __syncthreads();
  Cx<R>* img = spec + (size_t)p * NSEQ * N;
  {
    constexpr int SPT = (NSEQ * N + T - 1) / T;
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSEQ * N) % T == 0 || e < NSEQ * N) img[e] = lds[lidx<N>(e / N, e % N)];
    }
  }
}

// ---------------------------------------------------------------------------
// K3
// ---------------------------------------------------------------------------
template <typename R, int LOG2N, typename TZ>
__global__ __launch_bounds__((PcCfg<R, LOG2N>::T)) void k_pc_inverse(
    const Cx<R>* __restrict__ spec, const Cx<R>* __restrict__ sep,
    const int* __restrict__ done, const double* __restrict__ lo,
    const double* __restrict__ di, const double* __restrict__ up,
    const double* __restrict__ winv, const Cx<R>* __restrict__ tw,
    const Cx<double>* __restrict__ mu, TZ* __restrict__ z, int nx, int P, int NS,
    int nwg_pad) {
  using Cfg = PcCfg<R, LOG2N>;
  constexpr int N = Cfg::N, B = Cfg::B, NSEQ = Cfg::NSEQ, T = Cfg::T;
  __shared__ Cx<R> lds[Cfg::LDS_ELEMS];
  __shared__ R co[3 * B];
  if (done != nullptr && *done) return;
  const int p = xcd_tile(blockIdx.x, nwg_pad);
  if (p >= P) return;
  const int tid = threadIdx.x;
  const int i0 = p * B;
  const int ncols = min(B, nx - i0);
  if (tid < 3 * B) {
    const int b = tid / 3, c = tid % 3;
    R val = R(0);
    if (b < ncols) val = (R)(c == 0 ? lo[i0 + b] : (c == 1 ? di[i0 + b] : up[i0 + b]));
    co[tid] = val;
  }
  const Cx<R>* img = spec + (size_t)p * NSEQ * N;
  {
    constexpr int SPT = (NSEQ * N + T - 1) / T;
    Cx<R> iv[SPT];
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSEQ * N) % T == 0 || e < NSEQ * N) iv[q] = img[e];
    }
#pragma unroll
    for (int q = 0; q < SPT; ++q) {
      const int e = tid + q * T;
      if ((NSEQ * N) % T == 0 || e < NSEQ * N) lds[lidx<N>(e / N, e % N)] = iv[q];
    }
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
      const Cx<double> md = mu[j];
      const Cx<R> m{(R)md.x, (R)md.y};
      const Cx<R> zero{R(0), R(0)};
      const Cx<R> sl = has_left ? sep[(size_t)j * NS + p - 1] : zero;
      const Cx<R> sr = has_sep ? sep[(size_t)j * NS + p] : zero;
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
  fft_run<R, LOG2N, NSEQ, T, true, Cfg::MAXLOG, 0>(lds, tw);
  const R* ldsr = reinterpret_cast<const R*>(lds);
  {
    constexpr int LPT = (N * B + T - 1) / T;
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int e = tid + q * T;
      const int k = e / B, b = e % B;
      if (((N * B) % T == 0 || e < N * B) && b < ncols) {
        const double val = (double)ldsr[2 * lidx<N>(b >> 1, k) + (b & 1)] * winv[k];
        z[(size_t)k * nx + i0 + b] = (TZ)val;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K2: interface (separator) systems, one workgroup per frequency line j.
//   rho_s = d_s + lo_s y_last(s) + up_s y_first(s+1)           (s = 0..NS-1)
//   forward  rho'_s = a_s rho'_{s-1} + rho_s,       a_s  = -m_s
//   backward S_s    = ap_s S_{s+1} + inv_s rho'_s,  ap_s = -c_s inv_s
// Each recurrence is an affine scan: chunk-local composition, a Hillis-Steele
// scan of the chunk maps in LDS, then a replay with the carried value.
// ---------------------------------------------------------------------------
constexpr int K2_THREADS = 256;

__device__ __forceinline__ void affine_scan(Cx<double>& A, Cx<double>& Bv, Cx<double>* sA,
                                            Cx<double>* sB, int pos, int n) {
  sA[pos] = A;
  sB[pos] = Bv;
  __syncthreads();
  for (int off = 1; off < n; off <<= 1) {
    Cx<double> pa{1.0, 0.0}, pb{0.0, 0.0};
    const bool has = pos >= off;
    if (has) {
      pa = sA[pos - off];
      pb = sB[pos - off];
    }
    __syncthreads();
    if (has) {
      const Cx<double> nA = A * pa;
      const Cx<double> nB = A * pb + Bv;
      A = nA;
      Bv = nB;
      sA[pos] = A;
      sB[pos] = Bv;
    }
    __syncthreads();
  }
}

template <typename R>
__global__ __launch_bounds__(K2_THREADS) void k_pc_reduced(
    const Cx<R>* __restrict__ iface, Cx<R>* __restrict__ sep,
    const Cx<double>* __restrict__ ra, const Cx<double>* __restrict__ rap,
    const Cx<double>* __restrict__ rinv, Cx<double>* __restrict__ rtmp,
    const double* __restrict__ lo, const double* __restrict__ up, int P, int NS, int B,
    const int* __restrict__ done) {
  __shared__ Cx<double> sA[K2_THREADS], sB[K2_THREADS];
  if (done != nullptr && *done) return;
  const int j = blockIdx.x;
  const int tid = threadIdx.x, n = blockDim.x;
  const int chunk = (NS + n - 1) / n;
  const int s0 = min(NS, tid * chunk), s1 = min(NS, s0 + chunk);
  const size_t row = (size_t)j * NS;
  const Cx<R>* f = iface + (size_t)j * P * 3;
  auto rho = [&](int s) -> Cx<double> {
    const int is = (s + 1) * B - 1;
    const Cx<R> d = f[(size_t)s * 3 + 0], yl = f[(size_t)s * 3 + 1], yf = f[(size_t)(s + 1) * 3 + 2];
    const double l = lo[is], u = up[is];
    return Cx<double>{(double)d.x + l * (double)yl.x + u * (double)yf.x,
                      (double)d.y + l * (double)yl.y + u * (double)yf.y};
  };
  // forward sweep
  Cx<double> A{1.0, 0.0}, Bv{0.0, 0.0};
  for (int s = s0; s < s1; ++s) {
    const Cx<double> a = ra[row + s];
    Bv = a * Bv + rho(s);
    A = a * A;
  }
  affine_scan(A, Bv, sA, sB, tid, n);
  Cx<double> r = tid > 0 ? sB[tid - 1] : Cx<double>{0.0, 0.0};
  for (int s = s0; s < s1; ++s) {
    r = ra[row + s] * r + rho(s);
    rtmp[row + s] = r;
  }
  __syncthreads();
  // backward sweep, scanned from the last chunk
  const int pos = n - 1 - tid;
  A = Cx<double>{1.0, 0.0};
  Bv = Cx<double>{0.0, 0.0};
  for (int s = s1 - 1; s >= s0; --s) {
    const Cx<double> a = rap[row + s];
    Bv = a * Bv + rinv[row + s] * rtmp[row + s];
    A = a * A;
  }
  affine_scan(A, Bv, sA, sB, pos, n);
  Cx<double> S = pos > 0 ? sB[pos - 1] : Cx<double>{0.0, 0.0};
  for (int s = s1 - 1; s >= s0; --s) {
    S = rap[row + s] * S + rinv[row + s] * rtmp[row + s];
    sep[row + s] = Cx<R>{(R)S.x, (R)S.y};
  }
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

__global__ void k_setup_reduced(const double* __restrict__ lo, const double* __restrict__ di,
                                const double* __restrict__ up, const Cx<double>* __restrict__ mu,
                                const Cx<double>* __restrict__ spk, int P, int NS, int B, int F,
                                Cx<double>* __restrict__ ra, Cx<double>* __restrict__ rap,
                                Cx<double>* __restrict__ rinv, int* __restrict__ err) {
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
    ra[row + s] = Cx<double>{-mlt.x, -mlt.y};
    rinv[row + s] = inv;
    const Cx<double> capi = Cm * inv;
    rap[row + s] = Cx<double>{-capi.x, -capi.y};
    beta_prev = beta;
    cm_prev = Cm;
  }
  if (bad) atomicOr(err, 2);
}

// ---------------------------------------------------------------------------
// launchers: dispatch on the precision and on log2(N_t)
// ---------------------------------------------------------------------------
template <typename R, int L>
static void cfg_of(int* B, int* T) {
  *B = PcCfg<R, L>::B;
  *T = PcCfg<R, L>::T;
}

#define CN_LOG2N_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13)

void pc_config(int prec, int log2n, int* B, int* T) {
  switch (log2n) {
#define X(L)                       \
  case L:                          \
    if (prec)                      \
      cfg_of<float, L>(B, T);      \
    else                           \
      cfg_of<double, L>(B, T);     \
    break;
    CN_LOG2N_CASES(X)
#undef X
    default:
      *B = *T = 0;
  }
}

static inline int pad8(int v) { return (v + 7) / 8 * 8; }

template <typename R, int L>
static hipError_t launch_fwd(const PcPlan& pl, const double* v, const double* scale,
                             const int* done, hipStream_t s) {
  using Cfg = PcCfg<R, L>;
  const int nwg = pad8(pl.P);
  const Cx<R>* tw = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f;
  hipLaunchKernelGGL((k_pc_forward<R, L>), dim3(nwg), dim3(Cfg::T), 0, s, v, scale, done, pl.lo,
                     pl.di, pl.up, pl.wfw, tw, pl.mu, pl.il2, (Cx<R>*)pl.spec, (Cx<R>*)pl.iface,
                     pl.nx, pl.P, nwg);
  return hipGetLastError();
}

template <typename R, int L>
static hipError_t launch_inv(const PcPlan& pl, void* z, int zf, const int* done, hipStream_t s) {
  using Cfg = PcCfg<R, L>;
  const int nwg = pad8(pl.P);
  const Cx<R>* tw = std::is_same<R, double>::value ? (const Cx<R>*)pl.tw : (const Cx<R>*)pl.tw_f;
  if (zf)
    hipLaunchKernelGGL((k_pc_inverse<R, L, float>), dim3(nwg), dim3(Cfg::T), 0, s,
                       (const Cx<R>*)pl.spec, (const Cx<R>*)pl.sep, done, pl.lo, pl.di, pl.up,
                       pl.winv, tw, pl.mu, (float*)z, pl.nx, pl.P, pl.NS, nwg);
  else
    hipLaunchKernelGGL((k_pc_inverse<R, L, double>), dim3(nwg), dim3(Cfg::T), 0, s,
                       (const Cx<R>*)pl.spec, (const Cx<R>*)pl.sep, done, pl.lo, pl.di, pl.up,
                       pl.winv, tw, pl.mu, (double*)z, pl.nx, pl.P, pl.NS, nwg);
  return hipGetLastError();
}

hipError_t pc_forward(const PcPlan& pl, const double* v, const double* scale, const int* done,
                      hipStream_t s) {
  switch (pl.log2n) {
#define X(L)                                                    \
  case L:                                                       \
    return pl.prec ? launch_fwd<float, L>(pl, v, scale, done, s) \
                   : launch_fwd<double, L>(pl, v, scale, done, s);
    CN_LOG2N_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t pc_inverse(const PcPlan& pl, void* z, int zf, const int* done, hipStream_t s) {
  switch (pl.log2n) {
#define X(L)                                                   \
  case L:                                                      \
    return pl.prec ? launch_inv<float, L>(pl, z, zf, done, s) \
                   : launch_inv<double, L>(pl, z, zf, done, s);
    CN_LOG2N_CASES(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t pc_reduced(const PcPlan& pl, const int* done, hipStream_t s) {
  if (pl.NS <= 0) return hipSuccess;
  int thr = 64;
  while (thr < K2_THREADS && thr < pl.NS) thr *= 2;
  if (pl.prec)
    hipLaunchKernelGGL((k_pc_reduced<float>), dim3(pl.F), dim3(thr), 0, s,
                       (const Cx<float>*)pl.iface, (Cx<float>*)pl.sep, pl.red_a, pl.red_ap,
                       pl.red_inv, pl.red_tmp, pl.lo, pl.up, pl.P, pl.NS, pl.B, done);
  else
    hipLaunchKernelGGL((k_pc_reduced<double>), dim3(pl.F), dim3(thr), 0, s,
                       (const Cx<double>*)pl.iface, (Cx<double>*)pl.sep, pl.red_a, pl.red_ap,
                       pl.red_inv, pl.red_tmp, pl.lo, pl.up, pl.P, pl.NS, pl.B, done);
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
    hipLaunchKernelGGL(k_setup_reduced, dim3(b2), dim3(t2), 0, s, pl.lo, pl.di, pl.up, pl.mu,
                       spk, pl.P, pl.NS, pl.B, pl.F, pl.red_a, pl.red_ap, pl.red_inv, err);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace cn
