// Learned warm start on gfx950: a 4-layer perceptron (n_in -> w -> w -> w ->
// n_out, ReLU) trained and evaluated with hand-written kernels:
//   * GEMMs on the matrix cores: bf16 operands (weights kept as float32
//     masters with bf16 copies, activations rounded to bf16 as they are
//     staged in LDS), float32 accumulation, fused bias / ReLU / ReLU-mask
//     epilogues;
//   * input standardisation and output de-standardisation in float32 (the
//     network works on standardised features and targets);
//   * mean-squared-error gradient, bias gradients, Adam;
//   * restriction of fine space-time solutions to the 128 x 64 coarse grid
//     (training targets) and bilinear interpolation of a coarse prediction
//     back to the fine grid (the initial guess), with the initial condition
//     as the t = 0 row and the Dirichlet data as the space-boundary columns.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "cn_internal.hpp"
#include "cn_warmstart.h"

namespace cn_ws {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// float32 -> bf16, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }
__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(unsigned short v) { return bf2f(v); }

// ---------------------------------------------------------------------------
// C[M x N] = alpha * sum_k A(m, k) B(k, n), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn]; epilogue: 0 none, 1 bias + ReLU, 2 bias,
// 3 keep where mask(m, n) > 0 (ReLU derivative), C row-major with ldc.
// 64 x 64 tile per workgroup, four waves of 32 x 32 (MFMA 32x32x8 bf16).
// ---------------------------------------------------------------------------
constexpr int BM = 64, BN = 64, BK = 32, PADK = 8;

template <typename TA, typename TB, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const TA* __restrict__ A,
                                              long long sam, long long sak,
                                              const TB* __restrict__ B, long long sbk,
                                              long long sbn, float* __restrict__ C,
                                              long long ldc, const float* __restrict__ bias,
                                              const float* __restrict__ mask, float alpha) {
  __shared__ unsigned short As[BM][BK + PADK];
  __shared__ unsigned short Bs[BN][BK + PADK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv & 1, wn = wv >> 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  f16v acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  const bool a_kc = sak == 1, b_kc = sbk == 1;
  for (int k0 = 0; k0 < K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int m, k;
      if (a_kc) {
        m = e / BK;
        k = e % BK;
      } else {
        k = e / BM;
        m = e % BM;
      }
      const int gm = m0 + m, gk = k0 + k;
      const float v = (gm < M && gk < K) ? to_f(A[(long long)gm * sam + (long long)gk * sak]) : 0.f;
      As[m][k] = f2bf(v);
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int n, k;
      if (b_kc) {
        n = e / BK;
        k = e % BK;
      } else {
        k = e / BN;
        n = e % BN;
      }
      const int gn = n0 + n, gk = k0 + k;
      const float v = (gn < N && gk < K) ? to_f(B[(long long)gk * sbk + (long long)gn * sbn]) : 0.f;
      Bs[n][k] = f2bf(v);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 8) {
      const s4 a = *(const s4*)&As[wm * 32 + (lane & 31)][kk + (lane >> 5) * 4];
      const s4 b = *(const s4*)&Bs[wn * 32 + (lane & 31)][kk + (lane >> 5) * 4];
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int m = m0 + wm * 32 + (v / 4) * 8 + (lane >> 5) * 4 + (v % 4);
    const int n = n0 + wn * 32 + (lane & 31);
    if (m < M && n < N) {
      float r = alpha * acc[v];
      if (EPI == 1 || EPI == 2) r += bias[n];
      if (EPI == 1) r = fmaxf(r, 0.f);
      if (EPI == 3) r = mask[(long long)m * ldc + n] > 0.f ? r : 0.f;
      C[(long long)m * ldc + n] = r;
    }
  }
}

// d = z - (t - mu) / sd (standardised output against standardised target),
// dOut = scale d; per-block partial sums of d^2
__global__ __launch_bounds__(256) void k_mse_grad(const float* __restrict__ out,
                                                  const float* __restrict__ tgt, long long n,
                                                  int cols, const float* __restrict__ mu,
                                                  const float* __restrict__ sd, float scale,
                                                  float* __restrict__ dout,
                                                  float* __restrict__ partial) {
  __shared__ float red[256];
  float s = 0.f;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int c = (int)(e % cols);
    const float d = out[e] - (tgt[e] - mu[c]) / sd[c];
    dout[e] = scale * d;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// y = (x - mu) / sd (standardise, columns of a row-major [rows x cols]) or
// y = mu + sd x (INV: de-standardise)
template <bool INV>
__global__ __launch_bounds__(256) void k_affine(const float* __restrict__ x, long long n, int cols,
                                                const float* __restrict__ mu,
                                                const float* __restrict__ sd,
                                                float* __restrict__ y) {
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int c = (int)(e % cols);
    y[e] = INV ? mu[c] + sd[c] * x[e] : (x[e] - mu[c]) / sd[c];
  }
}

__global__ void k_fill(float* __restrict__ p, long long n, float v) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    p[e] = v;
}

__global__ void k_sum(const float* __restrict__ partial, int n, float scale, float* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float s = 0.f;
  for (int i = 0; i < n; ++i) s += partial[i];
  *out = scale * s;
}

// out[c] = sum_r X[r*cols + c] (bias gradient), fixed order
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ X, int rows, int cols,
                                                float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.f;
  for (int r = 0; r < rows; ++r) s += X[(long long)r * cols + c];
  out[c] = s;
}

// Adam on the float32 masters, then the bf16 copies of the weight matrices
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              long long n, float lr, float b1, float b2,
                                              float eps, float bc1, float bc2) {
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
  }
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ w,
                                                 unsigned short* __restrict__ wb, long long n) {
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256)
    wb[e] = f2bf(w[e]);
}

// ---------------------------------------------------------------------------
// coarse grid: 128 points in space x 64 in time, stored [q][c].  Fine point
// (k, i) of an N_x x N_t grid with (N_x + 1) = 128 sx and N_t = 64 st:
// coarse node c sits at fine i = sx c + sx/2 - 1, node q at fine k = st q + st - 1.
// ---------------------------------------------------------------------------
constexpr int CX = 128, CT = 64;

__global__ __launch_bounds__(256) void k_restrict(const double* __restrict__ x, int count, int nx,
                                                  int nt, const double* __restrict__ inv_scale,
                                                  float* __restrict__ coarse) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)count * CX * CT) return;
  const int inst = (int)(e / (CX * CT));
  const int r = (int)(e % (CX * CT));
  const int q = r / CX, c = r % CX;
  const int sx = (nx + 1) / CX, st = nt / CT;
  const int i = sx * c + sx / 2 - 1, k = st * q + st - 1;
  const long long n = (long long)nx * nt;
  coarse[e] = (float)(x[inst * n + (long long)k * nx + i] * inv_scale[inst]);
}

// x0(k, i) = bilinear interpolation of scale * coarse, extended by u0 at
// t = 0 and by the Dirichlet data gl(t), gr(t) at the space ends, for one
// instance: cs its CX x CT coarse values, gL/gR its N_t boundary values, u0
// its N_x initial values.  Contraction into fused multiply-adds is off, so
// every kernel that calls this gets the same bits for the same inputs.
__device__ __forceinline__ double interp_value(const float* __restrict__ cs, double sc,
                                               const double* __restrict__ gL,
                                               const double* __restrict__ gR,
                                               const double* __restrict__ u0, int nx, int nt,
                                               int k, int i) {
#pragma clang fp contract(off)
  const int sx = (nx + 1) / CX, st = nt / CT;
  // space position in coarse units: node c at (i - (sx/2 - 1))/sx = c; the
  // boundaries sit at -1/2 (left) and CX - 1/2 (right)
  const double pc = (double)(i - (sx / 2 - 1)) / sx;
  // value of coarse time row q (q >= 0) at fine column i
  auto row = [&](int q, int kk) -> double {
    if (pc < 0.0) {
      const double w = (pc + 0.5) / 0.5;
      return (1.0 - w) * gL[kk] + w * sc * cs[q * CX];
    }
    if (pc > CX - 1) {
      const double w = (pc - (CX - 1)) / 0.5;
      return (1.0 - w) * sc * cs[q * CX + CX - 1] + w * gR[kk];
    }
    const int c0 = min((int)pc, CX - 2);
    const double w = pc - c0;
    return (1.0 - w) * sc * cs[q * CX + c0] + w * sc * cs[q * CX + c0 + 1];
  };
  // time position: node q at fine level st q + st - 1; q = -1 is t = 0 (u0)
  const double pq = (double)(k + 1) / st - 1.0;
  const int q0 = (int)floor(pq);
  const double wt = pq - q0;
  // fine level of coarse row q (for the boundary data of that row)
  const int k0 = st * q0 + st - 1;
  const double v0 = q0 < 0 ? u0[i] : row(q0, k0);
  double v = v0;
  if (wt > 0.0 && q0 + 1 < CT) v = (1.0 - wt) * v0 + wt * row(q0 + 1, k0 + st);
  return v;
}

// `count` instances of one shape, back to back
__global__ __launch_bounds__(256) void k_interp(const float* __restrict__ coarse, int count, int nx,
                                                int nt, const double* __restrict__ u0,
                                                const double* __restrict__ gl,
                                                const double* __restrict__ gr,
                                                const double* __restrict__ scale,
                                                double* __restrict__ x0) {
  const long long n = (long long)nx * nt;
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long long)count * n) return;
  const int inst = (int)(e / n);
  const long long r = e % n;
  const int k = (int)(r / nx), i = (int)(r % nx);
  x0[e] = interp_value(coarse + (long long)inst * CX * CT, scale[inst], gl + (long long)inst * nt,
                       gr + (long long)inst * nt, u0 + (long long)inst * nx, nx, nt, k, i);
}

// The same for a batch of uneven instances: element e of the packed vector
// belongs to the instance whose offset range holds it (binary search over the
// offsets); that instance's N_x, N_t, initial condition and boundary data come
// from the batch layout (see BatchLayout).
__global__ __launch_bounds__(256) void k_interp_batch(const float* __restrict__ coarse, int count,
                                                      const long long* __restrict__ lay,
                                                      const double* __restrict__ u0,
                                                      const double* __restrict__ gl,
                                                      const double* __restrict__ gr,
                                                      const double* __restrict__ scale,
                                                      double* __restrict__ x0) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= lay[count]) return;
  int lo = 0, hi = count - 1;  // lay[lo] <= e < lay[hi + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lay[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  const int inst = lo;
  const int nx = (int)lay[3 * count + 1 + inst], nt = (int)lay[4 * count + 1 + inst];
  const long long r = e - lay[inst];
  const int k = (int)(r / nx), i = (int)(r % nx);
  const long long go = lay[2 * count + 1 + inst];
  x0[e] = interp_value(coarse + (long long)inst * CX * CT, scale[inst], gl + go, gr + go,
                       u0 + lay[count + 1 + inst], nx, nt, k, i);
}

}  // namespace cn_ws

using namespace cn_ws;

static thread_local std::string g_ws_err;

struct cn_mlp {
  int n_in = 0, w = 0, n_out = 0, max_batch = 0;
  hipStream_t s = nullptr;
  long long np = 0;            // parameters
  long long off[8] = {};       // W1 b1 W2 b2 W3 b3 W4 b4 offsets in the flat layout
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;   // params, grads, Adam moments
  unsigned short* pb = nullptr;  // bf16 copy of the parameters
  float *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *out = nullptr;  // activations
  float *d3 = nullptr, *d2 = nullptr, *d1 = nullptr, *dout = nullptr;  // gradients of activations
  float* partial = nullptr;
  float *in_mu = nullptr, *in_sd = nullptr, *out_mu = nullptr, *out_sd = nullptr;
  float* xn = nullptr;  // standardised input rows
  int step = 0;
};

static cn_status ws_fail(cn_status s, const std::string& m) {
  g_ws_err = m;
  return s;
}

#define WS_TRY(expr)                                                                \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ws_fail(e_ == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP,               \
                     std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

template <typename TA, typename TB, int EPI>
static hipError_t gemm(hipStream_t s, int M, int N, int K, const TA* A, long long sam,
                       long long sak, const TB* B, long long sbk, long long sbn, float* C,
                       long long ldc, const float* bias, const float* mask, float alpha) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
  hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk,
                     sbn, C, ldc, bias, mask, alpha);
  return hipGetLastError();
}

static int nblk(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

static void free_mlp(cn_mlp* net) {
  if (net == nullptr) return;
  for (void* q : {(void*)net->p, (void*)net->g, (void*)net->m, (void*)net->v, (void*)net->pb,
                  (void*)net->h1, (void*)net->h2, (void*)net->h3, (void*)net->out,
                  (void*)net->d3, (void*)net->d2, (void*)net->d1, (void*)net->dout,
                  (void*)net->partial, (void*)net->in_mu, (void*)net->in_sd,
                  (void*)net->out_mu, (void*)net->out_sd, (void*)net->xn})
    if (q != nullptr) (void)hipFree(q);
  delete net;
}

// forward pass of net on X[B x n_in] into net->out (standardised output,
// activations and the standardised input n->xn kept for the backward pass)
static hipError_t forward(cn_mlp* n, const float* Xraw, int B) {
  const unsigned short* W = n->pb;
  const float* P = n->p;
  const int w = n->w;
  const long long nin = (long long)B * n->n_in;
  hipLaunchKernelGGL(k_affine<false>, dim3(nblk(nin)), dim3(256), 0, n->s, Xraw, nin, n->n_in,
                     n->in_mu, n->in_sd, n->xn);
  const float* X = n->xn;
  hipError_t e = gemm<float, unsigned short, 1>(n->s, B, w, n->n_in, X, n->n_in, 1, W + n->off[0],
                                                1, n->n_in, n->h1, w, P + n->off[1], nullptr, 1.f);
  if (e == hipSuccess)
    e = gemm<float, unsigned short, 1>(n->s, B, w, w, n->h1, w, 1, W + n->off[2], 1, w, n->h2, w,
                                       P + n->off[3], nullptr, 1.f);
  if (e == hipSuccess)
    e = gemm<float, unsigned short, 1>(n->s, B, w, w, n->h2, w, 1, W + n->off[4], 1, w, n->h3, w,
                                       P + n->off[5], nullptr, 1.f);
  if (e == hipSuccess)
    e = gemm<float, unsigned short, 2>(n->s, B, n->n_out, w, n->h3, w, 1, W + n->off[6], 1, w,
                                       n->out, n->n_out, P + n->off[7], nullptr, 1.f);
  return e;
}

extern "C" {

const char* cn_ws_last_error(void) { return g_ws_err.c_str(); }

cn_status cn_mlp_create(int32_t n_in, int32_t width, int32_t n_out, int32_t max_batch,
                        void* stream, cn_mlp** out) {
  if (out == nullptr) return ws_fail(CN_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_in < 1 || width < 1 || n_out < 1 || max_batch < 1)
    return ws_fail(CN_EINVAL, "sizes must be >= 1");
  cn_mlp* n = new cn_mlp();
  n->n_in = n_in;
  n->w = width;
  n->n_out = n_out;
  n->max_batch = max_batch;
  n->s = (hipStream_t)stream;
  const long long sizes[8] = {(long long)width * n_in, width, (long long)width * width, width,
                              (long long)width * width, width, (long long)n_out * width, n_out};
  long long o = 0;
  for (int i = 0; i < 8; ++i) {
    n->off[i] = o;
    o += sizes[i];
  }
  n->np = o;
  const long long act = (long long)max_batch * width;
  const long long outn = (long long)max_batch * n_out;
  hipError_t e = hipSuccess;
  auto al = [&](auto** ptr, long long elems, size_t es) {
    if (e == hipSuccess) e = hipMalloc((void**)ptr, (size_t)elems * es);
  };
  al(&n->p, o, 4);
  al(&n->g, o, 4);
  al(&n->m, o, 4);
  al(&n->v, o, 4);
  al(&n->pb, o, 2);
  al(&n->h1, act, 4);
  al(&n->h2, act, 4);
  al(&n->h3, act, 4);
  al(&n->d1, act, 4);
  al(&n->d2, act, 4);
  al(&n->d3, act, 4);
  al(&n->out, outn, 4);
  al(&n->dout, outn, 4);
  al(&n->partial, 4096, 4);
  al(&n->in_mu, n_in, 4);
  al(&n->in_sd, n_in, 4);
  al(&n->out_mu, n_out, 4);
  al(&n->out_sd, n_out, 4);
  al(&n->xn, (long long)max_batch * n_in, 4);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, n->s, n->in_mu, (long long)n_in, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(1), dim3(256), 0, n->s, n->in_sd, (long long)n_in, 1.f);
    hipLaunchKernelGGL(k_fill, dim3(32), dim3(256), 0, n->s, n->out_mu, (long long)n_out, 0.f);
    hipLaunchKernelGGL(k_fill, dim3(32), dim3(256), 0, n->s, n->out_sd, (long long)n_out, 1.f);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemsetAsync(n->p, 0, (size_t)o * 4, n->s);
  if (e == hipSuccess) e = hipMemsetAsync(n->pb, 0, (size_t)o * 2, n->s);
  if (e == hipSuccess) e = hipMemsetAsync(n->m, 0, (size_t)o * 4, n->s);
  if (e == hipSuccess) e = hipMemsetAsync(n->v, 0, (size_t)o * 4, n->s);
  if (e == hipSuccess) e = hipStreamSynchronize(n->s);
  if (e != hipSuccess) {
    free_mlp(n);
    return ws_fail(e == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP,
                   std::string("cn_mlp_create: ") + hipGetErrorString(e));
  }
  *out = n;
  return CN_OK;
}

cn_status cn_mlp_destroy(cn_mlp* n) {
  if (n == nullptr) return ws_fail(CN_EINVAL, "net is NULL");
  (void)hipStreamSynchronize(n->s);
  free_mlp(n);
  return CN_OK;
}

cn_status cn_mlp_num_params(const cn_mlp* n, int64_t* np) {
  if (n == nullptr || np == nullptr) return ws_fail(CN_EINVAL, "NULL argument");
  *np = n->np;
  return CN_OK;
}

cn_status cn_mlp_set_params(cn_mlp* n, const float* params) {
  if (n == nullptr || params == nullptr) return ws_fail(CN_EINVAL, "NULL argument");
  WS_TRY(hipMemcpyAsync(n->p, params, (size_t)n->np * 4, hipMemcpyDeviceToDevice, n->s));
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n->np)), dim3(256), 0, n->s, n->p, n->pb, n->np);
  WS_TRY(hipGetLastError());
  WS_TRY(hipMemsetAsync(n->m, 0, (size_t)n->np * 4, n->s));
  WS_TRY(hipMemsetAsync(n->v, 0, (size_t)n->np * 4, n->s));
  n->step = 0;
  return CN_OK;
}

cn_status cn_mlp_get_params(const cn_mlp* n, float* params) {
  if (n == nullptr || params == nullptr) return ws_fail(CN_EINVAL, "NULL argument");
  WS_TRY(hipMemcpyAsync(params, n->p, (size_t)n->np * 4, hipMemcpyDeviceToDevice, n->s));
  return CN_OK;
}

cn_status cn_mlp_set_normalization(cn_mlp* n, const float* in_mean, const float* in_scale,
                                   const float* out_mean, const float* out_scale) {
  if (n == nullptr || in_mean == nullptr || in_scale == nullptr || out_mean == nullptr ||
      out_scale == nullptr)
    return ws_fail(CN_EINVAL, "NULL argument");
  WS_TRY(hipMemcpyAsync(n->in_mu, in_mean, (size_t)n->n_in * 4, hipMemcpyDeviceToDevice, n->s));
  WS_TRY(hipMemcpyAsync(n->in_sd, in_scale, (size_t)n->n_in * 4, hipMemcpyDeviceToDevice, n->s));
  WS_TRY(hipMemcpyAsync(n->out_mu, out_mean, (size_t)n->n_out * 4, hipMemcpyDeviceToDevice, n->s));
  WS_TRY(hipMemcpyAsync(n->out_sd, out_scale, (size_t)n->n_out * 4, hipMemcpyDeviceToDevice, n->s));
  return CN_OK;
}

cn_status cn_mlp_forward(cn_mlp* n, const float* X, int32_t B, float* Y) {
  if (n == nullptr || X == nullptr || Y == nullptr) return ws_fail(CN_EINVAL, "NULL argument");
  if (B < 1 || B > n->max_batch) return ws_fail(CN_EINVAL, "batch outside [1, max_batch]");
  WS_TRY(forward(n, X, B));
  const long long no = (long long)B * n->n_out;
  hipLaunchKernelGGL(k_affine<true>, dim3(nblk(no)), dim3(256), 0, n->s, n->out, no, n->n_out,
                     n->out_mu, n->out_sd, Y);
  WS_TRY(hipGetLastError());
  return CN_OK;
}

cn_status cn_mlp_loss_grad(cn_mlp* n, const float* X, const float* Yt, int32_t B, float* grads,
                           float* loss) {
  if (n == nullptr || X == nullptr || Yt == nullptr) return ws_fail(CN_EINVAL, "NULL argument");
  if (B < 1 || B > n->max_batch) return ws_fail(CN_EINVAL, "batch outside [1, max_batch]");
  const int w = n->w, no = n->n_out;
  const unsigned short* W = n->pb;
  float* G = n->g;
  WS_TRY(forward(n, X, B));
  // loss = mean d^2 over B x n_out with d = z - (t - mu)/sd; dz = 2 d / (B n_out)
  const long long nout = (long long)B * no;
  const int nb = nblk(nout);
  const float sc = 2.f / (float)nout;
  hipLaunchKernelGGL(k_mse_grad, dim3(nb), dim3(256), 0, n->s, n->out, Yt, nout, no, n->out_mu,
                     n->out_sd, sc, n->dout, n->partial);
  if (loss != nullptr)
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, n->s, n->partial, nb, 1.f / (float)nout, loss);
  WS_TRY(hipGetLastError());
  // layer 4: dW4 = dout^T h3, db4 = colsum dout, d3 = (dout W4) * [h3 > 0]
  WS_TRY((gemm<float, float, 0>(n->s, no, w, B, n->dout, 1, no, n->h3, w, 1, G + n->off[6], w,
                                nullptr, nullptr, 1.f)));
  hipLaunchKernelGGL(k_colsum, dim3((no + 255) / 256), dim3(256), 0, n->s, n->dout, B, no,
                     G + n->off[7]);
  WS_TRY((gemm<float, unsigned short, 3>(n->s, B, w, no, n->dout, no, 1, W + n->off[6], w, 1,
                                         n->d3, w, nullptr, n->h3, 1.f)));
  // layer 3
  WS_TRY((gemm<float, float, 0>(n->s, w, w, B, n->d3, 1, w, n->h2, w, 1, G + n->off[4], w,
                                nullptr, nullptr, 1.f)));
  hipLaunchKernelGGL(k_colsum, dim3((w + 255) / 256), dim3(256), 0, n->s, n->d3, B, w,
                     G + n->off[5]);
  WS_TRY((gemm<float, unsigned short, 3>(n->s, B, w, w, n->d3, w, 1, W + n->off[4], w, 1, n->d2,
                                         w, nullptr, n->h2, 1.f)));
  // layer 2
  WS_TRY((gemm<float, float, 0>(n->s, w, w, B, n->d2, 1, w, n->h1, w, 1, G + n->off[2], w,
                                nullptr, nullptr, 1.f)));
  hipLaunchKernelGGL(k_colsum, dim3((w + 255) / 256), dim3(256), 0, n->s, n->d2, B, w,
                     G + n->off[3]);
  WS_TRY((gemm<float, unsigned short, 3>(n->s, B, w, w, n->d2, w, 1, W + n->off[2], w, 1, n->d1,
                                         w, nullptr, n->h1, 1.f)));
  // layer 1 (no gradient for the input)
  WS_TRY((gemm<float, float, 0>(n->s, w, n->n_in, B, n->d1, 1, w, n->xn, n->n_in, 1, G + n->off[0],
                                n->n_in, nullptr, nullptr, 1.f)));
  hipLaunchKernelGGL(k_colsum, dim3((w + 255) / 256), dim3(256), 0, n->s, n->d1, B, w,
                     G + n->off[1]);
  WS_TRY(hipGetLastError());
  if (grads != nullptr)
    WS_TRY(hipMemcpyAsync(grads, G, (size_t)n->np * 4, hipMemcpyDeviceToDevice, n->s));
  return CN_OK;
}

cn_status cn_mlp_adam_step(cn_mlp* n, float lr, float beta1, float beta2, float eps) {
  if (n == nullptr) return ws_fail(CN_EINVAL, "net is NULL");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return ws_fail(CN_EINVAL, "invalid Adam hyper-parameters");
  n->step += 1;
  const float bc1 = 1.f - powf(beta1, (float)n->step);
  const float bc2 = 1.f - powf(beta2, (float)n->step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(n->np)), dim3(256), 0, n->s, n->p, n->g, n->m, n->v, n->np,
                     lr, beta1, beta2, eps, bc1, bc2);
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n->np)), dim3(256), 0, n->s, n->p, n->pb, n->np);
  WS_TRY(hipGetLastError());
  return CN_OK;
}

cn_status cn_ws_restrict(const double* x, int32_t count, int32_t nx, int32_t nt,
                         const double* inv_scale, float* coarse, void* stream) {
  if (x == nullptr || inv_scale == nullptr || coarse == nullptr)
    return ws_fail(CN_EINVAL, "NULL argument");
  if (count < 1 || nx < 1 || nt < CT || (nx + 1) % CX != 0 || nt % CT != 0 || (nx + 1) / CX < 2)
    return ws_fail(CN_EINVAL, "need nx + 1 a multiple of 128 (>= 256) and nt a multiple of 64");
  const long long n = (long long)count * CX * CT;
  hipLaunchKernelGGL(k_restrict, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, x, count, nx, nt, inv_scale, coarse);
  WS_TRY(hipGetLastError());
  return CN_OK;
}

cn_status cn_ws_interpolate(const float* coarse, int32_t count, int32_t nx, int32_t nt,
                            const double* u0, const double* gl, const double* gr,
                            const double* scale, double* x0, void* stream) {
  if (coarse == nullptr || u0 == nullptr || gl == nullptr || gr == nullptr || scale == nullptr ||
      x0 == nullptr)
    return ws_fail(CN_EINVAL, "NULL argument");
  if (count < 1 || nx < 1 || nt < CT || (nx + 1) % CX != 0 || nt % CT != 0 || (nx + 1) / CX < 2)
    return ws_fail(CN_EINVAL, "need nx + 1 a multiple of 128 (>= 256) and nt a multiple of 64");
  const long long n = (long long)count * nx * nt;
  hipLaunchKernelGGL(k_interp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, coarse, count, nx, nt, u0, gl, gr, scale, x0);
  WS_TRY(hipGetLastError());
  return CN_OK;
}

cn_status cn_ws_predict(cn_mlp* n, const float* features, int32_t count, int32_t nx, int32_t nt,
                        const double* u0, const double* gl, const double* gr,
                        const double* scale, float* coarse, double* x0) {
  if (n == nullptr || features == nullptr || coarse == nullptr || x0 == nullptr)
    return ws_fail(CN_EINVAL, "NULL argument");
  if (n->n_out != CX * CT) return ws_fail(CN_EINVAL, "the network must predict 128 x 64 values");
  if (count < 1) return ws_fail(CN_EINVAL, "count must be >= 1");
  for (int c0 = 0; c0 < count; c0 += n->max_batch) {
    const int B = std::min(n->max_batch, count - c0);
    const cn_status st = cn_mlp_forward(n, features + (size_t)c0 * n->n_in, B,
                                        coarse + (size_t)c0 * n->n_out);
    if (st != CN_OK) return st;
  }
  return cn_ws_interpolate(coarse, count, nx, nt, u0, gl, gr, scale, x0, n->s);
}

cn_status cn_ws_predict_batch(cn_mlp* n, const float* features, const cn_batch* b,
                              const double* u0, const double* gl, const double* gr,
                              const double* scale, float* coarse, double* x0) {
  if (n == nullptr || features == nullptr || b == nullptr || u0 == nullptr || gl == nullptr ||
      gr == nullptr || scale == nullptr || coarse == nullptr || x0 == nullptr)
    return ws_fail(CN_EINVAL, "NULL argument");
  if (n->n_out != CX * CT) return ws_fail(CN_EINVAL, "the network must predict 128 x 64 values");
  cn::BatchLayout lay;
  if (!cn::batch_layout(b, &lay)) return ws_fail(CN_EINVAL, "batch has no layout");
  for (int i = 0; i < lay.count; ++i) {
    const int nx = lay.nx[i], nt = lay.nt[i];
    if (nt < CT || (nx + 1) % CX != 0 || nt % CT != 0 || (nx + 1) / CX < 2)
      return ws_fail(CN_EINVAL, "instance " + std::to_string(i) +
                                    ": need nx + 1 a multiple of 128 (>= 256) and nt a multiple of 64");
  }
  for (int c0 = 0; c0 < lay.count; c0 += n->max_batch) {
    const int B = std::min(n->max_batch, lay.count - c0);
    const cn_status st = cn_mlp_forward(n, features + (size_t)c0 * n->n_in, B,
                                        coarse + (size_t)c0 * n->n_out);
    if (st != CN_OK) return st;
  }
  hipLaunchKernelGGL(k_interp_batch, dim3((unsigned)((lay.total + 255) / 256)), dim3(256), 0,
                     n->s, coarse, lay.count, lay.dev, u0, gl, gr, scale, x0);
  WS_TRY(hipGetLastError());
  return CN_OK;
}

}  // extern "C"
