// Device building blocks for the alpha-circulant preconditioner on gfx950:
// complex arithmetic, in-register DFTs, an LDS-staged Stockham FFT pass and
// the tile-local tridiagonal solve of the partitioned step-(b) solver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cn {

// Global-memory pointers.  Pointers read from an instance descriptor are
// generic to the compiler, which then emits flat memory instructions (they
// also count against the LDS counter, so an LDS wait waits for memory too);
// the hot loops take their vectors as global-qualified pointers instead.
#define CN_G __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ CN_G T* gp(T* p) {
  return (CN_G T*)p;
}

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename R>
struct Cx {
  R x, y;
};

// Complex values through global-qualified pointers, as one 8- or 16-byte access
// (a struct copy through such a pointer would need an address-space-aware
// assignment operator).
typedef float cn_f2 __attribute__((ext_vector_type(2)));
typedef double cn_d2 __attribute__((ext_vector_type(2)));
template <typename R>
struct CxVec;
template <>
struct CxVec<float> {
  using T = cn_f2;
};
template <>
struct CxVec<double> {
  using T = cn_d2;
};
template <typename R>
__device__ __forceinline__ Cx<R> gld(const CN_G Cx<R>* p) {
  const typename CxVec<R>::T v = *(const CN_G typename CxVec<R>::T*)p;
  return Cx<R>{v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void gst(CN_G Cx<R>* p, Cx<R> c) {
  typename CxVec<R>::T v;
  v.x = c.x;
  v.y = c.y;
  *(CN_G typename CxVec<R>::T*)p = v;
}
// generic pointers keep plain accesses
template <typename R>
__device__ __forceinline__ Cx<R> gld(const Cx<R>* p) { return *p; }

template <typename R>
__device__ __forceinline__ Cx<R> mk(R a, R b) { return Cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator+(Cx<R> a, Cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator-(Cx<R> a, Cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> operator*(Cx<R> a, Cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ Cx<R> operator*(R s, Cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> conj(Cx<R> a) { return {a.x, -a.y}; }
// multiply by -i (forward) or +i (inverse)
template <typename R, bool INV>
__device__ __forceinline__ Cx<R> mul_mi(Cx<R> a) {
  return INV ? Cx<R>{-a.y, a.x} : Cx<R>{a.y, -a.x};
}

// Reciprocals.  float64: hardware estimate refined by two Newton steps
// (error ~1 ulp); float32: hardware estimate (1 ulp).
__device__ __forceinline__ double rcp(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = __builtin_fma(-a, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-a, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp(float a) { return __builtin_amdgcn_rcpf(a); }

template <typename R>
__device__ __forceinline__ Cx<R> crcp(Cx<R> a) {
  R s = rcp(a.x * a.x + a.y * a.y);
  return {a.x * s, -a.y * s};
}
__device__ __forceinline__ double crcp(double a) { return rcp(a); }
__device__ __forceinline__ float crcp(float a) { return rcp(a); }

// ---------------------------------------------------------------------------
// in-register DFT of size RAD (RAD = 1, 2, 4, 8, 16), decimation in time.
// forward: X_q = sum_r u_r exp(-2 pi i r q / RAD); inverse: exp(+...).
// ---------------------------------------------------------------------------
// cos and sin of 2 pi m / 16, m = 0..15
__host__ __device__ constexpr double cos16(int m) {
  constexpr double t[16] = {
      1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
      0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
      -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
      0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  return t[m & 15];
}
__host__ __device__ constexpr double sin16(int m) { return cos16(m + 12); }

template <typename R, int RAD, bool INV, int S = 1>
struct Dft {
  // in-place DFT of u[0], u[S], ..., u[(RAD-1) S]
  static __device__ __forceinline__ void run(Cx<R>* u) {
    if constexpr (RAD == 1) {
      return;
    } else if constexpr (RAD == 2) {
      Cx<R> a = u[0], b = u[S];
      u[0] = a + b;
      u[S] = a - b;
    } else {
      // split into even and odd halves (stride 2S), transform each, combine
      Dft<R, RAD / 2, INV, 2 * S>::run(u);
      Dft<R, RAD / 2, INV, 2 * S>::run(u + S);
      Cx<R> t[RAD];
#pragma unroll
      for (int q = 0; q < RAD; ++q) t[q] = u[q * S];
      // now t[2q] = E_q (q < RAD/2), t[2q+1] = O_q
#pragma unroll
      for (int q = 0; q < RAD / 2; ++q) {
        Cx<R> e = t[2 * q], o = t[2 * q + 1];
        Cx<R> w;
        constexpr int step = 16 / RAD;
        if (q == 0) {
          w = o;
        } else if (4 * q == RAD) {
          w = mul_mi<R, INV>(o);
        } else {
          const R c = (R)cos16(q * step);
          const R s = INV ? (R)sin16(q * step) : -(R)sin16(q * step);
          w = Cx<R>{o.x * c - o.y * s, o.x * s + o.y * c};
        }
        u[q * S] = e + w;
        u[(q + RAD / 2) * S] = e - w;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// transform kernel configuration for a given precision and N_t = 2^LOG2N
// ---------------------------------------------------------------------------
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int clog2(int v) { return v <= 1 ? 0 : 1 + clog2(v / 2); }

// Reads through a buffer resource: a uniform base address, a per-thread
// 32-bit byte offset and a uniform 32-bit byte offset per load, so a run of
// loads whose addresses differ by uniform amounts needs one address register
// in all (global loads take a 64-bit address register pair each).  The
// caller keeps every offset below 2^32 bytes (the resource's range is not
// used as a bound).  Word 3 = 0x00020000: 32-bit data format, which raw
// (untyped) loads of the CDNA family require.
struct BufRd {
  __amdgpu_buffer_rsrc_t r;
  template <typename P>
  __device__ __forceinline__ explicit BufRd(P base)
      : r(__builtin_amdgcn_make_buffer_rsrc((void*)(base), (short)0, -1, 0x00020000)) {}
  __device__ __forceinline__ double f64(unsigned voff, unsigned soff) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
};

// Two-level tables of a length-N sequence (N a power of two): entry k is
// lo[k mod SL] * hi[k / SL], with lo = the first SL entries and hi = every
// SL-th one, SL = min(N, 64).  Used for the twiddles when the full table
// would cost the tile a workgroup per CU: 64 + N/64 entries instead of N,
// at the price of one extra product (about one unit of rounding).
template <int N>
struct Split2 {
  static constexpr int SL = N < 64 ? N : 64;
  static constexpr int LOGSL = clog2(SL);
  static constexpr int SH = N / SL;
  static constexpr int SIZE = SL + SH;
};

constexpr int kLdsCap = 160 * 1024;  // LDS of a gfx950 compute unit (and most per workgroup)
// a table of `extra` bytes beside `base` fits and keeps `wgs` workgroups per CU
constexpr bool lds_keeps(int base, int extra, int wgs) {
  return base + extra <= kLdsCap && kLdsCap / (base + extra) >= wgs;
}

// Default tile width B (columns, even) and workgroup size T of the transform
// kernels: the widest tile whose image fits 128 KB of LDS, ~16 complex
// elements per thread.
template <typename R, int LOG2N>
struct PcDefault {
  static constexpr int N = 1 << LOG2N;
  static constexpr int B = cmax(2, cmin(16, (128 * 1024) / (N * (int)sizeof(R))));
  static constexpr int T = cmax(64, cmin(1024, (B / 2) * N / 16));
};

template <typename R, int LOG2N, int B_, int T_>
struct PcCfg {
  static constexpr int N = 1 << LOG2N;
  static constexpr int B = B_;                             // tile columns (even)
  static constexpr int NSEQ = B / 2;                       // complex sequences
  static constexpr int ELEMS = NSEQ * N;                   // complex elements
  static constexpr int T = T_;
  static constexpr int E = cmax(1, ELEMS / T);             // elements per thread
  static constexpr int MAXLOG = cmax(1, cmin(4, clog2(E)));  // largest radix 2^MAXLOG
  // padded LDS layout: one spare complex slot every 16, plus one per sequence
  static constexpr int SSTRIDE = N + N / 16 + 1;
  static constexpr int LDS_ELEMS = NSEQ * SSTRIDE;
  static constexpr int LDS_BASE = LDS_ELEMS * 2 * (int)sizeof(R) + 3 * B * (int)sizeof(R);
  // the twiddle table e^{-2 pi i m/N} sits in LDS (its global reads would
  // otherwise sit on every FFT pass): whole, first half (w^{m+N/2} = -w^m) or
  // two-level, the largest that keeps the workgroups per CU the tile allows
  static constexpr int TW_BYTES = N * 2 * (int)sizeof(R);
  static constexpr int TW2_BYTES = Split2<N>::SIZE * 2 * (int)sizeof(R);
  static constexpr int WGS = kLdsCap / (LDS_BASE + TW2_BYTES);
  static constexpr int TWMODE = lds_keeps(LDS_BASE, TW_BYTES, WGS)       ? 2
                                : lds_keeps(LDS_BASE, TW_BYTES / 2, WGS) ? 1
                                                                         : 3;
  static constexpr bool TWL = true;
  static constexpr int TWN = TWMODE == 2 ? N : (TWMODE == 1 ? cmax(1, N / 2) : Split2<N>::SIZE);
  static constexpr int LDS_BYTES = LDS_BASE + TWN * 2 * (int)sizeof(R);
  static constexpr int TWPT = (TWN + T - 1) / T;            // table entries per thread
  static constexpr int TASKS = N >= 2 ? N / 2 : 1;          // step-(b) tasks
  static constexpr int NTK = (TASKS + T - 1) / T;           // tasks per thread
};

// Candidate (B, T) variants the create-time autotuner times; index 0 is the
// default.  A candidate is compiled for 64 <= N_t <= 4096 when its tile
// image fits the LDS, every thread owns at least one element and the
// tile-solve registers fit the VGPR budget of its workgroup size.
// S: workgroups per tile of K3.  With S = 2 each workgroup inverts half of
// the tile's sequences (the interface correction, which couples all B
// columns, is formed by both), so K3 needs half the LDS per workgroup and
// runs twice as many workgroups per CU; K1 is the same as for S = 1.
// F = 2 (float32 only): K1 transforms and solves the tile one frequency
// parity at a time (two length-N_t/2 FFTs after one radix-2 decimation-in-
// frequency step, the odd half held in registers meanwhile), in half the
// LDS and at most 128 registers, so two workgroups share a CU and one's
// loads overlap the other's transforms.  The tile image is stored by parity
// and K3 runs by parity as well (S = 1: one workgroup per tile, half the
// LDS, each interface correction formed once).
constexpr int kNumCand = 14;
constexpr int kCandB[kNumCand] = {0, 16, 16, 16, 8, 8, 8, 4, 4, 16, 16, 8, 8, 8};
constexpr int kCandT[kNumCand] = {0, 256, 512, 1024, 256, 512, 1024, 256, 512, 256, 512, 256, 512, 512};
constexpr int kCandS[kNumCand] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 1};
constexpr int kCandF[kNumCand] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 2};

template <typename R, int LOG2N, int CI>
struct PcCand {
  static constexpr int B = CI == 0 ? PcDefault<R, LOG2N>::B : kCandB[CI];
  static constexpr int T = CI == 0 ? PcDefault<R, LOG2N>::T : kCandT[CI];
  static constexpr int S = kCandS[CI];
  static constexpr int F = kCandF[CI];
  using Cfg = PcCfg<R, LOG2N, B, T>;
  using CfgF = PcCfg<R, LOG2N, B / S, T>;  // K3's part of a tile
  using CfgH = PcCfg<R, (LOG2N > 0 ? LOG2N - 1 : 0), B, T>;  // K1's half with F = 2
  static constexpr int HALF_LDS = CfgH::LDS_ELEMS * 2 * (int)sizeof(R) +
                                  Split2<(1 << LOG2N)>::SIZE * 2 * (int)sizeof(R) +
                                  3 * B * (int)sizeof(R);
  static constexpr bool dup =
      CI != 0 && S == 1 && B == PcDefault<R, LOG2N>::B && T == PcDefault<R, LOG2N>::T;
  static constexpr bool ok =
      CI == 0 || (!dup && LOG2N >= 6 && LOG2N <= 12 && Cfg::LDS_BYTES <= kLdsCap &&
                  Cfg::ELEMS >= T && (T < 1024 || B * (int)sizeof(R) <= 64) &&
                  (S == 1 || (B >= 8 && CfgF::ELEMS >= T)) &&
                  (F == 1 || (sizeof(R) == 4 && S == 1 && T == 512 && LOG2N >= 7 && 2 * HALF_LDS <= kLdsCap &&
                              CfgH::ELEMS >= T && ((1 << LOG2N) / 2) % (T / B) == 0)));
};

// threadIdx.x through an empty asm: index arithmetic derived from it cannot be
// hoisted above the call or shared with an earlier phase, so a long kernel
// recomputes its (cheap) per-phase indices instead of keeping them live in
// registers across the whole launch.
template <int T>
__device__ __forceinline__ int phase_tid() {
  static_assert((T & (T - 1)) == 0, "workgroup size must be a power of two");
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t & (T - 1);  // the known range keeps the index arithmetic narrow
}

template <int N>
__device__ __forceinline__ int lidx(int s, int e) {
  return s * (N + N / 16 + 1) + e + (e >> 4);
}

// One Stockham radix-2^LR pass over NSEQ sequences of length N held in LDS.
// p is the product of the radices of earlier passes.  All inputs of the pass
// are read to registers before a barrier, so the pass runs in place.
template <typename R, int N, int NSEQ, int T, bool INV, int LR, int P, typename TW>
__device__ __forceinline__ void fft_pass(Cx<R>* lds, const TW& tw, int tid) {
  constexpr int RAD = 1 << LR;
  constexpr int NQ = N / RAD;             // butterflies per sequence
  constexpr int NB = NSEQ * NQ;           // butterflies in the pass
  constexpr int PER = (NB + T - 1) / T;   // per thread
  Cx<R> u[PER][RAD];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      const int s = b / NQ, i = b % NQ;
#pragma unroll
      for (int r = 0; r < RAD; ++r) u[q][r] = lds[lidx<N>(s, i + r * NQ)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      const int s = b / NQ, i = b % NQ;
      const int k = i & (P - 1);
      if constexpr (P > 1) {
        // twiddle exp(-+2 pi i r k / (P RAD)) = tw[r k N/(P RAD)]
        constexpr int SCL = N / (P * RAD);
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          Cx<R> w = tw(r * k * SCL);
          if (INV) w.y = -w.y;
          u[q][r] = u[q][r] * w;
        }
      }
      Dft<R, RAD, INV>::run(u[q]);
      const int j = (i - k) * RAD + k;
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds[lidx<N>(s, j + r * P)] = u[q][r];
    }
  }
  __syncthreads();
}

// Twiddle staging in two halves so that the table's global reads can be
// issued after (and overlap) the tile's own loads: fetch the first TWN
// entries, then store them to LDS (visible after the next barrier).
template <typename R, int TWN, int T, int TWPT>
struct TwStage {
  Cx<R> v[TWPT];
  template <typename PTR>
  __device__ __forceinline__ void fetch(PTR tw) {
#pragma unroll
    for (int q = 0; q < TWPT; ++q) {
      const int m = threadIdx.x + q * T;
      if (TWN % T == 0 || m < TWN) v[q] = gld(tw + m);
    }
  }
  __device__ __forceinline__ void store(Cx<R>* ltw) {
#pragma unroll
    for (int q = 0; q < TWPT; ++q) {
      const int m = threadIdx.x + q * T;
      if (TWN % T == 0 || m < TWN) ltw[m] = v[q];
    }
  }
};

// Twiddle w^m, m in [0, N), from a full table (HALF = false) or from its
// first half (w^{m+N/2} = -w^m).
template <typename R, int N, bool HALF>
struct TwTab {
  const Cx<R>* t;
  __device__ __forceinline__ Cx<R> operator()(int m) const {
    if constexpr (HALF) {
      const bool up = m >= N / 2;
      const Cx<R> w = t[up ? m - N / 2 : m];
      return up ? Cx<R>{-w.x, -w.y} : w;
    } else {
      return t[m];
    }
  }
};

// Twiddle w^m from the two-level table: w^{m mod SL} w^{SL floor(m/SL)}.
template <typename R, int N>
struct TwTab2 {
  const Cx<R>* t;
  __device__ __forceinline__ Cx<R> operator()(int m) const {
    using S = Split2<N>;
    return t[m & (S::SL - 1)] * t[S::SL + (m >> S::LOGSL)];
  }
};

// Twiddle of the length-N/2 transform, w_{N/2}^m = w_N^{2m}, from the
// two-level table of length N.
template <typename R, int N>
struct TwTab2Half {
  const Cx<R>* t;
  __device__ __forceinline__ Cx<R> operator()(int m) const { return TwTab2<R, N>{t}(2 * m); }
};

template <typename R, int LOG2N, int NSEQ, int T, bool INV, int MAXLOG, int DONE, typename TW>
__device__ __forceinline__ void fft_run(Cx<R>* lds, const TW& tw, int tid) {
  if constexpr (DONE < LOG2N) {
    constexpr int LR = (DONE == 0 && (LOG2N % MAXLOG) != 0) ? (LOG2N % MAXLOG) : MAXLOG;
    fft_pass<R, (1 << LOG2N), NSEQ, T, INV, LR, (1 << DONE)>(lds, tw, tid);
    fft_run<R, LOG2N, NSEQ, T, INV, MAXLOG, DONE + LR>(lds, tw, tid);
  }
}

// Forward transform of length NH = N/2 whose input, when `pre` is set, is
// first multiplied elementwise by w_N^e (e = 0..NH-1): the odd-frequency
// half of a length-N transform split by decimation in frequency.  The
// multiplication is folded into the first pass, which reads every element
// once; all twiddles come from the two-level table of length N in LDS.
template <typename R, int LOG2N, int NSEQ, int T, int MAXLOG>
__device__ __forceinline__ void fft_half(Cx<R>* lds, const Cx<R>* ltw, int tid, bool pre) {
  constexpr int N = 1 << LOG2N, LOGH = LOG2N - 1, NH = N / 2;
  constexpr int LR = (LOGH % MAXLOG) != 0 ? (LOGH % MAXLOG) : MAXLOG;
  constexpr int RAD = 1 << LR;
  constexpr int NQ = NH / RAD;
  constexpr int NB = NSEQ * NQ;
  constexpr int PER = (NB + T - 1) / T;
  const TwTab2<R, N> twf{ltw};
  Cx<R> u[PER][RAD];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      const int s = b / NQ, i = b % NQ;
#pragma unroll
      for (int r = 0; r < RAD; ++r) u[q][r] = lds[lidx<NH>(s, i + r * NQ)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      const int s = b / NQ, i = b % NQ;
      if (pre) {
#pragma unroll
        for (int r = 0; r < RAD; ++r) u[q][r] = u[q][r] * twf(i + r * NQ);
      }
      Dft<R, RAD, false>::run(u[q]);
      // first pass (P = 1): output j = i RAD + r
#pragma unroll
      for (int r = 0; r < RAD; ++r) lds[lidx<NH>(s, i * RAD + r)] = u[q][r];
    }
  }
  __syncthreads();
  fft_run<R, LOGH, NSEQ, T, false, MAXLOG, LR>(lds, TwTab2Half<R, N>{ltw}, tid);
}

// FFT with the twiddles from the LDS table staged as Cfg says.
// tid: the thread index the passes derive their element indices from (one
// opaque value per transform, see phase_tid)
template <typename Cfg, typename R, int LOG2N, bool INV>
__device__ __forceinline__ void fft_tile(Cx<R>* lds, const Cx<R>* ltw, const Cx<R>* __restrict__ tw,
                                         int tid) {
  constexpr int N = 1 << LOG2N;
  (void)tw;
  if constexpr (Cfg::TWMODE == 2) {
    fft_run<R, LOG2N, Cfg::NSEQ, Cfg::T, INV, Cfg::MAXLOG, 0>(lds, TwTab<R, N, false>{ltw}, tid);
  } else if constexpr (Cfg::TWMODE == 1) {
    fft_run<R, LOG2N, Cfg::NSEQ, Cfg::T, INV, Cfg::MAXLOG, 0>(lds, TwTab<R, N, true>{ltw}, tid);
  } else {
    fft_run<R, LOG2N, Cfg::NSEQ, Cfg::T, INV, Cfg::MAXLOG, 0>(lds, TwTab2<R, N>{ltw}, tid);
  }
}

// ---------------------------------------------------------------------------
// Tile-local solve of (mu I - A~) restricted to the nb interior columns of a
// tile (rows b = 0..nb-1, global column i0 + b).  Couplings to the columns
// left of b = 0 and right of b = nb-1 are excluded (they are the interface
// unknowns of the partitioned solve).  Plain Thomas elimination, no pivoting
// (the matrix is strictly diagonally dominant for 0 < alpha < 1).
// C is Cx<R> for a complex shift, R for a real one.  lo/di/up hold tau*A.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ Cx<R> shift_sub(Cx<R> mu, R d) { return {mu.x - d, mu.y}; }
template <typename R>
__device__ __forceinline__ R shift_sub(R mu, R d) { return mu - d; }
template <typename R>
__device__ __forceinline__ Cx<R> zero_of(Cx<R>) { return {R(0), R(0)}; }
template <typename R>
__device__ __forceinline__ R zero_of(R) { return R(0); }
template <typename R>
__device__ __forceinline__ Cx<R> axpy_r(Cx<R> a, R s, Cx<R> b) {  // a - s*b
  return {a.x - s * b.x, a.y - s * b.y};
}
__device__ __forceinline__ double axpy_r(double a, double s, double b) { return a - s * b; }
__device__ __forceinline__ float axpy_r(float a, float s, float b) { return a - s * b; }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) { return a * b; }
__device__ __forceinline__ double cmul(double a, double b) { return a * b; }
__device__ __forceinline__ float cmul(float a, float b) { return a * b; }
template <typename R>
__device__ __forceinline__ Cx<R> rmul(R s, Cx<R> a) { return {s * a.x, s * a.y}; }
__device__ __forceinline__ double rmul(double s, double a) { return s * a; }
__device__ __forceinline__ float rmul(float s, float a) { return s * a; }

// co: LDS, per column b of the tile: co[3b] = lo, co[3b+1] = di, co[3b+2] = up
template <typename R, typename C, int B>
__device__ __forceinline__ void tile_solve(C (&d)[B], C mu, const R* co, int nb) {
  C c[B];
  C yp = zero_of(mu);
  C cp = zero_of(mu);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if (b < nb) {
      const R lb = (b == 0) ? R(0) : -co[3 * b];
      // pivot = (mu - di) - lb * c_{b-1}
      const C piv = axpy_r(shift_sub(mu, co[3 * b + 1]), lb, cp);
      const C q = crcp(piv);
      cp = (b < nb - 1) ? rmul(-co[3 * b + 2], q) : zero_of(mu);
      c[b] = cp;
      yp = cmul(axpy_r(d[b], lb, yp), q);
      d[b] = yp;
    }
  }
#pragma unroll
  for (int b = B - 2; b >= 0; --b) {
    if (b < nb - 1) d[b] = d[b] - cmul(c[b], d[b + 1]);
  }
}

// Remap a flat workgroup index so that consecutive tiles run on the same XCD
// (workgroups are dealt round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_tile(int wg, int nwg_padded) {
  const int per = nwg_padded >> 3;
  return (wg & 7) * per + (wg >> 3);
}

}  // namespace cn
