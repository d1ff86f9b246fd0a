// Host runtime of libcn_aao: the opaque handles (one problem, or a batch of
// uneven problems), argument validation, the float64 tables of the
// alpha-circulant diagonalisation (Sec. 3.1), the workspace, the
// create-time autotuner and the GMRES(m) driver.  Every computational step
// runs in the kernels of cn_pc*.hip and cn_krylov.hip; a handle is a launch
// context of one instance descriptor, a batch concatenates the descriptors
// and work lists of its instances so that each step is one launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cn_internal.hpp"

using namespace cn;

static thread_local std::string g_err;

// Autotuned transform variant per (precision, log2 N_t, N_x) on this device:
// kept per process, and on disk so that later processes skip the timing.  The
// file (CN_TUNE_CACHE, else $XDG_CACHE_HOME/cn_aao/tune.txt, else
// $HOME/.cache/cn_aao/tune.txt; CN_TUNE_CACHE="" turns it off) holds one line
// per choice: tag, device, precision, log2 N_t, N_x, tile width, workgroup
// size.  The tag is the build time of this library, so a rebuilt library
// tunes again; the device is its architecture name and compute-unit count.
struct TuneKey {
  int prec, log2n, nx;
  bool operator<(const TuneKey& o) const {
    return std::tie(prec, log2n, nx) < std::tie(o.prec, o.log2n, o.nx);
  }
};
static std::mutex g_tune_mu;
static std::map<TuneKey, int> g_tune;

static std::string tune_tag() {
  std::string t = __DATE__ "T" __TIME__;
  for (char& c : t)
    if (c == ' ') c = '_';
  return t;
}

static std::string tune_device() {
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess)
    return "";
  std::string a = pr.gcnArchName;
  for (char& c : a)
    if (c == ' ') c = '_';
  return a + "/" + std::to_string(pr.multiProcessorCount);
}

static std::string tune_path() {
  if (const char* e = getenv("CN_TUNE_CACHE")) return e;
  const char* x = getenv("XDG_CACHE_HOME");
  if (x != nullptr && *x) return std::string(x) + "/cn_aao/tune.txt";
  const char* hm = getenv("HOME");
  if (hm != nullptr && *hm) return std::string(hm) + "/.cache/cn_aao/tune.txt";
  return "";
}

// Compiled candidate of `cands` recorded for key (process map, then file), or -1.
static int tune_lookup(const TuneKey& k, const std::vector<int>& cands) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(k);
  if (it != g_tune.end() && std::find(cands.begin(), cands.end(), it->second) != cands.end())
    return it->second;
  const std::string path = tune_path(), dev = tune_device(), tag = tune_tag();
  if (path.empty() || dev.empty()) return -1;
  FILE* f = fopen(path.c_str(), "r");
  if (f == nullptr) return -1;
  int found = -1;
  char line[512], ftag[128], fdev[256];
  while (fgets(line, sizeof line, f) != nullptr) {
    int pr = -1, l2 = -1, nx = -1, B = 0, T = 0, S = 0, FS = 1;
    // (a line without the ninth field, the K1 split, means 1)
    if (sscanf(line, "%127s %255s %d %d %d %d %d %d %d", ftag, fdev, &pr, &l2, &nx, &B, &T, &S,
               &FS) < 8)
      continue;
    if (tag != ftag || dev != fdev || pr != k.prec || l2 != k.log2n || nx != k.nx) continue;
    for (int ci : cands) {
      int cb = 0, ct = 0, cs = 0, cf = 0;
      if (pc_candidate(k.prec, k.log2n, ci, &cb, &ct, &cs, &cf) && cb == B && ct == T && cs == S &&
          cf == FS)
        found = ci;
    }
  }
  fclose(f);
  if (found >= 0) g_tune[k] = found;
  return found;
}

static void tune_store(const TuneKey& k, int ci) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[k] = ci;
  const std::string path = tune_path(), dev = tune_device();
  int B = 0, T = 0, S = 0, FS = 1;
  if (path.empty() || dev.empty() || !pc_candidate(k.prec, k.log2n, ci, &B, &T, &S, &FS)) return;
  // create the directory levels of the default location (failures only
  // mean that nothing is kept)
  for (size_t p = path.find('/', 1); p != std::string::npos; p = path.find('/', p + 1))
    (void)mkdir(path.substr(0, p).c_str(), 0755);
  FILE* f = fopen(path.c_str(), "a");
  if (f == nullptr) return;
  fprintf(f, "%s %s %d %d %d %d %d %d %d\n", tune_tag().c_str(), dev.c_str(), k.prec, k.log2n, k.nx,
          B, T, S, FS);
  fclose(f);
}

static cn_status fail(cn_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      return fail(e_ == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP,                      \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    }                                                                                   \
  } while (0)

// work lists of one launch context (device arrays)
struct WorkLists {
  int2* pc = nullptr;   // (instance, tile) for the transform kernels
  int2* k2 = nullptr;   // (instance, frequency) for the interface solve
  int2* mv = nullptr;   // (instance, matvec block)
  int2* st = nullptr;   // (instance, streaming block)
  Items I_pc, I_k2, I_mv, I_st;
  void release() {
    for (int2* p : {pc, k2, mv, st})
      if (p != nullptr) (void)hipFree(p);
    pc = k2 = mv = st = nullptr;
    I_pc = I_k2 = I_mv = I_st = Items{};
  }
};

static hipError_t upload_items(const std::vector<int2>& v, int2** dptr, Items* it) {
  if (*dptr != nullptr) {
    (void)hipFree(*dptr);
    *dptr = nullptr;
  }
  *it = Items{};
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dptr, v.size() * sizeof(int2));
  if (e == hipSuccess) e = hipMemcpy(*dptr, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    it->it = *dptr;
    it->n = (int)v.size();
  }
  return e;
}


struct cn_aao {
  int nx = 0, nt = 0, m_max = 0, flags = 0;
  double T = 0, alpha = 0, tau = 0;
  int prec = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  long long n = 0, npad = 0;
  int ldx = 0;        // internal row pitch (N_x rounded up to 16, padded, see create)
  long long pgrid = 0;  // partial sums per dot (largest grid of a reducing kernel)
  long long nin = 0;  // N_t ldx
  PcPlan pl;
  double* dw = nullptr;   // time weights (device) or null
  double* V = nullptr;    // (m_max+1) x npad float64
  void* Z = nullptr;      // m_max x npad, float64 or float32
  double* w = nullptr;    // npad
  double* partials = nullptr;
  GState* st = nullptr;
  GSummary* hsum = nullptr;      // pinned coherent host memory, 4 slots
  GSummary* hsum_dev = nullptr;  // the same slots as seen by kernels
  int seqc = 0;                  // last sequence number handed to a kernel
  // launch context: one descriptor and its work lists
  InstDesc desc{};
  InstDesc* d_desc = nullptr;
  StopCtl* d_ctl = nullptr;        // stopping controls (device) and their host
  StopCtl* h_ctl = nullptr;        // staging copy (pinned); see SolveCtx::ctl
  StopCtl last_ctl{1.0, 0, 0};     // what the device holds
  WorkLists wl;
  Launch L{};
  int k2_thr = 32 * 16;  // interface-solve variant (k2_chunk_class)
  std::vector<void*> dev_allocs;
  std::vector<double> rt;    // remembered rtol target (SolveCtx::rt)
  double rt_for[2] = {0.0, 0.0};
};

static void release(cn_aao* h) {
  if (h == nullptr) return;
  (void)hipStreamSynchronize(h->stream);
  h->wl.release();
  for (void* p : h->dev_allocs) (void)hipFree(p);
  if (h->hsum != nullptr) (void)hipHostFree(h->hsum);
  if (h->h_ctl != nullptr) (void)hipHostFree(h->h_ctl);
  delete h;
}

template <typename P>
static hipError_t dalloc(cn_aao* h, P** ptr, size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes > 0 ? bytes : 16);
  if (e == hipSuccess) {
    h->dev_allocs.push_back(p);
    *ptr = (P*)p;
  }
  return e;
}

static bool overlaps(const void* a, const void* b, size_t bytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

// Fill the instance descriptor of h from its plan and workspace.
static void fill_desc(cn_aao* h, InstDesc* d) {
  d->pl = h->pl;
  d->dw = h->dw;
  d->nx = h->nx;
  d->nt = h->nt;
  d->rows = matvec_rows(h->nx, h->nt);
  d->mv_cols = (h->nx + MVT - 1) / MVT;
  d->mv_grid = d->mv_cols * ((h->nt + d->rows - 1) / d->rows);
  d->st_grid = stream_grid(h->nin);
  d->n = h->n;
  d->ldx = h->ldx;
  d->nin = h->nin;
  d->vstride = h->npad;
  d->off = 0;
  d->V = h->V;
  d->Z = h->Z;
  d->w = h->w;
  d->partials = h->partials;
  d->partials2 = h->partials + h->pgrid * NVMAX;
  d->st = h->st;
  d->host = h->hsum_dev;
  d->zf = h->prec;
  int zl = 0;
  while ((1 << zl) < h->pl.B) ++zl;
  d->zlog = zl;
  d->ctl = h->d_ctl;
}

// Work items of one instance (appended with instance index `inst`).
static void append_items(const InstDesc& d, int inst, std::vector<int2>* pc, std::vector<int2>* k2,
                         std::vector<int2>* mv, std::vector<int2>* stv) {
  if (pc != nullptr)
    for (int p = 0; p < d.pl.P; ++p) pc->push_back(make_int2(inst, p));
  if (k2 != nullptr && d.pl.NS > 0)
    for (int j = 0; j < d.pl.F; ++j) k2->push_back(make_int2(inst, j));
  if (mv != nullptr)
    for (int b = 0; b < d.mv_grid; ++b) mv->push_back(make_int2(inst, b));
  if (stv != nullptr)
    for (int b = 0; b < d.st_grid; ++b) stv->push_back(make_int2(inst, b));
}

// (Re)build the one-instance launch context of h.
static hipError_t build_launch(cn_aao* h) {
  fill_desc(h, &h->desc);
  hipError_t e = hipMemcpy(h->d_desc, &h->desc, sizeof(InstDesc), hipMemcpyHostToDevice);
  std::vector<int2> pc, k2, mv, stv;
  append_items(h->desc, 0, &pc, &k2, &mv, &stv);
  if (e == hipSuccess) e = upload_items(pc, &h->wl.pc, &h->wl.I_pc);
  if (e == hipSuccess) e = upload_items(k2, &h->wl.k2, &h->wl.I_k2);
  if (e == hipSuccess) e = upload_items(mv, &h->wl.mv, &h->wl.I_mv);
  if (e == hipSuccess) e = upload_items(stv, &h->wl.st, &h->wl.I_st);
  h->L = Launch{h->d_desc, 1, h->prec};
  // one instance: kernels derive the work items from the block index, which
  // saves a dependent load at the start of every workgroup
  h->wl.I_pc.it = h->wl.I_k2.it = h->wl.I_mv.it = h->wl.I_st.it = nullptr;
  h->k2_thr = k2_chunk_class(h->pl.NS, h->prec);
  // CN_K2_CLASS=32W+CH forces an interface-solve variant (tests); a
  // register variant too small for the chunk falls back to the default
  if (const char* f = getenv("CN_K2_CLASS")) {
    const int c = atoi(f);
    if (c >= K2_ROUNDS) {  // rounds layout: two rounds of 4096 separators
      if (c == K2_ROUNDS + 2 && h->pl.NS <= 2 * 4096) h->k2_thr = c;
    } else if (c >= 4096) {  // strided layout: blocks of 1024 separators per lane set
      const int ch = c - 4096, blocks = (h->pl.NS + 1023) / 1024;
      if ((ch == 1 || ch == 2 || ch == 4 || ch == 8 || ch == 16) && blocks <= ch) h->k2_thr = c;
    } else {
      const int w = c / 32, ch = c % 32;
      const int chunk = (h->pl.NS + 64 * w - 1) / (64 * std::max(w, 1));
      const bool known = (w == 1 || w == 4 || w == 8 || w == 16) &&
                         (ch == 0 ? w == 16 : (ch == 1 || ch == 2 || ch == 4 || (ch == 8 && w < 16)));
      if (known && (ch == 0 || chunk <= ch)) h->k2_thr = c;
    }
  }
  return e;
}

// Spin until a kernel has published sequence number `seq` into `slot`
// (coherent pinned host memory), then copy the summary out.
static cn_status wait_slot(hipStream_t stream, GSummary* slot, int seq, GSummary* out) {
  volatile int* p = &slot->seq;
  long spins = 0;
  while (*p != seq) {
    if ((++spins & 4095) == 0) {
      const hipError_t e = hipStreamQuery(stream);
      if (e != hipSuccess && e != hipErrorNotReady)
        return fail(CN_EHIP, std::string("solver stream: ") + hipGetErrorString(e));
      if (e == hipSuccess && *p != seq)
        return fail(CN_EHIP, "solver kernels finished without publishing their summary");
    }
    __builtin_ia32_pause();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  volatile GSummary* v = slot;
  out->bnorm = v->bnorm;
  out->beta = v->beta;
  out->est = v->est;
  out->relres = v->relres;
  out->k = v->k;
  out->done = v->done;
  out->breakdown = v->breakdown;
  out->x0_rejected = v->x0_rejected;
  out->seq = seq;
  return CN_OK;
}

#define CN_TRY(expr)               \
  do {                             \
    const cn_status st_ = (expr);  \
    if (st_ != CN_OK) return st_;  \
  } while (0)

extern "C" {
const char* cn_status_string(cn_status s) {
  switch (s) {
    case CN_OK: return "ok";
    case CN_NOT_CONVERGED: return "not converged";
    case CN_EINVAL: return "invalid argument";
    case CN_ENOMEM: return "out of device memory";
    case CN_EHIP: return "HIP runtime error";
    case CN_ESINGULAR: return "singular shifted system";
  }
  return "unknown status";
}

const char* cn_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// Create a handle; force_cand >= 0 skips autotuning and uses that variant.
static cn_status create_handle(const cn_problem* p, int force_cand, cn_aao** out) {
  if (out == nullptr) return fail(CN_EINVAL, "out is NULL");
  *out = nullptr;
  if (p == nullptr) return fail(CN_EINVAL, "problem is NULL");
  if (p->nx < 1) return fail(CN_EINVAL, "nx must be >= 1");
  if (p->nt < 1 || p->nt > 8192 || (p->nt & (p->nt - 1)) != 0)
    return fail(CN_EINVAL, "nt must be a power of two in [1, 8192]");
  // the transform reads a tile's column block through 32-bit byte offsets
  if ((unsigned long long)p->nt * ((p->nx + 15) / 16 * 16) * 8 >= (1ull << 32))
    return fail(CN_EINVAL, "nt * nx must stay below 2^29 (about 5.4e8 unknowns per instance)");
  if (p->m_max < 1 || p->m_max > MMAX) return fail(CN_EINVAL, "m_max must be in [1, 64]");
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(CN_EINVAL, "T must be finite and > 0");
  const bool allow1 = (p->flags & CN_FLAG_ALLOW_ALPHA_ONE) != 0;
  if (!(p->alpha > 0.0) || !(p->alpha < 1.0 || (allow1 && p->alpha == 1.0)))
    return fail(CN_EINVAL, "alpha must satisfy 0 < alpha < 1 (alpha = 1 needs CN_FLAG_ALLOW_ALPHA_ONE)");
  if (p->pc_prec != CN_PC_FP64 && p->pc_prec != CN_PC_FP32)
    return fail(CN_EINVAL, "pc_prec must be CN_PC_FP64 or CN_PC_FP32");
  if (p->a_lo == nullptr || p->a_di == nullptr || p->a_up == nullptr)
    return fail(CN_EINVAL, "A diagonals must be device pointers");
  const long long n = (long long)p->nx * p->nt;
  if (n > (1LL << 40)) return fail(CN_EINVAL, "problem too large");

  cn_aao* h = new cn_aao();
  h->nx = p->nx;
  h->nt = p->nt;
  h->m_max = p->m_max;
  h->flags = p->flags;
  h->T = p->T;
  h->alpha = p->alpha;
  h->tau = p->T / p->nt;
  h->prec = p->pc_prec == CN_PC_FP32 ? 1 : 0;
  h->stream = (hipStream_t)p->stream;
  h->n = n;
  // Row pitch: N_x rounded up to 16.  A pitch that is a multiple of 8 KB puts
  // the rows of a tile at one offset modulo a large power of two, and with
  // vectors beyond the last-level cache the transforms' 64-byte row reads
  // then crowd a few HBM channels: such a pitch is padded by 128 bytes
  // (65535 x 4096: K1 1002 -> 824 us, the two Krylov passes about 2 % slower,
  // a net 2-3 % per inner iteration; 2 KB and 8 KB pads gained less, 4 KB lost;
  // cache-resident sizes are left alone).
  h->ldx = (p->nx + 15) / 16 * 16;
  if (h->ldx % 1024 == 0 && (long long)p->nt * h->ldx * (long long)sizeof(double) > (256LL << 20))
    h->ldx += 16;
  h->nin = (long long)p->nt * h->ldx;
  h->npad = (h->nin + 63) / 64 * 64;
  auto bail = [&](cn_status s) {
    release(h);
    return s;
  };
#define TRY(expr)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      fail(e_ == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP,                              \
           std::string(#expr) + ": " + hipGetErrorString(e_));                           \
      return bail(e_ == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP);                      \
    }                                                                                    \
  } while (0)
  TRY(hipGetDevice(&h->device));

  // -- operator rows: A~ = tau A, boundary entries cleared ----------------------
  const int nx = h->nx, nt = h->nt;
  std::vector<double> lo(nx), di(nx), up(nx);
  TRY(hipMemcpy(lo.data(), p->a_lo, nx * sizeof(double), hipMemcpyDeviceToHost));
  TRY(hipMemcpy(di.data(), p->a_di, nx * sizeof(double), hipMemcpyDeviceToHost));
  TRY(hipMemcpy(up.data(), p->a_up, nx * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < nx; ++i) {
    if (i == 0) lo[i] = 0.0;
    if (i == nx - 1) up[i] = 0.0;
    if (!std::isfinite(lo[i]) || !std::isfinite(di[i]) || !std::isfinite(up[i])) {
      fail(CN_EINVAL, "A has non-finite entries");
      return bail(CN_EINVAL);
    }
    lo[i] *= h->tau;
    di[i] *= h->tau;
    up[i] *= h->tau;
  }
  double dbar = 1.0;
  std::vector<double> dw;
  if (p->d_half != nullptr) {
    dw.resize(nt);
    TRY(hipMemcpy(dw.data(), p->d_half, nt * sizeof(double), hipMemcpyDeviceToHost));
    long double s = 0;
    for (int k = 0; k < nt; ++k) {
      if (!std::isfinite(dw[k]) || !(dw[k] > 0.0)) {
        fail(CN_EINVAL, "time weights must be finite and > 0");
        return bail(CN_EINVAL);
      }
      s += dw[k];
    }
    dbar = (double)(s / nt);
  }

  // -- plan -----------------------------------------------------------------------
  PcPlan& pl = h->pl;
  pl.nx = nx;
  pl.nt = nt;
  pl.log2n = 0;
  while ((1 << pl.log2n) < nt) ++pl.log2n;
  pl.F = nt / 2 + 1;
  pl.prec = h->prec;
  pl.alpha = h->alpha;
  pl.dbar = dbar;
  const size_t rsz = pl.prec ? sizeof(float) : sizeof(double);
  // compiled (B, T) variants of the transform kernels for this N_t
  std::vector<int> cands;
  for (int ci = 0; ci < kNumCand; ++ci) {
    int B = 0, T = 0;
    if (pc_candidate(pl.prec, pl.log2n, ci, &B, &T)) cands.push_back(ci);
  }
  {
    // CN_PC_TILE="B,T", "B,T,S" or "B,T,S,F" forces a variant (S: K3
    // workgroups per tile, F = 2: K1 by frequency parity; 1 if not given);
    // CN_AUTOTUNE=0 keeps the default
    const char* force = getenv("CN_PC_TILE");
    const char* at = getenv("CN_AUTOTUNE");
    int fb = 0, ft = 0, fs = 1, ff = 1;
    if (force != nullptr && sscanf(force, "%d,%d,%d,%d", &fb, &ft, &fs, &ff) >= 2) {
      std::vector<int> keep;
      for (int ci : cands) {
        int B = 0, T = 0, S = 0, FS = 0;
        pc_candidate(pl.prec, pl.log2n, ci, &B, &T, &S, &FS);
        if (B == fb && T == ft && S == fs && FS == ff) keep.push_back(ci);
      }
      if (keep.empty()) {
        fail(CN_EINVAL, std::string("CN_PC_TILE=") + force + " is not a compiled variant");
        return bail(CN_EINVAL);
      }
      cands = keep;
    } else if (at != nullptr && at[0] == '0') {
      cands.assign(1, 0);
    }
    if (force_cand >= 0) {
      int B = 0, T = 0;
      if (!pc_candidate(pl.prec, pl.log2n, force_cand, &B, &T)) {
        fail(CN_EINVAL, "requested transform variant is not compiled");
        return bail(CN_EINVAL);
      }
      cands.assign(1, force_cand);
    }
  }
  // buffers sized for the most demanding candidate
  size_t spec_elems = 0, nsep_max = 1, ptile_max = 1;
  for (int ci : cands) {
    int B = 0, T = 0;
    pc_candidate(pl.prec, pl.log2n, ci, &B, &T);
    const size_t P = (size_t)(nx + B - 1) / B;
    spec_elems = std::max(spec_elems, P * B * (size_t)nt);
    ptile_max = std::max(ptile_max, P);
    nsep_max = std::max(nsep_max, P > 1 ? P - 1 : (size_t)1);
  }

  // workspace size check against free memory
  size_t need = 0;
  need += (size_t)(h->m_max + 1) * h->npad * sizeof(double);         // V
  need += (size_t)h->m_max * h->npad * rsz;                           // Z
  need += (size_t)h->npad * sizeof(double);                           // w
  need += spec_elems * rsz;                                           // spectrum tiles
  need += (size_t)pl.F * ptile_max * 2 * 2 * rsz;                     // interface values
  need += (size_t)pl.F * nsep_max * 2 * rsz + (size_t)pl.F * nsep_max * 4 * sizeof(Cx<double>);
  need += (size_t)pl.F * ptile_max * 4 * sizeof(Cx<double>);          // set-up spikes
  size_t freeb = 0, totalb = 0;
  TRY(hipMemGetInfo(&freeb, &totalb));
  if (need + (64u << 20) > freeb) {
    fail(CN_ENOMEM, "workspace of " + std::to_string(need) + " bytes does not fit in " +
                        std::to_string(freeb) + " free bytes");
    return bail(CN_ENOMEM);
  }

  TRY(dalloc(h, &pl.lo, nx * sizeof(double)));
  TRY(dalloc(h, &pl.di, nx * sizeof(double)));
  TRY(dalloc(h, &pl.up, nx * sizeof(double)));
  TRY(hipMemcpy(pl.lo, lo.data(), nx * sizeof(double), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.di, di.data(), nx * sizeof(double), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.up, up.data(), nx * sizeof(double), hipMemcpyHostToDevice));
  if (!dw.empty()) {
    TRY(dalloc(h, &h->dw, nt * sizeof(double)));
    TRY(hipMemcpy(h->dw, dw.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  }

  // -- float64 tables (computed in long double) -------------------------------------
  const long double la = logl((long double)h->alpha);
  const long double PI = 3.141592653589793238462643383279502884L;
  std::vector<double> wfw(nt), winv(nt);
  std::vector<Cx<double>> tw(nt), mu(pl.F), il2(pl.F);
  std::vector<Cx<float>> twf(nt);
  for (int k = 0; k < nt; ++k) {
    wfw[k] = (double)expl(la * k / nt);                  // alpha^{k/N_t}
    winv[k] = (double)(expl(-la * k / nt) / nt);         // alpha^{-k/N_t} / N_t
    const long double ang = -2.0L * PI * k / nt;         // omega^k, omega = e^{-2 pi i/N_t}
    tw[k] = Cx<double>{(double)cosl(ang), (double)sinl(ang)};
    twf[k] = Cx<float>{(float)tw[k].x, (float)tw[k].y};
  }
  const int wsl = std::min(nt, 64), wsh = nt / wsl;   // two-level twiddle table
  std::vector<Cx<double>> tw2(wsl + wsh);
  std::vector<Cx<float>> tw2f(wsl + wsh);
  for (int e = 0; e < wsl + wsh; ++e) {
    const int k = e < wsl ? e : (e - wsl) * wsl;
    tw2[e] = tw[k];
    tw2f[e] = twf[k];
  }
  const long double a1 = expl(la / nt);                  // alpha^{1/N_t}
  for (int j = 0; j < pl.F; ++j) {
    // omega^j; the modes j = 0 and j = N_t/2 are real (omega^j = +-1 exactly)
    long double wr, wi;
    if (j == 0) {
      wr = 1.0L;
      wi = 0.0L;
    } else if (2 * j == nt) {
      wr = -1.0L;
      wi = 0.0L;
    } else {
      const long double ang = -2.0L * PI * j / nt;
      wr = cosl(ang);
      wi = sinl(ang);
    }
    // lambda_1 = 1 - a omega^j, lambda_2 = dbar (1 + a omega^j) / 2
    const long double l1r = 1.0L - a1 * wr, l1i = -a1 * wi;
    long double l2r = 0.5L * dbar * (1.0L + a1 * wr), l2i = 0.5L * dbar * a1 * wi;
    // lambda_2 vanishes only for alpha = 1 at j = N_t/2, where the shifted
    // system reduces to lambda_1 I; a relative floor of 1e-15 keeps the
    // (mu I - A~)/lambda_2 form finite (a perturbation far below rounding)
    const long double l1m = sqrtl(l1r * l1r + l1i * l1i);
    if (sqrtl(l2r * l2r + l2i * l2i) < 1e-15L * l1m) {
      l2r = 1e-15L * l1m;
      l2i = 0.0L;
    }
    const long double den = l2r * l2r + l2i * l2i;
    mu[j] = Cx<double>{(double)((l1r * l2r + l1i * l2i) / den),
                       (double)((l1i * l2r - l1r * l2i) / den)};
    il2[j] = Cx<double>{(double)(l2r / den), (double)(-l2i / den)};
  }
  TRY(dalloc(h, &pl.wfw, nt * sizeof(double)));
  TRY(dalloc(h, &pl.winv, nt * sizeof(double)));
  TRY(dalloc(h, &pl.tw, nt * sizeof(Cx<double>)));
  TRY(dalloc(h, &pl.tw_f, nt * sizeof(Cx<float>)));
  TRY(dalloc(h, &pl.mu, pl.F * sizeof(Cx<double>)));
  TRY(dalloc(h, &pl.il2, pl.F * sizeof(Cx<double>)));
  TRY(hipMemcpy(pl.wfw, wfw.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.winv, winv.data(), nt * sizeof(double), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.tw, tw.data(), nt * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.tw_f, twf.data(), nt * sizeof(Cx<float>), hipMemcpyHostToDevice));
  TRY(dalloc(h, &pl.tw2, (wsl + wsh) * sizeof(Cx<double>)));
  TRY(dalloc(h, &pl.tw2_f, (wsl + wsh) * sizeof(Cx<float>)));
  TRY(hipMemcpy(pl.tw2, tw2.data(), (wsl + wsh) * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.tw2_f, tw2f.data(), (wsl + wsh) * sizeof(Cx<float>), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.mu, mu.data(), pl.F * sizeof(Cx<double>), hipMemcpyHostToDevice));
  TRY(hipMemcpy(pl.il2, il2.data(), pl.F * sizeof(Cx<double>), hipMemcpyHostToDevice));

  // -- GMRES basis (also the autotuner's scratch) and solver state -------------------
  TRY(dalloc(h, &h->V, (size_t)(h->m_max + 1) * h->npad * sizeof(double)));
  TRY(dalloc(h, &h->Z, (size_t)h->m_max * h->npad * rsz));
  TRY(dalloc(h, &h->w, (size_t)h->npad * sizeof(double)));
  // the pad columns of V and w take part in the Gram-Schmidt passes as zeros
  TRY(hipMemsetAsync(h->V, 0, (size_t)(h->m_max + 1) * h->npad * sizeof(double), h->stream));
  TRY(hipMemsetAsync(h->w, 0, (size_t)h->npad * sizeof(double), h->stream));
  {
    const int rows = matvec_rows(nx, nt);
    const long long mgrid = (long long)((nx + MVT - 1) / MVT) * ((nt + rows - 1) / rows);
    h->pgrid = std::max<long long>(mgrid, stream_grid(h->nin));
    TRY(dalloc(h, &h->partials, (size_t)2 * h->pgrid * NVMAX * sizeof(double)));
  }
  TRY(dalloc(h, &h->st, sizeof(GState)));
  TRY(hipMemsetAsync(h->st, 0, sizeof(GState), h->stream));
  TRY(hipHostMalloc((void**)&h->hsum, 4 * sizeof(GSummary),
                    hipHostMallocCoherent | hipHostMallocMapped));
  memset(h->hsum, 0, 4 * sizeof(GSummary));
  TRY(hipHostGetDevicePointer((void**)&h->hsum_dev, h->hsum, 0));
  TRY(dalloc(h, &h->d_desc, sizeof(InstDesc)));
  TRY(dalloc(h, &h->d_ctl, sizeof(StopCtl)));
  TRY(hipHostMalloc((void**)&h->h_ctl, sizeof(StopCtl), hipHostMallocDefault));
  *h->h_ctl = h->last_ctl;
  TRY(hipMemcpyAsync(h->d_ctl, h->h_ctl, sizeof(StopCtl), hipMemcpyHostToDevice, h->stream));

  // -- preconditioner workspace, interface factorisation, variant choice -------------
  TRY(dalloc(h, &pl.spec, spec_elems * rsz));
  TRY(dalloc(h, &pl.iface, (size_t)pl.F * ptile_max * 2 * 2 * rsz));
  TRY(dalloc(h, &pl.sep, (size_t)pl.F * nsep_max * 2 * rsz));
  TRY(dalloc(h, &pl.recf, (size_t)pl.F * nsep_max * 2 * 2 * rsz));
  TRY(dalloc(h, &pl.recb, (size_t)pl.F * nsep_max * 2 * rsz));
  TRY(dalloc(h, &pl.red_tmp, (size_t)pl.F * nsep_max * sizeof(Cx<double>)));
  {
    Cx<double>* spk = nullptr;
    int* err = nullptr;
    TRY(hipMalloc((void**)&spk, (size_t)pl.F * ptile_max * 4 * sizeof(Cx<double>)));
    if (hipMalloc((void**)&err, sizeof(int)) != hipSuccess) {
      (void)hipFree(spk);
      fail(CN_ENOMEM, "set-up flag");
      return bail(CN_ENOMEM);
    }
    auto free_tmp = [&]() {
      (void)hipStreamSynchronize(h->stream);
      (void)hipFree(spk);
      (void)hipFree(err);
    };
    // set up the interface factors and launch context of candidate ci
    auto setup = [&](int ci, int* singular) -> hipError_t {
      int B = 0, T = 0, S = 1, FS = 1;
      pc_candidate(pl.prec, pl.log2n, ci, &B, &T, &S, &FS);
      pl.cand = ci;
      pl.B = B;
      pl.T = T;
      pl.S = S;
      pl.FS = FS;
      pl.P = (nx + B - 1) / B;
      pl.NS = pl.P - 1;
      hipError_t e = hipMemsetAsync(err, 0, sizeof(int), h->stream);
      if (e == hipSuccess) e = pc_setup(pl, spk, err, h->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
      int herr = 0;
      if (e == hipSuccess) e = hipMemcpy(&herr, err, sizeof(int), hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = build_launch(h);
      *singular = herr != 0;
      return e;
    };
    int best = -1;
    const TuneKey key{pl.prec, pl.log2n, nx};
    if (force_cand < 0) best = tune_lookup(key, cands);
    if (best < 0 && cands.size() == 1) best = cands[0];
    hipError_t e = hipSuccess;
    if (best < 0) {
      // time every candidate on this problem's shape as it runs inside a
      // solve: caches cold (the basis buffer, up to 1 GB, is overwritten
      // before each timed apply; its first vector, all zero, is the input),
      // one warm-up apply, the best of three
      hipEvent_t e0 = nullptr, e1 = nullptr;
      e = hipEventCreate(&e0);
      if (e == hipSuccess) e = hipEventCreate(&e1);
      const size_t flush = std::min<size_t>((size_t)(h->m_max + 1) * h->npad * sizeof(double),
                                            (size_t)1 << 30);
      if (e == hipSuccess) e = hipMemsetAsync(h->V, 0, flush, h->stream);
      float best_ms = 1e30f;
      for (size_t c = 0; c < cands.size() && e == hipSuccess; ++c) {
        const int ci = cands[c];
        int sing = 0;
        e = setup(ci, &sing);
        if (e != hipSuccess || sing) continue;
        auto apply = [&]() -> hipError_t {
          hipError_t r = pc_forward(pl.prec, pl.log2n, ci, h->L, h->wl.I_pc, 0, h->V, 0, h->stream);
          if (r == hipSuccess) r = pc_reduced(pl.prec, h->L, h->wl.I_k2, h->k2_thr, 0, 1, h->stream);
          if (r == hipSuccess)
            r = pc_inverse(pl.prec, pl.log2n, ci, h->L, h->wl.I_pc, 0, h->Z, pl.prec, 0, h->stream);
          return r;
        };
        float t3 = 1e30f;
        e = apply();
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
          e = hipMemsetAsync(h->V, 0, flush, h->stream);
          if (e == hipSuccess) e = hipEventRecord(e0, h->stream);
          if (e == hipSuccess) e = apply();
          if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          if (e == hipSuccess) t3 = std::min(t3, ms);
        }
        if (e == hipSuccess && t3 < best_ms) {
          best_ms = t3;
          best = ci;
        }
      }
      if (e0 != nullptr) (void)hipEventDestroy(e0);
      if (e1 != nullptr) (void)hipEventDestroy(e1);
      if (e == hipSuccess && best >= 0 && force_cand < 0) tune_store(key, best);
    }
    int sing = 1;
    if (e == hipSuccess && best >= 0) e = setup(best, &sing);
    free_tmp();
    if (e != hipSuccess) {
      fail(CN_EHIP, std::string("preconditioner set-up: ") + hipGetErrorString(e));
      return bail(CN_EHIP);
    }
    if (sing) {
      fail(CN_ESINGULAR, "a shifted system of step (b) is singular (alpha = " +
                             std::to_string(h->alpha) + ")");
      return bail(CN_ESINGULAR);
    }
  }
  TRY(hipStreamSynchronize(h->stream));
#undef TRY
  *out = h;
  return CN_OK;
}

// ---------------------------------------------------------------------------
// the solve driver, shared by a handle (one instance) and a batch
// ---------------------------------------------------------------------------
struct PcGroup {
  int prec, log2n, cand;
  Items items;
};

struct SolveCtx {
  hipStream_t s = nullptr;
  Launch L{};
  std::vector<PcGroup> groups;  // transform launches (one per N_t group)
  Items k2, mv, stv;
  int k2_thr = 32 * 16;  // interface-solve variant (k2_chunk_class)
  int prec = 0;
  bool batched = false;
  // one instance: its host slots and sequence counter
  GSummary* hs = nullptr;
  int* seqc = nullptr;
  // batch: batch-summary slots (host and device view), device counter, host count
  GSummary* bh = nullptr;
  GSummary* bh_dev = nullptr;
  int* dcounter = nullptr;
  int* bseq = nullptr;
  std::vector<GSummary*> inst_host;  // per-instance host slots
  std::vector<long long> off, len;   // packed offsets and lengths
  // per-instance stopping controls: the host staging array (pinned, so its
  // upload is asynchronous; every solve ends with a stream synchronisation
  // before the host writes it again), the device array the descriptors point
  // to, and the last values uploaded (uploads are skipped when unchanged);
  // rt: the rtol targets error-controlled stopping remembers between solves
  StopCtl* ctl = nullptr;
  StopCtl* ctl_dev = nullptr;
  StopCtl* ctl_last = nullptr;
  std::vector<double>* rt = nullptr;
  double* rt_for = nullptr;  // the (rtol, err_tol) the targets were made for
  // batch: captured inner iterations (null: launch kernel by kernel); with
  // cycle_graphs the first *cycle_k iterations of a cycle as one graph
  // (*cycle_k: the last solve's first-cycle iteration count)
  struct GraphCache* graphs = nullptr;
  bool cycle_graphs = false;
  int* cycle_k = nullptr;
};

// One captured graph per inner-iteration index j of a batch: the transform
// launches of every N_t group, the interface solves, the Krylov kernels with
// their finishing reductions and the batch summary.  Every argument of those
// launches is fixed for a batch except (j, stop_iter, rtol), the cache key.
struct GraphCache {
  hipStream_t cap = nullptr;  // capture stream (the solve stream may be the null stream)
  struct Entry {
    int j, stop_iter;
    double rtol;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<Entry> entries;
  void release() {
    for (Entry& e : entries) {
      (void)hipGraphExecDestroy(e.x);
      (void)hipGraphDestroy(e.g);
    }
    entries.clear();
    if (cap != nullptr) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }
};

static hipError_t enqueue_iteration(SolveCtx& c, int j, int stop_iter, double rtol, int slot,
                                    int seq) {
  hipError_t e = hipSuccess;
  for (const PcGroup& g : c.groups)
    if (e == hipSuccess) e = pc_forward(g.prec, g.log2n, g.cand, c.L, g.items, j, nullptr, 0, c.s);
  if (e == hipSuccess) e = pc_reduced(c.prec, c.L, c.k2, c.k2_thr, j, 0, c.s);
  for (const PcGroup& g : c.groups)
    if (e == hipSuccess)
      e = pc_inverse(g.prec, g.log2n, g.cand, c.L, g.items, j, nullptr, c.L.zf, 0, c.s);
  if (e == hipSuccess) e = launch_arnoldi(c.L, c.mv, c.stv, j, stop_iter, rtol, slot, seq, c.s);
  return e;
}

// Publish a batch summary (instances still iterating) and return its sequence number.
static cn_status batch_publish(SolveCtx& c, int slot, int* seq) {
  HIP_TRY(launch_batch_summary(c.L, c.dcounter, c.bh_dev + slot, c.s));
  *seq = ++(*c.bseq);
  return CN_OK;
}

// Launch the captured graph of inner iteration j (capturing it on first use):
// the same launches as enqueue_iteration + batch_publish on slot j & 1.
// With `cycle` = K > 0, the graph holds inner iterations 0..K-1 of a cycle,
// each followed by its batch summary (key j = -K): the host then waits once,
// for the summary of iteration K-1, instead of once per iteration.
static cn_status launch_iteration_graph(SolveCtx& c, int j, int stop_iter, double rtol,
                                        int cycle = 0) {
  GraphCache& gc = *c.graphs;
  const int key = cycle > 0 ? -cycle : j;
  for (const GraphCache::Entry& e : gc.entries)
    if (e.j == key && e.stop_iter == stop_iter && e.rtol == rtol) {
      HIP_TRY(hipGraphLaunch(e.x, c.s));
      return CN_OK;
    }
  if (gc.cap == nullptr) HIP_TRY(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
  SolveCtx cc = c;
  cc.s = gc.cap;
  HIP_TRY(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  const int j0 = cycle > 0 ? 0 : j, j1 = cycle > 0 ? cycle : j + 1;
  for (int jj = j0; jj < j1 && e == hipSuccess; ++jj) {
    e = enqueue_iteration(cc, jj, stop_iter, rtol, jj & 1, 0);
    if (e == hipSuccess) e = launch_batch_summary(cc.L, cc.dcounter, cc.bh_dev + (jj & 1), gc.cap);
  }
  hipGraph_t g = nullptr;
  const hipError_t e2 = hipStreamEndCapture(gc.cap, &g);
  if (e == hipSuccess) e = e2;
  hipGraphExec_t x = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    if (g != nullptr) (void)hipGraphDestroy(g);
    return fail(CN_EHIP, std::string("iteration graph: ") + hipGetErrorString(e));
  }
  gc.entries.push_back(GraphCache::Entry{key, stop_iter, rtol, g, x});
  HIP_TRY(hipGraphLaunch(x, c.s));
  return CN_OK;
}

// Summary slot `slot` of instance i (read after the stream has drained).
static const volatile GSummary* inst_slot(const SolveCtx& c, int i, int slot) {
  return (c.batched ? c.inst_host[i] : c.hs) + slot;
}

// Copy the stopping controls to the device (if they changed).
static hipError_t upload_ctl(SolveCtx& c) {
  const size_t bytes = (size_t)c.L.ninst * sizeof(StopCtl);
  if (memcmp(c.ctl, c.ctl_last, bytes) == 0) return hipSuccess;
  memcpy(c.ctl_last, c.ctl, bytes);
  return hipMemcpyAsync(c.ctl_dev, c.ctl, bytes, hipMemcpyHostToDevice, c.s);
}

// One restarted GMRES solve of every instance of the context; instance i
// stops at relres <= rtol * (*c.ctl)[i].rscale (uploaded by the caller).
// Fills infos[0..ninst).
static cn_status run_solve(SolveCtx& c, const double* b, double* x, const cn_gmres_opts* opts,
                           cn_gmres_info* infos) {
  const auto wall0 = std::chrono::steady_clock::now();
  const int ninst = c.L.ninst;
  const double rtol = opts->rtol;
  std::vector<double> fac(ninst);
  for (int i = 0; i < ninst; ++i) fac[i] = c.ctl[i].rscale;
  const double rtol_min = rtol * *std::min_element(fac.begin(), fac.end());
  std::vector<int> iters(ninst, 0), pcs(ninst, 0), mvs(ninst, 1), rest(ninst, 0);
  std::vector<double> est(ninst, 0.0);
  std::vector<GSummary> cur(ninst), fin(ninst);
  // r_0 = b - M x_0 into v_0 (x_0 = 0 is never read); the stop flag covers
  // instances that already meet rtol, so nothing waits here
  int seq_res = c.batched ? 0 : ++(*c.seqc);
  HIP_TRY(launch_residual(c.L, c.mv, c.stv, b, x, opts->use_x0 ? 0 : 1, rtol, 2, seq_res, c.s,
                          opts->use_x0 == 2 ? 2 : 1));
  bool x_zero = !opts->use_x0;
  int done_iters = 0;
  int first_cycle_k = -1;
  int seqs[MMAX];
  double ests[MMAX];
  GSummary it{};
  while (true) {
    const int m_eff = std::min(opts->m, opts->max_iters - done_iters);
    int known = 0;  // iterations of this cycle whose summary the host has read
    // speculative cycle end queued behind the iteration the host waits for
    bool spec = false, spec_taken = false;
    int spec_fin = 0, spec_res = 0;
    int enq = 0;  // inner iterations queued in this cycle
    for (int j = 0; j < m_eff; ++j) {
      spec = false;
      seqs[j] = c.batched ? 0 : ++(*c.seqc);
      enq = j + 1;
      const int K = c.cycle_k != nullptr ? *c.cycle_k : 0;
      if (j == 0 && c.graphs != nullptr && c.cycle_graphs && K >= 2 && K <= m_eff) {
        // the first K iterations (as many as the last solve's first cycle
        // took) as one graph, and one wait for the summary of the last;
        // iterations queued after convergence return at entry
        CN_TRY(launch_iteration_graph(c, 0, m_eff, rtol, K));
        *c.bseq += K;
        seqs[K - 1] = *c.bseq;
        enq = K;
        CN_TRY(wait_slot(c.s, c.bh + ((K - 1) & 1), seqs[K - 1], &it));
        for (int q = 0; q < K; ++q) ests[q] = it.est;
        known = K;
        if (it.done) break;
        j = K - 1;
        continue;
      }
      if (c.graphs != nullptr) {
        CN_TRY(launch_iteration_graph(c, j, m_eff, rtol));
        seqs[j] = ++(*c.bseq);
      } else {
        HIP_TRY(enqueue_iteration(c, j, m_eff, rtol, j & 1, seqs[j]));
        if (c.batched) CN_TRY(batch_publish(c, j & 1, &seqs[j]));
      }
      GSummary* slots = c.batched ? c.bh : c.hs;
      if (j >= 1) {
        if (known < j) {
          CN_TRY(wait_slot(c.s, slots + ((j - 1) & 1), seqs[j - 1], &it));
          ests[j - 1] = it.est;
          known = j;
          if (it.done) break;
        }
        // The residual estimate falls at least geometrically (usually
        // faster).  When the rate of the last two steps brings iteration j
        // within 50x of rtol, wait for it instead of queueing iteration j+1:
        // an iteration queued after convergence still costs its kernel
        // dispatches (~45 us), a wrong guess only a short idle gap (~15 us).
        double prev = 1.0;
        if (j >= 2) {
          prev = ests[j - 2];
        } else if (!c.batched) {
          volatile GSummary* r0 = c.hs + 2;
          prev = (r0->seq == seq_res && r0->relres > 0.0) ? r0->relres : 1.0;
        }
        const double rate = prev > 0.0 ? ests[j - 1] / prev : 1.0;
        if (j + 1 < m_eff && ests[j - 1] * rate < 50.0 * rtol_min) {
          // one instance: queue the cycle end behind iteration j before
          // waiting (its kernels return at entry unless the cycle stopped),
          // so a converged solve goes on without a host round trip
          if (!c.batched) {
            spec_fin = ++(*c.seqc);
            spec_res = ++(*c.seqc);
            if (x_zero) {
              HIP_TRY(launch_cycle_end_zero(c.L, c.mv, enq, b, x, rtol, 3, spec_fin, 2, spec_res,
                                            c.s, true, false));
            } else {
              HIP_TRY(launch_cycle_end(c.L, c.stv, x, 0, 3, spec_fin, c.s, true));
              HIP_TRY(launch_residual(c.L, c.mv, c.stv, b, x, 0, rtol, 2, spec_res, c.s, 0, true));
            }
            spec = true;
          }
          CN_TRY(wait_slot(c.s, slots + (j & 1), seqs[j], &it));
          ests[j] = it.est;
          known = j + 1;
          if (it.done) {
            spec_taken = spec;
            break;
          }
        }
      }
    }
    // y from the triangular factors (cycle summaries -> slot 3), x += Z y,
    // then the true residuals (-> slot 2), unless already queued; a cycle
    // from x = 0 does the update and the residual in one pass, and for one
    // instance leaves r unstored (formed again below if the cycle restarts)
    const bool r_unstored = x_zero && !c.batched;
    int seq_fin = spec_fin;
    if (spec_taken) {
      seq_res = spec_res;
    } else {
      seq_fin = c.batched ? 0 : ++(*c.seqc);
      seq_res = c.batched ? 0 : ++(*c.seqc);
      if (x_zero) {
        HIP_TRY(launch_cycle_end_zero(c.L, c.mv, enq, b, x, rtol, 3, seq_fin, 2, seq_res, c.s,
                                      false, c.batched));
      } else {
        HIP_TRY(launch_cycle_end(c.L, c.stv, x, 0, 3, seq_fin, c.s));
        HIP_TRY(launch_residual(c.L, c.mv, c.stv, b, x, 0, rtol, 2, seq_res, c.s, 0));
      }
    }
    x_zero = false;
    if (c.batched) {
      int sq = 0;
      CN_TRY(batch_publish(c, 2, &sq));
      CN_TRY(wait_slot(c.s, c.bh + 2, sq, &it));
      std::atomic_thread_fence(std::memory_order_acquire);
      for (int i = 0; i < ninst; ++i) {
        volatile GSummary* f3 = c.inst_host[i] + 3;
        volatile GSummary* f2 = c.inst_host[i] + 2;
        fin[i].k = f3->k;
        fin[i].est = f3->est;
        cur[i].relres = f2->relres;
        cur[i].bnorm = f2->bnorm;
        cur[i].x0_rejected = f2->x0_rejected;
      }
    } else {
      CN_TRY(wait_slot(c.s, c.hs + 3, seq_fin, &fin[0]));
      CN_TRY(wait_slot(c.s, c.hs + 2, seq_res, &cur[0]));
    }
    int kmax = 0;
    bool all_conv = true;
    for (int i = 0; i < ninst; ++i) {
      const int k = fin[i].k;
      if (k > 0) est[i] = fin[i].est;
      iters[i] += k;
      pcs[i] += k;
      mvs[i] += k + 1;
      kmax = std::max(kmax, k);
      if (!(cur[i].relres <= rtol * fac[i])) all_conv = false;
    }
    if (first_cycle_k < 0) first_cycle_k = kmax;
    done_iters += kmax;
    if (kmax == 0 || all_conv || done_iters >= opts->max_iters) break;
    if (r_unstored) {
      // the restart's v_0: r = b - M x again (and FIN 1 on it)
      seq_res = ++(*c.seqc);
      HIP_TRY(launch_residual(c.L, c.mv, c.stv, b, x, 0, rtol, 2, seq_res, c.s, 0));
      ++mvs[0];
    }
    for (int i = 0; i < ninst; ++i)
      if (!(cur[i].relres <= rtol * fac[i])) ++rest[i];
  }
  // b = 0: the solution is x = 0 whatever the initial guess
  for (int i = 0; i < ninst; ++i) {
    if (cur[i].bnorm == 0.0) {
      HIP_TRY(hipMemsetAsync(x + c.off[i], 0, (size_t)c.len[i] * sizeof(double), c.s));
      cur[i].relres = 0.0;
      est[i] = 0.0;
    }
  }
  HIP_TRY(hipStreamSynchronize(c.s));
  if (c.cycle_k != nullptr && first_cycle_k > 0) *c.cycle_k = first_cycle_k;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  bool ok = true;
  for (int i = 0; i < ninst; ++i) {
    cn_gmres_info in{};
    in.iters = iters[i];
    in.restarts = rest[i];
    in.matvecs = mvs[i];
    in.pc_applies = pcs[i];
    in.x0_rejected = cur[i].x0_rejected;
    in.relres_true = cur[i].relres;
    in.relres_est = iters[i] > 0 ? est[i] : cur[i].relres;
    in.seconds = secs;
    in.err_est = -1.0;
    infos[i] = in;
    if (!(cur[i].relres <= rtol * fac[i])) ok = false;
  }
  return ok ? CN_OK : CN_NOT_CONVERGED;
}

// Relative max-norm error estimate of every instance's x whose est_skip is 0
// (see launch_err_estimate): r = b - M x in V_0 (a batch's last cycle end
// left it there; one instance forms it again), the preconditioner of
// iteration 0 on it, the estimate into summary slot 2.  err[i] < 0: not
// estimated.
static cn_status estimate_errors(SolveCtx& c, const double* b, double* x, std::vector<double>* err) {
  const int seq = c.batched ? 0 : ++(*c.seqc);
  if (c.batched)
    HIP_TRY(launch_err_begin(c.L, c.s));
  else
    HIP_TRY(launch_residual(c.L, c.mv, c.stv, b, x, 0, -1.0, 2, seq, c.s, 0));
  for (const PcGroup& g : c.groups)
    HIP_TRY(pc_forward(g.prec, g.log2n, g.cand, c.L, g.items, 0, nullptr, 0, c.s));
  HIP_TRY(pc_reduced(c.prec, c.L, c.k2, c.k2_thr, 0, 0, c.s));
  for (const PcGroup& g : c.groups)
    HIP_TRY(pc_inverse(g.prec, g.log2n, g.cand, c.L, g.items, 0, nullptr, c.L.zf, 0, c.s));
  HIP_TRY(launch_err_estimate(c.L, c.stv, x, 2, seq, c.s));
  HIP_TRY(hipStreamSynchronize(c.s));
  std::atomic_thread_fence(std::memory_order_acquire);
  for (int i = 0; i < c.L.ninst; ++i) (*err)[i] = inst_slot(c, i, 2)->err;
  return CN_OK;
}

// The solve of cn_gmres_solve / cn_batch_solve.
//
// Error-controlled stopping (opts->err_tol > 0): instance i first stops at its
// remembered target rt_i <= rtol (on a handle's or batch's first such solve
// with these rtol and err_tol, min(rtol, err_tol / 10)).  Then every
// instance's error is estimated; an instance above err_tol continues from
// its x with the target relres times err_tol / (4 * estimate) (on the
// assumption that its error falls in proportion to its residual, at least
// halving the target), and only the instances that continued are estimated
// again, at most kErrRounds times.  The targets only tighten and are kept for
// the next solve (a relaxed target can miss by a whole inner iteration's
// reduction and cost a continuation pass on the next solve).
constexpr int kErrRounds = 3;
static cn_status solve_driver(SolveCtx& c, const double* b, double* x, const cn_gmres_opts* opts,
                              cn_gmres_info* infos, cn_gmres_info* total) {
  const auto wall0 = std::chrono::steady_clock::now();
  const int ninst = c.L.ninst;
  const double rtol = opts->rtol, etol = opts->err_tol;
  const bool ec = etol > 0.0 && rtol > 0.0;
  StopCtl* ctl = c.ctl;
  std::vector<double>& rt = *c.rt;
  for (int i = 0; i < ninst; ++i) ctl[i] = StopCtl{1.0, 0, 0};
  if (ec) {
    if ((int)rt.size() != ninst || c.rt_for[0] != rtol || c.rt_for[1] != etol) {
      rt.assign(ninst, std::min(rtol, 0.1 * etol));
      c.rt_for[0] = rtol;
      c.rt_for[1] = etol;
    }
    for (int i = 0; i < ninst; ++i) ctl[i].rscale = std::min(1.0, rt[i] / rtol);
  }
  HIP_TRY(upload_ctl(c));
  std::vector<cn_gmres_info> inf(ninst), more(ninst);
  int passes = 0;
  cn_status rc = run_solve(c, b, x, opts, inf.data());
  if (rc == CN_OK && ec) {
    std::vector<double> err(ninst, 0.0);
    cn_gmres_opts o2 = *opts;
    o2.use_x0 = 1;
    // continuations neither use nor record the first-cycle iteration count
    c.cycle_k = nullptr;
    for (int round = 0;; ++round) {
      CN_TRY(estimate_errors(c, b, x, &err));
      bool above = false;
      for (int i = 0; i < ninst; ++i) {
        StopCtl& ci = ctl[i];
        if (ci.est_skip) continue;
        inf[i].err_est = err[i];
        if (err[i] <= etol) {
          ci.est_skip = 1;  // accurate: nothing more to do
        } else {
          above = true;
          const double want = inf[i].relres_true * 0.25 * etol / err[i];
          ci.rscale = std::max(1e-8, std::min(0.5 * ci.rscale, want / rtol));
          rt[i] = rtol * ci.rscale;
        }
      }
      if (!above) break;
      if (round == kErrRounds) {
        rc = CN_NOT_CONVERGED;
        break;
      }
      // instances already accurate stop at their first residual (their
      // threshold is left loose enough to hold: relres <= rtol)
      for (int i = 0; i < ninst; ++i)
        if (ctl[i].est_skip) ctl[i].rscale = 1.0;
      HIP_TRY(upload_ctl(c));
      rc = run_solve(c, b, x, &o2, more.data());
      ++passes;
      for (int i = 0; i < ninst; ++i) {
        if (ctl[i].est_skip) continue;
        ++inf[i].err_passes;
        inf[i].iters += more[i].iters;
        inf[i].restarts += more[i].restarts;
        inf[i].matvecs += more[i].matvecs;
        inf[i].pc_applies += more[i].pc_applies;
        inf[i].relres_true = more[i].relres_true;
        if (more[i].iters > 0) inf[i].relres_est = more[i].relres_est;
      }
      if (rc != CN_OK) break;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count();
  cn_gmres_info tot{};
  tot.err_est = -1.0;
  for (int i = 0; i < ninst; ++i) {
    cn_gmres_info& in = inf[i];
    in.seconds = secs;
    if (infos != nullptr) infos[i] = in;
    tot.iters = std::max(tot.iters, in.iters);
    tot.restarts = std::max(tot.restarts, in.restarts);
    tot.matvecs += in.matvecs;
    tot.pc_applies += in.pc_applies;
    tot.x0_rejected += in.x0_rejected;
    tot.relres_true = std::max(tot.relres_true, in.relres_true);
    tot.relres_est = std::max(tot.relres_est, in.relres_est);
    tot.err_est = std::max(tot.err_est, in.err_est);
  }
  tot.seconds = secs;
  tot.err_passes = passes;
  if (total != nullptr) *total = tot;
  return rc;
}

static SolveCtx handle_ctx(cn_aao* h) {
  SolveCtx c;
  c.s = h->stream;
  c.L = h->L;
  c.groups.push_back(PcGroup{h->prec, h->pl.log2n, h->pl.cand, h->wl.I_pc});
  c.k2 = h->wl.I_k2;
  c.mv = h->wl.I_mv;
  c.stv = h->wl.I_st;
  c.k2_thr = h->k2_thr;
  c.prec = h->prec;
  c.batched = false;
  c.hs = h->hsum;
  c.seqc = &h->seqc;
  c.off.assign(1, 0);
  c.len.assign(1, h->n);
  c.ctl = h->h_ctl;
  c.ctl_dev = h->d_ctl;
  c.ctl_last = &h->last_ctl;
  c.rt = &h->rt;
  c.rt_for = h->rt_for;
  return c;
}

// ---------------------------------------------------------------------------
// batch of uneven instances
// ---------------------------------------------------------------------------
struct cn_batch {
  std::vector<cn_aao*> inst;
  std::vector<long long> off;      // count + 1 offsets into packed vectors
  std::vector<long long> uoff;     // count + 1 offsets into packed u0 (space only)
  hipStream_t stream = nullptr;
  int prec = 0, m_min = 0;
  InstDesc* d_desc = nullptr;
  WorkLists wl;                    // k2, mv, st lists (pc lists per group below)
  std::vector<int2*> pc_lists;
  std::vector<PcGroup> groups;
  int k2_thr = 32 * 16;  // interface-solve variant (k2_chunk_class)
  GSummary* bh = nullptr;          // 3 batch-summary slots (pinned coherent)
  GSummary* bh_dev = nullptr;
  int* dcounter = nullptr;
  int bseq = 0;
  GraphCache graphs;
  long long* d_layout = nullptr;   // BatchLayout::dev
  std::vector<int> nxs, nts;       // per-instance N_x, N_t (host)
  StopCtl* d_ctl = nullptr;        // stopping controls (SolveCtx::ctl): device,
  StopCtl* h_ctl = nullptr;        // pinned host staging,
  std::vector<StopCtl> last_ctl;   // last uploaded
  std::vector<double> rt;          // remembered rtol targets (SolveCtx::rt)
  double rt_for[2] = {0.0, 0.0};
  int cycle_k = 0;                 // first-cycle iterations of the last solve
};

static void batch_release(cn_batch* b) {
  if (b == nullptr) return;
  (void)hipStreamSynchronize(b->stream);
  b->graphs.release();
  for (cn_aao* h : b->inst) release(h);
  b->wl.release();
  for (int2* p : b->pc_lists) (void)hipFree(p);
  if (b->d_desc != nullptr) (void)hipFree(b->d_desc);
  if (b->d_ctl != nullptr) (void)hipFree(b->d_ctl);
  if (b->h_ctl != nullptr) (void)hipHostFree(b->h_ctl);
  if (b->d_layout != nullptr) (void)hipFree(b->d_layout);
  if (b->dcounter != nullptr) (void)hipFree(b->dcounter);
  if (b->bh != nullptr) (void)hipHostFree(b->bh);
  delete b;
}

extern "C" {

cn_status cn_aao_create(const cn_problem* p, cn_aao** out) { return create_handle(p, -1, out); }

cn_status cn_aao_destroy(cn_aao* h) {
  if (h == nullptr) return fail(CN_EINVAL, "handle is NULL");
  release(h);
  return CN_OK;
}

cn_status cn_aao_query(const cn_aao* h, int32_t* tile_cols, int32_t* tiles, int32_t* threads,
                       int32_t* inverse_split, int32_t* forward_split) {
  if (h == nullptr) return fail(CN_EINVAL, "handle is NULL");
  if (tile_cols != nullptr) *tile_cols = h->pl.B;
  if (tiles != nullptr) *tiles = h->pl.P;
  if (threads != nullptr) *threads = h->pl.T;
  if (inverse_split != nullptr) *inverse_split = h->pl.S;
  if (forward_split != nullptr) *forward_split = h->pl.FS;
  return CN_OK;
}

cn_status cn_aao_cycle(cn_aao* h, int32_t k, double* gram, double* rfac, double* scale) {
  if (h == nullptr) return fail(CN_EINVAL, "handle is NULL");
  if (k < 0 || k > h->m_max) return fail(CN_EINVAL, "k must be in [0, m_max]");
  std::vector<char> buf(sizeof(GState));
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(buf.data(), h->st, sizeof(GState), hipMemcpyDeviceToHost));
  const GState& st = *reinterpret_cast<const GState*>(buf.data());
  const int kk = k;
  for (int p = 0; p <= kk; ++p) {
    if (scale != nullptr) scale[p] = st.vscale[p];
    for (int q = 0; q <= kk && gram != nullptr; ++q) gram[p * (kk + 1) + q] = st.gram[p * NVMAX + q];
  }
  for (int j = 0; j < kk && rfac != nullptr; ++j)
    for (int q = 0; q <= kk; ++q) rfac[j * (kk + 1) + q] = q <= j ? st.H[j * (MMAX + 1) + q] : 0.0;
  return CN_OK;
}

cn_status cn_aao_basis(cn_aao* h, int32_t q, double* out) {
  if (h == nullptr || out == nullptr) return fail(CN_EINVAL, "NULL argument");
  if (q < 0 || q > h->m_max) return fail(CN_EINVAL, "basis index out of range");
  HIP_TRY(hipMemcpy2DAsync(out, (size_t)h->nx * sizeof(double), h->V + (size_t)q * h->npad,
                           (size_t)h->ldx * sizeof(double), (size_t)h->nx * sizeof(double), h->nt,
                           hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return CN_OK;
}

cn_status cn_rhs(cn_aao* h, const double* u0, const double* f, double* b) {
  if (h == nullptr || u0 == nullptr || f == nullptr || b == nullptr)
    return fail(CN_EINVAL, "NULL argument");
  if (overlaps(f, b, h->n * sizeof(double)) || overlaps(u0, b, h->n * sizeof(double)))
    return fail(CN_EINVAL, "b must not overlap u0 or f");
  HIP_TRY(launch_rhs(h->pl.lo, h->pl.di, h->pl.up, h->dw, h->tau, u0, f, b, h->nx, h->n,
                     h->stream));
  return CN_OK;
}

cn_status cn_matvec(cn_aao* h, const double* x, double* y) {
  if (h == nullptr || x == nullptr || y == nullptr) return fail(CN_EINVAL, "NULL argument");
  if (overlaps(x, y, h->n * sizeof(double))) return fail(CN_EINVAL, "x and y overlap");
  HIP_TRY(launch_matvec_plain(h->L, h->wl.I_mv, x, y, h->stream));
  return CN_OK;
}

cn_status cn_pc_apply(cn_aao* h, const double* v, double* z) {
  if (h == nullptr || v == nullptr || z == nullptr) return fail(CN_EINVAL, "NULL argument");
  const PcPlan& pl = h->pl;
  HIP_TRY(pc_forward(pl.prec, pl.log2n, pl.cand, h->L, h->wl.I_pc, 0, v, h->nx, h->stream));
  HIP_TRY(pc_reduced(pl.prec, h->L, h->wl.I_k2, h->k2_thr, 0, 1, h->stream));
  HIP_TRY(pc_inverse(pl.prec, pl.log2n, pl.cand, h->L, h->wl.I_pc, 0, z, 0, h->nx, h->stream));
  return CN_OK;
}

cn_status cn_gmres_solve(cn_aao* h, const double* b, double* x, const cn_gmres_opts* opts,
                         cn_gmres_info* info) {
  if (h == nullptr || b == nullptr || x == nullptr || opts == nullptr)
    return fail(CN_EINVAL, "NULL argument");
  if (opts->m < 1 || opts->m > h->m_max) return fail(CN_EINVAL, "opts->m must be in [1, m_max]");
  if (opts->max_iters < 1) return fail(CN_EINVAL, "opts->max_iters must be >= 1");
  if (opts->use_x0 < 0 || opts->use_x0 > 2) return fail(CN_EINVAL, "opts->use_x0 must be 0, 1 or 2");
  if (opts->flags & ~(CN_SOLVE_NO_GRAPHS | CN_SOLVE_ITERATION_GRAPHS))
    return fail(CN_EINVAL, "unknown bits in opts->flags");
  if (!(opts->rtol >= 0.0) || !std::isfinite(opts->rtol))
    return fail(CN_EINVAL, "opts->rtol must be finite and >= 0");
  if (!(opts->err_tol >= 0.0) || !std::isfinite(opts->err_tol))
    return fail(CN_EINVAL, "opts->err_tol must be finite and >= 0");
  if (overlaps(b, x, h->n * sizeof(double))) return fail(CN_EINVAL, "b and x overlap");
  SolveCtx c = handle_ctx(h);
  const cn_status st = solve_driver(c, b, x, opts, info, nullptr);
  return st;
}

cn_status cn_profile_step(cn_aao* h, int32_t j, int32_t reps, double* ms, double* bytes) {
  if (h == nullptr || ms == nullptr || bytes == nullptr) return fail(CN_EINVAL, "NULL argument");
  if (j < 0 || j >= h->m_max || reps < 1) return fail(CN_EINVAL, "j or reps out of range");
  hipStream_t s = h->stream;
  GState* st = h->st;
  const int zf = h->prec;
  const size_t zes = zf ? sizeof(float) : sizeof(double);
  const size_t rsz = h->prec ? sizeof(float) : sizeof(double);
  // keep every kernel of the step active
  const int zero = 0;
  HIP_TRY(hipMemcpyAsync(&st->sum.done, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  hipEvent_t ev[2];
  HIP_TRY(hipEventCreate(&ev[0]));
  HIP_TRY(hipEventCreate(&ev[1]));
  const PcPlan& pl = h->pl;
  const double n = (double)h->n;
  const double nimg = (double)pl.P * pl.B * pl.nt;
  const double nsep = (double)pl.F * pl.NS;
  bytes[0] = n * 8 + nimg * rsz + (double)pl.F * pl.P * 4 * rsz;
  // partial right-hand sides (two per separator), factor records (three), S
  bytes[1] = nsep * (4 * rsz + 6 * rsz + 2 * rsz);
  bytes[2] = nimg * rsz + (double)pl.F * pl.P * 4 * rsz + n * zes;
  bytes[3] = n * zes + (double)(j + 1) * n * 8;  // z_j and the basis (w is not stored)
  bytes[4] = n * zes + (double)(j + 2) * n * 8;  // z_j, the basis, v_{j+1}
  cn_status rc = CN_OK;
  for (int kk = 0; kk < CN_PROFILE_KERNELS && rc == CN_OK; ++kk) {
    hipError_t e = hipEventRecord(ev[0], s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
      switch (kk) {
        case 0: e = pc_forward(pl.prec, pl.log2n, pl.cand, h->L, h->wl.I_pc, j, nullptr, 0, s); break;
        case 1: e = pc_reduced(pl.prec, h->L, h->wl.I_k2, h->k2_thr, j, 0, s); break;
        case 2: e = pc_inverse(pl.prec, pl.log2n, pl.cand, h->L, h->wl.I_pc, j, nullptr, zf, 0, s); break;
        // the two streaming Krylov kernels alone (their one-workgroup
        // finishing reductions are left out, so each entry is one kernel)
        case 3: e = launch_arnoldi(h->L, h->wl.I_mv, h->wl.I_st, j, 1 << 30, 0.0, 0, 0, s, 1, false); break;
        case 4: e = launch_arnoldi(h->L, h->wl.I_mv, h->wl.I_st, j, 1 << 30, 0.0, 0, 0, s, 4, false); break;
      }
    }
    if (e == hipSuccess) e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
    if (e != hipSuccess) {
      rc = fail(CN_EHIP, std::string("profile: ") + hipGetErrorString(e));
      break;
    }
    ms[kk] = (double)t / reps;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return rc;
}

// ---------------------------------------------------------------------------
// batch entry points
// ---------------------------------------------------------------------------
cn_status cn_batch_create(const cn_problem* probs, int32_t count, cn_batch** out) {
  if (out == nullptr) return fail(CN_EINVAL, "out is NULL");
  *out = nullptr;
  if (probs == nullptr || count < 1) return fail(CN_EINVAL, "need at least one problem");
  for (int i = 1; i < count; ++i) {
    if (probs[i].pc_prec != probs[0].pc_prec)
      return fail(CN_EINVAL, "all problems of a batch need the same pc_prec");
    if (probs[i].stream != probs[0].stream)
      return fail(CN_EINVAL, "all problems of a batch need the same stream");
  }
  cn_batch* b = new cn_batch();
  b->stream = (hipStream_t)probs[0].stream;
  b->prec = probs[0].pc_prec == CN_PC_FP32 ? 1 : 0;
  b->inst.assign(count, nullptr);
  // transform variant per N_t group: tuned on the group's widest instance
  std::map<int, int> group_cand;  // log2 N_t -> candidate
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return probs[a].nx > probs[c].nx; });
  for (int i : order) {
    int l2 = 0;
    while ((1 << l2) < probs[i].nt && l2 < 31) ++l2;
    auto it = group_cand.find(l2);
    cn_aao* h = nullptr;
    const cn_status st = create_handle(&probs[i], it == group_cand.end() ? -1 : it->second, &h);
    if (st != CN_OK) {
      g_err = "problem " + std::to_string(i) + ": " + g_err;
      batch_release(b);
      return st;
    }
    b->inst[i] = h;
    if (it == group_cand.end()) group_cand[l2] = h->pl.cand;
  }
  // packed offsets, descriptors and work lists
  b->off.assign(count + 1, 0);
  b->uoff.assign(count + 1, 0);
  b->m_min = MMAX;
  for (int i = 0; i < count; ++i) {
    b->off[i + 1] = b->off[i] + b->inst[i]->n;
    b->uoff[i + 1] = b->uoff[i] + b->inst[i]->nx;
    b->m_min = std::min(b->m_min, b->inst[i]->m_max);
  }
  std::vector<InstDesc> desc(count);
  std::vector<int2> k2, mv, stv;
  std::map<int, std::vector<int2>> pcs;
  int max_ns = 0;
  for (int i = 0; i < count; ++i) {
    desc[i] = b->inst[i]->desc;
    desc[i].off = b->off[i];
    // the batch has parallelism across instances: matvec blocks of at least
    // MV_BATCH_ROWS time levels keep per-workgroup latency chains and partial
    // sums few (a lone small instance keeps its finer blocks)
    if (desc[i].rows < MV_BATCH_ROWS) {
      desc[i].rows = std::min(MV_BATCH_ROWS, desc[i].nt);
      desc[i].mv_grid = desc[i].mv_cols * ((desc[i].nt + desc[i].rows - 1) / desc[i].rows);
    }
    append_items(desc[i], i, &pcs[b->inst[i]->pl.log2n], &k2, &mv, &stv);
    max_ns = std::max(max_ns, desc[i].pl.NS);
  }
  b->last_ctl.assign(count, StopCtl{1.0, 0, 0});
  hipError_t e = hipMalloc((void**)&b->d_ctl, count * sizeof(StopCtl));
  if (e == hipSuccess)
    e = hipMemcpy(b->d_ctl, b->last_ctl.data(), count * sizeof(StopCtl), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_ctl, count * sizeof(StopCtl), hipHostMallocDefault);
  for (int i = 0; i < count; ++i) desc[i].ctl = b->d_ctl + i;
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_desc, count * sizeof(InstDesc));
  if (e == hipSuccess)
    e = hipMemcpy(b->d_desc, desc.data(), count * sizeof(InstDesc), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = upload_items(k2, &b->wl.k2, &b->wl.I_k2);
  if (e == hipSuccess) e = upload_items(mv, &b->wl.mv, &b->wl.I_mv);
  if (e == hipSuccess) e = upload_items(stv, &b->wl.st, &b->wl.I_st);
  for (auto& kv : pcs) {
    if (e != hipSuccess) break;
    int2* dptr = nullptr;
    Items it;
    e = upload_items(kv.second, &dptr, &it);
    b->pc_lists.push_back(dptr);
    b->groups.push_back(PcGroup{b->prec, kv.first, group_cand[kv.first], it});
  }
  b->k2_thr = k2_chunk_class(max_ns, b->prec);
  {
    // layout for per-instance kernels outside the solver (the learned guess)
    std::vector<long long> lay(1 + 5 * (size_t)count);
    long long go = 0;
    for (int i = 0; i < count; ++i) {
      b->nxs.push_back(b->inst[i]->nx);
      b->nts.push_back(b->inst[i]->nt);
    }
    for (int i = 0; i <= count; ++i) lay[i] = b->off[i];
    for (int i = 0; i < count; ++i) {
      lay[count + 1 + i] = b->uoff[i];
      lay[2 * count + 1 + i] = go;
      go += b->nts[i];
      lay[3 * count + 1 + i] = b->nxs[i];
      lay[4 * count + 1 + i] = b->nts[i];
    }
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_layout, lay.size() * sizeof(long long));
    if (e == hipSuccess)
      e = hipMemcpy(b->d_layout, lay.data(), lay.size() * sizeof(long long), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMalloc((void**)&b->dcounter, sizeof(int));
  if (e == hipSuccess) e = hipMemset(b->dcounter, 0, sizeof(int));
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&b->bh, 3 * sizeof(GSummary),
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) {
    memset(b->bh, 0, 3 * sizeof(GSummary));
    e = hipHostGetDevicePointer((void**)&b->bh_dev, b->bh, 0);
  }
  if (e != hipSuccess) {
    const cn_status st = fail(e == hipErrorOutOfMemory ? CN_ENOMEM : CN_EHIP,
                              std::string("batch set-up: ") + hipGetErrorString(e));
    batch_release(b);
    return st;
  }
  *out = b;
  return CN_OK;
}

}  // extern "C"

bool cn::batch_layout(const cn_batch* b, BatchLayout* out) {
  if (b == nullptr || out == nullptr || b->d_layout == nullptr) return false;
  out->dev = b->d_layout;
  out->count = (int)b->inst.size();
  out->nx = b->nxs.data();
  out->nt = b->nts.data();
  out->total = b->off.back();
  return true;
}

extern "C" {

cn_status cn_batch_destroy(cn_batch* b) {
  if (b == nullptr) return fail(CN_EINVAL, "batch is NULL");
  batch_release(b);
  return CN_OK;
}

cn_status cn_batch_offsets(const cn_batch* b, int64_t* off, int64_t* space_off) {
  if (b == nullptr) return fail(CN_EINVAL, "batch is NULL");
  for (size_t i = 0; i < b->off.size(); ++i) {
    if (off != nullptr) off[i] = b->off[i];
    if (space_off != nullptr) space_off[i] = b->uoff[i];
  }
  return CN_OK;
}

cn_status cn_batch_rhs(cn_batch* b, const double* u0, const double* f, double* bp) {
  if (b == nullptr || u0 == nullptr || f == nullptr || bp == nullptr)
    return fail(CN_EINVAL, "NULL argument");
  for (size_t i = 0; i < b->inst.size(); ++i) {
    const cn_status st = cn_rhs(b->inst[i], u0 + b->uoff[i], f + b->off[i], bp + b->off[i]);
    if (st != CN_OK) return st;
  }
  return CN_OK;
}

cn_status cn_batch_solve(cn_batch* b, const double* bp, double* xp, const cn_gmres_opts* opts,
                         cn_gmres_info* infos, cn_gmres_info* total) {
  if (b == nullptr || bp == nullptr || xp == nullptr || opts == nullptr)
    return fail(CN_EINVAL, "NULL argument");
  if (opts->m < 1 || opts->m > b->m_min)
    return fail(CN_EINVAL, "opts->m must be in [1, smallest m_max of the batch]");
  if (opts->max_iters < 1) return fail(CN_EINVAL, "opts->max_iters must be >= 1");
  if (opts->use_x0 < 0 || opts->use_x0 > 2) return fail(CN_EINVAL, "opts->use_x0 must be 0, 1 or 2");
  if (opts->flags & ~(CN_SOLVE_NO_GRAPHS | CN_SOLVE_ITERATION_GRAPHS))
    return fail(CN_EINVAL, "unknown bits in opts->flags");
  if (!(opts->rtol >= 0.0) || !std::isfinite(opts->rtol))
    return fail(CN_EINVAL, "opts->rtol must be finite and >= 0");
  if (!(opts->err_tol >= 0.0) || !std::isfinite(opts->err_tol))
    return fail(CN_EINVAL, "opts->err_tol must be finite and >= 0");
  if (overlaps(bp, xp, b->off.back() * sizeof(double))) return fail(CN_EINVAL, "b and x overlap");
  SolveCtx c;
  c.s = b->stream;
  c.L = Launch{b->d_desc, (int)b->inst.size(), b->prec};
  c.groups = b->groups;
  c.k2 = b->wl.I_k2;
  c.mv = b->wl.I_mv;
  c.stv = b->wl.I_st;
  c.k2_thr = b->k2_thr;
  c.prec = b->prec;
  c.batched = true;
  c.bh = b->bh;
  c.bh_dev = b->bh_dev;
  c.dcounter = b->dcounter;
  c.bseq = &b->bseq;
  if (!(opts->flags & CN_SOLVE_NO_GRAPHS)) c.graphs = &b->graphs;
  c.cycle_graphs = (opts->flags & CN_SOLVE_ITERATION_GRAPHS) == 0;
  c.cycle_k = &b->cycle_k;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    c.inst_host.push_back(b->inst[i]->hsum);
    c.off.push_back(b->off[i]);
    c.len.push_back(b->inst[i]->n);
  }
  c.ctl = b->h_ctl;
  c.ctl_dev = b->d_ctl;
  c.ctl_last = b->last_ctl.data();
  c.rt = &b->rt;
  c.rt_for = b->rt_for;
  return solve_driver(c, bp, xp, opts, infos, total);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free preconditioner apply.  Every table and work array of one
// apply lives in `scratch`, a file-scope device array of
// CN_NOALLOC_SCRATCH_BYTES (one copy per GPU, held until the process ends,
// shared by all calls on that GPU).  Host code uses the array only through
// the device address looked up per device (the symbol itself is a host-side
// stand-in).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[CN_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_ptr;

// Device address of `scratch` on the current device: looked up on the first
// call on each device (with that device current) and kept.
static hipError_t scratch_base(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (ptr == nullptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = (unsigned char*)ptr;
  *out = (unsigned char*)ptr;
  return hipSuccess;
}

// The tables of one apply, computed on the device from the same definitions
// as the handle's host-side tables (float64 here, long double there):
// tau A rows with the boundary couplings cleared, alpha^{k/N_t} and
// alpha^{-k/N_t}/N_t, the twiddles exp(-2 pi i m/N_t) (full and two-level),
// mu_j = lambda_{1,j}/lambda_{2,j} and 1/lambda_{2,j} with
// lambda_{1,j} = 1 - alpha^{1/N_t} w^j, lambda_{2,j} = dbar (1 + alpha^{1/N_t} w^j)/2
// (dbar: the mean time weight, 1 without weights).  Block 0 also writes the
// instance descriptor and clears the set-up flag.
__global__ void k_noalloc_tables(const double* __restrict__ a_lo, const double* __restrict__ a_di,
                                 const double* __restrict__ a_up, const double* __restrict__ dw,
                                 int nx, int nt, double tau, double alpha, InstDesc desc,
                                 InstDesc* dst, int* err) {
  __shared__ double red[256];
  const PcPlan& pl = desc.pl;
  const int t = threadIdx.x;
  double s = 0.0;
  if (dw != nullptr)
    for (int k = t; k < nt; k += 256) s += dw[k];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double dbar = dw != nullptr ? red[0] / nt : 1.0;
  const int gid = blockIdx.x * 256 + t, gs = gridDim.x * 256;
  if (gid == 0) {
    *dst = desc;
    *err = 0;
  }
  for (int i = gid; i < nx; i += gs) {
    pl.lo[i] = i == 0 ? 0.0 : tau * a_lo[i];
    pl.di[i] = tau * a_di[i];
    pl.up[i] = i == nx - 1 ? 0.0 : tau * a_up[i];
  }
  const double la = log(alpha);
  const int wsl = nt < 64 ? nt : 64, wsh = nt / wsl;
  for (int k = gid; k < nt; k += gs) {
    pl.wfw[k] = exp(la * k / nt);
    pl.winv[k] = exp(-la * k / nt) / nt;
    double sn, cs;
    sincospi(-2.0 * k / nt, &sn, &cs);
    pl.tw[k] = Cx<double>{cs, sn};
    pl.tw_f[k] = Cx<float>{(float)cs, (float)sn};
  }
  for (int e = gid; e < wsl + wsh; e += gs) {
    const int k = e < wsl ? e : (e - wsl) * wsl;
    double sn, cs;
    sincospi(-2.0 * k / nt, &sn, &cs);
    pl.tw2[e] = Cx<double>{cs, sn};
    pl.tw2_f[e] = Cx<float>{(float)cs, (float)sn};
  }
  const double a1 = exp(la / nt);
  for (int j = gid; j < pl.F; j += gs) {
    double wr = 1.0, wi = 0.0;
    if (2 * j == nt) {
      wr = -1.0;
    } else if (j != 0) {
      sincospi(-2.0 * j / nt, &wi, &wr);
    }
    const double l1r = 1.0 - a1 * wr, l1i = -a1 * wi;
    const double l2r = 0.5 * dbar * (1.0 + a1 * wr), l2i = 0.5 * dbar * a1 * wi;
    const double den = l2r * l2r + l2i * l2i;
    pl.mu[j] = Cx<double>{(l1r * l2r + l1i * l2i) / den, (l1i * l2r - l1r * l2i) / den};
    pl.il2[j] = Cx<double>{l2r / den, -l2i / den};
  }
}

extern "C" {

cn_status cn_pc_apply_noalloc(const cn_problem* p, const double* v, double* z) {
  if (p == nullptr || v == nullptr || z == nullptr) return fail(CN_EINVAL, "NULL argument");
  if (p->nx < 1) return fail(CN_EINVAL, "nx must be >= 1");
  if (p->nt < 1 || p->nt > 8192 || (p->nt & (p->nt - 1)) != 0)
    return fail(CN_EINVAL, "nt must be a power of two in [1, 8192]");
  if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(CN_EINVAL, "T must be finite and > 0");
  if (!(p->alpha > 0.0) || !(p->alpha < 1.0)) return fail(CN_EINVAL, "alpha must satisfy 0 < alpha < 1");
  if (p->pc_prec != CN_PC_FP64 && p->pc_prec != CN_PC_FP32)
    return fail(CN_EINVAL, "pc_prec must be CN_PC_FP64 or CN_PC_FP32");
  if (p->a_lo == nullptr || p->a_di == nullptr || p->a_up == nullptr)
    return fail(CN_EINVAL, "A diagonals must be device pointers");
  const int nx = p->nx, nt = p->nt;
  const int prec = p->pc_prec == CN_PC_FP32 ? 1 : 0;
  const size_t rsz = prec ? sizeof(float) : sizeof(double);
  int log2n = 0;
  while ((1 << log2n) < nt) ++log2n;
  int B = 0, T = 0;
  if (!pc_candidate(prec, log2n, 0, &B, &T)) return fail(CN_EINVAL, "no transform variant");
  const int F = nt / 2 + 1, P = (nx + B - 1) / B, NS = P - 1;
  const size_t ns1 = (size_t)std::max(NS, 1);
  const int wsl = std::min(nt, 64), wsh = nt / wsl;
  // layout of the scratch array (256-byte aligned pieces)
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t o_desc = take(sizeof(InstDesc));
  const size_t o_lo = take(nx * sizeof(double)), o_di = take(nx * sizeof(double)),
               o_up = take(nx * sizeof(double));
  const size_t o_wfw = take(nt * sizeof(double)), o_winv = take(nt * sizeof(double));
  const size_t o_tw = take(nt * sizeof(Cx<double>)), o_twf = take(nt * sizeof(Cx<float>));
  const size_t o_tw2 = take((wsl + wsh) * sizeof(Cx<double>)),
               o_tw2f = take((wsl + wsh) * sizeof(Cx<float>));
  const size_t o_mu = take(F * sizeof(Cx<double>)), o_il2 = take(F * sizeof(Cx<double>));
  const size_t o_spec = take((size_t)P * B * nt * rsz);
  const size_t o_iface = take((size_t)F * P * 2 * 2 * rsz);
  const size_t o_sep = take((size_t)F * ns1 * 2 * rsz);
  const size_t o_recf = take((size_t)F * ns1 * 2 * 2 * rsz), o_recb = take((size_t)F * ns1 * 2 * rsz);
  const size_t o_tmp = take((size_t)F * ns1 * sizeof(Cx<double>));
  const size_t o_spk = take((size_t)F * P * 4 * sizeof(Cx<double>));
  const size_t o_err = take(sizeof(int));
  if (off > (size_t)CN_NOALLOC_SCRATCH_BYTES)
    return fail(CN_EINVAL, "problem needs " + std::to_string(off) + " bytes of scratch, more than " +
                               std::to_string((size_t)CN_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = nullptr;
  HIP_TRY(scratch_base(&base));
  PcPlan pl;
  pl.nx = nx;
  pl.nt = nt;
  pl.log2n = log2n;
  pl.F = F;
  pl.prec = prec;
  pl.B = B;
  pl.P = P;
  pl.NS = NS;
  pl.T = T;
  pl.cand = 0;
  pl.alpha = p->alpha;
  pl.lo = (double*)(base + o_lo);
  pl.di = (double*)(base + o_di);
  pl.up = (double*)(base + o_up);
  pl.wfw = (double*)(base + o_wfw);
  pl.winv = (double*)(base + o_winv);
  pl.tw = (Cx<double>*)(base + o_tw);
  pl.tw_f = (Cx<float>*)(base + o_twf);
  pl.tw2 = (Cx<double>*)(base + o_tw2);
  pl.tw2_f = (Cx<float>*)(base + o_tw2f);
  pl.mu = (Cx<double>*)(base + o_mu);
  pl.il2 = (Cx<double>*)(base + o_il2);
  pl.spec = base + o_spec;
  pl.iface = base + o_iface;
  pl.sep = base + o_sep;
  pl.recf = base + o_recf;
  pl.recb = base + o_recb;
  pl.red_tmp = (Cx<double>*)(base + o_tmp);
  InstDesc desc{};
  desc.pl = pl;
  desc.nx = nx;
  desc.nt = nt;
  desc.n = (long long)nx * nt;
  desc.ldx = (nx + 15) / 16 * 16;
  desc.nin = (long long)nt * desc.ldx;
  desc.zf = 0;
  InstDesc* d_desc = (InstDesc*)(base + o_desc);
  int* err = (int*)(base + o_err);
  hipStream_t s = (hipStream_t)p->stream;
  const int grid = (int)std::min<long long>(1024, (std::max(nx, nt) + 255) / 256);
  hipLaunchKernelGGL(k_noalloc_tables, dim3(grid), dim3(256), 0, s, p->a_lo, p->a_di, p->a_up,
                     p->d_half, nx, nt, p->T / nt, p->alpha, desc, d_desc, err);
  HIP_TRY(hipGetLastError());
  HIP_TRY(pc_setup(pl, (Cx<double>*)(base + o_spk), err, s));
  const Launch L{d_desc, 1, 0};
  const Items ipc{nullptr, P}, ik2{nullptr, NS > 0 ? F : 0};
  HIP_TRY(pc_forward(prec, log2n, 0, L, ipc, 0, v, nx, s));
  HIP_TRY(pc_reduced(prec, L, ik2, k2_chunk_class(NS, prec), 0, 1, s));
  HIP_TRY(pc_inverse(prec, log2n, 0, L, ipc, 0, z, 0, nx, s));
  return CN_OK;
}

}  // extern "C"
