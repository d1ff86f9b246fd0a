// Internal declarations shared by the translation units of libcn_aao.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "cn_aao.h"
#include "cn_device.hpp"

namespace cn {

constexpr int MMAX = 64;        // largest supported restart length
constexpr int NVMAX = MMAX + 1; // basis vectors

// Preconditioner plan: sizes, float64 tables and workspace of the
// partitioned three-step apply (eq. (3.2)).
struct PcPlan {
  int nx = 0, nt = 0, log2n = 0, F = 0;  // F = nt/2 + 1 frequency lines kept
  int prec = 0;                           // 0: float64, 1: float32
  int B = 0, P = 0, NS = 0, T = 0;        // tile cols, tiles, separators, threads
  int S = 1;                              // K3 workgroups per tile
  int FS = 1;                             // 2: K1 by frequency parity (half the LDS)
  int cand = 0;                           // compiled (B, T, S, FS) variant (0 = default)
  double alpha = 0, dbar = 1;
  // device tables
  double *lo = nullptr, *di = nullptr, *up = nullptr;   // tau*A rows
  double *wfw = nullptr, *winv = nullptr;               // alpha^{k/N}, alpha^{-k/N}/N
  Cx<double>* tw = nullptr;                             // exp(-2 pi i m/N)
  Cx<float>* tw_f = nullptr;
  Cx<double>* tw2 = nullptr;                            // two-level form (64 + N/64 entries)
  Cx<float>* tw2_f = nullptr;
  Cx<double>* mu = nullptr;                             // lambda1/lambda2, [F]
  Cx<double>* il2 = nullptr;                            // 1/lambda2, [F]
  // interface system factors [F][NS], precision of the PC: forward {a, inv}
  // (recf) and backward ap (recb)
  void* recf = nullptr;
  void* recb = nullptr;
  Cx<double>* red_tmp = nullptr;
  void* spec = nullptr;                                 // tile images
  void* iface = nullptr;                                // [F][P][2] partial rhs
  void* sep = nullptr;                                  // [F][NS]
};

// Scalars the host driver polls (written by kernels into pinned host memory).
// A batch summary reuses the layout: k = instances still iterating.
struct GSummary {
  double bnorm;   // ||b||
  double beta;    // ||b - M x|| at the start of the current cycle
  double est;     // least-squares residual estimate / ||b||
  double relres;  // beta / ||b||
  int k;          // inner iterations completed in the current cycle
  int done;       // nonzero: the cycle has stopped, remaining kernels return
  int breakdown;  // lucky breakdown (h_{j+1,j} == 0)
  int x0_rejected;  // the initial guess was replaced by zero (fallback start)
  int pad;
  double err;     // error estimate of a stopped solve (error-controlled stopping)
  int seq;        // sequence number of the write (host polling), written last
};

// Device state of one GMRES solve (float64), read and written by kernels.
struct GState {
  GSummary sum;
  double H[(MMAX + 1) * MMAX];  // triangular factor, column j at H[j*(MMAX+1)]
  double g[MMAX + 1];
  double cs[MMAX], sn[MMAX];
  double vscale[NVMAX];         // 1/||v_q|| of the stored (unnormalised) basis
  double h1[NVMAX], c1[NVMAX];  // first Gram-Schmidt projection: coefficients
  double h2[NVMAX], c2[NVMAX];  // second projection
  double y[MMAX];
  // Gram matrix of the normalised basis, gram[p*NVMAX + q] = <v_p, v_q> /
  // (||v_p|| ||v_q||) (unit diagonal), rows 0..k of the current cycle
  double gram[NVMAX * NVMAX];
  // error estimate in progress: max |Z_0| and max |x| as float64 bit patterns
  // (zero between estimates)
  unsigned long long emax[2];
};

// Per-instance stopping controls, set by the host for each solve.
struct StopCtl {
  double rscale;  // the instance stops at relres <= rtol * rscale (1 unless
                  // error-controlled stopping tightened it)
  int est_skip;   // an error estimate is not asked for this instance
  int pad;
};

// Everything a kernel needs to know about one instance.  Kernels receive an
// array of these plus a work list of (instance, block) items, so one launch
// serves one instance (a handle) or many (a batch).
struct InstDesc {
  PcPlan pl;              // transform tables and preconditioner workspace
  const double* dw;       // time weights d_k or null
  int nx, nt;
  int rows;               // time levels per matvec workgroup
  int mv_cols;            // column blocks of the matvec
  int mv_grid;            // matvec workgroups (partials per dot)
  int st_grid;            // workgroups of the streaming passes
  long long n;            // unknowns (caller layout: row k of N_x values at k N_x)
  int ldx;                // row pitch of the internal row-major vectors (V, w): N_x rounded
                          // up to 16, so every row starts on a 128-byte line
  long long nin;          // elements of an internal vector, N_t ldx (pads stay 0)
  long long vstride;      // elements between basis vectors
  long long off;          // offset of the instance in packed b / x arrays
  double* V;              // basis (m_max + 1 vectors)
  void* Z;                // preconditioned vectors (float64 or float32)
  double* w;              // matvec output
  double* partials;       // per-workgroup partial sums [q][block]: matvec
  double* partials2;      // second buffer: the update pass (written while its
                          // workgroups still read the matvec's partials)
  GState* st;             // solver state
  GSummary* host;         // the instance's summary slot in pinned host memory
  int zf;                 // Z stored in float32
  int zlog;               // Z is tile-blocked with block width 2^zlog (the
                          // transform tile width): element (k, i) of Z_j at
                          // ((i >> zlog) N_t + k) 2^zlog + (i mod 2^zlog);
                          // -1: row-major with pitch ldx
  const StopCtl* ctl;     // per-solve stopping controls of the instance
};

// Element addressing of one column of a space-time vector: element (k, i) at
// col(i) + k * row.  Row-major vectors (the caller's, the basis): col(i) = i,
// row = the pitch.  The preconditioned vectors Z: tile-blocked, so that the
// inverse transform writes each tile as one contiguous block.
struct VecLayout {
  int row;   // elements between consecutive levels of one column
  int zlog;  // tile-blocked: log2 of the tile width; -1: row-major
  int nt;
  __device__ __forceinline__ size_t col(int i) const {
    return zlog < 0 ? (size_t)i
                    : (((size_t)(i >> zlog) * (size_t)nt) << zlog) + (size_t)(i & ((1 << zlog) - 1));
  }
};
__device__ __forceinline__ VecLayout row_major(int pitch, int nt) { return VecLayout{pitch, -1, nt}; }
__device__ __forceinline__ VecLayout z_layout(const InstDesc& d) {
  return d.zlog < 0 ? VecLayout{d.ldx, -1, d.nt} : VecLayout{1 << d.zlog, d.zlog, d.nt};
}

// Launch context shared by the kernels of one handle or batch.
struct Launch {
  const InstDesc* D;      // device array of descriptors
  int ninst;
  int zf;                 // preconditioned vectors stored in float32 (all instances)
};

// Work list of one kernel kind: items[i] = (instance, local block).
struct Items {
  const int2* it = nullptr;  // null: one instance, item i = (0, i) (no list to read)
  int n = 0;
};

// Work item i of a launch (instance, local block).
__device__ __forceinline__ int2 work_item(const int2* __restrict__ items, int i) {
  return items != nullptr ? items[i] : make_int2(0, i);
}

// Launchers (cn_pc.hip, cn_pc_f64.hip, cn_pc_f32.hip).  `v`/`z` override the
// basis vector V_j / Z_j of a single instance (standalone apply, no stop flag);
// `pitch` is their row pitch (0: the internal layout: V_j row-major with pitch
// ldx, Z_j tile-blocked).
hipError_t pc_setup(PcPlan& pl, Cx<double>* spk, int* err_dev, hipStream_t s);
hipError_t pc_forward(int prec, int log2n, int cand, const Launch& L, const Items& it, int j,
                      const double* v, int pitch, hipStream_t s);
// chunk_class: k2_chunk_class(largest NS of the launch, precision): 32 W + CH
// (W wavefronts per line, CH separators per lane), K2_STRIDED + CH (blocks
// of 1024 separators) or K2_ROUNDS + 2 (two rounds of 4096 separators)
constexpr int K2_STRIDED = 4096;
constexpr int K2_ROUNDS = 8192;
int k2_chunk_class(int ns, int prec);
hipError_t pc_reduced(int prec, const Launch& L, const Items& it, int chunk_class, int j,
                      int standalone, hipStream_t s);
hipError_t pc_inverse(int prec, int log2n, int cand, const Launch& L, const Items& it, int j,
                      void* z, int zf, int pitch, hipStream_t s);
// (B, T) of compiled candidate `ci`; false if that candidate is not compiled
bool pc_candidate(int prec, int log2n, int ci, int* B, int* T, int* S = nullptr,
                  int* FS = nullptr);
// Krylov launchers (cn_krylov.hip)
constexpr int KT = 512;     // threads per workgroup of the streaming Krylov kernels
constexpr int KGRID = 512;  // most workgroups of a streaming pass (= partial sums
                            // per dot, which every consumer workgroup re-reduces)
constexpr int MVT = 512;       // threads per workgroup of the matvec (one column each)
constexpr int MV_KGRID = 512;  // target workgroups of the matvec (marching depth)
constexpr int MV_BATCH_ROWS = 8;  // least time levels per matvec block in a batch
int matvec_rows(int nx, int nt);
int stream_grid(long long n);
// y = M x for one instance (standalone matvec)
hipError_t launch_matvec_plain(const Launch& L, const Items& mv, const double* x, double* y,
                               hipStream_t s);
// r = b - M x into V_0 of every instance (x = 0 is not read when x_zero), then
// the per-instance cycle start (norms, stop flag, summary to the host slot).
// start: 0 restart of a solve, 1 first residual of a solve, 2 first residual
// with fallback (an instance whose ||r|| >= ||b|| restarts from x = 0: its
// V_0 becomes b and its x is cleared, on the device)
// guard: speculative (queued before the host knows the cycle stopped): every
// kernel returns at entry for an instance whose cycle is still running
hipError_t launch_residual(const Launch& L, const Items& mv, const Items& stv,
                           const double* b_base, double* x_base, int x_zero, double rtol,
                           int slot, int seq, hipStream_t s, int start = 0, bool guard = false);
// one inner iteration's Krylov part: w = M z_j with the dots against the
// basis, the update pass (both CGS2 projections, the new vector's norm and
// Gram row) and the Givens update (`finish` = false leaves out the finishing
// kernel, for timing the streaming kernels alone)
// passes: bit 0 matvec + dots, bit 2 update + norm + Gram row (bit 1 unused)
hipError_t launch_arnoldi(const Launch& L, const Items& mv, const Items& stv, int j, int stop_iter,
                          double rtol, int slot, int seq, hipStream_t s, int passes = 7,
                          bool finish = true);
// end of a cycle: triangular solve, x += Z y
hipError_t launch_cycle_end(const Launch& L, const Items& stv, double* x_base, int x_zero,
                            int slot, int seq, hipStream_t s, bool guard = false);
// end of a cycle that started from x = 0 (every instance of the launch), in
// two kernels: y, x = Z y and the true residual (into V_0 when store_r) in one
// pass (cycle summary -> slot_fin), then FIN 1 in restart mode (-> slot_res).
// kmax: the most inner iterations any instance of this cycle can have run.
hipError_t launch_cycle_end_zero(const Launch& L, const Items& mv, int kmax,
                                 const double* b_base, double* x_base, double rtol, int slot_fin,
                                 int seq_fin, int slot_res, int seq_res, hipStream_t s,
                                 bool guard = false, bool store_r = true);
// start of an error estimate of a batch from the residual its last cycle end
// stored in V_0 (instead of launch_residual with rtol < 0)
hipError_t launch_err_begin(const Launch& L, hipStream_t s);
// error estimate of a stopped solve, after launch_residual (V_0 = r) and the
// preconditioner of iteration 0 (Z_0 = P^{-1} r / ||r||): ||r|| max|Z_0| /
// max|x| of every instance into its summary slot `slot` (field err)
hipError_t launch_err_estimate(const Launch& L, const Items& stv, const double* x_base, int slot,
                               int seq, hipStream_t s);
// publish the number of instances still iterating (batch polling)
hipError_t launch_batch_summary(const Launch& L, int* counter, GSummary* host, hipStream_t s);
// Per-instance layout of a batch for kernels outside the solver: `dev` (device)
// holds 1 + 5 count int64 values: the packed offsets of the space-time vectors
// [count + 1], of the initial conditions [count] (sums of N_x), of the
// boundary data [count] (sums of N_t), then N_x [count] and N_t [count].
struct BatchLayout {
  const long long* dev = nullptr;
  int count = 0;
  const int* nx = nullptr;  // host copies
  const int* nt = nullptr;
  long long total = 0;      // space-time unknowns of the batch
};
bool batch_layout(const cn_batch* b, BatchLayout* out);
hipError_t launch_rhs(const double* lo, const double* di, const double* up, const double* dw,
                      double tau, const double* u0, const double* f, double* b, int nx,
                      long long n, hipStream_t s);

}  // namespace cn
