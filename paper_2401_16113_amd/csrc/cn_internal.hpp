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
  int cand = 0;                           // compiled (B, T) variant (0 = default)
  double alpha = 0, dbar = 1;
  // device tables
  double *lo = nullptr, *di = nullptr, *up = nullptr;   // tau*A rows
  double *wfw = nullptr, *winv = nullptr;               // alpha^{k/N}, alpha^{-k/N}/N
  Cx<double>* tw = nullptr;                             // exp(-2 pi i m/N)
  Cx<float>* tw_f = nullptr;
  Cx<double>* mu = nullptr;                             // lambda1/lambda2, [F]
  Cx<double>* il2 = nullptr;                            // 1/lambda2, [F]
  Cx<double>* red_a = nullptr;                          // interface system factors [F][NS]
  Cx<double>* red_ap = nullptr;
  Cx<double>* red_inv = nullptr;
  Cx<double>* red_tmp = nullptr;
  void* spec = nullptr;                                 // tile images
  void* iface = nullptr;                                // [F][P][3]
  void* sep = nullptr;                                  // [F][NS]
};

// Scalars the host driver polls (copied to pinned host memory).
struct GSummary {
  double bnorm;   // ||b||
  double beta;    // ||b - M x|| at the start of the current cycle
  double est;     // least-squares residual estimate / ||b||
  double relres;  // beta / ||b||
  int k;          // inner iterations completed in the current cycle
  int done;       // nonzero: the cycle has stopped, remaining kernels return
  int breakdown;  // lucky breakdown (h_{j+1,j} == 0)
  int seq;        // sequence number of the write (host polling), written last
};

// Device state of one GMRES solve (float64), read and written by kernels.
struct GState {
  GSummary sum;
  double H[(MMAX + 1) * MMAX];  // triangular factor, column j at H[j*(MMAX+1)]
  double g[MMAX + 1];
  double cs[MMAX], sn[MMAX];
  double vscale[NVMAX];         // 1/||v_q|| of the stored (unnormalised) basis
  double h1[NVMAX], c1[NVMAX];  // first Gram-Schmidt pass: coefficients
  double h2[NVMAX], c2[NVMAX];  // second pass
  double y[MMAX];
};

// Launchers (cn_pc.hip)
hipError_t pc_setup(PcPlan& pl, Cx<double>* spk, int* err_dev, hipStream_t s);
hipError_t pc_forward(const PcPlan& pl, const double* v, const double* scale_dev,
                      const int* done, hipStream_t s);
hipError_t pc_reduced(const PcPlan& pl, const int* done, hipStream_t s);
hipError_t pc_inverse(const PcPlan& pl, void* z, int z_is_float, const int* done,
                      hipStream_t s);
// (B, T) of compiled candidate `ci`; false if that candidate is not compiled
bool pc_candidate(int prec, int log2n, int ci, int* B, int* T);

// Krylov launchers (cn_krylov.hip)
struct KArgs {
  const double* lo;       // tau*A rows
  const double* di;
  const double* up;
  const double* dw;       // time weights d_k or null
  int nx, nt;
  int rows;               // time levels per matvec workgroup
  long long n;
  const double* V;        // basis base pointer
  long long vstride;      // elements between basis vectors
  int nv;                 // vectors taking part
  GState* st;
  double* partials;       // [grid][NVMAX]
};
constexpr int KGRID = 2048;  // target number of workgroups of a streaming pass
int matvec_rows(int nx, int nt);
// mode 0: y = M x; 1: y = b - M x + norms (finish: cycle start, summary to
// `host`); 2: y = M x + first Gram-Schmidt dots
hipError_t launch_matvec(const KArgs& a, const void* x, int x_is_float, const double* b,
                         double* y, int mode, hipStream_t s, double rtol = 0.0,
                         GSummary* host = nullptr, int seq = 0, bool finish = true);
// passes: 1 = second Gram-Schmidt dots, 2 = update + norm + Givens, 3 = both
hipError_t launch_cgs(const KArgs& a, const double* w, double* vout, int j, int stop_iter,
                      hipStream_t s, int passes = 3, double rtol = 0.0,
                      GSummary* host = nullptr, int seq = 0, bool finish = true);
hipError_t launch_finish_update(GState* st, const void* Z, int z_is_float, long long zstride,
                                double* x, long long n, int x_zero, GSummary* host, int seq,
                                hipStream_t s);
hipError_t launch_rhs(const double* lo, const double* di, const double* up, const double* dw,
                      double tau, const double* u0, const double* f, double* b, int nx,
                      long long n, hipStream_t s);

}  // namespace cn
