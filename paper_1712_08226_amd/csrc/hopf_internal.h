// Internal declarations shared by the host setup code and the HIP solver.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/hopfpd.h"

namespace hopf {

constexpr int NODE_BLOCK = 16;     // table nodes per MFMA row tile
constexpr int POW_LEVELS = 21;     // binary powers e^{2^b delta A}, delta = t_max / 2^20
constexpr int POW_BITS = 20;
constexpr int RDIG_LEVELS = 3;     // base-16 digits of r / dr below one node step

// Host copy of one system plus its device tables.
constexpr int KRON_BMAX = 8;       // largest block of a Kronecker-structured system

struct SysTables {
  hopf_system desc{};
  std::vector<double> A, B, Qu, W, c;   // host copies (row-major), in the solver's coordinates
  bool rotated = false;                 // W was not diagonal: the solver works in x' = U^T x
  std::vector<double> U;                // [n][n] orthogonal, W = U diag(d) U^T (rotated only)
  int n = 0, m = 0, N = 0, n_pad = 0, nkb = 0;
  int m_user = 0;                      // the caller's m; m >= m_user is the padded kernel size
  // k > 1 copies of a b-dimensional system that share the control: A =
  // I_k (x) A_b, B = 1_k (x) B_b, c = 1_k (x) c_b, W = blockdiag(W_b / alpha_c)
  // (W_b diagonal, alpha_0 = 1); value solves then run on the reduced system
  // (ctx->ksys[kron_red], target W_b / sum alpha)
  int kron_k = 0, kron_b = 0, kron_red = -1;
  double kron_atot = 0.0;              // sum of the copies' weights alpha_c
  std::vector<double> kron_winv;       // [b] 1 / diag(W_b), then [k] alpha_c
  double *kron_winv_d = nullptr;
  double h = 0.0, delta = 0.0;
  // host tables
  std::vector<double> phi;     // [N][m][n] node blocks Phi_k = -Qu^T B^T e^{k h A^T}
  std::vector<double> lpref;   // [N+1] upper bound of ||Phi_{0..j-1}||_2^2
  std::vector<double> epow;    // [POW_LEVELS][n][n] e^{2^b delta A}
  // probe setup: x_f = e^{T A} x0 and the extra node's block for T = M h + r,
  // r = q dr + rho, as e^{rho A} e^{q dr A} e^{M h A}
  int n_hbin = 0;              // binary node powers e^{2^b h A}, b < n_hbin (2^n_hbin > last node)
  std::vector<double> hbin;    // [n_hbin][n][n]
  std::vector<double> rdig;    // [RDIG_LEVELS][15][n][n] e^{d 16^b dr A}, d = 1..15
  double dr = 0.0;             // h / 16^RDIG_LEVELS
  double anorm = 0.0;          // max(||A||_1, ||A||_inf): Taylor term count of e^{rho A}
  // device tables
  float *K32 = nullptr;        // [nkb][m][16][n_pad]   dual-operand layout
  double *K64 = nullptr;       // [nkb][m][16][n_pad]
  float *K32T = nullptr;       // [nkb][m][n_pad][16]   primal-operand layout
  double *K64T = nullptr;      // [nkb][m][n_pad][16]
  __bf16 *Kd16h = nullptr, *Kd16l = nullptr;   // BF16 hi/lo split, dual layout
  __bf16 *Kp16h = nullptr, *Kp16l = nullptr;   // BF16 hi/lo split, primal layout
  double *lpref_d = nullptr;   // [N+1]
  double *epow_d = nullptr;    // [POW_LEVELS][n][n]
  // the probe-setup matrices on the device are stored by columns:
  // element (i, k) of each n x n matrix at [k n + i]
  double *hbin_d = nullptr;    // [n_hbin][n][n]
  double *rdig_d = nullptr;    // [RDIG_LEVELS][15][n][n]
  double *At_d = nullptr;      // [n][n]   A by columns
  double *U_d = nullptr;       // [n][n] (rotated systems only)
  double *A_d = nullptr;       // [n][n]
  double *BQ_d = nullptr;      // [n][m]   -B Qu
  double *Wd_d = nullptr;      // [n_pad]  diag W (1 in the padding)
  double *c_d = nullptr;       // [n_pad]
  double *Eh_d = nullptr;      // [n][n]   e^{h A}
  double *Qu_d = nullptr;      // [m_user][m_user]
};

constexpr int MLP_WIDTH = 256;

// Warm-start network of one system (device memory).
struct MlpState {
  int n = 0, H = 0;
  size_t nparam = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr;   // parameters and Adam moments
  float *xm = nullptr, *xs = nullptr;                   // input normalisation
  float t_scale = 1.0f, lam_scale = 1.0f;
  int step = 0, valid = 0;
};
void mlp_free(MlpState &w);

struct Ctx {
  int device = 0;
  int n_cu = 1;                // compute units of the device
  hipStream_t stream = nullptr;
  hopf_opts opts{};
  std::vector<SysTables> sys;
  std::vector<SysTables> ksys;     // reduced systems of the Kronecker-structured ones
  std::vector<MlpState> mlp;       // one per system (optional)
  std::string err;
  // optional probe log of the next solve (filled by the warm-start trainer)
  int *log_pt = nullptr;
  float *log_T = nullptr, *log_lam = nullptr;
  long log_cap = 0;
  long log_count = 0;
  float *net_buf = nullptr;        // first-probe network evaluation (grown on demand)
  size_t net_cap = 0;
  // timing of the last solve
  double t_total = 0.0, t_iter = 0.0, point_rows = 0.0, alg_flops = 0.0;
  double t_tail = 0.0, tail_rows = 0.0;
  long iter_launches = 0, tail_points = 0;
  double t_wide = 0.0, wide_rows = 0.0;   // the 64-point kernel's share of the iteration launches
  long wide_launches = 0;
  // point-state buffers of each job (one job per system in a call), grown on demand
  struct Buf { void *p = nullptr; size_t bytes = 0; };
  std::vector<std::vector<Buf>> jbufs;
  // extra streams (default priority) on which the jobs of a multi-system call run
  std::vector<hipStream_t> pool;
  // events reused by every call (created on first use), pinned words for round checks
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  int *hcount = nullptr;
  long hcount_cap = 0;
  void *scratch = nullptr;         // this device's no-allocation scratch (hipGetSymbolAddress)
};

// host setup (hopf_setup.cpp)
hopf_status build_tables(Ctx *ctx, const hopf_system &s, SysTables &t);
void free_tables(SysTables &t);

// device solver (hopf_solver.hip)
// first-probe network evaluation of one job's points (hopf_mlp.hip)
struct MlpView;
struct PtState;
hopf_status mlp_first_probe(Ctx *ctx, const MlpView &mv, int warm, const PtState &st, long npts, int np,
                            bool caller_lam0, hipStream_t s);
hopf_status solve_dev(Ctx *ctx, int mode, long npts, const int *sys_id, const double *x,
                      const double *t_in, const double *lam0, const double *t_bracket, double *T_out,
                      double *gap_out, double *philo_out, double *phihi_out, double *lam_out,
                      int *probes_out, int *iters_out, int *status_out, hipStream_t user_stream);
hopf_status trajectory_dev(Ctx *ctx, int sys_id, const double *x0_h, double T, int *n_nodes,
                           double *s, double *u, double *xs, double *p_star, double *philo,
                           double *phihi);

hopf_status set_err(Ctx *ctx, hopf_status st, const std::string &msg);

// the device scratch of the no-allocation entry point (hopf_solver.hip)
hopf_status scratch_init(int device, void **out);

}  // namespace hopf
