// Device-side declarations shared by the solver and the kernel instance
// files: per-point state, per-system view, MFMA wrappers and the two
// templated hot kernels (fused PDHG iterations, FP64 certificate).
#pragma once

#include <hip/hip_runtime.h>

#include "hopf_internal.h"

namespace hopf {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int WAVES = 4;
constexpr int PTS_WAVE = 16;
constexpr int PTS_WG = WAVES * PTS_WAVE;
constexpr int PTS_TILE = 16;       // points per workgroup in the iteration and certificate kernels
constexpr int THREADS = WAVES * 64;
constexpr int LDS_BYTES = 76 * 1024;

enum { MODE_VALUE = 0, MODE_MINTIME = 1 };
// search phase of a point: PH_SCAN probes the uniform scan horizons in
// ascending order; PH_PROBE refines the first cell with a sign change;
// PH_FINAL continues the solve at T = hi to the gap tolerance
enum { PH_PROBE = 0, PH_FINAL = 1, PH_DONE = 2, PH_SCAN = 3 };

__device__ __forceinline__ floatx4 mfma(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of the 16x16 accumulator held in register q of a lane in group g
// (g = lane / 16; the column is lane % 16).  Measured on gfx950:
// v_mfma_f32_16x16x4f32 -> row 4 g + q;  v_mfma_f64_16x16x4f64 -> row g + 4 q.
// Operands A (16 x 4) and B (4 x 16) are A[lane % 16][lane / 16] and
// B[lane / 16][lane % 16] for both.
template <typename Tv> __device__ __forceinline__ constexpr int acc_row(int g, int q) {
  return sizeof(Tv) == 4 ? 4 * g + q : g + 4 * q;
}

__device__ __forceinline__ float gelu_f(float v) { return 0.5f * v * (1.0f + erff(v * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float v) {
  return 0.5f * (1.0f + erff(v * 0.70710678118654752f)) + v * expf(-0.5f * v * v) * 0.3989422804014327f;
}

template <typename Tv> struct V4;
template <> struct V4<float> { typedef floatx4 t; };
template <> struct V4<double> { typedef doublex4 t; };

// ------------------------------------------------------------------ per-point state

struct SysView {
  int n, m, N, n_pad, nkb, quad, uset, m_user;
  double t_max, h, delta, c_tau;   // c_tau: the system's step ratio (0: the call's)
  int n_hbin;
  double dr, anorm;
  const double *hbin, *rdig, *At;  // probe-setup powers and A, stored by columns (see SysTables)
  const double *U;                 // [n][n] x = U x' for a rotated system (non-diagonal W), else null
  const float *K32, *K32T;
  const __bf16 *Kd16h, *Kd16l, *Kp16h, *Kp16l;     // BF16 hi/lo copies (dual and primal layouts)
  const double *K64, *K64T, *lpref, *epow, *A, *BQ, *Wd, *c, *Eh, *Qu;
};

struct PtState {
  long npts;
  int ystride;               // floats of y per point (nkb * m * 16)
  int mpad;                  // floats of the partial-node dual per point
  double *x0;                // [npts][n_pad]
  int *status, *phase, *flags, *probes, *iters_tot, *iters_probe, *rows, *M, *partial;
  int *nscan;                // scan probes decided
  int *ncell;                // probes of the first sign-change cell decided
  int *newt;                 // bit 0: the running probe was placed by a Newton step; bit 1: no Newton step next;
                             // bit 2: the running probe runs to the Newton accuracy
  double *wbef;              // bracket width when the running probe was placed
  double *ha, *hb;           // probe hints inside the cell (caller's t_bracket or the network's)
  double *lam0s;             // [npts][n_pad] caller's starting costate of the first probe, or null
  // minimum time on the reduced system of k copies (else null): the copies'
  // spread s(T) at the point's probe horizon and ds/dT, which turn the
  // reduced problem's bounds into the full system's (phi = phi_red + s)
  double *kspread, *kdspread;
  double *T, *lo, *hi, *r, *tau, *sig, *P, *D;
  double *xf;                // [npts][n_pad]
  double *axf;               // [npts][n_pad]  A x_f (time derivative of x_f, for the Newton slope)
  float *xfc32;              // [npts][n_pad]  x_f - c
  double *R64;               // [npts][m][n_pad]
  float *R32;                // [npts][m][n_pad]
  float *lam, *lamb;         // [npts][n_pad]
  float *y;                  // [npts][ystride]
  float *yR;                 // [npts][mpad]
  int *perm;                 // [npts]
  int *setup_list;           // [npts] points waiting for a probe setup
  int *counters;             // [0] active, [1] setup-list length, [2] probe-log length
  int *stage;                // [npts] hints still to probe: 0 both (hb then ha), 1 ha only, 2 none
  int *esc;                  // [npts] 1: iterate in FP32 (escalated from BF16 hi+lo)
  float *lamref, *yref;      // tail solver: iterate at the last restart ([npts][n_pad], [npts][ystride])
  // FP64 iterations only (else null): the iterate in FP64 between launches, with
  // s64[p] = 1 when it is current; lam/lamb/y/yR then hold its FP32 rounding,
  // which the certificate and the read-out use
  double *lam64, *lamb64, *y64, *yR64;
  int *s64;
  float *bT, *bD;            // [npts] predicted minimum time and log-bracket half-width
  int *log_pt;               // optional probe log: point, horizon, final lam of each probe
  float *log_T, *log_lam;
  int log_cap;
  double *rowsum;            // accumulated point-rows for flop accounting
};

struct Opts {
  double c_tau, gap_tol, t_rel_tol, t_abs_frac;
  int max_iter, check_every, warm, prec, esc_iters;
  int root, newton_after;
  double newton_rho;
  int adapt;
  int scan;                  // scan horizons: table nodes nearest t_max (j / scan)^2, j = 1..scan
};

// Table nodes as probe horizons.  K = index of the node at t_max; the scan
// probes the node nearest to t_max (j / scan)^2 (at least node 1) for
// j = 1..scan, repeats skipped, the last one K: the spacing grows like
// sqrt(t), finest near t = 0 where reachable intervals of horizons are
// short, and a node needs no extra quadrature node.
__host__ __device__ __forceinline__ int last_node(int N, int quad) { return quad == HOPF_Q_TRAP ? N - 1 : N; }
__host__ __device__ __forceinline__ double node_horizon(double t_max, double h, int K, int k) {
  return k >= K ? t_max : (double)k * h;
}
__host__ __device__ __forceinline__ int scan_node(int K, int scan, int j) {
  if (j >= scan) return K;
  const double s = (double)j / (double)scan;
  const int k = (int)rint((double)K * s * s);
  return k < 1 ? 1 : (k > K ? K : k);
}
// the table node at t when t is one (within 1e-12 relative), else the node below
__host__ __device__ __forceinline__ int node_floor(double t, double h, bool &exact) {
  const double q = t / h;
  const double qr = rint(q);
  exact = fabs(q - qr) <= 1e-12 * fmax(1.0, q);
  return exact ? (int)qr : (int)floor(q);
}

// point range of one iteration launch: 0 = FP32-escalated points
// [0, counters[3]), 1 = the others [counters[3], counters[0]), 2 = all
__device__ __forceinline__ void launch_range(const PtState &st, int part, int &beg, int &end) {
  beg = part == 1 ? st.counters[3] : 0;
  end = part == 0 ? st.counters[3] : st.counters[0];
}

// Read-only view of a trained warm-start network (see hopf_mlp.hip).
struct MlpView {
  const float *theta, *xm, *xs;
  float t_scale, lam_scale;
  int n, H, valid;
};

enum { FL_SETUP = 1 };

// append (point, horizon, final lam) of a finished probe to the optional log
__device__ __forceinline__ void log_probe(const PtState &st, long p, int np) {
  if (!st.log_pt) return;
  const int e = atomicAdd(&st.counters[2], 1);
  if (e >= st.log_cap) return;
  st.log_pt[e] = (int)p;
  st.log_T[e] = (float)st.T[p];
  for (int i = 0; i < np; ++i) st.log_lam[(long)e * np + i] = st.lam[p * np + i];
}

// queue point p for a probe setup at its (new) horizon st.T[p]
__device__ __forceinline__ void mark_setup(const PtState &st, long p) {
  st.flags[p] = FL_SETUP;
  st.setup_list[atomicAdd(&st.counters[1], 1)] = (int)p;
}

// quadrature weight of table node k for a point with (M, r)
__device__ __forceinline__ double node_weight(int k, int M, double r, double h, int quad) {
  if (quad == HOPF_Q_TRAP) {
    if (k < M) return k == 0 ? 0.5 * h : h;
    if (k == M) return (M > 0 ? 0.5 * h : 0.0) + 0.5 * r;
    return 0.0;
  }
  if (k < M) return h;
  if (k == M) return r;
  return 0.0;
}

// ------------------------------------------------------------------ fused PDHG iterations

// Tile = 16 points (the MFMA column dimension); the 4 waves of a workgroup
// split the tile's node blocks (wave w takes blocks w, w+4, ...), so one
// tile's iteration runs on all four SIMDs of a CU.  Operand A of both GEMMs
// is read straight from L2 in two pre-swizzled copies of the node table:
//   dual   Kd[kb][j][16 nodes][n_pad]  -> lane reads 4 consecutive state columns
//   primal Kp[kb][j][n_pad][16 nodes]  -> lane reads 4 consecutive nodes
// Each lane owns column cl = lane % 16 and accumulator rows acc_row(g, q).
// The per-wave partial G is summed over the waves through LDS once per
// iteration; every wave then applies the (cheap) prox redundantly so that
// all of them hold sigma * lam_bar for the next dual GEMM.
template <typename Tv, int NT, int MM, int WV>
__global__ __launch_bounds__(WV * 64, WV == 4 ? 2 : 1) void k_pdhg(SysView S, PtState st, int iters, int part) {
  typedef typename V4<Tv>::t vec4;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Tv *gred = reinterpret_cast<Tv *>(lds_raw);                       // [2][WV][NT][4][64]
  Tv *pscr = gred + 2 * WV * NT * 4 * 64;                        // partial-node scratch
  const int tile = blockIdx.x;
  int beg, nact;
  launch_range(st, part, beg, nact);
  if (beg + tile * PTS_TILE >= nact) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  constexpr int m = MM;          // components (the tables are zero-padded to MM)
  constexpr int np = 16 * NT;    // padded state dimension
  const int slot = beg + tile * PTS_TILE + cl;
  const bool live = slot < nact;
  const long p = live ? st.perm[slot] : -1;
  const long pd = live ? p : st.npts;     // lanes without a point use the spare row npts
  const int rows_max = st.rows[st.perm[beg + tile * PTS_TILE]];
  const int nkb = (rows_max + NODE_BLOCK - 1) / NODE_BLOCK;
  __shared__ int any_part;
  if (threadIdx.x == 0) any_part = 0;
  __syncthreads();
  if (wave == 0 && g == 0 && live && st.partial[p]) atomicOr(&any_part, 1);
  __syncthreads();
  const bool wg_part = any_part != 0;

  const Tv *Kd = (sizeof(Tv) == 4) ? reinterpret_cast<const Tv *>(S.K32) : reinterpret_cast<const Tv *>(S.K64);
  const Tv *Kp = (sizeof(Tv) == 4) ? reinterpret_cast<const Tv *>(S.K32T) : reinterpret_cast<const Tv *>(S.K64T);

  Tv tau = 0, sig = 0, rr = 0;
  const Tv hw = (Tv)S.h;
  int M = -1, rowsp = 0;
  if (live) {
    tau = (Tv)st.tau[p];
    sig = (Tv)st.sig[p];
    rr = (Tv)st.r[p];
    M = st.M[p];
    rowsp = st.rows[p];
  }
  // FP64 iterations continue from the FP64 iterate of the previous launch
  const bool v64 = sizeof(Tv) == 8 && st.s64 != nullptr && live && st.s64[p] != 0;
  Tv lam[NT][4], bop[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * t + acc_row<Tv>(g, q);
      if (v64) {
        lam[t][q] = (Tv)st.lam64[pd * np + i];
        bop[t][q] = sig * (Tv)st.lamb64[pd * np + i];
      } else {
        lam[t][q] = (Tv)st.lam[pd * np + i];
        bop[t][q] = sig * (Tv)st.lamb[pd * np + i];
      }
    }
  float *yp = st.y + (size_t)pd * st.ystride;
  double *yp64 = st.y64 ? st.y64 + (size_t)pd * st.ystride : nullptr;

  for (int it = 0; it < iters; ++it) {
    vec4 G[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) G[t] = vec4{0, 0, 0, 0};

    // ---- private node at tau = T (trapezoid rule, T off the grid): wave 0.
    // FP32: in registers in one pass over R, as in k_pdhg_wide (the four
    // lanes of a point hold all of its lambda_bar rows, 16 t + 4 g + q); the
    // term enters wave 0's share of G only.
    if constexpr (sizeof(Tv) == 4) {
      if (wave == 0 && wg_part) {
        const bool ppart = live && st.partial[p] != 0;
        const float wR = ppart ? 0.5f * (float)rr : 0.f;
        const float *Rp = ppart ? st.R32 + (size_t)p * m * np : nullptr;
        float *yRp = ppart ? st.yR + (size_t)p * st.mpad : nullptr;
        const bool box = S.uset != HOPF_U_L2;
        float ssq = 0.f;
        float4 rn[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          rn[t] = ppart ? *reinterpret_cast<const float4 *>(Rp + 16 * t + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 1
        for (int j = 0; j < m; ++j) {
          float4 rv[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) rv[t] = rn[t];
          if (j + 1 < m)
#pragma unroll
            for (int t = 0; t < NT; ++t)
              rn[t] = ppart ? *reinterpret_cast<const float4 *>(Rp + (size_t)(j + 1) * np + 16 * t + 4 * g)
                            : make_float4(0.f, 0.f, 0.f, 0.f);
          float acc = 0.f;
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc += rv[t].x * bop[t][0] + rv[t].y * bop[t][1] + rv[t].z * bop[t][2] + rv[t].w * bop[t][3];
          acc += __shfl_xor(acc, 16);
          acc += __shfl_xor(acc, 32);
          float v = ppart ? yRp[j] + acc : 0.f;
          if (box) v = fminf(fmaxf(v, -wR), wR);
          ssq += v * v;
          if (ppart && g == 0) {
            yRp[j] = v;                              // the l2 ball's scale is applied below
            if (st.yR64) st.yR64[(size_t)p * st.mpad + j] = (double)v;
          }
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            G[t][0] += rv[t].x * v;
            G[t][1] += rv[t].y * v;
            G[t][2] += rv[t].z * v;
            G[t][3] += rv[t].w * v;
          }
        }
        if (!box) {
          const float nv = sqrtf(ssq);
          const float sc = (nv > wR) ? (nv > 0.f ? wR / nv : 0.f) : 1.f;
          if (ppart && g == 0)
            for (int j = 0; j < m; ++j) {
              yRp[j] *= sc;
              if (st.yR64) st.yR64[(size_t)p * st.mpad + j] = (double)yRp[j];
            }
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) G[t][q] *= sc;
        }
      }
    } else if (wg_part) {
      Tv *lb_s = pscr;                 // [16][np]
      Tv *gr_s = lb_s + 16 * np;       // [16][np]
      Tv *yr_s = gr_s + 16 * np;       // [16][MM]
      if (wave == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) lb_s[cl * np + 16 * t + acc_row<Tv>(g, q)] = (sig > 0 ? bop[t][q] / sig : (Tv)0);
      }
      __syncthreads();
      if (wave == 0) {
        const int pp = lane >> 2, qq = lane & 3;     // point pp of the tile, lane quarter qq
        const int pslot = beg + tile * PTS_TILE + pp;
        const bool plive = pslot < nact;
        const long P2 = plive ? st.perm[pslot] : -1;
        const bool ppart = plive && st.partial[P2];
        const Tv *Rr = (sizeof(Tv) == 4) ? reinterpret_cast<const Tv *>(st.R32) : reinterpret_cast<const Tv *>(st.R64);
        Tv vj[(MM + 3) / 4];
        Tv ssq = 0;
        const Tv sig2 = ppart ? (Tv)st.sig[P2] : (Tv)0;
        const Tv wR = ppart ? (Tv)(0.5 * st.r[P2]) : (Tv)0;
#pragma unroll
        for (int a = 0; a < (MM + 3) / 4; ++a) {
          const int j = qq + 4 * a;
          Tv v = 0;
          if (ppart && j < m) {
            const Tv *row = Rr + ((size_t)P2 * m + j) * np;
            Tv acc = 0;
            for (int i = 0; i < np; ++i) acc += row[i] * lb_s[pp * np + i];
            const bool r64 = sizeof(Tv) == 8 && st.s64 != nullptr && st.s64[P2] != 0;
            v = (r64 ? (Tv)st.yR64[(size_t)P2 * st.mpad + j] : (Tv)st.yR[(size_t)P2 * st.mpad + j]) + sig2 * acc;
          }
          vj[a] = v;
          ssq += v * v;
        }
        if (S.uset == HOPF_U_L2) {
          ssq += __shfl_xor(ssq, 1);
          ssq += __shfl_xor(ssq, 2);
          const Tv nv = sqrt(ssq);
          const Tv sc = (nv > wR) ? (nv > 0 ? wR / nv : (Tv)0) : (Tv)1;
#pragma unroll
          for (int a = 0; a < (MM + 3) / 4; ++a) vj[a] *= sc;
        } else {
#pragma unroll
          for (int a = 0; a < (MM + 3) / 4; ++a) vj[a] = fmin(fmax(vj[a], -wR), wR);
        }
#pragma unroll
        for (int a = 0; a < (MM + 3) / 4; ++a) {
          const int j = qq + 4 * a;
          if (j < MM) yr_s[pp * MM + j] = vj[a];
          if (ppart && j < m) {
            st.yR[(size_t)P2 * st.mpad + j] = (float)vj[a];
            if (st.yR64) st.yR64[(size_t)P2 * st.mpad + j] = (double)vj[a];
          }
        }
      }
      __syncthreads();
      if (wave == 0) {
        const int pp = lane >> 2, qq = lane & 3;
        const int pslot = beg + tile * PTS_TILE + pp;
        const bool plive = pslot < nact;
        const long P2 = plive ? st.perm[pslot] : -1;
        const bool ppart = plive && st.partial[P2];
        const Tv *Rr = (sizeof(Tv) == 4) ? reinterpret_cast<const Tv *>(st.R32) : reinterpret_cast<const Tv *>(st.R64);
        for (int i = qq; i < np; i += 4) {
          Tv acc = 0;
          if (ppart)
            for (int j = 0; j < m; ++j) acc += Rr[((size_t)P2 * m + j) * np + i] * yr_s[pp * MM + j];
          gr_s[pp * np + i] = acc;
        }
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) G[t][q] = gr_s[cl * np + 16 * t + acc_row<Tv>(g, q)];
      }
    }

    // ---- this wave's share of the node table
    for (int kb = wave; kb < nkb; kb += WV) {
      // y is stored node-major within a block: offset kk = node % 16
      vec4 V[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const float *src = yp + (size_t)(kb * m + j) * NODE_BLOCK;
        if constexpr (sizeof(Tv) == 4) {
          const float4 f = *reinterpret_cast<const float4 *>(src + 4 * g);
          V[j] = vec4{(Tv)f.x, (Tv)f.y, (Tv)f.z, (Tv)f.w};
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            V[j][q] = v64 ? (Tv)yp64[(size_t)(kb * m + j) * NODE_BLOCK + acc_row<Tv>(g, q)]
                          : (Tv)src[acc_row<Tv>(g, q)];
        }
      }
      // dual GEMM: V_j += K_j (sigma lam_bar), A = Kd[kb][j][node cl][16 t + acc_row(g, q)];
      // the operands of step t + 1 are loaded before the MFMAs of step t
      const Tv *kd = Kd + ((size_t)kb * m * NODE_BLOCK + cl) * np;
      Tv af[2][MM][4];
      auto load_af = [&](int t, Tv (&dst)[MM][4]) {
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          const Tv *a = kd + (size_t)j * NODE_BLOCK * np + 16 * t;
          if constexpr (sizeof(Tv) == 4) {
            const float4 f = *reinterpret_cast<const float4 *>(a + 4 * g);
            dst[j][0] = f.x; dst[j][1] = f.y; dst[j][2] = f.z; dst[j][3] = f.w;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[j][q] = a[acc_row<Tv>(g, q)];
          }
        }
      };
      load_af(0, af[0]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t + 1 < NT) load_af(t + 1, af[(t + 1) & 1]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < MM; ++j) V[j] = mfma(af[t & 1][j][q], bop[t][q], V[j]);
        __builtin_amdgcn_sched_barrier(0);
      }
      // projection onto w_k C per (node, point)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kb * NODE_BLOCK + acc_row<Tv>(g, q);
        const Tv w = (k < rowsp) ? (Tv)node_weight(k, M, (double)rr, (double)hw, S.quad) : (Tv)0;
        if (S.uset == HOPF_U_L2) {
          Tv s = 0;
#pragma unroll
          for (int j = 0; j < MM; ++j) s += V[j][q] * V[j][q];
          const Tv nv = sqrt(s);
          const Tv sc = (nv > w) ? (nv > 0 ? w / nv : (Tv)0) : (Tv)1;
#pragma unroll
          for (int j = 0; j < MM; ++j) V[j][q] *= sc;
        } else {
#pragma unroll
          for (int j = 0; j < MM; ++j) V[j][q] = fmin(fmax(V[j][q], -w), w);
        }
      }
      // store Y
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        float *dst = yp + (size_t)(kb * m + j) * NODE_BLOCK;
        if constexpr (sizeof(Tv) == 4) {
          float4 f;
          f.x = (float)V[j][0]; f.y = (float)V[j][1]; f.z = (float)V[j][2]; f.w = (float)V[j][3];
          *reinterpret_cast<float4 *>(dst + 4 * g) = f;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            dst[acc_row<Tv>(g, q)] = (float)V[j][q];
            if (yp64) yp64[(size_t)(kb * m + j) * NODE_BLOCK + acc_row<Tv>(g, q)] = (double)V[j][q];
          }
        }
      }
      // primal GEMM: G += K_j^T Y_j, A = Kp[kb][j][16 t + cl][node acc_row(g, q)]
      const Tv *kp = Kp + (size_t)kb * m * np * NODE_BLOCK;
      Tv ap[2][NT][4];
      auto load_ap = [&](int j, Tv (&dst)[NT][4]) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const Tv *a = kp + ((size_t)j * np + 16 * t + cl) * NODE_BLOCK;
          if constexpr (sizeof(Tv) == 4) {
            const float4 f = *reinterpret_cast<const float4 *>(a + 4 * g);
            dst[t][0] = f.x; dst[t][1] = f.y; dst[t][2] = f.z; dst[t][3] = f.w;
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[t][q] = a[acc_row<Tv>(g, q)];
          }
        }
      };
      load_ap(0, ap[0]);
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        if (j + 1 < MM) load_ap(j + 1, ap[(j + 1) & 1]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int t = 0; t < NT; ++t) G[t] = mfma(ap[j & 1][t][q], V[j][q], G[t]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    // ---- sum G over the waves (double-buffered LDS), then prox and extrapolation
    Tv *gb = gred + (size_t)(it & 1) * WV * NT * 4 * 64;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) gb[((wave * NT + t) * 4 + q) * 64 + lane] = G[t][q];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        Tv gs = 0;
#pragma unroll
        for (int w2 = 0; w2 < WV; ++w2) gs += gb[((w2 * NT + t) * 4 + q) * 64 + lane];
        const int i = 16 * t + acc_row<Tv>(g, q);
        const Tv xfc = (Tv)st.xfc32[pd * np + i];
        const Tv wd = (Tv)S.Wd[i];
        const Tv ln = (lam[t][q] - tau * (gs - xfc)) / ((Tv)1 + tau * wd);
        bop[t][q] = sig * ((Tv)2 * ln - lam[t][q]);
        lam[t][q] = ln;
      }
  }
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 16 * t + acc_row<Tv>(g, q);
        st.lam[pd * np + i] = (float)lam[t][q];
        st.lamb[pd * np + i] = (float)(sig > 0 ? bop[t][q] / sig : (Tv)0);
        if (sizeof(Tv) == 8 && st.lam64) {
          st.lam64[pd * np + i] = (double)lam[t][q];
          st.lamb64[pd * np + i] = (double)(sig > 0 ? bop[t][q] / sig : (Tv)0);
        }
      }
    if (live && g == 0) {
      st.iters_probe[p] += iters;
      st.iters_tot[p] += iters;
      if (sizeof(Tv) == 8 && st.s64) st.s64[p] = 1;
    }
  }
}

// ------------------------------------------------------------------ wide FP32 iterations (64 points, K staged in LDS)

// The same iteration as k_pdhg for FP32 with a workgroup of 64 points: wave
// w owns points 16 w .. 16 w + 15 of the workgroup's slots and runs every
// node block for them, so its G = K^T Y needs no cross-wave sum.  Each
// 16-node block of the table (dual layout, one row of n_pad values per
// (component, node)) is copied once into LDS and read by all four waves:
// one global read of K serves 64 points instead of 16.  Operand reads from
// LDS: dual GEMM A = K_j[node cl][16 t + 4 g .. +3] (one 16-byte read),
// primal GEMM A = K_j[node 4 g + q][16 t + cl]; the row stride n_pad + 4
// spreads the rows of a 16-byte read over the banks.  The extra node at
// tau = T (trapezoid, T off the grid) is applied per point in registers:
// the four lanes of a point hold all of its lambda_bar rows, reduce R lam_bar
// with two shuffles, project, and add R^T y_R to their rows of G.
constexpr int WIDE_PTS = 64;
__host__ __device__ constexpr int wide_row_stride(int NT) { return 16 * NT + 4; }

template <int NT, int MM>
__global__ __launch_bounds__(THREADS, 2) void k_pdhg_wide(SysView S, PtState st, int iters, int part) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int np = 16 * NT;
  constexpr int KS = wide_row_stride(NT);
  constexpr int m = MM;
  float *ks = reinterpret_cast<float *>(lds_raw);           // [MM][16][KS]
  int beg, nact;
  launch_range(st, part, beg, nact);
  const int wg0 = beg + blockIdx.x * WIDE_PTS;
  if (wg0 >= nact) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int slot = wg0 + wave * PTS_WAVE + cl;
  const bool live = slot < nact;
  const long p = live ? st.perm[slot] : -1;
  const long pd = live ? p : st.npts;
  const int rows_max = st.rows[st.perm[wg0]];     // slots are sorted by rows, descending
  const int nkb = (rows_max + NODE_BLOCK - 1) / NODE_BLOCK;

  float tau = 0.f, sig = 0.f, rr = 0.f;
  int M = -1, rowsp = 0;
  bool ppart = false;
  if (live) {
    tau = (float)st.tau[p];
    sig = (float)st.sig[p];
    rr = (float)st.r[p];
    M = st.M[p];
    rowsp = st.rows[p];
    ppart = st.partial[p] != 0;
  }
  const bool wave_part = __any(ppart);
  const float wR = ppart ? 0.5f * rr : 0.f;
  const float hw = (float)S.h;
  // sigma lam_bar stays in registers (operand of the dual GEMM); lam itself
  // is read and written in memory once per iteration, at the prox step
  float bop[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) bop[t][q] = sig * st.lamb[pd * np + 16 * t + 4 * g + q];
  float *lamp = st.lam + pd * np;
  float *yp = st.y + (size_t)pd * st.ystride;
  const float *Rp = ppart ? st.R32 + (size_t)p * m * np : nullptr;
  const int nchunk = m * NODE_BLOCK * (np / 4);               // float4 chunks of one node block

  for (int it = 0; it < iters; ++it) {
    floatx4 G[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) G[t] = floatx4{0, 0, 0, 0};

    // ---- extra node at tau = T, in registers, one pass over R: for each
    // component j, v_j = y_R,j + R_j . (sigma lam_bar) (the four lanes of a
    // point reduce with two shuffles) and the primal term R_j^T (.) is added
    // to G with the same loaded row: the clamped v_j for the box; for the l2
    // ball v_j itself, G being scaled by the projection factor afterwards
    // (G holds only this term at that point)
    if (wave_part) {
      float ssq = 0.f;
      const bool box = S.uset != HOPF_U_L2;
      float *yRp = ppart ? st.yR + (size_t)p * st.mpad : nullptr;
      // row j + 1 of R is loaded while row j is used
      float4 rn[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t)
        rn[t] = ppart ? *reinterpret_cast<const float4 *>(Rp + 16 * t + 4 * g) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 1
      for (int j = 0; j < m; ++j) {
        float4 rv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) rv[t] = rn[t];
        if (j + 1 < m)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            rn[t] = ppart ? *reinterpret_cast<const float4 *>(Rp + (size_t)(j + 1) * np + 16 * t + 4 * g)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc += rv[t].x * bop[t][0] + rv[t].y * bop[t][1] + rv[t].z * bop[t][2] + rv[t].w * bop[t][3];
        acc += __shfl_xor(acc, 16);
        acc += __shfl_xor(acc, 32);
        float v = ppart ? yRp[j] + acc : 0.f;
        if (box) v = fminf(fmaxf(v, -wR), wR);
        ssq += v * v;
        if (ppart && g == 0) yRp[j] = v;           // the l2 ball's scale is applied below
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          G[t][0] += rv[t].x * v;
          G[t][1] += rv[t].y * v;
          G[t][2] += rv[t].z * v;
          G[t][3] += rv[t].w * v;
        }
      }
      if (!box) {
        const float nv = sqrtf(ssq);
        const float sc = (nv > wR) ? (nv > 0.f ? wR / nv : 0.f) : 1.f;
        if (ppart && g == 0)
          for (int j = 0; j < m; ++j) yRp[j] *= sc;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) G[t][q] *= sc;
      }
    }

    for (int kb = 0; kb < nkb; ++kb) {
      // ---- stage node block kb of the dual table in LDS
      __syncthreads();                                    // every wave is done with the previous block
      const float4 *src = reinterpret_cast<const float4 *>(S.K32 + (size_t)kb * m * NODE_BLOCK * np);
      for (int e = threadIdx.x; e < nchunk; e += THREADS) {
        const int row = e / (np / 4), c4 = e - row * (np / 4);
        *reinterpret_cast<float4 *>(ks + row * KS + 4 * c4) = src[e];
      }
      __syncthreads();
      // ---- dual GEMM: V_j = Y_j + K_j (sigma lam_bar)
      floatx4 V[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const float4 f = *reinterpret_cast<const float4 *>(yp + (size_t)(kb * m + j) * NODE_BLOCK + 4 * g);
        V[j] = floatx4{f.x, f.y, f.z, f.w};
      }
      // A = K_j[node cl][16 t + 4 g + q]: one 16-byte LDS read per (j, t)
      // gives the four steps q of column group t (the row stride puts the 16
      // rows of a read in distinct banks); the reads of group t + 1 are
      // issued at the last step of group t, so their latency hides behind
      // that step's matrix-core work
      {
        const float *kd = ks + cl * KS + 4 * g;
        float4 a4[MM];
#pragma unroll
        for (int j = 0; j < MM; ++j) a4[j] = *reinterpret_cast<const float4 *>(kd + j * NODE_BLOCK * KS);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float a[MM];
#pragma unroll
            for (int j = 0; j < MM; ++j) a[j] = q == 0 ? a4[j].x : q == 1 ? a4[j].y : q == 2 ? a4[j].z : a4[j].w;
            if (q == 3 && t + 1 < NT)
#pragma unroll
              for (int j = 0; j < MM; ++j)
                a4[j] = *reinterpret_cast<const float4 *>(kd + j * NODE_BLOCK * KS + 16 * (t + 1));
#pragma unroll
            for (int j = 0; j < MM; ++j) V[j] = mfma(a[j], bop[t][q], V[j]);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      // ---- projection onto w_k C per (node, point), rows 4 g + q
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kb * NODE_BLOCK + 4 * g + q;
        const float w = (k < rowsp) ? (float)node_weight(k, M, (double)rr, (double)hw, S.quad) : 0.f;
        if (S.uset == HOPF_U_L2) {
          float ss = 0.f;
#pragma unroll
          for (int j = 0; j < MM; ++j) ss += V[j][q] * V[j][q];
          const float nv = sqrtf(ss);
          const float sc = (nv > w) ? (nv > 0.f ? w / nv : 0.f) : 1.f;
#pragma unroll
          for (int j = 0; j < MM; ++j) V[j][q] *= sc;
        } else {
#pragma unroll
          for (int j = 0; j < MM; ++j) V[j][q] = fminf(fmaxf(V[j][q], -w), w);
        }
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        float4 f;
        f.x = V[j][0]; f.y = V[j][1]; f.z = V[j][2]; f.w = V[j][3];
        *reinterpret_cast<float4 *>(yp + (size_t)(kb * m + j) * NODE_BLOCK + 4 * g) = f;
      }
      // ---- primal GEMM: G_t += K_j^T Y_j, A = K_j[node 4 g + q][16 t + cl]
      {
        float b[2][NT];
        const float *kp = ks + 4 * g * KS + cl;
#pragma unroll
        for (int t = 0; t < NT; ++t) b[0][t] = kp[16 * t];
#pragma unroll
        for (int sidx = 0; sidx < 4 * MM; ++sidx) {
          const int j = sidx >> 2, q = sidx & 3;
          if (sidx + 1 < 4 * MM) {
            const int j1 = (sidx + 1) >> 2, q1 = (sidx + 1) & 3;
            const float *row = kp + (j1 * NODE_BLOCK + q1) * KS;
#pragma unroll
            for (int t = 0; t < NT; ++t) b[(sidx + 1) & 1][t] = row[16 * t];
          }
#pragma unroll
          for (int t = 0; t < NT; ++t) G[t] = mfma(b[sidx & 1][t], V[j][q], G[t]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // ---- prox of G and extrapolation (theta = 1), rows 16 t + 4 g + q
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const float4 l4 = *reinterpret_cast<const float4 *>(lamp + 16 * t + 4 * g);
      const float4 x4 = *reinterpret_cast<const float4 *>(st.xfc32 + pd * np + 16 * t + 4 * g);
      const float l0[4] = {l4.x, l4.y, l4.z, l4.w}, xc[4] = {x4.x, x4.y, x4.z, x4.w};
      float ln[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float wd = (float)S.Wd[16 * t + 4 * g + q];
        ln[q] = (l0[q] - tau * (G[t][q] - xc[q])) / (1.0f + tau * wd);
        bop[t][q] = sig * (2.0f * ln[q] - l0[q]);
      }
      *reinterpret_cast<float4 *>(lamp + 16 * t + 4 * g) = make_float4(ln[0], ln[1], ln[2], ln[3]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) st.lamb[pd * np + 16 * t + 4 * g + q] = sig > 0.f ? bop[t][q] / sig : 0.f;
  if (live && g == 0) {
    st.iters_probe[p] += iters;
    st.iters_tot[p] += iters;
  }
}

// ------------------------------------------------------------------ FP64 certificate + decisions

// Certificate bookkeeping and the search step for point p (Sec. IV: the
// minimum time is the smallest horizon where phi(x, .) falls to zero): the
// certified interval [-P, -D] from the FP64 sums (sP = 1/2 lam^T W lam -
// <x_f - c, lam>, wsig = sum_k w_k sigma_C(K_k lam), sJ = (x_T - c)^T W^-1
// (x_T - c)), the sign or gap decision, then
//   PH_SCAN   certified unreachable at the scan horizon: next scan horizon
//             (t_max itself unreachable: T = +inf); certified reach: the
//             cell [previous scan horizon, this one] holds the first crossing;
//   PH_PROBE  a certified reach moves hi, unreachable moves lo; next probe:
//             a pending hint inside (lo, hi), else the hybrid Newton step
//             (slope sAx - slast) or the midpoint;
//   PH_FINAL  the solve at T = hi runs to the gap tolerance.
// Returns true when the point needs a probe setup at the new horizon st.T[p].
__device__ __forceinline__ double search_tol(const Opts &o, double t_max, double hi) {
  return fmax(o.t_rel_tol * hi, o.t_abs_frac * t_max);
}

__device__ bool decide(const SysView &S, const PtState &st, const Opts &o, long p, int np, double sP,
                       double wsig, double sJ, double sAx, double slast) {
  // primal bound: the better of the iterate and lam = 0 (P(0) = 1/2 = -min J);
  // a reduced system of copies shifts both bounds by the copies' spread
  const double spread = st.kspread ? st.kspread[p] : 0.0;
  const double Pv = fmin(sP + 0.5 + wsig, 0.5) - spread;
  const double Dv = -0.5 * (sJ - 1.0) - spread;
  st.P[p] = Pv;
  st.D[p] = Dv;
  const double gap = (Pv - Dv) / fmax(1.0, fabs(Dv));
  const int ph = st.phase[p];
  const double T = st.T[p];
  if (!isfinite(Pv) || !isfinite(Dv)) {
    st.status[p] = HOPF_PT_NONFINITE;
    st.phase[p] = PH_DONE;
    return false;
  }
  if (ph == PH_FINAL) {
    if (gap <= o.gap_tol) { st.phase[p] = PH_DONE; log_probe(st, p, np); return false; }
    if (st.iters_probe[p] >= o.max_iter) { st.status[p] = HOPF_PT_NOCONV; st.phase[p] = PH_DONE; }
    else if (o.prec == HOPF_BF16X3 && st.iters_probe[p] >= o.esc_iters) st.esc[p] = 1;   // finish in FP32
    return false;
  }
  // certified sign of phi_N(x, T); a probe placed for the Newton hybrid
  // (between table nodes, from the newton_after-th probe of the cell on) also
  // needs a value accurate to newton_rho relative
  const bool scan = ph == PH_SCAN;
  const bool tight = !scan && (st.newt[p] & 4);
  int outcome = -1;   // 1 reach, 0 unreach
  if (gap <= o.gap_tol) outcome = (-Pv > 0.0) ? 0 : 1;
  else if (tight && Pv - Dv > o.newton_rho * 0.5 * fabs(Pv + Dv)) outcome = -1;
  else if (-Dv <= 0.0) outcome = 1;
  else if (-Pv > 0.0) outcome = 0;
  if (outcome < 0) {
    if (st.iters_probe[p] >= o.max_iter) { st.status[p] = HOPF_PT_NOCONV; st.phase[p] = PH_DONE; }
    else if (o.prec == HOPF_BF16X3 && st.iters_probe[p] >= o.esc_iters) st.esc[p] = 1;   // finish in FP32
    return false;
  }
  log_probe(st, p, np);
  double lo = st.lo[p], hi = st.hi[p];
  const int K = last_node(S.N, S.quad);
  if (scan) {
    if (outcome == 0) {
      st.lo[p] = T;
      int j = st.nscan[p];
      const int kc = scan_node(K, o.scan, j);
      if (kc >= K) {                 // every scan horizon, t_max included, certified unreachable
        st.status[p] = HOPF_PT_UNREACH;
        st.phase[p] = PH_DONE;
        st.T[p] = INFINITY;
        st.hi[p] = INFINITY;
        return false;
      }
      while (scan_node(K, o.scan, j) <= kc) ++j;
      st.nscan[p] = j;
      st.T[p] = node_horizon(S.t_max, S.h, K, scan_node(K, o.scan, j));
      return true;
    }
    hi = T;                          // first certified reach: refine [lo, hi]
    st.phase[p] = PH_PROBE;
  } else {
    if (outcome == 1) hi = T; else lo = T;
    st.ncell[p] += 1;
    // a Newton probe that left the bracket wider than half its width before
    // the step forces a midpoint next (the width halves at least every two probes)
    const double wb = st.wbef[p];
    st.newt[p] = ((st.newt[p] & 1) && hi - lo > 0.5 * wb) ? 2 : 0;   // the tight bit was read above
  }
  st.lo[p] = lo;
  st.hi[p] = hi;
  if (hi - lo <= search_tol(o, S.t_max, hi)) {
    st.phase[p] = PH_FINAL;
    if (outcome == 1) {
      if (gap <= o.gap_tol) { st.phase[p] = PH_DONE; log_probe(st, p, np); }   // already certified at T = hi
    } else {
      st.T[p] = hi;
      return true;
    }
    return false;
  }
  // next probe inside the cell: a pending hint (hb, then ha) inside (lo, hi);
  // else the middle table node strictly inside (lo, hi); else the Newton
  // step of Sec. IV from this probe (when it ran tight and no midpoint is
  // forced), moved off its root estimate towards the farther end of the
  // bracket by 0.4 of the stopping tolerance plus the estimate's own
  // uncertainty; else the midpoint
  double Tn = 0.5 * (lo + hi);
  bool placed = false, newton = false, cont = true;
  while (st.stage[p] < 2) {
    const double t = st.stage[p] == 0 ? st.hb[p] : st.ha[p];
    st.stage[p] += 1;
    if (t > lo && t < hi) { Tn = t; placed = true; break; }
  }
  if (!placed) {
    bool ex_lo, ex_hi;
    const int ka = node_floor(lo, S.h, ex_lo) + 1;
    const int kh = node_floor(hi, S.h, ex_hi);
    const int kb = min(ex_hi ? kh - 1 : kh, K);
    if (ka <= kb) {                                  // bisection over the table nodes inside
      Tn = node_horizon(S.t_max, S.h, K, (ka + kb) / 2);
      cont = false;
    } else if (tight && !(st.newt[p] & 2)) {
      const double slope = sAx - slast + (st.kdspread ? st.kdspread[p] : 0.0);   // d phi / dT = -H_x(p*, x0)
      if (slope < 0.0 && isfinite(slope)) {
        const double r = T - (-0.5 * (Pv + Dv)) / slope;
        const double shift = 0.4 * search_tol(o, S.t_max, hi) + 0.5 * (Pv - Dv) / fabs(slope);
        const double tn = (hi - r > r - lo) ? r + shift : r - shift;
        if (tn > lo && tn < hi) { Tn = tn; newton = true; }
      }
    }
  }
  const bool tight_next = o.root == HOPF_ROOT_NEWTON && cont && st.ncell[p] + 1 >= o.newton_after;
  st.newt[p] = (newton ? 1 : 0) | (tight_next ? 4 : 0);
  st.wbef[p] = hi - lo;
  st.T[p] = Tn;
  return true;
}


// Per point: P(lam) from K lam, D(y^) from K^T y^ with y^ the FP64
// projection of the stored y onto w_k C (moved onto the boundary when within
// 1e-5 of it; any point of w_k C gives a valid bound).  Then the sign / gap
// decision and the bisection update (paper Sec. IV).  Same tiling as the
// iteration kernel: 16 points per workgroup, node blocks split over waves,
// operands from the FP64 copies of the two table layouts.  Two workgroups
// per CU up to NT = 7 (n_pad <= 112): the register cap spills a few values
// there but cuts the launch time by a third; wider tiles would spill hundreds.
template <int NT>
__global__ __launch_bounds__(THREADS, NT <= 7 ? 2 : 1) void k_certify(SysView S, PtState st, Opts o, int mode) {
  const int part = 2;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int tile = blockIdx.x;
  int beg, nact;
  launch_range(st, part, beg, nact);
  if (beg + tile * PTS_TILE >= nact) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int m = S.m;
  constexpr int np = 16 * NT;
  const int slot = beg + tile * PTS_TILE + cl;
  const bool live = slot < nact;
  const long p = live ? st.perm[slot] : -1;
  const long pd = live ? p : st.npts;
  const int rows_max = st.rows[st.perm[beg + tile * PTS_TILE]];
  const int nkb = (rows_max + NODE_BLOCK - 1) / NODE_BLOCK;
  double *gred = reinterpret_cast<double *>(lds_raw);            // [WAVES-1][2][4][64] + [WAVES][64]
  double *sred = gred + (WAVES - 1) * 2 * 4 * 64;

  double rr = 0.0;
  int M = -1, rowsp = 0;
  if (live) { rr = st.r[p]; M = st.M[p]; rowsp = st.rows[p]; }
  const double hw = S.h;

  float lam[NT][4];   // the iterates are FP32, so float holds them exactly (rows 4g+q)
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) lam[t][q] = st.lam[pd * np + 16 * t + 4 * g + q];
  doublex4 G[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) G[t] = doublex4{0, 0, 0, 0};
  double wsig = 0.0;    // sum_k w_k sigma_C(K_k lam) over this lane's rows
  double slast = 0.0;   // sigma_C(K_k lam) of the last table node (Newton slope)
  const int klast = (live && !st.partial[p]) ? rowsp - 1 : -1;
  const float *yp = st.y + (size_t)pd * st.ystride;

  for (int kb = wave; kb < nkb; kb += WAVES) {
    // w[q], ysc[q]: node 4g+q (FP32 y layout, operand B of K^T y^);
    // wu[q], snorm[q]: node g+4q (FP64 accumulator rows of U = K lam)
    double w[4], ysc[4], snorm[4], wu[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = kb * NODE_BLOCK + 4 * g + q;
      w[q] = (k < rowsp) ? node_weight(k, M, rr, hw, S.quad) : 0.0;
      const int ku = kb * NODE_BLOCK + acc_row<double>(g, q);
      wu[q] = (ku < rowsp) ? node_weight(ku, M, rr, hw, S.quad) : 0.0;
      snorm[q] = 0.0;
      ysc[q] = 1.0;
    }
    if (S.uset == HOPF_U_L2) {
      double s[4] = {0, 0, 0, 0};
      for (int j = 0; j < m; ++j) {
        const float4 f = *reinterpret_cast<const float4 *>(yp + ((size_t)(kb * m + j) * NODE_BLOCK + 4 * g));
        s[0] += (double)f.x * f.x; s[1] += (double)f.y * f.y; s[2] += (double)f.z * f.z; s[3] += (double)f.w * f.w;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double nv = sqrt(s[q]);
        if (w[q] <= 0.0 || nv == 0.0) ysc[q] = 0.0;
        else if (nv >= (1.0 - 1e-5) * w[q]) ysc[q] = w[q] / nv;     // on the boundary
        else ysc[q] = 1.0;
      }
    }
    const double *kd = S.K64 + ((size_t)kb * m * NODE_BLOCK + cl) * np;
    const double *kp = S.K64T + (size_t)kb * m * np * NODE_BLOCK;
    for (int j = 0; j < m; ++j) {
      // U = K_j lam  (16 nodes x 16 points), contraction over rows 16t + 4g + q
      doublex4 U{0, 0, 0, 0};
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double *a = kd + (size_t)j * NODE_BLOCK * np + 16 * t + 4 * g;
        const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
        U = mfma(a0, (double)lam[t][0], U);
        U = mfma(a1, (double)lam[t][1], U);
        U = mfma(a2, (double)lam[t][2], U);
        U = mfma(a3, (double)lam[t][3], U);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) snorm[q] += (S.uset == HOPF_U_L2) ? U[q] * U[q] : fabs(U[q]);
      // y^_j on nodes 4g+q
      double yh[4];
      {
        const float4 f = *reinterpret_cast<const float4 *>(yp + ((size_t)(kb * m + j) * NODE_BLOCK + 4 * g));
        const double yv[4] = {(double)f.x, (double)f.y, (double)f.z, (double)f.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (S.uset == HOPF_U_L2) yh[q] = yv[q] * ysc[q];
          else {
            double v = fmin(fmax(yv[q], -w[q]), w[q]);
            if (w[q] > 0.0 && fabs(v) >= (1.0 - 1e-5) * w[q]) v = copysign(w[q], v);
            yh[q] = v;
          }
        }
      }
      // G += K_j^T y^_j, A = Kp[kb][j][16 t + cl][node 4g + q]
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double *a = kp + ((size_t)j * np + 16 * t + cl) * NODE_BLOCK + 4 * g;
        const double a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
        G[t] = mfma(a0, yh[0], G[t]);
        G[t] = mfma(a1, yh[1], G[t]);
        G[t] = mfma(a2, yh[2], G[t]);
        G[t] = mfma(a3, yh[3], G[t]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double sg = (S.uset == HOPF_U_L2) ? sqrt(snorm[q]) : snorm[q];
      wsig += wu[q] * sg;
      if (kb * NODE_BLOCK + acc_row<double>(g, q) == klast) slast = sg;
    }
  }
  // sum over the waves into wave 0, CT tiles at a time (bounded LDS)
  constexpr int CT = 2;
#pragma unroll
  for (int t0 = 0; t0 < NT; t0 += CT) {
    if (wave > 0) {
#pragma unroll
      for (int tt = 0; tt < CT; ++tt)
        if (t0 + tt < NT)
#pragma unroll
          for (int q = 0; q < 4; ++q) gred[(((wave - 1) * CT + tt) * 4 + q) * 64 + lane] = G[t0 + tt < NT ? t0 + tt : 0][q];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int tt = 0; tt < CT; ++tt)
        if (t0 + tt < NT)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            for (int w2 = 0; w2 < WAVES - 1; ++w2) G[t0 + tt < NT ? t0 + tt : 0][q] += gred[((w2 * CT + tt) * 4 + q) * 64 + lane];
    }
    __syncthreads();
  }
  sred[wave * 64 + lane] = wsig;
  gred[wave * 64 + lane] = slast;    // the G reduction area is free again
  __syncthreads();
  if (wave != 0) return;
  wsig = 0.0;
  slast = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < WAVES; ++w2) { wsig += sred[w2 * 64 + lane]; slast += gred[w2 * 64 + lane]; }

  double sP = 0.0;   // 1/2 W lam^2 - (x_f - c) lam
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * t + 4 * g + q;          // lam registers: rows 4g+q
      double xf = 0.0, cc = 0.0, wd = 1.0;
      if (live && i < S.n) { xf = st.xf[p * np + i]; cc = S.c[i]; wd = S.Wd[i]; }
      const double l = lam[t][q];
      sP += 0.5 * wd * l * l - (xf - cc) * l;
      const int ig = 16 * t + acc_row<double>(g, q);   // G registers: rows g+4q
      const double xg = (live && ig < S.n) ? st.xf[p * np + ig] : 0.0;
      G[t][q] = (live && ig < S.n) ? xg - G[t][q] : 0.0;   // G now holds x_T
    }

  // private node (trapezoid, off-grid T): sigma_C(R lam) and R^T y^_R, in wave 0
  bool any_part = false;
  {
    const bool mine = live && st.partial[p];
    any_part = __any(mine);
  }
  if (any_part) {
    // scratch: lam [16][np] (float), R^T y^ [16][np], y^ [16][mp]; reuses the reduction area
    const int mp = st.mpad;
    unsigned char *base = reinterpret_cast<unsigned char *>(sred + WAVES * 64);
    float *lam_s = reinterpret_cast<float *>(base);
    double *xr_s = reinterpret_cast<double *>(base + 16 * np * 4);
    double *yr_s = xr_s + 16 * np;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) lam_s[cl * np + 16 * t + 4 * g + q] = lam[t][q];
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const int pp = lane >> 2, qq = lane & 3;
    const int pslot = beg + tile * PTS_TILE + pp;
    const bool plive = pslot < nact;
    const long P2 = plive ? st.perm[pslot] : -1;
    const bool ppart = plive && st.partial[P2];
    const double wR = ppart ? 0.5 * st.r[P2] : 0.0;
    double ssU = 0.0, ssY = 0.0;
    for (int j = qq; j < mp; j += 4) {
      double u = 0.0, yv = 0.0;
      if (ppart && j < m) {
        const double *row = st.R64 + ((size_t)P2 * m + j) * np;
        for (int i = 0; i < np; ++i) u += row[i] * (double)lam_s[pp * np + i];
        yv = st.yR[(size_t)P2 * mp + j];
      }
      ssU += (S.uset == HOPF_U_L2) ? u * u : fabs(u);
      ssY += yv * yv;
      yr_s[pp * mp + j] = yv;
    }
    ssU += __shfl_xor(ssU, 1); ssU += __shfl_xor(ssU, 2);
    ssY += __shfl_xor(ssY, 1); ssY += __shfl_xor(ssY, 2);
    double scY = 1.0;
    if (S.uset == HOPF_U_L2) {
      const double nv = sqrt(ssY);
      if (wR <= 0.0 || nv == 0.0) scY = 0.0;
      else if (nv >= (1.0 - 1e-5) * wR) scY = wR / nv;
    }
    for (int j = qq; j < mp; j += 4) {
      double v = yr_s[pp * mp + j];
      if (S.uset == HOPF_U_L2) v *= scY;
      else {
        v = fmin(fmax(v, -wR), wR);
        if (wR > 0.0 && fabs(v) >= (1.0 - 1e-5) * wR) v = copysign(wR, v);
      }
      yr_s[pp * mp + j] = v;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    for (int i = qq; i < np; i += 4) {
      double acc = 0.0;
      if (ppart)
        for (int j = 0; j < m; ++j) acc += st.R64[((size_t)P2 * m + j) * np + i] * yr_s[pp * mp + j];
      xr_s[pp * np + i] = acc;
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    // the private node's term w_R sigma_C(R lam), moved to the lane holding column pp with g = 0
    const double part_sig = wR * ((S.uset == HOPF_U_L2) ? sqrt(ssU) : ssU);
    const double ps = __shfl(part_sig, 4 * cl);
    if (g == 0) wsig += ps;
    const double sR = __shfl((S.uset == HOPF_U_L2) ? sqrt(ssU) : ssU, 4 * cl);
    if (g == 0 && live && st.partial[p]) slast = sR;     // the node at tau = T is the last one
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ig = 16 * t + acc_row<double>(g, q);
        G[t][q] -= (live && ig < S.n) ? xr_s[cl * np + ig] : 0.0;
      }
  }

  // J(x_T) partial sums (G registers: rows g + 4q)
  double sJ = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * t + acc_row<double>(g, q);
      if (live && i < S.n) {
        const double d = G[t][q] - S.c[i];
        sJ += d * d / S.Wd[i];
      }
    }
  // <A x_f, lam> (lam registers: rows 4g+q)
  double sAx = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * t + 4 * g + q;
      if (live && i < S.n) sAx += st.axf[p * np + i] * (double)lam[t][q];
    }
  // reduce over the four lane groups holding the same point
  sAx += __shfl_xor(sAx, 16); sAx += __shfl_xor(sAx, 32);
  slast += __shfl_xor(slast, 16); slast += __shfl_xor(slast, 32);
  sP += __shfl_xor(sP, 16); sP += __shfl_xor(sP, 32);
  sJ += __shfl_xor(sJ, 16); sJ += __shfl_xor(sJ, 32);
  wsig += __shfl_xor(wsig, 16); wsig += __shfl_xor(wsig, 32);
  if (!live || g != 0) return;

  if (decide(S, st, o, p, np, sP, wsig, sJ, sAx, slast)) mark_setup(st, p);
}


// ------------------------------------------------------------------ streaming variant (any m, large n, BF16 hi+lo)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ floatx4 mfma_bf16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// hi = bf16(v), lo = bf16(v - hi): v ~ hi + lo to about 2^-17 relative
__device__ __forceinline__ void split_bf16(float v, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// Components are processed a pair at a time, so registers do not grow with
// m: for the box the pair is projected right after its dual GEMM; for the l2
// ball a first pass stores the unprojected V and accumulates the node norms,
// a second pass scales, stores and runs the primal GEMM.  Wave 0 owns lam
// (in L2) and broadcasts sigma*lam_bar through LDS.  With BF: K is held as a
// hi + lo pair of bf16 tables, operands are split the same way on the fly,
// and each product takes three bf16 MFMAs (hi*hi + hi*lo + lo*hi) with FP32
// accumulation; the contraction chunk of 32 is (tiles t, t+1) for the dual
// GEMM and (components j, j+1) x 16 nodes for the primal GEMM.
template <int NT, bool BF>
__global__ __launch_bounds__(THREADS, 1) void k_pdhg_stream(SysView S, PtState st, int iters, int part) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int TCH = 4;                                             // tiles per reduction chunk
  float *gred = reinterpret_cast<float *>(lds_raw);                  // [WAVES-1][TCH][4][64]
  float *bopb = gred + (WAVES - 1) * TCH * 4 * 64;                   // [NT][4][64]
  float *pscr = bopb + NT * 4 * 64;                                  // private-node scratch
  const int tile = blockIdx.x;
  int beg, nact;
  launch_range(st, part, beg, nact);
  if (beg + tile * PTS_TILE >= nact) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int m = S.m;
  constexpr int np = 16 * NT;
  const int slot = beg + tile * PTS_TILE + cl;
  const bool live = slot < nact;
  const long p = live ? st.perm[slot] : -1;
  const long pd = live ? p : st.npts;
  const int rows_max = st.rows[st.perm[beg + tile * PTS_TILE]];
  const int nkb = (rows_max + NODE_BLOCK - 1) / NODE_BLOCK;
  __shared__ int any_part;
  if (threadIdx.x == 0) any_part = 0;
  __syncthreads();
  if (wave == 0 && g == 0 && live && st.partial[p]) atomicOr(&any_part, 1);
  __syncthreads();
  const bool wg_part = any_part != 0;

  float tau = 0.f, sig = 0.f, rr = 0.f;
  int M = -1, rowsp = 0;
  if (live) {
    tau = (float)st.tau[p];
    sig = (float)st.sig[p];
    rr = (float)st.r[p];
    M = st.M[p];
    rowsp = st.rows[p];
  }
  const float hw = (float)S.h;
  float bop[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) bop[t][q] = sig * st.lamb[pd * np + 16 * t + 4 * g + q];
  float *yp = st.y + (size_t)pd * st.ystride;
  float *lamp = st.lam + pd * np;

  for (int it = 0; it < iters; ++it) {
    floatx4 G[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) G[t] = floatx4{0, 0, 0, 0};

    // ---- private node (trapezoid, T off the grid): wave 0, FP32
    if (wg_part) {
      float *lb_s = pscr, *gr_s = pscr + 16 * np, *yr_s = pscr + 32 * np;   // yr_s [16][mpad]
      const int mp = st.mpad;
      if (wave == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) lb_s[cl * np + 16 * t + 4 * g + q] = (sig > 0 ? bop[t][q] / sig : 0.f);
      }
      __syncthreads();
      if (wave == 0) {
        const int pp = lane >> 2, qq = lane & 3;
        const int pslot = beg + tile * PTS_TILE + pp;
        const long P2 = pslot < nact ? st.perm[pslot] : -1;
        const bool ppart = P2 >= 0 && st.partial[P2];
        const float sig2 = ppart ? (float)st.sig[P2] : 0.f;
        const float wR = ppart ? (float)(0.5 * st.r[P2]) : 0.f;
        float ssq = 0.f;
        for (int j = qq; j < mp; j += 4) {
          float v = 0.f;
          if (ppart && j < m) {
            const float *row = st.R32 + ((size_t)P2 * m + j) * np;
            float acc = 0.f;
            for (int i = 0; i < np; ++i) acc += row[i] * lb_s[pp * np + i];
            v = st.yR[(size_t)P2 * mp + j] + sig2 * acc;
          }
          yr_s[pp * mp + j] = v;
          ssq += v * v;
        }
        if (S.uset == HOPF_U_L2) {
          ssq += __shfl_xor(ssq, 1);
          ssq += __shfl_xor(ssq, 2);
        }
        const float nv = sqrtf(ssq);
        const float sc = (nv > wR) ? (nv > 0 ? wR / nv : 0.f) : 1.f;
        for (int j = qq; j < mp; j += 4) {
          float v = yr_s[pp * mp + j];
          v = (S.uset == HOPF_U_L2) ? v * sc : fminf(fmaxf(v, -wR), wR);
          yr_s[pp * mp + j] = v;
          if (ppart && j < m) st.yR[(size_t)P2 * mp + j] = v;
        }
      }
      __syncthreads();
      if (wave == 0) {
        const int pp = lane >> 2, qq = lane & 3;
        const int pslot = beg + tile * PTS_TILE + pp;
        const long P2 = pslot < nact ? st.perm[pslot] : -1;
        const bool ppart = P2 >= 0 && st.partial[P2];
        for (int i = qq; i < np; i += 4) {
          float acc = 0.f;
          if (ppart)
            for (int j = 0; j < m; ++j) acc += st.R32[((size_t)P2 * m + j) * np + i] * yr_s[pp * mp + j];
          gr_s[pp * np + i] = acc;
        }
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) G[t][q] = gr_s[cl * np + 16 * t + 4 * g + q];
      }
    }

    // B operand of the dual GEMM, split once per iteration
    bf16x8 bdh[(NT + 1) / 2], bdl[(NT + 1) / 2];
    if constexpr (BF) {
#pragma unroll
      for (int c = 0; c < (NT + 1) / 2; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int t = 2 * c + (e >> 2);
          const float v = (t < NT) ? bop[t < NT ? t : 0][e & 3] : 0.f;
          __bf16 hi, lo;
          split_bf16(v, hi, lo);
          bdh[c][e] = hi;
          bdl[c][e] = lo;
        }
    }

    for (int kb = wave; kb < nkb; kb += WAVES) {
      float w4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kb * NODE_BLOCK + 4 * g + q;
        w4[q] = (k < rowsp) ? (float)node_weight(k, M, (double)rr, (double)hw, S.quad) : 0.f;
      }
      const bool l2 = S.uset == HOPF_U_L2;
      float s4[4] = {0.f, 0.f, 0.f, 0.f};
      for (int pass = 0; pass < (l2 ? 2 : 1); ++pass) {
        float sc4[4];
        if (l2 && pass == 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float nv = sqrtf(s4[q]);
            sc4[q] = (nv > w4[q]) ? (nv > 0 ? w4[q] / nv : 0.f) : 1.f;
          }
        }
        for (int j = 0; j < m; j += 2) {
          const bool has2 = j + 1 < m;
          floatx4 V[2];
          // y (node-major within the block)
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            V[u] = floatx4{0, 0, 0, 0};
            if (u == 0 || has2) {
              const float4 f = *reinterpret_cast<const float4 *>(yp + (size_t)(kb * m + j + u) * NODE_BLOCK + 4 * g);
              V[u] = floatx4{f.x, f.y, f.z, f.w};
            }
          }
          if (!l2 || pass == 0) {
            // dual GEMM for components j, j+1
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              if (u == 1 && !has2) break;
              if constexpr (BF) {
                const __bf16 *kh = S.Kd16h + (((size_t)kb * m + j + u) * NODE_BLOCK + cl) * np;
                const __bf16 *kl = S.Kd16l + (((size_t)kb * m + j + u) * NODE_BLOCK + cl) * np;
#pragma unroll
                for (int c = 0; c < (NT + 1) / 2; ++c) {
                  bf16x8 ah, al;
#pragma unroll
                  for (int e = 0; e < 8; ++e) {
                    const int t = 2 * c + (e >> 2);
                    const int col = 16 * (t < NT ? t : 0) + 4 * g + (e & 3);
                    ah[e] = (t < NT) ? kh[col] : (__bf16)0.0f;
                    al[e] = (t < NT) ? kl[col] : (__bf16)0.0f;
                  }
                  V[u] = mfma_bf16(ah, bdh[c], V[u]);
                  V[u] = mfma_bf16(ah, bdl[c], V[u]);
                  V[u] = mfma_bf16(al, bdh[c], V[u]);
                }
              } else {
                const float *kd = S.K32 + (((size_t)kb * m + j + u) * NODE_BLOCK + cl) * np;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                  const float4 f = *reinterpret_cast<const float4 *>(kd + 16 * t + 4 * g);
                  V[u] = mfma(f.x, bop[t][0], V[u]);
                  V[u] = mfma(f.y, bop[t][1], V[u]);
                  V[u] = mfma(f.z, bop[t][2], V[u]);
                  V[u] = mfma(f.w, bop[t][3], V[u]);
                }
              }
            }
          }
          if (l2 && pass == 0) {       // store unprojected, accumulate node norms
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              if (u == 1 && !has2) break;
#pragma unroll
              for (int q = 0; q < 4; ++q) s4[q] += V[u][q] * V[u][q];
              float4 f;
              f.x = V[u][0]; f.y = V[u][1]; f.z = V[u][2]; f.w = V[u][3];
              *reinterpret_cast<float4 *>(yp + (size_t)(kb * m + j + u) * NODE_BLOCK + 4 * g) = f;
            }
            continue;
          }
          // project, store, primal GEMM
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (u == 1 && !has2) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) V[u][q] = l2 ? V[u][q] * sc4[q] : fminf(fmaxf(V[u][q], -w4[q]), w4[q]);
            float4 f;
            f.x = V[u][0]; f.y = V[u][1]; f.z = V[u][2]; f.w = V[u][3];
            *reinterpret_cast<float4 *>(yp + (size_t)(kb * m + j + u) * NODE_BLOCK + 4 * g) = f;
          }
          if constexpr (BF) {
            bf16x8 byh, byl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              __bf16 hi, lo;
              split_bf16((e < 4 || has2) ? V[e >> 2][e & 3] : 0.f, hi, lo);
              byh[e] = hi;
              byl[e] = lo;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              bf16x8 ah, al;
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                const int u = e >> 2;
                const bool okc = u == 0 || has2;
                const size_t off = (((size_t)kb * m + j + (okc ? u : 0)) * np + 16 * t + cl) * NODE_BLOCK + 4 * g + (e & 3);
                ah[e] = okc ? S.Kp16h[off] : (__bf16)0.0f;
                al[e] = okc ? S.Kp16l[off] : (__bf16)0.0f;
              }
              G[t] = mfma_bf16(ah, byh, G[t]);
              G[t] = mfma_bf16(ah, byl, G[t]);
              G[t] = mfma_bf16(al, byh, G[t]);
            }
          } else {
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              if (u == 1 && !has2) break;
              const float *kp = S.K32T + ((size_t)kb * m + j + u) * np * NODE_BLOCK;
#pragma unroll
              for (int t = 0; t < NT; ++t) {
                const float4 f = *reinterpret_cast<const float4 *>(kp + (size_t)(16 * t + cl) * NODE_BLOCK + 4 * g);
                G[t] = mfma(f.x, V[u][0], G[t]);
                G[t] = mfma(f.y, V[u][1], G[t]);
                G[t] = mfma(f.z, V[u][2], G[t]);
                G[t] = mfma(f.w, V[u][3], G[t]);
              }
            }
          }
        }
      }
    }

    // ---- sum G over the waves into wave 0, in chunks of TCH tiles
#pragma unroll
    for (int t0 = 0; t0 < NT; t0 += TCH) {
      if (wave > 0) {
#pragma unroll
        for (int tt = 0; tt < TCH; ++tt)
          if (t0 + tt < NT)
#pragma unroll
            for (int q = 0; q < 4; ++q) gred[(((wave - 1) * TCH + tt) * 4 + q) * 64 + lane] = G[t0 + tt < NT ? t0 + tt : 0][q];
      }
      __syncthreads();
      if (wave == 0) {
#pragma unroll
        for (int tt = 0; tt < TCH; ++tt)
          if (t0 + tt < NT)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              for (int w2 = 0; w2 < WAVES - 1; ++w2) G[t0 + tt < NT ? t0 + tt : 0][q] += gred[((w2 * TCH + tt) * 4 + q) * 64 + lane];
      }
      __syncthreads();
    }
    // ---- prox and extrapolation in wave 0, broadcast of sigma * lam_bar
    if (wave == 0) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * t + 4 * g + q;
          const float xfc = st.xfc32[pd * np + i];
          const float wd = (float)S.Wd[i];
          const float l0 = lamp[i];
          const float ln = (l0 - tau * (G[t][q] - xfc)) / (1.0f + tau * wd);
          lamp[i] = ln;
          bopb[(t * 4 + q) * 64 + lane] = sig * (2.0f * ln - l0);
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) bop[t][q] = bopb[(t * 4 + q) * 64 + lane];
  }
  if (wave == 0) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) st.lamb[pd * np + 16 * t + 4 * g + q] = sig > 0 ? bop[t][q] / sig : 0.f;
    if (live && g == 0) {
      st.iters_probe[p] += iters;
      st.iters_tot[p] += iters;
    }
  }
}

// ------------------------------------------------------------------ 64-point streaming variant (any m, BF16 hi+lo)

// The streaming iteration for a workgroup of 64 points (wave w owns points
// 16 w .. 16 w + 15 and runs every node block for them, as in k_pdhg_wide):
// for each node block and component pair (j, j+1) the table rows are copied
// once into LDS and read by all four waves.  FP32: one copy in the dual
// layout, rows (component, node) of n_pad floats at stride n_pad + 4 (dual
// operand: one 16-byte read per column group; primal operand: 4-byte reads
// at node 4 g + q).  BF16 hi+lo: the dual-layout hi and lo rows at stride
// n_pad + 4 bf16 (an odd multiple of 8 bytes: the 16 rows of an 8-byte read
// fall in distinct banks) and the primal-layout hi and lo copies
// [component][n_pad][16 nodes] (two 8-byte reads give a lane its 8 values of
// the 16x16x32 operand).  The extra node is applied per point in registers.
__host__ __device__ constexpr int swide_bf_stride(int NT) { return 16 * NT + 4; }
__host__ __device__ inline size_t swide_lds_bytes(int NT, bool bf) {
  return bf ? (size_t)2 * (2 * 16 * swide_bf_stride(NT)) * 2 + (size_t)2 * (2 * 16 * NT * 16) * 2
            : (size_t)2 * 16 * wide_row_stride(NT) * 4;
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <int NT, bool BF>
__global__ __launch_bounds__(THREADS, NT <= 12 ? 2 : 1) void k_pdhg_swide(SysView S, PtState st, int iters, int part) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int np = 16 * NT;
  constexpr int KS = wide_row_stride(NT);
  constexpr int KB = swide_bf_stride(NT);
  float *ks = reinterpret_cast<float *>(lds_raw);                 // FP32: [2][16][KS]
  __bf16 *kdh = reinterpret_cast<__bf16 *>(lds_raw);             // BF16: [2][16][KB] hi, lo
  __bf16 *kdl = kdh + 2 * 16 * KB;
  __bf16 *kph = kdl + 2 * 16 * KB;                                // [2][np][16] hi, lo
  __bf16 *kpl = kph + 2 * np * 16;
  int beg, nact;
  launch_range(st, part, beg, nact);
  const int wg0 = beg + blockIdx.x * WIDE_PTS;
  if (wg0 >= nact) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int m = S.m;
  const int slot = wg0 + wave * PTS_WAVE + cl;
  const bool live = slot < nact;
  const long p = live ? st.perm[slot] : -1;
  const long pd = live ? p : st.npts;
  const int rows_max = st.rows[st.perm[wg0]];     // slots are sorted by rows, descending
  const int nkb = (rows_max + NODE_BLOCK - 1) / NODE_BLOCK;

  float tau = 0.f, sig = 0.f, rr = 0.f;
  int M = -1, rowsp = 0;
  bool ppart = false;
  if (live) {
    tau = (float)st.tau[p];
    sig = (float)st.sig[p];
    rr = (float)st.r[p];
    M = st.M[p];
    rowsp = st.rows[p];
    ppart = st.partial[p] != 0;
  }
  const bool wave_part = __any(ppart);
  const float wR = ppart ? 0.5f * rr : 0.f;
  const float hw = (float)S.h;
  const bool l2 = S.uset == HOPF_U_L2;
  float bop[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) bop[t][q] = sig * st.lamb[pd * np + 16 * t + 4 * g + q];
  float *lamp = st.lam + pd * np;
  float *yp = st.y + (size_t)pd * st.ystride;
  const float *Rp = ppart ? st.R32 + (size_t)p * m * np : nullptr;

  for (int it = 0; it < iters; ++it) {
    floatx4 G[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) G[t] = floatx4{0, 0, 0, 0};

    // ---- extra node at tau = T, in registers (see k_pdhg_wide)
    if (wave_part) {
      float ssq = 0.f;
      float *yRp = ppart ? st.yR + (size_t)p * st.mpad : nullptr;
#pragma unroll 1
      for (int j = 0; j < m; ++j) {
        float4 rv[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          rv[t] = ppart ? *reinterpret_cast<const float4 *>(Rp + (size_t)j * np + 16 * t + 4 * g)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc += rv[t].x * bop[t][0] + rv[t].y * bop[t][1] + rv[t].z * bop[t][2] + rv[t].w * bop[t][3];
        acc += __shfl_xor(acc, 16);
        acc += __shfl_xor(acc, 32);
        float v = ppart ? yRp[j] + acc : 0.f;
        if (!l2) v = fminf(fmaxf(v, -wR), wR);
        ssq += v * v;
        if (ppart && g == 0) yRp[j] = v;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          G[t][0] += rv[t].x * v;
          G[t][1] += rv[t].y * v;
          G[t][2] += rv[t].z * v;
          G[t][3] += rv[t].w * v;
        }
      }
      if (l2) {
        const float nv = sqrtf(ssq);
        const float sc = (nv > wR) ? (nv > 0.f ? wR / nv : 0.f) : 1.f;
        if (ppart && g == 0)
          for (int j = 0; j < m; ++j) yRp[j] *= sc;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) G[t][q] *= sc;
      }
    }

    // B operand of the dual GEMM as hi + lo, split once per iteration
    bf16x8 bdh[(NT + 1) / 2], bdl[(NT + 1) / 2];
    if constexpr (BF) {
#pragma unroll
      for (int c = 0; c < (NT + 1) / 2; ++c)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int t = 2 * c + (e >> 2);
          const float v = (t < NT) ? bop[t < NT ? t : 0][e & 3] : 0.f;
          __bf16 hi, lo;
          split_bf16(v, hi, lo);
          bdh[c][e] = hi;
          bdl[c][e] = lo;
        }
    }

    // staging of the rows of one (node block, pass, component pair) through
    // registers: PF / PD / PP chunks per thread
    const int npass = l2 ? 2 : 1;
    struct Stage { int kb, pass, j; };
    constexpr int FCH = 2 * 16 * (np / 4);              // FP32 float4 chunks
    constexpr int DCH = 2 * 16 * (np / 4);              // BF16 dual 8-byte chunks (per table)
    constexpr int PCH = 2 * np * NODE_BLOCK / 8;        // BF16 primal 16-byte chunks (per table)
    constexpr int PF = BF ? 1 : (FCH + THREADS - 1) / THREADS;
    constexpr int PD = BF ? (DCH + THREADS - 1) / THREADS : 1;
    constexpr int PP = BF ? (PCH + THREADS - 1) / THREADS : 1;
    float4 rf[PF];
    uint2 rdh[PD], rdl[PD];
    uint4 rph[PP], rpl[PP];
    auto stage_load = [&](const Stage &q) {
      const bool h2 = q.j + 1 < m;
      if constexpr (BF) {
        if (!l2 || q.pass == 0) {
          const uint2 *sh = reinterpret_cast<const uint2 *>(S.Kd16h + ((size_t)q.kb * m + q.j) * NODE_BLOCK * np);
          const uint2 *sl = reinterpret_cast<const uint2 *>(S.Kd16l + ((size_t)q.kb * m + q.j) * NODE_BLOCK * np);
#pragma unroll
          for (int r = 0; r < PD; ++r) {
            const int e = threadIdx.x + r * THREADS;
            const bool ok = e < DCH && (e < DCH / 2 || h2);
            rdh[r] = ok ? sh[e] : make_uint2(0u, 0u);
            rdl[r] = ok ? sl[e] : make_uint2(0u, 0u);
          }
        }
        if (!l2 || q.pass == 1) {
          const uint4 *sh = reinterpret_cast<const uint4 *>(S.Kp16h + ((size_t)q.kb * m + q.j) * np * NODE_BLOCK);
          const uint4 *sl = reinterpret_cast<const uint4 *>(S.Kp16l + ((size_t)q.kb * m + q.j) * np * NODE_BLOCK);
#pragma unroll
          for (int r = 0; r < PP; ++r) {
            const int e = threadIdx.x + r * THREADS;
            const bool ok = e < PCH && (e < PCH / 2 || h2);
            rph[r] = ok ? sh[e] : make_uint4(0u, 0u, 0u, 0u);
            rpl[r] = ok ? sl[e] : make_uint4(0u, 0u, 0u, 0u);
          }
        }
      } else {
        const float4 *src = reinterpret_cast<const float4 *>(S.K32 + ((size_t)q.kb * m + q.j) * NODE_BLOCK * np);
#pragma unroll
        for (int r = 0; r < PF; ++r) {
          const int e = threadIdx.x + r * THREADS;
          const bool ok = e < FCH && (e < FCH / 2 || h2);
          rf[r] = ok ? src[e] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      }
    };
    auto stage_store = [&](const Stage &q) {
      if constexpr (BF) {
        if (!l2 || q.pass == 0) {
          constexpr int C2 = np / 4;
#pragma unroll
          for (int r = 0; r < PD; ++r) {
            const int e = threadIdx.x + r * THREADS;
            if (e < DCH) {
              const int row = e / C2, c2 = e - row * C2;
              *reinterpret_cast<uint2 *>(kdh + row * KB + 4 * c2) = rdh[r];
              *reinterpret_cast<uint2 *>(kdl + row * KB + 4 * c2) = rdl[r];
            }
          }
        }
        if (!l2 || q.pass == 1) {
#pragma unroll
          for (int r = 0; r < PP; ++r) {
            const int e = threadIdx.x + r * THREADS;
            if (e < PCH) {
              reinterpret_cast<uint4 *>(kph)[e] = rph[r];
              reinterpret_cast<uint4 *>(kpl)[e] = rpl[r];
            }
          }
        }
      } else {
        constexpr int C4 = np / 4;
#pragma unroll
        for (int r = 0; r < PF; ++r) {
          const int e = threadIdx.x + r * THREADS;
          if (e < FCH) {
            const int row = e / C4, c4 = e - row * C4;
            *reinterpret_cast<float4 *>(ks + row * KS + 4 * c4) = rf[r];
          }
        }
      }
    };
    Stage cur{0, 0, 0};
    if (nkb > 0) stage_load(cur);

    for (int kb = 0; kb < nkb; ++kb) {
      float w4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = kb * NODE_BLOCK + 4 * g + q;
        w4[q] = (k < rowsp) ? (float)node_weight(k, M, (double)rr, (double)hw, S.quad) : 0.f;
      }
      float s4[4] = {0.f, 0.f, 0.f, 0.f};
      for (int pass = 0; pass < (l2 ? 2 : 1); ++pass) {
        const bool dual = !l2 || pass == 0, primal = !l2 || pass == 1;
        float sc4[4] = {1.f, 1.f, 1.f, 1.f};
        if (l2 && pass == 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float nv = sqrtf(s4[q]);
            sc4[q] = (nv > w4[q]) ? (nv > 0 ? w4[q] / nv : 0.f) : 1.f;
          }
        }
        for (int j = 0; j < m; j += 2) {
          const bool has2 = j + 1 < m;
          // ---- the prefetched rows of components j, j+1 into LDS, then the
          // next pair's rows from memory into registers (in flight during
          // this pair's matrix-core work)
          __syncthreads();                     // every wave is done with the previous pair
          stage_store(cur);
          __syncthreads();
          {
            int nkb2 = kb, np2 = pass, nj = j + 2;
            if (nj >= m) { nj = 0; if (++np2 >= npass) { np2 = 0; ++nkb2; } }
            cur = Stage{nkb2, np2, nj};
            if (nkb2 < nkb) stage_load(cur);
          }
          // ---- y of the pair (node-major within the block)
          floatx4 V[2];
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            V[u] = floatx4{0, 0, 0, 0};
            if (u == 0 || has2) {
              const float4 f = *reinterpret_cast<const float4 *>(yp + (size_t)(kb * m + j + u) * NODE_BLOCK + 4 * g);
              V[u] = floatx4{f.x, f.y, f.z, f.w};
            }
          }
          if (dual) {
            // ---- dual GEMM V_u += K_{j+u} (sigma lam_bar)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              if constexpr (BF) {
                const __bf16 *rh = kdh + (u * 16 + cl) * KB + 4 * g;
                const __bf16 *rl = kdl + (u * 16 + cl) * KB + 4 * g;
#pragma unroll
                for (int c = 0; c < (NT + 1) / 2; ++c) {
                  const bf16x4 h0 = *reinterpret_cast<const bf16x4 *>(rh + 32 * c);
                  const bf16x4 l0 = *reinterpret_cast<const bf16x4 *>(rl + 32 * c);
                  bf16x4 h1 = {}, l1 = {};
                  if (2 * c + 1 < NT) {
                    h1 = *reinterpret_cast<const bf16x4 *>(rh + 32 * c + 16);
                    l1 = *reinterpret_cast<const bf16x4 *>(rl + 32 * c + 16);
                  }
                  const bf16x8 ah = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
                  const bf16x8 al = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
                  V[u] = mfma_bf16(ah, bdh[c], V[u]);
                  V[u] = mfma_bf16(ah, bdl[c], V[u]);
                  V[u] = mfma_bf16(al, bdh[c], V[u]);
                }
              } else {
                const float *kd = ks + (u * 16 + cl) * KS + 4 * g;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                  const float4 f = *reinterpret_cast<const float4 *>(kd + 16 * t);
                  V[u] = mfma(f.x, bop[t][0], V[u]);
                  V[u] = mfma(f.y, bop[t][1], V[u]);
                  V[u] = mfma(f.z, bop[t][2], V[u]);
                  V[u] = mfma(f.w, bop[t][3], V[u]);
                }
              }
            }
          }
          if (l2 && pass == 0) {       // store unprojected, accumulate node norms
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              if (u == 1 && !has2) break;
#pragma unroll
              for (int q = 0; q < 4; ++q) s4[q] += V[u][q] * V[u][q];
              *reinterpret_cast<float4 *>(yp + (size_t)(kb * m + j + u) * NODE_BLOCK + 4 * g) =
                  make_float4(V[u][0], V[u][1], V[u][2], V[u][3]);
            }
            continue;
          }
          // ---- project, store, primal GEMM G_t += K_{j+u}^T V_u
#pragma unroll
          for (int u = 0; u < 2; ++u) {
#pragma unroll
            for (int q = 0; q < 4; ++q) V[u][q] = l2 ? V[u][q] * sc4[q] : fminf(fmaxf(V[u][q], -w4[q]), w4[q]);
            if (u == 0 || has2)
              *reinterpret_cast<float4 *>(yp + (size_t)(kb * m + j + u) * NODE_BLOCK + 4 * g) =
                  make_float4(V[u][0], V[u][1], V[u][2], V[u][3]);
          }
          if constexpr (BF) {
            bf16x8 byh, byl;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              __bf16 hi, lo;
              split_bf16(V[e >> 2][e & 3], hi, lo);
              byh[e] = hi;
              byl[e] = lo;
            }
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const int o = (16 * t + cl) * NODE_BLOCK + 4 * g;
              const bf16x4 h0 = *reinterpret_cast<const bf16x4 *>(kph + o);
              const bf16x4 h1 = *reinterpret_cast<const bf16x4 *>(kph + np * NODE_BLOCK + o);
              const bf16x4 l0 = *reinterpret_cast<const bf16x4 *>(kpl + o);
              const bf16x4 l1 = *reinterpret_cast<const bf16x4 *>(kpl + np * NODE_BLOCK + o);
              const bf16x8 ah = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
              const bf16x8 al = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
              G[t] = mfma_bf16(ah, byh, G[t]);
              G[t] = mfma_bf16(ah, byl, G[t]);
              G[t] = mfma_bf16(al, byh, G[t]);
            }
          } else {
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const float *row = ks + (u * 16 + 4 * g + q) * KS + cl;
#pragma unroll
                for (int t = 0; t < NT; ++t) G[t] = mfma(row[16 * t], V[u][q], G[t]);
              }
          }
        }
      }
    }
    // ---- prox of G and extrapolation (theta = 1), rows 16 t + 4 g + q
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const float4 l4 = *reinterpret_cast<const float4 *>(lamp + 16 * t + 4 * g);
      const float4 x4 = *reinterpret_cast<const float4 *>(st.xfc32 + pd * np + 16 * t + 4 * g);
      const float l0[4] = {l4.x, l4.y, l4.z, l4.w}, xc[4] = {x4.x, x4.y, x4.z, x4.w};
      float ln[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float wd = (float)S.Wd[16 * t + 4 * g + q];
        ln[q] = (l0[q] - tau * (G[t][q] - xc[q])) / (1.0f + tau * wd);
        bop[t][q] = sig * (2.0f * ln[q] - l0[q]);
      }
      *reinterpret_cast<float4 *>(lamp + 16 * t + 4 * g) = make_float4(ln[0], ln[1], ln[2], ln[3]);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) st.lamb[pd * np + 16 * t + 4 * g + q] = sig > 0.f ? bop[t][q] / sig : 0.f;
  if (live && g == 0) {
    st.iters_probe[p] += iters;
    st.iters_tot[p] += iters;
  }
}

typedef void (*pdhg_fn)(SysView, PtState, int, int);
typedef void (*cert_fn)(SysView, PtState, Opts, int);

// kernel instances, one lookup per NT (hopf_inst_nt*.hip); nullptr if absent
pdhg_fn pdhg_lookup(int NT, int m, int prec, int waves, int *MM_out);
pdhg_fn wide_lookup(int NT, int m);
cert_fn cert_lookup(int NT);
pdhg_fn stream_lookup(int NT, int bf16);
pdhg_fn swide_lookup(int NT, int bf16);

}  // namespace hopf
