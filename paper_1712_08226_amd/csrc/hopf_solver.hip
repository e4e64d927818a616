// Device solver: batched primal-dual (Chambolle-Pock) solves of the
// quadrature form of the generalized Hopf formula (paper Sec. III-A,
// eqs. (15)-(23)), certified in FP64, inside a per-point bisection on the
// horizon (Sec. IV), on gfx950.
//
// Notation (terminal-costate form, lam = e^{-T A^T} p):
//   K_k   = -Qu^T B^T e^{tau_k A^T}         m x n node block, tau_k = k h
//   x_f   = e^{T A} x0                       free terminal state
//   P(lam) = 1/2 lam^T W lam - <x_f - c, lam> + 1/2 + sum_k w_k sigma_C(K_k lam)
//   D(y)   = -J(x_f - sum_k K_k^T y_k),  y_k in w_k C
// with C the unit l2 ball or box and sigma_C its support function.
//
// Work decomposition.  Points are the GEMM column dimension: a workgroup
// holds 64 points (4 waves x 16), all points of one system.  Every point
// uses a prefix of the shared node table (rows 0..rows-1) plus, for the
// trapezoid rule at a horizon off the grid, one private node at tau = T
// ("partial" node, kept per point).  Per iteration and 16-node block:
//   V_j  = Y_j + K_j (sigma lam_bar)          MFMA 16x16x4, Y as accumulator
//   Y_j  = proj_{w C}(V_j)                     in registers (all j of a node)
//   G   += K_j^T Y_j                           MFMA, Y in registers as operand B
// then lam+ = (lam - tau (G - (x_f - c))) / (1 + tau W),
// lam_bar = 2 lam+ - lam (theta = 1).  y lives in HBM in the MFMA
// accumulator order, so every load/store is a 16-byte per-lane access.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hopf_device.h"

namespace hopf {

// ------------------------------------------------------------------ init

// x0[p] = row idx[p] (or p) of the caller's x, whose rows are xs doubles
// apart; for a rotated system x0 = U^T x (the solver's coordinates)
__global__ void k_pack(const double *__restrict__ x, double *__restrict__ x0, long npts, int n, int n_pad,
                       int xs, const int *__restrict__ idx, const double *__restrict__ U) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts * n_pad) return;
  long p = i / n_pad;
  int k = (int)(i % n_pad);
  const long q = idx ? idx[p] : p;
  if (k >= n) { x0[i] = 0.0; return; }
  if (!U) { x0[i] = x[q * xs + k]; return; }
  double acc = 0.0;
  for (int j = 0; j < n; ++j) acc += U[(size_t)j * n + k] * x[q * xs + j];
  x0[i] = acc;
}

// counters and flop accounting of a job start at zero (a kernel, not a
// memset, so that the sequence needs no runtime memset nodes)
__global__ void k_clear(PtState st) {
  if (threadIdx.x < 4) st.counters[threadIdx.x] = 0;
  if (threadIdx.x < 3) st.rowsum[threadIdx.x] = 0.0;
}

// t_in: value-mode horizons; lam0 (rows of stride ls) and tb (pairs a, b):
// the caller's starting costate of the first probe and probe hints
// (min-time mode, either may be null)
__global__ void k_init(SysView S, PtState st, Opts o, int mode, const double *__restrict__ t_in,
                       const int *__restrict__ idx, const double *__restrict__ lam0,
                       const double *__restrict__ tb, int ls) {
  long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= st.npts) return;
  const double *x = st.x0 + p * S.n_pad;
  bool finite = true;
  double Jx = 0.0;
  for (int i = 0; i < S.n; ++i) {
    const double v = x[i];
    if (!isfinite(v)) finite = false;
    const double d = v - S.c[i];
    Jx += d * d / S.Wd[i];
  }
  Jx = 0.5 * (Jx - 1.0);
  const double s0 = st.kspread ? st.kspread[p] : 0.0;   // reduced copies: J = J_red(mean) + s(0)
  Jx += s0;
  const long q = idx ? idx[p] : p;
  st.rows[p] = 0;
  st.partial[p] = 0;
  st.esc[p] = 0;
  st.bT[p] = 0.0f;
  st.bD[p] = 0.0f;
  if (st.s64) st.s64[p] = 0;
  st.probes[p] = 0;
  st.iters_tot[p] = 0;
  st.iters_probe[p] = 0;
  st.nscan[p] = 0;
  st.ncell[p] = 0;
  st.newt[p] = 0;
  st.wbef[p] = 0.0;
  st.stage[p] = 2;
  st.ha[p] = 0.0;
  st.hb[p] = 0.0;
  if (st.lam0s)
    for (int i = 0; i < S.n_pad; ++i) {
      double v = 0.0;
      if (lam0 && i < S.n) {
        if (S.U)
          for (int j = 0; j < S.n; ++j) v += S.U[(size_t)j * S.n + i] * lam0[q * ls + j];   // U^T lam0
        else
          v = lam0[q * ls + i];
      }
      st.lam0s[p * S.n_pad + i] = v;
    }
  st.P[p] = 0.0;
  st.D[p] = 0.0;
  st.flags[p] = 0;
  if (!finite) {
    st.status[p] = HOPF_PT_NONFINITE;
    st.phase[p] = PH_DONE;
    st.T[p] = NAN;
    return;
  }
  if (mode == MODE_MINTIME) {
    if (Jx <= 0.0) {   // inside the target: T = 0, lam = W^{-1}(x - c), phi = J(x)
      st.status[p] = HOPF_PT_INSIDE;
      st.phase[p] = PH_DONE;
      st.T[p] = 0.0;
      st.hi[p] = 0.0;
      double Pv = 0.5;
      for (int i = 0; i < S.n_pad; ++i) {
        const double l = i < S.n ? (x[i] - S.c[i]) / S.Wd[i] : 0.0;
        st.lam[p * S.n_pad + i] = (float)l;
        if (i < S.n) Pv += 0.5 * S.Wd[i] * l * l - (x[i] - S.c[i]) * l;
      }
      st.P[p] = Pv - s0;
      st.D[p] = -Jx;
      return;
    }
    st.status[p] = HOPF_PT_OK;
    st.phase[p] = PH_SCAN;
    st.nscan[p] = 1;
    st.T[p] = node_horizon(S.t_max, S.h, last_node(S.N, S.quad), scan_node(last_node(S.N, S.quad), o.scan, 1));
    st.lo[p] = 0.0;
    st.hi[p] = INFINITY;
    if (tb) {
      st.ha[p] = tb[2 * q];
      st.hb[p] = tb[2 * q + 1];
      st.stage[p] = 0;
    }
    mark_setup(st, p);
  } else {
    const double tv = t_in[q];
    st.status[p] = HOPF_PT_OK;
    st.phase[p] = PH_FINAL;
    st.T[p] = tv;
    st.lo[p] = tv;
    st.hi[p] = tv;
    mark_setup(st, p);
  }
}

// ------------------------------------------------------------------ probe setup

// Probe setup: the horizon split T = M h + r, x_f = e^{T A} x0 and (trapezoid,
// off-grid T) the extra node's block R = -Qu^T B^T e^{T A^T} = K_M e^{r A^T},
// all in FP64, then the warm or cold start and the step sizes.
//   1. x_M = e^{M h A} x0 by the binary node powers e^{2^b h A};
//   2. e^{r A} applied to [x_M | rows of K_M] (ncols columns, a few at a
//      time): r = q dr + rho, the base-16 digits of q pick the powers
//      e^{d 16^b dr A}, then a Taylor series for rho < dr with as many terms
//      as (rho ||A||)^k / k! needs to fall below 1e-17.
// A group of GS threads (one wave, GS = 64, or a workgroup, GS = 256) does
// the linear algebra of one probe.  Thread l of the group owns rows l + GS g
// of every vector; the CW vectors being transformed sit in LDS as
// vs[i CW + c] (row i of column c), and the matrices are stored by columns,
// so one column of a matrix is a single contiguous read of the group.
struct SetupInfo {
  int M, rows, part;
  double r, Rfro;
};

// columns per pass of step 2: a wave keeps 6 (3 for n > 128) in registers,
// a workgroup 4
template <int GS, int RG>
__host__ __device__ constexpr int setup_cw() { return GS == 64 ? (RG <= 2 ? 6 : 3) : 4; }

// Make the group's LDS writes visible to all of its threads before later reads.
template <int GS>
__device__ __forceinline__ void group_sync() {
  if constexpr (GS == 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// acc[c][g] = sum_k E(l + GS g, k) vs[k CW + c], c < CC, for an n x n matrix
// E stored by columns (E(i, k) at Ec[k n + i]).  U columns of E are loaded
// before their products, so that many loads are in flight together.
template <int GS, int RG, int CC, int CW>
__device__ __forceinline__ void group_apply(const double *__restrict__ Ec, const double *vs, int n, int l,
                                            double (&acc)[CC][RG]) {
  constexpr int U = CC == 1 ? 8 : 2;
#pragma unroll
  for (int c = 0; c < CC; ++c)
#pragma unroll
    for (int g = 0; g < RG; ++g) acc[c][g] = 0.0;
  int k = 0;
  for (; k + U <= n; k += U) {
    double e[U][RG];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const int i = l + GS * g;
        e[u][g] = (i < n) ? Ec[(size_t)(k + u) * n + i] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const double v = vs[(k + u) * CW + c];
#pragma unroll
        for (int g = 0; g < RG; ++g) acc[c][g] = fma(e[u][g], v, acc[c][g]);
      }
  }
  for (; k < n; ++k) {
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int i = l + GS * g;
      const double e = (i < n) ? Ec[(size_t)k * n + i] : 0.0;
#pragma unroll
      for (int c = 0; c < CC; ++c) acc[c][g] = fma(e, vs[k * CW + c], acc[c][g]);
    }
  }
}

// vs <- E vs on the first CC columns
template <int GS, int RG, int CC, int CW>
__device__ __forceinline__ void group_transform(const double *__restrict__ Ec, double *vs, int n, int l) {
  double acc[CC][RG];
  group_apply<GS, RG, CC, CW>(Ec, vs, n, l, acc);
  group_sync<GS>();   // every thread has read vs
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int i = l + GS * g;
    if (i < n)
#pragma unroll
      for (int c = 0; c < CC; ++c) vs[i * CW + c] = acc[c][g];
  }
  group_sync<GS>();
}

// vs <- e^{rho A} vs = sum_{k <= kt} (rho A)^k vs / k! on the first CC columns
// (the running term stays in vs, the sum in registers)
template <int GS, int RG, int CC, int CW>
__device__ __forceinline__ void group_taylor(const double *__restrict__ At, double *vs, int n, int l, double rho,
                                             int kt) {
  double sum[CC][RG];
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int i = l + GS * g;
#pragma unroll
    for (int c = 0; c < CC; ++c) sum[c][g] = (i < n) ? vs[i * CW + c] : 0.0;
  }
  for (int k = 1; k <= kt; ++k) {
    double acc[CC][RG];
    group_apply<GS, RG, CC, CW>(At, vs, n, l, acc);
    group_sync<GS>();
    const double f = rho / k;
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int i = l + GS * g;
      if (i < n)
#pragma unroll
        for (int c = 0; c < CC; ++c) {
          const double t = acc[c][g] * f;
          vs[i * CW + c] = t;
          sum[c][g] += t;
        }
    }
    group_sync<GS>();
  }
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int i = l + GS * g;
    if (i < n)
#pragma unroll
      for (int c = 0; c < CC; ++c) vs[i * CW + c] = sum[c][g];
  }
  group_sync<GS>();
}

// The linear algebra of the setup of point p by a group of GS threads
// (l: the thread's index in it, every thread of the group calls this):
// horizon split, x_f, A x_f and (off-grid trapezoid) the extra node's block
// and its Frobenius norm.  vs: n_pad setup_cw<GS, RG>() doubles of LDS;
// red: GS / 64 doubles of LDS for the norm (GS > 64).  Needs RG GS >= n.
template <int GS, int RG>
__device__ SetupInfo setup_linear(const SysView &S, const PtState &st, long p, int l, double *vs, double *red) {
  constexpr int CW = setup_cw<GS, RG>();
  const int n = S.n, m = S.m, np = S.n_pad;
  const double T = st.T[p];
  SetupInfo in;
  // horizon split T = M h + r (snapped to the grid within 1e-12 relative)
  const double q = T / S.h;
  const double qr = rint(q);
  int M;
  double r;
  if (fabs(q - qr) <= 1e-12 * fmax(1.0, q)) { M = (int)qr; r = 0.0; }
  else { M = (int)floor(q); r = T - M * S.h; }
  int rows, part;
  if (S.quad == HOPF_Q_TRAP) {
    if (M > S.N - 1) { M = S.N - 1; r = 0.0; }
    rows = (T > 0.0) ? M + 1 : 0;
    part = (r > 0.0) ? 1 : 0;
  } else {
    if (M > S.N) { M = S.N; r = 0.0; }
    rows = M + (r > 0.0 ? 1 : 0);
    if (rows > S.N) rows = S.N;
    part = 0;
  }
  const int ncols = 1 + (part ? m : 0);
  const long qd = (r > 0.0) ? (long)floor(r / S.dr) : 0;
  const long qdig = qd > 4095 ? 4095 : (qd < 0 ? 0 : qd);
  const double rho = (r > 0.0) ? r - (double)qdig * S.dr : 0.0;
  int kt = 0;
  if (rho > 0.0) {
    const double a = rho * S.anorm;
    double term = 1.0;
    while (kt < 30) {
      ++kt;
      term *= a / kt;
      if (term < 1e-17) break;
    }
  }
  // 1. x_M in column 0
  for (int i = l; i < n; i += GS) vs[i * CW] = st.x0[p * np + i];
  group_sync<GS>();
  for (int b = 0; b < S.n_hbin; ++b)
    if ((M >> b) & 1) group_transform<GS, RG, 1, CW>(S.hbin + (size_t)b * n * n, vs, n, l);
  // 2. e^{r A} on [x_M | K_M rows], CW columns at a time
  const int kb_M = M / NODE_BLOCK, kk_M = M % NODE_BLOCK;
  double Rfro = 0.0;
  for (int c0 = 0; c0 < ncols; c0 += CW) {
    const int cc = min(CW, ncols - c0);
    if (ncols > 1) {
      // columns c0 + cl: x_M (already in place), then rows j = col - 1 of
      // K_M; columns past ncols are zero
      for (int cl = (c0 == 0 ? 1 : 0); cl < CW; ++cl) {
        const int col = c0 + cl;
        for (int i = l; i < n; i += GS)
          vs[i * CW + cl] =
              col < ncols ? S.K64[(((size_t)kb_M * m + (col - 1)) * NODE_BLOCK + kk_M) * np + i] : 0.0;
      }
      group_sync<GS>();
    }
    for (int lv = 0; lv < RDIG_LEVELS; ++lv) {
      const int d = (int)((qdig >> (4 * lv)) & 15);
      if (!d) continue;
      const double *E = S.rdig + ((size_t)lv * 15 + (d - 1)) * n * n;
      if (ncols == 1) group_transform<GS, RG, 1, CW>(E, vs, n, l);
      else group_transform<GS, RG, CW, CW>(E, vs, n, l);
    }
    if (kt > 0) {
      if (ncols == 1) group_taylor<GS, RG, 1, CW>(S.At, vs, n, l, rho, kt);
      else group_taylor<GS, RG, CW, CW>(S.At, vs, n, l, rho, kt);
    }
    // store: column 0 is x_f (with A x_f), the others rows of R
    for (int cl = 0; cl < cc; ++cl) {
      const int col = c0 + cl;
      for (int i = l; i < np; i += GS) {
        const double v = i < n ? vs[i * CW + cl] : 0.0;
        if (col == 0) {
          st.xf[p * np + i] = v;
          st.xfc32[p * np + i] = (float)(i < n ? v - S.c[i] : 0.0);
        } else {
          const size_t o2 = ((size_t)p * m + (col - 1)) * np + i;
          st.R64[o2] = v;
          st.R32[o2] = (float)v;
          Rfro += v * v;
        }
      }
    }
    if (c0 == 0) {
      double ax[1][RG];
      group_apply<GS, RG, 1, CW>(S.At, vs, n, l, ax);
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        const int i = l + GS * g;
        if (i < np) st.axf[p * np + i] = i < n ? ax[0][g] : 0.0;
      }
    }
    group_sync<GS>();   // every thread is done reading vs before the next columns land
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) Rfro += __shfl_xor(Rfro, off, 64);
  if constexpr (GS > 64) {
    if ((l & 63) == 0) red[l >> 6] = Rfro;
    __syncthreads();
    Rfro = 0.0;
    for (int w = 0; w < GS / 64; ++w) Rfro += red[w];
    __syncthreads();
  }
  in.M = M;
  in.rows = rows;
  in.part = part;
  in.r = r;
  in.Rfro = Rfro;
  return in;
}

// Cold or continued start of point p's new probe by a group of GS threads
// (l: the thread's index in it): lambda from 0 (or the caller's lam0 at the
// first probe) or carried over, dual rows carried over where both probes
// have them, every other row at zero.
template <int GS>
__device__ void setup_start(const PtState &st, const Opts &o, long p, int m, int np, int rows, int l) {
  const int old_rows = st.rows[p];
  const bool first = st.probes[p] == 0;
  const bool cold = (o.warm == HOPF_WARM_COLD) || first;   // CONT and MLP keep y
  // FP64 iterations keep their own FP64 iterate (carried over when it is current)
  const bool f64 = st.s64 != nullptr;
  const bool had64 = f64 && st.s64[p] != 0;
  if (cold) {
    const bool given = st.lam0s != nullptr && first;
    for (int i = l; i < np; i += GS) {
      const double l = given ? st.lam0s[p * np + i] : 0.0;
      st.lam[p * np + i] = (float)l;
      st.lamb[p * np + i] = (float)l;
      if (f64) { st.lam64[p * np + i] = l; st.lamb64[p * np + i] = l; }
    }
  } else {
    for (int i = l; i < np; i += GS) {
      st.lamb[p * np + i] = st.lam[p * np + i];
      if (f64) {
        const double l = had64 ? st.lam64[p * np + i] : (double)st.lam[p * np + i];
        st.lam64[p * np + i] = l;
        st.lamb64[p * np + i] = l;
      }
    }
  }
  // The iteration kernels read the node blocks of a tile's longest point, so
  // every row of a point's dual iterate holds a finite value.  Rows at or
  // past the point's node count are zero after every setup and every
  // iteration (outside the horizon a node's weight is 0 and its dual projects
  // to 0), so only rows [keep, old_rows) can hold values to clear; the first
  // probe clears every row.
  const int keep = cold ? 0 : min(old_rows, rows);
  const int m16 = m * NODE_BLOCK;
  if (f64) {
    for (int e = l; e < st.ystride; e += GS) {
      const int kb = e / m16, kk = e % NODE_BLOCK;
      const size_t ye = (size_t)p * st.ystride + e;
      const bool zero = kb * NODE_BLOCK + kk >= keep;
      if (zero) st.y[ye] = 0.0f;
      st.y64[ye] = zero ? 0.0 : (had64 ? st.y64[ye] : (double)st.y[ye]);
    }
  } else {
    const int end = first ? st.ystride / m : max(keep, old_rows);
    const int e0 = (keep / NODE_BLOCK) * m16, e1 = ((end + NODE_BLOCK - 1) / NODE_BLOCK) * m16;
    for (int e = e0 + l; e < e1; e += GS) {
      const int kb = e / m16, kk = e % NODE_BLOCK;
      if (kb * NODE_BLOCK + kk >= keep) st.y[(size_t)p * st.ystride + e] = 0.0f;
    }
  }
  for (int j = l; j < st.mpad; j += GS) {
    st.yR[(size_t)p * st.mpad + j] = 0.0f;
    if (f64) st.yR64[(size_t)p * st.mpad + j] = 0.0;
  }
}

// Per-point fields of the new probe and its step sizes (one thread).
__device__ void setup_finish(const SysView &S, const PtState &st, const Opts &o, long p, const SetupInfo &in) {
  const double L2 = S.lpref[in.rows] + (in.part ? in.Rfro : 0.0);
  const double L = sqrt(L2);
  st.M[p] = in.M;
  st.r[p] = in.r;
  st.rows[p] = in.rows;
  st.partial[p] = in.part;
  if (L > 0.0) {
    const double ct = S.c_tau > 0.0 ? S.c_tau : o.c_tau;
    st.tau[p] = ct / L;
    st.sig[p] = 0.999 / (ct * L);
  } else {   // no quadrature nodes: the prox of G alone is exact in one step
    st.tau[p] = 1e20;
    st.sig[p] = 0.0;
  }
  st.iters_probe[p] = 0;
  st.probes[p] += 1;
  st.flags[p] = 0;
  if (st.s64 != nullptr) st.s64[p] = 1;
}

// Block scratch of setup_point (doubles): the vectors | norm partial sums |
// network activations (4 x 260 floats)
constexpr int SETUP_VS = 256 * setup_cw<256, 1>();
constexpr int SETUP_SCRATCH = SETUP_VS + 8 + 520;

// The setup of point p by a workgroup of 256 threads (one row per thread),
// with the learned warm start.  sm: SETUP_SCRATCH doubles of LDS (the
// caller's; free during the call).
__device__ void setup_point(SysView S, PtState st, Opts o, MlpView mv, long p, double *sm) {
  __syncthreads();
  const int tid = threadIdx.x;
  const int n = S.n, np = S.n_pad;
  const SetupInfo info = setup_linear<256, 1>(S, st, p, tid, sm, sm + SETUP_VS);
  setup_start<256>(st, o, p, S.m, np, info.rows, tid);
  __syncthreads();
  const double T = st.T[p];
  const bool f64 = st.s64 != nullptr;
  // learned warm start at a later probe (mode mlp_lam): lam_0 = network(x, T);
  // the first probe's network output was evaluated for all points at once
  if (o.warm == HOPF_WARM_MLP_LAM && st.probes[p] > 0 && mv.valid && mv.n == n && mv.H == 256) {
    float *zin = reinterpret_cast<float *>(sm + SETUP_VS + 8), *ha = zin + 260, *hb = ha + 260, *outv = hb + 260;
    const int di = n + 1, dout = n + 2, H = 256;
    __syncthreads();
    for (int i = tid; i < di; i += 256)
      zin[i] = (i < n) ? (float)((st.x0[p * np + i] - mv.xm[i]) / mv.xs[i]) : (float)(T / mv.t_scale);
    __syncthreads();
    const float *W1 = mv.theta, *b1 = W1 + (size_t)di * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H,
                *W3 = b2 + H, *b3 = W3 + (size_t)H * H, *W4 = b3 + H, *b4 = W4 + (size_t)H * dout;
    {
      float a = b1[tid];
      for (int i = 0; i < di; ++i) a += zin[i] * W1[(size_t)i * H + tid];
      ha[tid] = gelu_f(a);
    }
    __syncthreads();
    {
      float a = b2[tid];
      for (int i = 0; i < H; ++i) a += ha[i] * W2[(size_t)i * H + tid];
      hb[tid] = gelu_f(a);
    }
    __syncthreads();
    {
      float a = b3[tid];
      for (int i = 0; i < H; ++i) a += hb[i] * W3[(size_t)i * H + tid];
      ha[tid] = gelu_f(a);
    }
    __syncthreads();
    for (int k = tid; k < dout; k += 256) {
      float a = b4[k];
      for (int i = 0; i < H; ++i) a += ha[i] * W4[(size_t)i * dout + k];
      outv[k] = a;
    }
    __syncthreads();
    // a network output that is not finite, or a costate more than 1000 times
    // the training costates' scale, is not used (the start stays cold or
    // continued): a damaged network can slow a solve down, not change it
    if (tid == 0) {
      int bad = !(isfinite(mv.lam_scale) && mv.lam_scale > 0.0f);
      for (int k = 0; k < dout; ++k) bad |= !isfinite(outv[k] * (k < n ? mv.lam_scale : 1.0f));
      for (int k = 0; k < n; ++k) bad |= fabsf(outv[k]) > 1e3f;
      reinterpret_cast<int *>(outv)[dout] = bad;
    }
    __syncthreads();
    const bool net_bad = reinterpret_cast<const int *>(outv)[dout] != 0;
    if (!net_bad) {
      for (int i = tid; i < np; i += 256) {
        const float l = i < n ? outv[i] * mv.lam_scale : 0.0f;
        st.lam[p * np + i] = l;
        st.lamb[p * np + i] = l;
        if (f64) { st.lam64[p * np + i] = l; st.lamb64[p * np + i] = l; }
      }
    }
    __syncthreads();
  }
  if (tid == 0) setup_finish(S, st, o, p, info);
}

// Probe setups without the network: one wave per point on the setup list,
// RG 64 >= n.  Dynamic LDS: 4 n_pad setup_cw<64, RG>() doubles.
template <int RG>
__global__ __launch_bounds__(256) void k_setup_waves(SysView S, PtState st, Opts o) {
  extern __shared__ __align__(16) double sw[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *vs = sw + (size_t)wave * S.n_pad * setup_cw<64, RG>();
  const int nset = st.counters[1];
  for (int li = blockIdx.x * 4 + wave; li < nset; li += gridDim.x * 4) {
    const long p = st.setup_list[li];
    const SetupInfo in = setup_linear<64, RG>(S, st, p, lane, vs, nullptr);
    setup_start<64>(st, o, p, S.m, S.n_pad, in.rows, lane);
    if (lane == 0) setup_finish(S, st, o, p, in);
    group_sync<64>();
  }
}

typedef void (*SetupWavesFn)(SysView, PtState, Opts);
SetupWavesFn setup_waves_for(int n) {
  if (n <= 64) return k_setup_waves<1>;
  if (n <= 128) return k_setup_waves<2>;
  if (n <= 192) return k_setup_waves<3>;
  return k_setup_waves<4>;
}

// Probe setups with the learned warm start: one workgroup per point.
__global__ __launch_bounds__(256) void k_setup(SysView S, PtState st, Opts o, MlpView mv) {
  __shared__ double sm[SETUP_SCRATCH];
  const int nset = st.counters[1];
  for (int li = blockIdx.x; li < nset; li += gridDim.x) {
    const long p = st.setup_list[li];
    setup_point(S, st, o, mv, p, sm);
    __syncthreads();
  }
}

// ------------------------------------------------------------------ per-point tail solver

// When few points remain, a 16-point MFMA tile is mostly empty and a round
// (setup, sort, iteration and certificate launches) costs the same however
// few points it carries.  The tail solver gives each remaining point a
// workgroup of its own and runs the rest of its search inside one launch:
// FP32 iterations as matrix-vector products (the node table streams from L2,
// chunks of node blocks staged in LDS), the FP64 certificate and the search
// step (decide) every check_every iterations, and the next probe's setup in
// place.  The arithmetic is the same as the tiled path's (same tables, same
// projections, same certificate); only the summation order differs.
constexpr int TAIL_MAX_POINTS = 8192;

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s);
  return v;
}

// Dual product of one chunk of node-block rows, V[r] = K[r,:] . b (rows of
// the chunk contiguous in the dual table layout, n_pad values each): four
// lanes per row, float4 (double2) loads, four rows in flight per quad.
template <typename T, typename T4>
__device__ __forceinline__ void tail_dual(const T *__restrict__ Kc, const T *__restrict__ b, T *__restrict__ V,
                                          int nrow, int np, int tid) {
  constexpr int EL = sizeof(T4) / sizeof(T);      // elements per vector load
  const int q = tid & 3, quad = tid >> 2;
  const int nv = np / EL;                           // vector loads per row (multiple of 4)
  const T4 *K4 = reinterpret_cast<const T4 *>(Kc);
  const T4 *b4 = reinterpret_cast<const T4 *>(b);
  for (int r0 = quad; r0 < nrow; r0 += 4 * 64) {
    T acc[4] = {0, 0, 0, 0};
    const T4 *rp[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 64 * u;
      rp[u] = K4 + (size_t)(r < nrow ? r : r0) * nv;
    }
#pragma unroll 2
    for (int c = q; c < nv; c += 4) {
      const T4 bb = b4[c];
      T4 a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = rp[u][c];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if constexpr (EL == 4) acc[u] += a[u].x * bb.x + a[u].y * bb.y + a[u].z * bb.z + a[u].w * bb.w;
        else acc[u] += a[u].x * bb.x + a[u].y * bb.y;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      T v = acc[u];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      const int r = r0 + 64 * u;
      if (q == 0 && r < nrow) V[r] = v;
    }
  }
}

// Primal product of one chunk, g += K[rows,:]^T y[rows]: lane (c, group)
// owns column chunk c (EL columns) and the rows of its group; partial sums
// stay in registers across chunks.
template <typename T, typename T4>
__device__ __forceinline__ void tail_primal(const T *__restrict__ Kc, const T *__restrict__ y, T4 &g, int nrow,
                                            int np, int tid) {
  constexpr int EL = sizeof(T4) / sizeof(T);
  const int nv = np / EL, ngrp = 256 / nv;
  const int c = tid % nv, grp = tid / nv;
  if (grp >= ngrp) return;
  const T4 *K4 = reinterpret_cast<const T4 *>(Kc) + c;
#pragma unroll 8
  for (int r = grp; r < nrow; r += ngrp) {
    const T4 a = K4[(size_t)r * nv];
    const T yv = y[r];
    g.x += a.x * yv;
    g.y += a.y * yv;
    if constexpr (EL == 4) {
      g.z += a.z * yv;
      g.w += a.w * yv;
    }
  }
}

// Dynamic LDS of k_tail_multi (the probe setup reuses the same bytes):
//   bop 256 floats | l64 256 doubles | gp 256 x 16 B | red 5 x 4 doubles | vb CH doubles
__host__ __device__ inline int tail_chunk_blocks(int m) { return m >= 256 ? 1 : (256 / m < 16 ? 256 / m : 16); }
__host__ __device__ inline size_t tail_lds_bytes(int m) {
  const size_t it = 256 * 4 + 256 * 8 + 256 * 16 + 20 * 8 + (size_t)16 * tail_chunk_blocks(m) * m * 8;
  const size_t su = (size_t)SETUP_SCRATCH * 8;
  return it > su ? it : su;
}

// The whole remaining search of point p by one workgroup of 256 threads;
// tl_raw: tail_lds_bytes(S.m) bytes of LDS, s_ctl: one shared int.
__device__ void tail_point(const SysView &S, const PtState &st, const Opts &o, const MlpView &mv, long p,
                           unsigned char *tl_raw, int &s_ctl) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = S.m, np = S.n_pad, n = S.n;
  const int CB = tail_chunk_blocks(m);
  float *bop = reinterpret_cast<float *>(tl_raw);
  double *l64 = reinterpret_cast<double *>(tl_raw + 1024);
  float4 *gpf4 = reinterpret_cast<float4 *>(tl_raw + 1024 + 2048);
  double2 *gpd2 = reinterpret_cast<double2 *>(gpf4);
  float *gpf = reinterpret_cast<float *>(gpf4);
  double *gpd = reinterpret_cast<double *>(gpf4);
  double *red = reinterpret_cast<double *>(tl_raw + 1024 + 2048 + 4096);
  double *vb = red + 20;
  float *vbf = reinterpret_cast<float *>(vb);
  double *sm = reinterpret_cast<double *>(tl_raw);        // probe setup scratch (aliases all of the above)
  float *yp = st.y + (size_t)p * st.ystride;
  const int mp = st.mpad;
  const int nv4 = np / 4, ng4 = 256 / nv4, nv2 = np / 2, ng2 = 256 / nv2;
  // every interval runs check_every iterations (or none: the certificate of a
  // fresh probe's starting point); the search ends within scan + 64 probes
  // (scan, then a cell whose width halves at least every two probes) of at
  // most max_iter iterations each
  const long guard_max = (long)(o.scan + 64) * (o.max_iter / o.check_every + 3);
  bool fresh = true;     // the running probe has not iterated yet: certify its starting point first
  // step adaptation: iterate and certified gap at the last restart (thread 0)
  __shared__ int s_restart;
  double gap_r = INFINITY, gap_prev = INFINITY;
  double w_base = 0.0;   // the probe's starting primal weight; adapted weights stay within 4x of it
  int since = 0;         // certificates since the last restart
  bool need_ref = o.adapt != 0;
  float *lref = st.lamref + (size_t)p * np, *yref = st.yref + (size_t)p * st.ystride;
  for (long guard = 0; guard < guard_max; ++guard) {
    __syncthreads();   // every wave has read s_ctl of the previous interval
    if (tid == 0) s_ctl = st.phase[p];
    __syncthreads();
    if (s_ctl == PH_DONE) break;
    const int rows = st.rows[p], M = st.M[p], part = st.partial[p];
    const double rr = st.r[p];
    const int nkb = (rows + NODE_BLOCK - 1) / NODE_BLOCK;
    if (need_ref) {   // a new probe (or entry): its starting iterate is the reference
      for (int i = tid; i < np; i += 256) lref[i] = st.lam[p * np + i];
      for (int e = tid; e < nkb * m * NODE_BLOCK; e += 256) yref[e] = yp[e];
      gap_r = INFINITY;
      gap_prev = INFINITY;
      since = 0;
      w_base = (st.tau[p] > 0.0 && st.sig[p] > 0.0) ? sqrt(st.sig[p] / (0.999 * st.tau[p])) : 0.0;
      need_ref = false;
    }
    const float tau = (float)st.tau[p], sig = (float)st.sig[p];
    float lam_i = 0.f, xfc = 0.f, wd = 1.f;
    if (tid < np) {
      lam_i = st.lam[p * np + tid];
      xfc = st.xfc32[p * np + tid];
      wd = (float)S.Wd[tid];
    }
    bop[tid] = tid < np ? sig * st.lamb[p * np + tid] : 0.f;
    // ---------------- check_every FP32 iterations (none for a fresh probe)
    for (int it = 0; it < (fresh ? 0 : o.check_every); ++it) {
      float4 g4 = make_float4(0.f, 0.f, 0.f, 0.f);
      __syncthreads();                       // bop of this iteration
      for (int kb0 = 0; kb0 < nkb; kb0 += CB) {
        const int cb = min(CB, nkb - kb0), nrow = cb * m * NODE_BLOCK;
        const float *Kc = S.K32 + (size_t)kb0 * m * NODE_BLOCK * np;
        tail_dual<float, float4>(Kc, bop, vbf, nrow, np, tid);   // V = K (sigma lam_bar)
        __syncthreads();
        if (tid < cb * NODE_BLOCK) {   // y_k = projection of y_k + V_k onto w_k C, one node per thread
          const int kbl = tid >> 4, kk = tid & 15, k = (kb0 + kbl) * NODE_BLOCK + kk;
          const float w = (k < rows) ? (float)node_weight(k, M, rr, S.h, S.quad) : 0.f;
          float *yr = yp + (size_t)(kb0 + kbl) * m * NODE_BLOCK + kk;
          float *vr = vbf + kbl * m * NODE_BLOCK + kk;
          if (S.uset == HOPF_U_L2) {
            float ss = 0.f;
            for (int j = 0; j < m; ++j) {
              const float v = yr[j * NODE_BLOCK] + vr[j * NODE_BLOCK];
              vr[j * NODE_BLOCK] = v;
              ss += v * v;
            }
            const float nv = sqrtf(ss);
            const float sc = (nv > w) ? (nv > 0.f ? w / nv : 0.f) : 1.f;
            for (int j = 0; j < m; ++j) {
              const float v = vr[j * NODE_BLOCK] * sc;
              vr[j * NODE_BLOCK] = v;
              yr[j * NODE_BLOCK] = v;
            }
          } else {
            for (int j = 0; j < m; ++j) {
              const float v = fminf(fmaxf(yr[j * NODE_BLOCK] + vr[j * NODE_BLOCK], -w), w);
              vr[j * NODE_BLOCK] = v;
              yr[j * NODE_BLOCK] = v;
            }
          }
        }
        __syncthreads();
        tail_primal<float, float4>(Kc, vbf, g4, nrow, np, tid);   // g += K^T y
        __syncthreads();
      }
      if (part) {   // the private node at tau = T with weight r/2
        for (int j = wave; j < m; j += 4) {
          const float *row = st.R32 + ((size_t)p * m + j) * np;
          float acc = 0.f;
          for (int i = lane; i < np; i += 64) acc += row[i] * bop[i];
          acc = wave_sum_f(acc);
          if (lane == 0) vbf[j] = st.yR[(size_t)p * mp + j] + acc;
        }
        __syncthreads();
        if (tid == 0) {
          const float wR = (float)(0.5 * rr);
          if (S.uset == HOPF_U_L2) {
            float ss = 0.f;
            for (int j = 0; j < m; ++j) ss += vbf[j] * vbf[j];
            const float nv = sqrtf(ss);
            const float sc = (nv > wR) ? (nv > 0.f ? wR / nv : 0.f) : 1.f;
            for (int j = 0; j < m; ++j) vbf[j] *= sc;
          } else {
            for (int j = 0; j < m; ++j) vbf[j] = fminf(fmaxf(vbf[j], -wR), wR);
          }
          for (int j = 0; j < m; ++j) st.yR[(size_t)p * mp + j] = vbf[j];
        }
        __syncthreads();
      }
      if (tid / nv4 < ng4) gpf4[tid] = g4;     // column chunk tid % nv4 of group tid / nv4
      __syncthreads();
      if (tid < np) {   // lam+ = (lam - tau (K^T y - (x_f - c))) / (1 + tau W);  theta = 1
        float gs = 0.f;
        for (int r2 = 0; r2 < ng4; ++r2) gs += gpf[r2 * np + tid];
        if (part)
          for (int j = 0; j < m; ++j) gs += st.R32[((size_t)p * m + j) * np + tid] * vbf[j];
        const float ln = (lam_i - tau * (gs - xfc)) / (1.f + tau * wd);
        bop[tid] = sig * (2.f * ln - lam_i);
        lam_i = ln;
      }
    }
    __syncthreads();
    if (tid < np) {
      if (!fresh) {
        st.lam[p * np + tid] = lam_i;
        st.lamb[p * np + tid] = sig > 0.f ? bop[tid] / sig : 0.f;
      }
      l64[tid] = (double)lam_i;
    }
    if (tid == 0 && !fresh) {
      st.iters_probe[p] += o.check_every;
      st.iters_tot[p] += o.check_every;
      atomicAdd(&st.rowsum[1], (double)(rows + part));
    }
    __syncthreads();
    // ---------------- FP64 certificate from (lam, y)
    double wsig = 0.0, slast = 0.0;
    double2 g2 = make_double2(0.0, 0.0);
    for (int kb0 = 0; kb0 < nkb; kb0 += CB) {
      const int cb = min(CB, nkb - kb0), nrow = cb * m * NODE_BLOCK;
      const double *Kc = S.K64 + (size_t)kb0 * m * NODE_BLOCK * np;
      tail_dual<double, double2>(Kc, l64, vb, nrow, np, tid);    // U = K lam
      __syncthreads();
      if (tid < cb * NODE_BLOCK) {
        const int kbl = tid >> 4, kk = tid & 15, k = (kb0 + kbl) * NODE_BLOCK + kk;
        const double w = (k < rows) ? node_weight(k, M, rr, S.h, S.quad) : 0.0;
        const float *yr = yp + (size_t)(kb0 + kbl) * m * NODE_BLOCK + kk;
        double *ur = vb + kbl * m * NODE_BLOCK + kk;
        double sg = 0.0, ysq = 0.0;
        for (int j = 0; j < m; ++j) {
          const double u = ur[j * NODE_BLOCK];
          sg += (S.uset == HOPF_U_L2) ? u * u : fabs(u);
          const double yv = (double)yr[j * NODE_BLOCK];
          ysq += yv * yv;
        }
        if (S.uset == HOPF_U_L2) sg = sqrt(sg);
        wsig += w * sg;
        if (!part && k == rows - 1) slast = sg;
        double ysc = 1.0;
        if (S.uset == HOPF_U_L2) {
          const double nv = sqrt(ysq);
          if (w <= 0.0 || nv == 0.0) ysc = 0.0;
          else if (nv >= (1.0 - 1e-5) * w) ysc = w / nv;
        }
        for (int j = 0; j < m; ++j) {   // y^ (replaces U in LDS)
          double v = (double)yr[j * NODE_BLOCK];
          if (S.uset == HOPF_U_L2) v *= ysc;
          else {
            v = fmin(fmax(v, -w), w);
            if (w > 0.0 && fabs(v) >= (1.0 - 1e-5) * w) v = copysign(w, v);
          }
          ur[j * NODE_BLOCK] = v;
        }
      }
      __syncthreads();
      tail_primal<double, double2>(Kc, vb, g2, nrow, np, tid);   // K^T y^
      __syncthreads();
    }
    if (part) {
      for (int j = wave; j < m; j += 4) {
        const double *row = st.R64 + ((size_t)p * m + j) * np;
        double acc = 0.0;
        for (int i = lane; i < np; i += 64) acc += row[i] * l64[i];
        acc = wave_sum_d(acc);
        if (lane == 0) {
          vb[j] = acc;                                    // U_R
          vb[64 + j] = (double)st.yR[(size_t)p * mp + j];  // y_R
        }
      }
      __syncthreads();
      if (tid == 0) {
        const double wR = 0.5 * rr;
        double sg = 0.0, ysq = 0.0;
        for (int j = 0; j < m; ++j) {
          sg += (S.uset == HOPF_U_L2) ? vb[j] * vb[j] : fabs(vb[j]);
          ysq += vb[64 + j] * vb[64 + j];
        }
        if (S.uset == HOPF_U_L2) sg = sqrt(sg);
        wsig += wR * sg;
        slast = sg;
        double ysc = 1.0;
        if (S.uset == HOPF_U_L2) {
          const double nv = sqrt(ysq);
          if (wR <= 0.0 || nv == 0.0) ysc = 0.0;
          else if (nv >= (1.0 - 1e-5) * wR) ysc = wR / nv;
        }
        for (int j = 0; j < m; ++j) {
          double v = vb[64 + j];
          if (S.uset == HOPF_U_L2) v *= ysc;
          else {
            v = fmin(fmax(v, -wR), wR);
            if (wR > 0.0 && fabs(v) >= (1.0 - 1e-5) * wR) v = copysign(wR, v);
          }
          vb[64 + j] = v;
        }
      }
      __syncthreads();
    }
    if (tid / nv2 < ng2) gpd2[tid] = g2;
    __syncthreads();
    double sP = 0.0, sJ = 0.0, sAx = 0.0;
    if (tid < n) {
      double G = 0.0;
      for (int r2 = 0; r2 < ng2; ++r2) G += gpd[r2 * np + tid];
      if (part)
        for (int j = 0; j < m; ++j) G += st.R64[((size_t)p * m + j) * np + tid] * vb[64 + j];
      const double l = l64[tid], xf = st.xf[p * np + tid], cc = S.c[tid], wdd = S.Wd[tid];
      sP = 0.5 * wdd * l * l - (xf - cc) * l;
      const double d = xf - G - cc;      // x_T - c
      sJ = d * d / wdd;
      sAx = st.axf[p * np + tid] * l;
    }
    {
      const double v[5] = {wave_sum_d(sP), wave_sum_d(sJ), wave_sum_d(sAx), wave_sum_d(wsig), wave_sum_d(slast)};
      if (lane == 0)
        for (int q = 0; q < 5; ++q) red[q * 4 + wave] = v[q];
    }
    __syncthreads();
    if (tid == 0) {
      double a[5];
      for (int q = 0; q < 5; ++q) a[q] = (red[q * 4] + red[q * 4 + 1]) + (red[q * 4 + 2] + red[q * 4 + 3]);
      s_ctl = decide(S, st, o, p, np, a[0], a[3], a[1], a[2], a[4]) ? 1 : 0;
      s_restart = 0;
      if (o.adapt && !s_ctl && st.phase[p] != PH_DONE) {
        const double Pv = st.P[p], Dv = st.D[p];
        const double gap = (Pv - Dv) / fmax(1.0, fabs(Dv));
        ++since;
        // the first certificate of a probe always restarts; later ones at least 4 certificates apart
        s_restart = (gap_r == INFINITY || (since >= 4 && (gap <= 0.2 * gap_r || (gap <= 0.8 * gap_r && gap > gap_prev))))
                        ? 1 : 0;
        if (s_restart) {
          gap_r = gap;
          since = 0;
        }
        gap_prev = gap;
      }
    }
    __syncthreads();
    if (s_restart) {   // |dlam|^2, |dy|^2 since the last restart; the current iterate becomes the reference
      double dl = 0.0, dy = 0.0;
      for (int i = tid; i < np; i += 256) {
        const float l = st.lam[p * np + i];
        const double d = (double)l - (double)lref[i];
        dl += d * d;
        lref[i] = l;
      }
      for (int e = tid; e < nkb * m * NODE_BLOCK; e += 256) {
        const float v = yp[e];
        const double d = (double)v - (double)yref[e];
        dy += d * d;
        yref[e] = v;
      }
      dl = wave_sum_d(dl);
      dy = wave_sum_d(dy);
      if (lane == 0) {
        red[wave] = dl;
        red[4 + wave] = dy;
      }
      __syncthreads();
      if (tid == 0) {
        const double dl2 = (red[0] + red[1]) + (red[2] + red[3]);
        const double dy2 = (red[4] + red[5]) + (red[6] + red[7]);
        const double ta = st.tau[p], sg = st.sig[p];
        if (dl2 > 0.0 && dy2 > 0.0 && isfinite(dl2) && isfinite(dy2) && ta > 0.0 && sg > 0.0) {
          const double w_old = sqrt(sg / (0.999 * ta));             // omega = 1 / c_tau
          double w_new = sqrt(w_old * sqrt(dy2 / dl2));            // geometric mean with |dy| / |dlam|
          if (w_base > 0.0) w_new = fmin(fmax(w_new, 0.25 * w_base), 4.0 * w_base);
          st.tau[p] = ta * (w_old / w_new);
          st.sig[p] = sg * (w_new / w_old);
        }
      }
    }
    fresh = s_ctl != 0;
    if (s_ctl) {
      setup_point(S, st, o, mv, p, sm);
      need_ref = o.adapt != 0;
    }
  }
}

// Every parked job of a call in one launch: jobs[j] owns workgroups
// [base[j], base[j+1]), workgroup base[j] + i takes the job's i-th active point.
struct TailJob {
  SysView S;
  PtState st;
  MlpView mv;
  long base;
};

__global__ __launch_bounds__(256) void k_tail_multi(const TailJob *__restrict__ jobs, int njobs, Opts o) {
  extern __shared__ __align__(16) unsigned char tl_raw[];
  __shared__ int s_ctl;
  const long b = blockIdx.x;
  int j = 0;
  while (j + 1 < njobs && jobs[j + 1].base <= b) ++j;
  const TailJob &J = jobs[j];
  const long i = b - J.base;
  if (i >= J.st.counters[0]) return;
  tail_point(J.S, J.st, o, J.mv, J.st.perm[i], tl_raw, s_ctl);
}


// ------------------------------------------------------------------ tile formation

// Active points (not done and not waiting for a probe setup) sorted by class
// (FP32-escalated first) and by rows (descending) so that a tile's points
// need similar table prefixes.  reset_setup: the setup list was consumed by
// the k_setup launch before this one; count_rows: add the active point-rows
// to the flop accounting (the iteration launch after this sort runs them:
// 1 on the 16-point tiles, 2 on the 64-point kernel).
__global__ __launch_bounds__(1024) void k_sort(PtState st, int N, int reset_setup, int count_rows) {
  __shared__ int hist[2 * 4097 + 2];
  __shared__ double rsum[1024];
  const int tid = threadIdx.x;
  const int nb = 2 * (N + 1);
  for (int b = tid; b < nb; b += 1024) hist[b] = 0;
  __syncthreads();
  double loc = 0.0;
  for (long p = tid; p < st.npts; p += 1024) {
    if (st.phase[p] == PH_DONE || st.flags[p]) continue;
    const int rw = st.rows[p];
    const int bin = (st.esc[p] ? 0 : N + 1) + (N - rw);
    atomicAdd(&hist[bin], 1);
    loc += (double)(rw + st.partial[p]);
  }
  rsum[tid] = loc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (tid < s) rsum[tid] += rsum[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    if (reset_setup) st.counters[1] = 0;
    int acc = 0, nesc = 0;
    for (int b = 0; b < nb; ++b) {   // exclusive scan
      const int v = hist[b];
      hist[b] = acc;
      acc += v;
      if (b == N) nesc = acc;
    }
    st.counters[0] = acc;
    st.counters[3] = nesc;
    if (count_rows) st.rowsum[count_rows == 2 ? 2 : 0] += rsum[0];
  }
  __syncthreads();
  for (long p = tid; p < st.npts; p += 1024) {
    if (st.phase[p] == PH_DONE || st.flags[p]) continue;
    const int bin = (st.esc[p] ? 0 : N + 1) + (N - st.rows[p]);
    const int pos = atomicAdd(&hist[bin], 1);
    st.perm[pos] = (int)p;
  }
}

// ------------------------------------------------------------------ control and trajectory read-out

// v <- e^{dt A} v (or e^{dt A^T} v) for one LDS vector of length n, by the
// binary-power table and a Taylor series for the remainder below delta.
__device__ void exp_apply(const SysView &S, double dt, double *v, double *w, double *term, bool transpose) {
  const int n = S.n, tid = threadIdx.x;
  long qq = (long)floor(dt / S.delta);
  if (qq < 0) qq = 0;
  if (qq > (1L << POW_BITS)) qq = 1L << POW_BITS;
  const double rho = dt - qq * S.delta;
  for (int b = 0; b <= POW_BITS; ++b) {
    if (!((qq >> b) & 1L)) continue;
    const double *E = S.epow + (size_t)b * n * n;
    for (int i = tid; i < n; i += blockDim.x) {
      double acc = 0.0;
      for (int l = 0; l < n; ++l) acc += (transpose ? E[(size_t)l * n + i] : E[(size_t)i * n + l]) * v[l];
      w[i] = acc;
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) v[i] = w[i];
    __syncthreads();
  }
  if (rho > 0.0) {
    for (int i = tid; i < n; i += blockDim.x) term[i] = v[i];
    __syncthreads();
    for (int k = 1; k <= 8; ++k) {
      for (int i = tid; i < n; i += blockDim.x) {
        double acc = 0.0;
        for (int l = 0; l < n; ++l) acc += (transpose ? S.A[(size_t)l * n + i] : S.A[(size_t)i * n + l]) * term[l];
        w[i] = acc * (rho / k);
      }
      __syncthreads();
      for (int i = tid; i < n; i += blockDim.x) { term[i] = w[i]; v[i] += w[i]; }
      __syncthreads();
    }
  }
}

// Point 0 of the state after a value solve at horizon T: nodes in order of
// increasing physical time s = T - tau, the control u = Qu y^/w at each node
// (y^: FP64 projection of the dual block onto w C), the state after each
// node's impulse e^{tau A} B Qu y^ (so the last state is the certified x_T),
// and p* = e^{T A^T} lam*.
__global__ __launch_bounds__(256) void k_traj(SysView S, PtState st, double T, double *s_out, double *u_out,
                                              double *xs_out, double *p_out, int *nn_out) {
  __shared__ double z[256], w2[256], term[256], yh[64];
  __shared__ double s_prev_sh;
  const int tid = threadIdx.x, n = S.n, m = S.m, mu = S.m_user;
  const int rows = st.rows[0], part = st.partial[0], M = st.M[0];
  const double r = st.r[0];
  const int nn = rows + part;
  for (int i = tid; i < n; i += 256) z[i] = st.x0[i];
  if (tid == 0) { *nn_out = nn; s_prev_sh = 0.0; }
  __syncthreads();
  for (int j = 0; j < nn; ++j) {
    // node j: the private node (tau = T, s = 0) first, then table nodes k = rows-1 .. 0
    const bool isp = part && j == 0;
    const int k = isp ? -1 : rows - 1 - (j - part);
    const double tau = isp ? T : k * S.h;
    const double s = T - tau;
    const double w = isp ? 0.5 * r : node_weight(k, M, r, S.h, S.quad);
    // y^ for this node
    if (tid < m) {
      double v;
      const bool u64 = st.s64 != nullptr && st.s64[0] != 0;
      const size_t ye = ((size_t)(k / NODE_BLOCK) * m + tid) * NODE_BLOCK + (k % NODE_BLOCK);
      if (isp) v = u64 ? st.yR64[tid] : st.yR[tid];
      else v = u64 ? st.y64[ye] : st.y[ye];
      yh[tid] = v;
    }
    __syncthreads();
    if (tid == 0) {
      double nv = 0.0;
      for (int a = 0; a < m; ++a) nv += yh[a] * yh[a];
      nv = sqrt(nv);
      for (int a = 0; a < m; ++a) {
        double v = yh[a];
        if (S.uset == HOPF_U_L2) {
          if (w <= 0.0 || nv == 0.0) v = 0.0;
          else if (nv >= (1.0 - 1e-5) * w) v = v * (w / nv);
        } else {
          v = fmin(fmax(v, -w), w);
          if (w > 0.0 && fabs(v) >= (1.0 - 1e-5) * w) v = copysign(w, v);
        }
        yh[a] = v;
      }
    }
    __syncthreads();
    // advance the state from the previous node's time to s
    const double dt = s - s_prev_sh;
    __syncthreads();
    if (dt > 0.0) {
      if (fabs(dt - S.h) <= 1e-12 * S.h) {
        for (int i = tid; i < n; i += 256) {
          double acc = 0.0;
          for (int l = 0; l < n; ++l) acc += S.Eh[(size_t)i * n + l] * z[l];
          w2[i] = acc;
        }
        __syncthreads();
        for (int i = tid; i < n; i += 256) z[i] = w2[i];
        __syncthreads();
      } else {
        exp_apply(S, dt, z, w2, term, false);
      }
    }
    // impulse B Qu y^ (BQ holds -B Qu)
    for (int i = tid; i < n; i += 256) {
      double acc = 0.0;
      for (int a = 0; a < m; ++a) acc -= S.BQ[(size_t)i * m + a] * yh[a];
      z[i] += acc;
    }
    __syncthreads();
    for (int i = tid; i < n; i += 256) xs_out[(size_t)j * n + i] = z[i];
    if (tid < mu) {
      double acc = 0.0;
      if (w > 0.0)
        for (int a = 0; a < mu; ++a) acc += S.Qu[(size_t)tid * mu + a] * yh[a];
      u_out[(size_t)j * mu + tid] = w > 0.0 ? acc / w : 0.0;
    }
    if (tid == 0) { s_out[j] = s; s_prev_sh = s; }
    __syncthreads();
  }
  // p* = e^{T A^T} lam
  for (int i = tid; i < n; i += 256) z[i] = (st.s64 != nullptr && st.s64[0] != 0) ? st.lam64[i] : (double)st.lam[i];
  __syncthreads();
  exp_apply(S, T, z, w2, term, true);
  for (int i = tid; i < n; i += 256) p_out[i] = z[i];
}

// ------------------------------------------------------------------ outputs

// results of job point p go to the caller's index idx[p] (or p); lam rows are ls apart
__global__ void k_outputs(SysView S, PtState st, int mode, double *T_out, double *gap_out,
                          double *philo, double *phihi, double *lam_out, int *probes_out,
                          int *iters_out, int *status_out, const int *__restrict__ idx, int ls) {
  const long p0 = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p0 >= st.npts) return;
  const long p = p0;
  const long q = idx ? idx[p0] : p0;
  const double Pv = st.P[p], Dv = st.D[p];
  const int stt = st.status[p];
  if (T_out) {
    double Tv = st.T[p];
    if (mode == MODE_MINTIME) {
      if (stt == HOPF_PT_OK || stt == HOPF_PT_INSIDE) Tv = st.hi[p];
      else if (stt == HOPF_PT_NOCONV || stt == HOPF_PT_NONFINITE) Tv = NAN;
    }
    T_out[q] = Tv;
  }
  if (gap_out) gap_out[q] = (Pv - Dv) / fmax(1.0, fabs(Dv));
  if (philo) philo[q] = -Pv;
  if (phihi) phihi[q] = -Dv;
  if (lam_out) {
    const bool f64 = st.s64 != nullptr && st.s64[p] != 0;
    for (int i = 0; i < S.n; ++i) {
      double v = 0.0;
      if (S.U)   // lam = U lam' (back to the caller's coordinates)
        for (int j = 0; j < S.n; ++j)
          v += S.U[(size_t)i * S.n + j] * (f64 ? st.lam64[p * S.n_pad + j] : (double)st.lam[p * S.n_pad + j]);
      else
        v = f64 ? st.lam64[p * S.n_pad + i] : (double)st.lam[p * S.n_pad + i];
      lam_out[q * ls + i] = v;
    }
  }
  if (probes_out) probes_out[q] = st.probes[p];
  if (iters_out) iters_out[q] = st.iters_tot[p];
  status_out[q] = stt;
}

// ------------------------------------------------------------------ Kronecker-structured systems

// A system of k copies of one b-dimensional system that share the control
// (A = I_k (x) A_b, B = 1_k (x) B_b, c = 1_k (x) c_b, target blocks W_b / a_c)
// has x_c(t) = e^{t A_b} x_c + z(u) for every copy c, so with m_c =
// e^{t A_b} x_c - c_b, a = sum_c a_c and the weighted mean mean = sum_c a_c m_c / a
//   sum_c a_c |m_c + z|^2_{W_b^-1} = a |mean + z|^2_{W_b^-1} + sum_c a_c |m_c - mean|^2_{W_b^-1}
// and phi(x, t) = phi_red(weighted mean of the copies, t) + spread: phi_red the
// value of the b-dimensional system with target matrix W_b / a, spread =
// (1/2) sum_c a_c |e^{t A_b}(x_c - mean)|^2_{W_b^-1}.  The minimiser per copy is
// lambda_c = a_c (W_b^-1 e^{t A_b}(x_c - mean) + lambda_red / a).
// wts = [1 / diag(W_b) (b) | a_c (k)].

// x0 of the reduced solve: the weighted mean of point q's k blocks
__global__ void k_kron_pack(const double *__restrict__ x, double *__restrict__ x0, long npts, int k, int b,
                            int n_pad, int xs, const int *__restrict__ idx, const double *__restrict__ wts,
                            double atot) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npts * n_pad) return;
  const long p = i / n_pad;
  const int r = (int)(i % n_pad);
  if (r >= b) { x0[i] = 0.0; return; }
  const long q = idx ? idx[p] : p;
  double s = 0.0;
  for (int c = 0; c < k; ++c) s += wts[b + c] * x[q * xs + (long)c * b + r];
  x0[i] = s / atot;
}

// v <- e^{T A} v for a system of at most KRON_BMAX states, from its probe-setup
// tables (the horizon split, binary node powers, base-16 remainder digits and
// the Taylor series of the probe setup)
__device__ void small_expm_apply(const SysView &S, double T, double *v) {
  const int n = S.n;
  const double q = T / S.h;
  const double qr = rint(q);
  int M;
  double r;
  if (fabs(q - qr) <= 1e-12 * fmax(1.0, q)) { M = (int)qr; r = 0.0; }
  else { M = (int)floor(q); r = T - M * S.h; }
  const int Mmax = S.quad == HOPF_Q_TRAP ? S.N - 1 : S.N;
  if (M > Mmax) { M = Mmax; r = 0.0; }
  double w[KRON_BMAX];
  auto apply = [&](const double *Ec) {   // v <- E v, E stored by columns
    for (int i = 0; i < n; ++i) {
      double a = 0.0;
      for (int k2 = 0; k2 < n; ++k2) a += Ec[(size_t)k2 * n + i] * v[k2];
      w[i] = a;
    }
    for (int i = 0; i < n; ++i) v[i] = w[i];
  };
  for (int bb = 0; bb < S.n_hbin; ++bb)
    if ((M >> bb) & 1) apply(S.hbin + (size_t)bb * n * n);
  if (r > 0.0) {
    const long qd = (long)floor(r / S.dr);
    const long qdig = qd > 4095 ? 4095 : (qd < 0 ? 0 : qd);
    for (int lv = 0; lv < RDIG_LEVELS; ++lv) {
      const int d = (int)((qdig >> (4 * lv)) & 15);
      if (d) apply(S.rdig + ((size_t)lv * 15 + (d - 1)) * n * n);
    }
    const double rho = r - (double)qdig * S.dr;
    if (rho > 0.0) {   // e^{rho A} v = sum_k (rho A)^k v / k!
      double term[KRON_BMAX], sum[KRON_BMAX];
      for (int i = 0; i < n; ++i) term[i] = sum[i] = v[i];
      const double a = rho * S.anorm;
      double bound = 1.0;
      for (int kk = 1; kk <= 30; ++kk) {
        for (int i = 0; i < n; ++i) {
          double acc = 0.0;
          for (int k2 = 0; k2 < n; ++k2) acc += S.At[(size_t)k2 * n + i] * term[k2];
          w[i] = acc * (rho / kk);
        }
        for (int i = 0; i < n; ++i) { term[i] = w[i]; sum[i] += w[i]; }
        bound *= a / kk;
        if (bound < 1e-17) break;
      }
      for (int i = 0; i < n; ++i) v[i] = sum[i];
    }
  }
}

// The copies' spread s(T) = (1/2) sum_c a_c |e^{T A_b}(x_c - mean)|^2_{W_b^-1}
// and ds/dT = sum_c a_c (e^{T A_b} d_c)^T W_b^-1 A_b e^{T A_b} d_c of the
// minimum-time search on a reduced system, at the horizon of every point on
// the setup list (from_list), or at T = 0 for every point (before k_init).
__global__ void k_kron_spread(SysView S, PtState st, const double *__restrict__ x, int k,
                              const double *__restrict__ wts, const int *__restrict__ idx, int xs, int from_list) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (from_list ? (long)st.counters[1] : st.npts)) return;
  const long p = from_list ? (long)st.setup_list[i] : i;
  const long q = idx ? idx[p] : p;
  const int b = S.n, np = S.n_pad;
  const double T = from_list ? st.T[p] : 0.0;
  double s = 0.0, ds = 0.0;
  if (isfinite(T))
    for (int c = 0; c < k; ++c) {
      const double ac = wts[b + c];
      double d[KRON_BMAX];
      for (int r = 0; r < b; ++r) d[r] = x[q * xs + (long)c * b + r] - st.x0[p * np + r];
      if (T > 0.0) small_expm_apply(S, T, d);
      for (int r = 0; r < b; ++r) {
        double ad = 0.0;   // (A_b e^{T A_b} d_c)_r, A_b stored by columns
        for (int j = 0; j < b; ++j) ad += S.At[(size_t)j * b + r] * d[j];
        s += 0.5 * ac * wts[r] * d[r] * d[r];
        ds += ac * wts[r] * d[r] * ad;
      }
    }
  st.kspread[p] = s;
  st.kdspread[p] = ds;
}

// outputs of a reduced solve in the full system's terms (one thread per
// point): value bounds with the spread added and the copies' costates; a
// minimum-time call takes the costates at the final horizon (the last scan
// horizon for unreachable points) and its other outputs from k_outputs
__global__ void k_kron_outputs(SysView S, PtState st, const double *__restrict__ x, int k,
                               const double *__restrict__ wts, double atot, double *philo, double *phihi,
                               double *lam_out, int *iters_out, int *status_out, const int *__restrict__ idx,
                               int xs, int min_time) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= st.npts) return;
  const long q = idx ? idx[p] : p;
  const int b = S.n, np = S.n_pad;
  double T = st.T[p];
  if (min_time) {
    if (!isfinite(T)) T = st.status[p] == HOPF_PT_UNREACH ? S.t_max : 0.0;
    if (!lam_out) return;
  }
  const bool f64 = st.s64 != nullptr && st.s64[p] != 0;
  double mean[KRON_BMAX], lred[KRON_BMAX];
  for (int r = 0; r < b; ++r) {
    mean[r] = st.x0[p * np + r];
    lred[r] = f64 ? st.lam64[p * np + r] : (double)st.lam[p * np + r];
  }
  double spread = 0.0;
  for (int c = 0; c < k; ++c) {
    const double ac = wts[b + c];
    double d[KRON_BMAX];
    for (int r = 0; r < b; ++r) d[r] = x[q * xs + (long)c * b + r] - mean[r];
    small_expm_apply(S, T, d);
    for (int r = 0; r < b; ++r) {
      spread += 0.5 * ac * wts[r] * d[r] * d[r];
      if (lam_out) lam_out[q * xs + (long)c * b + r] = ac * (wts[r] * d[r] + lred[r] / atot);
    }
  }
  if (min_time) return;
  if (philo) philo[q] = -st.P[p] + spread;
  if (phihi) phihi[q] = -st.D[p] + spread;
  if (iters_out) iters_out[q] = st.iters_tot[p];
  status_out[q] = st.status[p];
}

// ------------------------------------------------------------------ host orchestration

namespace {

template <typename T>
T *grow(std::vector<Ctx::Buf> &bufs, int idx, size_t count) {
  if ((int)bufs.size() <= idx) bufs.resize(idx + 1);
  auto &b = bufs[idx];
  const size_t bytes = std::max<size_t>(count * sizeof(T), 256);
  if (b.bytes < bytes) {
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) return nullptr;
    b.bytes = bytes;
  }
  return reinterpret_cast<T *>(b.p);
}

// Per-point state layout (same for every call with the same system sizes;
// row npts of lam/lamb/xfc32/y is a spare row that lanes without a point
// read and write).  The allocator hands out typed arrays in a fixed order:
// GrowAlloc from the context's reusable buffers (grown with hipMalloc when a
// call needs more), ArenaAlloc from one fixed block without allocating.
struct GrowAlloc {
  std::vector<Ctx::Buf> &bufs;
  int bi = 0;
  template <typename T> T *get(size_t count) { return grow<T>(bufs, bi++, count); }
};
struct ArenaAlloc {
  unsigned char *base;           // nullptr: only count the bytes (the arrays are never touched)
  size_t cap, used = 0;
  template <typename T> T *get(size_t count) {
    const size_t bytes = (std::max<size_t>(count * sizeof(T), 1) + 255) & ~(size_t)255;
    if (used + bytes > cap) { used = cap + 1; return nullptr; }
    static T dummy;
    T *p = base ? reinterpret_cast<T *>(base + used) : &dummy;
    used += bytes;
    return p;
  }
};

template <class Alloc>
bool layout_state(Alloc &al, const SysTables &tab, long npts, PtState &st, bool with_lam0, bool fp64,
                  bool kron_spread = false) {
  const int np = tab.n_pad, m = tab.m;
  st = PtState{};
  st.npts = npts;
  st.ystride = tab.nkb * m * NODE_BLOCK;
  st.mpad = ((m + 3) / 4) * 4;
  st.x0 = al.template get<double>(npts * np);
  st.status = al.template get<int>(npts);
  st.phase = al.template get<int>(npts);
  st.flags = al.template get<int>(npts);
  st.probes = al.template get<int>(npts);
  st.iters_tot = al.template get<int>(npts);
  st.iters_probe = al.template get<int>(npts);
  st.rows = al.template get<int>(npts);
  st.M = al.template get<int>(npts);
  st.partial = al.template get<int>(npts);
  st.nscan = al.template get<int>(npts);
  st.ncell = al.template get<int>(npts);
  st.newt = al.template get<int>(npts);
  st.wbef = al.template get<double>(npts);
  st.ha = al.template get<double>(npts);
  st.hb = al.template get<double>(npts);
  st.T = al.template get<double>(npts);
  st.lo = al.template get<double>(npts);
  st.hi = al.template get<double>(npts);
  st.r = al.template get<double>(npts);
  st.tau = al.template get<double>(npts);
  st.sig = al.template get<double>(npts);
  st.P = al.template get<double>(npts);
  st.D = al.template get<double>(npts);
  st.xf = al.template get<double>(npts * np);
  st.axf = al.template get<double>(npts * np);
  st.xfc32 = al.template get<float>((npts + 1) * np);
  const bool trap = tab.desc.quad == HOPF_Q_TRAP;
  st.R64 = al.template get<double>(trap ? npts * m * np : 1);
  st.R32 = al.template get<float>(trap ? npts * m * np : 1);
  st.lam = al.template get<float>((npts + 1) * np);
  st.lamb = al.template get<float>((npts + 1) * np);
  st.y = al.template get<float>((size_t)(npts + 1) * st.ystride);
  st.yR = al.template get<float>(npts * st.mpad);
  st.perm = al.template get<int>(npts);
  st.setup_list = al.template get<int>(npts);
  st.stage = al.template get<int>(npts);
  st.esc = al.template get<int>(npts);
  st.lamref = al.template get<float>(npts * np);
  if (fp64) {   // the FP64 iterate (spare row included)
    st.lam64 = al.template get<double>((npts + 1) * np);
    st.lamb64 = al.template get<double>((npts + 1) * np);
    st.y64 = al.template get<double>((size_t)(npts + 1) * st.ystride);
    st.yR64 = al.template get<double>(npts * st.mpad);
    st.s64 = al.template get<int>(npts);
    if (!st.lam64 || !st.lamb64 || !st.y64 || !st.yR64 || !st.s64) return false;
  }
  st.yref = al.template get<float>((size_t)npts * st.ystride);
  st.bT = al.template get<float>(npts);
  st.bD = al.template get<float>(npts);
  st.counters = al.template get<int>(4);
  st.rowsum = al.template get<double>(3);   // [0] 16-point rounds, [1] tail solver, [2] 64-point rounds
  st.lam0s = nullptr;
  if (with_lam0 && !(st.lam0s = al.template get<double>(npts * np))) return false;
  if (kron_spread &&
      (!(st.kspread = al.template get<double>(npts)) || !(st.kdspread = al.template get<double>(npts))))
    return false;
  return st.x0 && st.status && st.phase && st.flags && st.probes && st.iters_tot && st.iters_probe &&
         st.rows && st.M && st.partial && st.nscan && st.ncell && st.newt && st.wbef && st.ha && st.hb && st.T &&
         st.lo && st.hi && st.r && st.tau && st.sig && st.P && st.D && st.xf && st.axf && st.xfc32 && st.R64 &&
         st.R32 && st.lam && st.lamb && st.y && st.yR && st.perm && st.setup_list && st.stage && st.esc &&
         st.lamref && st.yref && st.bT && st.bD && st.counters && st.rowsum;
}

// Point state of job `job` in the context's reusable buffers.
bool make_state(Ctx *ctx, int job, const SysTables &tab, long npts, PtState &st, bool with_lam0,
                bool kron_spread = false) {
  if ((int)ctx->jbufs.size() <= job) ctx->jbufs.resize(job + 1);
  GrowAlloc al{ctx->jbufs[job]};
  if (!layout_state(al, tab, npts, st, with_lam0, ctx->opts.prec == HOPF_FP64, kron_spread)) return false;
  st.log_pt = ctx->log_pt;
  st.log_T = ctx->log_T;
  st.log_lam = ctx->log_lam;
  st.log_cap = (int)std::min<long>(ctx->log_cap, 2000000000L);
  return true;
}

SysView view(const SysTables &t) {
  SysView v;
  v.n = t.n; v.m = t.m; v.N = t.N; v.n_pad = t.n_pad; v.nkb = t.nkb;
  v.quad = t.desc.quad; v.uset = t.desc.uset;
  v.t_max = t.desc.t_max; v.h = t.h; v.delta = t.delta; v.c_tau = t.desc.c_tau;
  v.K32 = t.K32; v.K64 = t.K64; v.K32T = t.K32T; v.K64T = t.K64T;
  v.Kd16h = t.Kd16h; v.Kd16l = t.Kd16l; v.Kp16h = t.Kp16h; v.Kp16l = t.Kp16l; v.lpref = t.lpref_d; v.epow = t.epow_d;
  v.A = t.A_d; v.BQ = t.BQ_d; v.Wd = t.Wd_d; v.c = t.c_d;
  v.Eh = t.Eh_d; v.Qu = t.Qu_d; v.m_user = t.m_user;
  v.n_hbin = t.n_hbin; v.dr = t.dr; v.anorm = t.anorm; v.hbin = t.hbin_d; v.rdig = t.rdig_d; v.At = t.At_d;
  v.U = t.rotated ? t.U_d : nullptr;
  return v;
}

#define HIPCHK(x)                                                                            \
  do {                                                                                       \
    hipError_t e_ = (x);                                                                     \
    if (e_ != hipSuccess) return set_err(ctx, HOPF_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

namespace {

// One system's share of a call: its points, kernels, point state and stream.
struct Job {
  int sid = 0;
  const SysTables *tab = nullptr;
  const SysTables *kron = nullptr;   // solve of a Kronecker-structured system: its full tables
                                     // (tab is then the reduced system's)
  const double *kx = nullptr;        // the call's x (the copies), for the spread of a minimum-time search
  int kxs = 0;
  SysView S{};
  pdhg_fn fp = nullptr, fp32_esc = nullptr;
  pdhg_fn fw = nullptr;          // 64-point LDS-staged FP32 iterations (nullptr: none for this shape)
  pdhg_fn fd = nullptr;          // 16-point FP32 iterations on 8 waves (few tiles)
  pdhg_fn fsw = nullptr;         // 64-point streaming iterations (FP32 or BF16 hi+lo)
  pdhg_fn fsw32 = nullptr;       // 64-point FP32 streaming iterations of escalated BF16 points
  SetupWavesFn fs = nullptr;     // probe setups without the network
  cert_fn fc = nullptr;
  size_t lds_pdhg = 0, lds_esc = 0, lds_cert = 0, lds_wide = 0, lds_setup = 0, lds_deep = 0, lds_swide = 0,
         lds_swide32 = 0;
  long last_active = 0;          // active points at the last check read (picks the iteration kernel)
  PtState st{};
  long npts = 0;
  const int *idx = nullptr;      // device: job point -> caller's point (nullptr: identity)
  hipStream_t s = nullptr;
  unsigned ngrid = 0;
  long rounds = 0, max_rounds = 0;
  int *hcount = nullptr;         // pinned: active count of the last check of each group slot
  hipEvent_t gev[2] = {nullptr, nullptr};   // completion of the two most recent round groups
  int ngroups = 0, gdone = 0;    // groups issued / groups whose count was read
  bool done = false;
  MlpView mv{};
  std::vector<hipEvent_t> kev;
  std::vector<char> kwide;   // per timed round: the 64-point kernel ran it
  bool tail_ok = false;          // FP32 iterations: the tail solver may take over
  bool parked = false;           // waiting for the combined tail launch
  hipEvent_t park_ev = nullptr;
  long tail_points = 0;
  bool timed = true;             // timing events and the asynchronous round checks (off: no runtime objects made)
};

constexpr int GROUP_ROUNDS = 4;   // rounds between active-count checks

// Kernel choice and LDS sizes for one system at the requested precision.
hopf_status plan_job(Ctx *ctx, Job &J) {
  const SysTables &tab = *J.tab;
  const hopf_opts &ho = ctx->opts;
  const int NT = tab.n_pad / 16;
  int MMc = 0;
  // register-resident kernel where an instance exists (FP32/FP64, small m
  // and n), the streaming kernel otherwise and for BF16 hi+lo
  bool streaming = false;
  if (ho.prec != HOPF_BF16X3) J.fp = pdhg_lookup(NT, tab.m, ho.prec, WAVES, &MMc);
  if (!J.fp && ho.prec != HOPF_FP64) {
    J.fp = stream_lookup(NT, ho.prec == HOPF_BF16X3 ? 1 : 0);
    streaming = true;
  }
  J.fc = cert_lookup(NT);
  if (!J.fp || !J.fc)
    return set_err(ctx, HOPF_EUNSUPPORTED, "no kernel instance for n=" + std::to_string(tab.n) + ", m=" +
                                               std::to_string(tab.m) + " at this precision");
  const size_t elt = ho.prec == HOPF_FP64 ? 8 : 4;
  const int mpad = ((tab.m + 3) / 4) * 4;
  const size_t lds_stream =
      ((size_t)(WAVES - 1) * 4 * 4 * 64 + (size_t)NT * 4 * 64 + 32 * (size_t)tab.n_pad + 16 * (size_t)mpad) * 4;
  if (streaming)   // cross-wave G chunks + broadcast of sigma*lam_bar + private-node scratch
    J.lds_pdhg = lds_stream;
  else             // double-buffered cross-wave G sums + the private-node scratch
    J.lds_pdhg = (size_t)2 * WAVES * NT * 4 * 64 * elt + (size_t)(2 * 16 * tab.n_pad + 16 * MMc) * elt;
  // certificate: G chunks, sigma sums, private-node scratch
  J.lds_cert = (size_t)(WAVES - 1) * 2 * 4 * 64 * 8 + (size_t)WAVES * 64 * 8 + (size_t)16 * tab.n_pad * 4 +
               (size_t)16 * tab.n_pad * 8 + (size_t)16 * mpad * 8;
  if (J.lds_pdhg > 150 * 1024 || J.lds_cert > 150 * 1024)
    return set_err(ctx, HOPF_EUNSUPPORTED, "system too large for the LDS tiling of the kernels");
  if (ho.prec == HOPF_BF16X3 && !tab.Kd16h) return set_err(ctx, HOPF_ESTATE, "BF16 tables missing");
  if (ho.prec == HOPF_FP32 && !streaming && ho.wide_min > 0) {
    J.fw = wide_lookup(NT, tab.m);
    if (J.fw) {
      J.lds_wide = (size_t)NODE_BLOCK * MMc * wide_row_stride(NT) * sizeof(float);
      HIPCHK(hipFuncSetAttribute((const void *)J.fw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_wide));
    }
  }
  // large m or n: the streaming iteration on 64-point workgroups
  if (streaming && ho.wide_min > 0) {
    J.fsw = swide_lookup(NT, ho.prec == HOPF_BF16X3 ? 1 : 0);
    J.lds_swide = swide_lds_bytes(NT, ho.prec == HOPF_BF16X3);
    if (J.fsw && J.lds_swide <= 150 * 1024)
      HIPCHK(hipFuncSetAttribute((const void *)J.fsw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_swide));
    else
      J.fsw = nullptr;
    if (J.fsw && ho.prec == HOPF_BF16X3) {
      J.fsw32 = swide_lookup(NT, 0);
      J.lds_swide32 = swide_lds_bytes(NT, false);
      if (J.fsw32)
        HIPCHK(hipFuncSetAttribute((const void *)J.fsw32, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)J.lds_swide32));
    }
  }
  // BF16 hi+lo: points that stall are escalated to an FP32 kernel
  if (ho.prec == HOPF_BF16X3) {
    int mm2 = 0;
    J.fp32_esc = pdhg_lookup(NT, tab.m, HOPF_FP32, WAVES, &mm2);
    if (J.fp32_esc) J.lds_esc = (size_t)2 * WAVES * NT * 4 * 64 * 4 + (size_t)(2 * 16 * tab.n_pad + 16 * mm2) * 4;
    else {
      J.fp32_esc = stream_lookup(NT, 0);
      J.lds_esc = lds_stream;
    }
    HIPCHK(hipFuncSetAttribute((const void *)J.fp32_esc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_esc));
  }
  HIPCHK(hipFuncSetAttribute((const void *)J.fp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_pdhg));
  // launches with at most one tile per compute unit: the tile's node blocks
  // over 8 waves
  if (ho.prec == HOPF_FP32 && !streaming) {
    int mm3 = 0;
    J.fd = pdhg_lookup(NT, tab.m, HOPF_FP32, 8, &mm3);
    J.lds_deep = (size_t)2 * 8 * NT * 4 * 64 * 4 + (size_t)(2 * 16 * tab.n_pad + 16 * mm3) * 4;
    if (J.fd && J.lds_deep <= 150 * 1024)
      HIPCHK(hipFuncSetAttribute((const void *)J.fd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_deep));
    else
      J.fd = nullptr;
  }
  HIPCHK(hipFuncSetAttribute((const void *)J.fc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_cert));
  J.fs = setup_waves_for(tab.n);
  J.lds_setup = (size_t)4 * tab.n_pad * (tab.n <= 128 ? setup_cw<64, 1>() : setup_cw<64, 3>()) * sizeof(double);
  HIPCHK(hipFuncSetAttribute((const void *)J.fs, hipFuncAttributeMaxDynamicSharedMemorySize, (int)J.lds_setup));
  return HOPF_OK;
}

// Probe setups of the points on the setup list: one wave per point, or one
// workgroup per point when a network gives the warm start.
void launch_setup(const Job &J, const Opts &o) {
  const bool net = J.mv.valid && o.warm == HOPF_WARM_MLP_LAM;
  if (net)
    k_setup<<<(unsigned)std::min<long>(J.npts, 2048), 256, 0, J.s>>>(J.S, J.st, o, J.mv);
  else
    J.fs<<<(unsigned)std::min<long>((J.npts + 3) / 4, 4096), 256, J.lds_setup, J.s>>>(J.S, J.st, o);
}

// Timing events come from a pool the context keeps (created on first use,
// reused by later calls, destroyed with the context).
hipEvent_t take_event(Ctx *ctx) {
  if (ctx->ev_used == ctx->evpool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->evpool.push_back(e);
  }
  return ctx->evpool[ctx->ev_used++];
}

// Queue one group of rounds and an active-count check whose result lands in
// hcount[2 slot .. 2 slot + 1] when gev[slot] fires.  A round: probe setups,
// tile formation, the FP64 certificate of every active point (the starting
// point of a fresh probe, else the iterate after the last iterations) with
// the search step, tile formation without the points that now wait for a
// setup, then check_every fused iterations.
hopf_status issue_group(Ctx *ctx, Job &J, const Opts &o, int mode) {
  const hopf_opts &ho = ctx->opts;
  const hipStream_t s = J.s;
  for (int r = 0; r < GROUP_ROUNDS && J.rounds < J.max_rounds; ++r) {
    launch_setup(J, o);
    if (J.kx)   // the copies' spread at the new horizons (the setup list is still set)
      k_kron_spread<<<(unsigned)((J.npts + 255) / 256), 256, 0, s>>>(J.S, J.st, J.kx, J.kron->kron_k,
                                                                      J.kron->kron_winv_d, J.idx, J.kxs, 1);
    k_sort<<<1, 1024, 0, s>>>(J.st, J.tab->N, 1, 0);
    J.fc<<<J.ngrid, THREADS, J.lds_cert, s>>>(J.S, J.st, o, mode);
    const bool wide = (J.fw || J.fsw) && J.last_active >= ho.wide_min;
    k_sort<<<1, 1024, 0, s>>>(J.st, J.tab->N, 0, wide ? 2 : 1);
    hipEvent_t a = nullptr, b = nullptr;
    if (J.timed) {
      a = take_event(ctx);
      b = take_event(ctx);
      if (!a || !b) return set_err(ctx, HOPF_EDEVICE, "hipEventCreate failed");
      HIPCHK(hipEventRecord(a, s));
    }
    if (J.fp32_esc) {   // escalated BF16 points (sorted first) in FP32
      if (wide && J.fsw32)
        J.fsw32<<<(unsigned)((J.npts + WIDE_PTS - 1) / WIDE_PTS), THREADS, J.lds_swide32, s>>>(J.S, J.st,
                                                                                               ho.check_every, 0);
      else
        J.fp32_esc<<<J.ngrid, THREADS, J.lds_esc, s>>>(J.S, J.st, ho.check_every, 0);
    }
    if (wide) {
      const unsigned wgrid = (unsigned)((J.npts + WIDE_PTS - 1) / WIDE_PTS);
      if (J.fw) J.fw<<<wgrid, THREADS, J.lds_wide, s>>>(J.S, J.st, ho.check_every, J.fp32_esc ? 1 : 2);
      else J.fsw<<<wgrid, THREADS, J.lds_swide, s>>>(J.S, J.st, ho.check_every, J.fp32_esc ? 1 : 2);
    } else if (J.fd && J.last_active <= (ho.deep_max < 0 ? (long)PTS_TILE * ctx->n_cu : (long)ho.deep_max)) {
      J.fd<<<J.ngrid, 8 * 64, J.lds_deep, s>>>(J.S, J.st, ho.check_every, 2);
    } else {
      J.fp<<<J.ngrid, THREADS, J.lds_pdhg, s>>>(J.S, J.st, ho.check_every, J.fp32_esc ? 1 : 2);
    }
    if (J.timed) {
      HIPCHK(hipEventRecord(b, s));
      J.kev.push_back(a);
      J.kev.push_back(b);
      J.kwide.push_back(wide ? 1 : 0);
    }
    ctx->iter_launches++;
    ++J.rounds;
  }
  if (!J.timed) return HOPF_OK;   // the caller reads the counters itself
  // active points after the last certificate, and points waiting for a setup
  const int slot = J.ngroups & 1;
  HIPCHK(hipMemcpyAsync(J.hcount + 2 * slot, J.st.counters, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(J.gev[slot], s));
  ++J.ngroups;
  return HOPF_OK;
}

// Park the job for the tail solver: consume pending probe setups and sort its
// (at most `count`) active points; the combined tail launch picks them up.
hopf_status park_job(Ctx *ctx, Job &J, const Opts &o, long count) {
  const hipStream_t s = J.s;
  launch_setup(J, o);
  k_sort<<<1, 1024, 0, s>>>(J.st, J.tab->N, 1, 0);
  if (J.timed) {
    J.park_ev = take_event(ctx);
    if (!J.park_ev) return set_err(ctx, HOPF_EDEVICE, "hipEventCreate failed");
    HIPCHK(hipEventRecord(J.park_ev, s));
  }
  J.parked = true;
  J.tail_points = count;
  return HOPF_OK;
}

}  // namespace

// Solve every point of the call.  Points are grouped by system into jobs;
// each job runs its own rounds (probe setup, tile formation, check_every
// fused iterations, FP64 certificate and bisection step) until all of its
// points are done.  A single-system call runs on the caller's stream; a
// multi-system call runs its jobs on a pool of streams and interleaves their
// rounds from this thread, keeping up to two round groups of each job in
// flight so that the device does not wait for the host's checks.
hopf_status solve_dev(Ctx *ctx, int mode, long npts, const int *sys_id, const double *x,
                      const double *t_in, const double *lam0, const double *t_bracket, double *T_out,
                      double *gap_out, double *philo_out, double *phihi_out, double *lam_out,
                      int *probes_out, int *iters_out, int *status_out, hipStream_t user_stream) {
  if (ctx->sys.empty()) return set_err(ctx, HOPF_ESTATE, "no systems set");
  if (npts < 0) return set_err(ctx, HOPF_EINVAL, "npts < 0");
  if (!status_out || !x) return set_err(ctx, HOPF_EINVAL, "x and pt_status are required");
  if (npts == 0) return HOPF_OK;
  if (npts > (1L << 26)) return set_err(ctx, HOPF_EINVAL, "too many points in one call");
  const int nsys = (int)ctx->sys.size();
  hipStream_t base = user_stream ? user_stream : ctx->stream;
  // ---- group the points by system (counting sort on the host)
  std::vector<long> cnt(nsys, 0), off(nsys + 1, 0);
  std::vector<int> ids;
  if (sys_id) {
    ids.resize(npts);
    HIPCHK(hipMemcpyAsync(ids.data(), sys_id, npts * sizeof(int), hipMemcpyDeviceToHost, base));
    HIPCHK(hipStreamSynchronize(base));
    for (long i = 0; i < npts; ++i) {
      if (ids[i] < 0 || ids[i] >= nsys) return set_err(ctx, HOPF_EINVAL, "sys_id out of range");
      cnt[ids[i]]++;
    }
  } else {
    cnt[0] = npts;
  }
  int xs = 0;      // row stride of x and lam: the largest n among the systems used
  std::vector<int> used;
  for (int k = 0; k < nsys; ++k)
    if (cnt[k] > 0) {
      used.push_back(k);
      xs = std::max(xs, ctx->sys[k].n);
    }
  for (int k = 0; k < nsys; ++k) off[k + 1] = off[k] + cnt[k];
  const int nj = (int)used.size();
  int *d_idx = nullptr;
  if (nj > 1) {
    std::vector<int> order(npts);
    std::vector<long> pos(off.begin(), off.end() - 1);
    for (long i = 0; i < npts; ++i) order[pos[ids[i]]++] = (int)i;
    if ((int)ctx->jbufs.size() < nj + 1) ctx->jbufs.resize(nj + 1);
    d_idx = grow<int>(ctx->jbufs[nj], 0, npts);
    if (!d_idx) return set_err(ctx, HOPF_ENOMEM, "index buffer");
    HIPCHK(hipMemcpyAsync(d_idx, order.data(), npts * sizeof(int), hipMemcpyHostToDevice, base));
    HIPCHK(hipStreamSynchronize(base));
  }
  // ---- streams: the caller's for one job, the pool (and the caller's) otherwise
  const int NPOOL = 4;
  if (nj > 1)
    while ((int)ctx->pool.size() < NPOOL) {
      hipStream_t ps = nullptr;
      HIPCHK(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
      ctx->pool.push_back(ps);
    }
  const hopf_opts &ho = ctx->opts;
  Opts o{ho.c_tau, ho.gap_tol, ho.t_rel_tol, ho.t_abs_frac, ho.max_iter, ho.check_every, ho.warm, ho.prec, 4000,
         ho.root, ho.newton_after, ho.newton_rho, ho.adapt, ho.scan};
  // a search takes at most scan + 64 probes (scan horizons, then a cell whose
  // width halves at least every two probes, two hints and the final solve)
  const int max_probes = ho.scan + 64;
  ctx->ev_used = 0;
  hipEvent_t e0 = take_event(ctx), e1 = take_event(ctx), ebase = take_event(ctx);
  if (!e0 || !e1 || !ebase) return set_err(ctx, HOPF_EDEVICE, "hipEventCreate failed");
  HIPCHK(hipEventRecord(e0, base));
  HIPCHK(hipEventRecord(ebase, base));
  std::vector<Job> jobs(nj);
  // pinned host words for the round checks: 2 slots x (active, pending setups) per job
  if (ctx->hcount_cap < 4L * nj) {
    if (ctx->hcount) hipHostFree(ctx->hcount);
    ctx->hcount = nullptr;
    ctx->hcount_cap = 0;
    HIPCHK(hipHostMalloc((void **)&ctx->hcount, 4L * nj * sizeof(int), hipHostMallocDefault));
    ctx->hcount_cap = 4L * nj;
  }
  int *hcount = ctx->hcount;
  hopf_status rc = HOPF_OK;
  ctx->iter_launches = 0;
  for (int j = 0; j < nj && rc == HOPF_OK; ++j) {
    Job &J = jobs[j];
    J.sid = used[j];
    J.tab = &ctx->sys[J.sid];
    J.S = view(*J.tab);
    // value solves, and minimum-time searches without a caller's lam0 (whose
    // rows are the copies'), of a Kronecker-structured system
    if (ho.structure && J.tab->kron_red >= 0 && (mode == MODE_VALUE || (mode == MODE_MINTIME && !lam0))) {
      // the reduced system of the copies' weighted mean; with equal weights
      // its step ratio sqrt(k) c_tau makes its iterates those of the full
      // system (||K||^2 is k times the reduced one's, and the reduced costate
      // is the sum of the copies'); with unequal weights the same ratio is a
      // choice of step only (the certified result does not depend on it)
      J.kron = J.tab;
      J.tab = &ctx->ksys[J.kron->kron_red];
      J.S = view(*J.tab);
      const double ct = J.kron->desc.c_tau > 0.0 ? J.kron->desc.c_tau : ho.c_tau;
      J.S.c_tau = std::sqrt((double)J.kron->kron_k) * ct;
      if (mode == MODE_MINTIME) {
        J.kx = x;
        J.kxs = nj > 1 ? xs : J.kron->n;
      }
    }
    J.npts = cnt[J.sid];
    J.idx = nj > 1 ? d_idx + off[J.sid] : nullptr;
    J.s = nj > 1 ? ctx->pool[j % NPOOL] : base;
    J.ngrid = (unsigned)((J.npts + PTS_TILE - 1) / PTS_TILE);
    J.last_active = J.npts;
    J.max_rounds = (long)(ho.max_iter / ho.check_every + 3) * (max_probes + 2);
    J.hcount = hcount + 4 * j;
    // (the tail solver's in-kernel probe setup has no spread term)
    J.tail_ok = ho.prec == HOPF_FP32 && J.tab->n_pad <= 256 && J.tab->m <= 64 && !J.kx;
    if ((rc = plan_job(ctx, J)) != HOPF_OK) break;
    const bool net = (ho.warm == HOPF_WARM_MLP || ho.warm == HOPF_WARM_MLP_LAM || ho.warm == HOPF_WARM_MLP_FIRST) &&
                     J.sid < (int)ctx->mlp.size() && ctx->mlp[J.sid].valid && !J.kron;
    if (!make_state(ctx, j, *J.tab, J.npts, J.st, (lam0 != nullptr && mode == MODE_MINTIME) || net, J.kx != nullptr)) {
      rc = set_err(ctx, HOPF_ENOMEM, "device allocation of the point state failed");
      break;
    }
    for (int k = 0; k < 2 && rc == HOPF_OK; ++k)
      if (!(J.gev[k] = take_event(ctx))) rc = set_err(ctx, HOPF_EDEVICE, "event");
    if (rc != HOPF_OK) break;
    if (J.s != base && hipStreamWaitEvent(J.s, ebase, 0) != hipSuccess) {
      rc = set_err(ctx, HOPF_EDEVICE, "stream wait");
      break;
    }
    if (net) {
      const MlpState &w = ctx->mlp[J.sid];
      J.mv = MlpView{w.theta, w.xm, w.xs, w.t_scale, w.lam_scale, w.n, w.H, 1};
    }
    const PtState &st = J.st;
    const long np_ = J.npts;
    const hipStream_t s = J.s;
    const long tot = np_ * J.tab->n_pad;
    const int ls = nj > 1 ? xs : (J.kron ? J.kron->n : J.tab->n);     // row stride of x, lam0 and lam
    k_clear<<<1, 64, 0, s>>>(st);
    if (J.kron) {
      k_kron_pack<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(x, st.x0, np_, J.kron->kron_k, J.kron->kron_b,
                                                                 J.tab->n_pad, ls, J.idx, J.kron->kron_winv_d,
                                                                 J.kron->kron_atot);
      if (J.kx)   // the spread at T = 0 decides which points start inside the target
        k_kron_spread<<<(unsigned)((np_ + 255) / 256), 256, 0, s>>>(J.S, st, J.kx, J.kron->kron_k,
                                                                     J.kron->kron_winv_d, J.idx, J.kxs, 0);
    } else {
      k_pack<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(x, st.x0, np_, J.tab->n, J.tab->n_pad, ls, J.idx, J.S.U);
    }
    k_init<<<(unsigned)((np_ + 255) / 256), 256, 0, s>>>(J.S, st, o, mode, t_in, J.idx, lam0, t_bracket, ls);
    // learned start: the network at every point's first probe, batched on
    // the matrix cores (later probes of mode mlp_lam evaluate it in the setup)
    if (net && J.mv.n == J.tab->n && J.mv.H == 256)
      rc = mlp_first_probe(ctx, J.mv, ho.warm, st, np_, J.tab->n_pad, lam0 != nullptr && mode == MODE_MINTIME, s);
  }
  // ---- interleaved rounds: each job keeps up to two groups in flight until
  // its points are done or at most tail_max remain (then it is parked); the
  // parked jobs of the call finish together in one tail launch.
  const long tail_lim = std::min(ho.tail_max, TAIL_MAX_POINTS);
  long live = 0;
  for (int j = 0; j < nj && rc == HOPF_OK; ++j) {
    Job &J = jobs[j];
    if (J.tail_ok && J.npts <= tail_lim) rc = park_job(ctx, J, o, J.npts);   // straight to the tail
    else ++live;
  }
  while (rc == HOPF_OK && live > 0) {
    bool progressed = false;
    for (int j = 0; j < nj && rc == HOPF_OK; ++j) {
      Job &J = jobs[j];
      if (J.done || J.parked) continue;
      // read the oldest outstanding check if it has completed
      if (J.gdone < J.ngroups) {
        const hipError_t q = hipEventQuery(J.gev[J.gdone & 1]);
        if (q == hipSuccess) {
          const int c = J.hcount[2 * (J.gdone & 1)] + J.hcount[2 * (J.gdone & 1) + 1];
          J.last_active = c;
          ++J.gdone;
          progressed = true;
          if (c == 0 || J.rounds >= J.max_rounds) {
            J.done = true;
            --live;
            continue;
          }
          if (J.tail_ok && c <= tail_lim) {
            rc = park_job(ctx, J, o, c);
            --live;
            continue;
          }
        } else if (q != hipErrorNotReady) {
          rc = set_err(ctx, HOPF_EDEVICE, std::string("round check: ") + hipGetErrorString(q));
          break;
        }
      }
      if (J.ngroups - J.gdone < 2 && J.rounds < J.max_rounds) {
        rc = issue_group(ctx, J, o, mode);
        progressed = true;
      }
    }
    if (rc != HOPF_OK) break;
    if (!progressed) {   // every running job has two groups in flight: wait for the oldest check of one
      for (int j = 0; j < nj; ++j)
        if (!jobs[j].done && !jobs[j].parked && jobs[j].gdone < jobs[j].ngroups) {
          if (hipEventSynchronize(jobs[j].gev[jobs[j].gdone & 1]) != hipSuccess)
            rc = set_err(ctx, HOPF_EDEVICE, "round check failed");
          break;
        }
    }
  }
  // ---- the combined tail launch over every parked job
  double tail_s = 0.0;
  long tail_pts = 0;
  {
    std::vector<TailJob> tj;
    long tb = 0;
    size_t lds = 0;
    for (int j = 0; j < nj && rc == HOPF_OK; ++j) {
      Job &J = jobs[j];
      if (!J.parked) continue;
      tj.push_back(TailJob{J.S, J.st, J.mv, tb});
      tb += J.tail_points;
      lds = std::max(lds, tail_lds_bytes(J.tab->m));
      if (hipStreamWaitEvent(base, J.park_ev, 0) != hipSuccess) rc = set_err(ctx, HOPF_EDEVICE, "stream wait");
    }
    if (rc == HOPF_OK && tb > 0) {
      if ((int)ctx->jbufs.size() < nj + 1) ctx->jbufs.resize(nj + 1);
      TailJob *d_tj = grow<TailJob>(ctx->jbufs[nj], 1, tj.size());
      if (!d_tj) rc = set_err(ctx, HOPF_ENOMEM, "tail job table");
      hipEvent_t t0 = take_event(ctx), t1 = take_event(ctx), tdone = take_event(ctx);
      if (rc == HOPF_OK) {
        const bool ok =
            t0 && t1 && tdone &&
            hipMemcpyAsync(d_tj, tj.data(), tj.size() * sizeof(TailJob), hipMemcpyHostToDevice, base) == hipSuccess &&
            hipFuncSetAttribute((const void *)k_tail_multi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) ==
                hipSuccess &&
            hipEventRecord(t0, base) == hipSuccess;
        if (!ok) rc = set_err(ctx, HOPF_EDEVICE, "tail launch setup failed");
      }
      if (rc == HOPF_OK) {
        k_tail_multi<<<(unsigned)tb, 256, lds, base>>>(d_tj, (int)tj.size(), o);
        hipEventRecord(t1, base);
        hipEventRecord(tdone, base);
        for (int j = 0; j < nj; ++j)   // each parked job's outputs wait for the tail
          if (jobs[j].parked && jobs[j].s != base) hipStreamWaitEvent(jobs[j].s, tdone, 0);
        // the host table must outlive the asynchronous copy
        if (hipEventSynchronize(t1) != hipSuccess) rc = set_err(ctx, HOPF_EDEVICE, "tail solver failed");
        float km = 0.f;
        if (rc == HOPF_OK) hipEventElapsedTime(&km, t0, t1);
        tail_s = km * 1e-3;
        tail_pts = tb;
      }
    }
    for (int j = 0; j < nj; ++j)
      if (jobs[j].parked) jobs[j].done = true;
  }
  if (rc == HOPF_OK) {
    if (hipGetLastError() != hipSuccess) rc = set_err(ctx, HOPF_EDEVICE, "kernel launch failed");
  }
  bool hit_limit = false;
  double it_s = 0.0, rows_tot = 0.0, flops = 0.0, tail_rows = 0.0, wide_s = 0.0, wide_rows = 0.0;
  long wide_n = 0;
  for (int j = 0; j < nj; ++j) {
    Job &J = jobs[j];
    if (rc == HOPF_OK && J.st.x0) {
      if (J.kron && mode == MODE_VALUE) {
        k_kron_outputs<<<(unsigned)((J.npts + 255) / 256), 256, 0, J.s>>>(
            J.S, J.st, x, J.kron->kron_k, J.kron->kron_winv_d, J.kron->kron_atot, philo_out, phihi_out, lam_out,
            iters_out, status_out, J.idx, nj > 1 ? xs : J.kron->n, 0);
      } else {
        // (a minimum-time search on a reduced system: its bounds are already
        // the full system's; the copies' costates follow)
        k_outputs<<<(unsigned)((J.npts + 255) / 256), 256, 0, J.s>>>(
            J.S, J.st, mode, T_out, gap_out, philo_out, phihi_out, J.kron ? nullptr : lam_out, probes_out,
            iters_out, status_out, J.idx, nj > 1 ? xs : J.tab->n);
        if (J.kron && lam_out)
          k_kron_outputs<<<(unsigned)((J.npts + 255) / 256), 256, 0, J.s>>>(
              J.S, J.st, x, J.kron->kron_k, J.kron->kron_winv_d, J.kron->kron_atot, nullptr, nullptr, lam_out,
              nullptr, nullptr, J.idx, nj > 1 ? xs : J.kron->n, 1);
      }
      hipEvent_t fin = J.s != base ? take_event(ctx) : nullptr;
      if (fin) {
        hipEventRecord(fin, J.s);
        hipStreamWaitEvent(base, fin, 0);
      }
    }
    if (J.rounds >= J.max_rounds) hit_limit = true;
  }
  hipEventRecord(e1, base);
  if (hipStreamSynchronize(base) != hipSuccess && rc == HOPF_OK) rc = set_err(ctx, HOPF_EDEVICE, "solve failed");
  for (int j = 0; j < nj; ++j) {
    Job &J = jobs[j];
    for (size_t i = 0; i + 1 < J.kev.size(); i += 2) {
      float km = 0.f;
      if (rc == HOPF_OK) hipEventElapsedTime(&km, J.kev[i], J.kev[i + 1]);
      it_s += km * 1e-3;
      if (J.kwide[i / 2]) {
        wide_s += km * 1e-3;
        ++wide_n;
      }
    }
    if (rc == HOPF_OK && J.st.rowsum) {
      double rs[3] = {0.0, 0.0, 0.0};
      hipMemcpy(rs, J.st.rowsum, 3 * sizeof(double), hipMemcpyDeviceToHost);
      // point-rows are summed once per round (per interval in the tail
      // solver); each runs check_every iterations
      rows_tot += (rs[0] + rs[2]) * ho.check_every;
      wide_rows += rs[2] * ho.check_every;
      tail_rows += rs[1] * ho.check_every;
      flops += 4.0 * J.tab->m_user * J.tab->n * (rs[0] + rs[1] + rs[2]) * ho.check_every;
    }
    if (rc == HOPF_OK && ctx->log_pt && j == 0) {
      int lc = 0;
      hipMemcpy(&lc, J.st.counters + 2, sizeof(int), hipMemcpyDeviceToHost);
      ctx->log_count = std::min<long>(lc, ctx->log_cap);
    }
  }
  float ms = 0.f;
  if (rc == HOPF_OK) hipEventElapsedTime(&ms, e0, e1);
  ctx->t_total = ms * 1e-3;
  ctx->t_iter = it_s;
  ctx->point_rows = rows_tot;
  ctx->alg_flops = flops;
  ctx->t_tail = tail_s;
  ctx->tail_rows = tail_rows;
  ctx->tail_points = tail_pts;
  ctx->t_wide = wide_s;
  ctx->wide_rows = wide_rows;
  ctx->wide_launches = wide_n;
  if (nj > 1)
    for (auto ps : ctx->pool) hipStreamSynchronize(ps);   // nothing of this call may outlive it
  if (rc == HOPF_OK && hit_limit) ctx->err = "round limit reached; unfinished points report NOCONV";
  return rc;
}

// ------------------------------------------------------------------ minimum time without allocations

// Device scratch for callers that cannot allocate (graph capture, serving
// loops): the per-point state of hopf_min_time_dev_noalloc lives here.  Each
// GPU the library runs on holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress gives
// on that device (scratch_init), never through the array's name.
constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

hopf_status scratch_init(int device, void **out) {
  static std::mutex mu;
  static std::vector<void *> addr;      // per device
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HOPF_EDEVICE;
    addr[device] = ptr;
  }
  *out = addr[device];
  return HOPF_OK;
}

size_t scratch_bytes() { return SCRATCH_BYTES; }

// One system's minimum-time call with every array of the point state carved
// from the device scratch: no device, pinned-host or event allocation, no
// extra streams; round checks read the active count synchronously.  The
// kernels and the search are those of solve_dev.
hopf_status solve_noalloc(Ctx *ctx, int sid, long npts, const double *x, const double *lam0, const double *tb,
                          double *T_out, double *gap_out, double *lam_out, int *probes_out, int *iters_out,
                          int *status_out, hipStream_t s) {
  if (ctx->sys.empty()) return set_err(ctx, HOPF_ESTATE, "no systems set");
  if (sid < 0 || sid >= (int)ctx->sys.size()) return set_err(ctx, HOPF_EINVAL, "sys out of range");
  if (npts < 0 || !x || !status_out) return set_err(ctx, HOPF_EINVAL, "x and pt_status are required");
  if (npts == 0) return HOPF_OK;
  if (!ctx->scratch) return set_err(ctx, HOPF_ESTATE, "device scratch not initialised");
  const hopf_opts &ho = ctx->opts;
  Job J;
  J.sid = sid;
  J.tab = &ctx->sys[sid];
  J.S = view(*J.tab);
  J.npts = npts;
  J.s = s;
  J.timed = false;
  J.ngrid = (unsigned)((npts + PTS_TILE - 1) / PTS_TILE);
  J.last_active = npts;
  J.max_rounds = (long)(ho.max_iter / ho.check_every + 3) * (ho.scan + 64 + 2);
  J.tail_ok = ho.prec == HOPF_FP32 && J.tab->n_pad <= 256 && J.tab->m <= 64;
  hopf_status rc = plan_job(ctx, J);
  if (rc != HOPF_OK) return rc;
  // the point state and the tail solver's job entry, in the scratch
  ArenaAlloc need{nullptr, ~(size_t)0};
  PtState probe_st;
  layout_state(need, *J.tab, npts, probe_st, lam0 != nullptr, ho.prec == HOPF_FP64);
  const size_t bytes = need.used + ((sizeof(TailJob) + 255) & ~(size_t)255);
  if (bytes > SCRATCH_BYTES)
    return set_err(ctx, HOPF_EINVAL, "this call needs " + std::to_string(bytes) + " bytes of scratch, more than the " +
                                         std::to_string(SCRATCH_BYTES) + " the no-allocation entry point holds; "
                                         "split the points over several calls");
  ArenaAlloc ar{reinterpret_cast<unsigned char *>(ctx->scratch), SCRATCH_BYTES};
  if (!layout_state(ar, *J.tab, npts, J.st, lam0 != nullptr, ho.prec == HOPF_FP64))
    return set_err(ctx, HOPF_EINVAL, "scratch layout failed");
  TailJob *d_tj = ar.template get<TailJob>(1);
  if (!d_tj) return set_err(ctx, HOPF_EINVAL, "scratch layout failed");
  if ((ho.warm == HOPF_WARM_MLP || ho.warm == HOPF_WARM_MLP_LAM || ho.warm == HOPF_WARM_MLP_FIRST) &&
      sid < (int)ctx->mlp.size() && ctx->mlp[sid].valid) {
    const MlpState &w = ctx->mlp[sid];
    J.mv = MlpView{w.theta, w.xm, w.xs, w.t_scale, w.lam_scale, w.n, w.H, 1};
  }
  Opts o{ho.c_tau, ho.gap_tol, ho.t_rel_tol, ho.t_abs_frac, ho.max_iter, ho.check_every, ho.warm, ho.prec, 4000,
         ho.root, ho.newton_after, ho.newton_rho, ho.adapt, ho.scan};
  const int n = J.tab->n;
  const long tot = npts * J.tab->n_pad;
  k_clear<<<1, 64, 0, s>>>(J.st);
  k_pack<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(x, J.st.x0, npts, n, J.tab->n_pad, n, nullptr, J.S.U);
  k_init<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(J.S, J.st, o, MODE_MINTIME, nullptr, nullptr, lam0, tb, n);
  ctx->iter_launches = 0;
  const long tail_lim = std::min(ho.tail_max, TAIL_MAX_POINTS);
  int cnt[2] = {0, 0};
  while (J.rounds < J.max_rounds) {
    if ((rc = issue_group(ctx, J, o, MODE_MINTIME)) != HOPF_OK) return rc;
    HIPCHK(hipMemcpyAsync(cnt, J.st.counters, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const long act = (long)cnt[0] + cnt[1];
    J.last_active = act;
    if (act == 0) break;
    if (J.tail_ok && act <= tail_lim) {
      if ((rc = park_job(ctx, J, o, act)) != HOPF_OK) return rc;
      const TailJob tj{J.S, J.st, J.mv, 0};
      HIPCHK(hipMemcpyAsync(d_tj, &tj, sizeof(TailJob), hipMemcpyHostToDevice, s));
      HIPCHK(hipFuncSetAttribute((const void *)k_tail_multi, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)tail_lds_bytes(J.tab->m)));
      k_tail_multi<<<(unsigned)act, 256, tail_lds_bytes(J.tab->m), s>>>(d_tj, 1, o);
      HIPCHK(hipStreamSynchronize(s));    // the host copy of the job entry lives until here
      break;
    }
  }
  k_outputs<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(J.S, J.st, MODE_MINTIME, T_out, gap_out, nullptr,
                                                          nullptr, lam_out, probes_out, iters_out, status_out,
                                                          nullptr, n);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  ctx->t_total = ctx->t_iter = ctx->point_rows = ctx->alg_flops = ctx->t_tail = ctx->tail_rows = 0.0;
  ctx->t_wide = ctx->wide_rows = 0.0;
  ctx->tail_points = ctx->wide_launches = 0;
  if (J.rounds >= J.max_rounds) ctx->err = "round limit reached; unfinished points report NOCONV";
  return HOPF_OK;
}

hopf_status trajectory_dev(Ctx *ctx, int sid, const double *x0_h, double T, int *n_nodes, double *s_h,
                           double *u_h, double *xs_h, double *p_h, double *philo, double *phihi) {
  if (ctx->sys.empty()) return set_err(ctx, HOPF_ESTATE, "no systems set");
  if (sid < 0 || sid >= (int)ctx->sys.size()) return set_err(ctx, HOPF_EINVAL, "sys_id out of range");
  if (!x0_h || !n_nodes || !s_h || !u_h || !xs_h || !p_h) return set_err(ctx, HOPF_EINVAL, "null output");
  const SysTables &tab = ctx->sys[sid];
  if (!(T >= 0.0 && T <= tab.desc.t_max)) return set_err(ctx, HOPF_EINVAL, "T must lie in [0, t_max]");
  const int n = tab.n, mu = tab.m_user, N = tab.N;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x0_h[i])) return set_err(ctx, HOPF_EINVAL, "x0 is not finite");
  double *dx = nullptr, *dt = nullptr, *dlo = nullptr, *dhi = nullptr, *dT = nullptr, *dgap = nullptr;
  double *ds = nullptr, *du = nullptr, *dxs = nullptr, *dp = nullptr;
  int *dsid = nullptr, *dst = nullptr, *dnn = nullptr;
  hopf_status rc = HOPF_OK;
  auto al = [&](void **p, size_t b) { if (rc == HOPF_OK && hipMalloc(p, b) != hipSuccess) rc = HOPF_ENOMEM; };
  al((void **)&dx, n * sizeof(double)); al((void **)&dt, sizeof(double)); al((void **)&dlo, sizeof(double));
  al((void **)&dhi, sizeof(double)); al((void **)&dT, sizeof(double)); al((void **)&dgap, sizeof(double));
  al((void **)&dsid, sizeof(int)); al((void **)&dst, sizeof(int)); al((void **)&dnn, sizeof(int));
  al((void **)&ds, (N + 1) * sizeof(double)); al((void **)&du, (size_t)(N + 1) * mu * sizeof(double));
  al((void **)&dxs, (size_t)(N + 1) * n * sizeof(double)); al((void **)&dp, n * sizeof(double));
  if (rc == HOPF_OK) {
    hipMemcpy(dx, x0_h, n * sizeof(double), hipMemcpyHostToDevice);
    hipMemcpy(dt, &T, sizeof(double), hipMemcpyHostToDevice);
    hipMemcpy(dsid, &sid, sizeof(int), hipMemcpyHostToDevice);
    rc = solve_dev(ctx, MODE_VALUE, 1, dsid, dx, dt, nullptr, nullptr, dT, dgap, dlo, dhi, nullptr, nullptr,
                   nullptr, dst, nullptr);
    if (rc == HOPF_OK) {
      PtState st{};
      if (!make_state(ctx, 0, tab, 1, st, false)) rc = set_err(ctx, HOPF_ENOMEM, "point state");
      else {
        k_traj<<<1, 256, 0, ctx->stream>>>(view(tab), st, T, ds, du, dxs, dp, dnn);
        if (hipStreamSynchronize(ctx->stream) != hipSuccess || hipGetLastError() != hipSuccess)
          rc = set_err(ctx, HOPF_EDEVICE, "trajectory kernel failed");
      }
    }
    if (rc == HOPF_OK) {
      int nn = 0;
      hipMemcpy(&nn, dnn, sizeof(int), hipMemcpyDeviceToHost);
      *n_nodes = nn;
      hipMemcpy(s_h, ds, nn * sizeof(double), hipMemcpyDeviceToHost);
      hipMemcpy(u_h, du, (size_t)nn * mu * sizeof(double), hipMemcpyDeviceToHost);
      hipMemcpy(xs_h, dxs, (size_t)nn * n * sizeof(double), hipMemcpyDeviceToHost);
      hipMemcpy(p_h, dp, n * sizeof(double), hipMemcpyDeviceToHost);
      if (tab.rotated) {   // states and costate back to the caller's coordinates: v = U v'
        std::vector<double> tmp(n);
        auto rot = [&](double *v) {
          for (int i = 0; i < n; ++i) {
            double a = 0.0;
            for (int j = 0; j < n; ++j) a += tab.U[(size_t)i * n + j] * v[j];
            tmp[i] = a;
          }
          std::copy(tmp.begin(), tmp.end(), v);
        };
        for (int j = 0; j < nn; ++j) rot(xs_h + (size_t)j * n);
        rot(p_h);
      }
      if (philo) hipMemcpy(philo, dlo, sizeof(double), hipMemcpyDeviceToHost);
      if (phihi) hipMemcpy(phihi, dhi, sizeof(double), hipMemcpyDeviceToHost);
    }
  } else {
    set_err(ctx, rc, "device allocation failed");
  }
  hipFree(dx); hipFree(dt); hipFree(dlo); hipFree(dhi); hipFree(dT); hipFree(dgap); hipFree(dsid); hipFree(dst);
  hipFree(dnn); hipFree(ds); hipFree(du); hipFree(dxs); hipFree(dp);
  return rc;
}

}  // namespace hopf

using hopf::Ctx;

extern "C" {

hopf_status hopf_min_time_dev(hopf_ctx *h, long npts, const int *sys_id, const double *x, const double *lam0,
                              const double *t_bracket, double *T, double *gap, double *lam, int *probes,
                              int *iters, int *pt_status, void *stream) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c) return HOPF_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return hopf::set_err(c, HOPF_EDEVICE, "hipSetDevice failed");
  return hopf::solve_dev(c, hopf::MODE_MINTIME, npts, sys_id, x, nullptr, lam0, t_bracket, T, gap, nullptr,
                         nullptr, lam, probes, iters, pt_status, (hipStream_t)stream);
}

hopf_status hopf_min_time_dev_noalloc(hopf_ctx *h, long npts, int sys, const double *x, const double *lam0,
                                      const double *t_bracket, double *T, double *gap, double *lam, int *probes,
                                      int *iters, int *pt_status, void *stream) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c) return HOPF_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return hopf::set_err(c, HOPF_EDEVICE, "hipSetDevice failed");
  return hopf::solve_noalloc(c, sys, npts, x, lam0, t_bracket, T, gap, lam, probes, iters, pt_status,
                             stream ? (hipStream_t)stream : c->stream);
}

hopf_status hopf_value_dev(hopf_ctx *h, long npts, const int *sys_id, const double *x, const double *t,
                           double *phi_lo, double *phi_hi, double *lam, int *iters, int *pt_status,
                           void *stream) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c) return HOPF_EINVAL;
  if (c->sys.empty()) return hopf::set_err(c, HOPF_ESTATE, "no systems set");
  if (npts < 0 || !x || !t || !phi_lo || !phi_hi || !pt_status)
    return hopf::set_err(c, HOPF_EINVAL, "x, t, phi_lo, phi_hi and pt_status are required");
  if (npts == 0) return HOPF_OK;
  if (npts > (1L << 26)) return hopf::set_err(c, HOPF_EINVAL, "too many points in one call");
  if (hipSetDevice(c->device) != hipSuccess) return hopf::set_err(c, HOPF_EDEVICE, "hipSetDevice failed");
  hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  // the horizons (and system ids) are checked on the host before any kernel
  // runs: a horizon outside [0, t_max] would address nodes beyond the table
  std::vector<double> th(npts);
  std::vector<int> ih(sys_id ? npts : 0);
  if (hipMemcpyAsync(th.data(), t, npts * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      (sys_id && hipMemcpyAsync(ih.data(), sys_id, npts * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return hopf::set_err(c, HOPF_EDEVICE, "reading t / sys_id from the device failed");
  const int nsys = (int)c->sys.size();
  for (long i = 0; i < npts; ++i) {
    const int sid = sys_id ? ih[i] : 0;
    if (sid < 0 || sid >= nsys) return hopf::set_err(c, HOPF_EINVAL, "sys_id out of range");
    if (!(th[i] >= 0.0 && th[i] <= c->sys[sid].desc.t_max))
      return hopf::set_err(c, HOPF_EINVAL, "t must lie in [0, t_max]");
  }
  return hopf::solve_dev(c, hopf::MODE_VALUE, npts, sys_id, x, t, nullptr, nullptr, nullptr, nullptr, phi_lo,
                         phi_hi, lam, nullptr, iters, pt_status, s);
}

static hopf_status host_call(Ctx *c, int mode, long npts, const int *sys_id, const double *x,
                             const double *t, const double *lam0, const double *tbr, double *T, double *gap,
                             double *philo, double *phihi, double *lam, int *probes, int *iters,
                             int *pt_status) {
  if (!c) return HOPF_EINVAL;
  if (c->sys.empty()) return hopf::set_err(c, HOPF_ESTATE, "no systems set");
  if (npts < 0 || !x || !pt_status) return hopf::set_err(c, HOPF_EINVAL, "x and pt_status are required");
  if (mode == hopf::MODE_VALUE && !t) return hopf::set_err(c, HOPF_EINVAL, "t is required");
  if (npts == 0) return HOPF_OK;
  if (hipSetDevice(c->device) != hipSuccess) return hopf::set_err(c, HOPF_EDEVICE, "hipSetDevice failed");
  int n = 0;   // row stride of x and lam: the largest n among the systems used
  for (long i = 0; i < (sys_id ? npts : 1); ++i) {
    const int sid = sys_id ? sys_id[i] : 0;
    if (sid < 0 || sid >= (int)c->sys.size()) return hopf::set_err(c, HOPF_EINVAL, "sys_id out of range");
    n = std::max(n, c->sys[sid].n);
  }
  if (mode == hopf::MODE_VALUE)
    for (long i = 0; i < npts; ++i)
      if (!(t[i] >= 0.0 && t[i] <= c->sys[sys_id ? sys_id[i] : 0].desc.t_max))
        return hopf::set_err(c, HOPF_EINVAL, "t must lie in [0, t_max]");
  // device buffers for this call
  double *dx = nullptr, *dt = nullptr, *dT = nullptr, *dgap = nullptr, *dlo = nullptr, *dhi = nullptr, *dlam = nullptr;
  double *dl0 = nullptr, *dtb = nullptr;
  int *dsid = nullptr, *dpr = nullptr, *dit = nullptr, *dst = nullptr;
  hopf_status rc = HOPF_OK;
  auto al = [&](void **p, size_t b) { if (rc == HOPF_OK && hipMalloc(p, b) != hipSuccess) rc = HOPF_ENOMEM; };
  al((void **)&dx, npts * n * sizeof(double));
  al((void **)&dT, npts * sizeof(double));
  al((void **)&dgap, npts * sizeof(double));
  al((void **)&dlo, npts * sizeof(double));
  al((void **)&dhi, npts * sizeof(double));
  al((void **)&dpr, npts * sizeof(int));
  al((void **)&dit, npts * sizeof(int));
  al((void **)&dst, npts * sizeof(int));
  if (lam) al((void **)&dlam, npts * n * sizeof(double));
  if (lam0) al((void **)&dl0, npts * n * sizeof(double));
  if (tbr) al((void **)&dtb, npts * 2 * sizeof(double));
  if (t) al((void **)&dt, npts * sizeof(double));
  if (sys_id) al((void **)&dsid, npts * sizeof(int));
  if (rc == HOPF_OK) {
    hipMemcpy(dx, x, npts * n * sizeof(double), hipMemcpyHostToDevice);
    if (t) hipMemcpy(dt, t, npts * sizeof(double), hipMemcpyHostToDevice);
    if (sys_id) hipMemcpy(dsid, sys_id, npts * sizeof(int), hipMemcpyHostToDevice);
    if (lam0) hipMemcpy(dl0, lam0, npts * n * sizeof(double), hipMemcpyHostToDevice);
    if (tbr) hipMemcpy(dtb, tbr, npts * 2 * sizeof(double), hipMemcpyHostToDevice);
    rc = hopf::solve_dev(c, mode, npts, dsid, dx, dt, dl0, dtb, dT, dgap, dlo, dhi, dlam, dpr, dit, dst, nullptr);
    if (rc == HOPF_OK) {
      if (T) hipMemcpy(T, dT, npts * sizeof(double), hipMemcpyDeviceToHost);
      if (gap) hipMemcpy(gap, dgap, npts * sizeof(double), hipMemcpyDeviceToHost);
      if (philo) hipMemcpy(philo, dlo, npts * sizeof(double), hipMemcpyDeviceToHost);
      if (phihi) hipMemcpy(phihi, dhi, npts * sizeof(double), hipMemcpyDeviceToHost);
      if (lam) hipMemcpy(lam, dlam, npts * n * sizeof(double), hipMemcpyDeviceToHost);
      if (probes) hipMemcpy(probes, dpr, npts * sizeof(int), hipMemcpyDeviceToHost);
      if (iters) hipMemcpy(iters, dit, npts * sizeof(int), hipMemcpyDeviceToHost);
      hipMemcpy(pt_status, dst, npts * sizeof(int), hipMemcpyDeviceToHost);
    }
  } else {
    hopf::set_err(c, rc, "device allocation failed");
  }
  hipFree(dx); hipFree(dt); hipFree(dT); hipFree(dgap); hipFree(dlo); hipFree(dhi); hipFree(dlam);
  hipFree(dsid); hipFree(dpr); hipFree(dit); hipFree(dst); hipFree(dl0); hipFree(dtb);
  return rc;
}

hopf_status hopf_min_time(hopf_ctx *h, long npts, const int *sys_id, const double *x, const double *lam0,
                          const double *t_bracket, double *T, double *gap, double *lam, int *probes, int *iters,
                          int *pt_status) {
  return host_call(reinterpret_cast<Ctx *>(h), hopf::MODE_MINTIME, npts, sys_id, x, nullptr, lam0, t_bracket, T,
                   gap, nullptr, nullptr, lam, probes, iters, pt_status);
}

hopf_status hopf_value(hopf_ctx *h, long npts, const int *sys_id, const double *x, const double *t,
                       double *phi_lo, double *phi_hi, double *lam, int *iters, int *pt_status) {
  return host_call(reinterpret_cast<Ctx *>(h), hopf::MODE_VALUE, npts, sys_id, x, t, nullptr, nullptr, nullptr,
                   nullptr, phi_lo, phi_hi, lam, nullptr, iters, pt_status);
}

hopf_status hopf_trajectory(hopf_ctx *h, int sys_id, const double *x0, double T, int *n_nodes, double *s,
                            double *u, double *xs, double *p_star, double *phi_lo, double *phi_hi) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c) return HOPF_EINVAL;
  return hopf::trajectory_dev(c, sys_id, x0, T, n_nodes, s, u, xs, p_star, phi_lo, phi_hi);
}

}  // extern "C"

namespace hopf {

#define HOPF_DECL(k)                                   \
  pdhg_fn pdhg_lookup_nt##k(int m, int prec, int waves, int *MM); \
  pdhg_fn wide_lookup_nt##k(int m);                    \
  pdhg_fn stream_lookup_nt##k(int bf16);               \
  pdhg_fn swide_lookup_nt##k(int bf16);                \
  cert_fn cert_lookup_nt##k();
HOPF_DECL(1) HOPF_DECL(2) HOPF_DECL(3) HOPF_DECL(4) HOPF_DECL(5) HOPF_DECL(6) HOPF_DECL(7) HOPF_DECL(8)
HOPF_DECL(9) HOPF_DECL(10) HOPF_DECL(11) HOPF_DECL(12) HOPF_DECL(13) HOPF_DECL(14) HOPF_DECL(15) HOPF_DECL(16)
#undef HOPF_DECL

#define HOPF_SW(expr_k)                                                               \
  switch (NT) {                                                                       \
    case 1: return expr_k(1); case 2: return expr_k(2); case 3: return expr_k(3);      \
    case 4: return expr_k(4); case 5: return expr_k(5); case 6: return expr_k(6);      \
    case 7: return expr_k(7); case 8: return expr_k(8); case 9: return expr_k(9);      \
    case 10: return expr_k(10); case 11: return expr_k(11); case 12: return expr_k(12); \
    case 13: return expr_k(13); case 14: return expr_k(14); case 15: return expr_k(15); \
    case 16: return expr_k(16);                                                       \
  }                                                                                   \
  return nullptr;

pdhg_fn pdhg_lookup(int NT, int m, int prec, int waves, int *MM) {
#define E(k) pdhg_lookup_nt##k(m, prec, waves, MM)
  HOPF_SW(E)
#undef E
}

pdhg_fn wide_lookup(int NT, int m) {
#define E(k) wide_lookup_nt##k(m)
  HOPF_SW(E)
#undef E
}

pdhg_fn stream_lookup(int NT, int bf16) {
#define E(k) stream_lookup_nt##k(bf16)
  HOPF_SW(E)
#undef E
}

pdhg_fn swide_lookup(int NT, int bf16) {
#define E(k) swide_lookup_nt##k(bf16)
  HOPF_SW(E)
#undef E
}

cert_fn cert_lookup(int NT) {
#define E(k) cert_lookup_nt##k()
  HOPF_SW(E)
#undef E
}

}  // namespace hopf
