// Learned warm start: a small MLP (x, t) -> (lam_0, log T_hat, bracket
// width) trained on pairs the solver itself generates (the final costate of
// every probe), with hand-written HIP kernels for the forward pass, the
// backward pass and Adam.  Cold-start PDHG stays the fallback: the network only
// proposes starting points and probe horizons; every result is still certified
// by the FP64 duality gap.
//
// Network (per system, n states): z = ((x - mean)/std, t/t_max) in R^{n+1};
// three hidden layers of width H = 256 with the exact GELU; linear output
// [lam_hat/lam_scale (n), log T_hat, r], bracket half-width
// delta = softplus(r) + 1e-3 in log-time.  Loss per sample:
//   (1/n)|lam_hat - lam|^2 + reach * ((e)^2 + max(0,|e| - delta) + 0.05 delta),
//   e = log T_hat - log T*.
// Parameters are one flat FP32 vector [W1 (n+1,H), b1, W2, b2, W3, b3, W4 (H,n+2), b4].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "hopf_device.h"

namespace hopf {

constexpr float MLP_DELTA_MIN = 1e-3f;
constexpr float MLP_ETA = 0.05f;


// ------------------------------------------------------------------ GEMM

// C (M x N) = op(A) (M x K) * op(B) (K x N) on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32), with A(i,k) at A[i*ars + k*acs] and B(k,j) at
// B[k*brs + j*bcs] (strides express the transposes of the backward pass).
// A workgroup of four waves computes a 64 x 64 tile of C, each wave a
// 32 x 32 quarter as 2 x 2 MFMA tiles; K runs in chunks of 16 through LDS
// (row stride 80 floats: the four k rows of an operand read fall in distinct
// banks).  Options:
//   ones_row >= 0  row ones_row of op(A) is all ones (row ones_row of C then
//                  holds the column sums of op(B): a bias gradient computed
//                  with its weight gradient)
//   gridDim.z > 1  split K: workgroup z takes K chunks z, z + gridDim.z, ...
//                  and adds its partial tile to C atomically (C zeroed first)
//   epi            GEMM_STORE: C = acc + bias_j;  GEMM_GELU: C = acc + bias_j
//                  and H = gelu(C) (same layout);  GEMM_GELU_BWD:
//                  C = acc * gelu'(aux) (aux in C's layout);  GEMM_GELU_ONLY:
//                  C = gelu(acc + bias_j)
constexpr int GEMM_STORE = 0, GEMM_GELU = 1, GEMM_GELU_BWD = 2, GEMM_GELU_ONLY = 3;
constexpr int GEMM_LDS = 80;

__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A, long ars, long acs,
                                              const float *__restrict__ B, long brs, long bcs, float *__restrict__ C,
                                              long ldc, const float *__restrict__ bias, int ones_row, int epi,
                                              float *__restrict__ Hout, const float *__restrict__ aux) {
  __shared__ __align__(16) float As[16 * GEMM_LDS];   // As[k][row]
  __shared__ __align__(16) float Bs[16 * GEMM_LDS];   // Bs[k][col]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cl = lane & 15, g = lane >> 4;
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nchunk = (K + 15) / 16;
  for (int ch = blockIdx.z; ch < nchunk; ch += gridDim.z) {
    const int k0 = ch * 16;
    // stage op(A)[i0 .. +64][k0 .. +16] and op(B)[k0 .. +16][j0 .. +64];
    // consecutive threads take the operand's unit-stride index
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      int kk, r;
      if (acs == 1) { r = e >> 4; kk = e & 15; } else { kk = e >> 6; r = e & 63; }
      const int ia = i0 + r, ka = k0 + kk;
      float v = 0.0f;
      if (ia < M && ka < K) v = (ia == ones_row) ? 1.0f : A[(long)ia * ars + (long)ka * acs];
      As[kk * GEMM_LDS + r] = v;
      if (bcs == 1) { kk = e >> 6; r = e & 63; } else { r = e >> 4; kk = e & 15; }
      const int jb = j0 + r, kb = k0 + kk;
      Bs[kk * GEMM_LDS + r] = (jb < N && kb < K) ? B[(long)kb * brs + (long)jb * bcs] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < 16; k4 += 4) {
      float av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[(k4 + g) * GEMM_LDS + wr + 16 * a + cl];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[(k4 + g) * GEMM_LDS + wc + 16 * b + cl];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  // lane (cl, g) holds rows 4 g + q, column cl of each 16 x 16 tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + wr + 16 * a + 4 * g + q, j = j0 + wc + 16 * b + cl;
        if (i >= M || j >= N) continue;
        const long o = (long)i * ldc + j;
        float v = acc[a][b][q];
        if (gridDim.z > 1) {
          atomicAdd(&C[o], v);
        } else if (epi == GEMM_GELU_BWD) {
          C[o] = v * gelu_grad_f(aux[o]);
        } else {
          v += bias ? bias[j] : 0.0f;
          C[o] = epi == GEMM_GELU_ONLY ? gelu_f(v) : v;
          if (epi == GEMM_GELU) Hout[o] = gelu_f(v);
        }
      }
}

__global__ void k_fill(float *__restrict__ p, long count, float v) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// loss and gradient with respect to the output rows; loss += the batch
// mean, esum (if given) += the batch sum
__global__ void k_loss_grad(const float *__restrict__ out, const float *__restrict__ Y, int Bn, int n,
                            float *__restrict__ gout, double *__restrict__ loss, double *__restrict__ esum) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= Bn) return;
  const int d = n + 2;
  const float *o = out + (long)s * d;
  const float *y = Y + (long)s * d;
  float *go = gout + (long)s * d;
  double ls = 0.0;
  for (int i = 0; i < n; ++i) {
    const float df = o[i] - y[i];
    ls += (double)df * df / n;
    go[i] = 2.0f * df / ((float)n * Bn);
  }
  const float mk = y[n + 1];
  const float r = o[n + 1];
  const float delta = log1pf(expf(-fabsf(r))) + fmaxf(r, 0.0f) + MLP_DELTA_MIN;
  const float e = o[n] - y[n];
  const bool miss = fabsf(e) > delta;
  ls += mk * ((double)e * e + fmax(0.0, (double)fabsf(e) - delta) + MLP_ETA * delta);
  go[n] = mk * (2.0f * e + (miss ? (e > 0 ? 1.0f : (e < 0 ? -1.0f : 0.0f)) : 0.0f)) / Bn;
  const float sg = 1.0f / (1.0f + expf(-r));
  go[n + 1] = mk * ((miss ? -1.0f : 0.0f) + MLP_ETA) * sg / Bn;
  atomicAdd(loss, ls / Bn);
  if (esum) atomicAdd(esum, ls);
}

__global__ void k_zero_d(double *__restrict__ p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0.0;
}

__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long count, float lr, float c1, float c2) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// training rows from the probe log: Z = ((x - mean)/std, T/t_max),
// Y = (lam/lam_scale, log T*, reach)
__global__ void k_make_rows(const int *__restrict__ idx, int Bn, const int *__restrict__ log_pt,
                            const float *__restrict__ log_T, const float *__restrict__ log_lam, int lstride,
                            const double *__restrict__ xq, const double *__restrict__ Tq,
                            const int *__restrict__ stq, int n, const float *__restrict__ xm,
                            const float *__restrict__ xs, float t_scale, float lam_scale,
                            float *__restrict__ Z, float *__restrict__ Y) {
  const int s = blockIdx.x;
  if (s >= Bn) return;
  const int e = idx[s];
  const int p = log_pt[e];
  for (int i = threadIdx.x; i < n + 2; i += blockDim.x) {
    if (i < n) {
      Z[(long)s * (n + 1) + i] = (float)((xq[(long)p * n + i] - xm[i]) / xs[i]);
      Y[(long)s * (n + 2) + i] = log_lam[(long)e * lstride + i] / lam_scale;
    } else if (i == n) {
      Z[(long)s * (n + 1) + n] = log_T[e] / t_scale;
      const bool reach = stq[p] == HOPF_PT_OK;
      Y[(long)s * (n + 2) + n] = reach ? (float)log(Tq[p]) : 0.0f;
    } else {
      Y[(long)s * (n + 2) + n + 1] = (stq[p] == HOPF_PT_OK) ? 1.0f : 0.0f;
    }
  }
}

// ------------------------------------------------------------------ host side

namespace {

struct MlpBufs {
  float *Z = nullptr, *Y = nullptr, *a1 = nullptr, *h1 = nullptr, *a2 = nullptr, *h2 = nullptr, *a3 = nullptr,
        *h3 = nullptr, *out = nullptr, *g = nullptr, *g2 = nullptr, *grad = nullptr;
  double *loss = nullptr, *esum = nullptr;
  int cap = 0;
  size_t np = 0;
  void free_all() {
    hipFree(Z); hipFree(Y); hipFree(a1); hipFree(h1); hipFree(a2); hipFree(h2); hipFree(a3); hipFree(h3);
    hipFree(out); hipFree(g); hipFree(g2); hipFree(grad); hipFree(loss); hipFree(esum);
    *this = MlpBufs();
  }
};

size_t nparams(int n, int H) {
  const size_t di = n + 1, dout = n + 2;
  return di * H + H + (size_t)H * H + H + (size_t)H * H + H + (size_t)H * dout + dout;
}

void gemm(hipStream_t s, int M, int N, int K, const float *A, long ars, long acs, const float *B, long brs,
          long bcs, float *C, long ldc, const float *bias, int epi = GEMM_STORE, float *Hout = nullptr,
          const float *aux = nullptr, int ones_row = -1, int split = 1) {
  dim3 grid((N + 63) / 64, (M + 63) / 64, split);
  k_gemm<<<grid, 256, 0, s>>>(M, N, K, A, ars, acs, B, brs, bcs, C, ldc, bias, ones_row, epi, Hout, aux);
}

// weight and bias gradient of one layer in one GEMM: [gW; gb] = [X^T; 1] G,
// X (Bn x rows) the layer's input, G (Bn x cols) the gradient at its output;
// gb follows gW in the parameter vector (row `rows` of a (rows+1) x cols
// matrix).  K = Bn is split so that about 512 workgroups run; the partial
// tiles add into gW, which the caller has zeroed.
void wgrad(hipStream_t s, int rows, int cols, int Bn, const float *X, const float *G, float *gW) {
  const int tiles = ((cols + 63) / 64) * ((rows + 1 + 63) / 64);
  const int split = std::max(1, std::min((Bn + 15) / 16, (512 + tiles - 1) / tiles));
  gemm(s, rows + 1, cols, Bn, X, 1, rows, G, cols, 1, gW, cols, nullptr, GEMM_STORE, nullptr, nullptr, rows, split);
}

bool alloc_bufs(MlpBufs &b, int Bn, int n, int H, size_t np_) {
  if (b.cap >= Bn && b.grad) return true;
  b.free_all();
  auto al = [&](float **p, size_t c) { return hipMalloc(p, c * sizeof(float)) == hipSuccess; };
  bool ok = al(&b.Z, (size_t)Bn * (n + 1)) && al(&b.Y, (size_t)Bn * (n + 2)) && al(&b.a1, (size_t)Bn * H) &&
            al(&b.h1, (size_t)Bn * H) && al(&b.a2, (size_t)Bn * H) && al(&b.h2, (size_t)Bn * H) &&
            al(&b.a3, (size_t)Bn * H) && al(&b.h3, (size_t)Bn * H) && al(&b.out, (size_t)Bn * (n + 2)) &&
            al(&b.g, (size_t)Bn * std::max(H, n + 2)) && al(&b.g2, (size_t)Bn * std::max(H, n + 2)) &&
            al(&b.grad, np_) && hipMalloc(&b.loss, sizeof(double)) == hipSuccess &&
            hipMalloc(&b.esum, sizeof(double)) == hipSuccess;
  if (!ok) { b.free_all(); return false; }
  b.cap = Bn;
  b.np = np_;
  return true;
}

// forward + loss + backward on rows Z, Y (device); gradient into b.grad, the
// batch's mean loss into b.loss (and its sum added to esum when given)
void loss_grad(hipStream_t s, const float *th, MlpBufs &b, int Bn, int n, int H, double *esum = nullptr) {
  const int di = n + 1, dout = n + 2;
  const float *W1 = th, *b1 = W1 + (size_t)di * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H, *W3 = b2 + H,
              *b3 = W3 + (size_t)H * H, *W4 = b3 + H, *b4 = W4 + (size_t)H * dout;
  float *gW1 = b.grad, *gW2 = gW1 + (size_t)di * H + H, *gW3 = gW2 + (size_t)H * H + H,
        *gW4 = gW3 + (size_t)H * H + H;
  // forward: a_l = h_{l-1} W_l + b_l and h_l = gelu(a_l) in one pass
  gemm(s, Bn, H, di, b.Z, di, 1, W1, H, 1, b.a1, H, b1, GEMM_GELU, b.h1);
  gemm(s, Bn, H, H, b.h1, H, 1, W2, H, 1, b.a2, H, b2, GEMM_GELU, b.h2);
  gemm(s, Bn, H, H, b.h2, H, 1, W3, H, 1, b.a3, H, b3, GEMM_GELU, b.h3);
  gemm(s, Bn, dout, H, b.h3, H, 1, W4, dout, 1, b.out, dout, b4);
  k_zero_d<<<1, 64, 0, s>>>(b.loss);
  k_loss_grad<<<(Bn + 127) / 128, 128, 0, s>>>(b.out, b.Y, Bn, n, b.g, b.loss, esum);   // g = dL/dout
  k_fill<<<(unsigned)((b.np + 255) / 256), 256, 0, s>>>(b.grad, (long)b.np, 0.0f);
  // backward: layer l's weight and bias gradient, then the gradient at the
  // previous layer's pre-activation, (g W_l^T) * gelu'(a_{l-1}), in one pass
  wgrad(s, H, dout, Bn, b.h3, b.g, gW4);
  gemm(s, Bn, H, dout, b.g, dout, 1, W4, 1, dout, b.g2, H, nullptr, GEMM_GELU_BWD, nullptr, b.a3);
  wgrad(s, H, H, Bn, b.h2, b.g2, gW3);
  gemm(s, Bn, H, H, b.g2, H, 1, W3, 1, H, b.g, H, nullptr, GEMM_GELU_BWD, nullptr, b.a2);
  wgrad(s, H, H, Bn, b.h1, b.g, gW2);
  gemm(s, Bn, H, H, b.g, H, 1, W2, 1, H, b.g2, H, nullptr, GEMM_GELU_BWD, nullptr, b.a1);
  wgrad(s, di, H, Bn, b.Z, b.g2, gW1);
}

// network inputs of the first probe: Z = ((x0 - mean)/std, T/t_scale), one
// workgroup per point
__global__ void k_net_in(MlpView mv, PtState st, long npts, int np, float *__restrict__ Z) {
  const long p = blockIdx.x;
  if (p >= npts) return;
  const int n = mv.n;
  for (int i = threadIdx.x; i <= n; i += blockDim.x)
    Z[p * (n + 1) + i] = i < n ? (float)((st.x0[p * np + i] - mv.xm[i]) / mv.xs[i]) : (float)(st.T[p] / mv.t_scale);
}

// network outputs of the first probe, one thread per point.  An output that
// is not finite, or a costate more than 1000 times the training costates'
// scale, is not used (lambda_0 = 0, no bracket): a damaged network can slow a
// solve down, not change it.
__global__ void k_net_out(MlpView mv, PtState st, long npts, int np, const float *__restrict__ out, int warm,
                          int caller_lam0) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts) return;
  const int n = mv.n, dout = n + 2;
  const float *o = out + p * dout;
  bool bad = !(isfinite(mv.lam_scale) && mv.lam_scale > 0.0f);
  for (int k = 0; k < dout; ++k) bad |= !isfinite(o[k] * (k < n ? mv.lam_scale : 1.0f));
  for (int k = 0; k < n; ++k) bad |= fabsf(o[k]) > 1e3f;
  if ((warm == HOPF_WARM_MLP_FIRST || warm == HOPF_WARM_MLP_LAM) && !caller_lam0 && st.lam0s)
    for (int i = 0; i < np; ++i) st.lam0s[p * np + i] = (!bad && i < n) ? (double)(o[i] * mv.lam_scale) : 0.0;
  if (bad) return;
  const float r2 = o[n + 1];
  st.bT[p] = expf(o[n]);
  st.bD[p] = log1pf(expf(-fabsf(r2))) + fmaxf(r2, 0.0f) + MLP_DELTA_MIN;
  // the network's bracket [T e^-d, T e^d] as probe hints inside the first
  // sign-change cell, unless the caller gave hints
  if ((warm == HOPF_WARM_MLP || warm == HOPF_WARM_MLP_LAM) && st.stage[p] == 2) {
    st.ha[p] = (double)st.bT[p] * exp(-(double)st.bD[p]);
    st.hb[p] = (double)st.bT[p] * exp((double)st.bD[p]);
    st.stage[p] = 0;
  }
}

}  // namespace

hopf_status mlp_first_probe(Ctx *ctx, const MlpView &mv, int warm, const PtState &st, long npts, int np,
                            bool caller_lam0, hipStream_t s) {
  if (npts < 1) return HOPF_OK;
  const int n = mv.n, H = mv.H, di = n + 1, dout = n + 2;
  const size_t need = (size_t)npts * ((size_t)di + 2 * (size_t)H + (size_t)dout);
  if (ctx->net_cap < need) {
    hipFree(ctx->net_buf);
    ctx->net_buf = nullptr;
    ctx->net_cap = 0;
    if (hipMalloc((void **)&ctx->net_buf, need * sizeof(float)) != hipSuccess)
      return set_err(ctx, HOPF_ENOMEM, "network evaluation buffers");
    ctx->net_cap = need;
  }
  float *Z = ctx->net_buf, *h1 = Z + (size_t)npts * di, *h2 = h1 + (size_t)npts * H, *out = h2 + (size_t)npts * H;
  const float *W1 = mv.theta, *b1 = W1 + (size_t)di * H, *W2 = b1 + H, *b2 = W2 + (size_t)H * H, *W3 = b2 + H,
              *b3 = W3 + (size_t)H * H, *W4 = b3 + H, *b4 = W4 + (size_t)H * dout;
  const int M = (int)npts;
  k_net_in<<<(unsigned)npts, 128, 0, s>>>(mv, st, npts, np, Z);
  gemm(s, M, H, di, Z, di, 1, W1, H, 1, h1, H, b1, GEMM_GELU_ONLY);
  gemm(s, M, H, H, h1, H, 1, W2, H, 1, h2, H, b2, GEMM_GELU_ONLY);
  gemm(s, M, H, H, h2, H, 1, W3, H, 1, h1, H, b3, GEMM_GELU_ONLY);
  gemm(s, M, dout, H, h1, H, 1, W4, dout, 1, out, dout, b4);
  k_net_out<<<(unsigned)((npts + 255) / 256), 256, 0, s>>>(mv, st, npts, np, out, warm, caller_lam0 ? 1 : 0);
  return hipGetLastError() == hipSuccess ? HOPF_OK : set_err(ctx, HOPF_EDEVICE, "network evaluation launch failed");
}

void mlp_free(MlpState &w) {
  hipFree(w.theta); hipFree(w.m); hipFree(w.v); hipFree(w.xm); hipFree(w.xs);
  w.theta = w.m = w.v = w.xm = w.xs = nullptr;
  w.valid = 0;
}

static hopf_status mlp_ensure(Ctx *ctx, int sid, MlpState &w) {
  const SysTables &t = ctx->sys[sid];
  const int n = t.n, H = MLP_WIDTH;
  const size_t np_ = nparams(n, H);
  if (w.theta && w.n == n && w.nparam == np_) return HOPF_OK;
  mlp_free(w);
  w.n = n;
  w.H = H;
  w.nparam = np_;
  if (hipMalloc(&w.theta, np_ * 4) != hipSuccess || hipMalloc(&w.m, np_ * 4) != hipSuccess ||
      hipMalloc(&w.v, np_ * 4) != hipSuccess || hipMalloc(&w.xm, n * 4) != hipSuccess ||
      hipMalloc(&w.xs, n * 4) != hipSuccess) {
    mlp_free(w);
    return set_err(ctx, HOPF_ENOMEM, "warm-start network allocation failed");
  }
  w.t_scale = (float)t.desc.t_max;
  w.lam_scale = 1.0f;
  std::vector<float> one(n, 1.0f), zero(n, 0.0f);
  hipMemcpy(w.xm, zero.data(), n * 4, hipMemcpyHostToDevice);
  hipMemcpy(w.xs, one.data(), n * 4, hipMemcpyHostToDevice);
  return HOPF_OK;
}

static void he_init(std::vector<float> &th, int n, int H, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<float> nd(0.0f, 1.0f);
  const int di = n + 1, dout = n + 2;
  size_t o = 0;
  auto fill = [&](int fan_in, size_t count, bool weight) {
    const float sc = weight ? std::sqrt(2.0f / fan_in) : 0.0f;
    for (size_t i = 0; i < count; ++i) th[o++] = weight ? sc * nd(rng) : 0.0f;
  };
  fill(di, (size_t)di * H, true); fill(di, H, false);
  fill(H, (size_t)H * H, true); fill(H, H, false);
  fill(H, (size_t)H * H, true); fill(H, H, false);
  fill(H, (size_t)H * dout, true); fill(H, dout, false);
  // the output layer starts small so that early predictions are near the bias
  o = (size_t)di * H + H + 2 * ((size_t)H * H + H);
  for (size_t i = 0; i < (size_t)H * dout; ++i) th[o + i] *= 0.1f;
}

__global__ void k_sumsq_rows(const float *__restrict__ a, long rows, int n, int stride, double *__restrict__ out) {
  long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    const double v = a[r * stride + i];
    s += v * v;
  }
  atomicAdd(out, s);
}

}  // namespace hopf

using hopf::Ctx;
using hopf::set_err;

extern "C" {

hopf_status hopf_warm_init(hopf_ctx *h, int sys_id, unsigned seed) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c) return HOPF_EINVAL;
  if (sys_id < 0 || sys_id >= (int)c->sys.size()) return set_err(c, HOPF_EINVAL, "sys_id out of range");
  hipSetDevice(c->device);
  if ((int)c->mlp.size() < (int)c->sys.size()) c->mlp.resize(c->sys.size());
  hopf::MlpState &w = c->mlp[sys_id];
  hopf_status st = hopf::mlp_ensure(c, sys_id, w);
  if (st != HOPF_OK) return st;
  std::vector<float> th(w.nparam);
  hopf::he_init(th, w.n, w.H, seed);
  hipMemcpy(w.theta, th.data(), w.nparam * 4, hipMemcpyHostToDevice);
  hipMemset(w.m, 0, w.nparam * 4);
  hipMemset(w.v, 0, w.nparam * 4);
  w.step = 0;
  w.valid = 0;
  return HOPF_OK;
}

hopf_status hopf_warm_params(hopf_ctx *h, int sys_id, int set, float *theta, long count, float *norm) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c || !theta) return HOPF_EINVAL;
  if (sys_id < 0 || sys_id >= (int)c->mlp.size() || !c->mlp[sys_id].theta)
    return set_err(c, HOPF_ESTATE, "no warm-start network for this system (call hopf_warm_init)");
  hopf::MlpState &w = c->mlp[sys_id];
  if (count != (long)w.nparam) return set_err(c, HOPF_EINVAL, "parameter count mismatch");
  hipSetDevice(c->device);
  const int n = w.n;
  if (set) {
    hipMemcpy(w.theta, theta, w.nparam * 4, hipMemcpyHostToDevice);
    if (norm) {   // norm = [x_mean (n), x_std (n), t_scale, lam_scale]
      hipMemcpy(w.xm, norm, n * 4, hipMemcpyHostToDevice);
      hipMemcpy(w.xs, norm + n, n * 4, hipMemcpyHostToDevice);
      w.t_scale = norm[2 * n];
      w.lam_scale = norm[2 * n + 1];
      w.valid = 1;
    }
  } else {
    hipMemcpy(theta, w.theta, w.nparam * 4, hipMemcpyDeviceToHost);
    if (norm) {
      hipMemcpy(norm, w.xm, n * 4, hipMemcpyDeviceToHost);
      hipMemcpy(norm + n, w.xs, n * 4, hipMemcpyDeviceToHost);
      norm[2 * n] = w.t_scale;
      norm[2 * n + 1] = w.lam_scale;
    }
  }
  return HOPF_OK;
}

// Checkpoint file of one network (little-endian): "HOPFWARM", u32 version 1,
// u32 n, u32 H, u64 parameter count, f32 t_scale, f32 lam_scale, then f32
// x_mean[n], x_std[n], theta[count].  Load checks every header field against
// the system's network before it replaces anything.
hopf_status hopf_warm_save(hopf_ctx *h, int sys_id, const char *path) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c || !path) return HOPF_EINVAL;
  if (sys_id < 0 || sys_id >= (int)c->mlp.size() || !c->mlp[sys_id].theta || !c->mlp[sys_id].valid)
    return set_err(c, HOPF_ESTATE, "no trained warm-start network for this system");
  hopf::MlpState &w = c->mlp[sys_id];
  hipSetDevice(c->device);
  std::vector<float> th(w.nparam), xm(w.n), xs(w.n);
  if (hipMemcpy(th.data(), w.theta, w.nparam * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(xm.data(), w.xm, w.n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(xs.data(), w.xs, w.n * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return set_err(c, HOPF_EDEVICE, "reading the network from the device failed");
  FILE *f = std::fopen(path, "wb");
  if (!f) return set_err(c, HOPF_EINVAL, std::string("cannot open ") + path + " for writing");
  const uint32_t hdr[3] = {1u, (uint32_t)w.n, (uint32_t)w.H};
  const uint64_t cnt = w.nparam;
  const float sc[2] = {w.t_scale, w.lam_scale};
  bool ok = std::fwrite("HOPFWARM", 1, 8, f) == 8 && std::fwrite(hdr, 4, 3, f) == 3 &&
            std::fwrite(&cnt, 8, 1, f) == 1 && std::fwrite(sc, 4, 2, f) == 2 &&
            std::fwrite(xm.data(), 4, w.n, f) == (size_t)w.n && std::fwrite(xs.data(), 4, w.n, f) == (size_t)w.n &&
            std::fwrite(th.data(), 4, w.nparam, f) == w.nparam;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? HOPF_OK : set_err(c, HOPF_EINVAL, std::string("writing ") + path + " failed");
}

hopf_status hopf_warm_load(hopf_ctx *h, int sys_id, const char *path) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c || !path) return HOPF_EINVAL;
  if (sys_id < 0 || sys_id >= (int)c->sys.size()) return set_err(c, HOPF_EINVAL, "sys_id out of range");
  hipSetDevice(c->device);
  if ((int)c->mlp.size() < (int)c->sys.size()) c->mlp.resize(c->sys.size());
  hopf::MlpState &w = c->mlp[sys_id];
  hopf_status st = hopf::mlp_ensure(c, sys_id, w);
  if (st != HOPF_OK) return st;
  FILE *f = std::fopen(path, "rb");
  if (!f) return set_err(c, HOPF_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  uint32_t hdr[3];
  uint64_t cnt = 0;
  float sc[2];
  std::vector<float> xm(w.n), xs(w.n), th(w.nparam);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "HOPFWARM", 8) == 0 &&
            std::fread(hdr, 4, 3, f) == 3 && hdr[0] == 1u && hdr[1] == (uint32_t)w.n && hdr[2] == (uint32_t)w.H &&
            std::fread(&cnt, 8, 1, f) == 1 && cnt == (uint64_t)w.nparam && std::fread(sc, 4, 2, f) == 2 &&
            std::fread(xm.data(), 4, w.n, f) == (size_t)w.n && std::fread(xs.data(), 4, w.n, f) == (size_t)w.n &&
            std::fread(th.data(), 4, w.nparam, f) == w.nparam;
  std::fclose(f);
  if (!ok) return set_err(c, HOPF_EINVAL, std::string(path) + " is not a warm-start checkpoint of this system's network");
  for (float v : th)
    if (!std::isfinite(v)) return set_err(c, HOPF_EINVAL, std::string(path) + " holds non-finite parameters");
  if (hipMemcpy(w.theta, th.data(), w.nparam * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.xm, xm.data(), w.n * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(w.xs, xs.data(), w.n * 4, hipMemcpyHostToDevice) != hipSuccess)
    return set_err(c, HOPF_EDEVICE, "copying the network to the device failed");
  w.t_scale = sc[0];
  w.lam_scale = sc[1];
  w.valid = 1;
  return HOPF_OK;
}

hopf_status hopf_warm_loss_grad(hopf_ctx *h, int sys_id, int nrows, const float *Z, const float *Y, double *loss,
                                float *grad) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c || !Z || !Y || !loss || !grad || nrows < 1) return HOPF_EINVAL;
  if (sys_id < 0 || sys_id >= (int)c->mlp.size() || !c->mlp[sys_id].theta)
    return set_err(c, HOPF_ESTATE, "no warm-start network for this system (call hopf_warm_init)");
  hopf::MlpState &w = c->mlp[sys_id];
  hipSetDevice(c->device);
  hopf::MlpBufs b;
  if (!hopf::alloc_bufs(b, nrows, w.n, w.H, w.nparam)) return set_err(c, HOPF_ENOMEM, "MLP buffers");
  hipMemcpy(b.Z, Z, (size_t)nrows * (w.n + 1) * 4, hipMemcpyHostToDevice);
  hipMemcpy(b.Y, Y, (size_t)nrows * (w.n + 2) * 4, hipMemcpyHostToDevice);
  hopf::loss_grad(c->stream, w.theta, b, nrows, w.n, w.H);
  hipStreamSynchronize(c->stream);
  hipMemcpy(loss, b.loss, sizeof(double), hipMemcpyDeviceToHost);
  hipMemcpy(grad, b.grad, w.nparam * 4, hipMemcpyDeviceToHost);
  hipError_t e = hipGetLastError();
  b.free_all();
  if (e != hipSuccess) return set_err(c, HOPF_EDEVICE, hipGetErrorString(e));
  return HOPF_OK;
}

hopf_status hopf_warm_train(hopf_ctx *h, int sys_id, long npts, const double *x, int epochs, int batch, float lr,
                            unsigned seed, double *epoch_loss, long *pairs) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c || !x || npts < 1 || epochs < 0 || batch < 1 || !(lr > 0.0f)) return HOPF_EINVAL;
  if (sys_id < 0 || sys_id >= (int)c->sys.size()) return set_err(c, HOPF_EINVAL, "sys_id out of range");
  hipSetDevice(c->device);
  if ((int)c->mlp.size() < (int)c->sys.size()) c->mlp.resize(c->sys.size());
  hopf::MlpState &w = c->mlp[sys_id];
  if (!w.theta) {
    hopf_status st = hopf_warm_init(h, sys_id, seed);
    if (st != HOPF_OK) return st;
  }
  const hopf::SysTables &tab = c->sys[sys_id];
  const int n = tab.n, np = tab.n_pad;
  // the network sees the start point in the solver's coordinates (rotated
  // when the target matrix is not diagonal), as the probe setup does
  std::vector<double> xr;
  const double *xf = x;
  if (tab.rotated) {
    xr.assign((size_t)npts * n, 0.0);
    for (long p = 0; p < npts; ++p)
      for (int j = 0; j < n; ++j) {
        const double v = x[p * n + j];
        for (int i = 0; i < n; ++i) xr[(size_t)p * n + i] += tab.U[(size_t)j * n + i] * v;
      }
    xf = xr.data();
  }
  // input normalisation from the training points
  std::vector<float> xm(n, 0.0f), xs(n, 1.0f);
  for (int i = 0; i < n; ++i) {
    double s = 0.0, s2 = 0.0;
    for (long p = 0; p < npts; ++p) { const double v = xf[p * n + i]; s += v; s2 += v * v; }
    const double mu = s / npts, var = std::max(s2 / npts - mu * mu, 1e-24);
    xm[i] = (float)mu;
    xs[i] = (float)std::sqrt(var);
  }
  hipMemcpy(w.xm, xm.data(), n * 4, hipMemcpyHostToDevice);
  hipMemcpy(w.xs, xs.data(), n * 4, hipMemcpyHostToDevice);
  w.t_scale = (float)tab.desc.t_max;
  // 1. solve the training points with the probe log on
  const long cap = npts * 48;
  double *dx = nullptr, *dxf = nullptr, *dT = nullptr, *dgap = nullptr;
  int *dst = nullptr, *dsid = nullptr;
  hopf_status rc = HOPF_OK;
  auto al = [&](void **p, size_t b) { if (rc == HOPF_OK && hipMalloc(p, b) != hipSuccess) rc = HOPF_ENOMEM; };
  al((void **)&dx, (size_t)npts * n * 8);
  if (tab.rotated) al((void **)&dxf, (size_t)npts * n * 8);
  al((void **)&dT, npts * 8);
  al((void **)&dgap, npts * 8);
  al((void **)&dst, npts * 4);
  al((void **)&c->log_pt, cap * 4);
  al((void **)&c->log_T, cap * 4);
  al((void **)&c->log_lam, (size_t)cap * np * 4);
  if (sys_id != 0) al((void **)&dsid, npts * 4);
  hopf::MlpBufs b;
  int *didx = nullptr;
  double *dss = nullptr;
  if (rc == HOPF_OK) {
    c->log_cap = cap;
    c->log_count = 0;
    hipMemcpy(dx, x, (size_t)npts * n * 8, hipMemcpyHostToDevice);
    if (dxf) hipMemcpy(dxf, xf, (size_t)npts * n * 8, hipMemcpyHostToDevice);
    if (dsid) {
      std::vector<int> ids(npts, sys_id);
      hipMemcpy(dsid, ids.data(), npts * 4, hipMemcpyHostToDevice);
    }
    rc = hopf::solve_dev(c, 1, npts, dsid, dx, nullptr, nullptr, nullptr, dT, dgap, nullptr, nullptr, nullptr,
                         nullptr, nullptr, dst, nullptr);
  }
  const long rows = c->log_count;
  if (pairs) *pairs = rows;
  if (rc == HOPF_OK && rows < 1) rc = set_err(c, HOPF_ESTATE, "the training solve logged no probes");
  // 2. costate scale
  if (rc == HOPF_OK) {
    al((void **)&dss, 8);
    if (rc == HOPF_OK) {
      hipMemset(dss, 0, 8);
      hopf::k_sumsq_rows<<<(unsigned)((rows + 255) / 256), 256, 0, c->stream>>>(c->log_lam, rows, n, np, dss);
      double ss = 0.0;
      hipStreamSynchronize(c->stream);
      hipMemcpy(&ss, dss, 8, hipMemcpyDeviceToHost);
      w.lam_scale = (float)std::max(std::sqrt(ss / ((double)rows * n)), 1e-12);
    }
  }
  // 3. Adam epochs over shuffled rows
  if (rc == HOPF_OK) {
    const int Bn = (int)std::min<long>(batch, rows);
    if (!hopf::alloc_bufs(b, Bn, n, w.H, w.nparam)) rc = set_err(c, HOPF_ENOMEM, "MLP buffers");
    al((void **)&didx, rows * 4);
  }
  if (rc == HOPF_OK) {
    std::vector<int> order(rows);
    for (long i = 0; i < rows; ++i) order[i] = (int)i;
    std::mt19937_64 rng(seed ^ 0x9e3779b97f4a7c15ULL);
    const int Bn = b.cap;
    for (int ep = 0; ep < epochs; ++ep) {
      std::shuffle(order.begin(), order.end(), rng);
      hipMemcpy(didx, order.data(), rows * 4, hipMemcpyHostToDevice);
      // the epoch's loss is summed on the device and read once at its end
      // (the stream is idle then, so the next epoch's order can be copied in)
      long seen = 0;
      hopf::k_zero_d<<<1, 64, 0, c->stream>>>(b.esum);
      for (long s0 = 0; s0 + Bn <= rows || (s0 == 0 && rows < Bn); s0 += Bn) {
        const int nb = (int)std::min<long>(Bn, rows - s0);
        hopf::k_make_rows<<<nb, 128, 0, c->stream>>>(didx + s0, nb, c->log_pt, c->log_T, c->log_lam, np,
                                                     dxf ? dxf : dx, dT, dst,
                                                     n, w.xm, w.xs, w.t_scale, w.lam_scale, b.Z, b.Y);
        hopf::loss_grad(c->stream, w.theta, b, nb, n, w.H, b.esum);
        w.step += 1;
        const float c1 = 1.0f - std::pow(0.9f, (float)w.step), c2 = 1.0f - std::pow(0.999f, (float)w.step);
        hopf::k_adam<<<(unsigned)((w.nparam + 255) / 256), 256, 0, c->stream>>>(w.theta, b.grad, w.m, w.v,
                                                                                 (long)w.nparam, lr, c1, c2);
        seen += nb;
      }
      double tot = 0.0;
      hipMemcpyAsync(&tot, b.esum, 8, hipMemcpyDeviceToHost, c->stream);
      hipStreamSynchronize(c->stream);
      if (epoch_loss) epoch_loss[ep] = seen ? tot / seen : 0.0;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) rc = set_err(c, HOPF_EDEVICE, hipGetErrorString(e));
    else w.valid = 1;
  }
  b.free_all();
  hipFree(didx); hipFree(dss); hipFree(dx); hipFree(dxf); hipFree(dT); hipFree(dgap); hipFree(dst); hipFree(dsid);
  hipFree(c->log_pt); hipFree(c->log_T); hipFree(c->log_lam);
  c->log_pt = nullptr; c->log_T = nullptr; c->log_lam = nullptr;
  c->log_cap = 0;
  if (rc != HOPF_OK && c->err.empty()) c->err = "warm-start training failed";
  return rc;
}

}  // extern "C"
