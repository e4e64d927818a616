// Host side of the library: argument validation, the FP64 node tables built
// once per system, and the C-ABI entry points that marshal host arrays.
//
// Tables (paper Sec. III-A, eqs. (16)-(20), in the terminal costate
// lam = e^{-T A^T} p): K_k = -Qu^T B^T e^{tau_k A^T} at the time-to-go nodes
// tau_k = k h.  The matrix exponential is the scaling-and-squaring method
// with a diagonal [13/13] Pade approximant (Higham, SIAM J. Matrix Anal.
// Appl. 26 (2005)); the paper evaluates the same exponential action with
// Al-Mohy & Higham's algorithm (Sec. VI).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hopf_internal.h"

namespace hopf {

hopf_status set_err(Ctx *ctx, hopf_status st, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return st;
}

namespace {

using Mat = std::vector<double>;  // row-major n x n

void matmul(const double *A, const double *B, double *C, int n, int k, int m) {
  // C (n x m) = A (n x k) * B (k x m)
  std::fill(C, C + (size_t)n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      const double a = A[(size_t)i * k + l];
      if (a == 0.0) continue;
      const double *b = B + (size_t)l * m;
      double *c = C + (size_t)i * m;
      for (int j = 0; j < m; ++j) c[j] += a * b[j];
    }
}

double norm1(const Mat &A, int n) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += std::fabs(A[(size_t)i * n + j]);
    best = std::max(best, s);
  }
  return best;
}

// Solve P X = R in place (R becomes X), LU with partial pivoting.
bool lu_solve(Mat P, Mat &R, int n) {
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(P[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double v = std::fabs(P[(size_t)i * n + k]);
      if (v > best) { best = v; p = i; }
    }
    if (best == 0.0 || !std::isfinite(best)) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) {
        std::swap(P[(size_t)k * n + j], P[(size_t)p * n + j]);
        std::swap(R[(size_t)k * n + j], R[(size_t)p * n + j]);
      }
    }
    const double inv = 1.0 / P[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      const double f = P[(size_t)i * n + k] * inv;
      if (f == 0.0) continue;
      for (int j = k; j < n; ++j) P[(size_t)i * n + j] -= f * P[(size_t)k * n + j];
      for (int j = 0; j < n; ++j) R[(size_t)i * n + j] -= f * R[(size_t)k * n + j];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    const double inv = 1.0 / P[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      double s = R[(size_t)k * n + j];
      for (int l = k + 1; l < n; ++l) s -= P[(size_t)k * n + l] * R[(size_t)l * n + j];
      R[(size_t)k * n + j] = s * inv;
    }
  }
  return true;
}

// Diagonal Pade [13/13] coefficients b_j = (26-j)! 13! / (26! j! (13-j)!).
std::vector<double> pade13() {
  std::vector<double> b(14);
  for (int j = 0; j <= 13; ++j) {
    double lg = std::lgamma(27.0 - j) + std::lgamma(14.0) - std::lgamma(27.0) - std::lgamma(j + 1.0) -
                std::lgamma(14.0 - j);
    b[j] = std::exp(lg);
  }
  return b;
}

// e^{X} for ||X||_1 <= 0.5 by the Pade approximant alone.
bool pade_exp(const Mat &X, Mat &out, int n) {
  static const std::vector<double> b = pade13();
  const size_t nn = (size_t)n * n;
  Mat X2(nn), X4(nn), X6(nn), t1(nn), t2(nn), U(nn), V(nn);
  matmul(X.data(), X.data(), X2.data(), n, n, n);
  matmul(X2.data(), X2.data(), X4.data(), n, n, n);
  matmul(X4.data(), X2.data(), X6.data(), n, n, n);
  for (size_t i = 0; i < nn; ++i) t1[i] = b[13] * X6[i] + b[11] * X4[i] + b[9] * X2[i];
  matmul(X6.data(), t1.data(), t2.data(), n, n, n);
  for (size_t i = 0; i < nn; ++i) t2[i] += b[7] * X6[i] + b[5] * X4[i] + b[3] * X2[i];
  for (int i = 0; i < n; ++i) t2[(size_t)i * n + i] += b[1];
  matmul(X.data(), t2.data(), U.data(), n, n, n);             // odd part
  for (size_t i = 0; i < nn; ++i) t1[i] = b[12] * X6[i] + b[10] * X4[i] + b[8] * X2[i];
  matmul(X6.data(), t1.data(), V.data(), n, n, n);
  for (size_t i = 0; i < nn; ++i) V[i] += b[6] * X6[i] + b[4] * X4[i] + b[2] * X2[i];
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] += b[0];  // even part
  Mat P(nn), R(nn);
  for (size_t i = 0; i < nn; ++i) { P[i] = V[i] - U[i]; R[i] = V[i] + U[i]; }
  if (!lu_solve(P, R, n)) return false;
  out.swap(R);
  return true;
}

bool expm(const Mat &A, double t, Mat &out, int n) {
  Mat X(A);
  for (auto &v : X) v *= t;
  int s = 0;
  double nrm = norm1(X, n);
  while (nrm > 0.5) { nrm *= 0.5; ++s; }
  const double sc = std::ldexp(1.0, -s);
  for (auto &v : X) v *= sc;
  if (!pade_exp(X, out, n)) return false;
  Mat tmp(out.size());
  for (int i = 0; i < s; ++i) {
    matmul(out.data(), out.data(), tmp.data(), n, n, n);
    out.swap(tmp);
  }
  return true;
}

// Symmetric eigendecomposition W = U diag(d) U^T by cyclic Jacobi rotations
// (U orthogonal, row-major; column k is the eigenvector of d[k]).
void sym_eig(const Mat &W, int n, Mat &U, std::vector<double> &d) {
  Mat a(W);
  U.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = a[(size_t)i * n + j] * a[(size_t)i * n + j];
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
          a[(size_t)k * n + p] = c * akp - sn * akq;
          a[(size_t)k * n + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
          a[(size_t)p * n + k] = c * apk - sn * aqk;
          a[(size_t)q * n + k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double ukp = U[(size_t)k * n + p], ukq = U[(size_t)k * n + q];
          U[(size_t)k * n + p] = c * ukp - sn * ukq;
          U[(size_t)k * n + q] = sn * ukp + c * ukq;
        }
      }
  }
  d.resize(n);
  for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
}

bool all_finite(const double *p, size_t k) {
  for (size_t i = 0; i < k; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

void free_tables(SysTables &t) {
  hipFree(t.K32); hipFree(t.K64); hipFree(t.K32T); hipFree(t.K64T); hipFree(t.lpref_d); hipFree(t.epow_d);
  hipFree(t.hbin_d); hipFree(t.rdig_d); hipFree(t.At_d); hipFree(t.U_d);
  t.hbin_d = t.rdig_d = t.At_d = t.U_d = nullptr;
  hipFree(t.Kd16h); hipFree(t.Kd16l); hipFree(t.Kp16h); hipFree(t.Kp16l);
  t.K32T = nullptr; t.K64T = nullptr;
  t.Kd16h = t.Kd16l = t.Kp16h = t.Kp16l = nullptr;
  hipFree(t.A_d); hipFree(t.BQ_d); hipFree(t.Wd_d); hipFree(t.c_d); hipFree(t.Eh_d); hipFree(t.Qu_d);
  hipFree(t.kron_winv_d);
  t.kron_winv_d = nullptr;
  t.Eh_d = nullptr; t.Qu_d = nullptr;
  t.K32 = nullptr; t.K64 = nullptr; t.lpref_d = nullptr; t.epow_d = nullptr;
  t.A_d = nullptr; t.BQ_d = nullptr; t.Wd_d = nullptr; t.c_d = nullptr;
}

hopf_status build_tables(Ctx *ctx, const hopf_system &s, SysTables &t) {
  const int n = s.n, m = s.m, N = s.N;
  if (n < 1 || n > 256 || m < 1 || m > 64 || N < 2 || N > 4096)
    return set_err(ctx, HOPF_EINVAL, "system sizes out of range (1<=n<=256, 1<=m<=64, 2<=N<=4096)");
  if (!(s.t_max > 0.0) || !std::isfinite(s.t_max)) return set_err(ctx, HOPF_EINVAL, "t_max must be finite and > 0");
  if (!(s.c_tau >= 0.0) || !std::isfinite(s.c_tau)) return set_err(ctx, HOPF_EINVAL, "c_tau must be finite and >= 0");
  if (s.quad != HOPF_Q_TRAP && s.quad != HOPF_Q_LEFT) return set_err(ctx, HOPF_EINVAL, "bad quadrature rule");
  if (s.uset != HOPF_U_L2 && s.uset != HOPF_U_BOX) return set_err(ctx, HOPF_EINVAL, "bad control set");
  if (!s.A || !s.B || !s.W) return set_err(ctx, HOPF_EINVAL, "A, B and W are required");
  t.desc = s;
  t.n = n; t.N = N;
  t.m_user = m;
  // the kernels hold the m components of a node in registers with m fixed at
  // compile time; the tables are padded with zero components up to that size
  // (zero rows of K leave every norm and clamp unchanged)
  {
    static const int kMM[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};
    int mk = m;
    for (int v : kMM)
      if (v >= m) { mk = v; break; }
    t.m = mk;
  }
  t.A.assign(s.A, s.A + (size_t)n * n);
  t.B.assign(s.B, s.B + (size_t)n * m);
  t.W.assign(s.W, s.W + (size_t)n * n);
  t.Qu.assign((size_t)m * m, 0.0);
  if (s.Qu) t.Qu.assign(s.Qu, s.Qu + (size_t)m * m);
  else for (int i = 0; i < m; ++i) t.Qu[(size_t)i * m + i] = 1.0;
  t.c.assign(n, 0.0);
  if (s.c) t.c.assign(s.c, s.c + n);
  if (!all_finite(t.A.data(), t.A.size()) || !all_finite(t.B.data(), t.B.size()) ||
      !all_finite(t.W.data(), t.W.size()) || !all_finite(t.Qu.data(), t.Qu.size()) ||
      !all_finite(t.c.data(), t.c.size()))
    return set_err(ctx, HOPF_EINVAL, "non-finite system data");
  // W must be symmetric positive definite.  A diagonal W is used as is; any
  // other is diagonalised, W = U diag(d) U^T, and the system is solved in the
  // rotated state x' = U^T x (A' = U^T A U, B' = U^T B, c' = U^T c, W' = diag(d)):
  // an orthogonal change of coordinates leaves phi, T*, u and the certified
  // gap unchanged, and the library rotates x in and lam, x(s), p* out.
  {
    double wmax = 0.0;
    bool diag = true;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        wmax = std::max(wmax, std::fabs(t.W[(size_t)i * n + j]));
        if (i != j && t.W[(size_t)i * n + j] != 0.0) diag = false;
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j)
        if (std::fabs(t.W[(size_t)i * n + j] - t.W[(size_t)j * n + i]) > 1e-12 * wmax)
          return set_err(ctx, HOPF_EINVAL, "W is not symmetric");
    t.rotated = !diag;
    t.U.clear();
    if (diag) {
      for (int i = 0; i < n; ++i)
        if (!(t.W[(size_t)i * n + i] > 0.0)) return set_err(ctx, HOPF_EINVAL, "W is not positive definite");
    } else {
      std::vector<double> d;
      sym_eig(t.W, n, t.U, d);
      for (int i = 0; i < n; ++i)
        if (!(d[i] > 1e-14 * wmax)) return set_err(ctx, HOPF_EINVAL, "W is not positive definite");
      Mat Ut((size_t)n * n), AU((size_t)n * n), Ar((size_t)n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ut[(size_t)i * n + j] = t.U[(size_t)j * n + i];
      matmul(t.A.data(), t.U.data(), AU.data(), n, n, n);
      matmul(Ut.data(), AU.data(), Ar.data(), n, n, n);
      std::vector<double> Br((size_t)n * m), cr(n, 0.0);
      matmul(Ut.data(), t.B.data(), Br.data(), n, n, m);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) cr[i] += Ut[(size_t)i * n + j] * t.c[j];
      t.A.swap(Ar);
      t.B.swap(Br);
      t.c.swap(cr);
      t.W.assign((size_t)n * n, 0.0);
      for (int i = 0; i < n; ++i) t.W[(size_t)i * n + i] = d[i];
    }
  }
  t.desc.A = t.A.data(); t.desc.B = t.B.data(); t.desc.W = t.W.data();
  t.desc.Qu = t.Qu.data(); t.desc.c = t.c.data();

  t.n_pad = ((n + 15) / 16) * 16;
  t.nkb = (N + NODE_BLOCK - 1) / NODE_BLOCK;
  t.h = (s.quad == HOPF_Q_TRAP) ? s.t_max / (N - 1) : s.t_max / N;
  t.delta = std::ldexp(s.t_max, -POW_BITS);

  // BQ = B Qu (n x m_user), then zero-padded to n x t.m
  const int mu = m;
  std::vector<double> BQu((size_t)n * mu);
  matmul(t.B.data(), t.Qu.data(), BQu.data(), n, mu, mu);
  const int mk = t.m;
  std::vector<double> BQ((size_t)n * mk, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < mu; ++j) BQ[(size_t)i * mk + j] = BQu[(size_t)i * mu + j];

  // node blocks Phi_k = -(e^{k h A} B Qu)^T, by Phi_k = Phi_{k-1} e^{h A^T}
  Mat Eh;
  if (!expm(t.A, t.h, Eh, n)) return set_err(ctx, HOPF_EINVAL, "matrix exponential failed (singular Pade denominator)");
  t.phi.assign((size_t)N * mk * n, 0.0);
  for (int j = 0; j < mk; ++j)
    for (int i = 0; i < n; ++i) t.phi[(size_t)j * n + i] = -BQ[(size_t)i * mk + j];
  for (int k = 1; k < N; ++k) {
    const double *prev = &t.phi[(size_t)(k - 1) * mk * n];
    double *cur = &t.phi[(size_t)k * mk * n];
    for (int j = 0; j < mk; ++j)
      for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int l = 0; l < n; ++l) acc += prev[(size_t)j * n + l] * Eh[(size_t)i * n + l];
        cur[(size_t)j * n + i] = acc;
      }
  }
  if (!all_finite(t.phi.data(), t.phi.size()))
    return set_err(ctx, HOPF_EINVAL, "node table overflowed (e^{t A} too large on [0, t_max])");

  // prefix bounds lpref[j] >= lambda_max(sum_{k<j} Phi_k^T Phi_k): power
  // iteration warm-started from the previous prefix, with a 1e-4 margin; the
  // Frobenius norm is used where the iteration does not settle.
  t.lpref.assign(N + 1, 0.0);
  {
    Mat S((size_t)n * n, 0.0);
    std::vector<double> v(n, 1.0 / std::sqrt((double)n)), w(n);
    for (int j = 1; j <= N; ++j) {
      const double *P = &t.phi[(size_t)(j - 1) * mk * n];
      for (int a = 0; a < mk; ++a)
        for (int i = 0; i < n; ++i) {
          const double pi = P[(size_t)a * n + i];
          if (pi == 0.0) continue;
          for (int l = 0; l < n; ++l) S[(size_t)i * n + l] += pi * P[(size_t)a * n + l];
        }
      double theta = 0.0, prev = -1.0;
      bool conv = false;
      for (int it = 0; it < 3000; ++it) {
        for (int i = 0; i < n; ++i) {
          double acc = 0.0;
          for (int l = 0; l < n; ++l) acc += S[(size_t)i * n + l] * v[l];
          w[i] = acc;
        }
        theta = 0.0;
        double nw = 0.0;
        for (int i = 0; i < n; ++i) { theta += v[i] * w[i]; nw += w[i] * w[i]; }
        nw = std::sqrt(nw);
        if (nw == 0.0) { conv = true; theta = 0.0; break; }
        for (int i = 0; i < n; ++i) v[i] = w[i] / nw;
        if (it >= 8 && std::fabs(theta - prev) <= 1e-13 * theta) { conv = true; break; }
        prev = theta;
      }
      if (conv) {
        t.lpref[j] = theta * (1.0 + 1e-4);
      } else {
        double fro = 0.0;
        for (double x : S) fro += x * x;
        t.lpref[j] = std::sqrt(fro);
      }
    }
  }

  // binary powers e^{2^b delta A}: Pade while the argument is small, then squaring
  t.epow.assign((size_t)POW_LEVELS * n * n, 0.0);
  {
    const double nA = norm1(t.A, n);
    Mat E;
    for (int b = 0; b < POW_LEVELS; ++b) {
      const double tb = std::ldexp(t.delta, b);
      if (b == 0 || tb * nA <= 0.5) {
        Mat X(t.A);
        for (auto &x : X) x *= tb;
        if (tb * nA <= 0.5) {
          if (!pade_exp(X, E, n)) return set_err(ctx, HOPF_EINVAL, "matrix exponential failed");
        } else if (!expm(t.A, tb, E, n)) {
          return set_err(ctx, HOPF_EINVAL, "matrix exponential failed");
        }
      } else {
        Mat prev(t.epow.begin() + (size_t)(b - 1) * n * n, t.epow.begin() + (size_t)b * n * n);
        E.assign((size_t)n * n, 0.0);
        matmul(prev.data(), prev.data(), E.data(), n, n, n);
      }
      std::copy(E.begin(), E.end(), t.epow.begin() + (size_t)b * n * n);
    }
    if (!all_finite(t.epow.data(), t.epow.size()))
      return set_err(ctx, HOPF_EINVAL, "e^{t A} overflows on [0, t_max]");
  }

  // probe-setup powers: e^{2^b h A} by squaring e^{h A}; e^{d 16^b dr A}
  // (d = 1..15) from e^{dr A} by products, dr = h / 16^RDIG_LEVELS
  {
    const int K = (s.quad == HOPF_Q_TRAP) ? N - 1 : N;
    t.n_hbin = 1;
    while ((1 << t.n_hbin) <= K) ++t.n_hbin;
    const size_t nn = (size_t)n * n;
    t.hbin.assign((size_t)t.n_hbin * nn, 0.0);
    std::copy(Eh.begin(), Eh.end(), t.hbin.begin());
    for (int b = 1; b < t.n_hbin; ++b)
      matmul(&t.hbin[(b - 1) * nn], &t.hbin[(b - 1) * nn], &t.hbin[b * nn], n, n, n);
    t.dr = std::ldexp(t.h, -4 * RDIG_LEVELS);
    Mat base;
    if (!expm(t.A, t.dr, base, n)) return set_err(ctx, HOPF_EINVAL, "matrix exponential failed");
    t.rdig.assign((size_t)RDIG_LEVELS * 15 * nn, 0.0);
    Mat unit(base);   // e^{16^b dr A}
    for (int b = 0; b < RDIG_LEVELS; ++b) {
      double *lev = &t.rdig[(size_t)b * 15 * nn];
      std::copy(unit.begin(), unit.end(), lev);
      for (int d = 2; d <= 15; ++d) matmul(&lev[(d - 2) * nn], unit.data(), &lev[(d - 1) * nn], n, n, n);
      Mat next(nn);
      matmul(&lev[14 * nn], unit.data(), next.data(), n, n, n);   // e^{16^{b+1} dr A}
      unit.swap(next);
    }
    double ninf = 0.0;
    for (int i = 0; i < n; ++i) {
      double r = 0.0;
      for (int j = 0; j < n; ++j) r += std::fabs(t.A[(size_t)i * n + j]);
      ninf = std::max(ninf, r);
    }
    t.anorm = std::max(norm1(t.A, n), ninf);
    if (!all_finite(t.hbin.data(), t.hbin.size()) || !all_finite(t.rdig.data(), t.rdig.size()))
      return set_err(ctx, HOPF_EINVAL, "e^{t A} overflows on [0, t_max]");
  }

  // device copies in the kernels' layout: K[kb][j][kk][i] = Phi_{16 kb + kk}[j][i]
  const size_t kel = (size_t)t.nkb * mk * NODE_BLOCK * t.n_pad;
  std::vector<float> K32(kel, 0.0f), K32T(kel, 0.0f);
  std::vector<double> K64(kel, 0.0), K64T(kel, 0.0);
  std::vector<__bf16> Kdh(kel, (__bf16)0.0f), Kdl(kel, (__bf16)0.0f), Kph(kel, (__bf16)0.0f), Kpl(kel, (__bf16)0.0f);
  for (int k = 0; k < N; ++k) {
    const int kb = k / NODE_BLOCK, kk = k % NODE_BLOCK;
    for (int j = 0; j < mk; ++j)
      for (int i = 0; i < n; ++i) {
        const size_t dst = (((size_t)kb * mk + j) * NODE_BLOCK + kk) * t.n_pad + i;
        const size_t dstT = (((size_t)kb * mk + j) * t.n_pad + i) * NODE_BLOCK + kk;
        const double v = t.phi[((size_t)k * mk + j) * n + i];
        K64[dst] = v;
        K32[dst] = (float)v;
        K64T[dstT] = v;
        K32T[dstT] = (float)v;
        // hi = bf16(v), lo = bf16(v - hi), both rounded to nearest even
        const __bf16 hi = (__bf16)(float)v;
        const __bf16 lo = (__bf16)(float)(v - (double)(float)hi);
        Kdh[dst] = hi; Kdl[dst] = lo; Kph[dstT] = hi; Kpl[dstT] = lo;
      }
  }
  std::vector<double> Wd(t.n_pad, 1.0), cc(t.n_pad, 0.0);
  for (int i = 0; i < n; ++i) { Wd[i] = t.W[(size_t)i * n + i]; cc[i] = t.c[i]; }
  std::vector<double> mBQ(BQ);
  for (auto &v : mBQ) v = -v;
  // the probe setup reads its matrices by columns
  auto by_columns = [n](const std::vector<double> &src) {
    const size_t nn = (size_t)n * n;
    std::vector<double> dst(src.size());
    for (size_t b = 0; b < src.size() / nn; ++b)
      for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) dst[b * nn + (size_t)k * n + i] = src[b * nn + (size_t)i * n + k];
    return dst;
  };
  const std::vector<double> hbin_c = by_columns(t.hbin), rdig_c = by_columns(t.rdig), A_c = by_columns(t.A);

  free_tables(t);
  auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
    if (hipMalloc(dst, bytes) != hipSuccess) return false;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool ok = up((void **)&t.K32, K32.data(), kel * sizeof(float)) &&
            up((void **)&t.K64, K64.data(), kel * sizeof(double)) &&
            up((void **)&t.K32T, K32T.data(), kel * sizeof(float)) &&
            up((void **)&t.K64T, K64T.data(), kel * sizeof(double)) &&
            up((void **)&t.Kd16h, Kdh.data(), kel * sizeof(__bf16)) &&
            up((void **)&t.Kd16l, Kdl.data(), kel * sizeof(__bf16)) &&
            up((void **)&t.Kp16h, Kph.data(), kel * sizeof(__bf16)) &&
            up((void **)&t.Kp16l, Kpl.data(), kel * sizeof(__bf16)) &&
            up((void **)&t.lpref_d, t.lpref.data(), t.lpref.size() * sizeof(double)) &&
            up((void **)&t.epow_d, t.epow.data(), t.epow.size() * sizeof(double)) &&
            up((void **)&t.hbin_d, hbin_c.data(), hbin_c.size() * sizeof(double)) &&
            up((void **)&t.rdig_d, rdig_c.data(), rdig_c.size() * sizeof(double)) &&
            up((void **)&t.At_d, A_c.data(), A_c.size() * sizeof(double)) &&
            up((void **)&t.A_d, t.A.data(), t.A.size() * sizeof(double)) &&
            up((void **)&t.BQ_d, mBQ.data(), mBQ.size() * sizeof(double)) &&
            up((void **)&t.Wd_d, Wd.data(), Wd.size() * sizeof(double)) &&
            up((void **)&t.c_d, cc.data(), cc.size() * sizeof(double)) &&
            up((void **)&t.Eh_d, Eh.data(), Eh.size() * sizeof(double)) &&
            up((void **)&t.Qu_d, t.Qu.data(), t.Qu.size() * sizeof(double)) &&
            (!t.rotated || up((void **)&t.U_d, t.U.data(), t.U.size() * sizeof(double)));
  if (!ok) {
    free_tables(t);
    return set_err(ctx, HOPF_ENOMEM, "device allocation/copy of the node tables failed");
  }
  return HOPF_OK;
}

}  // namespace hopf

using hopf::Ctx;
using hopf::set_err;

extern "C" {

hopf_status hopf_default_opts(hopf_opts *o) {
  if (!o) return HOPF_EINVAL;
  o->c_tau = 1.0;
  o->gap_tol = 1e-6;
  o->t_rel_tol = 0.5e-4;
  o->t_abs_frac = 1e-6;
  o->max_iter = 200000;
  o->check_every = 50;
  o->warm = HOPF_WARM_COLD;
  o->prec = HOPF_FP32;
  o->root = HOPF_ROOT_BISECT;
  o->newton_after = 1;
  o->newton_rho = 0.5;
  o->tail_max = 2048;
  o->adapt = 1;
  o->scan = 48;
  o->wide_min = 16384;
  o->deep_max = -1;
  o->structure = 1;
  return HOPF_OK;
}

const char *hopf_strerror(hopf_status s) {
  switch (s) {
    case HOPF_OK: return "ok";
    case HOPF_EINVAL: return "invalid argument";
    case HOPF_ENOMEM: return "out of memory";
    case HOPF_EDEVICE: return "HIP device error";
    case HOPF_ESTATE: return "call out of order";
    case HOPF_EUNSUPPORTED: return "not supported by the library";
  }
  return "unknown status";
}

hopf_status hopf_create(int device, hopf_ctx **out) {
  if (!out) return HOPF_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HOPF_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return HOPF_EDEVICE;
  Ctx *c = new (std::nothrow) Ctx();
  if (!c) return HOPF_ENOMEM;
  c->device = device;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1)
    c->n_cu = 1;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return HOPF_EDEVICE;
  }
  hopf_default_opts(&c->opts);
  // the no-allocation entry point's scratch: its address on this device
  if (hopf::scratch_init(device, &c->scratch) != HOPF_OK) {
    hipStreamDestroy(c->stream);
    delete c;
    return HOPF_EDEVICE;
  }
  *out = reinterpret_cast<hopf_ctx *>(c);
  return HOPF_OK;
}

void hopf_destroy(hopf_ctx *h) {
  if (!h) return;
  Ctx *c = reinterpret_cast<Ctx *>(h);
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto &t : c->sys) hopf::free_tables(t);
  for (auto &t : c->ksys) hopf::free_tables(t);
  for (auto &w : c->mlp) hopf::mlp_free(w);
  for (auto &v : c->jbufs)
    for (auto &b : v) hipFree(b.p);
  for (auto &ps : c->pool) {
    hipStreamSynchronize(ps);
    hipStreamDestroy(ps);
  }
  for (auto &e : c->evpool) hipEventDestroy(e);
  if (c->hcount) hipHostFree(c->hcount);
  hipFree(c->net_buf);
  hipStreamDestroy(c->stream);
  delete c;
}

const char *hopf_last_error(const hopf_ctx *h) {
  if (!h) return "null context";
  return reinterpret_cast<const Ctx *>(h)->err.c_str();
}

hopf_status hopf_set_opts(hopf_ctx *h, const hopf_opts *o) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c || !o) return HOPF_EINVAL;
  if (!(o->c_tau > 0.0) || !(o->gap_tol > 0.0) || !(o->t_rel_tol >= 0.0) || !(o->t_abs_frac >= 0.0) ||
      o->max_iter < 1 || o->check_every < 1 || o->warm < 0 || o->warm > 4 || o->prec < 0 || o->prec > 2 ||
      o->root < 0 || o->root > 1 || o->newton_after < 0 || !(o->newton_rho > 0.0) ||
      o->tail_max < 0 || o->tail_max > 8192 || o->adapt < 0 || o->adapt > 1 || o->scan < 1 || o->scan > 4096 || o->wide_min < 0 ||
      o->deep_max < -1 || o->structure < 0 || o->structure > 1)
    return set_err(c, HOPF_EINVAL, "invalid solver options");
  c->opts = *o;
  return HOPF_OK;
}

namespace hopf {

// The smallest block size b (n = k b, k > 1) for which the system is k copies
// of one b-dimensional system sharing the control (A = I_k (x) A_b, B = 1_k (x)
// B_b, c = 1_k (x) c_b, W block-diagonal with blocks W_b / alpha_c, W_b
// diagonal, alpha_0 = 1, alpha_c > 0), or 0; alpha receives the k weights.
// Blocks must match to 1e-14 relative; the system's own coordinates.
int kron_block(const SysTables &t, std::vector<double> &alpha) {
  const int n = t.n, m = t.m_user;
  if (t.rotated) return 0;
  double amax = 0.0, bmax = 0.0;
  for (double v : t.A) amax = std::max(amax, std::fabs(v));
  for (double v : t.B) bmax = std::max(bmax, std::fabs(v));
  auto close = [](double a, double b, double scale) { return std::fabs(a - b) <= 1e-14 * std::max(scale, 1e-300); };
  for (int b = 1; 2 * b <= n && b <= KRON_BMAX; ++b) {
    if (n % b) continue;
    const int k = n / b;
    bool ok = true;
    for (int i = 0; i < n && ok; ++i)
      for (int j = 0; j < n && ok; ++j) {
        const int ci = i / b, cj = j / b;
        const double v = t.A[(size_t)i * n + j];
        if (ci != cj) ok = v == 0.0;
        else ok = close(v, t.A[(size_t)(i % b) * n + (j % b)], amax);
      }
    for (int i = b; i < n && ok; ++i)
      for (int j = 0; j < m && ok; ++j) ok = close(t.B[(size_t)i * m + j], t.B[(size_t)(i % b) * m + j], bmax);
    alpha.assign(k, 1.0);
    for (int cc = 1; cc < k && ok; ++cc) {
      const double a = t.W[0] / t.W[(size_t)(cc * b) * n + cc * b];
      ok = a > 0.0 && std::isfinite(a);
      for (int r = 0; r < b && ok; ++r) {
        const int i = cc * b + r;
        ok = close(t.W[(size_t)r * n + r] / t.W[(size_t)i * n + i], a, a) && t.c[i] == t.c[r];
      }
      alpha[cc] = a;
    }
    if (ok && k > 1) return b;
  }
  return 0;
}

}  // namespace hopf

hopf_status hopf_set_systems(hopf_ctx *h, int nsys, const hopf_system *sys) {
  Ctx *c = reinterpret_cast<Ctx *>(h);
  if (!c) return HOPF_EINVAL;
  if (nsys < 1 || !sys) return set_err(c, HOPF_EINVAL, "need at least one system");
  if (hipSetDevice(c->device) != hipSuccess) return set_err(c, HOPF_EDEVICE, "hipSetDevice failed");
  hipStreamSynchronize(c->stream);
  for (auto &t : c->sys) hopf::free_tables(t);
  for (auto &t : c->ksys) hopf::free_tables(t);
  for (auto &w : c->mlp) hopf::mlp_free(w);
  c->mlp.clear();
  c->sys.clear();
  c->ksys.clear();
  std::vector<hopf::SysTables> tabs(nsys), ktabs;
  auto fail = [&](int i, hopf_status st) {
    for (auto &t : tabs) hopf::free_tables(t);
    for (auto &t : ktabs) hopf::free_tables(t);
    c->err = "system " + std::to_string(i) + ": " + c->err;
    return st;
  };
  for (int i = 0; i < nsys; ++i) {
    hopf_status st = hopf::build_tables(c, sys[i], tabs[i]);
    if (st != HOPF_OK) return fail(i, st);
    // Kronecker structure: the reduced system of the copies' weighted mean,
    // target matrix W_b / a with a = sum_c a_c (a z^T W_b^-1 z = z^T (W_b / a)^-1 z)
    hopf::SysTables &t = tabs[i];
    std::vector<double> alpha;
    const int b = hopf::kron_block(t, alpha);
    if (b > 0) {
      const int k = t.n / b, m = t.m_user;
      double atot = 0.0;
      for (double a : alpha) atot += a;
      std::vector<double> Ab((size_t)b * b), Bb((size_t)b * m), Wb((size_t)b * b, 0.0), cb(b);
      for (int r = 0; r < b; ++r) {
        for (int j = 0; j < b; ++j) Ab[(size_t)r * b + j] = t.A[(size_t)r * t.n + j];
        for (int j = 0; j < m; ++j) Bb[(size_t)r * m + j] = t.B[(size_t)r * m + j];
        Wb[(size_t)r * b + r] = t.W[(size_t)r * t.n + r] / atot;
        cb[r] = t.c[r];
      }
      hopf_system rs = sys[i];
      rs.n = b;
      rs.A = Ab.data();
      rs.B = Bb.data();
      rs.W = Wb.data();
      rs.c = cb.data();
      rs.Qu = t.Qu.data();
      ktabs.emplace_back();
      st = hopf::build_tables(c, rs, ktabs.back());
      if (st != HOPF_OK) return fail(i, st);
      t.kron_k = k;
      t.kron_b = b;
      t.kron_red = (int)ktabs.size() - 1;
      // [winv (b) | alpha (k)]: 1 / diag(W_b) and the copies' weights
      t.kron_winv.resize(b + k);
      for (int r = 0; r < b; ++r) t.kron_winv[r] = 1.0 / t.W[(size_t)r * t.n + r];
      for (int cc = 0; cc < k; ++cc) t.kron_winv[b + cc] = alpha[cc];
      t.kron_atot = atot;
      if (hipMalloc((void **)&t.kron_winv_d, (b + k) * sizeof(double)) != hipSuccess ||
          hipMemcpy(t.kron_winv_d, t.kron_winv.data(), (b + k) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return fail(i, set_err(c, HOPF_ENOMEM, "device copy of the copies' target weights failed"));
    }
  }
  c->sys.swap(tabs);
  c->ksys.swap(ktabs);
  return HOPF_OK;
}

hopf_status hopf_last_timing(const hopf_ctx *h, hopf_timing *out) {
  const Ctx *c = reinterpret_cast<const Ctx *>(h);
  if (!c || !out) return HOPF_EINVAL;
  out->total_s = c->t_total;
  out->iter_kernel_s = c->t_iter;
  out->iter_launches = c->iter_launches;
  out->iter_point_rows = c->point_rows;
  out->alg_flops = c->alg_flops;
  out->tail_kernel_s = c->t_tail;
  out->tail_point_rows = c->tail_rows;
  out->tail_points = c->tail_points;
  out->wide_kernel_s = c->t_wide;
  out->wide_launches = c->wide_launches;
  out->wide_point_rows = c->wide_rows;
  return HOPF_OK;
}

}  // extern "C"
