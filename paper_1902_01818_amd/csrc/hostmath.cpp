// Host-side numerics of the setup phase (see hostmath.h).
#include "hostmath.h"

#include <algorithm>
#include <cmath>

namespace igamg {

GaussRule gauss_rule(int q) {
  if (q < 1 || q > MAXQ) fail(IGAMG_EINVAL, "Gauss rule size out of range");
  GaussRule g{};
  g.q = q;
  for (int i = 0; i < q; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 1; k < q; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = x; p0 = 1.0; }
      dp = q * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    // recompute derivative at the converged node for the weight
    double p0 = 1.0, p1 = x;
    for (int k = 1; k < q; ++k) {
      double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = x; p0 = 1.0; }
    dp = q * (x * p1 - p0) / (x * x - 1.0);
    // nodes come out in descending order of x; store ascending on [0,1]
    g.x[q - 1 - i] = 0.5 * (1.0 + x);
    g.w[q - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
  return g;
}

std::vector<double> open_knots(int n_el, int p) {
  std::vector<double> t;
  for (int i = 0; i <= p; ++i) t.push_back(0.0);
  for (int j = 1; j < n_el; ++j) t.push_back((double)j / (double)n_el);
  for (int i = 0; i <= p; ++i) t.push_back(1.0);
  return t;
}

void bspline_span_ders(const std::vector<double> &t, int p, int m, double x, int nd,
                       double out[][MAXP + 1]) {
  // N[j][a]: degree-j splines N_{m-j+a, j}(x), a = 0..j
  double N[MAXP + 1][MAXP + 1];
  N[0][0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    for (int a = 0; a <= j; ++a) {
      int i = m - j + a;
      double v = 0.0;
      if (a >= 1) {
        double den = t[i + j] - t[i];
        if (den > 0) v += (x - t[i]) / den * N[j - 1][a - 1];
      }
      if (a <= j - 1) {
        double den = t[i + j + 1] - t[i + 1];
        if (den > 0) v += (t[i + j + 1] - x) / den * N[j - 1][a];
      }
      N[j][a] = v;
    }
  }
  for (int k = 0; k <= nd; ++k) {
    for (int a = 0; a <= MAXP; ++a) out[k][a] = 0.0;
    if (k > p) continue;
    // start from degree p-k, differentiate k times
    double W[MAXP + 1];
    int j0 = p - k;
    for (int a = 0; a <= j0; ++a) W[a] = N[j0][a];
    for (int j = j0 + 1; j <= p; ++j) {
      double Wn[MAXP + 1];
      for (int a = 0; a <= j; ++a) {
        int i = m - j + a;
        double v = 0.0;
        if (a >= 1) {
          double den = t[i + j] - t[i];
          if (den > 0) v += j * W[a - 1] / den;
        }
        if (a <= j - 1) {
          double den = t[i + j + 1] - t[i + 1];
          if (den > 0) v -= j * W[a] / den;
        }
        Wn[a] = v;
      }
      for (int a = 0; a <= j; ++a) W[a] = Wn[a];
    }
    for (int a = 0; a <= p; ++a) out[k][a] = W[a];
  }
}

void element_tables(int n_el, int p, const GaussRule &gr, std::vector<double> &B,
                    std::vector<double> &D) {
  std::vector<double> t = open_knots(n_el, p);
  int q = gr.q;
  B.assign((size_t)n_el * q * (p + 1), 0.0);
  D.assign((size_t)n_el * q * (p + 1), 0.0);
  double out[2][MAXP + 1];
  for (int e = 0; e < n_el; ++e)
    for (int g = 0; g < q; ++g) {
      double x = ((double)e + gr.x[g]) / (double)n_el;
      bspline_span_ders(t, p, p + e, x, 1, out);
      for (int a = 0; a <= p; ++a) {
        B[((size_t)e * q + g) * (p + 1) + a] = out[0][a];
        D[((size_t)e * q + g) * (p + 1) + a] = out[1][a];
      }
    }
}

bool cholesky(std::vector<double> &A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
    if (!(s > 0)) return false;
    double d = std::sqrt(s);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double v = A[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
      A[(size_t)i * n + j] = v / d;
    }
    for (int i = 0; i < j; ++i) A[(size_t)i * n + j] = 0.0;
  }
  return true;
}

void chol_solve(const std::vector<double> &L, int n, double *b) {
  for (int i = 0; i < n; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[(size_t)i * n + k] * b[k];
    b[i] = v / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double v = b[i];
    for (int k = i + 1; k < n; ++k) v -= L[(size_t)k * n + i] * b[k];
    b[i] = v / L[(size_t)i * n + i];
  }
}

std::vector<double> spd_inverse(const std::vector<double> &A, int n) {
  std::vector<double> L = A;
  if (!cholesky(L, n)) fail(IGAMG_EINVAL, "matrix of a smoother piece or the coarse level is not SPD");
  // X = L^-T L^-1, computed column by column of L^-1
  std::vector<double> Li((size_t)n * n, 0.0);  // L^-1, lower
  for (int j = 0; j < n; ++j) {
    for (int i = j; i < n; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) v -= L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = v / L[(size_t)i * n + i];
    }
  }
  std::vector<double> X((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
      X[(size_t)i * n + j] = s;
      X[(size_t)j * n + i] = s;
    }
  return X;
}

void jacobi_eigen(std::vector<double> A, int n, std::vector<double> &w, std::vector<double> &V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = A[(size_t)i * n + j];
        tot += a * a;
        if (i != j) off += a * a;
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (apq == 0.0) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        double theta = (aqq - app) / (2.0 * apq);
        double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {  // A <- A J
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V J
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
}

std::vector<double> null_space(const std::vector<double> &C, int m, int n) {
  // Householder QR of C^T (n x m); the last n-m columns of Q span null(C).
  std::vector<double> At((size_t)n * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) At[(size_t)j * m + i] = C[(size_t)i * n + j];
  std::vector<std::vector<double>> vs;
  for (int k = 0; k < m; ++k) {
    std::vector<double> v(n, 0.0);
    double nrm = 0.0;
    for (int i = k; i < n; ++i) nrm += At[(size_t)i * m + k] * At[(size_t)i * m + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) fail(IGAMG_EINVAL, "rank-deficient SCMS constraints");
    double a0 = At[(size_t)k * m + k];
    double alpha = a0 >= 0 ? -nrm : nrm;
    for (int i = k; i < n; ++i) v[i] = At[(size_t)i * m + k];
    v[k] -= alpha;
    double vn = 0.0;
    for (int i = k; i < n; ++i) vn += v[i] * v[i];
    for (int j = k; j < m; ++j) {
      double s = 0.0;
      for (int i = k; i < n; ++i) s += v[i] * At[(size_t)i * m + j];
      s = 2.0 * s / vn;
      for (int i = k; i < n; ++i) At[(size_t)i * m + j] -= s * v[i];
    }
    vs.push_back(v);
  }
  int r = n - m;
  std::vector<double> Z((size_t)n * r, 0.0);
  for (int c = 0; c < r; ++c) {
    std::vector<double> e(n, 0.0);
    e[m + c] = 1.0;
    for (int k = m - 1; k >= 0; --k) {  // Q e = H_0 H_1 ... H_{m-1} e
      const std::vector<double> &v = vs[k];
      double vn = 0.0, s = 0.0;
      for (int i = k; i < n; ++i) {
        vn += v[i] * v[i];
        s += v[i] * e[i];
      }
      s = 2.0 * s / vn;
      for (int i = k; i < n; ++i) e[i] -= s * v[i];
    }
    for (int i = 0; i < n; ++i) Z[(size_t)i * r + c] = e[i];
  }
  return Z;
}

static void mass_stiffness(int n_el, int p, std::vector<double> &M, std::vector<double> &K) {
  GaussRule gr = gauss_rule(p + 1);
  std::vector<double> B, D;
  element_tables(n_el, p, gr, B, D);
  int n = n_el + p;
  M.assign((size_t)n * n, 0.0);
  K.assign((size_t)n * n, 0.0);
  double h = 1.0 / n_el;
  for (int e = 0; e < n_el; ++e)
    for (int g = 0; g < gr.q; ++g) {
      double w = gr.w[g] * h;
      const double *b = &B[((size_t)e * gr.q + g) * (p + 1)];
      const double *d = &D[((size_t)e * gr.q + g) * (p + 1)];
      for (int a = 0; a <= p; ++a)
        for (int c = 0; c <= p; ++c) {
          M[(size_t)(e + a) * n + e + c] += w * b[a] * b[c];
          K[(size_t)(e + a) * n + e + c] += w * d[a] * d[c];
        }
    }
}

static std::vector<double> matmul(const std::vector<double> &A, const std::vector<double> &B, int m,
                                  int k, int n, bool transA = false) {
  // C (m x n) = op(A) B; A is (m x k) or, if transA, (k x m)
  std::vector<double> C((size_t)m * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int l = 0; l < k; ++l) {
      double a = transA ? A[(size_t)l * m + i] : A[(size_t)i * k + l];
      if (a == 0.0) continue;
      for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)l * n + j];
    }
  return C;
}

// X (n x c) <- X L^-T for lower-triangular L (c x c)
static void right_solve_LT(std::vector<double> &X, int n, const std::vector<double> &L, int c) {
  for (int r = 0; r < n; ++r) {
    double *x = &X[(size_t)r * c];
    for (int j = 0; j < c; ++j) {
      double v = x[j];
      for (int k = 0; k < j; ++k) v -= x[k] * L[(size_t)j * c + k];
      x[j] = v / L[(size_t)j * c + j];
    }
  }
}

void scms_factors_1d(int n_el, int p, std::vector<double> &Q, std::vector<double> &lam) {
  int n = n_el + p, ni = n - 2;
  std::vector<double> M, K;
  mass_stiffness(n_el, p, M, K);
  std::vector<double> Mi((size_t)ni * ni), Ki((size_t)ni * ni);
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < ni; ++j) {
      Mi[(size_t)i * ni + j] = M[(size_t)(i + 1) * n + j + 1];
      Ki[(size_t)i * ni + j] = K[(size_t)(i + 1) * n + j + 1];
    }
  // constraint rows h^{2l} N_i^{(2l)}(0), h^{2l} N_i^{(2l)}(1), 1 <= l, 2l < p
  std::vector<double> t = open_knots(n_el, p);
  double h = 1.0 / n_el;
  std::vector<double> C;
  int mc = 0;
  for (int l = 1; 2 * l < p; ++l) {
    double out[MAXP + 1][MAXP + 1];
    double sc = std::pow(h, 2 * l);
    for (int side = 0; side < 2; ++side) {
      int m = side == 0 ? p : p + n_el - 1;
      bspline_span_ders(t, p, m, side == 0 ? 0.0 : 1.0, 2 * l, out);
      std::vector<double> row(ni, 0.0);
      for (int a = 0; a <= p; ++a) {
        int i = m - p + a;
        if (i >= 1 && i <= n - 2) row[i - 1] = sc * out[2 * l][a];
      }
      C.insert(C.end(), row.begin(), row.end());
      ++mc;
    }
  }
  if (mc >= ni) fail(IGAMG_EINVAL, "too few elements for the SCMS splitting at this degree");
  Q.assign((size_t)ni * ni, 0.0);
  lam.assign(ni, 0.0);
  int r = ni - mc;
  // M-orthonormal basis of S~ = null(C): Z (Z^T M Z)^{-1/2 Cholesky}
  std::vector<double> Z = mc ? null_space(C, mc, ni) : std::vector<double>();
  if (!mc) {
    Z.assign((size_t)ni * ni, 0.0);
    for (int i = 0; i < ni; ++i) Z[(size_t)i * ni + i] = 1.0;
  }
  std::vector<double> G = matmul(Z, matmul(Mi, Z, ni, ni, r), r, ni, r, true);
  if (!cholesky(G, r)) fail(IGAMG_EINVAL, "SCMS mass matrix not SPD");
  right_solve_LT(Z, ni, G, r);
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < r; ++j) Q[(size_t)i * ni + j] = Z[(size_t)i * r + j];
  if (!mc) return;
  // complement S1 = M^-1 C^T, generalized eigenvectors of (K, M) on it
  std::vector<double> L = Mi;
  if (!cholesky(L, ni)) fail(IGAMG_EINVAL, "SCMS mass matrix not SPD");
  std::vector<double> Z1((size_t)ni * mc);
  for (int c = 0; c < mc; ++c) {
    std::vector<double> b(ni);
    for (int i = 0; i < ni; ++i) b[i] = C[(size_t)c * ni + i];
    chol_solve(L, ni, b.data());
    for (int i = 0; i < ni; ++i) Z1[(size_t)i * mc + c] = b[i];
  }
  std::vector<double> G1 = matmul(Z1, matmul(Mi, Z1, ni, ni, mc), mc, ni, mc, true);
  std::vector<double> H1 = matmul(Z1, matmul(Ki, Z1, ni, ni, mc), mc, ni, mc, true);
  if (!cholesky(G1, mc)) fail(IGAMG_EINVAL, "SCMS complement not SPD");
  // C1 = L1^-1 H1 L1^-T
  std::vector<double> T = H1;
  right_solve_LT(T, mc, G1, mc);  // H1 L1^-T
  std::vector<double> Tt((size_t)mc * mc);
  for (int i = 0; i < mc; ++i)
    for (int j = 0; j < mc; ++j) Tt[(size_t)i * mc + j] = T[(size_t)j * mc + i];
  right_solve_LT(Tt, mc, G1, mc);  // (L1^-1 H1 L1^-T)^T = same (symmetric)
  std::vector<double> w, V;
  jacobi_eigen(Tt, mc, w, V);
  right_solve_LT(Z1, ni, G1, mc);  // Z1 L1^-T
  std::vector<double> Q1 = matmul(Z1, V, ni, mc, mc);
  for (int i = 0; i < ni; ++i)
    for (int j = 0; j < mc; ++j) Q[(size_t)i * ni + r + j] = Q1[(size_t)i * mc + j];
  for (int j = 0; j < mc; ++j) lam[r + j] = w[j];
}

std::vector<double> embedding_1d(int n_c, int p) {
  int nf = 2 * n_c + p, nc = n_c + p;
  GaussRule gr = gauss_rule(p + 1);
  std::vector<double> tf = open_knots(2 * n_c, p), tc = open_knots(n_c, p);
  std::vector<double> Mff((size_t)nf * nf, 0.0), Mfc((size_t)nf * nc, 0.0);
  double h = 1.0 / (2 * n_c);
  double bf[2][MAXP + 1], bc[2][MAXP + 1];
  for (int e = 0; e < 2 * n_c; ++e)
    for (int g = 0; g < gr.q; ++g) {
      double x = ((double)e + gr.x[g]) / (double)(2 * n_c);
      double w = gr.w[g] * h;
      bspline_span_ders(tf, p, p + e, x, 0, bf);
      bspline_span_ders(tc, p, p + e / 2, x, 0, bc);
      for (int a = 0; a <= p; ++a) {
        for (int c = 0; c <= p; ++c) Mff[(size_t)(e + a) * nf + e + c] += w * bf[0][a] * bf[0][c];
        for (int c = 0; c <= p; ++c) Mfc[(size_t)(e + a) * nc + e / 2 + c] += w * bf[0][a] * bc[0][c];
      }
    }
  if (!cholesky(Mff, nf)) fail(IGAMG_EINVAL, "fine mass matrix not SPD");
  std::vector<double> P((size_t)nf * nc);
  std::vector<double> col(nf);
  for (int j = 0; j < nc; ++j) {
    for (int i = 0; i < nf; ++i) col[i] = Mfc[(size_t)i * nc + j];
    chol_solve(Mff, nf, col.data());
    for (int i = 0; i < nf; ++i) P[(size_t)i * nc + j] = std::fabs(col[i]) < 1e-11 ? 0.0 : col[i];
  }
  return P;
}

}  // namespace igamg
