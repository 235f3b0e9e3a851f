// Host-side set-up: quadrature, 1D C0IP factors, row-class coefficient
// tables, patch eigenpairs, transfer table, coarse inverse.
#include "setup.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace c0ip {

namespace {

// Legendre P_n and its first two derivatives at x by the three-term recurrence.
void legendre(int n, double x, double& p, double& dp, double& d2p) {
  double p0 = 1, p1 = x, d0 = 0, d1 = 1, e0 = 0, e1 = 0;
  if (n == 0) { p = 1; dp = 0; d2p = 0; return; }
  for (int m = 1; m < n; ++m) {
    double p2 = ((2 * m + 1) * x * p1 - m * p0) / (m + 1);
    double d2 = d0 + (2 * m + 1) * p1;   // P'_{m+1} = P'_{m-1} + (2m+1) P_m
    double e2 = e0 + (2 * m + 1) * d1;   // same recurrence differentiated once more
    p0 = p1; p1 = p2; d0 = d1; d1 = d2; e0 = e1; e1 = e2;
  }
  p = p1; dp = d1; d2p = e1;
}

// Barycentric weights of nodes z.
std::vector<double> bary_weights(const std::vector<double>& z) {
  int n = (int)z.size();
  std::vector<double> w(n, 1.0);
  for (int j = 0; j < n; ++j)
    for (int m = 0; m < n; ++m)
      if (m != j) w[j] /= (z[j] - z[m]);
  return w;
}

// Differentiation matrix D[i*n+j] = l_j'(z_i) (exact for the degree-k basis).
std::vector<double> diff_matrix(const std::vector<double>& z) {
  int n = (int)z.size();
  std::vector<double> w = bary_weights(z), D((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        D[i * n + j] = (w[j] / w[i]) / (z[i] - z[j]);
        s += D[i * n + j];
      }
    D[i * n + i] = -s;
  }
  return D;
}

// Values of the Lagrange basis of nodes z at point t (barycentric form).
std::vector<double> lagrange_values(const std::vector<double>& z, double t) {
  int n = (int)z.size();
  std::vector<double> v(n, 0.0);
  for (int j = 0; j < n; ++j)
    if (t == z[j]) { v[j] = 1.0; return v; }
  std::vector<double> w = bary_weights(z);
  double den = 0;
  for (int j = 0; j < n; ++j) { v[j] = w[j] / (t - z[j]); den += v[j]; }
  for (int j = 0; j < n; ++j) v[j] /= den;
  return v;
}

std::vector<double> matmul(int n, const std::vector<double>& A, const std::vector<double>& B) {
  std::vector<double> C((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < n; ++l)
      for (int j = 0; j < n; ++j) C[i * n + j] += A[i * n + l] * B[l * n + j];
  return C;
}

// In-place lower Cholesky of a row-major SPD matrix; false if not SPD.
bool cholesky(int n, std::vector<double>& A) {
  for (int j = 0; j < n; ++j) {
    double d = A[(size_t)j * n + j];
    for (int l = 0; l < j; ++l) d -= A[(size_t)j * n + l] * A[(size_t)j * n + l];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    A[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[(size_t)i * n + j];
      for (int l = 0; l < j; ++l) s -= A[(size_t)i * n + l] * A[(size_t)j * n + l];
      A[(size_t)i * n + j] = s / d;
    }
    for (int i = 0; i < j; ++i) A[(size_t)i * n + j] = 0.0;
  }
  return true;
}

// Cyclic Jacobi eigen-decomposition of a symmetric matrix S (row-major):
// S = U diag(lam) U^T.
void jacobi_eigen(int n, std::vector<double> S, std::vector<double>& U, std::vector<double>& lam) {
  U.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) U[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += S[i * n + j] * S[i * n + j];
        if (i != j) off += S[i * n + j] * S[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = S[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = S[p * n + p], aqq = S[q * n + q];
        double theta = (aqq - app) / (2 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int r = 0; r < n; ++r) {  // S <- J^T S J
          double srp = S[r * n + p], srq = S[r * n + q];
          S[r * n + p] = c * srp - s * srq;
          S[r * n + q] = s * srp + c * srq;
        }
        for (int r = 0; r < n; ++r) {
          double spr = S[p * n + r], sqr = S[q * n + r];
          S[p * n + r] = c * spr - s * sqr;
          S[q * n + r] = s * spr + c * sqr;
        }
        for (int r = 0; r < n; ++r) {
          double urp = U[r * n + p], urq = U[r * n + q];
          U[r * n + p] = c * urp - s * urq;
          U[r * n + q] = s * urp + c * urq;
        }
      }
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = S[i * n + i];
}

}  // namespace

std::vector<double> gll_points(int k) {
  std::vector<double> x(k + 1);
  x[0] = -1.0;
  x[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    double t = -std::cos(M_PI * i / k);  // Chebyshev-Lobatto start
    for (int it = 0; it < 100; ++it) {
      double p, dp, d2p;
      legendre(k, t, p, dp, d2p);
      double dt = dp / d2p;  // Newton on P_k'
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  std::vector<double> z(k + 1);
  for (int i = 0; i <= k; ++i) z[i] = 0.5 * (0.5 * (x[i] - x[k - i]) + 1.0);  // symmetric
  return z;
}

void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w) {
  x.resize(q);
  w.resize(q);
  for (int i = 0; i < q; ++i) {
    double t = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
    double p = 0, dp = 1, d2p;
    for (int it = 0; it < 100; ++it) {
      legendre(q, t, p, dp, d2p);
      double dt = p / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    legendre(q, t, p, dp, d2p);
    x[i] = 0.5 * (t + 1.0);
    w[i] = 1.0 / ((1 - t * t) * dp * dp);  // 2/((1-t^2)P'^2) mapped to [0,1]
  }
}

Level1D build_level_1d(int k, int N, double gamma) {
  Level1D lv;
  lv.k = k;
  lv.N = N;
  lv.n1 = k * N + 1;
  lv.h = 1.0 / N;
  lv.gamma = gamma;
  const int n = k + 1, hw = 2 * k;
  const double h = lv.h, pen = gamma / h;
  std::vector<double> z = gll_points(k), tq, wq;
  gauss_rule(k + 1, tq, wq);
  std::vector<double> D1 = diff_matrix(z), D2 = matmul(n, D1, D1);
  // basis values / first / second derivatives at the quadrature points
  std::vector<double> V((size_t)(k + 1) * n), V1(V.size()), V2(V.size());
  for (int q = 0; q <= k; ++q) {
    std::vector<double> l = lagrange_values(z, tq[q]);
    for (int j = 0; j < n; ++j) {
      double d1 = 0, d2 = 0;
      for (int i = 0; i < n; ++i) { d1 += l[i] * D1[i * n + j]; d2 += l[i] * D2[i * n + j]; }
      V[q * n + j] = l[j];
      V1[q * n + j] = d1;
      V2[q * n + j] = d2;
    }
  }
  // element matrices on a cell of size h
  std::vector<double> Me(n * n, 0), Le(n * n, 0), Be(n * n, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int q = 0; q <= k; ++q) {
        Me[i * n + j] += wq[q] * h * V[q * n + i] * V[q * n + j];
        Le[i * n + j] += wq[q] / h * V1[q * n + i] * V1[q * n + j];
        Be[i * n + j] += wq[q] / (h * h * h) * V2[q * n + i] * V2[q * n + j];
      }
  lv.M.init(lv.n1, hw);
  lv.L.init(lv.n1, hw);
  lv.B.init(lv.n1, hw);
  for (int c = 0; c < N; ++c)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        lv.M.at(c * k + i, c * k + j) += Me[i * n + j];
        lv.L.at(c * k + i, c * k + j) += Le[i * n + j];
        lv.B.at(c * k + i, c * k + j) += Be[i * n + j];
      }
  // point terms at every grid point x_f = f h: normal-derivative jump and
  // mean second derivative of the two cells' traces (one-sided, full
  // weight at the two boundary points)
  for (int f = 0; f <= N; ++f) {
    std::vector<int> idx;
    std::vector<double> jump, mean;
    if (f > 0) {  // cell f-1, its right end (reference t = 1), outward normal +x
      for (int j = 0; j < n; ++j) {
        idx.push_back((f - 1) * k + j);
        jump.push_back(D1[k * n + j] / h);
        mean.push_back((f < N ? 0.5 : 1.0) * D2[k * n + j] / (h * h));
      }
    }
    if (f < N) {  // cell f, its left end (t = 0), outward normal -x
      for (int j = 0; j < n; ++j) {
        idx.push_back(f * k + j);
        jump.push_back(-D1[0 * n + j] / h);
        mean.push_back((f > 0 ? 0.5 : 1.0) * D2[0 * n + j] / (h * h));
      }
    }
    for (size_t a = 0; a < idx.size(); ++a)
      for (size_t b = 0; b < idx.size(); ++b)
        lv.B.at(idx[a], idx[b]) += pen * jump[a] * jump[b] - mean[b] * jump[a] - jump[b] * mean[a];
  }
  // boundary nodes carry no DoF
  for (Band* m : {&lv.M, &lv.L, &lv.B})
    for (int i = 0; i < lv.n1; ++i)
      for (int o = -hw; o <= hw; ++o) {
        int j = i + o;
        if (j < 0 || j >= lv.n1) continue;
        if (i == 0 || i == lv.n1 - 1 || j == 0 || j == lv.n1 - 1) m->at(i, j) = 0.0;
      }
  return lv;
}

RowClasses row_classes(const Level1D& lv) {
  RowClasses rc;
  const int k = lv.k, n1 = lv.n1;
  const int left = 2 * k + 1;
  if (n1 <= 2 * left + k) {  // small level: one class per row
    rc.nclass = n1;
    rc.left = n1;
    rc.right0 = n1;
    rc.periodic = 0;
    for (int i = 0; i < n1; ++i) rc.row_of_class.push_back(i);
    return rc;
  }
  rc.left = left;
  rc.right0 = n1 - left;
  rc.periodic = 1;
  rc.nclass = 2 * left + k;
  rc.row_of_class.resize(rc.nclass);
  for (int i = 0; i < left; ++i) rc.row_of_class[i] = i;
  for (int i = 0; i < left; ++i) rc.row_of_class[left + i] = n1 - 1 - i;
  for (int p = 0; p < k; ++p) {
    int r = left + ((p - left % k) % k + k) % k;  // first periodic row with r mod k == p
    rc.row_of_class[2 * left + p] = r;
  }
  return rc;
}

std::vector<double> coefficient_table(const Level1D& lv, const RowClasses& rc) {
  const int k = lv.k, w = 4 * k + 1;
  std::vector<double> t((size_t)3 * rc.nclass * w, 0.0);
  const Band* mats[3] = {&lv.M, &lv.L, &lv.B};
  for (int m = 0; m < 3; ++m)
    for (int c = 0; c < rc.nclass; ++c) {
      int i = rc.row_of_class[c];
      for (int o = -2 * k; o <= 2 * k; ++o) {
        int j = i + o;
        t[((size_t)m * rc.nclass + c) * w + (o + 2 * k)] = (j >= 0 && j < lv.n1) ? mats[m]->get(i, j) : 0.0;
      }
    }
  return t;
}

bool generalized_eigen(int n, const std::vector<double>& A, const std::vector<double>& M,
                       std::vector<double>& Q, std::vector<double>& lam) {
  std::vector<double> C = M;
  if (!cholesky(n, C)) return false;
  // S = C^{-1} A C^{-T}: solve C X = A, then C S^T = X^T
  std::vector<double> X = A;
  for (int col = 0; col < n; ++col)
    for (int i = 0; i < n; ++i) {
      double s = X[i * n + col];
      for (int l = 0; l < i; ++l) s -= C[i * n + l] * X[l * n + col];
      X[i * n + col] = s / C[i * n + i];
    }
  std::vector<double> S((size_t)n * n);
  for (int row = 0; row < n; ++row)  // S[row][:] solves C y = X[row][:]^T
    for (int i = 0; i < n; ++i) {
      double s = X[row * n + i];
      for (int l = 0; l < i; ++l) s -= C[i * n + l] * S[row * n + l];
      S[row * n + i] = s / C[i * n + i];
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double a = 0.5 * (S[i * n + j] + S[j * n + i]);
      S[i * n + j] = S[j * n + i] = a;
    }
  std::vector<double> U;
  jacobi_eigen(n, S, U, lam);
  // Q = C^{-T} U (back substitution with C^T)
  Q.assign((size_t)n * n, 0.0);
  for (int col = 0; col < n; ++col)
    for (int i = n - 1; i >= 0; --i) {
      double s = U[i * n + col];
      for (int l = i + 1; l < n; ++l) s -= C[l * n + i] * Q[l * n + col];
      Q[i * n + col] = s / C[i * n + i];
    }
  return true;
}

bool build_patch_eigen(const Level1D& lv, PatchEigen& pe, std::string& err) {
  const int k = lv.k, N = lv.N, n = 2 * k - 1;
  pe.n = n;
  int rep[4] = {-1, -1, -1, -1};
  for (int v = 1; v <= N - 1; ++v) {
    int t = patch_variant(v, N);
    if (rep[t] < 0) rep[t] = v;
  }
  for (int t = 0; t < 4; ++t) {
    if (rep[t] < 0) continue;
    int v = rep[t], i0 = (v - 1) * k + 1;
    std::vector<double> Bp((size_t)n * n), Mp((size_t)n * n);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        Bp[a * n + b] = lv.B.get(i0 + a, i0 + b);
        Mp[a * n + b] = lv.M.get(i0 + a, i0 + b);
      }
    if (!generalized_eigen(n, Bp, Mp, pe.Q[t], pe.lam[t])) {
      err = "patch mass matrix not positive definite";
      return false;
    }
    for (double l : pe.lam[t])
      if (!(l > 0)) { err = "patch bi-Laplace factor not positive definite"; return false; }
    pe.present[t] = true;
  }
  return true;
}

std::vector<double> prolongation_table(int k) {
  std::vector<double> z = gll_points(k), T((size_t)2 * k * (k + 1));
  for (int s = 0; s < 2; ++s)
    for (int p = 0; p < k; ++p) {
      std::vector<double> l = lagrange_values(z, 0.5 * (s + z[p]));
      for (int a = 0; a <= k; ++a) T[((size_t)s * k + p) * (k + 1) + a] = l[a];
    }
  return T;
}

bool patch_exact_inverse(const Level1D& lv, int dim, const int* v, std::vector<double>& Ainv, std::string& err) {
  const int k = lv.k, n = 2 * k - 1;
  int n0 = 1, i0[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) {
    n0 *= n;
    i0[d] = (v[d] - 1) * k + 1;  // first interior node of the patch along axis d
  }
  auto M = [&](int d, int i, int j) { return lv.M.get(i0[d] + i, i0[d] + j); };
  auto L = [&](int d, int i, int j) { return lv.L.get(i0[d] + i, i0[d] + j); };
  auto B = [&](int d, int i, int j) { return lv.B.get(i0[d] + i, i0[d] + j); };
  std::vector<double> A((size_t)n0 * n0);
  for (int r = 0; r < n0; ++r)
    for (int c = 0; c < n0; ++c) {
      int ri[3] = {r % n, (r / n) % n, r / (n * n)}, ci[3] = {c % n, (c / n) % n, c / (n * n)};
      double val;
      if (dim == 2) {
        val = B(0, ri[0], ci[0]) * M(1, ri[1], ci[1]) + 2 * L(0, ri[0], ci[0]) * L(1, ri[1], ci[1]) +
              M(0, ri[0], ci[0]) * B(1, ri[1], ci[1]);
      } else {
        double m0 = M(0, ri[0], ci[0]), m1 = M(1, ri[1], ci[1]), m2 = M(2, ri[2], ci[2]);
        double l0 = L(0, ri[0], ci[0]), l1 = L(1, ri[1], ci[1]), l2 = L(2, ri[2], ci[2]);
        double b0 = B(0, ri[0], ci[0]), b1 = B(1, ri[1], ci[1]), b2 = B(2, ri[2], ci[2]);
        val = b0 * m1 * m2 + m0 * b1 * m2 + m0 * m1 * b2 + 2 * (l0 * l1 * m2 + m0 * l1 * l2 + l0 * m1 * l2);
      }
      A[(size_t)r * n0 + c] = val;
    }
  std::vector<double> C = A;
  if (!cholesky(n0, C)) { err = "local operator not positive definite"; return false; }
  // inverse from the Cholesky factor: solve C C^T X = I column by column
  Ainv.assign((size_t)n0 * n0, 0.0);
  std::vector<double> y(n0);
  for (int col = 0; col < n0; ++col) {
    for (int i = 0; i < n0; ++i) {
      double s = (i == col) ? 1.0 : 0.0;
      for (int l = 0; l < i; ++l) s -= C[(size_t)i * n0 + l] * y[l];
      y[i] = s / C[(size_t)i * n0 + i];
    }
    for (int i = n0 - 1; i >= 0; --i) {
      double s = y[i];
      for (int l = i + 1; l < n0; ++l) s -= C[(size_t)l * n0 + i] * Ainv[(size_t)l * n0 + col];
      Ainv[(size_t)i * n0 + col] = s / C[(size_t)i * n0 + i];
    }
  }
  return true;
}

bool coarse_inverse(const Level1D& lv0, int dim, std::vector<double>& Ainv, std::string& err) {
  const int v[3] = {1, 1, 1};
  if (!patch_exact_inverse(lv0, dim, v, Ainv, err)) {
    err = "coarse operator not positive definite";
    return false;
  }
  return true;
}

}  // namespace c0ip
