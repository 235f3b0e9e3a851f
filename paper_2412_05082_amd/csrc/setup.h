// Host-side set-up of the 1D ingredients of the C0IP operator and of the
// fast-diagonalisation local solvers (plain C++17, no HIP).
//
// On a uniform Cartesian mesh of [0,1]^d the C0IP matrix is a sum of
// Kronecker products of three global 1D matrices along each axis (Sec. 4,
// eqs. c0iptensorvp / c0iptensorvp3D):
//   M  (mass),  L  (stiffness),  B  (cellwise int phi'' phi'' plus, at every
//   grid point, the 1D penalty / consistency / adjoint-consistency terms).
// Vertex-patch matrices are restrictions of these to the patch's 2k-1
// interior nodes per axis; their separable approximation (eq.
// localsolverbila) is inverted by fast diagonalisation (eq. inverse) from
// the generalised eigenpairs B q = lambda M q, Q^T M Q = I.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace c0ip {

// k+1 Gauss-Lobatto-Legendre points on [0,1].
std::vector<double> gll_points(int k);
// q-point Gauss-Legendre rule on [0,1].
void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w);

// Banded n x n matrix, half-bandwidth hw, row-major band storage
// a[i * (2 hw + 1) + (j - i + hw)].
struct Band {
  int n = 0, hw = 0;
  std::vector<double> a;
  void init(int n_, int hw_) { n = n_; hw = hw_; a.assign((size_t)n * (2 * hw + 1), 0.0); }
  double get(int i, int j) const {
    int o = j - i;
    return (o < -hw || o > hw) ? 0.0 : a[(size_t)i * (2 * hw + 1) + (o + hw)];
  }
  double& at(int i, int j) { return a[(size_t)i * (2 * hw + 1) + (j - i + hw)]; }
};

// Global 1D matrices of one level (N cells, degree k, penalty gamma / h):
// n1 = kN+1 nodes including both boundary nodes, whose rows and columns are
// zero (u = 0 on the boundary is built into V_l).
struct Level1D {
  int k = 0, N = 0, n1 = 0;
  double h = 0, gamma = 0;
  Band M, L, B;  // half-bandwidth 2k for all three (M and L use only k)
};
Level1D build_level_1d(int k, int N, double gamma);

// Row classes for compact coefficient tables: rows within 2k of either end
// get their own class, the rest repeat with period k.
struct RowClasses {
  int nclass = 0;
  int left = 0;     // rows [0, left) are classes 0..left-1
  int right0 = 0;   // rows [right0, n1) are classes left + (n1-1-i)
  int periodic = 0; // other rows: class 2*left + (i mod k) (0 if per-row)
  std::vector<int> row_of_class;  // a representative row for each class
};
RowClasses row_classes(const Level1D& lv);
// Table [3 matrices][nclass][4k+1] (M, L, B; offset j-i in [-2k, 2k]).
std::vector<double> coefficient_table(const Level1D& lv, const RowClasses& rc);

// Patch variants along one axis: 0 interior, 1 touching x=0, 2 touching
// x=1, 3 touching both (N = 2).  Returns the variant of vertex v in [1,N-1].
inline int patch_variant(int v, int N) { return (v == 1 ? 1 : 0) | (v == N - 1 ? 2 : 0); }

// Generalised symmetric eigenproblem A q = lambda M q with M SPD:
// Q (n x n, column j = eigenvector j, row-major Q[i*n+j]) with Q^T M Q = I.
// Returns false if M is not positive definite.
bool generalized_eigen(int n, const std::vector<double>& A, const std::vector<double>& M,
                       std::vector<double>& Q, std::vector<double>& lam);

// Fast-diagonalisation data of the 4 patch variants of one level:
// Q[v][n*n] row-major (Q[c'*n + c] = component c' of eigenvector c),
// lam[v][n].  Variants that do not occur on this level are left empty.
struct PatchEigen {
  int n = 0;
  std::vector<double> Q[4], lam[4];
  bool present[4] = {false, false, false, false};
};
bool build_patch_eigen(const Level1D& lv, PatchEigen& pe, std::string& err);

// 1D embedding of Q_k on Nc cells into Q_k on 2Nc cells: table
// T[s][p][a] = value of coarse cell basis a at the fine node of position p
// in fine cell 2cc+s (s in {0,1}, p in [0,k), a in [0,k]).
std::vector<double> prolongation_table(int k);

// Dense coarse operator of level 0 (2 cells per axis) on its (2k-1)^dim
// interior nodes, and its inverse (via Cholesky).  Row-major.
bool coarse_inverse(const Level1D& lv0, int dim, std::vector<double>& Ainv, std::string& err);

// The exact local matrix A_v = R_v A R_v^T of the vertex patch at vertex
// v[0..dim-1] (each in [1, N-1]) on level lv -- the restriction of the
// Kronecker form (Sec. 4) to the patch's (2k-1)^dim interior nodes, mixed
// terms included -- and its inverse (via Cholesky).  Row-major, patch
// nodes x fastest.  The coarse inverse is the case N = 2, v = (1, ..., 1).
bool patch_exact_inverse(const Level1D& lv, int dim, const int* v, std::vector<double>& Ainv, std::string& err);

}  // namespace c0ip
