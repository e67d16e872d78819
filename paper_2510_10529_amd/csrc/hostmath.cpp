// Host-side numerics: 1-D quadrature and Lagrange tables, small dense FP64
// linear algebra (Cholesky, triangular inverse, cyclic Jacobi eigensolver).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace invdft {

namespace {
// Legendre P_k(x) for k = m and m-1 by the three-term recurrence.
void legendre_pair(int m, double x, double* pm, double* pm1) {
  double p0 = 1.0, p1 = x;
  if (m == 0) {
    *pm = 1.0;
    *pm1 = 0.0;
    return;
  }
  for (int k = 2; k <= m; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pm = p1;
  *pm1 = p0;
}
}  // namespace

// Gauss-Lobatto-Legendre nodes: -1, roots of P_p', +1; weights 2/(p(p+1)P_p^2).
// Newton iteration on x P_p(x) - P_{p-1}(x) = 0 (whose roots are the GLL nodes),
// started from the Chebyshev-Gauss-Lobatto points (von Winckel's method).
void gll_rule(int p, double* x, double* w) {
  for (int j = 0; j <= p; ++j) {
    double xj = -std::cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double pp, pm1;
      legendre_pair(p, xj, &pp, &pm1);
      double dx = (xj * pp - pm1) / ((p + 1) * pp);
      xj -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    x[j] = xj;
  }
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 0; j <= p / 2; ++j) {  // enforce exact symmetry
    double s = 0.5 * (x[p - j] - x[j]);
    x[j] = -s;
    x[p - j] = s;
  }
  if (p % 2 == 0) x[p / 2] = 0.0;
  for (int j = 0; j <= p; ++j) {
    double pp, pm1;
    legendre_pair(p, x[j], &pp, &pm1);
    w[j] = 2.0 / (p * (p + 1.0) * pp * pp);
  }
}

// Gauss-Legendre rule with m points: Newton on P_m from cos(pi (i + 3/4)/(m + 1/2)).
void gauss_rule(int m, double* x, double* w) {
  for (int i = 0; i < m; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double pm, pm1;
      legendre_pair(m, z, &pm, &pm1);
      dp = m * (z * pm - pm1) / (z * z - 1.0);
      double dz = pm / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double pm, pm1;
    legendre_pair(m, z, &pm, &pm1);
    dp = m * (z * pm - pm1) / (z * z - 1.0);
    x[m - 1 - i] = z;  // ascending
    w[m - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Reference element matrices on [-1,1] for the order-p Lagrange basis on GLL nodes:
// K^_ij = int l_i' l_j', M^_ij = int l_i l_j by (p+1)-point Gauss (exact).
void reference_matrices(int p, double* Kh, double* Mh, double* xi, double* wi) {
  const int n = p + 1;
  gll_rule(p, xi, wi);
  std::vector<double> xq(n), wq(n);
  gauss_rule(n, xq.data(), wq.data());
  std::vector<double> L(n * n), D(n * n);  // [q][i]
  for (int q = 0; q < n; ++q) {
    for (int i = 0; i < n; ++i) {
      double l = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != i) l *= (xq[q] - xi[j]) / (xi[i] - xi[j]);
      L[q * n + i] = l;
      double d = 0.0;
      for (int m = 0; m < n; ++m) {
        if (m == i) continue;
        double t = 1.0 / (xi[i] - xi[m]);
        for (int j = 0; j < n; ++j)
          if (j != i && j != m) t *= (xq[q] - xi[j]) / (xi[i] - xi[j]);
        d += t;
      }
      D[q * n + i] = d;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double k = 0.0, mm = 0.0;
      for (int q = 0; q < n; ++q) {
        k += wq[q] * D[q * n + i] * D[q * n + j];
        mm += wq[q] * L[q * n + i] * L[q * n + j];
      }
      Kh[i * n + j] = k;
      Mh[i * n + j] = mm;
    }
  for (int i = 0; i < n; ++i)  // symmetrise the rounding
    for (int j = 0; j < i; ++j) {
      double a = 0.5 * (Kh[i * n + j] + Kh[j * n + i]);
      Kh[i * n + j] = Kh[j * n + i] = a;
      double b = 0.5 * (Mh[i * n + j] + Mh[j * n + i]);
      Mh[i * n + j] = Mh[j * n + i] = b;
    }
}

bool cholesky_lower(int n, double* A) {
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    d = std::sqrt(d);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = s / d;
    }
    for (int i = 0; i < j; ++i) A[i * n + j] = 0.0;
  }
  return true;
}

void invert_lower(int n, const double* L, double* Li) {
  std::fill(Li, Li + (size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Li[j * n + j] = 1.0 / L[j * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * n + k] * Li[k * n + j];
      Li[i * n + j] = -s / L[i * n + i];
    }
  }
}

// Cyclic Jacobi eigenvalue method for a symmetric matrix (Golub and Van Loan, Sec. 8.5):
// rotations annihilate each off-diagonal entry in turn until the off-diagonal
// Frobenius norm is negligible. A is destroyed. Eigenvalues ascending; column k
// of `evecs` (row-major n x n) is the eigenvector of evals[k].
void jacobi_eigh(int n, double* A, double* evals, double* evecs) {
  std::vector<double> V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  double fro = 0.0;
  for (size_t i = 0; i < (size_t)n * n; ++i) fro += A[i] * A[i];
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    if (std::sqrt(off) <= 1e-17 * fro || off == 0.0) break;
    for (int pi = 0; pi < n; ++pi)
      for (int qi = pi + 1; qi < n; ++qi) {
        double apq = A[(size_t)pi * n + qi];
        if (apq == 0.0) continue;
        double app = A[(size_t)pi * n + pi], aqq = A[(size_t)qi * n + qi];
        double theta = (aqq - app) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
          double akp = A[(size_t)k * n + pi], akq = A[(size_t)k * n + qi];
          A[(size_t)k * n + pi] = c * akp - sn * akq;
          A[(size_t)k * n + qi] = sn * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
          double apk = A[(size_t)pi * n + k], aqk = A[(size_t)qi * n + k];
          A[(size_t)pi * n + k] = c * apk - sn * aqk;
          A[(size_t)qi * n + k] = sn * apk + c * aqk;
        }
        A[(size_t)pi * n + qi] = A[(size_t)qi * n + pi] = 0.0;
        for (int k = 0; k < n; ++k) {
          double vkp = V[(size_t)k * n + pi], vkq = V[(size_t)k * n + qi];
          V[(size_t)k * n + pi] = c * vkp - sn * vkq;
          V[(size_t)k * n + qi] = sn * vkp + c * vkq;
        }
      }
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
  for (int k = 0; k < n; ++k) {
    evals[k] = A[(size_t)order[k] * n + order[k]];
    if (evecs)
      for (int i = 0; i < n; ++i) evecs[(size_t)i * n + k] = V[(size_t)i * n + order[k]];
  }
}

double max_eig_sym(int n, const double* A) {
  std::vector<double> a(A, A + (size_t)n * n), e(n);
  jacobi_eigh(n, a.data(), e.data(), nullptr);
  return e[n - 1];
}

}  // namespace invdft
