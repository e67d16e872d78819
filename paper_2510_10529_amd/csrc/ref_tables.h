// Compile-time 1-D element tables of the order-P spectral element on the unit cell.
//
// With the assembled GLL-lumped mass W1 (vertex: h w_0, interior: h w_i / 2) and
// s_i = W1_i^{-1/2}, the scaled element matrices are
//   m~_ik = s_i (h/2) M^_ik s_k      (independent of h),
//   k~_ik = s_i (2/h) K^_ik s_k = k~ref_ik / h^2,
// with M^, K^ the exact (Gauss) mass and stiffness of the Lagrange basis on the GLL
// nodes (Eq. 12). Each term of the kinetic operator carries exactly one k~ factor,
// so kernels apply the h = 1 tables and scale the result by 1/h^2. Evaluated by the
// compiler (C++17 constexpr), the entries become literals in the kernels.
#pragma once

namespace invdft {
namespace ref {

constexpr double cabs(double x) { return x < 0 ? -x : x; }

constexpr double csqrt(double x) {
  if (x <= 0) return 0.0;
  double y = x > 1 ? x : 1.0;
  for (int i = 0; i < 200; ++i) {
    const double yn = 0.5 * (y + x / y);
    if (yn == y) break;
    y = yn;
  }
  return y;
}

// cos on [0, pi] by a Taylor series around pi/2 shifted to [-pi/2, pi/2]
constexpr double ccos(double x) {
  const double pi = 3.14159265358979323846;
  double sign = 1.0;
  if (x > pi / 2) {  // cos(x) = -cos(pi - x)
    x = pi - x;
    sign = -1.0;
  }
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 30; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sign * sum;
}

constexpr void legendre_pair(int m, double x, double& pm, double& pm1) {
  double p0 = 1.0, p1 = x;
  if (m == 0) {
    pm = 1.0;
    pm1 = 0.0;
    return;
  }
  for (int k = 2; k <= m; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pm = p1;
  pm1 = p0;
}

template <int P>
struct Tables {
  double mt[P + 1][P + 1];
  double kt[P + 1][P + 1];
};

template <int P>
constexpr Tables<P> make_tables() {
  constexpr int N = P + 1;
  const double pi = 3.14159265358979323846;
  double xi[N] = {}, wi[N] = {}, xq[N] = {}, wq[N] = {};
  // GLL nodes: Newton on x P_p - P_{p-1} from Chebyshev-Gauss-Lobatto points
  for (int j = 0; j <= P; ++j) {
    double x = -ccos(pi * j / P);
    for (int it = 0; it < 100; ++it) {
      double pp = 0, pm1 = 0;
      legendre_pair(P, x, pp, pm1);
      const double dx = (x * pp - pm1) / ((P + 1) * pp);
      x -= dx;
      if (cabs(dx) < 1e-16) break;
    }
    xi[j] = x;
  }
  xi[0] = -1.0;
  xi[P] = 1.0;
  for (int j = 0; j <= P / 2; ++j) {
    const double s = 0.5 * (xi[P - j] - xi[j]);
    xi[j] = -s;
    xi[P - j] = s;
  }
  if (P % 2 == 0) xi[P / 2] = 0.0;
  for (int j = 0; j <= P; ++j) {
    double pp = 0, pm1 = 0;
    legendre_pair(P, xi[j], pp, pm1);
    wi[j] = 2.0 / (P * (P + 1.0) * pp * pp);
  }
  // Gauss-Legendre, N points
  for (int i = 0; i < N; ++i) {
    double z = ccos(pi * (i + 0.75) / (N + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pm = 0, pm1 = 0;
      legendre_pair(N, z, pm, pm1);
      const double dp = N * (z * pm - pm1) / (z * z - 1.0);
      const double dz = pm / dp;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    double pm = 0, pm1 = 0;
    legendre_pair(N, z, pm, pm1);
    const double dp = N * (z * pm - pm1) / (z * z - 1.0);
    xq[N - 1 - i] = z;
    wq[N - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // Lagrange basis values and derivatives at the Gauss points
  double L[N][N] = {}, D[N][N] = {};
  for (int q = 0; q < N; ++q)
    for (int i = 0; i < N; ++i) {
      double l = 1.0;
      for (int j = 0; j < N; ++j)
        if (j != i) l *= (xq[q] - xi[j]) / (xi[i] - xi[j]);
      L[q][i] = l;
      double d = 0.0;
      for (int m = 0; m < N; ++m) {
        if (m == i) continue;
        double t = 1.0 / (xi[i] - xi[m]);
        for (int j = 0; j < N; ++j)
          if (j != i && j != m) t *= (xq[q] - xi[j]) / (xi[i] - xi[j]);
        d += t;
      }
      D[q][i] = d;
    }
  double s[N] = {};
  for (int i = 0; i < N; ++i) s[i] = 1.0 / csqrt((i == 0 || i == P) ? wi[0] : 0.5 * wi[i]);
  Tables<P> t{};
  double mr[N][N] = {}, kr[N][N] = {};
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k) {
      double kk = 0.0, mm = 0.0;
      for (int q = 0; q < N; ++q) {
        kk += wq[q] * D[q][i] * D[q][k];
        mm += wq[q] * L[q][i] * L[q][k];
      }
      mr[i][k] = s[i] * 0.5 * mm * s[k];
      kr[i][k] = s[i] * 2.0 * kk * s[k];
    }
  // exact symmetry and centrosymmetry
  for (int i = 0; i < N; ++i)
    for (int k = 0; k < N; ++k) {
      t.mt[i][k] = 0.25 * (mr[i][k] + mr[k][i] + mr[P - i][P - k] + mr[P - k][P - i]);
      t.kt[i][k] = 0.25 * (kr[i][k] + kr[k][i] + kr[P - i][P - k] + kr[P - k][P - i]);
    }
  return t;
}

template <int P>
struct Table {
  static constexpr Tables<P> value = make_tables<P>();
};

}  // namespace ref
}  // namespace invdft
