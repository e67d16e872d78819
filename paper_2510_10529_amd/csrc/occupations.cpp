// Finite temperature: Fermi-Dirac occupations and the component of the adjoint
// functions along the occupied orbitals (Sec. 2, Eqs. 4, 5, 8, 9).
//
// With occupations f_i = s phi(x_i), phi(x) = 1 / (1 + e^x), x_i = (eps_i - mu)/kT,
// and mu fixed by sum_i f_i = N_e, the derivative of L = sum_a W_a (rho_d - rho)^2
// with respect to the nodal potential splits into
//   * the part that couples each included orbital i to the orbitals outside the
//     included set S: g_b += psi_{b,i} q_{b,i}, q_i the MINRES solution on the
//     complement of S (adjoint_solve with the fractional f_i in the right-hand side);
//   * the part inside S, which needs no linear solve:
//       g_b += sum_{i,j in S} psi_{b,i} C_ij psi_{b,j},
//       C_ij = F_ij M_ij (i != j),  C_ii = f'_i (M_ii - etabar),
//     with M = Psi^T diag(2 (rho - rho_d)) Psi, F_ij = (f_i - f_j)/(eps_i - eps_j)
//     (the divided difference, F_ii = f'_i = d f_i / d eps_i) and
//     etabar = sum_i f'_i M_ii / sum_i f'_i. The diagonal blocks of C, over each
//     degenerate group, are the overlap condition of Eq. 8 (the paper's
//     multiplier of Eq. 9 is eta = -etabar); the blocks between groups are the
//     components along the other included orbitals that a solve projecting only
//     its own group would return, split symmetrically between the pair.
// adjoint_along_psi adds Psi C to the MINRES solution, so that
// grad_b = sum_i psi_{b,i} p_{b,i} (Eq. 10) with p = q + Psi C.
//
// The divided difference is evaluated without cancellation from
//   phi(x) - phi(y) = -phi(x) phi(-y) expm1(x - y),
// taken with x <= y so that expm1 stays in (-1, 0]: no overflow at any temperature,
// and F_ij tends to f'_i continuously as eps_j -> eps_i (degenerate groups need no
// special case).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace invdft {

namespace {

double logistic(double x) {  // 1 / (1 + e^x) without overflow
  if (x >= 0.0) {
    const double e = std::exp(-x);
    return e / (1.0 + e);
  }
  return 1.0 / (1.0 + std::exp(x));
}

double expm1_over(double d) {  // expm1(d) / d, continuous at 0
  if (std::fabs(d) < 1e-5) return 1.0 + d * (0.5 + d / 6.0);
  return std::expm1(d) / d;
}

// (f(e1) - f(e2)) / (e1 - e2) for f = s phi((e - mu)/kT); f'(e1) when e1 == e2.
double divided_difference(double e1, double e2, double mu, double kT, double smax) {
  double x = (e1 - mu) / kT, y = (e2 - mu) / kT;
  if (x > y) std::swap(x, y);
  return -(smax / kT) * logistic(x) * logistic(-y) * expm1_over(x - y);
}

double occupation_sum(const double* eig, int n, double mu, double kT, double smax) {
  double t = 0.0;
  for (int i = 0; i < n; ++i) t += smax * logistic((eig[i] - mu) / kT);
  return t;
}

constexpr double kTieHa = 1e-6;  // Ritz values closer than this are one degenerate group

}  // namespace

size_t along_psi_work_bytes(int64_t N, int n) {
  return ((gram_work_bytes(N, n, n) + 255) / 256) * 256 + 2 * (size_t)n * n * sizeof(double);
}

}  // namespace invdft

using namespace invdft;

extern "C" fe_status fermi_occupations(const double* eig_h, int n, double n_elec, double kT, double smax,
                                       double occ_cut, double* occ_h, double* dfde_h, double* mu_h, int* n_incl_h) {
  if (!eig_h || !occ_h) return fail(FE_EINVAL, "fermi_occupations: eig_h and occ_h are required");
  if (n < 1) return fail(FE_EINVAL, "fermi_occupations: n must be >= 1");
  if (!(kT > 0.0) || !(smax > 0.0)) return fail(FE_EINVAL, "fermi_occupations: kT > 0 and smax > 0 required");
  if (!(occ_cut >= 0.0 && occ_cut < 1.0)) return fail(FE_EINVAL, "fermi_occupations: occ_cut must be in [0, 1)");
  if (!(n_elec > 0.0 && n_elec < smax * n))
    return fail(FE_EINVAL, "fermi_occupations: need 0 < n_elec < smax * n");
  for (int i = 1; i < n; ++i)
    if (!(eig_h[i] >= eig_h[i - 1])) return fail(FE_EINVAL, "fermi_occupations: eigenvalues must ascend");
  // sum_i f_i(mu) increases with mu from ~0 to ~s n over this bracket
  double lo = eig_h[0] - 60.0 * kT, hi = eig_h[n - 1] + 60.0 * kT;
  for (int it = 0; it < 4096; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (occupation_sum(eig_h, n, mid, kT, smax) < n_elec)
      lo = mid;
    else
      hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  for (int i = 0; i < n; ++i) {
    const double x = (eig_h[i] - mu) / kT;
    occ_h[i] = smax * logistic(x);
    if (dfde_h) dfde_h[i] = -(smax / kT) * logistic(x) * logistic(-x);
  }
  if (mu_h) *mu_h = mu;
  int keep = 0;  // occupations decrease along the ascending eigenvalues
  while (keep < n && occ_h[keep] > occ_cut * smax) ++keep;
  while (keep > 0 && keep < n && eig_h[keep] - eig_h[keep - 1] < kTieHa) ++keep;
  if (n_incl_h) *n_incl_h = keep;
  if (occ_h[n - 1] > occ_cut * smax)
    return fail(FE_ESTATES, "fermi_occupations: the highest state passed is occupied above occ_cut");
  return FE_OK;
}

extern "C" fe_status adjoint_along_psi(fe_mesh mesh, const double* Psi, int n, const double* eps_h, double mu,
                                       double kT, double smax, const double* rho, const double* rho_data, double* Q,
                                       double* eta_h, double* C_h, void* work, void* stream) {
  int64_t nf = 0;
  if (!mesh) return fail(FE_EINVAL, "mesh handle is NULL");
  if (fe_mesh_info(mesh, &nf, nullptr, nullptr, nullptr) != FE_OK) return FE_EINVAL;
  if (!Psi || !eps_h || !rho || !rho_data || !Q || !work)
    return fail(FE_EINVAL, "adjoint_along_psi: NULL argument");
  if (n < 1 || n > kMaxShiftCols) return fail(FE_EINVAL, "adjoint_along_psi: n must be in [1, 256]");
  if (!(kT > 0.0) || !(smax > 0.0)) return fail(FE_EINVAL, "adjoint_along_psi: kT > 0 and smax > 0 required");
  if (((reinterpret_cast<uintptr_t>(Psi) | reinterpret_cast<uintptr_t>(Q) | reinterpret_cast<uintptr_t>(work)) &
       15u) != 0)
    return fail(FE_EINVAL, "adjoint_along_psi: Psi, Q and work must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(work);
  void* gw = w;
  double* Gd = reinterpret_cast<double*>(w + ((gram_work_bytes(nf, n, n) + 255) / 256) * 256);
  double* Cd = Gd + (size_t)n * n;
  // G = Psi^T diag(rho - rho_d) Psi, M = 2 G
  fe_status st = gram_weighted(Psi, n, rho, rho_data, nf, n, Gd, gw, s);
  if (st != FE_OK) return st;
  std::vector<double> M((size_t)n * n), C((size_t)n * n);
  INVDFT_HIP(hipMemcpyAsync(M.data(), Gd, M.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  std::vector<double> dfde(n);
  double num = 0.0, den = 0.0;
  for (int i = 0; i < n; ++i) {
    const double x = (eps_h[i] - mu) / kT;
    dfde[i] = -(smax / kT) * logistic(x) * logistic(-x);
    for (int j = 0; j < n; ++j) M[(size_t)i * n + j] *= 2.0;
    num += dfde[i] * M[(size_t)i * n + i];
    den += dfde[i];
  }
  const double etabar = den != 0.0 ? num / den : 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double Mij = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);  // symmetric to the last bit
      C[(size_t)i * n + j] = i == j ? dfde[i] * (Mij - etabar)
                                    : divided_difference(eps_h[i], eps_h[j], mu, kT, smax) * Mij;
    }
  INVDFT_HIP(hipMemcpyAsync(Cd, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s));
  st = rotate_add(Psi, n, nf, n, Cd, n, Q, n, s);
  INVDFT_HIP(hipStreamSynchronize(s));  // the host copy of C must outlive the transfer
  if (st != FE_OK) return st;
  if (eta_h) *eta_h = -etabar;
  if (C_h)
    for (size_t e = 0; e < C.size(); ++e) C_h[e] = C[e];
  return FE_OK;
}
