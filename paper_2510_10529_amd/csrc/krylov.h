// Internal launchers of the loss/gradient and MINRES kernels (krylov.hip).
#pragma once

#include "internal.h"

namespace invdft {

fe_status k_nodes(const Mesh& m, double* xyz, double* w, hipStream_t s);
fe_status k_kdiag(const Mesh& m, double* d, hipStream_t s);
fe_status k_dinv(const Mesh& m, double* dinv, hipStream_t s);
fe_status k_density(const Mesh& m, const double* Psi, int nocc, const double* occ_h, double* rho, hipStream_t s);
size_t loss_work_bytes();
fe_status k_loss(const Mesh& m, const double* rho, const double* rho_d, double* out, void* work, hipStream_t s);
fe_status k_rhs(const Mesh& m, const double* Psi, int nocc, const double* occ_h, const double* rho,
                const double* rho_d, double* R, hipStream_t s);
fe_status k_grad(const Mesh& m, const double* Psi, const double* Q, int nocc, const double* rho_d, double tau,
                 double* g, hipStream_t s);

// per-column scalar state (struct of arrays, each of length k)
enum MrState {
  S_BETA = 0, S_OLDB, S_DBAR, S_EPSLN, S_PHIBAR, S_BETA1, S_CS, S_SN, S_ALFA, S_C1, S_C2,
  S_INVBETA, S_INVBETA_OLD, S_OLDEPS, S_DELTA, S_INVGAMMA, S_PHI, S_ACTIVE, S_ITERS, S_RELRES, S_D1, S_D2,
  S_COUNT
};

int mr_state_count();
int mr_state_iters();
int mr_state_active();
int mr_state_invbeta();
fe_status mr_init(double* st, const double* dot_r_z, int k, hipStream_t s);
fe_status mr_alfa(double* st, const double* d1, const double* d2, int k, bool first, hipStream_t s);
fe_status mr_givens(double* st, const double* dot_r_z, int k, double tol, hipStream_t s);
template <typename T>
fe_status k_precond(const T* x, const double* dinv, int k, int64_t nf, T* y, hipStream_t s);
fe_status k_add_f32(const float* d, double* q, int64_t total, hipStream_t s);
template <typename T>
fe_status k_select_cols(const T* src, int ko, T* dst, int kn, const int* map, int64_t nf, hipStream_t s);
template <typename T>
fe_status k_scatter_cols(const T* src, int kc, T* dst, int kf, const int* map, int64_t nf, hipStream_t s);
fe_status k_mask_cols(float* r, const double* rr, const double* bb, double tol, int k, int64_t nf, hipStream_t s);
fe_status k_sub_from(const double* b, double* r, int64_t total, hipStream_t s);

// deflated preconditioner of the adjoint (small per-column corrections; krylov.hip)
// V = [Psi U(:, 0..nb)] (U with row pitch ldu), N x (k0 + nb)
fe_status defl_pack(const double* Psi, int k0, const double* U, int ldu, int nb, double* V, int64_t nf,
                    hipStream_t s);
fe_status defl_d2(double* d2, const double* cR1, const double* cR2, const double* theta, const double* eps, int k,
                  int nb, hipStream_t s);
// The U rows of G1 / G2 (from the fused passes, k0 = their Psi width) hold the first nbf
// deflation vectors; Gr ((nb - nbf) x k) holds the rest, or is unused when nbf == nb.
fe_status defl_cnew(const double* G1, int k0, int nbf, const double* Gr, int nb, const double* cR1, const double* cR2,
                    const double* st, int k, double* cnew, hipStream_t s);
fe_status defl_beta_g2(double* d, double* G2, int k0, int nbf, double* Gr, int nb, const double* cnew,
                       const double* theta, const double* eps, int k, hipStream_t s);
fe_status defl_scale(const double* c, const double* theta, const double* eps, int k, int nb, double* out,
                     hipStream_t s);

}  // namespace invdft
