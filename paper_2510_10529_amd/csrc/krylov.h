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

int mr_state_count();
int mr_state_iters();
int mr_state_relres();
int mr_state_active();
int mr_state_invbeta();
int mr_state_c1();
int mr_state_c2();
fe_status mr_init(double* st, const double* dot_r_z, int k, hipStream_t s);
size_t mr_dots_work_bytes(int64_t nf, int k);
template <typename T>
fe_status mr_dots(const T* z, const T* y, const T* r1, int k, int64_t nf, double* d1, double* d2,
                  double* partial, hipStream_t s);
fe_status mr_alfa(double* st, const double* d1, const double* d2, int k, bool first, hipStream_t s);
fe_status mr_givens(double* st, const double* dot_r_z, int k, double tol, hipStream_t s);
template <typename T>
fe_status mr_resid_precond(T* y, T* r1, const T* r2, const double* st, const double* dinv, int k,
                           int64_t nf, hipStream_t s);
template <typename T>
fe_status mr_update(const T* zold, T* w1, const T* w2, T* x, const double* st, int k, int64_t nf,
                    hipStream_t s);
template <typename T>
fe_status k_precond(const T* x, const double* dinv, int k, int64_t nf, T* y, hipStream_t s);
fe_status k_add_f32(const float* d, double* q, int64_t total, hipStream_t s);
template <typename T>
fe_status k_select_cols(const T* src, int ko, T* dst, int kn, const int* map, int64_t nf, hipStream_t s);
template <typename T>
fe_status k_scatter_cols(const T* src, int kc, T* dst, int kf, const int* map, int64_t nf, hipStream_t s);
fe_status k_mask_cols(float* r, const double* rr, const double* bb, double tol, int k, int64_t nf, hipStream_t s);
fe_status k_sub_from(const double* b, double* r, int64_t total, hipStream_t s);

}  // namespace invdft
