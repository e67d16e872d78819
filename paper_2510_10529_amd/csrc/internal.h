// Internal declarations of the gfx950 inverse-DFT library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "invdft.h"

namespace invdft {

constexpr int kMaxP = 8;
constexpr int kMaxP1 = kMaxP + 1;
constexpr int kMaxShiftCols = 256;

// Mesh handle: immutable after creation.
struct Mesh {
  int p = 0, n = 0, n1 = 0;   // order, cells per axis, free nodes per axis (p n - 1)
  double L = 0, h = 0;
  int64_t nf = 0;             // free nodes
  double kin_bound = 0;       // Fried element bound on lambda_max(K~/2)
  // 1-D element matrices scaled by the assembled W1^{-1/2} at the element's
  // local nodes (identical for every element of the uniform mesh), row-major
  // (p+1) x (p+1): mt = s (h/2) M^ s, kt = s (2/h) K^ s.
  double mt[kMaxP1 * kMaxP1] = {};
  double kt[kMaxP1 * kMaxP1] = {};
  std::vector<double> x1, w1, kd1, md1;  // per free 1-D node: coordinate, W1, diag(K~1), diag(M~1)
  int device = 0;
  double* d_x1 = nullptr;     // device copies of the 1-D tables (n1 each)
  double* d_w1 = nullptr;
  double* d_kd1 = nullptr;
  double* d_md1 = nullptr;
  // graded meshes (cells of different widths; h above is then the smallest): per 1-D
  // cell, the stiffness factor (h/h_e)^2 and the end-node factors of the W1^{-1/2}
  // scaling relative to the uniform tables (device copies, n each)
  bool graded = false;
  std::vector<double> cell_h;
  double* d_ckap = nullptr;
  double* d_cgl = nullptr;
  double* d_cgr = nullptr;
  // mapped meshes (cells curved by a smooth map of the box; every cell its own dense
  // matrix): per free node W, diag(K~/2) and coordinates, and the per-cell scaled matrices
  // in MFMA fragment order (map_mt 16-row tiles x map_ks 4-column steps x 64 per cell)
  bool mapped = false;
  double amp = 0.0;
  int map_mt = 0, map_ks = 0;
  double* d_wn = nullptr;
  double* d_kdn = nullptr;
  double* d_xyz = nullptr;
  double* d_Ke64 = nullptr;
  float* d_Ke32 = nullptr;
};

// the tables behind a mesh handle (NULL for a NULL handle)
const Mesh* mesh_tables(fe_mesh mesh);

// thread-local error text
void set_error(const std::string& msg);
fe_status fail(fe_status st, const std::string& msg);
fe_status hip_fail(hipError_t e, const char* what);

#define INVDFT_HIP(call)                                      \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return ::invdft::hip_fail(e_, #call); \
  } while (0)

// ---------------------------------------------------------------- host math
void gll_rule(int p, double* x, double* w);                  // p+1 GLL nodes/weights
void gauss_rule(int m, double* x, double* w);                // m Gauss-Legendre nodes/weights
void reference_matrices(int p, double* Kh, double* Mh, double* xi, double* wi);
bool cholesky_lower(int n, double* A);                       // A = L L^T in place (lower), row-major
void invert_lower(int n, const double* L, double* Linv);     // row-major
void jacobi_eigh(int n, double* A, double* evals, double* evecs);  // ascending; evecs columns, row-major
double max_eig_sym(int n, const double* A);

// ---------------------------------------------------------------- kernels
// Apply parameters; Y = alpha (K~/2 X + (v - cshift - colshift_j) X) + beta Z.
struct ApplyArgs {
  const void* X;
  void* Y;
  const void* Z;
  const double* v;
  int nv, ld;
  double alpha, beta, cshift;
  const double* colshift;     // host array (nv) or nullptr; copied into kernel arguments
  const double* d_colscale;   // device array (nv) or nullptr: output column j scaled by it
};
fe_status launch_apply(const Mesh& m, const ApplyArgs& a, fe_prec prec, hipStream_t s);
// mapped meshes: per-cell matrices and node tables (m.mapped set, m.nf etc. filled), the apply,
// and the bytes of one precision's matrices
fe_status mapped_setup(Mesh& m, double amp);
fe_status launch_apply_mapped(const Mesh& m, const ApplyArgs& a, fe_prec prec, hipStream_t s);
size_t mapped_matrix_bytes(const Mesh& m, fe_prec prec);
// Launch timing (a measurement aid): while enabled, timed_begin records a start event on s and
// returns a slot (-1 when timing is off), timed_end records the stop event. kind is an fe_prec for
// operator applies and kTimedSweep + pass (0, 1, 2 = A, B, C) for the MINRES row sweeps.
constexpr int kTimedSweep = 16;
fe_status apply_timing(int enable);
fe_status apply_timing_read(fe_prec prec, int64_t* launches, double* ms, double* bytes, double* columns);
fe_status sweep_timing_read(int pass, int64_t* launches, double* ms, double* bytes, double* columns);
fe_status timed_begin(int kind, double bytes, double cols, hipStream_t s, int* slot);
fe_status timed_end(int slot, hipStream_t s);

// Block operations (FP64 reductions; T = double or float storage).
// Gram: out (nx x ny, row-major, FP64 device) = X^T Y over the first N rows.
size_t gram_work_bytes(int64_t N, int nx, int ny);
fe_status gram(const void* X, int ldx, const void* Y, int ldy, int64_t N, int nx, int ny, bool f32,
               double* out, void* work, hipStream_t s);
// out[a, j] = sum_k X[a, k] C[k, j] (C FP64 device, nin x nout, row-major); out may equal X up to
// 64 columns in and out (wider blocks are rotated in 64 x 64 tiles and out must not overlap X).
fe_status rotate(const double* X, int ldx, int64_t N, int nin, const double* C, int nout, double* out,
                 int ldo, hipStream_t s);
// Column-wise dot products d_j = sum_a X[a,j] Y[a,j] (FP64 result, device array nv).
// out = X^T diag(wa - wb) X (n x n, X: N x n with leading dimension ld); work: gram_work_bytes(N, n, n).
fe_status gram_weighted(const double* X, int ld, const double* wa, const double* wb, int64_t N, int n, double* out,
                        void* work, hipStream_t s);
size_t along_psi_work_bytes(int64_t N, int n);
size_t poisson_work_bytes(int64_t nf);
// Y += X C over N rows (X: N x nin, C: nin x nout row-major on the device, Y: N x nout).
fe_status rotate_add(const double* X, int ldx, int64_t N, int nin, const double* C, int nout, double* Y, int ldy,
                     hipStream_t s);
// Y += alpha X C
fe_status rotate_axpy(const double* X, int ldx, int64_t N, int nin, const double* C, int nout, double alpha, double* Y,
                      int ldy, hipStream_t s);
size_t coldot_work_bytes(int64_t N, int nv);
fe_status coldot(const void* X, const void* Y, int ld, int64_t N, int nv, bool f32, double* out, void* work,
                 hipStream_t s);
// out[j] = sum_a (HX[a,j] - lam_j X[a,j])^2 (lam on device); work: coldot_work_bytes.
fe_status colresid(const double* HX, const double* X, const double* lam, int ld, int64_t N, int nv, double* out,
                   void* work, hipStream_t s);
// Scalar dot product of two FP64 vectors (device result).
fe_status dot1(const double* x, const double* y, int64_t n, double* out, void* work, hipStream_t s);
fe_status max1(const double* x, int64_t n, double* out, void* work, hipStream_t s);

// bf16 storage: the upper 16 bits of an IEEE binary32 (FE_BF16 blocks hold these bit patterns)
typedef unsigned short bf16_t;

// Kernels used by the Krylov and loss/gradient code (defined in blockops.hip).
fe_status cast_block_to_f32(const double* src, float* dst, int64_t count, hipStream_t s);
// FP64 -> bf16 with round-to-nearest-even; bf16 -> FP64 (exact) of columns [c0, ld)
fe_status cast_block_to_bf16(const double* src, bf16_t* dst, int64_t count, hipStream_t s);
fe_status cast_cols_bf16_to_f64(const bf16_t* src, double* dst, int64_t nrow, int ld, int c0, hipStream_t s);
fe_status cast_block_to_f64(const float* src, double* dst, int64_t count, hipStream_t s);
// columns [c0, ld) of an nrow x ld block (row pitch ld in both)
fe_status cast_cols_to_f64(const float* src, double* dst, int64_t nrow, int ld, int c0, hipStream_t s);
fe_status axpby(double alpha, const double* x, double beta, double* y, int64_t n, hipStream_t s);
fe_status fill(double* y, double val, int64_t n, hipStream_t s);

// Projection X <- X - Psi (Psi^T X) (Psi: N x k, ld k; X: N x nv, ld nv), any widths, in groups
// of at most 64 columns of X. work: project_work_bytes(N, k, nv).
size_t project_work_bytes(int64_t N, int k, int nv);
// f32: Psi and X are float blocks (products accumulated in FP64).
fe_status project_out(const void* Psi, int k, void* X, int nv, int64_t N, bool f32, void* work, hipStream_t s);
// The same with Psi's row pitch ldp >= k (Psi a column range of a wider block).
fe_status project_out_ld(const void* Psi, int ldp, int k, void* X, int nv, int64_t N, bool f32, void* work,
                         hipStream_t s);
// X <- X - Psi G with a given G (k x nv, FP64 device).
fe_status fill_f32(float* y, float val, int64_t n, hipStream_t s);
fe_status copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t s);

// loss_grad's two phases (Eqs. 1, 4, 7, 10, 11, 20, 22) over caller-given buffers: rho_w is an
// N_f density buffer used when rho is NULL; scratch holds loss_grad_scratch_bytes(nf, nocc).
size_t loss_grad_scratch_bytes(int64_t nf, int nocc);
fe_status loss_grad_impl(const Mesh& m, const double* Psi, const double* occ_h, int nocc, const double* rho_data,
                         const double* Q, double tau_bc, double* rho, double* B, double* grad, double* loss_h,
                         double* rho_w, void* scratch, const char* name, hipStream_t s);

}  // namespace invdft
