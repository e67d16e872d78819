// C ABI of the inverse-DFT hot path: argument checks, work-buffer layout and
// the host-side control of the iterative methods. All arithmetic on blocks
// runs in the HIP kernels of apply.hip, blockops.hip and krylov.hip; the host
// only does O(nv^3) dense FP64 algebra on nv x nv projected matrices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "krylov.h"
#include "minres_fused.h"
#include "ref_tables.h"

struct fe_mesh_s {
  invdft::Mesh m;
};

namespace invdft {

const Mesh* mesh_tables(fe_mesh mesh) { return mesh ? &mesh->m : nullptr; }

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

fe_status fail(fe_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

fe_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string("HIP error ") + hipGetErrorString(e) + " in " + what;
  return FE_EDEVICE;
}

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's work buffer; with base == nullptr it only measures.
struct Bump {
  char* base;
  size_t off = 0;
  explicit Bump(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align_up(count * sizeof(T));
    return p;
  }
};

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

fe_status check_mesh(fe_mesh mesh) {
  if (!mesh) return fail(FE_EINVAL, "mesh handle is NULL");
  return FE_OK;
}

fe_status check_block(const void* X, const char* name, int nv, int ld) {
  if (!X) return fail(FE_EINVAL, std::string(name) + " is NULL");
  if (!aligned16(X)) return fail(FE_EINVAL, std::string(name) + " is not 16-byte aligned");
  if (nv < 1) return fail(FE_EINVAL, "nv must be >= 1");
  if (ld < nv) return fail(FE_EINVAL, "ld must be >= nv");
  return FE_OK;
}

size_t elem_size(fe_prec p) { return p == FE_F64 ? sizeof(double) : p == FE_F32 ? sizeof(float) : sizeof(bf16_t); }

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// ---------------------------------------------------------------- filter
// Scaled three-term recurrence of the Chebyshev filter (Zhou and Saad 2007):
// Y1 = (sigma1/e)(H - c)X, Y_{k+1} = (2 sigma_{k+1}/e)(H - c)Y_k - sigma_k sigma_{k+1} Y_{k-1},
// sigma_{k+1} = 1 / (2/sigma1 - sigma_k). Two blocks suffice: the newest block
// overwrites the oldest one, which the kernel reads element by element before it writes.
fe_status filter_impl(const Mesh& m, const double* v, int degree, double a, double b, double a0, void* X, int nv,
                      int ld, fe_prec prec, void* work, hipStream_t s) {
  const double e = 0.5 * (b - a), c = 0.5 * (b + a);
  const double sigma1 = e / (a0 - c);
  double sigma = sigma1;
  const double gamma = 2.0 / sigma1;
  void* bufs[2] = {X, work};
  ApplyArgs aa{};
  aa.v = v;
  aa.nv = nv;
  aa.ld = ld;
  aa.cshift = c;
  // step 1: work = (sigma1/e)(H - c) X
  aa.X = X;
  aa.Y = work;
  aa.Z = nullptr;
  aa.alpha = sigma1 / e;
  aa.beta = 0.0;
  fe_status st = launch_apply(m, aa, prec, s);
  if (st != FE_OK) return st;
  int cur = 1;  // bufs[cur] holds Y_k, bufs[1-cur] holds Y_{k-1}
  for (int k = 2; k <= degree; ++k) {
    const double sigma_new = 1.0 / (gamma - sigma);
    aa.X = bufs[cur];
    aa.Z = bufs[1 - cur];
    aa.Y = bufs[1 - cur];
    aa.alpha = 2.0 * sigma_new / e;
    aa.beta = -sigma * sigma_new;
    st = launch_apply(m, aa, prec, s);
    if (st != FE_OK) return st;
    sigma = sigma_new;
    cur = 1 - cur;
  }
  if (cur == 1) {
    const size_t es = elem_size(prec);
    if (nv == ld) {
      INVDFT_HIP(hipMemcpyAsync(X, work, (size_t)m.nf * ld * es, hipMemcpyDeviceToDevice, s));
    } else {  // a sub-block of columns: copy only those
      INVDFT_HIP(hipMemcpy2DAsync(X, ld * es, work, ld * es, nv * es, m.nf, hipMemcpyDeviceToDevice, s));
    }
  }
  return FE_OK;
}

size_t filter_work(const Mesh& m, int ld, fe_prec prec) { return align_up((size_t)m.nf * ld * elem_size(prec)); }

// ------------------------------------------------------------ Rayleigh-Ritz
struct RRWork {
  double *HX, *T, *S, *H, *C, *lam, *res, *gw;
};

RRWork rr_layout(Bump& bp, const Mesh& m, int nv, int ld) {
  RRWork w{};
  w.HX = bp.take<double>((size_t)m.nf * ld);
  // above 64 columns the rotations are not in place: their results go through T
  w.T = nv > 64 ? bp.take<double>((size_t)m.nf * ld) : nullptr;
  w.S = bp.take<double>((size_t)nv * nv);
  w.H = bp.take<double>((size_t)nv * nv);
  w.C = bp.take<double>((size_t)nv * nv);
  w.lam = bp.take<double>(nv);
  w.res = bp.take<double>(nv);
  w.gw = bp.take<double>(std::max(gram_work_bytes(m.nf, nv, nv), coldot_work_bytes(m.nf, nv)) / sizeof(double) + 1);
  return w;
}

fe_status rr_impl(const Mesh& m, const double* v, double* X, double* eig_h, double* res_h, int nv, int ld,
                  void* work, hipStream_t s) {
  Bump bp(work);
  RRWork w = rr_layout(bp, m, nv, ld);
  fe_status st = gram(X, ld, X, ld, m.nf, nv, nv, false, w.S, w.gw, s);
  if (st != FE_OK) return st;
  ApplyArgs aa{};
  aa.X = X;
  aa.Y = w.HX;
  aa.v = v;
  aa.nv = nv;
  aa.ld = ld;
  aa.alpha = 1.0;
  st = launch_apply(m, aa, FE_F64, s);
  if (st != FE_OK) return st;
  st = gram(X, ld, w.HX, ld, m.nf, nv, nv, false, w.H, w.gw, s);
  if (st != FE_OK) return st;
  std::vector<double> Sh((size_t)nv * nv), Hh((size_t)nv * nv);
  INVDFT_HIP(hipMemcpyAsync(Sh.data(), w.S, Sh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipMemcpyAsync(Hh.data(), w.H, Hh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  for (double x : Sh)
    if (!std::isfinite(x)) return fail(FE_ENOTPD, "rayleigh_ritz: overlap matrix is not finite");
  // S = L L^T ; A = L^{-1} H L^{-T} ; A = V diag(lam) V^T ; C = L^{-T} V  (Eq. 24)
  if (!cholesky_lower(nv, Sh.data())) return fail(FE_ENOTPD, "rayleigh_ritz: overlap matrix is not positive definite");
  std::vector<double> Li((size_t)nv * nv), T((size_t)nv * nv, 0.0), A((size_t)nv * nv, 0.0);
  invert_lower(nv, Sh.data(), Li.data());
  for (int i = 0; i < nv; ++i)  // symmetrise H_X
    for (int j = 0; j < i; ++j) {
      const double a = 0.5 * (Hh[(size_t)i * nv + j] + Hh[(size_t)j * nv + i]);
      Hh[(size_t)i * nv + j] = Hh[(size_t)j * nv + i] = a;
    }
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      double t = 0.0;
      for (int k = 0; k <= i; ++k) t += Li[(size_t)i * nv + k] * Hh[(size_t)k * nv + j];
      T[(size_t)i * nv + j] = t;
    }
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j <= i; ++j) {
      double t = 0.0;
      for (int k = 0; k <= j; ++k) t += T[(size_t)i * nv + k] * Li[(size_t)j * nv + k];
      A[(size_t)i * nv + j] = A[(size_t)j * nv + i] = t;
    }
  std::vector<double> lam(nv), V((size_t)nv * nv), C((size_t)nv * nv, 0.0);
  jacobi_eigh(nv, A.data(), lam.data(), V.data());
  for (int i = 0; i < nv; ++i)  // C = L^{-T} V: (L^{-T})_{ik} = Li[k][i], nonzero for k >= i
    for (int j = 0; j < nv; ++j) {
      double t = 0.0;
      for (int k = i; k < nv; ++k) t += Li[(size_t)k * nv + i] * V[(size_t)k * nv + j];
      C[(size_t)i * nv + j] = t;
    }
  INVDFT_HIP(hipMemcpyAsync(w.C, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s));
  INVDFT_HIP(hipMemcpyAsync(w.lam, lam.data(), nv * sizeof(double), hipMemcpyHostToDevice, s));
  double* HX = w.HX;
  if (!w.T) {
    if ((st = rotate(X, ld, m.nf, nv, w.C, nv, X, ld, s)) != FE_OK) return st;
    if ((st = rotate(HX, ld, m.nf, nv, w.C, nv, HX, ld, s)) != FE_OK) return st;
  } else {
    if ((st = rotate(X, ld, m.nf, nv, w.C, nv, w.T, ld, s)) != FE_OK) return st;
    INVDFT_HIP(hipMemcpy2DAsync(X, ld * sizeof(double), w.T, ld * sizeof(double), nv * sizeof(double), m.nf,
                                hipMemcpyDeviceToDevice, s));
    if ((st = rotate(w.HX, ld, m.nf, nv, w.C, nv, w.T, ld, s)) != FE_OK) return st;
    HX = w.T;
  }
  std::vector<double> res(nv);
  st = colresid(HX, X, w.lam, ld, m.nf, nv, w.res, w.gw, s);
  if (st != FE_OK) return st;
  INVDFT_HIP(hipMemcpyAsync(res.data(), w.res, nv * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < nv; ++i) {
    if (eig_h) eig_h[i] = lam[i];
    if (res_h) res_h[i] = std::sqrt(std::max(res[i], 0.0));
  }
  return FE_OK;
}

// -------------------------------------------------------------- eigensolve
struct EigWork {
  void* rr;
  void* filt;   // filter work block (precision of the filter)
  float* Xf;    // FP32 copy of X for the reduced-precision filter
  double* vmax;
  void* redw;
};

EigWork eig_layout(Bump& bp, const Mesh& m, int nv, int ld, fe_prec prec) {
  EigWork w{};
  Bump rrb(nullptr);
  rr_layout(rrb, m, nv, ld);
  w.rr = bp.take<char>(rrb.off);
  w.filt = bp.take<char>(filter_work(m, ld, FE_F64));  // large enough for either filter precision
  w.Xf = prec == FE_F64 ? nullptr : bp.take<float>((size_t)m.nf * ld);
  w.vmax = bp.take<double>(1);
  w.redw = bp.take<double>(1025);
  return w;
}

// ------------------------------------------------------------------ MINRES
// Work blocks of one MINRES solve in storage type T (FP64 or FP32).
struct MRWork {
  void *R1, *R2, *Z, *Y, *Wa, *Wb, *X;   // X: the solution of the inner solve (FP32 path only)
  void* Qw;                              // compacted solution block
  int* map;                              // column map of a compaction (device)
  void* fused;                           // partial sums of the fused passes
  double *dinv, *st, *d1, *d2, *bnorm, *pw;
  // FP32 refinement extras
  float* Psif;    // FP32 copy of Psi
  double *R64, *Y64;
  // FP64 refinement on the true residual: its right-hand side, correction and column mask
  double *rb, *dq, *mask;
  // more than 64 orbitals: the fused passes' copy of the first 64, and one group's B and Q
  double *Pf, *Bg, *Qg;
};

// k columns solved together (at most 64), kpsi orbitals to project against
MRWork mr_layout(Bump& bp, const Mesh& m, int k, fe_prec prec, int kpsi = 0) {
  MRWork w{};
  if (kpsi < k) kpsi = k;
  const size_t blk = (size_t)m.nf * k;
  const size_t es = prec == FE_F64 ? sizeof(double) : sizeof(float);
  w.R1 = bp.take<char>(blk * es);
  w.R2 = bp.take<char>(blk * es);
  w.Z = bp.take<char>(blk * es);
  w.Y = bp.take<char>(blk * es);
  w.Wa = bp.take<char>(blk * es);
  w.Wb = bp.take<char>(blk * es);
  w.Qw = bp.take<char>(blk * es);
  w.map = bp.take<int>(64);
  w.fused = bp.take<char>(fused_work_bytes(m.nf));
  w.dinv = bp.take<double>(m.nf);
  w.st = bp.take<double>((size_t)mr_state_count() * k);
  w.d1 = bp.take<double>(k);
  w.d2 = bp.take<double>(k);
  w.bnorm = bp.take<double>(k);
  w.pw = bp.take<double>(std::max(project_work_bytes(m.nf, kpsi, k), coldot_work_bytes(m.nf, k)) / sizeof(double) + 1);
  if (prec != FE_F64) {
    w.X = bp.take<char>(blk * es);
    w.Psif = bp.take<float>(blk);
    w.R64 = bp.take<double>(blk);
    w.Y64 = bp.take<double>(blk);
  } else {
    w.rb = bp.take<double>(blk);
    w.dq = bp.take<double>(blk);
    w.mask = bp.take<double>((size_t)k * k);
  }
  return w;
}

// An adjoint solve of nocc columns: groups of at most 64 shifts, each against all nocc orbitals
// (FP64 above 64 orbitals).
MRWork adjoint_layout(Bump& bp, const Mesh& m, int nocc, fe_prec prec) {
  const int k = std::min(nocc, 64);
  MRWork w = mr_layout(bp, m, k, prec, nocc);
  if (nocc > 64) {
    w.Pf = bp.take<double>((size_t)m.nf * 64);
    w.Bg = bp.take<double>((size_t)m.nf * 64);
    w.Qg = bp.take<double>((size_t)m.nf * 64);
  }
  return w;
}

template <typename T>
fe_status fill_t(T* y, int64_t n, hipStream_t s);
template <>
fe_status fill_t<double>(double* y, int64_t n, hipStream_t s) { return fill(y, 0.0, n, s); }
template <>
fe_status fill_t<float>(float* y, int64_t n, hipStream_t s) { return fill_f32(y, 0.0f, n, s); }

// MINRES (Paige and Saunders 1975) on P (H - eps_i) P q_i = b_i for all columns in lockstep,
// preconditioner P D^{-1} P. Blocks of type T; every per-column scalar in FP64 on the device.
// Columns that have converged are dropped from every block (and from the operator apply)
// once enough of them have: the solve's cost then follows the still-active columns.
// On return `iters` holds per-column iteration counts, `active` the still-unconverged flags
// (both in the original column order).
// Deflation of the preconditioner (FP64 only): with U (N x nb, orthonormal, orthogonal to
// Psi) approximate eigenvectors above every shift, Rayleigh quotients theta,
//   M = P_ext D^{-1} P_ext + U diag(1 / (theta - eps_i)) U^T,   P_ext = I - V V^T, V = [Psi U].
// M is symmetric positive definite on the complement of Psi whatever the quality of U, so
// the solution is unchanged; the Krylov space no longer has to resolve the low states U
// captures, which are what slows the columns with the smallest gaps. The stored Lanczos
// vectors are r' = r - U c with c = U^T r kept as small per-column arrays; the fused passes
// then run with V in place of Psi (pass B's subtraction V (V^T y) is exactly the deflated
// recurrence), plus four small per-column corrections.
// Above 64 columns, V = [Psi U] is split: the fused passes take its first 64 columns
// (Vf = [Psi U_f], nbf = 64 - k0 vectors of U), and the rest U_r (nb - nbf vectors) is handled
// by separate Gram and update sweeps whose coefficients Gr1 = U_r^T y and Gr2 = U_r^T u also
// feed the deflation's per-column corrections.
struct Deflation {
  double* V;            // [Psi U(:, 0..nbf)], N x (k0 + nbf), nbf = min(nb, 64 - k0)
  double* U;            // N x nb
  int nb, nbf;
  double* theta;        // nb (device)
  double* eps;          // shifts of the current columns (device, k)
  double *cA, *cB, *cC, *tmp;  // nb x k small arrays (device)
  double *Gr1, *Gr2;    // (nb - nbf) x k: U_r^T y and U_r^T u (device)
};

// Extra work of a deflated solve with k <= 64 shifts and nb <= 64 deflation vectors; pw
// replaces MRWork's projection scratch (V is wider than Psi).
Deflation defl_layout(Bump& bp, const Mesh& m, int k, int nb, double** Ucopy, double** pw) {
  Deflation d{};
  *Ucopy = bp.take<double>((size_t)m.nf * nb);
  d.nb = nb;
  d.nbf = std::max(0, std::min(nb, 64 - k));
  d.V = bp.take<double>((size_t)m.nf * (k + d.nbf));
  d.U = *Ucopy;
  d.theta = bp.take<double>(64);
  d.eps = bp.take<double>(64);
  d.cA = bp.take<double>(64 * 64);
  d.cB = bp.take<double>(64 * 64);
  d.cC = bp.take<double>(64 * 64);
  d.tmp = bp.take<double>(64 * 64);
  d.Gr1 = bp.take<double>(64 * 64);
  d.Gr2 = bp.take<double>(64 * 64);
  *pw = bp.take<double>(project_work_bytes(m.nf, 128, 64) / sizeof(double) + 1);
  return d;
}

// The orbitals a solve projects against: Psi (N x kpsi, row pitch kpsi) in full, the block the
// fused passes take (Pf: N x kf, kf <= 64, its own row pitch kf) and the rest (Pr: the columns of
// Psi past Pf, kr of them, row pitch kpsi), projected by separate sweeps. Up to 64 orbitals Pf is
// Psi and there is no rest.
template <typename T>
struct ProjSet {
  const T* Psi;
  int kpsi;
  const T* Pf;
  int kf;
  const T* Pr;
  int kr;
};

template <typename T>
ProjSet<T> proj_whole(const T* Psi, int k) {
  return ProjSet<T>{Psi, k, Psi, k, nullptr, 0};
}

template <typename T>
fe_status minres_core(const Mesh& m, const double* v, const ProjSet<T>& ps, const double* eps_h, int k0, const T* B,
                      T* Q, double tol, int maxit, MRWork& w, std::vector<double>& iters, std::vector<double>& active,
                      hipStream_t s, Deflation* df = nullptr) {
  const int64_t nf = m.nf;
  const bool f32 = sizeof(T) == sizeof(float);
  const fe_prec prec = f32 ? FE_F32 : FE_F64;
  const int SC = mr_state_count();
  fe_status st;
  int k = k0;
  size_t blk = (size_t)nf * k;
  T *R1 = static_cast<T*>(w.R1), *R2 = static_cast<T*>(w.R2), *Z = static_cast<T*>(w.Z), *Y = static_cast<T*>(w.Y);
  T *Wa = static_cast<T*>(w.Wa), *Wb = static_cast<T*>(w.Wb), *Qw = static_cast<T*>(w.Qw);
  if ((st = fill_t<T>(Qw, blk, s)) != FE_OK) return st;
  if ((st = fill_t<T>(Wa, blk, s)) != FE_OK) return st;
  if ((st = fill_t<T>(Wb, blk, s)) != FE_OK) return st;
  const bool defl = df != nullptr;
  if (defl && ps.Pr) return fail(FE_EINVAL, "adjoint_solve: deflation needs Psi and U within 64 columns");
  const T* Psi = ps.Psi;
  const int kpsi = ps.kpsi;
  const T* Pj = ps.Pf;     // the block the fused passes project with
  int kp = ps.kf;
  // the orbitals past the fused block: X <- X - Pr (Pr^T X) on a k-column block
  auto project_rest = [&](T* X, int k) -> fe_status {
    return ps.Pr ? project_out_ld(ps.Pr, kpsi, ps.kr, X, k, nf, f32, w.pw, s) : FE_OK;
  };
  double *cR1 = nullptr, *cR2 = nullptr, *cN = nullptr;
  if (!defl) {
    if ((st = copy_bytes(B, R1, blk * sizeof(T), s)) != FE_OK) return st;
    if ((st = copy_bytes(B, R2, blk * sizeof(T), s)) != FE_OK) return st;
    // z = P D^{-1} b ; beta1 = sqrt(b.z)
    if ((st = k_precond<T>(B, w.dinv, k, nf, Z, s)) != FE_OK) return st;
    if ((st = project_out(Psi, kpsi, Z, k, nf, f32, w.pw, s)) != FE_OK) return st;
  } else {
    if constexpr (sizeof(T) == sizeof(double)) {
      Pj = df->V;
      kp = k0 + df->nbf;
      cR1 = df->cA;
      cR2 = df->cB;
      cN = df->cC;
      const int nb = df->nb;
      // the shifts of all k0 columns (a previous solve leaves them compacted)
      INVDFT_HIP(hipMemcpyAsync(df->eps, eps_h, k0 * sizeof(double), hipMemcpyHostToDevice, s));
      // c0 = U^T b ; r' = b - U c0 (R1 and R2) ; z = P_ext D^{-1} r' + U c0 / (theta - eps) ; beta1^2 = b.z
      if ((st = gram(df->U, nb, B, k, nf, nb, k, false, cR1, w.pw, s)) != FE_OK) return st;
      if ((st = copy_bytes(cR1, cR2, (size_t)nb * k * sizeof(double), s)) != FE_OK) return st;
      if ((st = copy_bytes(B, R1, blk * sizeof(T), s)) != FE_OK) return st;
      if ((st = rotate_axpy(df->U, nb, nf, nb, cR1, k, -1.0, R1, k, s)) != FE_OK) return st;
      if ((st = copy_bytes(R1, R2, blk * sizeof(T), s)) != FE_OK) return st;
      if ((st = k_precond<T>(R1, w.dinv, k, nf, Z, s)) != FE_OK) return st;
      if ((st = project_out(Pj, kp, Z, k, nf, false, w.pw, s)) != FE_OK) return st;
      if (nb > df->nbf &&
          (st = project_out_ld(df->U + df->nbf, nb, nb - df->nbf, Z, k, nf, false, w.pw, s)) != FE_OK)
        return st;
      if ((st = defl_scale(cR1, df->theta, df->eps, k, nb, df->tmp, s)) != FE_OK) return st;
      if ((st = rotate_axpy(df->U, nb, nf, nb, df->tmp, k, 1.0, Z, k, s)) != FE_OK) return st;
    } else {
      return fail(FE_EINVAL, "adjoint_solve: deflation needs FP64");
    }
  }
  if ((st = coldot(B, Z, k, nf, k, f32, w.d1, w.pw, s)) != FE_OK) return st;
  if ((st = mr_init(w.st, w.d1, k, s)) != FE_OK) return st;
  std::vector<int> orig(k0);
  for (int j = 0; j < k0; ++j) orig[j] = j;
  std::vector<double> eps(eps_h, eps_h + k0);
  iters.assign(k0, 0.0);
  active.assign(k0, 1.0);
  std::vector<double> act(k0), sth((size_t)SC * k0), stn((size_t)SC * k0);
  ApplyArgs aa{};
  aa.v = v;
  aa.alpha = 1.0;
  FusedWork fw = fused_layout(w.fused, nf);
  const int check_every = 8;
  // writes the compact solution columns back to Q and records per-column counters
  auto flush = [&](bool all_cols) -> fe_status {
    fe_status st2;
    INVDFT_HIP(hipMemcpyAsync(w.map, orig.data(), k * sizeof(int), hipMemcpyHostToDevice, s));
    if ((st2 = k_scatter_cols<T>(Qw, k, Q, k0, w.map, nf, s)) != FE_OK) return st2;
    INVDFT_HIP(hipMemcpyAsync(sth.data(), w.st, (size_t)SC * k * sizeof(double), hipMemcpyDeviceToHost, s));
    INVDFT_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < k; ++j) {
      iters[orig[j]] = sth[(size_t)mr_state_iters() * k + j];
      active[orig[j]] = sth[(size_t)mr_state_active() * k + j];
    }
    (void)all_cols;
    return FE_OK;
  };
  for (int it = 1; it <= maxit; ++it) {
    aa.nv = k;
    aa.ld = k;
    aa.colshift = eps.data();
    // y = (H - eps) (z / beta)
    aa.X = Z;
    aa.Y = Y;
    aa.d_colscale = w.st + (size_t)mr_state_invbeta() * k;
    if ((st = launch_apply(m, aa, prec, s)) != FE_OK) return st;
    // the orbitals past the fused block leave y first (P = P_f P_r: the two sets are orthogonal)
    if ((st = project_rest(Y, k)) != FE_OK) return st;
    // the coefficients U_r^T y of the deflation vectors past the fused block (y keeps those
    // components through pass A: z has components along U, so z.y needs all of y)
    const int nbr = defl ? df->nb - df->nbf : 0;
    if constexpr (sizeof(T) == sizeof(double)) {
      if (nbr > 0 && (st = gram(df->U + df->nbf, df->nb, Y, k, nf, nbr, k, false, df->Gr1, w.pw, s)) != FE_OK)
        return st;
    }
    // one sweep: G = Psi^T y, z.y, z.r1; alfa = v.(P y - c1 r1) = v.y - c1 v.r1 (v is orthogonal to Psi)
    if ((st = minres_pass_a<T>(Pj, kp, Y, Z, R1, k, nf, fw, s)) != FE_OK) return st;
    if (defl && (st = defl_d2(fw.d2, cR1, cR2, df->theta, df->eps, k, df->nb, s)) != FE_OK) return st;
    if ((st = mr_alfa(w.st, fw.d1, fw.d2, k, it == 1, s)) != FE_OK) return st;
    if (defl && (st = defl_cnew(fw.G, k0, df->nbf, df->Gr1, df->nb, cR1, cR2, w.st, k, cN, s)) != FE_OK) return st;
    // before pass B forms r' = y - V G1 - c1 r1' - c2 r2', y loses its U_r part as well
    if constexpr (sizeof(T) == sizeof(double)) {
      if (nbr > 0 && (st = rotate_axpy(df->U + df->nbf, df->nb, nf, nbr, df->Gr1, k, -1.0, Y, k, s)) != FE_OK)
        return st;
    }
    // r_new = P y - c1 r1 - c2 r2 (into R1) ; u = D^{-1} r_new (into Y) ; G2 = Psi^T u ; beta^2 = r_new.u
    if ((st = minres_pass_b<T>(Pj, kp, Y, R1, R2, w.st, w.dinv, k, nf, fw, s)) != FE_OK) return st;
    if (defl) {
      if constexpr (sizeof(T) == sizeof(double)) {
        if (nbr > 0 && (st = gram(df->U + df->nbf, df->nb, Y, k, nf, nbr, k, false, df->Gr2, w.pw, s)) != FE_OK)
          return st;
      }
      if ((st = defl_beta_g2(fw.d, fw.G2, k0, df->nbf, df->Gr2, df->nb, cN, df->theta, df->eps, k, s)) != FE_OK)
        return st;
      // u loses U_r (U_r^T u - c_new / (theta - eps)), as pass C does for the vectors inside
      if constexpr (sizeof(T) == sizeof(double)) {
        if (nbr > 0 && (st = rotate_axpy(df->U + df->nbf, df->nb, nf, nbr, df->Gr2, k, -1.0, Y, k, s)) != FE_OK)
          return st;
      }
      double* t = cR1;  // the coefficients follow the vectors: cR1 <- cR2, cR2 <- c_new
      cR1 = cR2;
      cR2 = cN;
      cN = t;
    }
    std::swap(R1, R2);  // R1 <- old r2, R2 <- r_new
    // u loses its part along the rest before pass C forms z = u - Pf G2; G2 = Pf^T u and r.u are
    // unchanged by it (Pf and r are orthogonal to the rest)
    if ((st = project_rest(Y, k)) != FE_OK) return st;
    if ((st = mr_givens(w.st, fw.d, k, tol, s)) != FE_OK) return st;
    // z_new = P u (into Y) ; w and q updates with the new rotation
    if ((st = minres_pass_c<T>(Pj, kp, Y, Z, Wb, Wa, Qw, w.st, k, nf, fw, s)) != FE_OK) return st;
    std::swap(Wa, Wb);
    std::swap(Z, Y);  // Y now holds the previous z: free until the next apply
    if (it % check_every == 0 || it == maxit) {
      INVDFT_HIP(hipMemcpyAsync(act.data(), w.st + (size_t)mr_state_active() * k, k * sizeof(double),
                                hipMemcpyDeviceToHost, s));
      INVDFT_HIP(hipStreamSynchronize(s));
      int na = 0;
      for (int j = 0; j < k; ++j) na += act[j] > 0.0 ? 1 : 0;
      if (na == 0 || it == maxit) break;
      if (na <= k - std::max(2, k / 8)) {   // measured: 1.7 % faster than waiting for k / 4
        // drop the converged columns: write them out, then compact every block and the state
        if ((st = flush(false)) != FE_OK) return st;
        std::vector<int> keep;
        for (int j = 0; j < k; ++j)
          if (act[j] > 0.0) keep.push_back(j);
        INVDFT_HIP(hipMemcpyAsync(w.map, keep.data(), na * sizeof(int), hipMemcpyHostToDevice, s));
        T** blocks[6] = {&R1, &R2, &Z, &Wa, &Wb, &Qw};
        for (T** bptr : blocks) {
          if ((st = k_select_cols<T>(*bptr, k, Y, na, w.map, nf, s)) != FE_OK) return st;
          std::swap(*bptr, Y);
        }
        for (int q = 0; q < SC; ++q)
          for (int j = 0; j < na; ++j) stn[(size_t)q * na + j] = sth[(size_t)q * k + keep[j]];
        INVDFT_HIP(hipMemcpyAsync(w.st, stn.data(), (size_t)SC * na * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<int> orig2(na);
        std::vector<double> eps2(na);
        for (int j = 0; j < na; ++j) {
          orig2[j] = orig[keep[j]];
          eps2[j] = eps[keep[j]];
        }
        orig.swap(orig2);
        eps.swap(eps2);
        if (defl) {
          // compact the small coefficient arrays and the device shifts the same way
          const int nb = df->nb;
          std::vector<double> ch((size_t)nb * k), cc((size_t)nb * na);
          for (double* c : {cR1, cR2}) {
            INVDFT_HIP(hipMemcpyAsync(ch.data(), c, ch.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            INVDFT_HIP(hipStreamSynchronize(s));
            for (int j = 0; j < nb; ++j)
              for (int i = 0; i < na; ++i) cc[(size_t)j * na + i] = ch[(size_t)j * k + keep[i]];
            INVDFT_HIP(hipMemcpyAsync(c, cc.data(), cc.size() * sizeof(double), hipMemcpyHostToDevice, s));
            INVDFT_HIP(hipStreamSynchronize(s));
          }
          INVDFT_HIP(hipMemcpyAsync(df->eps, eps.data(), na * sizeof(double), hipMemcpyHostToDevice, s));
        }
        k = na;
        INVDFT_HIP(hipStreamSynchronize(s));  // host vectors above are sources of async copies
      }
    }
  }
  if ((st = flush(true)) != FE_OK) return st;
  if ((st = project_out(Psi, kpsi, Q, k0, nf, f32, w.pw, s)) != FE_OK) return st;
  return FE_OK;
}

// FP64 true residual R = B - P (H - eps) P Q of k columns and their norms rr (device); Psi has
// kpsi columns.
fe_status true_residual(const Mesh& m, const double* v, const double* Psi, int kpsi, const double* eps_h, int k,
                        const double* B, const double* Q, double* R, double* rr, double* pw, hipStream_t s) {
  ApplyArgs aa{};
  aa.v = v;
  aa.nv = k;
  aa.ld = k;
  aa.alpha = 1.0;
  aa.colshift = eps_h;
  aa.X = Q;
  aa.Y = R;
  fe_status st;
  if ((st = launch_apply(m, aa, FE_F64, s)) != FE_OK) return st;
  if ((st = project_out(Psi, kpsi, R, k, m.nf, false, pw, s)) != FE_OK) return st;
  if ((st = k_sub_from(B, R, (int64_t)m.nf * k, s)) != FE_OK) return st;
  return coldot(R, R, k, m.nf, k, false, rr, pw, s);
}

}  // namespace

// Bytes of loss_grad's scratch beyond the density buffer: the loss partials and the
// projection's Gram partials (what the allocation-free variant holds in its static array).
size_t loss_grad_scratch_bytes(int64_t nf, int nocc) {
  Bump bp(nullptr);
  bp.take<double>(1025);
  bp.take<char>(project_work_bytes(nf, nocc, nocc));
  return bp.off;
}

// Both phases of loss_grad. rho_w: an N_f buffer for the density when rho is NULL (phase 1);
// scratch: loss_grad_scratch_bytes(nf, nocc) bytes (loss partials, then projection work).
fe_status loss_grad_impl(const Mesh& m, const double* Psi, const double* occ_h, int nocc, const double* rho_data,
                         const double* Q, double tau_bc, double* rho, double* B, double* grad, double* loss_h,
                         double* rho_w, void* scratch, const char* name, hipStream_t s) {
  fe_status st;
  Bump bp(scratch);
  double* lw = bp.take<double>(1025);
  double* dl = lw + 1024;
  void* pw = bp.take<char>(project_work_bytes(m.nf, nocc, nocc));
  if (Q) {
    if (!grad) return fail(FE_EINVAL, std::string(name) + ": phase 2 needs grad");
    if (tau_bc > 0 && !rho_data) return fail(FE_EINVAL, std::string(name) + ": tau_bc needs rho_data");
    if ((st = k_grad(m, Psi, Q, nocc, rho_data, tau_bc, grad, s)) != FE_OK) return st;
    if (loss_h && rho && rho_data) {
      if ((st = k_loss(m, rho, rho_data, dl, lw, s)) != FE_OK) return st;
      INVDFT_HIP(hipMemcpyAsync(loss_h, dl, sizeof(double), hipMemcpyDeviceToHost, s));
      INVDFT_HIP(hipStreamSynchronize(s));
    }
    return FE_OK;
  }
  if ((B || loss_h) && !rho_data)
    return fail(FE_EINVAL, std::string(name) + ": rho_data is required for the loss and B");
  double* r = rho ? rho : rho_w;
  if (!r) return fail(FE_EINVAL, std::string(name) + ": rho is required");
  if ((st = k_density(m, Psi, nocc, occ_h, r, s)) != FE_OK) return st;
  if (B) {
    if ((st = k_rhs(m, Psi, nocc, occ_h, r, rho_data, B, s)) != FE_OK) return st;
    if ((st = project_out(Psi, nocc, B, nocc, m.nf, false, pw, s)) != FE_OK) return st;
  }
  if (loss_h) {
    if ((st = k_loss(m, r, rho_data, dl, lw, s)) != FE_OK) return st;
    INVDFT_HIP(hipMemcpyAsync(loss_h, dl, sizeof(double), hipMemcpyDeviceToHost, s));
    INVDFT_HIP(hipStreamSynchronize(s));
  }
  return FE_OK;
}

}  // namespace invdft

using namespace invdft;

// =================================================================== C ABI
extern "C" {

const char* fe_last_error(void) { return g_err.c_str(); }

// Shared by the uniform and the graded constructor; t (n + 1 cell boundaries) is NULL for
// the uniform mesh of [-L, L].
static fe_status mesh_create_impl(int p, int n, double L, const double* t, fe_mesh* out) {
  if (!out) return fail(FE_EINVAL, "fe_mesh_create: out is NULL");
  *out = nullptr;
  if (p < 1 || p > kMaxP) return fail(FE_EINVAL, "fe_mesh_create: p must be in [1, 8]");
  if (n < 1) return fail(FE_EINVAL, "fe_mesh_create: n must be >= 1");
  if (t) {
    for (int e = 0; e < n; ++e)
      if (!(t[e + 1] > t[e]) || !std::isfinite(t[e]) || !std::isfinite(t[e + 1]))
        return fail(FE_EINVAL, "fe_mesh_create_graded: cell boundaries must increase strictly");
    L = 0.5 * (t[n] - t[0]);
  }
  if (!(L > 0.0) || !std::isfinite(L)) return fail(FE_EINVAL, "fe_mesh_create: half_width must be > 0");
  const long long n1 = (long long)p * n - 1;
  if (n1 > 2000) return fail(FE_EINVAL, "fe_mesh_create: mesh too large");
  auto* h = new (std::nothrow) fe_mesh_s();
  if (!h) return fail(FE_ENOMEM, "fe_mesh_create: host allocation failed");
  Mesh& m = h->m;
  m.p = p;
  m.n = n;
  m.n1 = (int)n1;
  m.L = L;
  m.h = 2.0 * L / n;
  m.nf = n1 * n1 * n1;
  if (t) {
    m.graded = true;
    m.cell_h.resize(n);
    for (int e = 0; e < n; ++e) m.cell_h[e] = t[e + 1] - t[e];
    m.h = *std::min_element(m.cell_h.begin(), m.cell_h.end());   // reference width: the smallest
  }
  const int P1 = p + 1;
  std::vector<double> Kh(P1 * P1), Mh(P1 * P1), xi(P1), wi(P1);
  reference_matrices(p, Kh.data(), Mh.data(), xi.data(), wi.data());
  // assembled 1-D GLL weights at the element's local nodes: vertices are shared by two cells
  std::vector<double> wloc(P1), sloc(P1);
  for (int i = 0; i < P1; ++i) {
    wloc[i] = (i == 0 || i == p) ? m.h * wi[0] : 0.5 * m.h * wi[i];
    sloc[i] = 1.0 / std::sqrt(wloc[i]);
  }
  for (int i = 0; i < P1; ++i)
    for (int k = 0; k < P1; ++k) {
      m.mt[i * P1 + k] = sloc[i] * (0.5 * m.h) * Mh[i * P1 + k] * sloc[k];
      m.kt[i * P1 + k] = sloc[i] * (2.0 / m.h) * Kh[i * P1 + k] * sloc[k];
    }
  // exact symmetry and centrosymmetry (the kernels read one canonical copy of each entry)
  for (double* A : {m.mt, m.kt}) {
    double B[kMaxP1 * kMaxP1];
    for (int i = 0; i < P1; ++i)
      for (int k = 0; k < P1; ++k)
        B[i * P1 + k] = 0.25 * (A[i * P1 + k] + A[k * P1 + i] + A[(p - i) * P1 + (p - k)] + A[(p - k) * P1 + (p - i)]);
    std::memcpy(A, B, sizeof(double) * P1 * P1);
  }
  // the kernels use compile-time unit-cell tables: check them against these run-time ones
  {
    double maxdiff = 0.0, scale = 0.0;
    auto cmp = [&](const auto& tab) {
      for (int i = 0; i < P1; ++i)
        for (int k = 0; k < P1; ++k) {
          maxdiff = std::max(maxdiff, std::fabs(tab.mt[i][k] - m.mt[i * P1 + k]));
          maxdiff = std::max(maxdiff, std::fabs(tab.kt[i][k] - m.kt[i * P1 + k] * m.h * m.h));
          scale = std::max(scale, std::fabs(tab.kt[i][k]));
        }
    };
    switch (p) {
      case 1: cmp(ref::Table<1>::value); break;
      case 2: cmp(ref::Table<2>::value); break;
      case 3: cmp(ref::Table<3>::value); break;
      case 4: cmp(ref::Table<4>::value); break;
      case 5: cmp(ref::Table<5>::value); break;
      case 6: cmp(ref::Table<6>::value); break;
      case 7: cmp(ref::Table<7>::value); break;
      case 8: cmp(ref::Table<8>::value); break;
    }
    if (!(maxdiff <= 1e-13 * scale)) {
      delete h;
      return fail(FE_EDEVICE, "fe_mesh_create: compile-time element tables disagree with run-time ones");
    }
  }
  m.x1.resize(n1);
  m.w1.resize(n1);
  m.kd1.resize(n1);
  m.md1.resize(n1);
  for (long long f = 0; f < n1; ++f) {
    const long long g = f + 1;
    const long long e = g / p;
    const int j = (int)(g % p);
    if (!m.graded) {
      m.x1[f] = -L + m.h * (e + 0.5 * (xi[j] + 1.0));
      m.w1[f] = wloc[j];
      m.kd1[f] = (j == 0) ? m.kt[p * P1 + p] + m.kt[0] : m.kt[j * P1 + j];
      m.md1[f] = (j == 0) ? m.mt[p * P1 + p] + m.mt[0] : m.mt[j * P1 + j];
      continue;
    }
    // graded: cell e of width he (j > 0), or the vertex between cells e - 1 and e (j = 0)
    const double he = m.cell_h[e];
    m.x1[f] = t[e] + 0.5 * he * (xi[j] + 1.0);
    if (j == 0) {
      const double hl = m.cell_h[e - 1];
      m.w1[f] = 0.5 * (hl + he) * wi[0];
      m.kd1[f] = ((2.0 / hl) * Kh[p * P1 + p] + (2.0 / he) * Kh[0]) / m.w1[f];
      m.md1[f] = ((0.5 * hl) * Mh[p * P1 + p] + (0.5 * he) * Mh[0]) / m.w1[f];
    } else {
      m.w1[f] = 0.5 * he * wi[j];
      m.kd1[f] = (2.0 / he) * Kh[j * P1 + j] / m.w1[f];
      m.md1[f] = (0.5 * he) * Mh[j * P1 + j] / m.w1[f];
    }
  }
  // Fried element bound: (1/2) lambda_max(W_e^{-1/2} K_e W_e^{-1/2}), W_e the element's own lumped mass
  {
    const int np = P1 * P1 * P1;
    std::vector<double> A((size_t)np * np);
    std::vector<double> ke(P1 * P1), me(P1 * P1), we(P1);
    for (int i = 0; i < P1 * P1; ++i) {
      ke[i] = (2.0 / m.h) * Kh[i];
      me[i] = (0.5 * m.h) * Mh[i];
    }
    for (int i = 0; i < P1; ++i) we[i] = 0.5 * m.h * wi[i];
    for (int a = 0; a < np; ++a) {
      const int ai = a % P1, aj = (a / P1) % P1, ak = a / (P1 * P1);
      for (int b = 0; b < np; ++b) {
        const int bi = b % P1, bj = (b / P1) % P1, bk = b / (P1 * P1);
        const double kk = ke[ai * P1 + bi] * me[aj * P1 + bj] * me[ak * P1 + bk] +
                          me[ai * P1 + bi] * ke[aj * P1 + bj] * me[ak * P1 + bk] +
                          me[ai * P1 + bi] * me[aj * P1 + bj] * ke[ak * P1 + bk];
        const double wa = we[ai] * we[aj] * we[ak], wb = we[bi] * we[bj] * we[bk];
        A[(size_t)a * np + b] = kk / std::sqrt(wa * wb);
      }
    }
    double lmax;
    if (p <= 5) {
      lmax = max_eig_sym(np, A.data());
    } else {  // Gershgorin: rigorous, looser
      lmax = 0.0;
      for (int a = 0; a < np; ++a) {
        double r = 0.0;
        for (int b = 0; b < np; ++b) r += std::fabs(A[(size_t)a * np + b]);
        lmax = std::max(lmax, r);
      }
    }
    m.kin_bound = 0.5 * lmax;
  }
  hipError_t e = hipGetDevice(&m.device);
  if (e == hipSuccess) e = hipMalloc(&m.d_x1, n1 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_w1, n1 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_kd1, n1 * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_md1, n1 * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(m.d_x1, m.x1.data(), n1 * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m.d_w1, m.w1.data(), n1 * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m.d_kd1, m.kd1.data(), n1 * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m.d_md1, m.md1.data(), n1 * sizeof(double), hipMemcpyHostToDevice);
  if (m.graded) {
    // per cell: (h/h_e)^2 and the end-node W1^{-1/2} factors relative to the uniform tables,
    // whose end nodes carry the weight of two cells of width h_e: sqrt(2 h_e / (h_e + h_nb))
    std::vector<double> kap(n), gl(n), gr(n);
    for (int c = 0; c < n; ++c) {
      const double hc = m.cell_h[c];
      kap[c] = (m.h / hc) * (m.h / hc);
      gl[c] = c > 0 ? std::sqrt(2.0 * hc / (hc + m.cell_h[c - 1])) : 1.0;
      gr[c] = c + 1 < n ? std::sqrt(2.0 * hc / (hc + m.cell_h[c + 1])) : 1.0;
    }
    if (e == hipSuccess) e = hipMalloc(&m.d_ckap, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&m.d_cgl, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&m.d_cgr, n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(m.d_ckap, kap.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m.d_cgl, gl.data(), n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m.d_cgr, gr.data(), n * sizeof(double), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    fe_mesh_destroy(h);
    return e == hipErrorOutOfMemory ? fail(FE_ENOMEM, "fe_mesh_create: device allocation failed")
                                    : hip_fail(e, "fe_mesh_create");
  }
  *out = h;
  return FE_OK;
}

fe_status fe_mesh_create(int p, int n, double L, fe_mesh* out) { return mesh_create_impl(p, n, L, nullptr, out); }

fe_status fe_mesh_create_graded(int p, int n, const double* breaks_h, fe_mesh* out) {
  if (!breaks_h) return fail(FE_EINVAL, "fe_mesh_create_graded: breaks_h is NULL");
  return mesh_create_impl(p, n, 0.0, breaks_h, out);
}

fe_status fe_mesh_create_mapped(int p, int n, double L, double amp, fe_mesh* out) {
  if (!out) return fail(FE_EINVAL, "fe_mesh_create_mapped: out is NULL");
  *out = nullptr;
  if (p < 1 || p > 5) return fail(FE_EINVAL, "fe_mesh_create_mapped: p must be in [1, 5]");
  if (!std::isfinite(amp) || std::fabs(amp) >= 1.0)
    return fail(FE_EINVAL, "fe_mesh_create_mapped: amp must satisfy |amp| < 1");
  if (n >= 1 && (long long)n * n * n > (1LL << 31) / 64)
    return fail(FE_EINVAL, "fe_mesh_create_mapped: too many cells");
  fe_mesh h = nullptr;
  fe_status st = mesh_create_impl(p, n, L, nullptr, &h);
  if (st != FE_OK) return st;
  Mesh& m = h->m;
  m.mapped = true;
  m.amp = amp;
  st = mapped_setup(m, amp);
  if (st != FE_OK) {
    const std::string msg = fe_last_error();
    fe_mesh_destroy(h);
    return fail(st, msg);
  }
  *out = h;
  return FE_OK;
}

fe_status fe_mesh_info(fe_mesh mesh, int64_t* n_free_h, int64_t* n_cells_h, int* nodes_per_cell_h,
                       double* kin_bound_h) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  const Mesh& m = mesh->m;
  if (n_free_h) *n_free_h = m.nf;
  if (n_cells_h) *n_cells_h = (int64_t)m.n * m.n * m.n;
  if (nodes_per_cell_h) *nodes_per_cell_h = (m.p + 1) * (m.p + 1) * (m.p + 1);
  if (kin_bound_h) *kin_bound_h = m.kin_bound;
  return FE_OK;
}

fe_status fe_mesh_nodes(fe_mesh mesh, double* xyz, double* w, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  if (!xyz && !w) return FE_OK;
  return k_nodes(mesh->m, xyz, w, S(stream));
}

fe_status fe_mesh_kinetic_diag(fe_mesh mesh, double* d, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  if (!d) return fail(FE_EINVAL, "fe_mesh_kinetic_diag: d is NULL");
  return k_kdiag(mesh->m, d, S(stream));
}

fe_status fe_mesh_destroy(fe_mesh mesh) {
  if (!mesh) return FE_OK;
  Mesh& m = mesh->m;
  if (m.d_x1) (void)hipFree(m.d_x1);
  if (m.d_w1) (void)hipFree(m.d_w1);
  if (m.d_kd1) (void)hipFree(m.d_kd1);
  if (m.d_md1) (void)hipFree(m.d_md1);
  if (m.d_ckap) (void)hipFree(m.d_ckap);
  if (m.d_cgl) (void)hipFree(m.d_cgl);
  if (m.d_cgr) (void)hipFree(m.d_cgr);
  if (m.d_wn) (void)hipFree(m.d_wn);
  if (m.d_kdn) (void)hipFree(m.d_kdn);
  if (m.d_xyz) (void)hipFree(m.d_xyz);
  if (m.d_Ke64) (void)hipFree(m.d_Ke64);
  if (m.d_Ke32) (void)hipFree(m.d_Ke32);
  delete mesh;
  return FE_OK;
}

size_t fe_workspace_bytes(fe_mesh mesh, int op, int nv, fe_prec prec) {
  if (!mesh || nv < 1) return 0;
  const Mesh& m = mesh->m;
  Bump bp(nullptr);
  switch (op) {
    case FE_OP_KS_APPLY: return 0;
    case FE_OP_CHEB_FILTER: return filter_work(m, nv, prec);
    case FE_OP_RAYLEIGH_RITZ: rr_layout(bp, m, nv, nv); return bp.off;
    case FE_OP_EIGENSOLVE: eig_layout(bp, m, nv, nv, prec); return bp.off;
    case FE_OP_ADJOINT_SOLVE: adjoint_layout(bp, m, nv, prec); return bp.off;
    case FE_OP_ADJOINT_DEFLATED: {  // nv = nocc + nbuf: a bound for every split of nv
      if (nv > 128) return 0;
      const int k = std::min(nv, 64);
      double *u, *pw;
      mr_layout(bp, m, k, FE_F64);
      defl_layout(bp, m, k, k, &u, &pw);   // U: min(nv, 64) columns; V: min(nv, 64) or more
      return bp.off;
    }
    case FE_OP_LOSS_GRAD:
      bp.take<double>(m.nf);
      bp.take<char>(loss_grad_scratch_bytes(m.nf, nv));
      return bp.off;
    case FE_OP_ALONG_PSI: return along_psi_work_bytes(m.nf, nv);
    case FE_OP_POISSON: return poisson_work_bytes(m.nf);
    default: return 0;
  }
}

fe_status ks_apply(fe_mesh mesh, const double* v, const double* shift_h, const void* X, void* Y, int nv, int ld,
                   fe_prec prec, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  fe_status st;
  if ((st = check_block(X, "X", nv, ld)) != FE_OK) return st;
  if ((st = check_block(Y, "Y", nv, ld)) != FE_OK) return st;
  if (!v) return fail(FE_EINVAL, "ks_apply: v is NULL");
  if (X == Y) return fail(FE_EINVAL, "ks_apply: Y must not alias X");
  if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16) return fail(FE_EINVAL, "ks_apply: unsupported precision");
  ApplyArgs aa{};
  aa.X = X;
  aa.Y = Y;
  aa.v = v;
  aa.nv = nv;
  aa.ld = ld;
  aa.alpha = 1.0;
  aa.colshift = shift_h;
  return launch_apply(mesh->m, aa, prec, S(stream));
}

fe_status cheb_filter(fe_mesh mesh, const double* v, int degree, double a, double b, double a0, void* X, int nv,
                      int ld, fe_prec prec, void* work, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  fe_status st;
  if ((st = check_block(X, "X", nv, ld)) != FE_OK) return st;
  if (!v) return fail(FE_EINVAL, "cheb_filter: v is NULL");
  if (!work) return fail(FE_EINVAL, "cheb_filter: work is NULL");
  if (degree < 1) return fail(FE_EINVAL, "cheb_filter: degree must be >= 1");
  if (!(a < b) || !(a0 < a)) return fail(FE_EINVAL, "cheb_filter: need a0 < a < b");
  if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16)
    return fail(FE_EINVAL, "cheb_filter: unsupported precision");
  return filter_impl(mesh->m, v, degree, a, b, a0, X, nv, ld, prec, work, S(stream));
}

fe_status rayleigh_ritz(fe_mesh mesh, const double* v, double* X, double* eig_h, double* resnorm_h, int nv, int ld,
                        void* work, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  fe_status st;
  if ((st = check_block(X, "X", nv, ld)) != FE_OK) return st;
  if (!v || !work || !eig_h) return fail(FE_EINVAL, "rayleigh_ritz: v, work and eig_h are required");
  return rr_impl(mesh->m, v, X, eig_h, resnorm_h, nv, ld, work, S(stream));
}

fe_status ks_eigensolve(fe_mesh mesh, const double* v, double* X, int nv, int ld, int nocc, int degree, double tol,
                        int maxpass, fe_prec prec, double switch_tol, double* eig_h, double* resnorm_h,
                        int* passes_h, int* stage_passes_h, void* work, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  fe_status st;
  if ((st = check_block(X, "X", nv, ld)) != FE_OK) return st;
  if (!v || !work || !eig_h || !resnorm_h) return fail(FE_EINVAL, "ks_eigensolve: v, work, eig_h, resnorm_h required");
  if (nocc < 1 || nocc >= nv) return fail(FE_EINVAL, "ks_eigensolve: need 1 <= nocc < nv");
  if (degree < 1 || maxpass < 0) return fail(FE_EINVAL, "ks_eigensolve: degree >= 1 and maxpass >= 0 required");
  if (prec != FE_F64 && prec != FE_F32 && prec != FE_BF16)
    return fail(FE_EINVAL, "ks_eigensolve: unsupported precision");
  const Mesh& m = mesh->m;
  if (prec == FE_BF16 && m.mapped) return fail(FE_EINVAL, "ks_eigensolve: FE_BF16 needs a uniform or graded mesh");
  hipStream_t s = S(stream);
  Bump bp(work);
  EigWork w = eig_layout(bp, m, nv, ld, prec);
  if ((st = max1(v, m.nf, w.vmax, w.redw, s)) != FE_OK) return st;
  double vmax = 0.0;
  INVDFT_HIP(hipMemcpyAsync(&vmax, w.vmax, sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  const double b = m.kin_bound + vmax;
  if ((st = rr_impl(m, v, X, eig_h, resnorm_h, nv, ld, w.rr, s)) != FE_OK) return st;
  int pass = 0;
  int stage_passes[3] = {0, 0, 0};   // FP64, FP32, bf16 passes
  bool conv = false;
  // Reduced-precision filter passes until the residual is below switch_tol or stops improving
  // (its rounding floor), then FP64 passes. FE_BF16 starts one stage lower: bf16 passes until
  // they stop halving the residual (or it is below switch_tol), then FP32 as above.
  fe_prec stage = prec;
  double rprev = 1e300;
  for (;;) {
    double rmax = 0.0;
    for (int i = 0; i < nocc; ++i) rmax = std::max(rmax, resnorm_h[i]);
    if (rmax <= tol) {
      conv = true;
      break;
    }
    if (pass >= maxpass) break;
    const double a = eig_h[nv - 1], a0 = eig_h[0];
    if (!(a < b) || !(a0 < a)) return fail(FE_EINVAL, "ks_eigensolve: degenerate filter interval");
    if (stage == FE_BF16 && (rmax <= switch_tol || rmax > 0.5 * rprev)) {
      stage = FE_F32;
      rprev = 1e300;     // the FP32 stage judges its own progress
    }
    if (stage == FE_F32 && (rmax <= switch_tol || rmax > 0.5 * rprev)) stage = FE_F64;
    const bool low = stage != FE_F64;
    rprev = rmax;
    // Locking: the leading Ritz pairs that already meet tol are not filtered again (rounded
    // down to a multiple of 8 columns, so that the filtered sub-block keeps 16-byte aligned
    // rows in both precisions). Rayleigh-Ritz still runs over the whole block, so a locked
    // pair that drifts above tol is filtered again on the next pass. A reduced-precision
    // pass also leaves alone the pairs already below switch_tol: it could not improve them,
    // only round them to its own level.
    const double lock_tol = low ? std::max(tol, switch_tol) : tol;
    int j0 = 0;
    while (j0 < nocc && resnorm_h[j0] <= lock_tol) ++j0;
    j0 &= ~7;
    const int nfilt = nv - j0;
    if (stage == FE_BF16) {
      bf16_t* Xb = reinterpret_cast<bf16_t*>(w.Xf);
      if ((st = cast_block_to_bf16(X, Xb, (int64_t)m.nf * ld, s)) != FE_OK) return st;
      if ((st = filter_impl(m, v, degree, a, b, a0, Xb + j0, nfilt, ld, FE_BF16,
                            static_cast<bf16_t*>(static_cast<void*>(w.filt)) + j0, s)) != FE_OK)
        return st;
      if ((st = cast_cols_bf16_to_f64(Xb, X, m.nf, ld, j0, s)) != FE_OK) return st;
    } else if (low) {
      if ((st = cast_block_to_f32(X, w.Xf, (int64_t)m.nf * ld, s)) != FE_OK) return st;
      if ((st = filter_impl(m, v, degree, a, b, a0, w.Xf + j0, nfilt, ld, FE_F32,
                            static_cast<float*>(static_cast<void*>(w.filt)) + j0, s)) != FE_OK)
        return st;
      if (j0 == 0) {
        if ((st = cast_block_to_f64(w.Xf, X, (int64_t)m.nf * ld, s)) != FE_OK) return st;
      } else if ((st = cast_cols_to_f64(w.Xf, X, m.nf, ld, j0, s)) != FE_OK) {
        return st;
      }
    } else {
      if ((st = filter_impl(m, v, degree, a, b, a0, X + j0, nfilt, ld, FE_F64,
                            static_cast<double*>(static_cast<void*>(w.filt)) + j0, s)) != FE_OK)
        return st;
    }
    if ((st = rr_impl(m, v, X, eig_h, resnorm_h, nv, ld, w.rr, s)) != FE_OK) return st;
    ++pass;
    ++stage_passes[stage == FE_F64 ? 0 : stage == FE_F32 ? 1 : 2];
  }
  if (passes_h) *passes_h = pass;
  if (stage_passes_h) {
    stage_passes_h[0] = stage_passes[2];
    stage_passes_h[1] = stage_passes[1];
    stage_passes_h[2] = stage_passes[0];
  }
  if (!conv) return fail(FE_ENOCONV, "ks_eigensolve: residual tolerance not reached in maxpass passes");
  if (eig_h[nocc] - eig_h[nocc - 1] < 1e-6) return fail(FE_EGAP, "ks_eigensolve: no gap at the Fermi level");
  return FE_OK;
}

fe_status loss_grad(fe_mesh mesh, const double* Psi, const double* occ_h, int nocc, const double* rho_data,
                    const double* Q, double tau_bc, double* rho, double* B, double* grad, double* loss_h, void* work,
                    void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  if (!Psi || !occ_h) return fail(FE_EINVAL, "loss_grad: Psi and occ_h are required");
  if (nocc < 1 || nocc > kMaxShiftCols) return fail(FE_EINVAL, "loss_grad: nocc must be in [1, 256]");
  const Mesh& m = mesh->m;
  const bool needs_work = !Q || (loss_h && rho && rho_data);
  if (needs_work && !work) return fail(FE_EINVAL, "loss_grad: work is NULL");
  // work layout: the density buffer (used when rho is NULL), then the scratch
  Bump bp(work);
  double* rho_w = bp.take<double>(m.nf);
  void* scratch = bp.take<char>(loss_grad_scratch_bytes(m.nf, nocc));
  return loss_grad_impl(m, Psi, occ_h, nocc, rho_data, Q, tau_bc, rho, B, grad, loss_h, work ? rho_w : nullptr,
                        work ? scratch : nullptr, "loss_grad", S(stream));
}

// The FP64 solve and its true residual; reports per-column counts and relative residuals.
// MINRES stops on its residual estimate in the preconditioner's norm; the result is held to
// the Euclidean bar ||b - A q|| <= 2 tol ||b|| on every column: columns above it are refined
// (at most three rounds). maxit bounds the whole solve: the first solve and the refinement
// rounds draw on one budget, counted in iterations of the slowest column.
fe_status adjoint_f64(const Mesh& m, const double* v, const ProjSet<double>& ps, const double* eps_h, int k,
                      const double* B, double* Q, double tol, int maxit, int* iters_h, double* relres_h, MRWork& w,
                      Deflation* df, const char* name, hipStream_t s) {
  fe_status st;
  std::vector<double> its, active, rr(k), bb(k);
  bool conv = true;
  // deflated: a tighter stop test for the first solve, since its residual norm weighs the
  // deflated directions by 1 / (theta - eps) and so understates the Euclidean one (by 6 to 17
  // times on the model molecules); refinement below covers what this factor misses
  const double tol1 = df ? tol / 6.0 : tol;
  if ((st = minres_core<double>(m, v, ps, eps_h, k, B, Q, tol1, maxit, w, its, active, s, df)) != FE_OK) return st;
  int used = 0;
  for (int j = 0; j < k; ++j) {
    if (active[j] > 0.0) conv = false;
    used = std::max(used, (int)its[j]);
  }
  if ((st = true_residual(m, v, ps.Psi, ps.kpsi, eps_h, k, B, Q, w.rb, w.d1, w.pw, s)) != FE_OK) return st;
  if ((st = coldot(B, B, k, m.nf, k, false, w.bnorm, w.pw, s)) != FE_OK) return st;
  INVDFT_HIP(hipMemcpyAsync(rr.data(), w.d1, k * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipMemcpyAsync(bb.data(), w.bnorm, k * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  auto above = [&](int j) { return rr[j] > 4.0 * tol * tol * bb[j]; };
  // Refinement: solve (H - eps) d = r for the true residual r of the columns above 2 tol, to
  // half of what the worst of them still needs, and add d.
  for (int round = 0; conv && round < 3; ++round) {
    double need = 1e300;
    std::vector<double> mask((size_t)k * k, 0.0);  // diag(1 for the columns still above 2 tol)
    for (int j = 0; j < k; ++j)
      if (above(j)) {
        need = std::min(need, std::sqrt(bb[j] / rr[j]));
        mask[(size_t)j * k + j] = 1.0;
      }
    if (need == 1e300) break;
    if (used >= maxit) break;
    // the other columns get a zero right-hand side: inactive from the start, soon compacted away
    INVDFT_HIP(hipMemcpyAsync(w.mask, mask.data(), mask.size() * sizeof(double), hipMemcpyHostToDevice, s));
    if ((st = rotate(w.rb, k, m.nf, k, w.mask, k, w.rb, k, s)) != FE_OK) return st;
    const double tol2 = std::min(0.5, std::max(1e-14, 0.5 * tol * need));
    std::vector<double> its2, act2;
    if ((st = minres_core<double>(m, v, ps, eps_h, k, w.rb, w.dq, tol2, maxit - used, w, its2, act2, s, df)) !=
        FE_OK)
      return st;
    int mx = 0;
    for (int j = 0; j < k; ++j) {
      its[j] += its2[j];
      mx = std::max(mx, (int)its2[j]);
      if (act2[j] > 0.0) conv = false;
    }
    used += mx;
    if ((st = axpby(1.0, w.dq, 1.0, Q, (int64_t)m.nf * k, s)) != FE_OK) return st;
    if ((st = true_residual(m, v, ps.Psi, ps.kpsi, eps_h, k, B, Q, w.rb, w.d1, w.pw, s)) != FE_OK) return st;
    INVDFT_HIP(hipMemcpyAsync(rr.data(), w.d1, k * sizeof(double), hipMemcpyDeviceToHost, s));
    INVDFT_HIP(hipStreamSynchronize(s));
  }
  for (int j = 0; j < k; ++j) {
    if (iters_h) iters_h[j] = (int)its[j];
    if (relres_h) relres_h[j] = bb[j] > 0 ? std::sqrt(std::max(rr[j], 0.0) / bb[j]) : 0.0;
    if (above(j)) conv = false;
  }
  if (!conv) {
    std::string msg = std::string(name) + ": some columns did not reach tol (Euclidean residual) in maxit iterations";
    return fail(FE_ENOCONV, msg.c_str());
  }
  return FE_OK;
}

fe_status adjoint_solve_deflated(fe_mesh mesh, const double* v, const double* Psi, const double* eps_h, int nocc,
                                 const double* U, const double* theta_h, int nbuf, const double* B, double* Q,
                                 double tol, int maxit, int* iters_h, double* relres_h, void* work, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  if (!v || !Psi || !eps_h || !U || !theta_h || !B || !Q || !work)
    return fail(FE_EINVAL, "adjoint_solve_deflated: NULL argument");
  if (!aligned16(Psi) || !aligned16(U) || !aligned16(B) || !aligned16(Q) || !aligned16(work))
    return fail(FE_EINVAL, "adjoint_solve_deflated: Psi, U, B, Q and work must be 16-byte aligned");
  if (nocc < 1 || nocc > 64 || nbuf < 1 || nbuf > 64)
    return fail(FE_EINVAL, "adjoint_solve_deflated: 1 <= nocc <= 64 and 1 <= nbuf <= 64 required");
  if (!(tol > 0.0) || maxit < 1) return fail(FE_EINVAL, "adjoint_solve_deflated: tol > 0 and maxit >= 1 required");
  double emax = -INFINITY;
  for (int i = 0; i < nocc; ++i) {
    if (!std::isfinite(eps_h[i])) return fail(FE_EINVAL, "adjoint_solve_deflated: shifts must be finite");
    emax = std::max(emax, eps_h[i]);
  }
  for (int j = 0; j < nbuf; ++j)  // also refuses NaN
    if (!(theta_h[j] > emax) || !std::isfinite(theta_h[j]))
      return fail(FE_EINVAL, "adjoint_solve_deflated: every theta must lie above every shift");
  const Mesh& m = mesh->m;
  hipStream_t s = S(stream);
  Bump bp(work);
  MRWork w = mr_layout(bp, m, nocc, FE_F64);
  double *Uc, *pw;
  Deflation df = defl_layout(bp, m, nocc, nbuf, &Uc, &pw);
  w.pw = pw;
  fe_status st;
  if ((st = k_dinv(m, w.dinv, s)) != FE_OK) return st;
  // U with Psi projected out (twice: the Ritz vectors are orthogonal to Psi only to rounding)
  if ((st = copy_bytes(U, Uc, (size_t)m.nf * nbuf * sizeof(double), s)) != FE_OK) return st;
  for (int pass = 0; pass < 2; ++pass)
    if ((st = project_out(Psi, nocc, Uc, nbuf, m.nf, false, w.pw, s)) != FE_OK) return st;
  if ((st = defl_pack(Psi, nocc, Uc, nbuf, df.nbf, df.V, m.nf, s)) != FE_OK) return st;
  INVDFT_HIP(hipMemcpyAsync(df.theta, theta_h, nbuf * sizeof(double), hipMemcpyHostToDevice, s));
  return adjoint_f64(m, v, proj_whole(Psi, nocc), eps_h, nocc, B, Q, tol, maxit, iters_h, relres_h, w, &df,
                     "adjoint_solve_deflated", s);
}

fe_status adjoint_solve(fe_mesh mesh, const double* v, const double* Psi, const double* eps_h, int nocc,
                        const double* B, double* Q, double tol, int maxit, int* iters_h, double* relres_h, fe_prec prec,
                        void* work, void* stream) {
  if (check_mesh(mesh) != FE_OK) return FE_EINVAL;
  if (!v || !Psi || !eps_h || !B || !Q || !work) return fail(FE_EINVAL, "adjoint_solve: NULL argument");
  if (!aligned16(Psi) || !aligned16(B) || !aligned16(Q) || !aligned16(work))
    return fail(FE_EINVAL, "adjoint_solve: Psi, B, Q and work must be 16-byte aligned");
  if (nocc < 1 || nocc > kMaxShiftCols) return fail(FE_EINVAL, "adjoint_solve: nocc must be in [1, 256]");
  if (!(tol > 0.0) || maxit < 1) return fail(FE_EINVAL, "adjoint_solve: tol > 0 and maxit >= 1 required");
  if (prec != FE_F64 && prec != FE_F32) return fail(FE_EINVAL, "adjoint_solve: unsupported precision");
  if (prec == FE_F32 && nocc > 64) return fail(FE_EINVAL, "adjoint_solve: FE_F32 takes at most 64 orbitals");
  const Mesh& m = mesh->m;
  hipStream_t s = S(stream);
  Bump bp(work);
  MRWork w = adjoint_layout(bp, m, nocc, prec);
  const int k = nocc;
  const size_t blk = (size_t)m.nf * k;
  fe_status st;
  if ((st = k_dinv(m, w.dinv, s)) != FE_OK) return st;
  std::vector<double> its, active, total_its(k, 0.0), rr(k), bb(k);
  bool conv = true;
  if (prec == FE_F64 && k <= 64) {
    return adjoint_f64(m, v, proj_whole(Psi, k), eps_h, k, B, Q, tol, maxit, iters_h, relres_h, w, nullptr,
                       "adjoint_solve", s);
  } else if (prec == FE_F64) {
    // More than 64 orbitals: the shifts in groups of at most 64 columns, each solved against all
    // of Psi. The fused passes take the first 64 orbitals (a block of their own, 64-column rows);
    // the others are projected by separate sweeps.
    const size_t es = sizeof(double);
    INVDFT_HIP(hipMemcpy2DAsync(w.Pf, 64 * es, Psi, k * es, 64 * es, m.nf, hipMemcpyDeviceToDevice, s));
    const ProjSet<double> ps{Psi, k, w.Pf, 64, Psi + 64, k - 64};
    std::string nc_msg;
    for (int c0 = 0; c0 < k; c0 += 64) {
      const int kc = std::min(64, k - c0);
      INVDFT_HIP(hipMemcpy2DAsync(w.Bg, kc * es, B + c0, k * es, kc * es, m.nf, hipMemcpyDeviceToDevice, s));
      st = adjoint_f64(m, v, ps, eps_h + c0, kc, w.Bg, w.Qg, tol, maxit, iters_h ? iters_h + c0 : nullptr,
                       relres_h ? relres_h + c0 : nullptr, w, nullptr, "adjoint_solve", s);
      if (st == FE_ENOCONV && nc_msg.empty()) nc_msg = g_err;
      if (st != FE_OK && st != FE_ENOCONV) return st;
      INVDFT_HIP(hipMemcpy2DAsync(Q + c0, k * es, w.Qg, kc * es, kc * es, m.nf, hipMemcpyDeviceToDevice, s));
    }
    INVDFT_HIP(hipStreamSynchronize(s));
    return nc_msg.empty() ? FE_OK : fail(FE_ENOCONV, nc_msg);
  } else {
    // FP32 MINRES inner solves with FP64 iterative refinement: q += d, (H - eps) d = r in FP32,
    // r = b - (H - eps) q in FP64, until every column reaches tol.
    const double tol_inner = std::max(tol, 1e-4);
    if ((st = cast_block_to_f32(Psi, w.Psif, blk, s)) != FE_OK) return st;
    if ((st = fill(Q, 0.0, blk, s)) != FE_OK) return st;
    if ((st = copy_bytes(B, w.R64, blk * sizeof(double), s)) != FE_OK) return st;
    if ((st = coldot(B, B, k, m.nf, k, false, w.bnorm, w.pw, s)) != FE_OK) return st;
    INVDFT_HIP(hipMemcpyAsync(bb.data(), w.bnorm, k * sizeof(double), hipMemcpyDeviceToHost, s));
    if ((st = copy_bytes(w.bnorm, w.d1, k * sizeof(double), s)) != FE_OK) return st;  // r = b at q = 0
    INVDFT_HIP(hipStreamSynchronize(s));
    rr = bb;
    int used = 0;
    const int max_outer = 20;
    conv = false;
    for (int outer = 0; outer < max_outer && used < maxit; ++outer) {
      bool done = true;
      for (int j = 0; j < k; ++j)
        if (rr[j] > tol * tol * bb[j]) done = false;
      if (done) {
        conv = true;
        break;
      }
      float* Rf = static_cast<float*>(w.X);  // right-hand side of the inner solve
      if ((st = cast_block_to_f32(w.R64, Rf, blk, s)) != FE_OK) return st;
      if ((st = k_mask_cols(Rf, w.d1, w.bnorm, tol, k, m.nf, s)) != FE_OK) return st;
      // the FP32 correction is stored in the (larger) FP64 scratch block Y64
      float* Dsol = reinterpret_cast<float*>(w.Y64);
      if ((st = minres_core<float>(m, v, proj_whole<float>(w.Psif, k), eps_h, k, Rf, Dsol, tol_inner, maxit - used, w,
                                   its, active, s)) != FE_OK)
        return st;
      int mx = 0;
      for (int j = 0; j < k; ++j) {
        total_its[j] += its[j];
        mx = std::max(mx, (int)its[j]);
      }
      used += std::max(mx, 1);
      if ((st = k_add_f32(Dsol, Q, blk, s)) != FE_OK) return st;
      if ((st = project_out(Psi, k, Q, k, m.nf, false, w.pw, s)) != FE_OK) return st;
      if ((st = true_residual(m, v, Psi, k, eps_h, k, B, Q, w.R64, w.d1, w.pw, s)) != FE_OK) return st;
      INVDFT_HIP(hipMemcpyAsync(rr.data(), w.d1, k * sizeof(double), hipMemcpyDeviceToHost, s));
      INVDFT_HIP(hipStreamSynchronize(s));
    }
    if (!conv) {
      bool done = true;
      for (int j = 0; j < k; ++j)
        if (rr[j] > tol * tol * bb[j]) done = false;
      conv = done;
    }
    if ((st = coldot(B, B, k, m.nf, k, false, w.bnorm, w.pw, s)) != FE_OK) return st;
  }
  INVDFT_HIP(hipMemcpyAsync(rr.data(), w.d1, k * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipMemcpyAsync(bb.data(), w.bnorm, k * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    if (iters_h) iters_h[j] = (int)total_its[j];
    if (relres_h) relres_h[j] = bb[j] > 0 ? std::sqrt(std::max(rr[j], 0.0) / bb[j]) : 0.0;
  }
  if (!conv) return fail(FE_ENOCONV, "adjoint_solve: some columns did not converge in maxit iterations");
  return FE_OK;
}

fe_status fe_dot(const double* x, const double* y, int64_t n, double* out_h, void* work, void* stream) {
  if (!x || !y || !out_h || !work || n < 0) return fail(FE_EINVAL, "fe_dot: bad argument");
  hipStream_t s = S(stream);
  double* w = static_cast<double*>(work);
  fe_status st = dot1(x, y, n, w + 1024, w, s);
  if (st != FE_OK) return st;
  INVDFT_HIP(hipMemcpyAsync(out_h, w + 1024, sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  return FE_OK;
}

fe_status fe_axpby(double alpha, const double* x, double beta, double* y, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && (!x || !y))) return fail(FE_EINVAL, "fe_axpby: bad argument");
  return axpby(alpha, x, beta, y, n, S(stream));
}

fe_status fe_apply_timing(int enable) { return apply_timing(enable); }

fe_status fe_apply_timing_read(fe_prec prec, int64_t* launches, double* ms, double* bytes, double* columns) {
  return apply_timing_read(prec, launches, ms, bytes, columns);
}

fe_status fe_sweep_timing_read(int pass, int64_t* launches, double* ms, double* bytes, double* columns) {
  return sweep_timing_read(pass, launches, ms, bytes, columns);
}

}  // extern "C"
