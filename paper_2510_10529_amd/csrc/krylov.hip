// Density, loss, adjoint right-hand side, gradient (Eqs. 1, 4, 7, 10, 11, 22)
// and the vector/scalar kernels of the batched projected MINRES adjoint solve
// (Sec. 3.2.2; Paige and Saunders 1975). Blocks are node-major, one column per
// occupied orbital; all per-column MINRES scalars live on the device, so an
// iteration makes no host round trip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "krylov.h"

namespace invdft {

namespace {

unsigned grid_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 16384)); }

__device__ __forceinline__ void node_xyz(long long a, int n1, int* ix, int* iy, int* iz) {
  const long long n1l = n1;
  *ix = (int)(a % n1l);
  const long long r = a / n1l;
  *iy = (int)(r % n1l);
  *iz = (int)(r / n1l);
}

// wn, xyzn: per-node tables of a mapped mesh (NULL: products of the 1-D tables)
__global__ void nodes_kernel(const double* __restrict__ x1, const double* __restrict__ w1, const double* __restrict__ wn,
                             const double* __restrict__ xyzn, int n1, long long nf, double* __restrict__ xyz,
                             double* __restrict__ w) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    node_xyz(a, n1, &ix, &iy, &iz);
    if (xyz) {
      xyz[3 * a + 0] = xyzn ? xyzn[3 * a + 0] : x1[ix];
      xyz[3 * a + 1] = xyzn ? xyzn[3 * a + 1] : x1[iy];
      xyz[3 * a + 2] = xyzn ? xyzn[3 * a + 2] : x1[iz];
    }
    if (w) w[a] = wn ? wn[a] : w1[ix] * w1[iy] * w1[iz];
  }
}

// diag(K~/2)_a = (kd(x) md(y) md(z) + md(x) kd(y) md(z) + md(x) md(y) kd(z)) / 2
// (kdn: the per-node diagonal of a mapped mesh, or NULL)
__global__ void kdiag_kernel(const double* __restrict__ kd1, const double* __restrict__ md1,
                             const double* __restrict__ kdn, int n1, long long nf, double* __restrict__ d) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    node_xyz(a, n1, &ix, &iy, &iz);
    d[a] = kdn ? kdn[a]
               : 0.5 * (kd1[ix] * md1[iy] * md1[iz] + md1[ix] * kd1[iy] * md1[iz] + md1[ix] * md1[iy] * kd1[iz]);
  }
}

struct Occ {
  double f[kMaxShiftCols];
};

// rho_a = sum_i f_i psi_{a,i}^2 / W_a   (Eq. 4)
__global__ void density_kernel(const double* __restrict__ Psi, int nocc, Occ occ, const double* __restrict__ w1,
                               const double* __restrict__ wn, int n1, long long nf, double* __restrict__ rho) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    node_xyz(a, n1, &ix, &iy, &iz);
    const double* row = Psi + a * nocc;
    double s = 0.0;
    for (int i = 0; i < nocc; ++i) s += occ.f[i] * row[i] * row[i];
    rho[a] = s / (wn ? wn[a] : w1[ix] * w1[iy] * w1[iz]);
  }
}

// partial sums of W_a (rho_data,a - rho_a)^2   (Eq. 1, w = 1)
__global__ void loss_partial_kernel(const double* __restrict__ rho, const double* __restrict__ rho_d,
                                    const double* __restrict__ w1, const double* __restrict__ wn, int n1,
                                    long long nf, long long per, double* __restrict__ partial) {
  __shared__ double red[256];
  const long long b0 = (long long)blockIdx.x * per;
  const long long b1 = min(nf, b0 + per);
  double s = 0.0;
  for (long long a = b0 + threadIdx.x; a < b1; a += 256) {
    int ix, iy, iz;
    node_xyz(a, n1, &ix, &iy, &iz);
    const double d = rho_d[a] - rho[a];
    s += (wn ? wn[a] : w1[ix] * w1[iy] * w1[iz]) * d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_serial_kernel(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += partial[b];
    *out = s;
  }
}

// R[a, i] = -4 f_i (rho_a - rho_data,a) psi_{a,i}   (the unprojected adjoint source, Eq. 7)
__global__ void rhs_kernel(const double* __restrict__ Psi, int nocc, Occ occ, const double* __restrict__ rho,
                           const double* __restrict__ rho_d, long long nf, double* __restrict__ R) {
  const long long total = nf * nocc;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long a = e / nocc;
    const int i = (int)(e % nocc);
    R[e] = -4.0 * occ.f[i] * (rho[a] - rho_d[a]) * Psi[e];
  }
}

// grad_b = sum_i psi_{b,i} q_{b,i}, zeroed where rho_data < tau   (Eqs. 11, 22; Sec. 3.1.2)
__global__ void grad_kernel(const double* __restrict__ Psi, const double* __restrict__ Q, int nocc,
                            const double* __restrict__ rho_d, double tau, long long nf, double* __restrict__ g) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nocc; ++i) s += Psi[a * nocc + i] * Q[a * nocc + i];
    if (tau > 0.0 && rho_d && rho_d[a] < tau) s = 0.0;
    g[a] = s;
  }
}

// ------------------------------------------------------------------ MINRES

template <typename T>
__global__ void mr_init_kernel(double* __restrict__ st, const double* __restrict__ dot_r_z, int k) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double* s = st;
  const double b1 = sqrt(fmax(dot_r_z[j], 0.0));
  s[S_BETA * k + j] = b1;
  s[S_BETA1 * k + j] = b1;
  s[S_OLDB * k + j] = 0.0;
  s[S_DBAR * k + j] = 0.0;
  s[S_EPSLN * k + j] = 0.0;
  s[S_PHIBAR * k + j] = b1;
  s[S_CS * k + j] = -1.0;
  s[S_SN * k + j] = 0.0;
  s[S_INVBETA * k + j] = b1 > 0.0 ? 1.0 / b1 : 0.0;
  s[S_INVBETA_OLD * k + j] = 0.0;
  s[S_ACTIVE * k + j] = b1 > 0.0 ? 1.0 : 0.0;
  s[S_ITERS * k + j] = 0.0;
  s[S_RELRES * k + j] = b1 > 0.0 ? 1.0 : 0.0;
  s[S_C1 * k + j] = 0.0;
  s[S_C2 * k + j] = 0.0;
  s[S_PHI * k + j] = 0.0;
}

// after the two dots d1 = z.y / beta (= v.y) and d2 = z.r1 / beta (= v.r1):
// alfa = v.(y - c1 r1) = d1 - c1 d2, c2 = alfa / beta
__global__ void mr_alfa_kernel(double* __restrict__ st, const double* __restrict__ d1, const double* __restrict__ d2,
                               int k, int first) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double* s = st;
  const double beta = s[S_BETA * k + j];
  const double ib = s[S_INVBETA * k + j];
  const double c1 = first ? 0.0 : beta / s[S_OLDB * k + j];
  const double alfa = ib * d1[j] - c1 * ib * d2[j];
  s[S_C1 * k + j] = (s[S_ACTIVE * k + j] > 0.0) ? c1 : 0.0;
  s[S_ALFA * k + j] = alfa;
  s[S_C2 * k + j] = (s[S_ACTIVE * k + j] > 0.0) ? alfa * ib : 0.0;
}

// Givens update after beta_new^2 = r2.z_new (Paige-Saunders recurrences).
__global__ void mr_givens_kernel(double* __restrict__ st, const double* __restrict__ dot_r_z, int k, double tol) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double* s = st;
  if (!(s[S_ACTIVE * k + j] > 0.0)) {
    s[S_PHI * k + j] = 0.0;
    s[S_INVGAMMA * k + j] = 0.0;
    s[S_OLDEPS * k + j] = 0.0;
    s[S_DELTA * k + j] = 0.0;
    s[S_INVBETA_OLD * k + j] = 0.0;
    return;
  }
  const double alfa = s[S_ALFA * k + j];
  const double oldb_new = s[S_BETA * k + j];
  const double beta = sqrt(fmax(dot_r_z[j], 0.0));
  const double cs = s[S_CS * k + j], sn = s[S_SN * k + j];
  const double dbar = s[S_DBAR * k + j];
  const double oldeps = s[S_EPSLN * k + j];
  const double delta = cs * dbar + sn * alfa;
  const double gbar = sn * dbar - cs * alfa;
  const double epsln = sn * beta;
  const double dbar_new = -cs * beta;
  double gamma = sqrt(gbar * gbar + beta * beta);
  gamma = fmax(gamma, 1e-300);
  const double cs_new = gbar / gamma, sn_new = beta / gamma;
  const double phibar = s[S_PHIBAR * k + j];
  const double phi = cs_new * phibar;
  const double phibar_new = sn_new * phibar;
  s[S_OLDB * k + j] = oldb_new;
  s[S_INVBETA_OLD * k + j] = s[S_INVBETA * k + j];
  s[S_BETA * k + j] = beta;
  s[S_INVBETA * k + j] = beta > 0.0 ? 1.0 / beta : 0.0;
  s[S_CS * k + j] = cs_new;
  s[S_SN * k + j] = sn_new;
  s[S_DBAR * k + j] = dbar_new;
  s[S_EPSLN * k + j] = epsln;
  s[S_OLDEPS * k + j] = oldeps;
  s[S_DELTA * k + j] = delta;
  s[S_INVGAMMA * k + j] = 1.0 / gamma;
  s[S_PHI * k + j] = phi;
  s[S_PHIBAR * k + j] = phibar_new;
  s[S_ITERS * k + j] += 1.0;
  const double rel = phibar_new / s[S_BETA1 * k + j];
  s[S_RELRES * k + j] = rel;
  if (rel <= tol || beta == 0.0) s[S_ACTIVE * k + j] = 0.0;
}




// ------------------------------------------------- deflated preconditioner
// M = P_ext D^{-1} P_ext + U diag(1 / (theta - eps_i)) U^T with V = [Psi U] orthonormal,
// P_ext = I - V V^T; the stored Lanczos vectors are r' = r - U c, c = U^T r (nb x k small
// arrays c[j k + i]); G blocks from the fused passes are (k0 + nb) x k row-major.

// V[a, 0..k0) = Psi[a, :], V[a, k0..k0+nb) = U[a, 0..nb) (U with row pitch ldu >= nb)
__global__ void defl_pack_kernel(const double* __restrict__ Psi, int k0, const double* __restrict__ U, int ldu,
                                 int nb, double* __restrict__ V, long long nf) {
  const int kp = k0 + nb;
  const long long total = nf * kp;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long a = e / kp;
    const int c = (int)(e % kp);
    V[e] = c < k0 ? Psi[a * k0 + c] : U[a * ldu + (c - k0)];
  }
}

// d2_i += sum_j cR1[j, i] cR2[j, i] / (theta_j - eps_i): z.r1 with r1 = r1' + U cR1 and U^T z = cR2 / (theta - eps)
__global__ void defl_d2_kernel(double* __restrict__ d2, const double* __restrict__ cR1, const double* __restrict__ cR2,
                               const double* __restrict__ theta, const double* __restrict__ eps, int k, int nb) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double t = 0.0;
    for (int j = 0; j < nb; ++j) t += cR1[j * k + i] * cR2[j * k + i] / (theta[j] - eps[i]);
    d2[i] += t;
  }
}

// c_new = U^T y - c1 cR1 - c2 cR2. U^T y: rows k0.. of G1 from pass A for the first nbf vectors
// (those inside the fused passes' block), the rows of Gr for the rest (nb - nbf of them).
__global__ void defl_cnew_kernel(const double* __restrict__ G1, int k0, int nbf, const double* __restrict__ Gr,
                                 int nb, const double* __restrict__ cR1, const double* __restrict__ cR2,
                                 const double* __restrict__ st, int k, double* __restrict__ cnew) {
  for (int e = threadIdx.x; e < nb * k; e += blockDim.x) {
    const int j = e / k, i = e % k;
    const double uy = j < nbf ? G1[(k0 + j) * k + i] : Gr[(j - nbf) * k + i];
    cnew[e] = uy - st[S_C1 * k + i] * cR1[e] - st[S_C2 * k + i] * cR2[e];
  }
}

// beta^2 = r'.D^{-1} r' + sum_j c_new^2 / (theta_j - eps_i); the U rows of G2 (and of Gr for the
// vectors past the fused block) lose c_new / (theta - eps), so that the update with them forms
// z = P_ext D^{-1} r' + U c_new / (theta - eps)
__global__ void defl_beta_g2_kernel(double* __restrict__ d, double* __restrict__ G2, int k0, int nbf,
                                    double* __restrict__ Gr, int nb, const double* __restrict__ cnew,
                                    const double* __restrict__ theta, const double* __restrict__ eps, int k) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    double t = 0.0;
    for (int j = 0; j < nb; ++j) {
      const double c = cnew[j * k + i];
      const double g = 1.0 / (theta[j] - eps[i]);
      t += c * c * g;
      if (j < nbf)
        G2[(k0 + j) * k + i] -= c * g;
      else
        Gr[(j - nbf) * k + i] -= c * g;
    }
    d[i] += t;
  }
}

// out[j, i] = c[j, i] / (theta_j - eps_i)
__global__ void defl_scale_kernel(const double* __restrict__ c, const double* __restrict__ theta,
                                  const double* __restrict__ eps, int k, int nb, double* __restrict__ out) {
  for (int e = threadIdx.x; e < nb * k; e += blockDim.x) {
    const int j = e / k, i = e % k;
    out[e] = c[e] / (theta[j] - eps[i]);
  }
}

__global__ void dinv_kernel(const double* __restrict__ kd1, const double* __restrict__ md1,
                            const double* __restrict__ kdn, int n1, long long nf, double* __restrict__ dinv) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    node_xyz(a, n1, &ix, &iy, &iz);
    const double d =
        kdn ? kdn[a] : 0.5 * (kd1[ix] * md1[iy] * md1[iz] + md1[ix] * kd1[iy] * md1[iz] + md1[ix] * md1[iy] * kd1[iz]);
    dinv[a] = 1.0 / d;
  }
}

// y = x / D row-wise (block)
template <typename T>
__global__ void precond_kernel(const T* __restrict__ x, const double* __restrict__ dinv, int k, long long nf,
                               T* __restrict__ y) {
  const long long total = nf * k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x)
    y[e] = (T)((double)x[e] * dinv[e / k]);
}

// dst[a, jn] = src[a, map[jn]] (dst has kn columns, src ko)
template <typename T>
__global__ void select_cols_kernel(const T* __restrict__ src, int ko, T* __restrict__ dst, int kn,
                                   const int* __restrict__ map, long long nf) {
  const long long total = nf * kn;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long a = e / kn;
    dst[e] = src[a * ko + map[e % kn]];
  }
}

// dst[a, map[jc]] = src[a, jc]  (scatter kc compact columns into a kf-wide block)
template <typename T>
__global__ void scatter_cols_kernel(const T* __restrict__ src, int kc, T* __restrict__ dst, int kf,
                                    const int* __restrict__ map, long long nf) {
  const long long total = nf * kc;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long a = e / kc;
    dst[a * kf + map[e % kc]] = src[e];
  }
}

// q += (double) d  (refinement update from the FP32 correction)
__global__ void add_f32_kernel(const float* __restrict__ d, double* __restrict__ q, long long total) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x)
    q[e] += (double)d[e];
}

// columns whose relative residual is at or below tol get a zero right-hand side (they stay frozen)
__global__ void mask_cols_kernel(float* __restrict__ r, const double* __restrict__ rr, const double* __restrict__ bb,
                                 double tol, int k, long long nf) {
  const long long total = nf * k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % k);
    if (rr[j] <= tol * tol * bb[j]) r[e] = 0.0f;
  }
}

// r = b - r (in place): residual from r = A q
__global__ void sub_from_kernel(const double* __restrict__ b, double* __restrict__ r, long long total) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x)
    r[e] = b[e] - r[e];
}

}  // namespace

fe_status k_nodes(const Mesh& m, double* xyz, double* w, hipStream_t s) {
  hipLaunchKernelGGL(nodes_kernel, dim3(grid_for(m.nf)), dim3(256), 0, s, m.d_x1, m.d_w1, m.d_wn, m.d_xyz, m.n1,
                     (long long)m.nf, xyz, w);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status k_kdiag(const Mesh& m, double* d, hipStream_t s) {
  hipLaunchKernelGGL(kdiag_kernel, dim3(grid_for(m.nf)), dim3(256), 0, s, m.d_kd1, m.d_md1, m.d_kdn, m.n1,
                     (long long)m.nf, d);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status k_dinv(const Mesh& m, double* dinv, hipStream_t s) {
  hipLaunchKernelGGL(dinv_kernel, dim3(grid_for(m.nf)), dim3(256), 0, s, m.d_kd1, m.d_md1, m.d_kdn, m.n1,
                     (long long)m.nf, dinv);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status k_density(const Mesh& m, const double* Psi, int nocc, const double* occ_h, double* rho, hipStream_t s) {
  Occ o{};
  for (int i = 0; i < nocc; ++i) o.f[i] = occ_h[i];
  hipLaunchKernelGGL(density_kernel, dim3(grid_for(m.nf)), dim3(256), 0, s, Psi, nocc, o, m.d_w1, m.d_wn, m.n1,
                     (long long)m.nf, rho);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

size_t loss_work_bytes() { return 1025 * sizeof(double); }

fe_status k_loss(const Mesh& m, const double* rho, const double* rho_d, double* out, void* work, hipStream_t s) {
  const int nblk = (int)std::max<long long>(1, std::min<long long>((m.nf + 4095) / 4096, 1024));
  const long long per = (m.nf + nblk - 1) / nblk;
  double* partial = static_cast<double*>(work);
  hipLaunchKernelGGL(loss_partial_kernel, dim3(nblk), dim3(256), 0, s, rho, rho_d, m.d_w1, m.d_wn, m.n1, (long long)m.nf,
                     per, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_serial_kernel, dim3(1), dim3(64), 0, s, partial, nblk, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status k_rhs(const Mesh& m, const double* Psi, int nocc, const double* occ_h, const double* rho,
                const double* rho_d, double* R, hipStream_t s) {
  Occ o{};
  for (int i = 0; i < nocc; ++i) o.f[i] = occ_h[i];
  hipLaunchKernelGGL(rhs_kernel, dim3(grid_for(m.nf * nocc)), dim3(256), 0, s, Psi, nocc, o, rho, rho_d,
                     (long long)m.nf, R);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status k_grad(const Mesh& m, const double* Psi, const double* Q, int nocc, const double* rho_d, double tau,
                 double* g, hipStream_t s) {
  hipLaunchKernelGGL(grad_kernel, dim3(grid_for(m.nf)), dim3(256), 0, s, Psi, Q, nocc, rho_d, tau, (long long)m.nf, g);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

// ----------------------------------------------------------------- MINRES
int mr_state_count() { return S_COUNT; }
int mr_state_iters() { return S_ITERS; }
int mr_state_active() { return S_ACTIVE; }
int mr_state_invbeta() { return S_INVBETA; }

fe_status defl_pack(const double* Psi, int k0, const double* U, int ldu, int nb, double* V, int64_t nf,
                    hipStream_t s) {
  hipLaunchKernelGGL(defl_pack_kernel, dim3(grid_for(nf * (k0 + nb))), dim3(256), 0, s, Psi, k0, U, ldu, nb, V,
                     (long long)nf);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status defl_d2(double* d2, const double* cR1, const double* cR2, const double* theta, const double* eps, int k,
                  int nb, hipStream_t s) {
  hipLaunchKernelGGL(defl_d2_kernel, dim3(1), dim3(64), 0, s, d2, cR1, cR2, theta, eps, k, nb);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status defl_cnew(const double* G1, int k0, int nbf, const double* Gr, int nb, const double* cR1, const double* cR2,
                    const double* st, int k, double* cnew, hipStream_t s) {
  hipLaunchKernelGGL(defl_cnew_kernel, dim3(1), dim3(256), 0, s, G1, k0, nbf, Gr, nb, cR1, cR2, st, k, cnew);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status defl_beta_g2(double* d, double* G2, int k0, int nbf, double* Gr, int nb, const double* cnew,
                       const double* theta, const double* eps, int k, hipStream_t s) {
  hipLaunchKernelGGL(defl_beta_g2_kernel, dim3(1), dim3(64), 0, s, d, G2, k0, nbf, Gr, nb, cnew, theta, eps, k);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status defl_scale(const double* c, const double* theta, const double* eps, int k, int nb, double* out,
                     hipStream_t s) {
  hipLaunchKernelGGL(defl_scale_kernel, dim3(1), dim3(256), 0, s, c, theta, eps, k, nb, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status mr_init(double* st, const double* dot_r_z, int k, hipStream_t s) {
  hipLaunchKernelGGL(mr_init_kernel<double>, dim3(1), dim3(256), 0, s, st, dot_r_z, k);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}


fe_status mr_alfa(double* st, const double* d1, const double* d2, int k, bool first, hipStream_t s) {
  hipLaunchKernelGGL(mr_alfa_kernel, dim3(1), dim3(256), 0, s, st, d1, d2, k, first ? 1 : 0);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status mr_givens(double* st, const double* dot_r_z, int k, double tol, hipStream_t s) {
  hipLaunchKernelGGL(mr_givens_kernel, dim3(1), dim3(256), 0, s, st, dot_r_z, k, tol);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}



template <typename T>
fe_status k_precond(const T* x, const double* dinv, int k, int64_t nf, T* y, hipStream_t s) {
  hipLaunchKernelGGL(precond_kernel<T>, dim3(grid_for(nf * k)), dim3(256), 0, s, x, dinv, k, (long long)nf, y);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

template <typename T>
fe_status k_select_cols(const T* src, int ko, T* dst, int kn, const int* map, int64_t nf, hipStream_t s) {
  hipLaunchKernelGGL(select_cols_kernel<T>, dim3(grid_for(nf * kn)), dim3(256), 0, s, src, ko, dst, kn, map,
                     (long long)nf);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

template <typename T>
fe_status k_scatter_cols(const T* src, int kc, T* dst, int kf, const int* map, int64_t nf, hipStream_t s) {
  hipLaunchKernelGGL(scatter_cols_kernel<T>, dim3(grid_for(nf * kc)), dim3(256), 0, s, src, kc, dst, kf, map,
                     (long long)nf);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

template fe_status k_select_cols<double>(const double*, int, double*, int, const int*, int64_t, hipStream_t);
template fe_status k_select_cols<float>(const float*, int, float*, int, const int*, int64_t, hipStream_t);
template fe_status k_scatter_cols<double>(const double*, int, double*, int, const int*, int64_t, hipStream_t);
template fe_status k_scatter_cols<float>(const float*, int, float*, int, const int*, int64_t, hipStream_t);

fe_status k_add_f32(const float* d, double* q, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL(add_f32_kernel, dim3(grid_for(total)), dim3(256), 0, s, d, q, (long long)total);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status k_mask_cols(float* r, const double* rr, const double* bb, double tol, int k, int64_t nf, hipStream_t s) {
  hipLaunchKernelGGL(mask_cols_kernel, dim3(grid_for(nf * k)), dim3(256), 0, s, r, rr, bb, tol, k, (long long)nf);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

template fe_status k_precond<double>(const double*, const double*, int, int64_t, double*, hipStream_t);
template fe_status k_precond<float>(const float*, const double*, int, int64_t, float*, hipStream_t);

fe_status k_sub_from(const double* b, double* r, int64_t total, hipStream_t s) {
  hipLaunchKernelGGL(sub_from_kernel, dim3(grid_for(total)), dim3(256), 0, s, b, r, (long long)total);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

}  // namespace invdft
