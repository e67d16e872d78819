// Physics front end (gfx950): the Hartree potential of a density by a finite-element
// Poisson solve on the orbital mesh, and the initial guess of Eq. 25.
//
// Hartree: -lap v_H = 4 pi rho with zero values on the box and the GLL-lumped
// right-hand side, in standard form (K~/2) phi~ = 2 pi W^{1/2} rho, phi = W^{-1/2} phi~.
// The monopole is split off first: Q = sum_a W_a rho_a and the centroid c, then
// rho' = rho - Q g_s(r - c) with the normalised Gaussian g_s, whose potential
// Q erf(|r - c| / (sqrt(2) s)) / |r - c| is added in closed form; rho' has no charge
// and no dipole about c, so the box's zero boundary values cost only its quadrupole
// and higher terms. The linear system is solved by conjugate gradients with the
// kinetic diagonal as preconditioner, each product one ks_apply with a zero
// potential (the same matrix-free stiffness as the Kohn-Sham operator).
//
// Initial guess: v = f v0 + (1 - f) alpha (-v_H / N_e), f = rho / (rho + tau),
// v0 = exchange + Perdew-Wang 1992 correlation of the unpolarised gas, node by node.
// Exchange: Slater -(3 rho / pi)^{1/3}, or van Leeuwen-Baerends (LB94), which adds
// -beta rho_s^{1/3} x^2 / (1 + 3 beta x asinh x), x = |grad rho_s| / rho_s^{4/3},
// rho_s = rho / 2, beta = 0.05. The gradient is that of the order-p interpolant of the
// nodal density: per axis the GLL Lagrange derivative of the node's cell, the two
// one-sided values averaged at a vertex shared by two cells, zero Dirichlet values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "krylov.h"

namespace invdft {
namespace {

constexpr int kMomentsThreads = 256;
constexpr double kPi = 3.14159265358979323846;

__device__ __forceinline__ void node_of(long long a, int n1, int& ix, int& iy, int& iz) {
  ix = (int)(a % n1);
  iy = (int)((a / n1) % n1);
  iz = (int)(a / ((long long)n1 * n1));
}

// per-block partial sums of W rho, W rho x, W rho y, W rho z (fixed-order tree in LDS)
__global__ __launch_bounds__(kMomentsThreads) void moments_partial_kernel(const double* __restrict__ x1,
                                                                          const double* __restrict__ w1, int n1,
                                                                          long long nf, const double* __restrict__ rho,
                                                                          long long per_blk,
                                                                          double* __restrict__ partial) {
  __shared__ double red[4][kMomentsThreads];
  const long long b0 = (long long)blockIdx.x * per_blk;
  const long long b1 = min(nf, b0 + per_blk);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long a = b0 + threadIdx.x; a < b1; a += kMomentsThreads) {
    int ix, iy, iz;
    node_of(a, n1, ix, iy, iz);
    const double q = w1[ix] * w1[iy] * w1[iz] * rho[a];
    s[0] += q;
    s[1] += q * x1[ix];
    s[2] += q * x1[iy];
    s[3] += q * x1[iz];
  }
  for (int c = 0; c < 4; ++c) red[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = kMomentsThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) partial[(long long)blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

struct Monopole {
  double Q, cx, cy, cz, s;  // s <= 0: no split
};

// b = 2 pi W^{1/2} (rho - Q g_s(r - c))
__global__ void poisson_rhs_kernel(const double* __restrict__ x1, const double* __restrict__ w1, int n1, long long nf,
                                   const double* __restrict__ rho, Monopole mp, double* __restrict__ b) {
  const double norm = mp.s > 0 ? 1.0 / (2.0 * kPi * mp.s * mp.s * sqrt(2.0 * kPi * mp.s * mp.s)) : 0.0;
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    node_of(a, n1, ix, iy, iz);
    double r = rho[a];
    if (mp.s > 0) {
      const double dx = x1[ix] - mp.cx, dy = x1[iy] - mp.cy, dz = x1[iz] - mp.cz;
      r -= mp.Q * norm * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * mp.s * mp.s));
    }
    b[a] = 2.0 * kPi * sqrt(w1[ix] * w1[iy] * w1[iz]) * r;
  }
}

// phi = W^{-1/2} x + Q erf(|r - c| / (sqrt(2) s)) / |r - c|
__global__ void poisson_finish_kernel(const double* __restrict__ x1, const double* __restrict__ w1, int n1,
                                      long long nf, const double* __restrict__ xt, Monopole mp,
                                      double* __restrict__ phi) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    int ix, iy, iz;
    node_of(a, n1, ix, iy, iz);
    double v = xt[a] / sqrt(w1[ix] * w1[iy] * w1[iz]);
    if (mp.s > 0) {
      const double dx = x1[ix] - mp.cx, dy = x1[iy] - mp.cy, dz = x1[iz] - mp.cz;
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      v += mp.Q * (r < 1e-8 * mp.s ? sqrt(2.0 / kPi) / mp.s : erf(r / (sqrt(2.0) * mp.s)) / r);
    }
    phi[a] = v;
  }
}

// Preconditioned CG with its scalars on the device, so that an iteration needs no host round trip.
// S[0] = b.b, S[1] and S[2] = r.z of alternate iterations, S[3] = p.q, S[4] = r.r, S[5] = 1 once
// converged, S[6] = iterations done, S[7] = relative residual. Every update is a no-op once S[5]
// is set, so the iterations launched after convergence (until the host next looks) change nothing.
enum { kCgBB = 0, kCgPQ = 3, kCgRR = 4, kCgDone = 5, kCgIters = 6, kCgRel = 7 };

__global__ void cg_init_kernel(double* __restrict__ S) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S[kCgDone] = S[kCgBB] > 0.0 ? 0.0 : 1.0;
    S[kCgIters] = 0.0;
    S[kCgRel] = S[kCgBB] > 0.0 ? 1.0 : 0.0;
  }
}

// x += alpha p, r -= alpha q with alpha = (r.z) / (p.q)
__global__ void cg_xr_kernel(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                             const double* __restrict__ q, const double* __restrict__ S, int irz, long long n) {
  if (S[kCgDone] != 0.0) return;
  const double alpha = S[irz] / S[kCgPQ];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    x[i] = fma(alpha, p[i], x[i]);
    r[i] = fma(-alpha, q[i], r[i]);
  }
}

__global__ void cg_check_kernel(double* __restrict__ S, double tol) {
  if (blockIdx.x != 0 || threadIdx.x != 0 || S[kCgDone] != 0.0) return;
  S[kCgIters] += 1.0;
  const double rel = sqrt(S[kCgRR] / S[kCgBB]);
  S[kCgRel] = rel;
  if (rel <= tol) S[kCgDone] = 1.0;
}

// p = z + beta p with beta = (r.z)_new / (r.z)_old
__global__ void cg_p_kernel(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ S,
                            int inew, int iold, long long n) {
  if (S[kCgDone] != 0.0) return;
  const double beta = S[inew] / S[iold];
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = fma(beta, p[i], z[i]);
}

// Perdew-Wang 1992 correlation of the unpolarised gas (J. P. Perdew and Y. Wang, Phys. Rev. B 45,
// 13244 (1992), the published parameters of its fit): e_c(r_s) and v_c = e_c - (r_s/3) de_c/dr_s
__device__ __forceinline__ double pw92_vc(double rho) {
  const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double rs = cbrt(3.0 / (4.0 * kPi * rho));
  const double s = sqrt(rs);
  const double q = 2.0 * A * (b1 * s + b2 * rs + b3 * rs * s + b4 * rs * rs);
  const double dq = A * (b1 / s + 2.0 * b2 + 3.0 * b3 * s + 4.0 * b4 * rs);
  const double lg = log1p(1.0 / q);
  const double ec = -2.0 * A * (1.0 + a1 * rs) * lg;
  const double dec = -2.0 * A * a1 * lg + 2.0 * A * (1.0 + a1 * rs) * dq / (q * q + q);
  return ec - rs / 3.0 * dec;
}

struct DerivTable {
  double d[kMaxP1 * kMaxP1];  // d[j (p+1) + k] = N_k'(xi_j) on [-1, 1]
  int p;
};

// derivative of the interpolant along one axis at 1-D free node f (g = f + 1) of the line
// whose free node f' sits at base + f' stride; 2/h_e per cell from inv_h2 (n entries)
__device__ double axis_derivative(const double* __restrict__ rho, long long base, long long stride, int f, int n,
                                  int n1, const DerivTable& D, const double* __restrict__ two_over_h) {
  const int p = D.p;
  const int g = f + 1;
  const int e = g / p, j = g % p;
  auto val = [&](int gg) { return (gg >= 1 && gg <= n1) ? rho[base + (long long)(gg - 1) * stride] : 0.0; };
  double dr = 0.0;
  for (int k = 0; k <= p; ++k) dr += D.d[j * (p + 1) + k] * val(e * p + k);
  dr *= two_over_h[e];
  if (j == 0) {  // vertex: the left cell's row p as well, averaged
    double dl = 0.0;
    for (int k = 0; k <= p; ++k) dl += D.d[p * (p + 1) + k] * val((e - 1) * p + k);
    dr = 0.5 * (dr + dl * two_over_h[e - 1]);
  }
  return dr;
}

__global__ void xc_init_kernel(const double* __restrict__ rho, const double* __restrict__ vh, long long n, int n1,
                               int ncell, DerivTable D, const double* __restrict__ two_over_h, int lb94,
                               double n_elec, double tau, double alpha, double* __restrict__ v) {
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (long long)gridDim.x * blockDim.x) {
    const double r = rho[a];
    const double f = r / (r + tau);
    double v0 = 0.0;
    if (r > 1e-30) {
      v0 = -cbrt(3.0 * r / kPi) + pw92_vc(r);
      if (lb94) {
        int ix, iy, iz;
        node_of(a, n1, ix, iy, iz);
        const long long sy = n1, sz = (long long)n1 * n1;
        const double gx = axis_derivative(rho, a - ix, 1, ix, ncell, n1, D, two_over_h);
        const double gy = axis_derivative(rho, a - iy * sy, sy, iy, ncell, n1, D, two_over_h);
        const double gz = axis_derivative(rho, a - iz * sz, sz, iz, ncell, n1, D, two_over_h);
        const double rs = 0.5 * r;
        const double x = 0.5 * sqrt(gx * gx + gy * gy + gz * gz) / (rs * cbrt(rs));
        v0 -= 0.05 * cbrt(rs) * x * x / (1.0 + 0.15 * x * asinh(x));
      }
    }
    v[a] = f * v0 + (1.0 - f) * alpha * (-vh[a] / n_elec);
  }
}

// N_k'(xi_j) at the GLL nodes from the barycentric form of the Lagrange basis
void derivative_table(int p, DerivTable& D) {
  std::vector<double> Kh((p + 1) * (p + 1)), Mh((p + 1) * (p + 1)), xi(p + 1), wi(p + 1);
  reference_matrices(p, Kh.data(), Mh.data(), xi.data(), wi.data());
  std::vector<double> bw(p + 1, 1.0);
  for (int j = 0; j <= p; ++j)
    for (int k = 0; k <= p; ++k)
      if (k != j) bw[j] /= (xi[j] - xi[k]);
  D.p = p;
  for (int j = 0; j <= p; ++j) {
    double diag = 0.0;
    for (int k = 0; k <= p; ++k) {
      if (k == j) continue;
      const double djk = (bw[k] / bw[j]) / (xi[j] - xi[k]);
      D.d[j * (p + 1) + k] = djk;
      diag -= djk;
    }
    D.d[j * (p + 1) + j] = diag;
  }
}

unsigned grid_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192)); }

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t poisson_work_bytes(int64_t nf) { return 7 * round256((size_t)nf * sizeof(double)) + round256(8192 * 8) + 256; }

}  // namespace invdft

using namespace invdft;

extern "C" fe_status poisson_solve(fe_mesh mesh, const double* rho, double sigma, double* phi, double tol, int maxit,
                                   int* iters_h, double* relres_h, double* charge_h, void* work, void* stream) {
  const Mesh* mp = mesh_tables(mesh);
  if (!mp) return fail(FE_EINVAL, "mesh handle is NULL");
  if (!rho || !phi || !work) return fail(FE_EINVAL, "poisson_solve: NULL argument");
  if (mp->mapped) return fail(FE_EINVAL, "poisson_solve: mapped meshes are not supported");
  if (!(tol > 0.0) || maxit < 1) return fail(FE_EINVAL, "poisson_solve: tol > 0 and maxit >= 1 required");
  if (!(sigma >= 0.0)) return fail(FE_EINVAL, "poisson_solve: sigma must be >= 0");
  const Mesh& m = *mp;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long nf = m.nf;
  char* w = static_cast<char*>(work);
  const size_t vb = round256((size_t)nf * sizeof(double));
  double* x = reinterpret_cast<double*>(w);
  double* r = reinterpret_cast<double*>(w + vb);
  double* z = reinterpret_cast<double*>(w + 2 * vb);
  double* p = reinterpret_cast<double*>(w + 3 * vb);
  double* q = reinterpret_cast<double*>(w + 4 * vb);
  double* dinv = reinterpret_cast<double*>(w + 5 * vb);
  double* vzero = reinterpret_cast<double*>(w + 6 * vb);
  double* scratch = reinterpret_cast<double*>(w + 7 * vb);   // 1024 partials + scalars
  double* scal = scratch + 8000;
  fe_status st;
  // charge and centroid: per-block partials, summed on the host in block order
  const int nblk = (int)std::max<long long>(1, std::min<long long>((nf + 4095) / 4096, 1024));
  const long long per = (nf + nblk - 1) / nblk;
  hipLaunchKernelGGL(moments_partial_kernel, dim3(nblk), dim3(kMomentsThreads), 0, s, m.d_x1, m.d_w1, m.n1, nf, rho,
                     per, scratch);
  INVDFT_HIP(hipGetLastError());
  std::vector<double> part((size_t)nblk * 4);
  INVDFT_HIP(hipMemcpyAsync(part.data(), scratch, part.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  INVDFT_HIP(hipStreamSynchronize(s));
  double mom[4] = {0.0, 0.0, 0.0, 0.0};
  for (int bk = 0; bk < nblk; ++bk)
    for (int c = 0; c < 4; ++c) mom[c] += part[(size_t)bk * 4 + c];
  Monopole mono{mom[0], 0.0, 0.0, 0.0, 0.0};
  if (sigma > 0.0 && mom[0] != 0.0) {
    mono.cx = mom[1] / mom[0];
    mono.cy = mom[2] / mom[0];
    mono.cz = mom[3] / mom[0];
    mono.s = sigma;
  }
  if (charge_h) *charge_h = mom[0];
  // r = b, x = 0, z = D^{-1} r, p = z
  hipLaunchKernelGGL(poisson_rhs_kernel, dim3(grid_for(nf)), dim3(256), 0, s, m.d_x1, m.d_w1, m.n1, nf, rho, mono, r);
  INVDFT_HIP(hipGetLastError());
  if ((st = fill(x, 0.0, nf, s)) != FE_OK) return st;
  if ((st = fill(vzero, 0.0, nf, s)) != FE_OK) return st;
  if ((st = k_dinv(m, dinv, s)) != FE_OK) return st;
  double* S = scal;   // the CG scalars (device)
  if ((st = dot1(r, r, nf, S + kCgBB, scratch, s)) != FE_OK) return st;
  if ((st = k_precond<double>(r, dinv, 1, nf, z, s)) != FE_OK) return st;
  if ((st = copy_bytes(z, p, (size_t)nf * sizeof(double), s)) != FE_OK) return st;
  if ((st = dot1(r, z, nf, S + 1, scratch, s)) != FE_OK) return st;
  hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(64), 0, s, S);
  INVDFT_HIP(hipGetLastError());
  ApplyArgs aa{};
  aa.X = p;
  aa.Y = q;
  aa.v = vzero;
  aa.nv = 1;
  aa.ld = 1;
  aa.alpha = 1.0;
  double hs[3] = {1.0, 0.0, 0.0};   // done, iterations, relative residual, as last read
  auto read_state = [&]() -> fe_status {
    INVDFT_HIP(hipMemcpyAsync(hs, S + kCgDone, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    INVDFT_HIP(hipStreamSynchronize(s));
    return FE_OK;
  };
  if ((st = read_state()) != FE_OK) return st;
  const int check_every = 8;   // host looks at the convergence flag this often
  const unsigned g = grid_for(nf);
  for (int it = 0; hs[0] == 0.0 && it < maxit; ++it) {
    const int irz = 1 + (it & 1), inew = 1 + ((it + 1) & 1);
    if ((st = launch_apply(m, aa, FE_F64, s)) != FE_OK) return st;   // q = (K~/2) p
    if ((st = dot1(p, q, nf, S + kCgPQ, scratch, s)) != FE_OK) return st;
    hipLaunchKernelGGL(cg_xr_kernel, dim3(g), dim3(256), 0, s, x, r, p, q, S, irz, nf);
    INVDFT_HIP(hipGetLastError());
    if ((st = dot1(r, r, nf, S + kCgRR, scratch, s)) != FE_OK) return st;
    hipLaunchKernelGGL(cg_check_kernel, dim3(1), dim3(64), 0, s, S, tol);
    INVDFT_HIP(hipGetLastError());
    if ((st = k_precond<double>(r, dinv, 1, nf, z, s)) != FE_OK) return st;
    if ((st = dot1(r, z, nf, S + inew, scratch, s)) != FE_OK) return st;
    hipLaunchKernelGGL(cg_p_kernel, dim3(g), dim3(256), 0, s, p, z, S, inew, irz, nf);
    INVDFT_HIP(hipGetLastError());
    if ((it + 1) % check_every == 0 && (st = read_state()) != FE_OK) return st;
  }
  if ((st = read_state()) != FE_OK) return st;
  const int it = (int)hs[1];
  const double rel = hs[2];
  hipLaunchKernelGGL(poisson_finish_kernel, dim3(grid_for(nf)), dim3(256), 0, s, m.d_x1, m.d_w1, m.n1, nf, x, mono,
                     phi);
  INVDFT_HIP(hipGetLastError());
  INVDFT_HIP(hipStreamSynchronize(s));
  if (iters_h) *iters_h = it;
  if (relres_h) *relres_h = rel;
  if (rel > tol) return fail(FE_ENOCONV, "poisson_solve: tolerance not reached in maxit iterations");
  return FE_OK;
}

extern "C" fe_status xc_initial_guess(fe_mesh mesh, const double* rho, const double* v_h, double n_elec, double tau,
                                      double alpha, int exchange, double* v, void* work, void* stream) {
  const Mesh* mp = mesh_tables(mesh);
  if (!mp) return fail(FE_EINVAL, "mesh handle is NULL");
  if (!rho || !v_h || !v) return fail(FE_EINVAL, "xc_initial_guess: NULL argument");
  if (mp->mapped) return fail(FE_EINVAL, "xc_initial_guess: mapped meshes are not supported");
  if (!(n_elec > 0.0) || !(tau > 0.0)) return fail(FE_EINVAL, "xc_initial_guess: n_elec > 0 and tau > 0 required");
  if (exchange != FE_XC_SLATER && exchange != FE_XC_LB94) return fail(FE_EINVAL, "xc_initial_guess: unknown exchange");
  if (exchange == FE_XC_LB94 && !work) return fail(FE_EINVAL, "xc_initial_guess: LB94 needs work");
  const Mesh& m = *mp;
  hipStream_t s = static_cast<hipStream_t>(stream);
  DerivTable D{};
  double* two_over_h = static_cast<double*>(work);
  std::vector<double> th;
  if (exchange == FE_XC_LB94) {
    derivative_table(m.p, D);
    th.resize(m.n);
    for (int e = 0; e < m.n; ++e) th[e] = 2.0 / (m.graded ? m.cell_h[e] : m.h);
    INVDFT_HIP(hipMemcpyAsync(two_over_h, th.data(), th.size() * sizeof(double), hipMemcpyHostToDevice, s));
  }
  if (m.nf > 0)
    hipLaunchKernelGGL(xc_init_kernel, dim3(grid_for(m.nf)), dim3(256), 0, s, rho, v_h, (long long)m.nf, m.n1, m.n, D,
                       two_over_h, exchange == FE_XC_LB94 ? 1 : 0, n_elec, tau, alpha, v);
  INVDFT_HIP(hipGetLastError());
  if (exchange == FE_XC_LB94) INVDFT_HIP(hipStreamSynchronize(s));   // th is read by the copy
  return FE_OK;
}
