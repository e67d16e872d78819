// The exchange-correlation potential on its own linear mesh (Eq. 14) and the
// transfer to and from the orbital mesh's GLL nodes (gfx950).
//
// The linear mesh is a tensor product of three 1-D vertex lists t^x, t^y, t^z
// with trilinear hat functions; vertex b = ix + (mx+1)(iy + (my+1) iz). With the
// orbital mesh's GLL quadrature the potential is needed only at the orbital
// nodes, v_a = sum_b N_b(x_a) u_b = (P u)_a, and the gradient with respect to
// the linear unknowns is f = P^T g for the nodal gradient g (Eq. 22). Both
// meshes are tensor products, so P = Px (x) Py (x) Pz with 1-D interpolation
// matrices of two nonzeros a row, and each 1-D hat function is supported on a
// contiguous range of orbital nodes. The handle keeps, per axis:
//   cell[g], s[g]   the linear cell holding free node g and the weight s of its
//                   right vertex (the left one has 1 - s);
//   lo[i], hi[i]    the free nodes in the support of vertex i, [lo, hi).
// prolong: one thread per orbital node, eight gathers from u (small, L2-resident).
// restrict: P^T = Px^T (x) Py^T (x) Pz^T in three 1-D passes (x, then y, then z),
// each thread summing one 1-D support in a fixed order: coalesced, balanced (a
// support along one axis is at most a few dozen nodes even in the coarse outer
// cells) and bitwise reproducible without atomics. The two intermediate arrays
// (n1^2 (mx+1) and n1 (my+1)(mx+1) doubles) belong to the handle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "internal.h"

struct vxc_mesh_s {
  int n1 = 0;                       // free orbital nodes per axis
  int nv[3] = {0, 0, 0};            // vertices per axis
  int64_t nvert = 0;
  int64_t nf = 0;
  int* d_cell[3] = {nullptr, nullptr, nullptr};
  double* d_s[3] = {nullptr, nullptr, nullptr};
  int* d_lo[3] = {nullptr, nullptr, nullptr};
  int* d_hi[3] = {nullptr, nullptr, nullptr};
  double* d_t1 = nullptr;           // [gz][gy][ix]
  double* d_t2 = nullptr;           // [gz][iy][ix]
};

namespace invdft {
namespace {

struct Axes {
  const int* cell[3];
  const double* s[3];
  const int* lo[3];
  const int* hi[3];
  int nv[3];
  int n1;
};

Axes axes_of(const vxc_mesh_s& v) {
  Axes a{};
  for (int d = 0; d < 3; ++d) {
    a.cell[d] = v.d_cell[d];
    a.s[d] = v.d_s[d];
    a.lo[d] = v.d_lo[d];
    a.hi[d] = v.d_hi[d];
    a.nv[d] = v.nv[d];
  }
  a.n1 = v.n1;
  return a;
}

__global__ void prolong_kernel(Axes ax, const double* __restrict__ u, const double* __restrict__ base,
                               double* __restrict__ v, long long nf) {
  const int n1 = ax.n1;
  for (long long a = (long long)blockIdx.x * blockDim.x + threadIdx.x; a < nf; a += (long long)gridDim.x * blockDim.x) {
    const int gx = (int)(a % n1);
    const int gy = (int)((a / n1) % n1);
    const int gz = (int)(a / ((long long)n1 * n1));
    const int cx = ax.cell[0][gx], cy = ax.cell[1][gy], cz = ax.cell[2][gz];
    const double sx = ax.s[0][gx], sy = ax.s[1][gy], sz = ax.s[2][gz];
    const double wx[2] = {1.0 - sx, sx}, wy[2] = {1.0 - sy, sy}, wz[2] = {1.0 - sz, sz};
    const long long sxy = (long long)ax.nv[0] * ax.nv[1];
    double t = 0.0;
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
          t += wx[dx] * wy[dy] * wz[dz] * u[(cx + dx) + (long long)ax.nv[0] * (cy + dy) + sxy * (cz + dz)];
    v[a] = (base ? base[a] : 0.0) + t;
  }
}

__device__ __forceinline__ double hat(const Axes& ax, int d, int i, int g) {
  const int c = ax.cell[d][g];
  const double s = ax.s[d][g];
  return c == i ? 1.0 - s : (c + 1 == i ? s : 0.0);
}

// t1[gz][gy][ix] = sum over the x-support of vertex ix of N_ix(x_gx) g[gz][gy][gx]
__global__ void restrict_x_kernel(Axes ax, const double* __restrict__ g, double* __restrict__ t1, long long total) {
  const long long n1 = ax.n1, nx = ax.nv[0];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(e % nx);
    const long long row = e / nx;                 // gy + n1 gz
    const double* r = g + row * n1;
    double t = 0.0;
    for (int gx = ax.lo[0][ix]; gx < ax.hi[0][ix]; ++gx) t += hat(ax, 0, ix, gx) * r[gx];
    t1[e] = t;
  }
}

// t2[gz][iy][ix] = sum over the y-support of vertex iy of N_iy(y_gy) t1[gz][gy][ix]
__global__ void restrict_y_kernel(Axes ax, const double* __restrict__ t1, double* __restrict__ t2, long long total) {
  const long long n1 = ax.n1, nx = ax.nv[0], ny = ax.nv[1];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(e % nx);
    const int iy = (int)((e / nx) % ny);
    const long long gz = e / (nx * ny);
    double t = 0.0;
    for (int gy = ax.lo[1][iy]; gy < ax.hi[1][iy]; ++gy) t += hat(ax, 1, iy, gy) * t1[ix + nx * (gy + n1 * gz)];
    t2[e] = t;
  }
}

// f[iz][iy][ix] = sum over the z-support of vertex iz of N_iz(z_gz) t2[gz][iy][ix]
__global__ void restrict_z_kernel(Axes ax, const double* __restrict__ t2, double* __restrict__ f, long long total) {
  const long long nxy = (long long)ax.nv[0] * ax.nv[1];
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const long long ixy = e % nxy;
    const int iz = (int)(e / nxy);
    double t = 0.0;
    for (int gz = ax.lo[2][iz]; gz < ax.hi[2][iz]; ++gz) t += hat(ax, 2, iz, gz) * t2[ixy + nxy * gz];
    f[e] = t;
  }
}

unsigned grid_for(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192)); }

void free_tables(vxc_mesh_s* v) {
  for (int d = 0; d < 3; ++d) {
    if (v->d_cell[d]) (void)hipFree(v->d_cell[d]);
    if (v->d_s[d]) (void)hipFree(v->d_s[d]);
    if (v->d_lo[d]) (void)hipFree(v->d_lo[d]);
    if (v->d_hi[d]) (void)hipFree(v->d_hi[d]);
  }
  if (v->d_t1) (void)hipFree(v->d_t1);
  if (v->d_t2) (void)hipFree(v->d_t2);
}

template <typename T>
fe_status upload(const std::vector<T>& h, T** d) {
  if (hipMalloc(reinterpret_cast<void**>(d), std::max<size_t>(1, h.size()) * sizeof(T)) != hipSuccess) {
    *d = nullptr;
    return fail(FE_ENOMEM, "vxc_mesh_create: device allocation failed");
  }
  INVDFT_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return FE_OK;
}

}  // namespace
}  // namespace invdft

using namespace invdft;

extern "C" fe_status vxc_mesh_create(fe_mesh mesh, int mx, const double* tx_h, int my, const double* ty_h, int mz,
                                     const double* tz_h, vxc_mesh* out) {
  const Mesh* m = mesh_tables(mesh);
  if (!m || !out) return fail(FE_EINVAL, "vxc_mesh_create: mesh and out are required");
  *out = nullptr;
  if (m->mapped) return fail(FE_EINVAL, "vxc_mesh_create: mapped orbital meshes are not supported");
  const int ms[3] = {mx, my, mz};
  const double* ts[3] = {tx_h, ty_h, tz_h};
  for (int d = 0; d < 3; ++d) {
    if (!ts[d] || ms[d] < 1) return fail(FE_EINVAL, "vxc_mesh_create: each axis needs >= 1 cell and its vertices");
    for (int i = 0; i < ms[d]; ++i)
      if (!(ts[d][i + 1] > ts[d][i])) return fail(FE_EINVAL, "vxc_mesh_create: vertices must increase strictly");
    if (ts[d][0] > m->x1.front() + 1e-12 || ts[d][ms[d]] < m->x1.back() - 1e-12)
      return fail(FE_EINVAL, "vxc_mesh_create: the linear mesh must cover every free orbital node");
  }
  const int n1 = m->n1;
  vxc_mesh_s* v = new vxc_mesh_s;
  v->n1 = n1;
  v->nf = m->nf;
  v->nvert = 1;
  fe_status st = FE_OK;
  for (int d = 0; d < 3 && st == FE_OK; ++d) {
    const int nvd = ms[d] + 1;
    const double* t = ts[d];
    v->nv[d] = nvd;
    v->nvert *= nvd;
    std::vector<int> cell(n1), lo(nvd, n1), hi(nvd, 0);
    std::vector<double> s(n1);
    for (int g = 0; g < n1; ++g) {
      const double x = std::min(std::max(m->x1[g], t[0]), t[ms[d]]);
      // last cell c with t[c] <= x, at most ms - 1
      int c = (int)(std::upper_bound(t, t + ms[d] + 1, x) - t) - 1;
      c = std::min(std::max(c, 0), ms[d] - 1);
      cell[g] = c;
      s[g] = (x - t[c]) / (t[c + 1] - t[c]);
      for (int i = c; i <= c + 1; ++i) {  // the nodes in the support of vertex i form a range
        lo[i] = std::min(lo[i], g);
        hi[i] = std::max(hi[i], g + 1);
      }
    }
    for (int i = 0; i < nvd; ++i)
      if (hi[i] <= lo[i]) lo[i] = hi[i] = 0;  // no orbital node under this vertex
    if ((st = upload(cell, &v->d_cell[d])) != FE_OK) break;
    if ((st = upload(s, &v->d_s[d])) != FE_OK) break;
    if ((st = upload(lo, &v->d_lo[d])) != FE_OK) break;
    if ((st = upload(hi, &v->d_hi[d])) != FE_OK) break;
  }
  if (st == FE_OK) {
    const size_t b1 = (size_t)n1 * n1 * v->nv[0] * sizeof(double);
    const size_t b2 = (size_t)n1 * v->nv[1] * v->nv[0] * sizeof(double);
    if (hipMalloc(reinterpret_cast<void**>(&v->d_t1), b1) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&v->d_t2), b2) != hipSuccess)
      st = fail(FE_ENOMEM, "vxc_mesh_create: device allocation failed");
  }
  if (st != FE_OK) {
    free_tables(v);
    delete v;
    return st;
  }
  *out = v;
  return FE_OK;
}

extern "C" fe_status vxc_mesh_info(vxc_mesh vm, int64_t* n_vertices_h, int* vertices_per_axis_h) {
  if (!vm) return fail(FE_EINVAL, "vxc_mesh handle is NULL");
  if (n_vertices_h) *n_vertices_h = vm->nvert;
  if (vertices_per_axis_h)
    for (int d = 0; d < 3; ++d) vertices_per_axis_h[d] = vm->nv[d];
  return FE_OK;
}

extern "C" fe_status vxc_mesh_destroy(vxc_mesh vm) {
  if (!vm) return FE_OK;
  free_tables(vm);
  delete vm;
  return FE_OK;
}

extern "C" fe_status vxc_prolong(vxc_mesh vm, const double* u, const double* base, double* v, void* stream) {
  if (!vm || !u || !v) return fail(FE_EINVAL, "vxc_prolong: NULL argument");
  if (u == v || (base && u == base)) return fail(FE_EINVAL, "vxc_prolong: u must not alias v or base");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(prolong_kernel, dim3(grid_for(vm->nf)), dim3(256), 0, s, axes_of(*vm), u, base, v,
                     (long long)vm->nf);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

extern "C" fe_status vxc_restrict(vxc_mesh vm, const double* g, double* f, void* stream) {
  if (!vm || !g || !f) return fail(FE_EINVAL, "vxc_restrict: NULL argument");
  if (g == f) return fail(FE_EINVAL, "vxc_restrict: f must not alias g");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Axes ax = axes_of(*vm);
  const long long n1 = vm->n1, nx = vm->nv[0], ny = vm->nv[1];
  const long long e1 = n1 * n1 * nx, e2 = n1 * ny * nx;
  hipLaunchKernelGGL(restrict_x_kernel, dim3(grid_for(e1)), dim3(256), 0, s, ax, g, vm->d_t1, e1);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(restrict_y_kernel, dim3(grid_for(e2)), dim3(256), 0, s, ax, vm->d_t1, vm->d_t2, e2);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(restrict_z_kernel, dim3(grid_for(vm->nvert)), dim3(256), 0, s, ax, vm->d_t2, f,
                     (long long)vm->nvert);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}
