// Mapped hexahedral meshes: every cell carries its own dense element matrix, and the
// operator is the batched product of per-cell matrices with gather and scatter of the
// paper's Sec. 3.2.3, on the FP64 matrix cores.
//
// Geometry. The nodes are the uniform mesh's GLL nodes moved by the map
//   Phi_d(xi) = xi_d + amp (L/pi) sin(pi xi_d / L) sin(pi xi_{d+1} / L)   (d + 1 cyclic),
// which takes each face of [-L, L]^3 into itself; a cell's shape is the order-p
// interpolant of its node coordinates (isoparametric), so its cells are curved and no
// element matrix factorises per axis.
//
// Set-up (once per mesh, on the device):
//   1. per cell: node coordinates, the lumped mass W_e at the GLL nodes (|det J| w^w^w^),
//      and G(q) = w_q |det J| J^{-1} J^{-T} at the q^3 Gauss points, q = ceil((3p + 1)/2)
//      (enough for the stiffness of any linear field to be integrated exactly);
//      K_e = Abar^T T with Abar[(q, d)][a] = d N_a / d xi_d at point q and
//      T[(q, d)][b] = sum_f G_df(q) Abar[(q, f)][b]: a (n_p x 3q^3) (3q^3 x n_p) product on
//      FP64 MFMA, upper tiles only, mirrored exactly;
//   2. per free node, in a fixed cell order: W_a, the stiffness diagonal, the coordinates;
//   3. per cell: K~_e = (1/2) s K_e s with s = W^{-1/2} (0 at Dirichlet nodes), stored in
//      the MFMA A-operand order (one 64-double fragment per 16 x 4 tile, so that each
//      wavefront loads one contiguous 512-byte piece per instruction), in FP64 and FP32;
//      and a Gershgorin bound of (1/2) W_e^{-1/2} K_e W_e^{-1/2} (Fried's element bound).
//
// Apply: Y = alpha cs_j ((K~/2) X + (v - c - s_j) X) + beta Z as eight launches of cell
// products, one per parity class (ex, ey, ez mod 2): cells of one class share no node, so
// each launch adds its contributions with plain read-modify-write, in a fixed order, bitwise
// reproducibly. The first class that holds a node writes it, with the diagonal and Chebyshev
// terms (X from the gathered block); the later ones add.
// A workgroup gathers a cell's X_e (n_p x up to 64 columns) into LDS, and each wavefront
// streams its M-tiles of K~_e from HBM through v_mfma_f64_16x16x4f64, all its tiles at once,
// with the A fragments three steps ahead in registers (FP32 storage is widened to FP64 there).
// Up to 64 columns the matrices stream once per apply; the product is HBM-bound up to about 32
// FP64 columns and FP64-MFMA-bound beyond.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace invdft {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l holds A[l%16][l/16] and B[l/16][l%16]; the result D is
// D[l/16 + 4r][l%16] in register r.
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kMapThreads = 256;
constexpr int kMaxQ = 13;   // Gauss points per axis for p <= 8

struct MapGeom {
  int p, n, N, n1;    // order, cells per axis, nodes per axis (p n + 1), free nodes per axis
  double L, h, amp;
};

struct MapTables {
  double xi[kMaxP1];             // GLL nodes
  double wg[kMaxP1];             // GLL weights
  double Dg[kMaxP1 * kMaxP1];    // Dg[j][i] = N_i'(xi_j)
  double Bq[kMaxQ * kMaxP1];     // Bq[q][i] = N_i(x_q)
  double Dq[kMaxQ * kMaxP1];     // Dq[q][i] = N_i'(x_q)
  double wq[kMaxQ];
  int q;
};

__device__ __forceinline__ double ref_coord(const MapGeom& g, const MapTables& t, int idx) {
  int e = idx / g.p, j = idx - e * g.p;
  if (e == g.n) {
    e = g.n - 1;
    j = g.p;
  }
  return -g.L + g.h * (e + 0.5 * (t.xi[j] + 1.0));
}

__device__ __forceinline__ void warp_point(const MapGeom& g, double r[3], double x[3]) {
  double s[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = sin(M_PI * r[d] / g.L);
#pragma unroll
  for (int d = 0; d < 3; ++d) x[d] = r[d] + g.amp * (g.L / M_PI) * s[d] * s[(d + 1) % 3];
}

__device__ __forceinline__ double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Step 1: one workgroup per cell. Kraw: n_c x n_p x n_p (row-major per cell), We: n_c x n_p.
// Abar: KP x NP16 (rows (q, d), zero padded). flag: set to 1 when a cell is inverted.
template <int P>
__global__ __launch_bounds__(kMapThreads) void mapped_element_kernel(MapGeom g, MapTables t,
                                                                     const double* __restrict__ Abar, int KP,
                                                                     int NP16, double* __restrict__ Kraw,
                                                                     double* __restrict__ We, int* flag) {
  constexpr int P1 = P + 1, NP = P1 * P1 * P1;
  __shared__ double sX[NP][3];
  extern __shared__ double sG[];   // q^3 x 6: G00 G01 G02 G11 G12 G22 (times w_q)
  const int cell = blockIdx.x;
  const int ex = cell % g.n, ey = (cell / g.n) % g.n, ez = cell / (g.n * g.n);
  const int tid = threadIdx.x;
  for (int a = tid; a < NP; a += kMapThreads) {
    const int i = a % P1, j = (a / P1) % P1, k = a / (P1 * P1);
    double r[3] = {ref_coord(g, t, ex * P + i), ref_coord(g, t, ey * P + j), ref_coord(g, t, ez * P + k)};
    double x[3];
    warp_point(g, r, x);
    sX[a][0] = x[0];
    sX[a][1] = x[1];
    sX[a][2] = x[2];
  }
  __syncthreads();
  // lumped mass at the GLL nodes: the interpolant's Jacobian there
  for (int a = tid; a < NP; a += kMapThreads) {
    const int i = a % P1, j = (a / P1) % P1, k = a / (P1 * P1);
    double J[3][3] = {};
    for (int m = 0; m < P1; ++m) {
      const double di = t.Dg[i * P1 + m], dj = t.Dg[j * P1 + m], dk = t.Dg[k * P1 + m];
      const int ai = m + P1 * (j + P1 * k), aj = i + P1 * (m + P1 * k), ak = i + P1 * (j + P1 * m);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        J[c][0] += di * sX[ai][c];
        J[c][1] += dj * sX[aj][c];
        J[c][2] += dk * sX[ak][c];
      }
    }
    const double det = det3(J);
    if (!(det > 0.0)) *flag = 1;
    We[(size_t)cell * NP + a] = t.wg[i] * t.wg[j] * t.wg[k] * fabs(det);
  }
  // the metric at the Gauss points
  const int q = t.q, q3 = q * q * q;
  for (int qq = tid; qq < q3; qq += kMapThreads) {
    const int qx = qq % q, qy = (qq / q) % q, qz = qq / (q * q);
    double J[3][3] = {};
    for (int a = 0; a < NP; ++a) {
      const int i = a % P1, j = (a / P1) % P1, k = a / (P1 * P1);
      const double bx = t.Bq[qx * P1 + i], by = t.Bq[qy * P1 + j], bz = t.Bq[qz * P1 + k];
      const double g0 = t.Dq[qx * P1 + i] * by * bz, g1 = bx * t.Dq[qy * P1 + j] * bz, g2 = bx * by * t.Dq[qz * P1 + k];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        J[c][0] += sX[a][c] * g0;
        J[c][1] += sX[a][c] * g1;
        J[c][2] += sX[a][c] * g2;
      }
    }
    const double det = det3(J);
    if (!(det > 0.0)) *flag = 1;
    // adj(J) = det J^{-1}; G = w |det| J^{-1} J^{-T} = w adj adj^T / det
    double A[3][3];
    A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double s = t.wq[qx] * t.wq[qy] * t.wq[qz] / fabs(det);
    auto gg = [&](int d, int f) { return s * (A[d][0] * A[f][0] + A[d][1] * A[f][1] + A[d][2] * A[f][2]); };
    sG[qq * 6 + 0] = gg(0, 0);
    sG[qq * 6 + 1] = gg(0, 1);
    sG[qq * 6 + 2] = gg(0, 2);
    sG[qq * 6 + 3] = gg(1, 1);
    sG[qq * 6 + 4] = gg(1, 2);
    sG[qq * 6 + 5] = gg(2, 2);
  }
  __syncthreads();
  // K_e = Abar^T T on the upper 16 x 16 tiles
  const int wave = tid / 64, lane = tid % 64, lr = lane % 16, lk = lane / 16;
  const int TT = NP16 / 16;
  const int ntile = TT * (TT + 1) / 2;
  const int KR = 3 * q3;
  for (int tix = wave; tix < ntile; tix += kMapThreads / 64) {
    int mt = 0, rem = tix;
    while (rem >= TT - mt) {
      rem -= TT - mt;
      ++mt;
    }
    const int nt = mt + rem;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const int col = nt * 16 + lr;
    for (int k0 = 0; k0 < KP; k0 += 4) {
      const int kap = k0 + lk;
      const double a = Abar[(size_t)kap * NP16 + mt * 16 + lr];
      double b = 0.0;
      if (kap < KR) {
        const int qq = kap / 3, d = kap - 3 * qq;
        const double* Gq = sG + qq * 6;
        const double gd0 = (d == 0) ? Gq[0] : (d == 1 ? Gq[1] : Gq[2]);
        const double gd1 = (d == 0) ? Gq[1] : (d == 1 ? Gq[3] : Gq[4]);
        const double gd2 = (d == 0) ? Gq[2] : (d == 1 ? Gq[4] : Gq[5]);
        const double* Ar = Abar + (size_t)(3 * qq) * NP16 + col;
        b = gd0 * Ar[0] + gd1 * Ar[NP16] + gd2 * Ar[2 * NP16];
      }
      acc = mfma16(a, b, acc);
    }
    double* Kc = Kraw + (size_t)cell * NP * NP;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = mt * 16 + lk + 4 * r;
      if (row < NP && col < NP) {
        Kc[(size_t)row * NP + col] = acc[r];
        if (mt != nt) Kc[(size_t)col * NP + row] = acc[r];
      }
    }
  }
}

// Step 2: per free node, the cells holding it in a fixed order (z, then y, then x).
template <int P>
__global__ void mapped_node_kernel(MapGeom g, MapTables t, const double* __restrict__ Kraw,
                                   const double* __restrict__ We, double* __restrict__ wn,
                                   double* __restrict__ kdn, double* __restrict__ xyz) {
  constexpr int P1 = P + 1, NP = P1 * P1 * P1;
  const long long nf = (long long)g.n1 * g.n1 * g.n1;
  for (long long af = (long long)blockIdx.x * blockDim.x + threadIdx.x; af < nf;
       af += (long long)gridDim.x * blockDim.x) {
    const int gx = (int)(af % g.n1) + 1, gy = (int)((af / g.n1) % g.n1) + 1, gz = (int)(af / ((long long)g.n1 * g.n1)) + 1;
    int cx[2], lx[2], nx = 0, cy[2], ly[2], ny = 0, cz[2], lz[2], nz = 0;
    auto cells_of = [&](int gc, int* c, int* l, int& cnt) {
      if (gc % P == 0) {
        c[0] = gc / P - 1;
        l[0] = P;
        c[1] = gc / P;
        l[1] = 0;
        cnt = 2;
      } else {
        c[0] = gc / P;
        l[0] = gc % P;
        cnt = 1;
      }
    };
    cells_of(gx, cx, lx, nx);
    cells_of(gy, cy, ly, ny);
    cells_of(gz, cz, lz, nz);
    double w = 0.0, kd = 0.0;
    for (int iz = 0; iz < nz; ++iz)
      for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
          const long long cell = cx[ix] + (long long)g.n * (cy[iy] + (long long)g.n * cz[iz]);
          const int a = lx[ix] + P1 * (ly[iy] + P1 * lz[iz]);
          w += We[cell * NP + a];
          kd += Kraw[(size_t)cell * NP * NP + (size_t)a * NP + a];
        }
    wn[af] = w;
    kdn[af] = 0.5 * kd / w;
    double r[3] = {ref_coord(g, t, gx), ref_coord(g, t, gy), ref_coord(g, t, gz)};
    double x[3];
    warp_point(g, r, x);
    xyz[3 * af + 0] = x[0];
    xyz[3 * af + 1] = x[1];
    xyz[3 * af + 2] = x[2];
  }
}

// Step 3: scaled matrices in A-fragment order, and the per-cell element bound.
template <int P>
__global__ __launch_bounds__(kMapThreads) void mapped_scale_kernel(MapGeom g, const double* __restrict__ Kraw,
                                                                   const double* __restrict__ We,
                                                                   const double* __restrict__ wn, int MT, int KS,
                                                                   double* __restrict__ K64, float* __restrict__ K32,
                                                                   double* __restrict__ bound) {
  constexpr int P1 = P + 1, NP = P1 * P1 * P1;
  __shared__ double sS[NP];
  __shared__ double sR[kMapThreads];
  const int cell = blockIdx.x;
  const int ex = cell % g.n, ey = (cell / g.n) % g.n, ez = cell / (g.n * g.n);
  const int tid = threadIdx.x;
  for (int a = tid; a < NP; a += kMapThreads) {
    const int gx = ex * P + a % P1, gy = ey * P + (a / P1) % P1, gz = ez * P + a / (P1 * P1);
    const bool fr = gx >= 1 && gx <= g.N - 2 && gy >= 1 && gy <= g.N - 2 && gz >= 1 && gz <= g.N - 2;
    sS[a] = fr ? 1.0 / sqrt(wn[(gx - 1) + (long long)g.n1 * ((gy - 1) + (long long)g.n1 * (gz - 1))]) : 0.0;
  }
  __syncthreads();
  const double* Kc = Kraw + (size_t)cell * NP * NP;
  const double* Wc = We + (size_t)cell * NP;
  const size_t base = (size_t)cell * MT * KS * 64;
  for (int e = tid; e < MT * KS * 64; e += kMapThreads) {
    const int lane = e % 64, ks = (e / 64) % KS, mt = e / (64 * KS);
    const int row = mt * 16 + lane % 16, col = ks * 4 + lane / 16;
    const double val = (row < NP && col < NP) ? 0.5 * sS[row] * Kc[(size_t)row * NP + col] * sS[col] : 0.0;
    K64[base + e] = val;
    K32[base + e] = (float)val;
  }
  double r = 0.0;
  for (int a = tid; a < NP; a += kMapThreads) {
    double s = 0.0;
    const double wa = Wc[a];
    for (int b = 0; b < NP; ++b) s += fabs(Kc[(size_t)a * NP + b]) / sqrt(wa * Wc[b]);
    r = fmax(r, s);
  }
  sR[tid] = r;
  __syncthreads();
  for (int w = kMapThreads / 2; w > 0; w >>= 1) {
    if (tid < w) sR[tid] = fmax(sR[tid], sR[tid + w]);
    __syncthreads();
  }
  if (tid == 0) bound[cell] = 0.5 * sR[0];
}

// ------------------------------------------------------------------ apply
struct MapApply {
  const void* X;
  void* Y;
  const void* Z;
  const double* v;
  const double* colscale;
  const void* K;
  int n, n1, nv, ld, MT, KS;
  int cx, cy, cz, ncx, ncy;   // parity class and its cell counts along x, y
  int jchunks;
  int has_colshift;
  double alpha, beta, cshift;
  double colshift[kMaxShiftCols];
};

// One parity class: workgroup = (cell of the class, chunk of 16 NTL columns). Wavefront w
// owns the M-tiles w, w + 4, ... (MTI of them) and keeps MTI x NTL independent accumulators,
// so consecutive MFMAs never wait on each other and every fragment of K~_e loaded from HBM
// feeds NTL products. The gathered block lives in LDS in the storage precision (LT).
template <typename T, int P, int NTL, int NT>
__global__ __launch_bounds__(NT) void mapped_cell_kernel(const MapApply a) {
  constexpr int P1 = P + 1, NP = P1 * P1 * P1;
  constexpr int NP4 = (NP + 3) / 4 * 4;
  constexpr int JC = 16 * NTL;
  constexpr int MT = (NP + 15) / 16, KS = NP4 / 4;
  constexpr int NW = NT / 64;
  constexpr int MTI = (MT + NW - 1) / NW;
  constexpr int EV = 16 / sizeof(T);          // elements per 16-byte load
  // a B fragment reads 16 columns of 4 consecutive rows: a row pitch of 16 (mod 32) elements
  // puts the four rows on different LDS banks (FP32) or bank halves (FP64)
  constexpr int JP = JC + ((JC == 32 || (JC == 64 && sizeof(T) == 4)) ? 16 : 0);
  __shared__ __attribute__((aligned(16))) T sX[NP4][JP];
  __shared__ long long sNode[NP4];   // free-node index of each local node, -1 at Dirichlet nodes
  __shared__ unsigned char sFirst[NP4];   // 1: this cell's class is the first launched that holds the node
  const T* X = static_cast<const T*>(a.X);
  T* Y = static_cast<T*>(a.Y);
  const T* Z = static_cast<const T*>(a.Z);
  const T* K = static_cast<const T*>(a.K);
  const int tid = threadIdx.x;
  const int jc = blockIdx.x % a.jchunks;
  const int c = blockIdx.x / a.jchunks;
  const int ex = a.cx + 2 * (c % a.ncx), ey = a.cy + 2 * ((c / a.ncx) % a.ncy), ez = a.cz + 2 * (c / (a.ncx * a.ncy));
  const int j0 = jc * JC;
  const int pn = P * a.n;
  for (int l = tid; l < NP4; l += NT) {
    long long idx = -1;
    unsigned char first = 0;
    if (l < NP) {
      const int gx = ex * P + l % P1, gy = ey * P + (l / P1) % P1, gz = ez * P + l / (P1 * P1);
      if (gx >= 1 && gx <= pn - 1 && gy >= 1 && gy <= pn - 1 && gz >= 1 && gz <= pn - 1) {
        idx = (gx - 1) + (long long)a.n1 * ((gy - 1) + (long long)a.n1 * (gz - 1));
        // the classes run in the order (cz, cy, cx) = (0, 0, 0), (0, 0, 1), ...: the first that
        // holds the node takes, along each axis, the smaller parity of the cells holding it (a
        // vertex plane lies in two cells, one of each parity)
        const int px = gx % P == 0 ? 0 : (gx / P) % 2;
        const int py = gy % P == 0 ? 0 : (gy / P) % 2;
        const int pz = gz % P == 0 ? 0 : (gz / P) % 2;
        first = (px == a.cx && py == a.cy && pz == a.cz) ? 1 : 0;
      }
    }
    sNode[l] = idx;
    sFirst[l] = first;
  }
  __syncthreads();
  // gather X_e: 16-byte pieces where the row pitch keeps them aligned and inside the block
  typedef T TV __attribute__((ext_vector_type(EV)));
  const bool vec = (a.ld % EV) == 0;
  for (int e = tid; e < NP4 * (JC / EV); e += NT) {
    const int l = e / (JC / EV), jj = (e % (JC / EV)) * EV;
    const long long node = sNode[l];
    const int j = j0 + jj;
    TV val;
    if (node >= 0 && vec && j + EV <= a.nv) {
      val = *reinterpret_cast<const TV*>(X + (size_t)node * a.ld + j);
    } else {
#pragma unroll
      for (int q = 0; q < EV; ++q) val[q] = (node >= 0 && j + q < a.nv) ? X[(size_t)node * a.ld + j + q] : T(0);
    }
    *reinterpret_cast<TV*>(&sX[l][jj]) = val;
  }
  __syncthreads();
  const int wave = tid / 64, lane = tid % 64, lr = lane % 16, lk = lane / 16;
  const size_t cell = ex + (size_t)a.n * (ey + (size_t)a.n * ez);
  const T* Kc = K + cell * (size_t)MT * KS * 64 + lane;
  d4 acc[MTI][NTL];
#pragma unroll
  for (int i = 0; i < MTI; ++i)
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[i][t] = d4{0.0, 0.0, 0.0, 0.0};
  // tiles beyond MT (the last wavefronts' missing ones) read tile MT - 1 and are not stored
  const T* Km[MTI];
#pragma unroll
  for (int i = 0; i < MTI; ++i) Km[i] = Kc + (size_t)min(wave + NW * i, MT - 1) * KS * 64;
  // A fragments three steps ahead in registers (a ring of PFD slots per tile): one step ahead
  // leaves too few loads in flight to cover HBM latency (measured: 10 % slower at p = 5), and
  // three beat two by 5-7 % at 16 columns
  constexpr int PFD = 3;
  T an[PFD][MTI];
#pragma unroll
  for (int d = 0; d < PFD; ++d)
#pragma unroll
    for (int i = 0; i < MTI; ++i) an[d][i] = d < KS ? Km[i][(size_t)d * 64] : T(0);
  for (int k0 = 0; k0 < KS; k0 += PFD) {
#pragma unroll
    for (int d = 0; d < PFD; ++d) {
      const int ks = k0 + d;
      if (ks < KS) {
        double av[MTI], bv[NTL];
#pragma unroll
        for (int i = 0; i < MTI; ++i) av[i] = (double)an[d][i];
        if (ks + PFD < KS) {
#pragma unroll
          for (int i = 0; i < MTI; ++i) an[d][i] = Km[i][(size_t)(ks + PFD) * 64];
        }
#pragma unroll
        for (int t = 0; t < NTL; ++t) bv[t] = (double)sX[ks * 4 + lk][t * 16 + lr];
#pragma unroll
        for (int i = 0; i < MTI; ++i)
#pragma unroll
          for (int t = 0; t < NTL; ++t) acc[i][t] = mfma16(av[i], bv[t], acc[i][t]);
      }
    }
  }
  // The output in two phases for 16-column chunks, and for FP64 at p >= 4, whose LDS block
  // already limits a CU to the workgroups the extra registers allow. Otherwise per element:
  // holding the loaded values beside the accumulators would cost workgroups per CU (FP32,
  // p = 5, 64 columns: 10.1 ms in two phases against 8.2 ms per element).
  constexpr bool kBatchOut = NTL == 1 || (sizeof(T) == 8 && P >= 4);
  if constexpr (kBatchOut) {
    // Every load (the column constants, v, Z for the first class, Y for the others) is
    // issued before the first store and no load follows a store: memory operations are counted
    // in order, so a wait for a load issued after a store would also wait for that store, one
    // round trip per element. Loads of entries that are not written read a valid address (index
    // 0) and are discarded.
    double cs[NTL], sh[NTL];
#pragma unroll
    for (int t = 0; t < NTL; ++t) {
      const int j = j0 + t * 16 + lr;
      const int jc = j < a.nv ? j : 0;
      cs[t] = a.alpha * (a.colscale ? a.colscale[jc] : 1.0);
      sh[t] = a.cshift + (a.has_colshift ? a.colshift[jc] : 0.0);
    }
    long long onode[MTI][4];
    bool ofirst[MTI][4];
    double vn[MTI][4];
    double old[MTI][NTL][4];
#pragma unroll
    for (int i = 0; i < MTI; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int mt = wave + NW * i;
        const int row = mt * 16 + lk + 4 * r;
        const bool rok = mt < MT && row < NP;
        onode[i][r] = rok ? sNode[row] : -1;
        ofirst[i][r] = rok && sFirst[row];
        vn[i][r] = a.v[onode[i][r] >= 0 ? onode[i][r] : 0];
      }
#pragma unroll
    for (int i = 0; i < MTI; ++i)
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + t * 16 + lr;
          const bool ok = onode[i][r] >= 0 && j < a.nv;
          const size_t idx = ok ? (size_t)onode[i][r] * a.ld + j : 0;
          // the first class reads beta Z (Y may alias Z: read before any store), the others Y
          const T* src = ofirst[i][r] ? Z : Y;
          old[i][t][r] = (src != nullptr) ? (double)src[idx] : 0.0;
        }
    // every value first (the empty asm keeps the compiler from moving the arithmetic into the
    // conditional stores below, where it would wait on the loads again after each store)
#pragma unroll
    for (int i = 0; i < MTI; ++i)
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min((wave + NW * i) * 16 + lk + 4 * r, NP - 1);
          // the node's first class also adds the diagonal and Chebyshev terms: Y = alpha cs_j
          // ((K~/2) X + (v - c - s_j) X) + beta Z
          const double yf = cs[t] * (acc[i][t][r] + (vn[i][r] - sh[t]) * (double)sX[row][t * 16 + lr]) +
                            (Z ? a.beta * old[i][t][r] : 0.0);
          double y = ofirst[i][r] ? yf : old[i][t][r] + cs[t] * acc[i][t][r];
          asm volatile("" : "+v"(y));
          old[i][t][r] = y;
        }
#pragma unroll
    for (int i = 0; i < MTI; ++i)
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = j0 + t * 16 + lr;
          if (onode[i][r] >= 0 && j < a.nv) Y[(size_t)onode[i][r] * a.ld + j] = (T)old[i][t][r];
        }
  } else {
#pragma unroll
    for (int i = 0; i < MTI; ++i) {
      const int mt = wave + NW * i;
      if (mt >= MT) continue;
#pragma unroll
      for (int t = 0; t < NTL; ++t) {
        const int j = j0 + t * 16 + lr;
        if (j >= a.nv) continue;
        const double cs = a.alpha * (a.colscale ? a.colscale[j] : 1.0);
        const double sh = a.cshift + (a.has_colshift ? a.colshift[j] : 0.0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = mt * 16 + lk + 4 * r;
          if (row >= NP) continue;
          const long long node = sNode[row];
          if (node < 0) continue;
          const size_t idx = (size_t)node * a.ld + j;
          if (sFirst[row]) {
            // the node's first class also adds the diagonal and Chebyshev terms: Y = alpha cs_j
            // ((K~/2) X + (v - c - s_j) X) + beta Z (Y may alias Z: Z is read first)
            double y = cs * (acc[i][t][r] + (a.v[node] - sh) * (double)sX[row][t * 16 + lr]);
            if (Z) y += a.beta * (double)Z[idx];
            Y[idx] = (T)y;
          } else {
            Y[idx] = (T)((double)Y[idx] + cs * acc[i][t][r]);
          }
        }
      }
    }
  }
}

// Sixteen wavefronts when a cell has 12 or more M-tiles (p = 5: one tile each, 22 % faster at
// 64 columns, the MFMA-bound case); eight instead of four when it has 8 or more (p = 4: up to
// 21 % faster at 64 columns and 7 % at 16 FP32 columns), when a workgroup's LDS block exceeds
// 80 KB (one workgroup per CU) or when four wavefronts would each hold more than 8 accumulator
// tiles.
template <typename T, int P, int NTL>
fe_status launch_class(MapApply& a, long long grid, hipStream_t s) {
  constexpr int NP = (P + 1) * (P + 1) * (P + 1), NP4 = (NP + 3) / 4 * 4, MT = (NP + 15) / 16;
  constexpr int JC = 16 * NTL, JP = JC + ((JC == 32 || (JC == 64 && sizeof(T) == 4)) ? 16 : 0);
  constexpr int NT = MT >= 12 ? 1024 : (MT >= 8 || (size_t)NP4 * JP * sizeof(T) > 80 * 1024 || ((MT + 3) / 4) * NTL > 8) ? 512 : 256;
  hipLaunchKernelGGL((mapped_cell_kernel<T, P, NTL, NT>), dim3((unsigned)grid), dim3(NT), 0, s, a);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

template <typename T, int P>
fe_status launch_cells(const Mesh& m, MapApply& a, hipStream_t s) {
  // columns in chunks of at most 64: the matrices stream once per chunk
  const int ntl = std::min(4, (a.nv + 15) / 16);
  a.jchunks = (a.nv + 16 * ntl - 1) / (16 * ntl);
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        a.cx = cx;
        a.cy = cy;
        a.cz = cz;
        a.ncx = (m.n - cx + 1) / 2;
        a.ncy = (m.n - cy + 1) / 2;
        const int ncz = (m.n - cz + 1) / 2;
        const long long grid = (long long)a.ncx * a.ncy * ncz * a.jchunks;
        if (grid == 0) continue;
        fe_status st;
        switch (ntl) {
          case 1: st = launch_class<T, P, 1>(a, grid, s); break;
          case 2: st = launch_class<T, P, 2>(a, grid, s); break;
          case 3: st = launch_class<T, P, 3>(a, grid, s); break;
          default: st = launch_class<T, P, 4>(a, grid, s); break;
        }
        if (st != FE_OK) return st;
      }
  return FE_OK;
}

template <typename T>
fe_status launch_mapped_typed(const Mesh& m, MapApply& a, hipStream_t s) {
  switch (m.p) {
    case 1: return launch_cells<T, 1>(m, a, s);
    case 2: return launch_cells<T, 2>(m, a, s);
    case 3: return launch_cells<T, 3>(m, a, s);
    case 4: return launch_cells<T, 4>(m, a, s);
    case 5: return launch_cells<T, 5>(m, a, s);
    default: return fail(FE_EINVAL, "ks_apply: mapped meshes support p <= 5");
  }
}

// host Lagrange tables on the GLL nodes: values and derivatives at points x
void lagrange_at(const double* nodes, int k, const double* x, int m, double* val, double* der) {
  for (int q = 0; q < m; ++q)
    for (int i = 0; i < k; ++i) {
      double v = 1.0, d = 0.0;
      for (int j = 0; j < k; ++j) {
        if (j == i) continue;
        const double f = (x[q] - nodes[j]) / (nodes[i] - nodes[j]);
        d = d * f + v / (nodes[i] - nodes[j]);
        v *= f;
      }
      val[q * k + i] = v;
      der[q * k + i] = d;
    }
}

template <int P>
fe_status setup_typed(Mesh& m, const MapGeom& g, const MapTables& t, hipStream_t s) {
  constexpr int P1 = P + 1, NP = P1 * P1 * P1;
  const int q = t.q, q3 = q * q * q;
  const int NP16 = (NP + 15) / 16 * 16;
  const int KR = 3 * q3, KP = (KR + 3) / 4 * 4;
  const long long nc = (long long)m.n * m.n * m.n;
  // Abar[(q, d)][a]: reference gradients at the Gauss points
  std::vector<double> Ab((size_t)KP * NP16, 0.0);
  for (int qq = 0; qq < q3; ++qq) {
    const int qx = qq % q, qy = (qq / q) % q, qz = qq / (q * q);
    for (int a = 0; a < NP; ++a) {
      const int i = a % P1, j = (a / P1) % P1, k = a / (P1 * P1);
      const double bx = t.Bq[qx * P1 + i], by = t.Bq[qy * P1 + j], bz = t.Bq[qz * P1 + k];
      Ab[(size_t)(3 * qq + 0) * NP16 + a] = t.Dq[qx * P1 + i] * by * bz;
      Ab[(size_t)(3 * qq + 1) * NP16 + a] = bx * t.Dq[qy * P1 + j] * bz;
      Ab[(size_t)(3 * qq + 2) * NP16 + a] = bx * by * t.Dq[qz * P1 + k];
    }
  }
  double *dA = nullptr, *dK = nullptr, *dW = nullptr, *dB = nullptr;
  int* dflag = nullptr;
  auto cleanup = [&]() {
    if (dA) (void)hipFree(dA);
    if (dK) (void)hipFree(dK);
    if (dW) (void)hipFree(dW);
    if (dB) (void)hipFree(dB);
    if (dflag) (void)hipFree(dflag);
  };
  hipError_t e = hipMalloc(&dA, Ab.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&dK, (size_t)nc * NP * NP * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&dW, (size_t)nc * NP * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&dB, (size_t)nc * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&dflag, sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(dA, Ab.data(), Ab.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(dflag, 0, sizeof(int));
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "mapped mesh set-up");
  }
  const size_t lds = (size_t)q3 * 6 * sizeof(double);
  hipLaunchKernelGGL((mapped_element_kernel<P>), dim3((unsigned)nc), dim3(kMapThreads), lds, s, g, t, dA, KP, NP16,
                     dK, dW, dflag);
  e = hipGetLastError();
  const unsigned gn = (unsigned)std::min<long long>((m.nf + 255) / 256, 1 << 16);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((mapped_node_kernel<P>), dim3(gn), dim3(256), 0, s, g, t, dK, dW, m.d_wn, m.d_kdn, m.d_xyz);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL((mapped_scale_kernel<P>), dim3((unsigned)nc), dim3(kMapThreads), 0, s, g, dK, dW, m.d_wn,
                       m.map_mt, m.map_ks, m.d_Ke64, m.d_Ke32, dB);
    e = hipGetLastError();
  }
  int flag = 0;
  std::vector<double> bnd(nc);
  if (e == hipSuccess) e = hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(bnd.data(), dB, nc * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "mapped mesh set-up");
  if (flag) return fail(FE_EINVAL, "fe_mesh_create_mapped: the map inverts a cell (det J <= 0); use a smaller amp");
  m.kin_bound = *std::max_element(bnd.begin(), bnd.end());
  return FE_OK;
}

}  // namespace

fe_status mapped_setup(Mesh& m, double amp) {
  const int p = m.p, P1 = p + 1;
  if (p > 5) return fail(FE_EINVAL, "fe_mesh_create_mapped: p must be in [1, 5]");
  MapGeom g{p, m.n, p * m.n + 1, m.n1, m.L, m.h, amp};
  MapTables t{};
  gll_rule(p, t.xi, t.wg);
  t.q = (3 * p + 2) / 2;   // ceil((3p + 1)/2)
  double xq[kMaxQ];
  gauss_rule(t.q, xq, t.wq);
  std::vector<double> dv(P1 * P1);
  lagrange_at(t.xi, P1, t.xi, P1, dv.data(), t.Dg);
  lagrange_at(t.xi, P1, xq, t.q, t.Bq, t.Dq);
  const int NP = P1 * P1 * P1;
  m.map_mt = (NP + 15) / 16;
  m.map_ks = (NP + 3) / 4;
  const long long nc = (long long)m.n * m.n * m.n;
  const size_t nfrag = (size_t)nc * m.map_mt * m.map_ks * 64;
  hipError_t e = hipMalloc(&m.d_wn, m.nf * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_kdn, m.nf * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_xyz, 3 * m.nf * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_Ke64, nfrag * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&m.d_Ke32, nfrag * sizeof(float));
  if (e != hipSuccess) return hip_fail(e, "fe_mesh_create_mapped: device allocation");
  hipStream_t s = nullptr;
  switch (p) {
    case 1: return setup_typed<1>(m, g, t, s);
    case 2: return setup_typed<2>(m, g, t, s);
    case 3: return setup_typed<3>(m, g, t, s);
    case 4: return setup_typed<4>(m, g, t, s);
    default: return setup_typed<5>(m, g, t, s);
  }
}

fe_status launch_apply_mapped(const Mesh& m, const ApplyArgs& aa, fe_prec prec, hipStream_t s) {
  MapApply a;
  std::memset(&a, 0, sizeof(a));
  a.X = aa.X;
  a.Y = aa.Y;
  a.Z = aa.Z;
  a.v = aa.v;
  a.colscale = aa.d_colscale;
  a.n = m.n;
  a.n1 = m.n1;
  a.nv = aa.nv;
  a.ld = aa.ld;
  a.MT = m.map_mt;
  a.KS = m.map_ks;
  a.alpha = aa.alpha;
  a.beta = aa.beta;
  a.cshift = aa.cshift;
  if (aa.colshift) {
    if (aa.nv > kMaxShiftCols) return fail(FE_EINVAL, "ks_apply: per-column shifts limited to 256 columns");
    a.has_colshift = 1;
    for (int j = 0; j < aa.nv; ++j) a.colshift[j] = aa.colshift[j];
  }
  if (prec == FE_F64) {
    a.K = m.d_Ke64;
    return launch_mapped_typed<double>(m, a, s);
  }
  if (prec == FE_F32) {
    a.K = m.d_Ke32;
    return launch_mapped_typed<float>(m, a, s);
  }
  return fail(FE_EINVAL, "ks_apply: mapped meshes take FE_F64 or FE_F32 blocks");
}

size_t mapped_matrix_bytes(const Mesh& m, fe_prec prec) {
  const size_t nfrag = (size_t)m.n * m.n * m.n * m.map_mt * m.map_ks * 64;
  return nfrag * (prec == FE_F64 ? sizeof(double) : sizeof(float));
}

}  // namespace invdft
