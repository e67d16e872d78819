// Matrix-free spectral-FE Kohn-Sham operator on node-major blocks (gfx950).
//
//   Y = alpha * ( (1/2) W^{-1/2} K W^{-1/2} X + (v - c - s_j) X ) + beta * Z
//
// The paper's operator (Eqs. 17, 19; Sec. 3.2.3) is a sum of per-cell dense
// products K_e X_e followed by an assembly. On a tensor-product mesh the exact
// element stiffness is K_e = (h/2)(K^ (x) M^ (x) M^ + M^ (x) K^ (x) M^ + M^ (x) M^ (x) K^)
// (Eq. 12's basis is a tensor product), and the W^{-1/2} scaling factorises per
// axis, so the assembled operator is
//   K~ = K~1 (x) M~ (x) M~ + M~ (x) K~1 (x) M~ + M~ (x) M~ (x) K~1
// with 1-D banded assembled matrices built from one scaled (p+1)x(p+1) element
// pair (mt, kt). The kernel applies it by sum factorisation: six 1-D
// contractions instead of one (p+1)^3 x (p+1)^3 dense product per cell, which
// makes the apply bound by HBM instead of by FP64 matrix throughput.
//
// One workgroup owns an xy-tile of BXE x BYE cells (its nodes [e0 p, (e0+B) p) on
// each axis), J consecutive columns of the block, and a range of cells along z,
// which it marches through plane by plane:
//   x-pass  (global -> LDS): U1 = M~x X, U2 = K~x X on the tile's rows plus the
//                            y-halo, owner-computes (a vertex sums both cells);
//   y-pass  (LDS -> LDS)   : A = M~y U1, B = M~y U2 + K~y U1 on owned nodes;
//   z-step  (registers)    : each owned (x, y, j) column accumulates
//                            M~z B + K~z A for the p+1 output planes of the
//                            current cell and carries the shared top vertex
//                            plane into the next cell.
// Every output is written exactly once by its owner, so there are no atomics
// and the result is bitwise reproducible. Dirichlet nodes are zero.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "internal.h"
#include "ref_tables.h"

namespace invdft {

struct KParams {
  const void* X;
  void* Y;
  const void* Z;
  const double* v;
  const double* colscale;   // device, nv entries, or null
  int n, n1, nv, ld;
  int zseg, tiles_x, tiles_y, jchunks, zsegs;
  int has_colshift;
  double alpha, beta, cshift;
  double kscale;  // 1/(2 h^2): the kinetic accumulators hold 2 h^2 K~/2 X
  double dscale;  // 2 h^2: the diagonal term is stored in the same units
  // graded meshes only (h is then the smallest cell): per 1-D cell e, the stiffness
  // factor (h/h_e)^2 and the end-node factors of the W^{-1/2} scaling relative to the
  // uniform tables, sqrt(2 h_e / (h_e + h_neighbour)) on the left and right
  const double* ckap;
  const double* cgl;
  const double* cgr;
  double colshift[kMaxShiftCols];
};

// Storage and arithmetic types: FP64 and FP32 blocks are computed in their own precision;
// bf16 blocks (FE_BF16: bit patterns of the upper half of an FP32) are widened to FP32 on
// load and rounded to nearest even on store.
template <typename T>
struct Calc {
  using type = T;
};
template <>
struct Calc<bf16_t> {
  using type = float;
};
template <typename T>
__device__ __forceinline__ typename Calc<T>::type widen(T x) {
  return x;
}
template <>
__device__ __forceinline__ float widen<bf16_t>(bf16_t x) {
  return __uint_as_float((unsigned)x << 16);
}
template <typename T>
__device__ __forceinline__ T narrow(typename Calc<T>::type x) {
  return x;
}
template <>
__device__ __forceinline__ bf16_t narrow<bf16_t>(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}

// Tile shape per order: BEX x BEY cells per workgroup in x and y (a z-range of
// cells is marched), chosen by measurement. Larger tiles read less halo per owned
// node but cost LDS and registers: at P = 5 in FP64 the 2 x 2 tile takes about
// 62 KB of LDS and 225 VGPRs, two workgroups per CU.
template <int P, typename T>
struct TileShape {
  static constexpr int BEX = (P == 1) ? 4 : (P == 2) ? 4 : (P <= 5) ? 2 : 1;
  static constexpr int BEY = (P == 1) ? 4 : (P <= 5) ? 2 : 1;
};

// Distinct entries of a symmetric, centrosymmetric (P+1)x(P+1) matrix: slot of (i, k).
template <int P>
struct Canon {
  static constexpr int rep(int i, int k) {
    int a = i < k ? i : k, b = i < k ? k : i;
    const int a2 = P - b, b2 = P - a;
    if (a2 < a || (a2 == a && b2 < b)) {
      a = a2;
      b = b2;
    }
    return a * (P + 1) + b;
  }
  struct Map {
    int slot[P + 1][P + 1];
    int rep_of[(P + 1) * (P + 1)];
    int count;
  };
  static constexpr Map make() {
    Map m{};
    int seen[(P + 1) * (P + 1)] = {};
    for (int q = 0; q < (P + 1) * (P + 1); ++q) seen[q] = -1;
    m.count = 0;
    for (int i = 0; i <= P; ++i)
      for (int k = 0; k <= P; ++k) {
        const int r = rep(i, k);
        if (seen[r] < 0) {
          seen[r] = m.count;
          m.rep_of[m.count] = r;
          ++m.count;
        }
        m.slot[i][k] = seen[r];
      }
    return m;
  }
  static constexpr Map map = make();
  static constexpr int N = map.count;
};

// Logical block order: column chunk fastest, then tile x, tile y, z-segment.
// The hardware deals consecutive block ids round-robin to the 8 XCDs; this
// remap gives each XCD a contiguous range of logical ids, so the column chunks
// of one tile and its neighbour tiles share that XCD's L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nblk) {
  const int q = nblk / 8, r = nblk % 8;
  const int x = b % 8, i = b / 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + i;
}

// acc[c][i] += m~(i, k) b_c + k~ref(i, k) a_c (+ d_c for i = k), for the block-uniform
// plane index k, unrolled per value of k so that every coefficient is a compile-time
// constant of the unit-cell tables.
template <typename CT, int P, int CPT, int NU, int K>
__device__ __forceinline__ void z_acc_k(const CT (&cM)[NU], const CT (&cK)[NU], CT (&acc)[CPT][P + 1],
                                        const CT (&av)[CPT], const CT (&bv)[CPT], const CT (&dv)[CPT]) {
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
#pragma unroll
    for (int i = 0; i <= P; ++i) {
      acc[c][i] = fma(cM[Canon<P>::map.slot[i][K]], bv[c], acc[c][i]);
      acc[c][i] = fma(cK[Canon<P>::map.slot[i][K]], av[c], acc[c][i]);
    }
    acc[c][K] += dv[c];
  }
}

template <typename CT, int P, int CPT, int NU, int K = 0>
__device__ __forceinline__ void z_accumulate(int k, const CT (&cM)[NU], const CT (&cK)[NU], CT (&acc)[CPT][P + 1],
                                             const CT (&av)[CPT], const CT (&bv)[CPT], const CT (&dv)[CPT]) {
  if constexpr (K <= P) {
    if (k == K)
      z_acc_k<CT, P, CPT, NU, K>(cM, cK, acc, av, bv, dv);
    else
      z_accumulate<CT, P, CPT, NU, K + 1>(k, cM, cK, acc, av, bv, dv);
  }
}

// Graded cell: the element pair is g_i g_k (m~(i, k), kap k~ref(i, k)) with g = gl at node 0,
// gr at node P and 1 inside. Plane k contributes g_i g_k (m~ b + kap k~ a) to output i; the
// diagonal term is a nodal quantity and is not scaled.
template <typename CT, int P, int CPT, int NU, int K>
__device__ __forceinline__ void z_acc_k_graded(const CT (&cM)[NU], const CT (&cK)[NU], CT (&acc)[CPT][P + 1],
                                               const CT (&av)[CPT], const CT (&bv)[CPT], const CT (&dv)[CPT],
                                               CT kap, CT gl, CT gr) {
  const CT gk = (K == 0) ? gl : ((K == P) ? gr : CT(1));
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const CT b = gk * bv[c];
    const CT a = gk * kap * av[c];
#pragma unroll
    for (int i = 0; i <= P; ++i) {
      CT t = cM[Canon<P>::map.slot[i][K]] * b;
      t = fma(cK[Canon<P>::map.slot[i][K]], a, t);
      if (i == 0) t *= gl;
      if (i == P) t *= gr;
      acc[c][i] += t;
    }
    acc[c][K] += dv[c];
  }
}

template <typename CT, int P, int CPT, int NU, int K = 0>
__device__ __forceinline__ void z_accumulate_graded(int k, const CT (&cM)[NU], const CT (&cK)[NU],
                                                    CT (&acc)[CPT][P + 1], const CT (&av)[CPT], const CT (&bv)[CPT],
                                                    const CT (&dv)[CPT], CT kap, CT gl, CT gr) {
  if constexpr (K <= P) {
    if (k == K)
      z_acc_k_graded<CT, P, CPT, NU, K>(cM, cK, acc, av, bv, dv, kap, gl, gr);
    else
      z_accumulate_graded<CT, P, CPT, NU, K + 1>(k, cM, cK, acc, av, bv, dv, kap, gl, gr);
  }
}

template <typename T, int P, int J, int NT, bool GR>
__global__ __launch_bounds__(NT) void ks_apply_kernel(const KParams prm) {
  using CT = typename Calc<T>::type;  // compute type: the storage type, FP32 for bf16 storage
  constexpr int P1 = P + 1;
  constexpr int BEX = TileShape<P, T>::BEX, BEY = TileShape<P, T>::BEY;
  constexpr int BX = BEX * P, BY = BEY * P;  // owned nodes per tile edge
  constexpr int NYI = (BEY + 1) * P + 1;     // input rows (owned + halo)
  constexpr int NXN = (BEX + 1) * P + 1;     // input nodes per row (owned + halo)
  constexpr int NXI = BEX * NYI * J;         // x-pass items
  constexpr int NYP = BX * BEY * J;          // y-pass items
  constexpr int NCOL = BX * BY * J;          // owned (x, y, column) z-columns
  constexpr int CPT = (NCOL + NT - 1) / NT;
  constexpr int EPC = 16 / sizeof(T);        // elements per 16-byte chunk
  constexpr int CPN = J / EPC;               // chunks per node
  constexpr int NCHUNK = NYI * NXN * CPN;    // 16-byte chunks of one input plane
  constexpr int LPT = (NCHUNK + NT - 1) / NT;
  constexpr int NVO = BX * BY;               // owned nodes (potential values)
  constexpr int VPT = (NVO + NT - 1) / NT;
  static_assert(J % EPC == 0, "column chunk must be a whole number of 16-byte pieces");

  typedef T T16 __attribute__((ext_vector_type(EPC)));
  __shared__ __attribute__((aligned(16))) CT sIn[NYI][NXN][J];  // raw input plane
  __shared__ CT sU1[NYI][BX][J];
  __shared__ CT sU2[NYI][BX][J];
  __shared__ CT sA[BY][BX][J];
  __shared__ CT sB[BY][BX][J];
  __shared__ CT sD[2][BY][BX][J];            // diagonal term (v - c - s_j) x, double-buffered
  __shared__ double sV[BY][BX];              // potential at the owned nodes of the plane

  const T* __restrict__ X = static_cast<const T*>(prm.X);
  T* Y = static_cast<T*>(prm.Y);  // may alias Z, never X
  const T* Z = static_cast<const T*>(prm.Z);
  const int tid = threadIdx.x;
  const int n = prm.n, n1 = prm.n1, ld = prm.ld, nv = prm.nv;
  const int pn = P * n;

  int bid = xcd_logical_block(blockIdx.x, gridDim.x);
  const int jc = bid % prm.jchunks;
  bid /= prm.jchunks;
  const int tx = bid % prm.tiles_x;
  bid /= prm.tiles_x;
  const int ty = bid % prm.tiles_y;
  const int zs = bid / prm.tiles_y;
  const int ex0 = tx * BEX, ey0 = ty * BEY, j0 = jc * J;
  const int ez0 = zs * prm.zseg;
  const int ez1 = min(n, ez0 + prm.zseg);
  const int ezs = (ez0 > 0) ? ez0 - 1 : 0;
  // 16-byte vector loads need the chunk start aligned: ld a multiple of EPC (j0 is)
  const bool vec_ok = (ld % EPC) == 0;

  auto node_ok = [&](int g) { return g >= 1 && g <= pn - 1; };
  auto node_index = [&](int gx, int gy, int gz) -> long long {
    return (long long)(gx - 1) + (long long)n1 * ((long long)(gy - 1) + (long long)n1 * (gz - 1));
  };
  // Coefficients. FP32: compile-time literals. FP64 (no 64-bit literal operands): the
  // distinct entries are read once from an LDS table into registers, so the loop does
  // not hold 2 x NU doubles in scalar registers.
  constexpr int NU = Canon<P>::N;
  __shared__ double sTab[2][NU];
  if constexpr (sizeof(CT) == sizeof(double)) {
    for (int q = tid; q < 2 * NU; q += NT) {
      const int r = Canon<P>::map.rep_of[q % NU];
      sTab[q / NU][q % NU] = (q < NU) ? ref::Table<P>::value.mt[r / (P + 1)][r % (P + 1)]
                                      : ref::Table<P>::value.kt[r / (P + 1)][r % (P + 1)];
    }
    __syncthreads();
  }
  CT cM[NU], cK[NU];
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    if constexpr (sizeof(CT) == sizeof(double)) {
      // split: mass entries stay scalar (uniform), stiffness entries in vector registers
      const int r = Canon<P>::map.rep_of[q];
      cM[q] = (CT)ref::Table<P>::value.mt[r / (P + 1)][r % (P + 1)];
      cK[q] = sTab[1][q];
    } else {
      const int r = Canon<P>::map.rep_of[q];
      cM[q] = (CT)ref::Table<P>::value.mt[r / (P + 1)][r % (P + 1)];
      cK[q] = (CT)ref::Table<P>::value.kt[r / (P + 1)][r % (P + 1)];
    }
  }
  auto MT = [&](int i, int k) { return cM[Canon<P>::map.slot[i][k]]; };
  auto KT = [&](int i, int k) { return cK[Canon<P>::map.slot[i][k]]; };

  // graded meshes: factors (kap, gl, gr) of the tile's x- and y-cells and their left
  // neighbours in LDS, sFac[axis][q][kind] for cell e0 - 1 + q (cells outside the mesh only
  // meet zero inputs; their entries are clamped copies)
  constexpr int NFQ = (BEX > BEY ? BEX : BEY) + 1;
  __shared__ CT sFac[2][NFQ][3];
  auto cell_factors = [&](int e, CT& kap, CT& gl, CT& gr) {
    const int ec = e < 0 ? 0 : (e >= n ? n - 1 : e);
    kap = (CT)prm.ckap[ec];
    gl = (CT)prm.cgl[ec];
    gr = (CT)prm.cgr[ec];
  };
  if constexpr (GR) {
    if (tid < 2 * NFQ) {
      const int ax = tid / NFQ, q = tid % NFQ;
      cell_factors((ax == 0 ? ex0 : ey0) - 1 + q, sFac[ax][q][0], sFac[ax][q][1], sFac[ax][q][2]);
    }
  }

  // ---- plane loader: non-redundant 16-byte chunks into registers (prefetch), then LDS.
  // The (x, y, column) part of every chunk's address is the same on all planes.
  T16 pre[LPT];
  double vpre[VPT];
  int coff[LPT];   // element offset of the chunk in plane gz = 1, or -1 when outside
  int cfull[LPT];        // 1: whole chunk in range and 16-byte aligned
  int voff[VPT];
  const long long plane_stride = (long long)n1 * n1;
#pragma unroll
  for (int t = 0; t < LPT; ++t) {
    const int c = tid + t * NT;
    coff[t] = -1;
    cfull[t] = 0;
    if (c < NCHUNK) {
      const int part = c % CPN;
      const int r = c / CPN;
      const int gx = ex0 * P - P + r % NXN, gy = ey0 * P - P + r / NXN;
      const int jb = j0 + part * EPC;
      if (node_ok(gx) && node_ok(gy) && jb < nv) {
        coff[t] = (int)(node_index(gx, gy, 1) * ld + jb);
        cfull[t] = (vec_ok && jb + EPC <= nv) ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < VPT; ++t) {
    const int o = tid + t * NT;
    voff[t] = -1;
    if (o < NVO) {
      const int gx = ex0 * P + o % BX, gy = ey0 * P + o / BX;
      if (node_ok(gx) && node_ok(gy)) voff[t] = (int)node_index(gx, gy, 1);
    }
  }
  auto load_plane = [&](int gz) {
    const bool zok = node_ok(gz);
    const long long zo = (long long)(gz - 1) * plane_stride;
    const T* Xz = X + zo * ld;
    const double* vz = prm.v + zo;
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
      T16 val;
#pragma unroll
      for (int e = 0; e < EPC; ++e) val[e] = T(0);
      if (zok && coff[t] >= 0) {
        const T* src = Xz + coff[t];
        if (cfull[t]) {
          val = *reinterpret_cast<const T16*>(src);
        } else {
          const int jb = coff[t] % ld;
#pragma unroll
          for (int e = 0; e < EPC; ++e) val[e] = (jb + e < nv) ? src[e] : T(0);
        }
      }
      pre[t] = val;
    }
#pragma unroll
    for (int t = 0; t < VPT; ++t) vpre[t] = (zok && voff[t] >= 0) ? vz[voff[t]] : 0.0;
  };
  auto store_plane = [&]() {
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
      const int c = tid + t * NT;
      if (c < NCHUNK) {
        const int part = c % CPN;
        const int r = c / CPN;
        if constexpr (sizeof(T) == sizeof(CT)) {
          *reinterpret_cast<T16*>(&sIn[r / NXN][r % NXN][part * EPC]) = pre[t];
        } else {
#pragma unroll
          for (int e = 0; e < EPC; ++e) sIn[r / NXN][r % NXN][part * EPC + e] = widen<T>(pre[t][e]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < VPT; ++t) {
      const int o = tid + t * NT;
      if (o < NVO) sV[o / BX][o % BX] = vpre[t];
    }
  };

  // Column constants of this thread, read once: every x-pass item and z-column of a thread
  // has the column tid % J (NT is a multiple of J). A global load of them inside the plane
  // loop would make the wave wait for the plane prefetch in flight as well (memory loads
  // complete in order), leaving the prefetch nothing to overlap.
  static_assert(NT % J == 0, "a thread's items share one column");
  const int jt = j0 + tid % J;
  const double sh_t = prm.cshift + ((prm.has_colshift && jt < nv) ? prm.colshift[jt] : 0.0);
  const CT cs_t = (CT)(prm.kscale * prm.alpha) * ((prm.colscale && jt < nv) ? (CT)prm.colscale[jt] : CT(1));

  // per-thread z-column accumulators: outputs of the P+1 planes of the current cell
  CT acc[CPT][P1];
#pragma unroll
  for (int c = 0; c < CPT; ++c)
#pragma unroll
    for (int i = 0; i <= P; ++i) acc[c][i] = 0;

  const int gz0 = ezs * P, gz1 = ez1 * P;
  load_plane(gz0);
  store_plane();
  __syncthreads();
  int buf = 0;
#pragma unroll 1
  for (int gz = gz0; gz <= gz1; ++gz) {
    // prefetch, in flight during this plane's passes. Issued and stored on every plane (after
    // the last, plane 0: zeros, no memory access), so that no load is pending across the
    // loop's back edge and the next plane's loads do not wait for this plane's stores.
    load_plane(gz < gz1 ? gz + 1 : 0);
    // ---- x-pass (LDS -> LDS): U1 = M~x X, U2 = K~x X on owned x, all NYI rows; diagonal term
    for (int item = tid; item < NXI; item += NT) {
      const int jj = item % J;
      const int r = item / J;
      const int exl = r % BEX;
      const int yl = r / BEX;
      CT in[2 * P + 1];
#pragma unroll
      for (int k = 0; k <= 2 * P; ++k) in[k] = sIn[yl][exl * P + k][jj];
      if constexpr (!GR) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
          CT u1 = MT(i, 0) * in[P], u2 = KT(i, 0) * in[P];
#pragma unroll
          for (int k = 1; k <= P; ++k) {
            u1 = fma(MT(i, k), in[P + k], u1);
            u2 = fma(KT(i, k), in[P + k], u2);
          }
          if (i == 0) {  // shared vertex: the left cell's row P as well
#pragma unroll
            for (int k = 0; k <= P; ++k) {
              u1 = fma(MT(P, k), in[k], u1);
              u2 = fma(KT(P, k), in[k], u2);
            }
          }
          sU1[yl][exl * P + i][jj] = u1;
          sU2[yl][exl * P + i][jj] = u2;
        }
      } else {
        // this cell (factors q = exl + 1) on in[P..2P], its left neighbour (q = exl) on in[0..P]
        const CT kc = sFac[0][exl + 1][0], glc = sFac[0][exl + 1][1], grc = sFac[0][exl + 1][2];
        const CT kl = sFac[0][exl][0], grl = sFac[0][exl][2];
        const CT e0 = glc * in[P], eP = grc * in[2 * P];
        const CT l0 = sFac[0][exl][1] * in[0], lP = grl * in[P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
          CT u1 = MT(i, 0) * e0, u2 = KT(i, 0) * e0;
#pragma unroll
          for (int k = 1; k < P; ++k) {
            u1 = fma(MT(i, k), in[P + k], u1);
            u2 = fma(KT(i, k), in[P + k], u2);
          }
          u1 = fma(MT(i, P), eP, u1);
          u2 = kc * fma(KT(i, P), eP, u2);
          if (i == 0) {  // shared vertex: the left cell's row P, with that cell's factors
            CT w1 = MT(P, 0) * l0, w2 = KT(P, 0) * l0;
#pragma unroll
            for (int k = 1; k < P; ++k) {
              w1 = fma(MT(P, k), in[k], w1);
              w2 = fma(KT(P, k), in[k], w2);
            }
            w1 = fma(MT(P, P), lP, w1);
            w2 = kl * fma(KT(P, P), lP, w2);
            u1 = fma(glc, u1, grl * w1);
            u2 = fma(glc, u2, grl * w2);
          }
          sU1[yl][exl * P + i][jj] = u1;
          sU2[yl][exl * P + i][jj] = u2;
        }
      }
      if (yl >= P && yl < P + BY) {
#pragma unroll
        for (int i = 0; i < P; ++i)
          sD[buf][yl - P][exl * P + i][jj] = (CT)(prm.dscale * (sV[yl - P][exl * P + i] - sh_t) * (double)in[P + i]);
      }
    }
    __syncthreads();
    // ---- y-pass: A = M~y U1, B = M~y U2 + K~y U1 on owned nodes
    for (int item = tid; item < NYP; item += NT) {
      const int jj = item % J;
      const int r = item / J;
      const int xl = r % BX;
      const int eyl = r / BX;
      CT a1[2 * P + 1], a2[2 * P + 1];
#pragma unroll
      for (int k = 0; k <= 2 * P; ++k) {
        a1[k] = sU1[eyl * P + k][xl][jj];
        a2[k] = sU2[eyl * P + k][xl][jj];
      }
      if constexpr (!GR) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
          CT A = MT(i, 0) * a1[P], B = MT(i, 0) * a2[P];
          B = fma(KT(i, 0), a1[P], B);
#pragma unroll
          for (int k = 1; k <= P; ++k) {
            A = fma(MT(i, k), a1[P + k], A);
            B = fma(MT(i, k), a2[P + k], B);
            B = fma(KT(i, k), a1[P + k], B);
          }
          if (i == 0) {
#pragma unroll
            for (int k = 0; k <= P; ++k) {
              A = fma(MT(P, k), a1[k], A);
              B = fma(MT(P, k), a2[k], B);
              B = fma(KT(P, k), a1[k], B);
            }
          }
          sA[eyl * P + i][xl][jj] = A;
          sB[eyl * P + i][xl][jj] = B;
        }
      } else {
        const CT kc = sFac[1][eyl + 1][0], glc = sFac[1][eyl + 1][1], grc = sFac[1][eyl + 1][2];
        const CT kl = sFac[1][eyl][0], gll = sFac[1][eyl][1], grl = sFac[1][eyl][2];
        const CT p0 = glc * a1[P], pP = grc * a1[2 * P], q0 = glc * a2[P], qP = grc * a2[2 * P];
#pragma unroll
        for (int i = 0; i < P; ++i) {
          CT A = MT(i, 0) * p0, Bm = MT(i, 0) * q0, Bk = KT(i, 0) * p0;
#pragma unroll
          for (int k = 1; k < P; ++k) {
            A = fma(MT(i, k), a1[P + k], A);
            Bm = fma(MT(i, k), a2[P + k], Bm);
            Bk = fma(KT(i, k), a1[P + k], Bk);
          }
          A = fma(MT(i, P), pP, A);
          Bm = fma(MT(i, P), qP, Bm);
          Bk = fma(KT(i, P), pP, Bk);
          CT B = fma(kc, Bk, Bm);
          if (i == 0) {
            const CT r0 = gll * a1[0], rP = grl * a1[P], s0 = gll * a2[0], sP = grl * a2[P];
            CT Al = MT(P, 0) * r0, Bml = MT(P, 0) * s0, Bkl = KT(P, 0) * r0;
#pragma unroll
            for (int k = 1; k < P; ++k) {
              Al = fma(MT(P, k), a1[k], Al);
              Bml = fma(MT(P, k), a2[k], Bml);
              Bkl = fma(KT(P, k), a1[k], Bkl);
            }
            Al = fma(MT(P, P), rP, Al);
            Bml = fma(MT(P, P), sP, Bml);
            Bkl = fma(KT(P, P), rP, Bkl);
            A = fma(glc, A, grl * Al);
            B = fma(glc, B, grl * fma(kl, Bkl, Bml));
          }
          sA[eyl * P + i][xl][jj] = A;
          sB[eyl * P + i][xl][jj] = B;
        }
      }
    }
    // the raw plane and potential were last read by this plane's x-pass (before the barrier above)
    store_plane();
    __syncthreads();
    // ---- z-step: plane gz is node k of the current cell (k = 0 only for the first plane).
    // The accumulators hold 2 h^2 times the output (unit-cell tables; kscale on output);
    // k is block-uniform, so the dispatch on it is a scalar branch.
    const int rel = gz - gz0;
    const int k = (rel == 0) ? 0 : ((rel - 1) % P) + 1;
    CT av[CPT], bv[CPT], dv[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = tid + c * NT;
      av[c] = bv[c] = dv[c] = 0;
      if (col >= NCOL) continue;
      const int jj = col % J;
      const int xl = (col / J) % BX;
      const int yl = col / (J * BX);
      av[c] = sA[yl][xl][jj];
      bv[c] = sB[yl][xl][jj];
      dv[c] = sD[buf][yl][xl][jj];
    }
    // graded meshes: factors of the current z-cell (plane gz is its node k) and of the next
    CT zk = 1, zl = 1, zr = 1, nk = 1, nl = 1, nr = 1;
    if constexpr (GR) {
      const int ezc = (rel == 0) ? ezs : ezs + (rel - 1) / P;
      cell_factors(ezc, zk, zl, zr);
      cell_factors(ezc + 1, nk, nl, nr);
      z_accumulate_graded<CT, P, CPT, NU>(k, cM, cK, acc, av, bv, dv, zk, zl, zr);
    } else {
      z_accumulate<CT, P, CPT, NU>(k, cM, cK, acc, av, bv, dv);
    }
    if (k == P) {
      // cell ez complete: planes ez P + i, i < P, are final
      const int ez = (rel - 1) / P + ezs;
      if (ez >= ez0) {
        // The outputs replace acc[c][0..P-1] in place. Every load of Z is issued before the
        // first store, and no load follows a store: memory operations are counted in order,
        // so a wait for a later load would also wait for every store before it. (Y may alias
        // Z element for element; each element's Z is read before any store.)
        const long long pstride = (long long)n1 * n1 * ld;
        long long obase[CPT];
        bool ook[CPT];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int col = tid + c * NT;
          const int jj = col % J;
          const int xl = (col / J) % BX;
          const int yl = col / (J * BX);
          const int gx = ex0 * P + xl, gy = ey0 * P + yl, j = j0 + jj;
          ook[c] = col < NCOL && node_ok(gx) && node_ok(gy) && j < nv;
          obase[c] = ook[c] ? node_index(gx, gy, ez * P) * ld + j : 0;
        }
        if (Z) {
          CT zv[CPT][P];
#pragma unroll
          for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i)
              zv[c][i] = (ook[c] && node_ok(ez * P + i)) ? widen<T>(Z[obase[c] + i * pstride]) : CT(0);
#pragma unroll
          for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) acc[c][i] = fma(cs_t, acc[c][i], (CT)prm.beta * zv[c][i]);
        } else {
#pragma unroll
          for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) acc[c][i] *= cs_t;
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
          for (int i = 0; i < P; ++i)
            if (ook[c] && node_ok(ez * P + i)) Y[obase[c] + i * pstride] = narrow<T>(acc[c][i]);
      }
      // this vertex plane is also node 0 of the next cell
      if constexpr (!GR) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const CT carry = acc[c][P];
#pragma unroll
          for (int i = 0; i <= P; ++i)
            acc[c][i] = fma(KT(i, 0), av[c], fma(MT(i, 0), bv[c], i == 0 ? carry : CT(0)));
        }
      } else {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const CT carry = acc[c][P];
          const CT b = nl * bv[c], a = nl * nk * av[c];
#pragma unroll
          for (int i = 0; i <= P; ++i) {
            CT t = fma(KT(i, 0), a, MT(i, 0) * b);
            if (i == 0) t *= nl;
            if (i == P) t *= nr;
            acc[c][i] = (i == 0) ? carry + t : t;
          }
        }
      }
    }
    buf ^= 1;
  }
}


// Same operator with the y-pass and the z-step merged: a thread owns one x-node, one cell
// row in y and one column, forms A and B for that cell's P y-nodes and accumulates their
// z-columns in registers. Per plane there is one LDS intermediate (the x-pass output) and
// two barriers; the x-pass also stores the diagonal term of the owned nodes.
template <typename T, int P, int J, int BEX, int BEY, int NT>
__global__ __launch_bounds__(NT) void ks_apply_yz_kernel(const KParams prm) {
  using CT = typename Calc<T>::type;
  constexpr int BX = BEX * P, BY = BEY * P;  // owned nodes per tile edge
  constexpr int NYI = BY + P + 1;            // input rows (owned + halo)
  constexpr int NXN = BX + P + 1;            // input nodes per row (owned + halo)
  constexpr int NXI = BEX * NYI * J;         // x-pass items
  constexpr int NYZ = BX * BEY * J;          // y/z items: one per thread
  static_assert(NYZ <= NT, "one y-cell column per thread");
  constexpr int EPC = 16 / sizeof(T);
  constexpr int CPN = J / EPC;
  constexpr int NCHUNK = NYI * NXN * CPN;
  constexpr int LPT = (NCHUNK + NT - 1) / NT;
  constexpr int NVO = BX * BY;
  constexpr int VPT = (NVO + NT - 1) / NT;
  static_assert(J % EPC == 0, "column chunk must be a whole number of 16-byte pieces");

  typedef T T16 __attribute__((ext_vector_type(EPC)));
  __shared__ __attribute__((aligned(16))) CT sIn[NYI][NXN][J];
  __shared__ CT sU1[NYI][BX][J];
  __shared__ CT sU2[NYI][BX][J];
  __shared__ CT sD[BY][BX][J];
  __shared__ double sV[BY][BX];

  const T* __restrict__ X = static_cast<const T*>(prm.X);
  T* Y = static_cast<T*>(prm.Y);  // may alias Z, never X
  const T* Z = static_cast<const T*>(prm.Z);
  const int tid = threadIdx.x;
  const int n = prm.n, n1 = prm.n1, ld = prm.ld, nv = prm.nv;
  const int pn = P * n;

  int bid = xcd_logical_block(blockIdx.x, gridDim.x);
  const int jc = bid % prm.jchunks;
  bid /= prm.jchunks;
  const int tx = bid % prm.tiles_x;
  bid /= prm.tiles_x;
  const int ty = bid % prm.tiles_y;
  const int zs = bid / prm.tiles_y;
  const int ex0 = tx * BEX, ey0 = ty * BEY, j0 = jc * J;
  const int ez0 = zs * prm.zseg;
  const int ez1 = min(n, ez0 + prm.zseg);
  const int ezs = (ez0 > 0) ? ez0 - 1 : 0;
  const bool vec_ok = (ld % EPC) == 0;

  auto node_ok = [&](int g) { return g >= 1 && g <= pn - 1; };
  auto node_index = [&](int gx, int gy, int gz) -> long long {
    return (long long)(gx - 1) + (long long)n1 * ((long long)(gy - 1) + (long long)n1 * (gz - 1));
  };
  constexpr int NU = Canon<P>::N;
  __shared__ double sTab[2][NU];
  if constexpr (sizeof(CT) == sizeof(double)) {
    for (int q = tid; q < 2 * NU; q += NT) {
      const int r = Canon<P>::map.rep_of[q % NU];
      sTab[q / NU][q % NU] = (q < NU) ? ref::Table<P>::value.mt[r / (P + 1)][r % (P + 1)]
                                      : ref::Table<P>::value.kt[r / (P + 1)][r % (P + 1)];
    }
    __syncthreads();
  }
  CT cM[NU], cK[NU];
#pragma unroll
  for (int q = 0; q < NU; ++q) {
    const int r = Canon<P>::map.rep_of[q];
    if constexpr (sizeof(CT) == sizeof(double)) {
      cM[q] = (CT)ref::Table<P>::value.mt[r / (P + 1)][r % (P + 1)];
      cK[q] = sTab[1][q];
    } else {
      cM[q] = (CT)ref::Table<P>::value.mt[r / (P + 1)][r % (P + 1)];
      cK[q] = (CT)ref::Table<P>::value.kt[r / (P + 1)][r % (P + 1)];
    }
  }
  auto MT = [&](int i, int k) { return cM[Canon<P>::map.slot[i][k]]; };
  auto KT = [&](int i, int k) { return cK[Canon<P>::map.slot[i][k]]; };

  // ---- plane loader (as in ks_apply_kernel)
  T16 pre[LPT];
  double vpre[VPT];
  int coff[LPT];
  int cfull[LPT];
  int voff[VPT];
  const long long plane_stride = (long long)n1 * n1;
#pragma unroll
  for (int t = 0; t < LPT; ++t) {
    const int c = tid + t * NT;
    coff[t] = -1;
    cfull[t] = 0;
    if (c < NCHUNK) {
      const int part = c % CPN;
      const int r = c / CPN;
      const int gx = ex0 * P - P + r % NXN, gy = ey0 * P - P + r / NXN;
      const int jb = j0 + part * EPC;
      if (node_ok(gx) && node_ok(gy) && jb < nv) {
        coff[t] = (int)(node_index(gx, gy, 1) * ld + jb);
        cfull[t] = (vec_ok && jb + EPC <= nv) ? 1 : 0;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < VPT; ++t) {
    const int o = tid + t * NT;
    voff[t] = -1;
    if (o < NVO) {
      const int gx = ex0 * P + o % BX, gy = ey0 * P + o / BX;
      if (node_ok(gx) && node_ok(gy)) voff[t] = (int)node_index(gx, gy, 1);
    }
  }
  auto load_plane = [&](int gz) {
    const bool zok = node_ok(gz);
    const long long zo = (long long)(gz - 1) * plane_stride;
    const T* Xz = X + zo * ld;
    const double* vz = prm.v + zo;
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
      T16 val;
#pragma unroll
      for (int e = 0; e < EPC; ++e) val[e] = T(0);
      if (zok && coff[t] >= 0) {
        const T* src = Xz + coff[t];
        if (cfull[t]) {
          val = *reinterpret_cast<const T16*>(src);
        } else {
          const int jb = coff[t] % ld;
#pragma unroll
          for (int e = 0; e < EPC; ++e) val[e] = (jb + e < nv) ? src[e] : T(0);
        }
      }
      pre[t] = val;
    }
#pragma unroll
    for (int t = 0; t < VPT; ++t) vpre[t] = (zok && voff[t] >= 0) ? vz[voff[t]] : 0.0;
  };
  auto store_plane = [&]() {
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
      const int c = tid + t * NT;
      if (c < NCHUNK) {
        const int part = c % CPN;
        const int r = c / CPN;
        if constexpr (sizeof(T) == sizeof(CT)) {
          *reinterpret_cast<T16*>(&sIn[r / NXN][r % NXN][part * EPC]) = pre[t];
        } else {
#pragma unroll
          for (int e = 0; e < EPC; ++e) sIn[r / NXN][r % NXN][part * EPC + e] = widen<T>(pre[t][e]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < VPT; ++t) {
      const int o = tid + t * NT;
      if (o < NVO) sV[o / BX][o % BX] = vpre[t];
    }
  };

  // y/z item of this thread: x-node yxl, cell row yey, column yjj
  const bool yz = tid < NYZ;
  const int yjj = tid % J, yxl = (tid / J) % BX, yey = tid / (J * BX);
  const int ogx = ex0 * P + yxl, oj = j0 + yjj;
  const bool col_ok = yz && node_ok(ogx) && oj < nv;
  // column constants, read once (every x-pass item of this thread has the column tid % J as
  // well): a global load inside the plane loop would also wait for the plane prefetch
  static_assert(NT % J == 0, "a thread's items share one column");
  const double sh_t = prm.cshift + ((prm.has_colshift && oj < nv) ? prm.colshift[oj] : 0.0);
  const CT cs_t = (CT)(prm.kscale * prm.alpha) * ((prm.colscale && oj < nv) ? (CT)prm.colscale[oj] : CT(1));
  CT acc[P][P + 1];
#pragma unroll
  for (int c = 0; c < P; ++c)
#pragma unroll
    for (int i = 0; i <= P; ++i) acc[c][i] = 0;

  const int gz0 = ezs * P, gz1 = ez1 * P;
  load_plane(gz0);
  store_plane();
  __syncthreads();
#pragma unroll 1
  for (int gz = gz0; gz <= gz1; ++gz) {
    // prefetch, in flight during this plane's passes. Issued and stored on every plane (after
    // the last, plane 0: zeros, no memory access), so that no load is pending across the
    // loop's back edge and the next plane's loads do not wait for this plane's stores.
    load_plane(gz < gz1 ? gz + 1 : 0);
    // ---- x-pass: U1 = M~x X, U2 = K~x X on owned x, all NYI rows; diagonal term of owned nodes
    for (int item = tid; item < NXI; item += NT) {
      const int jj = item % J;
      const int r = item / J;
      const int exl = r % BEX;
      const int yl = r / BEX;
      CT in[2 * P + 1];
#pragma unroll
      for (int k = 0; k <= 2 * P; ++k) in[k] = sIn[yl][exl * P + k][jj];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        CT u1 = MT(i, 0) * in[P], u2 = KT(i, 0) * in[P];
#pragma unroll
        for (int k = 1; k <= P; ++k) {
          u1 = fma(MT(i, k), in[P + k], u1);
          u2 = fma(KT(i, k), in[P + k], u2);
        }
        if (i == 0) {
#pragma unroll
          for (int k = 0; k <= P; ++k) {
            u1 = fma(MT(P, k), in[k], u1);
            u2 = fma(KT(P, k), in[k], u2);
          }
        }
        sU1[yl][exl * P + i][jj] = u1;
        sU2[yl][exl * P + i][jj] = u2;
      }
      if (yl >= P && yl < P + BY) {
#pragma unroll
        for (int i = 0; i < P; ++i)
          sD[yl - P][exl * P + i][jj] = (CT)(prm.dscale * (sV[yl - P][exl * P + i] - sh_t) * (double)in[P + i]);
      }
    }
    __syncthreads();
    // ---- y-pass and z-step of this thread's y-cell column
    const int rel = gz - gz0;
    const int k = (rel == 0) ? 0 : ((rel - 1) % P) + 1;
    CT av[P], bv[P];
    if (yz) {
      CT a1[2 * P + 1], a2[2 * P + 1];
#pragma unroll
      for (int q = 0; q <= 2 * P; ++q) {
        a1[q] = sU1[yey * P + q][yxl][yjj];
        a2[q] = sU2[yey * P + q][yxl][yjj];
      }
      CT dv[P];
#pragma unroll
      for (int i = 0; i < P; ++i) {
        CT A = MT(i, 0) * a1[P], B = MT(i, 0) * a2[P];
        B = fma(KT(i, 0), a1[P], B);
#pragma unroll
        for (int q = 1; q <= P; ++q) {
          A = fma(MT(i, q), a1[P + q], A);
          B = fma(MT(i, q), a2[P + q], B);
          B = fma(KT(i, q), a1[P + q], B);
        }
        if (i == 0) {
#pragma unroll
          for (int q = 0; q <= P; ++q) {
            A = fma(MT(P, q), a1[q], A);
            B = fma(MT(P, q), a2[q], B);
            B = fma(KT(P, q), a1[q], B);
          }
        }
        av[i] = A;
        bv[i] = B;
        dv[i] = sD[yey * P + i][yxl][yjj];
      }
      z_accumulate<CT, P, P, NU>(k, cM, cK, acc, av, bv, dv);
    }
    // the raw plane and potential were last read by this plane's x-pass (before the barrier
    // above); storing the prefetched plane before this plane's outputs keeps its wait from
    // also waiting for the output stores
    store_plane();
    if (yz && k == P) {
      const int ez = (rel - 1) / P + ezs;
      if (ez >= ez0 && col_ok) {
        // outputs in place in acc[c][0..P-1]; every load of Z before the first store, no load
        // after a store (Y may alias Z element for element)
        const long long pstride = (long long)n1 * n1 * ld;
        const long long obase = node_index(ogx, ey0 * P + yey * P, ez * P) * ld + oj;
        const long long rstride = (long long)n1 * ld;
        if (Z) {
          CT zv[P][P];
#pragma unroll
          for (int c = 0; c < P; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i)
              zv[c][i] = (node_ok(ey0 * P + yey * P + c) && node_ok(ez * P + i))
                             ? widen<T>(Z[obase + c * rstride + i * pstride])
                             : CT(0);
#pragma unroll
          for (int c = 0; c < P; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) acc[c][i] = fma(cs_t, acc[c][i], (CT)prm.beta * zv[c][i]);
        } else {
#pragma unroll
          for (int c = 0; c < P; ++c)
#pragma unroll
            for (int i = 0; i < P; ++i) acc[c][i] *= cs_t;
        }
#pragma unroll
        for (int c = 0; c < P; ++c)
#pragma unroll
          for (int i = 0; i < P; ++i)
            if (node_ok(ey0 * P + yey * P + c) && node_ok(ez * P + i))
              Y[obase + c * rstride + i * pstride] = narrow<T>(acc[c][i]);
      }
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const CT carry = acc[c][P];
#pragma unroll
        for (int i = 0; i <= P; ++i)
          acc[c][i] = fma(KT(i, 0), av[c], fma(MT(i, 0), bv[c], i == 0 ? carry : CT(0)));
      }
    }
    __syncthreads();
  }
}

namespace {

template <typename T, int P, int J, bool GR = false>
fe_status launch_typed(const Mesh& m, KParams& prm, hipStream_t s) {
  constexpr int NT = 256;
  prm.tiles_x = (m.n + TileShape<P, T>::BEX - 1) / TileShape<P, T>::BEX;
  prm.tiles_y = (m.n + TileShape<P, T>::BEY - 1) / TileShape<P, T>::BEY;
  prm.jchunks = (prm.nv + J - 1) / J;
  const long long base = (long long)prm.tiles_x * prm.tiles_y * prm.jchunks;
  // enough workgroups to fill 256 CUs several times; each z-segment re-walks one
  // extra cell to pick up the shared bottom vertex plane
  int zsegs = (int)std::min<long long>(m.n, std::max<long long>(1, (2048 + base - 1) / base));
  int zseg = (m.n + zsegs - 1) / zsegs;
  zseg = std::max(zseg, std::min(m.n, 4));
  zsegs = (m.n + zseg - 1) / zseg;
  prm.zseg = zseg;
  prm.zsegs = zsegs;
  const long long grid = base * zsegs;
  if (grid > 0x7fffffffLL) return fail(FE_EINVAL, "ks_apply: problem too large for one launch");
  hipLaunchKernelGGL((ks_apply_kernel<T, P, J, NT, GR>), dim3((unsigned)grid), dim3(NT), 0, s, prm);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}


template <typename T, int P, int J, int BEX, int BEY>
fe_status launch_yz(const Mesh& m, KParams& prm, hipStream_t s) {
  constexpr int NT = 256;
  prm.tiles_x = (m.n + BEX - 1) / BEX;
  prm.tiles_y = (m.n + BEY - 1) / BEY;
  prm.jchunks = (prm.nv + J - 1) / J;
  const long long base = (long long)prm.tiles_x * prm.tiles_y * prm.jchunks;
  int zsegs = (int)std::min<long long>(m.n, std::max<long long>(1, (2048 + base - 1) / base));
  int zseg = (m.n + zsegs - 1) / zsegs;
  zseg = std::max(zseg, std::min(m.n, 4));
  zsegs = (m.n + zseg - 1) / zseg;
  prm.zseg = zseg;
  prm.zsegs = zsegs;
  const long long grid = base * zsegs;
  if (grid > 0x7fffffffLL) return fail(FE_EINVAL, "ks_apply: problem too large for one launch");
  hipLaunchKernelGGL((ks_apply_yz_kernel<T, P, J, BEX, BEY, NT>), dim3((unsigned)grid), dim3(NT), 0, s, prm);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

// graded meshes: the separate-pass kernel with per-cell factors, every order and precision
template <typename T, int J>
fe_status launch_p_graded(const Mesh& m, KParams& prm, hipStream_t s) {
  switch (m.p) {
    case 1: return launch_typed<T, 1, J, true>(m, prm, s);
    case 2: return launch_typed<T, 2, J, true>(m, prm, s);
    case 3: return launch_typed<T, 3, J, true>(m, prm, s);
    case 4: return launch_typed<T, 4, J, true>(m, prm, s);
    case 5: return launch_typed<T, 5, J, true>(m, prm, s);
    case 6: return launch_typed<T, 6, J, true>(m, prm, s);
    case 7: return launch_typed<T, 7, J, true>(m, prm, s);
    case 8: return launch_typed<T, 8, J, true>(m, prm, s);
    default: return fail(FE_EINVAL, "ks_apply: unsupported order p");
  }
}

template <typename T, int J>
fe_status launch_p(const Mesh& m, KParams& prm, hipStream_t s) {
  // (FP32 and bf16 graded: 8-column chunks; 16 would cost the second wave per SIMD at p = 5)
  if (m.graded) return launch_p_graded<T, (sizeof(T) < 8 ? 8 : J)>(m, prm, s);
  switch (m.p) {
    case 1: return launch_typed<T, 1, J>(m, prm, s);
    case 2: return launch_typed<T, 2, J>(m, prm, s);
    case 3: return launch_typed<T, 3, J>(m, prm, s);
    case 4: return launch_typed<T, 4, J>(m, prm, s);
    case 5:
      // FP32 arithmetic (FP32 or bf16 storage): merged y/z kernel on 3 x 1 cell tiles (faster at
      // this order); FP64: separate passes
      if constexpr (sizeof(T) < 8) return launch_yz<T, 5, J, 3, 1>(m, prm, s);
      else return launch_typed<T, 5, J>(m, prm, s);
    case 6: return launch_typed<T, 6, J>(m, prm, s);
    case 7: return launch_typed<T, 7, J>(m, prm, s);
    case 8: return launch_typed<T, 8, J>(m, prm, s);
    default: return fail(FE_EINVAL, "ks_apply: unsupported order p");
  }
}

}  // namespace

// ---- the apply, optionally timed (launch timing is a measurement aid)
static fe_status launch_apply_untimed(const Mesh& m, const ApplyArgs& a, fe_prec prec, hipStream_t s);

fe_status launch_apply(const Mesh& m, const ApplyArgs& a, fe_prec prec, hipStream_t s) {
  if (m.nf == 0) return launch_apply_untimed(m, a, prec, s);
  // algorithmic bytes: X read, Y written, Z read when given (the Chebyshev term), v read
  const double blocks = a.Z ? 3.0 : 2.0;
  const double bytes = (double)m.nf * (blocks * a.nv * (prec == FE_F64 ? 8.0 : prec == FE_F32 ? 4.0 : 2.0) + 8.0) +
                       (m.mapped ? (double)mapped_matrix_bytes(m, prec) : 0.0);
  int slot;
  fe_status st = timed_begin((int)prec, bytes, (double)a.nv, s, &slot);
  if (st != FE_OK) return st;
  st = launch_apply_untimed(m, a, prec, s);
  const fe_status st2 = timed_end(slot, s);
  return st != FE_OK ? st : st2;
}

static fe_status launch_apply_untimed(const Mesh& m, const ApplyArgs& a, fe_prec prec, hipStream_t s) {
  if (m.mapped) return m.nf == 0 ? FE_OK : launch_apply_mapped(m, a, prec, s);
  KParams prm;
  std::memset(&prm, 0, sizeof(prm));
  prm.X = a.X;
  prm.Y = a.Y;
  prm.Z = a.Z;
  prm.v = a.v;
  prm.colscale = a.d_colscale;
  prm.n = m.n;
  prm.n1 = m.n1;
  prm.nv = a.nv;
  prm.ld = a.ld;
  prm.alpha = a.alpha;
  prm.beta = a.beta;
  prm.cshift = a.cshift;
  prm.kscale = 0.5 / (m.h * m.h);
  prm.dscale = 2.0 * m.h * m.h;
  prm.ckap = m.d_ckap;
  prm.cgl = m.d_cgl;
  prm.cgr = m.d_cgr;
  if (a.colshift) {
    if (a.nv > kMaxShiftCols) return fail(FE_EINVAL, "ks_apply: per-column shifts limited to 256 columns");
    prm.has_colshift = 1;
    for (int j = 0; j < a.nv; ++j) prm.colshift[j] = a.colshift[j];
  }
  if (m.nf == 0) return FE_OK;
  // the kernels address one z-plane of the block with 32-bit element offsets
  if ((long long)m.n1 * m.n1 * a.ld > 0x7fffffffLL)
    return fail(FE_EINVAL, "ks_apply: one z-plane of the block exceeds 2^31 elements");
  switch (prec) {
    case FE_F64: return launch_p<double, 8>(m, prm, s);
    case FE_F32: return launch_p<float, 16>(m, prm, s);
    case FE_BF16: return launch_p<bf16_t, 16>(m, prm, s);
    default: return fail(FE_EINVAL, "ks_apply: precision not supported by this operator");
  }
}

}  // namespace invdft
