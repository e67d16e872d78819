// Fused row sweeps of a batched, projected, preconditioned MINRES iteration (gfx950).
// With Psi the N x k0 block of occupied orbitals, P = I - Psi Psi^T, D the diagonal
// preconditioner and y = (H - eps)(z / beta) from the operator apply, one iteration is
//   pass A:  G1 = Psi^T y,  d1 = z.y,  d2 = z.r1                 (alfa from d1, d2)
//   pass B:  r = y - Psi G1 - c1 r1 - c2 r2,  u = D^{-1} r,
//            G2 = Psi^T u,  d = r.u                              (beta from d)
//   pass C:  z = u - Psi G2,  w = (z_old / beta_old - e w1 - d w2) / gamma,  q += phi w
// so P y and P D^{-1} P r never make a round trip through memory of their own. alfa may use
// the unprojected y because v = z / beta is orthogonal to Psi, and r.u equals r.(P u)
// because r is orthogonal to Psi.
//
// Every pass walks 16-row chunks. A row-major chunk of an N x k block is one contiguous
// piece of memory, so each thread loads fixed 16-byte pieces of it (fully coalesced) and
// does the elementwise work on exactly the elements it loaded. Only the Psi products need
// a matrix layout: the chunk of Psi is staged in LDS, the products run on the FP64 matrix
// cores (16x16x4, one wavefront per 16-column tile), and their results go through LDS back
// to the threads that own the elements. Partial sums are per workgroup and are reduced in
// a fixed order by separate kernels, so the results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "krylov.h"
#include "minres_fused.h"

namespace invdft {

typedef double dv4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kRows = 16;     // rows per chunk
constexpr int kThreads = 256;
constexpr int kTile = 64;     // widest k0 and k
constexpr int kPsiLd = 65;    // LDS row stride of the Psi chunk (odd: conflict-free column reads)
constexpr int kMaxBlocks = 1024;

// 16x16x4 FP64 MFMA: lane l = 16 a + b holds A[b][a] and B[a][b]; register q of the
// result holds D[a + 4 q][b].
__device__ __forceinline__ dv4 mfma(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wsum64(double v) {  // fixed-order butterfly over the wavefront
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The elements of a chunk that one thread owns: NS pieces of EPV consecutive elements,
// piece j starting at element (threadIdx.x + kThreads j) EPV. The map is the same for every
// chunk. A full chunk (16 rows) holds 16 k elements, a multiple of EPV, so its pieces are
// either wholly inside or wholly outside.
template <typename T>
struct Piece {
  static constexpr int EPV = 16 / sizeof(T);
  static constexpr int NS = (kRows * kTile / EPV + kThreads - 1) / kThreads;
  typedef T V __attribute__((ext_vector_type(EPV)));
};

template <typename T>
struct Slots {
  static constexpr int NS = Piece<T>::NS, EPV = Piece<T>::EPV;
  int e0[NS];        // first element of piece j
  bool own[NS];      // piece j lies inside a full chunk
  int row[NS][EPV];  // chunk-local row and column of each element (row -1: not owned)
  int col[NS][EPV];
  __device__ void init(int k) {
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      e0[j] = (threadIdx.x + kThreads * j) * EPV;
      own[j] = e0[j] + EPV <= kRows * k;
#pragma unroll
      for (int m = 0; m < EPV; ++m) {
        row[j][m] = own[j] ? (e0[j] + m) / k : -1;
        col[j][m] = own[j] ? (e0[j] + m) % k : 0;
      }
    }
  }
};

// Loads of this thread's pieces. FULL: one unconditional 16-byte load per piece (pieces
// outside read piece 0 and are zeroed), so nothing branches between the loads and their use.
// Otherwise (the last, partial chunk only) element by element up to nvalid.
template <bool FULL, typename T>
__device__ __forceinline__ void load_pieces(const T* __restrict__ p, int nvalid, const Slots<T>& sl,
                                            double (&out)[Piece<T>::NS][Piece<T>::EPV]) {
  constexpr int EPV = Piece<T>::EPV;
#pragma unroll
  for (int j = 0; j < Piece<T>::NS; ++j) {
    if constexpr (FULL) {
      const typename Piece<T>::V v = *reinterpret_cast<const typename Piece<T>::V*>(p + (sl.own[j] ? sl.e0[j] : 0));
#pragma unroll
      for (int m = 0; m < EPV; ++m) out[j][m] = sl.own[j] ? (double)v[m] : 0.0;
    } else {
#pragma unroll
      for (int m = 0; m < EPV; ++m) {
        const int e = sl.e0[j] + m;
        out[j][m] = (sl.own[j] && e < nvalid) ? (double)p[e] : 0.0;
      }
    }
  }
}

template <bool FULL, typename T>
__device__ __forceinline__ void store_pieces(T* __restrict__ p, int nvalid, const Slots<T>& sl,
                                             const double (&in)[Piece<T>::NS][Piece<T>::EPV]) {
  constexpr int EPV = Piece<T>::EPV;
#pragma unroll
  for (int j = 0; j < Piece<T>::NS; ++j) {
    if constexpr (FULL) {
      typename Piece<T>::V v;
#pragma unroll
      for (int m = 0; m < EPV; ++m) v[m] = (T)in[j][m];
      if (sl.own[j]) *reinterpret_cast<typename Piece<T>::V*>(p + sl.e0[j]) = v;
    } else {
#pragma unroll
      for (int m = 0; m < EPV; ++m)
        if (sl.own[j] && sl.e0[j] + m < nvalid) p[sl.e0[j] + m] = (T)in[j][m];
    }
  }
}

// Psi chunk (16 x k0, row-major): this thread's pieces of it and their LDS slots
// (rows of stride kPsiLd; columns k0..63 stay zero).
template <typename T>
struct PsiSlots {
  Slots<T> sl;
  int lds[Piece<T>::NS][Piece<T>::EPV];
  __device__ void init(int k0) {
    sl.init(k0);
#pragma unroll
    for (int j = 0; j < Piece<T>::NS; ++j)
#pragma unroll
      for (int m = 0; m < Piece<T>::EPV; ++m)
        lds[j][m] = sl.own[j] ? sl.row[j][m] * kPsiLd + sl.col[j][m] : -1;
  }
};

template <typename T>
__device__ __forceinline__ void put_psi(const PsiSlots<T>& ps, const double (&v)[Piece<T>::NS][Piece<T>::EPV],
                                        double* sPsi) {
#pragma unroll
  for (int j = 0; j < Piece<T>::NS; ++j)
#pragma unroll
    for (int m = 0; m < Piece<T>::EPV; ++m)
      if (ps.lds[j][m] >= 0) sPsi[ps.lds[j][m]] = v[j][m];
}

// Wave w (< TJ) forms rows x [16 w, 16 w + 16) of Psi G (G: k0 x k, B operand in gB) into sOut.
__device__ __forceinline__ void psi_times_g(const double* sPsi, int k0, const double (&gB)[16], int w, int li,
                                            int lk, double* sOut) {
  double a[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) a[s] = sPsi[li * kPsiLd + 4 * s + lk];
  dv4 acc = dv4{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 16; ++s)
    if (4 * s < k0) acc = mfma(a[s], gB[s], acc);
#pragma unroll
  for (int q = 0; q < 4; ++q) sOut[(lk + 4 * q) * kTile + 16 * w + li] = acc[q];
}

// acc[t] += (Psi^T X) tile (16 t.., 16 w..) over the chunk's rows; X in LDS with row stride kTile.
__device__ __forceinline__ void psiT_times_x(const double* sPsi, const double* sX, int TI, int w, int li, int lk,
                                             dv4 (&acc)[4]) {
  double b[4], a[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    b[q] = sX[(4 * q + lk) * kTile + 16 * w + li];
#pragma unroll
    for (int t = 0; t < 4; ++t) a[t][q] = sPsi[(4 * q + lk) * kPsiLd + 16 * t + li];
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (t < TI) {
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[t] = mfma(a[t][q], b[q], acc[t]);
    }
}

// Per-column sums of per-element partials, fixed order: part[qd][j][m] belongs to the column
// of element (j, m). Result in out[qd * kTile + c] for c < k (block-level; red holds
// kThreads * NS * EPV doubles).
template <typename T, int NQ>
__device__ void column_sums(const double (&part)[NQ][Piece<T>::NS][Piece<T>::EPV], int k, double* red, double* out) {
  constexpr int EPV = Piece<T>::EPV;
  constexpr int PER = Piece<T>::NS * EPV;
  for (int qd = 0; qd < NQ; ++qd) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < Piece<T>::NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m) red[threadIdx.x * PER + j * EPV + m] = part[qd][j][m];
    __syncthreads();
    if (threadIdx.x < k) {
      const int c = threadIdx.x;
      double s = 0.0;
      // element e of the chunk is piece e / EPV (thread (e / EPV) % kThreads, slot (e / EPV) / kThreads)
      for (int e = c; e < kRows * k; e += k) {
        const int vi = e / EPV;
        s += red[(vi % kThreads) * PER + (vi / kThreads) * EPV + e % EPV];
      }
      out[qd * kTile + c] = s;
    }
  }
}

// Chunk loop shared by the passes: full chunks take the branch-free path, the one partial
// chunk at the end (if any) the guarded one, on the workgroup that the stride lands it on.
template <typename Body>
__device__ __forceinline__ void for_chunks(long long N, Body&& body) {
  const long long nfull = N / kRows;
  for (long long ch = blockIdx.x; ch < nfull; ch += gridDim.x) body(std::integral_constant<bool, true>(), ch, kRows);
  if (N % kRows != 0 && nfull % gridDim.x == blockIdx.x)
    body(std::integral_constant<bool, false>(), nfull, (int)(N % kRows));
}

// ---------------------------------------------------------------- pass A
template <typename T>
__global__ __launch_bounds__(kThreads) void pass_a_kernel(const T* __restrict__ Psi, int k0, const T* __restrict__ Y,
                                                          const T* __restrict__ Z, const T* __restrict__ R1, int k,
                                                          long long N, double* __restrict__ partG,
                                                          double* __restrict__ partD) {
  __shared__ double sPsi[kRows * kPsiLd];
  __shared__ double sY[kRows * kTile];
  __shared__ double red[kThreads * Piece<T>::NS * Piece<T>::EPV];
  __shared__ double sd[2 * kTile];
  constexpr int NS = Piece<T>::NS, EPV = Piece<T>::EPV;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int TI = (k0 + 15) / 16, TJ = (k + 15) / 16;
  Slots<T> sl;
  sl.init(k);
  PsiSlots<T> ps;
  ps.init(k0);
  for (int e = threadIdx.x; e < kRows * kPsiLd; e += kThreads) sPsi[e] = 0.0;
  for (int e = threadIdx.x; e < kRows * kTile; e += kThreads) sY[e] = 0.0;
  dv4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = dv4{0, 0, 0, 0};
  double dd[2][NS][EPV] = {};
  for_chunks(N, [&](auto full, long long ch, int nr) {
    constexpr bool FULL = decltype(full)::value;
    const long long row0 = ch * kRows;
    double yv[NS][EPV], zv[NS][EPV], rv[NS][EPV], pv[NS][EPV];
    // Psi first: it is needed first (LDS staging), the rest stays in flight meanwhile
    load_pieces<FULL>(Psi + row0 * k0, nr * k0, ps.sl, pv);
    load_pieces<FULL>(Y + row0 * k, nr * k, sl, yv);
    load_pieces<FULL>(Z + row0 * k, nr * k, sl, zv);
    load_pieces<FULL>(R1 + row0 * k, nr * k, sl, rv);
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m) {
        dd[0][j][m] = fma(zv[j][m], yv[j][m], dd[0][j][m]);
        dd[1][j][m] = fma(zv[j][m], rv[j][m], dd[1][j][m]);
      }
    __syncthreads();  // the previous chunk's product is done with sPsi and sY
    put_psi(ps, pv, sPsi);
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m)
        if (sl.row[j][m] >= 0) sY[sl.row[j][m] * kTile + sl.col[j][m]] = yv[j][m];
    __syncthreads();
    if (w < TJ) psiT_times_x(sPsi, sY, TI, w, li, lk, acc);
  });
  // G partial: wave w writes its column tile (zero for idle waves)
  double* outG = partG + (long long)blockIdx.x * kTile * kTile;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) outG[(16 * t + lk + 4 * q) * kTile + 16 * w + li] = acc[t][q];
  column_sums<T, 2>(dd, k, red, sd);
  __syncthreads();
  if (threadIdx.x < k) {
    partD[((long long)blockIdx.x * 2 + 0) * k + threadIdx.x] = sd[threadIdx.x];
    partD[((long long)blockIdx.x * 2 + 1) * k + threadIdx.x] = sd[kTile + threadIdx.x];
  }
}

// ---------------------------------------------------------------- pass B
template <typename T>
__global__ __launch_bounds__(kThreads) void pass_b_kernel(const T* __restrict__ Psi, int k0,
                                                          const double* __restrict__ G1, T* __restrict__ Y,
                                                          T* __restrict__ R1, const T* __restrict__ R2,
                                                          const double* __restrict__ st,
                                                          const double* __restrict__ dinv, int k, long long N,
                                                          double* __restrict__ partG, double* __restrict__ partD) {
  __shared__ double sPsi[kRows * kPsiLd];
  __shared__ double sPG[kRows * kTile];   // Psi G1, then u
  __shared__ double red[kThreads * Piece<T>::NS * Piece<T>::EPV];
  __shared__ double sd[kTile];
  __shared__ double sC[2][kTile];          // c1, c2 per column
  __shared__ double sDv[kRows];            // the chunk's rows of D^{-1}
  constexpr int NS = Piece<T>::NS, EPV = Piece<T>::EPV;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int TI = (k0 + 15) / 16, TJ = (k + 15) / 16;
  Slots<T> sl;
  sl.init(k);
  PsiSlots<T> ps;
  ps.init(k0);
  for (int e = threadIdx.x; e < kRows * kPsiLd; e += kThreads) sPsi[e] = 0.0;
  if (threadIdx.x < k) {
    sC[0][threadIdx.x] = st[S_C1 * k + threadIdx.x];
    sC[1][threadIdx.x] = st[S_C2 * k + threadIdx.x];
  }
  // G1 as the B operand of the wave's column tile
  double gB[16];
  {
    const int c = 16 * w + li;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int i = 4 * s + lk;
      gB[s] = (c < k && i < k0) ? G1[i * k + c] : 0.0;
    }
  }
  dv4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = dv4{0, 0, 0, 0};
  double dd[1][NS][EPV] = {};
  for_chunks(N, [&](auto full, long long ch, int nr) {
    constexpr bool FULL = decltype(full)::value;
    const long long row0 = ch * kRows;
    double yv[NS][EPV], r1v[NS][EPV], r2v[NS][EPV], pv[NS][EPV], dv[NS][EPV];
    // Psi first: it is needed first (LDS staging), the rest stays in flight meanwhile
    load_pieces<FULL>(Psi + row0 * k0, nr * k0, ps.sl, pv);
    load_pieces<FULL>(Y + row0 * k, nr * k, sl, yv);
    load_pieces<FULL>(R1 + row0 * k, nr * k, sl, r1v);
    load_pieces<FULL>(R2 + row0 * k, nr * k, sl, r2v);
    const double drow = threadIdx.x < nr ? dinv[row0 + threadIdx.x] : 0.0;
    __syncthreads();  // the previous chunk's Gram product is done with sPsi and sPG
    put_psi(ps, pv, sPsi);
    if (threadIdx.x < kRows) sDv[threadIdx.x] = drow;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m) {
        const int r = sl.row[j][m];
        dv[j][m] = (r >= 0 && r < nr) ? sDv[r] : 0.0;
      }
    if (w < TJ) psi_times_g(sPsi, k0, gB, w, li, lk, sPG);
    __syncthreads();
    double rn[NS][EPV], u[NS][EPV];
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m) {
        const int r = sl.row[j][m], c = sl.col[j][m];
        const double pg = r >= 0 ? sPG[r * kTile + c] : 0.0;
        rn[j][m] = (double)(T)(yv[j][m] - pg - sC[0][c] * r1v[j][m] - sC[1][c] * r2v[j][m]);
        u[j][m] = (double)(T)(rn[j][m] * dv[j][m]);
        dd[0][j][m] = fma(rn[j][m], u[j][m], dd[0][j][m]);
      }
    store_pieces<FULL>(R1 + row0 * k, nr * k, sl, rn);
    store_pieces<FULL>(Y + row0 * k, nr * k, sl, u);
    __syncthreads();  // every read of Psi G1 is done
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m)
        if (sl.row[j][m] >= 0) sPG[sl.row[j][m] * kTile + sl.col[j][m]] = u[j][m];
    __syncthreads();
    if (w < TJ) psiT_times_x(sPsi, sPG, TI, w, li, lk, acc);
  });
  double* outG = partG + (long long)blockIdx.x * kTile * kTile;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) outG[(16 * t + lk + 4 * q) * kTile + 16 * w + li] = acc[t][q];
  column_sums<T, 1>(dd, k, red, sd);
  __syncthreads();
  if (threadIdx.x < k) partD[(long long)blockIdx.x * k + threadIdx.x] = sd[threadIdx.x];
}

// ---------------------------------------------------------------- pass C
template <typename T>
__global__ __launch_bounds__(kThreads) void pass_c_kernel(const T* __restrict__ Psi, int k0,
                                                          const double* __restrict__ G2, T* __restrict__ U,
                                                          const T* __restrict__ Zold, T* __restrict__ W1,
                                                          const T* __restrict__ W2, T* __restrict__ X,
                                                          const double* __restrict__ st, int k, long long N) {
  __shared__ double sPsi[kRows * kPsiLd];
  __shared__ double sPG[kRows * kTile];
  __shared__ double sS[6][kTile];  // per-column scalars: active, 1/gamma, 1/beta_old, oldeps, delta, phi
  constexpr int NS = Piece<T>::NS, EPV = Piece<T>::EPV;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int TJ = (k + 15) / 16;
  Slots<T> sl;
  sl.init(k);
  PsiSlots<T> ps;
  ps.init(k0);
  for (int e = threadIdx.x; e < kRows * kPsiLd; e += kThreads) sPsi[e] = 0.0;
  if (threadIdx.x < k) {
    const int c = threadIdx.x;
    sS[0][c] = st[S_ACTIVE * k + c] > 0.0 ? 1.0 : 0.0;
    sS[1][c] = st[S_INVGAMMA * k + c];
    sS[2][c] = st[S_INVBETA_OLD * k + c];
    sS[3][c] = st[S_OLDEPS * k + c];
    sS[4][c] = st[S_DELTA * k + c];
    sS[5][c] = st[S_PHI * k + c];
  }
  double gB[16];
  {
    const int c = 16 * w + li;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int i = 4 * s + lk;
      gB[s] = (c < k && i < k0) ? G2[i * k + c] : 0.0;
    }
  }
  for_chunks(N, [&](auto full, long long ch, int nr) {
    constexpr bool FULL = decltype(full)::value;
    const long long row0 = ch * kRows;
    const int nv = nr * k;
    double uv[NS][EPV], zv[NS][EPV], w1v[NS][EPV], w2v[NS][EPV], xv[NS][EPV], pv[NS][EPV];
    // Psi first: it is needed first (LDS staging), the rest stays in flight meanwhile
    load_pieces<FULL>(Psi + row0 * k0, nr * k0, ps.sl, pv);
    load_pieces<FULL>(U + row0 * k, nv, sl, uv);
    load_pieces<FULL>(Zold + row0 * k, nv, sl, zv);
    load_pieces<FULL>(W1 + row0 * k, nv, sl, w1v);
    load_pieces<FULL>(W2 + row0 * k, nv, sl, w2v);
    load_pieces<FULL>(X + row0 * k, nv, sl, xv);
    __syncthreads();  // the previous chunk's product is done with sPsi, its results with sPG
    put_psi(ps, pv, sPsi);
    __syncthreads();
    if (w < TJ) psi_times_g(sPsi, k0, gB, w, li, lk, sPG);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NS; ++j)
#pragma unroll
      for (int m = 0; m < EPV; ++m) {
        const int r = sl.row[j][m], c = sl.col[j][m];
        const double pg = r >= 0 ? sPG[r * kTile + c] : 0.0;
        // converged columns get z = 0, which keeps them at zero in every later pass
        uv[j][m] = sS[0][c] * (uv[j][m] - pg);
        const double ig = sS[1][c];
        if (ig != 0.0) {
          const double wn = (zv[j][m] * sS[2][c] - sS[3][c] * w1v[j][m] - sS[4][c] * w2v[j][m]) * ig;
          w1v[j][m] = wn;
          xv[j][m] += sS[5][c] * wn;
        }
      }
    store_pieces<FULL>(U + row0 * k, nv, sl, uv);
    store_pieces<FULL>(W1 + row0 * k, nv, sl, w1v);
    store_pieces<FULL>(X + row0 * k, nv, sl, xv);
  });
}

// G[i][c] = sum over blocks of the partial tiles, d[q] likewise: one wavefront per entry.
__global__ __launch_bounds__(256) void reduce_kernel(const double* __restrict__ partG, const double* __restrict__ partD,
                                                     int nblk, int k0, int k, int nd, double* __restrict__ G,
                                                     double* __restrict__ d) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e < k0 * k) {
    const int i = e / k, c = e % k;
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += partG[((long long)b * kTile + i) * kTile + c];
    s = wsum64(s);
    if (lane == 0) G[e] = s;
  } else if (e < k0 * k + nd * k) {
    const int q = e - k0 * k;  // q = which * k + c
    double s = 0.0;
    for (int b = lane; b < nblk; b += 64) s += partD[(long long)b * nd * k + q];
    s = wsum64(s);
    if (lane == 0) d[(q / k) * kTile + q % k] = s;
  }
}

int fused_blocks(long long N) {
  return (int)std::max<long long>(1, std::min<long long>((N + kRows - 1) / kRows, kMaxBlocks));
}

fe_status check_widths(int k0, int k) {
  if (k0 < 1 || k0 > kTile || k < 1 || k > kTile)
    return fail(FE_EINVAL, "MINRES passes: Psi and block widths must be in [1, 64]");
  return FE_OK;
}

}  // namespace

size_t fused_work_bytes(int64_t N) {
  const size_t nb = fused_blocks(N);
  // partial G tiles (nb x 64 x 64), partial dots (nb x 2 x 64), G1, G2 (64 x 64), d1, d2, d (64)
  return (nb * kTile * kTile + nb * 2 * kTile + 2 * kTile * kTile + 3 * kTile) * sizeof(double);
}

FusedWork fused_layout(void* base, int64_t N) {
  FusedWork fw{};
  double* p = static_cast<double*>(base);
  const size_t nb = fused_blocks(N);
  fw.partG = p;
  p += nb * kTile * kTile;
  fw.partD = p;
  p += nb * 2 * kTile;
  fw.G = p;
  p += kTile * kTile;
  fw.G2 = p;
  p += kTile * kTile;
  fw.d1 = p;  // d1 and d2 are 64 apart: pass A's reduction writes both
  fw.d2 = p + kTile;
  p += 2 * kTile;
  fw.d = p;
  return fw;
}

template <typename T>
fe_status minres_pass_a(const T* Psi, int k0, const T* Y, const T* Z, const T* R1, int k, int64_t N, FusedWork& fw,
                        hipStream_t s) {
  fe_status st;
  if ((st = check_widths(k0, k)) != FE_OK) return st;
  if (N <= 0) return FE_OK;
  const int nb = fused_blocks(N);
  int slot;  // algorithmic bytes: Psi, Y, Z, R1 read
  if ((st = timed_begin(kTimedSweep + 0, (double)N * sizeof(T) * (k0 + 3.0 * k), k, s, &slot)) != FE_OK) return st;
  hipLaunchKernelGGL(pass_a_kernel<T>, dim3(nb), dim3(kThreads), 0, s, Psi, k0, Y, Z, R1, k, (long long)N, fw.partG,
                     fw.partD);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3((k0 * k + 2 * k + 3) / 4), dim3(256), 0, s, fw.partG, fw.partD, nb, k0, k, 2,
                     fw.G, fw.d1);
  INVDFT_HIP(hipGetLastError());
  return timed_end(slot, s);
}

template <typename T>
fe_status minres_pass_b(const T* Psi, int k0, T* Y, T* R1, const T* R2, const double* st, const double* dinv, int k,
                        int64_t N, FusedWork& fw, hipStream_t s) {
  fe_status stt;
  if ((stt = check_widths(k0, k)) != FE_OK) return stt;
  if (N <= 0) return FE_OK;
  const int nb = fused_blocks(N);
  int slot;  // algorithmic bytes: Psi, Y, R1, R2 and the diagonal read, R1 and Y written
  if ((stt = timed_begin(kTimedSweep + 1, (double)N * (sizeof(T) * (k0 + 5.0 * k) + 8.0), k, s, &slot)) != FE_OK)
    return stt;
  hipLaunchKernelGGL(pass_b_kernel<T>, dim3(nb), dim3(kThreads), 0, s, Psi, k0, fw.G, Y, R1, R2, st, dinv, k,
                     (long long)N, fw.partG, fw.partD);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3((k0 * k + k + 3) / 4), dim3(256), 0, s, fw.partG, fw.partD, nb, k0, k, 1,
                     fw.G2, fw.d);
  INVDFT_HIP(hipGetLastError());
  return timed_end(slot, s);
}

template <typename T>
fe_status minres_pass_c(const T* Psi, int k0, T* U, const T* Zold, T* W1, const T* W2, T* X, const double* st, int k,
                        int64_t N, FusedWork& fw, hipStream_t s) {
  fe_status stt;
  if ((stt = check_widths(k0, k)) != FE_OK) return stt;
  if (N <= 0) return FE_OK;
  int slot;  // algorithmic bytes: Psi, U, Zold, W1, W2, X read, U, W1, X written
  if ((stt = timed_begin(kTimedSweep + 2, (double)N * sizeof(T) * (k0 + 8.0 * k), k, s, &slot)) != FE_OK) return stt;
  hipLaunchKernelGGL(pass_c_kernel<T>, dim3(fused_blocks(N)), dim3(kThreads), 0, s, Psi, k0, fw.G2, U, Zold, W1, W2,
                     X, st, k, (long long)N);
  INVDFT_HIP(hipGetLastError());
  return timed_end(slot, s);
}

template fe_status minres_pass_a<double>(const double*, int, const double*, const double*, const double*, int, int64_t,
                                         FusedWork&, hipStream_t);
template fe_status minres_pass_a<float>(const float*, int, const float*, const float*, const float*, int, int64_t,
                                        FusedWork&, hipStream_t);
template fe_status minres_pass_b<double>(const double*, int, double*, double*, const double*, const double*,
                                         const double*, int, int64_t, FusedWork&, hipStream_t);
template fe_status minres_pass_b<float>(const float*, int, float*, float*, const float*, const double*, const double*,
                                        int, int64_t, FusedWork&, hipStream_t);
template fe_status minres_pass_c<double>(const double*, int, double*, const double*, double*, const double*, double*,
                                         const double*, int, int64_t, FusedWork&, hipStream_t);
template fe_status minres_pass_c<float>(const float*, int, float*, const float*, float*, const float*, float*,
                                        const double*, int, int64_t, FusedWork&, hipStream_t);
}  // namespace invdft
