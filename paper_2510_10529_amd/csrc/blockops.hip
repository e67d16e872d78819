// Tall-skinny block operations on node-major blocks (gfx950).
//
// Gram products X^T Y and rotations X C of N x nv blocks (nv <= 64 per tile)
// are dense contractions, so they run on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): each wavefront streams 4 rows per instruction
// straight from HBM into the A/B operands (16 consecutive doubles of a row per
// quarter-wave, i.e. 128-byte coalesced loads) and keeps the 16x16 output tiles
// in accumulation registers. Reductions over rows are written as per-workgroup
// partials and summed in a fixed order by a second kernel, so every result is
// bitwise reproducible (no floating-point atomics anywhere).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"

namespace invdft {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

template <typename T>
__device__ __forceinline__ double ld_d(const T* p) {
  return (double)(*p);
}

// MFMA FP64 16x16x4 operand layout on gfx950 (checked on the device): lane l holds
// A[l%16][l/16] and B[l/16][l%16]; the 16x16 result D is held as D[l/16 + 4r][l%16]
// in register r (rows interleaved across the four lane groups).
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kGramThreads = 256;
constexpr int kGramTile = 64;  // output tile edge handled by one workgroup (4 x 4 MFMA tiles)

// partial[blk][i][j] (for this output tile) = sum over the block's rows of X[r][i] Y[r][j], or with
// WEIGHTED of X[r][i] (wa[r] - wb[r]) Y[r][j] (a diagonal weight that keeps a symmetric product symmetric).
template <typename T, bool WEIGHTED>
__global__ __launch_bounds__(kGramThreads) void gram_partial_kernel(const T* __restrict__ X, int ldx,
                                                                    const T* __restrict__ Y, int ldy,
                                                                    const double* __restrict__ wa,
                                                                    const double* __restrict__ wb,
                                                                    long long N, int nx, int ny,
                                                                    long long rows_per_blk, int sym,
                                                                    double* __restrict__ partial) {
  __shared__ double red[kGramTile * kGramTile];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int tiles_j = (ny + kGramTile - 1) / kGramTile;
  const int i0 = (blockIdx.y / tiles_j) * kGramTile;
  const int j0 = (blockIdx.y % tiles_j) * kGramTile;
  const long long r_begin = (long long)blockIdx.x * rows_per_blk;
  const long long r_end = min(N, r_begin + rows_per_blk);
  const int li = lane & 15, lk = lane >> 4;

  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0, 0, 0, 0};

  const bool symtile = sym && (i0 == j0);
  // Each wave takes every 4th group of 4 rows, GU groups per trip: the loads of all GU groups are
  // issued before their products, so that a trip waits for memory once (one group per trip leaves
  // the kernel bound by memory latency). The rows accumulate in the same order either way.
  constexpr int GU = 8;
  constexpr long long kStride = 4 * (kGramThreads / 64);
  for (long long rb = r_begin + 4 * wave; rb < r_end; rb += GU * kStride) {
    double av[GU][4], bv[GU][4];
#pragma unroll
    for (int g = 0; g < GU; ++g) {
      const long long r = rb + g * kStride + lk;
      const bool rok = r < r_end;
      double wr = 1.0;
      if constexpr (WEIGHTED) wr = rok ? wa[r] - wb[r] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int ci = i0 + 16 * t + li;
        const int cj = j0 + 16 * t + li;
        av[g][t] = (rok && ci < nx) ? ld_d(X + r * ldx + ci) : 0.0;
        if constexpr (WEIGHTED) av[g][t] *= wr;
        bv[g][t] = (rok && cj < ny) ? ld_d(Y + r * ldy + cj) : 0.0;
      }
    }
#pragma unroll
    for (int g = 0; g < GU; ++g)
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (symtile && b < a) continue;
          acc[a][b] = mfma16(av[g][a], bv[g][b], acc[a][b]);
        }
  }
  // reduce the 4 waves through LDS in a fixed order
  for (int w = 0; w < kGramThreads / 64; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = 16 * a + lk + 4 * rr;
            const int j = 16 * b + li;
            const double val = acc[a][b][rr];
            if (w == 0)
              red[i * kGramTile + j] = val;
            else
              red[i * kGramTile + j] += val;
          }
    }
    __syncthreads();
  }
  // write the partial (full tile; symmetric tiles mirror the upper part)
  double* out = partial + ((long long)blockIdx.x * gridDim.y + blockIdx.y) * kGramTile * kGramTile;
  for (int e = threadIdx.x; e < kGramTile * kGramTile; e += kGramThreads) {
    const int i = e / kGramTile, j = e % kGramTile;
    double val = red[e];
    if (symtile && (j / 16) < (i / 16)) val = red[j * kGramTile + i];
    out[e] = val;
  }
}

// out[i][j] = sum over blocks of the partial tiles: one wavefront per entry, each lane sums
// a fixed strided subset, then a fixed-order butterfly across the lanes (deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const double* __restrict__ partial, int nblk, int ntiles,
                                                          int nx, int ny, double* __restrict__ out) {
  const int e = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (e >= nx * ny) return;
  const int i = e / ny, j = e % ny;
  const int tiles_j = (ny + kGramTile - 1) / kGramTile;
  const int tile = (i / kGramTile) * tiles_j + (j / kGramTile);
  const int off = (i % kGramTile) * kGramTile + (j % kGramTile);
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += partial[((long long)b * ntiles + tile) * kGramTile * kGramTile + off];
  s = wave_sum(s);
  if (lane == 0) out[e] = s;
}

int gram_blocks(long long N) {
  long long b = (N + 511) / 512;
  return (int)std::max<long long>(1, std::min<long long>(b, 1024));
}

// out = alpha * (A C) + beta * Xin  over N rows; A: N x nin (lda), C: nin x nout (row stride ldc,
// device), Xin/out: N x nout (ldo). Each wave owns 16 rows and all nout (<= 64) columns, nin <= 64;
// out may alias Xin, and A too: a wave reads all of its rows of A before it writes them.
template <typename T, int KQ, int TT>
__global__ __launch_bounds__(256) void rotate_kernel(
    const T* A, int lda, long long N, int nin, const double* __restrict__ C, int ldc, int nout, double alpha,
    double beta, const T* Xin, T* out, int ldo) {
  __shared__ double sC[64 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const long long r0 = ((long long)blockIdx.x * 4 + wave) * 16;
  const int li = lane & 15, lk = lane >> 4;
  // D[i = row][j = out col] = sum_k A[row][k] C[k][j] in 2 KQ MFMA steps of 4 k each (nin <= 8 KQ)
  // on TT output tiles of 16 columns (nout <= 16 TT), both fixed at compile time so that the
  // unrolled products carry no branches and narrow blocks do no padding work. Step s takes
  // k = 8 (s / 2) + 2 lk + s % 2 in lane group lk, so that a lane's operands of steps 2q and
  // 2q + 1 are two adjacent entries of its row of A: KQ pieces of 2 per lane, all loads in flight
  // together, issued before C is staged (one load and one wait per step would leave the kernel
  // bound by memory latency). Pieces outside A read row 0, column 0 and are discarded.
  const long long ra = r0 + li;
  const bool raok = ra < N;
  const T* Arow = A + (raok ? ra : 0) * lda;
  double av[2 * KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int k = 8 * q + 2 * lk;
    const double x0 = ld_d(Arow + (k < nin ? k : 0));
    const double x1 = ld_d(Arow + (k + 1 < nin ? k + 1 : 0));
    av[2 * q] = (raok && k < nin) ? x0 : 0.0;
    av[2 * q + 1] = (raok && k + 1 < nin) ? x1 : 0.0;
  }
  {
    double cv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = threadIdx.x + 256 * i;
      const int k = e / 64, j = e % 64;
      cv[i] = (k < nin && j < nout) ? C[(long long)k * ldc + j] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) sC[threadIdx.x + 256 * i] = cv[i];
  }
  __syncthreads();
  if (r0 >= N) return;
  d4 acc[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) acc[t] = d4{0, 0, 0, 0};
#pragma unroll
  for (int st = 0; st < 2 * KQ; ++st) {
    const int k = 8 * (st / 2) + 2 * lk + st % 2;
#pragma unroll
    for (int t = 0; t < TT; ++t) acc[t] = mfma16(av[st], sC[k * 64 + 16 * t + li], acc[t]);
  }
  // Output: every load of Xin before the first store (loads and stores complete in order: a
  // load after a store would wait for it); the empty asm keeps each value's arithmetic here
  // rather than in the conditional store below. A and Xin may alias out: both are read first.
  double val[TT][4];
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int j = 16 * t + li;
      const long long row = r0 + lk + 4 * rr;
      const bool ok = j < nout && row < N;
      const double x = beta != 0.0 ? ld_d(Xin + (ok ? row * ldo + j : 0)) : 0.0;
      val[t][rr] = ok ? x : 0.0;
    }
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      double v = alpha * acc[t][rr];
      if (beta != 0.0) v += beta * val[t][rr];
      asm volatile("" : "+v"(v));
      val[t][rr] = v;
    }
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int j = 16 * t + li;
      const long long row = r0 + lk + 4 * rr;
      if (j < nout && row < N) out[row * ldo + j] = (T)val[t][rr];
    }
}

// rotate_kernel instantiated for the block's widths: nin <= 8 KQ (KQ = 2, 4, 8), nout <= 16 TT
template <typename T, int KQ, int TT>
void launch_rotate_t(unsigned grid, const T* A, int lda, long long N, int nin, const double* C, int ldc, int nout,
                     double alpha, double beta, const T* Xin, T* out, int ldo, hipStream_t s) {
  hipLaunchKernelGGL((rotate_kernel<T, KQ, TT>), dim3(grid), dim3(256), 0, s, A, lda, N, nin, C, ldc, nout, alpha, beta,
                     Xin, out, ldo);
}

template <typename T, int KQ>
void launch_rotate_k(unsigned grid, const T* A, int lda, long long N, int nin, const double* C, int ldc, int nout,
                     double alpha, double beta, const T* Xin, T* out, int ldo, hipStream_t s) {
  switch ((nout + 15) / 16) {
    case 1: launch_rotate_t<T, KQ, 1>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s); break;
    case 2: launch_rotate_t<T, KQ, 2>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s); break;
    case 3: launch_rotate_t<T, KQ, 3>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s); break;
    default: launch_rotate_t<T, KQ, 4>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s); break;
  }
}

template <typename T>
void launch_rotate(unsigned grid, const T* A, int lda, long long N, int nin, const double* C, int ldc, int nout,
                   double alpha, double beta, const T* Xin, T* out, int ldo, hipStream_t s) {
  if (nin <= 16) launch_rotate_k<T, 2>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s);
  else if (nin <= 32) launch_rotate_k<T, 4>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s);
  else launch_rotate_k<T, 8>(grid, A, lda, N, nin, C, ldc, nout, alpha, beta, Xin, out, ldo, s);
}

// Column dot products: partial[blk][j] = sum over the block's rows of X[r][j] Y[r][j].
template <typename T>
__global__ __launch_bounds__(256) void coldot_partial_kernel(const T* __restrict__ X, const T* __restrict__ Y,
                                                             int ld, long long N, int nv, long long rows_per_blk,
                                                             double* __restrict__ partial) {
  __shared__ double red[256];
  const long long r_begin = (long long)blockIdx.x * rows_per_blk;
  const long long r_end = min(N, r_begin + rows_per_blk);
  const int j = blockIdx.y * 64 + (threadIdx.x & 63);
  const int rsub = threadIdx.x >> 6;
  double s = 0.0;
  if (j < nv)
    for (long long r = r_begin + rsub; r < r_end; r += 4) s += ld_d(X + r * ld + j) * ld_d(Y + r * ld + j);
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 64 && j < nv) {
    const double t = ((red[threadIdx.x] + red[threadIdx.x + 64]) + red[threadIdx.x + 128]) + red[threadIdx.x + 192];
    partial[(long long)blockIdx.x * nv + j] = t;
  }
}

// Residual column norms: partial[blk][j] = sum over rows of (HX[r][j] - lam_j X[r][j])^2.
__global__ __launch_bounds__(256) void resid_partial_kernel(const double* __restrict__ HX, const double* __restrict__ X,
                                                            const double* __restrict__ lam, int ld, long long N,
                                                            int nv, long long rows_per_blk,
                                                            double* __restrict__ partial) {
  __shared__ double red[256];
  const long long r_begin = (long long)blockIdx.x * rows_per_blk;
  const long long r_end = min(N, r_begin + rows_per_blk);
  const int j = blockIdx.y * 64 + (threadIdx.x & 63);
  const int rsub = threadIdx.x >> 6;
  double s = 0.0;
  if (j < nv) {
    const double l = lam[j];
    for (long long r = r_begin + rsub; r < r_end; r += 4) {
      const double d = HX[r * ld + j] - l * X[r * ld + j];
      s += d * d;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 64 && j < nv) {
    const double t = ((red[threadIdx.x] + red[threadIdx.x + 64]) + red[threadIdx.x + 128]) + red[threadIdx.x + 192];
    partial[(long long)blockIdx.x * nv + j] = t;
  }
}

__global__ __launch_bounds__(256) void sum_partials_kernel(const double* __restrict__ partial, int nblk, int nv,
                                                           double* __restrict__ out) {
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= nv) return;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += partial[(long long)b * nv + j];
  s = wave_sum(s);
  if (lane == 0) out[j] = s;
}

__global__ void dot1_partial_kernel(const double* __restrict__ x, const double* __restrict__ y, long long n,
                                    long long per_blk, double* __restrict__ partial) {
  __shared__ double red[256];
  const long long b0 = (long long)blockIdx.x * per_blk;
  const long long b1 = min(n, b0 + per_blk);
  double s = 0.0;
  for (long long i = b0 + threadIdx.x; i < b1; i += 256) s += x[i] * y[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void max1_partial_kernel(const double* __restrict__ x, long long n, long long per_blk,
                                    double* __restrict__ partial) {
  __shared__ double red[256];
  const long long b0 = (long long)blockIdx.x * per_blk;
  const long long b1 = min(n, b0 + per_blk);
  double s = -1.0e300;
  for (long long i = b0 + threadIdx.x; i < b1; i += 256) s = fmax(s, x[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void reduce_serial_kernel(const double* __restrict__ partial, int nblk, int op, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = (op == 0) ? 0.0 : -1.0e300;
  for (int b = 0; b < nblk; ++b) s = (op == 0) ? s + partial[b] : fmax(s, partial[b]);
  *out = s;
}

template <typename TS, typename TD>
__global__ void cast_kernel(const TS* __restrict__ src, TD* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = (TD)src[i];
}

// bf16 <-> wider: round to nearest, ties to even, on the FP32 value (an FP64 value is first
// rounded to FP32; NaN stays a quiet NaN, overflow goes to infinity as rounding dictates)
__device__ __forceinline__ bf16_t bf16_from_f32(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (bf16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(bf16_t b) { return __uint_as_float((unsigned)b << 16); }

__global__ void cast_to_bf16_kernel(const double* __restrict__ src, bf16_t* __restrict__ dst, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    dst[i] = bf16_from_f32((float)src[i]);
}

__global__ void cast_cols_from_bf16_kernel(const bf16_t* __restrict__ src, double* __restrict__ dst, long long nrow,
                                           int ld, int c0) {
  const int w = ld - c0;
  const long long total = nrow * w;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e / w;
    const long long idx = r * ld + c0 + (e - r * w);
    dst[idx] = (double)bf16_to_f32(src[idx]);
  }
}

// columns [c0, ld) of an nrow x ld row-major block (the trailing columns of every row)
template <typename TS, typename TD>
__global__ void cast_cols_kernel(const TS* __restrict__ src, TD* __restrict__ dst, long long nrow, int ld, int c0) {
  const int w = ld - c0;
  const long long n = nrow * w;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long a = e / w;
    const long long i = a * ld + c0 + (e - a * w);
    dst[i] = (TD)src[i];
  }
}

__global__ void axpby_kernel(double alpha, const double* __restrict__ x, double beta, double* __restrict__ y,
                             long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = alpha * x[i] + beta * y[i];
}

// The same on 16-byte pieces (both arrays 16-byte aligned), one piece per thread: a launch of
// many short-lived workgroups streams faster than a grid-stride loop on this chip (about 5.8
// against 4.7 TB/s for this kernel over 2^27 doubles).
typedef double d2v __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void axpby2_kernel(double alpha, const d2v* __restrict__ x, double beta,
                                                     d2v* __restrict__ y, long long n2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n2) y[i] = alpha * x[i] + beta * y[i];
}

__global__ void fill_kernel(double* __restrict__ y, double val, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = val;
}

__global__ void fill_f32_kernel(float* __restrict__ y, float val, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = val;
}

unsigned stream_grid(long long n) { return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192)); }

}  // namespace

size_t gram_work_bytes(int64_t N, int nx, int ny) {
  const int tiles = ((nx + kGramTile - 1) / kGramTile) * ((ny + kGramTile - 1) / kGramTile);
  return (size_t)gram_blocks(N) * tiles * kGramTile * kGramTile * sizeof(double);
}

fe_status gram(const void* X, int ldx, const void* Y, int ldy, int64_t N, int nx, int ny, bool f32, double* out,
               void* work, hipStream_t s) {
  if (nx <= 0 || ny <= 0) return FE_OK;
  const int nblk = gram_blocks(N);
  const int tiles_i = (nx + kGramTile - 1) / kGramTile, tiles_j = (ny + kGramTile - 1) / kGramTile;
  const long long rpb = (N + nblk - 1) / nblk;
  const int sym = (X == Y && ldx == ldy && nx == ny) ? 1 : 0;
  double* partial = static_cast<double*>(work);
  dim3 grid(nblk, tiles_i * tiles_j);
  if (f32)
    hipLaunchKernelGGL((gram_partial_kernel<float, false>), grid, dim3(kGramThreads), 0, s,
                       static_cast<const float*>(X), ldx, static_cast<const float*>(Y), ldy, nullptr, nullptr,
                       (long long)N, nx, ny, rpb, sym, partial);
  else
    hipLaunchKernelGGL((gram_partial_kernel<double, false>), grid, dim3(kGramThreads), 0, s,
                       static_cast<const double*>(X), ldx, static_cast<const double*>(Y), ldy, nullptr, nullptr,
                       (long long)N, nx, ny, rpb, sym, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((nx * ny + 3) / 4), dim3(256), 0, s, partial, nblk,
                     tiles_i * tiles_j, nx, ny, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status gram_weighted(const double* X, int ld, const double* wa, const double* wb, int64_t N, int n, double* out,
                        void* work, hipStream_t s) {
  if (n <= 0) return FE_OK;
  const int nblk = gram_blocks(N);
  const int tiles = (n + kGramTile - 1) / kGramTile;
  const long long rpb = (N + nblk - 1) / nblk;
  double* partial = static_cast<double*>(work);
  hipLaunchKernelGGL((gram_partial_kernel<double, true>), dim3(nblk, tiles * tiles), dim3(kGramThreads), 0, s, X, ld,
                     X, ld, wa, wb, (long long)N, n, n, rpb, 1, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((n * n + 3) / 4), dim3(256), 0, s, partial, nblk, tiles * tiles, n, n,
                     out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status rotate_add(const double* X, int ldx, int64_t N, int nin, const double* C, int nout, double* Y, int ldy,
                     hipStream_t s) {
  return rotate_axpy(X, ldx, N, nin, C, nout, 1.0, Y, ldy, s);
}

// out = alpha A C + beta Xin for any widths: 64 x 64 tiles of C, one launch each, accumulating
// over the input tiles into out (the first with beta Xin, the rest with out itself). Above 64
// columns in or out, out must not overlap A.
template <typename T>
fe_status rotate_tiled(const T* A, int lda, int64_t N, int nin, const double* C, int ldc, int nout, double alpha,
                       double beta, const T* Xin, T* out, int ldo, hipStream_t s) {
  if (N <= 0 || nin <= 0 || nout <= 0) return FE_OK;
  const unsigned grid = (unsigned)((N + 63) / 64);
  for (int j0 = 0; j0 < nout; j0 += 64) {
    const int nj = std::min(64, nout - j0);
    for (int k0 = 0; k0 < nin; k0 += 64) {
      const int nk = std::min(64, nin - k0);
      const bool first = k0 == 0;
      launch_rotate<T>(grid, A + k0, lda, (long long)N, nk, C + (long long)k0 * ldc + j0, ldc, nj, alpha,
                       first ? beta : 1.0, first ? (Xin ? Xin + j0 : nullptr) : out + j0, out + j0, ldo, s);
      INVDFT_HIP(hipGetLastError());
    }
  }
  return FE_OK;
}

// do the column ranges of two N-row blocks share memory?
bool blocks_overlap(const void* a, int lda, int na, const void* b, int ldb, int nb, int64_t N, size_t es) {
  const char* a0 = static_cast<const char*>(a);
  const char* b0 = static_cast<const char*>(b);
  const char* a1 = a0 + ((size_t)(N - 1) * lda + na) * es;
  const char* b1 = b0 + ((size_t)(N - 1) * ldb + nb) * es;
  return a0 < b1 && b0 < a1;
}

fe_status rotate_axpy(const double* X, int ldx, int64_t N, int nin, const double* C, int nout, double alpha, double* Y,
                      int ldy, hipStream_t s) {
  if (N <= 0) return FE_OK;
  if ((nin > 64 || nout > 64) && blocks_overlap(X, ldx, nin, Y, ldy, nout, N, sizeof(double)))
    return fail(FE_EINVAL, "rotate: above 64 columns the output must not overlap the input");
  return rotate_tiled<double>(X, ldx, N, nin, C, nout, nout, alpha, 1.0, Y, Y, ldy, s);
}

fe_status rotate(const double* X, int ldx, int64_t N, int nin, const double* C, int nout, double* out, int ldo,
                 hipStream_t s) {
  if (N <= 0) return FE_OK;
  if ((nin > 64 || nout > 64) && blocks_overlap(X, ldx, nin, out, ldo, nout, N, sizeof(double)))
    return fail(FE_EINVAL, "rotate: above 64 columns the output must not overlap the input");
  return rotate_tiled<double>(X, ldx, N, nin, C, nout, nout, 1.0, 0.0, nullptr, out, ldo, s);
}

size_t coldot_work_bytes(int64_t N, int nv) { return (size_t)gram_blocks(N) * nv * sizeof(double); }

fe_status coldot(const void* X, const void* Y, int ld, int64_t N, int nv, bool f32, double* out, void* work,
                 hipStream_t s) {
  const int nblk = gram_blocks(N);
  const long long rpb = (N + nblk - 1) / nblk;
  double* partial = static_cast<double*>(work);
  dim3 grid(nblk, (nv + 63) / 64);
  if (f32)
    hipLaunchKernelGGL(coldot_partial_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(X),
                       static_cast<const float*>(Y), ld, (long long)N, nv, rpb, partial);
  else
    hipLaunchKernelGGL(coldot_partial_kernel<double>, grid, dim3(256), 0, s, static_cast<const double*>(X),
                       static_cast<const double*>(Y), ld, (long long)N, nv, rpb, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3((nv + 3) / 4), dim3(256), 0, s, partial, nblk, nv, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status colresid(const double* HX, const double* X, const double* lam, int ld, int64_t N, int nv, double* out,
                   void* work, hipStream_t s) {
  const int nblk = gram_blocks(N);
  const long long rpb = (N + nblk - 1) / nblk;
  double* partial = static_cast<double*>(work);
  hipLaunchKernelGGL(resid_partial_kernel, dim3(nblk, (nv + 63) / 64), dim3(256), 0, s, HX, X, lam, ld, (long long)N,
                     nv, rpb, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_partials_kernel, dim3((nv + 3) / 4), dim3(256), 0, s, partial, nblk, nv, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}





fe_status dot1(const double* x, const double* y, int64_t n, double* out, void* work, hipStream_t s) {
  const int nblk = (int)std::max<long long>(1, std::min<long long>((n + 4095) / 4096, 1024));
  const long long per = (n + nblk - 1) / nblk;
  double* partial = static_cast<double*>(work);
  hipLaunchKernelGGL(dot1_partial_kernel, dim3(nblk), dim3(256), 0, s, x, y, (long long)n, per, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_serial_kernel, dim3(1), dim3(64), 0, s, partial, nblk, 0, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status max1(const double* x, int64_t n, double* out, void* work, hipStream_t s) {
  const int nblk = (int)std::max<long long>(1, std::min<long long>((n + 4095) / 4096, 1024));
  const long long per = (n + nblk - 1) / nblk;
  double* partial = static_cast<double*>(work);
  hipLaunchKernelGGL(max1_partial_kernel, dim3(nblk), dim3(256), 0, s, x, (long long)n, per, partial);
  INVDFT_HIP(hipGetLastError());
  hipLaunchKernelGGL(reduce_serial_kernel, dim3(1), dim3(64), 0, s, partial, nblk, 1, out);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}


fe_status cast_block_to_f32(const double* src, float* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL((cast_kernel<double, float>), dim3(stream_grid(count)), dim3(256), 0, s, src, dst,
                     (long long)count);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status cast_block_to_f64(const float* src, double* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL((cast_kernel<float, double>), dim3(stream_grid(count)), dim3(256), 0, s, src, dst,
                     (long long)count);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status cast_block_to_bf16(const double* src, bf16_t* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(cast_to_bf16_kernel, dim3(stream_grid(count)), dim3(256), 0, s, src, dst, (long long)count);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status cast_cols_bf16_to_f64(const bf16_t* src, double* dst, int64_t nrow, int ld, int c0, hipStream_t s) {
  if (c0 < 0 || c0 >= ld) return fail(FE_EINVAL, "cast_cols: column range");
  hipLaunchKernelGGL(cast_cols_from_bf16_kernel, dim3(stream_grid(nrow * (ld - c0))), dim3(256), 0, s, src, dst,
                     (long long)nrow, ld, c0);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status cast_cols_to_f64(const float* src, double* dst, int64_t nrow, int ld, int c0, hipStream_t s) {
  if (c0 < 0 || c0 >= ld) return fail(FE_EINVAL, "cast_cols: column range");
  hipLaunchKernelGGL((cast_cols_kernel<float, double>), dim3(stream_grid(nrow * (ld - c0))), dim3(256), 0, s, src, dst,
                     (long long)nrow, ld, c0);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status axpby(double alpha, const double* x, double beta, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return FE_OK;
  const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0 && n >= 2;
  if (!vec) {
    hipLaunchKernelGGL(axpby_kernel, dim3(stream_grid(n)), dim3(256), 0, s, alpha, x, beta, y, (long long)n);
    INVDFT_HIP(hipGetLastError());
    return FE_OK;
  }
  const long long n2 = n / 2;
  const long long blocks = (n2 + 255) / 256;
  if (blocks > 0x7fffffffLL) {   // beyond one launch's grid: the grid-stride kernel
    hipLaunchKernelGGL(axpby_kernel, dim3(stream_grid(n)), dim3(256), 0, s, alpha, x, beta, y, (long long)n);
    INVDFT_HIP(hipGetLastError());
    return FE_OK;
  }
  hipLaunchKernelGGL(axpby2_kernel, dim3((unsigned)blocks), dim3(256), 0, s, alpha, reinterpret_cast<const d2v*>(x),
                     beta, reinterpret_cast<d2v*>(y), n2);
  INVDFT_HIP(hipGetLastError());
  if (n % 2) {  // the last element of an odd length
    hipLaunchKernelGGL(axpby_kernel, dim3(1), dim3(64), 0, s, alpha, x + n - 1, beta, y + n - 1, 1LL);
    INVDFT_HIP(hipGetLastError());
  }
  return FE_OK;
}

fe_status fill(double* y, double val, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel, dim3(stream_grid(n)), dim3(256), 0, s, y, val, (long long)n);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

size_t project_work_bytes(int64_t N, int k, int nv) {
  // a group of at most 64 columns at a time: its k x 64 Gram block and one tile's partials
  const int cw = std::min(nv, 64);
  return gram_work_bytes(N, std::min(k, 64), cw) + (((size_t)k * cw * sizeof(double) + 255) / 256) * 256 + 256;
}

// X <- X - Psi (Psi^T X), one group of at most 64 columns of X at a time: the group's Gram
// blocks with every 64-column segment of Psi first, then its update (classical block
// projection, as for a single tile).
template <typename T>
fe_status project_out_t(const T* Psi, int ldp, int k, T* X, int nv, int64_t N, void* work, hipStream_t s) {
  const int cwmax = std::min(nv, 64);
  char* w = static_cast<char*>(work);
  double* G = reinterpret_cast<double*>(w);
  void* gw = w + (((size_t)k * cwmax * sizeof(double) + 255) / 256) * 256;
  const bool f32 = sizeof(T) == sizeof(float);
  fe_status st;
  for (int c0 = 0; c0 < nv; c0 += 64) {
    const int cw = std::min(64, nv - c0);
    for (int s0 = 0; s0 < k; s0 += 64) {
      const int kw = std::min(64, k - s0);
      if ((st = gram(Psi + s0, ldp, X + c0, nv, N, kw, cw, f32, G + (size_t)s0 * cw, gw, s)) != FE_OK) return st;
    }
    if ((st = rotate_tiled<T>(Psi, ldp, N, k, G, cw, cw, -1.0, 1.0, X + c0, X + c0, nv, s)) != FE_OK) return st;
  }
  return FE_OK;
}

fe_status project_out_ld(const void* Psi, int ldp, int k, void* X, int nv, int64_t N, bool f32, void* work,
                         hipStream_t s) {
  if (k < 1 || nv < 1 || N <= 0) return FE_OK;
  if (ldp < k) return fail(FE_EINVAL, "projection: the row pitch of Psi is below its width");
  if (f32)
    return project_out_t<float>(static_cast<const float*>(Psi), ldp, k, static_cast<float*>(X), nv, N, work, s);
  return project_out_t<double>(static_cast<const double*>(Psi), ldp, k, static_cast<double*>(X), nv, N, work, s);
}

fe_status project_out(const void* Psi, int k, void* X, int nv, int64_t N, bool f32, void* work, hipStream_t s) {
  return project_out_ld(Psi, k, k, X, nv, N, f32, work, s);
}

fe_status fill_f32(float* y, float val, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(stream_grid(n)), dim3(256), 0, s, y, val, (long long)n);
  INVDFT_HIP(hipGetLastError());
  return FE_OK;
}

fe_status copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t s) {
  INVDFT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return FE_OK;
}

}  // namespace invdft
