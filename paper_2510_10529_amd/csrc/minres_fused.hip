// Fused first pass of a batched, projected, preconditioned MINRES iteration (gfx950):
//   G = Psi^T y,  d1 = z.y,  d2 = z.r1
// in one sweep over the rows (Psi: N x k0 occupied orbitals). alfa may use the unprojected
// y because v = z / beta is orthogonal to Psi; G then projects y. The Gram product runs on
// the FP64 matrix cores (16x16x4), the dots on the vector ALU from the same loaded values.
// Partial sums are per workgroup and reduced in a fixed order by separate kernels, so the
// results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"
#include "minres_fused.h"

namespace invdft {

typedef double dv4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kRows = 64;     // rows per chunk (4 wavefronts x 16)
constexpr int kThreads = 256;
constexpr int kTile = 64;     // Gram partial tile (k0, k <= 64)

__device__ __forceinline__ dv4 mfma(double a, double b, dv4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double wsum16(double v) {  // sum over the 4 lane groups sharing lane % 16
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// ---------------------------------------------------------------- pass A
template <typename T>
__global__ __launch_bounds__(kThreads) void pass_a_kernel(const T* __restrict__ Psi, int k0, const T* __restrict__ Y,
                                                          const T* __restrict__ Z, const T* __restrict__ R1, int k,
                                                          long long N, long long rows_per_blk,
                                                          double* __restrict__ partG, double* __restrict__ partD) {
  __shared__ double red[kTile * kTile];
  __shared__ double redd[2][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const long long r_begin = (long long)blockIdx.x * rows_per_blk;
  const long long r_end = min(N, r_begin + rows_per_blk);
  const int TI = (k0 + 15) / 16, TJ = (k + 15) / 16;
  dv4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = dv4{0, 0, 0, 0};
  double d1[4] = {0, 0, 0, 0}, d2[4] = {0, 0, 0, 0};
  for (long long r0 = r_begin + 4 * wave; r0 < r_end; r0 += 16) {
    const long long r = r0 + lk;
    const bool rok = r < r_end;
    double av[4], bv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int ci = 16 * t + li;
      av[t] = (t < TI && rok && ci < k0) ? (double)Psi[r * k0 + ci] : 0.0;
      double y = 0, zz = 0, r1 = 0;
      if (t < TJ && rok && ci < k) {
        y = (double)Y[r * k + ci];
        zz = (double)Z[r * k + ci];
        r1 = (double)R1[r * k + ci];
      }
      bv[t] = y;
      d1[t] = fma(zz, y, d1[t]);
      d2[t] = fma(zz, r1, d2[t]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (a < TI && b < TJ) acc[a][b] = mfma(av[a], bv[b], acc[a][b]);
  }
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = 16 * a + lk + 4 * rr, j = 16 * b + li;
            if (w == 0)
              red[i * kTile + j] = acc[a][b][rr];
            else
              red[i * kTile + j] += acc[a][b][rr];
          }
    }
    __syncthreads();
  }
  double* outG = partG + (long long)blockIdx.x * kTile * kTile;
  for (int e = threadIdx.x; e < kTile * kTile; e += kThreads) outG[e] = red[e];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const double s1 = wsum16(d1[t]), s2 = wsum16(d2[t]);
    if (lk == 0) {
      redd[0][wave][16 * t + li] = s1;
      redd[1][wave][16 * t + li] = s2;
    }
  }
  __syncthreads();
  if (threadIdx.x < 64 && threadIdx.x < k) {
    const int j = threadIdx.x;
    partD[((long long)blockIdx.x * 2 + 0) * k + j] = ((redd[0][0][j] + redd[0][1][j]) + redd[0][2][j]) + redd[0][3][j];
    partD[((long long)blockIdx.x * 2 + 1) * k + j] = ((redd[1][0][j] + redd[1][1][j]) + redd[1][2][j]) + redd[1][3][j];
  }
}

int fused_blocks(long long N) {
  return (int)std::max<long long>(1, std::min<long long>((N + 4095) / 4096, 1024));
}

}  // namespace

size_t fused_work_bytes(int64_t N) {
  const size_t nb = fused_blocks(N);
  // G partials (nb tiles), dot partials (2 nb x 64), G (64 x 64), d1, d2 (64 each)
  return (nb * kTile * kTile + nb * 2 * 64 + 64 * 64 + 2 * 64 + 64) * sizeof(double);
}

template <typename T>
fe_status minres_pass_a(const T* Psi, int k0, const T* Y, const T* Z, const T* R1, int k, int64_t N, FusedWork& fw,
                        hipStream_t s) {
  const int nb = fused_blocks(N);
  const long long rpb = (N + nb - 1) / nb;
  hipLaunchKernelGGL(pass_a_kernel<T>, dim3(nb), dim3(kThreads), 0, s, Psi, k0, Y, Z, R1, k, (long long)N, rpb,
                     fw.partG, fw.partD);
  INVDFT_HIP(hipGetLastError());
  fe_status st;
  if ((st = reduce_tiles(fw.partG, nb, k0, k, fw.G, s)) != FE_OK) return st;
  if ((st = sum_columns_strided(fw.partD, nb, k, 2, 0, fw.d1, s)) != FE_OK) return st;
  return sum_columns_strided(fw.partD, nb, k, 2, 1, fw.d2, s);
}

FusedWork fused_layout(void* base, int64_t N) {
  FusedWork fw{};
  double* p = static_cast<double*>(base);
  const size_t nb = fused_blocks(N);
  fw.partG = p;
  p += nb * kTile * kTile;
  fw.partD = p;
  p += nb * 2 * 64;
  fw.G = p;
  p += 64 * 64;
  fw.d1 = p;
  p += 64;
  fw.d2 = p;
  return fw;
}

template fe_status minres_pass_a<double>(const double*, int, const double*, const double*, const double*, int, int64_t,
                                         FusedWork&, hipStream_t);
template fe_status minres_pass_a<float>(const float*, int, const float*, const float*, const float*, int, int64_t,
                                        FusedWork&, hipStream_t);
}  // namespace invdft
