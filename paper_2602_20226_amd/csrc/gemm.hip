// Dense GEMM kernels on the CDNA4 matrix cores.
//
//  * FP64 and FP32: 64x64 output tile per 256-thread workgroup, BK = 16,
//    four waves each owning a 32x32 quadrant made of 2x2 MFMA 16x16x4 tiles.
//    FP64 matrix throughput on gfx950 equals its vector FP64 rate, so the
//    small tile is already compute bound for FP64 (a 64x64x16 step is 16
//    MFMAs per wave against 16 KB of LDS traffic) while keeping many
//    workgroups for the modest matrix sizes of a QTT sweep.
//  * BF16 split: FP64 operands are split into three bf16 pieces on the way
//    into LDS (a = a0 + a1 + a2, each piece the RNE bf16 of the remainder);
//    3 or 6 cross products run on MFMA 16x16x32 bf16 with FP32 accumulation
//    inside each 32-deep k step, and the k-step partial sums are added in
//    FP64 registers.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"

namespace qtt {

namespace {

template <typename T>
struct Mfma;
// Result row of accumulator element v in a lane (column is lane % 16): the
// f64 instruction interleaves rows across the four values, the f32 one keeps
// four consecutive rows per lane group (checked on gfx950).
template <>
struct Mfma<double> {
  typedef double4_t acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct Mfma<float> {
  typedef float4_t acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int BM = 64, BN = 64, BK = 16, PADM = 1;

// 16x16x4 MFMA operands: lane holds A[lane % 16][lane / 16] and
// B[lane / 16][lane % 16]; result value v of a lane sits in column lane % 16
// and row Mfma<T>::row(lane, v).
// LOWER: only the output tiles on or below the tile diagonal (for symmetric
// updates whose upper triangle is never read); the others exit at once.
template <typename T, bool TA, bool TB, bool LOWER = false>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, T alpha, const T* __restrict__ A,
                                              long lda, long sA, const T* __restrict__ B, long ldb,
                                              long sB, T beta, T* __restrict__ C, long ldc, long sC) {
  if (LOWER && blockIdx.x > blockIdx.y) return;
  __shared__ T As[BK][BM + PADM];
  __shared__ T Bs[BK][BN + PADM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (!TA) {
        m = idx >> 4;
        k = idx & 15;
      } else {
        k = idx >> 6;
        m = idx & 63;
      }
      const int gm = m0 + m, gk = k0 + k;
      T v = 0;
      if (gm < M && gk < K) v = TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      As[k][m] = v;
      int n;
      if (!TB) {
        k = idx >> 6;
        n = idx & 63;
      } else {
        n = idx >> 4;
        k = idx & 15;
      }
      const int gn = n0 + n;
      const int gk2 = k0 + k;
      T w = 0;
      if (gn < N && gk2 < K) w = TB ? B[(long)gn * ldb + gk2] : B[(long)gk2 * ldb + gn];
      Bs[k][n] = w;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::op(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + i * 16 + Mfma<T>::row(lane, v);
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          T r = alpha * acc[i][j][v];
          if (beta != T(0)) r += beta * C[(long)gm * ldc + gn];
          C[(long)gm * ldc + gn] = r;
        }
      }
}

template <typename T>
hipError_t launch_gemm(hipStream_t s, bool ta, bool tb, int M, int N, int K, T alpha, const T* A,
                       long lda, long sA, const T* B, long ldb, long sB, T beta, T* C, long ldc,
                       long sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (K <= 0) {
    // C = beta * C : run with K = 0 through the kernel (the k loop is empty).
  }
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
  if (grid.y > 65535 || grid.z > 65535) return hipErrorInvalidValue;
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, false, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, true, false>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<T, false, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), grid, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC);
  return hipGetLastError();
}

// ------------------------------------------------------------------ bf16 split
// (bf16 split helpers: qtt_device.hpp)
constexpr int SBM = 64, SBN = 64, SBK = 32;

// 16x16x32 bf16 MFMA operand layout: lane holds 8 consecutive k of
// A[lane % 16][8 * (lane / 16) + 0..7] and of B^T[lane % 16][8 * (lane / 16) + 0..7].
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_bf16split(int M, int N, int K,
                                                        const double* __restrict__ A, long lda,
                                                        const double* __restrict__ B, long ldb,
                                                        double* __restrict__ C, long ldc,
                                                        int nprod) {
  // [piece][row][k] with k contiguous so a lane reads its 8 k values as one 16-byte load
  __shared__ __attribute__((aligned(16))) unsigned short As[3][SBM][SBK + 8];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[3][SBN][SBK + 8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * SBM, n0 = blockIdx.x * SBN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  double accd[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) accd[i][j][v] = 0.0;

  for (int k0 = 0; k0 < K; k0 += SBK) {
    // 64 x 32 elements per operand = 2048, 8 per thread
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (!TA) {
        m = idx >> 5;
        k = idx & 31;
      } else {
        k = idx >> 6;
        m = idx & 63;
      }
      double v = 0.0;
      if (m0 + m < M && k0 + k < K)
        v = TA ? A[(long)(k0 + k) * lda + m0 + m] : A[(long)(m0 + m) * lda + k0 + k];
      unsigned short p0, p1, p2;
      split3(v, p0, p1, p2);
      As[0][m][k] = p0;
      As[1][m][k] = p1;
      As[2][m][k] = p2;
      int n;
      if (!TB) {
        k = idx >> 6;
        n = idx & 63;
      } else {
        n = idx >> 5;
        k = idx & 31;
      }
      double w = 0.0;
      if (n0 + n < N && k0 + k < K)
        w = TB ? B[(long)(n0 + n) * ldb + k0 + k] : B[(long)(k0 + k) * ldb + n0 + n];
      split3(w, p0, p1, p2);
      Bs[0][n][k] = p0;
      Bs[1][n][k] = p1;
      Bs[2][n][k] = p2;
    }
    __syncthreads();
    bf16x8_t a[3][2], b[3][2];
    const int kb = 8 * (lane >> 4);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int i = 0; i < 2; ++i) a[p][i] = *reinterpret_cast<const bf16x8_t*>(&As[p][wm + i * 16 + (lane & 15)][kb]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[p][j] = *reinterpret_cast<const bf16x8_t*>(&Bs[p][wn + j * 16 + (lane & 15)][kb]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // small products first, dominant product last, all within one 32-deep step
        float4_t lo = {0.f, 0.f, 0.f, 0.f};
        if (nprod >= 6) {
          lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], lo, 0, 0, 0);
          lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], lo, 0, 0, 0);
          lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], lo, 0, 0, 0);
        }
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], lo, 0, 0, 0);
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], lo, 0, 0, 0);
        float4_t hi = {0.f, 0.f, 0.f, 0.f};
        hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], hi, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) accd[i][j][v] += (double)hi[v] + (double)lo[v];
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) C[(long)gm * ldc + gn] = accd[i][j][v];
      }
}

// FP64 operands rounded once to FP32, FP32 MFMA accumulation per 16-deep step.
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_viaf32(int M, int N, int K, const double* __restrict__ A,
                                                     long lda, const double* __restrict__ B, long ldb,
                                                     double* __restrict__ C, long ldc) {
  __shared__ float As[BK][BM + PADM];
  __shared__ float Bs[BK][BN + PADM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (!TA) { m = idx >> 4; k = idx & 15; } else { k = idx >> 6; m = idx & 63; }
      float v = 0.f;
      if (m0 + m < M && k0 + k < K)
        v = (float)(TA ? A[(long)(k0 + k) * lda + m0 + m] : A[(long)(m0 + m) * lda + k0 + k]);
      As[k][m] = v;
      int n;
      if (!TB) { k = idx >> 6; n = idx & 63; } else { n = idx >> 4; k = idx & 15; }
      float w = 0.f;
      if (n0 + n < N && k0 + k < K)
        w = (float)(TB ? B[(long)(n0 + n) * ldb + k0 + k] : B[(long)(k0 + k) * ldb + n0 + n]);
      Bs[k][n] = w;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) C[(long)gm * ldc + gn] = (double)acc[i][j][v];
      }
}

// C = alpha A A^T + beta C for K <= 64 on the tiles on or below the
// diagonal: one workgroup per 32-row x 64-column tile, the tile's rows of A
// (as the left operand) and the 64 rows of its columns (as the right one)
// staged in LDS at once with coalesced loads, the product on FP64 MFMA
// 16x16x4 (wave w owns rows 16 (w / 2) and columns 32 (w % 2) of the tile:
// two 16 x 16 results; lane layout as in k_gemm).  Tiles wholly above the
// diagonal exit at once.
__global__ __launch_bounds__(256) void k_syrk_k64(int N, int K, double alpha, const double* __restrict__ A, long lda,
                                                  double beta, double* __restrict__ C, long ldc) {
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 64;
  if (j0 > i0 + 31) return;
  __shared__ double As[64][33];  // As[k][i] = A[i0 + i][k]
  __shared__ double Bs[64][65];  // Bs[k][j] = A[j0 + j][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < 32 * 64; e += 256) {
    const int i = e >> 6, k = e & 63;
    As[k][i] = (i0 + i < N && k < K) ? A[(long)(i0 + i) * lda + k] : 0.0;
  }
  for (int e = tid; e < 64 * 64; e += 256) {
    const int j = e >> 6, k = e & 63;
    Bs[k][j] = (j0 + j < N && k < K) ? A[(long)(j0 + j) * lda + k] : 0.0;
  }
  __syncthreads();
  const int ti = w >> 1, tj0 = 2 * (w & 1), il = lane & 15, kq = lane >> 4;
  double4_t acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) acc[t] = double4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const int k = 4 * ks + kq;
    const double a = As[k][16 * ti + il];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[k][16 * (tj0 + t) + il], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int col = j0 + 16 * (tj0 + t) + il;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = i0 + 16 * ti + kq + 4 * v;
      if (row < N && col < N) {
        double r = alpha * acc[t][v];
        if (beta != 0.0) r += beta * C[(long)row * ldc + col];
        C[(long)row * ldc + col] = r;
      }
    }
  }
}

}  // namespace

hipError_t gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, long lda, long sA, const double* B, long ldb, long sB,
                    double beta, double* C, long ldc, long sC, int batch) {
  return launch_gemm<double>(s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
}

hipError_t gemm_f64_lower_nt(hipStream_t s, int N, int K, double alpha, const double* A, long lda, double beta,
                             double* C, long ldc) {
  if (N <= 0) return hipSuccess;
  if (K <= 64) {
    const int nr = (N + 31) / 32, nc = (N + 63) / 64;
    if (nr > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_syrk_k64, dim3(nc, nr, 1), dim3(256), 0, s, N, K, alpha, A, lda, beta, C, ldc);
    return hipGetLastError();
  }
  const int nt = (N + BN - 1) / BN;
  if (nt > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_gemm<double, false, true, true>), dim3(nt, nt, 1), dim3(256), 0, s, N, N, K, alpha, A, lda,
                     0L, A, lda, 0L, beta, C, ldc, 0L);
  return hipGetLastError();
}

hipError_t gemm_f32(hipStream_t s, bool ta, bool tb, int M, int N, int K, float alpha,
                    const float* A, long lda, long sA, const float* B, long ldb, long sB,
                    float beta, float* C, long ldc, long sC, int batch) {
  return launch_gemm<float>(s, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
}

hipError_t gemm_bf16split(hipStream_t s, bool ta, bool tb, int M, int N, int K, const double* A,
                          long lda, const double* B, long ldb, double* C, long ldc, int nprod) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + SBN - 1) / SBN, (M + SBM - 1) / SBM, 1);
  if (grid.y > 65535) return hipErrorInvalidValue;
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm_bf16split<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, nprod);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm_bf16split<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, nprod);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm_bf16split<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, nprod);
  else
    hipLaunchKernelGGL((k_gemm_bf16split<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc, nprod);
  return hipGetLastError();
}

hipError_t gemm_f64_via_f32(hipStream_t s, bool ta, bool tb, int M, int N, int K, const double* A,
                            long lda, const double* B, long ldb, double* C, long ldc) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, 1);
  if (grid.y > 65535) return hipErrorInvalidValue;
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm_viaf32<false, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm_viaf32<true, false>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm_viaf32<false, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  else
    hipLaunchKernelGGL((k_gemm_viaf32<true, true>), grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

}  // namespace qtt
