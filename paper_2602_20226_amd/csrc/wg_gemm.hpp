// Workgroup-level GEMM on the bf16 matrix cores for the batched kernel.
//
// C(m, n) = sum_k A(m, k) B(k, n) by one 256-thread workgroup: FP64 operands
// are split into three bf16 pieces on the way into LDS (a = a0 + a1 + a2,
// each piece the RNE bf16 of the remainder) and the six cross products run on
// MFMA 16x16x32 bf16, smallest first, with FP32 accumulation inside each
// 32-deep k step; the step sums are added in FP64 registers.  Operands are
// read and the result is written through functors, so strided and gathered
// layouts (the bond products of a QTT sweep) need no copies.
//
// Output tiles are TM x TN (TM, TN in {32, 64}); the four waves form a 2 x 2
// grid of (TM/2) x (TN/2) wave tiles made of 16 x 16 MFMA tiles.  Which tile
// shape runs for a call is chosen per shape bucket (gemm_bucket) from a
// TileMap measured by the batch plan's tuner.
#pragma once

#include "qtt_device.hpp"

namespace qtt {

// LDS staging of one 32-deep step: three bf16 pieces of each operand, k
// contiguous so that a lane reads its 8 k values with one 16-byte load.
struct GemmTiles {
  unsigned short A[3][64][40];
  unsigned short B[3][64][40];
};

constexpr int kTileVariants = 4;  // 0: 64x64, 1: 64x32, 2: 32x64, 3: 32x32
constexpr int kGemmBuckets = 8;

struct TileMap {
  unsigned char v[kGemmBuckets];
};

// Shape bucket: M > 32, N > 32, K > 64 (one bit each).
__host__ __device__ inline int gemm_bucket(int M, int N, int K) {
  return (M > 32 ? 1 : 0) | (N > 32 ? 2 : 0) | (K > 64 ? 4 : 0);
}

template <int TM, int TN, class LA, class LB, class SC>
__device__ void wg_gemm_split_tile(int M, int N, int K, const LA& la, const LB& lb, const SC& sc, GemmTiles& g) {
  constexpr int WM = TM / 2, WN = TN / 2;
  constexpr int FI = WM / 16, FJ = WN / 16;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
  const int kb = 8 * (lane >> 4);
  for (int m0 = 0; m0 < M; m0 += TM) {
    for (int n0 = 0; n0 < N; n0 += TN) {
      double acc[FI][FJ][4];
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[i][j][v] = 0.0;
      for (int k0 = 0; k0 < K; k0 += 32) {
        for (int e = tid; e < TM * 32; e += 256) {
          const int m = e >> 5, k = e & 31;
          const double v = (m0 + m < M && k0 + k < K) ? la(m0 + m, k0 + k) : 0.0;
          unsigned short p0, p1, p2;
          split3(v, p0, p1, p2);
          g.A[0][m][k] = p0;
          g.A[1][m][k] = p1;
          g.A[2][m][k] = p2;
        }
        for (int e = tid; e < TN * 32; e += 256) {
          const int k = e / TN, n = e % TN;
          const double v = (n0 + n < N && k0 + k < K) ? lb(k0 + k, n0 + n) : 0.0;
          unsigned short p0, p1, p2;
          split3(v, p0, p1, p2);
          g.B[0][n][k] = p0;
          g.B[1][n][k] = p1;
          g.B[2][n][k] = p2;
        }
        __syncthreads();
        bf16x8_t a[3][FI], b[3][FJ];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
#pragma unroll
          for (int i = 0; i < FI; ++i)
            a[p][i] = *reinterpret_cast<const bf16x8_t*>(&g.A[p][wm + i * 16 + (lane & 15)][kb]);
#pragma unroll
          for (int j = 0; j < FJ; ++j)
            b[p][j] = *reinterpret_cast<const bf16x8_t*>(&g.B[p][wn + j * 16 + (lane & 15)][kb]);
        }
#pragma unroll
        for (int i = 0; i < FI; ++i)
#pragma unroll
          for (int j = 0; j < FJ; ++j) {
            float4_t lo = {0.f, 0.f, 0.f, 0.f};
            lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2][i], b[0][j], lo, 0, 0, 0);
            lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[1][j], lo, 0, 0, 0);
            lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[2][j], lo, 0, 0, 0);
            lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], lo, 0, 0, 0);
            lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], lo, 0, 0, 0);
            float4_t hi = {0.f, 0.f, 0.f, 0.f};
            hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], hi, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[i][j][v] += (double)hi[v] + (double)lo[v];
          }
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gm = m0 + wm + i * 16 + 4 * (lane >> 4) + v;
            const int gn = n0 + wn + j * 16 + (lane & 15);
            if (gm < M && gn < N) sc(gm, gn, acc[i][j][v]);
          }
    }
  }
  __syncthreads();
}

template <class LA, class LB, class SC>
__device__ void wg_gemm_split_var(int variant, int M, int N, int K, const LA& la, const LB& lb, const SC& sc,
                                  GemmTiles& g) {
  switch (variant) {
    case 1:
      wg_gemm_split_tile<64, 32>(M, N, K, la, lb, sc, g);
      break;
    case 2:
      wg_gemm_split_tile<32, 64>(M, N, K, la, lb, sc, g);
      break;
    case 3:
      wg_gemm_split_tile<32, 32>(M, N, K, la, lb, sc, g);
      break;
    default:
      wg_gemm_split_tile<64, 64>(M, N, K, la, lb, sc, g);
      break;
  }
}

template <class LA, class LB, class SC>
__device__ void wg_gemm_split(const TileMap& tm, int M, int N, int K, const LA& la, const LB& lb, const SC& sc,
                              GemmTiles& g) {
  if (M <= 0 || N <= 0) return;
  wg_gemm_split_var(tm.v[gemm_bucket(M, N, K)], M, N, K, la, lb, sc, g);
}

}  // namespace qtt
