// Householder panel factorisation by one workgroup (shared by the
// single-chain kernels and the batched persistent kernel).
//
// Row-major A (m x n).  A panel of up to 16 columns is held in registers
// (each thread owns RPT rows of the panel), one Householder reflector per
// column:
//     x = A[j:m, j], beta = -sign(x0) ||x||, tau = (beta - x0)/beta,
//     v = x / (x0 - beta) with v0 = 1,   H = I - tau v v^T,   H x = beta e0
// (tau = 0, H = I when x has no entries below the diagonal).  The same
// workgroup reduction that forms v^T A for the update also yields the
// column V^T v_j, from which the compact-WY factor T (H_1..H_b = I - V T V^T,
// T upper triangular) is built column by column.
#pragma once

#include "qtt_device.hpp"

namespace qtt {

// stage (optional, NT * (PW + 1) doubles of LDS): when given, the panel is
// moved between global memory and registers through LDS in row-contiguous,
// coalesced order (a thread's own row segment read directly would touch one
// cache line per lane and instruction).  tau_out (optional) receives the pw
// reflector coefficients.
template <int NT, int RPT, int PW>
__device__ __forceinline__ void qr_panel_dev(double* __restrict__ A, long lda, int m, int j0, int pw,
                                             double* __restrict__ Tout, double* __restrict__ stage = nullptr,
                                             double* __restrict__ tau_out = nullptr) {
  constexpr int NW = NT / 64;
  __shared__ double red[NT];
  __shared__ double bc[16];
  __shared__ double sc[NW];
  __shared__ double Ts[16][17];
  __shared__ double alphaS;
  const int tid = threadIdx.x;
  const int mp = m - j0;
  constexpr int SW = PW + 1;  // LDS row stride (odd: conflict-free row reads)
  double a[RPT][PW];
  if (stage) {
    // all global loads first, in coalesced order: a[r][q] = element
    // e = tid + NT q of row block r (row e / PW, column e % PW) ...
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = tid + NT * q;
        const int gr = r * NT + e / PW, c = e % PW;
        a[r][q] = (gr < mp && c < pw) ? A[(long)(j0 + gr) * lda + j0 + c] : 0.0;
      }
    // ... then one LDS transpose per row block into a[r][c] = row tid + r NT
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = tid + NT * q;
        stage[(e / PW) * SW + e % PW] = a[r][q];
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < PW; ++c) a[r][c] = stage[tid * SW + c];
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = tid + r * NT;
#pragma unroll
      for (int c = 0; c < PW; ++c) a[r][c] = (lr < mp && c < pw) ? A[(long)(j0 + lr) * lda + j0 + c] : 0.0;
    }
  }
  for (int t = tid; t < 16 * 17; t += NT) (&Ts[0][0])[t] = 0.0;

#pragma unroll
  for (int j = 0; j < PW; ++j) {
    if (j < pw) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int lr = tid + r * NT;
        if (lr > j && lr < mp) s += a[r][j] * a[r][j];
      }
      if (tid == j) alphaS = a[0][j];
      s = block_sum<NT>(s, sc);
      const double alpha = alphaS;
      double tau, beta, scale;
      if (s == 0.0) {
        tau = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int lr = tid + r * NT;
        if (lr > j && lr < mp) a[r][j] *= scale;
      }
      if (tid == j) a[0][j] = beta;
      // p[c] (c > j): v_j^T A[:, c];  p[c] (c < j): v_c^T v_j  (column j of V^T V)
      double p[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) p[c] = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int lr = tid + r * NT;
        if (lr >= j && lr < mp) {
          const double v = (lr == j) ? 1.0 : a[r][j];
#pragma unroll
          for (int c = 0; c < PW; ++c) {
            if (c > j) {
              p[c] += v * a[r][c];
            } else if (c < j) {
              const double vc = (lr > c) ? a[r][c] : (lr == c ? 1.0 : 0.0);
              p[c] += v * vc;
            }
          }
        }
      }
      block_sum16<NT>(p, red, bc);
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int lr = tid + r * NT;
        if (lr >= j && lr < mp) {
          const double v = (lr == j) ? 1.0 : a[r][j];
#pragma unroll
          for (int c = 0; c < PW; ++c)
            if (c > j) a[r][c] -= tau * v * bc[c];
        }
      }
      // T[0:j, j] = -tau T[0:j, 0:j] (V^T v_j)[0:j],  T[j][j] = tau
      if (tid < j) {
        double acc = 0.0;
        for (int l = tid; l < j; ++l) acc += Ts[tid][l] * bc[l];
        Ts[tid][j] = -tau * acc;
      }
      if (tid == j) Ts[j][j] = tau;
      __syncthreads();
    }
  }
  if (stage) {
    // LDS transposes back to coalesced order, then all global stores
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
      for (int c = 0; c < PW; ++c) stage[tid * SW + c] = a[r][c];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = tid + NT * q;
        a[r][q] = stage[(e / PW) * SW + e % PW];
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = tid + NT * q;
        const int gr = r * NT + e / PW, c = e % PW;
        if (gr < mp && c < pw) A[(long)(j0 + gr) * lda + j0 + c] = a[r][q];
      }
  } else {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = tid + r * NT;
      if (lr < mp) {
#pragma unroll
        for (int c = 0; c < PW; ++c)
          if (c < pw) A[(long)(j0 + lr) * lda + j0 + c] = a[r][c];
      }
    }
  }
  for (int t = tid; t < 256; t += NT) Tout[t] = Ts[t >> 4][t & 15];
  if (tau_out && tid < pw) tau_out[tid] = Ts[tid][tid];
}


// Block reflector (V, op(T)) applied by one workgroup to the 16 columns
// [col0, cend) of Y, all rows [0, mp) of the block:
//   W = V^T Y, W <- op(T) W, Y <- Y - V W.
// NT threads: thread (g, c) owns column c and rows g (mod NT/16).
// red: LDS [NT/16][16][17], wsh / w2sh / tsh: LDS [16][17].
__device__ __forceinline__ void load_vrow16(const double* __restrict__ arow, int lr, int pw, double (&v)[16]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (i >= pw) ? 0.0 : (lr > i ? arow[i] : (lr == i ? 1.0 : 0.0));
}

template <int NT>
__device__ __forceinline__ void apply_tile_dev(const double* __restrict__ Ab, long lda, int mp, int pw,
                                               const double* __restrict__ T, double* __restrict__ Yb, long ldy,
                                               int col0, int cend, int trans, double (*red)[16][17],
                                               double (*wsh)[17], double (*w2sh)[17], double (*tsh)[17]) {
  constexpr int G = NT / 16;
  const int tid = threadIdx.x;
  const int c = tid & 15, g = tid >> 4;
  const int col = col0 + c;
  const bool valid = col < cend;
  for (int t = tid; t < 256; t += NT) tsh[t >> 4][t & 15] = T[t];
  double w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = 0.0;
  for (int lr = g; lr < mp; lr += G) {
    const double y = valid ? Yb[(long)lr * ldy + col] : 0.0;
    double v[16];
    load_vrow16(Ab + (long)lr * lda, lr, pw, v);
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] += v[i] * y;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) red[g][i][c] = w[i];
  __syncthreads();
  for (int t = tid; t < 256; t += NT) {
    const int i = t >> 4, cc = t & 15;
    double sum = 0.0;
    for (int q = 0; q < G; ++q) sum += red[q][i][cc];
    wsh[i][cc] = sum;
  }
  __syncthreads();
  for (int t = tid; t < 256; t += NT) {
    const int i = t >> 4, cc = t & 15;
    double sum = 0.0;
#pragma unroll
    for (int l = 0; l < 16; ++l) sum += (trans ? tsh[l][i] : tsh[i][l]) * wsh[l][cc];
    w2sh[i][cc] = sum;
  }
  __syncthreads();
  if (valid) {
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] = w2sh[i][c];
    for (int lr = g; lr < mp; lr += G) {
      double v[16];
      load_vrow16(Ab + (long)lr * lda, lr, pw, v);
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) sum += v[i] * w[i];
      Yb[(long)lr * ldy + col] -= sum;
    }
  }
  __syncthreads();
}

}  // namespace qtt
