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
// column V^T v_j of the earlier reflectors, from which the compact-WY factor
// T (H_1..H_b = I - V T V^T, T upper triangular) grows one column per step:
// T[0:j, j] = -tau_j T[0:j, 0:j] (V^T v_j)[0:j].
//
// Each column costs one single-barrier workgroup sum for the norm and one
// for the PW dot products (8 values by a 3-step row transpose, 16 by a
// 4-step one); the panel is bound by its vector-ALU work, so the
// reductions are kept short and the column loop is unrolled (every register
// index a constant).
#pragma once

#include "qtt_device.hpp"

namespace qtt {

// stage (optional, NT * (PW + 1) doubles of LDS): when given, the panel is
// moved between global memory and registers in coalesced order (16-byte
// accesses when the panel is full width and aligned), all loads issued
// before the LDS transposes into the per-thread row layout; a thread's own
// row segment read directly would touch one cache line per lane and
// instruction.  T (16 x 16, row-major, zero outside pw x pw) goes to Tout
// and the coefficients tau to tau_out (optional).
// 1/x over the whole normal range: double-precision hardware estimate
// (relative error e ~2^-24) and one third-order correction r (1 + e + e^2),
// within an ulp or two; the two reciprocals of a reflector need no IEEE
// division.
__device__ __forceinline__ double rcp_f64_full(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

template <int NT, int RPT, int PW>
__device__ __forceinline__ void qr_panel_dev(double* __restrict__ A, long lda, int m, int j0, int pw,
                                             double* __restrict__ Tout, double* __restrict__ stage = nullptr,
                                             double* __restrict__ tau_out = nullptr) {
  constexpr int NW = NT / 64;
  constexpr int SW = PW + 1;
  constexpr int HP = PW / 2;  // column pairs
  static_assert(PW == 8 || PW == 16, "panel width 8 or 16");
  __shared__ double red[2 * NW * PW];
  __shared__ double sc[2 * NW];
  __shared__ double alphaS[2];
  __shared__ double Ts[16][17];  // T, built one column per step
  const int tid = threadIdx.x;
  const int mp = m - j0;
  double a[RPT][PW];
  const bool pairs = stage && (pw == PW) && ((lda & 1) == 0) && ((j0 & 1) == 0);
  if (!stage) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = tid + r * NT;
#pragma unroll
      for (int c = 0; c < PW; ++c) a[r][c] = (lr < mp && c < pw) ? A[(long)(j0 + lr) * lda + j0 + c] : 0.0;
    }
  } else if (pairs) {
    // 16-byte loads: pair e = tid + NT q of row block r -> row e / HP, columns 2 (e % HP) + {0, 1}
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int q = 0; q < HP; ++q) {
        const int e = tid + NT * q;
        const int gr = r * NT + e / HP, c = 2 * (e % HP);
        double2 v = make_double2(0.0, 0.0);
        if (gr < mp) v = *reinterpret_cast<const double2*>(A + (long)(j0 + gr) * lda + j0 + c);
        a[r][2 * q] = v.x;
        a[r][2 * q + 1] = v.y;
      }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
      for (int q = 0; q < HP; ++q) {
        const int e = tid + NT * q;
        const int rr = e / HP, c = 2 * (e % HP);
        stage[rr * SW + c] = a[r][2 * q];
        stage[rr * SW + c + 1] = a[r][2 * q + 1];
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < PW; ++c) a[r][c] = stage[tid * SW + c];
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int q = 0; q < PW; ++q) {
        const int e = tid + NT * q;
        const int gr = r * NT + e / PW, c = e % PW;
        a[r][q] = (gr < mp && c < pw) ? A[(long)(j0 + gr) * lda + j0 + c] : 0.0;
      }
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
  }
  for (int t = tid; t < 16 * 17; t += NT) (&Ts[0][0])[t] = 0.0;
  // Rows outside the panel are zero and stay zero; only rows of r = 0 can
  // lie at or above the diagonal (j < 16 <= NT).
#pragma unroll
  for (int j = 0; j < PW; ++j) {
    if (j < pw) {
      const int par = j & 1;
      double sp[3] = {0.0, 0.0, 0.0};  // three partial sums: a third of the dependent chain
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r > 0 || tid > j) sp[r % 3] += a[r][j] * a[r][j];
      if (tid == j) alphaS[par] = a[0][j];
      double s = wg_sum1<NT>((sp[0] + sp[1]) + sp[2], sc, par);
      const double alpha = alphaS[par];
      double tau, beta, scale;
      if (s == 0.0) {
        tau = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        tau = (beta - alpha) * rcp_f64_full(beta);
        scale = rcp_f64_full(alpha - beta);
      }
      double v[RPT];
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        if (r > 0 || tid > j) a[r][j] *= scale;
        v[r] = (r > 0 || tid > j) ? a[r][j] : (tid == j ? 1.0 : 0.0);
      }
      if (tid == j) a[0][j] = beta;
      // columns still to come get v^T a (the update), columns already
      // factored give v_l^T v_j (rows >= j lie below their diagonal)
      double p[PW], d[PW];
#pragma unroll
      for (int c = 0; c < PW; ++c) p[c] = 0.0;
#pragma unroll
      for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int c = 0; c < PW; ++c)
          if (c != j) p[c] += v[r] * a[r][c];
      wg_sum_vals<NT, PW>(p, red, par, d);
#pragma unroll
      for (int r = 0; r < RPT; ++r) v[r] *= tau;
#pragma unroll
      for (int c = j + 1; c < PW; ++c) {
        if (c < pw) {
#pragma unroll
          for (int r = 0; r < RPT; ++r) a[r][c] -= v[r] * d[c];
        }
      }
      // column j of T
      if (tid < j) {
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < j; ++l)
          if (l >= tid) acc += Ts[tid][l] * d[l];
        Ts[tid][j] = -tau * acc;
      }
      if (tid == j) Ts[j][j] = tau;
    }
  }
  __syncthreads();
  for (int t = tid; t < 256; t += NT) Tout[t] = Ts[t >> 4][t & 15];
  if (tau_out && tid < pw) tau_out[tid] = Ts[tid][tid];
  if (!stage) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int lr = tid + r * NT;
      if (lr < mp) {
#pragma unroll
        for (int c = 0; c < PW; ++c)
          if (c < pw) A[(long)(j0 + lr) * lda + j0 + c] = a[r][c];
      }
    }
  } else if (pairs) {
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
#pragma unroll
      for (int c = 0; c < PW; ++c) stage[tid * SW + c] = a[r][c];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < HP; ++q) {
        const int e = tid + NT * q;
        const int rr = e / HP, c = 2 * (e % HP);
        a[r][2 * q] = stage[rr * SW + c];
        a[r][2 * q + 1] = stage[rr * SW + c + 1];
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int q = 0; q < HP; ++q) {
        const int e = tid + NT * q;
        const int gr = r * NT + e / HP, c = 2 * (e % HP);
        if (gr < mp) *reinterpret_cast<double2*>(A + (long)(j0 + gr) * lda + j0 + c) = make_double2(a[r][2 * q], a[r][2 * q + 1]);
      }
  } else {
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
  }
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
