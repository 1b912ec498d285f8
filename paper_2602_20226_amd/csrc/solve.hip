// Kernels of the DMRG-like linear solver (Sec. 5): the local matrix of the
// energy <x, W x> - 2 <x, b> for one core or a two-core super-core, the
// operator-core steps of the three-layer environments <x|W|x>, the product
// of two adjacent operator cores, and the upper-triangular solve that ends
// the local QR solve.  FP64 throughout (the local problems decide the
// solution's accuracy; they are small).
#include "qtt_device.hpp"
#include "qtt_internal.hpp"

#include <algorithm>

namespace qtt {

namespace {

inline int grid_of(long n) {
  long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > (1 << 20)) g = 1 << 20;
  return (int)g;
}

// A[(a,i,c),(x,j,y)] = sum_{al,be} LW[a,al,x] Wl[al,i,j,be] RW[c,be,y]
__global__ void k_local_matrix(const double* __restrict__ LW, const double* __restrict__ Wl,
                               const double* __restrict__ RW, int r0, int P, int r1, int w0, int w1,
                               double* __restrict__ A) {
  const long N = (long)r0 * P * r1;
  const long total = N * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / N, col = e % N;
    const int c = (int)(row % r1), i = (int)((row / r1) % P), a = (int)(row / ((long)r1 * P));
    const int y = (int)(col % r1), j = (int)((col / r1) % P), x = (int)(col / ((long)r1 * P));
    double acc = 0.0;
    for (int al = 0; al < w0; ++al) {
      const double l = LW[((long)a * w0 + al) * r0 + x];
      if (l == 0.0) continue;
      const double* wrow = Wl + (((long)al * P + i) * P + j) * w1;
      double s = 0.0;
      for (int be = 0; be < w1; ++be) s += wrow[be] * RW[((long)c * w1 + be) * r1 + y];
      acc += l * s;
    }
    A[e] = acc;
  }
}

// T2[a][i][be][y] = sum_{al,j} T1[a][al][j][y] W[al][i][j][be]
__global__ void k_env3_left_mid(const double* __restrict__ T1, const double* __restrict__ W, int r0, int w0, int d,
                                int w1, int r1, double* __restrict__ T2) {
  const long total = (long)r0 * d * w1 * r1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int y = (int)(t % r1);
    t /= r1;
    const int be = (int)(t % w1);
    t /= w1;
    const int i = (int)(t % d);
    const long a = t / d;
    double acc = 0.0;
    for (int al = 0; al < w0; ++al)
      for (int j = 0; j < d; ++j)
        acc += T1[((a * w0 + al) * d + j) * r1 + y] * W[(((long)al * d + i) * d + j) * w1 + be];
    T2[e] = acc;
  }
}

// U2[i][c][al][x] = sum_{j,be} W[al][i][j][be] U1[x][j][c][be]
__global__ void k_env3_right_mid(const double* __restrict__ U1, const double* __restrict__ W, int r0, int w0, int d,
                                 int w1, int r1, double* __restrict__ U2) {
  const long total = (long)d * r1 * w0 * r0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int x = (int)(t % r0);
    t /= r0;
    const int al = (int)(t % w0);
    t /= w0;
    const int c = (int)(t % r1);
    const int i = (int)(t / r1);
    double acc = 0.0;
    for (int j = 0; j < d; ++j)
      for (int be = 0; be < w1; ++be)
        acc += W[(((long)al * d + i) * d + j) * w1 + be] * U1[(((long)x * d + j) * r1 + c) * w1 + be];
    U2[e] = acc;
  }
}

// G[al][(i1,i2)][(j1,j2)][ga] = sum_be W1[al][i1][j1][be] W2[be][i2][j2][ga]
__global__ void k_mpo_pair(const double* __restrict__ W1, const double* __restrict__ W2, int w0, int d1, int w1,
                           int d2, int w2, double* __restrict__ G) {
  const int P = d1 * d2;
  const long total = (long)w0 * P * P * w2;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int ga = (int)(t % w2);
    t /= w2;
    const int J = (int)(t % P);
    t /= P;
    const int I = (int)(t % P);
    const int al = (int)(t / P);
    const int i1 = I / d2, i2 = I % d2, j1 = J / d2, j2 = J % d2;
    double acc = 0.0;
    for (int be = 0; be < w1; ++be)
      acc += W1[(((long)al * d1 + i1) * d1 + j1) * w1 + be] * W2[(((long)be * d2 + i2) * d2 + j2) * w2 + ga];
    G[e] = acc;
  }
}

// 1/x over the whole normal range: double-precision hardware estimate and
// one third-order correction (within an ulp or two; no IEEE division).
__device__ __forceinline__ double rcp_full(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Cholesky of the nb x nb diagonal block at A[j0][j0] (nb <= 64, lower
// triangle used and overwritten by L) and the inverse of L into Linv
// (64 x 64, row-major, zero outside the nb x nb lower triangle).  The block
// is padded with the identity to 64 x 64 and held in registers, a 4 x 4
// tile per thread (256 threads, 16 x 16 tiles), together with Y, which
// starts as I and ends as L^{-1}.  Four columns K = k..k+3 per step: the
// threads holding them publish the 64 x 4 column panel and those holding
// rows K of Y publish them (double-buffered LDS, one barrier per step);
// every thread then factors the 4 x 4 diagonal block Ld (and inverts it,
// Li) in registers, forms the multipliers l_i = Li p_i of its rows and
// columns from the published panel rows p_i (zero for rows and columns up
// to k+3), the rows of the inverse X_K = Li Y_K, and applies the rank-4
// updates a -= l l^T (only the trailing lower triangle is touched where it
// matters; the upper triangle, never read, takes what it gets) and
// Y -= l X_K; rows K of Y become X_K and columns K of L go to LDS.  A pivot
// that is not positive gives NaN, which propagates to the solution.
__global__ __launch_bounds__(256) void k_potrf_inv(double* __restrict__ A, long lda, int j0, int nb,
                                                   double* __restrict__ Linv) {
  __shared__ double P[2][64][5];
  __shared__ double Yr[2][4][65];
  __shared__ double Ls[64][65];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int i0 = 4 * tr, c0 = 4 * tc;
  double a[4][4], y[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + u, j = c0 + v;
      a[u][v] = (i < nb && j <= i) ? A[(long)(j0 + i) * lda + j0 + j] : (i == j ? 1.0 : 0.0);
      y[u][v] = (i == j) ? 1.0 : 0.0;
    }
  for (int k = 0; k < 64; k += 4) {
    const int buf = (k >> 2) & 1;
    if (tc == (k >> 2)) {  // this tile's columns are K: publish them for its rows
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[buf][i0 + u][v] = a[u][v];
    }
    if (tr == (k >> 2)) {  // this tile's rows are K: publish them for its columns
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) Yr[buf][u][c0 + v] = y[u][v];
    }
    __syncthreads();
    // all LDS reads of the step first
    double d[4][4], pi[4][4], pj[4][4], yk[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        d[t][q] = P[buf][k + t][q];
        pi[t][q] = P[buf][i0 + t][q];
        pj[t][q] = P[buf][c0 + t][q];
        yk[t][q] = Yr[buf][t][c0 + q];
      }
    // Ld = chol(D), Li = Ld^{-1} (lower, 4 x 4), written out
    const double l00 = sqrt(d[0][0]), r0 = rcp_full(l00);
    const double l10 = d[1][0] * r0, l20 = d[2][0] * r0, l30 = d[3][0] * r0;
    const double l11 = sqrt(d[1][1] - l10 * l10), r1 = rcp_full(l11);
    const double l21 = (d[2][1] - l20 * l10) * r1, l31 = (d[3][1] - l30 * l10) * r1;
    const double l22 = sqrt(d[2][2] - l20 * l20 - l21 * l21), r2 = rcp_full(l22);
    const double l32 = (d[3][2] - l30 * l20 - l31 * l21) * r2;
    const double l33 = sqrt(d[3][3] - l30 * l30 - l31 * l31 - l32 * l32), r3 = rcp_full(l33);
    const double m10 = -l10 * r0 * r1;
    const double m21 = -l21 * r1 * r2;
    const double m20 = -(l20 * r0 + l21 * m10) * r2;
    const double m32 = -l32 * r2 * r3;
    const double m31 = -(l31 * r1 + l32 * m21) * r3;
    const double m30 = -(l30 * r0 + l31 * m10 + l32 * m20) * r3;
    const double Li[4][4] = {{r0, 0.0, 0.0, 0.0}, {m10, r1, 0.0, 0.0}, {m20, m21, r2, 0.0}, {m30, m31, m32, r3}};
    const double L[4][4] = {{l00, 0.0, 0.0, 0.0}, {l10, l11, 0.0, 0.0}, {l20, l21, l22, 0.0}, {l30, l31, l32, l33}};
    // multipliers of this tile's rows and columns (zero up to k+3) and X_K
    double li[4][4], lj[4][4], xk[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double su = 0.0, sv = 0.0, sx = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q <= t) {
            su += Li[t][q] * pi[u][q];
            sv += Li[t][q] * pj[u][q];
            sx += Li[t][q] * yk[q][u];
          }
        li[u][t] = (i0 + u > k + 3) ? su : 0.0;
        lj[u][t] = (c0 + u > k + 3) ? sv : 0.0;
        xk[t][u] = sx;  // X_K[t][c0 + u]
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a[u][v] = fma(-li[u][t], lj[v][t], a[u][v]);
          y[u][v] = fma(-li[u][t], xk[t][v], y[u][v]);
        }
    if (tr == (k >> 2)) {  // rows K of the inverse
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) y[u][v] = xk[u][v];
    }
    if (tc == 0 && tr != (k >> 2)) {  // columns K of L outside the diagonal block
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int i = i0 + u;
          Ls[i][k + t] = (i > k + 3) ? li[u][t] : 0.0;
        }
    }
    if (tid < 16) {  // the diagonal block of L (selects: no run-time index into registers)
      const int t = tid >> 2, q = tid & 3;
      double v = 0.0;
#pragma unroll
      for (int tt = 0; tt < 4; ++tt)
#pragma unroll
        for (int qq = 0; qq <= tt; ++qq) v = (t == tt && q == qq) ? L[tt][qq] : v;
      Ls[k + t][k + q] = v;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + u, j = c0 + v;
      if (i < nb && j <= i) A[(long)(j0 + i) * lda + j0 + j] = Ls[i][j];
      Linv[i * 64 + j] = (i < nb && j < nb) ? y[u][v] : 0.0;
    }
}

// Wave sum, every lane ends with the total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

constexpr int kCholMaxN = 4096;

// y <- L^{-1} y with L (N x N, lower triangle of L, leading dimension ldl)
// given with the inverses of its 64 x 64 diagonal blocks (Linv, one 64 x 64
// block after the other): left-looking by blocks, r_B = y_B - L[B, 0:k0]
// y[0:k0] (rows of L read contiguously, one wave per row, lanes along it),
// y_B = Linv_B r_B.  One workgroup, y held in LDS, fixed operation order.
__global__ __launch_bounds__(1024) void k_chol_fwd(const double* __restrict__ L, int N, long ldl,
                                                   const double* __restrict__ Linv, double* __restrict__ y) {
  __shared__ double ys[kCholMaxN];
  __shared__ double rb[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < N; i += blockDim.x) ys[i] = y[i];
  __syncthreads();
  for (int k0 = 0, b = 0; k0 < N; k0 += 64, ++b) {
    const int nb = min(64, N - k0);
    // rows r = wave + nw q of the block, four at a time (independent loads)
    for (int r0 = wave; r0 < nb; r0 += 4 * nw) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      const double* row[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) row[q] = L + (long)(k0 + min(r0 + q * nw, nb - 1)) * ldl;
      for (int c = lane; c < k0; c += 64) {
        const double yc = ys[c];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += row[q][c] * yc;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double t = wave_sum(acc[q]);
        const int r = r0 + q * nw;
        if (lane == 0 && r < nb) rb[r] = ys[k0 + r] - t;
      }
    }
    __syncthreads();
    const double* Li = Linv + (long)b * 4096;
    for (int r = wave; r < nb; r += nw) {
      double acc = (lane < nb) ? Li[r * 64 + lane] * rb[lane] : 0.0;
      acc = wave_sum(acc);
      if (lane == 0) ys[k0 + r] = acc;
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += blockDim.x) y[i] = ys[i];
}

// x <- L^{-T} x with L and Linv as in k_chol_fwd: by blocks from the last,
// r_B = x_B - L[k1:N, B]^T x[k1:N] (rows of L read contiguously, lanes
// along the block's 64 columns, waves over rows, partial sums added in
// fixed order), x_B = Linv_B^T r_B.  One workgroup, x held in LDS.
__global__ __launch_bounds__(1024) void k_chol_bwd(const double* __restrict__ L, int N, long ldl,
                                                   const double* __restrict__ Linv, double* __restrict__ x) {
  __shared__ double xs[kCholMaxN];
  __shared__ double part[16][64];
  __shared__ double rb[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int i = tid; i < N; i += blockDim.x) xs[i] = x[i];
  __syncthreads();
  const int nblk = (N + 63) / 64;
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = 64 * b, k1 = min(N, k0 + 64), nb = k1 - k0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (lane < nb) {
      const double* col = L + k0 + lane;
      int i = k1 + wave;
      for (; i + 3 * nw < N; i += 4 * nw) {
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += col[(long)(i + q * nw) * ldl] * xs[i + q * nw];
      }
      for (; i < N; i += nw) acc[0] += col[(long)i * ldl] * xs[i];
    }
    part[wave][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (wave == 0) {
      double sum = 0.0;
      for (int w = 0; w < nw; ++w) sum += part[w][lane];
      rb[lane] = (lane < nb) ? xs[k0 + lane] - sum : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      const double* Li = Linv + (long)b * 4096;
      double s = 0.0;
      for (int r = 0; r < nb; ++r) s += Li[r * 64 + lane] * rb[r];
      if (lane < nb) xs[k0 + lane] = s;
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += blockDim.x) x[i] = xs[i];
}

}  // namespace

hipError_t local_matrix(hipStream_t s, const double* LW, const double* Wl, const double* RW, int r0, int P, int r1,
                        int w0, int w1, double* A) {
  const long N = (long)r0 * P * r1;
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_local_matrix, dim3(grid_of(N * N)), dim3(256), 0, s, LW, Wl, RW, r0, P, r1, w0, w1, A);
  return hipGetLastError();
}

hipError_t env3_left_mid(hipStream_t s, const double* T1, const double* W, int r0, int w0, int d, int w1, int r1,
                         double* T2) {
  const long total = (long)r0 * d * w1 * r1;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_env3_left_mid, dim3(grid_of(total)), dim3(256), 0, s, T1, W, r0, w0, d, w1, r1, T2);
  return hipGetLastError();
}

hipError_t env3_right_mid(hipStream_t s, const double* U1, const double* W, int r0, int w0, int d, int w1, int r1,
                          double* U2) {
  const long total = (long)d * r1 * w0 * r0;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_env3_right_mid, dim3(grid_of(total)), dim3(256), 0, s, U1, W, r0, w0, d, w1, r1, U2);
  return hipGetLastError();
}

hipError_t mpo_pair(hipStream_t s, const double* W1, const double* W2, int w0, int d1, int w1, int d2, int w2,
                    double* G) {
  const long total = (long)w0 * d1 * d2 * d1 * d2 * w2;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mpo_pair, dim3(grid_of(total)), dim3(256), 0, s, W1, W2, w0, d1, w1, d2, w2, G);
  return hipGetLastError();
}

hipError_t chol_solve(hipStream_t s, double* A, int N, long lda, double* x, double* work) {
  if (N <= 0) return hipSuccess;
  if (N > kCholMaxN) return hipErrorInvalidValue;
  const int nblk = (N + 63) / 64;
  double* Linv = work;                   // nblk blocks of 64 x 64
  double* P = work + (long)nblk * 4096;  // (N - 64) x 64 panel
  hipError_t e;
  for (int b = 0; b < nblk; ++b) {
    const int j0 = 64 * b, nb = std::min(64, N - j0);
    double* Li = Linv + (long)b * 4096;
    if (prof::active(prof::CHOL_BLOCK))
      prof::begin(s, prof::CHOL_BLOCK, 8.0 * ((double)nb * nb + 4096.0), 2.0 * nb * nb * nb / 3.0);
    hipLaunchKernelGGL(k_potrf_inv, dim3(1), dim3(256), 0, s, A, lda, j0, nb, Li);
    prof::end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int mr = N - j0 - nb;
    if (mr <= 0) break;
    double* A21 = A + (long)(j0 + nb) * lda + j0;
    // L21 = A21 L11^{-T}, then A22 -= L21 L21^T (the whole square; only its lower triangle is read later)
    if ((e = gemm_f64(s, false, true, mr, nb, nb, 1.0, A21, lda, 0, Li, 64, 0, 0.0, P, nb, 0, 1)) != hipSuccess)
      return e;
    if ((e = copy_pad_rows(s, P, mr, nb, nb, A21, mr, lda)) != hipSuccess) return e;
    // algorithmic work: the lower triangle of the update, mr^2 nb FLOP
    if (prof::active(prof::CHOL_UPDATE))
      prof::begin(s, prof::CHOL_UPDATE, 8.0 * ((double)mr * nb + (double)mr * mr), (double)mr * mr * nb);
    e = gemm_f64(s, false, true, mr, mr, nb, -1.0, P, nb, 0, P, nb, 0, 1.0, A21 + nb, lda, 0, 1);
    prof::end(s);
    if (e != hipSuccess) return e;
  }
  // each solve reads the lower triangle of L and the block inverses once: N^2 FLOP
  const double sbytes = 8.0 * ((double)N * (N + 1) / 2.0 + (double)nblk * 4096.0 + 2.0 * N);
  if (prof::active(prof::CHOL_SOLVE)) prof::begin(s, prof::CHOL_SOLVE, sbytes, (double)N * N);
  hipLaunchKernelGGL(k_chol_fwd, dim3(1), dim3(1024), 0, s, A, N, lda, Linv, x);  // L y = b
  prof::end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (prof::active(prof::CHOL_SOLVE)) prof::begin(s, prof::CHOL_SOLVE, sbytes, (double)N * N);
  hipLaunchKernelGGL(k_chol_bwd, dim3(1), dim3(1024), 0, s, A, N, lda, Linv, x);  // L^T x = y
  prof::end(s);
  return hipGetLastError();
}

}  // namespace qtt
