// Kernels of the DMRG-like linear solver (Sec. 5): the local matrix of the
// energy <x, W x> - 2 <x, b> for one core or a two-core super-core, the
// operator-core steps of the three-layer environments <x|W|x>, the product
// of two adjacent operator cores, and the upper-triangular solve that ends
// the local QR solve.  FP64 throughout (the local problems decide the
// solution's accuracy; they are small).
#include "qtt_device.hpp"
#include "qtt_internal.hpp"

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

// A[j][i] = A[i][j] for i < j: the upper triangle mirrored into the lower
// one (whose previous contents are dropped), by 32 x 32 tiles staged in LDS
// so that both the reads and the writes are row-contiguous.  Tiles above
// the diagonal go to disjoint tiles below it; a diagonal tile moves only its
// strictly upper entries, so no entry is both read and written.
__global__ __launch_bounds__(256) void k_reflect_upper(double* __restrict__ A, int N, long lda) {
  __shared__ double tile[32][33];
  const int nt = (N + 31) / 32;
  // blockIdx.x enumerates the tile pairs (bi <= bj) row by row
  int t = blockIdx.x, bi = 0;
  while (t >= nt - bi) {
    t -= nt - bi;
    ++bi;
  }
  const int bj = bi + t;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of 32 per pass
  for (int r = ty; r < 32; r += 8) {
    const int i = bi * 32 + r, j = bj * 32 + tx;
    tile[r][tx] = (i < N && j < N) ? A[(long)i * lda + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = bj * 32 + r, i = bi * 32 + tx;  // destination row j, column i
    if (j < N && i < N && i < j) A[(long)j * lda + i] = tile[tx][r];
  }
}

// x <- R^{-1} x for an upper-triangular R given by its transpose in the
// lower triangle of L (N x N, leading dimension ldl): blocked from the
// bottom in blocks B of 64 unknowns.  The diagonal block R_BB is staged in
// LDS and x_B solved by one wave (lane i holds x_i; x_k = x_k / R_kk,
// broadcast, lanes i < k subtract R_ik x_k); then every unknown above the
// block takes x_i -= sum_b L[b][i] x_b over the block's rows b of L, read
// contiguously along i (each thread keeps its 64 loads independent).  One
// workgroup; the operation order is fixed, so the result is deterministic.
constexpr int kTrsvB = 64;

__global__ __launch_bounds__(1024) void k_trsv_rt(const double* __restrict__ L, int N, long ldl,
                                                  double* __restrict__ x) {
  __shared__ double R[kTrsvB][kTrsvB + 1];
  __shared__ double xb[kTrsvB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int k1 = N; k1 > 0; k1 -= kTrsvB) {
    const int k0 = k1 > kTrsvB ? k1 - kTrsvB : 0;
    const int nb = k1 - k0;
    for (int e = tid; e < nb * nb; e += blockDim.x) {
      const int c = e / nb, r = e % nb;  // R_BB[r][c] = L[k0 + c][k0 + r]
      R[r][c] = (c >= r) ? L[(long)(k0 + c) * ldl + k0 + r] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double xi = lane < nb ? x[k0 + lane] : 0.0;
      for (int k = nb - 1; k >= 0; --k) {
        if (lane == k) xi = xi / R[k][k];
        const double xk = __shfl(xi, k);
        if (lane < k) xi -= R[lane][k] * xk;
      }
      if (lane < nb) {
        x[k0 + lane] = xi;
        xb[lane] = xi;
      }
    }
    __syncthreads();
    for (int i = tid; i < k0; i += blockDim.x) {
      const double* col = L + (long)k0 * ldl + i;
      double acc = 0.0;
      for (int b = 0; b < nb; ++b) acc += col[(long)b * ldl] * xb[b];
      x[i] -= acc;
    }
    __syncthreads();
  }
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

hipError_t trsv_upper(hipStream_t s, double* A, int N, long lda, double* x) {
  if (N <= 0) return hipSuccess;
  const int nt = (N + 31) / 32;
  hipLaunchKernelGGL(k_reflect_upper, dim3(nt * (nt + 1) / 2), dim3(256), 0, s, A, N, lda);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trsv_rt, dim3(1), dim3(1024), 0, s, A, N, lda, x);
  return hipGetLastError();
}

}  // namespace qtt
