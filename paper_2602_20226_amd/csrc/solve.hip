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

// sqrt(x) and 1/sqrt(x) of a pivot from one hardware estimate of 1/sqrt(x)
// (relative error e ~2^-24), one third-order correction of it,
// r (1 + e/2 + 3 e^2 / 8) with e = 1 - x r^2, and one Newton step of the
// square root l = x r: fewer dependent steps than an IEEE square root
// followed by a reciprocal, within an ulp or two of both.  A pivot that is
// zero, negative or NaN gives NaN or an infinity, as the IEEE pair would.
__device__ __forceinline__ void sqrt_rsqrt(double x, double& l, double& r) {
  const double r0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * r0, r0, 1.0);
  r = fma(r0 * e, fma(0.375, e, 0.5), r0);
  const double l0 = x * r;
  l = fma(fma(-l0, l0, x), 0.5 * r, l0);
}

// Cholesky of the nb x nb diagonal block at A[j0][j0] (nb <= 64, lower
// triangle used and overwritten by L) and the inverse of L into Linv
// (64 x 64, row-major, zero outside the nb x nb lower triangle).  The block
// is padded with the identity to 64 x 64; each of the 256 threads owns one
// 4 x 4 tile (tile row tr, tile column tc) in registers.  A tile holds A
// while its columns are still to be factored and, from the step that
// factors them on, the same tile of Y, which is built up to L^{-1}: its
// columns K of L are final at that step, and the tile of Y starts there
// (I on the diagonal, 0 below it).  Four columns K = k..k+3 per step: the
// threads of tile column K publish the 64 x 4 column panel, those of tile
// row K their rows of Y (double-buffered LDS, one barrier per step); every
// thread factors the 4 x 4 diagonal block Ld and inverts it (Li) in
// registers, forms the multipliers l_i = Li p_i of its rows (zero up to
// row k+3) and, for its columns, either the multipliers l_j = Li p_j (tile
// still holding A: a -= l_i l_j^T) or the rows X_K = Li Y_K of the inverse
// (tile holding Y: y -= l_i X_K), one rank-4 update either way; tile row K
// then takes X_K.  Tiles whose rows are finished (tile row below K) do no
// work, so waves drop out as the factorisation proceeds.  A pivot that is
// not positive gives NaN, which propagates to the solution.
__global__ __launch_bounds__(256) void k_potrf_inv(double* __restrict__ A, long lda, int j0, int nb,
                                                   double* __restrict__ Linv, double* __restrict__ x) {
  __shared__ double xs[64];
  __shared__ double P[2][64][5];
  __shared__ double Yr[2][4][65];
  __shared__ double Ls[64][65];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int i0 = 4 * tr, c0 = 4 * tc;
  double z[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + u, j = c0 + v;
      z[u][v] = (i < nb && j <= i) ? A[(long)(j0 + i) * lda + j0 + j] : (i == j ? 1.0 : 0.0);
    }
  for (int K = 0; K < 16; ++K) {
    const int k = 4 * K, buf = K & 1;
    const bool active = tr >= K;  // rows not yet final (wave-uniform once a whole wave is done)
    if (active && tc == K) {  // the column panel (rows above the block are never read)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) P[buf][i0 + u][v] = z[u][v];
    }
    if (tr == K) {  // rows K of Y: the Y tiles left of the block, I on it, 0 right of it
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) Yr[buf][u][c0 + v] = (tc < K) ? z[u][v] : ((tc == K && u == v) ? 1.0 : 0.0);
    }
    __syncthreads();
    // the 4 x 4 pivot block is the same for every thread: lanes 0-15 of each
    // wave read it and it is made wave-uniform (16 LDS values per wave
    // instead of per thread)
    const double dl = P[buf][k + ((tid >> 2) & 3)][tid & 3];
    double d[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) d[t][q] = readlane_f64(dl, 4 * t + q);
    if (!active) continue;
    const bool amode = tc > K;  // this tile still holds A
    // the multipliers' source: the panel rows of this tile's columns (A
    // tiles, P[c0 + t][q]) or the rows K of Y over them (Y tiles,
    // Yr[q][c0 + t]); one read per entry from the address chosen per thread
    const double* src = amode ? &P[buf][c0][0] : &Yr[buf][0][c0];
    const int st = amode ? 5 : 1, sq = amode ? 1 : 65;
    double pi[4][4], sel[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        pi[t][q] = P[buf][i0 + t][q];
        sel[t][q] = src[t * st + q * sq];
      }
    // Ld = chol(D), Li = Ld^{-1} (lower, 4 x 4), written out
    double l00, r0, l11, r1, l22, r2, l33, r3;
    sqrt_rsqrt(d[0][0], l00, r0);
    const double l10 = d[1][0] * r0, l20 = d[2][0] * r0, l30 = d[3][0] * r0;
    sqrt_rsqrt(d[1][1] - l10 * l10, l11, r1);
    const double l21 = (d[2][1] - l20 * l10) * r1, l31 = (d[3][1] - l30 * l10) * r1;
    sqrt_rsqrt(d[2][2] - l20 * l20 - l21 * l21, l22, r2);
    const double l32 = (d[3][2] - l30 * l20 - l31 * l21) * r2;
    sqrt_rsqrt(d[3][3] - l30 * l30 - l31 * l31 - l32 * l32, l33, r3);
    const double m10 = -l10 * r0 * r1;
    const double m21 = -l21 * r1 * r2;
    const double m20 = -(l20 * r0 + l21 * m10) * r2;
    const double m32 = -l32 * r2 * r3;
    const double m31 = -(l31 * r1 + l32 * m21) * r3;
    const double m30 = -(l30 * r0 + l31 * m10 + l32 * m20) * r3;
    const double Li[4][4] = {{r0, 0.0, 0.0, 0.0}, {m10, r1, 0.0, 0.0}, {m20, m21, r2, 0.0}, {m30, m31, m32, r3}};
    const double L[4][4] = {{l00, 0.0, 0.0, 0.0}, {l10, l11, 0.0, 0.0}, {l20, l21, l22, 0.0}, {l30, l31, l32, l33}};
    if (tc == K) {  // the tile switches from A to Y: I on the diagonal, 0 below
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) z[u][v] = (tr == K && u == v) ? 1.0 : 0.0;
    }
    // l_i of this tile's rows (zero up to k+3) and m = l_j (A tiles) or X_K (Y tiles)
    double li[4][4], m[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double su = 0.0, sm = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q <= t) {
            su += Li[t][q] * pi[u][q];
            sm += Li[t][q] * sel[u][q];
          }
        li[u][t] = (tr > K) ? su : 0.0;
        m[u][t] = sm;  // l_j[c0 + u][t] or X_K[t][c0 + u]
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int t = 0; t < 4; ++t) z[u][v] = fma(-li[u][t], m[v][t], z[u][v]);
    if (tr == K) {  // rows K of the inverse (zero right of the block)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) z[u][v] = amode ? 0.0 : m[v][u];
    }
    if (tc == 0 && tr > K) {  // columns K of L below the diagonal block
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 4; ++t) Ls[i0 + u][k + t] = li[u][t];
    }
    if (tr == K) {  // the diagonal block of L (selects: no run-time index into registers)
      const int t = tc >> 2, q = tc & 3;
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
      Linv[i * 64 + j] = (i < nb && j < nb) ? z[u][v] : 0.0;
    }
  // this block's step of the forward substitution: x_B <- L_BB^{-1} x_B
  // (x_B already holds b_B minus the earlier blocks' panels times their
  // solutions); each tile row is summed over its 16 lanes in fixed order
  if (tid < 64) xs[tid] = (tid < nb) ? x[j0 + tid] : 0.0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    double p = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) p = fma(z[u][v], xs[c0 + v], p);
    p = row_sum(p);
    if (tc == 0 && i0 + u < nb) x[j0 + i0 + u] = p;
  }
}

// Panel of the blocked Cholesky in place, and the matching step of the
// forward substitution: rows [r0, r0 + 32) of P (mr x nb, leading dimension
// ldp) <- P Li^T with Li (64 x 64, lower triangular, row-major, zero outside
// the nb x nb block) the inverse of the diagonal block's factor, then
// xr[row] -= P[row] . yb for the same rows (yb: the block's solved entries).
// One workgroup per 32 rows: the rows and Li^T are staged in LDS with
// coalesced loads (every read of the rows precedes the barrier, every write
// follows it), the 32 x 64 product runs on the FP64 matrix cores (wave w
// owns the 16-row half w / 2 and the two 16-column tiles 2 (w % 2) + {0, 1};
// operand lane layout A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k,
// result C[i][j] with i = lane / 16 + 4 v, j = lane % 16), and each row's
// dot product with yb is summed over its 16 lanes and the two waves of its
// half in fixed order.
typedef double f64x4_t __attribute__((ext_vector_type(4)));
constexpr int kPanelRows = 32;
__global__ __launch_bounds__(256) void k_panel_rmul(double* __restrict__ P, int mr, int nb, long ldp,
                                                    const double* __restrict__ Li, const double* __restrict__ yb,
                                                    double* __restrict__ xr) {
  constexpr int PR = kPanelRows;
  __shared__ double As[64][PR + 1];  // As[k][i] = P[r0 + i][k]
  __shared__ double Bs[64][65];      // Bs[k][j] = Li[j][k]
  __shared__ double ys[64];
  __shared__ double red[2][PR];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r0 = blockIdx.x * PR;
  for (int e = tid; e < PR * 64; e += 256) {
    const int i = e >> 6, k = e & 63;
    As[k][i] = (r0 + i < mr && k < nb) ? P[(long)(r0 + i) * ldp + k] : 0.0;
  }
  for (int e = tid; e < 4096; e += 256) Bs[e & 63][e >> 6] = Li[e];
  if (tid < 64) ys[tid] = (tid < nb) ? yb[tid] : 0.0;
  __syncthreads();
  const int ti = w >> 1, tj0 = 2 * (w & 1);
  const int il = lane & 15, kq = lane >> 4;
  f64x4_t acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) acc[t] = f64x4_t{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const int k = 4 * ks + kq;
    const double a = As[k][16 * ti + il];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[k][16 * (tj0 + t) + il], acc[t], 0, 0, 0);
  }
  // this wave's part of each row's dot product with yb: over its 32 columns
  double part[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double pv = 0.0;
#pragma unroll
    for (int t = 0; t < 2; ++t) pv = fma(acc[t][v], ys[16 * (tj0 + t) + il], pv);
    part[v] = row_sum(pv);  // the 16 lanes of a row of lanes hold the 16 columns of one output row
  }
  if (il == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) red[w & 1][16 * ti + kq + 4 * v] = part[v];
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int col = 16 * (tj0 + t) + il;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = r0 + 16 * ti + kq + 4 * v;
      if (row < mr && col < nb) P[(long)row * ldp + col] = acc[t][v];
    }
  }
  if (tid < PR && r0 + tid < mr) xr[r0 + tid] -= red[0][tid] + red[1][tid];
}

constexpr int kCholMaxN = 4096;

// x <- L^{-T} x with L (N x N, lower triangle, leading dimension ldl) given
// with the inverses of its 64 x 64 diagonal blocks (Linv, one 64 x 64 block
// after the other): by blocks from the last,
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
  double* Linv = work;  // nblk blocks of 64 x 64
  hipError_t e;
  for (int b = 0; b < nblk; ++b) {
    const int j0 = 64 * b, nb = std::min(64, N - j0);
    double* Li = Linv + (long)b * 4096;
    if (prof::active(prof::CHOL_BLOCK))
      prof::begin(s, prof::CHOL_BLOCK, 8.0 * ((double)nb * nb + 4096.0), 2.0 * nb * nb * nb / 3.0);
    hipLaunchKernelGGL(k_potrf_inv, dim3(1), dim3(256), 0, s, A, lda, j0, nb, Li, x);
    prof::end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int mr = N - j0 - nb;
    if (mr <= 0) break;
    double* A21 = A + (long)(j0 + nb) * lda + j0;
    // L21 = A21 L11^{-T}, in place, and x[j0 + nb:] -= L21 x_B
    hipLaunchKernelGGL(k_panel_rmul, dim3((mr + kPanelRows - 1) / kPanelRows), dim3(256), 0, s, A21, mr, nb, lda,
                       (const double*)Li,
                       (const double*)(x + j0), x + j0 + nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // A22 -= L21 L21^T on the tiles on or below the diagonal (only the lower
    // triangle is read later); algorithmic work: the lower triangle, mr^2 nb FLOP
    if (prof::active(prof::CHOL_UPDATE))
      prof::begin(s, prof::CHOL_UPDATE, 8.0 * ((double)mr * nb + (double)mr * mr), (double)mr * mr * nb);
    e = gemm_f64_lower_nt(s, mr, nb, -1.0, A21, lda, 1.0, A21 + nb, lda);
    prof::end(s);
    if (e != hipSuccess) return e;
  }
  // x now holds y with L y = b (forward substitution carried along the
  // factorisation); L^T x = y reads the lower triangle of L and the block
  // inverses once: N^2 FLOP
  const double sbytes = 8.0 * ((double)N * (N + 1) / 2.0 + (double)nblk * 4096.0 + 2.0 * N);
  if (prof::active(prof::CHOL_SOLVE)) prof::begin(s, prof::CHOL_SOLVE, sbytes, (double)N * N);
  hipLaunchKernelGGL(k_chol_bwd, dim3(1), dim3(1024), 0, s, A, N, lda, Linv, x);  // L^T x = y
  prof::end(s);
  return hipGetLastError();
}

}  // namespace qtt
