// Core-by-core contraction kernels (paper Sec. 3.1, eqs. quant_sum / einsum)
// and the small element-wise kernels of the rounding sweep.
//
// Bond flattening: xi = mu * r_B + nu (mu major), so a contracted core is
// C[(mu,nu), i, (mu',nu')] stored row-major as [rA*rB, d, rA'*rB'].
// All kernels here are memory bound; consecutive threads walk the fastest
// output index (nu') so that the operand with the fast index is read
// coalesced and the other one is broadcast.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"

namespace qtt {

namespace {

inline int grid_for(long n, int bs = 256) {
  long g = (n + bs - 1) / bs;
  if (g > (1L << 20)) g = 1L << 20;
  return (int)(g < 1 ? 1 : g);
}

// C[(a,c), i, (b,dd)] = A[a,i,b] * B[c,i,dd]
template <typename T>
__global__ void k_hadamard(const T* __restrict__ A, int ra0, int d, int ra1, const T* __restrict__ B,
                           int rb0, int rb1, T* __restrict__ C) {
  const long total = (long)ra0 * rb0 * d * ra1 * rb1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int dd = t % rb1; t /= rb1;
    const int b = t % ra1; t /= ra1;
    const int i = t % d; t /= d;
    const int c = t % rb0; t /= rb0;
    const int a = (int)t;
    C[e] = A[((long)a * d + i) * ra1 + b] * B[((long)c * d + i) * rb1 + dd];
  }
}

// C[(a,c), i, (b,dd)] = sum_j W[a,i,j,b] * X[c,j,dd]
template <typename T>
__global__ void k_mpo(const T* __restrict__ W, int rw0, int di, int dj, int rw1, const T* __restrict__ X,
                      int rx0, int rx1, T* __restrict__ C) {
  const long total = (long)rw0 * rx0 * di * rw1 * rx1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int dd = t % rx1; t /= rx1;
    const int b = t % rw1; t /= rw1;
    const int i = t % di; t /= di;
    const int c = t % rx0; t /= rx0;
    const int a = (int)t;
    T acc = 0;
    for (int j = 0; j < dj; ++j)
      acc += W[(((long)a * di + i) * dj + j) * rw1 + b] * X[((long)c * dj + j) * rx1 + dd];
    C[e] = acc;
  }
}

// M[(a,i),(b,dd)] = sum_{mu,j} Y[a,mu,j,dd] * W[mu,i,j,b]
__global__ void k_bond_mpo(const double* __restrict__ Y, int rho, int rw0, int dj, int rx1,
                           const double* __restrict__ W, int di, int rw1, double* __restrict__ M) {
  const long total = (long)rho * di * rw1 * rx1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int dd = t % rx1; t /= rx1;
    const int b = t % rw1; t /= rw1;
    const int i = t % di; t /= di;
    const long a = t;
    double acc = 0.0;
    for (int mu = 0; mu < rw0; ++mu)
      for (int j = 0; j < dj; ++j)
        acc += Y[((a * rw0 + mu) * dj + j) * rx1 + dd] * W[(((long)mu * di + i) * dj + j) * rw1 + b];
    M[e] = acc;
  }
}

// M[(a,i),(b,dd)] = sum_mu Y[a,mu,i,dd] * A[mu,i,b]
__global__ void k_bond_hadamard(const double* __restrict__ Y, int rho, int ra0, int d, int rb1,
                                const double* __restrict__ A, int ra1, double* __restrict__ M) {
  const long total = (long)rho * d * ra1 * rb1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int dd = t % rb1; t /= rb1;
    const int b = t % ra1; t /= ra1;
    const int i = t % d; t /= d;
    const long a = t;
    double acc = 0.0;
    for (int mu = 0; mu < ra0; ++mu)
      acc += Y[((a * ra0 + mu) * d + i) * rb1 + dd] * A[((long)mu * d + i) * ra1 + b];
    M[e] = acc;
  }
}

// dX[c,j,dd] = sum_{a,i,b} W[a,i,j,b] dC[(a,c),i,(b,dd)]   (Hadamard: j == i, W[a,i,b])
template <typename T>
__global__ void k_bwd_x(bool mpo, const T* __restrict__ W, int rw0, int di, int dj, int rw1,
                        const T* __restrict__ dC, int rx0, int rx1, T* __restrict__ dX) {
  const int dx = mpo ? dj : di;
  const long total = (long)rx0 * dx * rx1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int dd = t % rx1; t /= rx1;
    const int j = t % dx; t /= dx;
    const int c = (int)t;
    T acc = 0;
    for (int a = 0; a < rw0; ++a)
      for (int i = 0; i < di; ++i) {
        if (!mpo && i != j) continue;
        for (int b = 0; b < rw1; ++b) {
          const T w = mpo ? W[(((long)a * di + i) * dj + j) * rw1 + b] : W[((long)a * di + i) * rw1 + b];
          acc += w * dC[((((long)a * rx0 + c) * di + i) * rw1 + b) * rx1 + dd];
        }
      }
    dX[e] = acc;
  }
}

// dW[a,i,j,b] = sum_{c,dd} X[c,j,dd] dC[(a,c),i,(b,dd)]   (Hadamard: dW[a,i,b], j == i)
template <typename T>
__global__ void k_bwd_w(bool mpo, const T* __restrict__ X, int rx0, int dj, int rx1,
                        const T* __restrict__ dC, int rw0, int di, int rw1, T* __restrict__ dW) {
  const int djj = mpo ? dj : 1;
  const long total = (long)rw0 * di * djj * rw1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int b = t % rw1; t /= rw1;
    const int jj = t % djj; t /= djj;
    const int i = t % di; t /= di;
    const int a = (int)t;
    const int j = mpo ? jj : i;
    T acc = 0;
    for (int c = 0; c < rx0; ++c)
      for (int dd = 0; dd < rx1; ++dd)
        acc += X[((long)c * dj + j) * rx1 + dd] * dC[((((long)a * rx0 + c) * di + i) * rw1 + b) * rx1 + dd];
    dW[e] = acc;
  }
}

__global__ void k_fill(double* p, double v, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) p[e] = v;
}
__global__ void k_fill_u32(unsigned* p, unsigned v, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) p[e] = v;
}
__global__ void k_fill_f32(float* p, float v, long n) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) p[e] = v;
}
// Z (m x q) = [I_q; 0]
__global__ void k_eye_rect(double* Z, int m, int q) {
  const long n = (long)m * q;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    Z[e] = (e / q == e % q) ? 1.0 : 0.0;
}
// dst[r][c] = src[r][c] for r < rows, 0 for rows <= r < rows_out (c < cols)
__global__ void k_copy_pad(const double* __restrict__ src, int rows, int cols, long lds, double* __restrict__ dst,
                           int rows_out, long ldd) {
  const long n = (long)rows_out * cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / cols;
    const int c = (int)(e % cols);
    dst[r * ldd + c] = (r < rows) ? src[r * lds + c] : 0.0;
  }
}
__global__ void k_transpose(const double* __restrict__ A, int rows, int cols, long lda, double* __restrict__ B,
                            long ldb) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = by + k, c = bx + tx;
    if (r < rows && c < cols) tile[k][tx] = A[(long)r * lda + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = bx + k, r = by + tx;  // B[c][r] = A[r][c]
    if (r < rows && c < cols) B[(long)c * ldb + r] = tile[tx][k];
  }
}

// Frobenius norm of a vector; one workgroup, deterministic order.
// y += alpha x
__global__ void k_axpy(long n, double alpha, const double* __restrict__ x, double* __restrict__ y) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] += alpha * x[e];
}
// dst = src / (s2[0] + s2[1]) (a copy when the sum is zero); dst may be src.
__global__ void k_copy_scaled_inv(const double* src, int rows, int cols, long lds, const double* __restrict__ s2,
                                  double* dst, long ldd) {
  const double s = s2[0] + s2[1];
  const double f = s > 0.0 ? 1.0 / s : 1.0;
  const long n = (long)rows * cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const long r = e / cols;
    const int c = (int)(e % cols);
    dst[r * ldd + c] = src[r * lds + c] * f;
  }
}
__global__ __launch_bounds__(1024) void k_frob(const double* __restrict__ x, long n, double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (long e = threadIdx.x; e < n; e += 1024) s += x[e] * x[e];
  s = block_sum<1024>(s, red);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

// C[(a,c), i, k, (b,dd)] = sum_j A[a,i,j,b] * B[c,j,k,dd]   (operator product)
template <typename T>
__global__ void k_mpo_mpo(const T* __restrict__ A, int ra0, int di, int dj, int ra1, const T* __restrict__ B,
                          int rb0, int dk, int rb1, T* __restrict__ C) {
  const long total = (long)ra0 * rb0 * di * dk * ra1 * rb1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long t = e;
    const int dd = t % rb1; t /= rb1;
    const int b = t % ra1; t /= ra1;
    const int k = t % dk; t /= dk;
    const int i = t % di; t /= di;
    const int c = t % rb0; t /= rb0;
    const int a = (int)t;
    T acc = 0;
    for (int j = 0; j < dj; ++j)
      acc += A[(((long)a * di + i) * dj + j) * ra1 + b] * B[(((long)c * dj + j) * dk + k) * rb1 + dd];
    C[e] = acc;
  }
}

// One core of the exact sum of `count` trains (block structure of Sec. 3.1):
// core 0 is the row [c_1 X_1, c_2 X_2, ...] (terms side by side on the right
// bond), the last core the column of the terms (stacked on the left bond),
// the others block-diagonal in term order; with a single core the weighted
// sum itself (products and sums rounded separately, in term order: no
// fused multiply-add).
template <typename T>
__global__ void k_tt_add_core(AddTerms<T> t, int count, int P, int R0, int R1, int first, int last,
                              T* __restrict__ out) {
#pragma clang fp contract(off)
  const long total = (long)R0 * P * R1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e % R1);
    const long ai = e / R1;
    const int i = (int)(ai % P);
    const int a = (int)(ai / P);
    T v = 0;
    if (first && last) {
      for (int q = 0; q < count; ++q) v = v + (T)t.coef[q] * t.src[q][i];
    } else {
      int q = 0;
      if (last) {
        while (q + 1 < count && a >= t.off0[q + 1]) ++q;
      } else {
        while (q + 1 < count && b >= t.off1[q + 1]) ++q;
      }
      const int la = first ? 0 : a - t.off0[q];
      const int lb = last ? 0 : b - t.off1[q];
      if (la >= 0 && la < t.r0[q] && lb >= 0 && lb < t.r1[q]) {
        const T x = t.src[q][((long)la * P + i) * t.r1[q] + lb];
        v = first ? (T)t.coef[q] * x : x;
      }
    }
    out[e] = v;
  }
}

}  // namespace

template <typename T>
hipError_t contract_hadamard(hipStream_t s, const T* A, int ra0, int d, int ra1, const T* B, int rb0,
                             int rb1, T* C) {
  const long total = (long)ra0 * rb0 * d * ra1 * rb1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_hadamard<T>, dim3(grid_for(total)), dim3(256), 0, s, A, ra0, d, ra1, B, rb0, rb1, C);
  return hipGetLastError();
}
template <typename T>
hipError_t contract_mpo(hipStream_t s, const T* W, int rw0, int di, int dj, int rw1, const T* X, int rx0,
                        int rx1, T* C) {
  const long total = (long)rw0 * rx0 * di * rw1 * rx1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mpo<T>, dim3(grid_for(total)), dim3(256), 0, s, W, rw0, di, dj, rw1, X, rx0, rx1, C);
  return hipGetLastError();
}
template <typename T>
hipError_t contract_mpo_mpo(hipStream_t s, const T* A, int ra0, int di, int dj, int ra1, const T* B, int rb0,
                            int dk, int rb1, T* C) {
  const long total = (long)ra0 * rb0 * di * dk * ra1 * rb1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mpo_mpo<T>, dim3(grid_for(total)), dim3(256), 0, s, A, ra0, di, dj, ra1, B, rb0, dk, rb1, C);
  return hipGetLastError();
}
template hipError_t contract_mpo_mpo<double>(hipStream_t, const double*, int, int, int, int, const double*, int, int,
                                             int, double*);
template hipError_t contract_mpo_mpo<float>(hipStream_t, const float*, int, int, int, int, const float*, int, int,
                                            int, float*);

template <typename T>
hipError_t tt_add_core(hipStream_t s, const AddTerms<T>& terms, int count, int P, int R0, int R1, int first,
                       int last, T* out) {
  if (count < 1 || count > kMaxAddTerms) return hipErrorInvalidValue;
  const long total = (long)R0 * P * R1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tt_add_core<T>, dim3(grid_for(total)), dim3(256), 0, s, terms, count, P, R0, R1, first, last,
                     out);
  return hipGetLastError();
}
template hipError_t tt_add_core<double>(hipStream_t, const AddTerms<double>&, int, int, int, int, int, int, double*);
template hipError_t tt_add_core<float>(hipStream_t, const AddTerms<float>&, int, int, int, int, int, int, float*);

template hipError_t contract_hadamard<double>(hipStream_t, const double*, int, int, int, const double*, int, int, double*);
template hipError_t contract_hadamard<float>(hipStream_t, const float*, int, int, int, const float*, int, int, float*);
template hipError_t contract_mpo<double>(hipStream_t, const double*, int, int, int, int, const double*, int, int, double*);
template hipError_t contract_mpo<float>(hipStream_t, const float*, int, int, int, int, const float*, int, int, float*);

hipError_t bond_mpo_apply(hipStream_t s, const double* Y, int rho, int rw0, int dj, int rx1, const double* W,
                          int di, int rw1, double* M) {
  const long total = (long)rho * di * rw1 * rx1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bond_mpo, dim3(grid_for(total)), dim3(256), 0, s, Y, rho, rw0, dj, rx1, W, di, rw1, M);
  return hipGetLastError();
}
hipError_t bond_hadamard_apply(hipStream_t s, const double* Y, int rho, int ra0, int d, int rb1, const double* A,
                               int ra1, double* M) {
  const long total = (long)rho * d * ra1 * rb1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bond_hadamard, dim3(grid_for(total)), dim3(256), 0, s, Y, rho, ra0, d, rb1, A, ra1, M);
  return hipGetLastError();
}

template <typename T>
hipError_t contract_backward_x(hipStream_t s, bool mpo, const T* W, int rw0, int di, int dj, int rw1,
                               const T* dC, int rx0, int rx1, T* dX) {
  const long total = (long)rx0 * (mpo ? dj : di) * rx1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_x<T>, dim3(grid_for(total)), dim3(256), 0, s, mpo, W, rw0, di, dj, rw1, dC, rx0, rx1, dX);
  return hipGetLastError();
}
template <typename T>
hipError_t contract_backward_w(hipStream_t s, bool mpo, const T* X, int rx0, int dj, int rx1, const T* dC,
                               int rw0, int di, int rw1, T* dW) {
  const long total = (long)rw0 * di * (mpo ? dj : 1) * rw1;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_w<T>, dim3(grid_for(total)), dim3(256), 0, s, mpo, X, rx0, dj, rx1, dC, rw0, di, rw1, dW);
  return hipGetLastError();
}
template hipError_t contract_backward_x<double>(hipStream_t, bool, const double*, int, int, int, int, const double*, int, int, double*);
template hipError_t contract_backward_x<float>(hipStream_t, bool, const float*, int, int, int, int, const float*, int, int, float*);
template hipError_t contract_backward_w<double>(hipStream_t, bool, const double*, int, int, int, const double*, int, int, int, double*);
template hipError_t contract_backward_w<float>(hipStream_t, bool, const float*, int, int, int, const float*, int, int, int, float*);

hipError_t fill_f64(hipStream_t s, double* p, double v, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t fill_u32(hipStream_t s, unsigned* p, unsigned v, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t fill_f32(hipStream_t s, float* p, float v, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t set_eye_rect(hipStream_t s, double* Z, int m, int q) {
  if (m <= 0 || q <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eye_rect, dim3(grid_for((long)m * q)), dim3(256), 0, s, Z, m, q);
  return hipGetLastError();
}
hipError_t copy_pad_rows(hipStream_t s, const double* src, int rows, int cols, long lds, double* dst, int rows_out,
                         long ldd) {
  const long n = (long)rows_out * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_pad, dim3(grid_for(n)), dim3(256), 0, s, src, rows, cols, lds, dst, rows_out, ldd);
  return hipGetLastError();
}
hipError_t transpose(hipStream_t s, const double* A, int rows, int cols, long lda, double* B, long ldb) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32);
  hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, A, rows, cols, lda, B, ldb);
  return hipGetLastError();
}
hipError_t frob_norm(hipStream_t s, const double* x, long n, double* out) {
  hipLaunchKernelGGL(k_frob, dim3(1), dim3(1024), 0, s, x, n, out);
  return hipGetLastError();
}
hipError_t axpy_f64(hipStream_t s, long n, double alpha, const double* x, double* y) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(grid_for(n)), dim3(256), 0, s, n, alpha, x, y);
  return hipGetLastError();
}
hipError_t copy_scaled_inv(hipStream_t s, const double* src, int rows, int cols, long lds, const double* s2,
                           double* dst, long ldd) {
  const long n = (long)rows * cols;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_scaled_inv, dim3(grid_for(n)), dim3(256), 0, s, src, rows, cols, lds, s2, dst, ldd);
  return hipGetLastError();
}

}  // namespace qtt
