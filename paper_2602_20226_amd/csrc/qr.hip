// Blocked Householder QR for the rounding sweep (FP64).
//
// Panels of up to 16 columns are factored by one workgroup (qr_panel_dev in
// qr_device.hpp).  The trailing update and every later application of Q or
// Q^T go through apply_block: a pair of kernels split over 16-column tiles
// and 256-row chunks (W = V^T Y per chunk, then reduction, op(T) and the
// rank-pw update), so that narrow targets still occupy the whole GPU.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"
#include "qr_device.hpp"

#include <algorithm>

namespace qtt {

namespace {

template <int NT, int RPT, int PW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_qr_panel(
    double* __restrict__ A, long lda, int m, int j0, int pw, double* __restrict__ Tout) {
  qr_panel_dev<NT, RPT, PW>(A, lda, m, j0, pw, Tout);
}

inline void apply_cost(int mp, int pw, int ncols, double& bytes, double& flops);

// Block-reflector application, split over (16-column tile) x (row chunk)
// workgroups so that even a narrow target keeps the whole GPU busy:
//   k_apply_w:   W_chunk = V_chunk^T Y_chunk  (16 x 16 per workgroup, stored
//                per chunk in scratch[chunk][16][ncols]);
//   k_apply_upd: W = sum_chunk W_chunk, W <- op(T) W, Y_chunk -= V_chunk W.
// V: rows [r0, r0+mp) of A, columns [vc0, vc0+pw), unit lower trapezoidal.
// Y rows [yr0, yr0+mp), columns [c0, c0+ncols).
// trans: Y <- (I - V T^T V^T) Y, else Y <- (I - V T V^T) Y.
// 256 threads: thread (g, c) owns column c of the tile and rows g (mod 16)
// of the chunk; rows are streamed four at a time.
constexpr int AP_NT = 256, AP_G = AP_NT / 16, AP_CHUNK = 256;

__device__ __forceinline__ void load_vrow(const double* __restrict__ arow, int lr, int pw, double (&v)[16]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (i >= pw) ? 0.0 : (lr > i ? arow[i] : (lr == i ? 1.0 : 0.0));
}

__global__ __launch_bounds__(AP_NT) void k_apply_w(const double* __restrict__ A, long lda, int r0, int mp, int vc0,
                                                   int pw, const double* __restrict__ Y, long ldy, int yr0, int c0,
                                                   int ncols, int ntiles, double* __restrict__ part) {
  __shared__ double red[AP_G][16][17];
  const int tid = threadIdx.x;
  const int c = tid & 15, g = tid >> 4;
  const int tile = blockIdx.x % ntiles, chunk = blockIdx.x / ntiles;
  const int col = tile * 16 + c;
  const bool valid = col < ncols;
  const int rbeg = chunk * AP_CHUNK, rend = min(mp, rbeg + AP_CHUNK);
  const double* Ab = A + (long)r0 * lda + vc0;
  const double* Yb = Y + (long)yr0 * ldy + c0 + col;
  double w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = 0.0;
  int lr = rbeg + g;
  for (; lr + 3 * AP_G < rend; lr += 4 * AP_G) {
    double y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = valid ? Yb[(long)(lr + q * AP_G) * ldy] : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v[16];
      load_vrow(Ab + (long)(lr + q * AP_G) * lda, lr + q * AP_G, pw, v);
#pragma unroll
      for (int i = 0; i < 16; ++i) w[i] += v[i] * y[q];
    }
  }
  for (; lr < rend; lr += AP_G) {
    const double y = valid ? Yb[(long)lr * ldy] : 0.0;
    double v[16];
    load_vrow(Ab + (long)lr * lda, lr, pw, v);
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] += v[i] * y;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) red[g][i][c] = w[i];
  __syncthreads();
  {
    const int i = tid >> 4, cc = tid & 15;
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < AP_G; ++q) sum += red[q][i][cc];
    if (tile * 16 + cc < ncols) part[((long)chunk * 16 + i) * ncols + tile * 16 + cc] = sum;
  }
}

__global__ __launch_bounds__(AP_NT) void k_apply_upd(const double* __restrict__ A, long lda, int r0, int mp, int vc0,
                                                     int pw, const double* __restrict__ T, double* __restrict__ Y,
                                                     long ldy, int yr0, int c0, int ncols, int ntiles, int nchunks,
                                                     const double* __restrict__ part, int trans) {
  __shared__ double Ws[16][17];
  __shared__ double W2[16][17];
  __shared__ double Tsh[16][17];
  const int tid = threadIdx.x;
  const int c = tid & 15, g = tid >> 4;
  const int tile = blockIdx.x % ntiles, chunk = blockIdx.x / ntiles;
  const int col = tile * 16 + c;
  const bool valid = col < ncols;
  Tsh[tid >> 4][tid & 15] = T[tid];
  {
    const int i = tid >> 4, cc = tid & 15;
    double sum = 0.0;
    if (tile * 16 + cc < ncols)
      for (int q = 0; q < nchunks; ++q) sum += part[((long)q * 16 + i) * ncols + tile * 16 + cc];
    Ws[i][cc] = sum;
  }
  __syncthreads();
  {
    const int i = tid >> 4, cc = tid & 15;
    double sum = 0.0;
#pragma unroll
    for (int l = 0; l < 16; ++l) sum += (trans ? Tsh[l][i] : Tsh[i][l]) * Ws[l][cc];
    W2[i][cc] = sum;
  }
  __syncthreads();
  if (!valid) return;
  double w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = W2[i][c];
  const int rbeg = chunk * AP_CHUNK, rend = min(mp, rbeg + AP_CHUNK);
  const double* Ab = A + (long)r0 * lda + vc0;
  double* Yb = Y + (long)yr0 * ldy + c0 + col;
  int lr = rbeg + g;
  for (; lr + 3 * AP_G < rend; lr += 4 * AP_G) {
    double y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = Yb[(long)(lr + q * AP_G) * ldy];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v[16];
      load_vrow(Ab + (long)(lr + q * AP_G) * lda, lr + q * AP_G, pw, v);
      double sum = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) sum += v[i] * w[i];
      Yb[(long)(lr + q * AP_G) * ldy] = y[q] - sum;
    }
  }
  for (; lr < rend; lr += AP_G) {
    double v[16];
    load_vrow(Ab + (long)lr * lda, lr, pw, v);
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) sum += v[i] * w[i];
    Yb[(long)lr * ldy] -= sum;
  }
}

// One block-reflector application (two launches).
hipError_t apply_block(hipStream_t s, const double* A, long lda, int r0, int mp, int vc0, int pw, const double* T,
                       double* Y, long ldy, int yr0, int c0, int ncols, int trans, double* scratch) {
  const int ntiles = (ncols + 15) / 16;
  const int nchunks = (mp + AP_CHUNK - 1) / AP_CHUNK;
  if (prof::active(prof::APPLY_PANEL)) {
    double b, f;
    apply_cost(mp, pw, ncols, b, f);
    prof::begin(s, prof::APPLY_PANEL, b, f);
  }
  hipLaunchKernelGGL(k_apply_w, dim3(ntiles * nchunks), dim3(AP_NT), 0, s, A, lda, r0, mp, vc0, pw, (const double*)Y,
                     ldy, yr0, c0, ncols, ntiles, scratch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_apply_upd, dim3(ntiles * nchunks), dim3(AP_NT), 0, s, A, lda, r0, mp, vc0, pw, T, Y, ldy,
                       yr0, c0, ncols, ntiles, nchunks, (const double*)scratch, trans);
    e = hipGetLastError();
  }
  prof::end(s);
  return e;
}

__global__ void k_extract_r(const double* __restrict__ A, int kr, int n, long lda, double* __restrict__ R) {
  const long total = (long)kr * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n;
    const int j = (int)(e % n);
    R[e] = (j >= i) ? A[i * lda + j] : 0.0;
  }
}

// Algorithmic cost of one block-reflector application to an mp x ncols
// block: read and write the block once, read V and T once;
// W = V^T Y, W <- op(T) W, Y <- Y - V W.
inline void apply_cost(int mp, int pw, int ncols, double& bytes, double& flops) {
  bytes = 8.0 * (2.0 * mp * ncols + (double)mp * pw + 256.0);
  flops = 4.0 * mp * pw * (double)ncols + 2.0 * pw * pw * (double)ncols;
}

struct PanelCfg {
  int nt, rpt, pw;
};

inline PanelCfg panel_cfg(int mp) {
  if (mp <= 256) return {256, 1, 16};
  if (mp <= 512) return {256, 2, 16};
  if (mp <= 1024) return {256, 4, 16};
  if (mp <= 2048) return {1024, 2, 16};
  return {1024, 4, 8};
}

// Panel boundaries are a pure function of (m, kmax); both the factorisation
// and every later application of Q walk the same sequence.
template <typename F>
inline hipError_t for_each_panel(int m, int kmax, F f) {
  int j0 = 0, p = 0;
  while (j0 < kmax) {
    const PanelCfg c = panel_cfg(m - j0);
    const int pw = std::min(c.pw, kmax - j0);
    hipError_t e = f(p, j0, pw, c);
    if (e != hipSuccess) return e;
    j0 += pw;
    ++p;
  }
  return hipSuccess;
}

}  // namespace

int qr_num_panels(int m, int n) {
  const int kmax = std::min(m, n);
  int cnt = 0;
  (void)for_each_panel(m, kmax, [&](int, int, int, PanelCfg) {
    ++cnt;
    return hipSuccess;
  });
  return cnt;
}

hipError_t householder_qr(hipStream_t s, double* A, int m, int n, long lda, double* Tbuf, double* scratch) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (m > 4096) return hipErrorInvalidValue;
  const int kmax = std::min(m, n);
  return for_each_panel(m, kmax, [&](int p, int j0, int pw, PanelCfg c) -> hipError_t {
    double* T = Tbuf + (long)p * 256;
    if (prof::active(prof::QR_PANEL)) {
      const double mp = m - j0;
      prof::begin(s, prof::QR_PANEL, 8.0 * 2.0 * mp * pw, 4.0 * mp * pw * pw);
    }
    if (c.nt == 256 && c.rpt == 1)
      hipLaunchKernelGGL((k_qr_panel<256, 1, 16>), dim3(1), dim3(256), 0, s, A, lda, m, j0, pw, T);
    else if (c.nt == 256 && c.rpt == 2)
      hipLaunchKernelGGL((k_qr_panel<256, 2, 16>), dim3(1), dim3(256), 0, s, A, lda, m, j0, pw, T);
    else if (c.nt == 256)
      hipLaunchKernelGGL((k_qr_panel<256, 4, 16>), dim3(1), dim3(256), 0, s, A, lda, m, j0, pw, T);
    else if (c.rpt == 2)
      hipLaunchKernelGGL((k_qr_panel<1024, 2, 16>), dim3(1), dim3(1024), 0, s, A, lda, m, j0, pw, T);
    else
      hipLaunchKernelGGL((k_qr_panel<1024, 4, 8>), dim3(1), dim3(1024), 0, s, A, lda, m, j0, pw, T);
    hipError_t e = hipGetLastError();
    prof::end(s);
    if (e != hipSuccess) return e;
    const int c0 = j0 + pw;
    const int nc = n - c0;
    if (nc > 0) e = apply_block(s, A, lda, j0, m - j0, j0, pw, T, A, lda, j0, c0, nc, 1, scratch);
    return e;
  });
}

hipError_t apply_q(hipStream_t s, const double* A, int m, int kref, long lda, const double* Tbuf, double* Y,
                   int ncols, long ldy, bool trans, double* scratch) {
  if (m <= 0 || ncols <= 0 || kref <= 0) return hipSuccess;
  struct P {
    int p, j0, pw;
  };
  P list[4096 / 8 + 8];
  int np = 0;
  (void)for_each_panel(m, kref, [&](int p, int j0, int pw, PanelCfg) {
    list[np++] = {p, j0, pw};
    return hipSuccess;
  });
  for (int t = 0; t < np; ++t) {
    const P& q = trans ? list[t] : list[np - 1 - t];
    hipError_t e = apply_block(s, A, lda, q.j0, m - q.j0, q.j0, q.pw, Tbuf + (long)q.p * 256, Y, ldy, q.j0, 0, ncols,
                               trans ? 1 : 0, scratch);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t extract_r(hipStream_t s, const double* A, int kr, int n, long lda, double* Rout) {
  const long total = (long)kr * n;
  if (total <= 0) return hipSuccess;
  long g = (total + 255) / 256;
  if (g > (1 << 20)) g = 1 << 20;
  hipLaunchKernelGGL(k_extract_r, dim3((int)g), dim3(256), 0, s, A, kr, n, lda, Rout);
  return hipGetLastError();
}

}  // namespace qtt
