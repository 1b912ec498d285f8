// Blocked Householder QR for the rounding sweep (FP64).
//
// Row-major A (m x n).  Panels of up to 16 columns are factored by a single
// workgroup holding the panel in registers (each thread owns RPT rows of
// the panel), one Householder reflector per column:
//     x = A[j:m, j], beta = -sign(x0) ||x||, tau = (beta - x0)/beta,
//     v = x / (x0 - beta) with v0 = 1,   H = I - tau v v^T,   H x = beta e0
// (tau = 0, H = I when x has no entries below the diagonal).  The same
// workgroup reduction that forms v^T A for the update also yields the
// column V^T v_j, from which the compact-WY factor T (H_1..H_b = I - V T V^T,
// T upper triangular) is built column by column.
//
// The trailing update and every later application of Q or Q^T use one fused
// kernel: each workgroup owns 16 columns of the target and all its rows, so
// W = V^T Y, W <- op(T) W and Y <- Y - V W need no grid-wide reduction.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"

#include <algorithm>

namespace qtt {

namespace {

template <int NT, int RPT, int PW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_qr_panel(double* __restrict__ A, long lda, int m, int j0, int pw,
                                                 double* __restrict__ Tout) {
  constexpr int NW = NT / 64;
  __shared__ double red[NT];
  __shared__ double bc[16];
  __shared__ double sc[NW];
  __shared__ double Ts[16][17];
  __shared__ double alphaS;
  const int tid = threadIdx.x;
  const int mp = m - j0;
  double a[RPT][PW];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = tid + r * NT;
#pragma unroll
    for (int c = 0; c < PW; ++c) a[r][c] = (lr < mp && c < pw) ? A[(long)(j0 + lr) * lda + j0 + c] : 0.0;
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
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int lr = tid + r * NT;
    if (lr < mp) {
#pragma unroll
      for (int c = 0; c < PW; ++c)
        if (c < pw) A[(long)(j0 + lr) * lda + j0 + c] = a[r][c];
    }
  }
  for (int t = tid; t < 256; t += NT) Tout[t] = Ts[t >> 4][t & 15];
}

// Apply the block reflector of one panel to 16-column tiles of Y.
//   V: rows [r0, r0+mp) of A, columns [vc0, vc0+pw), unit lower trapezoidal.
//   Y rows [yr0, yr0+mp), columns [c0, c0+ncols).
//   trans: Y <- (I - V T^T V^T) Y  else  Y <- (I - V T V^T) Y.
// 512 threads: thread (g, c) owns column c of the tile and the rows
// lr = g (mod 32); rows are streamed four at a time so that several loads
// are in flight per thread.
constexpr int AP_NT = 512, AP_G = AP_NT / 16;

__device__ __forceinline__ void load_vrow(const double* __restrict__ arow, int lr, int pw, double (&v)[16]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = (i >= pw) ? 0.0 : (lr > i ? arow[i] : (lr == i ? 1.0 : 0.0));
}

__global__ __launch_bounds__(AP_NT) void k_apply_panel(const double* __restrict__ A, long lda, int r0, int mp,
                                                       int vc0, int pw, const double* __restrict__ T,
                                                       double* __restrict__ Y, long ldy, int yr0, int c0,
                                                       int ncols, int trans) {
  __shared__ double part[AP_G][16][17];
  __shared__ double Ws[16][17];
  __shared__ double W2[16][17];
  __shared__ double Tsh[16][17];
  const int tid = threadIdx.x;
  const int c = tid & 15, g = tid >> 4;
  const int gc = c0 + blockIdx.x * 16 + c;
  const bool valid = gc < c0 + ncols;
  if (tid < 256) Tsh[tid >> 4][tid & 15] = T[tid];
  const double* Ab = A + (long)r0 * lda + vc0;
  double* Yb = Y + (long)yr0 * ldy + gc;

  // phase 1: w[i] = sum_rows V[lr][i] * Y[lr][c]
  double w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = 0.0;
  int lr = g;
  for (; lr + 3 * AP_G < mp; lr += 4 * AP_G) {
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
  for (; lr < mp; lr += AP_G) {
    const double y = valid ? Yb[(long)lr * ldy] : 0.0;
    double v[16];
    load_vrow(Ab + (long)lr * lda, lr, pw, v);
#pragma unroll
    for (int i = 0; i < 16; ++i) w[i] += v[i] * y;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) part[g][i][c] = w[i];
  __syncthreads();
  if (tid < 256) {
    const int i = tid >> 4, cc = tid & 15;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < AP_G; ++q) s += part[q][i][cc];
    Ws[i][cc] = s;
  }
  __syncthreads();
  if (tid < 256) {
    const int i = tid >> 4, cc = tid & 15;
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < 16; ++l) s += (trans ? Tsh[l][i] : Tsh[i][l]) * Ws[l][cc];
    W2[i][cc] = s;
  }
  __syncthreads();
  if (!valid) return;
  // phase 3: Y[lr][c] -= sum_i V[lr][i] W2[i][c]
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = W2[i][c];
  lr = g;
  for (; lr + 3 * AP_G < mp; lr += 4 * AP_G) {
    double y[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) y[q] = Yb[(long)(lr + q * AP_G) * ldy];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v[16];
      load_vrow(Ab + (long)(lr + q * AP_G) * lda, lr + q * AP_G, pw, v);
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) s += v[i] * w[i];
      Yb[(long)(lr + q * AP_G) * ldy] = y[q] - s;
    }
  }
  for (; lr < mp; lr += AP_G) {
    double v[16];
    load_vrow(Ab + (long)lr * lda, lr, pw, v);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += v[i] * w[i];
    Yb[(long)lr * ldy] -= s;
  }
}

__global__ void k_extract_r(const double* __restrict__ A, int kr, int n, long lda, double* __restrict__ R) {
  const long total = (long)kr * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long i = e / n;
    const int j = (int)(e % n);
    R[e] = (j >= i) ? A[i * lda + j] : 0.0;
  }
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

hipError_t householder_qr(hipStream_t s, double* A, int m, int n, long lda, double* Tbuf) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (m > 4096) return hipErrorInvalidValue;
  const int kmax = std::min(m, n);
  return for_each_panel(m, kmax, [&](int p, int j0, int pw, PanelCfg c) -> hipError_t {
    double* T = Tbuf + (long)p * 256;
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
    if (e != hipSuccess) return e;
    const int c0 = j0 + pw;
    const int nc = n - c0;
    if (nc > 0) {
      hipLaunchKernelGGL(k_apply_panel, dim3((nc + 15) / 16), dim3(AP_NT), 0, s, (const double*)A, lda, j0, m - j0,
                         j0, pw, (const double*)T, A, lda, j0, c0, nc, 1);
      e = hipGetLastError();
    }
    return e;
  });
}

hipError_t apply_q(hipStream_t s, const double* A, int m, int kref, long lda, const double* Tbuf, double* Y,
                   int ncols, long ldy, bool trans) {
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
    hipLaunchKernelGGL(k_apply_panel, dim3((ncols + 15) / 16), dim3(AP_NT), 0, s, A, lda, q.j0, m - q.j0, q.j0, q.pw,
                       Tbuf + (long)q.p * 256, Y, ldy, q.j0, 0, ncols, trans ? 1 : 0);
    hipError_t e = hipGetLastError();
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
