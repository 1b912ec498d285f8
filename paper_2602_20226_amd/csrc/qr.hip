// Blocked Householder QR for the rounding sweep (FP64).
//
// Two levels.  Inner panels of up to 16 columns are factored by one
// workgroup each (qr_panel_dev in qr_device.hpp) and applied to the rest of
// their 64-column outer block by apply_block (one workgroup per column).
// The reflectors of an outer block are then aggregated into one compact-WY
// pair (V, T) with T of order <= 64, built from S = V^T V and the panels'
// own T blocks, and the trailing matrix -- and every later application of
// Q or Q^T -- is updated once per outer block by three kernels on FP64
// MFMA tiles:
//     P_c = V_c^T Y_c          (split over row chunks c of 64..256 rows),
//     W   = -op(T) sum_c P_c,
//     Y  += V W.
// V is never copied: the kernels read it from the unit lower trapezoid of
// the factored matrix.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"
#include "qr_device.hpp"

#include <algorithm>

namespace qtt {

namespace {

template <int NT, int RPT, int PW>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_qr_panel(
    double* __restrict__ A, long lda, int m, int j0, int pw, double* __restrict__ Tout, double* __restrict__ tau) {
  extern __shared__ double stage[];  // NT x (PW + 1)
  qr_panel_dev<NT, RPT, PW>(A, lda, m, j0, pw, Tout, stage, tau);
}

// ------------------------------------------------------------ outer blocks
constexpr int OB = 64;    // outer block width: reflectors aggregated per (V, T)
constexpr int KC = 256;   // largest row chunk of the split-K products
constexpr int KC_MIN = 64;      // smallest (one staged slab)
constexpr int MAX_CHUNKS = 64;  // m <= 4096 at the smallest chunk

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma16x16x4(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Element (k, i) of the unit lower trapezoidal V of an outer block whose
// origin is A[j0][j0]: 1 on the diagonal, the stored vector below, 0 above
// and outside [0, mp) x [0, nb).
__device__ __forceinline__ double vel(const double* __restrict__ Ab, long lda, int mp, int nb, int k, int i) {
  if (k >= mp || i >= nb || k < i) return 0.0;
  return k == i ? 1.0 : Ab[(long)k * lda + i];
}

// V of an outer block is staged in LDS in slabs of SL rows (double
// buffered: the next slab's global loads are in flight while the current
// one feeds the MFMAs), so that the four waves of a workgroup share it.
constexpr int SL = 64;      // rows per staged slab
constexpr int VT_LD = 80;   // LDS row stride for V^T operands: conflict-free
constexpr int VU_LD = 66;   // LDS row stride for V operands: conflict-free

// st[q] = V[r0 + e / 64][e % 64], e = tid + 256 q  (0 past kend)
__device__ __forceinline__ void fetch_vslab(const double* __restrict__ Ab, long lda, int mp, int nb, int r0, int kend,
                                            double (&st)[SL * OB / 256]) {
#pragma unroll
  for (int q = 0; q < SL * OB / 256; ++q) {
    const int e = threadIdx.x + 256 * q;
    const int k = r0 + e / OB;
    st[q] = (k < kend) ? vel(Ab, lda, mp, nb, k, e % OB) : 0.0;
  }
}
template <int LD>
__device__ __forceinline__ void put_vslab(double* __restrict__ Vs, const double (&st)[SL * OB / 256]) {
#pragma unroll
  for (int q = 0; q < SL * OB / 256; ++q) {
    const int e = threadIdx.x + 256 * q;
    Vs[(e / OB) * LD + e % OB] = st[q];
  }
}

// P[c][i][col] = sum over rows k of chunk c of V[k][i] * Yv[k][col],
// i < nb, col < ncols; Yv = V for col < s_cols, else Y[k][col].
// 256 threads; wave w owns output columns [16w, 16w + 16) of the 64-column
// tile and all four 16-row blocks of i.  MFMA f64 16x16x4 operand layout:
// A[i][k] in lane (i + 16 k), B[k][col] in lane (col + 16 k); result
// C[i][col] with i = lane / 16 + 4 v, col = lane % 16.
__global__ __launch_bounds__(256) void k_vty(const double* __restrict__ A, long lda, int j0, int mp, int nb,
                                             const double* __restrict__ Y, long ldy, int yr0, int yc0, int ncols,
                                             int s_cols, int ntiles, int kc, double* __restrict__ part) {
  __shared__ double Vs[2][SL * VT_LD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tile = blockIdx.x % ntiles, chunk = blockIdx.x / ntiles;
  const int col = tile * 64 + w * 16 + (lane & 15);
  const int kq = lane >> 4, il = lane & 15;
  const int kbeg = chunk * kc, kend = min(mp, kbeg + kc);
  const int nslab = (kend - kbeg + SL - 1) / SL;
  const double* Ab = A + (long)j0 * lda + j0;
  const double* Yc = Y + (long)yr0 * ldy + yc0 + col;
  const bool colok = col < ncols;
  const bool colv = col < s_cols;
  f64x4 acc[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
  double st[SL * OB / 256], b[SL / 4], b2[SL / 4];
  auto fetch_b = [&](int r0, double (&bb)[SL / 4]) {
#pragma unroll
    for (int t = 0; t < SL / 4; ++t) {
      const int k = r0 + 4 * t + kq;
      bb[t] = (colok && k < kend) ? (colv ? vel(Ab, lda, mp, nb, k, col) : Yc[(long)k * ldy]) : 0.0;
    }
  };
  fetch_vslab(Ab, lda, mp, nb, kbeg, kend, st);
  fetch_b(kbeg, b);
  put_vslab<VT_LD>(Vs[0], st);
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    const int r0 = kbeg + sl * SL;
    const bool more = sl + 1 < nslab;
    if (more) {
      fetch_vslab(Ab, lda, mp, nb, r0 + SL, kend, st);
      fetch_b(r0 + SL, b2);
    }
    const double* V = Vs[sl & 1];
#pragma unroll
    for (int t = 0; t < SL / 4; ++t)
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = mfma16x16x4(V[(4 * t + kq) * VT_LD + 16 * s + il], b[t], acc[s]);
    if (more) {
      put_vslab<VT_LD>(Vs[(sl + 1) & 1], st);
#pragma unroll
      for (int t = 0; t < SL / 4; ++t) b[t] = b2[t];
    }
    __syncthreads();
  }
  if (!colok) return;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = s * 16 + kq + 4 * v;
      if (i < nb) part[((long)chunk * OB + i) * ncols + col] = acc[s][v];
    }
}

// Panel boundaries inside one outer block (offsets relative to the block).
struct PanelList {
  int np;
  int off[OB / 8 + 1];  // panel q covers columns [off[q], off[q + 1])
};

// Compact-WY factor of an outer block from S = sum_c P_c[0:nb, 0:nb] = V^T V
// and the panels' own factors T_q (its diagonal blocks): block column q is
//     T[0:o, q] = -T[0:o, 0:o] S[0:o, q] T_q,   o = off[q],
// which is the column recurrence T[0:j, j] = -tau_j T[0:j, 0:j] S[0:j, j]
// taken one panel at a time.  One workgroup.
__global__ __launch_bounds__(256) void k_tbuild(const double* __restrict__ Sg, int sstride, int nb,
                                                const double* __restrict__ tin, PanelList pl,
                                                double* __restrict__ Tout) {
  __shared__ double S[OB][OB + 1];
  __shared__ double T[OB][OB + 1];
  __shared__ double X[OB][17];
  const int tid = threadIdx.x;
#pragma unroll
  for (int u = 0; u < OB * OB / 256; ++u) {
    const int e = tid + 256 * u;
    const int i = e / OB, j = e % OB;
    S[i][j] = (i < nb && j < nb && i < j) ? Sg[(long)i * sstride + j] : 0.0;
    T[i][j] = 0.0;
  }
  __syncthreads();
  for (int q = 0; q < pl.np; ++q) {
    const int o = pl.off[q], w = pl.off[q + 1] - o;
    for (int e = tid; e < w * w; e += 256) T[o + e / w][o + e % w] = tin[(long)q * 256 + (e / w) * 16 + e % w];
  }
  __syncthreads();
  for (int q = 1; q < pl.np; ++q) {
    const int o = pl.off[q], w = pl.off[q + 1] - o;
    // X = T[0:o, 0:o] S[0:o, o:o+w]   (T upper triangular)
    for (int e = tid; e < o * w; e += 256) {
      const int i = e / w, c = e % w;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};  // four partial sums: a quarter of the dependent chain
      int l = i;
      for (; l + 3 < o; l += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += T[i][l + u] * S[l + u][o + c];
      }
      for (; l < o; ++l) acc[0] += T[i][l] * S[l][o + c];
      X[i][c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    __syncthreads();
    // T[0:o, o:o+w] = -X T_q
    for (int e = tid; e < o * w; e += 256) {
      const int i = e / w, c = e % w;
      double acc = 0.0;
      for (int l = 0; l <= c; ++l) acc += X[i][l] * T[o + l][o + c];
      T[i][o + c] = -acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < OB * OB; e += 256) Tout[e] = T[e / OB][e % OB];
}

// W[i][col] = sum_c P_c[i][col] for i < nb, col < ncols (fixed summation
// order: deterministic).  One thread per entry, loads in flight 16 at a time.
__global__ __launch_bounds__(256) void k_red(const double* __restrict__ part, int nchunks, int ncols, int nb,
                                             double* __restrict__ W) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)nb * ncols) return;
  const int i = (int)(e / ncols), col = (int)(e % ncols);
  double sum = 0.0;
  for (int c0 = 0; c0 < nchunks; c0 += 16) {
    double v[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = (c0 + c < nchunks) ? part[((long)(c0 + c) * OB + i) * ncols + col] : 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) sum += v[c];
  }
  W[(long)i * ncols + col] = sum;
}

// Y[k][col] += sum_i V[k][i] W'[i][col] for the rows of one chunk and one
// 64-column tile, W' = -op(T) W.  The workgroup first forms its slice of W'
// (64 x 16 per wave, f64 MFMA); result element [16 s + kq + 4 v][col] is
// exactly the B operand of k-step q = 4 s + v, so no data movement is needed
// between the two.  Wave w owns columns [16w, 16w + 16); rows go in blocks
// of 16 (A = V rows from the staged slab, C = Y rows in the f64 MFMA result
// layout, fetched one slab ahead).
__global__ __launch_bounds__(256) void k_vupd(const double* __restrict__ A, long lda, int j0, int mp, int nb,
                                              const double* __restrict__ T, int trans, const double* __restrict__ W,
                                              long ldw, int wc0, double* __restrict__ Y, long ldy, int yr0, int yc0,
                                              int ncols, int ntiles, int kc) {
  __shared__ double Vs[2][SL * VU_LD];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int tile = blockIdx.x % ntiles, chunk = blockIdx.x / ntiles;
  const int col = tile * 64 + w * 16 + (lane & 15);
  const int kq = lane >> 4, il = lane & 15;
  const bool colok = col < ncols;
  const int kbeg = chunk * kc, kend = min(mp, kbeg + kc);
  const int nslab = (kend - kbeg + SL - 1) / SL;
  const double* Ab = A + (long)j0 * lda + j0;
  double* Yc = Y + (long)yr0 * ldy + yc0 + col;
  const int nk = (nb + 3) / 4;
  double st[SL * OB / 256];
  fetch_vslab(Ab, lda, mp, nb, kbeg, kend, st);
  double c[SL / 16][4], c2[SL / 16][4];
  auto fetch_c = [&](int r0, double (&cc)[SL / 16][4]) {
#pragma unroll
    for (int rb = 0; rb < SL / 16; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = r0 + 16 * rb + kq + 4 * v;
        cc[rb][v] = (colok && k < kend) ? Yc[(long)k * ldy] : 0.0;
      }
  };
  fetch_c(kbeg, c);
  double bw[OB / 4];
  {
    double wb[OB / 4];
#pragma unroll
    for (int q = 0; q < OB / 4; ++q) {
      const int i = 4 * q + kq;
      wb[q] = (i < nb && colok) ? W[(long)i * ldw + wc0 + col] : 0.0;
    }
    f64x4 acc[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[s] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < OB / 4; ++q) {
      const int k = 4 * q + kq;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int i = 16 * s + il;
        const double t = trans ? T[k * OB + i] : T[i * OB + k];
        acc[s] = mfma16x16x4(t, wb[q], acc[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v) bw[4 * s + v] = -acc[s][v];
  }
  put_vslab<VU_LD>(Vs[0], st);
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    const int r0 = kbeg + sl * SL;
    const bool more = sl + 1 < nslab;
    if (more) {
      fetch_vslab(Ab, lda, mp, nb, r0 + SL, kend, st);
      fetch_c(r0 + SL, c2);
    }
    const double* V = Vs[sl & 1];
#pragma unroll
    for (int rb = 0; rb < SL / 16; ++rb) {
      f64x4 acc = f64x4{c[rb][0], c[rb][1], c[rb][2], c[rb][3]};
#pragma unroll
      for (int q = 0; q < OB / 4; ++q)
        if (q < nk) acc = mfma16x16x4(V[(16 * rb + il) * VU_LD + 4 * q + kq], bw[q], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = r0 + 16 * rb + kq + 4 * v;
        if (colok && k < kend) Yc[(long)k * ldy] = acc[v];
      }
    }
    if (more) {
      put_vslab<VU_LD>(Vs[(sl + 1) & 1], st);
#pragma unroll
      for (int rb = 0; rb < SL / 16; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) c[rb][v] = c2[rb][v];
    }
    __syncthreads();
  }
}

inline void apply_cost(int mp, int pw, int ncols, double& bytes, double& flops);

// Block-reflector application inside an outer block, one launch:
// workgroup t owns column c0 + t of Y over all mp rows, so no workgroup
// reads what another one writes:
//     w = V^T y  (one workgroup sum of PWV values),  w <- op(T) w,
//     y <- y - V w.
// V: rows [r0, r0+mp) of A, columns [vc0, vc0+pw) (pw <= PWV), unit lower
// trapezoidal; y: rows [yr0, yr0+mp) of column c0 + t of Y.
// trans: Y <- (I - V T^T V^T) Y, else Y <- (I - V T V^T) Y.
// The NT lanes form quads; the quad (tid >> 2) holds rows NT/4 k + (tid >> 2),
// lane q of it V columns [q VPQ, (q+1) VPQ) of those rows, and all four
// lanes the y values.  V and y stay in registers between the two passes
// (KMAX = ceil(4 mp / NT) chunks); a quad's partial products are summed by
// two DPP exchanges, which leave the same bits in its four lanes.
// PAIRS: pw == PWV and lda even -- V is read 16 bytes at a time.
template <int NT, int PWV, int KMAX, bool PAIRS>
__global__ __launch_bounds__(NT) void k_apply1(const double* __restrict__ A, long lda, int r0, int mp, int vc0, int pw,
                                               const double* __restrict__ T, double* __restrict__ Y, long ldy,
                                               int yr0, int c0, int trans) {
  constexpr int VPQ = PWV / 4, RS = NT / 4;
  __shared__ double slots[2 * (NT / 64) * PWV];
  __shared__ double Ts[16 * 16];
  const int tid = threadIdx.x, q = tid & 3, sr = tid >> 2;
  for (int t = tid; t < 256; t += NT) Ts[t] = T[t];  // visible after the barrier of the sum below
  const double* __restrict__ Ab = A + (long)(r0 + sr) * lda + vc0 + q * VPQ;
  double* __restrict__ yb = Y + (long)(yr0 + sr) * ldy + c0 + blockIdx.x;
  const long astep = (long)RS * lda, ystep = (long)RS * ldy;
  double v[KMAX][VPQ], y[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int lr = RS * k + sr;
    const bool in = lr < mp;
    y[k] = in ? yb[k * ystep] : 0.0;
    if (PAIRS) {
#pragma unroll
      for (int e = 0; e < VPQ; e += 2) {
        double2 t2 = make_double2(0.0, 0.0);
        if (in) t2 = *reinterpret_cast<const double2*>(Ab + k * astep + e);
        v[k][e] = t2.x;
        v[k][e + 1] = t2.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < VPQ; ++e) v[k][e] = (in && q * VPQ + e < pw) ? Ab[k * astep + e] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < VPQ; ++e) {  // unit diagonal, zeros above it
      const int i = q * VPQ + e;
      if (lr <= i) v[k][e] = (lr == i && in && i < pw) ? 1.0 : 0.0;
    }
  }
  double acc[VPQ];
#pragma unroll
  for (int e = 0; e < VPQ; ++e) acc[e] = 0.0;
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
#pragma unroll
    for (int e = 0; e < VPQ; ++e) acc[e] += v[k][e] * y[k];
  double x[PWV], w[PWV];
#pragma unroll
  for (int i = 0; i < PWV; ++i) x[i] = (i / VPQ == q) ? acc[i % VPQ] : 0.0;
  wg_sum_vals<NT, PWV>(x, slots, 0, w);
  double w2[VPQ];
#pragma unroll
  for (int e = 0; e < VPQ; ++e) {
    const int i = q * VPQ + e;
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < PWV; ++l) t += (trans ? Ts[l * 16 + i] : Ts[i * 16 + l]) * w[l];
    w2[e] = t;
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    double pk = 0.0;
#pragma unroll
    for (int e = 0; e < VPQ; ++e) pk += v[k][e] * w2[e];
    pk += dpp<DPP_XOR1>(pk);
    pk += dpp<DPP_XOR2>(pk);
    if (q == 0 && RS * k + sr < mp) yb[k * ystep] = y[k] - pk;
  }
}

template <int NT, int PWV, int KMAX>
inline void launch_apply1(hipStream_t s, bool pairs, const double* A, long lda, int r0, int mp, int vc0, int pw,
                          const double* T, double* Y, long ldy, int yr0, int c0, int ncols, int trans) {
  static_assert(KMAX * NT / 4 >= 64, "");
  if (pairs)
    hipLaunchKernelGGL((k_apply1<NT, PWV, KMAX, true>), dim3(ncols), dim3(NT), 0, s, A, lda, r0, mp, vc0, pw, T, Y,
                       ldy, yr0, c0, trans);
  else
    hipLaunchKernelGGL((k_apply1<NT, PWV, KMAX, false>), dim3(ncols), dim3(NT), 0, s, A, lda, r0, mp, vc0, pw, T, Y,
                       ldy, yr0, c0, trans);
}

// One block-reflector application inside an outer block (mp <= 4096 rows,
// pw <= 16; pw <= 8 when mp > 2048).
hipError_t apply_block(hipStream_t s, const double* A, long lda, int r0, int mp, int vc0, int pw, const double* T,
                       double* Y, long ldy, int yr0, int c0, int ncols, int trans) {
  if (mp <= 0 || ncols <= 0) return hipSuccess;
  if (mp > 4096 || pw > 16 || (mp > 2048 && pw > 8)) return hipErrorInvalidValue;
  if (prof::active(prof::APPLY_PANEL)) {
    double b, f;
    apply_cost(mp, pw, ncols, b, f);
    prof::begin(s, prof::APPLY_PANEL, b, f);
  }
  const int pwv = mp > 2048 ? 8 : 16;
  const bool pairs = pw == pwv && (lda & 1) == 0 && (vc0 & 1) == 0 && ((uintptr_t)A & 15) == 0;
  if (mp <= 256)
    launch_apply1<256, 16, 4>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  else if (mp <= 512)
    launch_apply1<256, 16, 8>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  else if (mp <= 1024)
    launch_apply1<512, 16, 8>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  else if (mp <= 2048)
    launch_apply1<512, 16, 16>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  else if (mp <= 3072)
    launch_apply1<512, 8, 24>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  else if (mp <= 3584)
    launch_apply1<512, 8, 28>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  else
    launch_apply1<512, 8, 32>(s, pairs, A, lda, r0, mp, vc0, pw, T, Y, ldy, yr0, c0, ncols, trans);
  hipError_t e = hipGetLastError();
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

// One workgroup per panel; few waves keep the per-column reductions cheap
// (configurations measured on the 3D rank-256 rounding shapes).
inline PanelCfg panel_cfg(int mp) {
  if (mp <= 256) return {256, 1, 16};
  if (mp <= 512) return {256, 2, 16};
  if (mp <= 1024) return {256, 4, 16};
  if (mp <= 1792) return {256, 7, 16};
  if (mp <= 2048) return {512, 4, 16};
  if (mp <= 3072) return {256, 12, 8};
  if (mp <= 3584) return {512, 7, 8};
  return {512, 8, 8};
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Scratch layout (doubles) for ncols target columns: split-K partials
// [MAX_CHUNKS][OB][ncols], W [OB][ncols], inner T blocks [OB/8][256], tau [OB].
struct Scr {
  double *part, *w, *tin, *tau;
};
inline Scr scr_of(double* scratch, long ncols) {
  Scr r;
  r.part = scratch;
  r.w = r.part + (long)MAX_CHUNKS * OB * ncols;
  r.tin = r.w + (long)OB * ncols;
  r.tau = r.tin + (OB / 8) * 256;
  return r;
}

constexpr int kPanelBigLds = 512 * 17 * 8;  // k_qr_panel<512, 4, 16>: 512 x 17 doubles of staging

hipError_t launch_panel(hipStream_t s, double* A, long lda, int m, int j0, int pw, PanelCfg c, double* T,
                        double* tau) {
  if (prof::active(prof::QR_PANEL)) {
    const double mp = m - j0;
    prof::begin(s, prof::QR_PANEL, 8.0 * 2.0 * mp * pw, 4.0 * mp * pw * pw);
  }
  const size_t sh = (size_t)c.nt * (c.pw + 1) * sizeof(double);
  // only the 512-thread, 16-column instance stages more than the default
  // 64 KiB; its limit is raised by qr_configure() when a handle is created
  if (sh > (c.nt == 512 && c.pw == 16 ? kPanelBigLds : 64 * 1024)) return hipErrorInvalidValue;
  if (c.nt == 256 && c.rpt == 1)
    hipLaunchKernelGGL((k_qr_panel<256, 1, 16>), dim3(1), dim3(256), sh, s, A, lda, m, j0, pw, T, tau);
  else if (c.nt == 256 && c.rpt == 2)
    hipLaunchKernelGGL((k_qr_panel<256, 2, 16>), dim3(1), dim3(256), sh, s, A, lda, m, j0, pw, T, tau);
  else if (c.nt == 256 && c.rpt == 4)
    hipLaunchKernelGGL((k_qr_panel<256, 4, 16>), dim3(1), dim3(256), sh, s, A, lda, m, j0, pw, T, tau);
  else if (c.nt == 256 && c.rpt == 7)
    hipLaunchKernelGGL((k_qr_panel<256, 7, 16>), dim3(1), dim3(256), sh, s, A, lda, m, j0, pw, T, tau);
  else if (c.nt == 512 && c.rpt == 4)
    hipLaunchKernelGGL((k_qr_panel<512, 4, 16>), dim3(1), dim3(512), sh, s, A, lda, m, j0, pw, T, tau);
  else if (c.nt == 256 && c.rpt == 12)
    hipLaunchKernelGGL((k_qr_panel<256, 12, 8>), dim3(1), dim3(256), sh, s, A, lda, m, j0, pw, T, tau);
  else if (c.nt == 512 && c.rpt == 7)
    hipLaunchKernelGGL((k_qr_panel<512, 7, 8>), dim3(1), dim3(512), sh, s, A, lda, m, j0, pw, T, tau);
  else
    hipLaunchKernelGGL((k_qr_panel<512, 8, 8>), dim3(1), dim3(512), sh, s, A, lda, m, j0, pw, T, tau);
  hipError_t e = hipGetLastError();
  prof::end(s);
  return e;
}

// Row chunk of the split-K kernels: 256 rows, halved (down to one 64-row
// slab) while the grid has fewer than 160 workgroups, so that small
// trailing blocks still spread over the chip.
inline int pick_kc(int ncols, int mp) {
  const int ntiles = ceil_div(ncols, 64);
  int kc = KC;
  while (kc > KC_MIN && (long)ntiles * ceil_div(mp, kc) < 320) kc /= 2;
  return kc;
}

// P = V^T Yv over all row chunks of the block (mp rows); returns the number
// of chunks written (nch > 0), 0 on a launch error.
int launch_vty(hipStream_t s, const double* A, long lda, int j0, int mp, int nb, const double* Y, long ldy, int yr0,
               int yc0, int ncols, int s_cols, double* part) {
  const int kc = pick_kc(ncols, mp);
  const int ntiles = ceil_div(ncols, 64), nch = ceil_div(mp, kc);
  if (prof::active(prof::BLOCK_VTY))
    prof::begin(s, prof::BLOCK_VTY, 8.0 * ((double)mp * nb + (double)mp * (ncols - s_cols) + (double)nch * nb * ncols),
                2.0 * mp * (double)nb * ncols);
  hipLaunchKernelGGL(k_vty, dim3(ntiles * nch), dim3(256), 0, s, A, lda, j0, mp, nb, Y, ldy, yr0, yc0, ncols, s_cols,
                     ntiles, kc, part);
  hipError_t e = hipGetLastError();
  prof::end(s);
  return e == hipSuccess ? nch : 0;
}

hipError_t launch_vupd(hipStream_t s, const double* A, long lda, int j0, int mp, int nb, const double* T, int trans,
                       const double* W, long ldw, int wc0, double* Y, long ldy, int yr0, int yc0, int ncols) {
  const int kc = pick_kc(ncols, mp);
  const int ntiles = ceil_div(ncols, 64), nch = ceil_div(mp, kc);
  if (prof::active(prof::BLOCK_UPD))
    prof::begin(s, prof::BLOCK_UPD, 8.0 * (2.0 * mp * ncols + (double)mp * nb + (double)nb * ncols),
                2.0 * mp * (double)nb * ncols);
  hipLaunchKernelGGL(k_vupd, dim3(ntiles * nch), dim3(256), 0, s, A, lda, j0, mp, nb, T, trans, W, ldw, wc0, Y, ldy,
                     yr0, yc0, ncols, ntiles, kc);
  hipError_t e = hipGetLastError();
  prof::end(s);
  return e;
}

// Outer blocks [jb, jb + nb) of width OB (the last one narrower); inside
// each, inner panels of width panel_cfg(m - j).pw, clipped to the block.
// A pure function of (m, kmax): the factorisation and every later
// application of Q walk the same sequence.
template <typename F>
inline hipError_t for_each_outer(int kmax, F f) {
  for (int b = 0, jb = 0; jb < kmax; ++b, jb += OB) {
    hipError_t e = f(b, jb, std::min(OB, kmax - jb));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t qr_configure() {
  return hipFuncSetAttribute((const void*)k_qr_panel<512, 4, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kPanelBigLds);
}

long qr_t_doubles(int m, int n) { return (long)ceil_div(std::min(m, n), OB) * OB * OB; }

hipError_t householder_qr(hipStream_t s, double* A, int m, int n, long lda, double* Tbuf, double* scratch) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (m > KC_MIN * MAX_CHUNKS) return hipErrorInvalidValue;
  const int kmax = std::min(m, n);
  const Scr sc = scr_of(scratch, n);
  return for_each_outer(kmax, [&](int b, int jb, int nb) -> hipError_t {
    hipError_t e;
    // inner panels
    int q = 0;
    PanelList pl;
    pl.np = 0;
    for (int j = jb; j < jb + nb; ++q) {
      const PanelCfg c = panel_cfg(m - j);
      const int pw = std::min(c.pw, jb + nb - j);
      pl.off[q] = j - jb;
      pl.off[q + 1] = j - jb + pw;
      pl.np = q + 1;
      double* Tq = sc.tin + (long)q * 256;
      e = launch_panel(s, A, lda, m, j, pw, c, Tq, sc.tau + (j - jb));
      if (e != hipSuccess) return e;
      const int c0 = j + pw, nc = jb + nb - c0;
      if (nc > 0) {
        e = apply_block(s, A, lda, j, m - j, j, pw, Tq, A, lda, j, c0, nc, 1);
        if (e != hipSuccess) return e;
      }
      j += pw;
    }
    // aggregated (V, T) of the block, then the trailing update with Q_b^T
    const int mp = m - jb, ntrail = n - (jb + nb);
    const int ncw = nb + ntrail;
    const int nch = launch_vty(s, A, lda, jb, mp, nb, A, lda, jb, jb, ncw, nb, sc.part);
    if (nch == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_red, dim3(ceil_div((long)nb * ncw, 256)), dim3(256), 0, s, (const double*)sc.part, nch, ncw,
                       nb, sc.w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    double* T = Tbuf + (long)b * OB * OB;
    hipLaunchKernelGGL(k_tbuild, dim3(1), dim3(256), 0, s, (const double*)sc.w, ncw, nb, (const double*)sc.tin, pl, T);
    e = hipGetLastError();
    if (e != hipSuccess || ntrail <= 0) return e;
    return launch_vupd(s, A, lda, jb, mp, nb, T, 1, sc.w, ncw, nb, A, lda, jb, jb + nb, ntrail);
  });
}

hipError_t apply_q(hipStream_t s, const double* A, int m, int kref, long lda, const double* Tbuf, double* Y,
                   int ncols, long ldy, bool trans, double* scratch) {
  if (m <= 0 || ncols <= 0 || kref <= 0) return hipSuccess;
  if (m > KC_MIN * MAX_CHUNKS) return hipErrorInvalidValue;
  const Scr sc = scr_of(scratch, ncols);
  const int nblk = ceil_div(kref, OB);
  for (int t = 0; t < nblk; ++t) {
    const int b = trans ? t : nblk - 1 - t;
    const int jb = b * OB, nb = std::min(OB, kref - jb);
    const int mp = m - jb;
    const int nch = launch_vty(s, A, lda, jb, mp, nb, Y, ldy, jb, 0, ncols, 0, sc.part);
    if (nch == 0) return hipGetLastError();
    hipError_t e;
    hipLaunchKernelGGL(k_red, dim3(ceil_div((long)nb * ncols, 256)), dim3(256), 0, s, (const double*)sc.part, nch,
                       ncols, nb, sc.w);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_vupd(s, A, lda, jb, mp, nb, Tbuf + (long)b * OB * OB, trans ? 1 : 0, sc.w, ncols, 0, Y, ldy, jb, 0,
                    ncols);
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
