// Host-side declarations of the kernel launchers (internal to libqtt).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qtt {

// ---------------------------------------------------------------- GEMM
// Row-major C[M x N] = alpha * op(A)[M x K] * op(B)[K x N] + beta * C.
// op(A) = A (lda >= K) or A^T (A stored K x M, lda >= M); same for B.
// Batched with element strides sA, sB, sC.  FP64 on MFMA f64 16x16x4.
hipError_t gemm_f64(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha,
                    const double* A, long lda, long sA, const double* B, long ldb, long sB,
                    double beta, double* C, long ldc, long sC, int batch);
// C = alpha A A^T + beta C on the tiles of C (N x N) that hold part of its
// lower triangle (32 x 64 tiles for K <= 64, else 64 x 64; A: N x K,
// row-major); the tiles wholly above the diagonal are not touched.  For
// symmetric updates whose upper triangle is never read.
hipError_t gemm_f64_lower_nt(hipStream_t s, int N, int K, double alpha, const double* A, long lda, double beta,
                             double* C, long ldc);
hipError_t gemm_f32(hipStream_t s, bool ta, bool tb, int M, int N, int K, float alpha,
                    const float* A, long lda, long sA, const float* B, long ldb, long sB,
                    float beta, float* C, long ldc, long sC, int batch);
// FP64 operands, each split into three bf16 pieces; `nprod` = 3 or 6 split
// products accumulated in FP32 on MFMA bf16; result stored as FP64.
hipError_t gemm_bf16split(hipStream_t s, bool ta, bool tb, int M, int N, int K,
                          const double* A, long lda, const double* B, long ldb,
                          double* C, long ldc, int nprod);
// FP64 operands rounded to FP32, FP32 MFMA with FP32 accumulation, FP64 result.
hipError_t gemm_f64_via_f32(hipStream_t s, bool ta, bool tb, int M, int N, int K,
                            const double* A, long lda, const double* B, long ldb,
                            double* C, long ldc);

// ---------------------------------------------------------------- contraction
template <typename T>
hipError_t contract_hadamard(hipStream_t s, const T* A, int ra0, int d, int ra1,
                             const T* B, int rb0, int rb1, T* C);
template <typename T>
hipError_t contract_mpo(hipStream_t s, const T* W, int rw0, int di, int dj, int rw1,
                        const T* X, int rx0, int rx1, T* C);
// Operator product C[(a,c), i, k, (b,d)] = sum_j A[a,i,j,b] B[c,j,k,d].
template <typename T>
hipError_t contract_mpo_mpo(hipStream_t s, const T* A, int ra0, int di, int dj, int ra1, const T* B, int rb0,
                            int dk, int rb1, T* C);
// One core of an exact sum of up to kMaxAddTerms trains: term q's core
// (r0[q] x P x r1[q]) sits at row offset off0[q] / column offset off1[q] of
// the R0 x P x R1 output core (first: one row, terms side by side, scaled by
// coef[q]; last: one column; first && last: the weighted sum).
constexpr int kMaxAddTerms = 16;
template <typename T>
struct AddTerms {
  const T* src[kMaxAddTerms];
  int r0[kMaxAddTerms], r1[kMaxAddTerms], off0[kMaxAddTerms], off1[kMaxAddTerms];
  double coef[kMaxAddTerms];
};
template <typename T>
hipError_t tt_add_core(hipStream_t s, const AddTerms<T>& terms, int count, int P, int R0, int R1, int first,
                       int last, T* out);
// M[(a,i),(mu',nu')] = sum_{mu,j} Y[a,mu,j,nu'] W[mu,i,j,mu']  (FP64)
hipError_t bond_mpo_apply(hipStream_t s, const double* Y, int rho, int rw0, int dj, int rx1,
                          const double* W, int di, int rw1, double* M);
// M[(a,i),(mu',nu')] = sum_mu Y[a,mu,i,nu'] A[mu,i,mu']  (FP64, Hadamard factored)
hipError_t bond_hadamard_apply(hipStream_t s, const double* Y, int rho, int ra0, int d, int rb1,
                               const double* A, int ra1, double* M);
template <typename T>
hipError_t contract_backward_x(hipStream_t s, bool mpo, const T* W, int rw0, int di, int dj,
                               int rw1, const T* dC, int rx0, int rx1, T* dX);
template <typename T>
hipError_t contract_backward_w(hipStream_t s, bool mpo, const T* X, int rx0, int dj, int rx1,
                               const T* dC, int rw0, int di, int rw1, T* dW);

// ---------------------------------------------------------------- QR
// Blocked Householder QR of the m x n row-major matrix A (in place).  Reflector
// vectors below the diagonal, R on and above; one 64 x 64 compact-WY factor
// T per 64-column block of reflectors in Tbuf (qr_t_doubles(m, n) doubles;
// also enough for the 16 x 16 blocks of the batched workgroup QR).
// Supports m <= 4096.  scratch: qr_scratch_doubles(n).
hipError_t householder_qr(hipStream_t s, double* A, int m, int n, long lda, double* Tbuf, double* scratch);
// Y <- Q Y (trans=false, blocks in reverse order) or Q^T Y (trans=true,
// forward order); Y has m rows.  scratch: qr_scratch_doubles(ncols).
hipError_t apply_q(hipStream_t s, const double* A, int m, int kref, long lda, const double* Tbuf,
                   double* Y, int ncols, long ldy, bool trans, double* scratch);
// Scratch of one QR or Q application on ncols columns: split-K partials
// (up to 64 chunks x 64 x ncols), the 64 x ncols product, inner T blocks and tau.
inline long qr_scratch_doubles(long ncols) {
  const long nc = ncols < 1 ? 1 : ncols;
  return 64L * 64L * nc + 64L * nc + 8L * 256L + 64L;
}
// R = upper trapezoid of A[0:kr, 0:n] (zeros below the diagonal) into Rout (ld n).
hipError_t extract_r(hipStream_t s, const double* A, int kr, int n, long lda, double* Rout);

// ---------------------------------------------------------------- SVD
// One-sided Jacobi on the rows of X (p x L, row-major, ld L): on return the
// rows are mutually orthogonal (X <- Z^T X, Z orthogonal, not formed).
// counter: 8 + ceil(p / 8) unsigned of device scratch (cleared by the routine).
// sweeps_dev[0] receives the sweeps executed, sweeps_dev[1] 1 if a sweep
// without rotations was reached within max_sweeps (converged), else 0.
// ref_norm (device, nullable): the largest input row norm; rows whose norm
// falls below 8 u sqrt(p) times it (the rounding noise of the input) are
// deflated to zero.
hipError_t jacobi_rows(hipStream_t s, double* X, int p, int L, unsigned* counter, int max_sweeps,
                       int* sweeps_dev, const double* ref_norm = nullptr);
// dst[j] = src[perm[j]] (row gather).
hipError_t permute_rows(hipStream_t s, const double* src, int p, int L, const int* perm, double* dst);
// sigma_i = ||X_i||, perm = argsort descending (stable on ties).
hipError_t row_norms_sorted(hipStream_t s, const double* X, int p, int L, double* sig_sorted,
                            int* perm);

// ---------------------------------------------------------------- small kernels
hipError_t fill_f64(hipStream_t s, double* p, double v, long n);
hipError_t fill_u32(hipStream_t s, unsigned* p, unsigned v, long n);
hipError_t fill_f32(hipStream_t s, float* p, float v, long n);
hipError_t set_eye_rect(hipStream_t s, double* Z, int m, int q);
hipError_t copy_pad_rows(hipStream_t s, const double* src, int rows, int cols, long lds,
                         double* dst, int rows_out, long ldd);
hipError_t frob_norm(hipStream_t s, const double* x, long n, double* out);
// y += alpha x (n entries).
hipError_t axpy_f64(hipStream_t s, long n, double alpha, const double* x, double* y);
// dst = src / (s2[0] + s2[1]) with s2 on the device (a plain copy when the sum
// is zero); rows x cols, leading dimensions lds / ldd; dst may equal src.
hipError_t copy_scaled_inv(hipStream_t s, const double* src, int rows, int cols, long lds, const double* s2,
                           double* dst, long ldd);
hipError_t transpose(hipStream_t s, const double* A, int rows, int cols, long lda, double* B, long ldb);

struct TruncOut {
  int rank;
  int capped;
  double tail_r;
  double tail_rm1;
  double norm;
  double delta;
};
// Rank decision at one bond from sorted singular values (device).
hipError_t truncate_decide(hipStream_t s, const double* sig, int cnt, const double* norm_dev,
                           double rel_tol, int nbonds, long max_rank, TruncOut* out_dev);
// Rows perm[0:r] of X scaled to unit norm -> out (r x L); r read from t on device,
// rmax_host bounds the launch.
hipError_t gather_rows_normalized(hipStream_t s, const double* X, int L, const int* perm, const double* sig,
                                  const TruncOut* t, double* out, long ldo, int rmax_host);
// V (rb x L): rows perm[0:r] of X scaled to unit norm (r = t->rank on the
// device), zero rows r..rb-1.
hipError_t gather_rows_padded(hipStream_t s, const double* X, int L, const int* perm, const double* sig,
                              const TruncOut* t, double* V, int rb);
// out[a][i r + c] = B[a][i rb + c] for c < r (r = *r_dev on the device), zeros
// after the first d r entries of each row of length d rb.
hipError_t compact_cols(hipStream_t s, const double* B, int rows, int d, int rb, const int* r_dev, double* out);
// Compact core [r0, d r1] (r0 = *r0_dev, r1 = *r1_dev) from the leading
// entries of the first r0 rows of V (row length L); rows_bound >= r0.
hipError_t core_from_rows(hipStream_t s, const double* V, int rows_bound, int L, const int* r0_dev, int d,
                          const int* r1_dev, double* out);
// ranks[0..n] and a status word from the per-bond decisions t[0..n-2] and the
// Jacobi records sweeps[2 (n-1)] (see k_round_record).
hipError_t round_record(hipStream_t s, const TruncOut* t, const int* sweeps, int n, const double* norm_dev,
                        long long* ranks, int* status, int code_nonfinite, int code_noconv);
long qr_t_doubles(int m, int n);

// ---------------------------------------------------------------- linear solver (solve.hip)
// Local matrix of the energy over a block of P physical values:
// A[(a,i,c),(x,j,y)] = sum LW[a,al,x] Wl[al,i,j,be] RW[c,be,y]  (N = r0 P r1,
// A is N x N row-major; LW [r0][w0][r0], Wl [w0][P][P][w1], RW [r1][w1][r1]).
hipError_t local_matrix(hipStream_t s, const double* LW, const double* Wl, const double* RW, int r0, int P, int r1,
                        int w0, int w1, double* A);
// T2[a][i][be][y] = sum_{al,j} T1[a][al][j][y] W[al][i][j][be]
hipError_t env3_left_mid(hipStream_t s, const double* T1, const double* W, int r0, int w0, int d, int w1, int r1,
                         double* T2);
// U2[i][c][al][x] = sum_{j,be} W[al][i][j][be] U1[x][j][c][be]
hipError_t env3_right_mid(hipStream_t s, const double* U1, const double* W, int r0, int w0, int d, int w1, int r1,
                          double* U2);
// G[al][(i1,i2)][(j1,j2)][ga] = sum_be W1[al][i1][j1][be] W2[be][i2][j2][ga]
hipError_t mpo_pair(hipStream_t s, const double* W1, const double* W2, int w0, int d1, int w1, int d2, int w2,
                    double* G);
// x <- A^{-1} x for a symmetric positive definite A (N x N, leading
// dimension lda; its lower triangle is read): blocked Cholesky A = L L^T in
// place (64-column blocks: each diagonal block factored and inverted by one
// workgroup, the panel formed in place with that inverse, the trailing
// update as an FP64 GEMM on the tiles on or below the diagonal); L y = x is
// solved along the way (each block's step with the factorisation of its
// diagonal block and its panel), then L^T x = y by blocks with the diagonal
// blocks' inverses.  N <= 4096.
// A is overwritten; a pivot that is not positive gives NaN in x.  work:
// chol_work_doubles(N).
hipError_t chol_solve(hipStream_t s, double* A, int N, long lda, double* x, double* work);
inline long chol_work_doubles(long N) { return ((N + 63) / 64) * 4096L; }

// ---------------------------------------------------------------- kernel setup
// Raise the dynamic-LDS limit of the kernels that stage more than 64 KiB
// (on the current device); called once per handle before any launch.
hipError_t qr_configure();
hipError_t jacobi_configure();
hipError_t batched_configure();
inline hipError_t configure_kernels() {
  hipError_t e = qr_configure();
  if (e == hipSuccess) e = jacobi_configure();
  if (e == hipSuccess) e = batched_configure();
  return e;
}

// ---------------------------------------------------------------- launch profiling
namespace prof {
enum Class {
  APPLY_PANEL = 0,
  JACOBI = 1,
  QR_PANEL = 2,
  BLOCK_VTY = 3,
  BLOCK_UPD = 4,
  CHOL_BLOCK = 5,
  CHOL_UPDATE = 6,
  CHOL_SOLVE = 7
};
constexpr int kNumClasses = 8;
bool active(int cls);
void begin(hipStream_t st, int cls, double bytes, double flops);
void end(hipStream_t st);
hipError_t start(int cls, int max_launches);
hipError_t stop(long* launches, double* total_ms, double* bytes, double* flops);
}  // namespace prof

}  // namespace qtt
