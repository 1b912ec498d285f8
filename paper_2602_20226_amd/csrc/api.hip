// libqtt host side: argument validation, workspace planning and sequencing of
// the contraction / QR sweep / SVD sweep / environment sweeps on the caller's
// stream.  See include/qtt.h for the contract of every entry point.
#include "../../include/qtt.h"
#include "batched.hpp"
#include "qtt_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <type_traits>
#include <vector>

using namespace qtt;

struct qtt_context {
  int device;
  int max_sweeps;       // Jacobi sweep cap of this handle's calls
  TruncOut* pin_trunc;  // pinned host readback
  int* pin_int;
  double* pin_dbl;
  void* scratch;        // device address of this device's copy of `scratch`
};

// Workspace of qtt_contract_round_noalloc: one fixed array per device, held
// until the process ends.  Host code never uses the name `scratch` as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, once per device, in qtt_create.
static_assert(QTT_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");
static __device__ __align__(256) double scratch[QTT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up on
// the first call for that device).
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_dev[device] = ptr;
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}
}  // namespace

namespace {

// Default Jacobi sweep cap.  Full-rank inputs converge in 10-15 sweeps;
// inputs with exactly null directions (structurally rank-deficient
// super-cores of the decomposition algorithm) need up to about 40, since the
// rows that collapse to rounding level are made orthogonal only after the
// others have settled.  qtt_set_jacobi_max_sweeps changes it per handle.
constexpr int kMaxSweeps = 80;
constexpr int kMaxRows = 4096;

#define QTT_HIP(call)                          \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return QTT_ERR_HIP;  \
  } while (0)

struct Scoped {
  int prev = -1;
  explicit Scoped(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~Scoped() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int check_tt(const qtt_tt* t, int legs_expected) {
  if (!t || !t->phys || !t->ranks || !t->cores) return QTT_ERR_ARG;
  if (t->n < 1) return QTT_ERR_ARG;
  if (t->legs != 1 && t->legs != 2) return QTT_ERR_ARG;
  if (legs_expected && t->legs != legs_expected) return QTT_ERR_SHAPE;
  if (t->dtype != QTT_F64 && t->dtype != QTT_F32) return QTT_ERR_DTYPE;
  if (t->ranks[0] != 1 || t->ranks[t->n] != 1) return QTT_ERR_SHAPE;
  for (int k = 0; k <= t->n; ++k)
    if (t->ranks[k] < 1 || t->ranks[k] > (1 << 24)) return QTT_ERR_SHAPE;
  for (int k = 0; k < t->n * t->legs; ++k)
    if (t->phys[k] < 1) return QTT_ERR_SHAPE;
  for (int k = 0; k < t->n; ++k)
    if (!t->cores[k]) return QTT_ERR_ARG;
  return QTT_OK;
}

inline int dphys(const qtt_tt* t, int k) { return t->phys[k * t->legs]; }          // output leg
inline int dphys_in(const qtt_tt* t, int k) { return t->phys[k * t->legs + t->legs - 1]; }  // input leg

enum Kind { K_TT = 0, K_HAD = 1, K_MPO = 2, K_OPOP = 3 };

// Shapes of the operand(s) of a rounding sweep.
struct Shape {
  Kind kind;
  int n;
  std::vector<int> d;        // output physical size per core
  std::vector<long> rc;      // contracted bond ranks r_C (n+1)
  std::vector<long> ra, rb;  // operand ranks (factored kinds)
  std::vector<int> dj;       // MPO input leg
};

// Workspace plan (offsets in doubles) shared by size queries and execution.
struct Plan {
  std::vector<long> m;     // rows of M_k (k < n-1): rho_{k-1} d_k
  std::vector<long> rho;   // rank after QR, rho[-1] = 1 stored at index 0 => rho[k+1]
  std::vector<long> offM, offT;
  std::vector<long> rr;    // bound of the rounded rank per bond (n+1)
  long offCenter = 0, offR = 0, offY = 0, offZ = 0, offX = 0, offXc = 0, offYn = 0, offTB = 0;
  long offSig = 0, offPerm = 0, offTrunc = 0, offCtr = 0, offNorm = 0, offSweeps = 0, offOne = 0, offScr = 0;
  // SVD sweep with device-resident ranks: the compacted B_k (QR in place), the
  // padded V rows, R V, and a device int 1
  long offB = 0, offV = 0, offYt = 0, offOneI = 0;
  long total = 0;
  long maxr_bound = 0;
};

long round_up(long x, long a) { return (x + a - 1) / a * a; }

// svd = false plans the QR sweep only (orthogonalisation): no SVD-sweep
// buffers and none of their size limits.
// devranks = false: the batched kernel's per-problem plan (its sweep keeps
// ranks in workgroup registers and needs none of the device-rank buffers).
int make_plan(const Shape& s, long max_rank, Plan& P, bool svd = true, bool devranks = true) {
  const int n = s.n;
  P.m.assign(n, 0);
  P.rho.assign(n + 1, 1);
  P.offM.assign(n, 0);
  P.offT.assign(n, 0);
  long off = 0;
  auto take = [&](long cnt) {
    long o = off;
    off += round_up(std::max(cnt, 1L), 32);
    return o;
  };
  long maxR = 1, maxY = 1, maxQ = 1;
  for (int k = 0; k + 1 < n; ++k) {
    const long m = P.rho[k] * s.d[k];
    const long cols = s.rc[k + 1];
    if (m > kMaxRows) return QTT_ERR_UNSUPPORTED;
    P.m[k] = m;
    P.rho[k + 1] = std::min(m, cols);
    P.offM[k] = take(m * cols);
    P.offT[k] = take(qr_t_doubles((int)m, (int)cols));
    maxR = std::max(maxR, P.rho[k + 1] * cols);
    maxQ = std::max(maxQ, m * P.rho[k + 1]);  // explicit Q_k for qtt_orthogonalize
    if (s.kind != K_TT) {
      // Y = R X_k (rows rho_{k-1} * r_a, cols dj * r_b')
      const long dj = (s.kind == K_MPO) ? s.dj[k] : s.d[k];
      maxY = std::max(maxY, P.rho[k] * s.ra[k] * dj * s.rb[k + 1]);
    }
  }
  {
    const int k = n - 1;
    const long dj = (s.kind == K_MPO) ? s.dj[k] : s.d[k];
    if (s.kind != K_TT) maxY = std::max(maxY, P.rho[k] * s.ra[k] * dj * s.rb[k + 1]);
  }
  P.offCenter = take(P.rho[n - 1] * s.d[n - 1]);
  P.offR = take(maxR);
  P.offY = take(maxY);
  // SVD sweep bounds: r''_k <= min(rho_k, max_rank, d^(n-k) products)
  std::vector<long> rr(n + 1, 1);
  {
    long right = 1;
    for (int k = n - 1; k >= 1; --k) {
      right = std::min<long>(right * s.d[k], 1L << 40);
      long b = std::min(P.rho[k], right);
      if (max_rank > 0) b = std::min(b, max_rank);
      rr[k] = std::max(b, 1L);
    }
  }
  long maxZ = 1, maxX = 1, maxYn = 1, maxTB = 1, maxP = 1;
  for (int k = n - 1; svd && k >= 1; --k) {
    const long D = s.d[k] * rr[k + 1];
    const long rows = P.rho[k];  // rho_{k-1} in 1-based terms = rows of B
    // Q_k [Y; 0] lives in Z: m_k x r''_{k+1}  (for k = n-1 the centre is used)
    if (k < n - 1) maxZ = std::max(maxZ, P.m[k] * rr[k + 1]);
    maxZ = std::max(maxZ, rows * D);
    // D is a bound: the actual d r''_{k+1} can be smaller, which turns a
    // wide B tall (QR of rows x D', D' <= rows), so the QR factor is sized
    // for min(rows, D) whichever branch the bound takes.
    maxTB = std::max(maxTB, qr_t_doubles((int)rows, (int)std::min(rows, D)));
    if (rows >= D) {
      maxX = std::max(maxX, D * D);
      maxP = std::max(maxP, D);
    } else {
      maxX = std::max(maxX, rows * D);
      maxP = std::max(maxP, rows);
    }
    if (D > 1024) return QTT_ERR_UNSUPPORTED;  // Jacobi keeps 16 row slices of length D per lane group
    maxYn = std::max(maxYn, rows * rr[k]);
  }
  if (svd && n >= 2) maxZ = std::max(maxZ, P.m[0] * rr[1]);
  maxZ = std::max(maxZ, maxQ);
  P.offZ = take(maxZ);
  P.offX = take(maxX);
  P.offXc = take(maxX);
  P.offYn = take(maxYn);
  P.offTB = take(maxTB);
  P.offSig = take(maxP);
  P.offPerm = take(maxP / 2 + 1);
  // one rank decision and one Jacobi record (sweeps, converged) per bond
  P.offTrunc = take((long)std::max(n, 1) * (long)((sizeof(TruncOut) + 7) / 8));
  P.offCtr = take(96);  // Jacobi: 8 counter words + one version per 8-row block (p <= 1024)
  P.offNorm = take(1);
  P.offSweeps = take(std::max(n, 1));
  P.offOne = take(1);
  if (svd && devranks) {
    P.offB = take(maxZ);
    P.offV = take(maxX);
    P.offYt = take(maxX);
    P.offOneI = take(1);
  }
  {
    long maxc = 1;
    for (int k = 0; k <= n; ++k) maxc = std::max(maxc, s.rc[k]);
    for (int k = 0; svd && k < n; ++k) maxc = std::max(maxc, (long)s.d[k] * std::max(rr[k], rr[k + 1]));
    P.offScr = take(qr_scratch_doubles(maxc));
  }
  P.total = off;
  P.maxr_bound = 0;
  for (int k = 0; k <= n; ++k) P.maxr_bound = std::max(P.maxr_bound, rr[k]);
  P.rr = rr;
  return QTT_OK;
}

int shape_from_tt(const qtt_tt* t, Shape& s) {
  s.kind = K_TT;
  s.n = t->n;
  s.d.resize(t->n);
  s.rc.resize(t->n + 1);
  for (int k = 0; k < t->n; ++k) s.d[k] = dphys(t, k);
  for (int k = 0; k <= t->n; ++k) s.rc[k] = t->ranks[k];
  return QTT_OK;
}

int parse_spec(const char* spec, Kind& kind) {
  if (!spec) return QTT_ERR_ARG;
  std::string sp(spec);
  std::string t;
  for (char c : sp)
    if (c != ' ') t += c;
  if (t == "i,i->i") {
    kind = K_HAD;
    return QTT_OK;
  }
  if (t == "ij,j->i") {
    kind = K_MPO;
    return QTT_OK;
  }
  if (t == "ij,jk->ik") {
    kind = K_OPOP;
    return QTT_OK;
  }
  return QTT_ERR_SPEC;
}

int shape_from_pair(const char* spec, const qtt_tt* a, const qtt_tt* b, Shape& s) {
  Kind kind;
  int st = parse_spec(spec, kind);
  if (st) return st;
  // the operator product has its own entry (qtt_contract); the fused sweeps
  // take an MPS result
  if (kind == K_OPOP) return QTT_ERR_UNSUPPORTED;
  if ((st = check_tt(a, kind == K_MPO ? 2 : 1))) return st;
  if ((st = check_tt(b, 1))) return st;
  if (a->n != b->n) return QTT_ERR_SHAPE;
  const int n = a->n;
  s.kind = kind;
  s.n = n;
  s.d.resize(n);
  s.dj.resize(n);
  s.rc.resize(n + 1);
  s.ra.resize(n + 1);
  s.rb.resize(n + 1);
  for (int k = 0; k < n; ++k) {
    if (kind == K_HAD) {
      if (dphys(a, k) != dphys(b, k)) return QTT_ERR_SHAPE;
      s.d[k] = dphys(a, k);
      s.dj[k] = s.d[k];
    } else {
      if (dphys_in(a, k) != dphys(b, k)) return QTT_ERR_SHAPE;
      s.d[k] = dphys(a, k);
      s.dj[k] = dphys_in(a, k);
    }
  }
  for (int k = 0; k <= n; ++k) {
    s.ra[k] = a->ranks[k];
    s.rb[k] = b->ranks[k];
    s.rc[k] = a->ranks[k] * b->ranks[k];
  }
  return QTT_OK;
}

// Y = R * X (rows, K) x (K, cols) in the requested GEMM arithmetic.
hipError_t bond_gemm(hipStream_t st, int prec, int rows, int cols, int K, const double* R, long ldr,
                     const double* X, long ldx, double* Y, long ldy) {
  switch (prec) {
    case QTT_GEMM_FP32:
      return gemm_f64_via_f32(st, false, false, rows, cols, K, R, ldr, X, ldx, Y, ldy);
    case QTT_GEMM_BF16X3:
      return gemm_bf16split(st, false, false, rows, cols, K, R, ldr, X, ldx, Y, ldy, 3);
    case QTT_GEMM_BF16X6:
      return gemm_bf16split(st, false, false, rows, cols, K, R, ldr, X, ldx, Y, ldy, 6);
    default:
      return gemm_f64(st, false, false, rows, cols, K, 1.0, R, ldr, 0, X, ldx, 0, 0.0, Y, ldy, 0, 1);
  }
}

// C = op(A) op(B) (M x N, K deep) in the requested GEMM arithmetic (the
// reduced-precision forms take FP64 operands and write FP64 results).
hipError_t gemm_prec(hipStream_t st, int prec, bool ta, bool tb, int M, int N, int K, const double* A, long lda,
                     const double* B, long ldb, double* C, long ldc) {
  switch (prec) {
    case QTT_GEMM_FP32:
      return gemm_f64_via_f32(st, ta, tb, M, N, K, A, lda, B, ldb, C, ldc);
    case QTT_GEMM_BF16X3:
      return gemm_bf16split(st, ta, tb, M, N, K, A, lda, B, ldb, C, ldc, 3);
    case QTT_GEMM_BF16X6:
      return gemm_bf16split(st, ta, tb, M, N, K, A, lda, B, ldb, C, ldc, 6);
    default:
      return gemm_f64(st, ta, tb, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, ldc, 0, 1);
  }
}

struct Sweep {
  qtt_context* h;
  hipStream_t st;
  double* ws;
  const Shape* s;
  const Plan* P;
  int prec;
};

// QR sweep: M_k = R_{k-1} C_k factored in place; fills the centre core.
int qr_sweep(Sweep& w, const qtt_tt* t, const qtt_tt* a, const qtt_tt* b) {
  const Shape& s = *w.s;
  const Plan& P = *w.P;
  const int n = s.n;
  double* ws = w.ws;
  double* R = ws + P.offR;
  double* Yb = ws + P.offY;
  for (int k = 0; k < n; ++k) {
    const long rho0 = P.rho[k];
    const long cols = s.rc[k + 1];
    const bool last = (k == n - 1);
    double* M = last ? ws + P.offCenter : ws + P.offM[k];
    const long ldm = cols;
    if (s.kind == K_TT) {
      const double* Ck = (const double*)t->cores[k];
      if (k == 0) {
        QTT_HIP(copy_pad_rows(w.st, Ck, (int)(s.d[k]), (int)cols, cols, M, (int)(s.d[k]), ldm));
      } else {
        QTT_HIP(bond_gemm(w.st, w.prec, (int)rho0, (int)(s.d[k] * cols), (int)s.rc[k], R, s.rc[k], Ck,
                          s.d[k] * cols, M, s.d[k] * cols));
      }
    } else {
      // factored: Y[(a,mu),(j,nu')] = sum_nu R[(a,mu),nu] B[nu,(j,nu')]
      const double* Ak = (const double*)a->cores[k];
      const double* Bk = (const double*)b->cores[k];
      const long ra0 = s.ra[k], ra1 = s.ra[k + 1], rb0 = s.rb[k], rb1 = s.rb[k + 1];
      const long dj = s.dj[k];
      const double* Rk = R;
      if (k == 0) {
        // R_{-1} = [[1]]: Y = B_0 repeated over mu (ra0 == 1)
        QTT_HIP(fill_f64(w.st, ws + P.offOne, 1.0, 1));
        Rk = ws + P.offOne;
      }
      QTT_HIP(bond_gemm(w.st, w.prec, (int)(rho0 * ra0), (int)(dj * rb1), (int)rb0, Rk, rb0, Bk, dj * rb1, Yb,
                        dj * rb1));
      if (s.kind == K_MPO) {
        QTT_HIP(bond_mpo_apply(w.st, Yb, (int)rho0, (int)ra0, (int)dj, (int)rb1, Ak, s.d[k], (int)ra1, M));
      } else {
        QTT_HIP(bond_hadamard_apply(w.st, Yb, (int)rho0, (int)ra0, s.d[k], (int)rb1, Ak, (int)ra1, M));
      }
    }
    if (!last) {
      const long m = P.m[k];
      QTT_HIP(householder_qr(w.st, M, (int)m, (int)cols, ldm, ws + P.offT[k], ws + P.offScr));
      QTT_HIP(extract_r(w.st, M, (int)P.rho[k + 1], (int)cols, ldm, R));
    }
  }
  QTT_HIP(frob_norm(w.st, ws + P.offCenter, P.rho[n - 1] * s.d[n - 1], ws + P.offNorm));
  return QTT_OK;
}

int readback(qtt_context* h, hipStream_t st, const void* dev, size_t bytes, void* pinned) {
  QTT_HIP(hipMemcpyAsync(pinned, dev, bytes, hipMemcpyDeviceToHost, st));
  QTT_HIP(hipStreamSynchronize(st));
  return QTT_OK;
}

// SVD sweep from the right; writes the rounded cores into out.
//
// The ranks stay on the device: every launch is sized by the plan's rank
// bounds, and the rank r_{k+1} decided at the previous bond is read by the
// kernels that need it.  B_k = Q_k [U Sigma; 0] (whose columns beyond
// r_{k+1} are zero) is first compacted so that its zero columns trail; its
// Householder QR then has exactly zero rows beyond rank(B_k), which the
// Jacobi leaves untouched, so bonds whose rank falls below the bound cost
// only the bound's extra (zero) work.  Nothing is read back until the end,
// so the whole sweep is stream-ordered (sync = false: no host wait at all,
// and out's host ranks and info are not written; the record kernel leaves
// the ranks and a status in record_ranks / record_status).
int svd_sweep(Sweep& w, qtt_tt* out, double rel_tol, long max_rank, qtt_round_info* info, std::vector<long>& newr,
              bool sync = true, long long* record_ranks = nullptr, int* record_status = nullptr) {
  const Shape& s = *w.s;
  const Plan& P = *w.P;
  const int n = s.n;
  double* ws = w.ws;
  double* Z = ws + P.offZ;
  double* X = ws + P.offX;
  double* Xc = ws + P.offXc;
  double* Yn = ws + P.offYn;
  double* TB = ws + P.offTB;
  double* X0 = ws + P.offB;
  double* V = ws + P.offV;
  double* Yt = ws + P.offYt;
  double* sig = ws + P.offSig;
  int* perm = (int*)(ws + P.offPerm);
  TruncOut* trs = (TruncOut*)(ws + P.offTrunc);
  unsigned* ctr = (unsigned*)(ws + P.offCtr);
  int* sweeps = (int*)(ws + P.offSweeps);
  int* one_i = (int*)(ws + P.offOneI);
  newr.assign(n + 1, 1);
  QTT_HIP(fill_u32(w.st, (unsigned*)one_i, 1u, 1));
  const bool want_sig = sync && info && info->sigma && info->sigma_ld > 0;
  long rbnext = 1;              // launch bound of r_{k+1}
  const int* rnext_dev = one_i;  // r_{k+1} on the device
  for (int k = n - 1; k >= 1; --k) {
    const long rows = P.rho[k];
    const long D = s.d[k] * rbnext;
    if (k == n - 1) {
      QTT_HIP(copy_pad_rows(w.st, ws + P.offCenter, (int)rows, (int)D, D, X0, (int)rows, D));
    } else {
      // Z = Q_k [Y_{k+1}; 0]  (m_k x rb_{k+1}) = B_k as rows x D, then its kept columns to the front
      QTT_HIP(copy_pad_rows(w.st, Yn, (int)P.rho[k + 1], (int)rbnext, rbnext, Z, (int)P.m[k], rbnext));
      QTT_HIP(apply_q(w.st, ws + P.offM[k], (int)P.m[k], (int)P.rho[k + 1], s.rc[k + 1], ws + P.offT[k], Z,
                      (int)rbnext, rbnext, false, ws + P.offScr));
      QTT_HIP(compact_cols(w.st, Z, (int)rows, s.d[k], (int)rbnext, rnext_dev, X0));
    }
    // B = Q_B R; the Jacobi acts on the rows of F = R (p x D, p = min(rows, D)),
    // Xc keeps F for U Sigma = Q_B [F V; 0]
    const int p = (int)std::min(rows, D);
    const int L = (int)D;
    QTT_HIP(householder_qr(w.st, X0, (int)rows, (int)D, D, TB, ws + P.offScr));
    QTT_HIP(extract_r(w.st, X0, p, (int)D, D, Xc));
    // Jacobi from F's rows in descending-norm order (a row permutation changes
    // neither V nor F V)
    QTT_HIP(row_norms_sorted(w.st, Xc, p, L, sig, perm));
    QTT_HIP(permute_rows(w.st, Xc, p, L, perm, X));
    QTT_HIP(jacobi_rows(w.st, X, p, L, ctr, w.h->max_sweeps, sweeps + 2 * (k - 1), sig));  // sig[0]: largest norm
    QTT_HIP(row_norms_sorted(w.st, X, p, L, sig, perm));
    TruncOut* tr = trs + (k - 1);
    QTT_HIP(truncate_decide(w.st, sig, p, ws + P.offNorm, rel_tol, n - 1, max_rank, tr));
    if (want_sig) {
      const long cnt = std::min<long>(p, info->sigma_ld);
      QTT_HIP(hipMemcpyAsync(info->sigma + (long)(k - 1) * info->sigma_ld, sig, cnt * sizeof(double),
                             hipMemcpyDeviceToHost, w.st));
      QTT_HIP(hipStreamSynchronize(w.st));
      for (long i = cnt; i < info->sigma_ld; ++i) info->sigma[(long)(k - 1) * info->sigma_ld + i] = 0.0;
    }
    // V: the r kept right singular vectors (rows), zero rows up to the bound
    const int rb = (int)std::max(1L, std::min<long>(p, P.rr[k]));
    QTT_HIP(gather_rows_padded(w.st, X, L, perm, sig, tr, V, rb));
    // core k <- V_r^T  ([r_k, d_k, r_{k+1}], compact)
    QTT_HIP(core_from_rows(w.st, V, rb, L, &tr->rank, s.d[k], rnext_dev, (double*)out->cores[k]));
    // Y_k = U Sigma = B V_r = Q_B [F V_r; 0]  (rows x rb; columns beyond r_k are zero)
    QTT_HIP(gemm_prec(w.st, w.prec, false, true, p, rb, L, Xc, L, V, L, Yt, rb));
    QTT_HIP(copy_pad_rows(w.st, Yt, p, rb, rb, Yn, (int)rows, rb));
    QTT_HIP(apply_q(w.st, X0, (int)rows, p, D, TB, Yn, rb, rb, false, ws + P.offScr));
    rbnext = rb;
    rnext_dev = &tr->rank;
  }
  // core 0 = Q_0 [Y_1; 0], its first r_1 columns per physical index
  if (n == 1) {
    QTT_HIP(copy_pad_rows(w.st, ws + P.offCenter, 1, s.d[0], s.d[0], (double*)out->cores[0], 1, s.d[0]));
  } else {
    QTT_HIP(copy_pad_rows(w.st, Yn, (int)P.rho[1], (int)rbnext, rbnext, Z, (int)P.m[0], rbnext));
    QTT_HIP(apply_q(w.st, ws + P.offM[0], (int)P.m[0], (int)P.rho[1], s.rc[1], ws + P.offT[0], Z, (int)rbnext,
                    rbnext, false, ws + P.offScr));
    QTT_HIP(compact_cols(w.st, Z, 1, s.d[0], (int)rbnext, rnext_dev, (double*)out->cores[0]));
  }
  if (record_ranks || record_status) {
    if (!record_ranks || !record_status) return QTT_ERR_ARG;
    QTT_HIP(round_record(w.st, trs, sweeps, n, ws + P.offNorm, record_ranks, record_status, QTT_ERR_NONFINITE,
                         QTT_ERR_NOCONV));
  }
  if (!sync) return QTT_OK;
  // the only host wait of the sweep: decisions and Jacobi records of all bonds
  std::vector<TruncOut> ht(std::max(n - 1, 1));
  std::vector<int> hs(2 * std::max(n - 1, 1));
  double norm = 0.0;
  QTT_HIP(hipMemcpyAsync(&norm, ws + P.offNorm, sizeof(double), hipMemcpyDeviceToHost, w.st));
  if (n > 1) {
    QTT_HIP(hipMemcpyAsync(ht.data(), trs, (size_t)(n - 1) * sizeof(TruncOut), hipMemcpyDeviceToHost, w.st));
    QTT_HIP(hipMemcpyAsync(hs.data(), sweeps, (size_t)(n - 1) * 2 * sizeof(int), hipMemcpyDeviceToHost, w.st));
  }
  QTT_HIP(hipStreamSynchronize(w.st));
  if (!std::isfinite(norm)) return QTT_ERR_NONFINITE;
  double err2 = 0.0;
  int maxsw = 0;
  for (int k = 1; k < n; ++k) {
    const TruncOut& t = ht[k - 1];
    if (!hs[2 * (k - 1) + 1]) return QTT_ERR_NOCONV;
    maxsw = std::max(maxsw, hs[2 * (k - 1)]);
    newr[k] = t.rank;
    err2 += t.tail_r * t.tail_r;
    if (info) {
      if (info->tail) info->tail[k - 1] = t.tail_r;
      if (info->margin_lo) info->margin_lo[k - 1] = t.delta > 0 ? t.tail_rm1 / t.delta : INFINITY;
      if (info->margin_hi) info->margin_hi[k - 1] = t.delta > 0 ? t.tail_r / t.delta : 0.0;
      if (info->maxrank_hit) info->maxrank_hit[k - 1] = (uint8_t)t.capped;
    }
  }
  if (info) {
    info->norm = norm;
    info->delta = (n > 1) ? rel_tol * norm / std::sqrt((double)(n - 1)) : 0.0;
    info->err_bound = std::sqrt(err2);
    info->jacobi_sweeps_max = maxsw;
  }
  return QTT_OK;
}

size_t ws_bytes_of(const Plan& P) { return (size_t)P.total * sizeof(double) + 256; }

double* align_ws(void* ws) {
  uintptr_t p = (uintptr_t)ws;
  p = (p + 255) & ~(uintptr_t)255;
  return (double*)p;
}

// ---------------------------------------------------------------- inner products
struct InnerPlan {
  long offE0, offE1, offT, total;
};
InnerPlan inner_plan(const qtt_tt* a, const qtt_tt* b) {
  long maxE = 1, maxT = 1;
  for (int k = 0; k < a->n; ++k) {
    maxE = std::max(maxE, a->ranks[k + 1] * b->ranks[k + 1]);
    maxE = std::max(maxE, a->ranks[k] * b->ranks[k]);
    maxT = std::max(maxT, a->ranks[k] * (long)dphys(a, k) * b->ranks[k + 1]);
  }
  InnerPlan p;
  p.offE0 = 0;
  p.offE1 = round_up(maxE, 32);
  p.offT = p.offE1 + round_up(maxE, 32);
  p.total = p.offT + round_up(maxT, 32);
  return p;
}

struct EnvPlan {
  std::vector<long> offE, offF;
  long offT, offT2, total;
};
EnvPlan env_plan(const qtt_tt* a, const qtt_tt* b) {
  EnvPlan p;
  const int n = a->n;
  p.offE.resize(n + 1);
  p.offF.resize(n + 1);
  long off = 0, maxT = 1;
  for (int k = 0; k <= n; ++k) {
    p.offE[k] = off;
    off += round_up(a->ranks[k] * b->ranks[k], 32);
    p.offF[k] = off;
    off += round_up(a->ranks[k] * b->ranks[k], 32);
  }
  for (int k = 0; k < n; ++k) {
    const long d = dphys(a, k);
    maxT = std::max(maxT, a->ranks[k] * d * b->ranks[k + 1]);
    maxT = std::max(maxT, b->ranks[k] * d * a->ranks[k + 1]);
  }
  p.offT = off;
  off += round_up(maxT, 32);
  p.offT2 = off;
  off += round_up(maxT, 32);
  p.total = off;
  return p;
}

template <typename T>
hipError_t gemmT(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const T* A, long lda,
                 const T* B, long ldb, double beta, T* C, long ldc);
template <>
hipError_t gemmT<double>(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
                         long lda, const double* B, long ldb, double beta, double* C, long ldc) {
  return gemm_f64(s, ta, tb, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
}
template <>
hipError_t gemmT<float>(hipStream_t s, bool ta, bool tb, int M, int N, int K, double alpha, const float* A,
                        long lda, const float* B, long ldb, double beta, float* C, long ldc) {
  return gemm_f32(s, ta, tb, M, N, K, (float)alpha, A, lda, 0, B, ldb, 0, (float)beta, C, ldc, 0, 1);
}

template <typename T>
hipError_t fill_T(hipStream_t s, T* p, double v, long n);
template <>
hipError_t fill_T<double>(hipStream_t s, double* p, double v, long n) {
  return fill_f64(s, p, v, n);
}
template <>
hipError_t fill_T<float>(hipStream_t s, float* p, double v, long n) {
  return fill_f32(s, p, (float)v, n);
}

// E_{k+1} = sum_i a_k(i)^T E_k b_k(i)
template <typename T>
hipError_t env_step_left(hipStream_t st, const T* E, const T* ak, const T* bk, long ra0, long ra1, long rb0, long rb1,
                         long d, T* Tt, T* Enext) {
  hipError_t e = gemmT<T>(st, false, false, (int)ra0, (int)(d * rb1), (int)rb0, 1.0, E, rb0, bk, d * rb1, 0.0, Tt,
                          d * rb1);
  if (e != hipSuccess) return e;
  return gemmT<T>(st, true, false, (int)ra1, (int)rb1, (int)(ra0 * d), 1.0, ak, ra1, Tt, rb1, 0.0, Enext, rb1);
}
// F_k = sum_i a_k(i) F_{k+1} b_k(i)^T
template <typename T>
hipError_t env_step_right(hipStream_t st, const T* F, const T* ak, const T* bk, long ra0, long ra1, long rb0,
                          long rb1, long d, T* Tt, T* Fprev) {
  hipError_t e = gemmT<T>(st, false, false, (int)(ra0 * d), (int)rb1, (int)ra1, 1.0, ak, ra1, F, rb1, 0.0, Tt, rb1);
  if (e != hipSuccess) return e;
  return gemmT<T>(st, false, true, (int)ra0, (int)rb0, (int)(d * rb1), 1.0, Tt, d * rb1, bk, d * rb1, 0.0, Fprev,
                  rb0);
}

// The same step with the two GEMMs in the requested arithmetic (FP64 cores).
hipError_t env_step_left_prec(hipStream_t st, int prec, const double* E, const double* ak, const double* bk, long ra0,
                              long ra1, long rb0, long rb1, long d, double* Tt, double* Enext) {
  if (prec == QTT_GEMM_FP64) return env_step_left<double>(st, E, ak, bk, ra0, ra1, rb0, rb1, d, Tt, Enext);
  hipError_t e = gemm_prec(st, prec, false, false, (int)ra0, (int)(d * rb1), (int)rb0, E, rb0, bk, d * rb1, Tt,
                           d * rb1);
  if (e != hipSuccess) return e;
  return gemm_prec(st, prec, true, false, (int)ra1, (int)rb1, (int)(ra0 * d), ak, ra1, Tt, rb1, Enext, rb1);
}

template <typename T>
int inner_impl(qtt_context* h, const qtt_tt* a, const qtt_tt* b, double* out, void* ws_raw, hipStream_t st,
               int prec = QTT_GEMM_FP64) {
  InnerPlan p = inner_plan(a, b);
  T* ws = (T*)align_ws(ws_raw);
  T* E = ws + p.offE0;
  T* E2 = ws + p.offE1;
  T* Tt = ws + p.offT;
  QTT_HIP(fill_T<T>(st, E, 1.0, 1));
  for (int k = 0; k < a->n; ++k) {
    if constexpr (std::is_same<T, double>::value) {
      QTT_HIP(env_step_left_prec(st, prec, E, (const T*)a->cores[k], (const T*)b->cores[k], a->ranks[k],
                                 a->ranks[k + 1], b->ranks[k], b->ranks[k + 1], dphys(a, k), Tt, E2));
    } else {
      QTT_HIP(env_step_left<T>(st, E, (const T*)a->cores[k], (const T*)b->cores[k], a->ranks[k], a->ranks[k + 1],
                               b->ranks[k], b->ranks[k + 1], dphys(a, k), Tt, E2));
    }
    std::swap(E, E2);
  }
  T hv;
  QTT_HIP(hipMemcpyAsync(&hv, E, sizeof(T), hipMemcpyDeviceToHost, st));
  QTT_HIP(hipStreamSynchronize(st));
  *out = (double)hv;
  return QTT_OK;
}

template <typename T>
int inner_backward_impl(const qtt_tt* a, const qtt_tt* b, double g, qtt_tt* da, qtt_tt* db, void* ws_raw,
                        hipStream_t st) {
  EnvPlan p = env_plan(a, b);
  T* ws = (T*)align_ws(ws_raw);
  const int n = a->n;
  QTT_HIP(fill_T<T>(st, ws + p.offE[0], 1.0, 1));
  QTT_HIP(fill_T<T>(st, ws + p.offF[n], 1.0, 1));
  for (int k = 0; k < n; ++k)
    QTT_HIP(env_step_left<T>(st, ws + p.offE[k], (const T*)a->cores[k], (const T*)b->cores[k], a->ranks[k],
                             a->ranks[k + 1], b->ranks[k], b->ranks[k + 1], dphys(a, k), ws + p.offT,
                             ws + p.offE[k + 1]));
  for (int k = n - 1; k >= 0; --k)
    QTT_HIP(env_step_right<T>(st, ws + p.offF[k + 1], (const T*)a->cores[k], (const T*)b->cores[k], a->ranks[k],
                              a->ranks[k + 1], b->ranks[k], b->ranks[k + 1], dphys(a, k), ws + p.offT,
                              ws + p.offF[k]));
  for (int k = 0; k < n; ++k) {
    const long ra0 = a->ranks[k], ra1 = a->ranks[k + 1], rb0 = b->ranks[k], rb1 = b->ranks[k + 1], d = dphys(a, k);
    if (da) {
      // T = E_k b_k  (ra0 x d rb1);  da = g T F_{k+1}^T  ((ra0 d) x ra1)
      QTT_HIP(gemmT<T>(st, false, false, (int)ra0, (int)(d * rb1), (int)rb0, 1.0, ws + p.offE[k], rb0,
                       (const T*)b->cores[k], d * rb1, 0.0, ws + p.offT, d * rb1));
      QTT_HIP(gemmT<T>(st, false, true, (int)(ra0 * d), (int)ra1, (int)rb1, g, ws + p.offT, rb1, ws + p.offF[k + 1],
                       rb1, 0.0, (T*)da->cores[k], ra1));
    }
    if (db) {
      // T = E_k^T a_k  (rb0 x d ra1);  db = g T F_{k+1}  ((rb0 d) x rb1)
      QTT_HIP(gemmT<T>(st, true, false, (int)rb0, (int)(d * ra1), (int)ra0, 1.0, ws + p.offE[k], rb0,
                       (const T*)a->cores[k], d * ra1, 0.0, ws + p.offT, d * ra1));
      QTT_HIP(gemmT<T>(st, false, false, (int)(rb0 * d), (int)rb1, (int)ra1, g, ws + p.offT, ra1, ws + p.offF[k + 1],
                       rb1, 0.0, (T*)db->cores[k], rb1));
    }
  }
  return QTT_OK;
}

int same_layout(const qtt_tt* a, const qtt_tt* b) {
  if (a->n != b->n || a->dtype != b->dtype) return QTT_ERR_SHAPE;
  for (int k = 0; k < a->n; ++k)
    if (dphys(a, k) != dphys(b, k)) return QTT_ERR_SHAPE;
  return QTT_OK;
}

// ---------------------------------------------------------------- batched form
struct BatchLayout {
  long offTab, offOrder, offQueue, offRanks, offTails, offStatus, offInst;
  std::vector<long> instOff;  // per-instance workspace offset (bytes from the aligned base)
  std::vector<Plan> plans;
  std::vector<Shape> shapes;
  long total;  // bytes
  int maxL;
};

long align256(long b) { return (b + 255) / 256 * 256; }

int batch_layout(const char* spec, int count, const qtt_tt* a, const qtt_tt* b, long max_rank, BatchLayout& Lo) {
  if (count < 1 || !a || !b) return QTT_ERR_ARG;
  Lo.shapes.resize(count);
  Lo.plans.resize(count);
  Lo.instOff.resize(count);
  long off = 0;
  Lo.offTab = off;
  off = align256(off + (long)count * sizeof(BInst));
  Lo.offOrder = off;
  off = align256(off + (long)count * sizeof(int));
  Lo.offQueue = off;
  off = align256(off + 16);
  Lo.offRanks = off;
  off = align256(off + (long)count * (QTT_BATCH_MAXN + 1) * sizeof(long));
  Lo.offTails = off;
  off = align256(off + (long)count * QTT_BATCH_MAXN * sizeof(double));
  Lo.offStatus = off;
  off = align256(off + (long)count * sizeof(int));
  Lo.offInst = off;
  Lo.maxL = 1;
  for (int i = 0; i < count; ++i) {
    int st = shape_from_pair(spec, &a[i], &b[i], Lo.shapes[i]);
    if (st) return st;
    if (a[i].dtype != QTT_F64 || b[i].dtype != QTT_F64) return QTT_ERR_DTYPE;
    const Shape& sh = Lo.shapes[i];
    if (sh.n > QTT_BATCH_MAXN) return QTT_ERR_UNSUPPORTED;
    if ((st = make_plan(sh, max_rank, Lo.plans[i], true, false))) return st;
    const Plan& P = Lo.plans[i];
    for (int k = 0; k + 1 < sh.n; ++k)
      if (P.m[k] > 512) return QTT_ERR_UNSUPPORTED;  // register panel of the workgroup QR
    long rnext = 1;
    for (int k = sh.n - 1; k >= 1; --k) {
      long bnd = std::min<long>(P.rho[k], max_rank > 0 ? max_rank : P.rho[k]);
      const long D = (long)sh.d[k] * std::min<long>(rnext, 1L << 20);
      if (P.rho[k] > 512) return QTT_ERR_UNSUPPORTED;
      Lo.maxL = (int)std::max<long>(Lo.maxL, D);
      rnext = std::max<long>(1, std::min(bnd, D));
    }
    Lo.instOff[i] = off;
    off = align256(off + P.total * (long)sizeof(double));
  }
  if (16L * Lo.maxL * 8 > 96 * 1024) return QTT_ERR_UNSUPPORTED;  // Jacobi staging in LDS
  Lo.total = off + 256;
  return QTT_OK;
}

std::string tune_path() {
  const char* e = std::getenv("QTT_TUNE_CACHE");
  if (e && *e) return std::string(e);
  const char* home = std::getenv("HOME");
  std::string dir = std::string(home ? home : "/tmp") + "/.cache";
  mkdir(dir.c_str(), 0755);
  dir += "/qtt";
  mkdir(dir.c_str(), 0755);
  return dir + "/batched_tune.txt";
}

// Tuning cache: one line per workload signature, "signature variant".
int tune_lookup(const std::string& sig) {
  std::ifstream f(tune_path());
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    int v;
    if ((is >> k >> v) && k == sig) return v;
  }
  return -1;
}

void tune_store(const std::string& sig, int v) {
  std::ofstream f(tune_path(), std::ios::app);
  if (f) f << sig << " " << v << "\n";
}

}  // namespace

struct qtt_batch {
  qtt_context* h = nullptr;
  int count = 0;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BInst* dtab = nullptr;
  int* dorder = nullptr;
  unsigned* dqueue = nullptr;
  long* dranks = nullptr;
  double* dtails = nullptr;
  int* dstatus = nullptr;
  long* hranks = nullptr;
  double* htails = nullptr;
  int* hstatus = nullptr;
  std::vector<int> ncores;
  int variant = 0, grid = 0, maxL = 1;
  double tol = 0.0;
  long max_rank = 0;
  int max_sweeps = 0;
  float tuned_ms[4] = {0, 0, 0, 0};
  TileMap tiles{};                                  // GEMM tile variant per shape bucket
  int tile_shape[kGemmBuckets][3] = {};             // representative (M, N, K) of each bucket (0: unused)
  float tile_ms[kGemmBuckets][kTileVariants] = {};  // probe time per variant (0: not measured)
};

namespace {

void batch_free(qtt_batch* p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->hranks) (void)hipHostFree(p->hranks);
  if (p->htails) (void)hipHostFree(p->htails);
  if (p->hstatus) (void)hipHostFree(p->hstatus);
  delete p;
}

hipError_t batch_run(qtt_batch* p, hipStream_t s, int variant) {
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->h->device);
  const int grid = std::min(p->count, cus * ((variant & 2) ? 2 : 1));
  p->grid = grid;
  return batched_launch(s, variant, grid, p->dtab, p->dorder, p->count, p->dqueue, p->tiles, p->tol, p->max_rank,
                        p->max_sweeps, p->dranks, p->dtails, p->dstatus, p->maxL);
}

// Tile variant used for a bucket when none was measured: 64 rows / columns
// when the bucket's M / N exceed 32.
int default_tile(int bucket) {
  const bool bm = bucket & 1, bn = bucket & 2;
  return bm ? (bn ? 0 : 1) : (bn ? 2 : 3);
}

// The GEMM shapes the batched kernel will run, bucketed; per bucket the
// shape with the most work (M N K times its call count) represents it.
void batch_gemm_shapes(const BatchLayout& Lo, long max_rank, int (&rep)[kGemmBuckets][3]) {
  double best[kGemmBuckets] = {};
  auto add = [&](long M, long N, long K, long calls) {
    if (M <= 0 || N <= 0 || K <= 0) return;
    const int b = gemm_bucket((int)M, (int)N, (int)K);
    const double wgt = (double)M * N * K * calls;
    if (wgt > best[b]) {
      best[b] = wgt;
      rep[b][0] = (int)M;
      rep[b][1] = (int)N;
      rep[b][2] = (int)K;
    }
  };
  for (size_t i = 0; i < Lo.shapes.size(); ++i) {
    const Shape& sh = Lo.shapes[i];
    const Plan& P = Lo.plans[i];
    const bool mpo = sh.kind == K_MPO;
    for (int k = 0; k < sh.n; ++k) {
      add(P.rho[k] * sh.ra[k], (long)sh.dj[k] * sh.rb[k + 1], sh.rb[k], 1);
      add(P.rho[k], sh.ra[k + 1], sh.ra[k] * (mpo ? sh.dj[k] : 1), (long)sh.d[k] * sh.rb[k + 1]);
    }
    long rnext = 1;
    for (int k = sh.n - 1; k >= 1; --k) {
      const long rows = P.rho[k], D = (long)sh.d[k] * rnext;
      const long p = rows >= D ? D : rows;
      long r = std::min(p, rows);
      if (max_rank > 0) r = std::min<long>(r, max_rank);
      add(p, r, D, 1);
      rnext = std::max<long>(1, r);
    }
  }
}

// Tuner of the GEMM tiles: every tile variant runs the bucket's representative
// shape on `grid` workgroups side by side (median of three launches); the
// fastest wins.  Results are cached per (bucket shape, grid) in the tuning file.
int tune_tiles(qtt_batch* p, const BatchLayout& Lo, long max_rank, bool tune, char* base, hipStream_t us, int grid) {
  batch_gemm_shapes(Lo, max_rank, p->tile_shape);
  for (int b = 0; b < kGemmBuckets; ++b) p->tiles.v[b] = (unsigned char)default_tile(b);
  if (!tune) return QTT_OK;
  // probe operands in the largest instance's workspace (overwritten by every run)
  size_t big = 0;
  for (size_t i = 1; i < Lo.plans.size(); ++i)
    if (Lo.plans[i].total > Lo.plans[big].total) big = i;
  double* scr = (double*)(base + Lo.instOff[big]);
  const long cap = Lo.plans[big].total;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return QTT_ERR_HIP;
  int rc = QTT_OK;
  for (int b = 0; b < kGemmBuckets && rc == QTT_OK; ++b) {
    const int M = p->tile_shape[b][0], N = p->tile_shape[b][1], K = p->tile_shape[b][2];
    if (M <= 0) continue;
    const long need = (long)M * K + (long)K * N + (long)M * N;
    if (need > cap) continue;
    std::ostringstream sig;
    sig << "tile|" << b << "|" << M << "x" << N << "x" << K << "|" << grid;
    const int cached = tune_lookup(sig.str());
    if (cached >= 0 && cached < kTileVariants) {
      p->tiles.v[b] = (unsigned char)cached;
      continue;
    }
    double *A = scr, *B = scr + (long)M * K, *C = B + (long)K * N;
    if (fill_f64(us, scr, 0.5, need) != hipSuccess) {
      rc = QTT_ERR_HIP;
      break;
    }
    float bestms = 1e30f;
    int bestv = default_tile(b);
    for (int v = 0; v < kTileVariants; ++v) {
      float t[3];
      for (int rep = 0; rep < 3; ++rep) {
        if (hipEventRecord(e0, us) != hipSuccess || tile_probe_launch(us, v, grid, M, N, K, A, B, C) != hipSuccess ||
            hipEventRecord(e1, us) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = QTT_ERR_HIP;
          break;
        }
        (void)hipEventElapsedTime(&t[rep], e0, e1);
      }
      if (rc != QTT_OK) break;
      std::sort(t, t + 3);
      p->tile_ms[b][v] = t[1];
      if (t[1] < bestms) {
        bestms = t[1];
        bestv = v;
      }
    }
    if (rc != QTT_OK) break;
    p->tiles.v[b] = (unsigned char)bestv;
    tune_store(sig.str(), bestv);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

namespace {

// ---------------------------------------------------------------- decomposition (zip-up)
// Sec. 3.2: both operands move their normalisation centre to the left end;
// a super-core of N exact product cores then grows one product core at a
// time and is split off one truncated-SVD core whenever it holds N cores.
struct ZipPlan {
  int N = 1;
  std::vector<long> ra, rb;       // operand ranks after the right-to-left sweep
  std::vector<long> Pa, Pb;       // physical size per core (all legs)
  std::vector<long> offA, offB;   // operand copies
  std::vector<long> bound;        // result rank bounds (n+1)
  long offG = 0, offTq = 0, offQe = 0, offRr = 0, offTmp = 0;
  long offS = 0, offT = 0, offY = 0, offBt = 0, offTB = 0, offX = 0, offXc = 0, offYn = 0, offV = 0;
  long offSig = 0, offPerm = 0, offTrunc = 0, offCtr = 0, offSweeps = 0, offOne = 0, offNrm = 0, offScr = 0;
  long total = 0;
};

int make_zip_plan(const Shape& s, const qtt_tt* a, const qtt_tt* b, long max_rank, int ncores, ZipPlan& Z) {
  if (ncores < 1 || ncores > 2) return QTT_ERR_UNSUPPORTED;
  const int n = s.n;
  Z.N = std::min(ncores, n);
  Z.Pa.assign(n, 1);
  Z.Pb.assign(n, 1);
  for (int k = 0; k < n; ++k) {
    for (int l = 0; l < a->legs; ++l) Z.Pa[k] *= a->phys[k * a->legs + l];
    Z.Pb[k] = b->phys[k];
  }
  long off = 0;
  auto take = [&](long cnt) {
    long o = off;
    off += round_up(std::max(cnt, 1L), 32);
    return o;
  };
  // right-to-left sweep ranks and its scratch
  long maxG = 1, maxTq = 1, maxQe = 1, maxRr = 1, maxTmp = 1, maxScrCols = 1;
  auto right_ranks = [&](const std::vector<long>& r, const std::vector<long>& P, std::vector<long>& rho) {
    rho.assign(n + 1, 1);
    for (int k = n - 1; k >= 1; --k) {
      const long m = P[k] * rho[k + 1], c = r[k];
      if (m > kMaxRows) return QTT_ERR_UNSUPPORTED;
      rho[k] = std::min(m, c);
      maxG = std::max(maxG, m * c);
      maxTq = std::max(maxTq, qr_t_doubles((int)m, (int)c));
      maxQe = std::max(maxQe, m * rho[k]);
      maxRr = std::max(maxRr, rho[k] * c);
      maxTmp = std::max(maxTmp, r[k - 1] * P[k - 1] * rho[k]);
      maxScrCols = std::max(maxScrCols, c);
    }
    return QTT_OK;
  };
  int st;
  if ((st = right_ranks(s.ra, Z.Pa, Z.ra))) return st;
  if ((st = right_ranks(s.rb, Z.Pb, Z.rb))) return st;
  Z.offA.assign(n, 0);
  Z.offB.assign(n, 0);
  for (int k = 0; k < n; ++k) {
    Z.offA[k] = take(s.ra[k] * Z.Pa[k] * s.ra[k + 1]);
    Z.offB[k] = take(s.rb[k] * Z.Pb[k] * s.rb[k + 1]);
  }
  // zip-up sizes, simulated with the rank bounds
  Z.bound.assign(n + 1, 1);
  long maxS = 1, maxY = 1, maxBt = 1, maxTB = 1, maxX = 1, maxYn = 1, maxV = 1, maxP = 1;
  long r = 1, Pleg = 1, rcS = 1;
  int legs = 0, outc = 0;
  for (int k = 0; k < n; ++k) {
    const long rho0 = r * Pleg;
    const long dj = (s.kind == K_MPO) ? s.dj[k] : s.d[k];
    const long rc1 = Z.ra[k + 1] * Z.rb[k + 1];
    maxY = std::max(maxY, rho0 * Z.ra[k] * dj * Z.rb[k + 1]);
    maxS = std::max(maxS, rho0 * s.d[k] * rc1);
    Pleg *= s.d[k];
    rcS = rc1;
    ++legs;
    while ((legs == Z.N && k < n - 1) || (k == n - 1 && legs > 1)) {
      const long db = s.d[outc];
      const long m = r * db, cols = (Pleg / db) * rcS;
      if (m > 1024) return QTT_ERR_UNSUPPORTED;  // Jacobi row length
      // r is a bound: with a smaller kept rank the split can take the tall
      // branch (QR of the cols x m' transpose, m' <= min(m, cols)) even where
      // the bound takes the wide one, so both branches are sized.
      if (cols > kMaxRows) return QTT_ERR_UNSUPPORTED;
      const long mt = std::min(m, cols);
      maxBt = std::max(maxBt, cols * mt);
      maxTB = std::max(maxTB, qr_t_doubles((int)cols, (int)mt));
      maxX = std::max(maxX, mt * mt);
      if (cols < m) maxX = std::max(maxX, cols * m);
      const long p = mt;
      long rn = p;
      if (max_rank > 0) rn = std::min(rn, max_rank);
      maxYn = std::max(maxYn, cols * rn);
      maxV = std::max(maxV, rn * m);
      maxP = std::max(maxP, p);
      maxScrCols = std::max(maxScrCols, m);
      Z.bound[++outc] = rn;
      r = rn;
      Pleg /= db;
      --legs;
    }
  }
  Z.offG = take(maxG);
  Z.offTq = take(maxTq);
  Z.offQe = take(maxQe);
  Z.offRr = take(maxRr);
  Z.offTmp = take(maxTmp);
  Z.offS = take(maxS);
  Z.offT = take(maxS);
  Z.offY = take(maxY);
  Z.offBt = take(maxBt);
  Z.offTB = take(maxTB);
  Z.offX = take(maxX);
  Z.offXc = take(maxX);
  Z.offYn = take(maxYn);
  Z.offV = take(maxV);
  Z.offSig = take(maxP);
  Z.offPerm = take(maxP / 2 + 1);
  Z.offTrunc = take(8);
  Z.offCtr = take(96);
  Z.offSweeps = take(1);
  Z.offOne = take(1);
  Z.offNrm = take(1);
  Z.offScr = take(qr_scratch_doubles(maxScrCols));
  Z.total = off;
  return QTT_OK;
}

// Right-to-left QR sweep on an operand copy held in the workspace: core k
// (r_k x P_k r'_{k+1}) is replaced by Q^T from G^T = Q R and R^T moves into
// core k-1.  r holds the original ranks, rho the ranks after the sweep.
int right_sweep(hipStream_t st, double* ws, const ZipPlan& Z, const std::vector<long>& off,
                const std::vector<long>& r, const std::vector<long>& P, const std::vector<long>& rho, int n) {
  double* G = ws + Z.offG;
  double* Tq = ws + Z.offTq;
  double* Qe = ws + Z.offQe;
  double* Rr = ws + Z.offRr;
  double* Tmp = ws + Z.offTmp;
  double* scr = ws + Z.offScr;
  for (int k = n - 1; k >= 1; --k) {
    const int m = (int)(P[k] * rho[k + 1]), c = (int)r[k], q = (int)rho[k];
    double* core = ws + off[k];
    QTT_HIP(transpose(st, core, c, m, m, G, c));  // G^T: m x c
    QTT_HIP(householder_qr(st, G, m, c, c, Tq, scr));
    QTT_HIP(extract_r(st, G, q, c, c, Rr));  // q x c
    QTT_HIP(set_eye_rect(st, Qe, m, q));
    QTT_HIP(apply_q(st, G, m, q, c, Tq, Qe, q, q, false, scr));
    QTT_HIP(transpose(st, Qe, m, q, q, core, m));  // core k = Q^T: q x m
    // core k-1 <- core k-1 R^T: (r_{k-1} P_{k-1}) x q
    double* prev = ws + off[k - 1];
    const int rows = (int)(r[k - 1] * P[k - 1]);
    QTT_HIP(gemm_f64(st, false, true, rows, q, c, 1.0, prev, c, 0, Rr, c, 0, 0.0, Tmp, q, 0, 1));
    QTT_HIP(copy_pad_rows(st, Tmp, rows, q, q, prev, rows, q));
  }
  return QTT_OK;
}

// The zip-up proper on right-normalised operand copies; result cores go to out.
int zip_sweep(qtt_context* h, hipStream_t st, double* ws, const Shape& s, const ZipPlan& Z, int prec, double rel_tol,
              long max_rank, qtt_tt* out, qtt_round_info* info, std::vector<long>& newr) {
  const int n = s.n;
  double* S = ws + Z.offS;
  double* T = ws + Z.offT;
  double* Yb = ws + Z.offY;
  double* Bt = ws + Z.offBt;
  double* TB = ws + Z.offTB;
  double* X = ws + Z.offX;
  double* Xc = ws + Z.offXc;
  double* Yn = ws + Z.offYn;
  double* V = ws + Z.offV;
  double* sig = ws + Z.offSig;
  int* perm = (int*)(ws + Z.offPerm);
  TruncOut* tr = (TruncOut*)(ws + Z.offTrunc);
  unsigned* ctr = (unsigned*)(ws + Z.offCtr);
  int* sweeps = (int*)(ws + Z.offSweeps);
  double* nrm = ws + Z.offNrm;
  double* scr = ws + Z.offScr;
  newr.assign(n + 1, 1);
  QTT_HIP(fill_f64(st, S, 1.0, 1));
  long r = 1, Pleg = 1, rcS = 1;
  int legs = 0, outc = 0;
  double err2 = 0.0, first_norm = 0.0, first_delta = 0.0;
  int maxsw = 0;
  for (int k = 0; k < n; ++k) {
    // T = S C_k from the operand cores: (S X_k) then the operator / Hadamard factor
    const long rho0 = r * Pleg;
    const long ra0 = Z.ra[k], ra1 = Z.ra[k + 1], rb0 = Z.rb[k], rb1 = Z.rb[k + 1];
    const long dj = (s.kind == K_MPO) ? s.dj[k] : s.d[k];
    const double* Ak = ws + Z.offA[k];
    const double* Bk = ws + Z.offB[k];
    QTT_HIP(bond_gemm(st, prec, (int)(rho0 * ra0), (int)(dj * rb1), (int)rb0, S, rb0, Bk, dj * rb1, Yb, dj * rb1));
    if (s.kind == K_MPO)
      QTT_HIP(bond_mpo_apply(st, Yb, (int)rho0, (int)ra0, (int)dj, (int)rb1, Ak, s.d[k], (int)ra1, T));
    else
      QTT_HIP(bond_hadamard_apply(st, Yb, (int)rho0, (int)ra0, s.d[k], (int)rb1, Ak, (int)ra1, T));
    std::swap(S, T);
    Pleg *= s.d[k];
    rcS = ra1 * rb1;
    ++legs;
    while ((legs == Z.N && k < n - 1) || (k == n - 1 && legs > 1)) {
      const long db = s.d[outc];
      const int m = (int)(r * db), cols = (int)((Pleg / db) * rcS);
      // SVD of S (m x cols) through its transpose B = S^T: Jacobi on the rows
      // of F = R (QR of a tall B) or of B itself; U_S = V_B, Sig V_S^T = (B V_B)^T.
      const bool tall = cols >= m;
      const int L = m;
      int p;
      if (tall) {
        QTT_HIP(transpose(st, S, m, cols, cols, Bt, m));
        QTT_HIP(householder_qr(st, Bt, cols, m, m, TB, scr));
        QTT_HIP(extract_r(st, Bt, m, m, m, X));
        p = m;
      } else {
        QTT_HIP(transpose(st, S, m, cols, cols, X, m));
        p = cols;
      }
      QTT_HIP(copy_pad_rows(st, X, p, L, L, Xc, p, L));
      QTT_HIP(row_norms_sorted(st, Xc, p, L, sig, perm));
      QTT_HIP(permute_rows(st, Xc, p, L, perm, X));
      QTT_HIP(jacobi_rows(st, X, p, L, ctr, h->max_sweeps, sweeps, sig));  // sig[0]: largest row norm
      QTT_HIP(row_norms_sorted(st, X, p, L, sig, perm));
      QTT_HIP(frob_norm(st, sig, p, nrm));  // ||S||_F of the super-core being split
      QTT_HIP(truncate_decide(st, sig, p, nrm, rel_tol, n - 1, max_rank, tr));
      QTT_HIP(hipMemcpyAsync(h->pin_int, sweeps, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      int e = readback(h, st, tr, sizeof(TruncOut), h->pin_trunc);
      if (e) return e;
      const TruncOut t = *h->pin_trunc;
      const int swp = h->pin_int[0];
      if (!std::isfinite(t.norm)) return QTT_ERR_NONFINITE;
      if (!h->pin_int[1]) return QTT_ERR_NOCONV;
      maxsw = std::max(maxsw, swp);
      const int rn = t.rank;
      if (outc == 0) {
        first_norm = t.norm;
        first_delta = t.delta;
      }
      if (info) {
        const int bnd = outc;
        if (info->tail) info->tail[bnd] = t.tail_r;
        if (info->margin_lo) info->margin_lo[bnd] = t.delta > 0 ? t.tail_rm1 / t.delta : INFINITY;
        if (info->margin_hi) info->margin_hi[bnd] = t.delta > 0 ? t.tail_r / t.delta : 0.0;
        if (info->maxrank_hit) info->maxrank_hit[bnd] = (uint8_t)t.capped;
        if (info->sigma && info->sigma_ld > 0) {
          const long cnt = std::min<long>(p, info->sigma_ld);
          QTT_HIP(hipMemcpyAsync(info->sigma + (long)bnd * info->sigma_ld, sig, cnt * sizeof(double),
                                 hipMemcpyDeviceToHost, st));
          QTT_HIP(hipStreamSynchronize(st));
          for (long i = cnt; i < info->sigma_ld; ++i) info->sigma[(long)bnd * info->sigma_ld + i] = 0.0;
        }
      }
      err2 += t.tail_r * t.tail_r;
      // result core = V_B,r (m x rn): rows perm[:rn] of X normalised, transposed
      QTT_HIP(gather_rows_normalized(st, X, L, perm, sig, tr, V, L, rn));
      QTT_HIP(transpose(st, V, rn, m, m, (double*)out->cores[outc], rn));
      // Yn = B V_r (cols x rn); tall B = Q_B R  =>  Q_B [R V_r; 0]
      QTT_HIP(gemm_prec(st, prec, false, true, p, rn, L, Xc, L, V, L, Yn, rn));
      if (tall) {
        if (cols > p) QTT_HIP(fill_f64(st, Yn + (long)p * rn, 0.0, (long)(cols - p) * rn));
        QTT_HIP(apply_q(st, Bt, cols, p, m, TB, Yn, rn, rn, false, scr));
      }
      // remainder S = Yn^T (rn x cols) = Sig_r V_S,r^T
      QTT_HIP(transpose(st, Yn, cols, rn, rn, S, cols));
      newr[outc + 1] = rn;
      ++outc;
      r = rn;
      Pleg /= db;
      --legs;
    }
  }
  // last core = the one-leg remainder (r x d x 1)
  QTT_HIP(copy_pad_rows(st, S, (int)(r * s.d[n - 1]), 1, 1, (double*)out->cores[n - 1], (int)(r * s.d[n - 1]), 1));
  if (n == 1) {
    QTT_HIP(frob_norm(st, S, s.d[0], nrm));
    int e = readback(h, st, nrm, sizeof(double), h->pin_dbl);
    if (e) return e;
    first_norm = h->pin_dbl[0];
    if (!std::isfinite(first_norm)) return QTT_ERR_NONFINITE;
  }
  QTT_HIP(hipStreamSynchronize(st));
  if (info) {
    info->norm = first_norm;
    info->delta = first_delta;
    info->err_bound = std::sqrt(err2);
    info->jacobi_sweeps_max = maxsw;
  }
  return QTT_OK;
}

int zip_setup(const char* spec, const qtt_tt* a, const qtt_tt* b, long max_rank, int ncores, Shape& s, ZipPlan& Z) {
  int st = shape_from_pair(spec, a, b, s);
  if (st) return st;
  if (a->dtype != QTT_F64 || b->dtype != QTT_F64) return QTT_ERR_DTYPE;
  return make_zip_plan(s, a, b, max_rank, ncores, Z);
}

}  // namespace

namespace {

// ---------------------------------------------------------------- variational fitting
// Sec. 3.3: with the cores left of q left-orthonormal and those right of q
// right-orthonormal, the best core q is L_{q-1} Y_q R_{q+1} (the derivative
// of <C|Y> with respect to C_q), Y the exactly contracted product.
struct FitPlan {
  std::vector<long> ry, rc;        // product ranks, ranks of the fitted train (bounds)
  std::vector<long> offY, offL, offF;
  long offT = 0, offP = 0, offG = 0, offTq = 0, offQe = 0, offScr = 0, offNrm = 0;
  long total = 0;
};

int make_fit_plan(const Shape& s, const qtt_tt* c, FitPlan& F) {
  const int n = s.n;
  F.ry = s.rc;
  F.rc.assign(n + 1, 1);
  for (int k = 0; k <= n; ++k) F.rc[k] = c->ranks[k];
  long off = 0;
  auto take = [&](long cnt) {
    long o = off;
    off += round_up(std::max(cnt, 1L), 32);
    return o;
  };
  F.offY.assign(n, 0);
  F.offL.assign(n + 1, 0);
  F.offF.assign(n + 1, 0);
  long maxT = 1, maxP = 1, maxG = 1, maxTq = 1, maxQe = 1, maxc = 1;
  for (int k = 0; k < n; ++k) {
    const long d = s.d[k];
    F.offY[k] = take(F.ry[k] * d * F.ry[k + 1]);
    maxT = std::max(maxT, F.rc[k] * d * F.ry[k + 1]);  // E Y_k, C_k F and L Y_k share this size
    const long P = F.rc[k] * d * F.rc[k + 1];
    maxP = std::max(maxP, P);
    // right-to-left: QR of the (d rc1) x rc0 transpose; left-to-right: of (rc0 d) x rc1
    const long m1 = d * F.rc[k + 1], n1 = F.rc[k], m2 = F.rc[k] * d, n2 = F.rc[k + 1];
    if (m1 > kMaxRows || m2 > kMaxRows) return QTT_ERR_UNSUPPORTED;
    maxG = std::max(maxG, m1 * n1);
    maxTq = std::max({maxTq, qr_t_doubles((int)m1, (int)n1), qr_t_doubles((int)m2, (int)n2)});
    maxQe = std::max({maxQe, m1 * std::min(m1, n1), m2 * std::min(m2, n2)});
    maxc = std::max({maxc, n1, n2});
  }
  for (int k = 0; k <= n; ++k) {
    F.offL[k] = take(F.rc[k] * F.ry[k]);
    F.offF[k] = take(F.rc[k] * F.ry[k]);
  }
  F.offT = take(maxT);
  F.offP = take(maxP);
  F.offG = take(maxG);
  F.offTq = take(maxTq);
  F.offQe = take(maxQe);
  F.offScr = take(qr_scratch_doubles(maxc));
  F.offNrm = take(1);
  F.total = off;
  return QTT_OK;
}

// P = L Y_q R^T: (rc0 x ry0)(ry0 x d ry1) then ((rc0 d) x ry1)(ry1 x rc1)
hipError_t fit_project(hipStream_t st, const double* L, const double* Yq, const double* R, long rc0, long rc1,
                       long ry0, long ry1, long d, double* T, double* P) {
  hipError_t e = gemm_f64(st, false, false, (int)rc0, (int)(d * ry1), (int)ry0, 1.0, L, ry0, 0, Yq, d * ry1, 0, 0.0,
                          T, d * ry1, 0, 1);
  if (e != hipSuccess) return e;
  return gemm_f64(st, false, true, (int)(rc0 * d), (int)rc1, (int)ry1, 1.0, T, ry1, 0, R, ry1, 0, 0.0, P, rc1, 0, 1);
}

int fit_sweeps(hipStream_t st, double* ws, const Shape& s, const FitPlan& F, qtt_tt* c, std::vector<long>& rc,
               int nsweeps) {
  const int n = s.n;
  double* T = ws + F.offT;
  double* P = ws + F.offP;
  double* G = ws + F.offG;
  double* Tq = ws + F.offTq;
  double* Qe = ws + F.offQe;
  double* scr = ws + F.offScr;
  auto core = [&](int k) { return (double*)c->cores[k]; };
  auto Y = [&](int k) { return (const double*)(ws + F.offY[k]); };
  QTT_HIP(fill_f64(st, ws + F.offL[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offF[n], 1.0, 1));
  for (int k = 0; k + 1 < n; ++k)
    QTT_HIP(env_step_left<double>(st, ws + F.offL[k], core(k), Y(k), rc[k], rc[k + 1], F.ry[k], F.ry[k + 1], s.d[k],
                                  T, ws + F.offL[k + 1]));
  for (int sw = 0; sw < nsweeps; ++sw) {
    // right to left: the centre moves to core 1
    for (int q = n - 1; q >= 0; --q) {
      const long d = s.d[q];
      QTT_HIP(fit_project(st, ws + F.offL[q], Y(q), ws + F.offF[q + 1], rc[q], rc[q + 1], F.ry[q], F.ry[q + 1], d, T,
                          P));
      if (q > 0) {
        const int m = (int)(d * rc[q + 1]), nn = (int)rc[q], qq = std::min(m, nn);
        QTT_HIP(transpose(st, P, nn, m, m, G, nn));
        QTT_HIP(householder_qr(st, G, m, nn, nn, Tq, scr));
        QTT_HIP(set_eye_rect(st, Qe, m, qq));
        QTT_HIP(apply_q(st, G, m, qq, nn, Tq, Qe, qq, qq, false, scr));
        QTT_HIP(transpose(st, Qe, m, qq, qq, core(q), m));
        rc[q] = qq;
      } else {
        QTT_HIP(copy_pad_rows(st, P, (int)(d * rc[1]), 1, 1, core(0), (int)(d * rc[1]), 1));
      }
      QTT_HIP(env_step_right<double>(st, ws + F.offF[q + 1], core(q), Y(q), rc[q], rc[q + 1], F.ry[q], F.ry[q + 1], d,
                                     T, ws + F.offF[q]));
    }
    // left to right: the centre moves back to core n
    for (int q = 0; q < n; ++q) {
      const long d = s.d[q];
      QTT_HIP(fit_project(st, ws + F.offL[q], Y(q), ws + F.offF[q + 1], rc[q], rc[q + 1], F.ry[q], F.ry[q + 1], d, T,
                          P));
      if (q < n - 1) {
        const int m = (int)(rc[q] * d), nn = (int)rc[q + 1], qq = std::min(m, nn);
        QTT_HIP(householder_qr(st, P, m, nn, nn, Tq, scr));
        QTT_HIP(set_eye_rect(st, Qe, m, qq));
        QTT_HIP(apply_q(st, P, m, qq, nn, Tq, Qe, qq, qq, false, scr));
        QTT_HIP(copy_pad_rows(st, Qe, m, qq, qq, core(q), m, qq));
        rc[q + 1] = qq;
        QTT_HIP(env_step_left<double>(st, ws + F.offL[q], core(q), Y(q), rc[q], rc[q + 1], F.ry[q], F.ry[q + 1], d, T,
                                      ws + F.offL[q + 1]));
      } else {
        QTT_HIP(copy_pad_rows(st, P, (int)(rc[q] * d), 1, 1, core(q), (int)(rc[q] * d), 1));
      }
    }
  }
  QTT_HIP(frob_norm(st, core(n - 1), rc[n - 1] * s.d[n - 1], ws + F.offNrm));
  return QTT_OK;
}

// ---------------------------------------------------------------- two-core fitting
// Sec. 3.3, multi-core strategy with super-cores of two cores: with the cores
// left of the pair (q, q+1) left-orthonormal and those right of it
// right-orthonormal, the best super-core is
//   S[(a,i),(j,c)] = sum L_q[a,b] Y_q[b,i,d] Y_{q+1}[d,j,e] R_{q+2}[c,e],
// decomposed again by a truncated SVD (rank rule of the rounding with
// delta = rel_tol ||S||_F / sqrt(n-1), capped at max_rank), so the ranks of
// the fitted train adapt to the product.
struct Fit2Plan {
  std::vector<long> ry, bnd;  // product ranks, capacity of the fitted train's ranks
  std::vector<long> offY, offL, offF;
  long offT1 = 0, offT2 = 0, offS = 0, offSt = 0, offTB = 0, offX = 0, offXc = 0, offV = 0, offYt = 0, offMV = 0;
  long offSig = 0, offPerm = 0, offTrunc = 0, offCtr = 0, offSweeps = 0, offNrm = 0, offScr = 0;
  long total = 0;
};

// Rank capacity of every bond of the fitted train: the guess's rank, or the
// largest rank a split can produce (min of the left and right physical
// products, the product's rank, max_rank), whichever is larger.
std::vector<long> fit2_bounds(const Shape& s, const qtt_tt* c, long max_rank) {
  const int n = s.n;
  std::vector<long> left(n + 1, 1), right(n + 1, 1), b(n + 1, 1);
  for (int k = 1; k <= n; ++k) left[k] = std::min<long>(left[k - 1] * s.d[k - 1], 1L << 40);
  for (int k = n - 1; k >= 0; --k) right[k] = std::min<long>(right[k + 1] * s.d[k], 1L << 40);
  for (int k = 1; k < n; ++k) {
    long v = std::min({left[k], right[k], s.rc[k]});
    if (max_rank > 0) v = std::min(v, max_rank);
    b[k] = std::max<long>({v, c->ranks[k], 1L});
  }
  return b;
}

int make_fit2_plan(const Shape& s, const qtt_tt* c, long max_rank, Fit2Plan& F) {
  const int n = s.n;
  F.ry = s.rc;
  F.bnd = fit2_bounds(s, c, max_rank);
  long off = 0;
  auto take = [&](long cnt) {
    long o = off;
    off += round_up(std::max(cnt, 1L), 32);
    return o;
  };
  F.offY.assign(n, 0);
  F.offL.assign(n + 1, 0);
  F.offF.assign(n + 1, 0);
  long maxT1 = 1, maxT2 = 1, maxS = 1, maxTB = 1, maxX = 1, maxP = 1, maxc = 1, maxE = 1;
  for (int k = 0; k < n; ++k) {
    F.offY[k] = take(F.ry[k] * s.d[k] * F.ry[k + 1]);
    maxE = std::max(maxE, F.bnd[k] * s.d[k] * F.ry[k + 1]);  // environment step temporaries
  }
  for (int k = 0; k <= n; ++k) {
    F.offL[k] = take(F.bnd[k] * F.ry[k]);
    F.offF[k] = take(F.bnd[k] * F.ry[k]);
  }
  for (int q = 0; q + 1 < n; ++q) {
    const long m = F.bnd[q] * s.d[q], cols = (long)s.d[q + 1] * F.bnd[q + 2];
    maxT1 = std::max(maxT1, m * F.ry[q + 1]);
    maxT2 = std::max(maxT2, F.ry[q + 1] * cols);
    maxS = std::max(maxS, m * cols);
    // both orientations of the split: rows M x L with M, L in {m, cols}
    for (int o = 0; o < 2; ++o) {
      const long p0 = o ? cols : m, L = o ? m : cols;
      if (L > 1024 || p0 > kMaxRows) return QTT_ERR_UNSUPPORTED;
      const long p = std::min(p0, L);
      maxTB = std::max(maxTB, qr_t_doubles((int)p0, (int)p));
      maxX = std::max(maxX, p * L);
      maxP = std::max(maxP, p);
      maxc = std::max({maxc, L, p0});
    }
  }
  F.offT1 = take(std::max(maxT1, maxE));
  F.offT2 = take(maxT2);
  F.offS = take(maxS);
  F.offSt = take(maxS);
  F.offTB = take(maxTB);
  F.offX = take(maxX);
  F.offXc = take(maxX);
  F.offV = take(maxX);
  F.offYt = take(maxX);
  F.offMV = take(maxS);
  F.offSig = take(maxP);
  F.offPerm = take(maxP / 2 + 1);
  F.offTrunc = take(8);
  F.offCtr = take(96);
  F.offSweeps = take(1);
  F.offNrm = take(1);
  F.offScr = take(qr_scratch_doubles(maxc));
  F.total = off;
  return QTT_OK;
}

// Truncated SVD of M (p0 x L, row-major; overwritten by its Householder QR
// when tall): vt (rn x L, ld L) the kept right singular vectors as rows,
// mv (p0 x rn, ld rn) = M V_r = U_r Sigma_r.  The rank rule's threshold is
// rel_tol * ||M||_F / sqrt(nb), or rel_tol * (*norm_override) / sqrt(nb)
// with a device scalar given.  Reads the decision back.
// Device buffers of a truncated split (see split_rows).
struct SplitBufs {
  double *TB, *X, *Xc, *Yt, *sig, *nrm, *scr;
  int* perm;
  TruncOut* tr;
  unsigned* ctr;
  int* sweeps;
};

SplitBufs fit2_bufs(double* ws, const Fit2Plan& F) {
  SplitBufs b;
  b.TB = ws + F.offTB;
  b.X = ws + F.offX;
  b.Xc = ws + F.offXc;
  b.Yt = ws + F.offYt;
  b.sig = ws + F.offSig;
  b.perm = (int*)(ws + F.offPerm);
  b.tr = (TruncOut*)(ws + F.offTrunc);
  b.ctr = (unsigned*)(ws + F.offCtr);
  b.sweeps = (int*)(ws + F.offSweeps);
  b.nrm = ws + F.offNrm;
  b.scr = ws + F.offScr;
  return b;
}

int split_rows(qtt_context* h, hipStream_t st, const SplitBufs& bf, double* M, int p0, int L, double rel_tol, int nb,
               long max_rank, double* vt, double* mv, int& rn, double& tail, int& swp,
               const double* norm_override = nullptr) {
  double* TB = bf.TB;
  double* X = bf.X;
  double* Xc = bf.Xc;
  double* Yt = bf.Yt;
  double* sig = bf.sig;
  int* perm = bf.perm;
  TruncOut* tr = bf.tr;
  unsigned* ctr = bf.ctr;
  int* sweeps = bf.sweeps;
  double* nrm = bf.nrm;
  double* scr = bf.scr;
  const bool tall = p0 >= L;
  const int p = tall ? L : p0;
  if (tall) {
    QTT_HIP(householder_qr(st, M, p0, L, L, TB, scr));
    QTT_HIP(extract_r(st, M, L, L, L, Xc));
  } else {
    QTT_HIP(copy_pad_rows(st, M, p0, L, L, Xc, p0, L));
  }
  QTT_HIP(row_norms_sorted(st, Xc, p, L, sig, perm));
  QTT_HIP(permute_rows(st, Xc, p, L, perm, X));
  QTT_HIP(jacobi_rows(st, X, p, L, ctr, h->max_sweeps, sweeps, sig));  // sig[0]: largest row norm
  QTT_HIP(row_norms_sorted(st, X, p, L, sig, perm));
  // the threshold's scale: ||S||_F of the matrix being split, or a given one
  if (!norm_override) QTT_HIP(frob_norm(st, sig, p, nrm));
  QTT_HIP(truncate_decide(st, sig, p, norm_override ? norm_override : nrm, rel_tol, nb, max_rank, tr));
  QTT_HIP(hipMemcpyAsync(h->pin_int, sweeps, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  int e = readback(h, st, tr, sizeof(TruncOut), h->pin_trunc);
  if (e) return e;
  const TruncOut t = *h->pin_trunc;
  if (!std::isfinite(t.norm)) return QTT_ERR_NONFINITE;
  if (!h->pin_int[1]) return QTT_ERR_NOCONV;
  swp = h->pin_int[0];
  rn = t.rank;
  tail = t.tail_r;
  QTT_HIP(gather_rows_normalized(st, X, L, perm, sig, tr, vt, L, rn));
  QTT_HIP(gemm_f64(st, false, true, p, rn, L, 1.0, Xc, L, 0, vt, L, 0, 0.0, Yt, rn, 0, 1));
  QTT_HIP(copy_pad_rows(st, Yt, p, rn, rn, mv, p0, rn));
  if (tall) QTT_HIP(apply_q(st, M, p0, p, L, TB, mv, rn, rn, false, scr));
  return QTT_OK;
}

// S = L_q Y_q Y_{q+1} R_{q+2}^T as (rc_q d_q) x (d_{q+1} rc_{q+2}).
hipError_t fit2_supercore(hipStream_t st, double* ws, const Shape& s, const Fit2Plan& F, const std::vector<long>& rc,
                          int q, double* S) {
  const long rc0 = rc[q], rc2 = rc[q + 2], ry0 = F.ry[q], ry1 = F.ry[q + 1], ry2 = F.ry[q + 2];
  const long d0 = s.d[q], d1 = s.d[q + 1];
  double* T1 = ws + F.offT1;
  double* T2 = ws + F.offT2;
  hipError_t e = gemm_f64(st, false, false, (int)rc0, (int)(d0 * ry1), (int)ry0, 1.0, ws + F.offL[q], ry0, 0,
                          ws + F.offY[q], d0 * ry1, 0, 0.0, T1, d0 * ry1, 0, 1);
  if (e != hipSuccess) return e;
  e = gemm_f64(st, false, true, (int)(ry1 * d1), (int)rc2, (int)ry2, 1.0, ws + F.offY[q + 1], ry2, 0,
               ws + F.offF[q + 2], ry2, 0, 0.0, T2, rc2, 0, 1);
  if (e != hipSuccess) return e;
  return gemm_f64(st, false, false, (int)(rc0 * d0), (int)(d1 * rc2), (int)ry1, 1.0, T1, ry1, 0, T2, d1 * rc2, 0,
                  0.0, S, d1 * rc2, 0, 1);
}

int fit2_sweeps(qtt_context* h, hipStream_t st, double* ws, const Shape& s, const Fit2Plan& F, qtt_tt* c,
                std::vector<long>& rc, int nsweeps, double rel_tol, long max_rank, double* tails, int& maxsw) {
  const int n = s.n;
  auto core = [&](int k) { return (double*)c->cores[k]; };
  auto Y = [&](int k) { return (const double*)(ws + F.offY[k]); };
  double* S = ws + F.offS;
  double* St = ws + F.offSt;
  double* V = ws + F.offV;
  double* MV = ws + F.offMV;
  double* T = ws + F.offT1;
  QTT_HIP(fill_f64(st, ws + F.offL[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offF[n], 1.0, 1));
  for (int k = 0; k + 2 < n; ++k)
    QTT_HIP(env_step_left<double>(st, ws + F.offL[k], core(k), Y(k), rc[k], rc[k + 1], F.ry[k], F.ry[k + 1], s.d[k],
                                  T, ws + F.offL[k + 1]));
  maxsw = 0;
  int split_no = 0;
  for (int sw = 0; sw < nsweeps; ++sw) {
    // pairs from the right end: core q+1 <- V^T (right-orthonormal), core q <- U Sigma
    for (int q = n - 2; q >= 0; --q) {
      const long m = rc[q] * s.d[q], cols = (long)s.d[q + 1] * rc[q + 2];
      QTT_HIP(fit2_supercore(st, ws, s, F, rc, q, S));
      int rn = 0, swp = 0;
      double tail = 0.0;
      int e = split_rows(h, st, fit2_bufs(ws, F), S, (int)m, (int)cols, rel_tol, n - 1, max_rank, V, MV, rn, tail,
                         swp);
      if (e) return e;
      if (rn > F.bnd[q + 1]) return QTT_ERR_UNSUPPORTED;
      maxsw = std::max(maxsw, swp);
      if (tails) tails[split_no] = tail;
      ++split_no;
      QTT_HIP(copy_pad_rows(st, V, rn, (int)cols, cols, core(q + 1), rn, cols));
      QTT_HIP(copy_pad_rows(st, MV, (int)m, rn, rn, core(q), (int)m, rn));
      rc[q + 1] = rn;
      QTT_HIP(env_step_right<double>(st, ws + F.offF[q + 2], core(q + 1), Y(q + 1), rc[q + 1], rc[q + 2], F.ry[q + 1],
                                     F.ry[q + 2], s.d[q + 1], T, ws + F.offF[q + 1]));
    }
    // and back from the left end: core q <- U (left-orthonormal), core q+1 <- Sigma V^T
    for (int q = 0; q + 1 < n; ++q) {
      const long m = rc[q] * s.d[q], cols = (long)s.d[q + 1] * rc[q + 2];
      QTT_HIP(fit2_supercore(st, ws, s, F, rc, q, S));
      QTT_HIP(transpose(st, S, (int)m, (int)cols, cols, St, m));
      int rn = 0, swp = 0;
      double tail = 0.0;
      int e = split_rows(h, st, fit2_bufs(ws, F), St, (int)cols, (int)m, rel_tol, n - 1, max_rank, V, MV, rn, tail,
                         swp);
      if (e) return e;
      if (rn > F.bnd[q + 1]) return QTT_ERR_UNSUPPORTED;
      maxsw = std::max(maxsw, swp);
      if (tails) tails[split_no] = tail;
      ++split_no;
      QTT_HIP(transpose(st, V, rn, (int)m, m, core(q), rn));        // (rc_q d_q) x rn
      QTT_HIP(transpose(st, MV, (int)cols, rn, rn, core(q + 1), cols));  // rn x (d_{q+1} rc_{q+2})
      rc[q + 1] = rn;
      QTT_HIP(env_step_left<double>(st, ws + F.offL[q], core(q), Y(q), rc[q], rc[q + 1], F.ry[q], F.ry[q + 1], s.d[q],
                                    T, ws + F.offL[q + 1]));
    }
  }
  QTT_HIP(frob_norm(st, core(n - 1), rc[n - 1] * s.d[n - 1], ws + F.offNrm));
  return QTT_OK;
}

int fit2_setup(const char* spec, const qtt_tt* a, const qtt_tt* b, const qtt_tt* c, long max_rank, Shape& s,
               Fit2Plan& F, size_t& orth_bytes) {
  int st = shape_from_pair(spec, a, b, s);
  if (st) return st;
  if (a->dtype != QTT_F64 || b->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if ((st = check_tt(c, 1))) return st;
  if (c->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if (c->n != s.n) return QTT_ERR_SHAPE;
  for (int k = 0; k < s.n; ++k)
    if (dphys(c, k) != s.d[k]) return QTT_ERR_SHAPE;
  Shape sc;
  shape_from_tt(c, sc);
  Plan P;
  if ((st = make_plan(sc, 0, P, false))) return st;
  orth_bytes = ws_bytes_of(P);
  return make_fit2_plan(s, c, max_rank, F);
}

// ---------------------------------------------------------------- linear solver
// Sec. 5, DMRG-like strategy for W x = b with W symmetric positive definite:
// the energy J(x) = <x, W x> - 2 <x, b> is minimised over one core (ranks
// fixed) or a super-core of two cores (ranks adapt through the truncated
// split of the fitting).  With the cores outside the block orthonormal the
// block's minimiser solves A_loc x = b_loc, A_loc the block's local matrix
// (three-layer environments of <x|W|x> and the block's operator cores),
// b_loc = Lb b_block Rb^T.  A_loc is symmetric positive definite (an SPD
// operator between orthonormal frames), so the local system is solved by a
// blocked Cholesky factorisation (backward stable for SPD matrices) and two
// triangular solves.
struct SolvePlan {
  int nc = 1;
  std::vector<long> bnd, rw, rb;
  std::vector<long> offLW, offRW, offLb, offRb;
  long offA = 0, offRhs = 0, offT = 0, offE1 = 0, offE2 = 0, offG = 0, offBp = 0, offGt = 0, offTq = 0, offQe = 0;
  long offS = 0, offSt = 0, offV = 0, offMV = 0, offChol = 0;
  long offTB = 0, offX = 0, offXc = 0, offYt = 0, offSig = 0, offPerm = 0, offTrunc = 0, offCtr = 0, offSweeps = 0,
       offNrm = 0, offScr = 0;
  long total = 0;
};

SplitBufs solve_bufs(double* ws, const SolvePlan& F) {
  SplitBufs b;
  b.TB = ws + F.offTB;
  b.X = ws + F.offX;
  b.Xc = ws + F.offXc;
  b.Yt = ws + F.offYt;
  b.sig = ws + F.offSig;
  b.perm = (int*)(ws + F.offPerm);
  b.tr = (TruncOut*)(ws + F.offTrunc);
  b.ctr = (unsigned*)(ws + F.offCtr);
  b.sweeps = (int*)(ws + F.offSweeps);
  b.nrm = ws + F.offNrm;
  b.scr = ws + F.offScr;
  return b;
}

int solve_check(const qtt_tt* w, const qtt_tt* b, const qtt_tt* x) {
  int st;
  if ((st = check_tt(w, 2)) || (st = check_tt(b, 1)) || (st = check_tt(x, 1))) return st;
  if (w->dtype != QTT_F64 || b->dtype != QTT_F64 || x->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if (w->n != b->n || x->n != b->n) return QTT_ERR_SHAPE;
  for (int k = 0; k < w->n; ++k)
    if (dphys(w, k) != dphys_in(w, k) || dphys(b, k) != dphys(w, k) || dphys(x, k) != dphys(w, k))
      return QTT_ERR_SHAPE;
  return QTT_OK;
}

int make_solve_plan(const qtt_tt* w, const qtt_tt* b, const qtt_tt* x, int ncores, long max_rank, SolvePlan& F) {
  const int n = x->n;
  F.nc = ncores;
  F.bnd.assign(n + 1, 1);
  F.rw.assign(n + 1, 1);
  F.rb.assign(n + 1, 1);
  std::vector<long> left(n + 1, 1), right(n + 1, 1);
  std::vector<int> d(n);
  for (int k = 0; k < n; ++k) d[k] = dphys(x, k);
  for (int k = 1; k <= n; ++k) left[k] = std::min<long>(left[k - 1] * d[k - 1], 1L << 40);
  for (int k = n - 1; k >= 0; --k) right[k] = std::min<long>(right[k + 1] * d[k], 1L << 40);
  for (int k = 0; k <= n; ++k) {
    F.rw[k] = w->ranks[k];
    F.rb[k] = b->ranks[k];
    // after the left orthogonalisation of the guess its ranks are at most min(left, guess)
    long v = std::min<long>(left[k], x->ranks[k]);
    if (ncores == 2 && k > 0 && k < n) {
      long grow = std::min(left[k], right[k]);
      if (max_rank > 0) grow = std::min(grow, max_rank);
      v = std::max(v, grow);
    }
    F.bnd[k] = std::max(v, 1L);
  }
  long off = 0;
  auto take = [&](long cnt) {
    long o = off;
    off += round_up(std::max(cnt, 1L), 32);
    return o;
  };
  F.offLW.assign(n + 1, 0);
  F.offRW.assign(n + 1, 0);
  F.offLb.assign(n + 1, 0);
  F.offRb.assign(n + 1, 0);
  for (int k = 0; k <= n; ++k) {
    F.offLW[k] = take(F.bnd[k] * F.rw[k] * F.bnd[k]);
    F.offRW[k] = take(F.bnd[k] * F.rw[k] * F.bnd[k]);
    F.offLb[k] = take(F.bnd[k] * F.rb[k]);
    F.offRb[k] = take(F.bnd[k] * F.rb[k]);
  }
  long maxN = 1, maxT = 1, maxE = 1, maxG = 1, maxBp = 1, maxGt = 1, maxTq = 1, maxQe = 1, maxSplit = 1;
  long maxTB = 1, maxX = 1, maxP = 1, maxc = 1;
  for (int k = 0; k < n; ++k) {
    const long r0 = F.bnd[k], r1 = F.bnd[k + 1], w0 = F.rw[k], w1 = F.rw[k + 1];
    maxE = std::max({maxE, r0 * w0 * d[k] * r1, r0 * d[k] * w1 * r1, d[k] * r1 * w0 * r0});
    if (ncores == 1) {
      const long N = r0 * d[k] * r1;
      maxN = std::max(maxN, N);
      maxT = std::max(maxT, r0 * d[k] * F.rb[k + 1]);
      // QR moves: the solved core (r0 d) x r1 or its transpose (d r1) x r0
      const long m1 = d[k] * r1, m2 = r0 * d[k];
      if (m1 > kMaxRows || m2 > kMaxRows) return QTT_ERR_UNSUPPORTED;
      maxGt = std::max(maxGt, m1 * r0);
      maxTq = std::max({maxTq, qr_t_doubles((int)m1, (int)r0), qr_t_doubles((int)m2, (int)r1)});
      maxQe = std::max({maxQe, m1 * std::min(m1, r0), m2 * std::min(m2, r1)});
      maxc = std::max({maxc, r0, r1});
    } else if (k + 1 < n) {
      const long r2 = F.bnd[k + 2], P = (long)d[k] * d[k + 1];
      const long N = r0 * P * r2;
      maxN = std::max(maxN, N);
      maxT = std::max(maxT, r0 * P * F.rb[k + 2]);
      maxG = std::max(maxG, w0 * P * P * F.rw[k + 2]);
      maxBp = std::max(maxBp, F.rb[k] * P * F.rb[k + 2]);
      const long m = r0 * d[k], cols = (long)d[k + 1] * r2;
      maxSplit = std::max(maxSplit, m * cols);
      for (int o = 0; o < 2; ++o) {
        const long p0 = o ? cols : m, L = o ? m : cols;
        if (L > 1024 || p0 > kMaxRows) return QTT_ERR_UNSUPPORTED;
        const long p = std::min(p0, L);
        maxTB = std::max(maxTB, qr_t_doubles((int)p0, (int)p));
        maxX = std::max(maxX, p * L);
        maxP = std::max(maxP, p);
        maxc = std::max({maxc, L, p0});
      }
    }
  }
  if (maxN > kMaxRows) return QTT_ERR_UNSUPPORTED;  // the local QR solve
  F.offA = take(maxN * maxN);
  F.offRhs = take(maxN);
  F.offT = take(maxT);
  F.offE1 = take(maxE);
  F.offE2 = take(maxE);
  F.offG = take(maxG);
  F.offBp = take(maxBp);
  F.offGt = take(maxGt);
  F.offTq = take(maxTq);
  F.offQe = take(maxQe);
  F.offS = take(maxSplit);
  F.offSt = take(maxSplit);
  F.offV = take(maxX);
  F.offMV = take(maxSplit);
  F.offChol = take(chol_work_doubles(maxN));
  F.offTB = take(maxTB);
  F.offX = take(maxX);
  F.offXc = take(maxX);
  F.offYt = take(maxX);
  F.offSig = take(maxP);
  F.offPerm = take(maxP / 2 + 1);
  F.offTrunc = take(8);
  F.offCtr = take(96);
  F.offSweeps = take(1);
  F.offNrm = take(1);
  F.offScr = take(qr_scratch_doubles(maxc));
  F.total = off;
  return QTT_OK;
}

// LW' = sum x^T LW W x (three-layer step to the right of core x: r0 -> r1)
hipError_t env3_left(hipStream_t st, const double* LW, const double* x, const double* W, long r0, long d, long r1,
                     long w0, long w1, double* T1, double* T2, double* out) {
  hipError_t e = gemm_f64(st, false, false, (int)(r0 * w0), (int)(d * r1), (int)r0, 1.0, LW, r0, 0, x, d * r1, 0,
                          0.0, T1, d * r1, 0, 1);
  if (e != hipSuccess) return e;
  if ((e = env3_left_mid(st, T1, W, (int)r0, (int)w0, (int)d, (int)w1, (int)r1, T2)) != hipSuccess) return e;
  return gemm_f64(st, true, false, (int)r1, (int)(w1 * r1), (int)(r0 * d), 1.0, x, r1, 0, T2, w1 * r1, 0, 0.0, out,
                  w1 * r1, 0, 1);
}

// RW = sum x W x RW' (three-layer step to the left of core x: r1 -> r0)
hipError_t env3_right(hipStream_t st, const double* RW, const double* x, const double* W, long r0, long d, long r1,
                      long w0, long w1, double* U1, double* U2, double* out) {
  hipError_t e = gemm_f64(st, false, true, (int)(r0 * d), (int)(r1 * w1), (int)r1, 1.0, x, r1, 0, RW, r1, 0, 0.0, U1,
                          r1 * w1, 0, 1);
  if (e != hipSuccess) return e;
  if ((e = env3_right_mid(st, U1, W, (int)r0, (int)w0, (int)d, (int)w1, (int)r1, U2)) != hipSuccess) return e;
  return gemm_f64(st, false, false, (int)r0, (int)(w0 * r0), (int)(d * r1), 1.0, x, d * r1, 0, U2, w0 * r0, 0, 0.0,
                  out, w0 * r0, 0, 1);
}

// Local solve over the block starting at core q (ncores 1 or 2): writes the
// block's minimiser into F.offRhs (layout [r0][P][r_end]).
int solve_local(hipStream_t st, double* ws, const SolvePlan& F, const qtt_tt* w, const qtt_tt* b,
                const std::vector<long>& rc, const std::vector<int>& d, int q) {
  const int nc = F.nc;
  const long r0 = rc[q], r1 = rc[q + nc];
  const long w0 = F.rw[q], w1 = F.rw[q + nc];
  const long P = nc == 1 ? d[q] : (long)d[q] * d[q + 1];
  const long N = r0 * P * r1;
  double* A = ws + F.offA;
  double* rhs = ws + F.offRhs;
  const double* Wl = (const double*)w->cores[q];
  const double* bl = (const double*)b->cores[q];
  long rbl0 = F.rb[q], rbl1 = F.rb[q + nc];
  if (nc == 2) {
    QTT_HIP(mpo_pair(st, (const double*)w->cores[q], (const double*)w->cores[q + 1], (int)w0, d[q], (int)F.rw[q + 1],
                     d[q + 1], (int)w1, ws + F.offG));
    Wl = ws + F.offG;
    const long rbm = F.rb[q + 1];
    QTT_HIP(gemm_f64(st, false, false, (int)(rbl0 * d[q]), (int)(d[q + 1] * rbl1), (int)rbm, 1.0,
                     (const double*)b->cores[q], rbm, 0, (const double*)b->cores[q + 1], d[q + 1] * rbl1, 0, 0.0,
                     ws + F.offBp, d[q + 1] * rbl1, 0, 1));
    bl = ws + F.offBp;
  }
  QTT_HIP(local_matrix(st, ws + F.offLW[q], Wl, ws + F.offRW[q + nc], (int)r0, (int)P, (int)r1, (int)w0, (int)w1, A));
  QTT_HIP(fit_project(st, ws + F.offLb[q], bl, ws + F.offRb[q + nc], r0, r1, rbl0, rbl1, P, ws + F.offT, rhs));
  QTT_HIP(chol_solve(st, A, (int)N, N, rhs, ws + F.offChol));
  return QTT_OK;
}

int solve_sweeps(qtt_context* h, hipStream_t st, double* ws, const SolvePlan& F, const qtt_tt* w, const qtt_tt* b,
                 qtt_tt* x, std::vector<long>& rc, int nsweeps, double rel_tol, long max_rank, int& maxsw) {
  const int n = x->n;
  std::vector<int> d(n);
  for (int k = 0; k < n; ++k) d[k] = dphys(x, k);
  auto core = [&](int k) { return (double*)x->cores[k]; };
  auto W = [&](int k) { return (const double*)w->cores[k]; };
  auto B = [&](int k) { return (const double*)b->cores[k]; };
  double* E1 = ws + F.offE1;
  double* E2 = ws + F.offE2;
  double* T = ws + F.offT;
  double* sol = ws + F.offRhs;
  auto lw_step = [&](int k) -> int {
    QTT_HIP(env3_left(st, ws + F.offLW[k], core(k), W(k), rc[k], d[k], rc[k + 1], F.rw[k], F.rw[k + 1], E1, E2,
                      ws + F.offLW[k + 1]));
    QTT_HIP(env_step_left<double>(st, ws + F.offLb[k], core(k), B(k), rc[k], rc[k + 1], F.rb[k], F.rb[k + 1], d[k],
                                  T, ws + F.offLb[k + 1]));
    return QTT_OK;
  };
  auto rw_step = [&](int k) -> int {
    QTT_HIP(env3_right(st, ws + F.offRW[k + 1], core(k), W(k), rc[k], d[k], rc[k + 1], F.rw[k], F.rw[k + 1], E1, E2,
                       ws + F.offRW[k]));
    QTT_HIP(env_step_right<double>(st, ws + F.offRb[k + 1], core(k), B(k), rc[k], rc[k + 1], F.rb[k], F.rb[k + 1],
                                   d[k], T, ws + F.offRb[k]));
    return QTT_OK;
  };
  QTT_HIP(fill_f64(st, ws + F.offLW[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offLb[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offRW[n], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offRb[n], 1.0, 1));
  int e;
  for (int k = 0; k + F.nc < n; ++k)
    if ((e = lw_step(k))) return e;
  maxsw = 0;
  for (int sw = 0; sw < nsweeps; ++sw) {
    if (F.nc == 1) {
      // right to left: solve, then the solved core's transpose QR gives a right-orthonormal core
      for (int q = n - 1; q >= 0; --q) {
        if ((e = solve_local(st, ws, F, w, b, rc, d, q))) return e;
        if (q > 0) {
          const int m = (int)(d[q] * rc[q + 1]), nn = (int)rc[q], qq = std::min(m, nn);
          double* G = ws + F.offGt;
          double* Qe = ws + F.offQe;
          QTT_HIP(transpose(st, sol, nn, m, m, G, nn));
          QTT_HIP(householder_qr(st, G, m, nn, nn, ws + F.offTq, ws + F.offScr));
          QTT_HIP(set_eye_rect(st, Qe, m, qq));
          QTT_HIP(apply_q(st, G, m, qq, nn, ws + F.offTq, Qe, qq, qq, false, ws + F.offScr));
          QTT_HIP(transpose(st, Qe, m, qq, qq, core(q), m));
          rc[q] = qq;
          if ((e = rw_step(q))) return e;
        } else {
          QTT_HIP(copy_pad_rows(st, sol, (int)(d[0] * rc[1]), 1, 1, core(0), (int)(d[0] * rc[1]), 1));
          if ((e = rw_step(0))) return e;
        }
      }
      // left to right: solve, then a QR of the solved core gives a left-orthonormal core
      for (int q = 0; q < n; ++q) {
        if ((e = solve_local(st, ws, F, w, b, rc, d, q))) return e;
        if (q < n - 1) {
          const int m = (int)(rc[q] * d[q]), nn = (int)rc[q + 1], qq = std::min(m, nn);
          double* Qe = ws + F.offQe;
          QTT_HIP(householder_qr(st, sol, m, nn, nn, ws + F.offTq, ws + F.offScr));
          QTT_HIP(set_eye_rect(st, Qe, m, qq));
          QTT_HIP(apply_q(st, sol, m, qq, nn, ws + F.offTq, Qe, qq, qq, false, ws + F.offScr));
          QTT_HIP(copy_pad_rows(st, Qe, m, qq, qq, core(q), m, qq));
          rc[q + 1] = qq;
          if ((e = lw_step(q))) return e;
        } else {
          QTT_HIP(copy_pad_rows(st, sol, (int)(rc[q] * d[q]), 1, 1, core(q), (int)(rc[q] * d[q]), 1));
        }
      }
    } else {
      double* S = ws + F.offS;
      double* St = ws + F.offSt;
      double* V = ws + F.offV;
      double* MV = ws + F.offMV;
      const SplitBufs bf = solve_bufs(ws, F);
      for (int q = n - 2; q >= 0; --q) {  // pairs from the right end: core q+1 <- V^T, core q <- U Sigma
        if ((e = solve_local(st, ws, F, w, b, rc, d, q))) return e;
        const long m = rc[q] * d[q], cols = (long)d[q + 1] * rc[q + 2];
        QTT_HIP(copy_pad_rows(st, sol, (int)m, (int)cols, cols, S, (int)m, cols));
        int rn = 0, swp = 0;
        double tail = 0.0;
        if ((e = split_rows(h, st, bf, S, (int)m, (int)cols, rel_tol, n - 1, max_rank, V, MV, rn, tail, swp)))
          return e;
        if (rn > F.bnd[q + 1]) return QTT_ERR_UNSUPPORTED;
        maxsw = std::max(maxsw, swp);
        QTT_HIP(copy_pad_rows(st, V, rn, (int)cols, cols, core(q + 1), rn, cols));
        QTT_HIP(copy_pad_rows(st, MV, (int)m, rn, rn, core(q), (int)m, rn));
        rc[q + 1] = rn;
        if ((e = rw_step(q + 1))) return e;
      }
      for (int q = 0; q + 1 < n; ++q) {  // and back: core q <- U, core q+1 <- Sigma V^T
        if ((e = solve_local(st, ws, F, w, b, rc, d, q))) return e;
        const long m = rc[q] * d[q], cols = (long)d[q + 1] * rc[q + 2];
        QTT_HIP(transpose(st, sol, (int)m, (int)cols, cols, St, m));
        int rn = 0, swp = 0;
        double tail = 0.0;
        if ((e = split_rows(h, st, bf, St, (int)cols, (int)m, rel_tol, n - 1, max_rank, V, MV, rn, tail, swp)))
          return e;
        if (rn > F.bnd[q + 1]) return QTT_ERR_UNSUPPORTED;
        maxsw = std::max(maxsw, swp);
        QTT_HIP(transpose(st, V, rn, (int)m, m, core(q), rn));
        QTT_HIP(transpose(st, MV, (int)cols, rn, rn, core(q + 1), cols));
        rc[q + 1] = rn;
        if ((e = lw_step(q))) return e;
      }
    }
  }
  QTT_HIP(frob_norm(st, core(n - 1), rc[n - 1] * d[n - 1], ws + F.offNrm));
  return QTT_OK;
}

// ---------------------------------------------------------------- AMEn solver
// AMEn (Sec. 5, single-core sweeps with gradient enrichment): the one-core
// energy minimisation of the DMRG-like solver, then per step a truncated SVD
// of the solved core, the projection of the residual r = b - W x onto the
// frames of a second train z (z's new core) and onto z's frame on the side
// the sweep moves from and x's frame on the other (the enrichment core e).
// x's new core is the orthonormal basis of the rows of [V^T; e / s] and z's
// that of its projection (Jacobi SVD, directions whose discarded singular
// values have 2-norm <= kAmenSpanTol dropped, s = ||projected b|| +
// ||projected W x||): the projected residual has exactly null directions
// where the frames of x and z overlap, and a QR would complete them
// arbitrarily.  The factor the method absorbs into the next core is not
// formed: the next local solve replaces that core before anything reads it.
constexpr double kAmenSpanTol = 1e-10;

struct AmenPlan {
  SolvePlan S;               // x's environments, the local solve and the splits
  std::vector<long> bz;      // z's rank bounds
  std::vector<long> offLzW, offRzW, offLzb, offRzb;
  long offXt = 0, offZc = 0, offEn = 0, offWx = 0, offU1 = 0, offU2 = 0, offRE = 0, offRz = 0, offScale = 0,
       offOne = 0;
  long total = 0;
};

int amen_check(const qtt_tt* w, const qtt_tt* b, const qtt_tt* x, const qtt_tt* z) {
  int st = solve_check(w, b, x);
  if (st) return st;
  if ((st = check_tt(z, 1))) return st;
  if (z->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if (z->n != x->n) return QTT_ERR_SHAPE;
  for (int k = 0; k < x->n; ++k)
    if (dphys(z, k) != dphys(x, k)) return QTT_ERR_SHAPE;
  return QTT_OK;
}

// Rank bounds: z's ranks never grow past those of its left-orthogonalised
// guess; a bond of x holds at most the truncated rank (<= max_rank) plus
// z's rank, never more than the larger of its unfolding sizes (a pass
// moving right bounds it by the left one, a pass moving left by the right
// one), and at least what the orthogonalised guess had.
int make_amen_plan(const qtt_tt* w, const qtt_tt* b, const qtt_tt* x, const qtt_tt* z, long max_rank, AmenPlan& F) {
  const int n = x->n;
  SolvePlan& S = F.S;
  S.nc = 1;
  S.bnd.assign(n + 1, 1);
  S.rw.assign(n + 1, 1);
  S.rb.assign(n + 1, 1);
  F.bz.assign(n + 1, 1);
  std::vector<long> left(n + 1, 1), right(n + 1, 1);
  std::vector<int> d(n);
  for (int k = 0; k < n; ++k) d[k] = dphys(x, k);
  for (int k = 1; k <= n; ++k) left[k] = std::min<long>(left[k - 1] * d[k - 1], 1L << 40);
  for (int k = n - 1; k >= 0; --k) right[k] = std::min<long>(right[k + 1] * d[k], 1L << 40);
  const long cap = max_rank > 0 ? max_rank : (1L << 40);
  for (int k = 0; k <= n; ++k) {
    S.rw[k] = w->ranks[k];
    S.rb[k] = b->ranks[k];
    F.bz[k] = std::max(1L, std::min<long>(left[k], z->ranks[k]));
    const long g = std::min<long>(left[k], x->ranks[k]);
    long v = (k == 0 || k == n) ? 1 : std::min(std::max(left[k], right[k]), std::max(g, cap + F.bz[k]));
    S.bnd[k] = std::max(v, 1L);
  }
  const std::vector<long>& B = S.bnd;
  const std::vector<long>& Z = F.bz;
  long off = 0;
  auto take = [&](long cnt) {
    long o = off;
    off += round_up(std::max(cnt, 1L), 32);
    return o;
  };
  S.offLW.assign(n + 1, 0);
  S.offRW.assign(n + 1, 0);
  S.offLb.assign(n + 1, 0);
  S.offRb.assign(n + 1, 0);
  F.offLzW.assign(n + 1, 0);
  F.offRzW.assign(n + 1, 0);
  F.offLzb.assign(n + 1, 0);
  F.offRzb.assign(n + 1, 0);
  for (int k = 0; k <= n; ++k) {
    S.offLW[k] = take(B[k] * S.rw[k] * B[k]);
    S.offRW[k] = take(B[k] * S.rw[k] * B[k]);
    S.offLb[k] = take(B[k] * S.rb[k]);
    S.offRb[k] = take(B[k] * S.rb[k]);
    F.offLzW[k] = take(Z[k] * S.rw[k] * B[k]);
    F.offRzW[k] = take(Z[k] * S.rw[k] * B[k]);
    F.offLzb[k] = take(Z[k] * S.rb[k]);
    F.offRzb[k] = take(Z[k] * S.rb[k]);
  }
  long maxN = 1, maxT = 1, maxE = 1, maxU = 1, maxSplit = 1, maxTB = 1, maxX = 1, maxP = 1, maxc = 1;
  long maxXt = 1, maxZc = 1, maxRE = 1;
  // one Jacobi split of a p0 x L row matrix (its buffers)
  auto split_need = [&](long p0, long L) -> int {
    if (L > 1024 || p0 > kMaxRows) return QTT_ERR_UNSUPPORTED;
    const long p = std::min(p0, L);
    maxSplit = std::max(maxSplit, p0 * L);
    maxTB = std::max(maxTB, qr_t_doubles((int)p0, (int)p));
    maxX = std::max(maxX, p * L);
    maxP = std::max(maxP, p);
    maxc = std::max({maxc, L, p0});
    return QTT_OK;
  };
  for (int k = 0; k < n; ++k) {
    const long r0 = B[k], r1 = B[k + 1], z0 = Z[k], z1 = Z[k + 1], w0 = S.rw[k], w1 = S.rw[k + 1], dk = d[k];
    const long N = r0 * dk * r1;
    maxN = std::max(maxN, N);
    maxXt = std::max(maxXt, N);
    maxT = std::max(maxT, std::max(r0, z0) * dk * std::max({S.rb[k + 1], r1, z1}));
    // three-layer steps (bra x or z, ket x) and the residual projections
    maxE = std::max({maxE, std::max(r0, z0) * w0 * dk * r1, std::max(r0, z0) * dk * w1 * r1});
    maxU = std::max({maxU, r0 * dk * std::max(r1, z1) * w1, dk * std::max(r1, z1) * w0 * r0});
    maxZc = std::max({maxZc, z0 * dk * z1, z0 * dk * r1, r0 * dk * z1});
    int e;
    const long mL = dk * r1, mR = r0 * dk;
    if (k > 0) {  // moving left: truncation (r0) x (d r1), bases [V; e] (<= r0 + z0 rows) and z (z0 rows)
      const long cL = std::min(r0, mL) + z0;
      if ((e = split_need(r0, mL)) || (e = split_need(cL, mL)) || (e = split_need(z0, dk * z1))) return e;
      maxRE = std::max(maxRE, cL * mL);
    }
    if (k < n - 1) {  // moving right: the transposed forms, (r1) x (r0 d), [U, e]^T, z^T
      const long cR = std::min(r1, mR) + z1;
      if ((e = split_need(r1, mR)) || (e = split_need(cR, mR)) || (e = split_need(z1, z0 * dk))) return e;
      maxRE = std::max(maxRE, cR * mR);
    }
  }
  if (maxN > kMaxRows) return QTT_ERR_UNSUPPORTED;  // the local QR solve
  maxE = std::max(maxE, maxU);  // right steps with z as bra use the same buffers
  S.offA = take(maxN * maxN);
  S.offRhs = take(maxN);
  S.offT = take(maxT);
  S.offE1 = take(maxE);
  S.offE2 = take(maxE);
  S.offChol = take(chol_work_doubles(maxN));
  S.offS = take(maxSplit);
  S.offSt = take(maxSplit);
  S.offV = take(maxX);
  S.offMV = take(maxSplit);
  S.offTB = take(maxTB);
  S.offX = take(maxX);
  S.offXc = take(maxX);
  S.offYt = take(maxX);
  S.offSig = take(maxP);
  S.offPerm = take(maxP / 2 + 1);
  S.offTrunc = take(8);
  S.offCtr = take(96);
  S.offSweeps = take(1);
  S.offNrm = take(1);
  S.offScr = take(qr_scratch_doubles(maxc));
  F.offXt = take(maxXt);
  F.offZc = take(maxZc);
  F.offEn = take(maxZc);
  F.offWx = take(maxZc);
  F.offU1 = take(maxU);
  F.offU2 = take(maxU);
  F.offRE = take(maxRE);
  F.offRz = take(maxZc);
  F.offScale = take(4);
  F.offOne = take(1);
  F.total = S.total = off;
  return QTT_OK;
}

// Three-layer environment steps with bra u (ranks ru0, ru1) and ket v
// (rv0, rv1): LW' = sum u^T LW W v (left, LW: ru0 x w0 x rv0) and
// RW = sum u W v RW' (right, RW': ru1 x w1 x rv1).
hipError_t env3_left_bk(hipStream_t st, const double* LW, const double* u, const double* v, const double* W, long ru0,
                        long ru1, long rv0, long rv1, long d, long w0, long w1, double* T1, double* T2, double* out) {
  hipError_t e = gemm_f64(st, false, false, (int)(ru0 * w0), (int)(d * rv1), (int)rv0, 1.0, LW, rv0, 0, v, d * rv1,
                          0, 0.0, T1, d * rv1, 0, 1);
  if (e != hipSuccess) return e;
  if ((e = env3_left_mid(st, T1, W, (int)ru0, (int)w0, (int)d, (int)w1, (int)rv1, T2)) != hipSuccess) return e;
  return gemm_f64(st, true, false, (int)ru1, (int)(w1 * rv1), (int)(ru0 * d), 1.0, u, ru1, 0, T2, w1 * rv1, 0, 0.0,
                  out, w1 * rv1, 0, 1);
}

hipError_t env3_right_bk(hipStream_t st, const double* RW, const double* u, const double* v, const double* W, long ru0,
                         long ru1, long rv0, long rv1, long d, long w0, long w1, double* U1, double* U2, double* out) {
  hipError_t e = gemm_f64(st, false, true, (int)(rv0 * d), (int)(ru1 * w1), (int)rv1, 1.0, v, rv1, 0, RW, rv1, 0,
                          0.0, U1, ru1 * w1, 0, 1);
  if (e != hipSuccess) return e;
  if ((e = env3_right_mid(st, U1, W, (int)rv0, (int)w0, (int)d, (int)w1, (int)ru1, U2)) != hipSuccess) return e;
  return gemm_f64(st, false, false, (int)ru0, (int)(w0 * rv0), (int)(d * ru1), 1.0, u, d * ru1, 0, U2, w0 * rv0, 0,
                  0.0, out, w0 * rv0, 0, 1);
}

// out[a][i][c] = (Lb b_q Rb^T)[a][i][c] - sum LW[a][al][x] W[al][i][j][be] v[x][j][y] RW[c][be][y]:
// the projection of b - W x onto a left frame (ra0 columns, environments
// LW, Lb) and a right frame (rc1 rows, environments RW, Rb), x's core q = v
// (rv0 x d x rv1); norms[0], norms[1] (device) receive the Frobenius norms
// of the two terms.  wx: scratch of ra0 d rc1.
hipError_t residual_project(hipStream_t st, const double* LW, const double* RW, const double* Lb, const double* Rb,
                            const double* W, const double* bq, const double* v, long ra0, long rc1, long rv0,
                            long rv1, long rb0, long rb1, long d, long w0, long w1, double* T, double* U1,
                            double* U2, double* wx, double* out, double* norms) {
  hipError_t e = fit_project(st, Lb, bq, Rb, ra0, rc1, rb0, rb1, d, T, out);
  if (e != hipSuccess) return e;
  if ((e = gemm_f64(st, false, true, (int)(rv0 * d), (int)(rc1 * w1), (int)rv1, 1.0, v, rv1, 0, RW, rv1, 0, 0.0, U1,
                    rc1 * w1, 0, 1)) != hipSuccess)
    return e;
  if ((e = env3_right_mid(st, U1, W, (int)rv0, (int)w0, (int)d, (int)w1, (int)rc1, U2)) != hipSuccess) return e;
  if ((e = gemm_f64(st, false, true, (int)ra0, (int)(d * rc1), (int)(w0 * rv0), 1.0, LW, w0 * rv0, 0, U2, w0 * rv0,
                    0, 0.0, wx, d * rc1, 0, 1)) != hipSuccess)
    return e;
  const long cnt = ra0 * d * rc1;
  if ((e = frob_norm(st, out, cnt, norms)) != hipSuccess) return e;
  if ((e = frob_norm(st, wx, cnt, norms + 1)) != hipSuccess) return e;
  return axpy_f64(st, cnt, -1.0, wx, out);
}

int amen_sweeps(qtt_context* h, hipStream_t st, double* ws, const AmenPlan& F, const qtt_tt* w, const qtt_tt* b,
                qtt_tt* x, qtt_tt* z, std::vector<long>& rc, std::vector<long>& rz, int nsweeps, double rel_tol,
                long max_rank, int& maxsw) {
  const SolvePlan& S = F.S;
  const int n = x->n;
  std::vector<int> d(n);
  for (int k = 0; k < n; ++k) d[k] = dphys(x, k);
  auto X = [&](int k) { return (double*)x->cores[k]; };
  auto Zc = [&](int k) { return (double*)z->cores[k]; };
  auto W = [&](int k) { return (const double*)w->cores[k]; };
  auto B = [&](int k) { return (const double*)b->cores[k]; };
  double* E1 = ws + S.offE1;
  double* E2 = ws + S.offE2;
  double* T = ws + S.offT;
  double* sol = ws + S.offRhs;
  double* xt = ws + F.offXt;
  double* zc = ws + F.offZc;
  double* en = ws + F.offEn;
  double* RE = ws + F.offRE;
  double* Rz = ws + F.offRz;
  double* U1 = ws + F.offU1;
  double* U2 = ws + F.offU2;
  double* sc = ws + F.offScale;  // [0..1] scale terms of e, [2..3] of z's projection
  const double* one = ws + F.offOne;
  double* Sm = ws + S.offS;
  double* St = ws + S.offSt;
  double* V = ws + S.offV;
  double* MV = ws + S.offMV;
  const SplitBufs bf = solve_bufs(ws, S);
  const long* rw = S.rw.data();
  const long* rb = S.rb.data();
  // environments of x (bra = ket = x) and of z against x and b, one core on
  auto left_step = [&](int k) -> int {
    QTT_HIP(env3_left_bk(st, ws + S.offLW[k], X(k), X(k), W(k), rc[k], rc[k + 1], rc[k], rc[k + 1], d[k], rw[k],
                         rw[k + 1], E1, E2, ws + S.offLW[k + 1]));
    QTT_HIP(env_step_left<double>(st, ws + S.offLb[k], X(k), B(k), rc[k], rc[k + 1], rb[k], rb[k + 1], d[k], T,
                                  ws + S.offLb[k + 1]));
    QTT_HIP(env3_left_bk(st, ws + F.offLzW[k], Zc(k), X(k), W(k), rz[k], rz[k + 1], rc[k], rc[k + 1], d[k], rw[k],
                         rw[k + 1], E1, E2, ws + F.offLzW[k + 1]));
    QTT_HIP(env_step_left<double>(st, ws + F.offLzb[k], Zc(k), B(k), rz[k], rz[k + 1], rb[k], rb[k + 1], d[k], T,
                                  ws + F.offLzb[k + 1]));
    return QTT_OK;
  };
  auto right_step = [&](int k) -> int {
    QTT_HIP(env3_right_bk(st, ws + S.offRW[k + 1], X(k), X(k), W(k), rc[k], rc[k + 1], rc[k], rc[k + 1], d[k], rw[k],
                          rw[k + 1], E1, E2, ws + S.offRW[k]));
    QTT_HIP(env_step_right<double>(st, ws + S.offRb[k + 1], X(k), B(k), rc[k], rc[k + 1], rb[k], rb[k + 1], d[k], T,
                                   ws + S.offRb[k]));
    QTT_HIP(env3_right_bk(st, ws + F.offRzW[k + 1], Zc(k), X(k), W(k), rz[k], rz[k + 1], rc[k], rc[k + 1], d[k],
                          rw[k], rw[k + 1], E1, E2, ws + F.offRzW[k]));
    QTT_HIP(env_step_right<double>(st, ws + F.offRzb[k + 1], Zc(k), B(k), rz[k], rz[k + 1], rb[k], rb[k + 1], d[k], T,
                                   ws + F.offRzb[k]));
    return QTT_OK;
  };
  // projection of the residual with x's core q = v onto the frames given by
  // their environments (left: z or x, right: z or x); norms: its two terms
  auto project = [&](int q, bool zleft, bool zright, const double* v, double* out, double* norms) -> int {
    const long ra0 = zleft ? rz[q] : rc[q], rc1 = zright ? rz[q + 1] : rc[q + 1];
    QTT_HIP(residual_project(st, ws + (zleft ? F.offLzW[q] : S.offLW[q]),
                             ws + (zright ? F.offRzW[q + 1] : S.offRW[q + 1]), ws + (zleft ? F.offLzb[q] : S.offLb[q]),
                             ws + (zright ? F.offRzb[q + 1] : S.offRb[q + 1]), W(q), B(q), v, ra0, rc1, rc[q],
                             rc[q + 1], rb[q], rb[q + 1], d[q], rw[q], rw[q + 1], T, U1, U2, ws + F.offWx, out,
                             norms));
    return QTT_OK;
  };
  // orthonormal rows spanning the rows of M (p0 x L, overwritten): Jacobi
  // SVD, directions with discarded tail <= kAmenSpanTol dropped -> V (k x L)
  auto span_rows = [&](double* M, int p0, int L, int& k) -> int {
    int swp = 0;
    double tail = 0.0;
    int e = split_rows(h, st, bf, M, p0, L, kAmenSpanTol, 1, 0, V, MV, k, tail, swp, one);
    maxsw = std::max(maxsw, swp);
    return e;
  };
  QTT_HIP(fill_f64(st, ws + F.offOne, 1.0, 1));
  QTT_HIP(fill_f64(st, ws + S.offLW[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + S.offLb[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offLzW[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offLzb[0], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + S.offRW[n], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + S.offRb[n], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offRzW[n], 1.0, 1));
  QTT_HIP(fill_f64(st, ws + F.offRzb[n], 1.0, 1));
  int e;
  for (int k = 0; k + 1 < n; ++k)
    if ((e = left_step(k))) return e;
  maxsw = 0;
  for (int sw = 0; sw < nsweeps; ++sw) {
    for (int q = n - 1; q >= 0; --q) {  // right to left
      if ((e = solve_local(st, ws, S, w, b, rc, d, q))) return e;
      const long r0 = rc[q], r1 = rc[q + 1], m = d[q] * r1;
      if (q == 0) {
        QTT_HIP(copy_pad_rows(st, sol, 1, (int)m, m, X(0), 1, m));
        if ((e = project(0, true, true, sol, Zc(0), sc + 2))) return e;
        break;
      }
      // truncated split of the (r0) x (d r1) unfolding: V (rn x m) rows, MV = U S (r0 x rn)
      QTT_HIP(copy_pad_rows(st, sol, (int)r0, (int)m, m, Sm, (int)r0, m));
      int rn = 0, swp = 0;
      double tail = 0.0;
      if ((e = split_rows(h, st, bf, Sm, (int)r0, (int)m, rel_tol, n - 1, max_rank, V, MV, rn, tail, swp))) return e;
      maxsw = std::max(maxsw, swp);
      QTT_HIP(gemm_f64(st, false, false, (int)r0, (int)m, rn, 1.0, MV, rn, 0, V, m, 0, 0.0, xt, m, 0, 1));
      const long z0 = rz[q], z1 = rz[q + 1];
      if ((e = project(q, true, true, xt, zc, sc + 2))) return e;  // z's projection (z0 x d x z1)
      if ((e = project(q, true, false, xt, en, sc))) return e;     // enrichment (z0 x d x r1)
      // x's core: orthonormal rows spanning [V; en / s] ((rn + z0) x m)
      const int c = rn + (int)z0;
      QTT_HIP(copy_pad_rows(st, V, rn, (int)m, m, RE, rn, m));
      QTT_HIP(copy_scaled_inv(st, en, (int)z0, (int)m, m, sc, RE + (long)rn * m, m));
      int qq = 0;
      if ((e = span_rows(RE, c, (int)m, qq))) return e;
      if (qq > S.bnd[q]) return QTT_ERR_UNSUPPORTED;
      QTT_HIP(copy_pad_rows(st, V, qq, (int)m, m, X(q), qq, m));
      // z's core: orthonormal rows spanning its projection / s (z0 x d z1)
      const int mz = (int)(d[q] * z1);
      QTT_HIP(copy_scaled_inv(st, zc, (int)z0, mz, mz, sc + 2, Rz, mz));
      int qz = 0;
      if ((e = span_rows(Rz, (int)z0, mz, qz))) return e;
      QTT_HIP(copy_pad_rows(st, V, qz, mz, mz, Zc(q), qz, mz));
      rc[q] = qq;
      rz[q] = qz;
      if ((e = right_step(q))) return e;
    }
    for (int q = 0; q < n; ++q) {  // and back
      if ((e = solve_local(st, ws, S, w, b, rc, d, q))) return e;
      const long r0 = rc[q], r1 = rc[q + 1], m = r0 * d[q];
      if (q == n - 1) {
        QTT_HIP(copy_pad_rows(st, sol, (int)m, 1, 1, X(q), (int)m, 1));
        if ((e = project(q, true, true, sol, Zc(q), sc + 2))) return e;
        break;
      }
      // truncated split of the (r0 d) x r1 unfolding through its transpose:
      // V (rn x m) = U^T, MV (r1 x rn) = V S
      QTT_HIP(transpose(st, sol, (int)m, (int)r1, r1, St, m));
      int rn = 0, swp = 0;
      double tail = 0.0;
      if ((e = split_rows(h, st, bf, St, (int)r1, (int)m, rel_tol, n - 1, max_rank, V, MV, rn, tail, swp))) return e;
      maxsw = std::max(maxsw, swp);
      QTT_HIP(gemm_f64(st, true, true, (int)m, (int)r1, rn, 1.0, V, m, 0, MV, rn, 0, 0.0, xt, r1, 0, 1));
      const long z0 = rz[q], z1 = rz[q + 1];
      if ((e = project(q, true, true, xt, zc, sc + 2))) return e;  // z's projection (z0 x d x z1)
      if ((e = project(q, false, true, xt, en, sc))) return e;     // enrichment (r0 x d x z1)
      // x's core: orthonormal columns spanning [U, en / s] (m x (rn + z1)), as rows
      const int c = rn + (int)z1;
      QTT_HIP(copy_pad_rows(st, V, rn, (int)m, m, RE, rn, m));
      QTT_HIP(transpose(st, en, (int)m, (int)z1, z1, RE + (long)rn * m, m));
      QTT_HIP(copy_scaled_inv(st, RE + (long)rn * m, (int)z1, (int)m, m, sc, RE + (long)rn * m, m));
      int qq = 0;
      if ((e = span_rows(RE, c, (int)m, qq))) return e;
      if (qq > S.bnd[q + 1]) return QTT_ERR_UNSUPPORTED;
      QTT_HIP(transpose(st, V, qq, (int)m, m, X(q), qq));
      // z's core: orthonormal columns spanning its projection / s ((z0 d) x z1)
      const int mz = (int)(z0 * d[q]);
      QTT_HIP(transpose(st, zc, mz, (int)z1, z1, Rz, mz));
      QTT_HIP(copy_scaled_inv(st, Rz, (int)z1, mz, mz, sc + 2, Rz, mz));
      int qz = 0;
      if ((e = span_rows(Rz, (int)z1, mz, qz))) return e;
      QTT_HIP(transpose(st, V, qz, mz, mz, Zc(q), qz));
      rc[q + 1] = qq;
      rz[q + 1] = qz;
      if ((e = left_step(q))) return e;
    }
  }
  QTT_HIP(frob_norm(st, X(n - 1), rc[n - 1] * d[n - 1], ws + S.offNrm));
  return QTT_OK;
}

int fit_setup(const char* spec, const qtt_tt* a, const qtt_tt* b, const qtt_tt* c, Shape& s, FitPlan& F,
              size_t& orth_bytes) {
  int st = shape_from_pair(spec, a, b, s);
  if (st) return st;
  if (a->dtype != QTT_F64 || b->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if ((st = check_tt(c, 1))) return st;
  if (c->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if (c->n != s.n) return QTT_ERR_SHAPE;
  for (int k = 0; k < s.n; ++k)
    if (dphys(c, k) != s.d[k]) return QTT_ERR_SHAPE;
  Shape sc;
  shape_from_tt(c, sc);
  Plan P;
  if ((st = make_plan(sc, 0, P, false))) return st;
  orth_bytes = ws_bytes_of(P);
  return make_fit_plan(s, c, F);
}

}  // namespace

extern "C" {

const char* qtt_status_string(int status) {
  switch (status) {
    case QTT_OK: return "ok";
    case QTT_ERR_ARG: return "invalid argument";
    case QTT_ERR_SPEC: return "unsupported einsum specification";
    case QTT_ERR_SHAPE: return "shape mismatch";
    case QTT_ERR_DTYPE: return "unsupported dtype";
    case QTT_ERR_WORKSPACE: return "workspace too small";
    case QTT_ERR_NODEVICE: return "no gfx950 HIP device";
    case QTT_ERR_HIP: return "HIP runtime error";
    case QTT_ERR_NONFINITE: return "non-finite value";
    case QTT_ERR_NOCONV: return "Jacobi SVD did not converge";
    case QTT_ERR_UNSUPPORTED: return "size outside the implemented range";
    default: return "unknown status";
  }
}

int qtt_create(qtt_handle* h, int device) {
  if (!h) return QTT_ERR_ARG;
  *h = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return QTT_ERR_NODEVICE;
  if (device < 0 || device >= count) return QTT_ERR_NODEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return QTT_ERR_NODEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QTT_ERR_NODEVICE;
  Scoped sc(device);
  // kernels with more than 64 KiB of dynamic LDS get their limit raised on
  // this device before any launch
  if (configure_kernels() != hipSuccess) return QTT_ERR_HIP;
  qtt_context* c = new (std::nothrow) qtt_context();
  if (!c) return QTT_ERR_ARG;
  c->device = device;
  c->max_sweeps = kMaxSweeps;
  if (scratch_address(device, &c->scratch) != hipSuccess) {
    delete c;
    return QTT_ERR_HIP;
  }
  if (hipHostMalloc((void**)&c->pin_trunc, sizeof(TruncOut), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->pin_int, 64, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->pin_dbl, 64, hipHostMallocDefault) != hipSuccess) {
    if (c->pin_trunc) (void)hipHostFree(c->pin_trunc);
    if (c->pin_int) (void)hipHostFree(c->pin_int);
    if (c->pin_dbl) (void)hipHostFree(c->pin_dbl);
    delete c;
    return QTT_ERR_HIP;
  }
  *h = c;
  return QTT_OK;
}

int qtt_destroy(qtt_handle h) {
  if (!h) return QTT_ERR_ARG;
  Scoped sc(h->device);
  (void)hipHostFree(h->pin_trunc);
  (void)hipHostFree(h->pin_int);
  (void)hipHostFree(h->pin_dbl);
  delete h;
  return QTT_OK;
}

int qtt_set_jacobi_max_sweeps(qtt_handle h, int32_t max_sweeps) {
  if (!h || max_sweeps < 0 || max_sweeps > 100000) return QTT_ERR_ARG;
  h->max_sweeps = max_sweeps == 0 ? kMaxSweeps : max_sweeps;
  return QTT_OK;
}

int qtt_workspace_size(qtt_handle h, int op, const char* spec, const qtt_tt* a, const qtt_tt* b, int64_t max_rank,
                       int prec, size_t* bytes) {
  (void)h;  // pure shape arithmetic: a NULL handle is accepted
  if (!bytes) return QTT_ERR_ARG;
  *bytes = 0;
  int st;
  switch (op) {
    case QTT_OP_CONTRACT:
    case QTT_OP_CONTRACT_BACKWARD:
      *bytes = 0;
      return QTT_OK;
    case QTT_OP_ORTHOGONALIZE:
    case QTT_OP_ROUND: {
      if ((st = check_tt(a, 1))) return st;
      Shape s;
      shape_from_tt(a, s);
      Plan P;
      if ((st = make_plan(s, op == QTT_OP_ROUND ? max_rank : 0, P, op == QTT_OP_ROUND))) return st;
      *bytes = ws_bytes_of(P);
      return QTT_OK;
    }
    case QTT_OP_CONTRACT_ROUND: {
      Shape s;
      if ((st = shape_from_pair(spec, a, b, s))) return st;
      Plan P;
      if ((st = make_plan(s, max_rank, P))) return st;
      *bytes = ws_bytes_of(P);
      return QTT_OK;
    }
    case QTT_OP_INNER: {
      if ((st = check_tt(a, 1)) || (st = check_tt(b, 1))) return st;
      *bytes = (size_t)inner_plan(a, b).total * 8 + 256;
      return QTT_OK;
    }
    case QTT_OP_INNER_BACKWARD: {
      if ((st = check_tt(a, 1)) || (st = check_tt(b, 1))) return st;
      *bytes = (size_t)env_plan(a, b).total * 8 + 256;
      return QTT_OK;
    }
    default:
      return QTT_ERR_ARG;
  }
  (void)prec;
}

static int contract_opop(qtt_handle h, const qtt_tt* a, const qtt_tt* b, qtt_tt* c, void* stream) {
  int st;
  if ((st = check_tt(a, 2)) || (st = check_tt(b, 2)) || (st = check_tt(c, 2))) return st;
  const int n = a->n;
  if (b->n != n || c->n != n) return QTT_ERR_SHAPE;
  if (a->dtype != b->dtype || c->dtype != a->dtype) return QTT_ERR_SHAPE;
  for (int k = 0; k < n; ++k) {
    if (dphys_in(a, k) != dphys(b, k)) return QTT_ERR_SHAPE;
    if (dphys(c, k) != dphys(a, k) || dphys_in(c, k) != dphys_in(b, k)) return QTT_ERR_SHAPE;
  }
  for (int k = 0; k <= n; ++k)
    if (c->ranks[k] != a->ranks[k] * b->ranks[k]) return QTT_ERR_SHAPE;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  for (int k = 0; k < n; ++k) {
    const int ra0 = (int)a->ranks[k], ra1 = (int)a->ranks[k + 1], rb0 = (int)b->ranks[k], rb1 = (int)b->ranks[k + 1];
    const int di = dphys(a, k), dj = dphys_in(a, k), dk = dphys_in(b, k);
    hipError_t e;
    if (a->dtype == QTT_F64)
      e = contract_mpo_mpo<double>(strm, (const double*)a->cores[k], ra0, di, dj, ra1, (const double*)b->cores[k],
                                   rb0, dk, rb1, (double*)c->cores[k]);
    else
      e = contract_mpo_mpo<float>(strm, (const float*)a->cores[k], ra0, di, dj, ra1, (const float*)b->cores[k], rb0,
                                  dk, rb1, (float*)c->cores[k]);
    if (e != hipSuccess) return QTT_ERR_HIP;
  }
  return QTT_OK;
}

int qtt_contract(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* c, void* ws,
                 size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (!h) return QTT_ERR_ARG;
  {
    Kind kind;
    const int st = parse_spec(spec, kind);
    if (st) return st;
    if (kind == K_OPOP) return contract_opop(h, a, b, c, stream);
  }
  Shape s;
  int st = shape_from_pair(spec, a, b, s);
  if (st) return st;
  if ((st = check_tt(c, 1))) return st;
  if (c->n != a->n || a->dtype != b->dtype || c->dtype != a->dtype) return QTT_ERR_SHAPE;
  for (int k = 0; k <= a->n; ++k)
    if (c->ranks[k] != a->ranks[k] * b->ranks[k]) return QTT_ERR_SHAPE;
  for (int k = 0; k < a->n; ++k)
    if (dphys(c, k) != s.d[k]) return QTT_ERR_SHAPE;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  for (int k = 0; k < a->n; ++k) {
    const int ra0 = (int)a->ranks[k], ra1 = (int)a->ranks[k + 1], rb0 = (int)b->ranks[k], rb1 = (int)b->ranks[k + 1];
    hipError_t e;
    if (s.kind == K_HAD) {
      if (a->dtype == QTT_F64)
        e = contract_hadamard<double>(strm, (const double*)a->cores[k], ra0, s.d[k], ra1, (const double*)b->cores[k],
                                      rb0, rb1, (double*)c->cores[k]);
      else
        e = contract_hadamard<float>(strm, (const float*)a->cores[k], ra0, s.d[k], ra1, (const float*)b->cores[k],
                                     rb0, rb1, (float*)c->cores[k]);
    } else {
      if (a->dtype == QTT_F64)
        e = contract_mpo<double>(strm, (const double*)a->cores[k], ra0, s.d[k], s.dj[k], ra1,
                                 (const double*)b->cores[k], rb0, rb1, (double*)c->cores[k]);
      else
        e = contract_mpo<float>(strm, (const float*)a->cores[k], ra0, s.d[k], s.dj[k], ra1, (const float*)b->cores[k],
                                rb0, rb1, (float*)c->cores[k]);
    }
    if (e != hipSuccess) return QTT_ERR_HIP;
  }
  return QTT_OK;
}

int qtt_orthogonalize(qtt_handle h, qtt_tt* t, double* norm_host, void* ws, size_t ws_bytes, void* stream) {
  if (!h || !norm_host) return QTT_ERR_ARG;
  int st = check_tt(t, 1);
  if (st) return st;
  if (t->dtype != QTT_F64) return QTT_ERR_DTYPE;
  Shape s;
  shape_from_tt(t, s);
  Plan P;
  if ((st = make_plan(s, 0, P, false))) return st;
  if (!ws || ws_bytes < ws_bytes_of(P)) return QTT_ERR_WORKSPACE;
  Scoped sc(h->device);
  Sweep w{h, (hipStream_t)stream, align_ws(ws), &s, &P, QTT_GEMM_FP64};
  if ((st = qr_sweep(w, t, nullptr, nullptr))) return st;
  const int n = s.n;
  double* Z = w.ws + P.offZ;
  // core k = Q_k (explicit): Q_k [I; 0]
  for (int k = 0; k + 1 < n; ++k) {
    const int m = (int)P.m[k], q = (int)P.rho[k + 1];
    QTT_HIP(set_eye_rect(w.st, Z, m, q));
    QTT_HIP(apply_q(w.st, w.ws + P.offM[k], m, q, s.rc[k + 1], w.ws + P.offT[k], Z, q, q, false, w.ws + P.offScr));
    QTT_HIP(copy_pad_rows(w.st, Z, m, q, q, (double*)t->cores[k], m, q));
  }
  QTT_HIP(copy_pad_rows(w.st, w.ws + P.offCenter, (int)(P.rho[n - 1] * s.d[n - 1]), 1, 1,
                        (double*)t->cores[n - 1], (int)(P.rho[n - 1] * s.d[n - 1]), 1));
  QTT_HIP(hipMemcpyAsync(h->pin_dbl, w.ws + P.offNorm, sizeof(double), hipMemcpyDeviceToHost, w.st));
  QTT_HIP(hipStreamSynchronize(w.st));
  *norm_host = h->pin_dbl[0];
  if (!std::isfinite(*norm_host)) return QTT_ERR_NONFINITE;
  for (int k = 1; k < n; ++k) t->ranks[k] = P.rho[k];
  return QTT_OK;
}

static int round_common(qtt_handle h, const Shape& s, const qtt_tt* t, const qtt_tt* a, const qtt_tt* b,
                        qtt_tt* out, double rel_tol, int64_t max_rank, int prec, qtt_round_info* info, void* ws,
                        size_t ws_bytes, void* stream) {
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  if (prec < QTT_GEMM_FP64 || prec > QTT_GEMM_BF16X6) return QTT_ERR_ARG;
  Plan P;
  int st = make_plan(s, max_rank, P);
  if (st) return st;
  if (!ws || ws_bytes < ws_bytes_of(P)) return QTT_ERR_WORKSPACE;
  Scoped sc(h->device);
  Sweep w{h, (hipStream_t)stream, align_ws(ws), &s, &P, prec};
  if ((st = qr_sweep(w, t, a, b))) return st;
  std::vector<long> newr;
  if ((st = svd_sweep(w, out, rel_tol, max_rank, info, newr))) return st;
  out->ranks[0] = 1;
  out->ranks[s.n] = 1;
  for (int k = 1; k < s.n; ++k) out->ranks[k] = newr[k];
  return QTT_OK;
}

int qtt_round(qtt_handle h, qtt_tt* t, double rel_tol, int64_t max_rank, int prec, qtt_round_info* info, void* ws,
              size_t ws_bytes, void* stream) {
  if (!h) return QTT_ERR_ARG;
  int st = check_tt(t, 1);
  if (st) return st;
  if (t->dtype != QTT_F64) return QTT_ERR_DTYPE;
  Shape s;
  shape_from_tt(t, s);
  return round_common(h, s, t, nullptr, nullptr, t, rel_tol, max_rank, prec, info, ws, ws_bytes, stream);
}

static int contract_round_args(const char* spec, const qtt_tt* a, const qtt_tt* b, const qtt_tt* out, Shape& s) {
  int st = shape_from_pair(spec, a, b, s);
  if (st) return st;
  if (a->dtype != QTT_F64 || b->dtype != QTT_F64) return QTT_ERR_DTYPE;
  if (!out || !out->ranks || !out->cores || out->n != a->n || out->legs != 1) return QTT_ERR_ARG;
  if (out->dtype != QTT_F64) return QTT_ERR_DTYPE;
  for (int k = 0; k < out->n; ++k)
    if (!out->cores[k]) return QTT_ERR_ARG;
  return QTT_OK;
}

int qtt_contract_round(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* out,
                       double rel_tol, int64_t max_rank, int prec, qtt_round_info* info, void* ws, size_t ws_bytes,
                       void* stream) {
  if (!h) return QTT_ERR_ARG;
  Shape s;
  int st = contract_round_args(spec, a, b, out, s);
  if (st) return st;
  return round_common(h, s, nullptr, a, b, out, rel_tol, max_rank, prec, info, ws, ws_bytes, stream);
}

int qtt_contract_round_async(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* out,
                             double rel_tol, int64_t max_rank, int prec, int64_t* ranks_dev, int32_t* status_dev,
                             void* ws, size_t ws_bytes, void* stream) {
  if (!h || !ranks_dev || !status_dev) return QTT_ERR_ARG;
  Shape s;
  int st = contract_round_args(spec, a, b, out, s);
  if (st) return st;
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  if (prec < QTT_GEMM_FP64 || prec > QTT_GEMM_BF16X6) return QTT_ERR_ARG;
  Plan P;
  if ((st = make_plan(s, max_rank, P))) return st;
  if (!ws || ws_bytes < ws_bytes_of(P)) return QTT_ERR_WORKSPACE;
  Scoped sc(h->device);
  Sweep w{h, (hipStream_t)stream, align_ws(ws), &s, &P, prec};
  if ((st = qr_sweep(w, nullptr, a, b))) return st;
  std::vector<long> newr;
  static_assert(sizeof(long long) == sizeof(int64_t), "rank record width");
  return svd_sweep(w, out, rel_tol, max_rank, nullptr, newr, false, (long long*)ranks_dev, (int*)status_dev);
}

int qtt_contract_round_noalloc(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* out,
                               double rel_tol, int64_t max_rank, int prec, qtt_round_info* info, void* stream) {
  if (!h) return QTT_ERR_ARG;
  if (!h->scratch) return QTT_ERR_HIP;
  Shape s;
  int st = contract_round_args(spec, a, b, out, s);
  if (st) return st;
  // the same sweeps as qtt_contract_round on this device's fixed array;
  // round_common rejects a plan larger than the array with QTT_ERR_WORKSPACE
  // before anything is launched
  return round_common(h, s, nullptr, a, b, out, rel_tol, max_rank, prec, info, h->scratch,
                      (size_t)QTT_NOALLOC_SCRATCH_BYTES, stream);
}

int qtt_inner_prec(qtt_handle h, const qtt_tt* a, const qtt_tt* b, int prec, double* out_host, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!h || !out_host) return QTT_ERR_ARG;
  if (prec < QTT_GEMM_FP64 || prec > QTT_GEMM_BF16X6) return QTT_ERR_ARG;
  int st;
  if ((st = check_tt(a, 1)) || (st = check_tt(b, 1))) return st;
  if ((st = same_layout(a, b))) return st;
  // the reduced-precision forms take FP64 cores (FP32 cores already run FP32 GEMMs)
  if (prec != QTT_GEMM_FP64 && a->dtype != QTT_F64) return QTT_ERR_DTYPE;
  const size_t need = (size_t)inner_plan(a, b).total * 8 + 256;
  if (!ws || ws_bytes < need) return QTT_ERR_WORKSPACE;
  Scoped sc(h->device);
  if (a->dtype == QTT_F64) return inner_impl<double>(h, a, b, out_host, ws, (hipStream_t)stream, prec);
  return inner_impl<float>(h, a, b, out_host, ws, (hipStream_t)stream);
}

int qtt_inner(qtt_handle h, const qtt_tt* a, const qtt_tt* b, double* out_host, void* ws, size_t ws_bytes,
              void* stream) {
  return qtt_inner_prec(h, a, b, QTT_GEMM_FP64, out_host, ws, ws_bytes, stream);
}

int qtt_inner_backward(qtt_handle h, const qtt_tt* a, const qtt_tt* b, double g, qtt_tt* da, qtt_tt* db, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!h || (!da && !db)) return QTT_ERR_ARG;
  int st;
  if ((st = check_tt(a, 1)) || (st = check_tt(b, 1))) return st;
  if ((st = same_layout(a, b))) return st;
  if (da) {
    if ((st = check_tt(da, 1))) return st;
    if ((st = same_layout(a, da))) return st;
    for (int k = 0; k <= a->n; ++k)
      if (da->ranks[k] != a->ranks[k]) return QTT_ERR_SHAPE;
  }
  if (db) {
    if ((st = check_tt(db, 1))) return st;
    if ((st = same_layout(b, db))) return st;
    for (int k = 0; k <= b->n; ++k)
      if (db->ranks[k] != b->ranks[k]) return QTT_ERR_SHAPE;
  }
  const size_t need = (size_t)env_plan(a, b).total * 8 + 256;
  if (!ws || ws_bytes < need) return QTT_ERR_WORKSPACE;
  Scoped sc(h->device);
  if (a->dtype == QTT_F64) return inner_backward_impl<double>(a, b, g, da, db, ws, (hipStream_t)stream);
  return inner_backward_impl<float>(a, b, g, da, db, ws, (hipStream_t)stream);
}

int qtt_contract_backward(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, const qtt_tt* dc,
                          qtt_tt* da, qtt_tt* db, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (!h || (!da && !db)) return QTT_ERR_ARG;
  Shape s;
  int st = shape_from_pair(spec, a, b, s);
  if (st) return st;
  if ((st = check_tt(dc, 1))) return st;
  if (dc->n != a->n || dc->dtype != a->dtype || b->dtype != a->dtype) return QTT_ERR_SHAPE;
  for (int k = 0; k <= a->n; ++k)
    if (dc->ranks[k] != a->ranks[k] * b->ranks[k]) return QTT_ERR_SHAPE;
  if (da && (da->n != a->n || da->dtype != a->dtype)) return QTT_ERR_SHAPE;
  if (db && (db->n != b->n || db->dtype != b->dtype)) return QTT_ERR_SHAPE;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  const bool mpo = s.kind == K_MPO;
  for (int k = 0; k < a->n; ++k) {
    const int ra0 = (int)a->ranks[k], ra1 = (int)a->ranks[k + 1], rb0 = (int)b->ranks[k], rb1 = (int)b->ranks[k + 1];
    hipError_t e = hipSuccess;
    if (db) {
      if (a->dtype == QTT_F64)
        e = contract_backward_x<double>(strm, mpo, (const double*)a->cores[k], ra0, s.d[k], s.dj[k], ra1,
                                        (const double*)dc->cores[k], rb0, rb1, (double*)db->cores[k]);
      else
        e = contract_backward_x<float>(strm, mpo, (const float*)a->cores[k], ra0, s.d[k], s.dj[k], ra1,
                                       (const float*)dc->cores[k], rb0, rb1, (float*)db->cores[k]);
      if (e != hipSuccess) return QTT_ERR_HIP;
    }
    if (da) {
      if (a->dtype == QTT_F64)
        e = contract_backward_w<double>(strm, mpo, (const double*)b->cores[k], rb0, s.dj[k], rb1,
                                        (const double*)dc->cores[k], ra0, s.d[k], ra1, (double*)da->cores[k]);
      else
        e = contract_backward_w<float>(strm, mpo, (const float*)b->cores[k], rb0, s.dj[k], rb1,
                                       (const float*)dc->cores[k], ra0, s.d[k], ra1, (float*)da->cores[k]);
      if (e != hipSuccess) return QTT_ERR_HIP;
    }
  }
  return QTT_OK;
}

int qtt_profile_start(qtt_handle h, int kernel_class, int max_launches) {
  if (!h || kernel_class < 0 || kernel_class >= prof::kNumClasses || max_launches < 1 || max_launches > (1 << 22))
    return QTT_ERR_ARG;
  Scoped sc(h->device);
  return prof::start(kernel_class, max_launches) == hipSuccess ? QTT_OK : QTT_ERR_HIP;
}

int qtt_profile_stop(qtt_handle h, int64_t* launches, double* total_ms, double* alg_bytes, double* alg_flops) {
  if (!h || !launches || !total_ms || !alg_bytes || !alg_flops) return QTT_ERR_ARG;
  Scoped sc(h->device);
  long l = 0;
  if (prof::stop(&l, total_ms, alg_bytes, alg_flops) != hipSuccess) return QTT_ERR_HIP;
  *launches = l;
  return QTT_OK;
}

int qtt_batch_workspace_size(qtt_handle h, const char* spec, int32_t count, const qtt_tt* a, const qtt_tt* b,
                             int64_t max_rank, size_t* bytes) {
  (void)h;
  if (!bytes) return QTT_ERR_ARG;
  BatchLayout Lo;
  int st = batch_layout(spec, count, a, b, max_rank, Lo);
  if (st) return st;
  *bytes = (size_t)Lo.total;
  return QTT_OK;
}

int qtt_batch_plan_create(qtt_handle h, const char* spec, int32_t count, const qtt_tt* a, const qtt_tt* b,
                          qtt_tt* out, double rel_tol, int64_t max_rank, int tune, void* ws, size_t ws_bytes,
                          void* stream, qtt_batch_plan* plan) {
  if (!h || !plan || !out) return QTT_ERR_ARG;
  *plan = nullptr;
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  BatchLayout Lo;
  int st = batch_layout(spec, count, a, b, max_rank, Lo);
  if (st) return st;
  if (!ws || ws_bytes < (size_t)Lo.total) return QTT_ERR_WORKSPACE;
  for (int i = 0; i < count; ++i) {
    if (!out[i].cores || !out[i].ranks || out[i].n != a[i].n) return QTT_ERR_ARG;
    for (int k = 0; k < out[i].n; ++k)
      if (!out[i].cores[k]) return QTT_ERR_ARG;
  }
  Scoped sc(h->device);
  char* base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  // host instance table
  std::vector<BInst> tab(count);
  std::vector<double> cost(count, 0.0);
  for (int i = 0; i < count; ++i) {
    const Shape& sh = Lo.shapes[i];
    const Plan& P = Lo.plans[i];
    BInst& I = tab[i];
    std::memset(&I, 0, sizeof(BInst));
    I.n = sh.n;
    I.mpo = sh.kind == K_MPO ? 1 : 0;
    I.ws = (double*)(base + Lo.instOff[i]);
    for (int k = 0; k < sh.n; ++k) {
      I.a[k] = (const double*)a[i].cores[k];
      I.b[k] = (const double*)b[i].cores[k];
      I.out[k] = (double*)out[i].cores[k];
      I.offM[k] = P.offM[k];
      I.offT[k] = P.offT[k];
      I.d[k] = sh.d[k];
      I.dj[k] = sh.dj[k];
      I.m[k] = (int)P.m[k];
    }
    for (int k = 0; k <= sh.n; ++k) {
      I.ra[k] = (int)sh.ra[k];
      I.rb[k] = (int)sh.rb[k];
      I.rho[k] = (int)P.rho[k];
    }
    I.offCenter = P.offCenter;
    I.offR = P.offR;
    I.offY = P.offY;
    I.offZ = P.offZ;
    I.offX = P.offX;
    I.offXc = P.offXc;
    I.offYn = P.offYn;
    I.offTB = P.offTB;
    I.offSig = P.offSig;
    I.offPerm = P.offPerm;
    I.offTmp = P.offScr;
    I.offOne = P.offOne;
    for (int k = 0; k + 1 < sh.n; ++k) {
      const double m = (double)P.m[k], c = (double)sh.rc[k + 1];
      cost[i] += m * c * std::min(m, c) + std::pow(std::min(m, c), 3.0);
    }
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  qtt_batch* p = new (std::nothrow) qtt_batch();
  if (!p) return QTT_ERR_ARG;
  p->h = h;
  p->count = count;
  p->tol = rel_tol;
  p->max_rank = max_rank;
  p->max_sweeps = h->max_sweeps;
  p->maxL = Lo.maxL;
  p->dtab = (BInst*)(base + Lo.offTab);
  p->dorder = (int*)(base + Lo.offOrder);
  p->dqueue = (unsigned*)(base + Lo.offQueue);
  p->dranks = (long*)(base + Lo.offRanks);
  p->dtails = (double*)(base + Lo.offTails);
  p->dstatus = (int*)(base + Lo.offStatus);
  p->ncores.resize(count);
  for (int i = 0; i < count; ++i) p->ncores[i] = a[i].n;
  hipStream_t us = (hipStream_t)stream;
  auto fail = [&](int code) {
    batch_free(p);
    return code;
  };
  if (hipHostMalloc((void**)&p->hranks, (size_t)count * (QTT_BATCH_MAXN + 1) * sizeof(long), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&p->htails, (size_t)count * QTT_BATCH_MAXN * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&p->hstatus, (size_t)count * sizeof(int), hipHostMallocDefault) != hipSuccess)
    return fail(QTT_ERR_HIP);
  if (hipMemcpyAsync(p->dtab, tab.data(), (size_t)count * sizeof(BInst), hipMemcpyHostToDevice, us) != hipSuccess ||
      hipMemcpyAsync(p->dorder, order.data(), (size_t)count * sizeof(int), hipMemcpyHostToDevice, us) != hipSuccess ||
      hipStreamSynchronize(us) != hipSuccess)
    return fail(QTT_ERR_HIP);
  // GEMM tile per shape bucket (probe-timed or cached), then the kernel variant
  {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device);
    const int tst = tune_tiles(p, Lo, max_rank, tune != 0, base, us, std::min(count, cus));
    if (tst != QTT_OK) return fail(tst);
  }
  // variant: cached tuning result, measured now, or the default
  std::ostringstream sig;
  sig << spec << "|" << count << "|" << rel_tol << "|" << max_rank;
  {
    unsigned long long hsh = 1469598103934665603ull;
    for (int i = 0; i < count; ++i)
      for (int k = 0; k <= a[i].n; ++k) {
        hsh ^= (unsigned long long)(a[i].ranks[k] * 131 + b[i].ranks[k]);
        hsh *= 1099511628211ull;
      }
    sig << "|" << std::hex << hsh;
  }
  int variant = tune ? tune_lookup(sig.str()) : 0;
  if (variant < 0) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(QTT_ERR_HIP);
    float best = 1e30f;
    variant = 0;
    for (int v = 0; v < 4; ++v) {
      if (hipEventRecord(e0, us) != hipSuccess || batch_run(p, us, v) != hipSuccess ||
          hipEventRecord(e1, us) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(QTT_ERR_HIP);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      p->tuned_ms[v] = ms;
      if (ms < best) {
        best = ms;
        variant = v;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    tune_store(sig.str(), variant);
  } else {
    // one eager run: sets kernel attributes before capture and validates the launch
    if (batch_run(p, us, variant) != hipSuccess || hipStreamSynchronize(us) != hipSuccess) return fail(QTT_ERR_HIP);
  }
  p->variant = variant;
  // capture [queue reset, persistent kernel] into a graph on a private stream
  if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) return fail(QTT_ERR_HIP);
  if (hipStreamSynchronize(us) != hipSuccess) return fail(QTT_ERR_HIP);
  if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return fail(QTT_ERR_HIP);
  hipError_t le = batch_run(p, p->cap, variant);
  hipError_t ce = hipStreamEndCapture(p->cap, &p->graph);
  if (le != hipSuccess || ce != hipSuccess) return fail(QTT_ERR_HIP);
  if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) return fail(QTT_ERR_HIP);
  *plan = p;
  return QTT_OK;
}

int qtt_batch_plan_launch(qtt_batch_plan plan, void* stream) {
  if (!plan || !plan->exec) return QTT_ERR_ARG;
  Scoped sc(plan->h->device);
  return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? QTT_OK : QTT_ERR_HIP;
}

int qtt_batch_plan_results(qtt_batch_plan plan, int64_t* ranks, double* tails, void* stream) {
  if (!plan || !ranks) return QTT_ERR_ARG;
  Scoped sc(plan->h->device);
  hipStream_t s = (hipStream_t)stream;
  const int c = plan->count;
  if (hipMemcpyAsync(plan->hranks, plan->dranks, (size_t)c * (QTT_BATCH_MAXN + 1) * sizeof(long),
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(plan->htails, plan->dtails, (size_t)c * QTT_BATCH_MAXN * sizeof(double), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipMemcpyAsync(plan->hstatus, plan->dstatus, (size_t)c * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return QTT_ERR_HIP;
  long o = 0, ot = 0;
  int status = QTT_OK;
  for (int i = 0; i < c; ++i) {
    const int n = plan->ncores[i];
    for (int k = 0; k <= n; ++k) ranks[o + k] = plan->hranks[(long)i * (QTT_BATCH_MAXN + 1) + k];
    o += n + 1;
    if (tails) {
      for (int k = 0; k + 1 < n; ++k) tails[ot + k] = plan->htails[(long)i * QTT_BATCH_MAXN + k];
      ot += std::max(n - 1, 0);
    }
    if (plan->hstatus[i] == QTT_BSTATUS_NONFINITE) status = QTT_ERR_NONFINITE;
    if (plan->hstatus[i] == QTT_BSTATUS_NOCONV && status == QTT_OK) status = QTT_ERR_NOCONV;
  }
  return status;
}

int qtt_batch_plan_info(qtt_batch_plan plan, int32_t* variant, int32_t* grid, float* tuned_ms) {
  if (!plan || !variant || !grid) return QTT_ERR_ARG;
  *variant = plan->variant;
  *grid = plan->grid;
  if (tuned_ms)
    for (int v = 0; v < 4; ++v) tuned_ms[v] = plan->tuned_ms[v];
  return QTT_OK;
}

int qtt_batch_plan_tiles(qtt_batch_plan plan, uint8_t* tiles, int32_t* shapes, float* probe_ms) {
  if (!plan) return QTT_ERR_ARG;
  for (int b = 0; b < kGemmBuckets; ++b) {
    if (tiles) tiles[b] = plan->tiles.v[b];
    for (int c = 0; shapes && c < 3; ++c) shapes[3 * b + c] = plan->tile_shape[b][c];
    for (int v = 0; probe_ms && v < kTileVariants; ++v) probe_ms[kTileVariants * b + v] = plan->tile_ms[b][v];
  }
  return QTT_OK;
}

int qtt_batch_plan_destroy(qtt_batch_plan plan) {
  if (!plan) return QTT_ERR_ARG;
  Scoped sc(plan->h->device);
  batch_free(plan);
  return QTT_OK;
}

int qtt_zipup_query(const char* spec, const qtt_tt* a, const qtt_tt* b, int64_t max_rank, int32_t ncores,
                    int64_t* bounds, size_t* ws_bytes) {
  Shape s;
  ZipPlan Z;
  int st = zip_setup(spec, a, b, max_rank, ncores, s, Z);
  if (st) return st;
  if (bounds)
    for (int k = 0; k <= s.n; ++k) bounds[k] = Z.bound[k];
  if (ws_bytes) *ws_bytes = (size_t)Z.total * sizeof(double) + 256;
  return QTT_OK;
}

int qtt_contract_zipup(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* out,
                       double rel_tol, int64_t max_rank, int32_t ncores, int prec, qtt_round_info* info, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!h) return QTT_ERR_ARG;
  if (!(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  if (prec < QTT_GEMM_FP64 || prec > QTT_GEMM_BF16X6) return QTT_ERR_ARG;
  Shape s;
  ZipPlan Z;
  int st = zip_setup(spec, a, b, max_rank, ncores, s, Z);
  if (st) return st;
  if (!out || !out->ranks || !out->cores || out->n != a->n || out->legs != 1) return QTT_ERR_ARG;
  if (out->dtype != QTT_F64) return QTT_ERR_DTYPE;
  for (int k = 0; k < out->n; ++k)
    if (!out->cores[k]) return QTT_ERR_ARG;
  if (!ws || ws_bytes < (size_t)Z.total * sizeof(double) + 256) return QTT_ERR_WORKSPACE;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  double* w = align_ws(ws);
  const int n = s.n;
  for (int k = 0; k < n; ++k) {
    QTT_HIP(hipMemcpyAsync(w + Z.offA[k], a->cores[k], (size_t)(s.ra[k] * Z.Pa[k] * s.ra[k + 1]) * sizeof(double),
                           hipMemcpyDeviceToDevice, strm));
    QTT_HIP(hipMemcpyAsync(w + Z.offB[k], b->cores[k], (size_t)(s.rb[k] * Z.Pb[k] * s.rb[k + 1]) * sizeof(double),
                           hipMemcpyDeviceToDevice, strm));
  }
  if ((st = right_sweep(strm, w, Z, Z.offA, s.ra, Z.Pa, Z.ra, n))) return st;
  if ((st = right_sweep(strm, w, Z, Z.offB, s.rb, Z.Pb, Z.rb, n))) return st;
  std::vector<long> newr;
  if ((st = zip_sweep(h, strm, w, s, Z, prec, rel_tol, max_rank, out, info, newr))) return st;
  out->ranks[0] = 1;
  out->ranks[n] = 1;
  for (int k = 1; k < n; ++k) out->ranks[k] = newr[k];
  return QTT_OK;
}


int qtt_add(qtt_handle h, int32_t count, const qtt_tt* terms, const double* coeffs, qtt_tt* out, void* stream) {
  if (!h || !terms || !out) return QTT_ERR_ARG;
  if (count < 1) return QTT_ERR_ARG;
  if (count > kMaxAddTerms) return QTT_ERR_UNSUPPORTED;
  int st;
  const int legs = terms[0].legs;
  for (int t = 0; t < count; ++t)
    if ((st = check_tt(&terms[t], legs))) return st;
  if ((st = check_tt(out, legs))) return st;
  const int n = terms[0].n;
  const qtt_dtype dt = terms[0].dtype;
  if (out->n != n || out->dtype != dt) return QTT_ERR_SHAPE;
  for (int t = 0; t < count; ++t) {
    if (terms[t].n != n) return QTT_ERR_SHAPE;
    if (terms[t].dtype != dt) return QTT_ERR_DTYPE;
    for (int k = 0; k < n * legs; ++k)
      if (terms[t].phys[k] != terms[0].phys[k]) return QTT_ERR_SHAPE;
  }
  for (int k = 0; k < n * legs; ++k)
    if (out->phys[k] != terms[0].phys[k]) return QTT_ERR_SHAPE;
  for (int k = 1; k < n; ++k) {
    long sum = 0;
    for (int t = 0; t < count; ++t) sum += terms[t].ranks[k];
    if (out->ranks[k] != sum) return QTT_ERR_SHAPE;
  }
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  for (int k = 0; k < n; ++k) {
    int P = 1;
    for (int l = 0; l < legs; ++l) P *= terms[0].phys[k * legs + l];
    const int first = (k == 0), last = (k == n - 1);
    hipError_t e;
    auto fill = [&](auto& at) {
      int o0 = 0, o1 = 0;
      for (int t = 0; t < count; ++t) {
        at.r0[t] = (int)terms[t].ranks[k];
        at.r1[t] = (int)terms[t].ranks[k + 1];
        at.off0[t] = first ? 0 : o0;
        at.off1[t] = last ? 0 : o1;
        at.coef[t] = coeffs ? coeffs[t] : 1.0;
        o0 += at.r0[t];
        o1 += at.r1[t];
      }
    };
    if (dt == QTT_F64) {
      AddTerms<double> at{};
      for (int t = 0; t < count; ++t) at.src[t] = (const double*)terms[t].cores[k];
      fill(at);
      e = tt_add_core<double>(strm, at, count, P, (int)out->ranks[k], (int)out->ranks[k + 1], first, last,
                              (double*)out->cores[k]);
    } else {
      AddTerms<float> at{};
      for (int t = 0; t < count; ++t) at.src[t] = (const float*)terms[t].cores[k];
      fill(at);
      e = tt_add_core<float>(strm, at, count, P, (int)out->ranks[k], (int)out->ranks[k + 1], first, last,
                             (float*)out->cores[k]);
    }
    if (e != hipSuccess) return QTT_ERR_HIP;
  }
  return QTT_OK;
}

int qtt_fit_workspace_size(const char* spec, const qtt_tt* a, const qtt_tt* b, const qtt_tt* c, size_t* bytes) {
  if (!bytes) return QTT_ERR_ARG;
  Shape s;
  FitPlan F;
  size_t ob = 0;
  int st = fit_setup(spec, a, b, c, s, F, ob);
  if (st) return st;
  *bytes = std::max(ob, (size_t)F.total * sizeof(double) + 256);
  return QTT_OK;
}

int qtt_fit(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* c, int32_t nsweeps,
            double* norm_host, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return QTT_ERR_ARG;
  if (nsweeps < 0) return QTT_ERR_ARG;
  Shape s;
  FitPlan F;
  size_t ob = 0;
  int st = fit_setup(spec, a, b, c, s, F, ob);
  if (st) return st;
  if (!ws || ws_bytes < std::max(ob, (size_t)F.total * sizeof(double) + 256)) return QTT_ERR_WORKSPACE;
  double nrm = 0.0;
  // the guess, orthogonalised from the left (centre at core n; ranks may shrink)
  if ((st = qtt_orthogonalize(h, c, &nrm, ws, ws_bytes, stream))) return st;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  double* w = align_ws(ws);
  const int n = s.n;
  for (int k = 0; k < n; ++k) {
    const int ra0 = (int)s.ra[k], ra1 = (int)s.ra[k + 1], rb0 = (int)s.rb[k], rb1 = (int)s.rb[k + 1];
    hipError_t e;
    if (s.kind == K_HAD)
      e = contract_hadamard<double>(strm, (const double*)a->cores[k], ra0, s.d[k], ra1, (const double*)b->cores[k],
                                    rb0, rb1, w + F.offY[k]);
    else
      e = contract_mpo<double>(strm, (const double*)a->cores[k], ra0, s.d[k], s.dj[k], ra1,
                               (const double*)b->cores[k], rb0, rb1, w + F.offY[k]);
    if (e != hipSuccess) return QTT_ERR_HIP;
  }
  std::vector<long> rc(n + 1);
  for (int k = 0; k <= n; ++k) rc[k] = c->ranks[k];
  if ((st = fit_sweeps(strm, w, s, F, c, rc, nsweeps))) return st;
  int e = readback(h, strm, w + F.offNrm, sizeof(double), h->pin_dbl);
  if (e) return e;
  if (!std::isfinite(h->pin_dbl[0])) return QTT_ERR_NONFINITE;
  if (norm_host) *norm_host = h->pin_dbl[0];
  for (int k = 0; k <= n; ++k) c->ranks[k] = rc[k];
  return QTT_OK;
}

int qtt_solve_query(const qtt_tt* w, const qtt_tt* b, const qtt_tt* x, int32_t ncores, int64_t max_rank,
                    int64_t* bounds, size_t* bytes) {
  if (!bytes || (ncores != 1 && ncores != 2)) return QTT_ERR_ARG;
  int st = solve_check(w, b, x);
  if (st) return st;
  if (ncores == 2 && x->n < 2) return QTT_ERR_ARG;
  SolvePlan F;
  if ((st = make_solve_plan(w, b, x, ncores, max_rank, F))) return st;
  Shape sx;
  shape_from_tt(x, sx);
  Plan P;
  if ((st = make_plan(sx, 0, P, false))) return st;
  *bytes = std::max({ws_bytes_of(P), (size_t)F.total * sizeof(double) + 256,
                     (size_t)inner_plan(b, b).total * sizeof(double) + 256});
  if (bounds)
    for (int k = 0; k <= x->n; ++k) bounds[k] = F.bnd[k];
  return QTT_OK;
}

int qtt_solve(qtt_handle h, const qtt_tt* w, const qtt_tt* b, qtt_tt* x, int32_t nsweeps, int32_t ncores,
              double rel_tol, int64_t max_rank, qtt_round_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return QTT_ERR_ARG;
  if (nsweeps < 0 || !(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  size_t need = 0;
  int st = qtt_solve_query(w, b, x, ncores, max_rank, nullptr, &need);
  if (st) return st;
  if (!ws || ws_bytes < need) return QTT_ERR_WORKSPACE;
  SolvePlan F;
  if ((st = make_solve_plan(w, b, x, ncores, max_rank, F))) return st;
  double nrm = 0.0;
  const int n = x->n;
  {
    // b = 0: the solution is the zero train (rank 1), written directly; the
    // sweeps would split zero super-cores into zero, not orthonormal, cores
    double bb = 0.0;
    if ((st = inner_impl<double>(h, b, b, &bb, ws, (hipStream_t)stream))) return st;
    if (!std::isfinite(bb)) return QTT_ERR_NONFINITE;
    if (bb == 0.0) {
      Scoped sc(h->device);
      for (int k = 0; k < n; ++k) QTT_HIP(fill_f64((hipStream_t)stream, (double*)x->cores[k], 0.0, dphys(x, k)));
      QTT_HIP(hipStreamSynchronize((hipStream_t)stream));
      for (int k = 0; k <= n; ++k) x->ranks[k] = 1;
      if (info) {
        info->norm = 0.0;
        info->jacobi_sweeps_max = 0;
      }
      return QTT_OK;
    }
  }
  // the guess, orthogonalised from the left (centre at core n; ranks may shrink)
  if ((st = qtt_orthogonalize(h, x, &nrm, ws, ws_bytes, stream))) return st;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  double* wsa = align_ws(ws);
  std::vector<long> rc(n + 1);
  for (int k = 0; k <= n; ++k) rc[k] = x->ranks[k];
  int maxsw = 0;
  if ((st = solve_sweeps(h, strm, wsa, F, w, b, x, rc, nsweeps, rel_tol, max_rank, maxsw))) return st;
  int e = readback(h, strm, wsa + F.offNrm, sizeof(double), h->pin_dbl);
  if (e) return e;
  if (!std::isfinite(h->pin_dbl[0])) return QTT_ERR_NONFINITE;
  if (info) {
    info->norm = h->pin_dbl[0];
    info->jacobi_sweeps_max = maxsw;
  }
  for (int k = 0; k <= n; ++k) x->ranks[k] = rc[k];
  return QTT_OK;
}

int qtt_fit2_query(const char* spec, const qtt_tt* a, const qtt_tt* b, const qtt_tt* c, int64_t max_rank,
                   int64_t* bounds, size_t* bytes) {
  if (!bytes) return QTT_ERR_ARG;
  Shape s;
  Fit2Plan F;
  size_t ob = 0;
  int st = fit2_setup(spec, a, b, c, max_rank, s, F, ob);
  if (st) return st;
  *bytes = std::max(ob, (size_t)F.total * sizeof(double) + 256);
  if (bounds)
    for (int k = 0; k <= s.n; ++k) bounds[k] = F.bnd[k];
  return QTT_OK;
}

int qtt_fit2(qtt_handle h, const char* spec, const qtt_tt* a, const qtt_tt* b, qtt_tt* c, int32_t nsweeps,
             double rel_tol, int64_t max_rank, qtt_round_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return QTT_ERR_ARG;
  if (nsweeps < 0 || !(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  Shape s;
  Fit2Plan F;
  size_t ob = 0;
  int st = fit2_setup(spec, a, b, c, max_rank, s, F, ob);
  if (st) return st;
  if (!ws || ws_bytes < std::max(ob, (size_t)F.total * sizeof(double) + 256)) return QTT_ERR_WORKSPACE;
  double nrm = 0.0;
  // the guess, orthogonalised from the left (centre at core n; ranks may shrink)
  if ((st = qtt_orthogonalize(h, c, &nrm, ws, ws_bytes, stream))) return st;
  Scoped sc(h->device);
  hipStream_t strm = (hipStream_t)stream;
  double* w = align_ws(ws);
  const int n = s.n;
  for (int k = 0; k < n; ++k) {
    const int ra0 = (int)s.ra[k], ra1 = (int)s.ra[k + 1], rb0 = (int)s.rb[k], rb1 = (int)s.rb[k + 1];
    hipError_t e;
    if (s.kind == K_HAD)
      e = contract_hadamard<double>(strm, (const double*)a->cores[k], ra0, s.d[k], ra1, (const double*)b->cores[k],
                                    rb0, rb1, w + F.offY[k]);
    else
      e = contract_mpo<double>(strm, (const double*)a->cores[k], ra0, s.d[k], s.dj[k], ra1,
                               (const double*)b->cores[k], rb0, rb1, w + F.offY[k]);
    if (e != hipSuccess) return QTT_ERR_HIP;
  }
  std::vector<long> rc(n + 1);
  for (int k = 0; k <= n; ++k) rc[k] = c->ranks[k];
  int maxsw = 0;
  if (n == 1) {
    // one core: the product itself
    QTT_HIP(copy_pad_rows(strm, w + F.offY[0], 1, s.d[0], s.d[0], (double*)c->cores[0], 1, s.d[0]));
    QTT_HIP(frob_norm(strm, (double*)c->cores[0], s.d[0], w + F.offNrm));
  } else {
    std::vector<double> tails((size_t)2 * (n - 1) * std::max(nsweeps, 1));
    if ((st = fit2_sweeps(h, strm, w, s, F, c, rc, nsweeps, rel_tol, max_rank, tails.data(), maxsw))) return st;
    if (info && info->tail && nsweeps > 0)  // the discarded tails of the last sweep's left-to-right splits
      for (int k = 0; k + 1 < n; ++k) info->tail[k] = tails[(size_t)(2 * nsweeps - 1) * (n - 1) + k];
  }
  int e = readback(h, strm, w + F.offNrm, sizeof(double), h->pin_dbl);
  if (e) return e;
  if (!std::isfinite(h->pin_dbl[0])) return QTT_ERR_NONFINITE;
  if (info) {
    info->norm = h->pin_dbl[0];
    info->jacobi_sweeps_max = maxsw;
  }
  for (int k = 0; k <= n; ++k) c->ranks[k] = rc[k];
  return QTT_OK;
}

int qtt_solve_amen_query(const qtt_tt* w, const qtt_tt* b, const qtt_tt* x, const qtt_tt* z, int64_t max_rank,
                         int64_t* x_bounds, int64_t* z_bounds, size_t* bytes) {
  if (!bytes) return QTT_ERR_ARG;
  int st = amen_check(w, b, x, z);
  if (st) return st;
  AmenPlan F;
  if ((st = make_amen_plan(w, b, x, z, max_rank, F))) return st;
  Shape sx, sz;
  shape_from_tt(x, sx);
  shape_from_tt(z, sz);
  Plan Px, Pz;
  if ((st = make_plan(sx, 0, Px, false)) || (st = make_plan(sz, 0, Pz, false))) return st;
  *bytes = std::max({ws_bytes_of(Px), ws_bytes_of(Pz), (size_t)F.total * sizeof(double) + 256,
                     (size_t)inner_plan(b, b).total * sizeof(double) + 256});
  for (int k = 0; k <= x->n; ++k) {
    if (x_bounds) x_bounds[k] = F.S.bnd[k];
    if (z_bounds) z_bounds[k] = F.bz[k];
  }
  return QTT_OK;
}

int qtt_solve_amen(qtt_handle h, const qtt_tt* w, const qtt_tt* b, qtt_tt* x, qtt_tt* z, int32_t nsweeps,
                   double rel_tol, int64_t max_rank, qtt_round_info* info, void* ws, size_t ws_bytes, void* stream) {
  if (!h) return QTT_ERR_ARG;
  if (nsweeps < 0 || !(rel_tol >= 0.0) || !std::isfinite(rel_tol)) return QTT_ERR_ARG;
  size_t need = 0;
  int st = qtt_solve_amen_query(w, b, x, z, max_rank, nullptr, nullptr, &need);
  if (st) return st;
  if (!ws || ws_bytes < need) return QTT_ERR_WORKSPACE;
  AmenPlan F;
  if ((st = make_amen_plan(w, b, x, z, max_rank, F))) return st;
  const int n = x->n;
  hipStream_t strm = (hipStream_t)stream;
  {
    // b = 0: x and the residual train are the zero train (rank 1); the
    // truncated splits would normalise zero rows
    double bb = 0.0;
    if ((st = inner_impl<double>(h, b, b, &bb, ws, strm))) return st;
    if (!std::isfinite(bb)) return QTT_ERR_NONFINITE;
    if (bb == 0.0) {
      Scoped sc(h->device);
      for (int k = 0; k < n; ++k) {
        QTT_HIP(fill_f64(strm, (double*)x->cores[k], 0.0, dphys(x, k)));
        QTT_HIP(fill_f64(strm, (double*)z->cores[k], 0.0, dphys(z, k)));
      }
      QTT_HIP(hipStreamSynchronize(strm));
      for (int k = 0; k <= n; ++k) x->ranks[k] = z->ranks[k] = 1;
      if (info) {
        info->norm = 0.0;
        info->jacobi_sweeps_max = 0;
      }
      return QTT_OK;
    }
  }
  // the guess and the residual train, orthogonalised from the left (ranks may shrink)
  double nrm = 0.0;
  if ((st = qtt_orthogonalize(h, x, &nrm, ws, ws_bytes, stream))) return st;
  if ((st = qtt_orthogonalize(h, z, &nrm, ws, ws_bytes, stream))) return st;
  Scoped sc(h->device);
  double* wsa = align_ws(ws);
  std::vector<long> rc(n + 1), rz(n + 1);
  for (int k = 0; k <= n; ++k) {
    rc[k] = x->ranks[k];
    rz[k] = z->ranks[k];
  }
  int maxsw = 0;
  if ((st = amen_sweeps(h, strm, wsa, F, w, b, x, z, rc, rz, nsweeps, rel_tol, max_rank, maxsw))) return st;
  int e = readback(h, strm, wsa + F.S.offNrm, sizeof(double), h->pin_dbl);
  if (e) return e;
  if (!std::isfinite(h->pin_dbl[0])) return QTT_ERR_NONFINITE;
  if (info) {
    info->norm = h->pin_dbl[0];
    info->jacobi_sweeps_max = maxsw;
  }
  for (int k = 0; k <= n; ++k) {
    x->ranks[k] = rc[k];
    z->ranks[k] = rz[k];
  }
  return QTT_OK;
}

}  // extern "C"
