// One-sided Jacobi SVD and the device-side truncation decision (FP64).
//
// jacobi_rows orthogonalises the rows of X (p x L) by plane rotations,
// X <- Z^T X with Z orthogonal.  Afterwards the rows of X are Sigma V^T up
// to their order: normalising them gives the right singular vectors.  Z is
// not accumulated: the caller forms U Sigma = X_orig V with one GEMM, which
// keeps U Sigma V^T = X_orig V V^T exact up to the orthogonality of V
// (a product of thousands of rounded plane rotations drifts from orthogonal).
//
// Parallel ordering (block cyclic Jacobi): rows form blocks of 8; a
// persistent grid with one workgroup per block pair runs the round-robin
// tournament over blocks.  In a round a workgroup rotates the 64 cross pairs
// of its two blocks (8 steps of 8 disjoint pairs, one wave per pair, both
// rows held in registers, bottom rows passed between waves through LDS);
// in the first round of every sweep it also rotates the 28 + 28 pairs inside
// each block.  Every row pair is thus visited once per sweep.  Rounds are
// ordered by per-block version counters (a workgroup waits only for the two
// workgroups that produced its blocks), sweeps by a grid barrier that also
// sums the sweep's rotation count.  A rotation of rows a, c is skipped when
// |a.c| <= tol ||a|| ||c|| with tol = sqrt(L) eps; the iteration stops after
// the first sweep without any rotation.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"

#include <algorithm>

namespace qtt {

namespace {

constexpr int JB = 8;         // rows per block
constexpr int JNT = 64 * JB;  // one wave per row of the top block
constexpr int JCTR = 8;       // counter words before the block versions

__device__ __forceinline__ int rr_item(int pos, int round, int n) {
  // circle method: position 0 fixed, the others rotate
  return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (n - 1));
}

// Rotate the pair (u, v) of rows (E elements per lane, zero past the row end)
// so that they become orthogonal; returns true when a rotation was applied
// or a row was deflated.  A nonzero row whose squared norm is below negl is
// set to zero instead (see k_jacobi).
template <int E>
__device__ __forceinline__ bool rotate_pair(double (&u)[E], double (&v)[E], double tol, double negl) {
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    al += u[q] * u[q];
    be += v[q] * v[q];
    ga += u[q] * v[q];
  }
  al = wave_sum_bc(al);
  be = wave_sum_bc(be);
  ga = wave_sum_bc(ga);
  if (al < negl || be < negl) {
    bool changed = false;
    if (al < negl && al > 0.0) {
#pragma unroll
      for (int q = 0; q < E; ++q) u[q] = 0.0;
      changed = true;
    }
    if (be < negl && be > 0.0) {
#pragma unroll
      for (int q = 0; q < E; ++q) v[q] = 0.0;
      changed = true;
    }
    return changed;
  }
  double cs, sn;
  if (!jacobi_rotation(al, be, ga, tol, cs, sn)) return false;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const double a = u[q], c = v[q];
    u[q] = cs * a - sn * c;
    v[q] = sn * a + cs * c;
  }
  return true;
}

// Rows move between workgroups through global memory with agent-scope
// (coherent) accesses, so that no cache writeback or invalidation is needed
// when a block changes hands: the writer waits for its stores to complete
// before publishing the block's version, the reader reads the version and
// then the rows.
template <int E>
__device__ __forceinline__ void load_row(const double* __restrict__ src, int L, bool ok, double (&r)[E]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int c = lane + 64 * q;
    r[q] = (ok && c < L) ? __hip_atomic_load(src + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0.0;
  }
}

template <int E>
__device__ __forceinline__ void store_row(double* __restrict__ dst, int L, bool ok, const double (&r)[E]) {
  const int lane = threadIdx.x & 63;
  if (!ok) return;
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int c = lane + 64 * q;
    if (c < L) __hip_atomic_store(dst + c, r[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// LDS row slots hold 64 E doubles (row elements lane + 64 q).
template <int E>
__device__ __forceinline__ void lds_put(double* slot, const double (&r)[E]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < E; ++q) slot[lane + 64 * q] = r[q];
}
template <int E>
__device__ __forceinline__ void lds_get(const double* slot, double (&r)[E]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < E; ++q) r[q] = slot[lane + 64 * q];
}

// ctr[0..1]: grid barrier; ctr[2..4]: rotation counts of three consecutive
// sweeps; ctr[JCTR + b]: rounds completed by block b.
// Rows are deflated to exact zeros once their squared norm falls below
// negl = defl max_i ||x_i||^2 of the input, defl = (8 u sqrt(p))^2: a row
// at that level is rounding noise of the input (its singular value is
// within the error any backward-stable SVD makes), and left in, such rows
// cannot be rotated away -- a row that has become an exact tiny multiple of
// another shrinks by about eps per rotation while it stays parallel, so the
// relative test would fire on every sweep, and rows that collapse to the
// rounding level of an exactly rank-deficient input become orthogonal only
// after all the others.  ref (nullable) points at the largest input row
// norm.
template <int E>
__global__ __launch_bounds__(JNT) void k_jacobi(double* __restrict__ X, int p, int L, unsigned* __restrict__ ctr,
                                                int max_sweeps, int* sweeps_out, double tol,
                                                const double* __restrict__ ref, double defl) {
  const double negl = ref ? defl * (ref[0] * ref[0]) : 0.0;
  extern __shared__ double sh[];  // 16 row slots of 64 E doubles
  __shared__ double bes[2][JB];   // squared norms travelling with the bottom rows
  __shared__ unsigned s_tot;
  constexpr int RS = 64 * E;
  const int nblk = (p + JB - 1) / JB;
  const int nb2 = nblk + (nblk & 1);
  const int nrounds = nb2 - 1;
  const int pair = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  unsigned* ver = ctr + JCTR;
  unsigned local_rot = 0;
  int sweep = 0, converged = 0;
  for (; sweep < max_sweeps; ++sweep) {
    for (int round = 0; round < nrounds; ++round) {
      const int b0 = rr_item(pair, round, nb2);
      const int b1 = rr_item(nb2 - 1 - pair, round, nb2);
      const unsigned expect = (unsigned)(sweep * nrounds + round);
      if (tid < 2) {  // lanes 0 and 1 poll the two blocks' versions together
        const int bb = tid == 0 ? b0 : b1;
        while (__hip_atomic_load(&ver[bb], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != expect)
          __builtin_amdgcn_s_sleep(1);
      }
      __syncthreads();
      const int rt = b0 * JB + w;  // top row held by this wave
      const bool okt = rt < p;
      double top[E], bot[E];
      load_row<E>(X + (long)rt * L, L, okt, top);
      load_row<E>(X + (long)(b1 * JB + w) * L, L, b1 * JB + w < p, bot);
      if (round == 0) {
        // pairs inside each block: 7 steps, waves 0-3 on the top block, 4-7 on the bottom
        lds_put<E>(sh + w * RS, top);
        lds_put<E>(sh + (JB + w) * RS, bot);
        __syncthreads();
        const int blk = w >> 2, i = w & 3;
        for (int st = 0; st < JB - 1; ++st) {
          double* sa = sh + (blk * JB + rr_item(i, st, JB)) * RS;
          double* sc = sh + (blk * JB + rr_item(JB - 1 - i, st, JB)) * RS;
          double u[E], v[E];
          lds_get<E>(sa, u);
          lds_get<E>(sc, v);
          if (rotate_pair<E>(u, v, tol, negl)) {
            lds_put<E>(sa, u);
            lds_put<E>(sc, v);
            if (lane == 0) ++local_rot;
          }
          __syncthreads();
        }
        lds_get<E>(sh + w * RS, top);
        lds_get<E>(sh + (JB + w) * RS, bot);
        __syncthreads();
      }
      // cross pairs: at step s wave w rotates top row w with bottom row (w + s) % 8.
      // The squared row norms are formed once per round and then carried
      // through the rotations (||a'||^2 = ||a||^2 - t a.c, ||c'||^2 =
      // ||c||^2 + t a.c) and with the bottom rows through LDS, so a step
      // needs one dot product and one reduction.
      double al = 0.0, be = 0.0;
#pragma unroll
      for (int q = 0; q < E; ++q) {
        al += top[q] * top[q];
        be += bot[q] * bot[q];
      }
      al = wave_sum_bc(al);
      be = wave_sum_bc(be);
      if (al < negl && al > 0.0) {
#pragma unroll
        for (int q = 0; q < E; ++q) top[q] = 0.0;
        al = 0.0;
        if (lane == 0) ++local_rot;
      }
      if (be < negl && be > 0.0) {
#pragma unroll
        for (int q = 0; q < E; ++q) bot[q] = 0.0;
        be = 0.0;
        if (lane == 0) ++local_rot;
      }
      for (int s = 0; s < JB; ++s) {
        double ga = 0.0;
#pragma unroll
        for (int q = 0; q < E; ++q) ga += top[q] * bot[q];
        ga = wave_sum_bc(ga);
        double cs, sn, t;
        if (jacobi_rotation(al, be, ga, tol, cs, sn, t)) {
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const double a = top[q], c = bot[q];
            top[q] = cs * a - sn * c;
            bot[q] = sn * a + cs * c;
          }
          al -= t * ga;
          be += t * ga;
          if (lane == 0) ++local_rot;
        }
        if (s + 1 < JB) {
          double* buf = sh + (s & 1) * JB * RS;
          lds_put<E>(buf + ((w + s) % JB) * RS, bot);
          if (lane == 0) bes[s & 1][(w + s) % JB] = be;
          __syncthreads();
          lds_get<E>(buf + ((w + s + 1) % JB) * RS, bot);
          be = bes[s & 1][(w + s + 1) % JB];
        }
      }
      store_row<E>(X + (long)rt * L, L, okt, top);
      const int rb = b1 * JB + (w + JB - 1) % JB;
      store_row<E>(X + (long)rb * L, L, rb < p, bot);
      __builtin_amdgcn_s_waitcnt(0);  // this wave's row stores have completed
      __syncthreads();
      if (tid == 0) {
        __hip_atomic_store(&ver[b0], expect + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ver[b1], expect + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    // sweep bookkeeping: counter (sweep % 3) collects this sweep's rotations
    if (lane == 0 && local_rot) atomicAdd(&ctr[2 + (sweep % 3)], local_rot);
    local_rot = 0;
    grid_barrier(ctr, gridDim.x);
    if (tid == 0) {
      s_tot = __hip_atomic_load(&ctr[2 + (sweep % 3)], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (blockIdx.x == 0)
        __hip_atomic_store(&ctr[2 + ((sweep + 2) % 3)], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (s_tot == 0) {
      converged = 1;
      ++sweep;
      break;
    }
  }
  // sweeps executed (the last one without any rotation when converged) and
  // whether a sweep without rotations was reached within the cap
  if (blockIdx.x == 0 && tid == 0) {
    sweeps_out[0] = sweep;
    sweeps_out[1] = converged;
  }
}

// sigma_i = ||X_i||, perm sorts them descending (ties by index).
__global__ __launch_bounds__(1024) void k_norms_sort(const double* __restrict__ X, int p, int L,
                                                     double* __restrict__ sig_sorted, int* __restrict__ perm) {
  extern __shared__ double sg[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // four rows per wave at a time, all their loads in flight together
  for (int i0 = 4 * wave; i0 < p; i0 += 64) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = lane; c < L; c += 64) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (i0 + u < p) ? X[(long)(i0 + u) * L + c] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += v[u] * v[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double t = wave_sum(s[u]);
      if (lane == 0 && i0 + u < p) sg[i0 + u] = sqrt(t);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < p; i += 1024) {
    const double si = sg[i];
    int pos = 0;
    for (int j = 0; j < p; ++j) {
      const double sj = sg[j];
      pos += (sj > si) || (sj == si && j < i);
    }
    perm[pos] = i;
    sig_sorted[pos] = si;
  }
}

__global__ void k_truncate(const double* __restrict__ sig, int cnt, const double* __restrict__ norm_dev,
                           double rel_tol, int nbonds, long max_rank, TruncOut* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double nrm = norm_dev[0];
  const double delta = (nbonds > 0) ? rel_tol * nrm / sqrt((double)nbonds) : 0.0;
  // tail2(r) = sum_{i >= r} sigma_i^2, accumulated from the smallest value upwards
  int r = cnt;
  double acc = 0.0;
  double tail_r = 0.0, tail_rm1 = 0.0;
  // walk r from cnt down to 1; the smallest admissible r is the last one found
  for (int cand = cnt; cand >= 1; --cand) {
    // acc = tail2(cand)
    if (sqrt(acc) <= delta) {
      r = cand;
    } else {
      break;
    }
    acc += sig[cand - 1] * sig[cand - 1];
  }
  int capped = 0;
  if (max_rank > 0 && r > max_rank) {
    r = (int)max_rank;
    capped = 1;
  }
  if (r < 1) r = 1;
  if (r > cnt) r = cnt;
  double t2 = 0.0;
  for (int i = cnt - 1; i >= r; --i) t2 += sig[i] * sig[i];
  tail_r = sqrt(t2);
  tail_rm1 = sqrt(t2 + sig[r - 1] * sig[r - 1]);
  out->rank = r;
  out->capped = capped;
  out->tail_r = tail_r;
  out->tail_rm1 = tail_rm1;
  out->norm = nrm;
  out->delta = delta;
}

// dst[j][:] = src[perm[j]][:]  (rows in descending-norm order)
__global__ void k_permute_rows(const double* __restrict__ src, int p, int L, const int* __restrict__ perm,
                               double* __restrict__ dst) {
  const long total = (long)p * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / L), c = (int)(e % L);
    dst[e] = src[(long)perm[j] * L + c];
  }
}

__global__ void k_gather_rows(const double* __restrict__ X, int L, const int* __restrict__ perm,
                              const double* __restrict__ sig, const TruncOut* __restrict__ t,
                              double* __restrict__ out, long ldo) {
  const int r = t->rank;
  const long total = (long)r * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / L), c = (int)(e % L);
    const double s = sig[j];
    out[(long)j * ldo + c] = (s > 0.0) ? X[(long)perm[j] * L + c] / s : 0.0;
  }
}

// Rows of V (rb x L): V[j] = X[perm[j]] / sig[j] for j < r = t->rank (zero
// when sig[j] is zero), zero rows for r <= j < rb.
__global__ void k_gather_rows_padded(const double* __restrict__ X, int L, const int* __restrict__ perm,
                                     const double* __restrict__ sig, const TruncOut* __restrict__ t,
                                     double* __restrict__ V, int rb) {
  const int r = t->rank;
  const long total = (long)rb * L;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / L), c = (int)(e % L);
    double v = 0.0;
    if (j < r) {
      const double s = sig[j];
      v = (s > 0.0) ? X[(long)perm[j] * L + c] / s : 0.0;
    }
    V[e] = v;
  }
}

// out[a][i r + c] = B[a][i rb + c] for c < r = *r_dev (r <= rb); the rest of
// each output row (length d rb) is zero.  Moves the kept columns of every
// physical index to the front, so that a matrix whose rank r is known only on
// the device has exactly zero trailing columns.
__global__ void k_compact_cols(const double* __restrict__ B, int rows, int d, int rb, const int* __restrict__ r_dev,
                               double* __restrict__ out) {
  const int r = *r_dev;
  const long w = (long)d * rb;
  const long total = (long)rows * w;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long a = e / w;
    const int q = (int)(e % w);
    double v = 0.0;
    if (q < d * r) {
      const int i = q / r, c = q % r;
      v = B[a * w + (long)i * rb + c];
    }
    out[e] = v;
  }
}

// Compact core [r0, w] with w = d r1 (r0 = *r0_dev, r1 = *r1_dev): the
// leading w entries of the first r0 rows of V (row length L).
__global__ void k_core_from_rows(const double* __restrict__ V, int L, const int* __restrict__ r0_dev, int d,
                                 const int* __restrict__ r1_dev, double* __restrict__ out, int rows_bound) {
  const int r0 = *r0_dev, w = d * *r1_dev;
  const long total = (long)min(r0, rows_bound) * w;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long j = e / w;
    const int c = (int)(e % w);
    out[e] = V[j * L + c];
  }
}

// Ranks and status of a rounding from the per-bond decisions: ranks[0] =
// ranks[n] = 1, ranks[k] = t[k-1].rank; status 0, or the (negative) code of a
// non-finite norm or of a Jacobi run that did not converge (sweeps: two ints
// per bond, the second the converged flag).
__global__ void k_round_record(const TruncOut* __restrict__ t, const int* __restrict__ sweeps, int n,
                               const double* __restrict__ norm_dev, long long* __restrict__ ranks,
                               int* __restrict__ status, int code_nonfinite, int code_noconv) {
  if (blockIdx.x != 0) return;
  for (int k = threadIdx.x; k <= n; k += blockDim.x) ranks[k] = (k == 0 || k == n) ? 1 : t[k - 1].rank;
  if (threadIdx.x == 0) {
    int st = 0;
    const double nr = norm_dev[0];
    if (!(nr == nr) || nr > 1.7976931348623157e308) st = code_nonfinite;
    for (int k = 1; st == 0 && k < n; ++k)
      if (!sweeps[2 * (k - 1) + 1]) st = code_noconv;
    status[0] = st;
  }
}

inline int gsz(long n) {
  long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > (1 << 20)) g = 1 << 20;
  return (int)g;
}

constexpr int kJacobiBigLds = 2 * JB * 64 * 16 * 8;  // k_jacobi<16>: 16 row slots of 1024 doubles

}  // namespace

hipError_t jacobi_configure() {
  return hipFuncSetAttribute((const void*)k_jacobi<16>, hipFuncAttributeMaxDynamicSharedMemorySize, kJacobiBigLds);
}

hipError_t jacobi_rows(hipStream_t s, double* X, int p, int L, unsigned* counter, int max_sweeps,
                       int* sweeps_dev, const double* ref_norm) {
  if (p <= 0 || L <= 0) return hipSuccess;
  if (L > 1024 || p > 1024) return hipErrorInvalidValue;
  const int nblk = (p + JB - 1) / JB;
  const int nb2 = nblk + (nblk & 1);
  hipError_t e = fill_u32(s, counter, 0u, JCTR + nb2);
  if (e != hipSuccess) return e;
  const int grid = nb2 / 2;
  // tolerance on |a.c| / (||a|| ||c||)
  const double tol = 2.220446049250313e-16 * sqrt((double)L);
  // deflation level relative to the largest squared row norm: (8 u sqrt(p))^2
  double defl = 64.0 * 0x1p-106 * (double)p;
  void* args[] = {&X, &p, &L, &counter, &max_sweeps, &sweeps_dev, (void*)&tol, (void*)&ref_norm, (void*)&defl};
  const void* fn;
  int E;
  if (L <= 64) {
    fn = (const void*)k_jacobi<1>, E = 1;
  } else if (L <= 128) {
    fn = (const void*)k_jacobi<2>, E = 2;
  } else if (L <= 256) {
    fn = (const void*)k_jacobi<4>, E = 4;
  } else if (L <= 512) {
    fn = (const void*)k_jacobi<8>, E = 8;
  } else {
    fn = (const void*)k_jacobi<16>, E = 16;
  }
  const size_t shmem = (size_t)2 * JB * 64 * E * sizeof(double);
  // only the E = 16 instance needs more than 64 KiB; jacobi_configure()
  // raises its limit when a handle is created
  if (shmem > (E == 16 ? kJacobiBigLds : 64 * 1024)) return hipErrorInvalidValue;
  // Algorithmic work of the launch under the fixed SVD convention: 8 sweeps
  // of 9 n^3 (n = min(p, L)), whatever the sweeps taken; bytes: the matrix
  // read once and written once.
  if (prof::active(prof::JACOBI)) {
    const double nn = (double)std::min(p, L);
    prof::begin(s, prof::JACOBI, 2.0 * 8.0 * (double)p * L, 8.0 * 9.0 * nn * nn * nn);
  }
  e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(JNT), args, shmem, s);
  prof::end(s);
  return e;
}

hipError_t row_norms_sorted(hipStream_t s, const double* X, int p, int L, double* sig_sorted, int* perm) {
  if (p <= 0) return hipSuccess;
  const size_t shmem = (size_t)p * sizeof(double);
  if (shmem > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_norms_sort, dim3(1), dim3(1024), shmem, s, X, p, L, sig_sorted, perm);
  return hipGetLastError();
}

hipError_t permute_rows(hipStream_t s, const double* src, int p, int L, const int* perm, double* dst) {
  if (p <= 0 || L <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_rows, dim3(gsz((long)p * L)), dim3(256), 0, s, src, p, L, perm, dst);
  return hipGetLastError();
}

hipError_t truncate_decide(hipStream_t s, const double* sig, int cnt, const double* norm_dev, double rel_tol,
                           int nbonds, long max_rank, TruncOut* out_dev) {
  hipLaunchKernelGGL(k_truncate, dim3(1), dim3(64), 0, s, sig, cnt, norm_dev, rel_tol, nbonds, max_rank, out_dev);
  return hipGetLastError();
}

hipError_t gather_rows_padded(hipStream_t s, const double* X, int L, const int* perm, const double* sig,
                              const TruncOut* t, double* V, int rb) {
  if (rb <= 0 || L <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows_padded, dim3(gsz((long)rb * L)), dim3(256), 0, s, X, L, perm, sig, t, V, rb);
  return hipGetLastError();
}

hipError_t compact_cols(hipStream_t s, const double* B, int rows, int d, int rb, const int* r_dev, double* out) {
  if (rows <= 0 || d <= 0 || rb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact_cols, dim3(gsz((long)rows * d * rb)), dim3(256), 0, s, B, rows, d, rb, r_dev, out);
  return hipGetLastError();
}

hipError_t core_from_rows(hipStream_t s, const double* V, int rows_bound, int L, const int* r0_dev, int d,
                          const int* r1_dev, double* out) {
  if (rows_bound <= 0 || L <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_core_from_rows, dim3(gsz((long)rows_bound * L)), dim3(256), 0, s, V, L, r0_dev, d, r1_dev,
                     out, rows_bound);
  return hipGetLastError();
}

hipError_t round_record(hipStream_t s, const TruncOut* t, const int* sweeps, int n, const double* norm_dev,
                        long long* ranks, int* status, int code_nonfinite, int code_noconv) {
  hipLaunchKernelGGL(k_round_record, dim3(1), dim3(64), 0, s, t, sweeps, n, norm_dev, ranks, status, code_nonfinite,
                     code_noconv);
  return hipGetLastError();
}

hipError_t gather_rows_normalized(hipStream_t s, const double* X, int L, const int* perm, const double* sig,
                                  const TruncOut* t, double* out, long ldo, int rmax_host) {
  hipLaunchKernelGGL(k_gather_rows, dim3(gsz((long)rmax_host * L)), dim3(256), 0, s, X, L, perm, sig, t, out, ldo);
  return hipGetLastError();
}


}  // namespace qtt
