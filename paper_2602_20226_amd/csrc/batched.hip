// Batched contract + round: many independent QTT products of uneven ranks in
// one persistent launch.
//
// A grid of persistent workgroups (256 threads each) pulls instance indices
// from an atomic work queue; instances are queued in decreasing order of an
// estimated cost (sum over cores of rho^2 r_C + p^3), so that the largest
// ones start first and the small ones fill the tail.  A workgroup runs the
// whole pipeline of its instance with workgroup-level versions of the
// single-chain steps:
//   QR sweep:  bond product R_{k-1} C_k (factored: R X_k, then the A or
//              W core), blocked Householder QR (qr_panel_dev + apply_tile_dev);
//   SVD sweep: Q_k [U Sigma; 0], QR of tall unfoldings, one-sided block
//              Jacobi on the rows, device-side rank decision, V^T into the
//              output core and U Sigma = F V.
// The three product steps (R X_k, the core product, F V) run on the bf16
// matrix cores (wg_gemm.hpp: six products of a three-piece split, FP32
// accumulation inside each 32-deep step, FP64 across steps), with the tile
// shape of each shape bucket taken from the plan's TileMap.
// Ranks never leave the device during the launch, so the launch (with the
// queue reset before it) can be captured in a hipGraph and replayed.
#include "qtt_device.hpp"
#include "qtt_internal.hpp"
#include "qr_device.hpp"
#include "batched.hpp"
#include "wg_gemm.hpp"

namespace qtt {

namespace {

constexpr int BNT = 256;

struct Smem {
  union {  // the QR's tile reductions, or the staging of a matrix-core GEMM step
    double red[BNT / 16][16][17];
    GemmTiles gt;
  };
  double wsh[16][17];
  double w2sh[16][17];
  double tsh[16][17];
  double scal[16];
  double jn[16];  // squared norms of the 16 rows of a Jacobi visit
  int iscal[8];
};

__device__ __forceinline__ void wg_sync() { __syncthreads(); }

// Y = R (rows x K, ld ldr) * B (K x N, ld N)
__device__ void wg_gemm_nn(const TileMap& tm, int rows, int N, int K, const double* __restrict__ R, long ldr,
                           const double* __restrict__ B, double* __restrict__ Y, Smem& sm) {
  wg_gemm_split(
      tm, rows, N, K, [=](int m, int k) { return R[(long)m * ldr + k]; },
      [=](int k, int n) { return B[(long)k * N + n]; }, [=](int m, int n, double v) { Y[(long)m * N + n] = v; },
      sm.gt);
}

// Y (p x r) = F (p x L) * V^T, V = out core rows (r x L)
__device__ void wg_gemm_nt(const TileMap& tm, int p, int r, int L, const double* __restrict__ F,
                           const double* __restrict__ V, double* __restrict__ Y, Smem& sm) {
  wg_gemm_split(
      tm, p, r, L, [=](int m, int k) { return F[(long)m * L + k]; },
      [=](int k, int n) { return V[(long)n * L + k]; }, [=](int m, int n, double v) { Y[(long)m * r + n] = v; },
      sm.gt);
}

// Hadamard bond: M[(a,i),(b,dd)] = sum_mu Y[a,mu,i,dd] A[mu,i,b]
// MPO bond:      M[(a,i),(b,dd)] = sum_{mu,j} Y[a,mu,j,dd] W[mu,i,j,b]
// One GEMM per (i, dd): rows a, columns b, depth (mu, j).
__device__ void wg_bond_apply(const TileMap& tm, bool mpo, const double* __restrict__ Y, int rho, int ra0, int d,
                              int dj, int rb1, const double* __restrict__ A, int ra1, double* __restrict__ M,
                              Smem& sm) {
  const int dk = mpo ? dj : 1;  // contracted physical leg per mu
  const long ldo = (long)d * ra1 * rb1;
  for (int i = 0; i < d; ++i)
    for (int dd = 0; dd < rb1; ++dd) {
      if (mpo) {
        wg_gemm_split(
            tm, rho, ra1, ra0 * dk,
            [=](int a, int kk) { return Y[((long)a * ra0 * dk + kk) * rb1 + dd]; },
            [=](int kk, int b) {
              const int mu = kk / dk, j = kk % dk;
              return A[(((long)mu * d + i) * dj + j) * ra1 + b];
            },
            [=](int a, int b, double v) { M[(long)a * ldo + ((long)i * ra1 + b) * rb1 + dd] = v; }, sm.gt);
      } else {
        wg_gemm_split(
            tm, rho, ra1, ra0, [=](int a, int mu) { return Y[(((long)a * ra0 + mu) * d + i) * rb1 + dd]; },
            [=](int mu, int b) { return A[((long)mu * d + i) * ra1 + b]; },
            [=](int a, int b, double v) { M[(long)a * ldo + ((long)i * ra1 + b) * rb1 + dd] = v; }, sm.gt);
      }
    }
}

__device__ void wg_copy_pad(const double* __restrict__ src, int rows, int cols, long lds, double* __restrict__ dst,
                            int rows_out, long ldd) {
  const long n = (long)rows_out * cols;
  for (long e = threadIdx.x; e < n; e += BNT) {
    const long r = e / cols;
    const int c = (int)(e % cols);
    dst[r * ldd + c] = (r < rows) ? src[r * lds + c] : 0.0;
  }
  wg_sync();
}

__device__ void wg_extract_r(const double* __restrict__ A, int kr, int n, long lda, double* __restrict__ R) {
  const long total = (long)kr * n;
  for (long e = threadIdx.x; e < total; e += BNT) {
    const long i = e / n;
    const int j = (int)(e % n);
    R[e] = (j >= i) ? A[i * lda + j] : 0.0;
  }
  wg_sync();
}

// Householder QR of A (m x n, m <= 512) by this workgroup, T blocks in Tbuf.
__device__ void wg_householder_qr(double* __restrict__ A, int m, int n, long lda, double* __restrict__ Tbuf, Smem& sm) {
  const int kmax = min(m, n);
  for (int j0 = 0, p = 0; j0 < kmax; j0 += 16, ++p) {
    const int pw = min(16, kmax - j0);
    double* T = Tbuf + (long)p * 256;
    if (m - j0 <= 256)
      qr_panel_dev<BNT, 1, 16>(A, lda, m, j0, pw, T);
    else
      qr_panel_dev<BNT, 2, 16>(A, lda, m, j0, pw, T);
    wg_sync();
    for (int c0 = j0 + pw; c0 < n; c0 += 16)
      apply_tile_dev<BNT>(A + (long)j0 * lda + j0, lda, m - j0, pw, T, A + (long)j0 * lda, lda, c0, n, 1, sm.red,
                          sm.wsh, sm.w2sh, sm.tsh);
  }
}

// Y <- Q Y for the reflectors stored in A (m rows, kref reflectors).
__device__ void wg_apply_q(const double* __restrict__ A, int m, int kref, long lda, const double* __restrict__ Tbuf,
                           double* __restrict__ Y, int ncols, long ldy, Smem& sm) {
  const int np = (kref + 15) / 16;
  for (int p = np - 1; p >= 0; --p) {
    const int j0 = 16 * p, pw = min(16, kref - j0);
    for (int c0 = 0; c0 < ncols; c0 += 16)
      apply_tile_dev<BNT>(A + (long)j0 * lda + j0, lda, m - j0, pw, Tbuf + (long)p * 256, Y + (long)j0 * ldy, ldy, c0,
                          ncols, 0, sm.red, sm.wsh, sm.w2sh, sm.tsh);
  }
}

__device__ __forceinline__ int rr_item(int pos, int round, int n) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (n - 1));
}

// One-sided Jacobi on the rows of X (p x L) by this workgroup; blocks of JB
// rows, block pairs visited sequentially in the round-robin order, each pair
// staged in LDS with its squared row norms.  A visit rotates the JB x JB cross pairs (JB steps of JB
// disjoint pairs, waves taking pairs in turn); the pairs inside each block
// are rotated once per sweep, in the first round.  Returns the sweeps
// executed when a sweep without rotations was reached within max_sweeps,
// -1 otherwise.
constexpr int JEMAX = 12;  // row elements per lane: L <= 768

// Rotate rows xa, xc (LDS, length L) whose squared norms *na, *nc (LDS) are
// carried through the visit: one dot product and one wave sum per pair, each
// row read once; the new norms are ||a||^2 - t a.c and ||c||^2 + t a.c.
// A nonzero row whose squared norm is below negl is set to zero instead of
// being rotated (same rule as the single-chain Jacobi: a row that has become
// an exact tiny multiple of another cannot be rotated away).
__device__ __forceinline__ int wg_rotate(double* __restrict__ xa, double* __restrict__ xc, double* __restrict__ na,
                                         double* __restrict__ nc, int L, double tol, double negl) {
  const int lane = threadIdx.x & 63;
  {
    const double al = *na, be = *nc;
    if (al < negl || be < negl) {
      int changed = 0;
      if (al < negl && al > 0.0) {
        for (int c = lane; c < L; c += 64) xa[c] = 0.0;
        changed = 1;
      }
      if (be < negl && be > 0.0) {
        for (int c = lane; c < L; c += 64) xc[c] = 0.0;
        changed = 1;
      }
      if (changed && lane == 0) {
        if (al < negl) *na = 0.0;
        if (be < negl) *nc = 0.0;
      }
      return changed;
    }
  }
  double u[JEMAX], w[JEMAX];
  double ga = 0.0;
#pragma unroll
  for (int q = 0; q < JEMAX; ++q) {
    const int c = lane + 64 * q;
    u[q] = c < L ? xa[c] : 0.0;
    w[q] = c < L ? xc[c] : 0.0;
    ga += u[q] * w[q];
  }
  ga = wave_sum_bc(ga);
  const double al = *na, be = *nc;
  double cs, sn, t;
  if (!jacobi_rotation(al, be, ga, tol, cs, sn, t)) return 0;
#pragma unroll
  for (int q = 0; q < JEMAX; ++q) {
    const int c = lane + 64 * q;
    if (c < L) {
      xa[c] = cs * u[q] - sn * w[q];
      xc[c] = sn * u[q] + cs * w[q];
    }
  }
  if (lane == 0) {
    *na = al - t * ga;
    *nc = be + t * ga;
  }
  return 1;
}

// wg_rotate with row a held in registers by the calling wave (ua, its
// squared norm na in a register of every lane) and row c in LDS: the same
// arithmetic, so the same results.
__device__ __forceinline__ int wg_rotate_reg(double (&ua)[JEMAX], double& na, double* __restrict__ xc,
                                             double* __restrict__ nc, int L, double tol, double negl) {
  const int lane = threadIdx.x & 63;
  const double al = na, be = *nc;
  if (al < negl || be < negl) {
    int changed = 0;
    if (al < negl && al > 0.0) {
#pragma unroll
      for (int q = 0; q < JEMAX; ++q) ua[q] = 0.0;
      changed = 1;
    }
    if (be < negl && be > 0.0) {
      for (int c = lane; c < L; c += 64) xc[c] = 0.0;
      changed = 1;
    }
    if (changed) {
      if (al < negl) na = 0.0;
      if (lane == 0 && be < negl) *nc = 0.0;
    }
    return changed;
  }
  double w[JEMAX];
  double ga = 0.0;
#pragma unroll
  for (int q = 0; q < JEMAX; ++q) {
    const int c = lane + 64 * q;
    w[q] = c < L ? xc[c] : 0.0;
    ga += ua[q] * w[q];
  }
  ga = wave_sum_bc(ga);
  double cs, sn, t;
  if (!jacobi_rotation(al, be, ga, tol, cs, sn, t)) return 0;
#pragma unroll
  for (int q = 0; q < JEMAX; ++q) {
    const int c = lane + 64 * q;
    const double u = ua[q];
    if (c < L) {
      ua[q] = cs * u - sn * w[q];
      xc[c] = sn * u + cs * w[q];
    }
  }
  na = al - t * ga;
  if (lane == 0) *nc = be + t * ga;
  return 1;
}

template <int JB>
__device__ int wg_jacobi(double* __restrict__ X, int p, int L, double* __restrict__ sh, int max_sweeps, double tol,
                         Smem& sm) {
  constexpr int JR = 2 * JB;
  constexpr int NW = BNT / 64;
  const int nblk = (p + JB - 1) / JB;
  const int nb2 = nblk + (nblk & 1);
  const int npairs = nb2 / 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // deflation level: (8 u sqrt(p))^2 times the largest squared input row
  // norm (rows at the rounding noise of the input are set to zero, as in the
  // single-chain Jacobi)
  {
    double mx = 0.0;
    for (int i = wave; i < p; i += NW) {
      double s2 = 0.0;
      for (int c = lane; c < L; c += 64) s2 += X[(long)i * L + c] * X[(long)i * L + c];
      mx = fmax(mx, wave_sum_bc(s2));
    }
    if (lane == 0) sm.scal[12 + wave] = mx;
    wg_sync();
  }
  const double negl =
      64.0 * 0x1p-106 * (double)p * fmax(fmax(sm.scal[12], sm.scal[13]), fmax(sm.scal[14], sm.scal[15]));
  // a block pair's rows, this wave's share (rows t = wave + NW h of the pair),
  // loaded into registers with every load issued before any is used
  constexpr int RW = (2 * JB + NW - 1) / NW;
  double v[RW][JEMAX];
  auto fetch = [&](int f0, int f1) {
#pragma unroll
    for (int h = 0; h < RW; ++h) {
      const int t = wave + NW * h;
      const int gr = (t < JB ? f0 : f1) * JB + (t % JB);
      const bool ok = t < JR && gr < p;
#pragma unroll
      for (int e = 0; e < JEMAX; ++e) {
        const int c = lane + 64 * e;
        v[h][e] = (ok && c < L) ? X[(long)gr * L + c] : 0.0;
      }
    }
  };
  int sweep = 0;
  bool converged = false;
  for (; sweep < max_sweeps; ++sweep) {
    if (tid == 0) sm.iscal[0] = 0;
    wg_sync();
    for (int round = 0; round < max(nb2 - 1, 1); ++round) {
      for (int pair = 0; pair < npairs; ++pair) {
        const int b0 = rr_item(pair, round, nb2);
        const int b1 = (nb2 > 1) ? rr_item(nb2 - 1 - pair, round, nb2) : 1;
        // the pair's rows into LDS, squared row norms formed on the way and
        // carried through the visit
        {
          fetch(b0, b1);
#pragma unroll
          for (int h = 0; h < RW; ++h) {
            const int t = wave + NW * h;
            double s2 = 0.0;
            if (t < JR) {
#pragma unroll
              for (int e = 0; e < JEMAX; ++e) {
                const int c = lane + 64 * e;
                if (c < L) {
                  sh[t * L + c] = v[h][e];
                  s2 += v[h][e] * v[h][e];
                }
              }
            }
            s2 = wave_sum_bc(s2);
            if (lane == 0 && t < JR) sm.jn[t] = s2;
          }
        }
        wg_sync();
        int rot = 0;
        if (round == 0) {
          // pairs inside each block: JB - 1 steps of JB / 2 disjoint pairs per block
          for (int st = 0; st < JB - 1; ++st) {
            for (int q = wave; q < JB; q += NW) {
              const int blk = q / (JB / 2), i = q % (JB / 2);
              const int ta = blk * JB + rr_item(i, st, JB), tc = blk * JB + rr_item(JB - 1 - i, st, JB);
              rot += wg_rotate(sh + ta * L, sh + tc * L, &sm.jn[ta], &sm.jn[tc], L, tol, negl);
            }
            wg_sync();
          }
        }
        // cross pairs: at step s top row q meets bottom row (q + s) % JB.
        // Wave w keeps its top rows q = w + NW h in registers for the whole
        // visit; only the bottom rows pass through LDS.
        static_assert(JB % NW == 0 || JB < NW, "top rows per wave");
        constexpr int TH = JB >= NW ? JB / NW : 1;
        double ur[TH][JEMAX], nr[TH];
#pragma unroll
        for (int h = 0; h < TH; ++h) {
          const int q = wave + NW * h;
          const bool own = q < JB;
#pragma unroll
          for (int e = 0; e < JEMAX; ++e) {
            const int c = lane + 64 * e;
            ur[h][e] = (own && c < L) ? sh[q * L + c] : 0.0;
          }
          nr[h] = own ? sm.jn[q] : 0.0;
        }
        for (int s = 0; s < JB; ++s) {
#pragma unroll
          for (int h = 0; h < TH; ++h) {
            const int q = wave + NW * h;
            if (q < JB) {
              const int tc = JB + (q + s) % JB;
              rot += wg_rotate_reg(ur[h], nr[h], sh + tc * L, &sm.jn[tc], L, tol, negl);
            }
          }
          wg_sync();
        }
#pragma unroll
        for (int h = 0; h < TH; ++h) {
          const int q = wave + NW * h;
          if (q < JB) {
#pragma unroll
            for (int e = 0; e < JEMAX; ++e) {
              const int c = lane + 64 * e;
              if (c < L) sh[q * L + c] = ur[h][e];
            }
            if (lane == 0) sm.jn[q] = nr[h];
          }
        }
        wg_sync();
        if (lane == 0 && rot) atomicAdd(&sm.iscal[0], rot);
        for (int t = wave; t < JR; t += NW) {
          const int gr = (t < JB ? b0 : b1) * JB + (t % JB);
          if (gr < p)
            for (int c = lane; c < L; c += 64) X[(long)gr * L + c] = sh[t * L + c];
        }
        wg_sync();
      }
    }
    const int tot = sm.iscal[0];
    wg_sync();
    if (tot == 0) {
      converged = true;
      ++sweep;
      break;
    }
  }
  return converged ? sweep : -1;
}

// sigma (sorted descending) and perm of the row norms of X (p x L).
__device__ void wg_norms_sort(const double* __restrict__ X, int p, int L, double* __restrict__ sig,
                              int* __restrict__ perm, double* __restrict__ tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = wave; i < p; i += BNT / 64) {
    double s = 0.0;
    for (int c = lane; c < L; c += 64) {
      const double v = X[(long)i * L + c];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) tmp[i] = sqrt(s);
  }
  wg_sync();
  for (int i = threadIdx.x; i < p; i += BNT) {
    const double si = tmp[i];
    int pos = 0;
    for (int j = 0; j < p; ++j) {
      const double sj = tmp[j];
      pos += (sj > si) || (sj == si && j < i);
    }
    perm[pos] = i;
    sig[pos] = si;
  }
  wg_sync();
}

template <int JB>
__device__ void process_instance(const BInst& I, const TileMap& tm, double rel_tol, long max_rank, int max_sweeps,
                                 double* __restrict__ sh, Smem& sm,
                                 long* __restrict__ ranks_out, double* __restrict__ tail_out, int* __restrict__ status) {
  const int n = I.n;
  double* ws = I.ws;
  double* R = ws + I.offR;
  double* Yb = ws + I.offY;
  double* one = ws + I.offOne;
  const bool mpo = I.mpo != 0;
  const int tid = threadIdx.x;
  // ---------------- QR sweep
  for (int k = 0; k < n; ++k) {
    const int rho0 = I.rho[k];
    const int cols = I.ra[k + 1] * I.rb[k + 1];
    const bool last = (k == n - 1);
    double* M = last ? ws + I.offCenter : ws + I.offM[k];
    const int ra0 = I.ra[k], ra1 = I.ra[k + 1], rb0 = I.rb[k], rb1 = I.rb[k + 1];
    const int d = I.d[k], dj = I.dj[k];
    const double* Rk = R;
    if (k == 0) {
      if (tid == 0) one[0] = 1.0;
      wg_sync();
      Rk = one;
    }
    wg_gemm_nn(tm, rho0 * ra0, dj * rb1, rb0, Rk, rb0, I.b[k], Yb, sm);
    wg_bond_apply(tm, mpo, Yb, rho0, ra0, d, dj, rb1, I.a[k], ra1, M, sm);
    if (!last) {
      const int m = rho0 * d;
      wg_householder_qr(M, m, cols, cols, ws + I.offT[k], sm);
      wg_extract_r(M, I.rho[k + 1], cols, cols, R);
    }
  }
  // norm of the centre
  {
    const double* c = ws + I.offCenter;
    const long cnt = (long)I.rho[n - 1] * I.d[n - 1];
    double s = 0.0;
    for (long e = tid; e < cnt; e += BNT) s += c[e] * c[e];
    s = block_sum<BNT>(s, sm.scal);
    if (tid == 0) sm.scal[8] = sqrt(s);
    wg_sync();
  }
  const double nrm = sm.scal[8];
  if (!(nrm == nrm) || nrm > 1.7e308) {
    if (tid == 0) status[0] = QTT_BSTATUS_NONFINITE;
    return;
  }
  const double delta = (n > 1) ? rel_tol * nrm / sqrt((double)(n - 1)) : 0.0;
  double* Z = ws + I.offZ;
  double* X = ws + I.offX;
  double* Xc = ws + I.offXc;
  double* Yn = ws + I.offYn;
  double* TB = ws + I.offTB;
  double* sig = ws + I.offSig;
  int* perm = (int*)(ws + I.offPerm);
  double* tmp = ws + I.offTmp;
  const double eps = 2.220446049250313e-16;
  int rnext = 1;
  if (tid == 0) {
    ranks_out[0] = 1;
    ranks_out[n] = 1;
    status[0] = QTT_BSTATUS_OK;
  }
  for (int k = n - 1; k >= 1; --k) {
    const int rows = I.rho[k];
    const int D = I.d[k] * rnext;
    const double* B;
    if (k == n - 1) {
      B = ws + I.offCenter;
    } else {
      wg_copy_pad(Yn, I.rho[k + 1], rnext, rnext, Z, I.m[k], rnext);
      wg_apply_q(ws + I.offM[k], I.m[k], I.rho[k + 1], (long)I.ra[k + 1] * I.rb[k + 1], ws + I.offT[k], Z, rnext,
                 rnext, sm);
      B = Z;
    }
    const bool tall = rows >= D;
    const int L = D;
    int p;
    if (tall) {
      if (B != Z) wg_copy_pad(B, rows, D, D, Z, rows, D);
      wg_householder_qr(Z, rows, D, D, TB, sm);
      wg_extract_r(Z, D, D, D, X);
      p = D;
    } else {
      wg_copy_pad(B, rows, D, D, X, rows, D);
      p = rows;
    }
    wg_copy_pad(X, p, L, L, Xc, p, L);
    const int sweeps = wg_jacobi<JB>(X, p, L, sh, max_sweeps, eps * sqrt((double)L), sm);
    if (sweeps < 0 && tid == 0) status[0] = QTT_BSTATUS_NOCONV;
    wg_norms_sort(X, p, L, sig, perm, tmp);
    // rank decision (smallest r with discarded 2-norm <= delta, capped)
    if (tid == 0) {
      int r = p;
      double acc = 0.0;
      for (int cand = p; cand >= 1; --cand) {
        if (sqrt(acc) <= delta)
          r = cand;
        else
          break;
        acc += sig[cand - 1] * sig[cand - 1];
      }
      if (max_rank > 0 && r > max_rank) r = (int)max_rank;
      if (r < 1) r = 1;
      double t2 = 0.0;
      for (int i = p - 1; i >= r; --i) t2 += sig[i] * sig[i];
      sm.iscal[1] = r;
      tail_out[k - 1] = sqrt(t2);
    }
    wg_sync();
    const int r = sm.iscal[1];
    double* core = I.out[k];
    for (long e = tid; e < (long)r * L; e += BNT) {
      const int j = (int)(e / L), c = (int)(e % L);
      const double s = sig[j];
      core[(long)j * L + c] = (s > 0.0) ? X[(long)perm[j] * L + c] / s : 0.0;
    }
    wg_sync();
    wg_gemm_nt(tm, p, r, L, Xc, core, Yn, sm);
    if (tall) {
      for (long e = tid; e < (long)(rows - p) * r; e += BNT) Yn[(long)p * r + e] = 0.0;
      wg_sync();
      wg_apply_q(Z, rows, p, D, TB, Yn, r, r, sm);
    }
    if (tid == 0) ranks_out[k] = r;
    rnext = r;
  }
  if (n == 1) {
    wg_copy_pad(ws + I.offCenter, 1, I.d[0], I.d[0], I.out[0], 1, I.d[0]);
  } else {
    wg_copy_pad(Yn, I.rho[1], rnext, rnext, Z, I.m[0], rnext);
    wg_apply_q(ws + I.offM[0], I.m[0], I.rho[1], (long)I.ra[1] * I.rb[1], ws + I.offT[0], Z, rnext, rnext, sm);
    wg_copy_pad(Z, I.m[0], rnext, rnext, I.out[0], I.m[0], rnext);
  }
}

template <int JB>
__global__ __launch_bounds__(BNT) void k_batched(const BInst* __restrict__ insts, const int* __restrict__ order,
                                                 int count, unsigned* __restrict__ queue, TileMap tm, double rel_tol,
                                                 long max_rank, int max_sweeps, long* __restrict__ ranks_out,
                                                 double* __restrict__ tails_out, int* __restrict__ status) {
  extern __shared__ double sh[];
  __shared__ Smem sm;
  __shared__ int s_idx;
  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= count) break;
    const int inst = order[idx];
    process_instance<JB>(insts[inst], tm, rel_tol, max_rank, max_sweeps, sh, sm, ranks_out + (long)inst * (QTT_BATCH_MAXN + 1),
                         tails_out + (long)inst * QTT_BATCH_MAXN, status + inst);
    __syncthreads();
  }
}

// Tuner probe: every workgroup of the grid computes the same C = A B (A M x K,
// B K x N, row-major) with one tile variant, as the persistent kernel's
// workgroups do side by side; workgroup 0 writes C.
template <int TM, int TN>
__global__ __launch_bounds__(BNT) void k_tile_probe(int M, int N, int K, const double* __restrict__ A,
                                                    const double* __restrict__ B, double* __restrict__ C) {
  __shared__ GemmTiles gt;
  const bool w = blockIdx.x == 0;
  wg_gemm_split_tile<TM, TN>(
      M, N, K, [=](int m, int k) { return A[(long)m * K + k]; }, [=](int k, int n) { return B[(long)k * N + n]; },
      [=](int m, int n, double v) {
        if (w) C[(long)m * N + n] = v;
      },
      gt);
}

}  // namespace

hipError_t tile_probe_launch(hipStream_t s, int variant, int grid, int M, int N, int K, const double* A,
                             const double* B, double* C) {
  switch (variant) {
    case 1:
      hipLaunchKernelGGL((k_tile_probe<64, 32>), dim3(grid), dim3(BNT), 0, s, M, N, K, A, B, C);
      break;
    case 2:
      hipLaunchKernelGGL((k_tile_probe<32, 64>), dim3(grid), dim3(BNT), 0, s, M, N, K, A, B, C);
      break;
    case 3:
      hipLaunchKernelGGL((k_tile_probe<32, 32>), dim3(grid), dim3(BNT), 0, s, M, N, K, A, B, C);
      break;
    default:
      hipLaunchKernelGGL((k_tile_probe<64, 64>), dim3(grid), dim3(BNT), 0, s, M, N, K, A, B, C);
      break;
  }
  return hipGetLastError();
}

hipError_t batched_configure() {
  // up to 96 KiB of dynamic LDS (the Jacobi visit's 2 JB rows); raised for
  // both instances when a handle is created
  hipError_t e = hipFuncSetAttribute((const void*)k_batched<4>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_batched<8>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
}

hipError_t batched_launch(hipStream_t s, int variant, int grid, const BInst* insts, const int* order, int count,
                          unsigned* queue, const TileMap& tm, double rel_tol, long max_rank, int max_sweeps,
                          long* ranks_out, double* tails_out, int* status, int max_L) {
  hipError_t e = fill_u32(s, queue, 0u, 1);
  if (e != hipSuccess) return e;
  const int jb = (variant & 1) ? 4 : 8;
  const size_t shmem = (size_t)2 * jb * max_L * sizeof(double);
  if (shmem > 96 * 1024) return hipErrorInvalidValue;
  if (jb == 4) {
    hipLaunchKernelGGL(k_batched<4>, dim3(grid), dim3(BNT), shmem, s, insts, order, count, queue, tm, rel_tol, max_rank,
                       max_sweeps, ranks_out, tails_out, status);
  } else {
    hipLaunchKernelGGL(k_batched<8>, dim3(grid), dim3(BNT), shmem, s, insts, order, count, queue, tm, rel_tol, max_rank,
                       max_sweeps, ranks_out, tails_out, status);
  }
  return hipGetLastError();
}

}  // namespace qtt
