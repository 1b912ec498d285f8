// Device-side helpers shared by the QTT kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtt {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- bf16 split
__device__ __forceinline__ unsigned short bf16_bits_rne(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ double bf16_bits_to_double(unsigned short h) {
  return (double)__uint_as_float(((unsigned)h) << 16);
}
// a = p0 + p1 + p2 (+ remainder), each p the RNE bf16 of what is left.
__device__ __forceinline__ void split3(double a, unsigned short& p0, unsigned short& p1,
                                      unsigned short& p2) {
  p0 = bf16_bits_rne((float)a);
  double r = a - bf16_bits_to_double(p0);
  p1 = bf16_bits_rne((float)r);
  r -= bf16_bits_to_double(p1);
  p2 = bf16_bits_rne((float)r);
}

constexpr int WAVE = 64;

// DPP lane exchange inside a row of 16 lanes (no LDS traffic).
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8
constexpr int DPP_MIRROR = 0x140;       // lane i <-> 15 - i within 16
constexpr int DPP_ROW_ROR8 = 0x128;     // lane i <- lane (i + 8) % 16 within 16

// Sum over the 16 lanes of each row; all 16 lanes get the same bits.
__device__ __forceinline__ double row_sum(double v) {
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  v += dpp<DPP_HALF_MIRROR>(v);
  v += dpp<DPP_MIRROR>(v);
  return v;
}

// Bit-exact read of one lane's double (the readlane builtin converts a
// double operand to an integer, so the two 32-bit halves are read instead).
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave; uniform result.
__device__ __forceinline__ double wave_sum(double v) {
  v = row_sum(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

// Sum of one value over the whole workgroup; every thread gets the result.
// `scratch` must hold NT/64 doubles.  Contains two barriers.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  constexpr int NW = NT / WAVE;
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  v = wave_sum(v);
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += scratch[w];
  __syncthreads();
  return s;
}

// Row-level transpose reduction of 16 values per lane: afterwards lane L
// holds the sum over its row (16 lanes) of value index L % 16.  The pairing
// order (mirror, half mirror, xor 2, xor 1) keeps partners' index sets
// aligned: each step splits on one lane bit, 8 + 4 + 2 + 1 DPP exchanges.
__device__ __forceinline__ double row_sum16(const double (&x)[16]) {
  const int l = threadIdx.x & 15;
  double y[8];
  const bool b3 = (l & 8) != 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double send = b3 ? x[i] : x[i + 8];
    const double keep = b3 ? x[i + 8] : x[i];
    y[i] = keep + dpp<DPP_MIRROR>(send);
  }
  double z[4];
  const bool b2 = (l & 4) != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b2 ? y[i] : y[i + 4];
    const double keep = b2 ? y[i + 4] : y[i];
    z[i] = keep + dpp<DPP_HALF_MIRROR>(send);
  }
  double u[2];
  const bool b1 = (l & 2) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b1 ? z[i] : z[i + 2];
    const double keep = b1 ? z[i + 2] : z[i];
    u[i] = keep + dpp<DPP_XOR2>(send);
  }
  const bool b0 = (l & 1) != 0;
  const double send = b0 ? u[0] : u[1];
  const double keep = b0 ? u[1] : u[0];
  return keep + dpp<DPP_XOR1>(send);
}

// Workgroup sum of 16 values per thread; result written to out[16] (LDS),
// visible to all threads on return.  red must hold (NT/16)*16 doubles
// (one slot per row of 16 lanes and value).
template <int NT>
__device__ __forceinline__ void block_sum16(const double (&x)[16], double* red, double* out) {
  constexpr int NR = NT / 16;  // rows of 16 lanes
  const double r = row_sum16(x);
  red[threadIdx.x] = r;  // row (threadIdx.x / 16), value (threadIdx.x % 16)
  __syncthreads();
  if constexpr (NR > 16) {
    // two levels: 16 groups of NR/16 rows, then the 16 group sums
    constexpr int G = NR / 16;
    double s = 0.0;
    if (threadIdx.x < 256) {
#pragma unroll
      for (int w = 0; w < G; ++w) s += red[((threadIdx.x >> 4) * G + w) * 16 + (threadIdx.x & 15)];
    }
    __syncthreads();
    if (threadIdx.x < 256) red[threadIdx.x] = s;
    __syncthreads();
  }
  constexpr int NR2 = NR > 16 ? 16 : NR;
  if (threadIdx.x < 16) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NR2; ++w) s += red[w * 16 + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Row-level transpose reduction of 8 values per lane: afterwards lane L
// holds the sum over its row (16 lanes) of value index L % 8.  Three
// splitting steps inside each half row (partners by half mirror, xor 2,
// xor 1: 4 + 2 + 1 DPP exchanges), then the two half rows are added by a
// rotation of the row by 8 lanes.
__device__ __forceinline__ double row_sum8(const double (&x)[8]) {
  const int l = threadIdx.x & 15;
  double y[4];
  const bool b2 = (l & 4) != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b2 ? x[i] : x[i + 4];
    const double keep = b2 ? x[i + 4] : x[i];
    y[i] = keep + dpp<DPP_HALF_MIRROR>(send);
  }
  double z[2];
  const bool b1 = (l & 2) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b1 ? y[i] : y[i + 2];
    const double keep = b1 ? y[i + 2] : y[i];
    z[i] = keep + dpp<DPP_XOR2>(send);
  }
  const bool b0 = (l & 1) != 0;
  const double send = b0 ? z[0] : z[1];
  const double keep = b0 ? z[1] : z[0];
  const double u = keep + dpp<DPP_XOR1>(send);
  return u + dpp<DPP_ROW_ROR8>(u);
}

// Adds the four rows of 16 lanes lane by lane (row swaps of gfx950): every
// lane L gets the sum over lanes L % 16 + 16 q, q = 0..3.
__device__ __forceinline__ double rows_add(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v = __longlong_as_double((long long)(((unsigned long long)b[0] << 32) | a[0])) +
      __longlong_as_double((long long)(((unsigned long long)b[1] << 32) | a[1]));
  const unsigned long long w = (unsigned long long)__double_as_longlong(v);
  const unsigned lo2 = (unsigned)w, hi2 = (unsigned)(w >> 32);
  const auto c = __builtin_amdgcn_permlane32_swap(lo2, lo2, false, false);
  const auto d = __builtin_amdgcn_permlane32_swap(hi2, hi2, false, false);
  return __longlong_as_double((long long)(((unsigned long long)d[0] << 32) | c[0])) +
         __longlong_as_double((long long)(((unsigned long long)d[1] << 32) | c[1]));
}

// Workgroup sum of one value with a single barrier: slots holds 2 sets of
// NT/64 doubles used alternately (par), so that consecutive calls need no
// barrier to protect the slots.  Every thread gets the same bits.
template <int NT>
__device__ __forceinline__ double wg_sum1(double v, double* slots, int par) {
  constexpr int NW = NT / WAVE;
  v = rows_add(row_sum(v));
  if ((threadIdx.x & (WAVE - 1)) == 0) slots[par * NW + threadIdx.x / WAVE] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += slots[par * NW + w];
  return s;
}

// Workgroup sums of NV (8 or 16) values per thread with a single barrier;
// slots holds 2 sets of (NT/64) * NV doubles used alternately.  out[c] is
// the total of value c, the same bits in every thread (read back from one
// lane, so it is uniform across the wave).
template <int NT, int NV>
__device__ __forceinline__ void wg_sum_vals(const double (&x)[NV], double* slots, int par, double (&out)[NV]) {
  static_assert(NV == 8 || NV == 16, "8 or 16 values");
  constexpr int NW = NT / WAVE;
  double r;
  if constexpr (NV == 8) r = row_sum8(x);
  else r = row_sum16(x);
  r = rows_add(r);
  const int lane = threadIdx.x & (WAVE - 1);
  double* base = slots + par * NW * NV;
  if (lane < NV) base[(threadIdx.x / WAVE) * NV + lane] = r;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += base[w * NV + (lane & (NV - 1))];
#pragma unroll
  for (int c = 0; c < NV; ++c) out[c] = readlane_f64(t, c);
}

// Sum over the 64 lanes with the row broadcasts of DPP: after the row sums,
// row 3 accumulates rows 0-2 (row_bcast:15 into rows 1 and 3, row_bcast:31
// into rows 2 and 3); lane 63 holds the total, read back for every lane.
__device__ __forceinline__ double wave_sum_bc(double v) {
  v = row_sum(v);
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x142, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x143, 0xC, 0xF, false);
  return readlane_f64(v, 63);
}

// 1/sqrt(x) and 1/x for x in [2^-3, 2^3]: single-precision hardware
// estimate (relative error e ~ 2^-22), then one correction step of third
// order, r (1 + e/2 + 3 e^2 / 8) and r (1 + e + e^2), which leaves a
// truncation error ~e^3 (below double rounding) in fewer dependent steps
// than two Newton iterations.
__device__ __forceinline__ double rsq_f64(double x) {
  const double r = (double)__builtin_amdgcn_rsqf((float)x);
  const double e = fma(-x * r, r, 1.0);
  return fma(r * e, fma(0.375, e, 0.5), r);
}
__device__ __forceinline__ double rcp_f64(double x) {
  const double r = (double)__builtin_amdgcn_rcpf((float)x);
  const double e = fma(-x, r, 1.0);
  return fma(r, fma(e, e, e), r);
}

// Plane rotation of the one-sided Jacobi method for rows a, c with
// al = ||a||^2, be = ||c||^2, ga = a.c: returns false when the pair is
// orthogonal to the tolerance (|a.c| <= tol ||a|| ||c||), else (cs, sn) with
// [a; c] <- [cs a - sn c; sn a + cs c] making the pair orthogonal.
__device__ __forceinline__ bool jacobi_rotation(double al, double be, double ga, double tol, double& cs_out,
                                                double& sn_out, double& t_out) {
  // squared form of the test inside the safe range
  const bool safe = fmin(al, be) > 1e-140 && fmax(al, be) < 1e140;
  const bool rot = ga != 0.0 && (safe ? (ga * ga > (tol * tol) * (al * be)) : (fabs(ga) > tol * sqrt(al) * sqrt(be)));
  // With d = be - al, g = 2 ga (scaled by a power of two so that the larger
  // magnitude lies in [0.5, 1); the ratios below do not change):
  //   h = sqrt(d^2 + g^2), u = h + |d|, w = 1/sqrt(2 h u),
  //   cs = u w, sn = sign(d g) |g| w, t = sn/cs = sign(d g) |g| / u,
  // i.e. t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with zeta = d / g and
  // cs = (1 + t^2)^(-1/2), sn = cs t; 1/sqrt(2 h u) and 1/u are independent.
  // Evaluated whether or not the pair rotates, so that it overlaps the test.
  double d = be - al, g = 2.0 * ga;
  const int ke = __builtin_amdgcn_frexp_exp(fmax(fabs(d), fabs(g)));
  d = __builtin_amdgcn_ldexp(d, -ke);
  g = __builtin_amdgcn_ldexp(g, -ke);
  const double x = fma(d, d, g * g);  // in [0.25, 2)
  const double h = x * rsq_f64(x);
  const double u = h + fabs(d);       // in [0.5, 2.5)
  const double w = rsq_f64(2.0 * h * u);
  const double ru = rcp_f64(u);
  const double ag = copysign(fabs(g), d * g);
  cs_out = u * w;
  sn_out = ag * w;
  t_out = ag * ru;  // the new squared norms are al - t ga and be + t ga
  return rot;
}

__device__ __forceinline__ bool jacobi_rotation(double al, double be, double ga, double tol, double& cs_out,
                                                double& sn_out) {
  double t;
  return jacobi_rotation(al, be, ga, tol, cs_out, sn_out, t);
}

// Grid-wide barrier for co-resident persistent workgroups (cooperative launch).
// counter[0] = arrivals, counter[1] = generation.  Vector atomics only.
__device__ __forceinline__ void grid_barrier(unsigned* counter, unsigned nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned gen = __hip_atomic_load(&counter[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned arrived = __hip_atomic_fetch_add(&counter[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&counter[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&counter[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(&counter[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(2);
      }
    }
  }
  __syncthreads();
}

}  // namespace qtt
