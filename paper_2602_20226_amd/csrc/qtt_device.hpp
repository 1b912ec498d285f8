// Device-side helpers shared by the QTT kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qtt {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
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

// Wave-level reduction of 16 values per lane into one value per lane.
// After the call, lane L holds the wave sum of value index
//   v(L) = 8*bit5 + 4*bit4 + 2*bit3 + bit2,
// replicated over the four lanes that differ in bits 0..1.
// 17 exchanges instead of 16 full butterflies.
__device__ __forceinline__ double wave_sum16(const double (&x)[16], int& vidx) {
  const int lane = threadIdx.x & (WAVE - 1);
  double y[8];
  const bool hi5 = (lane & 32) != 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double send = hi5 ? x[i] : x[i + 8];
    double keep = hi5 ? x[i + 8] : x[i];
    y[i] = keep + __shfl_xor(send, 32, WAVE);
  }
  double z[4];
  const bool hi4 = (lane & 16) != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double send = hi4 ? y[i] : y[i + 4];
    double keep = hi4 ? y[i + 4] : y[i];
    z[i] = keep + __shfl_xor(send, 16, WAVE);
  }
  double u[2];
  const bool hi3 = (lane & 8) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    double send = hi3 ? z[i] : z[i + 2];
    double keep = hi3 ? z[i + 2] : z[i];
    u[i] = keep + __shfl_xor(send, 8, WAVE);
  }
  const bool hi2 = (lane & 4) != 0;
  double send = hi2 ? u[0] : u[1];
  double keep = hi2 ? u[1] : u[0];
  double r = keep + __shfl_xor(send, 4, WAVE);
  r += __shfl_xor(r, 2, WAVE);
  r += __shfl_xor(r, 1, WAVE);
  vidx = (hi5 ? 8 : 0) + (hi4 ? 4 : 0) + (hi3 ? 2 : 0) + (hi2 ? 1 : 0);
  return r;
}

// Workgroup sum of 16 values per thread; result written to out[16] (LDS),
// visible to all threads on return.  red must hold (NT/64)*16 doubles.
template <int NT>
__device__ __forceinline__ void block_sum16(const double (&x)[16], double* red, double* out) {
  constexpr int NW = NT / WAVE;
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  int v;
  double r = wave_sum16(x, v);
  if ((lane & 3) == 0) red[wid * 16 + v] = r;
  __syncthreads();
  if (threadIdx.x < 16) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w * 16 + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
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
