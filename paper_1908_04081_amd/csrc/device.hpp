// Device-side building blocks for gfx950 (wave64): CSR row products with a
// group of LPR lanes per row, deterministic reductions, XCD-aware tile maps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctl.hpp"

namespace assg {

constexpr int WAVE = 64;
constexpr int NXCD = 8;          // MI355X: 8 XCDs, workgroups dispatched round-robin

// ---------------------------------------------------------------- loads
template <typename T>
__device__ __forceinline__ T ldnt(const T* p) { return __builtin_nontemporal_load(p); }

// ------------------------------------------------------- wave reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, WAVE));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// Orders LDS traffic between lanes of one wave (a wave executes its LDS
// operations in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over a group of LPR consecutive lanes (butterfly, fixed order).
template <int LPR>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = LPR / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Sum of one value per thread over a workgroup of NT threads, deterministic;
// the result is valid in thread 0.  ``sh`` needs NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i) s += sh[i];
  }
  __syncthreads();
  return s;
}

// ------------------------------------------------------------ tile maps
// Workgroup b runs on XCD b % 8.  Logical id L makes every XCD own one
// contiguous range of logical ids, so neighbouring rows of a stencil
// (planes of a 3-D grid) are read through the same L2.  nb % 8 == 0.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  return (b % NXCD) * (nb / NXCD) + b / NXCD;
}
// Contiguous tile range [t0, t1) of logical workgroup L out of nb over ntiles.
__device__ __forceinline__ void tile_range(int L, int nb, int64_t ntiles, int64_t& t0,
                                           int64_t& t1) {
  t0 = (ntiles * L) / nb;
  t1 = (ntiles * (L + 1)) / nb;
}

// ----------------------------------------------------------- CSR rows
// Lane ``sub`` of a group of LPR lanes accumulates entries sub, sub+LPR, ...
// of the row; the group then sums with a butterfly.  A's arrays are read
// with non-temporal loads (streamed once per sweep, no reuse), the source
// vector through the caches (its entries are reused by neighbouring rows).
template <int LPR>
__device__ __forceinline__ double csr_dot(const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ ci,
                                          const double* __restrict__ va,
                                          const double* __restrict__ x, int64_t row, int sub,
                                          bool active) {
  double acc = 0.0;
  if (active) {
    const int32_t s = rp[row], e = rp[row + 1];
    for (int32_t k = s + sub; k < e; k += LPR) acc = fma(ldnt(va + k), x[ldnt(ci + k)], acc);
  }
  return group_sum<LPR>(acc);
}

// Two right-hand sides stored as pairs: both chains of the matrix powers
// share each read of A and each 16-byte gather.
template <int LPR>
__device__ __forceinline__ double2 csr_dot2(const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ ci,
                                            const double* __restrict__ va,
                                            const double2* __restrict__ x, int64_t row, int sub,
                                            bool active) {
  double ax = 0.0, ay = 0.0;
  if (active) {
    const int32_t s = rp[row], e = rp[row + 1];
    for (int32_t k = s + sub; k < e; k += LPR) {
      const double a = ldnt(va + k);
      const double2 v = x[ldnt(ci + k)];
      ax = fma(a, v.x, ax);
      ay = fma(a, v.y, ay);
    }
  }
  return make_double2(group_sum<LPR>(ax), group_sum<LPR>(ay));
}

// ------------------------------------------------ last-block reductions
// Each workgroup stores its partial, then the last one to arrive sums all
// partials in index order (deterministic for a fixed launch shape) and
// returns true in thread 0 with the total in ``total``.
__device__ __forceinline__ bool last_block_total(double part, double* partials, Ctl* ctl,
                                                 double* total, double* sh) {
  __shared__ bool am_last;
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = part;
    __threadfence();
    const uint32_t prev =
        __hip_atomic_fetch_add(&ctl->counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
  // fixed-order sum: thread t sums partials t, t+NT, ...; then a fixed tree
  double s = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
    s += __hip_atomic_load(partials + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s = wave_sum(s);
  const int w = threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) sh[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) t += sh[i];
    *total = t;
    ctl->counter = 0u;   // ready for the next reduction on this stream
  }
  return threadIdx.x == 0;
}

}  // namespace assg
