// Device-side building blocks for gfx950 (wave64): CSR-stream row blocks,
// deterministic reductions, XCD-aware workgroup maps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ctl.hpp"
#include "partition.hpp"

namespace assg {

// ------------------------------------------------------- debug builds
// Built with -DASSG_DEBUG, the kernels check the partition and index
// invariants they rely on and keep the first failed check's code in a
// device word of their translation unit, which the host reads (and clears)
// after each call; release builds compile the checks away.
#ifdef ASSG_DEBUG
static __device__ int g_debug_code;
#define ASSG_DCHECK(cond, code)                               \
  do {                                                        \
    if (!(cond) && g_debug_code == 0) g_debug_code = (code);  \
  } while (0)
#else
#define ASSG_DCHECK(cond, code) \
  do {                          \
  } while (0)
#endif

constexpr int WAVE = 64;

// ---------------------------------------------------------------- loads
// Streaming (non-temporal) accesses for data read or written once per
// kernel: they do not displace the gathered vectors from the caches, and on
// this part they raise the bandwidth of many concurrent streams.
template <typename T>
__device__ __forceinline__ T ldnt(const T* p) { return __builtin_nontemporal_load(p); }
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldnt2(const double2* p) {
  const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stnt(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void stnt2(double2* p, double2 v) {
  const dvec2 w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<dvec2*>(p));
}

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

// ------------------------------------------- DPP/readlane wave reductions
// Cross-lane moves within rows of 16 lanes by DPP (no LDS crossbar), the
// four row results combined through readlane.  The order of the additions
// is fixed, so the result is deterministic and uniform across the wave.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Lane l receives lane l + 1's value (DPP wave shift left by one); lane 63
// receives 0.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_shl1_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
__device__ __forceinline__ double wave_min_dpp(double v) {
  v = fmin(v, dpp_mov<0xB1>(v));
  v = fmin(v, dpp_mov<0x4E>(v));
  v = fmin(v, dpp_mov<0x141>(v));
  v = fmin(v, dpp_mov<0x140>(v));
  return fmin(fmin(readlane_d(v, 0), readlane_d(v, 16)), fmin(readlane_d(v, 32), readlane_d(v, 48)));
}
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_mov<0xB1>(v));
  v = fmax(v, dpp_mov<0x4E>(v));
  v = fmax(v, dpp_mov<0x141>(v));
  v = fmax(v, dpp_mov<0x140>(v));
  return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Orders LDS traffic between lanes of one wave (a wave executes its LDS
// operations in order; this keeps the compiler from moving them).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// ------------------------------------------------------ CSR-stream rows
// Source vectors of a product: x[c] (one chain), the pair (x_P[c], x_R[c])
// (both chains of the matrix powers from one 16-byte gather), or the P part
// of a pair vector.
struct Src1 {
  const double* __restrict__ x;
  __device__ __forceinline__ double2 get(int32_t c) const { return make_double2(x[c], 0.0); }
};
struct Src2 {
  const double2* __restrict__ x;
  __device__ __forceinline__ double2 get(int32_t c) const { return x[c]; }
};
struct SrcP {
  const double* __restrict__ x;   // pair vector viewed as doubles
  __device__ __forceinline__ double2 get(int32_t c) const {
    return make_double2(x[2 * (int64_t)c], 0.0);
  }
};

// Coalesced value/column loads of the nonzeros [e0, e0+ne) of one row
// block (ne <= CAP), thread t taking nonzeros t, t+NT, ...; indices are
// clamped into the block so every load is unconditional.  Issued apart
// from their use, so a kernel can fetch the next block while it works on
// the current one.
template <int NT, int CAP>
struct RowFetch {
  static constexpr int K = CAP / NT;
  double a[K];
  int32_t c[K];
  __device__ __forceinline__ void issue(const int32_t* __restrict__ ci,
                                        const double* __restrict__ va, int32_t e0, int32_t ne) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int32_t e = t + NT * k;
      const int32_t ee = e0 + (e < ne ? e : ne - 1);
      a[k] = ldnt(va + ee);
      c[k] = ldnt(ci + ee);
    }
  }
};

// Gathers src[c] for the fetched nonzeros and stores the products in LDS;
// after a barrier the owner of each row adds its row's products in column
// order (each product is rounded before the sum, as in a sequential CSR
// product).
template <int CH, int NT, int CAP, class S>
__device__ __forceinline__ void fetched_rows(const RowFetch<NT, CAP>& f, const S& src,
                                             int32_t ne, int32_t rs, int32_t re, bool own,
                                             double* prod, double& sx, double& sy,
                                             bool drain = false) {
  constexpr int K = CAP / NT;
  const int t = threadIdx.x;
  sx = 0.0;
  sy = 0.0;
  if (ne > 0) {
    double2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = src.get(f.c[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int32_t e = t + NT * k;
      if (e < ne) {
        if constexpr (CH == 2) {
          prod[2 * e] = f.a[k] * v[k].x;
          prod[2 * e + 1] = f.a[k] * v[k].y;
        } else {
          prod[e] = f.a[k] * v[k].x;
        }
      }
    }
  }
  // with direct-to-LDS loads in flight, every wave waits for them before the
  // barrier so their data is visible to the whole workgroup after it
  if (drain) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (own) {
    for (int32_t e = rs; e < re; ++e) {
      if constexpr (CH == 2) {
        const double2 p = reinterpret_cast<const double2*>(prod)[e];
        sx += p.x;
        sy += p.y;
      } else {
        sx += prod[e];
      }
    }
  }
}

// Row sums of a row longer than one block's nonzero capacity, reduced by
// the whole workgroup (valid in thread 0).
template <int CH, int NT, class S>
__device__ __forceinline__ void long_row(const int32_t* __restrict__ ci,
                                         const double* __restrict__ va, const S& src, int32_t e0,
                                         int32_t ne, double* red, double& sx, double& sy) {
  double px = 0.0, py = 0.0;
  for (int32_t e = threadIdx.x; e < ne; e += NT) {
    const double a = ldnt(va + e0 + e);
    const double2 v = src.get(ldnt(ci + e0 + e));
    px = fma(a, v.x, px);
    py = fma(a, v.y, py);
  }
  px = block_sum<NT>(px, red);
  if constexpr (CH == 2) py = block_sum<NT>(py, red);
  sx = px;
  sy = py;
}

// Row sums of one row block (rows r0.., nonzeros [e0, e0+ne)) for NT
// threads: fetch then products and row sums when the block fits (ne <=
// CAP), else the single long row by the whole workgroup.
template <int CH, int NT, int CAP, class S>
__device__ __forceinline__ void stream_rows(const int32_t* __restrict__ ci,
                                            const double* __restrict__ va, const S& src,
                                            int32_t e0, int32_t ne, int32_t rs, int32_t re,
                                            bool own, double* prod, double* red, double& sx,
                                            double& sy) {
  if (ne <= CAP) {
    RowFetch<NT, CAP> f;
    if (ne > 0) f.issue(ci, va, e0, ne);
    fetched_rows<CH, NT, CAP>(f, src, ne, rs, re, own, prod, sx, sy);
  } else {
    long_row<CH, NT>(ci, va, src, e0, ne, red, sx, sy);
  }
}

// Logical row-block range of this workgroup: [b0, b1) out of nblk, with
// the XCD-aware logical workgroup id.
__device__ __forceinline__ void block_range(int32_t nblk, int32_t& b0, int32_t& b1) {
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  b0 = (int32_t)(((int64_t)nblk * L) / gridDim.x);
  b1 = (int32_t)(((int64_t)nblk * (L + 1)) / gridDim.x);
}

// Chunk of a reduction kernel's workgroup (XCD-aware, one chunk per
// workgroup; the grid is nchunk) and its row blocks [b0, b1) and system.
template <class V>
__device__ __forceinline__ int32_t chunk_of(const V& A, int32_t& b0, int32_t& b1, int32_t& sys) {
  const int32_t c = xcd_logical(blockIdx.x, gridDim.x);
  ASSG_DCHECK(c >= 0 && c < A.nchunk, 11);
  b0 = A.cblk[c];
  b1 = A.cblk[c + 1];
  sys = A.csys ? A.csys[c] : 0;
  ASSG_DCHECK(b0 >= 0 && b0 <= b1 && b1 <= A.nblk, 12);
  ASSG_DCHECK(sys >= 0 && sys < A.nsys, 13);
  return c;
}
template <class V>
__device__ __forceinline__ int32_t block_sys(const V& A, int32_t b) {
  return A.bsys ? A.bsys[b] : 0;
}

// ------------------------------------------------------ grid reductions
// Grid kernels store one partial per workgroup (plain stores; the next
// kernel sees them at the kernel boundary, so no cross-workgroup fences are
// needed -- a device-scope release would write back the XCD's L2).  A
// one-workgroup kernel then sums them in index order: thread t adds
// partials t, t+NT, ... and the threads are combined by a fixed tree.
template <int NT>
__device__ __forceinline__ double finish_sum(const double* __restrict__ part, int n, double* sh) {
  constexpr int U = 16;   // independent loads in flight per thread; adds stay in index order
  double s = 0.0;
  for (int base = threadIdx.x; base < n; base += NT * U) {
    double v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int i = base + k * NT;
      v[k] = (i < n) ? part[i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k) s += v[k];
  }
  return block_sum<NT>(s, sh);
}


}  // namespace assg
