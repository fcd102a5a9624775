// Memory-bandwidth probes: a streaming read, a streaming copy, and reads
// that may be served by the caches (see bwprobe.h).  One workgroup of 256
// threads moves one contiguous 32 KiB piece: 8 rounds of 256 x 16-byte
// loads, all issued before the first use.
#include <hip/hip_runtime.h>

#include "bwprobe.h"

namespace {

constexpr int NT = 256;
constexpr int ROUNDS = 8;
constexpr size_t PIECE = (size_t)NT * 16 * ROUNDS;   // 32 KiB

typedef double dv2 __attribute__((ext_vector_type(2)));

template <bool NTL>
__global__ __launch_bounds__(NT) void k_read(const dv2* __restrict__ buf,
                                             double* __restrict__ partial) {
  const size_t base = (size_t)blockIdx.x * (PIECE / 16);
  dv2 v[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) {
    const dv2* p = buf + base + (size_t)j * NT + threadIdx.x;
    v[j] = NTL ? __builtin_nontemporal_load(p) : *p;
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j) s += v[j].x + v[j].y;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  __shared__ double sh[NT / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(NT) void k_copy(const dv2* __restrict__ src, dv2* __restrict__ dst) {
  const size_t base = (size_t)blockIdx.x * (PIECE / 16);
  dv2 v[ROUNDS];
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j)
    v[j] = __builtin_nontemporal_load(src + base + (size_t)j * NT + threadIdx.x);
#pragma unroll
  for (int j = 0; j < ROUNDS; ++j)
    __builtin_nontemporal_store(v[j], dst + base + (size_t)j * NT + threadIdx.x);
}

template <class F>
int timed(int iters, float* ms_avg, F launch) {
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -2;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return -2;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    launch(s);   // untimed first run
    if (hipEventRecord(e0, s) == hipSuccess) {
      for (int i = 0; i < iters; ++i) launch(s);
      float ms = 0.f;
      if (hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
          hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
        *ms_avg = ms / (float)iters;
        rc = 0;
      }
    }
  }
  (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  return rc;
}

bool bad_size(size_t bytes) { return bytes == 0 || bytes % PIECE != 0 || bytes / PIECE > 0x7fffffffu; }

}  // namespace

extern "C" int assg_bw_read(const void* buf, size_t bytes, int nontemporal, int iters,
                            double* partial, float* ms_avg) {
  if (!buf || !partial || !ms_avg || iters < 1 || bad_size(bytes)) return -1;
  const unsigned grid = (unsigned)(bytes / PIECE);
  const dv2* b = static_cast<const dv2*>(buf);
  return timed(iters, ms_avg, [&](hipStream_t s) {
    if (nontemporal)
      hipLaunchKernelGGL(k_read<true>, dim3(grid), dim3(NT), 0, s, b, partial);
    else
      hipLaunchKernelGGL(k_read<false>, dim3(grid), dim3(NT), 0, s, b, partial);
  });
}

extern "C" int assg_bw_copy(const void* src, void* dst, size_t bytes, int iters, float* ms_avg) {
  if (!src || !dst || !ms_avg || iters < 1 || bad_size(bytes)) return -1;
  const char* a = static_cast<const char*>(src);
  char* d = static_cast<char*>(dst);
  if (a < d + bytes && d < a + bytes) return -1;
  const unsigned grid = (unsigned)(bytes / PIECE);
  return timed(iters, ms_avg, [&](hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(NT), 0, s, reinterpret_cast<const dv2*>(a),
                       reinterpret_cast<dv2*>(d));
  });
}
