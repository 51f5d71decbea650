// lbpc_probe.hip -- memory-ceiling probes for the benchmark (not part of the
// step library): what the HBM delivers to streaming kernels over 16-byte
// vectors -- a copy, the same with non-temporal accesses, read only and write
// only.  (The step's own access pattern is timed by lbpc_memory_probe of the
// step library, which runs the step kernel's loads and stores without its
// arithmetic.)
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming kernels over 16-byte vectors: each thread moves UNR vectors per
// pass (all loads issued before the first store), grid-stride.  NT selects
// non-temporal accesses.
template <int UNR, bool NT>
__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ src,
                                              u32x4* __restrict__ dst,
                                              long long n) {
  const long long step = (long long)gridDim.x * 256 * UNR;
  for (long long base = (long long)blockIdx.x * 256 * UNR + threadIdx.x;
       base < n; base += step) {
    u32x4 v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) v[u] = NT ? __builtin_nontemporal_load(&src[i]) : src[i];
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) {
        if (NT)
          __builtin_nontemporal_store(v[u], &dst[i]);
        else
          dst[i] = v[u];
      }
    }
  }
}

// Read only: the vectors' xor, one 16-byte result per thread (kept so the
// loads are not removed).
template <int UNR>
__global__ __launch_bounds__(256) void k_read(const u32x4* __restrict__ src,
                                              u32x4* __restrict__ out,
                                              long long n) {
  u32x4 acc = {0u, 0u, 0u, 0u};
  const long long step = (long long)gridDim.x * 256 * UNR;
  for (long long base = (long long)blockIdx.x * 256 * UNR + threadIdx.x;
       base < n; base += step) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) {
        const u32x4 v = src[i];
        acc ^= v;
      }
    }
  }
  out[(long long)blockIdx.x * 256 + threadIdx.x] = acc;
}

// Write only.
template <int UNR>
__global__ __launch_bounds__(256) void k_write(u32x4* __restrict__ dst,
                                               long long n) {
  const u32x4 v = {1u, 2u, 3u, 4u};
  const long long step = (long long)gridDim.x * 256 * UNR;
  for (long long base = (long long)blockIdx.x * 256 * UNR + threadIdx.x;
       base < n; base += step) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) dst[i] = v;
    }
  }
}

}  // namespace

extern "C" {

// Streaming probes over `bytes` (a multiple of 16) on `stream`, with
// `blocks` blocks of 256 threads (grid-stride): kind 0 copies src to dst,
// 1 the same with non-temporal accesses, 2 reads src only (dst receives
// blocks x 256 x 16 bytes), 3 writes dst only.  Returns 0, -1 for an unknown
// kind, -2 when the launch fails.
int lbpc_probe_stream(int kind, const void* src, void* dst, size_t bytes,
                      int blocks, void* stream) {
  const long long n = (long long)(bytes / 16);
  hipStream_t s = (hipStream_t)stream;
  const u32x4* a = (const u32x4*)src;
  u32x4* b = (u32x4*)dst;
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    case 1: hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    case 2: hipLaunchKernelGGL((k_read<4>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    case 3: hipLaunchKernelGGL((k_write<4>), dim3(blocks), dim3(256), 0, s, b, n); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
