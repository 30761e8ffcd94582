// HBM streaming-copy probe: the practical ceiling of a kernel that reads N
// bytes and writes N bytes once each, the access budget of one lattice
// Boltzmann step (every population read once and written once).  A
// measurement tool beside the library, not part of the step.
//
// Each lane moves 16-byte (dwordx4) items with a grid-stride loop, UNROLL
// independent items in flight per iteration; stores are plain or
// nontemporal.  The caller sweeps the grid size (waves per CU) and these
// variants and keeps the fastest.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hbm_probe.h"

namespace {

// 16-byte item as a clang vector (the nontemporal builtin takes vectors of
// scalars, not HIP's u32x4 wrapper)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int UNROLL, bool NT>
__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                              size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
    u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      if (NT)
        __builtin_nontemporal_store(v[u], dst + i + u * stride);
      else
        dst[i + u * stride] = v[u];
    }
  }
  for (; i < n; i += stride) {
    const u32x4 v = src[i];
    if (NT)
      __builtin_nontemporal_store(v, dst + i);
    else
      dst[i] = v;
  }
}

template <int UNROLL>
hipError_t launch(const u32x4* s, u32x4* d, size_t n, int blocks, int threads, int nt,
                  hipStream_t st) {
  if (nt)
    hipLaunchKernelGGL((k_copy<UNROLL, true>), dim3(blocks), dim3(threads), 0, st, s, d, n);
  else
    hipLaunchKernelGGL((k_copy<UNROLL, false>), dim3(blocks), dim3(threads), 0, st, s, d, n);
  return hipGetLastError();
}

}  // namespace

extern "C" int hbm_copy(const void* src, void* dst, size_t bytes, int blocks, int threads, int nt,
                        int unroll, void* stream) {
  if (!src || !dst || bytes % 16 != 0 || blocks < 1 || threads < 64 || threads > 256 ||
      threads % 64 != 0)
    return -1;
  if ((uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0) return -1;
  const size_t n = bytes / 16;
  const u32x4* s = (const u32x4*)src;
  u32x4* d = (u32x4*)dst;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  switch (unroll) {
    case 1: e = launch<1>(s, d, n, blocks, threads, nt, st); break;
    case 2: e = launch<2>(s, d, n, blocks, threads, nt, st); break;
    case 4: e = launch<4>(s, d, n, blocks, threads, nt, st); break;
    default: return -1;
  }
  return e == hipSuccess ? 0 : -3;
}
