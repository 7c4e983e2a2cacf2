// copy.hip -- a plain streaming device-to-device copy: the measured
// bandwidth reference the kernels' HBM rates are read against, beside the
// published peak.  Each lane moves 16 bytes per access with U accesses in
// flight (all loads of a round issued before its stores), grid-stride over
// the buffer with enough 256-thread groups for eight wavefronts per SIMD;
// NT selects the non-temporal load/store forms (no reuse is expected).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/envpic.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int CB = 256;         // threads per group
constexpr int COPY_GROUPS = 2048;  // 256 CUs x 8 groups of 4 wavefronts

template <int U, bool NT>
__global__ __launch_bounds__(CB) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                    size_t n16) {
  const size_t stride = (size_t)gridDim.x * CB * U;
  for (size_t base = (size_t)blockIdx.x * CB * U + threadIdx.x; base < n16; base += stride) {
    u32x4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = base + (size_t)u * CB;
      if (k < n16) v[u] = NT ? __builtin_nontemporal_load(&src[k]) : src[k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const size_t k = base + (size_t)u * CB;
      if (k < n16) {
        if (NT)
          __builtin_nontemporal_store(v[u], &dst[k]);
        else
          dst[k] = v[u];
      }
    }
  }
}

}  // namespace

extern "C" int envpic_stream_copy(void* dst, const void* src, size_t bytes, int variant, void* stream) {
  if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0) return ENVPIC_EINVAL;
  if (variant < 0 || variant > 3) return ENVPIC_EINVAL;
  const size_t n16 = bytes / 16;
  if (n16 == 0) return ENVPIC_OK;
  const int unroll = variant & 1 ? 8 : 4;
  const size_t need = (n16 + (size_t)CB * unroll - 1) / ((size_t)CB * unroll);
  const int groups = (int)(need < (size_t)COPY_GROUPS ? need : (size_t)COPY_GROUPS);
  hipStream_t st = (hipStream_t)stream;
  const u32x4* s = (const u32x4*)src;
  u32x4* d = (u32x4*)dst;
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_stream_copy<4, false>), dim3(groups), dim3(CB), 0, st, s, d, n16); break;
    case 1: hipLaunchKernelGGL((k_stream_copy<8, false>), dim3(groups), dim3(CB), 0, st, s, d, n16); break;
    case 2: hipLaunchKernelGGL((k_stream_copy<4, true>), dim3(groups), dim3(CB), 0, st, s, d, n16); break;
    default: hipLaunchKernelGGL((k_stream_copy<8, true>), dim3(groups), dim3(CB), 0, st, s, d, n16); break;
  }
  return hipGetLastError() == hipSuccess ? ENVPIC_OK : ENVPIC_EDEVICE;
}
