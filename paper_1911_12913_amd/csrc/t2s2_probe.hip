// Reference copy kernel for the step kernel's roofline.  It reads the nine
// population planes of a state and writes them to another buffer, one
// element per lane and plane, with the step kernel's store policy
// (non-temporal stores for 8-byte elements, ordinary stores otherwise).  A
// step reads and writes every state element once, so the bandwidth of this
// copy on the same buffers is the practical ceiling of the step; the
// published HBM peak is the other reference.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "t2s2_internal.h"

namespace t2s2 {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void copy_planes_kernel(const T* __restrict__ src,
                                                          T* __restrict__ dst, long long plane) {
  const long long i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= plane) return;
  T v[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) v[q] = src[q * plane + i];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    if constexpr (sizeof(T) == 8)
      __builtin_nontemporal_store(v[q], dst + q * plane + i);
    else
      dst[q * plane + i] = v[q];
  }
}

template <typename T>
hipError_t launch_copy(const void* src, void* dst, long long plane, hipStream_t s) {
  const long long grid = (plane + 255) / 256;
  hipLaunchKernelGGL(copy_planes_kernel<T>, dim3(static_cast<unsigned>(grid)), dim3(256), 0, s,
                     static_cast<const T*>(src), static_cast<T*>(dst), plane);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_copy_probe(const void* src, void* dst, long long plane, int elem_bytes,
                             hipStream_t s) {
  switch (elem_bytes) {
    case 8: return launch_copy<unsigned long long>(src, dst, plane, s);
    case 4: return launch_copy<unsigned int>(src, dst, plane, s);
    case 2: return launch_copy<unsigned short>(src, dst, plane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace t2s2
