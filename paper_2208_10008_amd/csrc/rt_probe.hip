// Memory-system probes (declared in include/rt_probe.h): streaming reads over
// a chosen working set and a plain copy, for the traversal kernel's roofline
// and for calibrating the hardware byte counters.
#include <hip/hip_runtime.h>

#include "rt_internal.h"
#include "rt_probe.h"

namespace rt {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeGroups = 4096;  // copy kernel: 16 work-groups per compute unit
constexpr int kUnroll = 8;

// Work-group g reads `span` elements starting at element (g * span) mod
// elems, wrapping at the end of the buffer, `passes` times; lanes read
// consecutive 16-byte elements.
__global__ __launch_bounds__(kProbeThreads) void k_probe_read(const uint4* __restrict__ buf,
                                                              int64_t elems, int64_t span,
                                                              int passes,
                                                              uint32_t* __restrict__ sink) {
  const int64_t start = ((int64_t)blockIdx.x * span) % elems;
  uint32_t acc = 0;
  for (int p = 0; p < passes; ++p) {
    int64_t k = threadIdx.x;
    for (; k + (kUnroll - 1) * kProbeThreads < span; k += kUnroll * kProbeThreads) {
      uint4 v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        int64_t e = start + k + u * kProbeThreads;
        if (e >= elems) e -= elems;
        v[u] = buf[e];
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; k < span; k += kProbeThreads) {
      int64_t e = start + k;
      if (e >= elems) e -= elems;
      const uint4 v = buf[e];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
  __shared__ uint32_t s_acc[kProbeThreads / 64];
  if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = 0;
    for (int w = 0; w < kProbeThreads / 64; ++w) a ^= s_acc[w];
    sink[blockIdx.x] = a;
  }
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_copy(const uint4* __restrict__ src,
                                                              uint4* __restrict__ dst,
                                                              int64_t elems) {
  const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
  for (int64_t i = (int64_t)blockIdx.x * kProbeThreads + threadIdx.x; i < elems; i += stride)
    dst[i] = src[i];
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

int rt_probe_read(const void* buf, int64_t bytes, int64_t span, int32_t passes, int32_t groups,
                  uint32_t* sink, hipStream_t s) {
  if (!buf || !sink) return set_error(RT_EINVAL, "rt_probe_read: NULL pointer");
  if (!aligned16(buf) || !aligned16(sink))
    return set_error(RT_EINVAL, "rt_probe_read: buf and sink must be 16-byte aligned");
  if (bytes < 16 || bytes % 16 != 0 || span < 16 || span % 16 != 0 || span > bytes || passes < 1 ||
      groups < 1 || groups > 65536)
    return set_error(RT_EINVAL,
                     "rt_probe_read: bytes, span positive multiples of 16 with span <= bytes; "
                     "passes >= 1; groups in 1..65536");
  hipLaunchKernelGGL(k_probe_read, dim3(groups), dim3(kProbeThreads), 0, s,
                     static_cast<const uint4*>(buf), bytes / 16, span / 16, passes, sink);
  return check_hip(hipGetLastError(), "rt_probe_read");
}

int rt_probe_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  if (!src || !dst) return set_error(RT_EINVAL, "rt_probe_copy: NULL pointer");
  if (!aligned16(src) || !aligned16(dst))
    return set_error(RT_EINVAL, "rt_probe_copy: src and dst must be 16-byte aligned");
  if (bytes < 16 || bytes % 16 != 0)
    return set_error(RT_EINVAL, "rt_probe_copy: bytes must be a positive multiple of 16");
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + bytes && b < a + bytes) return set_error(RT_EINVAL, "rt_probe_copy: ranges overlap");
  const int64_t elems = bytes / 16;
  const int64_t groups = std::min<int64_t>(kProbeGroups, (elems + kProbeThreads - 1) / kProbeThreads);
  hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)groups), dim3(kProbeThreads), 0, s,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), elems);
  return check_hip(hipGetLastError(), "rt_probe_copy");
}

}  // extern "C"
