// Launched rays (Sec. III-A): rays from a source point along the directions
// of a resident direction table, for one launch or for many launches of a
// served batch in one kernel (declared in include/rt_mi355x.h).
#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_internal.h"

namespace rt {
namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// rays[i] = (o, tmin, dirs[i], tmax)
__global__ __launch_bounds__(256) void k_rays(const float* __restrict__ dirs, int64_t n, float ox,
                                              float oy, float oz, float tmin, float tmax,
                                              float4* __restrict__ rays) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  rays[2 * i] = make_float4(ox, oy, oz, tmin);
  rays[2 * i + 1] = make_float4(dirs[3 * i], dirs[3 * i + 1], dirs[3 * i + 2], tmax);
}

// Row i of a many-launch ray batch: the launch whose first row is the last
// one at or below i (binary search over the sorted table), if it covers i.
__global__ __launch_bounds__(256) void k_rays_many(const float* __restrict__ dirs, int64_t n_dirs,
                                                   const rt_ray_launch* __restrict__ table,
                                                   int count, float tmin, float tmax,
                                                   float4* __restrict__ rays, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total || count <= 0) return;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (table[mid].first <= i) lo = mid;
    else hi = mid - 1;
  }
  const rt_ray_launch e = table[lo];
  const int64_t k = i - e.first;
  if (e.first < 0 || e.n < 0 || e.n > n_dirs || e.first > total - e.n || k < 0 || k >= e.n) return;
  rays[2 * i] = make_float4(e.src[0], e.src[1], e.src[2], tmin);
  rays[2 * i + 1] = make_float4(dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2], tmax);
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

int rt_rays_from_directions(const float* dirs, int64_t n, float ox, float oy, float oz, float tmin,
                            float tmax, float* rays, hipStream_t s) {
  if (n < 0) return set_error(RT_EINVAL, "rt_rays_from_directions: n must be >= 0");
  if (n == 0) return RT_OK;
  if (!dirs || !rays) return set_error(RT_EINVAL, "rt_rays_from_directions: NULL pointer");
  if (!aligned16(rays) || (reinterpret_cast<uintptr_t>(dirs) & 3u))
    return set_error(RT_EINVAL, "rt_rays_from_directions: rays must be 16-byte aligned");
  if (!(tmin <= tmax) || !std::isfinite(ox) || !std::isfinite(oy) || !std::isfinite(oz) ||
      !std::isfinite(tmin))
    return set_error(RT_EINVAL, "rt_rays_from_directions: source and range must be finite, tmin <= tmax");
  hipLaunchKernelGGL(k_rays, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dirs, n, ox, oy, oz,
                     tmin, tmax, reinterpret_cast<float4*>(rays));
  return check_hip(hipGetLastError(), "rt_rays_from_directions");
}

int rt_rays_from_directions_many(const float* dirs, int64_t n_dirs, const rt_ray_launch* table,
                                 int32_t count, float tmin, float tmax, float* rays, int64_t total,
                                 hipStream_t s) {
  if (count < 0 || total < 0 || n_dirs < 0)
    return set_error(RT_EINVAL, "rt_rays_from_directions_many: count, total and n_dirs must be >= 0");
  if (count == 0 || total == 0) return RT_OK;
  if (!dirs || !table || !rays)
    return set_error(RT_EINVAL, "rt_rays_from_directions_many: NULL pointer");
  if (!aligned16(rays) || !aligned16(table) || (reinterpret_cast<uintptr_t>(dirs) & 3u))
    return set_error(RT_EINVAL, "rt_rays_from_directions_many: rays and table must be 16-byte aligned");
  if (!(tmin <= tmax) || !std::isfinite(tmin))
    return set_error(RT_EINVAL, "rt_rays_from_directions_many: range must be finite, tmin <= tmax");
  hipLaunchKernelGGL(k_rays_many, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, dirs,
                     n_dirs, table, (int)count, tmin, tmax, reinterpret_cast<float4*>(rays), total);
  return check_hip(hipGetLastError(), "rt_rays_from_directions_many");
}

}  // extern "C"
