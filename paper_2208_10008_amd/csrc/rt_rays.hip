// Launched rays (Sec. III-A): rays from a source point along the directions
// of a resident direction table, for one launch or for many launches of a
// served batch in one kernel, and a dispatch order of their batches from the
// directions (declared in include/rt_mi355x.h).
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

// Batch keys, one wave per batch of 64 consecutive rays: the smallest
// q = floor(1023 d_a^2 / |d|^2) among the batch's rays (float32, each
// operation rounded on its own, so the host can recompute it exactly).  A
// wave runs as long as its slowest chain, and the slowest chains start from
// the rays nearest the plane normal to the axis, so the batch's smallest q
// ranks it.
constexpr int kOrderQ = 1024;    // q and the keys lie in 0 .. 1023
constexpr int kOrderClasses = 16;
__global__ __launch_bounds__(256) void k_batch_keys(const float4* __restrict__ rays, int64_t n,
                                                    int64_t nb, int axis,
                                                    int32_t* __restrict__ keys) {
#pragma clang fp contract(off)
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= nb) return;  // whole waves: b is uniform in a wave
  const int64_t i = b * 64 + lane;
  int q = kOrderQ - 1;  // rows past n do not lower the minimum
  if (i < n) {
    const float4 d = rays[2 * i + 1];
    const float da = axis == 0 ? d.x : (axis == 1 ? d.y : d.z);
    const float d2 = (d.x * d.x + d.y * d.y) + d.z * d.z;
    q = 0;  // zero, infinite or NaN directions
    if (d2 > 0.f && isfinite(d2)) {
      const float t = (da * da) / d2;
      q = min(kOrderQ - 1, max(0, (int)floorf(1023.f * t)));
    }
  }
  for (int o = 32; o > 0; o >>= 1) q = min(q, __shfl_xor(q, o));
  if (lane == 0) keys[b] = q;
}

// Class of a key: c with (c / 16)^2 <= key / 1023 < ((c + 1) / 16)^2, i.e. the
// batch's |d_a| / |d| in sixteenths.
__device__ inline int order_class(int key) {
  int c = 0;
#pragma unroll
  for (int k = 1; k < kOrderClasses; ++k) c += key >= (1023 * k * k) / (kOrderClasses * kOrderClasses);
  return c;
}

// Stable partition of the batches by class in tiles of kTile batches, one
// 256-thread work-group per tile, thread t holding the tile's batches 4t ..
// 4t + 3.  k_batch_tiles counts each tile's batches per class; k_batch_scatter
// places batch j of class c after every batch of a lower class, after the
// class-c batches of earlier tiles, and after those of its own tile's earlier
// threads and earlier slots: ascending class, index order within a class.
constexpr int kTile = 1024, kTileThreads = 256, kTilePer = kTile / kTileThreads;

__device__ inline void tile_classes(const int32_t* __restrict__ keys, int64_t nb, int64_t tile,
                                    int cl[kTilePer], int cnt[kOrderClasses]) {
#pragma unroll
  for (int c = 0; c < kOrderClasses; ++c) cnt[c] = 0;
#pragma unroll
  for (int u = 0; u < kTilePer; ++u) {
    const int64_t j = tile * kTile + threadIdx.x * kTilePer + u;
    cl[u] = j < nb ? order_class(keys[j]) : -1;
#pragma unroll
    for (int c = 0; c < kOrderClasses; ++c) cnt[c] += cl[u] == c;
  }
}

__global__ __launch_bounds__(kTileThreads) void k_batch_tiles(const int32_t* __restrict__ keys,
                                                             int64_t nb,
                                                             int32_t* __restrict__ tcnt) {
  __shared__ int s_w[kTileThreads / 64][kOrderClasses];
  int cl[kTilePer], cnt[kOrderClasses];
  tile_classes(keys, nb, blockIdx.x, cl, cnt);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < kOrderClasses; ++c) {
    int v = cnt[c];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) s_w[wave][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < kOrderClasses) {
    int t = 0;
    for (int w = 0; w < kTileThreads / 64; ++w) t += s_w[w][threadIdx.x];
    tcnt[(int64_t)blockIdx.x * kOrderClasses + threadIdx.x] = t;
  }
}

__global__ __launch_bounds__(kTileThreads) void k_batch_scatter(const int32_t* __restrict__ keys,
                                                               int64_t nb,
                                                               const int32_t* __restrict__ tcnt,
                                                               int64_t tiles,
                                                               int32_t* __restrict__ order) {
  __shared__ int s_base[kOrderClasses];
  __shared__ int s_red[kTileThreads / 64][2][kOrderClasses];
  __shared__ int s_pre[kOrderClasses][kTileThreads];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t tile = blockIdx.x;
  // class c's start for this tile: every batch of a lower class, then the
  // class-c batches of earlier tiles (all threads sum the tiles' counts)
  {
    int tot[kOrderClasses], ear[kOrderClasses];
#pragma unroll
    for (int c = 0; c < kOrderClasses; ++c) tot[c] = ear[c] = 0;
    for (int64_t t = tid; t < tiles; t += kTileThreads) {
#pragma unroll
      for (int c = 0; c < kOrderClasses; ++c) {
        const int v = tcnt[t * kOrderClasses + c];
        tot[c] += v;
        ear[c] += t < tile ? v : 0;
      }
    }
#pragma unroll
    for (int c = 0; c < kOrderClasses; ++c) {
      int a = tot[c], e = ear[c];
      for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        e += __shfl_xor(e, o);
      }
      if (lane == 0) {
        s_red[wave][0][c] = a;
        s_red[wave][1][c] = e;
      }
    }
    __syncthreads();
    if (tid < kOrderClasses) {
      int below = 0, earlier = 0;
      for (int w = 0; w < kTileThreads / 64; ++w) {
        earlier += s_red[w][1][tid];
        for (int c = 0; c < tid; ++c) below += s_red[w][0][c];
      }
      s_base[tid] = below + earlier;
    }
  }
  int cl[kTilePer], cnt[kOrderClasses];
  tile_classes(keys, nb, tile, cl, cnt);
#pragma unroll
  for (int c = 0; c < kOrderClasses; ++c) s_pre[c][tid] = cnt[c];
  __syncthreads();
  // wave w: exclusive prefix over the threads of classes 4w .. 4w + 3
  for (int c = wave * 4; c < wave * 4 + 4; ++c) {
    int* row = s_pre[c];
    constexpr int kPer = kTileThreads / 64;
    int v[kPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      v[u] = row[lane * kPer + u];
      sum += v[u];
    }
    int x = sum;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    int run = x - sum;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      row[lane * kPer + u] = run;
      run += v[u];
    }
  }
  __syncthreads();
  int pos[kOrderClasses];
#pragma unroll
  for (int c = 0; c < kOrderClasses; ++c) pos[c] = s_base[c] + s_pre[c][tid];
#pragma unroll
  for (int u = 0; u < kTilePer; ++u) {
    if (cl[u] < 0) continue;
    int p = 0;
#pragma unroll
    for (int c = 0; c < kOrderClasses; ++c)
      if (cl[u] == c) p = pos[c]++;
    order[p] = (int32_t)(tile * kTile + tid * kTilePer + u);
  }
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

int64_t rt_rays_batch_order_ws_bytes(int64_t n) {
  if (n < 0) return 0;
  const int64_t nb = (n + 63) / 64, tiles = (nb + kTile - 1) / kTile;
  return 4 * (nb + kOrderClasses * tiles);
}

int rt_rays_batch_order(const float* rays, int64_t n, int32_t axis, int32_t* order,
                        int32_t* keys, hipStream_t s) {
  if (n < 0 || n >= (int64_t(1) << 31))
    return set_error(RT_EINVAL, "rt_rays_batch_order: n must lie in 0..2^31-1");
  if (axis < 0 || axis > 2) return set_error(RT_EINVAL, "rt_rays_batch_order: axis must be 0, 1 or 2");
  if (n == 0) return RT_OK;
  if (!rays || !order || !keys) return set_error(RT_EINVAL, "rt_rays_batch_order: NULL pointer");
  if (!aligned16(rays) || (reinterpret_cast<uintptr_t>(order) & 3u) ||
      (reinterpret_cast<uintptr_t>(keys) & 3u))
    return set_error(RT_EINVAL, "rt_rays_batch_order: misaligned rays, order or keys");
  const int64_t nb = (n + 63) / 64;
  hipLaunchKernelGGL(k_batch_keys, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s,
                     reinterpret_cast<const float4*>(rays), n, nb, (int)axis, keys);
  const int64_t tiles = (nb + kTile - 1) / kTile;
  int32_t* tcnt = keys + nb;  // the workspace's per-tile class counts
  hipLaunchKernelGGL(k_batch_tiles, dim3((unsigned)tiles), dim3(kTileThreads), 0, s, keys, nb,
                     tcnt);
  hipLaunchKernelGGL(k_batch_scatter, dim3((unsigned)tiles), dim3(kTileThreads), 0, s, keys, nb,
                     tcnt, tiles, order);
  return check_hip(hipGetLastError(), "rt_rays_batch_order");
}

}  // extern "C"
