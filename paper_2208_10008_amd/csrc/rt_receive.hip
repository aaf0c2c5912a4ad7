// Ray reception by receiving spheres (Sec. III-C, Eq. (4)) on gfx950:
//   rt_trace_receive     -- chains traced with every segment tested as it ends
//                           (the test sits in the trace loop, see rt_trace.hip)
//   rt_trace_energy      -- chains that also stop by energy (Sec. III-B),
//                           optionally with the same reception test
//   rt_receive_segments  -- the same test over stored chains, one ray per lane
//   rt_receive_dedup     -- one reception per (field point, order, facet sequence)
// The test itself (receive_segment, rt_internal.h) is float64 without
// contraction; receptions are appended with one atomic per wave and field point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rt_internal.h"

namespace rt {
namespace {

constexpr int kRecvBlock = 256;
constexpr int kScanBlock1 = 1024;

bool aligned_to(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

__global__ void k_zero_count(unsigned long long* c) { *c = 0ull; }

__global__ __launch_bounds__(kRecvBlock) void k_receive_segments(const float4* __restrict__ seg,
                                                                 const rt_hit* __restrict__ hits,
                                                                 int64_t n, int max_b, RecvArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kRecvBlock + threadIdx.x;
  if (i >= n) return;
  double L = 0.0;  // path length before segment b
  for (int b = 0; b < max_b; ++b) {
    const int64_t k = (int64_t)b * n + i;
    const float4 ra = seg[2 * k], rb = seg[2 * k + 1];
    const int4 h = reinterpret_cast<const int4*>(hits)[k];
    const bool hit = h.x >= 0;
    const float th = __int_as_float(h.y);
    receive_segment(a, i, b, ra.x, ra.y, ra.z, rb.x, rb.y, rb.z, ra.w, hit ? th : rb.w, L);
    if (!hit) break;
    L += seg_path(th, rb.x, rb.y, rb.z);
  }
}

// ---- duplicate grouping: counting sort of the records by field point, then
// every record looks for a better one of the same path in its bucket.
// Workspace (uint32): off[n_rx + 1] | fill[n_rx] | idx[cap].

__global__ void k_dd_clear(uint32_t* __restrict__ w, int64_t words) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words;
       k += (int64_t)gridDim.x * blockDim.x)
    w[k] = 0u;
}

__device__ __forceinline__ int64_t stored(const unsigned long long* count, int64_t cap) {
  const unsigned long long c = *count;
  return c < (unsigned long long)cap ? (int64_t)c : cap;
}

__global__ void k_dd_hist(const rt_reception* __restrict__ rec,
                          const unsigned long long* __restrict__ count, int64_t cap, int n_rx,
                          uint32_t* __restrict__ off) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= stored(count, cap)) return;
  const int r = rec[k].rx;
  if (r >= 0 && r < n_rx) atomicAdd(&off[r], 1u);
}

// Exclusive scan of v[0 .. len) in place by one work-group.
__global__ __launch_bounds__(kScanBlock1) void k_dd_scan(uint32_t* __restrict__ v, int64_t len) {
  __shared__ uint32_t part[kScanBlock1 / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t base = 0; base < len; base += kScanBlock1) {
    const int64_t i = base + threadIdx.x;
    const uint32_t x = i < len ? v[i] : 0u;
    uint32_t inc = x;
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(inc, d);
      if (lane >= d) inc += y;
    }
    if (lane == 63) part[w] = inc;
    __syncthreads();
    if (w == 0) {
      uint32_t p = lane < kScanBlock1 / 64 ? part[lane] : 0u;
      for (int d = 1; d < kScanBlock1 / 64; d <<= 1) {
        const uint32_t y = __shfl_up(p, d);
        if (lane >= d) p += y;
      }
      if (lane < kScanBlock1 / 64) part[lane] = p;
    }
    __syncthreads();
    const uint32_t before = w ? part[w - 1] : 0u;
    const uint32_t total = part[kScanBlock1 / 64 - 1];
    if (i < len) v[i] = carry + before + inc - x;
    __syncthreads();
    carry += total;
  }
}

__global__ void k_dd_scatter(const rt_reception* __restrict__ rec,
                             const unsigned long long* __restrict__ count, int64_t cap, int n_rx,
                             const uint32_t* __restrict__ off, uint32_t* __restrict__ fill,
                             uint32_t* __restrict__ idx) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= stored(count, cap)) return;
  const int r = rec[k].rx;
  if (r < 0 || r >= n_rx) return;
  idx[off[r] + atomicAdd(&fill[r], 1u)] = (uint32_t)k;
}

__global__ void k_dd_mark(rt_reception* __restrict__ rec, const unsigned long long* __restrict__ count,
                          int64_t cap, int n_rx, const uint32_t* __restrict__ off,
                          const uint32_t* __restrict__ idx, const int32_t* __restrict__ hit_ids,
                          int64_t n, int max_b) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= stored(count, cap)) return;
  const rt_reception e = rec[k];
  int keep = 0;
  if (e.rx >= 0 && e.rx < n_rx && e.ray >= 0 && e.ray < n && e.order >= 0 && e.order < max_b) {
    keep = 1;
    for (uint32_t p = off[e.rx]; p < off[e.rx + 1]; ++p) {
      const uint32_t j = idx[p];
      if (j == (uint32_t)k) continue;
      const rt_reception f = rec[j];
      if (f.order != e.order || f.ray < 0 || f.ray >= n) continue;
      if (!(f.dist < e.dist || (f.dist == e.dist && f.ray < e.ray))) continue;
      bool same = true;
      for (int b = 0; b < e.order && same; ++b)  // hit_ids: tri_id field, stride 4 words
        same = hit_ids[4 * ((int64_t)b * n + f.ray)] == hit_ids[4 * ((int64_t)b * n + e.ray)];
      if (same) {
        keep = 0;
        break;
      }
    }
  }
  rec[k].keep = keep;
}

int check_energy(const rt_energy* e) {
  if (!e) return set_error(RT_EINVAL, "rt_trace_energy: energy struct is NULL");
  if (!e->material || !aligned_to(e->material, 4))
    return set_error(RT_EINVAL, "rt_trace_energy: material must be non-NULL and 4-byte aligned");
  if (e->n_materials < 0 || e->reserved != 0)
    return set_error(RT_EINVAL, "rt_trace_energy: n_materials must be >= 0, reserved 0");
  if (e->n_materials > 0 && (!e->refl || !aligned_to(e->refl, 8)))
    return set_error(RT_EINVAL, "rt_trace_energy: refl must be non-NULL and 8-byte aligned");
  if (!std::isfinite(e->k0) || !(e->k0 > 0.0))
    return set_error(RT_EINVAL, "rt_trace_energy: k0 must be finite and > 0");
  if (!std::isfinite(e->min_power) || e->min_power < 0.0)
    return set_error(RT_EINVAL, "rt_trace_energy: min_power must be finite and >= 0");
  if (e->power && !aligned_to(e->power, 8))
    return set_error(RT_EINVAL, "rt_trace_energy: power must be 8-byte aligned");
  return RT_OK;
}

}  // namespace

int check_rx(const rt_receivers* rx, const char* who, WrittenRanges written) {
  const std::string w(who);
  if (!rx) return set_error(RT_EINVAL, w + ": receivers struct is NULL");
  if (rx->n < 0 || rx->reserved != 0) return set_error(RT_EINVAL, w + ": n must be >= 0, reserved 0");
  if (rx->n > 0 && (!rx->pos || !aligned_to(rx->pos, 8)))
    return set_error(RT_EINVAL, w + ": pos must be non-NULL and 8-byte aligned");
  if (!std::isfinite(rx->delta) || rx->delta < 0.0)
    return set_error(RT_EINVAL, w + ": delta must be finite and >= 0");
  if (rx->cap < 0 || rx->cap > INT32_MAX) return set_error(RT_EINVAL, w + ": cap outside 0..2^31-1");
  if (rx->cap > 0 && (!rx->rec || !aligned_to(rx->rec, 16)))
    return set_error(RT_EINVAL, w + ": rec must be non-NULL and 16-byte aligned");
  if (!rx->count || !aligned_to(rx->count, 8))
    return set_error(RT_EINVAL, w + ": count must be non-NULL and 8-byte aligned");
  // the kernels read the field points as constant data: nothing the call
  // writes may overlap them
  if (rx->n > 0) {
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(rx->pos);
    const uintptr_t p1 = p0 + static_cast<uintptr_t>(rx->n) * 3 * sizeof(double);
    auto overlaps = [&](const void* q, int64_t bytes) {
      const uintptr_t q0 = reinterpret_cast<uintptr_t>(q);
      return q != nullptr && bytes > 0 && q0 < p1 && p0 < q0 + static_cast<uintptr_t>(bytes);
    };
    bool clash = overlaps(rx->rec, rx->cap * (int64_t)sizeof(rt_reception)) ||
                 overlaps(rx->count, 8);
    for (const auto& wr : written) clash = clash || overlaps(wr.first, wr.second);
    if (clash) return set_error(RT_EINVAL, w + ": pos overlaps memory the call writes");
  }
  return RT_OK;
}

RecvArgs recv_args(const rt_receivers* rx) {
  RecvArgs a;
  a.pos = rx->pos;
  a.rec = rx->rec;
  a.count = reinterpret_cast<unsigned long long*>(rx->count);
  a.cap = rx->cap;
  a.delta = rx->delta;
  a.n_rx = rx->n;
  a.pad = 0;
  return a;
}

}  // namespace rt

using namespace rt;

extern "C" {

int rt_trace_receive(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                     rt_hit* out, double* path_len, int32_t* n_hits, const rt_receivers* rx,
                     hipStream_t s) {
  int rc = check_trace_args(b, rays, n, max_bounces, out, path_len, n_hits, nullptr);
  if (rc != RT_OK) return rc;
  rc = check_rx(rx, "rt_trace_receive",
                {{out, (int64_t)max_bounces * n * 16}, {path_len, n * 8}, {n_hits, n * 4}});
  if (rc != RT_OK) return rc;
  if (n > INT32_MAX) return set_error(RT_EINVAL, "rt_trace_receive: n must be < 2^31");
  RecvArgs a = recv_args(rx);
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, a.count);
  rc = check_hip(hipGetLastError(), "reception count reset");
  if (rc != RT_OK || n == 0) return rc;
  return launch_trace_receive(b->buf, b->info.node_format, b->info.depth, rays, n, max_bounces,
                              out, path_len, n_hits, a, trace_lanes(n, b->params.max_leaf),
                              (int)b->info.n_tris, s);
}

int rt_trace_energy(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                    const rt_energy* e, rt_hit* out, double* path_len, int32_t* n_hits,
                    const rt_receivers* rx, hipStream_t s) {
  int rc = check_energy(e);
  if (rc != RT_OK) return rc;
  rc = check_trace_args(b, rays, n, max_bounces, out, path_len, n_hits, nullptr);
  if (rc != RT_OK) return rc;
  RecvArgs a{};
  if (rx) {
    rc = check_rx(rx, "rt_trace_energy", {{out, (int64_t)max_bounces * n * 16}, {path_len, n * 8},
                                          {n_hits, n * 4}, {e->power, n * 8}});
    if (rc != RT_OK) return rc;
    if (n > INT32_MAX) return set_error(RT_EINVAL, "rt_trace_energy: n must be < 2^31 with receivers");
    a = recv_args(rx);
    hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, a.count);
    rc = check_hip(hipGetLastError(), "reception count reset");
    if (rc != RT_OK) return rc;
  }
  if (n == 0) return RT_OK;
  EnergyArgs en;
  en.material = e->material;
  en.refl = e->refl;
  en.power = e->power;
  en.k0 = e->k0;
  en.min_power = e->min_power;
  en.n_mat = e->n_materials;
  en.pad = 0;
  return launch_trace_energy(b->buf, b->info.node_format, b->info.depth, rays, n, max_bounces, out,
                             path_len, n_hits, rx ? &a : nullptr, en,
                             trace_lanes(n, b->params.max_leaf), (int)b->info.n_tris, s);
}

int rt_receive_segments(const float* seg_rays, const rt_hit* hits, int64_t n, int32_t max_bounces,
                        const rt_receivers* rx, hipStream_t s) {
  int rc = check_rx(rx, "rt_receive_segments");
  if (rc != RT_OK) return rc;
  if (n < 0 || n > INT32_MAX) return set_error(RT_EINVAL, "rt_receive_segments: n outside 0..2^31-1");
  if (max_bounces < 1 || max_bounces > RT_MAX_BOUNCES)
    return set_error(RT_EINVAL, "rt_receive_segments: max_bounces must lie in 1..64");
  if (n > 0 && (!seg_rays || !hits || !aligned_to(seg_rays, 16) || !aligned_to(hits, 16)))
    return set_error(RT_EINVAL, "rt_receive_segments: seg_rays and hits must be non-NULL, 16-byte aligned");
  RecvArgs a = recv_args(rx);
  hipLaunchKernelGGL(k_zero_count, dim3(1), dim3(1), 0, s, a.count);
  rc = check_hip(hipGetLastError(), "reception count reset");
  if (rc != RT_OK || n == 0 || a.n_rx == 0) return rc;
  hipLaunchKernelGGL(k_receive_segments, dim3((unsigned)((n + kRecvBlock - 1) / kRecvBlock)),
                     dim3(kRecvBlock), 0, s, reinterpret_cast<const float4*>(seg_rays), hits, n,
                     (int)max_bounces, a);
  return check_hip(hipGetLastError(), "reception launch");
}

int64_t rt_receive_dedup_workspace(int64_t cap, int32_t n_rx) {
  if (cap < 0 || cap > INT32_MAX || n_rx < 0) return -1;
  const int64_t bytes = 4 * (2 * (int64_t)n_rx + 1 + cap);
  return (bytes + 255) / 256 * 256;
}

int rt_receive_dedup(const rt_hit* hits, int64_t n, int32_t max_bounces, const rt_receivers* rx,
                     void* work, int64_t work_bytes, hipStream_t s) {
  int rc = check_rx(rx, "rt_receive_dedup");
  if (rc != RT_OK) return rc;
  if (n < 0 || n > INT32_MAX || max_bounces < 1 || max_bounces > RT_MAX_BOUNCES)
    return set_error(RT_EINVAL, "rt_receive_dedup: n outside 0..2^31-1 or bad max_bounces");
  if (rx->cap == 0) return RT_OK;
  if (n > 0 && (!hits || !aligned_to(hits, 16)))
    return set_error(RT_EINVAL, "rt_receive_dedup: hits must be non-NULL, 16-byte aligned");
  const int64_t need = rt_receive_dedup_workspace(rx->cap, rx->n);
  if (!work || !aligned_to(work, 256) || work_bytes < need)
    return set_error(RT_EINVAL, "rt_receive_dedup: workspace NULL, misaligned or too small");
  uint32_t* off = static_cast<uint32_t*>(work);
  uint32_t* fill = off + rx->n + 1;
  uint32_t* idx = fill + rx->n;
  const unsigned long long* cnt = reinterpret_cast<const unsigned long long*>(rx->count);
  const int64_t words = 2 * (int64_t)rx->n + 1;
  const unsigned gw = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
  const unsigned gk = (unsigned)((rx->cap + 255) / 256);
  hipLaunchKernelGGL(k_dd_clear, dim3(gw), dim3(256), 0, s, off, words);
  hipLaunchKernelGGL(k_dd_hist, dim3(gk), dim3(256), 0, s, rx->rec, cnt, rx->cap, rx->n, off);
  hipLaunchKernelGGL(k_dd_scan, dim3(1), dim3(kScanBlock1), 0, s, off, (int64_t)rx->n + 1);
  hipLaunchKernelGGL(k_dd_scatter, dim3(gk), dim3(256), 0, s, rx->rec, cnt, rx->cap, rx->n, off,
                     fill, idx);
  hipLaunchKernelGGL(k_dd_mark, dim3(gk), dim3(256), 0, s, rx->rec, cnt, rx->cap, rx->n, off, idx,
                     reinterpret_cast<const int32_t*>(hits), n, (int)max_bounces);
  return check_hip(hipGetLastError(), "dedup launch");
}

}  // extern "C"
