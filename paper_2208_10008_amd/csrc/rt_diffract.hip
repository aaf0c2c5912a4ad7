// Edge diffraction (declared in include/rt_mi355x.h; Sec. III-B: rays
// meeting facets give reflected and diffracted rays):
//   rt_wedges             -- neighbour of every half-edge: a 64-bit key per
//                            half-edge, a device radix sort, then each run of
//                            equal keys is grouped by exact end points
//   rt_diffract_segments  -- Keller-cone rays at the wedge or free edge nearest
//                            each stored hit, when it lies inside the ray tube
// Every float64 expression follows the documented order without contraction.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "rt_internal.h"

// Device memory of rt_wedges_noalloc: the half-edge keys and values (two
// buffers each for the radix sort), the non-finite flag and the sort's
// temporary storage, for up to kNoAllocMaxFacets facets.  One copy per GPU,
// held until the process ends.  Host code never passes this name to a
// kernel: it uses the device address hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[size_t(24) << 20];

namespace rt {
namespace {

constexpr int kDiffBlock = 256;
constexpr double kCos2Coplanar = 0.9996954135095479;  // cos^2(1 degree)

bool aligned_to(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

struct D3 {
  double x, y, z;
};

__device__ __forceinline__ D3 ld3(const float* p) { return {p[0], p[1], p[2]}; }

// ---------------------------------------------------------------------------
// wedges

// End points of half-edge h, -0 made +0, in lexicographic order.
__device__ __forceinline__ void half_edge(const float* __restrict__ tris, int64_t h, float lo[3],
                                          float hi[3]) {
  const int64_t f = h / 3;
  const int k = (int)(h % 3);
  const float* a = tris + 9 * f + 3 * k;
  const float* b = tris + 9 * f + 3 * ((k + 1) % 3);
  const float A[3] = {a[0] + 0.0f, a[1] + 0.0f, a[2] + 0.0f};
  const float B[3] = {b[0] + 0.0f, b[1] + 0.0f, b[2] + 0.0f};
  bool a_first = true;
  for (int q = 0; q < 3; ++q) {
    if (A[q] < B[q]) break;
    if (A[q] > B[q]) {
      a_first = false;
      break;
    }
  }
  for (int q = 0; q < 3; ++q) {
    lo[q] = a_first ? A[q] : B[q];
    hi[q] = a_first ? B[q] : A[q];
  }
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

__global__ void k_edge_keys(const float* __restrict__ tris, int64_t nh,
                            unsigned long long* __restrict__ keys, uint32_t* __restrict__ vals,
                            int* __restrict__ bad) {
  const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  float lo[3], hi[3];
  half_edge(tris, h, lo, hi);
  unsigned long long k = 0x9e3779b97f4a7c15ull;
  bool finite = true;
  for (int q = 0; q < 3; ++q) {
    finite = finite && isfinite(lo[q]) && isfinite(hi[q]);
    k = mix64(k ^ __float_as_uint(lo[q]));
    k = mix64(k ^ ((unsigned long long)__float_as_uint(hi[q]) << 32));
  }
  if (!finite) atomicOr(bad, 1);
  keys[h] = k;
  vals[h] = (uint32_t)h;
}

__device__ __forceinline__ D3 facet_normal64(const float* __restrict__ tris, int64_t f) {
#pragma clang fp contract(off)
  const D3 v0 = ld3(tris + 9 * f), v1 = ld3(tris + 9 * f + 3), v2 = ld3(tris + 9 * f + 6);
  const D3 e1 = {v1.x - v0.x, v1.y - v0.y, v1.z - v0.z};
  const D3 e2 = {v2.x - v0.x, v2.y - v0.y, v2.z - v0.z};
  return {e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z, e1.x * e2.y - e1.y * e2.x};
}

__device__ __forceinline__ bool not_coplanar(const float* __restrict__ tris, int64_t fa, int64_t fb) {
#pragma clang fp contract(off)
  const D3 na = facet_normal64(tris, fa), nb = facet_normal64(tris, fb);
  const double dot = na.x * nb.x + na.y * nb.y + na.z * nb.z;
  const double aa = na.x * na.x + na.y * na.y + na.z * na.z;
  const double bb = nb.x * nb.x + nb.y * nb.y + nb.z * nb.z;
  return dot * dot < kCos2Coplanar * aa * bb;
}

// One thread per run of equal keys in sorted order: groups its half-edges by
// exact end points and writes every member's neighbour.
__global__ void k_edge_group(const float* __restrict__ tris, int64_t nh,
                             const unsigned long long* __restrict__ keys,
                             const uint32_t* __restrict__ vals, int32_t* __restrict__ nbr) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nh || (i > 0 && keys[i] == keys[i - 1])) return;
  int64_t j = i + 1;
  while (j < nh && keys[j] == keys[i]) ++j;
  for (int64_t m = i; m < j; ++m) {
    float lo[3], hi[3];
    half_edge(tris, vals[m], lo, hi);
    int count = 0;
    int64_t other = -1;
    for (int64_t r = i; r < j; ++r) {
      float lo2[3], hi2[3];
      half_edge(tris, vals[r], lo2, hi2);
      const bool same = lo[0] == lo2[0] && lo[1] == lo2[1] && lo[2] == lo2[2] && hi[0] == hi2[0] &&
                        hi[1] == hi2[1] && hi[2] == hi2[2];
      if (same) {
        ++count;
        if (r != m) other = vals[r];
      }
    }
    const int64_t h = vals[m];
    int32_t v = -2;
    if (count == 1) v = -1;
    else if (count == 2 && not_coplanar(tris, h / 3, other / 3)) v = (int32_t)(other / 3);
    nbr[h] = v;
  }
}

// ---------------------------------------------------------------------------
// diffraction of stored chains

struct DiffArgs {
  const float* tris;
  const int32_t* nbr;
  const double* cone;
  rt_diffracted* out;
  unsigned long long* count;
  int64_t n_tris, cap;
  double delta;
  int32_t n_cone, pad;
};

__device__ __forceinline__ double dot3(const D3& a, const D3& b) {
#pragma clang fp contract(off)
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ D3 cross3(const D3& a, const D3& b) {
#pragma clang fp contract(off)
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ D3 sub3(const D3& a, const D3& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }

// In-plane unit vector across the edge (a, unit ehat) towards `third`.
__device__ __forceinline__ D3 across(const D3& a, const D3& third, const D3& ehat) {
#pragma clang fp contract(off)
  D3 x = sub3(third, a);
  const double k = dot3(x, ehat);
  x = {x.x - k * ehat.x, x.y - k * ehat.y, x.z - k * ehat.z};
  const double nx = sqrt(dot3(x, x));
  return {x.x / nx, x.y / nx, x.z / nx};
}

// Vertex i of (v0, v1, v2) by selects: indexing an array with a run-time
// index would place it in scratch memory.
__device__ __forceinline__ D3 pick(const D3& v0, const D3& v1, const D3& v2, int i) {
  return i == 0 ? v0 : (i == 1 ? v1 : v2);
}

// The diffracted rays of one hit; returns how many were kept (written only
// when `write`, from slot `base`).
__device__ int diffract_hit(const DiffArgs& A, int64_t ray, int order, int64_t f, const float4& ra,
                            const float4& rb, float t, double L, bool write,
                            unsigned long long base) {
#pragma clang fp contract(off)
  const float* tv = A.tris + 9 * f;
  const D3 v0 = ld3(tv), v1 = ld3(tv + 3), v2 = ld3(tv + 6);
  const D3 o = {ra.x, ra.y, ra.z}, d = {rb.x, rb.y, rb.z};
  const double T = t;
  const D3 p = {o.x + T * d.x, o.y + T * d.y, o.z + T * d.z};
  const double dn = sqrt(dot3(d, d));
  const double l = L + T * dn;
  const double rho = l * A.delta / sqrt(3.0);
  // single-precision rejection: an edge whose float32 distance from the hit
  // exceeds rho by 0.1 % plus 1e-4 of the coordinate scale (float32 rounding
  // moves these distances by a few 1e-7 of it) cannot pass the float64 test
  int maybe = 0;
  {
    const float px = fmaf(t, rb.x, ra.x), py = fmaf(t, rb.y, ra.y), pz = fmaf(t, rb.z, ra.z);
    const float scale = fmaxf(fmaxf(fabsf(px), fabsf(py)), fabsf(pz)) + 1.0f;
    const float r32 = (float)rho * 1.001f + 1e-4f * (scale + fmaxf(fmaxf(fabsf(tv[0]), fabsf(tv[1])),
                                                                   fabsf(tv[2])));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float* ka = tv + 3 * k;
      const float* kb = tv + 3 * ((k + 1) % 3);
      const float ex = kb[0] - ka[0], ey = kb[1] - ka[1], ez = kb[2] - ka[2];
      const float wx = px - ka[0], wy = py - ka[1], wz = pz - ka[2];
      const float ee = ex * ex + ey * ey + ez * ez;
      float sk = (wx * ex + wy * ey + wz * ez) / ee;
      sk = fminf(fmaxf(sk, 0.0f), 1.0f);
      const float qx = wx - sk * ex, qy = wy - sk * ey, qz = wz - sk * ez;
      const bool far = qx * qx + qy * qy + qz * qz > r32 * r32;
      if (!far) maybe |= 1 << k;   // NaN or overflow: kept for the float64 test
    }
  }
  if (maybe == 0) return 0;
  int bk = -1;
  double bdist = 0.0;
  D3 q{}, e{}, a{};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (!((maybe >> k) & 1) || A.nbr[3 * f + k] == -2) continue;
    const D3 ak = pick(v0, v1, v2, k), bkv = pick(v0, v1, v2, (k + 1) % 3);
    const D3 ek = sub3(bkv, ak);
    double s = dot3(sub3(p, ak), ek) / dot3(ek, ek);
    // clamp to the edge; a NaN (zero-length edge) stays NaN and never diffracts
    s = (0.0 > s) ? 0.0 : s;
    s = (1.0 < s) ? 1.0 : s;
    const D3 qk = {ak.x + s * ek.x, ak.y + s * ek.y, ak.z + s * ek.z};
    const D3 dq = sub3(p, qk);
    const double dist = sqrt(dot3(dq, dq));
    if (dist <= rho && (bk < 0 || dist < bdist)) {
      bk = k;
      bdist = dist;
      q = qk;
      e = ek;
      a = ak;
    }
  }
  if (bk < 0) return 0;
  const double en = sqrt(dot3(e, e));
  const D3 ehat = {e.x / en, e.y / en, e.z / en};
  const D3 ihat = {d.x / dn, d.y / dn, d.z / dn};
  const double c = dot3(ihat, ehat);
  const D3 r = {ihat.x - c * ehat.x, ihat.y - c * ehat.y, ihat.z - c * ehat.z};
  const double sb = sqrt(dot3(r, r));
  if (sb == 0.0) return 0;
  const D3 u = {r.x / sb, r.y / sb, r.z / sb};
  const D3 w = cross3(ehat, u);
  const int32_t g = A.nbr[3 * f + bk];
  bool wedge = g >= 0 && g < A.n_tris;
  D3 a_in{}, b_in{};
  double cab = 0.0;
  if (wedge) {
    const D3 bpt = pick(v0, v1, v2, (bk + 1) % 3);
    a_in = across(a, pick(v0, v1, v2, (bk + 2) % 3), ehat);
    const float* gv = A.tris + 9 * (int64_t)g;
    int third = -1;
    for (int x = 0; x < 3 && third < 0; ++x) {
      const D3 y = ld3(gv + 3 * x);
      const bool is_a = y.x == a.x && y.y == a.y && y.z == a.z;
      const bool is_b = y.x == bpt.x && y.y == bpt.y && y.z == bpt.z;
      if (!is_a && !is_b) third = x;
    }
    if (third < 0) {
      wedge = false;
    } else {
      b_in = across(a, ld3(gv + 3 * third), ehat);
      cab = dot3(cross3(a_in, b_in), ehat);
    }
  }
  const D3 qo = sub3(q, o);
  const double path = L + sqrt(dot3(qo, qo));
  int kept = 0;
  for (int j = 0; j < A.n_cone; ++j) {
    const double cj = A.cone[2 * j], sj = A.cone[2 * j + 1];
    const D3 perp = {sb * (cj * u.x + sj * w.x), sb * (cj * u.y + sj * w.y),
                     sb * (cj * u.z + sj * w.z)};
    if (wedge) {
      const double s1 = dot3(cross3(a_in, perp), ehat);
      const double s2 = dot3(cross3(perp, b_in), ehat);
      if ((s1 > 0 && s2 > 0 && cab > 0) || (s1 < 0 && s2 < 0 && cab < 0)) continue;
    }
    if (write) {
      const unsigned long long slot = base + kept;
      if (slot < (unsigned long long)A.cap) {
        rt_diffracted rec;
        rec.ray = (int32_t)ray;
        rec.order = order;
        rec.facet = (int32_t)f;
        rec.edge = bk;
        rec.cone = j;
        rec.pad = 0;
        rec.path = path;
        rec.ray8[0] = (float)q.x;
        rec.ray8[1] = (float)q.y;
        rec.ray8[2] = (float)q.z;
        rec.ray8[3] = ra.w;
        rec.ray8[4] = (float)(c * ehat.x + perp.x);
        rec.ray8[5] = (float)(c * ehat.y + perp.y);
        rec.ray8[6] = (float)(c * ehat.z + perp.z);
        rec.ray8[7] = rb.w;
        A.out[slot] = rec;
      }
    }
    ++kept;
  }
  return kept;
}

// One chain per lane; the wave steps through the segments together (lanes
// whose chain has ended sit out), adds up its lanes' diffracted rays with a
// wave scan and takes their slots with one atomic per wave and segment.
__global__ __launch_bounds__(kDiffBlock) void k_diffract(const float4* __restrict__ seg,
                                                         const rt_hit* __restrict__ hits, int64_t n,
                                                         int max_b, DiffArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kDiffBlock + threadIdx.x;
  const int lane = threadIdx.x & 63;
  bool alive = i < n;
  double L = 0.0;
  for (int b = 0; b < max_b; ++b) {
    if (__ballot(alive) == 0ull) break;
    int kept = 0, fid = -1;
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra;
    float th = 0.f;
    if (alive) {
      const int64_t k = (int64_t)b * n + i;
      const int4 h = reinterpret_cast<const int4*>(hits)[k];
      if (h.x < 0) {
        alive = false;
      } else {
        fid = h.x;
        ra = seg[2 * k];
        rb = seg[2 * k + 1];
        th = __int_as_float(h.y);
        if (fid < A.n_tris) kept = diffract_hit(A, i, b, fid, ra, rb, th, L, false, 0);
      }
    }
    int incl = kept;
    for (int d = 1; d < 64; d <<= 1) {
      const int y = __shfl_up(incl, d);
      if (lane >= d) incl += y;
    }
    const int total = __shfl(incl, 63);
    if (total > 0) {
      unsigned long long base = 0;
      if (lane == 63) base = atomicAdd(A.count, (unsigned long long)total);
      base = __shfl(base, 63);
      if (kept > 0) diffract_hit(A, i, b, fid, ra, rb, th, L, true, base + (incl - kept));
    }
    if (alive) L += seg_path(th, rb.x, rb.y, rb.z);
  }
}

__global__ void k_zero_u64(unsigned long long* c) { *c = 0ull; }
__global__ void k_zero_i32(int* c) { *c = 0; }

// Largest scene of rt_wedges_noalloc: keys and values of 3 * 2^18 half-edges
// take 18 MiB of the 24 MiB scratch, the radix sort's double-buffer storage
// the rest.
constexpr int64_t kNoAllocMaxFacets = int64_t(1) << 18;

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};

int scratch_of_device(unsigned char** out) {
  int dev = 0;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc != RT_OK) return rc;
  if (dev < 0 || dev >= kMaxDevices) return set_error(RT_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    if (rc != RT_OK) return rc;
    g_scratch[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch[dev];
  return RT_OK;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

int rt_wedges(const float* tris, int64_t n, int32_t* nbr, hipStream_t s) {
  if (!tris || !nbr || !aligned_to(tris, 4) || !aligned_to(nbr, 4))
    return set_error(RT_EINVAL, "rt_wedges: NULL or misaligned array");
  if (n < 1 || n >= (int64_t(1) << 29)) return set_error(RT_EINVAL, "rt_wedges: n outside 1..2^29-1");
  const int64_t nh = 3 * n;
  unsigned long long *k_in = nullptr, *k_out = nullptr;
  uint32_t *v_in = nullptr, *v_out = nullptr;
  int* bad = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  int rc = RT_OK;
  auto fail = [&](hipError_t e, const char* what) {
    if (rc == RT_OK && e != hipSuccess) rc = check_hip(e, what);
  };
  fail(hipMalloc((void**)&k_in, sizeof(unsigned long long) * nh), "hipMalloc");
  fail(hipMalloc((void**)&k_out, sizeof(unsigned long long) * nh), "hipMalloc");
  fail(hipMalloc((void**)&v_in, sizeof(uint32_t) * nh), "hipMalloc");
  fail(hipMalloc((void**)&v_out, sizeof(uint32_t) * nh), "hipMalloc");
  fail(hipMalloc((void**)&bad, sizeof(int)), "hipMalloc");
  if (rc == RT_OK)
    fail(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, k_in, k_out, v_in, v_out, (int)nh, 0,
                                            64, s),
         "radix sort size");
  if (rc == RT_OK) fail(hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16)), "hipMalloc");
  int host_bad = 0;
  if (rc == RT_OK) {
    const unsigned g = (unsigned)((nh + 255) / 256);
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, bad);
    hipLaunchKernelGGL(k_edge_keys, dim3(g), dim3(256), 0, s, tris, nh, k_in, v_in, bad);
    fail(hipGetLastError(), "edge keys");
    if (rc == RT_OK)
      fail(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, k_in, k_out, v_in, v_out, (int)nh, 0,
                                              64, s),
           "radix sort");
    hipLaunchKernelGGL(k_edge_group, dim3(g), dim3(256), 0, s, tris, nh, k_out, v_out, nbr);
    fail(hipGetLastError(), "edge groups");
    fail(hipMemcpyAsync(&host_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    fail(hipStreamSynchronize(s), "hipStreamSynchronize");
  }
  for (void* p : {(void*)k_in, (void*)k_out, (void*)v_in, (void*)v_out, (void*)bad, tmp})
    if (p) (void)hipFree(p);
  if (rc == RT_OK && host_bad) return set_error(RT_EINVAL, "rt_wedges: a facet has a non-finite vertex");
  return rc;
}

int rt_wedges_noalloc(const float* tris, int64_t n, int32_t* nbr, hipStream_t s) {
  if (!tris || !nbr || !aligned_to(tris, 4) || !aligned_to(nbr, 4))
    return set_error(RT_EINVAL, "rt_wedges_noalloc: NULL or misaligned array");
  if (n < 1 || n > kNoAllocMaxFacets)
    return set_error(RT_EINVAL, "rt_wedges_noalloc: n outside 1..262144 (the size of its device "
                                "scratch; rt_wedges takes larger scenes)");
  unsigned char* base = nullptr;
  int rc = scratch_of_device(&base);
  if (rc != RT_OK) return rc;
  const int64_t nh = 3 * n;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    unsigned char* p = base + off;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  auto* k0 = reinterpret_cast<unsigned long long*>(carve(sizeof(unsigned long long) * nh));
  auto* k1 = reinterpret_cast<unsigned long long*>(carve(sizeof(unsigned long long) * nh));
  auto* v0 = reinterpret_cast<uint32_t*>(carve(sizeof(uint32_t) * nh));
  auto* v1 = reinterpret_cast<uint32_t*>(carve(sizeof(uint32_t) * nh));
  int* bad = reinterpret_cast<int*>(carve(sizeof(int)));
  hipcub::DoubleBuffer<unsigned long long> keys(k0, k1);
  hipcub::DoubleBuffer<uint32_t> vals(v0, v1);
  size_t tmp_bytes = 0;
  rc = check_hip(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, keys, vals, (int)nh, 0, 64, s),
                 "radix sort size");
  if (rc != RT_OK) return rc;
  if (off + tmp_bytes > sizeof(scratch))
    return set_error(RT_EINVAL, "rt_wedges_noalloc: sort storage exceeds the device scratch");
  void* tmp = base + off;
  const unsigned g = (unsigned)((nh + 255) / 256);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, bad);  // the scratch keeps the last call's flag
  hipLaunchKernelGGL(k_edge_keys, dim3(g), dim3(256), 0, s, tris, nh, keys.Current(), vals.Current(), bad);
  rc = check_hip(hipGetLastError(), "edge keys");
  if (rc == RT_OK)
    rc = check_hip(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys, vals, (int)nh, 0, 64, s),
                   "radix sort");
  if (rc != RT_OK) return rc;
  hipLaunchKernelGGL(k_edge_group, dim3(g), dim3(256), 0, s, tris, nh, keys.Current(), vals.Current(),
                     nbr);
  rc = check_hip(hipGetLastError(), "edge groups");
  int host_bad = 0;
  if (rc == RT_OK)
    rc = check_hip(hipMemcpyAsync(&host_bad, bad, sizeof(int), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (rc == RT_OK) rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc == RT_OK && host_bad)
    return set_error(RT_EINVAL, "rt_wedges_noalloc: a facet has a non-finite vertex");
  return rc;
}

int rt_diffract_segments(const float* tris, int64_t n_tris, const int32_t* nbr,
                         const float* seg_rays, const rt_hit* hits, int64_t n,
                         int32_t max_bounces, double delta, const double* cone, int32_t n_cone,
                         rt_diffracted* out, int64_t cap, int64_t* count, hipStream_t s) {
  if (!tris || !nbr || !count || !aligned_to(tris, 4) || !aligned_to(nbr, 4) || !aligned_to(count, 8))
    return set_error(RT_EINVAL, "rt_diffract_segments: NULL or misaligned tris / nbr / count");
  if (n_tris < 1 || n_tris >= (int64_t(1) << 29))
    return set_error(RT_EINVAL, "rt_diffract_segments: n_tris outside 1..2^29-1");
  if (n < 0 || n > INT32_MAX || max_bounces < 1 || max_bounces > RT_MAX_BOUNCES)
    return set_error(RT_EINVAL, "rt_diffract_segments: n or max_bounces out of range");
  if (!std::isfinite(delta) || delta < 0.0)
    return set_error(RT_EINVAL, "rt_diffract_segments: delta must be finite and >= 0");
  if (n_cone < 0 || n_cone > 1024 || (n_cone > 0 && (!cone || !aligned_to(cone, 8))))
    return set_error(RT_EINVAL, "rt_diffract_segments: bad cone table");
  if (cap < 0 || cap > INT32_MAX || (cap > 0 && (!out || !aligned_to(out, 16))))
    return set_error(RT_EINVAL, "rt_diffract_segments: bad output buffer");
  if (n > 0 && (!seg_rays || !hits || !aligned_to(seg_rays, 16) || !aligned_to(hits, 16)))
    return set_error(RT_EINVAL, "rt_diffract_segments: seg_rays and hits must be non-NULL, 16-byte aligned");
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(count);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, s, cnt);
  int rc = check_hip(hipGetLastError(), "diffraction count reset");
  if (rc != RT_OK || n == 0 || n_cone == 0) return rc;
  DiffArgs A;
  A.tris = tris;
  A.nbr = nbr;
  A.cone = cone;
  A.out = out;
  A.count = cnt;
  A.n_tris = n_tris;
  A.cap = cap;
  A.delta = delta;
  A.n_cone = n_cone;
  A.pad = 0;
  hipLaunchKernelGGL(k_diffract, dim3((unsigned)((n + kDiffBlock - 1) / kDiffBlock)), dim3(kDiffBlock),
                     0, s, reinterpret_cast<const float4*>(seg_rays), hits, n, (int)max_bounces, A);
  return check_hip(hipGetLastError(), "diffraction launch");
}

}  // extern "C"
