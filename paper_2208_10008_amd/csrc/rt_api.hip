// C ABI of the gfx950 ray tracing library (declared in include/rt_mi355x.h):
// argument checks, device memory of a tree handle, error text.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "rt_build_plan.h"
#include "rt_internal.h"

namespace rt {

static thread_local std::string g_err = "no error";

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return RT_OK;
  if (e == hipErrorOutOfMemory)
    return set_error(RT_ENOMEM, std::string(what) + ": out of device memory");
  return set_error(RT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

void free_buffers(Buffers& B) {
  void* ptrs[] = {B.recs_a, B.recs_b, B.perm,   B.nodes,    B.cnodes,   B.used,
                  B.rank,   B.bsum,   B.mfront, B.sfront,   B.aitems,   B.accnt,   B.abins,
                  B.counters, B.root_box, B.tnodes, B.tfacets, B.wnodes, B.queue,
                  B.stat_work};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (B.rec_host) (void)hipHostFree(B.rec_host);
  B = Buffers();
}

template <class T>
int alloc(T*& p, size_t count, int64_t& bytes) {
  size_t b = sizeof(T) * (count ? count : 1);
  hipError_t e = hipMalloc((void**)&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    return check_hip(e, "hipMalloc");
  }
  bytes += (int64_t)b;
  return RT_OK;
}

int ensure_buffers(Buffers& B, int64_t n) {
  if (B.cap_n >= n && B.recs_a) return RT_OK;
  free_buffers(B);
  int64_t bytes = 0;
  int rc = RT_OK;
  const size_t nn = (size_t)n;
  if (rc == RT_OK) rc = alloc(B.recs_a, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.recs_b, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.perm, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.nodes, 2 * nn, bytes);
  const int64_t icap = item_capacity(n), acap = anode_capacity(n);
  if (rc == RT_OK) rc = alloc(B.cnodes, 2 * nn, bytes);
  if (rc == RT_OK) rc = alloc(B.used, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.rank, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.bsum, 2 * (nn / kScanBlock + 1), bytes);
  if (rc == RT_OK) rc = alloc(B.mfront, 2 * nn, bytes);
  if (rc == RT_OK) rc = alloc(B.sfront, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.aitems, 2 * (size_t)icap, bytes);
  if (rc == RT_OK) rc = alloc(B.accnt, 2 * (size_t)icap * 3 * RT_MAX_BINS, bytes);
  if (rc == RT_OK)
    rc = alloc(B.abins, 2 * (size_t)acap * kBinReplicas * bins_bytes(RT_MAX_BINS, true), bytes);
  if (rc == RT_OK) rc = alloc(B.counters, kStateWords, bytes);
  if (rc == RT_OK) rc = alloc(B.root_box, 12, bytes);
  if (rc == RT_OK) rc = alloc(B.tnodes, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.tfacets, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.wnodes, nn, bytes);
  if (rc == RT_OK) rc = alloc(B.queue, kQueueSlots, bytes);
  if (rc == RT_OK) rc = alloc(B.stat_work, kStatWords, bytes);
  if (rc != RT_OK) {
    free_buffers(B);
    return rc;
  }
  B.cap_n = n;
  B.item_cap = icap;
  B.anode_cap = acap;
  B.bytes = bytes;
  B.state_ready = false;
  return RT_OK;
}

int check_params(const rt_split_params* p) {
  if (!p) return set_error(RT_EINVAL, "split params: NULL");
  if (!(p->alpha >= 0.f && p->alpha <= 1.f))
    return set_error(RT_EINVAL, "split params: alpha must lie in [0, 1]");
  if (!(p->t_isect > 0.f) || !std::isfinite(p->t_isect))
    return set_error(RT_EINVAL, "split params: t_isect must be positive");
  if (!(p->t_trav >= 0.f) || !std::isfinite(p->t_trav))
    return set_error(RT_EINVAL, "split params: t_trav must be >= 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->src[a])) return set_error(RT_EINVAL, "split params: src not finite");
  if (p->max_leaf < 1) return set_error(RT_EINVAL, "split params: max_leaf must be >= 1");
  if (p->nbins < 2 || p->nbins > RT_MAX_BINS)
    return set_error(RT_EINVAL, "split params: nbins must lie in 2..64");
  if (p->d_mode < RT_D_CHILD_MEAN || p->d_mode > RT_D_PARENT)
    return set_error(RT_EINVAL, "split params: unknown d_mode");
  if (p->d_norm != RT_DNORM_UNIT && p->d_norm != RT_DNORM_RAW)
    return set_error(RT_EINVAL, "split params: unknown d_norm");
  if (p->max_depth < 0) return set_error(RT_EINVAL, "split params: max_depth must be >= 0");
  if (p->depth_limit < 1 || p->depth_limit > RT_MAX_DEPTH)
    return set_error(RT_EINVAL, "split params: depth_limit must lie in 1..64");
  if (p->node_format < RT_NODE_BIN2 || p->node_format > RT_NODE_Q4)
    return set_error(RT_EINVAL, "split params: unknown node_format");
  return RT_OK;
}

int check_build_args(const float* tris, int64_t n, const rt_split_params* p) {
  if (!tris) return set_error(RT_EINVAL, "rt_build: tris is NULL");
  if (n < 1 || n >= (int64_t(1) << 30)) return set_error(RT_EINVAL, "rt_build: n must lie in 1..2^30-1");
  if (!aligned(tris, 4)) return set_error(RT_EINVAL, "rt_build: tris must be 4-byte aligned");
  int rc = check_params(p);
  if (rc != RT_OK) return rc;
  // a halving schedule must reach the leaf size within the depth limit
  int64_t need = (n + p->max_leaf - 1) / p->max_leaf;
  int l = 0;
  while ((int64_t(1) << l) < need) ++l;
  if (l > p->depth_limit)
    return set_error(RT_EINVAL, "rt_build: depth_limit too small for n / max_leaf");
  return RT_OK;
}

// Reads the record of a build queued by rt_rebuild_async and makes the tree
// usable (or leaves it unusable with the build's error).
int complete_pending(rt_bvh* b) {
  if (!b->pending) return RT_OK;
  b->pending = false;
  rt_bvh_info info;
  std::memset(&info, 0, sizeof(info));
  int rc = build_complete(b->buf, b->pending_n, b->pending_params, b->pending_seq,
                          b->pending_stream, &info);
  if (rc != RT_OK) return rc;
  info.device_bytes = b->buf.bytes;
  b->info = info;
  b->params = b->pending_params;
  return RT_OK;
}

int do_build(rt_bvh* b, const float* tris, int64_t n, const rt_split_params* p, hipStream_t s) {
  (void)complete_pending(b);  // a build still in flight on the handle ends first
  int rc = check_build_args(tris, n, p);
  if (rc != RT_OK) return rc;
  rc = ensure_buffers(b->buf, n);
  if (rc != RT_OK) return rc;
  rt_bvh_info info;
  std::memset(&info, 0, sizeof(info));
  rc = build_tree(b->buf, tris, n, *p, s, &info);
  if (rc != RT_OK) return rc;
  info.device_bytes = b->buf.bytes;
  b->info = info;
  b->params = *p;
  return RT_OK;
}


}  // namespace

int check_trace_args(const rt_bvh* b, const float* rays, int64_t n, int32_t max_b, const rt_hit* out,
                     const double* path_len, const int32_t* n_hits, const rt_trace_opts* opts) {
  if (!b || b->info.n_tris <= 0) return set_error(RT_EINVAL, "trace: invalid tree handle");
  if (n < 0) return set_error(RT_EINVAL, "trace: n must be >= 0");
  if (n >= (int64_t(1) << 40)) return set_error(RT_EINVAL, "trace: n too large");
  if (max_b < 1 || max_b > RT_MAX_BOUNCES)
    return set_error(RT_EINVAL, "trace: max_bounces must lie in 1..64");
  if (n == 0) return RT_OK;
  if (!rays || !out) return set_error(RT_EINVAL, "trace: rays and out must not be NULL");
  if (!aligned(rays, 16) || !aligned(out, 16))
    return set_error(RT_EINVAL, "trace: rays and out must be 16-byte aligned");
  if ((path_len && !aligned(path_len, 8)) || (n_hits && !aligned(n_hits, 4)))
    return set_error(RT_EINVAL, "trace: misaligned path_len / n_hits");
  if (opts) {
    if (opts->seg_rays && !aligned(opts->seg_rays, 16))
      return set_error(RT_EINVAL, "trace: seg_rays must be 16-byte aligned");
    if (opts->ray_stats && !aligned(opts->ray_stats, 8))
      return set_error(RT_EINVAL, "trace: ray_stats must be 8-byte aligned");
    if ((opts->block != 0 && opts->block != 64) || opts->grid < 0 ||
        (opts->refill != 0 && opts->refill != 1))
      return set_error(RT_EINVAL, "trace: block must be 0 or 64, grid >= 0, refill 0 or 1");
    const int g = opts->lanes_per_ray;
    if (g != 0 && g != 1 && g != 4 && g != 16 && g != 64)
      return set_error(RT_EINVAL, "trace: lanes_per_ray must be 0, 1, 4, 16 or 64");
    if (g > 1 && (opts->seg_rays || opts->ray_stats || opts->grid > 0))
      return set_error(RT_EINVAL,
                       "trace: lanes_per_ray > 1 takes no seg_rays, ray_stats or grid");
    if (g > 1 && n > (int64_t)INT32_MAX * (64 / g))
      return set_error(RT_EINVAL, "trace: too many rays for lanes_per_ray");
    if (opts->cut < 0 || (opts->flags & ~RT_TRACE_NO_PAD) != 0)
      return set_error(RT_EINVAL, "trace: cut must be >= 0 and flags 0 or RT_TRACE_NO_PAD");
    if ((opts->flags & RT_TRACE_NO_PAD) && !n_hits)
      return set_error(RT_EINVAL, "trace: RT_TRACE_NO_PAD needs n_hits");
    if (opts->cut > 0) {
      if (opts->seg_rays || opts->ray_stats || opts->grid > 0 || g > 1)
        return set_error(RT_EINVAL,
                         "trace: cut >= 1 takes no seg_rays, ray_stats, grid or lanes_per_ray > 1");
      if (n > INT32_MAX) return set_error(RT_EINVAL, "trace: cut >= 1 takes n < 2^31");
      if (!opts->chain_ws || !aligned(opts->chain_ws, 256) ||
          opts->chain_ws_bytes < rt_trace_chain_ws_bytes(n))
        return set_error(RT_EINVAL, "trace: cut >= 1 needs a 256-byte aligned chain_ws of "
                                    "rt_trace_chain_ws_bytes(n) bytes");
    }
    if (opts->batch_order) {
      if (!aligned(opts->batch_order, 4))
        return set_error(RT_EINVAL, "trace: batch_order must be 4-byte aligned");
      if (opts->grid > 0 || g > 1)
        return set_error(RT_EINVAL, "trace: batch_order takes grid 0 and one lane per ray");
      if ((n + 63) / 64 > INT32_MAX) return set_error(RT_EINVAL, "trace: too many batches for batch_order");
    }
  }
  return RT_OK;
}

// Lanes per ray the library picks.  Sharing a ray among G lanes cuts the
// serial leaf tests of a chain by about G but multiplies the traversal and
// merge work by G, so it pays while the launch is small for the leaf size.
// Timed on the paper-size scenes (leaves of 16 to 820 facets, 642 to 2.6 M
// rays, every G), the fastest G follows n / max_leaf: 64 lanes up to 50
// rays per facet of leaf capacity, 16 up to 700, 4 up to 12,000 (within
// 1.25x of the fastest G in every case); G never exceeds max_leaf, and trees
// with small leaves keep one lane per ray.
int trace_lanes(int64_t n, int max_leaf) {
  constexpr int kGroupLeaf = 16;
  constexpr struct { int g; int64_t rays_per_facet; } kLimits[] = {{64, 50}, {16, 700}, {4, 12000}};
  if (max_leaf < kGroupLeaf || n <= 0) return 1;
  for (const auto& l : kLimits)
    if (l.g <= max_leaf && n <= l.rays_per_facet * max_leaf) return l.g;
  return 1;
}

// Lanes per ray of a trace call: the caller's choice, else the library's
// (one lane per ray whenever segments or statistics are recorded).
int lanes_of(const rt_bvh* b, int64_t n, const rt_trace_opts* opts) {
  if (opts && opts->lanes_per_ray > 0) return opts->lanes_per_ray;
  if (opts && (opts->seg_rays || opts->ray_stats || opts->grid > 0 || opts->cut > 0 ||
               opts->batch_order))
    return 1;
  return trace_lanes(n, b->params.max_leaf);
}

// Queue head of a persistent trace call: the handle's next slot, whatever
// kernel variant or node format the call launches (null without a grid).
unsigned long long* queue_of(const rt_bvh* b, const rt_trace_opts* opts) {
  if (!opts || opts->grid <= 0) return nullptr;
  const unsigned k = b->queue_slot.fetch_add(1u, std::memory_order_relaxed) % kQueueSlots;
  return b->buf.queue + k;
}
}  // namespace rt

using namespace rt;

extern "C" {

void rt_split_params_default(rt_split_params* p) {
  if (!p) return;
  p->alpha = 1.f;
  p->t_isect = 1.f;
  p->t_trav = 1.f;
  p->src[0] = p->src[1] = p->src[2] = 0.f;
  p->max_leaf = 4;
  p->nbins = 16;
  p->d_mode = RT_D_CHILD_MEAN;
  p->d_norm = RT_DNORM_UNIT;
  p->max_depth = 32;
  p->depth_limit = 64;
  p->node_format = RT_NODE_BIN2;
}

int rt_build(const float* tris, int64_t n, const rt_split_params* p, rt_bvh** out,
             hipStream_t s) {
  if (!out) return set_error(RT_EINVAL, "rt_build: out is NULL");
  *out = nullptr;
  int rc0 = check_build_args(tris, n, p);
  if (rc0 != RT_OK) return rc0;
  rt_bvh* b = new (std::nothrow) rt_bvh();
  if (!b) return set_error(RT_ENOMEM, "rt_build: host allocation failed");
  std::memset(&b->info, 0, sizeof(b->info));
  (void)hipGetDevice(&b->device);
  int rc = do_build(b, tris, n, p, s);
  if (rc != RT_OK) {
    free_buffers(b->buf);
    delete b;
    return rc;
  }
  *out = b;
  return RT_OK;
}

int rt_rebuild(rt_bvh* b, const float* tris, int64_t n, const rt_split_params* p, hipStream_t s) {
  if (!b) return set_error(RT_EINVAL, "rt_rebuild: handle is NULL");
  int rc = do_build(b, tris, n, p, s);
  if (rc != RT_OK) b->info.n_tris = 0;  // unusable until rebuilt
  return rc;
}

int rt_rebuild_async(rt_bvh* b, const float* tris, int64_t n, const rt_split_params* p,
                     hipStream_t s) {
  if (!b) return set_error(RT_EINVAL, "rt_rebuild_async: handle is NULL");
  (void)complete_pending(b);
  int rc = check_build_args(tris, n, p);
  if (rc == RT_OK) rc = ensure_buffers(b->buf, n);
  b->info.n_tris = 0;  // unusable until rt_bvh_wait has read the build's record
  if (rc != RT_OK) return rc;
  int seq = 0;
  rc = build_enqueue(b->buf, tris, n, *p, s, &seq);
  if (rc != RT_OK) return rc;
  b->pending = true;
  b->pending_seq = seq;
  b->pending_n = n;
  b->pending_params = *p;
  b->pending_stream = s;
  return RT_OK;
}

int rt_bvh_wait(rt_bvh* b) {
  if (!b) return set_error(RT_EINVAL, "rt_bvh_wait: handle is NULL");
  return complete_pending(b);
}

int rt_trace(const rt_bvh* b, const float* rays, int64_t n, rt_hit* out, hipStream_t s) {
  int rc = check_trace_args(b, rays, n, 1, out, nullptr, nullptr, nullptr);
  if (rc != RT_OK || n == 0) return rc;
  return launch_trace(b->buf, b->info.node_format, b->info.depth, rays, n, 1, out, nullptr, nullptr,
                      nullptr, lanes_of(b, n, nullptr), (int)b->info.n_tris, nullptr, s);
}

int64_t rt_trace_chain_ws_bytes(int64_t n) {
  return n < 0 ? 0 : chain_ws_bytes(n);
}

int rt_trace_bounces(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                     rt_hit* out, double* path_len, int32_t* n_hits, hipStream_t s) {
  return rt_trace_ex(b, rays, n, max_bounces, out, path_len, n_hits, nullptr, s);
}

int rt_trace_ex(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces, rt_hit* out,
                double* path_len, int32_t* n_hits, const rt_trace_opts* opts, hipStream_t s) {
  int rc = check_trace_args(b, rays, n, max_bounces, out, path_len, n_hits, opts);
  if (rc != RT_OK || n == 0) return rc;
  return launch_trace(b->buf, b->info.node_format, b->info.depth, rays, n, max_bounces, out,
                      path_len, n_hits, opts, lanes_of(b, n, opts), (int)b->info.n_tris,
                      queue_of(b, opts), s);
}

int rt_bvh_info_get(const rt_bvh* b, rt_bvh_info* info) {
  if (!b || !info) return set_error(RT_EINVAL, "rt_bvh_info_get: NULL argument");
  *info = b->info;
  return RT_OK;
}

int rt_bvh_stats(const rt_bvh* b, rt_bvh_info* info) {
  if (!b || !info) return set_error(RT_EINVAL, "rt_bvh_stats: NULL argument");
  if (b->info.n_tris <= 0) return set_error(RT_EINVAL, "rt_bvh_stats: tree not built");
  rt_bvh_info r = b->info;
  int rc = tree_stats(b->buf, r.n_nodes, (double)b->params.t_isect, (double)b->params.t_trav, &r);
  if (rc != RT_OK) return rc;
  *info = r;
  return RT_OK;
}

int rt_bvh_download(const rt_bvh* b, rt_node_rec* nodes, int64_t node_cap, int32_t* perm,
                    int64_t perm_cap) {
  if (!b || !nodes || !perm) return set_error(RT_EINVAL, "rt_bvh_download: NULL argument");
  if (b->info.n_tris <= 0) return set_error(RT_EINVAL, "rt_bvh_download: tree not built");
  if (node_cap < b->info.n_nodes || perm_cap < b->info.n_tris)
    return set_error(RT_EINVAL, "rt_bvh_download: capacity too small");
  int rc = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if (rc != RT_OK) return rc;
  const int64_t nn = b->info.n_nodes;
  BNode* tmp = new (std::nothrow) BNode[nn];
  if (!tmp) return set_error(RT_ENOMEM, "rt_bvh_download: host allocation failed");
  rc = check_hip(hipMemcpy(tmp, b->buf.cnodes, sizeof(BNode) * nn, hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc == RT_OK)
    rc = check_hip(hipMemcpy(perm, b->buf.perm, sizeof(int32_t) * b->info.n_tris,
                             hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc == RT_OK) {
    for (int64_t i = 0; i < nn; ++i) {
      rt_node_rec& r = nodes[i];
      const BNode& q = tmp[i];
      for (int a = 0; a < 3; ++a) {
        r.lo[a] = q.lo[a];
        r.hi[a] = q.hi[a];
      }
      r.left = q.left;
      r.first = q.first;
      r.count = q.count;
      r.depth = q.depth;
      r.axis = q.axis;
      r.plane = q.plane;
      r.flags = q.flags;
      r.reserved = 0;
      r.cost = q.cost;
    }
  }
  delete[] tmp;
  return rc;
}

int rt_bvh_export_trace_nodes(const rt_bvh* b, void* host, int64_t* bytes) {
  if (!b || !bytes) return set_error(RT_EINVAL, "rt_bvh_export_trace_nodes: NULL argument");
  if (b->info.n_tris <= 0) return set_error(RT_EINVAL, "rt_bvh_export_trace_nodes: tree not built");
  const int fmt = b->info.node_format;
  const int64_t rec = fmt == RT_NODE_F4 ? sizeof(FNode4) : fmt == RT_NODE_Q4 ? sizeof(QNode4) : sizeof(TNode);
  const int64_t need = rec * b->info.n_trace_nodes;
  if (!host) {
    *bytes = need;
    return RT_OK;
  }
  if (*bytes < need) return set_error(RT_EINVAL, "rt_bvh_export_trace_nodes: buffer too small");
  int rc = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if (rc != RT_OK) return rc;
  const void* src = fmt == RT_NODE_BIN2 ? (const void*)b->buf.tnodes : (const void*)b->buf.wnodes;
  rc = check_hip(hipMemcpy(host, src, need, hipMemcpyDeviceToHost), "hipMemcpy");
  *bytes = need;
  return rc;
}

void rt_bvh_destroy(rt_bvh* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  free_buffers(b->buf);
  delete b;
}

int rt_split_cus_mask(int32_t k, uint32_t* small_mask) {
  constexpr int kCUs = 256, kXcds = 8, kWords = kCUs / 32;
  if (!small_mask) return set_error(RT_EINVAL, "rt_split_cus_mask: NULL mask");
  if (k < 8 || k > 128 || k % 8 != 0)
    return set_error(RT_EINVAL, "rt_split_cus_mask: k must be a multiple of 8 in 8..128");
  for (int w = 0; w < kWords; ++w) small_mask[w] = 0;
  // block b gives its CUs of residue b mod 8 first, then of residue b + 1, ...:
  // block b's t-th CU has residue b + t / 4, so residue x collects one CU per t
  // from block x - t / 4, k / 8 in all, as block b does
  for (int b = 0; b < kXcds; ++b)
    for (int t = 0; t < k / kXcds; ++t) {
      const int cu = (kCUs / kXcds) * b + (b + t / 4) % kXcds + kXcds * (t % 4);
      small_mask[cu / 32] |= 1u << (cu % 32);
    }
  return RT_OK;
}

int rt_streams_split_cus(int32_t k, hipStream_t* small, hipStream_t* large) {
  if (!small || !large) return set_error(RT_EINVAL, "rt_streams_split_cus: NULL pointer");
  uint32_t small_mask[8], large_mask[8];
  int rc = rt_split_cus_mask(k, small_mask);
  if (rc != RT_OK) return rc;
  int dev = 0, ncu = 0;
  rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc != RT_OK) return rc;
  rc = check_hip(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev),
                 "hipDeviceGetAttribute");
  if (rc != RT_OK) return rc;
  constexpr int kWords = 8;
  if (ncu != 32 * kWords) return set_error(RT_EINVAL, "rt_streams_split_cus: needs a device with 256 CUs");
  for (int w = 0; w < kWords; ++w) large_mask[w] = ~small_mask[w];
  hipStream_t a = nullptr, c = nullptr;
  rc = check_hip(hipExtStreamCreateWithCUMask(&a, kWords, small_mask), "hipExtStreamCreateWithCUMask");
  if (rc != RT_OK) return rc;
  rc = check_hip(hipExtStreamCreateWithCUMask(&c, kWords, large_mask), "hipExtStreamCreateWithCUMask");
  if (rc != RT_OK) {
    (void)hipStreamDestroy(a);
    return rc;
  }
  *small = a;
  *large = c;
  return RT_OK;
}

int rt_stream_destroy(hipStream_t s) {
  if (!s) return set_error(RT_EINVAL, "rt_stream_destroy: NULL stream");
  return check_hip(hipStreamDestroy(s), "hipStreamDestroy");
}

const char* rt_last_error(void) { return g_err.c_str(); }

}  // extern "C"
