// Internal layouts and helpers of the gfx950 ray tracing library.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <initializer_list>
#include <utility>
#include <stdint.h>

#include <string>

#include "rt_mi355x.h"

namespace rt {

// ---- build-time node ----
// Node 0 is the root; the two children of a node are stored next to each
// other (left, left + 1), so an internal node is identified by its child pair
// (left - 1) / 2, which is also its traversal node index.
struct BNode {
  float lo[3], hi[3];      // volume: union of the facets' boxes
  int32_t left;            // left child id, -1 leaf
  int32_t first, count;    // facet range in the reference order
  int32_t depth;
  int32_t axis, plane, flags;
  int32_t tidx;            // unused (kept for the record layout)
  double cost;
  double cblo[3], cbhi[3]; // bounds of the facets' centroids
};

// ---- traversal node: one per internal node, 64 bytes ----
// Both child volumes sit in the parent so a visit is one 64-byte fetch.
//   a = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//   b = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//   c = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//   d = (ref0, ref1, -, -); ref >= 0: internal node index, ref < 0: leaf whose
//       facets start at position ~ref of the leaf-ordered facet array.
struct alignas(64) TNode {
  float4 a, b, c;
  int4 d;
};

// ---- 4-wide traversal nodes (one per even-depth internal node) ----
// Children are the node's grandchildren, or its children where those are
// leaves; `mask` marks the used slots.
struct alignas(64) FNode4 {  // 128 bytes
  float4 lox, hix, loy, hiy, loz, hiz;  // component c = child c
  int4 ref;
  uint4 meta;                           // x = mask
};
struct alignas(64) QNode4 {  // 64 bytes
  float4 h;    // origin xyz, w = bits (ex + 127) | (ey + 127) << 8 | (ez + 127) << 16 | mask << 24
  uint4 qa;    // bytes: qlo.x[4], qlo.y[4], qlo.z[4], qhi.x[4]
  uint4 qb;    // bytes: qhi.y[4], qhi.z[4], 0, 0
  int4 ref;
};

// ---- leaf-ordered facet: 48 bytes ----
//   p0 = (v0.xyz, id bits), p1 = (v1.xyz, 0), p2 = (v2.xyz, 0); the top bit of
//   the id marks the last facet of its leaf.
struct alignas(16) TFacet {
  float4 p0, p1, p2;
};
constexpr uint32_t kLastFacet = 0x80000000u;
constexpr int kQueueSlots = 64;  // persistent trace calls that may be in flight on one handle at once

// ---- a chain left alive by the first launch of a two-launch trace: 64 bytes ----
// The state its next segment starts from (Sec. III-B re-launch).
struct ChainCont {
  float4 o_tmin;   // reflected origin, tmin
  float4 d_tmax;   // reflected direction, tmax
  double path;     // path length of the segments traced so far
  int32_t ray;     // ray index
  int32_t skip;    // facet position the chain just left
  int32_t b;       // index of its next segment
  int32_t hits;    // hits so far
  int32_t pad[2];
};
static_assert(sizeof(ChainCont) == 64, "ChainCont is 64 bytes");
// Workspace of a two-launch trace: the live-chain count (a 256-byte header),
// then the records of the live chains in the order they were appended.
constexpr int64_t kChainWsHeader = 256;
inline int64_t chain_ws_bytes(int64_t n) { return kChainWsHeader + (int64_t)sizeof(ChainCont) * n; }

// ---- build-time facet record, kept in reference order: 32 bytes ----
//   lo = (box lo xyz, caller's id bits), hi = (box hi xyz, 0)
struct alignas(16) FacetRec {
  float4 lo, hi;
};

// One chunk of a big node's facets, binned and partitioned by one work-group.
struct AItem {
  int32_t node;        // node id
  int32_t slot;        // the node's bin slot on its level
  int32_t begin, end;  // facet range relative to the node's first facet
  int32_t first_item;  // list index of the node's first chunk
  int32_t n_items;     // chunks of the node
  int32_t pad[2];
};

// Build bookkeeping kept on the device: no pass waits for the host.
constexpr int kMaxPhaseLevels = 64;
struct BuildState {
  int32_t nonfinite;   // a facet has a non-finite vertex
  int32_t total;       // nodes of the finished tree
  int32_t depth;       // deepest node
  int32_t error;       // an internal capacity check failed
  int32_t n;           // facets of the build
  int32_t prep_done;   // work-groups of the facet pass that have finished
  int32_t pad[2];
  double inv_l2;       // 1 / squared root diagonal (0 if the root is a point)
  // per big-node level: (big nodes << 32) | chunk items, both taken by one
  // atomic add per parent
  unsigned long long a_pack[kMaxPhaseLevels + 1];
};
constexpr int kStateWords = 512;  // int32 words reserved for BuildState
static_assert(sizeof(BuildState) <= kStateWords * 4, "BuildState too large");

struct Buffers {
  // build scratch
  FacetRec* recs_a = nullptr;  // [n] facet records, ping-pong by node depth parity
  FacetRec* recs_b = nullptr;
  int32_t* perm = nullptr;  // [n] final leaf order
  BNode* nodes = nullptr;   // [2n] nodes at build ids: children of split boundary b are 2b+1, 2b+2
  BNode* cnodes = nullptr;  // [2n] the finished tree, ids compacted (2 n_internal + 1 nodes)
  int32_t* used = nullptr;  // [n] per split boundary: depth of its children, 0 if unused
  int32_t* rank = nullptr;  // [n] per used split boundary: its compact pair index
  int32_t* bsum = nullptr;  // [2][n / kScanBlock + 1] per-block used count and deepest child
  int32_t* mfront = nullptr; // [2][n] medium nodes by first facet (ping-pong by pass), -1 none
  int32_t* sfront = nullptr; // [n] subtree roots by first facet, -1 none
  AItem* aitems = nullptr;  // [2][item_cap] big-node chunks (ping-pong by level)
  int32_t* accnt = nullptr; // [2][item_cap][3 RT_MAX_BINS] per-chunk bin counts
  char* abins = nullptr;    // [2][anode_cap][kBinReplicas][bin bytes] bins of each big node
  int32_t* counters = nullptr;   // [kStateWords] BuildState
  long long* root_box = nullptr; // ordered-int root bounds (6 float + 6 double)
  int64_t item_cap = 0, anode_cap = 0;
  // traversal data
  TNode* tnodes = nullptr;  // [max(n_internal, 1)]
  FNode4* wnodes = nullptr; // [max(n_internal, 1)] wide nodes (QNode4 records use the first half)
  unsigned long long* queue = nullptr;  // [kQueueSlots] ray queue heads of persistent launches
  TFacet* tfacets = nullptr;  // [n]
  double* stat_work = nullptr;  // [kStatWords] tree statistics: per-block partial sums
  // BuildState and root bounds hold their starting values (set once after
  // allocation; every build's last kernel sets them again for the next one)
  bool state_ready = false;
  // pinned, device-mapped record that the last kernel of every build fills
  // (sequence number, tree size, errors, root box); one per handle, so builds
  // of different handles may be in flight at once
  int32_t* rec_host = nullptr;
  int32_t* rec_dev = nullptr;
  int rec_seq = 0;          // sequence number of the handle's last build
  int64_t cap_n = 0;        // facets the buffers can hold
  int64_t bytes = 0;
};

// tree statistics (rt_bvh_stats): per-block cost sums and leaf histograms
constexpr int kStatBlocks = 64;
constexpr int kStatHist = RT_LEAF_HIST + 1;  // buckets + the largest leaf
constexpr int kStatWords = kStatBlocks * (2 + kStatHist) + 2 + kStatHist;

// build sizes shared by the allocator and the build (the phase thresholds
// and the capacities derived from them are in rt_build_plan.h)
constexpr int kScanBlock = 1024;
constexpr int kBinReplicas = 4; // copies of a big node's bins that chunks add into (2 and 8 timed: no better)
// bytes of one bin set: counts, ordered-int boxes and (optionally) ordered-int64
// centroid bounds for 3 axes of B bins
__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }
__host__ __device__ inline size_t bins_bytes(int B, bool with_cb) {
  return align8(sizeof(int) * 3 * B) + align8(sizeof(int) * 3 * B * 6) +
         (with_cb ? align8(sizeof(long long) * 3 * B * 6) : 0);
}

// Ordered integer images of floats: signed comparison of the images equals
// the float order (finite values), so atomic integer min/max give exact float
// min/max independent of the order of the updates.
__device__ __host__ inline int32_t f2o(float f) {
  int32_t i;
  __builtin_memcpy(&i, &f, 4);
  return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __host__ inline float o2f(int32_t i) {
  i = i >= 0 ? i : i ^ 0x7fffffff;
  float f;
  __builtin_memcpy(&f, &i, 4);
  return f;
}
__device__ __host__ inline long long d2o(double d) {
  long long i;
  __builtin_memcpy(&i, &d, 8);
  return i >= 0 ? i : i ^ 0x7fffffffffffffffLL;
}
__device__ __host__ inline double o2d(long long i) {
  i = i >= 0 ? i : i ^ 0x7fffffffffffffffLL;
  double d;
  __builtin_memcpy(&d, &i, 8);
  return d;
}

// ---- ray reception (Sec. III-C, Eq. (4)) ----
struct RecvArgs {
  const double* pos;            // [n_rx][3]
  rt_reception* rec;            // [cap]
  unsigned long long* count;    // receptions found
  int64_t cap;
  double delta;
  int32_t n_rx;
  int32_t pad;
};

// One query of a batched trace launch (device table entry).
struct alignas(16) BatchQuery {
  const void* nodes;     // traversal nodes of the query's tree
  const TFacet* facets;  // its leaf-ordered facets
  const float4* rays;    // [n][2] float4
  rt_hit* out;           // [max_b][n]
  double* path_len;      // [n] or null
  int32_t* n_hits;       // [n] or null
  int64_t n;
  int64_t first_batch;   // first work-group number of the query in the launch
  int32_t max_b;
  int32_t pad[3];
  RecvArgs recv;         // field points of a reception launch (n_rx 0 otherwise)
};


// Path length t |d| of a segment in float64, without contraction, so that
// the tracer and the reception kernels accumulate the same bits.
__device__ __forceinline__ double seg_path(float t, float dx, float dy, float dz) {
#pragma clang fp contract(off)
  const double x = dx, y = dy, z = dz;
  return (double)t * sqrt(x * x + y * y + z * z);
}

// Tests one segment (origin o, direction d, range [t0, t1], path length L
// before it) of ray `ray` against every field point and appends the
// receptions.  Called by every active lane of a wave with the same field
// point list; one atomic per wave and field point with receptions.
//
// The decision is the float64 expression below.  Before it, a float32 test
// rejects pairs that cannot pass: with w = R - o and c = |w x d|^2 =
// dist^2 |d|^2, a received pair has dist <= (L + |w|) delta / sqrt(3) <=
// (L + |w|_1) delta / sqrt(3) (the 1-norm bounds |w| without a square root);
// the float32 values of w, c, |w|_1 and |d|^2 are within a few 1e-7 of
// |o|_1 + |w|_1 + L of the exact ones, and the test allows 1e-4 of that sum
// plus 0.1 % of the radius, so every pair the float64 test would receive
// passes it (a NaN or overflow in float32 also passes).  Most pairs are far
// from the line and stop here; the float64 test runs when a lane needs it.
// The field point's index is the same on every lane and the field points do
// not overlap anything a kernel writes (the host checks it), so their
// coordinates are read through the scalar cache as constant data.
__device__ __forceinline__ void receive_segment(const RecvArgs& a, int64_t ray, int order,
                                                float ox, float oy, float oz, float dx, float dy,
                                                float dz, float t0, float t1, double L) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const float ddk = (dx * dx + dy * dy + dz * dz) * 1.001f;
  const float Lf = (float)L;
  const float base = fabsf(ox) + fabsf(oy) + fabsf(oz) + Lf;
  const float kd = (float)(a.delta * 0.57735026918962576) * 1.001f;  // delta / sqrt(3)
  // radius (L + |w|_1) kd + 1e-4 (base + |w|_1) = rad0 + |w|_1 kw
  const float rad0 = fmaf(Lf, kd, 1e-4f * base);
  const float kw = kd + 1e-4f;
  typedef __attribute__((address_space(4))) const double ConstDouble;
  ConstDouble* pos = (ConstDouble*)a.pos;
  // the next field point is loaded while this one is tested
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if (a.n_rx > 0) {
    nx = pos[0];
    ny = pos[1];
    nz = pos[2];
  }
  for (int r = 0; r < a.n_rx; ++r) {
    const double Rx = nx, Ry = ny, Rz = nz;
    const int rn = __builtin_amdgcn_readfirstlane(r + 1 < a.n_rx ? r + 1 : r);
    nx = pos[3 * rn];
    ny = pos[3 * rn + 1];
    nz = pos[3 * rn + 2];
    const float wx = (float)Rx - ox, wy = (float)Ry - oy, wz = (float)Rz - oz;
    const float cx = wy * dz - wz * dy, cy = wz * dx - wx * dz, cz = wx * dy - wy * dx;
    const float c = cx * cx + cy * cy + cz * cz;
    const float rad = fmaf(fabsf(wx) + fabsf(wy) + fabsf(wz), kw, rad0);
    const bool maybe = !(c > ddk * rad * rad);
    if (__ballot(maybe) == 0ull) continue;
    bool ok = false;
    double l = 0.0, dist2 = 0.0;
    if (maybe) {
#pragma clang fp contract(off)
      const double Ox = ox, Oy = oy, Oz = oz, Dx = dx, Dy = dy, Dz = dz;
      const double dd = Dx * Dx + Dy * Dy + Dz * Dz;
      const double ex = Rx - Ox, ey = Ry - Oy, ez = Rz - Oz;
      const double s = (ex * Dx + ey * Dy + ez * Dz) / dd;
      const double px = ex - s * Dx, py = ey - s * Dy, pz = ez - s * Dz;
      dist2 = px * px + py * py + pz * pz;
      l = L + sqrt(ex * ex + ey * ey + ez * ez);
      const double rr = l * a.delta;
      ok = (s >= (double)t0) && (s <= (double)t1) && (3.0 * dist2 <= rr * rr);
    }
    const unsigned long long m = __ballot(ok);
    if (m == 0ull) continue;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base_k = 0;
    if (lane == leader) base_k = atomicAdd(a.count, (unsigned long long)__popcll(m));
    base_k = __shfl(base_k, leader);
    if (ok) {
      const unsigned long long k = base_k + __popcll(m & below);
      if (k < (unsigned long long)a.cap) {
        rt_reception e;
        e.rx = r;
        e.ray = (int32_t)ray;
        e.order = order;
        e.keep = 0;
        e.l = l;
        e.dist = sqrt(dist2);
        a.rec[k] = e;
      }
    }
  }
}

// ---- energy stop rule (Sec. III-B) ----
struct EnergyArgs {
  const int32_t* material;  // [n_tris] by caller facet id
  const double* refl;       // [n_mat]
  double* power;            // [n] or null
  double k0, min_power;
  int32_t n_mat;
  int32_t pad;
};

// Power ratio after a reflection: gain * k0 / l^2, float64 without contraction.
__device__ __forceinline__ double chain_power(double gain, double k0, double l) {
#pragma clang fp contract(off)
  return gain * k0 / (l * l);
}

// error reporting (thread-local message), defined in rt_api.hip
int set_error(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// Argument checks of the trace calls (api.hip).
int check_trace_args(const rt_bvh* b, const float* rays, int64_t n, int32_t max_b, const rt_hit* out,
                     const double* path_len, const int32_t* n_hits, const rt_trace_opts* opts);

// build.hip
int build_tree(Buffers& B, const float* tris, int64_t n, const rt_split_params& p,
               hipStream_t s, rt_bvh_info* info);
// build_tree in two halves: queue the build's kernels on s (*seq: the record
// its last kernel writes), then wait for that record and fill info.
int build_enqueue(Buffers& B, const float* tris, int64_t n, const rt_split_params& p,
                  hipStream_t s, int* seq);
int build_complete(Buffers& B, int64_t n, const rt_split_params& p, int seq, hipStream_t s,
                   rt_bvh_info* info);
// Eq. (1) tree cost and leaf histogram of the built tree into info (synchronous).
int tree_stats(const Buffers& B, int64_t n_nodes, double t_isect, double t_trav,
               rt_bvh_info* info);
// trace.hip
// lanes: 1, or 4 / 16 / 64 lanes tracing each ray together (then opts may not
// ask for seg_rays, ray_stats or a persistent grid); n_tf: facets of the tree;
// queue: the call's own queue head when opts asks for a persistent grid.
int launch_trace(const Buffers& B, int node_format, int depth, const float* rays, int64_t n,
                 int32_t max_bounces, rt_hit* out, double* path_len, int32_t* n_hits,
                 const rt_trace_opts* opts, int lanes, int n_tf, unsigned long long* queue,
                 hipStream_t s);
// Lanes per ray the library picks for n rays on a tree built with max_leaf
// (api.hip).
int trace_lanes(int64_t n, int max_leaf);
// Batched launch over table[0 .. nq) (device), all of one node format;
// total_batches work-groups, or `grid` persistent work-groups taking batches
// from `queue` when grid > 0.  depth: deepest tree of the queries.
// recv: the queries carry field points, every traced segment is tested
// (their counts must have been cleared, see launch_batch_clear_counts).
int launch_trace_batch(const BatchQuery* table, int nq, int64_t total_batches, int node_format,
                       bool recv, int depth, int grid, unsigned long long* queue, hipStream_t s);
// Clears the reception counts of table[0 .. nq) (a kernel: safe in a captured graph).
int launch_batch_clear_counts(const BatchQuery* table, int nq, hipStream_t s);
// Work-groups of the trace kernel that fit the device at once for this format and depth.
int trace_resident_groups(int node_format, bool recv, int depth);
// receive.hip: argument checks of a receivers struct and its kernel arguments.
// Ranges (pointer, bytes) a call writes besides the reception records.
using WrittenRanges = std::initializer_list<std::pair<const void*, int64_t>>;
int check_rx(const rt_receivers* rx, const char* who, WrittenRanges written = {});
RecvArgs recv_args(const rt_receivers* rx);
// Chains with the reception test of every segment (receive.hip zeroes the count first).
int launch_trace_receive(const Buffers& B, int node_format, int depth, const float* rays,
                         int64_t n, int32_t max_bounces, rt_hit* out, double* path_len,
                         int32_t* n_hits, const RecvArgs& recv, int lanes, int n_tf,
                         hipStream_t s);
// Chains stopped by energy, with the reception test when recv is not null.
int launch_trace_energy(const Buffers& B, int node_format, int depth, const float* rays,
                        int64_t n, int32_t max_bounces, rt_hit* out, double* path_len,
                        int32_t* n_hits, const RecvArgs* recv, const EnergyArgs& en, int lanes,
                        int n_tf, hipStream_t s);

}  // namespace rt

struct rt_bvh {
  rt::Buffers buf;
  rt_bvh_info info;
  rt_split_params params;
  int device;
  // Next of the handle's kQueueSlots queue heads: every persistent launch on
  // the handle, whatever its kernel variant or node format, takes the next
  // one, so calls in flight on different streams never share a head.
  mutable std::atomic<unsigned> queue_slot{0};
  // a build queued by rt_rebuild_async whose record has not been read yet
  // (info.n_tris stays 0 meanwhile, so no call uses the tree)
  bool pending = false;
  int pending_seq = 0;
  int64_t pending_n = 0;
  rt_split_params pending_params;
  hipStream_t pending_stream = nullptr;
};
