// Internal layouts and helpers of the gfx950 ray tracing library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rt_mi355x.h"

namespace rt {

// ---- build-time node (one per binary tree node, breadth-first order) ----
// The two children of a node are stored next to each other.
struct BNode {
  float lo[3], hi[3];      // volume: union of the facets' boxes
  int32_t left;            // left child id, -1 leaf
  int32_t first, count;    // facet range in the reference order
  int32_t depth;
  int32_t axis, plane, flags;
  int32_t tidx;            // index in the traversal node array (internal nodes)
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
constexpr int kQueueSlots = 64;  // trace calls that may be in flight on one handle at once

// ---- build-time facet record, kept in reference order: 32 bytes ----
//   lo = (box lo xyz, caller's id bits), hi = (box hi xyz, 0)
struct alignas(16) FacetRec {
  float4 lo, hi;
};

struct Buffers {
  // build scratch
  FacetRec* recs_a = nullptr;  // [n] facet records, ping-pong between levels
  FacetRec* recs_b = nullptr;
  int32_t* perm = nullptr;  // [n] final leaf order
  BNode* nodes = nullptr;   // [2n - 1]
  int32_t* act_a = nullptr; // [n] active node ids
  int32_t* act_b = nullptr;
  int32_t* cand = nullptr;  // [2n] facet count of a child that stays internal, else 0
  int32_t* big = nullptr;   // [n] level positions of nodes above the big-node size
  int32_t* small = nullptr; // [n] level positions of the other nodes
  int32_t* counters = nullptr;  // small device counters
  long long* root_box = nullptr; // ordered-int root bounds (6 float + 6 double)
  // traversal data
  TNode* tnodes = nullptr;  // [max(n_internal, 1)]
  FNode4* wnodes = nullptr; // [max(n_internal, 1)] wide nodes (QNode4 records use the first half)
  unsigned long long* queue = nullptr;  // [kQueueSlots] ray queue heads, one per trace call in flight
  TFacet* tfacets = nullptr;  // [n]
  int64_t cap_n = 0;        // facets the buffers can hold
  int64_t bytes = 0;
};

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

// error reporting (thread-local message), defined in rt_api.hip
int set_error(int code, const std::string& msg);
int check_hip(hipError_t e, const char* what);

// build.hip
int build_tree(Buffers& B, const float* tris, int64_t n, const rt_split_params& p,
               hipStream_t s, rt_bvh_info* info);
// trace.hip
int launch_trace(const Buffers& B, int node_format, int depth, const float* rays, int64_t n,
                 int32_t max_bounces, rt_hit* out, double* path_len, int32_t* n_hits,
                 const rt_trace_opts* opts, hipStream_t s);

}  // namespace rt

struct rt_bvh {
  rt::Buffers buf;
  rt_bvh_info info;
  rt_split_params params;
  int device;
};
