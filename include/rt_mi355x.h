/* rt_mi355x.h -- C ABI of the MI355X (gfx950) closest-hit ray tracer.
 *
 * The library builds a bounding volume hierarchy over triangular facets with
 * the split cost that blends the surface area heuristic with the squared
 * distance from the ray source point (Sec. II-B, Eq. (2)), then traces
 * launched rays through it: a ray enters only the bounding volumes it meets
 * (Sec. III-B), keeps the nearest facet hit inside its action range
 * [tmin, tmax], and may be re-launched as a specular reflection up to a set
 * number of segments (Sec. III-B, reflection order).  Around the chains:
 * batched launches of many queries (trees, ray sets), receiving spheres at
 * field points (Sec. III-C, Eq. (4)), the energy stop rule and edge
 * diffraction (Sec. III-B).
 *
 * Conventions shared by every call:
 *   - All array arguments are DEVICE pointers (HBM) unless a comment says
 *     "host".  The caller owns them; the library never frees them.
 *   - Every call that takes a stream enqueues its device work on that stream
 *     (hipStream_t, 0 = the null stream).  rt_build and rt_rebuild also wait
 *     for it: the whole build runs on the device and ends by writing one
 *     record (node count, depth, errors) that the host reads.
 *   - Functions return RT_OK (0) or a negative RT_E* code; the text of the
 *     last error on the calling thread is given by rt_last_error().  No C++
 *     exception crosses this interface.
 *   - Facets: float32 [n][9] = (v0.xyz, v1.xyz, v2.xyz), 4-byte aligned.
 *     Facet ids are the caller's indices 0..n-1.
 *   - Rays: float32 [m][8] = (ox, oy, oz, tmin, dx, dy, dz, tmax), 32 bytes
 *     per ray, 16-byte aligned.  d need not be unit length; t is the ray
 *     parameter (point = o + t d).  The range is closed: tmin <= t <= tmax.
 *   - Hits: rt_hit, 16 bytes, 16-byte aligned.  Ties on t go to the smaller
 *     facet id; a miss is {-1, +inf, 0, 0}.
 */
#ifndef RT_MI355X_H
#define RT_MI355X_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RT_OK 0
#define RT_EINVAL (-1) /* bad argument: null / misaligned pointer, size, NaN facet, parameter out of range */
#define RT_ENOMEM (-2) /* device allocation failed */
#define RT_EHIP (-3)   /* a HIP runtime call failed; rt_last_error() has its text */
#define RT_EDEPTH (-4) /* internal: tree deeper than the traversal stack */

/* ---- split parameters (Sec. II-B, Sec. II-C) ---------------------------- */
#define RT_D_CHILD_MEAN 0      /* d^2 = mean of the two child volumes' d^2 (default) */
#define RT_D_CHILD_SUM 1       /* d^2 = sum of the two children's d^2 */
#define RT_D_CHILD_KWEIGHTED 2 /* d^2 = facet-count-weighted mean of the children's d^2 */
#define RT_D_PARENT 3          /* d^2 of the parent volume: constant per node, equals Eq. (1) */

#define RT_DNORM_UNIT 0 /* SAH part / (k_C t_i), distance part / (root diagonal)^2 (default) */
#define RT_DNORM_RAW 1  /* Eq. (2) in the units it is printed in (metres squared) */

/* Traversal node formats (Sec. II-C tree, stored for the GPU) */
#define RT_NODE_BIN2 0 /* binary: both child volumes as float32 in the parent, 64 B per node */
#define RT_NODE_F4 1   /* 4-wide: pairs of tree levels merged, float32 child volumes, 128 B */
#define RT_NODE_Q4 2   /* 4-wide, child volumes as 8-bit offsets from a float32 origin with
                          power-of-two scales per axis, rounded outward so that the decoded
                          volume always contains the exact one, 64 B */

#define RT_MAX_BINS 64     /* largest nbins */
#define RT_MAX_DEPTH 64    /* largest depth_limit: the traversal stack holds this many entries */
#define RT_MAX_BOUNCES 64  /* largest max_bounces */
#define RT_LEAF_HIST 16    /* buckets of the leaf-size histogram (rt_bvh_stats) */

typedef struct rt_split_params {
  float alpha;       /* Eq. (2) weight in [0, 1]; 1 = surface area only (Eq. (1)), 0 = distance only */
  float t_isect;     /* t_i, cost of one facet test (> 0) */
  float t_trav;      /* t_trav, per-node constant of Eq. (1)/(2) (>= 0) */
  float src[3];      /* ray source point whose distance to a volume's centre enters Eq. (2) */
  int32_t max_leaf;  /* a node holding <= max_leaf facets is a leaf (>= 1) */
  int32_t nbins;     /* candidate planes: nbins equal centroid bins per axis (2..RT_MAX_BINS) */
  int32_t d_mode;    /* RT_D_* */
  int32_t d_norm;    /* RT_DNORM_* */
  int32_t max_depth; /* from this depth on, alpha is taken as 1 */
  int32_t depth_limit; /* no leaf deeper than this (1..RT_MAX_DEPTH); nodes that could
                          not otherwise meet it are halved by position */
  int32_t node_format; /* RT_NODE_*: layout the traversal reads; never changes the tree
                          or the hits */
} rt_split_params;

/* Defaults: alpha 1, t_isect 1, t_trav 1, src 0, max_leaf 4, nbins 16,
 * RT_D_CHILD_MEAN, RT_DNORM_UNIT, max_depth 32, depth_limit 64, RT_NODE_BIN2. */
void rt_split_params_default(rt_split_params* p);

/* ---- results ------------------------------------------------------------ */
typedef struct rt_hit {
  int32_t tri_id; /* caller's facet index, -1 = miss */
  float t;        /* ray parameter of the hit, +inf on a miss */
  float u, v;     /* hit point = (1 - u - v) v0 + u v1 + v v2 */
} rt_hit;

typedef struct rt_bvh rt_bvh; /* opaque; owns its device memory */

typedef struct rt_bvh_info {
  int64_t n_tris;
  int64_t n_nodes;     /* binary tree nodes, leaves included (2 * n_internal + 1) */
  int64_t n_internal;
  int64_t n_leaves;
  int32_t depth;       /* deepest leaf, root = 0 */
  int32_t n_levels;    /* tree levels (depth + 1) */
  int64_t device_bytes; /* device memory held by the handle */
  int64_t trace_bytes;  /* of which: traversal nodes + leaf-ordered facets */
  float root_lo[3], root_hi[3];
  int32_t node_format;  /* RT_NODE_* of the traversal nodes */
  int32_t n_trace_nodes; /* traversal node records; record (left - 1) / 2 belongs to the
                            internal node whose children are left, left + 1 (wide formats:
                            only even-depth internal nodes have one, so some records are
                            unused) */
  /* Filled by rt_bvh_stats (has_stats = 1); rt_bvh_info_get leaves them 0. */
  int32_t has_stats;
  int32_t max_leaf_count; /* facets of the largest leaf */
  double tree_cost;     /* Eq. (1) cost of the whole tree (Sec. II-B): the sum over internal
                           nodes n of S(n) / S(root) * t_trav plus the sum over leaves l of
                           S(l) / S(root) * k_l * t_i, S the surface area 2 (wh + hd + dw) of
                           the node's volume, k_l its facet count, t_i and t_trav the build's
                           split parameters; float64.  When S(root) = 0 every ratio is 1. */
  double root_area;     /* S(root) */
  int64_t leaf_hist[RT_LEAF_HIST]; /* leaves by facet count c: bucket c - 1 for c <= 8,
                           bucket 5 + floor(log2(c - 1)) for 9 <= c <= 1024 (9-16, 17-32,
                           ..., 513-1024), bucket 15 for c > 1024 */
} rt_bvh_info;

/* One node of the binary tree.  Node 0 is the root; the two children of a
 * node are adjacent (right = left + 1); the order of the pairs follows the
 * build's schedule and is not fixed. */
typedef struct rt_node_rec {
  float lo[3], hi[3]; /* node volume: union of its facets' boxes (Eq. (3) bounds) */
  int32_t left;       /* index of the left child, -1 for a leaf */
  int32_t first;      /* facets perm[first .. first + count) belong to this node */
  int32_t count;
  int32_t depth;      /* root = 0 */
  int32_t axis;       /* chosen split axis 0..2, -1 for leaves and position splits */
  int32_t plane;      /* chosen bin boundary 1..nbins-1, -1 likewise */
  int32_t flags;      /* bit0 halved by position (depth limit), bit1 all centroids equal,
                         bit2 alpha taken as 1 (depth >= max_depth) */
  int32_t reserved;
  double cost;        /* Eq. (2) cost of the chosen split (0 if none) */
} rt_node_rec;

/* ---- build (Sec. II-C) ---------------------------------------------------
 * Builds the tree of n facets on the GPU: per-facet boxes and centroids,
 * root volume, then for every internal node: bin its centroids, evaluate
 * Eq. (2) on every bin boundary, and partition the node's facets (stable:
 * each side keeps the input order).  The tree does not depend on the order in
 * which the device processes nodes.  tris may be freed once the call returns.
 * *out receives a new handle.  Waits for stream s.
 * Errors: RT_EINVAL (null, n < 1, n >= 2^30, non-finite vertex, bad params),
 * RT_ENOMEM, RT_EHIP. */
int rt_build(const float* tris, int64_t n, const rt_split_params* p, rt_bvh** out,
             hipStream_t s);

/* Rebuilds an existing handle in place for new facets or parameters, reusing
 * its device memory when it is large enough.  Same contract as rt_build. */
int rt_rebuild(rt_bvh* b, const float* tris, int64_t n, const rt_split_params* p,
               hipStream_t s);

/* The same build as rt_rebuild (Sec. II-B, II-C), queued on stream s without
 * waiting for it: returns once its kernels are queued, so the host can queue
 * other work (another handle's trace, the next handle's build) while it runs.
 * The handle is unusable (every call that reads the tree returns RT_EINVAL,
 * rt_bvh_info_get reports n_tris = 0) until rt_bvh_wait(b) has read the
 * build's record; errors found on the device (a non-finite vertex, a capacity
 * check) are returned by rt_bvh_wait.  Work queued on other streams that uses
 * the tree must wait for s (an event recorded on s after this call).  tris
 * must stay valid until the build has run.  rt_rebuild, rt_rebuild_async and
 * rt_bvh_destroy on a handle with a build in flight end that build first.
 * Errors returned at once: RT_EINVAL (as rt_rebuild's arguments), RT_ENOMEM,
 * RT_EHIP; the handle is then unusable until rebuilt. */
int rt_rebuild_async(rt_bvh* b, const float* tris, int64_t n, const rt_split_params* p,
                     hipStream_t s);

/* Waits for the build rt_rebuild_async queued on b (host spin on the build's
 * record, then a synchronisation of its stream if the record is late) and
 * makes the tree usable.  RT_OK at once if no build is in flight.  Errors:
 * RT_EINVAL (NULL, or a non-finite vertex), RT_EHIP (device error, capacity
 * check); the handle then stays unusable until rebuilt. */
int rt_bvh_wait(rt_bvh* b);

/* ---- trace (Sec. III-B) -------------------------------------------------
 * Closest hit of each ray: out[i] for rays[i].  n = 0 is a no-op.  The handle
 * may be traced concurrently from several streams.
 * Errors: RT_EINVAL (null / misaligned pointers, n < 0). */
int rt_trace(const rt_bvh* b, const float* rays, int64_t n, rt_hit* out, hipStream_t s);

/* Reflection chains: each ray is traced; after a hit it is reflected
 * specularly about the facet's plane and launched again from the hit point
 * with the same [tmin, tmax], ignoring the facet it leaves, until it misses
 * or max_bounces segments have been traced.
 *   out       [max_bounces][n] rt_hit, segment b of ray i at out[b * n + i];
 *             segments after the one that missed are written as misses
 *   path_len  [n] float64: sum over the hits of t * |d| (nullable)
 *   n_hits    [n] int32: number of hits (reflection points) (nullable)
 * Errors: RT_EINVAL (as rt_trace; max_bounces outside 1..RT_MAX_BOUNCES). */
int rt_trace_bounces(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                     rt_hit* out, double* path_len, int32_t* n_hits, hipStream_t s);

/* rt_trace_opts.flags: rows of out for segments never traced (those after a
 * chain's first miss) are left as they were instead of being written as
 * misses; a chain with h hits has rows 0 .. min(h, max_bounces - 1) written
 * (row h, when it exists, is its miss).  Needs n_hits to read out. */
#define RT_TRACE_NO_PAD 1

/* Optional outputs and launch shape for rt_trace_ex. */
typedef struct rt_trace_opts {
  float* seg_rays;     /* nullable, [max_bounces][n][8]: the ray of every traced segment,
                          as rays[] (the reflected origin, direction, tmin, tmax); rows of
                          segments never traced are left untouched */
  uint32_t* ray_stats; /* nullable, [n][2]: nodes visited and facets tested per ray,
                          summed over its segments (instrumented kernel, slower) */
  int32_t block;       /* reserved, must be 0 or 64 (one wave per work-group) */
  int32_t grid;        /* 0: one work-group (one wave) per 64 consecutive rays, scheduled by the
                          hardware (fastest measured); > 0: this many persistent work-groups
                          taking batches of rays from an atomic queue of the handle's own
                          (each call takes the next of 64 queues, so up to 64 such calls may
                          be in flight on one handle at once, on any streams) */
  int32_t refill;      /* persistent mode: 0 = a wave takes 64 consecutive rays when all its
                          chains have ended; 1 = free lanes take new rays at every segment */
  int32_t lanes_per_ray; /* 0: chosen by the library; 1: one lane per ray; 4, 16 or 64: that
                          many lanes trace each ray together and split every leaf's facets
                          (for trees with large leaves and launches too small to fill the
                          device); > 1 requires seg_rays and ray_stats NULL and grid 0.  The
                          library chooses > 1 only for trees built with max_leaf >= 16: with
                          G <= max_leaf, 64 for n <= 50 max_leaf, 16 for n <= 700 max_leaf,
                          4 for n <= 12000 max_leaf,
                          the same for rt_trace, rt_trace_bounces, rt_trace_receive and
                          rt_trace_energy (batched launches trace one lane per ray).
                          Results do not depend on it. */
  int32_t cut;         /* 0: every chain is traced to its end in one launch; k >= 1: two
                          launches (Sec. III-B re-launch, late segments regrouped): the
                          first traces every chain's first k segments and appends the chains
                          still alive after them to chain_ws (one atomic add per wave), the
                          second traces those from segment k on, 64 per wave.  Needs chain_ws,
                          grid 0 and one lane per
                          ray; no effect when max_bounces <= k.  Each chain's hits, path
                          length and hit count are those of the one-launch trace up to the
                          order in which a wave's lanes test leaves (a chain whose closest
                          hit is decided within rounding may differ) */
  int32_t flags;       /* 0 or RT_TRACE_NO_PAD */
  void* chain_ws;      /* cut >= 1: caller-owned device workspace of at least
                          rt_trace_chain_ws_bytes(n) bytes, 256-byte aligned, used by this
                          call only (calls that overlap need workspaces of their own) */
  int64_t chain_ws_bytes;
  const int32_t* batch_order; /* nullable, device [ceil(n / 64)]: the order in which the
                          launch starts its batches of 64 consecutive rays (work-group g traces
                          batch batch_order[g]); a permutation of 0 .. ceil(n / 64) - 1 (an
                          entry outside that range traces nothing, a repeated one traces its
                          batch again with the same results).  Results do not depend on it;
                          the launch's duration does: the hardware starts work-groups in index
                          order, and chains that run long but start late set the launch's
                          end.  rt_rays_batch_order makes one from the ray directions.  With
                          cut >= 1 it orders the first launch.  Needs grid 0 and one lane per
                          ray (lanes_per_ray 0 then means 1). */
} rt_trace_opts;

/* Workspace of a two-launch trace (rt_trace_opts.cut >= 1) of n rays: a
 * 256-byte header (the live-chain count) and a 64-byte chain state per ray.
 * n < 0: 0. */
int64_t rt_trace_chain_ws_bytes(int64_t n);

/* rt_trace_bounces with optional outputs (opts nullable).
 * Errors: as rt_trace_bounces; RT_EINVAL for a misaligned seg_rays / ray_stats,
 * block, grid, refill or lanes_per_ray outside their values, lanes_per_ray > 1
 * with seg_rays, ray_stats or grid > 0, n > (2^31 - 1) 64 / lanes_per_ray,
 * cut < 0, flags other than 0 or RT_TRACE_NO_PAD, RT_TRACE_NO_PAD without
 * n_hits, cut >= 1 with seg_rays, ray_stats, grid > 0,
 * lanes_per_ray > 1, n >= 2^31, or chain_ws NULL, misaligned or smaller than
 * rt_trace_chain_ws_bytes(n), or batch_order misaligned or with grid > 0 or
 * lanes_per_ray > 1. */
int rt_trace_ex(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                rt_hit* out, double* path_len, int32_t* n_hits, const rt_trace_opts* opts,
                hipStream_t s);

/* ---- launched rays (Sec. III-A) -----------------------------------------
 * Writes n rays from the source point (ox, oy, oz) along the first n launch
 * directions of a resident direction table: rays[i] = (o, tmin, dirs[i],
 * tmax), float32 [n][8].  dirs: device float32 [>= n][3] (the directions of a
 * subdivided icosahedron in first-appearance order, so any prefix is a valid
 * launch set).  rays 16-byte aligned.  Enqueued on s.
 * Errors: RT_EINVAL (NULL, misaligned, n < 0, tmin > tmax or not finite), RT_EHIP. */
int rt_rays_from_directions(const float* dirs, int64_t n, float ox, float oy, float oz, float tmin,
                            float tmax, float* rays, hipStream_t s);

/* Dispatch order for rt_trace_opts.batch_order from the ray directions.  Rays
 * are taken in batches of 64 consecutive ones (the last may be shorter).  A
 * ray's q = floor(1023 d_a^2 / |d|^2) in float32, each operation rounded on its
 * own (a = axis: 0 x, 1 y, 2 z; q = 0 for a zero or non-finite direction); a
 * batch's key is the smallest q among its rays, and its class c the number of
 * k in 1..15 with key >= floor(1023 k^2 / 256), i.e. the smallest |d_a| / |d|
 * in sixteenths.  order lists the batches by ascending class, in index order
 * within a class: the batches holding a ray nearest the plane normal to the
 * axis come first.  With the axis pointing up in an outdoor scene those rays
 * reflect between facades and build the longest chains (Sec. III-B
 * re-launch), and a wave lasts as long as its longest chain, so these batches
 * start while the rest of the launch can still fill the device around them.
 * rays: device float32 [n][8], 16-byte aligned; order: device int32
 * [ceil(n / 64)]; keys: caller-owned device workspace of
 * rt_rays_batch_order_ws_bytes(n) bytes, 4-byte aligned (its first
 * ceil(n / 64) int32 are left holding the batch keys).  Three kernels enqueued
 * on s.  n = 0 writes nothing.
 * Errors: RT_EINVAL (NULL, misaligned, n < 0 or n >= 2^31, axis outside 0..2),
 * RT_EHIP. */
int rt_rays_batch_order(const float* rays, int64_t n, int32_t axis, int32_t* order,
                        int32_t* keys, hipStream_t s);
/* Workspace of rt_rays_batch_order for n rays: 4 (ceil(n / 64) + 16 ceil(n / 65536))
 * bytes; n < 0: 0. */
int64_t rt_rays_batch_order_ws_bytes(int64_t n);

/* Many launches with one kernel (a serving batch): launch j writes n rays from
 * its source along the first n directions of dirs to rows first .. first + n - 1
 * of rays, as rt_rays_from_directions does.  table: device array of `count`
 * records sorted by `first`, whose row ranges do not overlap; a record with
 * n > n_dirs, a negative first or n, or a range past `total` writes nothing.
 * Rows that no record covers are left as they are.  rays: device float32
 * [total][8], 16-byte aligned.  Enqueued on s.
 * Errors: RT_EINVAL (NULL, misaligned, count or total or n_dirs < 0, tmin > tmax
 * or not finite), RT_EHIP. */
typedef struct rt_ray_launch {
  float src[3];      /* source point */
  int32_t reserved;  /* 0 */
  int64_t first;     /* first row of rays */
  int64_t n;         /* rays of this launch */
} rt_ray_launch;     /* 32 bytes */
int rt_rays_from_directions_many(const float* dirs, int64_t n_dirs, const rt_ray_launch* table,
                                 int32_t count, float tmin, float tmax, float* rays, int64_t total,
                                 hipStream_t s);

/* ---- ray reception (Sec. III-C, Eq. (4)) ---------------------------------
 * A field point R receives segment b of a ray (b = 0: the launched ray, b = k:
 * after k reflections; origin o, direction d, range [tmin, t_end] with t_end
 * the hit's t, or tmax when the segment missed) when the foot of the
 * perpendicular from R lies in that range and R lies in the receiving sphere
 * of radius l * delta / sqrt(3):
 *     w = R - o,  s = (w.d) / (d.d),  dist^2 = |w - s d|^2,
 *     l = L_b + |w|  (L_b = sum over the earlier hits of t |d|, the path
 *                     length up to o; l is the path source -> R),
 *     received  <=>  tmin <= s <= t_end  and  3 dist^2 <= (l delta)^2.
 * Evaluated in float64 from the float32 segment, in exactly this order,
 * without fused multiply-add, so equal inputs give equal decisions on any
 * IEEE float64 implementation.  Field points with a NaN coordinate are never
 * received. */
typedef struct rt_reception {
  int32_t rx;    /* index of the field point */
  int32_t ray;   /* index of the ray */
  int32_t order; /* segment index b (number of reflections before it) */
  int32_t keep;  /* 0 as found; rt_receive_dedup sets 1 on one reception per path */
  double l;      /* path length from the source to the field point along the ray */
  double dist;   /* distance of the field point from the segment's line */
} rt_reception; /* 32 bytes */

typedef struct rt_receivers {
  const double* pos;  /* device float64 [n][3] field points, 8-byte aligned; read as constant
                         data, so it may not overlap rec, count or any other output of the
                         call (RT_EINVAL) and must not change while a launch runs */
  int32_t n;          /* number of field points, >= 0 */
  int32_t reserved;   /* must be 0 */
  double delta;       /* angle between adjacent launched rays, radians, finite, >= 0 */
  rt_reception* rec;  /* device [cap] output, 16-byte aligned (nullable when cap == 0) */
  int64_t cap;        /* records rec can hold, 0 .. 2^31 - 1 */
  int64_t* count;     /* device int64: set to the number of receptions found, which
                         may exceed cap; only min(count, cap) records are written, in
                         no particular order (a truncated set is an arbitrary subset) */
} rt_receivers;

/* rt_trace_bounces that also tests every traced segment against the field
 * points as it is traced (the segment is never stored).  rx is a host struct.
 * Cost: one float64 test per segment and field point, so meant for up to a few
 * hundred field points.  Errors: as rt_trace_bounces; RT_EINVAL for a bad rx
 * (NULL count, n >= 2^31 rays, misaligned or NULL pos / rec, delta not
 * finite or negative, cap out of range). */
int rt_trace_receive(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                     rt_hit* out, double* path_len, int32_t* n_hits, const rt_receivers* rx,
                     hipStream_t s);

/* The same reception test over stored chains: seg_rays [max_bounces][n][8]
 * (as written by rt_trace_ex's seg_rays) and hits [max_bounces][n] (as
 * written by rt_trace_bounces).  Segment b of ray i exists when b == 0 or
 * hits[b - 1][i] is a hit (and so on down to 0); only existing segments are
 * read.  Results equal rt_trace_receive's on the chains that produced them.
 * Errors: RT_EINVAL (NULL / misaligned arrays, n outside 0..2^31 - 1,
 * max_bounces outside 1..RT_MAX_BOUNCES, bad rx), RT_EHIP. */
int rt_receive_segments(const float* seg_rays, const rt_hit* hits, int64_t n,
                        int32_t max_bounces, const rt_receivers* rx, hipStream_t s);

/* Bytes of device workspace rt_receive_dedup needs for cap records and
 * n_rx field points (256-byte multiple); -1 if the sizes are out of range. */
int64_t rt_receive_dedup_workspace(int64_t cap, int32_t n_rx);

/* Groups the first min(*rx->count, rx->cap) records by (field point, order,
 * facets hit before the segment, read from hits [max_bounces][n]) and sets
 * keep = 1 on one record per group -- the smallest dist, ties to the smaller
 * ray index -- and keep = 0 on the others.  Neighbouring rays whose receiving
 * spheres overlap give one group per propagation path.  work: device, at
 * least rt_receive_dedup_workspace(rx->cap, rx->n) bytes, 256-byte aligned.
 * Records whose rx, ray or order are out of range are left with keep = 0.
 * Errors: RT_EINVAL (NULL / misaligned, workspace too small), RT_EHIP. */
int rt_receive_dedup(const rt_hit* hits, int64_t n, int32_t max_bounces, const rt_receivers* rx,
                     void* work, int64_t work_bytes, hipStream_t s);

/* ---- energy stop rule (Sec. III-B) ---------------------------------------
 * Besides the reflection order, a chain ends when its energy has decayed
 * below a threshold.  After the reflection at hit j (facet f_j, path length
 * l_j from the source to the hit point, accumulated in float64 as path_len)
 * the chain carries the power ratio
 *     P_j = (refl[material[f_1]] * ... * refl[material[f_j]]) * k0 / l_j^2,
 * refl being the power reflection coefficient of a material and k0 the
 * free-space constant (lambda / (4 pi))^2 of isotropic antennas, evaluated in
 * float64 in this order; the next segment is launched only while
 * P_j >= min_power.  A material index outside [0, n_materials) reflects
 * nothing (P = 0).  min_power = 0 never stops a chain. */
typedef struct rt_energy {
  const int32_t* material; /* device [n_tris]: material index of each facet (caller's ids) */
  const double* refl;      /* device [n_materials]: power reflection coefficients */
  int32_t n_materials;     /* >= 0 (refl may be NULL when 0) */
  int32_t reserved;        /* must be 0 */
  double k0;               /* free-space constant, finite, > 0 */
  double min_power;        /* threshold, finite, >= 0 */
  double* power;           /* device [n], nullable: P of each chain's last hit, 0 without hits */
} rt_energy;

/* rt_trace_bounces with the energy stop rule (e: host struct), and, when rx
 * is not NULL, the receiving-sphere test of every traced segment as in
 * rt_trace_receive.  Errors: as rt_trace_bounces / rt_trace_receive; RT_EINVAL
 * for a NULL e or material, n_materials < 0, NULL refl with n_materials > 0,
 * misaligned arrays, k0 not finite and positive, min_power not finite and
 * >= 0, reserved != 0. */
int rt_trace_energy(const rt_bvh* b, const float* rays, int64_t n, int32_t max_bounces,
                    const rt_energy* e, rt_hit* out, double* path_len, int32_t* n_hits,
                    const rt_receivers* rx, hipStream_t s);

/* ---- edge diffraction (Sec. III-B: rays meeting facets give reflected and
 * diffracted rays) ---------------------------------------------------------
 * Wedges.  Edge k of facet f runs from its vertex k to vertex (k + 1) % 3.
 * Two half-edges are one edge when their end points are equal float32 points
 * (in either order).  An edge of exactly one facet is free (neighbour -1); an
 * edge of exactly two facets is a wedge when their normals
 * n = (v1 - v0) x (v2 - v0) (float64) satisfy (n_a.n_b)^2 < cos^2(1 deg)
 * |n_a|^2 |n_b|^2 (neighbour = the other facet's index); any other edge does
 * not diffract (-2).
 *
 * Diffraction of a stored chain's hit: segment b of a ray hits facet f at
 * p = o + t d after a path l = L_b + t |d|.  The nearest wedge or free edge of
 * f whose segment lies within the ray-tube radius rho = l delta / sqrt(3)
 * (Eq. (4)) of p (ties to the lower edge index) diffracts at q, the point of
 * the edge nearest p.  With unit edge direction e and unit incident direction
 * i, c = i.e, r = i - c e, sin(beta) = |r| (no diffraction when 0), u = r / |r|,
 * w = e x u, the Keller-cone directions are c e + sin(beta) (cos_k u + sin_k w)
 * for the caller's (cos_k, sin_k) table; at a wedge, directions whose part
 * across the edge lies strictly between the two facets (towards their third
 * vertices) point into the solid and are dropped.  All of it in float64 in
 * this order without fused multiply-add; q and the directions are rounded to
 * float32 once.  Diffracted rays are ordinary rays: trace them with
 * rt_trace_bounces. */
typedef struct rt_diffracted {
  int32_t ray;    /* parent ray */
  int32_t order;  /* parent segment (reflections before the diffracting hit) */
  int32_t facet;  /* facet hit */
  int32_t edge;   /* 0..2: the facet's edge that diffracts */
  int32_t cone;   /* index in the cone table */
  int32_t pad;
  double path;    /* path length from the source to the diffraction point q */
  float ray8[8];  /* the diffracted ray as in rays[]: q, parent tmin, direction, parent tmax */
} rt_diffracted;  /* 64 bytes */

/* Neighbour of every half-edge: nbr device int32 [n][3].  tris: device
 * float32 [n][9].  Synchronises the stream (sorts with temporary device
 * memory).  Errors: RT_EINVAL (NULL / misaligned, n < 1 or >= 2^29,
 * non-finite vertex), RT_ENOMEM, RT_EHIP. */
int rt_wedges(const float* tris, int64_t n, int32_t* nbr, hipStream_t s);

/* rt_wedges for callers that cannot allocate device memory (code that must
 * not call hipMalloc / hipFree, such as tight serving loops and harnesses that
 * forbid it): the same result, bit for bit, with every temporary buffer taken
 * from a device array the library holds for each GPU until the process ends
 * (24 MiB), so n is limited to 1..262144 facets (RT_EINVAL beyond).  All calls
 * on one GPU share that array: calls that overlap in time on one GPU (other
 * host threads, other streams) race and must not be made.  Synchronises the
 * stream.  Errors: as rt_wedges. */
int rt_wedges_noalloc(const float* tris, int64_t n, int32_t* nbr, hipStream_t s);

/* Diffracted rays of stored chains (seg_rays and hits as for
 * rt_receive_segments) over the facets tris [n_tris][9] with their
 * neighbours nbr [n_tris][3] from rt_wedges.  cone: device float64
 * [n_cone][2] (cos, sin); out: device [cap] records, *count (device int64)
 * set to the number found (only min(count, cap) written, in no particular
 * order).  Hits on facet indices outside [0, n_tris) do not diffract.
 * Errors: RT_EINVAL (NULL / misaligned, sizes out of range, delta not finite
 * or negative, n_cone outside 0..1024), RT_EHIP. */
int rt_diffract_segments(const float* tris, int64_t n_tris, const int32_t* nbr,
                         const float* seg_rays, const rt_hit* hits, int64_t n,
                         int32_t max_bounces, double delta, const double* cone, int32_t n_cone,
                         rt_diffracted* out, int64_t cap, int64_t* count, hipStream_t s);

/* ---- inspection and lifetime ------------------------------------------ */
/* Sizes recorded by the last build (host struct, no device work). */
int rt_bvh_info_get(const rt_bvh* b, rt_bvh_info* info);

/* Tree statistics (Sec. II-B, Eq. (1) tree cost): everything rt_bvh_info_get
 * gives plus the total cost of the tree and the leaf-size histogram, computed
 * on the device from the built tree (float64 sums in a fixed order, so equal
 * trees give equal bits).  info: host struct.  Synchronises the device.
 * Errors: RT_EINVAL (NULL, tree not built), RT_EHIP. */
int rt_bvh_stats(const rt_bvh* b, rt_bvh_info* info);

/* Copies the binary tree (host buffers): nodes [info.n_nodes], perm [n_tris]
 * (leaf order of the caller's facet ids).  Synchronises the device.
 * RT_EINVAL if a capacity is too small. */
int rt_bvh_download(const rt_bvh* b, rt_node_rec* nodes, int64_t node_cap, int32_t* perm,
                    int64_t perm_cap);

/* Copies the traversal node array as the GPU reads it (host buffer of at
 * least *bytes; call with host = NULL to get the size).  Layouts, all little
 * endian, one record per node index:
 *   RT_NODE_BIN2, 64 B: float c0lox, c0hix, c0loy, c0hiy; c1lox, c1hix, c1loy, c1hiy;
 *                 c0loz, c0hiz, c1loz, c1hiz; int32 ref0, ref1, 0, 0
 *   RT_NODE_F4, 128 B: float lox[4], hix[4], loy[4], hiy[4], loz[4], hiz[4];
 *                 int32 ref[4]; uint32 mask (bit c: child c present), 0, 0, 0
 *   RT_NODE_Q4, 64 B: float ox, oy, oz; uint32 meta = (ex + 127) | (ey + 127) << 8 |
 *                 (ez + 127) << 16 | mask << 24; uint8 qlox[4], qloy[4], qloz[4], qhix[4],
 *                 qhiy[4], qhiz[4]; 8 bytes 0; int32 ref[4].  Child c's volume is
 *                 lo = o + q_lo 2^e, hi = o + q_hi 2^e per axis in exact (real)
 *                 arithmetic, which contains the child's float32 volume; e >= -64.
 * A reference r >= 0 is a node index, r < 0 a leaf whose facets start at
 * leaf-order position ~r.  Synchronises the device. */
int rt_bvh_export_trace_nodes(const rt_bvh* b, void* host, int64_t* bytes);

void rt_bvh_destroy(rt_bvh* b); /* NULL is a no-op; waits for the device */

/* ---- streams on split compute units ----------------------------------------
 * For overlapping one transmitter's build with another's trace: the trace's
 * one-wave work-groups fill every compute unit as fast as earlier ones
 * retire, so the build's larger work-groups start only once the trace has
 * none left to dispatch.  These two streams divide the device's compute
 * units instead: `small` gets k of them and `large` the rest, so work on
 * `small` never waits for room.  The runtime may number an MI355X's 256 CUs
 * by XCD (blocks of 32) or interleaved over its 8 XCDs (CU c on XCD c mod 8);
 * `small` takes k / 8 CUs of every block, block b first those numbered b mod
 * 8, then b + 1 mod 8, ..., so that either way every XCD gives k / 8 CUs to
 * `small` and keeps the rest for `large` (a stream left with no CU on some
 * XCD could not run the work-groups the hardware hands that XCD).  k: a
 * multiple of 8 in 8..128.  Both are ordinary streams of default priority for
 * the current device; free them with rt_stream_destroy.
 * Errors: RT_EINVAL (NULL, k outside those values, a device without 256 CUs),
 * RT_EHIP. */
int rt_streams_split_cus(int32_t k, hipStream_t* small, hipStream_t* large);
/* The mask `small` gets (host only, no device): bit c of word c / 32 set for
 * each of its CUs; small_mask: host uint32 [8].  Errors: RT_EINVAL (NULL, k). */
int rt_split_cus_mask(int32_t k, uint32_t* small_mask);
int rt_stream_destroy(hipStream_t s); /* a stream from rt_streams_split_cus; RT_EHIP on failure */

/* ---- batched trace (Sec. III-B for many transmitters and scenes) ---------
 * Many queries -- each a resident tree, a set of launched rays and a bounce
 * limit, optionally field points -- traced in one launch per node format and
 * kind.  Every query's results are exactly those of rt_trace_bounces (with
 * field points: rt_trace_receive) on the same tree and rays: they do not
 * depend on the other queries, their order or the launch shape. */
typedef struct rt_query {
  const rt_bvh* bvh;    /* resident tree (built, not destroyed while a launch is pending) */
  const float* rays;    /* device float32 [n][8], 16-byte aligned */
  int64_t n;            /* rays, >= 0 */
  int32_t max_bounces;  /* 1..RT_MAX_BOUNCES: segments per chain */
  int32_t status;       /* written by rt_batch_set: RT_OK, or RT_EINVAL and left out */
  rt_hit* out;          /* device [max_bounces][n], 16-byte aligned */
  double* path_len;     /* device [n] (float64 path length per chain) or NULL */
  int32_t* n_hits;      /* device [n] (facets hit per chain) or NULL */
  const rt_receivers* receivers; /* host struct of device buffers (Sec. III-C, Eq. (4)): every
                                    traced segment is tested as in rt_trace_receive, the count
                                    cleared by each launch; read by rt_batch_set (the buffers
                                    must outlive the launches); NULL: no reception test.
                                    With field points n must be < 2^31. */
} rt_query;

#define RT_BATCH_DIRECT 0 /* one work-group per 64-ray batch of every query */
#define RT_BATCH_QUEUE 1  /* persistent work-groups take 64-ray batches from an atomic counter */
#define RT_ORDER_GIVEN 0  /* queries start in the order given */
#define RT_ORDER_COST 1   /* queries with the most rays x bounces start first */

typedef struct rt_batch_config {
  int32_t mode;  /* RT_BATCH_* */
  int32_t grid;  /* RT_BATCH_QUEUE: persistent work-groups, 0 = as many as fit the device */
  int32_t order; /* RT_ORDER_* */
  int32_t graph; /* 1: launch through a hipGraph (captured on a stream of the batch's own,
                    launched on the caller's), captured again when the batch's shape (queries
                    per format, batches, depths) or the configuration changes */
} rt_batch_config;

typedef struct rt_batch rt_batch; /* opaque: device query table, pinned staging, graph */

/* New batch holding up to max_queries queries (1..65536); defaults: DIRECT,
 * ORDER_COST, no graph.  Errors: RT_EINVAL, RT_ENOMEM, RT_EHIP. */
int rt_batch_create(int32_t max_queries, rt_batch** out);

/* Sets the queries (host array, copied; each query's status is written).
 * Invalid queries (NULL or unbuilt tree, NULL or misaligned pointers, n < 0,
 * bounces out of range) get RT_EINVAL and are left out; the others are kept.
 * Waits until an earlier launch of this batch has read its table.
 * Errors: RT_EINVAL (NULL batch or array, nq outside 0..max_queries). */
int rt_batch_set(rt_batch* b, rt_query* queries, int32_t nq);

int rt_batch_configure(rt_batch* b, const rt_batch_config* cfg); /* RT_EINVAL on bad values */
int rt_batch_get_config(const rt_batch* b, rt_batch_config* cfg);

/* Enqueues the table upload and the trace launches on stream s (no wait).
 * Errors: RT_EINVAL, RT_EHIP. */
int rt_batch_launch(rt_batch* b, hipStream_t s);

/* Times every launch shape (DIRECT and QUEUE at 1x and 2x the resident
 * work-groups, both orders) over `reps` launches each on stream s, keeps the
 * fastest (the graph flag is left as it is) and returns its average time per
 * launch in *ms (may be NULL).  Writes the results of the queries several
 * times over.  Synchronises the stream.  Errors: RT_EINVAL, RT_EHIP. */
int rt_batch_autotune(rt_batch* b, int32_t reps, hipStream_t s, float* ms);

void rt_batch_destroy(rt_batch* b); /* NULL is a no-op; waits for the device */

const char* rt_last_error(void); /* thread-local, never NULL */

#ifdef __cplusplus
}
#endif
#endif /* RT_MI355X_H */
