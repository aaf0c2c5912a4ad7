// GPU tree build (Sec. II-C) with the Eq. (2) split cost (Sec. II-B).
//
// Flow, one kernel pass per tree level:
//   k_prep     per facet: box, centroid (float64), reference list, root bounds
//   k_root     root node from the reduced bounds
//   k_level    one work-group per node of the level: bin the centroids on the
//              three axes, evaluate Eq. (2) on every bin boundary, pick the
//              cheapest (ties: lower axis, then lower boundary), partition the
//              facet references stably into the two children
//   k_compact  list the children that still hold more than max_leaf facets
//   k_emit     traversal nodes and leaf-ordered facets
//
// Every decision (bin index, Eq. (2) cost, argmin) is made in float64 with a
// fixed operation order and no contraction into fused multiply-adds, so the
// tree does not depend on thread scheduling: boxes are unions (exact min/max
// through ordered-integer atomics), counts are integers, and the partition
// keeps the input order on each side.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "rt_internal.h"

namespace rt {
namespace {

constexpr int kCompactThreads = 1024;

// counters[] slots
enum { C_NONFINITE = 0, C_NEXT = 1, C_BIG = 2, C_SMALL = 3 };

struct BuildConst {
  double alpha, t_isect, t_trav, src[3];
  double inv_l2;  // 1 / squared root diagonal (0 if the root is a point)
  int32_t max_leaf, nbins, d_mode, d_norm, max_depth, depth_limit;
};

__device__ inline double area(const double lo[3], const double hi[3]) {
  double ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
  return 2.0 * ((ex * ey + ey * ez) + ez * ex);
}

__device__ inline double dist2(const BuildConst& C, const double lo[3], const double hi[3]) {
  double cx = (lo[0] + hi[0]) * 0.5 - C.src[0];
  double cy = (lo[1] + hi[1]) * 0.5 - C.src[1];
  double cz = (lo[2] + hi[2]) * 0.5 - C.src[2];
  return (cx * cx + cy * cy) + cz * cz;
}

// Eq. (2): alpha (S(A)/S(C) k_A t_i + S(B)/S(C) k_B t_i) + (1 - alpha) d^2 + t_trav.
// RT_DNORM_UNIT divides the surface-area part by k_C t_i and d^2 by the squared
// root diagonal; RT_DNORM_RAW keeps the printed units.
__device__ double eq2_cost(const BuildConst& C, double alpha, const double alo[3],
                           const double ahi[3], int ka, const double blo[3],
                           const double bhi[3], int kb, const double clo[3],
                           const double chi[3], int kc) {
  double sa = area(alo, ahi), sb = area(blo, bhi), sc = area(clo, chi);
  double num = sa * (double)ka + sb * (double)kb;
  double da = dist2(C, alo, ahi), db = dist2(C, blo, bhi);
  double d;
  switch (C.d_mode) {
    case RT_D_CHILD_SUM: d = da + db; break;
    case RT_D_CHILD_KWEIGHTED: d = (da * (double)ka + db * (double)kb) / (double)kc; break;
    case RT_D_PARENT: d = dist2(C, clo, chi); break;
    default: d = (da + db) * 0.5; break;
  }
  double sah, tt;
  if (C.d_norm == RT_DNORM_RAW) {
    sah = num * C.t_isect / sc;
    tt = C.t_trav;
  } else {
    sah = num / (sc * (double)kc);
    d = d * C.inv_l2;
    tt = C.t_trav / (C.t_isect * (double)kc);
  }
  return alpha * sah + (1.0 - alpha) * d + tt;
}

// number of halvings that take k facets down to max_leaf
__device__ __host__ inline int halvings(int k, int max_leaf) {
  int need = (k + max_leaf - 1) / max_leaf;
  int l = 0;
  while ((1 << l) < need) ++l;
  return l;
}

// centroid of a facet = centre of its box, in float64 (exact for the sum of
// two float32 values in practice, and the same expression everywhere)
__device__ inline double centroid(float lo, float hi) { return ((double)lo + (double)hi) * 0.5; }

__device__ inline int bin_of(double c, double lo, double scale, int nb) {
  return min(nb - 1, (int)((c - lo) * scale));
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ tris, int n,
                                              FacetRec* __restrict__ recs, int32_t* __restrict__ perm,
                                              int32_t* __restrict__ counters,
                                              long long* __restrict__ root);

__global__ void k_root_init(long long* root) {
  int t = threadIdx.x;
  if (t < 3) {
    root[t] = f2o(INFINITY);
    root[3 + t] = f2o(-INFINITY);
    root[6 + t] = d2o(INFINITY);
    root[9 + t] = d2o(-INFINITY);
  }
}

__global__ void k_root(const long long* root, int n, BNode* nodes, double* inv_l2) {
  BNode r;
  for (int a = 0; a < 3; ++a) {
    r.lo[a] = o2f((int32_t)root[a]);
    r.hi[a] = o2f((int32_t)root[3 + a]);
    r.cblo[a] = o2d(root[6 + a]);
    r.cbhi[a] = o2d(root[9 + a]);
  }
  r.left = -1;
  r.first = 0;
  r.count = n;
  r.depth = 0;
  r.axis = r.plane = -1;
  r.flags = 0;
  r.tidx = 0;
  r.cost = 0.0;
  nodes[0] = r;
  double ex = (double)r.hi[0] - (double)r.lo[0];
  double ey = (double)r.hi[1] - (double)r.lo[1];
  double ez = (double)r.hi[2] - (double)r.lo[2];
  double l2 = (ex * ex + ey * ey) + ez * ez;
  *inv_l2 = l2 > 0.0 ? 1.0 / l2 : 0.0;
}

// ---------------------------------------------------------------------------
// wave-wide reductions and scans (64 lanes)
__device__ inline int lane_id() { return threadIdx.x & 63; }
__device__ inline float wmin(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o));
  return v;
}
__device__ inline float wmax(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wmin(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double wmax(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ inline int wscan_incl(int v) {
  const int lane = lane_id();
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}
// lanes of one wave see each other's LDS writes after this
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int G>
__device__ inline void group_sync() {
  if constexpr (G == 64) {
    wave_sync();
  } else {
    __syncthreads();
  }
}

// Level bookkeeping kept on the device, so several levels can be queued
// without waiting for the host.
struct LevelState {
  int32_t active;      // nodes of the current level
  int32_t n_big;       // of which above kBigNode facets
  int32_t n_small;
  int32_t child_base;  // first node id of the current level's children
  int32_t n_internal;  // internal nodes before the current level
  int32_t levels;      // levels with at least one node so far
  int32_t pad[2];
};

__global__ __launch_bounds__(256) void k_prep(const float* __restrict__ tris, int n,
                                              FacetRec* __restrict__ recs, int32_t* __restrict__ perm,
                                              int32_t* __restrict__ counters,
                                              long long* __restrict__ root) {
  __shared__ int s_box[6];
  __shared__ long long s_cb[6];
  if (threadIdx.x < 6) {
    s_box[threadIdx.x] = threadIdx.x < 3 ? f2o(INFINITY) : f2o(-INFINITY);
    s_cb[threadIdx.x] = threadIdx.x < 3 ? d2o(INFINITY) : d2o(-INFINITY);
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (i < n) {
    const float* v = tris + 9 * (int64_t)i;
    float x[9];
    for (int k = 0; k < 9; ++k) x[k] = v[k];
    bool finite = true;
    for (int k = 0; k < 9; ++k) finite = finite && isfinite(x[k]);
    if (!finite) atomicOr(&counters[C_NONFINITE], 1);
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(fminf(x[a], x[3 + a]), x[6 + a]);
      hi[a] = fmaxf(fmaxf(x[a], x[3 + a]), x[6 + a]);
      clo[a] = chi[a] = centroid(lo[a], hi[a]);
    }
    FacetRec r;
    r.lo = make_float4(lo[0], lo[1], lo[2], __int_as_float(i));
    r.hi = make_float4(hi[0], hi[1], hi[2], 0.f);
    recs[i] = r;
    perm[i] = i;  // final unless the facets are split
  }
  for (int a = 0; a < 3; ++a) {
    const float l = wmin(lo[a]), h = wmax(hi[a]);
    const double cl = wmin(clo[a]), ch = wmax(chi[a]);
    if (lane_id() == 0) {
      atomicMin(&s_box[a], f2o(l));
      atomicMax(&s_box[3 + a], f2o(h));
      atomicMin(&s_cb[a], d2o(cl));
      atomicMax(&s_cb[3 + a], d2o(ch));
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    atomicMin(&root[threadIdx.x], (long long)s_box[threadIdx.x]);
    atomicMax(&root[3 + threadIdx.x], (long long)s_box[3 + threadIdx.x]);
    atomicMin(&root[6 + threadIdx.x], s_cb[threadIdx.x]);
    atomicMax(&root[9 + threadIdx.x], s_cb[3 + threadIdx.x]);
  }
}

// nodes above kBigNode facets: one work-group of kBigThreads threads each
constexpr int kBigNode = 256;

// LDS of one node group, carved from dynamic shared memory; sized by nbins.
struct NodeLds {
  int ncopy;         // private bin copies (one per wave, or shared round-robin)
  int* cnt;          // [ncopy][3][B]
  int* box;          // [ncopy][3][B][6] ordered ints: lo xyz, hi xyz
  long long* cb;     // [ncopy][3][B][6] ordered int64: centroid lo xyz, hi xyz
  double* cost;      // [3 (B - 1)]
  int* wtot;         // [16] per-wave totals of a group scan
  int* wtot2;        // [kPartE][16] per-slice per-wave totals of the partition
  int* pick;         // [2]
  double* best;      // [1]
  int* cbox;         // [2][6]   child boxes (position splits)
  long long* ccb;    // [2][6]
};

__host__ __device__ inline size_t align8(size_t x) { return (x + 7) & ~size_t(7); }
__host__ __device__ inline size_t bin_copy_bytes(int B) {
  return align8(sizeof(int) * 3 * B) + align8(sizeof(int) * 3 * B * 6) +
         align8(sizeof(long long) * 3 * B * 6);
}
// Bin copies for a group of `waves` waves: one per wave while they fit in
// about 44 KB (fewer lanes contend for one bin), at least one.
__host__ __device__ inline int bin_copies(int B, int waves) {
  const int fit = (int)((44 * 1024) / bin_copy_bytes(B));
  return fit < 1 ? 1 : (fit < waves ? fit : waves);
}
__host__ __device__ inline size_t node_lds_bytes(int B, int ncopy) {
  size_t o = 0;
  o = align8(o + sizeof(int) * 3 * B * ncopy);
  o = align8(o + sizeof(int) * 3 * B * 6 * ncopy);
  o = align8(o + sizeof(long long) * 3 * B * 6 * ncopy);
  o = align8(o + sizeof(double) * 3 * (B - 1));
  o = align8(o + sizeof(int) * 16);
  o = align8(o + sizeof(int) * 16 * 8);
  o = align8(o + sizeof(int) * 2);
  o = align8(o + sizeof(double));
  o = align8(o + sizeof(int) * 12);
  o = align8(o + sizeof(long long) * 12);
  return o;
}
__device__ inline NodeLds node_lds(char* base, int B, int ncopy) {
  NodeLds L;
  size_t o = 0;
  L.ncopy = ncopy;
  L.cnt = (int*)(base + o);        o = align8(o + sizeof(int) * 3 * B * ncopy);
  L.box = (int*)(base + o);        o = align8(o + sizeof(int) * 3 * B * 6 * ncopy);
  L.cb = (long long*)(base + o);   o = align8(o + sizeof(long long) * 3 * B * 6 * ncopy);
  L.cost = (double*)(base + o);    o = align8(o + sizeof(double) * 3 * (B - 1));
  L.wtot = (int*)(base + o);       o = align8(o + sizeof(int) * 16);
  L.wtot2 = (int*)(base + o);      o = align8(o + sizeof(int) * 16 * 8);
  L.pick = (int*)(base + o);       o = align8(o + sizeof(int) * 2);
  L.best = (double*)(base + o);    o = align8(o + sizeof(double));
  L.cbox = (int*)(base + o);       o = align8(o + sizeof(int) * 12);
  L.ccb = (long long*)(base + o);
  return L;
}

struct LevelArgs {
  BNode* nodes;
  const FacetRec* in;   // facet records of the level, in reference order
  FacetRec* out;        // the same records partitioned for the next level
  int32_t* perm;
  const int32_t* act;   // node ids of the level, in order
  const int32_t* sel;   // positions in act handled by this kernel
  int32_t* cand;        // per child slot: its facet count if it stays internal, else 0
  const double* inv_l2;
  const LevelState* st;
  int32_t n;
  BuildConst C;
};

constexpr int kPartE = 8;  // consecutive records per thread and partition round

__device__ inline unsigned long long lanes_below() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Exclusive wave prefix of a small count v in 0..15 and the wave total, from
// four ballots (no cross-lane data movement).
__device__ inline int wave_excl_small(int v, int& total) {
  const unsigned long long below = lanes_below();
  int pre = 0, tot = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const unsigned long long m = __ballot((v >> b) & 1);
    pre += __popcll(m & below) << b;
    tot += __popcll(m) << b;
  }
  total = tot;
  return pre;
}

// Group exclusive prefixes of the left and right counts (each 0..15) of G
// threads, with the group totals.
template <int G>
__device__ inline void group_scan2(int nl, int nr, int& pl, int& pr, int& tl, int& tr,
                                   const NodeLds& S, int gtid) {
  int wl, wr;
  pl = wave_excl_small(nl, wl);
  pr = wave_excl_small(nr, wr);
  if constexpr (G == 64) {
    tl = wl;
    tr = wr;
  } else {
    const int wave = gtid >> 6;
    if (lane_id() == 0) S.wtot[wave] = wl | (wr << 16);
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < G / 64; ++w) {
      const int x = S.wtot[w];
      if (w < wave) pre += x;
      tot += x;
    }
    __syncthreads();
    pl += pre & 0xffff;
    pr += pre >> 16;
    tl = tot & 0xffff;
    tr = tot >> 16;
  }
}

// Run of consecutive facets that fall in one bin of one axis, kept in
// registers and merged into the bin when the bin changes.
struct Run {
  int bin, count;
  float lo[3], hi[3];
  double clo[3], chi[3];
};
__device__ inline void run_reset(Run& r, int bin) {
  r.bin = bin;
  r.count = 0;
  for (int q = 0; q < 3; ++q) {
    r.lo[q] = INFINITY;
    r.hi[q] = -INFINITY;
    r.clo[q] = INFINITY;
    r.chi[q] = -INFINITY;
  }
}
__device__ inline void run_flush(const Run& r, const NodeLds& S, int copy, int a, int B) {
  if (r.count == 0) return;
  const int slot = (copy * 3 + a) * B + r.bin;
  atomicAdd(&S.cnt[slot], r.count);
  int* bx = S.box + 6 * slot;
  long long* cb = S.cb + 6 * slot;
  for (int q = 0; q < 3; ++q) {
    atomicMin(&bx[q], f2o(r.lo[q]));
    atomicMax(&bx[3 + q], f2o(r.hi[q]));
    atomicMin(&cb[q], d2o(r.clo[q]));
    atomicMax(&cb[3 + q], d2o(r.chi[q]));
  }
}

// One node of the level: bin, evaluate Eq. (2), partition, emit children.
// G threads (one wave or one work-group) handle the node.
template <int G>
__device__ void process_node(const LevelArgs& A, int j, const NodeLds& S, int gtid) {
  const int lane = lane_id();
  const int id = A.act[j];
  const BNode nd = A.nodes[id];
  const int k = nd.count, s = nd.first;
  const int B = A.C.nbins;
  BuildConst C = A.C;
  C.inv_l2 = *A.inv_l2;
  const int child_base = A.st->child_base;

  double alpha = C.alpha;
  int flags = 0;
  const bool forced = nd.depth + halvings(k, C.max_leaf) >= C.depth_limit;
  if (forced) {
    flags = 1;
  } else if (nd.depth >= C.max_depth) {
    alpha = 1.0;
    flags |= 4;
  }
  double ext[3], scale[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ext[a] = nd.cbhi[a] - nd.cblo[a];
    scale[a] = ext[a] > 0.0 ? (double)B / ext[a] : 0.0;
  }
  if (gtid < 12) {
    const int side = gtid / 6, c = gtid % 6;
    S.cbox[6 * side + c] = c < 3 ? f2o(INFINITY) : f2o(-INFINITY);
    S.ccb[6 * side + c] = c < 3 ? d2o(INFINITY) : d2o(-INFINITY);
  }
  int axis = -1, plane = -1;
  double best = INFINITY;
  if (!forced) {
    const int my_copy = (gtid >> 6) % S.ncopy;
    for (int c = gtid; c < 3 * B * S.ncopy; c += G) {
      S.cnt[c] = 0;
      for (int q = 0; q < 3; ++q) {
        S.box[6 * c + q] = f2o(INFINITY);
        S.box[6 * c + 3 + q] = f2o(-INFINITY);
        S.cb[6 * c + q] = d2o(INFINITY);
        S.cb[6 * c + 3 + q] = d2o(-INFINITY);
      }
    }
    group_sync<G>();
    // binning: each thread walks a contiguous run of the node's facets
    const int per = (k + G - 1) / G;
    const int i0 = min(k, gtid * per), i1 = min(k, i0 + per);
    Run run[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) run_reset(run[a], -1);
    // loads of kBinU facets are issued together before they are merged
    constexpr int kBinU = 4;
    for (int i = i0; i < i1; i += kBinU) {
      float4 lo[kBinU], hi[kBinU];
      double cu[kBinU][3];
#pragma unroll
      for (int u = 0; u < kBinU; ++u) {
        const int q = min(i + u, i1 - 1);
        lo[u] = A.in[s + q].lo;
        hi[u] = A.in[s + q].hi;
      }
#pragma unroll
      for (int u = 0; u < kBinU; ++u) {
        cu[u][0] = centroid(lo[u].x, hi[u].x);
        cu[u][1] = centroid(lo[u].y, hi[u].y);
        cu[u][2] = centroid(lo[u].z, hi[u].z);
      }
#pragma unroll
      for (int u = 0; u < kBinU; ++u) {
        if (i + u >= i1) break;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (!(ext[a] > 0.0)) continue;
          const int b = bin_of(cu[u][a], nd.cblo[a], scale[a], B);
          if (b != run[a].bin) {
            run_flush(run[a], S, my_copy, a, B);
            run_reset(run[a], b);
          }
          Run& r = run[a];
          r.count += 1;
          r.lo[0] = fminf(r.lo[0], lo[u].x); r.lo[1] = fminf(r.lo[1], lo[u].y); r.lo[2] = fminf(r.lo[2], lo[u].z);
          r.hi[0] = fmaxf(r.hi[0], hi[u].x); r.hi[1] = fmaxf(r.hi[1], hi[u].y); r.hi[2] = fmaxf(r.hi[2], hi[u].z);
          r.clo[0] = fmin(r.clo[0], cu[u][0]); r.clo[1] = fmin(r.clo[1], cu[u][1]); r.clo[2] = fmin(r.clo[2], cu[u][2]);
          r.chi[0] = fmax(r.chi[0], cu[u][0]); r.chi[1] = fmax(r.chi[1], cu[u][1]); r.chi[2] = fmax(r.chi[2], cu[u][2]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) run_flush(run[a], S, my_copy, a, B);
    group_sync<G>();
    if (S.ncopy > 1) {  // fold the private copies into copy 0
      for (int c = gtid; c < 3 * B; c += G) {
        int cnt = S.cnt[c];
        int bx[6];
        long long cb[6];
        for (int q = 0; q < 6; ++q) {
          bx[q] = S.box[6 * c + q];
          cb[q] = S.cb[6 * c + q];
        }
        for (int cp = 1; cp < S.ncopy; ++cp) {
          const int o = cp * 3 * B + c;
          cnt += S.cnt[o];
          for (int q = 0; q < 3; ++q) {
            bx[q] = min(bx[q], S.box[6 * o + q]);
            bx[3 + q] = max(bx[3 + q], S.box[6 * o + 3 + q]);
            cb[q] = min(cb[q], S.cb[6 * o + q]);
            cb[3 + q] = max(cb[3 + q], S.cb[6 * o + 3 + q]);
          }
        }
        S.cnt[c] = cnt;
        for (int q = 0; q < 6; ++q) {
          S.box[6 * c + q] = bx[q];
          S.cb[6 * c + q] = cb[q];
        }
      }
      group_sync<G>();
    }
    const int ncand = 3 * (B - 1);
    double clo[3], chi[3];
    for (int q = 0; q < 3; ++q) {
      clo[q] = nd.lo[q];
      chi[q] = nd.hi[q];
    }
    for (int c = gtid; c < ncand; c += G) {
      const int a = c / (B - 1), pl = c % (B - 1) + 1;
      double cost = INFINITY;
      if (ext[a] > 0.0) {
        double alo[3] = {INFINITY, INFINITY, INFINITY}, ahi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int ka = 0, kb = 0;
        for (int b = 0; b < B; ++b) {
          const int slot = a * B + b;
          const int cnt = S.cnt[slot];
          if (cnt == 0) continue;
          const int* bx = S.box + 6 * slot;
          const double l0 = o2f(bx[0]), l1 = o2f(bx[1]), l2 = o2f(bx[2]);
          const double h0 = o2f(bx[3]), h1 = o2f(bx[4]), h2 = o2f(bx[5]);
          if (b < pl) {
            ka += cnt;
            alo[0] = fmin(alo[0], l0); alo[1] = fmin(alo[1], l1); alo[2] = fmin(alo[2], l2);
            ahi[0] = fmax(ahi[0], h0); ahi[1] = fmax(ahi[1], h1); ahi[2] = fmax(ahi[2], h2);
          } else {
            kb += cnt;
            blo[0] = fmin(blo[0], l0); blo[1] = fmin(blo[1], l1); blo[2] = fmin(blo[2], l2);
            bhi[0] = fmax(bhi[0], h0); bhi[1] = fmax(bhi[1], h1); bhi[2] = fmax(bhi[2], h2);
          }
        }
        if (ka > 0 && kb > 0) cost = eq2_cost(C, alpha, alo, ahi, ka, blo, bhi, kb, clo, chi, k);
      }
      S.cost[c] = cost;
    }
    group_sync<G>();
    if (gtid < 64) {
      // first strict minimum in (axis, plane) order: lexicographic (cost, index)
      double bc = INFINITY;
      int bi = 1 << 30;
      for (int c = gtid; c < ncand; c += 64) {
        const double x = S.cost[c];
        if (x < bc) {
          bc = x;
          bi = c;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double oc = __shfl_xor(bc, o);
        const int oi = __shfl_xor(bi, o);
        if (oc < bc || (oc == bc && oi < bi)) {
          bc = oc;
          bi = oi;
        }
      }
      if (gtid == 0) {
        const bool ok = bc < INFINITY;
        S.pick[0] = ok ? bi / (B - 1) : -1;
        S.pick[1] = ok ? bi % (B - 1) + 1 : -1;
        *S.best = bc;
      }
    }
    group_sync<G>();
    axis = S.pick[0];
    plane = S.pick[1];
    best = *S.best;
    if (axis < 0) flags |= 2;
  }
  const bool by_position = axis < 0;
  int nleft;
  if (by_position) {
    nleft = k / 2;
  } else {
    nleft = 0;
    for (int b = 0; b < plane; ++b) nleft += S.cnt[axis * B + b];
  }
  const int cnt0 = nleft, cnt1 = k - nleft;
  const int fst0 = s, fst1 = s + nleft;
  const bool leaf0 = cnt0 <= C.max_leaf, leaf1 = cnt1 <= C.max_leaf;
  // split axis constants as scalars (no dynamic indexing of small arrays)
  const int ax = by_position ? 0 : axis;
  const double ax_lo = ax == 0 ? nd.cblo[0] : (ax == 1 ? nd.cblo[1] : nd.cblo[2]);
  const double ax_scale = ax == 0 ? scale[0] : (ax == 1 ? scale[1] : scale[2]);

  // stable partition, kPartE consecutive records per thread and round
  float blo[2][3], bhi[2][3];
  double cbl[2][3], cbh[2][3];
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      blo[side][q] = INFINITY;
      bhi[side][q] = -INFINITY;
      cbl[side][q] = INFINITY;
      cbh[side][q] = -INFINITY;
    }
  // Round of G * kPartE records, slice e = records base + e G + [0, G):
  // loads and stores are coalesced; one exchange of per-wave slice totals
  // gives every record its stable rank.
  constexpr int NW = G / 64;
  int lbase = 0, rbase = 0;
  const int wave = gtid >> 6;
  const unsigned long long below = lanes_below();
  for (int base = 0; base < k; base += G * kPartE) {
    FacetRec r[kPartE];
    bool gl[kPartE], valid[kPartE];
    unsigned long long ml[kPartE], mr[kPartE];
#pragma unroll
    for (int e = 0; e < kPartE; ++e) {
      const int i = base + e * G + gtid;
      valid[e] = i < k;
      r[e] = A.in[s + min(i, k - 1)];
    }
#pragma unroll
    for (int e = 0; e < kPartE; ++e) {
      const int i = base + e * G + gtid;
      bool g = false;
      if (valid[e]) {
        if (by_position) {
          g = i < nleft;
        } else {
          const float l = ax == 0 ? r[e].lo.x : (ax == 1 ? r[e].lo.y : r[e].lo.z);
          const float h = ax == 0 ? r[e].hi.x : (ax == 1 ? r[e].hi.y : r[e].hi.z);
          g = bin_of(centroid(l, h), ax_lo, ax_scale, B) < plane;
        }
      }
      gl[e] = g;
      ml[e] = __ballot(g);
      mr[e] = __ballot(valid[e] && !g);
    }
    // per-slice offsets of this wave: earlier slices (all waves) + earlier waves of this slice
    int offl[kPartE], offr[kPartE];
    int tl = 0, tr = 0;
    if constexpr (NW == 1) {
#pragma unroll
      for (int e = 0; e < kPartE; ++e) {
        offl[e] = tl;
        offr[e] = tr;
        tl += __popcll(ml[e]);
        tr += __popcll(mr[e]);
      }
    } else {
      if (lane_id() < kPartE) {
        int cl = 0, cr = 0;
#pragma unroll
        for (int e = 0; e < kPartE; ++e)
          if (e == lane_id()) {
            cl = __popcll(ml[e]);
            cr = __popcll(mr[e]);
          }
        S.wtot2[lane_id() * NW + wave] = cl | (cr << 16);
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < kPartE; ++e) {
        int pre = 0, tot = 0;
        for (int w = 0; w < NW; ++w) {
          const int x = S.wtot2[e * NW + w];
          if (w < wave) pre += x;
          tot += x;
        }
        offl[e] = tl + (pre & 0xffff);
        offr[e] = tr + (pre >> 16);
        tl += tot & 0xffff;
        tr += tot >> 16;
      }
      __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kPartE; ++e) {
      if (!valid[e]) continue;
      const int dst = gl[e] ? fst0 + lbase + offl[e] + __popcll(ml[e] & below)
                            : fst1 + rbase + offr[e] + __popcll(mr[e] & below);
      A.out[dst] = r[e];
      if (gl[e] ? leaf0 : leaf1) A.perm[dst] = __float_as_int(r[e].lo.w);
      if (by_position) {  // no bins: child bounds from the facets themselves
        const float4 lo = r[e].lo, hi = r[e].hi;
        const double cx = centroid(lo.x, hi.x), cy = centroid(lo.y, hi.y), cz = centroid(lo.z, hi.z);
        if (gl[e]) {
          blo[0][0] = fminf(blo[0][0], lo.x); blo[0][1] = fminf(blo[0][1], lo.y); blo[0][2] = fminf(blo[0][2], lo.z);
          bhi[0][0] = fmaxf(bhi[0][0], hi.x); bhi[0][1] = fmaxf(bhi[0][1], hi.y); bhi[0][2] = fmaxf(bhi[0][2], hi.z);
          cbl[0][0] = fmin(cbl[0][0], cx); cbl[0][1] = fmin(cbl[0][1], cy); cbl[0][2] = fmin(cbl[0][2], cz);
          cbh[0][0] = fmax(cbh[0][0], cx); cbh[0][1] = fmax(cbh[0][1], cy); cbh[0][2] = fmax(cbh[0][2], cz);
        } else {
          blo[1][0] = fminf(blo[1][0], lo.x); blo[1][1] = fminf(blo[1][1], lo.y); blo[1][2] = fminf(blo[1][2], lo.z);
          bhi[1][0] = fmaxf(bhi[1][0], hi.x); bhi[1][1] = fmaxf(bhi[1][1], hi.y); bhi[1][2] = fmaxf(bhi[1][2], hi.z);
          cbl[1][0] = fmin(cbl[1][0], cx); cbl[1][1] = fmin(cbl[1][1], cy); cbl[1][2] = fmin(cbl[1][2], cz);
          cbh[1][0] = fmax(cbh[1][0], cx); cbh[1][1] = fmax(cbh[1][1], cy); cbh[1][2] = fmax(cbh[1][2], cz);
        }
      }
    }
    lbase += tl;
    rbase += tr;
  }
  if (by_position) {
    for (int side = 0; side < 2; ++side)
      for (int q = 0; q < 3; ++q) {
        const float l = wmin(blo[side][q]), h = wmax(bhi[side][q]);
        const double cl = wmin(cbl[side][q]), ch = wmax(cbh[side][q]);
        if (lane == 0) {
          atomicMin(&S.cbox[6 * side + q], f2o(l));
          atomicMax(&S.cbox[6 * side + 3 + q], f2o(h));
          atomicMin(&S.ccb[6 * side + q], d2o(cl));
          atomicMax(&S.ccb[6 * side + 3 + q], d2o(ch));
        }
      }
  }
  group_sync<G>();
  const int c0 = child_base + 2 * j;
  if (gtid < 2) {
    BNode ch;
    if (by_position) {
      for (int q = 0; q < 3; ++q) {
        ch.lo[q] = o2f(S.cbox[6 * gtid + q]);
        ch.hi[q] = o2f(S.cbox[6 * gtid + 3 + q]);
        ch.cblo[q] = o2d(S.ccb[6 * gtid + q]);
        ch.cbhi[q] = o2d(S.ccb[6 * gtid + 3 + q]);
      }
    } else {
      // union of the bins on this child's side of the plane
      int bl[6] = {f2o(INFINITY), f2o(INFINITY), f2o(INFINITY), f2o(-INFINITY), f2o(-INFINITY), f2o(-INFINITY)};
      long long cl[6] = {d2o(INFINITY), d2o(INFINITY), d2o(INFINITY), d2o(-INFINITY), d2o(-INFINITY), d2o(-INFINITY)};
      const int b0 = gtid == 0 ? 0 : plane, b1 = gtid == 0 ? plane : B;
      for (int b = b0; b < b1; ++b) {
        const int slot = axis * B + b;
        if (S.cnt[slot] == 0) continue;
        for (int q = 0; q < 3; ++q) {
          bl[q] = min(bl[q], S.box[6 * slot + q]);
          bl[3 + q] = max(bl[3 + q], S.box[6 * slot + 3 + q]);
          cl[q] = min(cl[q], S.cb[6 * slot + q]);
          cl[3 + q] = max(cl[3 + q], S.cb[6 * slot + 3 + q]);
        }
      }
      for (int q = 0; q < 3; ++q) {
        ch.lo[q] = o2f(bl[q]);
        ch.hi[q] = o2f(bl[3 + q]);
        ch.cblo[q] = o2d(cl[q]);
        ch.cbhi[q] = o2d(cl[3 + q]);
      }
    }
    ch.left = -1;
    ch.first = gtid == 0 ? fst0 : fst1;
    ch.count = gtid == 0 ? cnt0 : cnt1;
    ch.depth = nd.depth + 1;
    ch.axis = ch.plane = -1;
    ch.flags = 0;
    ch.tidx = -1;
    ch.cost = 0.0;
    A.nodes[c0 + gtid] = ch;
    A.cand[2 * j + gtid] = (gtid == 0 ? leaf0 : leaf1) ? 0 : ch.count;
  }
  if (gtid == 2) {
    BNode* p = &A.nodes[id];
    p->left = c0;
    p->axis = axis;
    p->plane = plane;
    p->flags = flags;
    p->cost = by_position ? 0.0 : best;
  }
}

constexpr int kBigThreads = 512;

__global__ __launch_bounds__(kBigThreads) void k_level_big(LevelArgs A) {
  extern __shared__ __align__(16) char lds[];
  if ((int)blockIdx.x >= A.st->n_big) return;
  process_node<kBigThreads>(A, A.sel[blockIdx.x],
                            node_lds(lds, A.C.nbins, bin_copies(A.C.nbins, kBigThreads / 64)),
                            threadIdx.x);
}

// smaller nodes: one wave each, several per work-group (no work-group barrier)
__global__ __launch_bounds__(256) void k_level_small(LevelArgs A) {
  extern __shared__ __align__(16) char lds[];
  const int w = threadIdx.x >> 6;
  const int q = blockIdx.x * (blockDim.x >> 6) + w;
  if (q >= A.st->n_small) return;
  process_node<64>(A, A.sel[q], node_lds(lds + w * node_lds_bytes(A.C.nbins, 1), A.C.nbins, 1),
                   threadIdx.x & 63);
}

// Lists the children that stay internal; they become the next level,
// numbered after every internal node so far, and are sorted into the big
// and small lists (positions into the level list).  Updates the level state
// and, for the host, a record {seq, next level size, nodes, internal nodes,
// levels}.
__global__ __launch_bounds__(kCompactThreads) void k_compact(
    const int32_t* __restrict__ cand, int32_t* __restrict__ act_next, int32_t* __restrict__ big,
    int32_t* __restrict__ small, BNode* __restrict__ nodes, LevelState* __restrict__ st,
    int32_t* __restrict__ host_out, int seq) {
  __shared__ int s_w[3][kCompactThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int active = st->active, child_base = st->child_base;
  const int n_internal = st->n_internal, levels = st->levels;
  const int tidx_base = n_internal + active;
  const int m = 2 * active;
  __syncthreads();  // every thread has read the state before thread 0 rewrites it
  int base_out = 0, base_big = 0, base_small = 0;
  for (int base = 0; base < m; base += kCompactThreads) {
    const int i = base + tid;
    const int c = i < m ? cand[i] : 0;
    const bool flag = c > 0;
    const bool isbig = c > kBigNode;
    const unsigned long long mk = __ballot(flag), mb = __ballot(isbig), ms = __ballot(flag && !isbig);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    if (lane == 0) {
      s_w[0][wave] = __popcll(mk);
      s_w[1][wave] = __popcll(mb);
      s_w[2][wave] = __popcll(ms);
    }
    __syncthreads();
    int pre[3] = {0, 0, 0}, tot[3] = {0, 0, 0};
    for (int w = 0; w < kCompactThreads / 64; ++w)
      for (int q = 0; q < 3; ++q) {
        if (w < wave) pre[q] += s_w[q][w];
        tot[q] += s_w[q][w];
      }
    if (flag) {
      const int pos = base_out + pre[0] + __popcll(mk & below);
      act_next[pos] = child_base + i;
      nodes[child_base + i].tidx = tidx_base + pos;
      if (isbig) big[base_big + pre[1] + __popcll(mb & below)] = pos;
      else small[base_small + pre[2] + __popcll(ms & below)] = pos;
    }
    base_out += tot[0];
    base_big += tot[1];
    base_small += tot[2];
    __syncthreads();
  }
  if (tid == 0) {
    LevelState n;
    n.active = base_out;
    n.n_big = base_big;
    n.n_small = base_small;
    n.child_base = child_base + m;
    n.n_internal = n_internal + active;
    n.levels = levels + (active > 0 ? 1 : 0);
    n.pad[0] = n.pad[1] = 0;
    *st = n;
    host_out[1] = n.active;
    host_out[2] = n.child_base;  // nodes so far
    host_out[3] = n.n_internal;
    host_out[4] = n.levels;
    __threadfence_system();
    __atomic_store_n(&host_out[0], seq, __ATOMIC_RELEASE);
  }
}

// First level: the root (node 0) is the only node unless it is already a leaf.
__global__ void k_level0(LevelState* st, int32_t* act, int32_t* big, int32_t* small, int n,
                         int max_leaf) {
  const bool split = n > max_leaf;
  LevelState z;
  z.active = split ? 1 : 0;
  z.n_big = split && n > kBigNode ? 1 : 0;
  z.n_small = split && n <= kBigNode ? 1 : 0;
  z.child_base = 1;
  z.n_internal = 0;
  z.levels = 0;
  z.pad[0] = z.pad[1] = 0;
  *st = z;
  act[0] = 0;
  big[0] = 0;
  small[0] = 0;
}

__device__ inline float4 f4(float x, float y, float z, float w) { return make_float4(x, y, z, w); }

// Traversal nodes (one per internal node) and leaf-ordered facets.
__global__ void k_emit(const BNode* __restrict__ nodes, int total, const int32_t* __restrict__ perm,
                       const float* __restrict__ tris, TNode* __restrict__ tn,
                       TFacet* __restrict__ tf) {
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const BNode nd = nodes[id];
  if (nd.left < 0) {
    for (int k = nd.first; k < nd.first + nd.count; ++k) {
      int f = perm[k];
      const float* v = tris + 9 * (int64_t)f;
      uint32_t tag = (uint32_t)f | (k == nd.first + nd.count - 1 ? kLastFacet : 0u);
      TFacet o;
      o.p0 = f4(v[0], v[1], v[2], __uint_as_float(tag));
      o.p1 = f4(v[3], v[4], v[5], 0.f);
      o.p2 = f4(v[6], v[7], v[8], 0.f);
      tf[k] = o;
    }
    if (id == 0) {  // the whole scene is one leaf: a root with one child
      TNode t;
      t.a = f4(nd.lo[0], nd.hi[0], nd.lo[1], nd.hi[1]);
      // an empty volume: lo = hi = +inf gives an empty slab on every axis
      t.b = f4(INFINITY, INFINITY, INFINITY, INFINITY);
      t.c = f4(nd.lo[2], nd.hi[2], INFINITY, INFINITY);
      t.d = make_int4(~0, ~0, 0, 0);
      tn[0] = t;
    }
    return;
  }
  const BNode l = nodes[nd.left], r = nodes[nd.left + 1];
  TNode t;
  t.a = f4(l.lo[0], l.hi[0], l.lo[1], l.hi[1]);
  t.b = f4(r.lo[0], r.hi[0], r.lo[1], r.hi[1]);
  t.c = f4(l.lo[2], l.hi[2], r.lo[2], r.hi[2]);
  t.d = make_int4(l.left < 0 ? ~l.first : l.tidx, r.left < 0 ? ~r.first : r.tidx, 0, 0);
  tn[nd.tidx] = t;
}

// ---------------------------------------------------------------------------
// 4-wide traversal nodes: every even-depth internal node becomes one wide
// node whose children are its grandchildren, or its children where those are
// leaves.  Stored at the node's breadth-first internal index.

__device__ inline float pow2f(int e) { return __int_as_float((e + 127) << 23); }  // e in [-126, 127]

// Per-axis exponent: smallest e with fmaf(255, 2^e, lo) >= hi, the decode
// expression of the traversal kernel.
__device__ inline int quant_exp(float lo, float hi) {
  int e = -126;
  const float ext = hi - lo;
  if (ext > 0.f) {
    int x;
    frexpf(ext / 255.f, &x);  // ext / 255 < 2^x
    e = max(-126, min(127, x - 1));
  }
  while (e < 127 && fmaf(255.f, pow2f(e), lo) < hi) ++e;
  while (e > -126 && fmaf(255.f, pow2f(e - 1), lo) >= hi) --e;
  return e;
}
// Largest q with decode(q) <= v (q in [0, 255]); decode(0) = lo <= v.
__device__ inline unsigned quant_lo(float v, float lo, float sc) {
  int q = (int)floorf((v - lo) / sc);
  q = max(0, min(255, q));
  while (q > 0 && fmaf((float)q, sc, lo) > v) --q;
  while (q < 255 && fmaf((float)(q + 1), sc, lo) <= v) ++q;
  return (unsigned)q;
}
// Smallest q with decode(q) >= v; decode(255) >= the parent's hi >= v.
__device__ inline unsigned quant_hi(float v, float lo, float sc) {
  int q = (int)ceilf((v - lo) / sc);
  q = max(0, min(255, q));
  while (q < 255 && fmaf((float)q, sc, lo) < v) ++q;
  while (q > 0 && fmaf((float)(q - 1), sc, lo) >= v) --q;
  return (unsigned)q;
}

template <int FMT>
__global__ void k_collapse(const BNode* __restrict__ nodes, int total, FNode4* __restrict__ wn) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= total) return;
  const BNode nd = nodes[id];
  const bool root_leaf = id == 0 && nd.left < 0;
  if (!root_leaf && (nd.left < 0 || (nd.depth & 1))) return;
  // gather up to four children
  BNode ch[4];
  int nc = 0;
  if (root_leaf) {
    ch[nc++] = nd;
  } else {
    for (int side = 0; side < 2; ++side) {
      const BNode c = nodes[nd.left + side];
      if (c.left < 0) {
        ch[nc++] = c;
      } else {
        ch[nc++] = nodes[c.left];
        ch[nc++] = nodes[c.left + 1];
      }
    }
  }
  int ref[4] = {0, 0, 0, 0};
  for (int c = 0; c < nc; ++c) ref[c] = ch[c].left < 0 ? ~ch[c].first : ch[c].tidx;
  const unsigned mask = (1u << nc) - 1u;
  const int slot = root_leaf ? 0 : nd.tidx;
  if (FMT == RT_NODE_F4) {
    FNode4 o;
    float v[6][4];
    for (int c = 0; c < 4; ++c)
      for (int q = 0; q < 3; ++q) {
        // unused slots: lo = hi = +inf (never entered; also masked out)
        v[2 * q][c] = c < nc ? ch[c].lo[q] : INFINITY;
        v[2 * q + 1][c] = c < nc ? ch[c].hi[q] : INFINITY;
      }
    o.lox = make_float4(v[0][0], v[0][1], v[0][2], v[0][3]);
    o.hix = make_float4(v[1][0], v[1][1], v[1][2], v[1][3]);
    o.loy = make_float4(v[2][0], v[2][1], v[2][2], v[2][3]);
    o.hiy = make_float4(v[3][0], v[3][1], v[3][2], v[3][3]);
    o.loz = make_float4(v[4][0], v[4][1], v[4][2], v[4][3]);
    o.hiz = make_float4(v[5][0], v[5][1], v[5][2], v[5][3]);
    o.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
    o.meta = make_uint4(mask, 0u, 0u, 0u);
    wn[slot] = o;
  } else {
    QNode4 o;
    int e[3];
    float sc[3];
    for (int q = 0; q < 3; ++q) {
      e[q] = quant_exp(nd.lo[q], nd.hi[q]);
      sc[q] = pow2f(e[q]);
    }
    unsigned ql[3] = {0u, 0u, 0u}, qh[3] = {0u, 0u, 0u};
    for (int c = 0; c < nc; ++c)
      for (int q = 0; q < 3; ++q) {
        ql[q] |= quant_lo(ch[c].lo[q], nd.lo[q], sc[q]) << (8 * c);
        qh[q] |= quant_hi(ch[c].hi[q], nd.lo[q], sc[q]) << (8 * c);
      }
    const unsigned meta = (unsigned)(e[0] + 127) | ((unsigned)(e[1] + 127) << 8) |
                          ((unsigned)(e[2] + 127) << 16) | (mask << 24);
    o.h = make_float4(nd.lo[0], nd.lo[1], nd.lo[2], __uint_as_float(meta));
    o.qa = make_uint4(ql[0], ql[1], ql[2], qh[0]);
    o.qb = make_uint4(qh[1], qh[2], 0u, 0u);
    o.ref = make_int4(ref[0], ref[1], ref[2], ref[3]);
    reinterpret_cast<QNode4*>(wn)[slot] = o;
  }
}

}  // namespace

#define HIPCHECK(call)                                  \
  do {                                                  \
    int _rc = check_hip((call), #call);                 \
    if (_rc != RT_OK) return _rc;                       \
  } while (0)

namespace {

// Pinned, device-mapped record the compaction kernel fills at the end of each
// level: {sequence, next level size, big nodes, small nodes}.
struct HostRecord {
  int32_t* host = nullptr;
  int32_t* dev = nullptr;
};

int host_record(HostRecord& r) {
  static thread_local HostRecord rec;
  if (!rec.host) {
    int rc = check_hip(hipHostMalloc((void**)&rec.host, 64, hipHostMallocMapped), "hipHostMalloc");
    if (rc != RT_OK) return rc;
    rc = check_hip(hipHostGetDevicePointer((void**)&rec.dev, rec.host, 0), "hipHostGetDevicePointer");
    if (rc != RT_OK) return rc;
    rec.host[0] = 0;
  }
  r = rec;
  return RT_OK;
}

// Waits until the device has written sequence number seq; falls back to a
// stream synchronisation (which reports device errors) after a while.
int wait_record(const HostRecord& r, int seq, hipStream_t s) {
  volatile int32_t* h = r.host;
  for (long spin = 0; spin < 2000000; ++spin) {
    if (__atomic_load_n(&h[0], __ATOMIC_ACQUIRE) == seq) return RT_OK;
    if (spin > 1000) __builtin_ia32_pause();
  }
  int rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc != RT_OK) return rc;
  if (__atomic_load_n(&h[0], __ATOMIC_ACQUIRE) != seq)
    return set_error(RT_EHIP, "rt_build: level record not written");
  return RT_OK;
}

}  // namespace

int build_tree(Buffers& B, const float* tris, int64_t n64, const rt_split_params& p,
               hipStream_t s, rt_bvh_info* info) {
  const int n = (int)n64;
  HostRecord rec;
  {
    int rc = host_record(rec);
    if (rc != RT_OK) return rc;
  }
  static thread_local int seq = 0;
  // counters: [0] non-finite flag, bytes 32..39 1/L^2, bytes 64..95 level state
  double* inv_l2 = reinterpret_cast<double*>(B.counters + 8);
  LevelState* st = reinterpret_cast<LevelState*>(B.counters + 16);

  HIPCHECK(hipMemsetAsync(B.counters, 0, 32 * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_root_init, dim3(1), dim3(64), 0, s, B.root_box);
  const int pb = 256;
  hipLaunchKernelGGL(k_prep, dim3((n + pb - 1) / pb), dim3(pb), 0, s, tris, n, B.recs_a, B.perm,
                     B.counters, B.root_box);
  hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, s, B.root_box, n, B.nodes, inv_l2);
  hipLaunchKernelGGL(k_level0, dim3(1), dim3(1), 0, s, st, B.act_a, B.big, B.small, n, p.max_leaf);
  HIPCHECK(hipGetLastError());

  BuildConst C;
  C.alpha = (double)p.alpha;
  C.t_isect = (double)p.t_isect;
  C.t_trav = (double)p.t_trav;
  for (int a = 0; a < 3; ++a) C.src[a] = (double)p.src[a];
  C.inv_l2 = 0.0;
  C.max_leaf = p.max_leaf;
  C.nbins = p.nbins;
  C.d_mode = p.d_mode;
  C.d_norm = p.d_norm;
  C.max_depth = p.max_depth;
  C.depth_limit = p.depth_limit;

  const size_t lds1 = node_lds_bytes(p.nbins, 1);
  const size_t lds_big = node_lds_bytes(p.nbins, bin_copies(p.nbins, kBigThreads / 64));
  const int small_groups = lds1 * 4 <= 48 * 1024 ? 4 : 2;  // node groups per small work-group
  const int big_cap = n / (kBigNode + 1);                   // nodes above kBigNode facets
  const int level_cap = n / (p.max_leaf + 1);               // internal nodes of one level
  constexpr int kBatch = 4;                                 // levels queued per host wait

  FacetRec* recs[2] = {B.recs_a, B.recs_b};
  int32_t* acts[2] = {B.act_a, B.act_b};
  int bound = n > p.max_leaf ? 1 : 0;  // upper bound on the size of the next level to run
  int level = 0;
  int total = 1, n_internal = 0, levels = 0;
  while (bound > 0) {
    for (int q = 0; q < kBatch; ++q, ++level) {
      if (level > RT_MAX_DEPTH + 1)
        return set_error(RT_EDEPTH, "rt_build: tree deeper than the depth limit");
      LevelArgs A;
      A.nodes = B.nodes;
      A.in = recs[level & 1];
      A.out = recs[(level + 1) & 1];
      A.perm = B.perm;
      A.act = acts[level & 1];
      A.cand = B.cand;
      A.inv_l2 = inv_l2;
      A.st = st;
      A.n = n;
      A.C = C;
      const int gb = std::min(bound, big_cap);
      if (gb > 0) {
        A.sel = B.big;
        hipLaunchKernelGGL(k_level_big, dim3(gb), dim3(kBigThreads), lds_big, s, A);
      }
      const int gs = (bound + small_groups - 1) / small_groups;
      A.sel = B.small;
      hipLaunchKernelGGL(k_level_small, dim3(gs), dim3(64 * small_groups), lds1 * small_groups, s, A);
      ++seq;
      hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, s, B.cand,
                         acts[(level + 1) & 1], B.big, B.small, B.nodes, st, rec.dev, seq);
      bound = std::min(2 * bound, level_cap);
    }
    HIPCHECK(hipGetLastError());
    {
      int rc = wait_record(rec, seq, s);
      if (rc != RT_OK) return rc;
    }
    bound = rec.host[1];
    total = rec.host[2];
    n_internal = rec.host[3];
    levels = rec.host[4];
  }
  const int eb = 256;
  hipLaunchKernelGGL(k_emit, dim3((total + eb - 1) / eb), dim3(eb), 0, s, B.nodes, total, B.perm,
                     tris, B.tnodes, B.tfacets);
  if (p.node_format == RT_NODE_F4)
    hipLaunchKernelGGL(k_collapse<RT_NODE_F4>, dim3((total + eb - 1) / eb), dim3(eb), 0, s,
                       B.nodes, total, B.wnodes);
  else if (p.node_format == RT_NODE_Q4)
    hipLaunchKernelGGL(k_collapse<RT_NODE_Q4>, dim3((total + eb - 1) / eb), dim3(eb), 0, s,
                       B.nodes, total, B.wnodes);
  HIPCHECK(hipGetLastError());
  int32_t nonfinite = 0;
  HIPCHECK(hipMemcpyAsync(&nonfinite, B.counters + C_NONFINITE, 4, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (nonfinite) return set_error(RT_EINVAL, "rt_build: a facet has a non-finite vertex");

  info->n_tris = n;
  info->n_nodes = total;
  info->n_internal = n_internal;
  info->n_leaves = total - n_internal;
  info->depth = levels;  // deepest leaf depth (root alone = 0)
  info->n_levels = levels;
  const int64_t node_bytes = p.node_format == RT_NODE_F4 ? sizeof(FNode4)
                             : p.node_format == RT_NODE_Q4 ? sizeof(QNode4) : sizeof(TNode);
  info->node_format = p.node_format;
  info->n_trace_nodes = std::max(n_internal, 1);
  info->trace_bytes = node_bytes * std::max(n_internal, 1) + (int64_t)sizeof(TFacet) * n;
  return RT_OK;
}

}  // namespace rt
