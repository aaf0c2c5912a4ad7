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

constexpr int kLevelThreads = 256;
constexpr int kCompactThreads = 1024;

// counters[] slots
enum { C_NONFINITE = 0, C_NEXT = 1 };

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

__device__ inline int bin_of(double c, double lo, double scale, int nb) {
  return min(nb - 1, (int)((c - lo) * scale));
}

// ---------------------------------------------------------------------------
__global__ void k_prep(const float* __restrict__ tris, int n, float4* __restrict__ flo,
                       float4* __restrict__ fhi, double* __restrict__ cen,
                       int32_t* __restrict__ refs, int32_t* __restrict__ counters,
                       long long* __restrict__ root) {
  __shared__ int s_box[6];
  __shared__ long long s_cb[6];
  if (threadIdx.x < 6) {
    s_box[threadIdx.x] = threadIdx.x < 3 ? f2o(INFINITY) : f2o(-INFINITY);
    s_cb[threadIdx.x] = threadIdx.x < 3 ? d2o(INFINITY) : d2o(-INFINITY);
  }
  __syncthreads();
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float* v = tris + 9 * (int64_t)i;
    float x[9];
    for (int k = 0; k < 9; ++k) x[k] = v[k];
    bool finite = true;
    for (int k = 0; k < 9; ++k) finite = finite && isfinite(x[k]);
    if (!finite) atomicOr(&counters[C_NONFINITE], 1);
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(fminf(x[a], x[3 + a]), x[6 + a]);
      hi[a] = fmaxf(fmaxf(x[a], x[3 + a]), x[6 + a]);
      double c = ((double)lo[a] + (double)hi[a]) * 0.5;
      cen[(int64_t)a * n + i] = c;
      atomicMin(&s_box[a], f2o(lo[a]));
      atomicMax(&s_box[3 + a], f2o(hi[a]));
      atomicMin(&s_cb[a], d2o(c));
      atomicMax(&s_cb[3 + a], d2o(c));
    }
    flo[i] = make_float4(lo[0], lo[1], lo[2], 0.f);
    fhi[i] = make_float4(hi[0], hi[1], hi[2], 0.f);
    refs[i] = i;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    atomicMin(&root[threadIdx.x], (long long)s_box[threadIdx.x]);
    atomicMax(&root[3 + threadIdx.x], (long long)s_box[3 + threadIdx.x]);
    atomicMin(&root[6 + threadIdx.x], s_cb[threadIdx.x]);
    atomicMax(&root[9 + threadIdx.x], s_cb[3 + threadIdx.x]);
  }
}

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
struct LevelArgs {
  BNode* nodes;
  const float4* flo;
  const float4* fhi;
  const double* cen;  // [3][n]
  const int32_t* refs_in;
  int32_t* refs_out;
  int32_t* perm;
  const int32_t* act;
  int32_t* cand;
  const double* inv_l2;
  int32_t child_base;
  int32_t n;
  BuildConst C;
};

__global__ __launch_bounds__(kLevelThreads) void k_level(LevelArgs A) {
  const int j = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int id = A.act[j];
  const BNode nd = A.nodes[id];
  const int k = nd.count, s = nd.first;
  const int B = A.C.nbins;
  BuildConst C = A.C;
  C.inv_l2 = *A.inv_l2;

  __shared__ int s_cnt[3][RT_MAX_BINS];
  __shared__ int s_blo[3][RT_MAX_BINS][3];
  __shared__ int s_bhi[3][RT_MAX_BINS][3];
  __shared__ double s_cost[3 * (RT_MAX_BINS - 1)];
  __shared__ int s_pick[2];  // axis, plane
  __shared__ double s_best;
  __shared__ int s_wl[kLevelThreads / 64], s_wr[kLevelThreads / 64];
  __shared__ int s_cbox[2][6];
  __shared__ long long s_ccb[2][6];

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
  for (int a = 0; a < 3; ++a) {
    ext[a] = nd.cbhi[a] - nd.cblo[a];
    scale[a] = ext[a] > 0.0 ? (double)B / ext[a] : 0.0;
  }
  if (tid < 12) {
    int side = tid / 6, c = tid % 6;
    s_cbox[side][c] = c < 3 ? f2o(INFINITY) : f2o(-INFINITY);
    s_ccb[side][c] = c < 3 ? d2o(INFINITY) : d2o(-INFINITY);
  }
  int axis = -1, plane = -1;
  double best = INFINITY;
  if (!forced) {
    for (int c = tid; c < 3 * B; c += kLevelThreads) {
      int a = c / B, b = c % B;
      s_cnt[a][b] = 0;
      for (int q = 0; q < 3; ++q) {
        s_blo[a][b][q] = f2o(INFINITY);
        s_bhi[a][b][q] = f2o(-INFINITY);
      }
    }
    __syncthreads();
    for (int i = tid; i < k; i += kLevelThreads) {
      int f = A.refs_in[s + i];
      float4 lo = A.flo[f], hi = A.fhi[f];
      for (int a = 0; a < 3; ++a) {
        if (!(ext[a] > 0.0)) continue;
        int b = bin_of(A.cen[(int64_t)a * A.n + f], nd.cblo[a], scale[a], B);
        atomicAdd(&s_cnt[a][b], 1);
        atomicMin(&s_blo[a][b][0], f2o(lo.x));
        atomicMin(&s_blo[a][b][1], f2o(lo.y));
        atomicMin(&s_blo[a][b][2], f2o(lo.z));
        atomicMax(&s_bhi[a][b][0], f2o(hi.x));
        atomicMax(&s_bhi[a][b][1], f2o(hi.y));
        atomicMax(&s_bhi[a][b][2], f2o(hi.z));
      }
    }
    __syncthreads();
    const int ncand = 3 * (B - 1);
    double clo[3], chi[3];
    for (int q = 0; q < 3; ++q) {
      clo[q] = nd.lo[q];
      chi[q] = nd.hi[q];
    }
    for (int c = tid; c < ncand; c += kLevelThreads) {
      int a = c / (B - 1), pl = c % (B - 1) + 1;
      double cost = INFINITY;
      if (ext[a] > 0.0) {
        double alo[3] = {INFINITY, INFINITY, INFINITY}, ahi[3] = {-INFINITY, -INFINITY, -INFINITY};
        double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int ka = 0, kb = 0;
        for (int b = 0; b < B; ++b) {
          int cnt = s_cnt[a][b];
          if (cnt == 0) continue;
          double* lo = b < pl ? alo : blo;
          double* hi = b < pl ? ahi : bhi;
          if (b < pl) ka += cnt; else kb += cnt;
          for (int q = 0; q < 3; ++q) {
            lo[q] = fmin(lo[q], (double)o2f(s_blo[a][b][q]));
            hi[q] = fmax(hi[q], (double)o2f(s_bhi[a][b][q]));
          }
        }
        if (ka > 0 && kb > 0) cost = eq2_cost(C, alpha, alo, ahi, ka, blo, bhi, kb, clo, chi, k);
      }
      s_cost[c] = cost;
    }
    __syncthreads();
    if (tid == 0) {
      int ba = -1, bp = -1;
      double bc = INFINITY;
      for (int c = 0; c < ncand; ++c) {
        if (s_cost[c] < bc) {
          bc = s_cost[c];
          ba = c / (B - 1);
          bp = c % (B - 1) + 1;
        }
      }
      s_pick[0] = ba;
      s_pick[1] = bp;
      s_best = bc;
    }
    __syncthreads();
    axis = s_pick[0];
    plane = s_pick[1];
    best = s_best;
    if (axis < 0) flags |= 2;
  }
  __syncthreads();
  const bool by_position = axis < 0;
  int nleft;
  if (by_position) {
    nleft = k / 2;
  } else {
    nleft = 0;
    for (int b = 0; b < plane; ++b) nleft += s_cnt[axis][b];
  }

  // stable partition with per-side bounds of the children
  float blo[2][3], bhi[2][3];
  double cblo[2][3], cbhi[2][3];
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      blo[side][q] = INFINITY;
      bhi[side][q] = -INFINITY;
      cblo[side][q] = INFINITY;
      cbhi[side][q] = -INFINITY;
    }
  int lbase = 0, rbase = 0;
  for (int base = 0; base < k; base += kLevelThreads) {
    int i = base + tid;
    bool valid = i < k;
    int f = valid ? A.refs_in[s + i] : 0;
    bool go_left = false;
    if (valid) {
      if (by_position) {
        go_left = i < nleft;
      } else {
        go_left = bin_of(A.cen[(int64_t)axis * A.n + f], nd.cblo[axis], scale[axis], B) < plane;
      }
    }
    bool go_right = valid && !go_left;
    unsigned long long ml = __ballot(go_left), mr = __ballot(go_right);
    unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int rl = __popcll(ml & below), rr = __popcll(mr & below);
    if (lane == 0) {
      s_wl[wave] = __popcll(ml);
      s_wr[wave] = __popcll(mr);
    }
    __syncthreads();
    int pl = 0, pr = 0, tl = 0, tr = 0;
    for (int w = 0; w < kLevelThreads / 64; ++w) {
      if (w < wave) {
        pl += s_wl[w];
        pr += s_wr[w];
      }
      tl += s_wl[w];
      tr += s_wr[w];
    }
    if (go_left) A.refs_out[s + lbase + pl + rl] = f;
    if (go_right) A.refs_out[s + nleft + rbase + pr + rr] = f;
    if (valid) {
      int side = go_left ? 0 : 1;
      float4 lo = A.flo[f], hi = A.fhi[f];
      float l3[3] = {lo.x, lo.y, lo.z}, h3[3] = {hi.x, hi.y, hi.z};
      for (int q = 0; q < 3; ++q) {
        double c = A.cen[(int64_t)q * A.n + f];
        if (side == 0) {
          blo[0][q] = fminf(blo[0][q], l3[q]);
          bhi[0][q] = fmaxf(bhi[0][q], h3[q]);
          cblo[0][q] = fmin(cblo[0][q], c);
          cbhi[0][q] = fmax(cbhi[0][q], c);
        } else {
          blo[1][q] = fminf(blo[1][q], l3[q]);
          bhi[1][q] = fmaxf(bhi[1][q], h3[q]);
          cblo[1][q] = fmin(cblo[1][q], c);
          cbhi[1][q] = fmax(cbhi[1][q], c);
        }
      }
    }
    lbase += tl;
    rbase += tr;
    __syncthreads();
  }
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      if (blo[side][q] <= bhi[side][q]) {
        atomicMin(&s_cbox[side][q], f2o(blo[side][q]));
        atomicMax(&s_cbox[side][3 + q], f2o(bhi[side][q]));
        atomicMin(&s_ccb[side][q], d2o(cblo[side][q]));
        atomicMax(&s_ccb[side][3 + q], d2o(cbhi[side][q]));
      }
    }
  __syncthreads();
  __threadfence_block();
  const int c0 = A.child_base + 2 * j;
  const int cnt[2] = {nleft, k - nleft};
  const int fst[2] = {s, s + nleft};
  if (tid < 2) {
    BNode ch;
    for (int q = 0; q < 3; ++q) {
      ch.lo[q] = o2f(s_cbox[tid][q]);
      ch.hi[q] = o2f(s_cbox[tid][3 + q]);
      ch.cblo[q] = o2d(s_ccb[tid][q]);
      ch.cbhi[q] = o2d(s_ccb[tid][3 + q]);
    }
    ch.left = -1;
    ch.first = fst[tid];
    ch.count = cnt[tid];
    ch.depth = nd.depth + 1;
    ch.axis = ch.plane = -1;
    ch.flags = 0;
    ch.tidx = -1;
    ch.cost = 0.0;
    A.nodes[c0 + tid] = ch;
    A.cand[2 * j + tid] = cnt[tid] > C.max_leaf ? 1 : 0;
  }
  if (tid == 2) {
    BNode* p = &A.nodes[id];
    p->left = c0;
    p->axis = axis;
    p->plane = plane;
    p->flags = flags;
    p->cost = by_position ? 0.0 : best;
  }
  // leaves are final: their references go to the output order
  for (int side = 0; side < 2; ++side) {
    if (cnt[side] > C.max_leaf) continue;
    for (int i = tid; i < cnt[side]; i += kLevelThreads)
      A.perm[fst[side] + i] = A.refs_out[fst[side] + i];
  }
}

// Lists the children that are still above the leaf threshold; they become the
// next level's work, numbered after every internal node of this level.
__global__ __launch_bounds__(kCompactThreads) void k_compact(
    const int32_t* __restrict__ cand, int m, int child_base, int tidx_base,
    int32_t* __restrict__ act_next, BNode* __restrict__ nodes, int32_t* __restrict__ counters) {
  __shared__ int s_w[kCompactThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int base_out = 0;
  for (int base = 0; base < m; base += kCompactThreads) {
    int i = base + tid;
    bool flag = i < m && cand[i] != 0;
    unsigned long long mk = __ballot(flag);
    unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int r = __popcll(mk & below);
    if (lane == 0) s_w[wave] = __popcll(mk);
    __syncthreads();
    int pre = 0, tot = 0;
    for (int w = 0; w < kCompactThreads / 64; ++w) {
      if (w < wave) pre += s_w[w];
      tot += s_w[w];
    }
    if (flag) {
      int pos = base_out + pre + r;
      act_next[pos] = child_base + i;
      nodes[child_base + i].tidx = tidx_base + pos;
    }
    base_out += tot;
    __syncthreads();
  }
  if (tid == 0) counters[C_NEXT] = base_out;
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

int halvings_host(int k, int max_leaf) {
  int need = (k + max_leaf - 1) / max_leaf;
  int l = 0;
  while ((1 << l) < need) ++l;
  return l;
}

}  // namespace

#define HIPCHECK(call)                                  \
  do {                                                  \
    int _rc = check_hip((call), #call);                 \
    if (_rc != RT_OK) return _rc;                       \
  } while (0)

int build_tree(Buffers& B, const float* tris, int64_t n64, const rt_split_params& p,
               hipStream_t s, rt_bvh_info* info) {
  const int n = (int)n64;
  static thread_local int32_t* host_ctr = nullptr;
  if (!host_ctr) HIPCHECK(hipHostMalloc((void**)&host_ctr, 64, hipHostMallocDefault));

  HIPCHECK(hipMemsetAsync(B.counters, 0, 64, s));
  hipLaunchKernelGGL(k_root_init, dim3(1), dim3(64), 0, s, B.root_box);
  const int pb = 256;
  hipLaunchKernelGGL(k_prep, dim3((n + pb - 1) / pb), dim3(pb), 0, s, tris, n, B.flo, B.fhi,
                     B.cen, B.refs_a, B.counters, B.root_box);
  double* inv_l2 = reinterpret_cast<double*>(B.counters + 8);
  hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, s, B.root_box, n, B.nodes, inv_l2);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(host_ctr, B.counters, 16, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  if (host_ctr[C_NONFINITE]) return set_error(RT_EINVAL, "rt_build: a facet has a non-finite vertex");

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

  int total = 1;        // nodes so far
  int n_internal = 0;   // internal nodes so far
  int levels = 0;
  int32_t* refs_in = B.refs_a;
  int32_t* refs_out = B.refs_b;
  int32_t* act = B.act_a;
  int32_t* act_next = B.act_b;
  int active = 0;
  if (n > p.max_leaf) {
    HIPCHECK(hipMemsetAsync(act, 0, sizeof(int32_t), s));  // level 0 = the root, node 0
    active = 1;
  } else {
    HIPCHECK(hipMemcpyAsync(B.perm, refs_in, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
  }
  int depth = 0;
  while (active > 0) {
    LevelArgs A;
    A.nodes = B.nodes;
    A.flo = B.flo;
    A.fhi = B.fhi;
    A.cen = B.cen;
    A.refs_in = refs_in;
    A.refs_out = refs_out;
    A.perm = B.perm;
    A.act = act;
    A.cand = B.cand;
    A.inv_l2 = inv_l2;
    A.child_base = total;
    A.n = n;
    A.C = C;
    hipLaunchKernelGGL(k_level, dim3(active), dim3(kLevelThreads), 0, s, A);
    n_internal += active;
    hipLaunchKernelGGL(k_compact, dim3(1), dim3(kCompactThreads), 0, s, B.cand, 2 * active,
                       total, n_internal, act_next, B.nodes, B.counters);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipMemcpyAsync(host_ctr, B.counters, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    total += 2 * active;
    active = host_ctr[C_NEXT];
    std::swap(refs_in, refs_out);
    std::swap(act, act_next);
    ++levels;
    ++depth;
    if (depth > RT_MAX_DEPTH + 1)
      return set_error(RT_EDEPTH, "rt_build: tree deeper than the depth limit");
  }
  const int eb = 256;
  hipLaunchKernelGGL(k_emit, dim3((total + eb - 1) / eb), dim3(eb), 0, s, B.nodes, total, B.perm,
                     tris, B.tnodes, B.tfacets);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));

  info->n_tris = n;
  info->n_nodes = total;
  info->n_internal = n_internal;
  info->n_leaves = total - n_internal;
  info->depth = levels;  // deepest leaf depth (root alone = 0)
  info->n_levels = levels;
  info->trace_bytes = (int64_t)sizeof(TNode) * std::max(n_internal, 1) + (int64_t)sizeof(TFacet) * n;
  (void)halvings_host;
  return RT_OK;
}

}  // namespace rt
