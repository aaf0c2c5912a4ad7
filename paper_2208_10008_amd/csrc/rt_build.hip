// GPU tree build (Sec. II-C) with the Eq. (2) split cost (Sec. II-B).
//
// Every internal node is split the same way: bin its facets' centroids on the
// three axes, evaluate Eq. (2) on every bin boundary, take the cheapest one
// (ties: lower axis, then lower boundary) and partition the facet references
// stably into the two children.  Three schedules apply that step, by node size:
//   big nodes     (> kBigNode facets) one pass per tree level; each node is cut
//                 into chunks of kChunk facets that separate work-groups bin
//                 (k_a_bin) and then partition (k_a_split)
//   medium nodes  (> kRegNode facets) one wave per node, one pass per level (k_m)
//   subtrees      one wave finishes a whole subtree (k_s); at or below kRegNode
//                 facets the facet records stay in the wave's registers, one
//                 per lane, and the wave walks the subtree depth-first
// A fixed number of passes is queued for each schedule; whatever is left over
// moves on to the next schedule, which handles nodes of any size.  Node ids
// follow from the split positions (no counter), pending nodes are filed by
// their first facet, a final pass compacts the ids, and the host reads a
// single record at the end.
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
#include <cstring>
#include <string>
#include <vector>

#include "rt_build_plan.h"
#include "rt_internal.h"

namespace rt {
namespace {

struct BuildConst {
  double alpha, t_isect, t_trav, src[3];
  double inv_l2;
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

// centroid of a facet = centre of its box, in float64
__device__ inline double centroid(float lo, float hi) { return ((double)lo + (double)hi) * 0.5; }

// bin of a centroid; the clamp at 0 only matters for values outside the node
__device__ inline int bin_of(double c, double lo, double scale, int nb) {
  return max(0, min(nb - 1, (int)((c - lo) * scale)));
}

// ---------------------------------------------------------------------------
// wave-wide helpers (64 lanes)
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
__device__ inline int wsum(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline unsigned long long lanes_below() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}
// lanes of one wave see each other's LDS writes after this
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// the wave's own global stores are visible to its later loads after this
__device__ inline void wave_global_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}
__device__ inline int bcast(int v) { return __shfl(v, 0); }

// ---------------------------------------------------------------------------
// Bins of one node: per axis a and bin b (slot a B + b) a facet count, the
// union of the facets' boxes (ordered ints: lo xyz, hi xyz) and, where the
// children's centroid bounds come from the bins, the centroid bounds
// (ordered int64: lo xyz, hi xyz).
struct Bins {
  int* cnt;
  int* box;
  long long* cb;  // null when not kept
};
__device__ inline Bins bins_at(char* base, int B, bool with_cb) {
  Bins b;
  b.cnt = (int*)base;
  b.box = (int*)(base + align8(sizeof(int) * 3 * B));
  b.cb = with_cb ? (long long*)(base + align8(sizeof(int) * 3 * B) + align8(sizeof(int) * 3 * B * 6))
                 : nullptr;
  return b;
}
__device__ inline void bins_clear(const Bins& S, int B, int t, int nt) {
  for (int c = t; c < 3 * B; c += nt) {
    S.cnt[c] = 0;
    for (int q = 0; q < 3; ++q) {
      S.box[6 * c + q] = f2o(INFINITY);
      S.box[6 * c + 3 + q] = f2o(-INFINITY);
      if (S.cb) {
        S.cb[6 * c + q] = d2o(INFINITY);
        S.cb[6 * c + 3 + q] = d2o(-INFINITY);
      }
    }
  }
}

// Node constants of one split.
struct NodeSetup {
  double alpha;
  int flags;       // 1 forced halving, 4 alpha taken as 1 (2 added when no plane separates)
  bool forced;
  bool axis_ok[3]; // nonzero centroid extent
  double scale[3]; // B / extent
};
__device__ inline NodeSetup node_setup(const BuildConst& C, int depth, int k, const double cblo[3],
                                       const double cbhi[3]) {
  NodeSetup u;
  u.alpha = C.alpha;
  u.flags = 0;
  u.forced = depth + halvings(k, C.max_leaf) >= C.depth_limit;
  if (u.forced) {
    u.flags = 1;
  } else if (depth >= C.max_depth) {
    u.alpha = 1.0;
    u.flags = 4;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ext = cbhi[a] - cblo[a];
    u.axis_ok[a] = ext > 0.0;
    u.scale[a] = ext > 0.0 ? (double)C.nbins / ext : 0.0;
  }
  return u;
}

// Eq. (2) on every bin boundary of one node, any bin count: each lane holds
// one bin; segmented prefix and suffix scans (lane shuffles) give the two
// sides of every boundary.
__device__ void wave_eval_any(const int* cnt, const int* box, const BuildConst& C, const NodeSetup& u,
                          const double clo[3], const double chi[3], int k, int& axis_out,
                          int& plane_out, double& best_out) {
  const int B = C.nbins;
  const int lane = lane_id();
  double bc = INFINITY;
  int bi = 1 << 30;
  const bool packed = 3 * B <= 64;
  const int passes = packed ? 1 : 3;
  for (int pass = 0; pass < passes; ++pass) {
    const int a = packed ? lane / B : pass;
    const int b = packed ? lane - a * B : lane;
    const bool valid = packed ? lane < 3 * B : lane < B;
    int c = 0;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (valid) {
      const int slot = a * B + b;
      c = cnt[slot];
      if (c > 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          lo[q] = o2f(box[6 * slot + q]);
          hi[q] = o2f(box[6 * slot + 3 + q]);
        }
      }
    }
    int pc = c, sc = c;
    float pl[3], ph[3], sl[3], sh[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      pl[q] = sl[q] = lo[q];
      ph[q] = sh[q] = hi[q];
    }
    for (int o = 1; o < B; o <<= 1) {
      const int tc = __shfl_up(pc, o);
      const int uc = __shfl_down(sc, o);
      float tl[3], th[3], ul[3], uh[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        tl[q] = __shfl_up(pl[q], o);
        th[q] = __shfl_up(ph[q], o);
        ul[q] = __shfl_down(sl[q], o);
        uh[q] = __shfl_down(sh[q], o);
      }
      if (b >= o) {
        pc += tc;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          pl[q] = fminf(pl[q], tl[q]);
          ph[q] = fmaxf(ph[q], th[q]);
        }
      }
      if (b + o < B) {
        sc += uc;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          sl[q] = fminf(sl[q], ul[q]);
          sh[q] = fmaxf(sh[q], uh[q]);
        }
      }
    }
    // boundary after bin b: bins [0, b] on the left, the suffix from bin b + 1 on the right
    const int rc = __shfl_down(sc, 1);
    float rl[3], rh[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      rl[q] = __shfl_down(sl[q], 1);
      rh[q] = __shfl_down(sh[q], 1);
    }
    const bool aok = a == 0 ? u.axis_ok[0] : (a == 1 ? u.axis_ok[1] : u.axis_ok[2]);
    if (valid && b <= B - 2 && aok && pc > 0 && rc > 0) {
      const double alo[3] = {pl[0], pl[1], pl[2]}, ahi[3] = {ph[0], ph[1], ph[2]};
      const double blo[3] = {rl[0], rl[1], rl[2]}, bhi[3] = {rh[0], rh[1], rh[2]};
      const double cost = eq2_cost(C, u.alpha, alo, ahi, pc, blo, bhi, rc, clo, chi, k);
      if (cost < bc) {  // passes visit increasing indices
        bc = cost;
        bi = a * (B - 1) + b;
      }
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
  const bool ok = bc < INFINITY;
  axis_out = ok ? bi / (B - 1) : -1;
  plane_out = ok ? bi % (B - 1) + 1 : -1;
  best_out = bc;
}

// Cross-lane moves inside 16-lane rows (DPP).  A lane whose source lies
// outside its row keeps `identity`.
constexpr int kRowShl = 0x100, kRowShr = 0x110;
template <int CTRL>
__device__ inline int dpp_i(int identity, int v) {
  return __builtin_amdgcn_update_dpp(identity, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline float dpp_f(float identity, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(identity), __float_as_int(v), CTRL,
                                                    0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp_d(double identity, double v) {
  const long long iv = __double_as_longlong(v), ii = __double_as_longlong(identity);
  const int lo = __builtin_amdgcn_update_dpp((int)ii, (int)iv, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(ii >> 32), (int)(iv >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave-wide min / max: DPP inside each 16-lane row, then the four row results.
constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kRowHalfMirror = 0x141, kRowMirror = 0x140;
__device__ inline float rmin(float v) {
  v = fminf(v, dpp_f<kQuadXor1>(v, v));
  v = fminf(v, dpp_f<kQuadXor2>(v, v));
  v = fminf(v, dpp_f<kRowHalfMirror>(v, v));
  v = fminf(v, dpp_f<kRowMirror>(v, v));
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return fminf(fminf(a, b), fminf(c, d));
}
__device__ inline float rmax(float v) { return -rmin(-v); }
__device__ inline double rlane(double v, int l) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double rmin(double v) {
  v = fmin(v, dpp_d<kQuadXor1>(v, v));
  v = fmin(v, dpp_d<kQuadXor2>(v, v));
  v = fmin(v, dpp_d<kRowHalfMirror>(v, v));
  v = fmin(v, dpp_d<kRowMirror>(v, v));
  return fmin(fmin(rlane(v, 0), rlane(v, 16)), fmin(rlane(v, 32), rlane(v, 48)));
}
__device__ inline double rmax(double v) { return -rmin(-v); }

// one step of the inclusive row scans: prefix from lower lanes, suffix from higher
template <int K>
__device__ inline void scan_step(int& pc, float pl[3], float ph[3], int& sc, float sl[3], float sh[3]) {
  pc += dpp_i<kRowShr | K>(0, pc);
  sc += dpp_i<kRowShl | K>(0, sc);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    pl[q] = fminf(pl[q], dpp_f<kRowShr | K>(INFINITY, pl[q]));
    ph[q] = fmaxf(ph[q], dpp_f<kRowShr | K>(-INFINITY, ph[q]));
    sl[q] = fminf(sl[q], dpp_f<kRowShl | K>(INFINITY, sl[q]));
    sh[q] = fmaxf(sh[q], dpp_f<kRowShl | K>(-INFINITY, sh[q]));
  }
}
template <int K>
__device__ inline void argmin_step(double& bc, int& bi) {
  const double oc = dpp_d<kRowShr | K>(INFINITY, bc);
  const int oi = dpp_i<kRowShr | K>(1 << 30, bi);
  if (oc < bc || (oc == bc && oi < bi)) {
    bc = oc;
    bi = oi;
  }
}

// Eq. (2) on every bin boundary with 16 bins: lane 16 a + b holds bin b of
// axis a (count c and box lo/hi; lanes 48..63 empty).  Row scans give each
// boundary's two sides; the first strict minimum in (axis, boundary) order
// wins, axis -1 when no boundary leaves facets on both sides.
__device__ void eval16(int c, const float lo[3], const float hi[3], const BuildConst& C,
                       const NodeSetup& u, const double clo[3], const double chi[3], int k,
                       int& axis_out, int& plane_out, double& best_out) {
  const int lane = lane_id();
  const int a = lane >> 4, b = lane & 15;
  int pc = c, sc = c;
  float pl[3], ph[3], sl[3], sh[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    pl[q] = sl[q] = lo[q];
    ph[q] = sh[q] = hi[q];
  }
  scan_step<1>(pc, pl, ph, sc, sl, sh);
  scan_step<2>(pc, pl, ph, sc, sl, sh);
  scan_step<4>(pc, pl, ph, sc, sl, sh);
  scan_step<8>(pc, pl, ph, sc, sl, sh);
  // boundary after bin b: prefix [0, b] on the left, suffix from b + 1 on the right
  const int rc = dpp_i<kRowShl | 1>(0, sc);
  float rl[3], rh[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    rl[q] = dpp_f<kRowShl | 1>(INFINITY, sl[q]);
    rh[q] = dpp_f<kRowShl | 1>(-INFINITY, sh[q]);
  }
  double bc = INFINITY;
  int bi = 1 << 30;
  const bool aok = a == 0 ? u.axis_ok[0] : (a == 1 ? u.axis_ok[1] : (a == 2 && u.axis_ok[2]));
  if (aok && b <= 14 && pc > 0 && rc > 0) {
    const double alo[3] = {pl[0], pl[1], pl[2]}, ahi[3] = {ph[0], ph[1], ph[2]};
    const double blo[3] = {rl[0], rl[1], rl[2]}, bhi[3] = {rh[0], rh[1], rh[2]};
    bc = eq2_cost(C, u.alpha, alo, ahi, pc, blo, bhi, rc, clo, chi, k);
    bi = a * 15 + b;
  }
  argmin_step<1>(bc, bi);
  argmin_step<2>(bc, bi);
  argmin_step<4>(bc, bi);
  argmin_step<8>(bc, bi);
  // the last lane of each row holds the row's minimum
  double best = INFINITY;
  int bidx = 1 << 30;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const long long bits = __double_as_longlong(bc);
    const int lo32 = __builtin_amdgcn_readlane((int)bits, 16 * r + 15);
    const int hi32 = __builtin_amdgcn_readlane((int)(bits >> 32), 16 * r + 15);
    const double rcst = __longlong_as_double(((long long)hi32 << 32) | (unsigned)lo32);
    const int ridx = __builtin_amdgcn_readlane(bi, 16 * r + 15);
    if (rcst < best || (rcst == best && ridx < bidx)) {
      best = rcst;
      bidx = ridx;
    }
  }
  const bool ok = best < INFINITY;
  axis_out = ok ? bidx / 15 : -1;
  plane_out = ok ? bidx % 15 + 1 : -1;
  best_out = best;
}

// Eq. (2) on every bin boundary of one node's bins (LDS); all 64 lanes of the
// wave call it and get the same answer.
__device__ void wave_eval(const int* cnt, const int* box, const BuildConst& C, const NodeSetup& u,
                          const double clo[3], const double chi[3], int k, int& axis_out,
                          int& plane_out, double& best_out) {
  if (C.nbins != 16) {
    wave_eval_any(cnt, box, C, u, clo, chi, k, axis_out, plane_out, best_out);
    return;
  }
  const int lane = lane_id();
  int c = 0;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  if (lane < 48) {
    c = cnt[lane];
    if (c > 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        lo[q] = o2f(box[6 * lane + q]);
        hi[q] = o2f(box[6 * lane + 3 + q]);
      }
    }
  }
  eval16(c, lo, hi, C, u, clo, chi, k, axis_out, plane_out, best_out);
}

// Union of the bins [b0, b1) of one axis: child volume and centroid bounds.
__device__ inline void bins_union(const Bins& S, int B, int axis, int b0, int b1, float lo[3],
                                  float hi[3], double clo[3], double chi[3]) {
  int bl[6] = {f2o(INFINITY), f2o(INFINITY), f2o(INFINITY), f2o(-INFINITY), f2o(-INFINITY), f2o(-INFINITY)};
  long long cl[6] = {d2o(INFINITY), d2o(INFINITY), d2o(INFINITY), d2o(-INFINITY), d2o(-INFINITY), d2o(-INFINITY)};
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
    lo[q] = o2f(bl[q]);
    hi[q] = o2f(bl[3 + q]);
    clo[q] = o2d(cl[q]);
    chi[q] = o2d(cl[3 + q]);
  }
}

// ---------------------------------------------------------------------------
// Where a new internal node goes next.
enum { TO_A = 0, TO_M = 1, TO_S = 2 };
__device__ inline int classify(const BuildConst& C, int k, int depth, const double cblo[3],
                               const double cbhi[3], bool a_ok, bool m_ok) {
  const bool forced = depth + halvings(k, C.max_leaf) >= C.depth_limit;
  const bool ext = cbhi[0] > cblo[0] || cbhi[1] > cblo[1] || cbhi[2] > cblo[2];
  if (a_ok && k > kBigNode && !forced && ext) return TO_A;
  if (m_ok && k > kRegNode) return TO_M;
  return TO_S;
}

struct Ctx {
  BNode* nodes;
  FacetRec* recs[2];  // by node depth parity
  int32_t* perm;
  BuildState* st;
  int32_t* used;
  int32_t* mfront[2];
  int32_t* sfront;
  AItem* items[2];
  int32_t* ccnt[2];
  char* abins[2];
  size_t abin_stride;  // bytes of one bin set; a node slot holds kBinReplicas of them
  int n, item_cap, anode_cap;
  int la, lm;  // queued big-node levels and medium-node passes
  BuildConst C;
};

__device__ inline void set_err(BuildState* st, int bit) { atomicOr(&st->error, bit); }

// Chunk items queued so far on big-node level `lvl`.
__device__ inline int level_items(const Ctx& X, int lvl) {
  return (int)(unsigned)X.st->a_pack[lvl];
}
// Takes bin slots for `nodes` big nodes of level `lvl` and `items` chunk
// items with one atomic add.  Returns false (and flags the error) when the
// capacities are exceeded.
__device__ inline bool take_big(const Ctx& X, int lvl, int nodes, int items, int& slot, int& base) {
  const unsigned long long old =
      atomicAdd(&X.st->a_pack[lvl], ((unsigned long long)nodes << 32) | (unsigned)items);
  slot = (int)(old >> 32);
  base = (int)(unsigned)old;
  if (slot + nodes > X.anode_cap || base + items > X.item_cap) {
    set_err(X.st, 1);
    return false;
  }
  return true;
}
// Chunk item j (of nit) of big node `id` (k facets) at list index base + j.
__device__ inline void write_item(const Ctx& X, int lvl, int id, int k, int slot, int base, int nit,
                                  int j) {
  AItem a;
  a.node = id;
  a.slot = slot;
  a.begin = j * kChunk;
  a.end = min(k, (j + 1) * kChunk);
  a.first_item = base;
  a.n_items = nit;
  a.pad[0] = a.pad[1] = 0;
  X.items[lvl & 1][base + j] = a;
}
__device__ inline char* node_bins(const Ctx& X, int lvl, int slot, int rep) {
  return X.abins[lvl & 1] + ((size_t)slot * kBinReplicas + rep) * X.abin_stride;
}
__device__ inline void clear_node_bins(const Ctx& X, int lvl, int slot, int t, int nt) {
  for (int r = 0; r < kBinReplicas; ++r)
    bins_clear(bins_at(node_bins(X, lvl, slot, r), X.C.nbins, true), X.C.nbins, t, nt);
}
// Medium nodes and subtree roots are filed under their first facet: no two
// pending nodes share one, so no counter is needed.
__device__ inline void push_m(const Ctx& X, int pass, int id, int first) {
  X.mfront[pass & 1][first] = id;
}
__device__ inline void push_s(const Ctx& X, int id, int first) { X.sfront[first] = id; }

// Writes the two children of `id` and the parent's split.  The children's ids
// come from the split boundary b (the left child's last facet): 2b + 1 and
// 2b + 2.  Distinct internal nodes have distinct boundaries, so ids never
// collide.  Returns the left child id.
__device__ int make_children(const Ctx& X, int id, const BNode& nd, int axis, int plane, int flags,
                             double cost, int nleft, const float lo[2][3], const float hi[2][3],
                             const double clo[2][3], const double chi[2][3]) {
  const int b = nd.first + nleft - 1;
  const int c0 = 2 * b + 1;
  if (nleft < 1 || nleft >= nd.count || b < 0 || b + 1 >= X.n) {  // both sides are never empty
    set_err(X.st, 8);
    return c0;
  }
  for (int side = 0; side < 2; ++side) {
    BNode ch;
    for (int q = 0; q < 3; ++q) {
      ch.lo[q] = lo[side][q];
      ch.hi[q] = hi[side][q];
      ch.cblo[q] = clo[side][q];
      ch.cbhi[q] = chi[side][q];
    }
    ch.left = -1;
    ch.first = side == 0 ? nd.first : nd.first + nleft;
    ch.count = side == 0 ? nleft : nd.count - nleft;
    ch.depth = nd.depth + 1;
    ch.axis = ch.plane = -1;
    ch.flags = 0;
    ch.tidx = -1;
    ch.cost = 0.0;
    X.nodes[c0 + side] = ch;
  }
  BNode* p = &X.nodes[id];
  p->left = c0;
  p->axis = axis;
  p->plane = plane;
  p->flags = flags;
  p->cost = cost;
  X.used[b] = nd.depth + 1;
  return c0;
}

// ---------------------------------------------------------------------------
__global__ void k_init(int32_t* words, long long* root, int n) {
  for (int i = threadIdx.x; i < kStateWords; i += blockDim.x) words[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) reinterpret_cast<BuildState*>(words)->n = n;
  if (threadIdx.x < 3) {
    const int t = threadIdx.x;
    root[t] = f2o(INFINITY);
    root[3 + t] = f2o(-INFINITY);
    root[6 + t] = d2o(INFINITY);
    root[9 + t] = d2o(-INFINITY);
  }
}

// Root node from the reduced bounds; queues it for the first schedule that
// takes it (nothing when it is a leaf or a facet is not finite).  Every
// thread of one work-group; the bounds and the non-finite flag were reduced
// by atomics of the whole grid, so they are read at device scope.
__device__ inline long long ld_dev(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ void setup_root(const Ctx& X, const long long* root) {
  __shared__ int s_slot, s_base;
  if (threadIdx.x == 0) s_slot = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
  BNode r;
  for (int a = 0; a < 3; ++a) {
    r.lo[a] = o2f((int32_t)ld_dev(&root[a]));
    r.hi[a] = o2f((int32_t)ld_dev(&root[3 + a]));
    r.cblo[a] = o2d(ld_dev(&root[6 + a]));
    r.cbhi[a] = o2d(ld_dev(&root[9 + a]));
  }
  r.left = -1;
  r.first = 0;
  r.count = X.n;
  r.depth = 0;
  r.axis = r.plane = -1;
  r.flags = 0;
  r.tidx = -1;
  r.cost = 0.0;
  X.nodes[0] = r;
  double ex = (double)r.hi[0] - (double)r.lo[0];
  double ey = (double)r.hi[1] - (double)r.lo[1];
  double ez = (double)r.hi[2] - (double)r.lo[2];
  double l2 = (ex * ex + ey * ey) + ez * ez;
  X.st->inv_l2 = l2 > 0.0 ? 1.0 / l2 : 0.0;
  const int nonfinite = __hip_atomic_load(&X.st->nonfinite, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (nonfinite == 0 && X.n > X.C.max_leaf) {
    const int to = classify(X.C, X.n, 0, r.cblo, r.cbhi, X.la > 0, X.lm > 0);
    if (to == TO_A) {
      int slot, base;
      if (take_big(X, 0, 1, (X.n + kChunk - 1) / kChunk, slot, base)) {
        s_slot = slot;
        s_base = base;
      }
    }
    else if (to == TO_M) push_m(X, 0, 0, 0);
    else push_s(X, 0, 0);
  }
  }
  __syncthreads();
  if (s_slot >= 0) {
    const int nit = (X.n + kChunk - 1) / kChunk;
    for (int j = threadIdx.x; j < nit; j += blockDim.x) write_item(X, 0, 0, X.n, s_slot, s_base, nit, j);
    clear_node_bins(X, 0, s_slot, threadIdx.x, blockDim.x);
  }
}

// Facet records, root bounds (ordered-int atomics), and the scratch the
// later passes expect; the last work-group to finish sets up the root.
__global__ __launch_bounds__(256) void k_prep(Ctx X, const float* __restrict__ tris,
                                              long long* __restrict__ root) {
  const int n = X.n;
  FacetRec* __restrict__ recs = X.recs[0];
  int32_t* __restrict__ perm = X.perm;
  BuildState* st = X.st;
  int32_t* __restrict__ used = X.used;
  int32_t* __restrict__ mfront = X.mfront[0];
  int32_t* __restrict__ sfront = X.sfront;
  if (blockIdx.x == 0 && threadIdx.x == 0) st->n = n;
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
    if (!finite) atomicOr(&st->nonfinite, 1);
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
    used[i] = 0;
    mfront[i] = -1;
    mfront[n + i] = -1;
    sfront[i] = -1;
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
  // the last work-group to get here sees every other one's root bounds
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    s_last = atomicAdd(&st->prep_done, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  setup_root(X, root);
}


// ---------------------------------------------------------------------------
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
__device__ inline void run_add(Run& r, const float4& lo, const float4& hi, const double cu[3]) {
  r.count += 1;
  r.lo[0] = fminf(r.lo[0], lo.x); r.lo[1] = fminf(r.lo[1], lo.y); r.lo[2] = fminf(r.lo[2], lo.z);
  r.hi[0] = fmaxf(r.hi[0], hi.x); r.hi[1] = fmaxf(r.hi[1], hi.y); r.hi[2] = fmaxf(r.hi[2], hi.z);
  r.clo[0] = fmin(r.clo[0], cu[0]); r.clo[1] = fmin(r.clo[1], cu[1]); r.clo[2] = fmin(r.clo[2], cu[2]);
  r.chi[0] = fmax(r.chi[0], cu[0]); r.chi[1] = fmax(r.chi[1], cu[1]); r.chi[2] = fmax(r.chi[2], cu[2]);
}
__device__ inline void run_flush(const Run& r, const Bins& S, int a, int B) {
  if (r.count == 0) return;
  const int slot = a * B + r.bin;
  atomicAdd(&S.cnt[slot], r.count);
  for (int q = 0; q < 3; ++q) {
    atomicMin(&S.box[6 * slot + q], f2o(r.lo[q]));
    atomicMax(&S.box[6 * slot + 3 + q], f2o(r.hi[q]));
    atomicMin(&S.cb[6 * slot + q], d2o(r.clo[q]));
    atomicMax(&S.cb[6 * slot + 3 + q], d2o(r.chi[q]));
  }
}

// Big nodes, pass 1: one work-group bins one chunk into LDS (one bin copy per
// wave while they fit) and stores the chunk's bins.
constexpr int kAThreads = 256;     // threads of a chunk's split work-group
constexpr int kABinThreads = 128;  // threads of a chunk's binning work-group (4 facets each)
__host__ __device__ inline int a_copies(int B, int threads) {
  const int fit = (int)((40 * 1024) / bins_bytes(B, true));
  return fit < 1 ? 1 : (fit < threads / 64 ? fit : threads / 64);
}

__global__ __launch_bounds__(kABinThreads) void k_a_bin(Ctx X, int lvl) {
  extern __shared__ __align__(16) char lds[];
  const int active = min(level_items(X, lvl), X.item_cap);
  if ((int)blockIdx.x >= active) return;
  {
    // the next level's bins (at most two big children per big node here),
    // cleared by this level's work-groups in turn: nothing reads or adds to
    // them before the next level's binning
    const int next_slots = min(X.anode_cap, 2 * (int)(X.st->a_pack[lvl] >> 32));
    for (int pr = blockIdx.x; pr < next_slots * kBinReplicas; pr += active)
      bins_clear(bins_at(node_bins(X, lvl + 1, pr / kBinReplicas, pr % kBinReplicas), X.C.nbins, true),
                 X.C.nbins, threadIdx.x, kABinThreads);
  }
  const int par = lvl & 1;
  const AItem it = X.items[par][blockIdx.x];
  const BNode nd = X.nodes[it.node];
  const int B = X.C.nbins;
  const int ncopy = a_copies(B, kABinThreads);
  const size_t cs = bins_bytes(B, true);
  const int tid = threadIdx.x;
  for (int cp = 0; cp < ncopy; ++cp) bins_clear(bins_at(lds + cp * cs, B, true), B, tid, kABinThreads);
  __syncthreads();
  const NodeSetup u = node_setup(X.C, nd.depth, nd.count, nd.cblo, nd.cbhi);
  const Bins S = bins_at(lds + ((tid >> 6) % ncopy) * cs, B, true);
  const FacetRec* in = X.recs[nd.depth & 1] + nd.first;
  // each thread walks a contiguous run of the chunk; consecutive facets that
  // share a bin are merged in registers before they reach LDS
  constexpr int kPer = kChunk / kABinThreads;
  const int i0 = it.begin + tid * kPer;
  FacetRec rr[kPer];
#pragma unroll
  for (int v = 0; v < kPer; ++v) rr[v] = in[min(i0 + v, it.end - 1)];
  Run run[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) run_reset(run[a], -1);
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    if (i0 + v >= it.end) break;
    const float4 lo = rr[v].lo, hi = rr[v].hi;
    const double cu[3] = {centroid(lo.x, hi.x), centroid(lo.y, hi.y), centroid(lo.z, hi.z)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!u.axis_ok[a]) continue;
      const int b = bin_of(cu[a], nd.cblo[a], u.scale[a], B);
      if (b != run[a].bin) {
        run_flush(run[a], S, a, B);
        run_reset(run[a], b);
      }
      run_add(run[a], lo, hi, cu);
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) run_flush(run[a], S, a, B);
  __syncthreads();
  // this chunk's counts, and its bins added to one replica of the node's bins
  const Bins G = bins_at(node_bins(X, lvl, it.slot, blockIdx.x % kBinReplicas), B, true);
  int32_t* cc = X.ccnt[par] + (size_t)blockIdx.x * 3 * RT_MAX_BINS;
  for (int c = tid; c < 3 * B; c += kABinThreads) {
    int cnt = 0;
    int bx[6] = {f2o(INFINITY), f2o(INFINITY), f2o(INFINITY), f2o(-INFINITY), f2o(-INFINITY), f2o(-INFINITY)};
    long long cb[6] = {d2o(INFINITY), d2o(INFINITY), d2o(INFINITY), d2o(-INFINITY), d2o(-INFINITY), d2o(-INFINITY)};
    for (int cp = 0; cp < ncopy; ++cp) {
      const Bins P = bins_at(lds + cp * cs, B, true);
      cnt += P.cnt[c];
      for (int q = 0; q < 3; ++q) {
        bx[q] = min(bx[q], P.box[6 * c + q]);
        bx[3 + q] = max(bx[3 + q], P.box[6 * c + 3 + q]);
        cb[q] = min(cb[q], P.cb[6 * c + q]);
        cb[3 + q] = max(cb[3 + q], P.cb[6 * c + 3 + q]);
      }
    }
    cc[c] = cnt;
    if (cnt > 0) {
      atomicAdd(&G.cnt[c], cnt);
      for (int q = 0; q < 3; ++q) {
        atomicMin(&G.box[6 * c + q], bx[q]);
        atomicMax(&G.box[6 * c + 3 + q], bx[3 + q]);
        atomicMin(&G.cb[6 * c + q], cb[q]);
        atomicMax(&G.cb[6 * c + 3 + q], cb[3 + q]);
      }
    }
  }
}

// Big nodes, pass 2: every work-group of a node folds the node's chunk bins
// and evaluates Eq. (2) on them (the same answer in each), places its chunk
// stably after the left-going facets of the chunks before it, and the node's
// first chunk writes the children and queues them.
__global__ __launch_bounds__(kAThreads) void k_a_split(Ctx X, int lvl) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_pick[2];
  __shared__ double s_best;
  __shared__ int s_red[kAThreads / 64];
  __shared__ int s_w[2][kAThreads / 64];
  if ((int)blockIdx.x >= min(level_items(X, lvl), X.item_cap)) return;
  const int par = lvl & 1;
  const AItem it = X.items[par][blockIdx.x];
  const BNode nd = X.nodes[it.node];
  const int B = X.C.nbins;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  BuildConst C = X.C;
  C.inv_l2 = X.st->inv_l2;
  const Bins S = bins_at(lds, B, true);
  // fold the replicas of the node's bins
  {
    Bins R[kBinReplicas];
#pragma unroll
    for (int r = 0; r < kBinReplicas; ++r) R[r] = bins_at(node_bins(X, lvl, it.slot, r), B, true);
    for (int c = tid; c < 3 * B; c += kAThreads) {
      int cnt = 0;
#pragma unroll
      for (int r = 0; r < kBinReplicas; ++r) cnt += R[r].cnt[c];
      S.cnt[c] = cnt;
    }
    for (int e = tid; e < 3 * B * 6; e += kAThreads) {
      const bool lo = e % 6 < 3;
      int bx = R[0].box[e];
      long long cb = R[0].cb[e];
#pragma unroll
      for (int r = 1; r < kBinReplicas; ++r) {
        const int x = R[r].box[e];
        const long long y = R[r].cb[e];
        bx = lo ? min(bx, x) : max(bx, x);
        cb = lo ? min(cb, y) : max(cb, y);
      }
      S.box[e] = bx;
      S.cb[e] = cb;
    }
  }
  __syncthreads();
  const NodeSetup u = node_setup(C, nd.depth, nd.count, nd.cblo, nd.cbhi);
  if (wave == 0) {
    const double clo[3] = {nd.lo[0], nd.lo[1], nd.lo[2]}, chi[3] = {nd.hi[0], nd.hi[1], nd.hi[2]};
    int axis, plane;
    double best;
    wave_eval(S.cnt, S.box, C, u, clo, chi, nd.count, axis, plane, best);
    if (lane == 0) {
      s_pick[0] = axis;
      s_pick[1] = plane;
      s_best = best;
    }
  }
  __syncthreads();
  const int axis = s_pick[0], plane = s_pick[1];
  if (axis < 0) {  // cannot happen for nodes queued here (nonzero extent)
    if (tid == 0) set_err(X.st, 16);
    return;
  }
  int nleft = 0;
  for (int b = 0; b < plane; ++b) nleft += S.cnt[axis * B + b];
  // left-going facets in the chunks before this one
  int loff = 0;
  {
    const int nprev = blockIdx.x - it.first_item;
    const int terms = nprev * plane;
    for (int t = tid; t < terms; t += kAThreads) {
      const int j = it.first_item + t / plane, b = t % plane;
      loff += X.ccnt[par][(size_t)j * 3 * RT_MAX_BINS + axis * B + b];
    }
    loff = wsum(loff);
    if (lane == 0) s_red[wave] = loff;
    __syncthreads();
    loff = 0;
    for (int w = 0; w < kAThreads / 64; ++w) loff += s_red[w];
  }
  const int roff = it.begin - loff;
  const int k = nd.count;
  const bool leaf0 = nleft <= C.max_leaf, leaf1 = k - nleft <= C.max_leaf;
  const double ax_lo = axis == 0 ? nd.cblo[0] : (axis == 1 ? nd.cblo[1] : nd.cblo[2]);
  const double ax_scale = axis == 0 ? u.scale[0] : (axis == 1 ? u.scale[1] : u.scale[2]);
  const FacetRec* in = X.recs[nd.depth & 1] + nd.first;
  FacetRec* out = X.recs[(nd.depth + 1) & 1] + nd.first;
  int32_t* perm = X.perm + nd.first;
  const unsigned long long below = lanes_below();
  int lb = 0, rb = 0;
  for (int s0 = it.begin; s0 < it.end; s0 += kAThreads) {
    const int i = s0 + tid;
    const bool valid = i < it.end;
    const FacetRec r = in[valid ? i : it.begin];
    bool g = false;
    if (valid) {
      const float l = axis == 0 ? r.lo.x : (axis == 1 ? r.lo.y : r.lo.z);
      const float h = axis == 0 ? r.hi.x : (axis == 1 ? r.hi.y : r.hi.z);
      g = bin_of(centroid(l, h), ax_lo, ax_scale, B) < plane;
    }
    const unsigned long long ml = __ballot(valid && g), mr = __ballot(valid && !g);
    if (lane == 0) {
      s_w[0][wave] = __popcll(ml);
      s_w[1][wave] = __popcll(mr);
    }
    __syncthreads();
    int pl = 0, pr = 0, tl = 0, tr = 0;
    for (int w = 0; w < kAThreads / 64; ++w) {
      if (w < wave) {
        pl += s_w[0][w];
        pr += s_w[1][w];
      }
      tl += s_w[0][w];
      tr += s_w[1][w];
    }
    __syncthreads();
    if (valid) {
      const int dst = g ? loff + lb + pl + __popcll(ml & below)
                        : nleft + roff + rb + pr + __popcll(mr & below);
      if (dst >= 0 && dst < k) {
        out[dst] = r;
        if (g ? leaf0 : leaf1) perm[dst] = __float_as_int(r.lo.w);
      } else {
        set_err(X.st, 128);
      }
    }
    lb += tl;
    rb += tr;
  }
  if (it.begin != 0) return;  // the node's first chunk writes the children
  // per side: bin slot (-1: not a big node), first chunk item, chunk items
  __shared__ int s_big[2][3];
  // the children's volumes and centroid bounds: the node's bins on the split
  // axis united per side, one bin per lane of the first wave
  __shared__ int s_bacc[12];
  __shared__ long long s_cacc[12];
  const int c0 = 2 * (nd.first + nleft - 1) + 1;
  if (wave == 0) {
    if (lane < 12) {
      s_bacc[lane] = lane % 6 < 3 ? f2o(INFINITY) : f2o(-INFINITY);
      s_cacc[lane] = lane % 6 < 3 ? d2o(INFINITY) : d2o(-INFINITY);
    }
    wave_sync();
    for (int b = lane; b < B; b += 64) {
      const int slot = axis * B + b, sd = b < plane ? 0 : 1;
      if (S.cnt[slot] == 0) continue;
      for (int q = 0; q < 3; ++q) {
        atomicMin(&s_bacc[6 * sd + q], S.box[6 * slot + q]);
        atomicMax(&s_bacc[6 * sd + 3 + q], S.box[6 * slot + 3 + q]);
        atomicMin(&s_cacc[6 * sd + q], S.cb[6 * slot + q]);
        atomicMax(&s_cacc[6 * sd + 3 + q], S.cb[6 * slot + 3 + q]);
      }
    }
    wave_sync();
  }
  if (tid == 0) {
    float lo[2][3], hi[2][3];
    double clo[2][3], chi[2][3];
    for (int sd = 0; sd < 2; ++sd)
      for (int q = 0; q < 3; ++q) {
        lo[sd][q] = o2f(s_bacc[6 * sd + q]);
        hi[sd][q] = o2f(s_bacc[6 * sd + 3 + q]);
        clo[sd][q] = o2d(s_cacc[6 * sd + q]);
        chi[sd][q] = o2d(s_cacc[6 * sd + 3 + q]);
      }
    make_children(X, it.node, nd, axis, plane, u.flags, s_best, nleft, lo, hi, clo, chi);
    int nit[2] = {0, 0};
    for (int side = 0; side < 2; ++side) {
      s_big[side][0] = -1;
      const int kc = side == 0 ? nleft : k - nleft;
      if (kc <= C.max_leaf) continue;
      const int first = nd.first + (side == 0 ? 0 : nleft);
      const int to = classify(C, kc, nd.depth + 1, clo[side], chi[side], lvl + 1 < X.la, X.lm > 0);
      if (to == TO_A) nit[side] = (kc + kChunk - 1) / kChunk;
      else if (to == TO_M) push_m(X, 0, c0 + side, first);
      else push_s(X, c0 + side, first);
    }
    // both big children's bin slots and chunk items in one atomic add
    const int nbig = (nit[0] > 0) + (nit[1] > 0);
    int slot, base;
    if (nbig > 0 && take_big(X, lvl + 1, nbig, nit[0] + nit[1], slot, base)) {
      for (int side = 0; side < 2; ++side) {
        if (nit[side] == 0) continue;
        s_big[side][0] = slot++;
        s_big[side][1] = base;
        s_big[side][2] = nit[side];
        base += nit[side];
      }
    }
  }
  __syncthreads();
  for (int side = 0; side < 2; ++side) {
    const int slot = s_big[side][0];
    if (slot < 0) continue;
    const int kc = side == 0 ? nleft : k - nleft;
    for (int j = tid; j < s_big[side][2]; j += kAThreads)
      write_item(X, lvl + 1, c0 + side, kc, slot, s_big[side][1], s_big[side][2], j);
  }
}

// ---------------------------------------------------------------------------
// One node split by one wave, facet records in global memory.  Returns the
// left child id (wave-uniform) and the children's sizes and centroid bounds.
constexpr int kPartE = 4;  // records per lane and partition round of a medium node above 64 facets (147 VGPRs, 3 waves per SIMD)

// Run of consecutive facets in one bin of one axis, counts and boxes only.
struct RunB {
  int bin, count;
  float lo[3], hi[3];
};
__device__ inline void runb_reset(RunB& r, int bin) {
  r.bin = bin;
  r.count = 0;
  for (int q = 0; q < 3; ++q) {
    r.lo[q] = INFINITY;
    r.hi[q] = -INFINITY;
  }
}
__device__ inline void runb_flush(const RunB& r, const Bins& S, int a, int B) {
  if (r.count == 0) return;
  const int slot = a * B + r.bin;
  atomicAdd(&S.cnt[slot], r.count);
  for (int q = 0; q < 3; ++q) {
    atomicMin(&S.box[6 * slot + q], f2o(r.lo[q]));
    atomicMax(&S.box[6 * slot + 3 + q], f2o(r.hi[q]));
  }
}

// Stable partition of a node's records (global memory) by the split: left
// side first, each side in input order; leaf children's facets go to perm.
// Each lane unites the boxes and centroids of the facets it moves, per side.
// PE records per lane and round.
template <int PE>
__device__ __forceinline__ void split_partition(BuildState* st, const FacetRec* in, FacetRec* out,
                                                int32_t* perm, int k, int nleft, bool by_position, int ax,
                                                double ax_lo, double ax_scale, int B, int plane,
                                                bool leaf0, bool leaf1, float blo[2][3], float bhi[2][3],
                                                double cbl[2][3], double cbh[2][3]) {
  const int lane = lane_id();
  const unsigned long long below = lanes_below();
  int lbase = 0, rbase = 0;
  for (int base = 0; base < k; base += 64 * PE) {
    FacetRec r[PE];
    bool gl[PE], valid[PE];
    unsigned long long ml[PE], mr[PE];
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      const int i = base + e * 64 + lane;
      valid[e] = i < k;
      r[e] = in[min(i, k - 1)];
    }
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      const int i = base + e * 64 + lane;
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
      ml[e] = __ballot(valid[e] && g);
      mr[e] = __ballot(valid[e] && !g);
    }
    int offl = 0, offr = 0;
#pragma unroll
    for (int e = 0; e < PE; ++e) {
      if (valid[e]) {
        const int dst = gl[e] ? lbase + offl + __popcll(ml[e] & below)
                              : nleft + rbase + offr + __popcll(mr[e] & below);
        if (dst >= 0 && dst < k) {
          out[dst] = r[e];
          if (gl[e] ? leaf0 : leaf1) perm[dst] = __float_as_int(r[e].lo.w);
        } else {
          set_err(st, 128);
        }
        const float4 lo = r[e].lo, hi = r[e].hi;
        const double cx = centroid(lo.x, hi.x), cy = centroid(lo.y, hi.y), cz = centroid(lo.z, hi.z);
        const int sd = gl[e] ? 0 : 1;
        blo[sd][0] = fminf(blo[sd][0], lo.x); blo[sd][1] = fminf(blo[sd][1], lo.y); blo[sd][2] = fminf(blo[sd][2], lo.z);
        bhi[sd][0] = fmaxf(bhi[sd][0], hi.x); bhi[sd][1] = fmaxf(bhi[sd][1], hi.y); bhi[sd][2] = fmaxf(bhi[sd][2], hi.z);
        cbl[sd][0] = fmin(cbl[sd][0], cx); cbl[sd][1] = fmin(cbl[sd][1], cy); cbl[sd][2] = fmin(cbl[sd][2], cz);
        cbh[sd][0] = fmax(cbh[sd][0], cx); cbh[sd][1] = fmax(cbh[sd][1], cy); cbh[sd][2] = fmax(cbh[sd][2], cz);
      }
      offl += __popcll(ml[e]);
      offr += __popcll(mr[e]);
    }
    lbase += offl;
    rbase += offr;
  }
}

// PE_MAX: records per lane and partition round for nodes above 64 facets (and
// binning loads in flight); k_s, whose nodes are mostly small, takes 1 to
// keep its registers (and so its waves per SIMD) down.
// The wave's bins count facets and unite their boxes per bin (the centroid
// bounds region of S is not used as bins here: it holds the 12 + 12 child
// accumulators, so S must come with centroid bounds).  The children's
// volumes and centroid bounds are exact unions of their facets', taken while
// partitioning: each lane unites its own facets, then adds them with ordered
// integer min / max into the accumulators.
template <int PE_MAX>
__device__ int wave_split_global(const Ctx& X, int id, const Bins& S, int& kc0, int& kc1,
                                 double ccb[2][6]) {
  const int lane = lane_id();
  const BNode nd = X.nodes[id];
  const int k = nd.count, B = X.C.nbins;
  BuildConst C = X.C;
  C.inv_l2 = X.st->inv_l2;
  const NodeSetup u = node_setup(C, nd.depth, k, nd.cblo, nd.cbhi);
  const FacetRec* in = X.recs[nd.depth & 1] + nd.first;
  FacetRec* out = X.recs[(nd.depth + 1) & 1] + nd.first;
  int32_t* perm = X.perm + nd.first;
  long long* cacc = S.cb;          // [side][centroid lo xyz, hi xyz]
  int* bacc = (int*)(S.cb + 12);   // [side][box lo xyz, hi xyz]
  if (lane < 12) {
    cacc[lane] = lane % 6 < 3 ? d2o(INFINITY) : d2o(-INFINITY);
    bacc[lane] = lane % 6 < 3 ? f2o(INFINITY) : f2o(-INFINITY);
  }
  int axis = -1, plane = -1, flags = u.flags;
  double best = INFINITY;
  if (!u.forced) {
    Bins Sb = S;
    Sb.cb = nullptr;
    bins_clear(Sb, B, lane, 64);
    wave_sync();
    // each lane walks a contiguous run of the node's facets
    const int per = (k + 63) / 64;
    const int i0 = min(k, lane * per), i1 = min(k, i0 + per);
    RunB run[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) runb_reset(run[a], -1);
    constexpr int kBinU = PE_MAX == 1 ? 1 : 4;
    for (int i = i0; i < i1; i += kBinU) {
      float4 lo[kBinU], hi[kBinU];
#pragma unroll
      for (int v = 0; v < kBinU; ++v) {
        const int q = min(i + v, i1 - 1);
        lo[v] = in[q].lo;
        hi[v] = in[q].hi;
      }
#pragma unroll
      for (int v = 0; v < kBinU; ++v) {
        if (i + v >= i1) break;
        const double cu[3] = {centroid(lo[v].x, hi[v].x), centroid(lo[v].y, hi[v].y),
                              centroid(lo[v].z, hi[v].z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          if (!u.axis_ok[a]) continue;
          const int b = bin_of(cu[a], nd.cblo[a], u.scale[a], B);
          if (b != run[a].bin) {
            runb_flush(run[a], Sb, a, B);
            runb_reset(run[a], b);
          }
          RunB& r = run[a];
          r.count += 1;
          r.lo[0] = fminf(r.lo[0], lo[v].x); r.lo[1] = fminf(r.lo[1], lo[v].y); r.lo[2] = fminf(r.lo[2], lo[v].z);
          r.hi[0] = fmaxf(r.hi[0], hi[v].x); r.hi[1] = fmaxf(r.hi[1], hi[v].y); r.hi[2] = fmaxf(r.hi[2], hi[v].z);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) runb_flush(run[a], Sb, a, B);
    wave_sync();
    const double clo[3] = {nd.lo[0], nd.lo[1], nd.lo[2]}, chi[3] = {nd.hi[0], nd.hi[1], nd.hi[2]};
    wave_eval(S.cnt, S.box, C, u, clo, chi, k, axis, plane, best);
    if (axis < 0) flags |= 2;
  }
  wave_sync();  // the accumulators' initial values
  const bool by_position = axis < 0;
  int nleft = 0;
  if (by_position) {
    nleft = k / 2;
  } else {
    for (int b = lane; b < plane; b += 64) nleft += S.cnt[axis * B + b];
    nleft = wsum(nleft);
  }
  const bool leaf0 = nleft <= C.max_leaf, leaf1 = k - nleft <= C.max_leaf;
  const int ax = by_position ? 0 : axis;
  const double ax_lo = ax == 0 ? nd.cblo[0] : (ax == 1 ? nd.cblo[1] : nd.cblo[2]);
  const double ax_scale = ax == 0 ? u.scale[0] : (ax == 1 ? u.scale[1] : u.scale[2]);
  float blo[2][3], bhi[2][3];
  double cbl[2][3], cbh[2][3];
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      blo[side][q] = INFINITY;
      bhi[side][q] = -INFINITY;
      cbl[side][q] = INFINITY;
      cbh[side][q] = -INFINITY;
    }
  if (PE_MAX == 1 || k <= 64)
    split_partition<1>(X.st, in, out, perm, k, nleft, by_position, ax, ax_lo, ax_scale, B, plane, leaf0,
                       leaf1, blo, bhi, cbl, cbh);
  else
    split_partition<PE_MAX>(X.st, in, out, perm, k, nleft, by_position, ax, ax_lo, ax_scale, B, plane,
                            leaf0, leaf1, blo, bhi, cbl, cbh);
  // the children's volumes and centroid bounds (a lane with no facet on a
  // side leaves that side's accumulators alone)
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      if (blo[side][q] <= bhi[side][q]) {
        atomicMin(&bacc[6 * side + q], f2o(blo[side][q]));
        atomicMax(&bacc[6 * side + 3 + q], f2o(bhi[side][q]));
        atomicMin(&cacc[6 * side + q], d2o(cbl[side][q]));
        atomicMax(&cacc[6 * side + 3 + q], d2o(cbh[side][q]));
      }
    }
  wave_sync();
  float lo[2][3], hi[2][3];
  double clo[2][3], chi[2][3];
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      lo[side][q] = o2f(bacc[6 * side + q]);
      hi[side][q] = o2f(bacc[6 * side + 3 + q]);
      clo[side][q] = o2d(cacc[6 * side + q]);
      chi[side][q] = o2d(cacc[6 * side + 3 + q]);
    }
  if (lane == 0)
    make_children(X, id, nd, axis, plane, flags, by_position ? 0.0 : best, nleft, lo, hi, clo, chi);
  const int c0 = 2 * (nd.first + nleft - 1) + 1;
  kc0 = nleft;
  kc1 = k - nleft;
  for (int side = 0; side < 2; ++side)
    for (int q = 0; q < 3; ++q) {
      ccb[side][q] = clo[side][q];
      ccb[side][3 + q] = chi[side][q];
    }
  wave_sync();  // the bins and accumulators are reused by the wave's next node
  return c0;
}

// Medium nodes: one wave per window of kMWindow facet positions; a pending
// node (more than kRegNode facets) is filed under its first facet, so a
// window holds at most one.
constexpr int kMWindow = kRegNode + 1;
// The wave kernels (k_m, k_s) serve up to four independent waves per
// work-group, each in its own LDS slice, and are launched with one: a wave
// that finishes frees its slot and LDS at once instead of waiting for its
// neighbours, which keeps the few compute units of a build that runs beside
// a trace busy.  The slice is found from the lane's own wave index, so the
// compiler sees the child-bound accumulators at lane-dependent LDS
// addresses and keeps their min / max as single LDS atomics (with a uniform
// address it expands each into a loop over the active lanes, which doubled
// the build time).
constexpr int kWaveThreads = 256;
__global__ __launch_bounds__(kWaveThreads) void k_m(Ctx X, int pass) {
  extern __shared__ __align__(16) char lds[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int B = X.C.nbins;
  const Bins S = bins_at(lds + w * bins_bytes(B, true), B, true);
  const int base = (blockIdx.x * (blockDim.x >> 6) + w) * kMWindow;
  if (base >= X.n) return;
  int32_t* front = X.mfront[pass & 1];
  const int slot = base + lane;
  const int mine = lane < kMWindow && slot < X.n ? front[slot] : -1;
  if (mine >= 0) front[slot] = -1;  // free for pass + 2
  unsigned long long todo = __ballot(mine >= 0);
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int id = __shfl(mine, src);
    const int depth = X.nodes[id].depth, first0 = X.nodes[id].first;
    int kc[2];
    double ccb[2][6];
    const int c0 = wave_split_global<kPartE>(X, id, S, kc[0], kc[1], ccb);
    if (lane < 2 && kc[lane] > X.C.max_leaf) {
      const double* cb = lane == 0 ? ccb[0] : ccb[1];
      const int to = classify(X.C, kc[lane], depth + 1, cb, cb + 3, false, pass + 1 < X.lm);
      const int first = first0 + (lane == 0 ? 0 : kc[0]);
      if (to == TO_M) push_m(X, pass + 1, c0 + lane, first);
      else push_s(X, c0 + lane, first);
    }
    wave_sync();
  }
}

// ---------------------------------------------------------------------------
// Subtrees.  A wave takes the subtree roots filed in its window of facet
// positions and splits each depth-first until every node is a leaf.  Nodes
// above kRegNode facets are split from global memory; a node at or below it
// is finished with its records in registers (lane i holds the node's i-th
// facet), the partition being a permutation of lanes.

// Node of a register subtree, kept on an LDS stack.
struct RNode {
  int32_t id, r0, cnt, depth;
  float lo[3], hi[3];
  double cblo[3], cbhi[3];
};
constexpr int kRStack = 64;   // a register subtree (<= kRegNode facets) is less deep
constexpr int kGStack = 72;   // nodes above kRegNode waiting on the global path

__host__ __device__ inline size_t s_wave_bytes(int B) {
  return bins_bytes(B, true) + align8(sizeof(RNode) * kRStack) + align8(sizeof(int) * kGStack);
}

// Bins of the node on lanes [r0, r0 + cnt) with 16 bins: lane 16 a + b walks
// the node's facets and keeps those in bin b of axis a.
__device__ inline void bins16_from_lanes(int r0, int cnt, int packed_bins, const float lo[3],
                                         const float hi[3], int& c, float bl[3], float bh[3]) {
  const int lane = lane_id();
  const int shift = 8 * min(lane >> 4, 2);
  const int mine = lane & 15;
  c = 0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    bl[q] = INFINITY;
    bh[q] = -INFINITY;
  }
  for (int j = r0; j < r0 + cnt; ++j) {
    const int pj = __builtin_amdgcn_readlane(packed_bins, j);
    float l[3], h[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      l[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lo[q]), j));
      h[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hi[q]), j));
    }
    if (((pj >> shift) & 255) == mine) {
      c += 1;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        bl[q] = fminf(bl[q], l[q]);
        bh[q] = fmaxf(bh[q], h[q]);
      }
    }
  }
  if (lane >= 48) c = 0;
}

// S must come with centroid bounds: that region holds the children's
// accumulators, the bins (any count but 16) are counts and boxes only.
__device__ void wave_subtree_regs(const Ctx& X, int id, const Bins& S, RNode* stk) {
  const int lane = lane_id();
  const int B = X.C.nbins;
  BuildConst C = X.C;
  C.inv_l2 = X.st->inv_l2;
  const BNode nd = X.nodes[id];
  const int base = nd.first;
  const FacetRec* in = X.recs[nd.depth & 1] + base;
  // lane i holds facet i of the subtree
  float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {0.f, 0.f, 0.f};
  int fid = -1;
  if (lane < nd.count) {
    const FacetRec r = in[lane];
    lo[0] = r.lo.x; lo[1] = r.lo.y; lo[2] = r.lo.z;
    hi[0] = r.hi.x; hi[1] = r.hi.y; hi[2] = r.hi.z;
    fid = __float_as_int(r.lo.w);
  }
  if (lane == 0) {
    RNode t;
    t.id = id;
    t.r0 = 0;
    t.cnt = nd.count;
    t.depth = nd.depth;
    for (int q = 0; q < 3; ++q) {
      t.lo[q] = nd.lo[q];
      t.hi[q] = nd.hi[q];
      t.cblo[q] = nd.cblo[q];
      t.cbhi[q] = nd.cbhi[q];
    }
    stk[0] = t;
  }
  int sp = 1;
  const unsigned long long below = lanes_below();
  while (sp > 0) {
    wave_sync();
    const RNode t = stk[--sp];
    const bool inr = lane >= t.r0 && lane < t.r0 + t.cnt;
    const NodeSetup u = node_setup(C, t.depth, t.cnt, t.cblo, t.cbhi);
    int axis = -1, plane = -1, flags = u.flags;
    double best = INFINITY;
    int mybins = 0;  // this lane's facet: bin on each axis, 8 bits each
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = u.axis_ok[a] ? bin_of(centroid(lo[a], hi[a]), t.cblo[a], u.scale[a], B) : 0;
      mybins |= b << (8 * a);
    }
    if (!u.forced) {
      const double clo[3] = {t.lo[0], t.lo[1], t.lo[2]}, chi[3] = {t.hi[0], t.hi[1], t.hi[2]};
      if (B == 16) {
        int c;
        float bl[3], bh[3];
        bins16_from_lanes(t.r0, t.cnt, mybins, lo, hi, c, bl, bh);
        eval16(c, bl, bh, C, u, clo, chi, t.cnt, axis, plane, best);
      } else {
        Bins Sb = S;
        Sb.cb = nullptr;
        bins_clear(Sb, B, lane, 64);
        wave_sync();
        if (inr) {
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            if (!u.axis_ok[a]) continue;
            const int slot = a * B + ((mybins >> (8 * a)) & 255);
            atomicAdd(&S.cnt[slot], 1);
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              atomicMin(&S.box[6 * slot + q], f2o(lo[q]));
              atomicMax(&S.box[6 * slot + 3 + q], f2o(hi[q]));
            }
          }
        }
        wave_sync();
        wave_eval_any(S.cnt, S.box, C, u, clo, chi, t.cnt, axis, plane, best);
      }
      if (axis < 0) flags |= 2;
    }
    const bool by_position = axis < 0;
    const bool g = by_position ? lane - t.r0 < t.cnt / 2
                               : ((mybins >> (8 * max(axis, 0))) & 255) < plane;
    const unsigned long long ml = __ballot(inr && g), mr = __ballot(inr && !g);
    const int nleft = __popcll(ml);
    const int dst = !inr ? lane
                    : g ? t.r0 + __popcll(ml & below)
                        : t.r0 + nleft + __popcll(mr & below);
    // stable partition of the node's lanes: every lane sends its record to dst
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      lo[q] = __int_as_float(__builtin_amdgcn_ds_permute(dst * 4, __float_as_int(lo[q])));
      hi[q] = __int_as_float(__builtin_amdgcn_ds_permute(dst * 4, __float_as_int(hi[q])));
    }
    fid = __builtin_amdgcn_ds_permute(dst * 4, fid);
    // child volumes and centroid bounds: exact unions through ordered-integer
    // min / max into the accumulators, one facet per lane
    const int side = !inr ? -1 : (lane < t.r0 + nleft ? 0 : 1);
    long long* cacc = S.cb;         // [side][centroid lo xyz, hi xyz]
    int* bacc = (int*)(S.cb + 12);  // [side][box lo xyz, hi xyz]
    wave_sync();  // the previous node's reads of the accumulators are done
    if (lane < 12) {
      cacc[lane] = lane % 6 < 3 ? d2o(INFINITY) : d2o(-INFINITY);
      bacc[lane] = lane % 6 < 3 ? f2o(INFINITY) : f2o(-INFINITY);
    }
    wave_sync();
    if (side >= 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        atomicMin(&bacc[6 * side + q], f2o(lo[q]));
        atomicMax(&bacc[6 * side + 3 + q], f2o(hi[q]));
        const long long c = d2o(centroid(lo[q], hi[q]));
        atomicMin(&cacc[6 * side + q], c);
        atomicMax(&cacc[6 * side + 3 + q], c);
      }
    }
    wave_sync();
    float clo_f[2][3], chi_f[2][3];
    double ccl[2][3], cch[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        clo_f[s][q] = o2f(bacc[6 * s + q]);
        chi_f[s][q] = o2f(bacc[6 * s + 3 + q]);
        ccl[s][q] = o2d(cacc[6 * s + q]);
        cch[s][q] = o2d(cacc[6 * s + 3 + q]);
      }
    BNode pn;
    pn.first = base + t.r0;
    pn.count = t.cnt;
    pn.depth = t.depth;
    if (lane == 0)
      make_children(X, t.id, pn, axis, plane, flags, by_position ? 0.0 : best, nleft, clo_f, chi_f,
                    ccl, cch);
    const int c0 = 2 * (base + t.r0 + nleft - 1) + 1;
    const int kc[2] = {nleft, t.cnt - nleft};
    // leaves: their facets are final; other children go on the stack (right first)
    for (int s = 1; s >= 0; --s) {
      if (kc[s] <= C.max_leaf) {
        if (side == s) X.perm[base + lane] = fid;
        continue;
      }
      if (sp >= kRStack) {  // cannot happen: register subtrees are shallower
        if (lane == 0) set_err(X.st, 32);
        return;
      }
      if (lane == 0) {
        RNode ch;
        ch.id = c0 + s;
        ch.r0 = s == 0 ? t.r0 : t.r0 + nleft;
        ch.cnt = kc[s];
        ch.depth = t.depth + 1;
        for (int q = 0; q < 3; ++q) {
          ch.lo[q] = clo_f[s][q];
          ch.hi[q] = chi_f[s][q];
          ch.cblo[q] = ccl[s][q];
          ch.cbhi[q] = cch[s][q];
        }
        stk[sp] = ch;
      }
      ++sp;
    }
  }
}

__global__ __launch_bounds__(kWaveThreads) void k_s(Ctx X) {
  extern __shared__ __align__(16) char lds[];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int B = X.C.nbins;
  char* mine = lds + w * s_wave_bytes(B);
  const Bins S = bins_at(mine, B, true);
  RNode* rstk = (RNode*)(mine + bins_bytes(B, true));
  int* gstk = (int*)(mine + bins_bytes(B, true) + align8(sizeof(RNode) * kRStack));
  // subtree roots hold more than max_leaf facets, so a window of
  // min(64, 2 (max_leaf + 1)) facet positions holds at most two of them,
  // taken in turn (half as many waves as one-root windows: fewer rounds of
  // resident waves)
  const int win = min(64, 2 * (X.C.max_leaf + 1));
  const int wbase = (blockIdx.x * (blockDim.x >> 6) + w) * win;
  if (wbase >= X.n) return;
  const int slot = wbase + lane;
  const int root = lane < win && slot < X.n ? X.sfront[slot] : -1;
  unsigned long long todo = __ballot(root >= 0);
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int rid = __shfl(root, src);
    if (lane == 0) gstk[0] = rid;
    int sp = 1;
    bool failed = false;
    while (sp > 0 && !failed) {
      wave_sync();
      const int id = gstk[--sp];
      const int k = X.nodes[id].count;
      if (k <= kRegNode) {
        wave_subtree_regs(X, id, S, rstk);
        continue;
      }
      int kc[2];
      double ccb[2][6];
      const int c0 = wave_split_global<1>(X, id, S, kc[0], kc[1], ccb);
      // the children's records and nodes were written by this wave
      wave_global_sync();
      for (int sd = 1; sd >= 0; --sd) {
        if (kc[sd] <= X.C.max_leaf) continue;
        if (sp >= kGStack) {
          if (lane == 0) set_err(X.st, 64);
          failed = true;
          break;
        }
        if (lane == 0) gstk[sp] = c0 + sd;
        ++sp;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Compaction: the used split boundaries, in order, become traversal indices
// 0, 1, ... (the root's and index 0 then trade places, so that traversal
// starts at 0); node ids follow (children of index r are 2 r + 1, 2 r + 2).
__global__ __launch_bounds__(kScanBlock) void k_count(const int32_t* __restrict__ used, int nb,
                                                      int32_t* __restrict__ bsum,
                                                      int32_t* __restrict__ bmax) {
  __shared__ int s_c[kScanBlock / 64], s_m[kScanBlock / 64];
  const int b = blockIdx.x * kScanBlock + threadIdx.x;
  const int u = b < nb ? used[b] : 0;
  int c = __popcll(__ballot(u > 0));
  int m = u;
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o));
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_c[wave] = c;
    s_m[wave] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int tc = 0, tm = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) {
      tc += s_c[w];
      tm = max(tm, s_m[w]);
    }
    bsum[blockIdx.x] = tc;
    bmax[blockIdx.x] = tm;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_rank(const int32_t* __restrict__ used, int nb,
                                                     const int32_t* __restrict__ bsum,
                                                     const int32_t* __restrict__ bmax,
                                                     int32_t* __restrict__ rank,
                                                     BuildState* __restrict__ st) {
  __shared__ int s_w[kScanBlock / 64];
  __shared__ int s_pre, s_max;
  const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
  const bool last = blockIdx.x == gridDim.x - 1;
  // exclusive prefix of the earlier blocks (and, in the last block, the deepest child)
  int pre = 0, dm = 0;
  for (int j = tid; j < (int)blockIdx.x; j += kScanBlock) pre += bsum[j];
  if (last)
    for (int j = tid; j < (int)gridDim.x; j += kScanBlock) dm = max(dm, bmax[j]);
  pre = wsum(pre);
  for (int o = 32; o > 0; o >>= 1) dm = max(dm, __shfl_xor(dm, o));
  if (lane == 0) s_w[wave] = pre;
  if (tid == 0) s_max = 0;
  __syncthreads();
  if (lane == 0) atomicMax(&s_max, dm);
  if (tid == 0) {
    int t = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) t += s_w[w];
    s_pre = t;
  }
  __syncthreads();
  const int b = blockIdx.x * kScanBlock + tid;
  const bool u = b < nb && used[b] > 0;
  const unsigned long long m = __ballot(u);
  if (lane == 0) s_w[wave] = __popcll(m);
  __syncthreads();
  int off = s_pre;
  for (int w = 0; w < wave; ++w) off += s_w[w];
  if (u) rank[b] = off + __popcll(m & lanes_below());
  if (last && tid == 0) {
    int t = s_pre;
    for (int w = 0; w < kScanBlock / 64; ++w) t += s_w[w];
    st->total = 2 * t + 1;
    st->depth = s_max;
  }
}

// End of a build, by every thread of one work-group after the build's other
// work: the host record {sequence, nodes, depth, non-finite, error, root lo
// xyz, root hi xyz}, then BuildState and the root bounds set back to their
// starting values for the next build on these buffers (nothing of this build
// reads them afterwards).
__device__ void finish_build(BuildState* st, long long* root, const BNode* nodes,
                             int32_t* host_out, int seq) {
  if (threadIdx.x == 0) {
    host_out[1] = st->total;
    host_out[2] = st->depth;
    host_out[3] = st->nonfinite;
    host_out[4] = st->error;
    for (int q = 0; q < 3; ++q) {
      host_out[5 + q] = __float_as_int(nodes[0].lo[q]);
      host_out[8 + q] = __float_as_int(nodes[0].hi[q]);
    }
    __threadfence_system();
    __atomic_store_n(&host_out[0], seq, __ATOMIC_RELEASE);
  }
  __syncthreads();
  int32_t* words = reinterpret_cast<int32_t*>(st);
  for (int i = threadIdx.x; i < kStateWords; i += blockDim.x) words[i] = 0;
  if (threadIdx.x < 3) {
    const int t = threadIdx.x;
    root[t] = f2o(INFINITY);
    root[3 + t] = f2o(-INFINITY);
    root[6 + t] = d2o(INFINITY);
    root[9 + t] = d2o(-INFINITY);
  }
}
__global__ void k_finish(BuildState* st, long long* root, const BNode* nodes, int32_t* host_out,
                         int seq) {
  finish_build(st, root, nodes, host_out, seq);
}

__device__ inline float4 f4(float x, float y, float z, float w) { return make_float4(x, y, z, w); }
// traversal index of an internal node: its child pair
__device__ inline int pair_index(const BNode& nd) { return (nd.left - 1) >> 1; }

// The facet at leaf-ordered position k.  The leaves tile the positions, and
// the boundary between two neighbouring leaves is the split position of some
// internal node, so the facet at k ends its leaf exactly when boundary k is
// used (or k is the last position).
__device__ inline void emit_facet(int k, int n, const int32_t* __restrict__ used,
                                  const int32_t* __restrict__ perm, const float* __restrict__ tris,
                                  TFacet* __restrict__ tf) {
  const int f = perm[k];
  const float* v = tris + 9 * (int64_t)f;
  const uint32_t tag = (uint32_t)f | (k == n - 1 || used[k] > 0 ? kLastFacet : 0u);
  TFacet o;
  o.p0 = f4(v[0], v[1], v[2], __uint_as_float(tag));
  o.p1 = f4(v[3], v[4], v[5], 0.f);
  o.p2 = f4(v[6], v[7], v[8], 0.f);
  tf[k] = o;
}
// One split boundary b (or, for the extra last index, the root): the facet at
// position b, and for a used boundary its two children copied to their
// compact ids and its traversal node.
// Traversal starts at index 0, so the root's pair swaps its rank with rank 0.
__device__ inline int remap(int r, int rr) { return r == rr ? 0 : (r == 0 ? rr : r); }
__device__ inline int compact_left(int left, const int32_t* __restrict__ rank, int rr) {
  return left < 0 ? -1 : 2 * remap(rank[(left - 1) >> 1], rr) + 1;
}

__device__ void emit_one(const BNode* __restrict__ nodes, const BuildState* __restrict__ st,
                         const int32_t* __restrict__ used, const int32_t* __restrict__ rank,
                         const int32_t* __restrict__ perm, const float* __restrict__ tris,
                         BNode* __restrict__ cn, TNode* __restrict__ tn, TFacet* __restrict__ tf) {
  const int n = st->n;
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (st->error || b >= n) return;
  emit_facet(b, n, used, perm, tris, tf);
  const int root_left = nodes[0].left;
  const int rr = root_left < 0 ? 0 : rank[(root_left - 1) >> 1];
  if (b == n - 1) {  // the root (a boundary index that is never used)
    BNode r = nodes[0];
    r.left = compact_left(r.left, rank, rr);
    cn[0] = r;
    if (r.left < 0) {  // the whole scene is one leaf: a root with one empty child
      TNode t;
      t.a = f4(r.lo[0], r.hi[0], r.lo[1], r.hi[1]);
      // an empty volume: lo = hi = +inf gives an empty slab on every axis
      t.b = f4(INFINITY, INFINITY, INFINITY, INFINITY);
      t.c = f4(r.lo[2], r.hi[2], INFINITY, INFINITY);
      t.d = make_int4(~0, ~0, 0, 0);
      tn[0] = t;
    }
    return;
  }
  if (used[b] <= 0) return;
  const int r = remap(rank[b], rr);
  BNode ch[2];
  for (int side = 0; side < 2; ++side) {
    ch[side] = nodes[2 * b + 1 + side];
    ch[side].left = compact_left(ch[side].left, rank, rr);
    cn[2 * r + 1 + side] = ch[side];
  }
  const BNode& l = ch[0];
  const BNode& q = ch[1];
  TNode t;
  t.a = f4(l.lo[0], l.hi[0], l.lo[1], l.hi[1]);
  t.b = f4(q.lo[0], q.hi[0], q.lo[1], q.hi[1]);
  t.c = f4(l.lo[2], l.hi[2], q.lo[2], q.hi[2]);
  t.d = make_int4(l.left < 0 ? ~l.first : pair_index(l), q.left < 0 ? ~q.first : pair_index(q), 0, 0);
  tn[r] = t;
}
// The build then ends with k_finish, one work-group.  (Ending it from the
// last work-group of this pass instead costs a device-scope fence in every
// work-group: measured slower, by 36 us on a 200k-facet build.)
__global__ void k_emit(const BNode* __restrict__ nodes, const BuildState* __restrict__ st,
                       const int32_t* __restrict__ used, const int32_t* __restrict__ rank,
                       const int32_t* __restrict__ perm, const float* __restrict__ tris,
                       BNode* __restrict__ cn, TNode* __restrict__ tn, TFacet* __restrict__ tf) {
  emit_one(nodes, st, used, rank, perm, tris, cn, tn, tf);
}

// ---------------------------------------------------------------------------
// 4-wide traversal nodes: every even-depth internal node becomes one wide
// node whose children are its grandchildren, or its children where those are
// leaves.  Stored at the node's traversal index (its child pair).

__device__ inline float pow2f(int e) { return __int_as_float((e + 127) << 23); }  // e in [-126, 127]

// The 8-bit bounds are exact: the child plane of code q is lo + q 2^e in real
// arithmetic (the traversal crosses it with one fused multiply-add and an
// outward-rounded node term, which encloses the exact plane).  Containment
// is therefore decided on the exact sum, from its float32 rounding
// r = fmaf(q, 2^e, lo): rounding to nearest is monotone and v is a float, so
// r < v implies lo + q 2^e <= v and r > v implies >= v; when r == v the
// comparison holds only if the sum is exact, i.e. r - lo == q 2^e, checked in
// double with the subtraction's own rounding error (two-sum) required zero.
// Exponents stay in [kQExpMin, 127] so that 2^e / d remains a normal float.
constexpr int kQExpMin = -64;

__device__ inline bool sum_exact(float q, float sc, float lo, float r) {
  const double a = r, b = -(double)lo;
  const double s = a + b;
  const double bb = s - a;
  const double err = (a - (s - bb)) + (b - bb);
  return err == 0.0 && s == (double)q * (double)sc;
}
// lo + q sc <= v exactly
__device__ inline bool dec_le(int q, float sc, float lo, float v) {
  const float r = fmaf((float)q, sc, lo);
  return r < v || (r == v && sum_exact((float)q, sc, lo, r));
}
// lo + q sc >= v exactly
__device__ inline bool dec_ge(int q, float sc, float lo, float v) {
  const float r = fmaf((float)q, sc, lo);
  return r > v || (r == v && sum_exact((float)q, sc, lo, r));
}

// Per-axis exponent: smallest e with lo + 255 2^e >= hi.
__device__ inline int quant_exp(float lo, float hi) {
  int e = kQExpMin;
  const float ext = hi - lo;
  if (ext > 0.f) {
    int x;
    frexpf(ext / 255.f, &x);  // ext / 255 < 2^x
    e = max(kQExpMin, min(127, x - 1));
  }
  while (e < 127 && !dec_ge(255, pow2f(e), lo, hi)) ++e;
  while (e > kQExpMin && dec_ge(255, pow2f(e - 1), lo, hi)) --e;
  return e;
}
// Largest q with lo + q sc <= v (q in [0, 255]; q = 0 qualifies: lo <= v).
__device__ inline unsigned quant_lo(float v, float lo, float sc) {
  int q = (int)floorf((v - lo) / sc);
  q = max(0, min(255, q));
  while (q > 0 && !dec_le(q, sc, lo, v)) --q;
  while (q < 255 && dec_le(q + 1, sc, lo, v)) ++q;
  return (unsigned)q;
}
// Smallest q with lo + q sc >= v (q = 255 qualifies: it reaches the parent's hi).
__device__ inline unsigned quant_hi(float v, float lo, float sc) {
  int q = (int)ceilf((v - lo) / sc);
  q = max(0, min(255, q));
  while (q < 255 && !dec_ge(q, sc, lo, v)) ++q;
  while (q > 0 && dec_ge(q - 1, sc, lo, v)) --q;
  return (unsigned)q;
}

// Four lanes per binary node: lane c of a node's group gathers child slot c
// of the wide node (and, for 8-bit nodes, encodes that child's six planes)
// and stores its own parts of the record, so a lane encodes one child
// instead of four and the launch has four times the waves (one lane per node
// left most of the device idle behind long serial encodings).
template <int FMT>
__global__ __launch_bounds__(256) void k_collapse(const BNode* __restrict__ nodes,
                                                  const BuildState* __restrict__ st,
                                                  FNode4* __restrict__ wn) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = (int)(gid & 3);
  if (st->error || gid >> 2 >= min(st->total, 2 * st->n - 1)) return;
  const int id = (int)(gid >> 2);
  const BNode& nd = nodes[id];
  const int left = nd.left;
  const bool root_leaf = id == 0 && left < 0;
  if (!root_leaf && (left < 0 || (nd.depth & 1))) return;
  // the slots: each side's child if it is a leaf, else that child's two
  // children, side 0 first
  int src = -1, nc = 1;
  if (root_leaf) {
    src = c == 0 ? id : -1;
  } else {
    const int la = nodes[left].left, lb = nodes[left + 1].left;
    const int na = la < 0 ? 1 : 2;
    nc = na + (lb < 0 ? 1 : 2);
    if (c < na)
      src = la < 0 ? left : la + c;
    else if (c < nc)
      src = lb < 0 ? left + 1 : lb + (c - na);
  }
  const unsigned mask = (1u << nc) - 1u;
  const int slot = root_leaf ? 0 : pair_index(nd);
  float lo[3], hi[3];
  int ref = 0;
  if (src >= 0) {
    const BNode& ch = nodes[src];
    ref = ch.left < 0 ? ~ch.first : pair_index(ch);
    for (int q = 0; q < 3; ++q) {
      lo[q] = ch.lo[q];
      hi[q] = ch.hi[q];
    }
  }
  if (FMT == RT_NODE_F4) {
    // words: lox, hix, loy, hiy, loz, hiz (component c = slot c), ref, meta
    uint32_t* w = reinterpret_cast<uint32_t*>(wn + slot);
    for (int q = 0; q < 3; ++q) {
      // unused slots: lo = hi = +inf (never entered; also masked out)
      w[8 * q + c] = __float_as_uint(src >= 0 ? lo[q] : INFINITY);
      w[8 * q + 4 + c] = __float_as_uint(src >= 0 ? hi[q] : INFINITY);
    }
    w[24 + c] = (uint32_t)ref;
    w[28 + c] = c == 0 ? mask : 0u;
  } else {
    // words: origin xyz and meta, then byte c of words 4-6 (qlo xyz) and 7-9
    // (qhi xyz) for slot c, two zero words, ref
    QNode4* o = reinterpret_cast<QNode4*>(wn) + slot;
    uint32_t* w = reinterpret_cast<uint32_t*>(o);
    unsigned char* b = reinterpret_cast<unsigned char*>(o);
    int e[3];
    for (int q = 0; q < 3; ++q) {
      e[q] = quant_exp(nd.lo[q], nd.hi[q]);
      const float sc = pow2f(e[q]);
      b[4 * (4 + q) + c] = (unsigned char)(src >= 0 ? quant_lo(lo[q], nd.lo[q], sc) : 0u);
      b[4 * (7 + q) + c] = (unsigned char)(src >= 0 ? quant_hi(hi[q], nd.lo[q], sc) : 0u);
    }
    w[12 + c] = (uint32_t)ref;
    if (c == 0) {
      const unsigned meta = (unsigned)(e[0] + 127) | ((unsigned)(e[1] + 127) << 8) |
                            ((unsigned)(e[2] + 127) << 16) | (mask << 24);
      w[0] = __float_as_uint(nd.lo[0]);
      w[1] = __float_as_uint(nd.lo[1]);
      w[2] = __float_as_uint(nd.lo[2]);
      w[3] = meta;
    } else if (c >= 2) {
      w[8 + c] = 0u;  // words 10 and 11
    }
  }
}

}  // namespace

#define HIPCHECK(call)                                  \
  do {                                                  \
    int _rc = check_hip((call), #call);                 \
    if (_rc != RT_OK) return _rc;                       \
  } while (0)

namespace {

// Pinned, device-mapped record that k_finish fills at the end of the build.
struct HostRecord {
  int32_t* host = nullptr;
  int32_t* dev = nullptr;
};

// The handle's record, made on its first build (freed with its buffers).
int host_record(Buffers& B, HostRecord& r) {
  if (!B.rec_host) {
    int rc = check_hip(hipHostMalloc((void**)&B.rec_host, 64, hipHostMallocMapped), "hipHostMalloc");
    if (rc != RT_OK) return rc;
    rc = check_hip(hipHostGetDevicePointer((void**)&B.rec_dev, B.rec_host, 0),
                   "hipHostGetDevicePointer");
    if (rc != RT_OK) {
      (void)hipHostFree(B.rec_host);
      B.rec_host = nullptr;
      return rc;
    }
    B.rec_host[0] = 0;
    B.rec_seq = 0;
  }
  r.host = B.rec_host;
  r.dev = B.rec_dev;
  return RT_OK;
}

// Waits until the device has written sequence number seq; falls back to a
// stream synchronisation (which reports device errors) after a while.
int wait_record(const HostRecord& r, int seq, hipStream_t s) {
  volatile int32_t* h = r.host;
  for (long spin = 0; spin < 20000000; ++spin) {
    if (__atomic_load_n(&h[0], __ATOMIC_ACQUIRE) == seq) return RT_OK;
    if (spin > 1000) __builtin_ia32_pause();
  }
  int rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc != RT_OK) return rc;
  if (__atomic_load_n(&h[0], __ATOMIC_ACQUIRE) != seq)
    return set_error(RT_EHIP, "rt_build: build record not written");
  return RT_OK;
}

}  // namespace

int build_tree(Buffers& B, const float* tris, int64_t n64, const rt_split_params& p,
               hipStream_t s, rt_bvh_info* info) {
  int seq = 0;
  int rc = build_enqueue(B, tris, n64, p, s, &seq);
  if (rc != RT_OK) return rc;
  return build_complete(B, n64, p, seq, s, info);
}

int build_enqueue(Buffers& B, const float* tris, int64_t n64, const rt_split_params& p,
                  hipStream_t s, int* seq_out) {
  const int n = (int)n64;
  HostRecord rec;
  {
    int rc = host_record(B, rec);
    if (rc != RT_OK) return rc;
  }
  const int seq = ++B.rec_seq;
  *seq_out = seq;
  BuildState* st = reinterpret_cast<BuildState*>(B.counters);

  Ctx X;
  X.nodes = B.nodes;
  X.recs[0] = B.recs_a;
  X.recs[1] = B.recs_b;
  X.perm = B.perm;
  X.st = st;
  X.used = B.used;
  X.mfront[0] = B.mfront;
  X.mfront[1] = B.mfront + n;
  X.sfront = B.sfront;
  X.items[0] = B.aitems;
  X.items[1] = B.aitems + B.item_cap;
  X.ccnt[0] = B.accnt;
  X.ccnt[1] = B.accnt + (size_t)B.item_cap * 3 * RT_MAX_BINS;
  X.abin_stride = bins_bytes(RT_MAX_BINS, true);
  X.abins[0] = B.abins;
  X.abins[1] = B.abins + (size_t)B.anode_cap * kBinReplicas * X.abin_stride;
  X.n = n;
  X.item_cap = (int)B.item_cap;
  X.anode_cap = (int)B.anode_cap;
  // big-node levels: enough for balanced halvings down to kBigNode, plus one
  int la = 0;
  if (n > kBigNode) {
    while ((int64_t(kBigNode) << la) < n) ++la;
    la = std::min(la + 1, kMaxPhaseLevels - 1);
  }
  // medium-node passes: balanced halvings from kBigNode down to kRegNode, plus two
  int lm = 0;
  if (n > kRegNode) {
    while ((kRegNode << lm) < std::min(n, kBigNode)) ++lm;
    lm = std::min(lm + 2, kMaxPhaseLevels - 1);
  }
  X.la = la;
  X.lm = lm;
  BuildConst& C = X.C;
  C.alpha = (double)p.alpha;
  C.t_isect = (double)p.t_isect;
  C.t_trav = (double)p.t_trav;
  for (int a = 0; a < 3; ++a) C.src[a] = (double)p.src[a];
  C.inv_l2 = 0.0;  // read from the device state by the kernels
  C.max_leaf = p.max_leaf;
  C.nbins = p.nbins;
  C.d_mode = p.d_mode;
  C.d_norm = p.d_norm;
  C.max_depth = p.max_depth;
  C.depth_limit = p.depth_limit;
  const int Bn = p.nbins;

  // the state's starting values: set once on new buffers, then by the end of
  // every build (finish_build)
  if (!B.state_ready) hipLaunchKernelGGL(k_init, dim3(1), dim3(256), 0, s, B.counters, B.root_box, n);
  B.state_ready = false;  // until this build has ended
  const int pb = 256;
  hipLaunchKernelGGL(k_prep, dim3((n + pb - 1) / pb), dim3(pb), 0, s, X, tris, B.root_box);
  const size_t lds_abin = a_copies(Bn, kABinThreads) * bins_bytes(Bn, true);
  const size_t lds_asplit = bins_bytes(Bn, true);
  for (int l = 0; l < la; ++l) {
    hipLaunchKernelGGL(k_a_bin, dim3(X.item_cap), dim3(kABinThreads), lds_abin, s, X, l);
    hipLaunchKernelGGL(k_a_split, dim3(X.item_cap), dim3(kAThreads), lds_asplit, s, X, l);
  }
  // one wave per window of facet positions
  const int m_windows = (n + kMWindow - 1) / kMWindow;
  for (int m = 0; m < lm; ++m)
    hipLaunchKernelGGL(k_m, dim3(m_windows), dim3(64), bins_bytes(Bn, true), s, X, m);
  const int s_win = std::min(64, 2 * (p.max_leaf + 1));
  const int s_windows = (n + s_win - 1) / s_win;
  hipLaunchKernelGGL(k_s, dim3(s_windows), dim3(64), s_wave_bytes(Bn), s, X);
  // compaction and traversal data
  const int nb = std::max(n - 1, 0);  // split boundaries
  const int nblk = std::max(1, (nb + kScanBlock - 1) / kScanBlock);
  int32_t* bsum = B.bsum;
  int32_t* bmax = B.bsum + (n / kScanBlock + 1);
  hipLaunchKernelGGL(k_count, dim3(nblk), dim3(kScanBlock), 0, s, B.used, nb, bsum, bmax);
  hipLaunchKernelGGL(k_rank, dim3(nblk), dim3(kScanBlock), 0, s, B.used, nb, bsum, bmax, B.rank, st);
  const int eb = 256;
  hipLaunchKernelGGL(k_emit, dim3((n + eb - 1) / eb), dim3(eb), 0, s, B.nodes, st, B.used, B.rank,
                     B.perm, tris, B.cnodes, B.tnodes, B.tfacets);
  const int64_t max_nodes = std::max(1, 2 * n - 1);
  const dim3 cgrid((unsigned)((4 * max_nodes + eb - 1) / eb));  // four lanes per node
  if (p.node_format == RT_NODE_F4)
    hipLaunchKernelGGL(k_collapse<RT_NODE_F4>, cgrid, dim3(eb), 0, s, B.cnodes, st, B.wnodes);
  else if (p.node_format == RT_NODE_Q4)
    hipLaunchKernelGGL(k_collapse<RT_NODE_Q4>, cgrid, dim3(eb), 0, s, B.cnodes, st, B.wnodes);
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, st, B.root_box, B.cnodes, rec.dev, seq);
  HIPCHECK(hipGetLastError());
  return RT_OK;
}

int build_complete(Buffers& B, int64_t n64, const rt_split_params& p, int seq, hipStream_t s,
                   rt_bvh_info* info) {
  const int n = (int)n64;
  const HostRecord rec{B.rec_host, B.rec_dev};
  {
    int rc = wait_record(rec, seq, s);
    if (rc != RT_OK) return rc;
  }
  B.state_ready = true;  // the build's end set the state back
  const int32_t* h = rec.host;
  if (h[3]) return set_error(RT_EINVAL, "rt_build: a facet has a non-finite vertex");
  if (h[4]) return set_error(RT_EHIP, "rt_build: internal capacity check failed (code " +
                                          std::to_string(h[4]) + ")");
  const int total = h[1];
  const int n_internal = (total - 1) / 2;
  info->n_tris = n;
  info->n_nodes = total;
  info->n_internal = n_internal;
  info->n_leaves = total - n_internal;
  info->depth = h[2];  // deepest leaf depth (root alone = 0)
  info->n_levels = h[2] + 1;
  for (int q = 0; q < 3; ++q) {
    int32_t lo = h[5 + q], hi = h[8 + q];
    std::memcpy(&info->root_lo[q], &lo, 4);
    std::memcpy(&info->root_hi[q], &hi, 4);
  }
  const int64_t node_bytes = p.node_format == RT_NODE_F4 ? sizeof(FNode4)
                             : p.node_format == RT_NODE_Q4 ? sizeof(QNode4) : sizeof(TNode);
  info->node_format = p.node_format;
  info->n_trace_nodes = std::max(n_internal, 1);
  info->trace_bytes = node_bytes * std::max(n_internal, 1) + (int64_t)sizeof(TFacet) * n;
  return RT_OK;
}

}  // namespace rt

// ---- tree statistics (rt_bvh_stats) ----------------------------------------
// Eq. (1) cost of the finished tree, Sec. II-B: internal nodes add
// S(n) t_trav, leaves S(l) k_l t_i (S the surface area of the node's volume),
// both sums divided by S(root) at the end; and the histogram of leaf sizes.
// A fixed grid walks the nodes with a fixed stride and reduces in a fixed
// order, so the same tree gives the same bits.
namespace rt {
namespace {

constexpr int kStatThreads = 256;

__device__ inline double box_area(const BNode& nd) {
  const double wx = (double)nd.hi[0] - (double)nd.lo[0];
  const double wy = (double)nd.hi[1] - (double)nd.lo[1];
  const double wz = (double)nd.hi[2] - (double)nd.lo[2];
  return 2.0 * (wx * wy + wy * wz + wz * wx);
}

__device__ inline int leaf_bucket(int c) {
  if (c <= 8) return c - 1;
  if (c > 1024) return RT_LEAF_HIST - 1;
  return 5 + (31 - __clz(c - 1));
}

// part[blk][2]: this block's internal and leaf sums; hist[blk][kStatHist]:
// its leaf counts per bucket and (last word) its largest leaf.
__global__ __launch_bounds__(kStatThreads) void k_tree_stats(const BNode* __restrict__ nodes,
                                                            int64_t nn, double t_i,
                                                            double t_trav,
                                                            double* __restrict__ part,
                                                            double* __restrict__ hist) {
  __shared__ double s_int[kStatThreads], s_leaf[kStatThreads];
  __shared__ int s_hist[kStatHist];
  if (threadIdx.x < kStatHist) s_hist[threadIdx.x] = 0;
  __syncthreads();
  double a_int = 0.0, a_leaf = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kStatThreads + threadIdx.x; i < nn;
       i += (int64_t)kStatBlocks * kStatThreads) {
    const BNode nd = nodes[i];
    const double s = box_area(nd);
    if (nd.left >= 0) {
      a_int += s * t_trav;
    } else {
      a_leaf += s * ((double)nd.count * t_i);
      atomicAdd(&s_hist[leaf_bucket(nd.count)], 1);
      atomicMax(&s_hist[kStatHist - 1], nd.count);
    }
  }
  s_int[threadIdx.x] = a_int;
  s_leaf[threadIdx.x] = a_leaf;
  __syncthreads();
  for (int h = kStatThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_int[threadIdx.x] += s_int[threadIdx.x + h];
      s_leaf[threadIdx.x] += s_leaf[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_int[0];
    part[2 * blockIdx.x + 1] = s_leaf[0];
  }
  if (threadIdx.x < kStatHist) hist[blockIdx.x * kStatHist + threadIdx.x] = (double)s_hist[threadIdx.x];
}

// out[0..1]: the internal and leaf sums over the blocks in block order;
// out[2..]: the histogram summed, the largest leaf as a maximum.
__global__ void k_tree_stats_sum(const double* __restrict__ part, const double* __restrict__ hist,
                                 double* __restrict__ out) {
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int k = 0; k < kStatBlocks; ++k) {
      a += part[2 * k];
      b += part[2 * k + 1];
    }
    out[0] = a;
    out[1] = b;
  }
  if (threadIdx.x < kStatHist) {
    double h = 0.0;
    for (int k = 0; k < kStatBlocks; ++k) {
      const double v = hist[k * kStatHist + threadIdx.x];
      h = threadIdx.x == kStatHist - 1 ? fmax(h, v) : h + v;
    }
    out[2 + threadIdx.x] = h;
  }
}

}  // namespace

int tree_stats(const Buffers& B, int64_t n_nodes, double t_isect, double t_trav,
               rt_bvh_info* info) {
  double* part = B.stat_work;
  double* hist = part + 2 * kStatBlocks;
  double* out = hist + kStatBlocks * kStatHist;
  HIPCHECK(hipDeviceSynchronize());
  hipLaunchKernelGGL(k_tree_stats, dim3(kStatBlocks), dim3(kStatThreads), 0, 0, B.cnodes, n_nodes,
                     t_isect, t_trav, part, hist);
  hipLaunchKernelGGL(k_tree_stats_sum, dim3(1), dim3(64), 0, 0, part, hist, out);
  HIPCHECK(hipGetLastError());
  BNode root;
  double h[2 + kStatHist];
  HIPCHECK(hipMemcpy(h, out, sizeof(h), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(&root, B.cnodes, sizeof(root), hipMemcpyDeviceToHost));
  const double wx = (double)root.hi[0] - (double)root.lo[0];
  const double wy = (double)root.hi[1] - (double)root.lo[1];
  const double wz = (double)root.hi[2] - (double)root.lo[2];
  const double s_root = 2.0 * (wx * wy + wy * wz + wz * wx);
  info->has_stats = 1;
  info->root_area = s_root;
  if (s_root > 0.0) {
    info->tree_cost = h[0] / s_root + h[1] / s_root;
  } else {  // every volume degenerate: each ratio is taken as 1
    info->tree_cost = t_trav * (double)info->n_internal + t_isect * (double)info->n_tris;
  }
  for (int k = 0; k < RT_LEAF_HIST; ++k) info->leaf_hist[k] = (int64_t)h[2 + k];
  info->max_leaf_count = (int32_t)h[2 + RT_LEAF_HIST];
  return RT_OK;
}

}  // namespace rt
