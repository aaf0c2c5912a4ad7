// Ray traversal, closest hit and specular re-launch (Sec. III-B).
//
// One ray per lane.  A ray visits a node by fetching its 64-byte record and
// testing both child volumes (closed slab test, robust to zero direction
// components); a child is entered when its slab interval meets
// [tmin, t_best], so hits already found shrink the action range and cull the
// volumes behind them.  Leaves test their facets with the watertight
// ray-triangle test in float32; the nearest hit wins, ties to the smaller
// facet id.  After a hit the ray may be reflected about the facet plane and
// traced again; the path length is summed in float64.
#include <hip/hip_runtime.h>
#include <climits>

#include <algorithm>
#include <atomic>

#include "rt_internal.h"

namespace rt {
namespace {

// Stand-in for 1/0 in the slab test: a power of two, so that o * kBig is
// exact and a zero direction component needs no rounding margin.
constexpr float kBig = 0x1p100f;
// Slab far distances grow by 2 * gamma(3) so rounding never rejects a volume
// the exact ray meets (Ize, "Robust BVH ray traversal", JCGT 2013).
constexpr float kFarGrow = 1.0f + 2.0f * (3.0f * 5.9604645e-8f) / (1.0f - 3.0f * 5.9604645e-8f);

struct RayPre {
  float ox, oy, oz, dx, dy, dz;
  float ix, iy, iz;  // 1/d (kBig for a zero component)
  // Fused-slab offsets: a plane at coordinate p is crossed at
  // fma(p, i, a), with a = -o * i rounded down for the plane the ray enters
  // first and up for the one it leaves by, so the single rounding of the
  // fused form can only widen the interval.  For the 4-wide float32 nodes
  // a0 / a1 belong to the lo / hi planes; for the 8-bit nodes, which pick
  // the entry and exit planes by the ray's signs, a0 is -o i rounded down
  // and a1 rounded up.
  float a0x, a1x, a0y, a1y, a0z, a1z;
  float tmin, tmax;
  int kx, ky, kz;    // axis permutation of the watertight test
  float sx, sy, sz;  // its shear constants
};

__device__ inline float sel(float x, float y, float z, int k) {
  return k == 0 ? x : (k == 1 ? y : z);
}

// Offsets of one axis.  a = fl(-o i) and its rounding error e = -o i - a,
// which one fused multiply-add gives exactly; the lo-plane offset of a ray
// with i > 0 is the float nearest below or at -o i and its hi-plane offset
// the float nearest above or at it (the reverse for i < 0), so
// fma(p, i, offset), rounded once, errs from the exact (p - o) i only by u
// of its own size (u = 2^-24) -- the relative error the far-distance growth
// already covers -- plus at most one ulp of o i toward the outside.  A zero
// component has i = kBig, a power of two: the product is exact (e = 0).
template <bool BY_SIGN>
__device__ inline void offsets(float o, float i, float& a0, float& a1) {
  const float a = -(o * i);
  const float e = fmaf(-o, i, -a);
  const float down = e < 0.f ? nextafterf(a, -INFINITY) : a;
  const float up = e > 0.f ? nextafterf(a, INFINITY) : a;
  a0 = BY_SIGN || i > 0.f ? down : up;
  a1 = BY_SIGN || i > 0.f ? up : down;
}

template <int FMT>
__device__ inline RayPre prepare(float ox, float oy, float oz, float dx, float dy, float dz,
                                 float tmin, float tmax) {
  RayPre r;
  r.ox = ox; r.oy = oy; r.oz = oz;
  r.dx = dx; r.dy = dy; r.dz = dz;
  r.ix = dx != 0.f ? 1.f / dx : kBig;
  r.iy = dy != 0.f ? 1.f / dy : kBig;
  r.iz = dz != 0.f ? 1.f / dz : kBig;
  if constexpr (FMT != RT_NODE_BIN2) {
    constexpr bool kBySign = FMT == RT_NODE_Q4;
    offsets<kBySign>(ox, r.ix, r.a0x, r.a1x);
    offsets<kBySign>(oy, r.iy, r.a0y, r.a1y);
    offsets<kBySign>(oz, r.iz, r.a0z, r.a1z);
  }
  r.tmin = tmin;
  r.tmax = tmax;
  float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
  int kz = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  float dkz = sel(dx, dy, dz, kz);
  if (dkz < 0.f) { int t = kx; kx = ky; ky = t; }
  r.kx = kx; r.ky = ky; r.kz = kz;
  r.sx = sel(dx, dy, dz, kx) / dkz;
  r.sy = sel(dx, dy, dz, ky) / dkz;
  r.sz = 1.f / dkz;
  return r;
}

// Closed slab test of one box against [tlo, thi]; returns the entry distance
// through tnear.  FUSED crosses each plane with one fused multiply-add and
// the ray's rounded offsets (six fewer operations per box, six more
// registers per ray): the wide nodes, whose child tests dominate their
// visits, use it; the binary nodes keep (p - o) / d, whose lower register
// count keeps one more wave per SIMD resident.
template <bool FUSED>
__device__ inline bool slab(const RayPre& r, float lox, float hix, float loy, float hiy,
                            float loz, float hiz, float tlo, float thi, float& tnear) {
  float x0, x1, y0, y1, z0, z1;
  if constexpr (FUSED) {
    x0 = fmaf(lox, r.ix, r.a0x); x1 = fmaf(hix, r.ix, r.a1x);
    y0 = fmaf(loy, r.iy, r.a0y); y1 = fmaf(hiy, r.iy, r.a1y);
    z0 = fmaf(loz, r.iz, r.a0z); z1 = fmaf(hiz, r.iz, r.a1z);
  } else {
    x0 = (lox - r.ox) * r.ix; x1 = (hix - r.ox) * r.ix;
    y0 = (loy - r.oy) * r.iy; y1 = (hiy - r.oy) * r.iy;
    z0 = (loz - r.oz) * r.iz; z1 = (hiz - r.oz) * r.iz;
  }
  float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fmaxf(fminf(z0, z1), tlo));
  float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fmaxf(z0, z1)) * kFarGrow;
  tf = fminf(tf, thi);
  tnear = tn;
  return tn <= tf;
}

// Watertight ray-triangle test (Woop, Benthin, Wald, JCGT 2013) in float32,
// two-sided.  The edge functions are products rounded one by one, so a
// shared edge gives exactly opposite values in its two facets.
__device__ inline bool facet_test(const RayPre& r, const float4& p0, const float4& p1,
                                  const float4& p2, float& t, float& u, float& v) {
#pragma clang fp contract(off)
  const float ax = p0.x - r.ox, ay = p0.y - r.oy, az = p0.z - r.oz;
  const float bx = p1.x - r.ox, by = p1.y - r.oy, bz = p1.z - r.oz;
  const float cx = p2.x - r.ox, cy = p2.y - r.oy, cz = p2.z - r.oz;
  const float Akz = sel(ax, ay, az, r.kz), Bkz = sel(bx, by, bz, r.kz), Ckz = sel(cx, cy, cz, r.kz);
  const float Ax = sel(ax, ay, az, r.kx) - r.sx * Akz;
  const float Ay = sel(ax, ay, az, r.ky) - r.sy * Akz;
  const float Bx = sel(bx, by, bz, r.kx) - r.sx * Bkz;
  const float By = sel(bx, by, bz, r.ky) - r.sy * Bkz;
  const float Cx = sel(cx, cy, cz, r.kx) - r.sx * Ckz;
  const float Cy = sel(cx, cy, cz, r.ky) - r.sy * Ckz;
  const float U = Cx * By - Cy * Bx;
  const float V = Ax * Cy - Ay * Cx;
  const float W = Bx * Ay - By * Ax;
  if ((U < 0.f || V < 0.f || W < 0.f) && (U > 0.f || V > 0.f || W > 0.f)) return false;
  const float det = U + V + W;
  if (det == 0.f) return false;
  const float T = U * (r.sz * Akz) + V * (r.sz * Bkz) + W * (r.sz * Ckz);
  const float rcp = 1.f / det;
  t = T * rcp;
  u = V * rcp;
  v = W * rcp;
  return true;
}

// ---- compensated float32 arithmetic (value = hi + lo) ----------------------
// Error-free sum (Knuth) and product (fused multiply-add) give each operation's
// rounding error exactly, so a short chain of them carries about twice the
// float32 precision without leaving float32.
struct F2 {
  float hi, lo;
};

__device__ inline F2 two_sum(float a, float b) {
#pragma clang fp contract(off)
  float s = a + b;
  float bb = s - a;
  float e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ inline F2 fast_two_sum(float a, float b) {  // |a| >= |b|
#pragma clang fp contract(off)
  float s = a + b;
  return {s, b - (s - a)};
}
__device__ inline F2 two_prod(float a, float b) {
#pragma clang fp contract(off)
  float p = a * b;
  return {p, fmaf(a, b, -p)};
}
__device__ inline F2 f2_add(F2 a, F2 b) {
#pragma clang fp contract(off)
  F2 s = two_sum(a.hi, b.hi);
  F2 t = two_sum(a.lo, b.lo);
  float lo = s.lo + t.hi;
  F2 u = fast_two_sum(s.hi, lo);
  return fast_two_sum(u.hi, u.lo + t.lo);
}
__device__ inline F2 f2_neg(F2 a) { return {-a.hi, -a.lo}; }
__device__ inline F2 f2_mul(F2 a, F2 b) {
#pragma clang fp contract(off)
  F2 p = two_prod(a.hi, b.hi);
  float lo = p.lo + (a.hi * b.lo + a.lo * b.hi);
  return fast_two_sum(p.hi, lo);
}
__device__ inline F2 f2_mulf(F2 a, float b) {
#pragma clang fp contract(off)
  F2 p = two_prod(a.hi, b);
  return fast_two_sum(p.hi, p.lo + a.lo * b);
}
__device__ inline float f2_div(F2 a, F2 b) {
#pragma clang fp contract(off)
  float q = a.hi / b.hi;
  // one correction step: r = a - q b, q += r / b
  F2 qb = f2_mulf(b, q);
  F2 r = f2_add(a, f2_neg(qb));
  return q + (r.hi + r.lo) / b.hi;
}

// Unnormalised facet normal (v1 - v0) x (v2 - v0) in compensated float32.
struct N2 {
  F2 x, y, z;
};
__device__ inline N2 facet_normal(const float4& p0, const float4& p1, const float4& p2) {
  const F2 e1x = two_sum(p1.x, -p0.x), e1y = two_sum(p1.y, -p0.y), e1z = two_sum(p1.z, -p0.z);
  const F2 e2x = two_sum(p2.x, -p0.x), e2y = two_sum(p2.y, -p0.y), e2z = two_sum(p2.z, -p0.z);
  N2 n;
  n.x = f2_add(f2_mul(e1y, e2z), f2_neg(f2_mul(e1z, e2y)));
  n.y = f2_add(f2_mul(e1z, e2x), f2_neg(f2_mul(e1x, e2z)));
  n.z = f2_add(f2_mul(e1x, e2y), f2_neg(f2_mul(e1y, e2x)));
  return n;
}

__device__ inline F2 f2_div2(F2 a, F2 b) {  // quotient kept as hi + lo
#pragma clang fp contract(off)
  float q = a.hi / b.hi;
  F2 r = f2_add(a, f2_neg(f2_mulf(b, q)));
  return fast_two_sum(q, (r.hi + r.lo) / b.hi);
}

// Distance to the facet's plane along the ray, t = n.(v0 - o) / n.d, with the
// edge vectors, the normal and both dot products carried in compensated
// float32: the result keeps float32 relative accuracy even when the facet is
// much larger than t (a reflected ray leaving a wall next to a km-wide
// ground facet).
__device__ inline float plane_t(const N2& n, const float4& p0, float ox, float oy, float oz,
                                float dx, float dy, float dz) {
  const F2 wx = two_sum(p0.x, -ox), wy = two_sum(p0.y, -oy), wz = two_sum(p0.z, -oz);
  const F2 num = f2_add(f2_add(f2_mul(n.x, wx), f2_mul(n.y, wy)), f2_mul(n.z, wz));
  const F2 den = f2_add(f2_add(f2_mulf(n.x, dx), f2_mulf(n.y, dy)), f2_mulf(n.z, dz));
  return f2_div(num, den);
}

// Specular reflection r = d - 2 (d.n) / (n.n) n, evaluated in compensated
// float32 and rounded once per component.
__device__ inline void reflect(const N2& n, float& dx, float& dy, float& dz) {
  const F2 dn = f2_add(f2_add(f2_mulf(n.x, dx), f2_mulf(n.y, dy)), f2_mulf(n.z, dz));
  const F2 nn = f2_add(f2_add(f2_mul(n.x, n.x), f2_mul(n.y, n.y)), f2_mul(n.z, n.z));
  F2 k = f2_div2(dn, nn);
  k.hi *= 2.f;
  k.lo *= 2.f;
  const F2 rx = f2_add(F2{dx, 0.f}, f2_neg(f2_mul(k, n.x)));
  const F2 ry = f2_add(F2{dy, 0.f}, f2_neg(f2_mul(k, n.y)));
  const F2 rz = f2_add(F2{dz, 0.f}, f2_neg(f2_mul(k, n.z)));
  dx = rx.hi + rx.lo;
  dy = ry.hi + ry.lo;
  dz = rz.hi + rz.lo;
}

struct Hit {
  int id;  // caller's facet id, -1 none
  int pos; // leaf-order position
  float t, u, v;
};

// Stack of pending subtrees, all of it in LDS: lane column layout (entry i
// of a lane at col[i * 64]) so the lanes of a wave hit distinct banks.  No
// private (scratch) memory is used, which would cap the waves in flight.
struct Stack {
  int* col;
  int sp = 0;
  __device__ void push(int r) {
    col[sp * 64] = r;
    ++sp;
  }
  __device__ bool pop(int& r) {
    if (sp == 0) return false;
    --sp;
    r = col[sp * 64];
    return true;
  }
};

__device__ inline void cswap(float& ka, int& ra, float& kb, int& rb) {
  if (kb < ka) {
    const float k = ka;
    ka = kb;
    kb = k;
    const int x = ra;
    ra = rb;
    rb = x;
  }
}

__device__ inline float qbyte(unsigned w, int c) { return (float)((w >> (8 * c)) & 255u); }
// x moved by at least one unit in the last place: down for step -2^-23, up
// for +2^-23 (|x| 2^-23 is one ulp of x or more, and the rounding of the
// fused result cannot come back past it); 0 stays 0.
__device__ inline float outward(float x, float step) { return fmaf(fabsf(x), step, x); }

// Tests the facets of one leaf (positions ~node .. the one tagged last).
template <bool STATS>
__device__ inline void leaf_test(const TFacet* __restrict__ tf, const RayPre& r, int node,
                                 int skip_pos, Hit& h, int& best_id, uint32_t& ntest) {
  for (int k = ~node;; ++k) {
    const TFacet f = tf[k];
    const uint32_t tag = __float_as_uint(f.p0.w);
    const int id = (int)(tag & ~kLastFacet);
    if (k != skip_pos) {
      if (STATS) ++ntest;
      float t, u, v;
      if (facet_test(r, f.p0, f.p1, f.p2, t, u, v) && t >= r.tmin &&
          (t < h.t || (t == h.t && id < best_id))) {
        h.t = t;
        h.u = u;
        h.v = v;
        h.pos = k;
        h.id = id;
        best_id = id;
      }
    }
    if (tag & kLastFacet) break;
  }
}

// The same leaf test shared by the G lanes that trace one ray: lane s of the
// group takes positions first + s, first + s + G, ... .  The round in which a
// lane of the group meets the facet tagged last ends the leaf (lanes after it
// hold the next leaf's facets and drop them; the facet array ends with a
// tagged facet, so no lane that tests reads past it).  The lanes' candidates
// are then merged by the closest-hit rule (smaller t, then smaller facet id),
// a total order, so every lane of the group ends with the hit the serial
// test finds.
template <int G>
__device__ inline void leaf_test_group(const TFacet* __restrict__ tf, int n_tf, const RayPre& r,
                                       int node, int skip_pos, Hit& h, int& best_id) {
  const int lane = threadIdx.x & 63;
  const int sub = lane & (G - 1);
  const int group_lane0 = lane & ~(G - 1);
  float bt = h.t, bu = h.u, bv = h.v;
  int bid = best_id, bpos = h.pos;
  for (int k0 = ~node;; k0 += G) {
    const int k = k0 + sub;
    const bool inside = k < n_tf;
    const TFacet f = tf[inside ? k : n_tf - 1];
    const uint32_t tag = __float_as_uint(f.p0.w);
    const unsigned long long ends = __ballot(inside && (tag & kLastFacet) != 0u);
    const unsigned long long mine =
        G == 64 ? ends : (ends >> group_lane0) & ((1ull << (G & 63)) - 1ull);
    const int last_sub = mine ? __ffsll((long long)mine) - 1 : G - 1;
    if (inside && sub <= last_sub && k != skip_pos) {
      const int id = (int)(tag & ~kLastFacet);
      float t, u, v;
      if (facet_test(r, f.p0, f.p1, f.p2, t, u, v) && t >= r.tmin &&
          (t < bt || (t == bt && id < bid))) {
        bt = t;
        bu = u;
        bv = v;
        bpos = k;
        bid = id;
      }
    }
    if (mine) break;
  }
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const float ot = __shfl_xor(bt, off), ou = __shfl_xor(bu, off), ov = __shfl_xor(bv, off);
    const int oid = __shfl_xor(bid, off), opos = __shfl_xor(bpos, off);
    if (ot < bt || (ot == bt && oid < bid)) {
      bt = ot;
      bu = ou;
      bv = ov;
      bid = oid;
      bpos = opos;
    }
  }
  h.t = bt;
  h.u = bu;
  h.v = bv;
  h.pos = bpos;
  if (bpos >= 0) h.id = bid;
  best_id = bid;
}

template <int FMT, bool STATS, int G = 1>
__device__ __forceinline__ Hit closest(const void* __restrict__ nodes, const TFacet* __restrict__ tf,
                       const RayPre& r, int skip_pos, int* stack_col, uint32_t& nvis,
                       uint32_t& ntest, int n_tf = 0) {
  Stack st;
  st.col = stack_col;
  int node = 0;
  Hit h;
  h.id = -1;
  h.pos = -1;
  h.t = r.tmax;
  h.u = h.v = 0.f;
  int best_id = 0x7fffffff;  // h.id, or the largest id while there is no hit
  if constexpr (FMT == RT_NODE_BIN2) {
    // speculative traversal: a lane parks the first leaf it reaches and keeps
    // descending; leaves are tested once every lane has one parked
    constexpr int kDone = INT_MIN;
    int leaf = 0;  // parked leaf (< 0), 0 none
    while (node != kDone) {
      while (node >= 0) {
        if (STATS) ++nvis;
        const TNode nd = static_cast<const TNode*>(nodes)[node];
        float n0, n1;
        const bool h0 = slab<false>(r, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.c.x, nd.c.y, r.tmin, h.t, n0);
        const bool h1 = slab<false>(r, nd.b.x, nd.b.y, nd.b.z, nd.b.w, nd.c.z, nd.c.w, r.tmin, h.t, n1);
        if (h0 && h1) {
          const bool first0 = n0 <= n1;
          st.push(first0 ? nd.d.y : nd.d.x);
          node = first0 ? nd.d.x : nd.d.y;
        } else if (h0) {
          node = nd.d.x;
        } else if (h1) {
          node = nd.d.y;
        } else if (!st.pop(node)) {
          node = kDone;
        }
        if (node < 0 && node != kDone && leaf == 0) {
          leaf = node;
          if (!st.pop(node)) node = kDone;
        }
        if (__ballot(leaf == 0 && node != kDone) == 0ull) break;
      }
      while (leaf < 0) {
        if constexpr (G == 1) leaf_test<STATS>(tf, r, leaf, skip_pos, h, best_id, ntest);
        else leaf_test_group<G>(tf, n_tf, r, leaf, skip_pos, h, best_id);
        leaf = 0;
        if (node < 0 && node != kDone) {
          leaf = node;
          if (!st.pop(node)) node = kDone;
        }
      }
    }
    return h;
  }
  // 4-wide nodes, the same speculative order: children sorted near first,
  // the first leaf a lane reaches is parked while it keeps descending
  constexpr int kDone = INT_MIN;
  int leaf = 0;
  while (node != kDone) {
    while (node >= 0) {
      if (STATS) ++nvis;
      float key[4];
      int ref[4];
      unsigned mask;
      if constexpr (FMT == RT_NODE_F4) {
        const FNode4 nd = static_cast<const FNode4*>(nodes)[node];
        mask = nd.meta.x;
        const float lx[4] = {nd.lox.x, nd.lox.y, nd.lox.z, nd.lox.w};
        const float hx[4] = {nd.hix.x, nd.hix.y, nd.hix.z, nd.hix.w};
        const float ly[4] = {nd.loy.x, nd.loy.y, nd.loy.z, nd.loy.w};
        const float hy[4] = {nd.hiy.x, nd.hiy.y, nd.hiy.z, nd.hiy.w};
        const float lz[4] = {nd.loz.x, nd.loz.y, nd.loz.z, nd.loz.w};
        const float hz[4] = {nd.hiz.x, nd.hiz.y, nd.hiz.z, nd.hiz.w};
        const int rr[4] = {nd.ref.x, nd.ref.y, nd.ref.z, nd.ref.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          float tn;
          const bool in = slab<true>(r, lx[c], hx[c], ly[c], hy[c], lz[c], hz[c], r.tmin, h.t, tn);
          key[c] = (in & (((mask >> c) & 1u) != 0u)) ? tn : INFINITY;
          ref[c] = rr[c];
        }
      } else {
        const QNode4 nd = static_cast<const QNode4*>(nodes)[node];
        const unsigned meta = __float_as_uint(nd.h.w);
        mask = meta >> 24;
        // The builder guarantees that the exact (unrounded) h + q 2^e encloses
        // every child.  A child plane is crossed at q (2^e i) + (h i - o i):
        // 2^e i is exact (a power of two times i), and the node term is formed
        // once per axis from the ray's directed offsets and moved outward by
        // one more unit in the last place for its own rounding, so one fused
        // multiply-add per plane errs only by u of the crossing distance.
        const float six = __uint_as_float((meta << 23) & 0x7f800000u) * r.ix;
        const float siy = __uint_as_float((meta << 15) & 0x7f800000u) * r.iy;
        const float siz = __uint_as_float((meta << 7) & 0x7f800000u) * r.iz;
        const float cnx = outward(fmaf(nd.h.x, r.ix, r.a0x), -0x1p-23f);
        const float cfx = outward(fmaf(nd.h.x, r.ix, r.a1x), 0x1p-23f);
        const float cny = outward(fmaf(nd.h.y, r.iy, r.a0y), -0x1p-23f);
        const float cfy = outward(fmaf(nd.h.y, r.iy, r.a1y), 0x1p-23f);
        const float cnz = outward(fmaf(nd.h.z, r.iz, r.a0z), -0x1p-23f);
        const float cfz = outward(fmaf(nd.h.z, r.iz, r.a1z), 0x1p-23f);
        // the bytes of the plane each child is entered by and left by
        const bool px = r.ix > 0.f, py = r.iy > 0.f, pz = r.iz > 0.f;
        const unsigned enx = px ? nd.qa.x : nd.qa.w, exx = px ? nd.qa.w : nd.qa.x;
        const unsigned eny = py ? nd.qa.y : nd.qb.x, exy = py ? nd.qb.x : nd.qa.y;
        const unsigned enz = pz ? nd.qa.z : nd.qb.y, exz = pz ? nd.qb.y : nd.qa.z;
        const int rr[4] = {nd.ref.x, nd.ref.y, nd.ref.z, nd.ref.w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float tnx = fmaf(qbyte(enx, c), six, cnx), tfx = fmaf(qbyte(exx, c), six, cfx);
          const float tny = fmaf(qbyte(eny, c), siy, cny), tfy = fmaf(qbyte(exy, c), siy, cfy);
          const float tnz = fmaf(qbyte(enz, c), siz, cnz), tfz = fmaf(qbyte(exz, c), siz, cfz);
          const float tn = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, r.tmin));
          const float tf = fminf(fminf(fminf(tfx, tfy), tfz) * kFarGrow, h.t);
          key[c] = ((tn <= tf) & (((mask >> c) & 1u) != 0u)) ? tn : INFINITY;
          ref[c] = rr[c];
        }
      }
      // nearest first
      cswap(key[0], ref[0], key[1], ref[1]);
      cswap(key[2], ref[2], key[3], ref[3]);
      cswap(key[0], ref[0], key[2], ref[2]);
      cswap(key[1], ref[1], key[3], ref[3]);
      cswap(key[1], ref[1], key[2], ref[2]);
      if (key[0] == INFINITY) {
        if (!st.pop(node)) node = kDone;
      } else {
        if (key[3] != INFINITY) st.push(ref[3]);
        if (key[2] != INFINITY) st.push(ref[2]);
        if (key[1] != INFINITY) st.push(ref[1]);
        node = ref[0];
      }
      if (node < 0 && node != kDone && leaf == 0) {
        leaf = node;
        if (!st.pop(node)) node = kDone;
      }
      if (__ballot(leaf == 0 && node != kDone) == 0ull) break;
    }
    while (leaf < 0) {
      if constexpr (G == 1) leaf_test<STATS>(tf, r, leaf, skip_pos, h, best_id, ntest);
      else leaf_test_group<G>(tf, n_tf, r, leaf, skip_pos, h, best_id);
      leaf = 0;
      if (node < 0 && node != kDone) {
        leaf = node;
        if (!st.pop(node)) node = kDone;
      }
    }
  }
  return h;
}

__device__ inline void store_hit(rt_hit* out, int64_t k, const Hit& h) {
  int4 w;
  if (h.id >= 0) {
    w = make_int4(h.id, __float_as_int(h.t), __float_as_int(h.u), __float_as_int(h.v));
  } else {
    w = make_int4(-1, __float_as_int(INFINITY), 0, 0);
  }
  reinterpret_cast<int4*>(out)[k] = w;
}

constexpr int kBlock = 64;  // one wave per work-group: the LDS stack is per wave

// One wave traces reflection chains, one per lane (Sec. III-B re-launch).
// Rays come either as the batch [base, base + 64) of this work-group (a work-
// group of the default launch; `drained` afterwards) or, with a queue, from a
// global counter with one atomic per wave (ballot + popcount give each free
// lane its ray): by default a new batch of 64 consecutive rays once all the
// wave's chains have ended, so a wave traces adjacent launch directions
// together; with `refill` it tops up free lanes at every segment.  A wave
// exits once its rays are done; no wave ever waits for another.
// With G > 1 (default launch only) the G lanes of each aligned group trace
// one chain together: every lane of the group holds the same chain state,
// the facets of each leaf are split over them, and only the group's first
// lane writes results; a wave then takes 64 / G consecutive rays.
// PHASE 1 (first launch of a two-launch trace, default launch shape): a
// chain still alive after `cut` segments is appended to `cont` (one atomic
// add on *cont_n per wave) instead of going on.  PHASE 2: the lanes take the
// records cont[batch_base ..) below n_src and go on from their saved state.
template <int FMT, bool BOUNCE, bool SEG, bool STATS, bool RECV, bool ENERGY = false, int G = 1,
          int PHASE = 0>
__device__ __forceinline__ void trace_chains(const void* __restrict__ tn, const TFacet* __restrict__ tf,
                             const float4* __restrict__ rays, int64_t n, int max_b,
                             rt_hit* __restrict__ out, double* __restrict__ path_len,
                             int32_t* __restrict__ n_hits, float4* __restrict__ seg,
                             uint32_t* __restrict__ stats, unsigned long long* __restrict__ queue,
                             int refill, int64_t batch_base, int* stack,
                             const RecvArgs& recv, const EnergyArgs& en = EnergyArgs{},
                             int n_tf = 0, ChainCont* __restrict__ cont = nullptr,
                             unsigned long long* __restrict__ cont_n = nullptr, int cut = 0,
                             int64_t n_src = -1, bool pad = true) {
  static_assert(G == 1 || !STATS, "per-ray statistics are kept by the one-lane form only");
  static_assert(PHASE == 0 || (BOUNCE && !SEG && !STATS && !RECV && !ENERGY && G == 1),
                "the two-launch trace is the plain chain trace");
  if (PHASE != 2) n_src = n;
  const int lane = threadIdx.x & 63;
  const bool writer = G == 1 || (lane & (G - 1)) == 0;
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int64_t i = -1;  // ray of this lane, -1 when free
  float ox = 0.f, oy = 0.f, oz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f, tmin = 0.f, tmax = 0.f;
  int skip = -1, b = 0, hits = 0;
  double path = 0.0, gain = 1.0, last_power = 0.0;
  uint32_t nvis = 0, ntest = 0;
  bool drained = false;
  for (;;) {
    const unsigned long long free_lanes = __ballot(i < 0);
    if (!drained && (refill ? free_lanes != 0ull : free_lanes == ~0ull)) {
      const int leader = __ffsll((long long)free_lanes) - 1;
      unsigned long long base = 0;
      if (queue == nullptr) {
        base = (unsigned long long)batch_base;
        drained = true;
      } else {
        if (lane == leader) base = atomicAdd(queue, (unsigned long long)__popcll(free_lanes));
        base = __shfl(base, leader);
      }
      if (base >= (unsigned long long)n_src) drained = true;
      if (i < 0) {
        const unsigned long long j =
            base + (G == 1 ? (unsigned long long)__popcll(free_lanes & below)
                           : (unsigned long long)(lane / G));
        if (j < (unsigned long long)n_src) {
          if (PHASE == 2) {
            const ChainCont c = cont[j];
            i = c.ray;
            ox = c.o_tmin.x; oy = c.o_tmin.y; oz = c.o_tmin.z; tmin = c.o_tmin.w;
            dx = c.d_tmax.x; dy = c.d_tmax.y; dz = c.d_tmax.z; tmax = c.d_tmax.w;
            skip = c.skip;
            b = c.b;
            hits = c.hits;
            path = c.path;
          } else {
            i = (int64_t)j;
            const float4 ra = rays[2 * i], rb = rays[2 * i + 1];
            ox = ra.x; oy = ra.y; oz = ra.z; tmin = ra.w;
            dx = rb.x; dy = rb.y; dz = rb.z; tmax = rb.w;
            skip = -1;
            b = 0;
            hits = 0;
            path = 0.0;
          }
          gain = 1.0;
          last_power = 0.0;
          nvis = ntest = 0;
        }
      }
    }
    if (__ballot(i >= 0) == 0ull) break;
    if (i < 0) continue;
    // one segment of this lane's chain
    if (SEG && writer) {
      seg[2 * ((int64_t)b * n + i)] = make_float4(ox, oy, oz, tmin);
      seg[2 * ((int64_t)b * n + i) + 1] = make_float4(dx, dy, dz, tmax);
    }
    const RayPre r = prepare<FMT>(ox, oy, oz, dx, dy, dz, tmin, tmax);
    Hit h = closest<FMT, STATS, G>(tn, tf, r, skip, stack, nvis, ntest, n_tf);
    N2 nrm;
    if (h.id >= 0) {
      // the facet is decided; its distance is recomputed accurately
      const TFacet f = tf[h.pos];
      nrm = facet_normal(f.p0, f.p1, f.p2);
      const float tp = plane_t(nrm, f.p0, ox, oy, oz, dx, dy, dz);
      if (isfinite(tp)) h.t = fminf(fmaxf(tp, tmin), tmax);
    }
    if (writer) store_hit(out, (int64_t)b * n + i, h);
    if (RECV && writer)  // receiving spheres (Sec. III-C): path holds the length before this segment
      receive_segment(recv, i, b, ox, oy, oz, dx, dy, dz, tmin, h.id >= 0 ? h.t : tmax, path);
    bool more = false;
    if (BOUNCE && h.id >= 0) {
      ++hits;
      path += seg_path(h.t, dx, dy, dz);
      bool alive = true;
      if (ENERGY) {  // stop by energy (Sec. III-B)
        const int mat = en.material[h.id];
        gain *= (mat >= 0 && mat < en.n_mat) ? en.refl[mat] : 0.0;
        last_power = chain_power(gain, en.k0, path);
        alive = last_power >= en.min_power;
      }
      if (alive && b + 1 < max_b) {
        // specular reflection about the facet plane, launched from the hit point
        ox = fmaf(h.t, dx, ox);
        oy = fmaf(h.t, dy, oy);
        oz = fmaf(h.t, dz, oz);
        reflect(nrm, dx, dy, dz);
        skip = h.pos;
        ++b;
        more = true;
      }
    }
    if (PHASE == 1) {  // chains alive after `cut` segments wait for the second launch
      const bool push = more && b == cut;
      const unsigned long long pm = __ballot(push);
      if (pm != 0ull) {
        const int leader = __ffsll((long long)pm) - 1;
        unsigned long long at = 0;
        if (lane == leader) at = atomicAdd(cont_n, (unsigned long long)__popcll(pm));
        at = __shfl(at, leader);
        if (push) {
          ChainCont c;
          c.o_tmin = make_float4(ox, oy, oz, tmin);
          c.d_tmax = make_float4(dx, dy, dz, tmax);
          c.path = path;
          c.ray = (int32_t)i;
          c.skip = skip;
          c.b = b;
          c.hits = hits;
          c.pad[0] = c.pad[1] = 0;
          cont[at + __popcll(pm & below)] = c;
          i = -1;
        }
      }
      if (i < 0) continue;
    }
    if (!more) {  // chain finished: segments never launched read as misses
      if (BOUNCE && writer) {
        Hit none;
        none.id = -1;
        if (pad)
          for (int q = b + 1; q < max_b; ++q) store_hit(out, (int64_t)q * n + i, none);
        if (path_len) path_len[i] = path;
        if (n_hits) n_hits[i] = hits;
        if (ENERGY && en.power) en.power[i] = last_power;
      }
      if (STATS) {
        stats[2 * i] = nvis;
        stats[2 * i + 1] = ntest;
      }
      i = -1;
    }
  }
}

// The LDS stack (dynamic shared memory) holds exactly the entries the tree
// can need: stack_need(depth) per lane, in lane-column layout.  With G > 1
// lanes per ray a work-group takes the 64 / G rays from blockIdx.x * 64 / G.
template <int FMT, bool BOUNCE, bool SEG, bool STATS, int G = 1, int PHASE = 0>
__global__ __launch_bounds__(kBlock) void k_trace(const void* __restrict__ tn,
                                                  const TFacet* __restrict__ tf,
                                                  const float4* __restrict__ rays, int64_t n,
                                                  int max_b, rt_hit* __restrict__ out,
                                                  double* __restrict__ path_len,
                                                  int32_t* __restrict__ n_hits,
                                                  float4* __restrict__ seg,
                                                  uint32_t* __restrict__ stats,
                                                  unsigned long long* __restrict__ queue,
                                                  int refill, int n_tf,
                                                  ChainCont* __restrict__ cont = nullptr,
                                                  unsigned long long* __restrict__ cont_n = nullptr,
                                                  int cut = 0, int pad = 1,
                                                  const int32_t* __restrict__ order = nullptr) {
  extern __shared__ int s_stack[];
  // the batch this work-group traces: its own index, or the caller's order
  // (an entry outside the launch's batches leaves the work-group idle)
  int64_t batch = blockIdx.x;
  if (order != nullptr) {
    batch = order[blockIdx.x];
    if (batch < 0 || batch * (kBlock / G) >= n) return;
  }
  trace_chains<FMT, BOUNCE, SEG, STATS, false, false, G, PHASE>(
      tn, tf, rays, n, max_b, out, path_len, n_hits, seg, stats, queue, refill,
      batch * (kBlock / G), s_stack + threadIdx.x, RecvArgs{}, EnergyArgs{}, n_tf,
      cont, cont_n, cut, -1, pad != 0);
}

// Second launch of a two-launch trace: work-group g resumes the live chains
// cont[64 g, 64 g + 64) of the *cont_n the first launch left.
template <int FMT>
__global__ __launch_bounds__(kBlock) void k_trace_resume(const void* __restrict__ tn,
                                                         const TFacet* __restrict__ tf, int64_t n,
                                                         int max_b, rt_hit* __restrict__ out,
                                                         double* __restrict__ path_len,
                                                         int32_t* __restrict__ n_hits, int n_tf,
                                                         const ChainCont* __restrict__ cont,
                                                         const unsigned long long* __restrict__ cont_n,
                                                         int pad) {
  extern __shared__ int s_stack[];
  const int64_t total = (int64_t)*cont_n;
  const int64_t base = (int64_t)blockIdx.x * kBlock;
  if (base >= total) return;
  trace_chains<FMT, true, false, false, false, false, 1, 2>(
      tn, tf, nullptr, n, max_b, out, path_len, n_hits, nullptr, nullptr, nullptr, 0, base,
      s_stack + threadIdx.x, RecvArgs{}, EnergyArgs{}, n_tf, const_cast<ChainCont*>(cont), nullptr, 0,
      total, pad != 0);
}

// Reflection chains whose segments are tested against field points as they
// are traced (Sec. III-C): nothing per segment is stored.
template <int FMT, int G = 1>
__global__ __launch_bounds__(kBlock) void k_trace_recv(const void* __restrict__ tn,
                                                       const TFacet* __restrict__ tf,
                                                       const float4* __restrict__ rays, int64_t n,
                                                       int max_b, rt_hit* __restrict__ out,
                                                       double* __restrict__ path_len,
                                                       int32_t* __restrict__ n_hits, RecvArgs recv,
                                                       int n_tf) {
  extern __shared__ int s_stack[];
  trace_chains<FMT, true, false, false, true, false, G>(
      tn, tf, rays, n, max_b, out, path_len, n_hits, nullptr, nullptr, nullptr, 0,
      (int64_t)blockIdx.x * (kBlock / G), s_stack + threadIdx.x, recv, EnergyArgs{}, n_tf);
}

// Reflection chains that also stop by energy (Sec. III-B), with or without
// the reception test of every segment.
template <int FMT, bool RECV, int G = 1>
__global__ __launch_bounds__(kBlock) void k_trace_energy(const void* __restrict__ tn,
                                                         const TFacet* __restrict__ tf,
                                                         const float4* __restrict__ rays, int64_t n,
                                                         int max_b, rt_hit* __restrict__ out,
                                                         double* __restrict__ path_len,
                                                         int32_t* __restrict__ n_hits,
                                                         RecvArgs recv, EnergyArgs en, int n_tf) {
  extern __shared__ int s_stack[];
  trace_chains<FMT, true, false, false, RECV, true, G>(
      tn, tf, rays, n, max_b, out, path_len, n_hits, nullptr, nullptr, nullptr, 0,
      (int64_t)blockIdx.x * (kBlock / G), s_stack + threadIdx.x, recv, en, n_tf);
}

// Many queries (trees, ray sets, bounce limits) in one launch: work-group g
// finds its query by binary search over the queries' first batch numbers and
// traces that query's batch g - first.  Queries of one launch share the node
// format and whether they carry field points (RECV: every traced segment is
// tested against the query's own field points, as in k_trace_recv); each
// brings its own tree.
template <int FMT, bool RECV>
__global__ __launch_bounds__(kBlock) void k_trace_batch(const BatchQuery* __restrict__ q, int nq) {
  extern __shared__ int s_stack[];
  const int64_t g = blockIdx.x;
  int lo = 0, hi = nq - 1;  // last query whose first batch <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (q[mid].first_batch <= g) lo = mid;
    else hi = mid - 1;
  }
  const BatchQuery Q = q[lo];
  const int64_t local = g - Q.first_batch;
  if (local * kBlock >= Q.n) return;
  trace_chains<FMT, true, false, false, RECV>(Q.nodes, Q.facets, Q.rays, Q.n, Q.max_b, Q.out,
                                              Q.path_len, Q.n_hits, nullptr, nullptr, nullptr, 0,
                                              local * kBlock, s_stack + threadIdx.x, Q.recv);
}

// Persistent form of the batched launch: each wave takes batch numbers from
// a global counter (one atomic per 64 rays) until all are done.
template <int FMT, bool RECV>
__global__ __launch_bounds__(kBlock) void k_trace_batch_q(const BatchQuery* __restrict__ q, int nq,
                                                          int64_t total,
                                                          unsigned long long* __restrict__ queue) {
  extern __shared__ int s_stack[];
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned long long g = 0;
    if (lane == 0) g = atomicAdd(queue, 1ull);
    g = __shfl(g, 0);
    if (g >= (unsigned long long)total) break;
    int lo = 0, hi = nq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (q[mid].first_batch <= (int64_t)g) lo = mid;
      else hi = mid - 1;
    }
    const BatchQuery Q = q[lo];
    const int64_t local = (int64_t)g - Q.first_batch;
    if (local * kBlock >= Q.n) continue;
    trace_chains<FMT, true, false, false, RECV>(Q.nodes, Q.facets, Q.rays, Q.n, Q.max_b, Q.out,
                                                Q.path_len, Q.n_hits, nullptr, nullptr, nullptr, 0,
                                                local * kBlock, s_stack + threadIdx.x, Q.recv);
  }
}

__global__ void k_queue_reset(unsigned long long* q) { *q = 0ull; }

// Clears the reception counts of the queries that have one.
__global__ void k_batch_clear_counts(const BatchQuery* __restrict__ q, int nq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nq && q[i].recv.count) *q[i].recv.count = 0ull;
}

// Stack entries a ray can need: one per binary level below the root, or up
// to three per 4-wide level.  Sizing the LDS stack to the tree keeps the
// most waves resident (20 entries = 5 KB per wave lets 8 waves share a
// compute unit's 160 KB).
template <int FMT>
constexpr int stack_need(int depth) {
  return FMT == RT_NODE_BIN2 ? depth : 3 * ((depth + 1) / 2);
}
template <int FMT>
size_t stack_bytes(int depth) {
  return sizeof(int) * kBlock * std::max(1, stack_need<FMT>(depth));
}

template <int FMT, bool BOUNCE, bool SEG, bool STATS>
void launch(const Buffers& B, int depth, const float* rays, int64_t n, int max_b, rt_hit* out,
            double* path_len, int32_t* n_hits, float* seg, uint32_t* stats, int grid,
            int refill, int n_tf, unsigned long long* queue, int cut, void* ws, int pad,
            const int32_t* order, hipStream_t s) {
  const int64_t batches = (n + kBlock - 1) / kBlock;
  const void* nodes = FMT == RT_NODE_BIN2 ? (const void*)B.tnodes : (const void*)B.wnodes;
  if constexpr (BOUNCE && !SEG && !STATS) {
    if (cut > 0 && cut < max_b && grid == 0) {  // two launches, regrouping the live chains
      unsigned long long* cont_n = reinterpret_cast<unsigned long long*>(ws);
      ChainCont* cont = reinterpret_cast<ChainCont*>(reinterpret_cast<char*>(ws) + kChainWsHeader);
      hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, cont_n);
      hipLaunchKernelGGL((k_trace<FMT, true, false, false, 1, 1>), dim3((unsigned)batches),
                         dim3(kBlock), stack_bytes<FMT>(depth), s, nodes, B.tfacets,
                         reinterpret_cast<const float4*>(rays), n, max_b, out, path_len, n_hits,
                         nullptr, nullptr, nullptr, 0, n_tf, cont, cont_n, cut, pad, order);
      hipLaunchKernelGGL((k_trace_resume<FMT>), dim3((unsigned)batches), dim3(kBlock),
                         stack_bytes<FMT>(depth), s, nodes, B.tfacets, n, max_b, out, path_len,
                         n_hits, n_tf, cont, cont_n, pad);
      return;
    }
  }
  unsigned long long* q = nullptr;
  int64_t blocks = batches;  // default: one work-group per batch of 64 rays
  if (grid > 0) {            // persistent work-groups pulling batches from the call's queue
    q = queue;
    blocks = std::min<int64_t>(grid, batches);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, q);
  }
  hipLaunchKernelGGL((k_trace<FMT, BOUNCE, SEG, STATS>), dim3((unsigned)blocks), dim3(kBlock),
                     stack_bytes<FMT>(depth), s, nodes, B.tfacets,
                     reinterpret_cast<const float4*>(rays), n, max_b, out, path_len, n_hits,
                     reinterpret_cast<float4*>(seg), stats, q, refill, n_tf, nullptr, nullptr, 0, pad,
                     grid > 0 ? nullptr : order);
}

// G lanes per ray: one work-group per 64 / G consecutive rays.
template <int FMT, int G>
void launch_group(const Buffers& B, int depth, const float* rays, int64_t n, int max_b,
                  rt_hit* out, double* path_len, int32_t* n_hits, int n_tf, int pad,
                  hipStream_t s) {
  constexpr int per_wave = kBlock / G;
  const int64_t blocks = (n + per_wave - 1) / per_wave;
  const void* nodes = FMT == RT_NODE_BIN2 ? (const void*)B.tnodes : (const void*)B.wnodes;
  hipLaunchKernelGGL((k_trace<FMT, true, false, false, G>), dim3((unsigned)blocks), dim3(kBlock),
                     stack_bytes<FMT>(depth), s, nodes, B.tfacets,
                     reinterpret_cast<const float4*>(rays), n, max_b, out, path_len, n_hits,
                     nullptr, nullptr, nullptr, 0, n_tf, nullptr, nullptr, 0, pad);
}

template <int FMT>
void launch_fmt(const Buffers& B, int depth, const float* rays, int64_t n, int max_b, rt_hit* out,
                double* path_len, int32_t* n_hits, float* seg, uint32_t* stats, int grid,
                int refill, int lanes, int n_tf, unsigned long long* q, int cut, void* ws, int pad,
                const int32_t* order, hipStream_t s) {
  switch (lanes) {  // the caller allows lanes > 1 only without seg, stats and grid
    case 4: return launch_group<FMT, 4>(B, depth, rays, n, max_b, out, path_len, n_hits, n_tf, pad, s);
    case 16: return launch_group<FMT, 16>(B, depth, rays, n, max_b, out, path_len, n_hits, n_tf, pad, s);
    case 64: return launch_group<FMT, 64>(B, depth, rays, n, max_b, out, path_len, n_hits, n_tf, pad, s);
    default: break;
  }
  const bool bounce = max_b > 1 || path_len || n_hits;
  if (!bounce && !seg && !stats) {
    launch<FMT, false, false, false>(B, depth, rays, n, 1, out, nullptr, nullptr, nullptr, nullptr, grid, refill, n_tf, q, cut, ws, pad, order, s);
  } else if (!seg && !stats) {
    launch<FMT, true, false, false>(B, depth, rays, n, max_b, out, path_len, n_hits, nullptr, nullptr, grid, refill, n_tf, q, cut, ws, pad, order, s);
  } else if (seg && !stats) {
    launch<FMT, true, true, false>(B, depth, rays, n, max_b, out, path_len, n_hits, seg, nullptr, grid, refill, n_tf, q, cut, ws, pad, order, s);
  } else if (!seg) {
    launch<FMT, true, false, true>(B, depth, rays, n, max_b, out, path_len, n_hits, nullptr, stats, grid, refill, n_tf, q, cut, ws, pad, order, s);
  } else {
    launch<FMT, true, true, true>(B, depth, rays, n, max_b, out, path_len, n_hits, seg, stats, grid, refill, n_tf, q, cut, ws, pad, order, s);
  }
}

template <int FMT, bool RECV>
void launch_batch_fmt(const BatchQuery* table, int nq, int64_t total, int depth, int grid,
                      unsigned long long* queue, hipStream_t s) {
  const size_t lds = stack_bytes<FMT>(depth);
  if (grid > 0) {
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, queue);
    hipLaunchKernelGGL((k_trace_batch_q<FMT, RECV>), dim3((unsigned)std::min<int64_t>(grid, total)),
                       dim3(kBlock), lds, s, table, nq, total, queue);
  } else {
    hipLaunchKernelGGL((k_trace_batch<FMT, RECV>), dim3((unsigned)total), dim3(kBlock), lds, s,
                       table, nq);
  }
}

template <int FMT, bool RECV>
int resident_fmt(int depth) {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_trace_batch_q<FMT, RECV>, kBlock,
                                                     stack_bytes<FMT>(depth));
  return std::max(1, cus * std::max(1, per_cu));
}

}  // namespace

int launch_trace_batch(const BatchQuery* table, int nq, int64_t total, int node_format, bool recv,
                       int depth, int grid, unsigned long long* queue, hipStream_t s) {
  if (nq <= 0 || total <= 0) return RT_OK;
  switch (node_format * 2 + (recv ? 1 : 0)) {
    case 2 * RT_NODE_F4: launch_batch_fmt<RT_NODE_F4, false>(table, nq, total, depth, grid, queue, s); break;
    case 2 * RT_NODE_F4 + 1: launch_batch_fmt<RT_NODE_F4, true>(table, nq, total, depth, grid, queue, s); break;
    case 2 * RT_NODE_Q4: launch_batch_fmt<RT_NODE_Q4, false>(table, nq, total, depth, grid, queue, s); break;
    case 2 * RT_NODE_Q4 + 1: launch_batch_fmt<RT_NODE_Q4, true>(table, nq, total, depth, grid, queue, s); break;
    case 2 * RT_NODE_BIN2 + 1: launch_batch_fmt<RT_NODE_BIN2, true>(table, nq, total, depth, grid, queue, s); break;
    default: launch_batch_fmt<RT_NODE_BIN2, false>(table, nq, total, depth, grid, queue, s); break;
  }
  return check_hip(hipGetLastError(), "batch trace launch");
}

int launch_batch_clear_counts(const BatchQuery* table, int nq, hipStream_t s) {
  if (nq <= 0) return RT_OK;
  hipLaunchKernelGGL(k_batch_clear_counts, dim3((nq + 255) / 256), dim3(256), 0, s, table, nq);
  return check_hip(hipGetLastError(), "batch reception count reset");
}

int trace_resident_groups(int node_format, bool recv, int depth) {
  switch (node_format * 2 + (recv ? 1 : 0)) {
    case 2 * RT_NODE_F4: return resident_fmt<RT_NODE_F4, false>(depth);
    case 2 * RT_NODE_F4 + 1: return resident_fmt<RT_NODE_F4, true>(depth);
    case 2 * RT_NODE_Q4: return resident_fmt<RT_NODE_Q4, false>(depth);
    case 2 * RT_NODE_Q4 + 1: return resident_fmt<RT_NODE_Q4, true>(depth);
    case 2 * RT_NODE_BIN2 + 1: return resident_fmt<RT_NODE_BIN2, true>(depth);
    default: return resident_fmt<RT_NODE_BIN2, false>(depth);
  }
}

namespace {
template <int FMT, int G>
void launch_recv_fmt(const Buffers& B, int depth, const float4* rays, int64_t n, int max_b,
                     rt_hit* out, double* path_len, int32_t* n_hits, const RecvArgs& recv,
                     int n_tf, hipStream_t s) {
  constexpr int per_wave = kBlock / G;
  const unsigned blocks = (unsigned)((n + per_wave - 1) / per_wave);
  const void* nodes = FMT == RT_NODE_BIN2 ? (const void*)B.tnodes : (const void*)B.wnodes;
  hipLaunchKernelGGL((k_trace_recv<FMT, G>), dim3(blocks), dim3(kBlock), stack_bytes<FMT>(depth),
                     s, nodes, B.tfacets, rays, n, max_b, out, path_len, n_hits, recv, n_tf);
}

template <int FMT>
void launch_recv_lanes(const Buffers& B, int depth, const float4* rays, int64_t n, int max_b,
                       rt_hit* out, double* path_len, int32_t* n_hits, const RecvArgs& recv,
                       int lanes, int n_tf, hipStream_t s) {
  switch (lanes) {
    case 4: return launch_recv_fmt<FMT, 4>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, n_tf, s);
    case 16: return launch_recv_fmt<FMT, 16>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, n_tf, s);
    case 64: return launch_recv_fmt<FMT, 64>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, n_tf, s);
    default: return launch_recv_fmt<FMT, 1>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, n_tf, s);
  }
}

}  // namespace

int launch_trace_receive(const Buffers& B, int node_format, int depth, const float* rays,
                         int64_t n, int32_t max_b, rt_hit* out, double* path_len,
                         int32_t* n_hits, const RecvArgs& recv, int lanes, int n_tf,
                         hipStream_t s) {
  if (n == 0) return RT_OK;
  const float4* r4 = reinterpret_cast<const float4*>(rays);
  switch (node_format) {
    case RT_NODE_F4:
      launch_recv_lanes<RT_NODE_F4>(B, depth, r4, n, max_b, out, path_len, n_hits, recv, lanes, n_tf, s);
      break;
    case RT_NODE_Q4:
      launch_recv_lanes<RT_NODE_Q4>(B, depth, r4, n, max_b, out, path_len, n_hits, recv, lanes, n_tf, s);
      break;
    default:
      launch_recv_lanes<RT_NODE_BIN2>(B, depth, r4, n, max_b, out, path_len, n_hits, recv, lanes, n_tf, s);
      break;
  }
  return check_hip(hipGetLastError(), "trace+receive launch");
}

namespace {
template <int FMT, int G>
void launch_energy_lanes(const Buffers& B, int depth, const float4* rays, int64_t n, int max_b,
                         rt_hit* out, double* path_len, int32_t* n_hits, const RecvArgs* recv,
                         const EnergyArgs& en, int n_tf, hipStream_t s) {
  constexpr int per_wave = kBlock / G;
  const unsigned blocks = (unsigned)((n + per_wave - 1) / per_wave);
  const void* nodes = FMT == RT_NODE_BIN2 ? (const void*)B.tnodes : (const void*)B.wnodes;
  if (recv)
    hipLaunchKernelGGL((k_trace_energy<FMT, true, G>), dim3(blocks), dim3(kBlock),
                       stack_bytes<FMT>(depth), s, nodes, B.tfacets, rays, n, max_b, out, path_len,
                       n_hits, *recv, en, n_tf);
  else
    hipLaunchKernelGGL((k_trace_energy<FMT, false, G>), dim3(blocks), dim3(kBlock),
                       stack_bytes<FMT>(depth), s, nodes, B.tfacets, rays, n, max_b, out, path_len,
                       n_hits, RecvArgs{}, en, n_tf);
}

template <int FMT>
void launch_energy_fmt(const Buffers& B, int depth, const float4* rays, int64_t n, int max_b,
                       rt_hit* out, double* path_len, int32_t* n_hits, const RecvArgs* recv,
                       const EnergyArgs& en, int lanes, int n_tf, hipStream_t s) {
  switch (lanes) {
    case 4: return launch_energy_lanes<FMT, 4>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, en, n_tf, s);
    case 16: return launch_energy_lanes<FMT, 16>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, en, n_tf, s);
    case 64: return launch_energy_lanes<FMT, 64>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, en, n_tf, s);
    default: return launch_energy_lanes<FMT, 1>(B, depth, rays, n, max_b, out, path_len, n_hits, recv, en, n_tf, s);
  }
}
}  // namespace

int launch_trace_energy(const Buffers& B, int node_format, int depth, const float* rays, int64_t n,
                        int32_t max_b, rt_hit* out, double* path_len, int32_t* n_hits,
                        const RecvArgs* recv, const EnergyArgs& en, int lanes, int n_tf,
                        hipStream_t s) {
  if (n == 0) return RT_OK;
  const float4* r4 = reinterpret_cast<const float4*>(rays);
  switch (node_format) {
    case RT_NODE_F4:
      launch_energy_fmt<RT_NODE_F4>(B, depth, r4, n, max_b, out, path_len, n_hits, recv, en, lanes, n_tf, s);
      break;
    case RT_NODE_Q4:
      launch_energy_fmt<RT_NODE_Q4>(B, depth, r4, n, max_b, out, path_len, n_hits, recv, en, lanes, n_tf, s);
      break;
    default:
      launch_energy_fmt<RT_NODE_BIN2>(B, depth, r4, n, max_b, out, path_len, n_hits, recv, en, lanes, n_tf, s);
      break;
  }
  return check_hip(hipGetLastError(), "trace+energy launch");
}

int launch_trace(const Buffers& B, int node_format, int depth, const float* rays, int64_t n,
                 int32_t max_b, rt_hit* out, double* path_len, int32_t* n_hits,
                 const rt_trace_opts* opts, int lanes, int n_tf, unsigned long long* q,
                 hipStream_t s) {
  if (n == 0) return RT_OK;
  float* seg = opts ? opts->seg_rays : nullptr;
  uint32_t* stats = opts ? opts->ray_stats : nullptr;
  const int grid = opts ? opts->grid : 0;
  const int refill = opts ? opts->refill : 0;
  const int cut = opts ? opts->cut : 0;
  void* ws = opts ? opts->chain_ws : nullptr;
  const int pad = opts && (opts->flags & RT_TRACE_NO_PAD) ? 0 : 1;
  const int32_t* order = opts ? opts->batch_order : nullptr;
  switch (node_format) {
    case RT_NODE_F4:
      launch_fmt<RT_NODE_F4>(B, depth, rays, n, max_b, out, path_len, n_hits, seg, stats, grid, refill, lanes, n_tf, q, cut, ws, pad, order, s);
      break;
    case RT_NODE_Q4:
      launch_fmt<RT_NODE_Q4>(B, depth, rays, n, max_b, out, path_len, n_hits, seg, stats, grid, refill, lanes, n_tf, q, cut, ws, pad, order, s);
      break;
    default:
      launch_fmt<RT_NODE_BIN2>(B, depth, rays, n, max_b, out, path_len, n_hits, seg, stats, grid, refill, lanes, n_tf, q, cut, ws, pad, order, s);
      break;
  }
  return check_hip(hipGetLastError(), "trace launch");
}

}  // namespace rt
