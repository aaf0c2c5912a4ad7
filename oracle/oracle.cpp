// CPU checker for the closest-hit ray tracing path: TEST INFRASTRUCTURE ONLY.
//
// Plain float64 reference.  Only tests, the package smoke check and the
// benchmark's CPU-baseline leg use it; nothing in the GPU library includes or
// links it.  Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared.
//
// Parity pins (tests/test_oracle_*.py):
//   or_brute     -- hand-built worked cases with exact hits (tests/golden),
//                   an independent numpy linear-solve brute force, ground and
//                   wall hits with closed-form distances.
//   or_build     -- tree invariants (bijection, containment, leaf rule, depth),
//                   hand-worked Eq. (2) split choices on small node sets,
//                   alpha = 1 / alpha = 0 limits of Eq. (2).
//   or_trace_bvh -- equal to or_brute on every ray (ids, t, capped margins).
//   or_bounces   -- image-source closed forms (ground + wall, corridor).
#include "oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

const double kInf = std::numeric_limits<double>::infinity();
const double kCap = OR_MARGIN_CAP;

struct V3 {
  double x, y, z;
};
V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 mul(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
double get(V3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

struct Tri {
  V3 a, b, c;
};
struct Ray {
  V3 o, d;
  double tmin, tmax;
};

Tri load_tri(const float* tris, int64_t j) {
  const float* p = tris + 9 * j;
  return {{p[0], p[1], p[2]}, {p[3], p[4], p[5]}, {p[6], p[7], p[8]}};
}
Ray load_ray(const float* rays, int64_t i) {
  const float* r = rays + 8 * i;
  return {{r[0], r[1], r[2]}, {r[4], r[5], r[6]}, r[3], r[7]};
}

// Crossing of the ray's line with the facet's plane, in barycentric form:
// o + t d = (1 - u - v) a + u b + v c.  Moller-Trumbore, float64.
struct Crossing {
  bool valid;  // false when the ray is parallel to the plane (det == 0)
  double t, u, v;
  bool inside() const { return valid && u >= 0.0 && v >= 0.0 && u + v <= 1.0; }
  double outside_by() const {  // > 0 when outside the triangle
    return std::max(std::max(-u, -v), u + v - 1.0);
  }
};

Crossing crossing(const Ray& r, const Tri& f) {
  V3 e1 = sub(f.b, f.a), e2 = sub(f.c, f.a);
  V3 p = cross(r.d, e2);
  double det = dot(e1, p);
  if (det == 0.0) return {false, 0.0, 0.0, 0.0};
  V3 s = sub(r.o, f.a);
  double u = dot(s, p) / det;
  V3 q = cross(s, e1);
  double v = dot(r.d, q) / det;
  double t = dot(e2, q) / det;
  return {true, t, u, v};
}

// Everything the margin needs about the facets a ray meets.
struct Result {
  int32_t id = -1;
  double t = kInf, u = 0.0, v = 0.0, margin = kCap, t2 = kInf;
};

struct Seen {  // one facet's crossing, kept until the winner is known
  int32_t id;
  Crossing c;
};

double rel(double a, double scale) { return a / std::max(std::fabs(scale), 1e-3); }

// Winner = lexicographic min of (t, id) over in-triangle crossings in
// [tmin, tmax]; margin = min of barycentric edge distance of the winner,
// relative gap to the next hit of another facet, how far outside the nearest
// missed facet in front of the winner is passed, and how close a crossing is
// to either end of the range.  Capped at kCap.
Result resolve(const Ray& r, const std::vector<Seen>& seen) {
  Result res;
  for (const Seen& s : seen) {
    if (!s.c.inside() || s.c.t < r.tmin || s.c.t > r.tmax) continue;
    if (s.c.t < res.t || (s.c.t == res.t && s.id < res.id)) {
      res.id = s.id;
      res.t = s.c.t;
      res.u = s.c.u;
      res.v = s.c.v;
    }
  }
  const bool hit = res.id >= 0;
  const double limit = hit ? res.t : r.tmax;
  double m = kCap;
  if (hit) {
    m = std::min(m, std::min(std::min(res.u, res.v), 1.0 - res.u - res.v));
    m = std::min(m, rel(std::min(res.t - r.tmin, r.tmax - res.t), res.t));
  }
  for (const Seen& s : seen) {
    if (!s.c.valid || s.id == res.id) continue;
    if (s.c.inside()) {
      if (s.c.t >= r.tmin && s.c.t <= r.tmax) {
        res.t2 = std::min(res.t2, s.c.t);
        if (hit) m = std::min(m, rel(s.c.t - res.t, res.t));
      } else if (s.c.t < r.tmin) {
        m = std::min(m, rel(r.tmin - s.c.t, s.c.t));
      } else if (!hit) {
        m = std::min(m, rel(s.c.t - r.tmax, s.c.t));
      }
    } else if (s.c.t >= r.tmin && s.c.t <= limit) {
      m = std::min(m, s.c.outside_by());
    }
  }
  res.margin = std::max(0.0, std::min(m, kCap));
  if (!hit) res.t = kInf;
  // a second hit is reported only inside the margin window
  if (!hit || !(rel(res.t2 - res.t, res.t) < kCap)) res.t2 = kInf;
  return res;
}

// A crossing can change the winner or lower a capped margin only if it lies
// inside the triangle or passes it by less than the cap.
bool matters(const Crossing& c) { return c.valid && (c.inside() || c.outside_by() < kCap); }

Result brute_one(const float* tris, int64_t n, const Ray& r, int32_t skip) {
  std::vector<Seen> seen;
  for (int64_t j = 0; j < n; ++j) {
    if (j == skip) continue;
    Crossing c = crossing(r, load_tri(tris, j));
    if (matters(c)) seen.push_back({(int32_t)j, c});
  }
  return resolve(r, seen);
}

template <class F>
void parallel_for(int64_t m, int32_t nthreads, F f) {
  int nt = nthreads > 0 ? nthreads : (int)std::max(1u, std::thread::hardware_concurrency());
  if (m < 64 || nt == 1) {
    for (int64_t i = 0; i < m; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = 64;
  std::atomic<int64_t> next(0);
  for (int k = 0; k < nt; ++k)
    th.emplace_back([&]() {
      for (;;) {
        int64_t s = next.fetch_add(chunk);
        if (s >= m) break;
        int64_t e = std::min(m, s + chunk);
        for (int64_t i = s; i < e; ++i) f(i);
      }
    });
  for (auto& t : th) t.join();
}

void store(const Result& r, int64_t i, int32_t* id, double* t, double* u, double* v,
           double* margin, double* t2) {
  id[i] = r.id;
  t[i] = r.t;
  u[i] = r.u;
  v[i] = r.v;
  if (margin) margin[i] = r.margin;
  if (t2) t2[i] = r.t2;
}

}  // namespace

// ----------------------------------------------------------------------------
// Tree build: Sec. II-C flow (import facets, root volume, best division by
// Eq. (2), recurse until the facet count reaches the threshold).
// ----------------------------------------------------------------------------
struct or_tree {
  struct Node {
    double lo[3], hi[3];
    int32_t left, right, first, count, depth, axis, plane, flags;
    double cost;
  };
  std::vector<Node> nodes;
  std::vector<int32_t> perm;
  int32_t depth = 0;
};

namespace {

struct Builder {
  const float* tris;
  or_params p;
  std::vector<double> flo, fhi, cen;  // per facet box and centroid, [n][3]
  std::vector<int32_t> refs;
  double inv_l2 = 0.0;
  or_tree* out;

  double area(const double* lo, const double* hi) const {
    double ex = hi[0] - lo[0], ey = hi[1] - lo[1], ez = hi[2] - lo[2];
    return 2.0 * ((ex * ey + ey * ez) + ez * ex);
  }
  double dist2(const double* lo, const double* hi) const {
    double cx = (lo[0] + hi[0]) * 0.5 - p.src[0];
    double cy = (lo[1] + hi[1]) * 0.5 - p.src[1];
    double cz = (lo[2] + hi[2]) * 0.5 - p.src[2];
    return (cx * cx + cy * cy) + cz * cz;
  }

  // Eq. (2); UNIT divides the surface-area part by k_C t_i and the distance
  // part by the squared root diagonal, RAW keeps the printed units.
  double cost(const double* alo, const double* ahi, int64_t ka, const double* blo,
              const double* bhi, int64_t kb, const double* clo, const double* chi,
              int64_t kc, double alpha) const {
    double sa = area(alo, ahi), sb = area(blo, bhi), sc = area(clo, chi);
    double num = sa * (double)ka + sb * (double)kb;
    double da = dist2(alo, ahi), db = dist2(blo, bhi);
    double d;
    switch (p.d_mode) {
      case 1: d = da + db; break;
      case 2: d = (da * (double)ka + db * (double)kb) / (double)kc; break;
      case 3: d = dist2(clo, chi); break;
      default: d = (da + db) * 0.5; break;
    }
    double sah, tt;
    if (p.d_norm == 1) {
      sah = num * p.t_isect / sc;
      tt = p.t_trav;
    } else {
      sah = num / (sc * (double)kc);
      d = d * inv_l2;
      tt = p.t_trav / (p.t_isect * (double)kc);
    }
    return alpha * sah + (1.0 - alpha) * d + tt;
  }

  static int32_t halvings(int64_t k, int32_t max_leaf) {
    int64_t need = (k + max_leaf - 1) / max_leaf;
    int32_t l = 0;
    while ((int64_t(1) << l) < need) ++l;
    return l;
  }

  int32_t rec(int64_t first, int64_t k, int32_t depth) {
    int32_t me = (int32_t)out->nodes.size();
    out->nodes.push_back({});
    or_tree::Node nd;
    double clo[3], chi[3], cblo[3], cbhi[3];
    for (int a = 0; a < 3; ++a) {
      clo[a] = cblo[a] = kInf;
      chi[a] = cbhi[a] = -kInf;
    }
    for (int64_t i = first; i < first + k; ++i) {
      int32_t f = refs[i];
      for (int a = 0; a < 3; ++a) {
        clo[a] = std::min(clo[a], flo[3 * f + a]);
        chi[a] = std::max(chi[a], fhi[3 * f + a]);
        cblo[a] = std::min(cblo[a], cen[3 * f + a]);
        cbhi[a] = std::max(cbhi[a], cen[3 * f + a]);
      }
    }
    for (int a = 0; a < 3; ++a) {
      nd.lo[a] = clo[a];
      nd.hi[a] = chi[a];
    }
    nd.left = nd.right = -1;
    nd.first = (int32_t)first;
    nd.count = (int32_t)k;
    nd.depth = depth;
    nd.axis = nd.plane = -1;
    nd.flags = 0;
    nd.cost = 0.0;
    out->depth = std::max(out->depth, depth);
    if (k <= p.max_leaf) {
      out->nodes[me] = nd;
      return me;
    }

    int64_t nleft = -1;  // set when the split is by position
    int best_axis = -1, best_plane = -1;
    double best = kInf;
    const int B = p.nbins;
    std::vector<double> scale(3, 0.0);
    if (depth + halvings(k, p.max_leaf) >= p.depth_limit) {
      nleft = k / 2;
      nd.flags |= 1;
    } else {
      double alpha = p.alpha;
      if (depth >= p.max_depth) {
        alpha = 1.0;
        nd.flags |= 4;
      }
      std::vector<int64_t> cnt(B);
      std::vector<double> blo(3 * B), bhi(3 * B);
      for (int a = 0; a < 3; ++a) {
        double ext = cbhi[a] - cblo[a];
        if (!(ext > 0.0)) continue;
        scale[a] = (double)B / ext;
        std::fill(cnt.begin(), cnt.end(), 0);
        std::fill(blo.begin(), blo.end(), kInf);
        std::fill(bhi.begin(), bhi.end(), -kInf);
        for (int64_t i = first; i < first + k; ++i) {
          int32_t f = refs[i];
          int b = std::min(B - 1, (int)((cen[3 * f + a] - cblo[a]) * scale[a]));
          cnt[b]++;
          for (int c = 0; c < 3; ++c) {
            blo[3 * b + c] = std::min(blo[3 * b + c], flo[3 * f + c]);
            bhi[3 * b + c] = std::max(bhi[3 * b + c], fhi[3 * f + c]);
          }
        }
        for (int pl = 1; pl < B; ++pl) {
          double alo[3] = {kInf, kInf, kInf}, ahi[3] = {-kInf, -kInf, -kInf};
          double rlo[3] = {kInf, kInf, kInf}, rhi[3] = {-kInf, -kInf, -kInf};
          int64_t ka = 0, kb = 0;
          for (int b = 0; b < B; ++b) {
            double* lo = b < pl ? alo : rlo;
            double* hi = b < pl ? ahi : rhi;
            (b < pl ? ka : kb) += cnt[b];
            if (cnt[b] == 0) continue;
            for (int c = 0; c < 3; ++c) {
              lo[c] = std::min(lo[c], blo[3 * b + c]);
              hi[c] = std::max(hi[c], bhi[3 * b + c]);
            }
          }
          if (ka == 0 || kb == 0) continue;
          double c = cost(alo, ahi, ka, rlo, rhi, kb, clo, chi, k, alpha);
          if (c < best) {
            best = c;
            best_axis = a;
            best_plane = pl;
          }
        }
      }
      if (best_axis < 0) {  // every centroid is the same point
        nleft = k / 2;
        nd.flags |= 2;
      }
    }
    if (nleft < 0) {
      // stable partition: facets keep their relative order on each side
      std::vector<int32_t> lside, rside;
      for (int64_t i = first; i < first + k; ++i) {
        int32_t f = refs[i];
        int b = std::min(B - 1, (int)((cen[3 * f + best_axis] - cblo[best_axis]) *
                                      scale[best_axis]));
        (b < best_plane ? lside : rside).push_back(f);
      }
      nleft = (int64_t)lside.size();
      std::copy(lside.begin(), lside.end(), refs.begin() + first);
      std::copy(rside.begin(), rside.end(), refs.begin() + first + nleft);
    }
    nd.axis = best_axis;
    nd.plane = best_plane;
    nd.cost = best_axis >= 0 ? best : 0.0;
    out->nodes[me] = nd;
    int32_t l = rec(first, nleft, depth + 1);
    int32_t rr = rec(first + nleft, k - nleft, depth + 1);
    out->nodes[me].left = l;
    out->nodes[me].right = rr;
    return me;
  }
};

// ----------------------------------------------------------------------------
// Sec. III-B collision detection against the tree: test a bounding volume,
// descend into the volumes the ray meets, test the facets of the leaves
// reached and keep the nearest crossing.  Every box is widened by
// 2 * cap * (box diagonal) + 1 um and the range by 2 * cap, which keeps each
// facet able to lower a capped margin in the tested set, so the outcome is the
// brute-force one.
// ----------------------------------------------------------------------------
bool box_hit(const double* lo, const double* hi, double grow, const Ray& r, double t0,
             double t1) {
  double tn = t0, tf = t1;
  for (int a = 0; a < 3; ++a) {
    double o = get(r.o, a), d = get(r.d, a);
    double l = lo[a] - grow, h = hi[a] + grow;
    if (d == 0.0) {
      if (o < l || o > h) return false;
      continue;
    }
    double ta = (l - o) / d, tb = (h - o) / d;
    if (ta > tb) std::swap(ta, tb);
    tn = std::max(tn, ta);
    tf = std::min(tf, tb);
    if (tn > tf) return false;
  }
  return true;
}

Result bvh_one(const float* tris, const or_tree& T, const Ray& r, int32_t skip,
               int32_t* nodes_visited, int32_t* tris_tested) {
  std::vector<Seen> seen;
  int32_t best_id = -1;
  double best_t = kInf;
  const double t_lo = r.tmin - 2 * kCap * std::max(std::fabs(r.tmin), 1e-3);
  int32_t nv = 0, nt = 0;
  std::vector<int32_t> stack;
  stack.push_back(0);
  while (!stack.empty()) {
    int32_t ni = stack.back();
    stack.pop_back();
    const or_tree::Node& nd = T.nodes[ni];
    double t_hi = best_id >= 0 ? best_t + 2 * kCap * std::max(best_t, 1e-3)
                               : r.tmax + 2 * kCap * std::max(r.tmax, 1e-3);
    double ex = nd.hi[0] - nd.lo[0], ey = nd.hi[1] - nd.lo[1], ez = nd.hi[2] - nd.lo[2];
    double grow = 2 * kCap * std::sqrt(ex * ex + ey * ey + ez * ez) + 1e-6;
    if (!box_hit(nd.lo, nd.hi, grow, r, t_lo, t_hi)) continue;
    ++nv;
    if (nd.left < 0) {
      for (int32_t k = nd.first; k < nd.first + nd.count; ++k) {
        int32_t f = T.perm[k];
        if (f == skip) continue;
        ++nt;
        Crossing c = crossing(r, load_tri(tris, f));
        if (!matters(c)) continue;
        seen.push_back({f, c});
        if (c.inside() && c.t >= r.tmin && c.t <= r.tmax &&
            (c.t < best_t || (c.t == best_t && f < best_id))) {
          best_t = c.t;
          best_id = f;
        }
      }
    } else {
      stack.push_back(nd.right);
      stack.push_back(nd.left);
    }
  }
  if (nodes_visited) *nodes_visited = nv;
  if (tris_tested) *tris_tested = nt;
  return resolve(r, seen);
}

Ray reflect(const float* tris, const Ray& r, const Result& h) {
  Tri f = load_tri(tris, h.id);
  V3 nrm = cross(sub(f.b, f.a), sub(f.c, f.a));
  nrm = mul(nrm, 1.0 / std::sqrt(dot(nrm, nrm)));
  Ray out = r;
  out.o = add(r.o, mul(r.d, h.t));
  out.d = sub(r.d, mul(nrm, 2.0 * dot(r.d, nrm)));
  return out;
}

}  // namespace

extern "C" {

int or_brute(const float* tris, int64_t n, const float* rays, int64_t m,
             const int32_t* skip, int32_t nthreads, int32_t* id, double* t, double* u,
             double* v, double* margin, double* t2) {
  if (!tris || !rays || !id || !t || !u || !v || n < 0 || m < 0) return -1;
  parallel_for(m, nthreads, [&](int64_t i) {
    Ray r = load_ray(rays, i);
    Result res = brute_one(tris, n, r, skip ? skip[i] : -1);
    store(res, i, id, t, u, v, margin, t2);
  });
  return 0;
}

int or_eval(const float* tris, int64_t n, const float* rays, int64_t m,
            const int32_t* ids, int32_t* valid, double* t, double* u, double* v) {
  if (!tris || !rays || !ids || !valid || !t || !u || !v) return -1;
  for (int64_t i = 0; i < m; ++i) {
    if (ids[i] < 0 || ids[i] >= n) {
      valid[i] = 0;
      t[i] = u[i] = v[i] = 0.0;
      continue;
    }
    Crossing c = crossing(load_ray(rays, i), load_tri(tris, ids[i]));
    valid[i] = c.valid ? 1 : 0;
    t[i] = c.t;
    u[i] = c.u;
    v[i] = c.v;
  }
  return 0;
}

or_tree* or_build(const float* tris, int64_t n, const or_params* p) {
  if (!tris || !p || n <= 0 || n > INT32_MAX) return nullptr;
  if (!(p->alpha >= 0.0 && p->alpha <= 1.0) || p->max_leaf < 1 || p->nbins < 2 ||
      p->nbins > 256 || p->depth_limit < 1 || p->d_mode < 0 || p->d_mode > 3 ||
      p->d_norm < 0 || p->d_norm > 1)
    return nullptr;
  or_tree* out = new or_tree;
  Builder b;
  b.tris = tris;
  b.p = *p;
  b.out = out;
  b.flo.resize(3 * n);
  b.fhi.resize(3 * n);
  b.cen.resize(3 * n);
  b.refs.resize(n);
  double rlo[3] = {kInf, kInf, kInf}, rhi[3] = {-kInf, -kInf, -kInf};
  for (int64_t j = 0; j < n; ++j) {
    const float* v = tris + 9 * j;
    for (int a = 0; a < 3; ++a) {
      double lo = std::min(std::min((double)v[a], (double)v[3 + a]), (double)v[6 + a]);
      double hi = std::max(std::max((double)v[a], (double)v[3 + a]), (double)v[6 + a]);
      b.flo[3 * j + a] = lo;
      b.fhi[3 * j + a] = hi;
      b.cen[3 * j + a] = (lo + hi) * 0.5;
      rlo[a] = std::min(rlo[a], lo);
      rhi[a] = std::max(rhi[a], hi);
    }
    b.refs[j] = (int32_t)j;
  }
  double ex = rhi[0] - rlo[0], ey = rhi[1] - rlo[1], ez = rhi[2] - rlo[2];
  double l2 = (ex * ex + ey * ey) + ez * ez;
  b.inv_l2 = l2 > 0.0 ? 1.0 / l2 : 0.0;
  b.rec(0, n, 0);
  out->perm = b.refs;
  return out;
}

void or_tree_free(or_tree* t) { delete t; }
int64_t or_tree_size(const or_tree* t) { return t ? (int64_t)t->nodes.size() : -1; }
int32_t or_tree_depth(const or_tree* t) { return t ? t->depth : -1; }

int or_tree_export(const or_tree* t, double* lo, double* hi, int32_t* left, int32_t* right,
                   int32_t* first, int32_t* count, int32_t* depth, int32_t* axis,
                   int32_t* plane, int32_t* flags, double* cost, int32_t* perm) {
  if (!t) return -1;
  for (size_t i = 0; i < t->nodes.size(); ++i) {
    const or_tree::Node& nd = t->nodes[i];
    for (int a = 0; a < 3; ++a) {
      lo[3 * i + a] = nd.lo[a];
      hi[3 * i + a] = nd.hi[a];
    }
    left[i] = nd.left;
    right[i] = nd.right;
    first[i] = nd.first;
    count[i] = nd.count;
    depth[i] = nd.depth;
    axis[i] = nd.axis;
    plane[i] = nd.plane;
    flags[i] = nd.flags;
    cost[i] = nd.cost;
  }
  std::copy(t->perm.begin(), t->perm.end(), perm);
  return 0;
}

int or_trace_bvh(const float* tris, int64_t n, const or_tree* tree, const float* rays,
                 int64_t m, const int32_t* skip, int32_t nthreads, int32_t* id, double* t,
                 double* u, double* v, double* margin, double* t2, int32_t* nodes_visited,
                 int32_t* tris_tested) {
  if (!tris || !tree || !rays || !id || !t || !u || !v || m < 0) return -1;
  if ((int64_t)tree->perm.size() != n) return -1;
  parallel_for(m, nthreads, [&](int64_t i) {
    Ray r = load_ray(rays, i);
    Result res = bvh_one(tris, *tree, r, skip ? skip[i] : -1,
                         nodes_visited ? nodes_visited + i : nullptr,
                         tris_tested ? tris_tested + i : nullptr);
    store(res, i, id, t, u, v, margin, t2);
  });
  return 0;
}

}  // extern "C"

namespace {

// Stop rule of Sec. III-B by energy: after the reflection at hit j (facet
// f_j, path length l_j from the source to the hit point) the chain carries
// the power ratio P_j = (prod_{i <= j} g(f_i)) * k0 / l_j^2, where g is the
// power reflection coefficient of the facet's material and k0 = (lambda /
// (4 pi))^2 the free-space constant; the next segment is launched only while
// P_j >= min_power.  A material index outside [0, n_mat) reflects nothing.
struct EnergyRule {
  const int32_t* material;
  const double* refl;
  int32_t n_mat;
  double k0, min_power;
};

void chains(const float* tris, int64_t n, const or_tree* tree, const float* rays, int64_t m,
            int32_t max_b, int32_t nthreads, int32_t* id, double* t, double* u, double* v,
            double* margin, double* seg, double* path_len, int32_t* n_hits,
            const EnergyRule* en, double* power) {
  parallel_for(m, nthreads, [&](int64_t i) {
    Ray r = load_ray(rays, i);
    int32_t skip = -1, hits = 0;
    double path = 0.0, gain = 1.0, last_power = 0.0;
    int32_t b = 0;
    for (; b < max_b; ++b) {
      const int64_t k = (int64_t)b * m + i;
      if (seg) {
        double* s = seg + 8 * k;
        s[0] = r.o.x; s[1] = r.o.y; s[2] = r.o.z; s[3] = r.tmin;
        s[4] = r.d.x; s[5] = r.d.y; s[6] = r.d.z; s[7] = r.tmax;
      }
      Result res = tree ? bvh_one(tris, *tree, r, skip, nullptr, nullptr)
                        : brute_one(tris, n, r, skip);
      store(res, k, id, t, u, v, margin, nullptr);
      if (res.id < 0) break;
      ++hits;
      path += res.t * std::sqrt(dot(r.d, r.d));
      if (en) {
        const int32_t mat = en->material[res.id];
        gain *= (mat >= 0 && mat < en->n_mat) ? en->refl[mat] : 0.0;
        last_power = gain * en->k0 / (path * path);
        if (!(last_power >= en->min_power)) break;
      }
      r = reflect(tris, r, res);
      skip = res.id;
    }
    for (++b; b < max_b; ++b) {  // segments never launched
      const int64_t k = (int64_t)b * m + i;
      Result none;
      none.t = kInf;
      store(none, k, id, t, u, v, margin, nullptr);
      if (seg)
        for (int c = 0; c < 8; ++c) seg[8 * k + c] = std::numeric_limits<double>::quiet_NaN();
    }
    path_len[i] = path;
    n_hits[i] = hits;
    if (power) power[i] = last_power;
  });
}

}  // namespace

extern "C" {

int or_bounces(const float* tris, int64_t n, const or_tree* tree, const float* rays,
               int64_t m, int32_t max_b, int32_t nthreads, int32_t* id, double* t,
               double* u, double* v, double* margin, double* seg, double* path_len,
               int32_t* n_hits) {
  if (!tris || !rays || !id || !t || !u || !v || !path_len || !n_hits || max_b < 1) return -1;
  if (tree && (int64_t)tree->perm.size() != n) return -1;
  chains(tris, n, tree, rays, m, max_b, nthreads, id, t, u, v, margin, seg, path_len, n_hits,
         nullptr, nullptr);
  return 0;
}

int or_bounces_energy(const float* tris, int64_t n, const or_tree* tree, const float* rays,
                      int64_t m, int32_t max_b, int32_t nthreads, const int32_t* material,
                      const double* refl, int32_t n_mat, double k0, double min_power,
                      int32_t* id, double* t, double* u, double* v, double* margin, double* seg,
                      double* path_len, int32_t* n_hits, double* power) {
  if (!tris || !rays || !id || !t || !u || !v || !path_len || !n_hits || !power || max_b < 1 ||
      !material || n_mat < 0 || (n_mat > 0 && !refl))
    return -1;
  if (tree && (int64_t)tree->perm.size() != n) return -1;
  const EnergyRule en{material, refl, n_mat, k0, min_power};
  chains(tris, n, tree, rays, m, max_b, nthreads, id, t, u, v, margin, seg, path_len, n_hits, &en,
         power);
  return 0;
}

}  // extern "C"
