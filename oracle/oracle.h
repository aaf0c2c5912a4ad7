/* CPU checker for the closest-hit ray tracing path: TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, float64 reference of what the GPU path computes.  Only the
 * tests, the package smoke check and the benchmark's CPU-baseline leg may
 * load it; the product path never calls it.  It shares no code, header or
 * constant with the GPU library.
 *
 * Inputs are the same float32 arrays the GPU path takes, promoted exactly
 * to float64:
 *   tris  float32 [n][9]  (v0.xyz, v1.xyz, v2.xyz), caller order
 *   rays  float32 [m][8]  (ox, oy, oz, tmin, dx, dy, dz, tmax)
 *
 * Parity status of every function is written in its comment. */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* margins are reported as min(margin, OR_MARGIN_CAP) */
#define OR_MARGIN_CAP 1e-3

typedef struct or_params {
  double alpha;      /* Eq. (2) weight in [0, 1]                               */
  double t_isect;    /* t_i of Eq. (1)/(2)                                     */
  double t_trav;     /* t_trav of Eq. (1)/(2)                                  */
  double src[3];     /* ray source point of the distance term                 */
  int32_t max_leaf;  /* leaf iff facet count <= max_leaf                       */
  int32_t nbins;     /* centroid bins per axis                                 */
  int32_t d_mode;    /* 0 mean of child d^2, 1 sum, 2 count-weighted, 3 parent */
  int32_t d_norm;    /* 0 unit-normalised terms, 1 raw (printed) units        */
  int32_t max_depth; /* from this depth on alpha is taken as 1                 */
  int32_t depth_limit; /* no leaf deeper than this (forced halving)            */
} or_params;

typedef struct or_tree or_tree;

/* Closest hit by definition: every ray against every facet (Moller-Trumbore
 * in float64), closed [tmin, tmax], ties on t to the smaller facet id.
 * skip (nullable): per ray, a facet id that is ignored (-1: none).
 * Outputs per ray: id (-1 miss), t (+inf miss), u, v, margin (capped),
 * t2 (next hit of another facet when its relative gap is below the cap,
 * +inf otherwise).  Returns 0. */
int or_brute(const float* tris, int64_t n, const float* rays, int64_t m,
             const int32_t* skip, int32_t nthreads, int32_t* id, double* t,
             double* u, double* v, double* margin, double* t2);

/* Float64 crossing of ray i with facet ids[i] (ids[i] < 0: zeros).
 * valid[i] = 0 when the ray is parallel to the facet plane (det == 0). */
int or_eval(const float* tris, int64_t n, const float* rays, int64_t m,
            const int32_t* ids, int32_t* valid, double* t, double* u, double* v);

/* The paper's top-down build (Sec. II-C) with the Eq. (2) split cost on
 * binned centroid candidates; returns NULL on bad arguments. */
or_tree* or_build(const float* tris, int64_t n, const or_params* p);
void or_tree_free(or_tree* t);
int64_t or_tree_size(const or_tree* t);
int32_t or_tree_depth(const or_tree* t);
/* Node arrays in depth-first pre-order (root = 0); lo/hi [nn][3];
 * left/right = child node ids (-1 for a leaf); [first, first + count) is the
 * node's range in perm; flags bit0 = forced halving, bit1 = all centroids
 * equal, bit2 = alpha taken as 1 by depth. */
int or_tree_export(const or_tree* t, double* lo, double* hi, int32_t* left,
                   int32_t* right, int32_t* first, int32_t* count, int32_t* depth,
                   int32_t* axis, int32_t* plane, int32_t* flags, double* cost,
                   int32_t* perm);

/* Sec. III-B traversal of the oracle's own tree in float64.  Produces the
 * same outputs as or_brute (identical id and t, identical capped margins):
 * boxes are inflated so that every facet able to lower a margin below the
 * cap is still tested.  nodes_visited / tris_tested (nullable) per ray. */
int or_trace_bvh(const float* tris, int64_t n, const or_tree* tree,
                 const float* rays, int64_t m, const int32_t* skip,
                 int32_t nthreads, int32_t* id, double* t, double* u, double* v,
                 double* margin, double* t2, int32_t* nodes_visited,
                 int32_t* tris_tested);

/* Reflection chains in float64 (Sec. III-B): up to max_b segments per ray;
 * after a hit the ray is reflected specularly about the facet plane, starts
 * at the hit point, keeps the primary ray's [tmin, tmax] and skips the facet
 * it left.  Per segment b and ray i (index b * m + i): id, t, u, v, margin;
 * seg (nullable) [max_b * m][8] float64 segment rays; path_len per ray =
 * sum over hits of t * |d|; n_hits per ray.  tree == NULL: brute force. */
int or_bounces(const float* tris, int64_t n, const or_tree* tree,
               const float* rays, int64_t m, int32_t max_b, int32_t nthreads,
               int32_t* id, double* t, double* u, double* v, double* margin,
               double* seg, double* path_len, int32_t* n_hits);

/* or_bounces with the energy stop rule of Sec. III-B: after the reflection at
 * hit j the chain carries P_j = (prod of refl[material[f_i]] over its hits)
 * * k0 / l_j^2 (l_j: path length to the hit, k0 = (lambda / 4 pi)^2); the next
 * segment is launched only while P_j >= min_power.  material [n] per facet id
 * (index outside [0, n_mat): reflects nothing); power [m] = P of the last hit,
 * 0 without hits. */
int or_bounces_energy(const float* tris, int64_t n, const or_tree* tree, const float* rays,
                      int64_t m, int32_t max_b, int32_t nthreads, const int32_t* material,
                      const double* refl, int32_t n_mat, double k0, double min_power,
                      int32_t* id, double* t, double* u, double* v, double* margin, double* seg,
                      double* path_len, int32_t* n_hits, double* power);

#ifdef __cplusplus
}
#endif
#endif
