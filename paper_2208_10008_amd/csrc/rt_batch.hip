// Batched trace (declared in include/rt_mi355x.h): many queries -- trees,
// ray sets, bounce limits, optionally field points -- in one launch per node
// format (and per kind: plain chains, or chains with the reception test),
// optionally through a captured hipGraph, with a small autotuner over launch
// shapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rt_internal.h"

namespace rt {
namespace {

constexpr int kFormats = 3;
constexpr int kGroups = 2 * kFormats;  // group 2 f + r: node format f, r = 1 with field points

struct Group {  // the queries of one node format and kind, contiguous in the table
  int first = 0, count = 0, depth = 0;
  int64_t batches = 0;
};

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int query_error(const rt_query& q) {
  if (!q.bvh || q.bvh->info.n_tris <= 0) return RT_EINVAL;
  if (q.n < 0 || q.n >= (int64_t(1) << 40)) return RT_EINVAL;
  if (q.max_bounces < 1 || q.max_bounces > RT_MAX_BOUNCES) return RT_EINVAL;
  if (q.n > 0) {
    if (!q.rays || !q.out || !aligned(q.rays, 16) || !aligned(q.out, 16)) return RT_EINVAL;
    if ((q.path_len && !aligned(q.path_len, 8)) || (q.n_hits && !aligned(q.n_hits, 4)))
      return RT_EINVAL;
  }
  if (q.receivers) {  // reception records hold 32-bit ray numbers
    if (check_rx(q.receivers, "rt_batch_set",
                 {{q.out, (int64_t)q.max_bounces * q.n * 16}, {q.path_len, q.n * 8},
                  {q.n_hits, q.n * 4}}) != RT_OK ||
        q.n > INT32_MAX)
      return RT_EINVAL;
  }
  return RT_OK;
}

}  // namespace
}  // namespace rt

using namespace rt;

struct rt_batch {
  int32_t cap = 0;
  int device = 0;
  BatchQuery* staging = nullptr;  // pinned host [cap]
  BatchQuery* table = nullptr;    // device [cap]
  unsigned long long* queues = nullptr;  // device [kGroups]
  hipEvent_t copied = nullptr;    // the last launch has read the staging table
  hipStream_t capture = nullptr;  // private stream the graph is captured on
  bool pending = false;
  std::vector<rt_query> queries;  // the valid queries, as given
  Group groups[kGroups];
  int nq = 0;
  rt_batch_config cfg{RT_BATCH_DIRECT, 0, RT_ORDER_COST, 0};
  int grid[kGroups] = {0, 0, 0, 0, 0, 0};  // persistent work-groups per group (QUEUE mode)
  // captured graph and the shape it was captured for
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> graph_key;
};

namespace {

void free_batch(rt_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->copied) (void)hipEventDestroy(b->copied);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->staging) (void)hipHostFree(b->staging);
  if (b->table) (void)hipFree(b->table);
  if (b->queues) (void)hipFree(b->queues);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Lays the valid queries out in the staging table: grouped by node format
// and kind, in the configured order, each with its first work-group number.
// A query with field points and no rays still takes its place (its count is
// cleared by the launch).
void layout(rt_batch* b) {
  std::vector<int> idx(b->queries.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  if (b->cfg.order == RT_ORDER_COST) {
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      const rt_query& a = b->queries[x];
      const rt_query& c = b->queries[y];
      return a.n * (int64_t)a.max_bounces > c.n * (int64_t)c.max_bounces;
    });
  }
  int pos = 0;
  for (int gi = 0; gi < kGroups; ++gi) {
    const int f = gi / 2;
    const bool rv = gi % 2;
    Group& g = b->groups[gi];
    g = Group();
    g.first = pos;
    for (int i : idx) {
      const rt_query& q = b->queries[i];
      if (q.bvh->info.node_format != f || (q.receivers != nullptr) != rv) continue;
      if (q.n == 0 && !rv) continue;
      BatchQuery e;
      std::memset(&e, 0, sizeof(e));
      const Buffers& B = q.bvh->buf;
      e.nodes = f == RT_NODE_BIN2 ? (const void*)B.tnodes : (const void*)B.wnodes;
      e.facets = B.tfacets;
      e.rays = reinterpret_cast<const float4*>(q.rays);
      e.out = q.out;
      e.path_len = q.path_len;
      e.n_hits = q.n_hits;
      e.n = q.n;
      e.first_batch = g.batches;
      e.max_b = q.max_bounces;
      if (rv) e.recv = recv_args(q.receivers);
      b->staging[pos++] = e;
      ++g.count;
      g.batches += (q.n + 63) / 64;
      g.depth = std::max(g.depth, (int)q.bvh->info.depth);
    }
  }
  b->nq = pos;
}

std::vector<int64_t> shape_key(const rt_batch* b) {
  std::vector<int64_t> k = {b->cfg.mode, b->cfg.grid, b->cfg.order, b->nq};
  for (int gi = 0; gi < kGroups; ++gi) {
    k.push_back(b->groups[gi].first);
    k.push_back(b->groups[gi].count);
    k.push_back(b->groups[gi].depth);
    k.push_back(b->groups[gi].batches);
  }
  return k;
}

// Persistent work-group counts for the QUEUE mode (before any capture).
void plan_grids(rt_batch* b) {
  for (int gi = 0; gi < kGroups; ++gi) {
    const Group& g = b->groups[gi];
    b->grid[gi] = 0;
    if (b->cfg.mode == RT_BATCH_QUEUE && g.count)
      b->grid[gi] = b->cfg.grid > 0 ? b->cfg.grid : trace_resident_groups(gi / 2, gi % 2, g.depth);
  }
}

// The table upload, the reception counts cleared, and one launch per group
// present, on stream s.
int enqueue(rt_batch* b, hipStream_t s) {
  int rc = check_hip(hipMemcpyAsync(b->table, b->staging, sizeof(BatchQuery) * std::max(b->nq, 1),
                                    hipMemcpyHostToDevice, s),
                     "rt_batch_launch: table upload");
  if (rc != RT_OK) return rc;
  for (int gi = 1; gi < kGroups; gi += 2) {
    const Group& g = b->groups[gi];
    if (g.count == 0) continue;
    rc = launch_batch_clear_counts(b->table + g.first, g.count, s);
    if (rc != RT_OK) return rc;
  }
  for (int gi = 0; gi < kGroups; ++gi) {
    const Group& g = b->groups[gi];
    if (g.count == 0 || g.batches == 0) continue;
    rc = launch_trace_batch(b->table + g.first, g.count, g.batches, gi / 2, gi % 2, g.depth,
                            b->grid[gi], b->queues + gi, s);
    if (rc != RT_OK) return rc;
  }
  return RT_OK;
}

int launch(rt_batch* b, hipStream_t s) {
  if (b->nq == 0) return RT_OK;
  int rc;
  plan_grids(b);
  if (b->cfg.graph) {
    // captured on the batch's own stream, launched on the caller's
    const std::vector<int64_t> key = shape_key(b);
    if (!b->exec || key != b->graph_key) {
      if (b->exec) (void)hipGraphExecDestroy(b->exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->exec = nullptr;
      b->graph = nullptr;
      rc = check_hip(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal),
                     "graph capture");
      if (rc != RT_OK) return rc;
      const int erc = enqueue(b, b->capture);
      hipGraph_t g = nullptr;
      rc = check_hip(hipStreamEndCapture(b->capture, &g), "graph capture end");
      if (erc != RT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return erc;
      }
      if (rc != RT_OK) return rc;
      b->graph = g;
      rc = check_hip(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
      if (rc != RT_OK) return rc;
      b->graph_key = key;
    }
    rc = check_hip(hipGraphLaunch(b->exec, s), "graph launch");
  } else {
    rc = enqueue(b, s);
  }
  if (rc != RT_OK) return rc;
  rc = check_hip(hipEventRecord(b->copied, s), "rt_batch_launch: event");
  if (rc != RT_OK) return rc;
  b->pending = true;
  return RT_OK;
}

int check_config(const rt_batch_config* c) {
  if (!c) return set_error(RT_EINVAL, "rt_batch_configure: NULL config");
  if ((c->mode != RT_BATCH_DIRECT && c->mode != RT_BATCH_QUEUE) || c->grid < 0 ||
      (c->order != RT_ORDER_GIVEN && c->order != RT_ORDER_COST) || (c->graph != 0 && c->graph != 1))
    return set_error(RT_EINVAL, "rt_batch_configure: mode 0/1, grid >= 0, order 0/1, graph 0/1");
  return RT_OK;
}

}  // namespace

extern "C" {

int rt_batch_create(int32_t max_queries, rt_batch** out) {
  if (!out) return set_error(RT_EINVAL, "rt_batch_create: out is NULL");
  *out = nullptr;
  if (max_queries < 1 || max_queries > 65536)
    return set_error(RT_EINVAL, "rt_batch_create: max_queries must lie in 1..65536");
  rt_batch* b = new (std::nothrow) rt_batch();
  if (!b) return set_error(RT_ENOMEM, "rt_batch_create: host allocation failed");
  b->cap = max_queries;
  (void)hipGetDevice(&b->device);
  int rc = check_hip(hipHostMalloc((void**)&b->staging, sizeof(BatchQuery) * max_queries),
                     "hipHostMalloc");
  if (rc == RT_OK)
    rc = check_hip(hipMalloc((void**)&b->table, sizeof(BatchQuery) * max_queries), "hipMalloc");
  if (rc == RT_OK)
    rc = check_hip(hipMalloc((void**)&b->queues, sizeof(unsigned long long) * kGroups), "hipMalloc");
  if (rc == RT_OK) rc = check_hip(hipEventCreateWithFlags(&b->copied, hipEventDisableTiming), "event");
  if (rc == RT_OK) rc = check_hip(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "stream");
  if (rc != RT_OK) {
    free_batch(b);
    delete b;
    return rc;
  }
  *out = b;
  return RT_OK;
}

int rt_batch_set(rt_batch* b, rt_query* queries, int32_t nq) {
  if (!b) return set_error(RT_EINVAL, "rt_batch_set: NULL batch");
  if (nq < 0 || nq > b->cap) return set_error(RT_EINVAL, "rt_batch_set: nq outside 0..max_queries");
  if (nq > 0 && !queries) return set_error(RT_EINVAL, "rt_batch_set: queries is NULL");
  if (b->pending) {
    int rc = check_hip(hipEventSynchronize(b->copied), "rt_batch_set: wait");
    if (rc != RT_OK) return rc;
    b->pending = false;
  }
  b->queries.clear();
  for (int i = 0; i < nq; ++i) {
    queries[i].status = query_error(queries[i]);
    if (queries[i].status == RT_OK) b->queries.push_back(queries[i]);
  }
  layout(b);
  return RT_OK;
}

int rt_batch_configure(rt_batch* b, const rt_batch_config* cfg) {
  if (!b) return set_error(RT_EINVAL, "rt_batch_configure: NULL batch");
  int rc = check_config(cfg);
  if (rc != RT_OK) return rc;
  const bool relayout = cfg->order != b->cfg.order;
  if (relayout && b->pending) {
    rc = check_hip(hipEventSynchronize(b->copied), "rt_batch_configure: wait");
    if (rc != RT_OK) return rc;
    b->pending = false;
  }
  b->cfg = *cfg;
  if (relayout) layout(b);
  return RT_OK;
}

int rt_batch_get_config(const rt_batch* b, rt_batch_config* cfg) {
  if (!b || !cfg) return set_error(RT_EINVAL, "rt_batch_get_config: NULL argument");
  *cfg = b->cfg;
  return RT_OK;
}

int rt_batch_launch(rt_batch* b, hipStream_t s) {
  if (!b) return set_error(RT_EINVAL, "rt_batch_launch: NULL batch");
  return launch(b, s);
}

int rt_batch_autotune(rt_batch* b, int32_t reps, hipStream_t s, float* ms) {
  if (!b) return set_error(RT_EINVAL, "rt_batch_autotune: NULL batch");
  if (reps < 1 || reps > 1000) return set_error(RT_EINVAL, "rt_batch_autotune: reps in 1..1000");
  const rt_batch_config keep = b->cfg;
  std::vector<rt_batch_config> cands;
  for (int order : {RT_ORDER_COST, RT_ORDER_GIVEN}) {
    cands.push_back({RT_BATCH_DIRECT, 0, order, 0});
    cands.push_back({RT_BATCH_QUEUE, 0, order, 0});
  }
  int res = 0;
  for (int gi = 0; gi < kGroups; ++gi)
    if (b->groups[gi].count)
      res = std::max(res, trace_resident_groups(gi / 2, gi % 2, RT_MAX_DEPTH));
  cands.push_back({RT_BATCH_QUEUE, 2 * std::max(res, 1), RT_ORDER_COST, 0});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = check_hip(hipEventCreate(&e0), "event");
  if (rc == RT_OK) rc = check_hip(hipEventCreate(&e1), "event");
  float best = -1.f;
  rt_batch_config best_cfg = keep;
  for (size_t c = 0; c < cands.size() && rc == RT_OK; ++c) {
    rc = rt_batch_configure(b, &cands[c]);
    if (rc == RT_OK) rc = launch(b, s);  // warm-up
    if (rc == RT_OK) rc = check_hip(hipEventRecord(e0, s), "event");
    for (int r = 0; r < reps && rc == RT_OK; ++r) rc = launch(b, s);
    if (rc == RT_OK) rc = check_hip(hipEventRecord(e1, s), "event");
    if (rc == RT_OK) rc = check_hip(hipEventSynchronize(e1), "event sync");
    float t = 0.f;
    if (rc == RT_OK) rc = check_hip(hipEventElapsedTime(&t, e0, e1), "event time");
    if (rc == RT_OK && (best < 0.f || t < best)) {
      best = t;
      best_cfg = cands[c];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  best_cfg.graph = keep.graph;
  const int rc2 = rt_batch_configure(b, rc == RT_OK ? &best_cfg : &keep);
  if (rc != RT_OK) return rc;
  if (ms) *ms = best / reps;
  return rc2;
}

void rt_batch_destroy(rt_batch* b) {
  if (!b) return;
  if (b->pending) (void)hipEventSynchronize(b->copied);
  (void)hipDeviceSynchronize();
  free_batch(b);
  delete b;
}

}  // extern "C"
