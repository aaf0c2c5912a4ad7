// Phase thresholds of the tree build and the scratch capacities that follow
// from them.  Shared by the allocator (rt_api.hip) and the build
// (rt_build.hip); the traversal does not depend on them.  They change only
// which kernel splits a node, never the split: node ids come from facet
// positions and every phase takes the same float64 decisions.
#pragma once

#include <stdint.h>

namespace rt {

constexpr int kChunk = 512;    // facets per big-node chunk
constexpr int kBigNode = 512;  // nodes above this many facets are split chunk-wise
constexpr int kRegNode = 12;   // subtrees at or below this many facets stay in registers
inline int64_t item_capacity(int64_t n) { return n / kChunk + n / (kBigNode + 1) + 2; }
inline int64_t anode_capacity(int64_t n) { return n / (kBigNode + 1) + 1; }

}  // namespace rt
