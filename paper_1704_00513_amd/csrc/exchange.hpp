// Launchers of the candidate exchange of the compressed 2D BFS (bfs.hip):
// the owners' unfiltered candidate sets as a batch of segments, and the
// receiver's merge and visited filter.
#pragma once

#include "common.hpp"

namespace bfsc {

size_t ex_ws_bytes(uint32_t V, uint64_t n_arcs, uint32_t nseg);
int launch_ex_init(bfsc_ctx *ctx, uint32_t V, uint64_t n_arcs, uint32_t nseg, void *ws, hipStream_t s);
int launch_candidates(bfsc_ctx *ctx, const bfsc_csr *g, const uint32_t *frontier, const uint32_t *frontier_len,
                      const uint32_t *bounds, uint32_t nseg, uint32_t *ids, uint64_t cap, uint64_t *seg_off,
                      uint32_t *seg_lo, uint32_t *seg_hi, void *ws, hipStream_t s);
int launch_merge_filter(bfsc_ctx *ctx, const bfsc_csr *g, int32_t cur_level, const uint32_t *ids,
                        const uint64_t *n_dev, int32_t *level, uint32_t *next, uint32_t *next_len, void *bfs_ws,
                        void *ws, hipStream_t s);

}  // namespace bfsc
