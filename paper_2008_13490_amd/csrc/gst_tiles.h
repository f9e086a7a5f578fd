// Tiles of the persistent batch kernels (host side, no device code).
//
// A request's sequences are sorted by length (descending, stable) and cut
// into tiles of a fixed number of sequences; tile t of a request owns row t of
// the request's partial-sum slab.  A batch lists the tiles of all its
// requests, longest first; a workgroup of the persistent kernel takes tiles
// from a queue and writes each one's partial sums into row `local` of its own
// request's slab (never a row derived from its workgroup index: the grid spans
// the tiles of every request, a slab only those of one).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace gst {

struct BatchTile {
  int32_t req;    // index into reqs
  int32_t local;  // tile index within its request (slab row)
  int64_t q0, q1; // positions in the request's order
};

// Length-sorted order of the S sequences of CSR `off` and the cut of that
// order into tiles of `tile_seqs` sequences: tile t covers positions
// tile_q[t] .. tile_q[t + 1] of `order`, cost[t] = the summed lengths.
void cut_tiles(const int64_t* off, int64_t S, int64_t tile_seqs, std::vector<int64_t>* order,
               std::vector<int64_t>* tile_q, std::vector<int64_t>* tile_cost);

// The tiles of a batch's requests (request x: its cut tile_q[x], costs
// tile_cost[x]), longest first; equal costs keep request and tile order.
std::vector<BatchTile> batch_tiles(const std::vector<const std::vector<int64_t>*>& tile_q,
                                   const std::vector<const std::vector<int64_t>*>& tile_cost,
                                   const std::vector<int>& req_index);

// Checks a batch's tile list against the requests' cuts: every tile names a
// request of the batch, its slab row is below that request's tile count, its
// range is that row's range of the cut, and every row of every request is
// listed exactly once.  Returns "" or a description of the first violation.
std::string check_batch_tiles(const std::vector<BatchTile>& tiles,
                              const std::vector<const std::vector<int64_t>*>& tile_q_of_req);

}  // namespace gst
