// C entry points over the library's host-side tile code (gst_tiles.cpp) for
// the CPU tests: cut requests into tiles, list a batch's tiles as the batch
// kernels receive them, and run the library's own check on that list.
#include <cstring>
#include <string>
#include <vector>

#include "gst_tiles.h"

static std::string g_msg;

extern "C" {

// Requests r = 0..n_req-1 with CSR offsets off[r] (S[r] sequences) and tile
// sizes tile_seqs[r].  Writes the batch's tiles (req, local, q0, q1) into
// out[4 * i ..] (at most cap tiles); corrupt >= 0 changes tile `corrupt`'s
// slab row to `corrupt_local` before the check.  Returns the tile count, or
// -1 if the check failed (message in tiles_msg()).
long tiles_batch(int n_req, const long* const* off, const long* S, const long* tile_seqs, long* out, long cap,
                 long corrupt, long corrupt_local) {
  std::vector<std::vector<int64_t>> order(n_req), q(n_req), cost(n_req);
  std::vector<const std::vector<int64_t>*> qp, cp;
  std::vector<int> idx;
  for (int r = 0; r < n_req; ++r) {
    gst::cut_tiles(reinterpret_cast<const int64_t*>(off[r]), S[r], tile_seqs[r], &order[r], &q[r], &cost[r]);
    qp.push_back(&q[r]);
    cp.push_back(&cost[r]);
    idx.push_back(r);
  }
  std::vector<gst::BatchTile> t = gst::batch_tiles(qp, cp, idx);
  if (corrupt >= 0 && corrupt < (long)t.size()) t[corrupt].local = (int32_t)corrupt_local;
  g_msg = gst::check_batch_tiles(t, qp);
  for (size_t i = 0; i < t.size() && (long)i < cap; ++i) {
    out[4 * i] = t[i].req;
    out[4 * i + 1] = t[i].local;
    out[4 * i + 2] = t[i].q0;
    out[4 * i + 3] = t[i].q1;
  }
  return g_msg.empty() ? (long)t.size() : -1;
}

const char* tiles_msg() { return g_msg.c_str(); }
}
