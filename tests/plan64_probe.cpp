// Test helper: the grouped-chain plan (gst_plan64.*) as flat arrays for the
// CPU tests, which execute it with numpy and compare with the oracle.
#include <cstring>

#include "gst_plan64.h"

namespace {
gst::Plan64 g;
int g_max_events = gst::Plan64Options().max_node_events;
}

extern "C" {

// Events per node the following builds allow (the library's bound by default;
// the CPU interpreter holds any number).
void plan64_set_max_events(int n) { g_max_events = n; }

// sizes: used, n_rows, n_tiles, n_levels, n_chains, n_slots, n_events,
//        n_records, words, tile steps, root_slot, root chains, n_nodes, chunks,
//        gradient tile-steps
int plan64_build(const int64_t* off, const uint8_t* gates, int64_t S, int K, double ratio, double fill,
                 int chunk, int64_t* sizes) {
  gst::Plan64Options opt;
  opt.max_row_ratio = ratio;
  opt.min_fill = fill;
  opt.chunk = chunk;
  opt.max_node_events = g_max_events;
  const bool used = gst::build_plan64(off, gates, S, K, opt, &g);
  const int64_t v[15] = {used, g.n_rows, g.n_tiles(), g.n_levels, g.n_chains, g.n_slots, (int64_t)g.ev_col.size(),
                         (int64_t)g.rec_b.size(), (int64_t)g.words.size(), g.tile_steps(), g.root_slot,
                         (int64_t)g.root_chains.size(), g.n_nodes, (int64_t)g.chunk_beg.size(),
                         (int64_t)g.ts_tile.size()};
  std::memcpy(sizes, v, sizeof v);
  return 0;
}

#define CP(dst, vec) std::memcpy(dst, g.vec.data(), g.vec.size() * sizeof(g.vec[0]))
void plan64_tiles(int64_t* level_tile_ptr, int64_t* row0, int32_t* len, int32_t* cols, int64_t* word,
                  int64_t* tev, int64_t* anchor, int64_t* chain, uint8_t* words) {
  CP(level_tile_ptr, level_tile_ptr); CP(row0, tile_row0); CP(len, tile_len); CP(cols, tile_cols);
  CP(word, tile_word); CP(tev, tile_ev); CP(anchor, col_anchor); CP(chain, col_chain); CP(words, words);
}
void plan64_events(int64_t* ev_ptr, int32_t* ev_col, int64_t* ev_src, int64_t* slot_row, int64_t* slot_ptr,
                   int64_t* slot_seq, int64_t* root_chains) {
  CP(ev_ptr, ev_ptr); CP(ev_col, ev_col); CP(ev_src, ev_src); CP(slot_row, slot_row); CP(slot_ptr, slot_ptr);
  CP(slot_seq, slot_seq); CP(root_chains, root_chains);
}
void plan64_records(int64_t* rec_b, int64_t* rec_f, int64_t* rec_gate_ptr, int64_t* chunk_beg, int64_t* chunk_end,
                    int64_t* gate_chunk_ptr) {
  CP(rec_b, rec_b); CP(rec_f, rec_f); CP(rec_gate_ptr, rec_gate_ptr); CP(chunk_beg, chunk_beg);
  CP(chunk_end, chunk_end); CP(gate_chunk_ptr, gate_chunk_ptr);
}
void plan64_ts(int64_t* ts_tile, int32_t* ts_step) {
  CP(ts_tile, ts_tile); CP(ts_step, ts_step);
}
// the per-tile-step column table (16 bytes per tile-step; none when the build
// allowed more than 15 events per node)
int64_t plan64_cend(uint8_t* out) {
  if (out) CP(out, ev_cend);
  return (int64_t)g.ev_cend.size();
}
#undef CP
}
