// Sharing plan with grouped chains (host side, no device code).
//
// Thesis Eq. GSTFullFiducialsGerms: every GST sequence is F_q g^l F_p.  In
// the trie of such a list, the chain g^l_max hanging below the preparation
// fiducial F_p has the same gate word for every p, and the short chains of the
// measurement fiducials hanging off every germ power have the same few words
// for every (p, g, l).  The plan cuts the trie into chains (heavy paths: a
// chain continues into the child with the deepest subtree) and puts chains
// with the same word at the same depth of the chain tree side by side, sixteen
// to a tile.  A tile applies one gate to all its chains at once, a 64 x 64
// transfer matrix times a 64 x 16 block of states: a dense product for the
// matrix cores, where the per-sequence evaluation is sixteen separate
// matrix-vector products.
//
// Rows.  Every trie node except the root owns a row of the state arena FA
// and of the adjoint arena BA; row 0 of FA is rho (the root).  Column c of a
// tile at step t (0-based) owns row tile_row0 + 16 t + c, so one step of a
// tile writes sixteen consecutive rows.  Columns beyond a tile's chains carry
// rho-anchored padding and are never read.
//
// Readouts and adjoints.  A sequence ends at its terminal node; all sequences
// ending at one node (duplicate words) form one seed slot.  The readout of a
// slot gives p for each of its sequences, and its seed, E^T (sum of the
// sequences' dL/dp), is the adjoint that the readouts deliver to the node.  In
// the reverse sweep of a chain the adjoint of every node is the sum of its
// seed, of the adjoints that chains anchored at the node deliver, and of the
// next node's adjoint carried back through the next gate.  All such vectors
// live in one array INJ: rows [0, n_slots) are seeds, rows n_slots + chain id
// the adjoint a chain delivers to its anchor.
#pragma once
#include <stdint.h>

#include <vector>

namespace gst {

// Events of one node at most: its seed and the chains anchored there, at most
// one per child (K <= 5 for three qubits; a chain that ends at a node leaves
// every child to chains anchored there); plans that would need more are refused.
constexpr int kMaxNodeEvents = 6;

struct Plan64Options {
  int tile_cols = 16;                 // chains per tile (the MFMA width)
  double max_row_ratio = 0.5;         // use the plan only if its rows (padding included) <= ratio * total steps
  double min_fill = 0.0;              // ... and live columns fill at least this share of tile rows
  int64_t max_nodes = 1LL << 26;
  int chunk = 8192;                   // gradient records per chunk (the records of the CPU tests)
  int ts_chunk = 64;                  // tile-steps per chunk of the gradient GEMM (<= GEMM64_TS_CHUNK_MAX)
  int max_node_events = kMaxNodeEvents;  // refuse plans with more events at one node
  int split_height = 32;              // a chain ends at a node with two children of at least this height
  bool short_asap = false;            // short chains run as soon as they are ready (else: in full tiles)
};

struct Plan64 {
  int K = 0;
  int64_t S = 0, sum_len = 0, n_nodes = 0, max_len = 0;
  int64_t n_rows = 0;                 // FA rows (row 0 = rho) = BA rows
  int64_t n_chains = 0, n_slots = 0;
  int64_t live_rows = 0;              // rows of real chain nodes (n_nodes - 1)
  // tiles, level by level; a tile's chains share their word and level
  int n_levels = 0;
  std::vector<int64_t> level_tile_ptr;   // [n_levels + 1]
  std::vector<int64_t> tile_row0;        // [n_tiles]
  std::vector<int32_t> tile_len;         // steps of the tile's word
  std::vector<int32_t> tile_cols;        // live columns
  std::vector<int64_t> tile_word;        // offset of the word in `words`
  std::vector<int64_t> tile_ev;          // offset of step 0 of the tile in ev_ptr
  std::vector<int64_t> col_anchor;       // [n_tiles * 16] FA row of the column's anchor (0 = rho)
  std::vector<int64_t> col_chain;        // [n_tiles * 16] chain id (-1 = padding)
  std::vector<uint8_t> words;
  // events of (tile, step): the INJ rows added to column `ev_col` before the
  // reverse sweep stores that step's adjoint (seed first, then chains by id)
  std::vector<int64_t> ev_ptr;           // [sum of tile lengths + 1]
  std::vector<int32_t> ev_col;           // ascending within a tile-step
  std::vector<int64_t> ev_src;
  // per tile-step 16 bytes, so that a column finds its events without a scan:
  // byte c < 15 counts the step's events of columns <= c, byte 15 is the most
  // events of one column (empty when the options allow more than 15 events
  // at a node: such plans only serve the host-side interpreter)
  std::vector<uint8_t> ev_cend;
  // readouts: slot -> FA row of its node, its sequences (ascending)
  std::vector<int64_t> slot_row;         // [n_slots]
  std::vector<int64_t> slot_ptr;         // [n_slots + 1]
  std::vector<int64_t> slot_seq;         // [S]
  // the root: seed slot of the empty words (-1 none) and chains anchored at rho
  int64_t root_slot = -1;
  std::vector<int64_t> root_chains;
  // gradient records grouped by gate: dG_k += BA[rec_b] FA[rec_f]^T
  std::vector<int64_t> rec_b, rec_f;
  std::vector<int64_t> rec_gate_ptr;     // [K + 1]
  // the same records as tile-steps (sixteen records each: the rows of the tile's
  // columns at step t, and the rows before them), grouped by gate, in chunks of
  // at most `ts_chunk` tile-steps of one gate
  std::vector<int64_t> ts_tile;          // tile of each tile-step
  std::vector<int32_t> ts_step;          // its step
  std::vector<int64_t> chunk_beg, chunk_end, gate_chunk_ptr;  // ranges of tile-steps; [K + 1]
  int64_t n_tiles() const { return (int64_t)tile_row0.size(); }
  int64_t tile_steps() const { return (int64_t)ev_ptr.size() - 1; }
};

// Builds the plan; false when sharing saves too little (or the trie is too
// large), and the sequences are then evaluated one by one.  Gate indices must
// already be validated (< K).
bool build_plan64(const int64_t* offsets, const uint8_t* gates, int64_t S, int K, const Plan64Options& opt,
                  Plan64* out);

}  // namespace gst
