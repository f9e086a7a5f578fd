// Prefix-sharing plan of a sequence list (host side).
//
// Thesis Eq. GSTFullFiducialsGerms: GST sequences are F_q g^l F_p, so for a
// fixed preparation fiducial and germ every power g^l is a prefix of the
// next one, and all measurement fiducials of one (p, g, l) share F_p g^l.
// The plan is a trie of the sequences in time order; every distinct prefix
// state is computed once.
//
// Decomposition:
//   * long chains of the trie ("trunks", heavy paths by remaining depth) are
//     evaluated by one team each; the state after every step is stored;
//   * every sequence becomes a work item for the sequence kernel: it starts
//     from the deepest stored state on its path (or rho) and applies the rest
//     of its own word (usually the measurement fiducial);
//   * in the reverse sweep the adjoints of the items are summed per stored
//     state ("injections") and the trunks carry them back to rho.
// Without germ-power jumps the probabilities computed this way are the same
// floating-point numbers as those of the plain per-sequence evaluation: the
// shared prefixes are the same operations on the same values.  A jump applies
// a matrix power of a germ instead of its gates one by one, which changes the
// rounding of the states after it (not their value in exact arithmetic).
#pragma once
#include <stdint.h>

#include <vector>

namespace gst {

struct HostPlan {
  int K = 0;
  int64_t S = 0;
  int64_t sum_len = 0;        // total steps of the plain evaluation
  int64_t n_nodes = 0;        // distinct prefixes (trie nodes, root included)
  int64_t max_len = 0;        // longest sequence
  // trunks, sorted by level then by length (descending)
  int n_levels = 0;
  std::vector<int64_t> trunk_level_ptr;  // [n_levels + 1] trunk index ranges per level
  std::vector<int64_t> trunk_anchor;     // [n_trunks] state location of the anchor, -1 = rho
  std::vector<int64_t> trunk_ptr;        // [n_trunks + 1] step ranges in trunk_gates / state locations
  std::vector<uint8_t> trunk_gates;      // [trunk_steps]
  std::vector<int32_t> trunk_inj;        // [trunk_steps] injection slot of the node reached by the step, -1 none
  std::vector<int64_t> trunk_anchor_inj; // [n_trunks] injection slot that receives the adjoint at the anchor (-1 = rho)
  int64_t trunk_max_len = 0;
  // items: (seq, beg, end, anchor location), sorted by end - beg descending
  std::vector<int64_t> items;            // [n_items * 4]
  std::vector<uint8_t> item_kv;          // [n_items * 16] the first 16 gate indices of each item's word, 0 past its end
  int64_t item_max_len = 0;
  // injection slots: state location and the items / trunks feeding it
  std::vector<int64_t> inj_loc;          // [n_inj]
  std::vector<int64_t> inj_ptr;          // [n_inj + 1] ranges into inj_src
  std::vector<int64_t> inj_src;          // item indices (>= 0) or -(trunk index + 1)
  // the last injection slot (location -1) collects the adjoints that trunks
  // anchored at rho carry back (added to dF/drho).
  int64_t root_slot = -1;
  // reverse-sweep records for the grouped gradient GEMM
  //   state rows:   0 = rho, 1 + j = state after trunk step j,
  //                 1 + trunk_steps + x = state before item step x
  //   adjoint rows: j = after trunk step j, trunk_steps + x = after item step x
  std::vector<int64_t> item_step_ptr;    // [n_items + 1] item step ranges
  std::vector<int64_t> rec_b, rec_f;     // [n_rec] adjoint row, state row; grouped by gate
  std::vector<int64_t> rec_gate_ptr;     // [K + 1]
  std::vector<int64_t> chunk_gate, chunk_beg, chunk_end;  // record chunks of one gate each
  // each trunk's gate word as periodic segments: pattern of period 1..4 repeated
  // `count` times (germ powers of Eq. GSTFullFiducialsGerms are such runs)
  std::vector<int64_t> seg_ptr;          // [n_trunks + 1]
  std::vector<int32_t> seg_start;        // step of the segment's first gate within its trunk
  std::vector<int32_t> seg_count;        // repetitions of the pattern
  std::vector<uint32_t> seg_pattern;     // period in bits 0..7, gates in bits 8..15, 16..23, 24..31 and
  std::vector<uint8_t> seg_gate3;        // the fourth gate
  std::vector<int64_t> seg_inj;          // injection slot of the state after the segment's last step, -1 none
  // Germ-power jumps.  A long periodic run of a trunk's jump pattern (one
  // pattern per trunk, its germ) is applied several repetitions at a time by
  // a power of the pattern's product matrix: a jump segment has period 0 in
  // seg_pattern, the steps per jump in bits 8..15 and e in bits 16..23, the
  // matrix being the pattern product to the power 2^e.  The chain then
  // stores only the state after each jump; the states inside a jump are
  // written by independent fill tasks that start from the stored state
  // before it.
  int jump_levels = 0;                   // e = 0 .. jump_levels - 1 (the most any trunk uses)
  std::vector<uint32_t> trunk_jump_pattern;  // [n_trunks] period and gates as in seg_pattern, 0 = no jumps
  std::vector<uint8_t> trunk_jump_gate3;     // fourth gate of the pattern
  std::vector<uint8_t> trunk_jump_levels;    // the trunk's levels (its longest jump: 2^(levels-1) repetitions)
  std::vector<int64_t> fill_first;       // [n_fill] trunk-arena index of the task's first step
  std::vector<int64_t> fill_in;          // state row (0 = rho, 1 + j = after trunk step j) before that step
  std::vector<int32_t> fill_n;           // steps covered by the jump (n - 1 states are filled)
  std::vector<uint32_t> fill_pattern;    // pattern repeated over the n steps
  std::vector<uint8_t> fill_gate3;
  // The trunk chains as flat op lists (what the trunk kernels run): an op is
  // one gate step or one jump; bits 0..6 hold the gate index, or the jump
  // level e with bit 7 set, and bits 8..15 the steps it spans.  op_slot is
  // the injection slot of the state after the op (-1 none).
  std::vector<int64_t> op_ptr;           // [n_trunks + 1]
  std::vector<uint32_t> op_desc;
  std::vector<int32_t> op_slot;
  // The adjoints that reach stored states, in source order: source z of the
  // injection lists (z < inj_ptr[root_slot]) is row z of the source arena, so
  // the sources of slot s are rows inj_ptr[s] .. inj_ptr[s + 1] - 1.  Item q
  // writes its adjoint to row item_src[q] and trunk t to row trunk_src[t]
  // (-1: anchored at rho, no row).
  std::vector<int32_t> item_src, trunk_src;
  int64_t n_items() const { return (int64_t)items.size() / 4; }
  int64_t n_trunks() const { return (int64_t)trunk_anchor.size(); }
  int64_t trunk_steps() const { return (int64_t)trunk_gates.size(); }
  int64_t plan_steps() const;            // trunk steps + item steps
  int64_t item_steps() const { return item_step_ptr.empty() ? 0 : item_step_ptr.back(); }
  int64_t n_chunks() const { return (int64_t)chunk_gate.size(); }
  int64_t n_fill() const { return (int64_t)fill_first.size(); }
  int64_t n_src_rows() const { return root_slot < 0 ? 0 : inj_ptr[root_slot]; }
  int64_t n_jump_trunks() const {
    int64_t n = 0;
    for (uint32_t p : trunk_jump_pattern) n += p != 0;
    return n;
  }
};

struct PlanOptions {
  int min_trunk = 24;        // shortest chain that is stored
  int reanchor_depth = 8;    // chains branching off at depth <= this restart from rho
  double max_share_ratio = 0.8;  // use the plan only if plan_steps <= ratio * sum_len
  int64_t max_nodes = 1LL << 26;
  int64_t max_item_steps = 1LL << 24;   // bound on stored item-step states (memory)
  int chunk = 128;                      // gradient GEMM records per chunk (the kernel takes at most 128)
  int jump = 8;                         // repetitions per germ-power jump (power of two, <= 16); 0 = none
  int jump_span = 16;                   // ... or more, a power of two, while a jump spans at most this many steps
  int jump_min_save = 3;                // jump a run only if it shortens the chain by this many steps
  int rep_anchor_min = 4;               // inside a periodic run of a trunk's word with at least this many
                                        // repetitions, items start only at repetition boundaries (0 = anywhere)
  int anchor_min_share = 6;             // ... and an item whose start state fewer items share moves back to
  int anchor_max_back = 12;             // an earlier boundary of the run that as many share, at most this far
};

// Builds the plan.  Returns false (plan unused: evaluate sequence by
// sequence) when sharing saves too little or the trie would be too large.
// Gate indices must already be validated (< K).
bool build_plan(const int64_t* offsets, const uint8_t* gates, int64_t S, int K, const PlanOptions& opt,
                HostPlan* out);

}  // namespace gst
