// Test helper: exposes the host sharing plan (paper_2008_13490_amd/csrc/gst_plan.*)
// to Python through a C function, so the plan can be checked on the CPU.
#include <cstring>

#include "gst_plan.h"

namespace {
gst::HostPlan g_plan;
int g_jump = gst::PlanOptions().jump;
int g_jump_min_save = gst::PlanOptions().jump_min_save;
int g_rep_anchor_min = gst::PlanOptions().rep_anchor_min;
int g_anchor_min_share = gst::PlanOptions().anchor_min_share;
int g_anchor_max_back = gst::PlanOptions().anchor_max_back;
int g_jump_span = gst::PlanOptions().jump_span;
}

// Longest span (steps) of a germ-power jump in the following plan_build calls.
extern "C" void plan_set_span(int span) { g_jump_span = span; }

// Start-state options of the following plan_build calls (items inside long
// periodic runs start at repetition boundaries that enough items share).
extern "C" void plan_set_anchor(int rep_min, int min_share, int max_back) {
  g_rep_anchor_min = rep_min;
  g_anchor_min_share = min_share;
  g_anchor_max_back = max_back;
}

// Germ-power jump options of the following plan_build calls.
extern "C" void plan_set_jump(int jump, int min_save) {
  g_jump = jump;
  g_jump_min_save = min_save;
}

extern "C" int plan_build(const int64_t* off, const uint8_t* gates, int64_t S, int K, int min_trunk,
                          int reanchor_depth, double ratio, int64_t* sizes) {
  gst::PlanOptions opt;
  opt.min_trunk = min_trunk;
  opt.reanchor_depth = reanchor_depth;
  opt.max_share_ratio = ratio;
  opt.jump = g_jump;
  opt.jump_min_save = g_jump_min_save;
  opt.rep_anchor_min = g_rep_anchor_min;
  opt.anchor_min_share = g_anchor_min_share;
  opt.anchor_max_back = g_anchor_max_back;
  opt.jump_span = g_jump_span;
  const bool used = gst::build_plan(off, gates, S, K, opt, &g_plan);
  const gst::HostPlan& P = g_plan;
  sizes[0] = used;
  sizes[1] = P.n_items();
  sizes[2] = P.n_trunks();
  sizes[3] = P.trunk_steps();
  sizes[4] = (int64_t)P.inj_loc.size();
  sizes[5] = (int64_t)P.inj_src.size();
  sizes[6] = P.n_levels;
  sizes[7] = P.n_nodes;
  sizes[8] = P.sum_len;
  sizes[9] = (int64_t)P.rec_b.size();
  sizes[10] = P.root_slot;
  sizes[11] = P.item_steps();
  sizes[12] = (int64_t)P.seg_start.size();
  return 0;
}

extern "C" void plan_copy(int64_t* items, int64_t* trunk_ptr, int64_t* trunk_anchor, uint8_t* trunk_gates,
                          int32_t* trunk_inj, int64_t* inj_loc, int64_t* inj_ptr, int64_t* inj_src,
                          int64_t* level_ptr) {
  const gst::HostPlan& P = g_plan;
  std::memcpy(items, P.items.data(), P.items.size() * 8);
  std::memcpy(trunk_ptr, P.trunk_ptr.data(), P.trunk_ptr.size() * 8);
  std::memcpy(trunk_anchor, P.trunk_anchor.data(), P.trunk_anchor.size() * 8);
  std::memcpy(trunk_gates, P.trunk_gates.data(), P.trunk_gates.size());
  std::memcpy(trunk_inj, P.trunk_inj.data(), P.trunk_inj.size() * 4);
  std::memcpy(inj_loc, P.inj_loc.data(), P.inj_loc.size() * 8);
  std::memcpy(inj_ptr, P.inj_ptr.data(), P.inj_ptr.size() * 8);
  std::memcpy(inj_src, P.inj_src.data(), P.inj_src.size() * 8);
  std::memcpy(level_ptr, P.trunk_level_ptr.data(), P.trunk_level_ptr.size() * 8);
}

extern "C" void plan_copy_records(int64_t* item_step_ptr, int64_t* rec_b, int64_t* rec_f, int64_t* rec_gate_ptr) {
  const gst::HostPlan& P = g_plan;
  std::memcpy(item_step_ptr, P.item_step_ptr.data(), P.item_step_ptr.size() * 8);
  std::memcpy(rec_b, P.rec_b.data(), P.rec_b.size() * 8);
  std::memcpy(rec_f, P.rec_f.data(), P.rec_f.size() * 8);
  std::memcpy(rec_gate_ptr, P.rec_gate_ptr.data(), P.rec_gate_ptr.size() * 8);
}

extern "C" void plan_copy_segments(int64_t* seg_ptr, int32_t* start, int32_t* count, uint32_t* pattern, uint8_t* g3) {
  const gst::HostPlan& P = g_plan;
  std::memcpy(seg_ptr, P.seg_ptr.data(), P.seg_ptr.size() * 8);
  std::memcpy(start, P.seg_start.data(), P.seg_start.size() * 4);
  std::memcpy(count, P.seg_count.data(), P.seg_count.size() * 4);
  std::memcpy(pattern, P.seg_pattern.data(), P.seg_pattern.size() * 4);
  std::memcpy(g3, P.seg_gate3.data(), P.seg_gate3.size());
}

extern "C" void plan_jump_sizes(int64_t* sizes) {
  const gst::HostPlan& P = g_plan;
  sizes[0] = P.jump_levels;
  sizes[1] = P.n_jump_trunks();
  sizes[2] = P.n_fill();
}

// pattern, g3: per trunk (pattern 0 = no jumps)
extern "C" void plan_copy_jumps(uint32_t* pattern, uint8_t* g3, int64_t* first, int64_t* in, int32_t* n,
                                uint32_t* fpat, uint8_t* fg3) {
  const gst::HostPlan& P = g_plan;
  std::memcpy(pattern, P.trunk_jump_pattern.data(), P.trunk_jump_pattern.size() * 4);
  std::memcpy(g3, P.trunk_jump_gate3.data(), P.trunk_jump_gate3.size());
  std::memcpy(first, P.fill_first.data(), P.fill_first.size() * 8);
  std::memcpy(in, P.fill_in.data(), P.fill_in.size() * 8);
  std::memcpy(n, P.fill_n.data(), P.fill_n.size() * 4);
  std::memcpy(fpat, P.fill_pattern.data(), P.fill_pattern.size() * 4);
  std::memcpy(fg3, P.fill_gate3.data(), P.fill_gate3.size());
}

extern "C" int64_t plan_n_ops() { return (int64_t)g_plan.op_desc.size(); }

extern "C" void plan_copy_ops(int64_t* op_ptr, uint32_t* desc, int32_t* slot) {
  const gst::HostPlan& P = g_plan;
  std::memcpy(op_ptr, P.op_ptr.data(), P.op_ptr.size() * 8);
  std::memcpy(desc, P.op_desc.data(), P.op_desc.size() * 4);
  std::memcpy(slot, P.op_slot.data(), P.op_slot.size() * 4);
}

extern "C" void plan_copy_sources(int32_t* item_src, int32_t* trunk_src) {
  const gst::HostPlan& P = g_plan;
  std::memcpy(item_src, P.item_src.data(), P.item_src.size() * 4);
  std::memcpy(trunk_src, P.trunk_src.data(), P.trunk_src.size() * 4);
}
