// Prefix-sharing plan (see gst_plan.h).
#include "gst_plan.h"

#include <algorithm>
#include <cstring>
#include <numeric>

namespace gst {

int64_t HostPlan::plan_steps() const {
  int64_t s = trunk_steps();
  for (int64_t q = 0; q < n_items(); ++q) s += items[4 * q + 2] - items[4 * q + 1];
  return s;
}

bool build_plan(const int64_t* off, const uint8_t* gates, int64_t S, int K, const PlanOptions& opt,
                HostPlan* out) {
  HostPlan& P = *out;
  P = HostPlan();
  P.K = K;
  P.S = S;
  P.sum_len = S > 0 ? off[S] - off[0] : 0;
  for (int64_t s = 0; s < S; ++s) P.max_len = std::max(P.max_len, off[s + 1] - off[s]);
  if (S == 0 || P.sum_len == 0) return false;

  // ---- 0. early rejection: distinct prefixes depth by depth ----
  // Once every word still running at depth t has its own prefix, no two words
  // share a node deeper than t, and the node count of the whole trie follows
  // from the length histogram.  Random words reach that point within a few
  // levels; structured lists (shared germ powers) do not and skip the test.
  {
    std::vector<int64_t> n_ge((size_t)P.max_len + 2, 0);  // words with length >= t
    for (int64_t s = 0; s < S; ++s) n_ge[off[s + 1] - off[s]] += 1;
    for (int64_t t = P.max_len - 1; t >= 0; --t) n_ge[t] += n_ge[t + 1];
    std::vector<int32_t> cur((size_t)S, 0);
    std::vector<int32_t> kid((size_t)K, -1);
    int64_t nodes = 1;
    const int64_t t_max = std::min<int64_t>(P.max_len, 64);
    for (int64_t t = 1; t <= t_max; ++t) {
      int64_t created = 0;
      for (int64_t s = 0; s < S; ++s) {
        if (off[s + 1] - off[s] < t) continue;
        const size_t at = (size_t)cur[s] * K + gates[off[s] + t - 1];
        if (kid[at] < 0) {
          kid[at] = (int32_t)nodes++;
          kid.resize((size_t)nodes * K, -1);
          ++created;
        }
        cur[s] = kid[at];
      }
      if (nodes >= opt.max_nodes) return false;
      if (created == n_ge[t]) {
        int64_t total = nodes;
        for (int64_t u = t + 1; u <= P.max_len; ++u) total += n_ge[u];
        if ((double)(total - 1) > opt.max_share_ratio * (double)P.sum_len) return false;
        break;
      }
    }
  }

  // ---- 1. trie over the words in time order ----
  std::vector<int32_t> parent{-1};
  std::vector<uint8_t> gate{0};
  std::vector<int32_t> depth{0};
  std::vector<int32_t> child((size_t)K, -1);
  std::vector<int32_t> term((size_t)S);
  for (int64_t s = 0; s < S; ++s) {
    int32_t n = 0;
    for (int64_t t = off[s]; t < off[s + 1]; ++t) {
      const int g = gates[t];
      int32_t c = child[(size_t)n * K + g];
      if (c < 0) {
        if ((int64_t)parent.size() >= opt.max_nodes) return false;
        c = (int32_t)parent.size();
        parent.push_back(n);
        gate.push_back((uint8_t)g);
        depth.push_back(depth[n] + 1);
        child.resize(child.size() + K, -1);
        child[(size_t)n * K + g] = c;
      }
      n = c;
    }
    term[s] = n;
  }
  const int64_t N = (int64_t)parent.size();
  P.n_nodes = N;
  // quick rejection: the trie alone bounds the saving
  if ((double)(N - 1) > opt.max_share_ratio * (double)P.sum_len) return false;

  // ---- 2. heights and heavy children (children have larger ids than parents) ----
  std::vector<int32_t> height((size_t)N, 0);
  for (int64_t n = N - 1; n >= 1; --n) height[parent[n]] = std::max(height[parent[n]], height[n] + 1);
  std::vector<int32_t> heavy((size_t)N, -1);
  for (int64_t n = 1; n < N; ++n) {
    const int32_t p = parent[n];
    if (heavy[p] < 0 || height[n] > height[heavy[p]]) heavy[p] = (int32_t)n;
  }

  // ---- 3. chains of the heavy-path decomposition; long ones become trunks ----
  // chain heads: heavy child of the root and every node that is not the heavy
  // child of its parent.
  std::vector<int32_t> heads;
  for (int64_t n = 1; n < N; ++n)
    if (heavy[parent[n]] != n || parent[n] == 0) heads.push_back((int32_t)n);
  // owner trunk and position of stored nodes
  std::vector<int32_t> owner((size_t)N, -1);
  std::vector<int32_t> chain_pos((size_t)N, -1);
  struct Trunk {
    int32_t head;
    int32_t anchor_node;  // 0 = root (recompute from rho)
    int32_t len_chain;
    int32_t len_prefix;   // unstored steps recomputed before the head
    int level;
  };
  std::vector<Trunk> trunks;
  for (int32_t h : heads) {
    if (height[h] + 1 < opt.min_trunk) continue;
    const int32_t t = (int32_t)trunks.size();
    int32_t len = 0;
    for (int32_t n = h; n >= 0; n = heavy[n]) {
      owner[n] = t;
      chain_pos[n] = len++;
    }
    trunks.push_back(Trunk{h, 0, len, 0, 0});
  }
  // anchors and levels; heads are in increasing node id, so a trunk's anchor
  // owner (an ancestor) has already been assigned a level when its head has a
  // smaller id -- not guaranteed in general, hence the fixed-point loop.
  for (auto& T : trunks) {
    int32_t a = parent[T.head];
    int32_t steps = 0;
    while (a != 0 && owner[a] < 0) {
      a = parent[a];
      ++steps;
    }
    if (a != 0 && depth[a] <= opt.reanchor_depth) {
      steps += depth[a];
      a = 0;
    }
    T.anchor_node = a;
    T.len_prefix = steps;
  }
  bool changed = true;
  for (int it = 0; changed && it < 64; ++it) {
    changed = false;
    for (auto& T : trunks) {
      const int lvl = T.anchor_node == 0 ? 0 : trunks[owner[T.anchor_node]].level + 1;
      if (lvl != T.level) {
        T.level = lvl;
        changed = true;
      }
    }
  }
  // order: level ascending, then total length descending, then head id
  std::vector<int32_t> order(trunks.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const Trunk &A = trunks[x], &B = trunks[y];
    if (A.level != B.level) return A.level < B.level;
    return A.len_prefix + A.len_chain > B.len_prefix + B.len_chain;
  });
  std::vector<int32_t> rank(trunks.size());
  for (size_t r = 0; r < order.size(); ++r) rank[order[r]] = (int32_t)r;
  // state locations: trunk r owns locations [trunk_ptr[r], trunk_ptr[r+1]);
  // the state after its j-th step is at trunk_ptr[r] + j.
  const int64_t nT = (int64_t)trunks.size();
  P.trunk_ptr.assign(nT + 1, 0);
  for (int64_t r = 0; r < nT; ++r) {
    const Trunk& T = trunks[order[r]];
    P.trunk_ptr[r + 1] = P.trunk_ptr[r] + T.len_prefix + T.len_chain;
  }
  auto loc_of = [&](int32_t n) -> int64_t {  // canonical location of a stored node
    const int32_t t = owner[n];
    return P.trunk_ptr[rank[t]] + trunks[t].len_prefix + chain_pos[n];
  };
  P.trunk_gates.resize(P.trunk_ptr[nT]);
  P.trunk_inj.assign(P.trunk_ptr[nT], -1);
  P.trunk_anchor.resize(nT);
  int max_level = 0;
  for (int64_t r = 0; r < nT; ++r) {
    const Trunk& T = trunks[order[r]];
    max_level = std::max(max_level, T.level);
    P.trunk_anchor[r] = T.anchor_node == 0 ? -1 : loc_of(T.anchor_node);
    // gates: walk up from the chain end to the anchor, then reverse
    int64_t w = P.trunk_ptr[r + 1] - 1;
    int32_t end = T.head;
    while (heavy[end] >= 0) end = heavy[end];
    for (int32_t n = end; n != T.anchor_node; n = parent[n]) P.trunk_gates[w--] = gate[n];
    P.trunk_max_len = std::max<int64_t>(P.trunk_max_len, T.len_prefix + T.len_chain);
  }
  P.n_levels = nT ? max_level + 1 : 0;
  P.trunk_level_ptr.assign(P.n_levels + 1, 0);
  for (int64_t r = 0; r < nT; ++r) P.trunk_level_ptr[trunks[order[r]].level + 1] = r + 1;
  for (int l = 1; l <= P.n_levels; ++l) P.trunk_level_ptr[l] = std::max(P.trunk_level_ptr[l], P.trunk_level_ptr[l - 1]);

  // ---- 3b. long periodic runs of the trunks' words ----
  // A germ power g^l is a run of repetitions of g's gates.  A state that an
  // item starts from ends the trunk's segment there (its adjoint is
  // injected), so a start inside a repetition, or at a boundary few items
  // share, breaks the run's germ-power jumps into short ones and single gate
  // steps on the chain.  Such items start earlier instead, at a repetition
  // boundary that others share, and take the steps in between themselves:
  // the items run in parallel, the chain does not.  Runs are found greedily
  // from the trunk's start, as the segments below find them; at each state
  // of a run of at least rep_anchor_min repetitions, run_per is the period
  // (0 elsewhere), run_ref the state before the run's first gate (boundaries
  // are run_ref + k run_per; base - 1 for a run from the trunk's start) and
  // run_lo the earliest state of the trunk an item may move back to.
  std::vector<int32_t> run_per((size_t)P.trunk_ptr[nT], 0);
  std::vector<int64_t> run_ref((size_t)P.trunk_ptr[nT], 0), run_lo((size_t)P.trunk_ptr[nT], 0);
  if (opt.rep_anchor_min > 0) {
    for (int64_t r = 0; r < nT; ++r) {
      const int64_t base = P.trunk_ptr[r], L = P.trunk_ptr[r + 1] - base;
      const uint8_t* w = P.trunk_gates.data() + base;
      for (int64_t j = 0; j < L;) {
        int bp = 1;
        int64_t bc = 1;
        for (int p = 1; p <= 4 && p <= L - j; ++p) {
          int64_t c = 1;
          while ((c + 1) * p <= L - j && std::memcmp(w + j, w + j + c * p, p) == 0) ++c;
          if (c * p > bc * bp) {
            bp = p;
            bc = c;
          }
        }
        if (bc >= opt.rep_anchor_min)
          for (int64_t x = std::max<int64_t>(j - 1, 0); x < j + bp * bc; ++x) {
            run_per[base + x] = bp;
            run_ref[base + x] = base + j - 1;
            run_lo[base + x] = base + std::max<int64_t>(j - 1, 0);
          }
        j += bp * bc;
      }
    }
  }
  // ---- 4. items: each sequence from its deepest stored prefix ----
  std::vector<int64_t> it((size_t)S * 4);
  for (int64_t s = 0; s < S; ++s) {
    int32_t n = term[s];
    while (n != 0 && owner[n] < 0) n = parent[n];
    int64_t loc = n == 0 ? -1 : loc_of(n), beg = off[s] + depth[n];
    if (loc >= 0 && run_per[loc] > 1) {  // back to the start of the repetition (within the trunk)
      const int64_t back = (loc - run_ref[loc]) % run_per[loc];
      if (loc - back >= run_lo[loc]) {
        loc -= back;
        beg -= back;
      }
    }
    it[4 * s + 0] = s;
    it[4 * s + 1] = beg;
    it[4 * s + 2] = off[s + 1];
    it[4 * s + 3] = loc;
  }
  if (opt.rep_anchor_min > 0 && opt.anchor_min_share > 1) {
    std::vector<int32_t> share((size_t)P.trunk_ptr[nT], 0);
    for (int64_t s = 0; s < S; ++s)
      if (it[4 * s + 3] >= 0) ++share[it[4 * s + 3]];
    for (int64_t s = 0; s < S; ++s) {
      const int64_t loc = it[4 * s + 3];
      if (loc < 0 || run_per[loc] == 0 || share[loc] >= opt.anchor_min_share) continue;
      for (int64_t b = loc - run_per[loc]; b >= run_lo[loc] && loc - b <= opt.anchor_max_back; b -= run_per[loc])
        if (share[b] >= opt.anchor_min_share) {
          it[4 * s + 1] -= loc - b;
          it[4 * s + 3] = b;
          break;
        }
    }
  }
  std::vector<int64_t> iorder((size_t)S);
  std::iota(iorder.begin(), iorder.end(), 0);
  std::stable_sort(iorder.begin(), iorder.end(), [&](int64_t x, int64_t y) {
    return it[4 * x + 2] - it[4 * x + 1] > it[4 * y + 2] - it[4 * y + 1];
  });
  P.items.resize((size_t)S * 4);
  for (int64_t q = 0; q < S; ++q)
    for (int c = 0; c < 4; ++c) P.items[4 * q + c] = it[4 * iorder[q] + c];
  for (int64_t q = 0; q < S; ++q) P.item_max_len = std::max(P.item_max_len, P.items[4 * q + 2] - P.items[4 * q + 1]);
  P.item_kv.assign((size_t)S * 16, 0);
  for (int64_t q = 0; q < S; ++q)
    for (int64_t x = P.items[4 * q + 1], c = 0; x < P.items[4 * q + 2] && c < 16; ++x, ++c)
      P.item_kv[(size_t)q * 16 + c] = gates[x];

  // ---- 5. injection slots: stored locations that receive adjoints ----
  // sources: items anchored there and trunks (level >= 1) anchored there.
  std::vector<std::pair<int64_t, int64_t>> src;  // (loc, source)
  for (int64_t q = 0; q < S; ++q)
    if (P.items[4 * q + 3] >= 0) src.emplace_back(P.items[4 * q + 3], q);
  for (int64_t r = 0; r < nT; ++r)
    if (P.trunk_anchor[r] >= 0) src.emplace_back(P.trunk_anchor[r], -(r + 1));
  std::stable_sort(src.begin(), src.end(),
                   [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
                     return a.first < b.first;
                   });
  P.inj_ptr.push_back(0);
  for (size_t x = 0; x < src.size();) {
    size_t y = x;
    while (y < src.size() && src[y].first == src[x].first) ++y;
    const int32_t slot = (int32_t)P.inj_loc.size();
    P.inj_loc.push_back(src[x].first);
    for (size_t z = x; z < y; ++z) P.inj_src.push_back(src[z].second);
    P.inj_ptr.push_back((int64_t)P.inj_src.size());
    P.trunk_inj[src[x].first] = slot;
    x = y;
  }
  // ---- periodic segments of every trunk's gate word; a segment never runs
  // past a step whose resulting state receives an injection, so injections
  // happen only at segment ends ----
  P.seg_ptr.assign(nT + 1, 0);
  const int B = opt.jump;
  const bool jump_on = B >= 2 && B <= 16 && (B & (B - 1)) == 0;
  // the longest jump of a pattern of period per: B repetitions, or more (a
  // power of two) while it spans at most jump_span steps; lb_of = its log2
  auto lb_of = [&](int per) {
    int lb = 0;
    while (lb < 4 && ((1 << (lb + 1)) <= B || (opt.jump_span > 0 && (2 << lb) * per <= opt.jump_span))) ++lb;
    return lb;  // at most 4: five levels, which the reverse trunk kernel holds in registers
  };
  P.jump_levels = 0;
  P.trunk_jump_pattern.assign(nT, 0);
  P.trunk_jump_gate3.assign(nT, 0);
  P.trunk_jump_levels.assign(nT, 0);
  struct Run {
    int64_t j, count;
    int per;
    uint32_t pat;
    uint8_t g3;
  };
  // chain mat-vecs of a run applied with jumps: count / 2^lb jumps by the
  // longest power, then one jump per set bit of the remainder (a one-gate
  // pattern takes its last single repetition as an ordinary step)
  auto chain_of = [&](const Run& u) {
    const int lb = lb_of(u.per);
    int64_t c = u.count >> lb;
    for (int e = 0; e < lb; ++e) c += (u.count >> e) & 1;
    return c;
  };
  std::vector<Run> runs;
  for (int64_t r = 0; r < nT; ++r) {
    const int64_t base = P.trunk_ptr[r];
    const uint8_t* w = P.trunk_gates.data() + base;
    const int64_t L = P.trunk_ptr[r + 1] - base;
    runs.clear();
    for (int64_t j = 0; j < L;) {
      int64_t piece_end = j;  // last step of the injection-free piece starting at j
      while (piece_end < L - 1 && P.trunk_inj[base + piece_end] < 0) ++piece_end;
      const int64_t n = piece_end - j + 1;
      int bp = 1;
      int64_t bc = 1;
      for (int p = 1; p <= 4 && p <= n; ++p) {
        int64_t c = 1;
        while ((c + 1) * p <= n && std::memcmp(w + j, w + j + c * p, p) == 0) ++c;
        if (c * p > bc * bp) {
          bp = p;
          bc = c;
        }
      }
      uint32_t pat = (uint32_t)bp;
      for (int q = 0; q < bp && q < 3; ++q) pat |= (uint32_t)w[j + q] << (8 * (q + 1));
      runs.push_back(Run{j, bc, bp, pat, (uint8_t)(bp == 4 ? w[j + 3] : 0)});
      j += bp * bc;
    }
    // the trunk's jump pattern: the one whose qualifying runs save the most
    // chain steps (its germ)
    auto saves = [&](const Run& u) { return u.per * u.count - chain_of(u); };
    uint32_t jp = 0;
    uint8_t jg3 = 0;
    if (jump_on) {
      int64_t best = 0;
      for (const Run& u : runs) {
        if (saves(u) < opt.jump_min_save) continue;
        int64_t tot = 0;
        for (const Run& v : runs)
          if (v.pat == u.pat && v.g3 == u.g3 && saves(v) >= opt.jump_min_save) tot += saves(v);
        if (tot > best) {
          best = tot;
          jp = u.pat;
          jg3 = u.g3;
        }
      }
    }
    P.trunk_jump_pattern[r] = jp;
    P.trunk_jump_gate3[r] = jg3;
    const int lb = jp ? lb_of((int)(jp & 0xffu)) : 0;
    const int64_t Bt = (int64_t)1 << lb;
    if (jp) {
      P.trunk_jump_levels[r] = (uint8_t)(lb + 1);
      P.jump_levels = std::max(P.jump_levels, lb + 1);
    }
    auto emit_plain = [&](int64_t start, int64_t count, uint32_t pat, uint8_t g3, int64_t inj) {
      P.seg_start.push_back((int32_t)start);
      P.seg_count.push_back((int32_t)count);
      P.seg_pattern.push_back(pat);
      P.seg_gate3.push_back(g3);
      P.seg_inj.push_back(inj);
    };
    for (const Run& u : runs) {
      const int64_t last = u.j + (int64_t)u.per * u.count - 1;
      const int64_t inj = P.trunk_inj[base + last];
      if (jp == 0 || u.pat != jp || u.g3 != jg3 || saves(u) < opt.jump_min_save) {
        emit_plain(u.j, u.count, u.pat, u.g3, inj);
        continue;
      }
      int64_t s = u.j;
      auto emit_jump = [&](int e, int64_t count) {
        const int64_t stride = ((int64_t)1 << e) * u.per;
        P.seg_start.push_back((int32_t)s);
        P.seg_count.push_back((int32_t)count);
        P.seg_pattern.push_back((uint32_t)stride << 8 | (uint32_t)e << 16);
        P.seg_gate3.push_back(0);
        P.seg_inj.push_back(s + count * stride - 1 == last ? inj : -1);
        for (int64_t c = 0; c < count; ++c, s += stride) {
          if (stride < 2) continue;
          P.fill_first.push_back(base + s);
          P.fill_in.push_back(s == 0 ? (P.trunk_anchor[r] < 0 ? 0 : 1 + P.trunk_anchor[r]) : 1 + base + s - 1);
          P.fill_n.push_back((int32_t)stride);
          P.fill_pattern.push_back(u.pat);
          P.fill_gate3.push_back(u.g3);
        }
      };
      const int64_t q_full = u.count >> lb, rem = u.count & (Bt - 1);
      if (q_full > 0) emit_jump(lb, q_full);
      for (int e = lb - 1; e >= 0; --e) {
        if (!((rem >> e) & 1)) continue;
        if (e == 0 && u.per == 1) {  // one gate: an ordinary step
          emit_plain(s, 1, u.pat, u.g3, s == last ? inj : -1);
          s += 1;
        } else {
          emit_jump(e, 1);
        }
      }
    }
    P.seg_ptr[r + 1] = (int64_t)P.seg_start.size();
  }
  // ops of each trunk's chain, from its segments
  P.op_ptr.assign(nT + 1, 0);
  for (int64_t r = 0; r < nT; ++r) {
    for (int64_t sg = P.seg_ptr[r]; sg < P.seg_ptr[r + 1]; ++sg) {
      const uint32_t pat = P.seg_pattern[sg];
      const int per = (int)(pat & 0xffu);
      const int64_t count = P.seg_count[sg];
      if (per == 0) {  // jumps
        const uint32_t span = (pat >> 8) & 0xffu, e = (pat >> 16) & 0x7fu;
        for (int64_t c = 0; c < count; ++c) {
          P.op_desc.push_back(0x80u | e | span << 8);
          P.op_slot.push_back(c == count - 1 ? (int32_t)P.seg_inj[sg] : -1);
        }
      } else {
        const uint32_t g[4] = {(pat >> 8) & 0xffu, (pat >> 16) & 0xffu, (pat >> 24) & 0xffu, P.seg_gate3[sg]};
        for (int64_t c = 0; c < count; ++c)
          for (int q = 0; q < per; ++q) {
            P.op_desc.push_back(g[q] | 1u << 8);
            P.op_slot.push_back(c == count - 1 && q == per - 1 ? (int32_t)P.seg_inj[sg] : -1);
          }
      }
    }
    P.op_ptr[r + 1] = (int64_t)P.op_desc.size();
  }
  // fill tasks grouped by pattern period, longest first within a period, and
  // each period's group padded to a multiple of four with empty tasks (one
  // step, nothing to fill): the four tasks of a wave share their period, so
  // the kernel keeps their pattern rows in registers and steps through the
  // phases in lockstep
  if (!P.fill_first.empty()) {
    std::vector<int64_t> ord(P.fill_first.size());
    for (size_t x = 0; x < ord.size(); ++x) ord[x] = (int64_t)x;
    auto per_of = [&](int64_t x) { return (int)(P.fill_pattern[x] & 0xffu); };
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
      return per_of(x) != per_of(y) ? per_of(x) < per_of(y) : P.fill_n[x] > P.fill_n[y];
    });
    std::vector<int64_t> first, in;
    std::vector<int32_t> nn;
    std::vector<uint32_t> pat;
    std::vector<uint8_t> g3;
    for (size_t x = 0; x < ord.size(); ++x) {
      const int64_t o = ord[x];
      first.push_back(P.fill_first[o]);
      in.push_back(P.fill_in[o]);
      nn.push_back(P.fill_n[o]);
      pat.push_back(P.fill_pattern[o]);
      g3.push_back(P.fill_gate3[o]);
      const bool group_end = x + 1 == ord.size() || per_of(ord[x + 1]) != per_of(o);
      while (group_end && first.size() % 4 != 0) {
        first.push_back(0);
        in.push_back(0);
        nn.push_back(1);
        pat.push_back((uint32_t)per_of(o));
        g3.push_back(0);
      }
    }
    P.fill_first.swap(first);
    P.fill_in.swap(in);
    P.fill_n.swap(nn);
    P.fill_pattern.swap(pat);
    P.fill_gate3.swap(g3);
  }

  P.trunk_anchor_inj.assign(nT, -1);
  for (int64_t r = 0; r < nT; ++r)
    if (P.trunk_anchor[r] >= 0) P.trunk_anchor_inj[r] = P.trunk_inj[P.trunk_anchor[r]];
  // root slot: trunks anchored at rho (items anchored at rho add their
  // adjoints to the per-workgroup partial sums of the item kernel)
  P.root_slot = (int64_t)P.inj_loc.size();
  P.inj_loc.push_back(-1);
  for (int64_t r = 0; r < nT; ++r)
    if (P.trunk_anchor[r] < 0) P.inj_src.push_back(-(r + 1));
  P.inj_ptr.push_back((int64_t)P.inj_src.size());
  // rows of the source arena (the root slot's sources have none)
  if (P.inj_src.size() >= (size_t)INT32_MAX) return false;
  P.item_src.assign(S, -1);
  P.trunk_src.assign(nT, -1);
  for (int64_t z = 0; z < P.inj_ptr[P.root_slot]; ++z) {
    const int64_t src = P.inj_src[z];
    if (src >= 0)
      P.item_src[src] = (int32_t)z;
    else
      P.trunk_src[-src - 1] = (int32_t)z;
  }

  if ((double)P.plan_steps() > opt.max_share_ratio * (double)P.sum_len) return false;

  // ---- 6. reverse-sweep records, grouped by gate ----
  P.item_step_ptr.assign(S + 1, 0);
  for (int64_t q = 0; q < S; ++q) P.item_step_ptr[q + 1] = P.item_step_ptr[q] + (P.items[4 * q + 2] - P.items[4 * q + 1]);
  if (P.item_steps() > opt.max_item_steps) return false;
  const int64_t nTS = P.trunk_steps();
  std::vector<std::vector<std::pair<int64_t, int64_t>>> by_gate(K);
  for (int64_t r = 0; r < nT; ++r) {
    const int64_t anchor_row = P.trunk_anchor[r] < 0 ? 0 : 1 + P.trunk_anchor[r];
    for (int64_t j = P.trunk_ptr[r]; j < P.trunk_ptr[r + 1]; ++j)
      by_gate[P.trunk_gates[j]].emplace_back(j, j == P.trunk_ptr[r] ? anchor_row : 1 + (j - 1));
  }
  for (int64_t q = 0; q < S; ++q) {
    const int64_t beg = P.items[4 * q + 1], end = P.items[4 * q + 2];
    for (int64_t x = beg; x < end; ++x) {
      const int64_t row = P.item_step_ptr[q] + (x - beg);
      by_gate[gates[x]].emplace_back(nTS + row, 1 + nTS + row);
    }
  }
  P.rec_gate_ptr.assign(K + 1, 0);
  for (int k = 0; k < K; ++k) {
    for (auto& pr : by_gate[k]) {
      P.rec_b.push_back(pr.first);
      P.rec_f.push_back(pr.second);
    }
    P.rec_gate_ptr[k + 1] = (int64_t)P.rec_b.size();
    for (int64_t c = P.rec_gate_ptr[k]; c < P.rec_gate_ptr[k + 1]; c += opt.chunk) {
      P.chunk_gate.push_back(k);
      P.chunk_beg.push_back(c);
      P.chunk_end.push_back(std::min<int64_t>(c + opt.chunk, P.rec_gate_ptr[k + 1]));
    }
  }
  return true;
}

}  // namespace gst
