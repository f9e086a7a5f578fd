// Sharing plan with grouped chains (see gst_plan64.h).
#include "gst_plan64.h"

#include <algorithm>
#include <string>
#include <unordered_map>

namespace gst {

namespace {

// Distinct prefixes of depth <= t0: if every word reaching depth t0 has its
// own prefix there, no two words share a node deeper than t0 and the trie's
// size follows from the lengths alone.  Returns that size, or -1 when words
// still share at depth t0 (the trie must then be built to know).
int64_t nodes_if_unshared_below(const int64_t* off, const uint8_t* gates, int64_t S, int K, int64_t t0) {
  std::vector<int32_t> child;
  child.assign((size_t)K, -1);
  int64_t nodes = 1, reach = 0, deeper = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t L = off[s + 1] - off[s];
    int32_t n = 0;
    const int64_t m = std::min(L, t0);
    for (int64_t t = 0; t < m; ++t) {
      const size_t at = (size_t)n * K + gates[off[s] + t];
      if (child[at] < 0) {
        child[at] = (int32_t)nodes++;
        child.resize((size_t)nodes * K, -1);
      }
      n = child[at];
    }
    if (L >= t0) {
      ++reach;
      deeper += L - t0;
    }
  }
  // nodes at depth t0 = words reaching it with distinct prefixes
  int64_t at_t0 = 0;
  {
    // count nodes of depth exactly t0 by a second walk over the prefix trie
    std::vector<int32_t> depth((size_t)nodes, 0);
    for (int64_t n = 0; n < nodes; ++n)
      for (int g = 0; g < K; ++g) {
        const int32_t c = child[(size_t)n * K + g];
        if (c >= 0) depth[c] = depth[n] + 1;
      }
    for (int64_t n = 0; n < nodes; ++n) at_t0 += depth[n] == t0;
  }
  return at_t0 == reach ? nodes + deeper : -1;
}

}  // namespace

bool build_plan64(const int64_t* off, const uint8_t* gates, int64_t S, int K, const Plan64Options& opt,
                  Plan64* out) {
  Plan64& P = *out;
  P = Plan64();
  P.K = K;
  P.S = S;
  P.sum_len = S > 0 ? off[S] - off[0] : 0;
  for (int64_t s = 0; s < S; ++s) P.max_len = std::max(P.max_len, off[s + 1] - off[s]);
  if (S == 0 || P.sum_len == 0) return false;
  const int W = opt.tile_cols;

  // ---- 0. early rejection of lists without deep sharing ----
  {
    const int64_t t0 = std::min<int64_t>(P.max_len, 24);
    const int64_t n = nodes_if_unshared_below(off, gates, S, K, t0);
    if (n >= 0 && (double)(n - 1) > opt.max_row_ratio * (double)P.sum_len) return false;
  }

  // ---- 1. trie over the words in time order ----
  std::vector<int32_t> parent{-1};
  std::vector<uint8_t> gate{0};
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
        child.resize(child.size() + K, -1);
        child[(size_t)n * K + g] = c;
      }
      n = c;
    }
    term[s] = n;
    if ((double)(parent.size() - 1) > opt.max_row_ratio * (double)P.sum_len) return false;
  }
  const int64_t N = (int64_t)parent.size();
  P.n_nodes = N;

  // ---- 2. heights and heavy children (children have larger ids) ----
  std::vector<int32_t> height((size_t)N, 0);
  for (int64_t n = N - 1; n >= 1; --n) height[parent[n]] = std::max(height[parent[n]], height[n] + 1);
  std::vector<int32_t> heavy((size_t)N, -1);
  std::vector<int32_t> long_kids((size_t)N, 0);
  for (int64_t n = 1; n < N; ++n) {
    const int32_t p = parent[n];
    if (p == 0) continue;  // the root is no chain node: every child of the root heads a chain
    if (heavy[p] < 0 || height[n] > height[heavy[p]]) heavy[p] = (int32_t)n;
    if (height[n] + 1 >= opt.split_height) long_kids[p] += 1;
  }
  // A chain ends at a node with two or more long children: the chains hanging
  // there then start together one level later, instead of the sibling chains
  // waiting for the end of a long chain that merely passes through the node
  // (the preparation fiducials of Eq. GSTFullFiducialsGerms are such nodes:
  // every germ power hangs below them).
  for (int64_t n = 1; n < N; ++n)
    if (long_kids[n] >= 2) heavy[n] = -1;

  // ---- 3. chains in increasing head id and their anchors ----
  std::vector<int32_t> chain_of((size_t)N, -1);
  std::vector<int32_t> head, anchor, clen;
  for (int64_t n = 1; n < N; ++n) {
    if (parent[n] != 0 && heavy[parent[n]] == n) continue;
    const int32_t c = (int32_t)head.size();
    int32_t len = 0;
    for (int32_t x = (int32_t)n; x >= 0; x = heavy[x]) {
      chain_of[x] = c;
      ++len;
    }
    head.push_back((int32_t)n);
    anchor.push_back(parent[n]);
    clen.push_back(len);
  }
  const int64_t C = (int64_t)head.size();
  P.n_chains = C;

  // ---- 4. groups: chains with the same word ----
  std::vector<int32_t> group_of((size_t)C);
  int32_t n_groups = 0;
  {
    std::unordered_map<std::string, int32_t> key_to_group;
    std::string key;
    for (int64_t c = 0; c < C; ++c) {
      key.clear();
      for (int32_t x = head[c]; x >= 0; x = heavy[x]) key.push_back((char)gate[x]);
      auto it = key_to_group.find(key);
      if (it == key_to_group.end()) it = key_to_group.emplace(key, n_groups++).first;
      group_of[c] = it->second;
    }
  }

  // ---- 5. levels and tiles ----
  // A chain can run once the chain holding its anchor has run at an earlier
  // level.  Level by level, the ready chains of a word run in full tiles of W;
  // a partial tile waits for more chains of its word unless all of them are
  // ready, and if no tile could run at a level, every ready chain runs (so the
  // schedule always advances).  Children become ready one level after their
  // parent, hence every anchor is computed before its chains and every chain's
  // reverse sweep ends before its anchor's chain starts its own.
  struct TileDesc {
    int32_t level, len, group;
    std::vector<int32_t> chains;
  };
  std::vector<TileDesc> tiles;
  {
    std::vector<std::vector<int32_t>> kids((size_t)C);  // chains anchored on chain c
    std::vector<int32_t> bucket0;
    for (int64_t c = 0; c < C; ++c) {
      if (anchor[c] == 0) bucket0.push_back((int32_t)c);
      else kids[chain_of[anchor[c]]].push_back((int32_t)c);
    }
    std::vector<int64_t> remaining((size_t)n_groups, 0);
    for (int64_t c = 0; c < C; ++c) remaining[group_of[c]] += 1;
    std::vector<std::vector<int32_t>> pending((size_t)n_groups);
    std::vector<int32_t> next = bucket0;
    int64_t done = 0, long_left = 0;
    for (int64_t c = 0; c < C; ++c) long_left += clen[c] >= opt.split_height;
    for (int32_t L = 0; done < C; ++L) {
      for (int32_t c : next) pending[group_of[c]].push_back(c);
      next.clear();
      std::vector<int32_t> open;  // groups with ready chains
      for (int32_t g = 0; g < n_groups; ++g)
        if (!pending[g].empty()) open.push_back(g);
      auto run = [&](int32_t g, size_t take) {
        std::vector<int32_t>& pl = pending[g];
        std::sort(pl.begin(), pl.end());
        for (size_t i = 0; i < take; i += (size_t)W) {
          TileDesc td{L, clen[pl[i]], g, {}};
          for (size_t j = i; j < std::min(take, i + (size_t)W); ++j) {
            td.chains.push_back(pl[j]);
            for (int32_t k : kids[pl[j]]) next.push_back(k);
          }
          tiles.push_back(std::move(td));
        }
        remaining[g] -= (int64_t)take;
        done += (int64_t)take;
        pl.erase(pl.begin(), pl.begin() + (std::ptrdiff_t)take);
      };
      // Short chains run as soon as their tiles fill.  Long chains wait until
      // every long chain is ready and then run together, at one level: the
      // time of a level is that of its longest tile, and a long chain has only
      // short chains anchored on it (a chain ends where two long ones part),
      // so holding the long chains back delays nothing they feed but short ones.
      bool progress = false;
      int64_t long_pending = 0;
      for (int32_t g : open) {
        const size_t n = pending[g].size();
        if (clen[pending[g][0]] >= opt.split_height) {
          long_pending += (int64_t)n;
          continue;
        }
        const size_t take = opt.short_asap || (int64_t)n == remaining[g] ? n : n / (size_t)W * (size_t)W;
        if (take) {
          run(g, take);
          progress = true;
        }
      }
      if (!progress && long_pending > 0 && long_pending == long_left) {
        for (int32_t g : open)
          if (!pending[g].empty() && clen[pending[g][0]] >= opt.split_height) {
            long_left -= (int64_t)pending[g].size();
            run(g, pending[g].size());
          }
        progress = true;
      }
      // no full tile anywhere: the waiting short chains run in partial tiles,
      // and only if there are none, the long ones
      if (!progress)
        for (int32_t g : open)
          if (!pending[g].empty() && clen[pending[g][0]] < opt.split_height) {
            run(g, pending[g].size());
            progress = true;
          }
      if (!progress)
        for (int32_t g : open)
          if (!pending[g].empty()) {
            long_left -= (int64_t)pending[g].size();
            run(g, pending[g].size());
          }
    }
  }
  std::stable_sort(tiles.begin(), tiles.end(), [&](const TileDesc& a, const TileDesc& b) {
    if (a.level != b.level) return a.level < b.level;
    if (a.len != b.len) return a.len > b.len;
    return a.chains[0] < b.chains[0];
  });
  const int64_t T = (int64_t)tiles.size();
  P.n_levels = tiles.empty() ? 0 : tiles.back().level + 1;
  P.level_tile_ptr.assign((size_t)P.n_levels + 1, 0);
  for (const auto& t : tiles) P.level_tile_ptr[t.level + 1] += 1;
  for (int l = 0; l < P.n_levels; ++l) P.level_tile_ptr[l + 1] += P.level_tile_ptr[l];

  // ---- 6. rows ----
  std::vector<int64_t> node_row((size_t)N, -1);
  node_row[0] = 0;
  P.tile_row0.resize((size_t)T);
  P.tile_len.resize((size_t)T);
  P.tile_cols.resize((size_t)T);
  P.tile_word.resize((size_t)T);
  P.col_anchor.assign((size_t)T * W, 0);
  P.col_chain.assign((size_t)T * W, -1);
  int64_t row = 1;
  for (int64_t ti = 0; ti < T; ++ti) {
    const TileDesc& td = tiles[ti];
    const int ncol = (int)td.chains.size();
    P.tile_row0[ti] = row;
    P.tile_len[ti] = td.len;
    P.tile_cols[ti] = ncol;
    P.tile_word[ti] = (int64_t)P.words.size();
    for (int32_t x = head[td.chains[0]]; x >= 0; x = heavy[x]) P.words.push_back(gate[x]);
    for (int c = 0; c < ncol; ++c) {
      const int32_t ch = td.chains[c];
      P.col_chain[ti * W + c] = ch;
      int64_t t = 0;
      for (int32_t x = head[ch]; x >= 0; x = heavy[x], ++t) node_row[x] = row + t * W + c;
    }
    row += (int64_t)td.len * W;
  }
  P.n_rows = row;
  P.live_rows = N - 1;
  // anchors after all rows are known (an anchor lies on a chain of a lower level)
  for (int64_t ti = 0; ti < T; ++ti)
    for (int c = 0; c < P.tile_cols[ti]; ++c) P.col_anchor[ti * W + c] = node_row[anchor[P.col_chain[ti * W + c]]];
  if ((double)(N - 1) < opt.min_fill * (double)(P.n_rows - 1)) return false;
  if ((double)(P.n_rows - 1) > opt.max_row_ratio * (double)P.sum_len) return false;

  // ---- 7. seed slots (terminal nodes in order of first appearance) ----
  std::vector<int64_t> slot_of_node((size_t)N, -1);
  std::vector<int64_t> slot_count;
  for (int64_t s = 0; s < S; ++s) {
    int64_t& sl = slot_of_node[term[s]];
    if (sl < 0) {
      sl = (int64_t)P.slot_row.size();
      P.slot_row.push_back(node_row[term[s]]);
      slot_count.push_back(0);
    }
    slot_count[sl] += 1;
  }
  P.n_slots = (int64_t)P.slot_row.size();
  P.slot_ptr.assign((size_t)P.n_slots + 1, 0);
  for (int64_t x = 0; x < P.n_slots; ++x) P.slot_ptr[x + 1] = P.slot_ptr[x] + slot_count[x];
  P.slot_seq.resize((size_t)S);
  {
    std::vector<int64_t> fill(P.slot_ptr.begin(), P.slot_ptr.end() - 1);
    for (int64_t s = 0; s < S; ++s) P.slot_seq[fill[slot_of_node[term[s]]]++] = s;
  }
  P.root_slot = slot_of_node[0];

  // ---- 8. events: seeds and the chains anchored at each node ----
  std::vector<int64_t> anch_ptr((size_t)N + 1, 0), anch_list((size_t)C);
  for (int64_t c = 0; c < C; ++c) anch_ptr[anchor[c] + 1] += 1;
  for (int64_t n = 0; n < N; ++n) anch_ptr[n + 1] += anch_ptr[n];
  {
    std::vector<int64_t> fill(anch_ptr.begin(), anch_ptr.end() - 1);
    for (int64_t c = 0; c < C; ++c) anch_list[fill[anchor[c]]++] = c;  // ascending chain id per node
  }
  for (int64_t k = anch_ptr[0]; k < anch_ptr[1]; ++k) P.root_chains.push_back(anch_list[k]);
  P.tile_ev.resize((size_t)T);
  P.ev_ptr.push_back(0);
  std::vector<int32_t> cur((size_t)W);
  const bool cend = opt.max_node_events <= 15 && W == 16;
  for (int64_t ti = 0; ti < T; ++ti) {
    P.tile_ev[ti] = (int64_t)P.ev_ptr.size() - 1;
    for (int c = 0; c < P.tile_cols[ti]; ++c) cur[c] = head[P.col_chain[ti * W + c]];
    for (int64_t t = 0; t < P.tile_len[ti]; ++t) {
      const size_t e_step = P.ev_col.size();
      uint8_t row[16] = {};
      int most = 0;
      for (int c = 0; c < P.tile_cols[ti]; ++c) {
        const size_t e_col = P.ev_col.size();
        const int32_t x = cur[c];  // the node of column c at step t
        cur[c] = heavy[x];
        if (slot_of_node[x] >= 0) {
          P.ev_col.push_back(c);
          P.ev_src.push_back(slot_of_node[x]);
        }
        // a node's events (its seed, the chains anchored there): the kernels
        // hold at most max_node_events of them in registers
        if ((slot_of_node[x] >= 0) + (anch_ptr[x + 1] - anch_ptr[x]) > opt.max_node_events) return false;
        for (int64_t k = anch_ptr[x]; k < anch_ptr[x + 1]; ++k) {
          P.ev_col.push_back(c);
          P.ev_src.push_back(P.n_slots + anch_list[k]);
        }
        most = std::max(most, (int)(P.ev_col.size() - e_col));
        if (c < 15) row[c] = (uint8_t)(P.ev_col.size() - e_step);
      }
      for (int c = P.tile_cols[ti]; c < 15; ++c) row[c] = (uint8_t)(P.ev_col.size() - e_step);
      row[15] = (uint8_t)most;
      if (cend) P.ev_cend.insert(P.ev_cend.end(), row, row + 16);
      P.ev_ptr.push_back((int64_t)P.ev_col.size());
    }
  }

  // ---- 9. gradient records grouped by gate ----
  P.rec_gate_ptr.assign((size_t)K + 1, 0);
  for (int64_t ti = 0; ti < T; ++ti)
    for (int64_t t = 0; t < P.tile_len[ti]; ++t)
      P.rec_gate_ptr[P.words[P.tile_word[ti] + t] + 1] += P.tile_cols[ti];
  for (int k = 0; k < K; ++k) P.rec_gate_ptr[k + 1] += P.rec_gate_ptr[k];
  P.rec_b.resize((size_t)P.rec_gate_ptr[K]);
  P.rec_f.resize((size_t)P.rec_gate_ptr[K]);
  {
    std::vector<int64_t> fill(P.rec_gate_ptr.begin(), P.rec_gate_ptr.end() - 1);
    for (int64_t ti = 0; ti < T; ++ti)
      for (int64_t t = 0; t < P.tile_len[ti]; ++t) {
        const int k = P.words[P.tile_word[ti] + t];
        for (int c = 0; c < P.tile_cols[ti]; ++c) {
          const int64_t r = fill[k]++;
          P.rec_b[r] = P.tile_row0[ti] + t * W + c;
          P.rec_f[r] = t ? P.tile_row0[ti] + (t - 1) * W + c : P.col_anchor[ti * W + c];
        }
      }
  }
  // tile-steps grouped by gate (tile order, then step), chunked per gate
  std::vector<int64_t> ts_ptr((size_t)K + 1, 0);
  for (int64_t ti = 0; ti < T; ++ti)
    for (int64_t t = 0; t < P.tile_len[ti]; ++t) ts_ptr[P.words[P.tile_word[ti] + t] + 1] += 1;
  for (int k = 0; k < K; ++k) ts_ptr[k + 1] += ts_ptr[k];
  P.ts_tile.resize((size_t)ts_ptr[K]);
  P.ts_step.resize((size_t)ts_ptr[K]);
  {
    std::vector<int64_t> fill(ts_ptr.begin(), ts_ptr.end() - 1);
    for (int64_t ti = 0; ti < T; ++ti)
      for (int64_t t = 0; t < P.tile_len[ti]; ++t) {
        const int64_t r = fill[P.words[P.tile_word[ti] + t]]++;
        P.ts_tile[r] = ti;
        P.ts_step[r] = (int32_t)t;
      }
  }
  P.gate_chunk_ptr.assign((size_t)K + 1, 0);
  for (int k = 0; k < K; ++k) {
    P.gate_chunk_ptr[k] = (int64_t)P.chunk_beg.size();
    for (int64_t b = ts_ptr[k]; b < ts_ptr[k + 1]; b += opt.ts_chunk) {
      P.chunk_beg.push_back(b);
      P.chunk_end.push_back(std::min<int64_t>(b + opt.ts_chunk, ts_ptr[k + 1]));
    }
  }
  P.gate_chunk_ptr[K] = (int64_t)P.chunk_beg.size();
  return true;
}

}  // namespace gst
