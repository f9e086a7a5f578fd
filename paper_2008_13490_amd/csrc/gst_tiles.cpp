// Tiles of the persistent batch kernels (see gst_tiles.h).
#include "gst_tiles.h"

#include <algorithm>

namespace gst {

void cut_tiles(const int64_t* off, int64_t S, int64_t tile_seqs, std::vector<int64_t>* order,
               std::vector<int64_t>* tile_q, std::vector<int64_t>* tile_cost) {
  order->resize((size_t)S);
  for (int64_t q = 0; q < S; ++q) (*order)[q] = q;
  std::stable_sort(order->begin(), order->end(),
                   [&](int64_t x, int64_t y) { return off[x + 1] - off[x] > off[y + 1] - off[y]; });
  tile_q->clear();
  tile_cost->clear();
  if (tile_seqs < 1) tile_seqs = 1;
  for (int64_t q0 = 0; q0 < S; q0 += tile_seqs) {
    tile_q->push_back(q0);
    int64_t cost = 0;
    for (int64_t q = q0; q < std::min(S, q0 + tile_seqs); ++q) cost += off[(*order)[q] + 1] - off[(*order)[q]];
    tile_cost->push_back(cost);
  }
  if (S > 0) tile_q->push_back(S);
}

std::vector<BatchTile> batch_tiles(const std::vector<const std::vector<int64_t>*>& tile_q,
                                   const std::vector<const std::vector<int64_t>*>& tile_cost,
                                   const std::vector<int>& req_index) {
  std::vector<std::pair<int64_t, BatchTile>> v;
  for (size_t x = 0; x < tile_q.size(); ++x) {
    const std::vector<int64_t>& q = *tile_q[x];
    const int64_t n = q.empty() ? 0 : (int64_t)q.size() - 1;
    for (int64_t t = 0; t < n; ++t) v.emplace_back((*tile_cost[x])[t], BatchTile{req_index[x], (int32_t)t, q[t], q[t + 1]});
  }
  std::stable_sort(v.begin(), v.end(), [](const std::pair<int64_t, BatchTile>& a, const std::pair<int64_t, BatchTile>& b) {
    return a.first > b.first;
  });
  std::vector<BatchTile> out;
  out.reserve(v.size());
  for (auto& pr : v) out.push_back(pr.second);
  return out;
}

std::string check_batch_tiles(const std::vector<BatchTile>& tiles,
                              const std::vector<const std::vector<int64_t>*>& tile_q_of_req) {
  const int64_t n_req = (int64_t)tile_q_of_req.size();
  std::vector<std::vector<int>> seen((size_t)n_req);
  for (int64_t x = 0; x < n_req; ++x) {
    const std::vector<int64_t>* q = tile_q_of_req[x];
    seen[x].assign(q && !q->empty() ? q->size() - 1 : 0, 0);
  }
  for (size_t i = 0; i < tiles.size(); ++i) {
    const BatchTile& T = tiles[i];
    const std::string at = "tile " + std::to_string(i) + ": ";
    if (T.req < 0 || T.req >= n_req || !tile_q_of_req[T.req]) return at + "request out of range";
    const std::vector<int64_t>& q = *tile_q_of_req[T.req];
    const int64_t n_tiles = (int64_t)seen[T.req].size();
    if (T.local < 0 || T.local >= n_tiles) return at + "slab row outside its request's tiles";
    if (T.q0 != q[T.local] || T.q1 != q[T.local + 1] || T.q0 >= T.q1) return at + "range differs from the cut";
    if (seen[T.req][T.local]++) return at + "slab row listed twice";
  }
  for (int64_t x = 0; x < n_req; ++x)
    for (size_t t = 0; t < seen[x].size(); ++t)
      if (!seen[x][t]) return "request " + std::to_string(x) + ": tile " + std::to_string(t) + " missing";
  return "";
}

}  // namespace gst
