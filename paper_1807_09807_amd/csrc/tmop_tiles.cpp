// Host construction of the owner-computes tiles of a 2D mesh (TileParams).
//
// Tiles grow by breadth-first search over elements that share a node, from
// the lowest-numbered element not yet in a tile, one whole search level at
// a time.  On a structured quadrilateral grid numbered row by row the
// levels are square rings around a corner, so the tiles come out as s x s
// squares laid in bands; m consecutive tiles are then merged into one.  s
// and m are chosen so that a tile's elements of each colour (the 2 x 2
// colouring of such a grid) fill one round of the workgroup, within the
// LDS node budget.  Any other connectivity gets valid but less regular
// tiles.  Within a tile, the elements are packed first-fit, in colour
// order, into rounds of at most tile_epr(Q) elements that share no node.
#include <algorithm>
#include <cstring>

#include "tmop_internal.h"

namespace tmop {

namespace {

// Nodes of an s x (m s) block of order-p quadrilaterals.
int64_t block_nodes(int p, int s, int m) { return (int64_t)(p * s + 1) * (p * s * m + 1); }

// Square side (even, so that each of the four colours of a 2 x 2 colouring
// holds s^2 / 4 elements) and merge count: the largest round fill
// m s^2 / (4 epr), then the most elements per element on the tile border
// (fewer shared nodes).
void pick_shape(int p, int epr, int64_t nn_cap, int* s_out, int* m_out) {
  int best_s = 2, best_m = 1;
  double best_fill = -1.0, best_ratio = 0.0;
  for (int s = 2; s <= 64; s += 2) {
    const int per = s * s / 4;
    if (per > epr || block_nodes(p, s, 1) > nn_cap) break;
    int m = epr / per;
    while (m > 1 && block_nodes(p, s, m) > nn_cap) --m;
    const double fill = (double)(m * per) / epr;
    const double ratio = (double)(s * s * m) / (2.0 * (s + s * m));   // area / perimeter
    if (fill > best_fill + 1e-12 || (fill > best_fill - 1e-12 && ratio > best_ratio)) {
      best_fill = fill;
      best_ratio = ratio;
      best_s = s;
      best_m = m;
    }
  }
  *s_out = best_s;
  *m_out = best_m;
}

}  // namespace

int build_tiles(const int32_t* en, int64_t n_elem, int npe, int64_t n_node, const int32_t* colour, int p, int Q,
                TileLayout& out) {
  const int P = p + 1, epr = tile_epr(Q);
  // the node budget of the largest element data (FP64 or FP32, both components)
  const int64_t elem_bytes = std::max(tile_lds_bytes(P, Q, 8, false, 0), tile_lds_bytes(P, Q, 4, false, 0));
  const int64_t nn_cap = std::min<int64_t>(65535, (TILE_LDS_BYTES - elem_bytes) / TILE_NODE_BYTES);
  if (nn_cap < npe || n_elem < 1) return -1;
  int side = 2, merge = 1;
  pick_shape(p, epr, nn_cap, &side, &merge);
  const int64_t te_bfs = (int64_t)side * side;

  // node -> elements
  std::vector<int64_t> ne_off(n_node + 1, 0);
  for (int64_t k = 0; k < n_elem * npe; ++k) ++ne_off[en[k] + 1];
  for (int64_t I = 0; I < n_node; ++I) ne_off[I + 1] += ne_off[I];
  std::vector<int32_t> ne(ne_off[n_node]);
  {
    std::vector<int64_t> pos(ne_off.begin(), ne_off.end() - 1);
    for (int64_t e = 0; e < n_elem; ++e)
      for (int l = 0; l < npe; ++l) ne[pos[en[e * npe + l]]++] = (int32_t)e;
  }

  // breadth-first tiles of up to te_bfs elements and nn_cap nodes
  std::vector<int32_t> tile_of(n_elem, -1), queued(n_elem, -1), in_tile(n_node, -1), trial(n_node, -1);
  std::vector<std::vector<int32_t>> bfs_tiles;
  int64_t seed = 0;
  int trial_id = 0;
  for (int32_t t = 0;; ++t) {
    while (seed < n_elem && tile_of[seed] >= 0) ++seed;
    if (seed == n_elem) break;
    std::vector<int32_t> members, level{(int32_t)seed}, next;
    queued[seed] = t;
    int64_t nn = 0;
    auto commit = [&](int32_t e) {
      members.push_back(e);
      for (int l = 0; l < npe; ++l) {
        const int32_t I = en[(int64_t)e * npe + l];
        if (in_tile[I] != t) { in_tile[I] = t; ++nn; }
      }
    };
    while (!level.empty()) {
      int64_t add = 0;   // nodes the whole level would add
      ++trial_id;
      for (int32_t e : level)
        for (int l = 0; l < npe; ++l) {
          const int32_t I = en[(int64_t)e * npe + l];
          if (in_tile[I] != t && trial[I] != trial_id) { trial[I] = trial_id; ++add; }
        }
      if ((int64_t)(members.size() + level.size()) <= te_bfs && nn + add <= nn_cap) {
        for (int32_t e : level) commit(e);
      } else {
        // a level that does not fit: only a tile under half its size takes a part of it
        if (2 * (int64_t)members.size() < te_bfs)
          for (int32_t e : level) {
            int64_t fresh = 0;
            for (int l = 0; l < npe; ++l) fresh += in_tile[en[(int64_t)e * npe + l]] != t;
            if ((int64_t)members.size() + 1 <= te_bfs && nn + fresh <= nn_cap) commit(e);
          }
        break;
      }
      next.clear();
      for (int32_t e : level)
        for (int l = 0; l < npe; ++l) {
          const int32_t I = en[(int64_t)e * npe + l];
          for (int64_t j = ne_off[I]; j < ne_off[I + 1]; ++j) {
            const int32_t f = ne[j];
            if (tile_of[f] < 0 && queued[f] != t) { queued[f] = t; next.push_back(f); }
          }
        }
      std::sort(next.begin(), next.end());
      level.swap(next);
    }
    for (int32_t e : members) tile_of[e] = t;
    bfs_tiles.push_back(std::move(members));
  }

  // merge runs of up to `merge` consecutive tiles within the node budget
  std::vector<std::vector<int32_t>> tiles;
  std::vector<int32_t> stamp(n_node, -1);
  for (size_t i = 0; i < bfs_tiles.size();) {
    std::vector<int32_t> mem = bfs_tiles[i];
    const int32_t id = (int32_t)tiles.size();
    int64_t nn = 0;
    for (int32_t e : mem)
      for (int l = 0; l < npe; ++l) {
        const int32_t I = en[(int64_t)e * npe + l];
        if (stamp[I] != id) { stamp[I] = id; ++nn; }
      }
    size_t j = i + 1;
    for (; j < bfs_tiles.size() && j < i + (size_t)merge; ++j) {
      int64_t add = 0;
      ++trial_id;
      for (int32_t e : bfs_tiles[j])
        for (int l = 0; l < npe; ++l) {
          const int32_t I = en[(int64_t)e * npe + l];
          if (stamp[I] != id && trial[I] != trial_id) { trial[I] = trial_id; ++add; }
        }
      if (nn + add > nn_cap) break;
      for (int32_t e : bfs_tiles[j]) {
        mem.push_back(e);
        for (int l = 0; l < npe; ++l) stamp[en[(int64_t)e * npe + l]] = id;
      }
      nn += add;
    }
    tiles.push_back(std::move(mem));
    i = j;
  }

  // per tile: nodes (ascending), local connectivity, rounds
  const int64_t n_tile = (int64_t)tiles.size();
  if (n_tile > INT32_MAX) return -1;
  out = TileLayout{};
  out.node_off.assign(1, 0);
  out.round_off.assign(1, 0);
  std::vector<int32_t> local(n_node, -1), touch(n_node, 0);
  std::vector<uint64_t> used;   // per local node: bit r = used by round r
  for (int64_t t = 0; t < n_tile; ++t) {
    std::vector<int32_t>& mem = tiles[t];
    const size_t nb = out.node.size();
    for (int32_t e : mem)
      for (int l = 0; l < npe; ++l) {
        const int32_t I = en[(int64_t)e * npe + l];
        if (local[I] != -2 - (int32_t)t) { local[I] = -2 - (int32_t)t; out.node.push_back(I); }
      }
    std::sort(out.node.begin() + nb, out.node.end());
    const int64_t nn = (int64_t)(out.node.size() - nb);
    out.nn_max = std::max<int32_t>(out.nn_max, (int32_t)nn);
    for (int64_t l = 0; l < nn; ++l) {
      local[out.node[nb + l]] = (int32_t)l;
      ++touch[out.node[nb + l]];
    }
    out.node_off.push_back((int32_t)out.node.size());
    std::stable_sort(mem.begin(), mem.end(), [&](int32_t a, int32_t b) {
      return colour[a] != colour[b] ? colour[a] < colour[b] : a < b;
    });
    used.assign(nn, 0);
    std::vector<std::vector<int32_t>> rounds;
    for (int32_t e : mem) {
      uint64_t busy = 0;
      for (int l = 0; l < npe; ++l) busy |= used[local[en[(int64_t)e * npe + l]]];
      size_t r = 0;
      while (r < rounds.size() && (rounds[r].size() >= (size_t)epr || ((busy >> r) & 1u))) ++r;
      if (r >= 64) return -1;
      if (r == rounds.size()) rounds.emplace_back();
      rounds[r].push_back(e);
      for (int l = 0; l < npe; ++l) used[local[en[(int64_t)e * npe + l]]] |= uint64_t(1) << r;
    }
    for (auto& rd : rounds) {
      for (int k = 0; k < epr; ++k) {
        const int32_t e = k < (int)rd.size() ? rd[k] : -1;
        out.slot_elem.push_back(e);
        for (int l = 0; l < npe; ++l)
          out.slot_lnode.push_back(e >= 0 ? (uint16_t)local[en[(int64_t)e * npe + l]] : (uint16_t)0);
      }
    }
    out.round_off.push_back(out.round_off.back() + (int32_t)rounds.size());
    if ((int64_t)out.slot_elem.size() > INT32_MAX) return -1;
  }

  // shared nodes: one slot per touching tile, in tile order
  std::vector<int64_t> first_slot(n_node, -1);
  out.halo_off.assign(1, 0);
  for (int64_t I = 0; I < n_node; ++I)
    if (touch[I] > 1) {
      first_slot[I] = out.halo_off.back();
      out.halo_node.push_back((int32_t)I);
      out.halo_off.push_back(out.halo_off.back() + touch[I]);
    }
  out.n_slot = out.halo_off.back();
  out.slot.resize(out.node.size());
  std::vector<int32_t> taken(n_node, 0);
  for (int64_t t = 0; t < n_tile; ++t)
    for (int32_t k = out.node_off[t]; k < out.node_off[t + 1]; ++k) {
      const int32_t I = out.node[k];
      out.slot[k] = touch[I] > 1 ? (int32_t)(first_slot[I] + taken[I]++) : -1;
    }
  return 0;
}

}  // namespace tmop
