// Host-only harness of the owner-computes tile builder (tmop_tiles.cpp) for
// the CPU tests: builds a layout and hands its arrays out by copy.
#include <cstring>

#include "tmop_internal.h"

namespace {
tmop::TileLayout g_layout;
}

extern "C" {

int tiles_build(const int32_t* en, int64_t n_elem, int npe, int64_t n_node, const int32_t* colour, int p, int Q) {
  return tmop::build_tiles(en, n_elem, npe, n_node, colour, p, Q, g_layout);
}

// which: 0 round_off, 1 slot_elem, 2 node_off, 3 node, 4 slot, 5 halo_node, 6 halo_off, 7 slot_lnode (uint16)
int64_t tiles_size(int which) {
  const tmop::TileLayout& L = g_layout;
  switch (which) {
    case 0: return (int64_t)L.round_off.size();
    case 1: return (int64_t)L.slot_elem.size();
    case 2: return (int64_t)L.node_off.size();
    case 3: return (int64_t)L.node.size();
    case 4: return (int64_t)L.slot.size();
    case 5: return (int64_t)L.halo_node.size();
    case 6: return (int64_t)L.halo_off.size();
    case 7: return (int64_t)L.slot_lnode.size();
    default: return -1;
  }
}

void tiles_copy(int which, void* dst) {
  const tmop::TileLayout& L = g_layout;
  const std::vector<int32_t>* v[7] = {&L.round_off, &L.slot_elem, &L.node_off, &L.node, &L.slot, &L.halo_node,
                                      &L.halo_off};
  if (which >= 0 && which < 7) memcpy(dst, v[which]->data(), v[which]->size() * sizeof(int32_t));
  if (which == 7) memcpy(dst, L.slot_lnode.data(), L.slot_lnode.size() * sizeof(uint16_t));
}

int64_t tiles_n_slot() { return g_layout.n_slot; }
int32_t tiles_nn_max() { return g_layout.nn_max; }
int tiles_epr(int Q) { return tmop::tile_epr(Q); }
int64_t tiles_lds_bytes(int P, int Q, int rsize, int split, int64_t nn) { return tmop::tile_lds_bytes(P, Q, rsize, split != 0, nn); }
int tiles_lds_limit() { return tmop::TILE_LDS_BYTES; }
}
