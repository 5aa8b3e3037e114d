// Host construction of the work tables of the grouped matrix-core launches:
// the order in which a launch's waves take their items.  The order decides
// which items share the assignment tiles and the state rows they read while
// those are still in an XCD's L2, so the measured HBM traffic of the kernels
// depends on it as much as on their code.
#include <vector>

#include "dode_internal.h"

// Items (cluster, a, b) with the cluster outermost and a cluster's groups
// consecutive in the group list.  Without `tile_major` a is the row u and b
// runs over (group, tile k) with k fastest: all day groups of a cluster that
// need the tiles of row u run back to back.  With `tile_major` a is the tile
// and b runs over (group, row).  `group_fastest` swaps the two parts of b so
// the day groups run fastest: neighbouring waves then read the same tiles
// (and the same rows of the tiles) for different days.  fwd: rows are
// minibatch slots, tiles link tiles (kFwdTileGroup per wave, tile = the
// first); adjoint: rows are descriptor or chunk indices, tiles OD tiles.
std::vector<WaveWork> work_table(const dode_dar* dar, const std::vector<int32_t>& gc,
                                 const std::vector<int32_t>& gf, const std::vector<int32_t>& gn,
                                 bool fwd, int32_t rows, bool tile_major, bool group_fastest) {
  const int32_t nLT = dar->tiles.nLT, nPT = dar->tiles.nPT;
  const std::vector<int32_t>& m = dar->h_tile_meta;
  const int32_t* ks = fwd ? m.data() + nLT : m.data() + 3 * nLT + nPT;
  const int32_t* lo = fwd ? m.data() : m.data() + 3 * nLT;
  const int32_t* ko = fwd ? m.data() + 2 * nLT : m.data() + 3 * nLT + 2 * nPT;
  const int32_t step = fwd ? kFwdTileGroup : 1;
  const int32_t n_tiles = fwd ? (nLT + step - 1) / step : nPT;
  const int32_t per = tile_major ? n_tiles : rows, inner = tile_major ? rows : n_tiles;
  std::vector<WaveWork> out;
  out.reserve((size_t)gc.size() * rows * n_tiles);
  auto push = [&](int32_t a, int32_t b, size_t g, size_t g0) {
    const int32_t row = tile_major ? b : a, tile = (tile_major ? a : b) * step;
    out.push_back(WaveWork{gc[g0], gf[g], gn[g], row, tile, ks[tile], lo[tile], ko[tile]});
  };
  for (size_t g0 = 0; g0 < gc.size();) {
    size_t g1 = g0 + 1;
    while (g1 < gc.size() && gc[g1] == gc[g0]) ++g1;
    for (int32_t a = 0; a < per; ++a)
      if (group_fastest) {
        for (int32_t b = 0; b < inner; ++b)
          for (size_t g = g0; g < g1; ++g) push(a, b, g, g0);
      } else {
        for (size_t g = g0; g < g1; ++g)
          for (int32_t b = 0; b < inner; ++b) push(a, b, g, g0);
      }
    g0 = g1;
  }
  return out;
}
