// Compile probe: the shape of the single-pass scan's carry tree, and that its
// state fits the scan workspace for every tile size, checked at compile time.
#include "hdc_host.hpp"
#include "hdc_scan.hpp"

using hdc::tree_levels;
using hdc::tree_nodes;

// Levels: the smallest K with 64^K >= tiles.
static_assert(tree_levels(1) == 1 && tree_levels(64) == 1);
static_assert(tree_levels(65) == 2 && tree_levels(4096) == 2);
static_assert(tree_levels(4097) == 3 && tree_levels(262144) == 3);
static_assert(tree_levels(262145) == 4);
// Nodes: level k holds ceil(tiles / 64^k) for k < K.
static_assert(tree_nodes(1) == 1 && tree_nodes(64) == 64);
static_assert(tree_nodes(65) == 65 + 2);
static_assert(tree_nodes(4097) == 4097 + 65 + 2);
static_assert(tree_nodes(262145) == 262145 + 4097 + 65 + 2);

// 256-byte header + kWords (at most 3) 8-byte words per node within the
// workspace hdc_workspace_size(HDC_OP_SCAN, ..., n) provides, for every block
// size and for n near every tile boundary up to 2^33.
consteval bool single_pass_state_fits() {
  for (int64_t block = 64; block <= 1024; block += 64) {
    const int64_t tile = block * hdc::kScanE;
    for (int64_t base = 1; base <= (int64_t(1) << 33); base = base * 3 / 2 + 1) {
      for (int64_t d = -1; d <= 1; ++d) {
        const int64_t n = (base / tile) * tile + d;
        if (n < 1) continue;
        const int64_t G = (n + tile - 1) / tile;
        if ((size_t)(256 + 8 * 3 * tree_nodes(G)) > hdc::scan_workspace_bytes(n)) return false;
      }
    }
  }
  return true;
}
static_assert(single_pass_state_fits());
