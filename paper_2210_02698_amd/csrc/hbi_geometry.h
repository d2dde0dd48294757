// Host geometry of the HODBF representation (Sec. 4.2): K-D cluster tree of
// the cell centres, node ranges and bounding boxes, boundary bands, and the
// proxy-row rule of eq. proxyv2v.
#pragma once
#include <stdint.h>

#include <functional>
#include <vector>

namespace hbi {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn);

struct Geometry {
  int dim = 2;
  int32_t nc[3] = {1, 1, 1};
  int64_t Nv = 0;
  int Lv = 0;
  std::vector<int32_t> perm;   // tree position -> natural index
  std::vector<int32_t> ipos;   // natural index -> tree position
  std::vector<int32_t> nstart, nend;   // node (l, i) at index (1<<l)-1+i
  std::vector<int32_t> bblo, bbhi;     // node bounding boxes in grid units [node*3+ax]
  std::vector<int64_t> band_off;       // boundary band CSR per node
  std::vector<int32_t> band;

  static int64_t node(int l, int64_t i) { return ((int64_t)1 << l) - 1 + i; }
  void grid_coords(int64_t nat, int32_t g[3]) const {
    g[0] = (int32_t)(nat % nc[0]);
    g[1] = (int32_t)((nat / nc[0]) % nc[1]);
    g[2] = (int32_t)(nat / ((int64_t)nc[0] * nc[1]));
  }
  // Complete binary tree: a node is split at the median of its cells along
  // its longest extent (ties: lowest axis; stable order within equal
  // coordinates), the lower half first, until leaves hold <= leaf cells.
  void build(int dim, const int32_t ncell[3], int leaf);
  // Cells of each non-leaf node within `width` cells (Chebyshev distance)
  // of a cell outside the node or outside the grid.
  void build_bands(int width);
};

struct ProxyParams {
  double chi = 20.0;
  double radius = 10.0;   // neighbour radius in cells
  bool band = true;       // half of the uniform rows over the boundary band
};

// Proxy rows of eq. proxyv2v for row node `nd` and candidate columns `cand`
// (tree positions; for segment columns, the cells that hold them): the
// cells of the node within `radius` cells of a candidate, plus
// ceil(chi*|cand|) cells spread uniformly, half over the node's boundary
// band and half over the whole node (all over the whole node without
// `band`, the rule for the cells x segments butterfly, Sec. 4.2).  Falls
// back to all cells of the node when that is not smaller.  Output
// ascending.  `stamp` is per-thread scratch of size Nv with values < `tag`.
void proxy_rows(const Geometry &G, int64_t nd, const int32_t *cand, int ncand,
                const ProxyParams &pp, std::vector<int32_t> &out,
                std::vector<int32_t> &stamp, int32_t tag);

}  // namespace hbi
