// Device-side records of the batched engine, shared by its per-step kernels
// (lbm_batch.hip) and its persistent kernel (lbm_persistent.hip).  Internal.
#pragma once

#include "lbm_tile.h"
#include "lbm_tile2.h"

namespace lbm {

// One domain: its geometry, its constants in working precision, its two
// distribution buffers and the number of tiles it has in the tile list that
// the launch uses (the persistent kernel's step barrier counts to it).
template <typename T>
struct BatchDomain {
  Geometry g;
  DevC<T> c;
  T* f[2];
  unsigned ntiles;
};

// One tile: its domain, the first stored column and row, and the direction
// the tile marches in (neighbouring row blocks alternate).
struct BatchTile {
  int domain, x0, y0, down;
};

}  // namespace lbm
