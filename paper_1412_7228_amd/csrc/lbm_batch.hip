// Batched engine: many independent periodic lattices (droplets of uneven size
// and parameters) advanced together on one GPU.
//
// Every domain is cut into tiles of tile_x columns x tile_y rows and each tile
// runs the same step_tile() / step2_tile() as the single-lattice kernel.  This
// file holds the per-step mode: one launch per step (or per two fused steps)
// over all tiles of all domains, kernel boundaries ordering the steps, chunks
// of launches captured in a HIP graph.  The persistent mode (one launch for
// many steps, per-domain barriers) is in lbm_persistent.hip.
#include <algorithm>
#include <vector>

#include "lbm_batch.h"

namespace lbm {

template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX)
    k_batch_step(const BatchDomain<T>* __restrict__ dom, const BatchTile* __restrict__ tiles,
                 int parity) {
  __shared__ typename V2<T>::t ring[4][BX + 2];
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int d = __builtin_amdgcn_readfirstlane(tiles[t].domain);
  const int x0 = __builtin_amdgcn_readfirstlane(tiles[t].x0);
  const int y0 = __builtin_amdgcn_readfirstlane(tiles[t].y0);
  const int down = __builtin_amdgcn_readfirstlane(tiles[t].down);
  const BatchDomain<T>& D = dom[d];
  step_tile<T, EOS, BX, BIG>(D.f[parity], D.f[parity ^ 1], D.g, D.c, x0, y0, down != 0, ring);
}

// Per-step mode with two fused steps per launch: the tiles are strips of
// BX - 6 stored columns (step2_tile).
template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX, sizeof(T) == 4 ? 5 : 1)
    k_batch_step2(const BatchDomain<T>* __restrict__ dom, const BatchTile* __restrict__ tiles,
                  int parity) {
  __shared__ Tile2Lds<T, BX> lds;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int d = __builtin_amdgcn_readfirstlane(tiles[t].domain);
  const int x0 = __builtin_amdgcn_readfirstlane(tiles[t].x0);
  const int y0 = __builtin_amdgcn_readfirstlane(tiles[t].y0);
  const int down = __builtin_amdgcn_readfirstlane(tiles[t].down);
  const BatchDomain<T>& D = dom[d];
  if (down)
    step2_tile<T, EOS, BX, BIG, true>(D.f[parity], D.f[parity ^ 1], D.g, D.c, x0, y0, lds);
  else
    step2_tile<T, EOS, BX, BIG, false>(D.f[parity], D.f[parity ^ 1], D.g, D.c, x0, y0, lds);
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
template <typename T, int EOS, int BX>
static hipError_t launch_b(const BatchRun& r, hipStream_t s) {
  const BatchDomain<T>* d = static_cast<const BatchDomain<T>*>(r.dom);
  const BatchTile* t = static_cast<const BatchTile*>(r.tiles);
  hipLaunchKernelGGL((k_batch_step<T, EOS, BX, false>), dim3(r.grid), dim3(BX), 0, s, d, t, r.parity);
  return hipGetLastError();
}

template <typename T, int EOS>
static hipError_t launch_e(int bx, const BatchRun& r, hipStream_t s) {
  switch (bx) {
    case 64: return launch_b<T, EOS, 64>(r, s);
    case 128: return launch_b<T, EOS, 128>(r, s);
    case 256: return launch_b<T, EOS, 256>(r, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_t(int eos, int bx, const BatchRun& r, hipStream_t s) {
  switch (eos) {
    case LBM_EOS_IDEAL: return launch_e<T, LBM_EOS_IDEAL>(bx, r, s);
    case LBM_EOS_CS: return launch_e<T, LBM_EOS_CS>(bx, r, s);
    case LBM_EOS_VDW: return launch_e<T, LBM_EOS_VDW>(bx, r, s);
    case LBM_EOS_PR: return launch_e<T, LBM_EOS_PR>(bx, r, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(lbm_precision prec, int eos, int tile_x, const BatchRun& r, hipStream_t s) {
  if (prec == LBM_FP32) return launch_t<float>(eos, tile_x, r, s);
  return launch_t<double>(eos, tile_x, r, s);
}

template <typename T, int EOS>
static hipError_t launch_step2_e(int bx, const BatchRun& r, hipStream_t s) {
  const BatchDomain<T>* d = static_cast<const BatchDomain<T>*>(r.dom);
  const BatchTile* t = static_cast<const BatchTile*>(r.tiles);
  switch (bx) {
    case 128:
      hipLaunchKernelGGL((k_batch_step2<T, EOS, 128, false>), dim3(r.grid), dim3(128), 0, s, d, t, r.parity);
      break;
    case 256:
      hipLaunchKernelGGL((k_batch_step2<T, EOS, 256, false>), dim3(r.grid), dim3(256), 0, s, d, t, r.parity);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_step2_t(int eos, int bx, const BatchRun& r, hipStream_t s) {
  switch (eos) {
    case LBM_EOS_IDEAL: return launch_step2_e<T, LBM_EOS_IDEAL>(bx, r, s);
    case LBM_EOS_CS: return launch_step2_e<T, LBM_EOS_CS>(bx, r, s);
    case LBM_EOS_VDW: return launch_step2_e<T, LBM_EOS_VDW>(bx, r, s);
    case LBM_EOS_PR: return launch_step2_e<T, LBM_EOS_PR>(bx, r, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_step2(lbm_precision prec, int eos, int tile_x, const BatchRun& r,
                              hipStream_t s) {
  if (prec == LBM_FP32) return launch_step2_t<float>(eos, tile_x, r, s);
  return launch_step2_t<double>(eos, tile_x, r, s);
}

size_t batch_domain_bytes(lbm_precision prec) {
  return prec == LBM_FP32 ? sizeof(BatchDomain<float>) : sizeof(BatchDomain<double>);
}

size_t batch_tile_bytes() { return sizeof(BatchTile); }

// Fills the device-side descriptor of one domain (host memory `out`).
void batch_fill_domain(lbm_precision prec, const Geometry& g, const ModelConsts& m, void* fa,
                       void* fb, unsigned ntiles, void* out) {
  if (prec == LBM_FP32) {
    BatchDomain<float> d{g, make_devc<float>(m), {static_cast<float*>(fa), static_cast<float*>(fb)}, ntiles};
    *static_cast<BatchDomain<float>*>(out) = d;
  } else {
    BatchDomain<double> d{g, make_devc<double>(m), {static_cast<double*>(fa), static_cast<double*>(fb)}, ntiles};
    *static_cast<BatchDomain<double>*>(out) = d;
  }
}

void batch_fill_tile(int domain, int x0, int y0, int down, void* out) {
  *static_cast<BatchTile*>(out) = BatchTile{domain, x0, y0, down};
}

}  // namespace lbm
