// Batched engine: many independent periodic lattices (droplets of uneven size
// and parameters) advanced together on one GPU.
//
// Every domain is cut into tiles of tile_x columns x tile_y rows and each tile
// runs the same step_tile() as the single-lattice kernel.  Two launch modes:
//
//  * persistent: one launch advances every domain by n steps.  The grid is no
//    larger than the number of workgroups the GPU holds at once, each
//    workgroup owns a fixed list of tiles (longest-processing-time
//    assignment), and a per-domain counter acts as that domain's step
//    barrier: a tile of domain d starts step s only when all of d's tiles
//    have finished step s - 1.  Waits are bounded: a wait that exceeds the
//    spin limit sets an error flag and every workgroup leaves, so the launch
//    always ends.  The counter reset and the launch are captured in a HIP graph.
//  * per-step: one launch per step over all tiles (kernel boundaries order
//    the steps); chunks of steps are captured in a HIP graph.
#include <algorithm>
#include <vector>

#include "lbm_tile.h"

namespace lbm {

template <typename T>
struct BatchDomain {
  Geometry g;
  DevC<T> c;
  T* f[2];
  unsigned ntiles;
};

struct BatchTile {
  int domain, x0, y0, down;
};

// Bounded wait of the whole workgroup until done[d] >= target.  Returns false
// (for every thread) if the batch has been aborted or this wait timed out.
__device__ __forceinline__ bool wait_domain(unsigned* done, int d, unsigned target, int* err,
                                            long long spin_limit, int* s_flag) {
  if (threadIdx.x == 0) {
    int ok = 1;
    long long it = 0;
    while (__hip_atomic_load(&done[d], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) { ok = 0; break; }
      if (++it > spin_limit) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    *s_flag = ok;
  }
  __syncthreads();
  return *s_flag != 0;
}

template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX)
    k_batch_persistent(const BatchDomain<T>* __restrict__ dom, const BatchTile* __restrict__ tiles,
                       const int* __restrict__ wg_begin, unsigned* __restrict__ done,
                       int* __restrict__ err, int nsteps, int parity, long long spin_limit) {
  __shared__ typename V2<T>::t ring[4][BX + 2];
  __shared__ int s_flag;
  const int t0 = wg_begin[blockIdx.x], t1 = wg_begin[blockIdx.x + 1];
  for (int s = 0; s < nsteps; ++s) {
    const int p = (parity + s) & 1;
    for (int t = t0; t < t1; ++t) {
      const int d = __builtin_amdgcn_readfirstlane(tiles[t].domain);
      const int x0 = __builtin_amdgcn_readfirstlane(tiles[t].x0);
      const int y0 = __builtin_amdgcn_readfirstlane(tiles[t].y0);
      const int down = __builtin_amdgcn_readfirstlane(tiles[t].down);
      const BatchDomain<T>& D = dom[d];
      if (s > 0 && !wait_domain(done, d, D.ntiles * (unsigned)s, err, spin_limit, &s_flag)) return;
      step_tile<T, EOS, BX, BIG>(D.f[p], D.f[p ^ 1], D.g, D.c, x0, y0, down != 0, ring);
      // make this thread's stores visible device-wide, then count the tile once
      __threadfence();
      __syncthreads();
      if (threadIdx.x == 0) __hip_atomic_fetch_add(&done[d], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

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

__global__ void k_batch_reset(unsigned* done, int n, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) done[i] = 0u;
  if (i == 0) *err = 0;
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------
template <typename T, int EOS, int BX>
static const void* persistent_fn() {
  return reinterpret_cast<const void*>(&k_batch_persistent<T, EOS, BX, false>);
}

template <typename T>
static hipError_t occupancy_t(int eos, int bx, int* per_cu) {
#define LBM_OCC(E, B)                                                                       \
  if (eos == E && bx == B)                                                                  \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, persistent_fn<T, E, B>(), B, 0);
  LBM_OCC(LBM_EOS_IDEAL, 64) LBM_OCC(LBM_EOS_IDEAL, 128) LBM_OCC(LBM_EOS_IDEAL, 256)
  LBM_OCC(LBM_EOS_CS, 64) LBM_OCC(LBM_EOS_CS, 128) LBM_OCC(LBM_EOS_CS, 256)
  LBM_OCC(LBM_EOS_VDW, 64) LBM_OCC(LBM_EOS_VDW, 128) LBM_OCC(LBM_EOS_VDW, 256)
  LBM_OCC(LBM_EOS_PR, 64) LBM_OCC(LBM_EOS_PR, 128) LBM_OCC(LBM_EOS_PR, 256)
#undef LBM_OCC
  return hipErrorInvalidValue;
}

hipError_t batch_occupancy(lbm_precision prec, int eos, int tile_x, int* per_cu) {
  if (prec == LBM_FP32) return occupancy_t<float>(eos, tile_x, per_cu);
  return occupancy_t<double>(eos, tile_x, per_cu);
}

template <typename T, int EOS, int BX>
static hipError_t launch_b(bool persistent, const void* dom, const BatchTile* tiles,
                           const int* wg_begin, unsigned* done, int* err, int grid, int nsteps,
                           int parity, long long spin_limit, hipStream_t s) {
  const BatchDomain<T>* d = static_cast<const BatchDomain<T>*>(dom);
  if (persistent)
    hipLaunchKernelGGL((k_batch_persistent<T, EOS, BX, false>), dim3(grid), dim3(BX), 0, s, d,
                       tiles, wg_begin, done, err, nsteps, parity, spin_limit);
  else
    hipLaunchKernelGGL((k_batch_step<T, EOS, BX, false>), dim3(grid), dim3(BX), 0, s, d, tiles,
                       parity);
  return hipGetLastError();
}

template <typename T, int EOS>
static hipError_t launch_e(int bx, bool persistent, const void* dom, const BatchTile* tiles,
                           const int* wg_begin, unsigned* done, int* err, int grid, int nsteps,
                           int parity, long long spin_limit, hipStream_t s) {
  switch (bx) {
    case 64: return launch_b<T, EOS, 64>(persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
    case 128: return launch_b<T, EOS, 128>(persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
    case 256: return launch_b<T, EOS, 256>(persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_t(int eos, int bx, bool persistent, const void* dom,
                           const BatchTile* tiles, const int* wg_begin, unsigned* done, int* err,
                           int grid, int nsteps, int parity, long long spin_limit, hipStream_t s) {
  switch (eos) {
    case LBM_EOS_IDEAL: return launch_e<T, LBM_EOS_IDEAL>(bx, persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
    case LBM_EOS_CS: return launch_e<T, LBM_EOS_CS>(bx, persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
    case LBM_EOS_VDW: return launch_e<T, LBM_EOS_VDW>(bx, persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
    case LBM_EOS_PR: return launch_e<T, LBM_EOS_PR>(bx, persistent, dom, tiles, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(lbm_precision prec, int eos, int tile_x, bool persistent, const void* dom,
                        const void* tiles, const int* wg_begin, unsigned* done, int* err, int grid,
                        int nsteps, int parity, long long spin_limit, hipStream_t s) {
  const BatchTile* t = static_cast<const BatchTile*>(tiles);
  if (prec == LBM_FP32)
    return launch_t<float>(eos, tile_x, persistent, dom, t, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
  return launch_t<double>(eos, tile_x, persistent, dom, t, wg_begin, done, err, grid, nsteps, parity, spin_limit, s);
}

hipError_t launch_batch_reset(unsigned* done, int n, int* err, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_reset, dim3((n + 255) / 256), dim3(256), 0, s, done, n, err);
  return hipGetLastError();
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
