// Batched engine: many independent periodic lattices (droplets of uneven size
// and parameters) advanced together on one GPU.
//
// Every domain is cut into tiles of tile_x columns x tile_y rows and each tile
// runs the same step_tile() as the single-lattice kernel.  Two launch modes:
//
//  * persistent: one launch advances every domain by n steps.  The domains are
//    split into one group per XCD (longest processing time first) and every
//    domain lives on the XCD of its group for the whole launch: a workgroup
//    reads the XCD it runs on from the hardware and takes tiles of that XCD's
//    group from a queue ordered step by step.  A per-domain counter is the
//    domain's step barrier: a tile of step s starts when all of the domain's
//    tiles of step s - 1 are done.  Producer and consumer of every barrier then
//    share one L2, so the barrier needs only the tile's stores to have reached
//    that L2 (a wait on the vector memory counter) and, on the consumer side,
//    an invalidation of the CU's L1; no L2 write-back or invalidation, which
//    is what device-wide release/acquire costs on a chip whose XCDs have
//    separate L2 caches.  Waits are bounded: one that exceeds the spin limit
//    sets an error flag and every workgroup leaves, so the launch always ends;
//    a check after the launch flags a group no workgroup served.  The queue
//    and counter reset, the launch and the check are captured in a HIP graph.
//  * per-step: one launch per step over all tiles (kernel boundaries order
//    the steps); chunks of steps are captured in a HIP graph.
#include <algorithm>
#include <vector>

#include "lbm_tile.h"
#include "lbm_tile2.h"

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

// The XCD this wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
}

// Current value of a counter that other workgroups change with atomics.  A
// compare-and-swap that never matches (no counter reaches 2^32 - 1) is a
// read-modify-write, performed where the increments are; a plain relaxed
// atomic load is not enough: it may keep hitting a copy of the line that the
// first poll left in this XCD's L2.
__device__ __forceinline__ unsigned poll(unsigned* p) {
  unsigned v = 0xFFFFFFFFu;
  __hip_atomic_compare_exchange_strong(p, &v, 0xFFFFFFFFu, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// Bounded wait of the whole workgroup until done[d] >= target.  On success
// every wave invalidates its CU's L1: the loads that follow then miss in L1
// and read the L2 that the producers' stores reached.  Returns false (for
// every thread) if the batch has been aborted or this wait timed out.
__device__ __forceinline__ bool wait_domain(unsigned* done, int d, unsigned target, int* err,
                                            long long spin_limit, int* s_flag) {
  if (threadIdx.x == 0) {
    int ok = 1;
    long long it = 0;
    while (poll(&done[d]) < target) {
      if (poll(reinterpret_cast<unsigned*>(err)) != 0u) { ok = 0; break; }
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
  // uniform: every exit of the tile loop must be a branch of the whole wave
  const bool ok = __builtin_amdgcn_readfirstlane(*s_flag) != 0;
  if (ok) asm volatile("buffer_inv sc0" ::: "memory");
  return ok;
}

template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX)
    k_batch_persistent(const BatchDomain<T>* __restrict__ dom, const BatchTile* __restrict__ tiles,
                       const int* __restrict__ group_begin, int ngroups, unsigned* __restrict__ head,
                       unsigned* __restrict__ done, int* __restrict__ err, int nsteps, int parity,
                       long long spin_limit) {
  __shared__ typename V2<T>::t ring[4][BX + 2];
  __shared__ int s_flag;
  __shared__ unsigned s_q;
  const int g = xcd_id();
  if (g >= ngroups) return;  // an XCD that holds no group
  const int b0 = group_begin[g];
  const unsigned nt = (unsigned)(group_begin[g + 1] - b0);
  const unsigned total = nt * (unsigned)nsteps;
  // Every branch that leaves or repeats the loop is uniform (read back with
  // readfirstlane), and the two single-thread sections (the wait's poll, and
  // counting a finished tile together with taking the next one) each end at
  // a barrier: no lane may start a tile before thread 0 has taken it.
  if (threadIdx.x == 0) s_q = __hip_atomic_fetch_add(&head[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  unsigned q = __builtin_amdgcn_readfirstlane(s_q);
  while (q < total) {
    const unsigned s = q / nt;
    const BatchTile tl = tiles[b0 + (int)(q - s * nt)];
    const int d = __builtin_amdgcn_readfirstlane(tl.domain);
    const int x0 = __builtin_amdgcn_readfirstlane(tl.x0);
    const int y0 = __builtin_amdgcn_readfirstlane(tl.y0);
    const int down = __builtin_amdgcn_readfirstlane(tl.down);
    const BatchDomain<T>& D = dom[d];
    if (s > 0 && !wait_domain(done, d, D.ntiles * s, err, spin_limit, &s_flag)) return;
    const int p = (parity + (int)s) & 1;
    step_tile<T, EOS, BX, BIG>(D.f[p], D.f[p ^ 1], D.g, D.c, x0, y0, down != 0, ring);
    // every wave's stores have reached this XCD's L2 before the tile is counted
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
      __hip_atomic_fetch_add(&done[d], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_q = __hip_atomic_fetch_add(&head[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    q = __builtin_amdgcn_readfirstlane(s_q);
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

__global__ void k_batch_reset(unsigned* done, int n, unsigned* head, int ngroups, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) done[i] = 0u;
  if (i < ngroups) head[i] = 0u;
  if (i == 0) *err = 0;
}

// After a persistent launch: every domain must have counted all its tiles of
// every step unless a wait aborted; otherwise no workgroup served its group.
template <typename T>
__global__ void k_batch_check(const BatchDomain<T>* __restrict__ dom, const unsigned* done, int n,
                              int nsteps, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && done[i] != dom[i].ntiles * (unsigned)nsteps && *err == 0) atomicOr(err, 2);
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
static hipError_t launch_b(bool persistent, const BatchRun& r, hipStream_t s) {
  const BatchDomain<T>* d = static_cast<const BatchDomain<T>*>(r.dom);
  const BatchTile* t = static_cast<const BatchTile*>(r.tiles);
  if (persistent)
    hipLaunchKernelGGL((k_batch_persistent<T, EOS, BX, false>), dim3(r.grid), dim3(BX), 0, s, d, t,
                       r.group_begin, r.ngroups, r.head, r.done, r.err, r.nsteps, r.parity,
                       r.spin_limit);
  else
    hipLaunchKernelGGL((k_batch_step<T, EOS, BX, false>), dim3(r.grid), dim3(BX), 0, s, d, t,
                       r.parity);
  return hipGetLastError();
}

template <typename T, int EOS>
static hipError_t launch_e(int bx, bool persistent, const BatchRun& r, hipStream_t s) {
  switch (bx) {
    case 64: return launch_b<T, EOS, 64>(persistent, r, s);
    case 128: return launch_b<T, EOS, 128>(persistent, r, s);
    case 256: return launch_b<T, EOS, 256>(persistent, r, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_t(int eos, int bx, bool persistent, const BatchRun& r, hipStream_t s) {
  switch (eos) {
    case LBM_EOS_IDEAL: return launch_e<T, LBM_EOS_IDEAL>(bx, persistent, r, s);
    case LBM_EOS_CS: return launch_e<T, LBM_EOS_CS>(bx, persistent, r, s);
    case LBM_EOS_VDW: return launch_e<T, LBM_EOS_VDW>(bx, persistent, r, s);
    case LBM_EOS_PR: return launch_e<T, LBM_EOS_PR>(bx, persistent, r, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch(lbm_precision prec, int eos, int tile_x, bool persistent, const BatchRun& r,
                        hipStream_t s) {
  if (prec == LBM_FP32) return launch_t<float>(eos, tile_x, persistent, r, s);
  return launch_t<double>(eos, tile_x, persistent, r, s);
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

hipError_t launch_batch_reset(const BatchRun& r, int ndomains, hipStream_t s) {
  const int n = std::max(ndomains, r.ngroups);
  hipLaunchKernelGGL(k_batch_reset, dim3((n + 255) / 256), dim3(256), 0, s, r.done, ndomains,
                     r.head, r.ngroups, r.err);
  return hipGetLastError();
}

hipError_t launch_batch_check(lbm_precision prec, const BatchRun& r, int ndomains, hipStream_t s) {
  const dim3 grid((ndomains + 255) / 256);
  if (prec == LBM_FP32)
    hipLaunchKernelGGL(k_batch_check<float>, grid, dim3(256), 0, s,
                       static_cast<const BatchDomain<float>*>(r.dom), r.done, ndomains, r.nsteps, r.err);
  else
    hipLaunchKernelGGL(k_batch_check<double>, grid, dim3(256), 0, s,
                       static_cast<const BatchDomain<double>*>(r.dom), r.done, ndomains, r.nsteps, r.err);
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
