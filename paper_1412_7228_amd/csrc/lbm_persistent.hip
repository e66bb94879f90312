// Persistent mode of the batched engine: one launch advances every domain of
// the batch by n pairs of time steps, each tile of the launch's work being one
// two-step pass (step2_tile) of one tile of one domain.
//
// Scheduling.  The domains are split into one group per XCD (on the host:
// longest processing time first onto the least loaded group).  A workgroup
// reads the XCD it runs on from the hardware (XCC_ID) and takes work items
// from that XCD's queue: the group's tiles, pair by pair (item q is tile
// q mod nt of pair q / nt, nt the group's tile count), by one atomic add on
// the queue head.  A per-domain counter of finished tiles is the domain's
// barrier: a tile of pair s starts once all of the domain's tiles of pair
// s - 1 have finished (counter >= ntiles * s).  That one condition orders
// both the reads of pair s after the writes of pair s - 1 and the writes of
// pair s (into the buffer pair s - 1 read) after those reads.
//
// Progress.  A work item is taken only by a running workgroup, and a queue
// hands out items in pair order, so the earliest unfinished item of a group
// never waits (everything it depends on came earlier in the queue and was
// taken by running workgroups); by induction every item finishes.  Every
// loop is bounded: the tile loop by the number of items (each iteration takes
// a new one), the wait by a spin limit, after which the wait sets an error
// flag that makes every other wait and every workgroup leave, so a launch
// always ends; a check kernel after it reports domains with missing tiles.
//
// Uniform control flow.  Every loop test and every exit is taken on values in
// scalar registers (read back with readfirstlane), so a loop never runs with
// part of a wave active: the wait loop runs on all 64 lanes of wave 0, lane 0
// alone making the atomic reads in a straight-line section whose result is
// broadcast; the other waves wait at a barrier.  The only per-lane sections
// are straight-line single-thread atomics, each followed by a barrier.
//
// Memory ordering.  Producer and consumer of a barrier run on one XCD and so
// share its L2: a tile is counted only after every wave's stores have been
// acknowledged by that L2 (s_waitcnt vmcnt(0), then a barrier), and a wave
// that passes a wait invalidates its CU's L1 at agent scope (buffer_inv sc1)
// before it loads.  A workgroup-scope invalidation (buffer_inv sc0) is not
// enough: outside thread-group-split mode the L1 counts as coherent for the
// workgroup and is left as it is, so a consumer could read lines of its
// domain that its CU cached before the producer on another CU wrote them.
// No L2 write-back is needed inside the launch (one per tile costs a factor of
// four or more); the kernel boundaries order everything across XCDs as for
// any launch.
#include "lbm_batch.h"

namespace lbm {

// The XCD this wave runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcd_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20);
}

// Value of a counter that other workgroups of this XCD advance with atomics:
// a compare-and-swap that never matches (no counter reaches 2^32 - 1), so the
// read is performed where the increments are.
__device__ __forceinline__ unsigned poll(unsigned* p) {
  unsigned v = 0xFFFFFFFFu;
  __hip_atomic_compare_exchange_strong(p, &v, 0xFFFFFFFFu, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

// Bounded wait of the whole workgroup until done[d] >= target.  Wave 0 runs
// the loop with all its lanes (the wave index is a scalar); lane 0 reads the
// counters and each test is on its values broadcast into scalar registers.
// Returns, to every thread, true once the counter has reached the target and
// false if the batch was aborted or this wait passed the spin limit (which
// aborts the batch).  On success every wave invalidates its CU's L1 (agent
// scope: the workgroup-scope form does not touch the L1).
__device__ __forceinline__ bool wait_domain(unsigned* done, int d, unsigned target, int* err,
                                            long long spin_limit, int* s_flag) {
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;
  if (wave == 0) {
    const bool lead = threadIdx.x == 0;
    int ok = 1;
    for (long long it = 0;; ++it) {
      unsigned v = 0u, e = 0u;
      if (lead) {
        v = poll(&done[d]);
        e = poll(reinterpret_cast<unsigned*>(err));
      }
      v = __builtin_amdgcn_readfirstlane(v);
      e = __builtin_amdgcn_readfirstlane(e);
      if (v >= target) break;
      if (e != 0u) {
        ok = 0;
        break;
      }
      if (it >= spin_limit) {
        if (lead) __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    if (lead) *s_flag = ok;
  }
  __syncthreads();
  const bool ok = __builtin_amdgcn_readfirstlane(*s_flag) != 0;
  if (ok) asm volatile("buffer_inv sc1" ::: "memory");
  return ok;
}

// Gathers two rows ahead (AHEAD = 2 of step2_tile); FP32: four waves per SIMD.
template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX, sizeof(T) == 4 ? 4 : 1)
    k_batch_persistent(const BatchDomain<T>* __restrict__ dom, const BatchTile* __restrict__ tiles,
                       const int* __restrict__ group_begin, int ngroups, unsigned* __restrict__ head,
                       unsigned* __restrict__ done, int* __restrict__ err, int npairs, int parity,
                       long long spin_limit) {
  __shared__ Tile2Lds<T, BX> lds;
  __shared__ int s_flag;
  __shared__ unsigned s_q;
  const int g = __builtin_amdgcn_readfirstlane(xcd_id());
  if (g >= ngroups) return;  // an XCD that holds no group
  const int b0 = group_begin[g];
  const unsigned nt = (unsigned)(group_begin[g + 1] - b0);
  const unsigned total = nt * (unsigned)npairs;
  if (threadIdx.x == 0) s_q = __hip_atomic_fetch_add(&head[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  unsigned q = __builtin_amdgcn_readfirstlane(s_q);
  // each iteration takes a new item, so at most `total` iterations
  for (unsigned it = 0; it < total && q < total; ++it) {
    const unsigned s = q / nt;
    const BatchTile* tp = tiles + b0 + (int)(q - s * nt);
    const int d = __builtin_amdgcn_readfirstlane(tp->domain);
    const int x0 = __builtin_amdgcn_readfirstlane(tp->x0);
    const int y0 = __builtin_amdgcn_readfirstlane(tp->y0);
    const int down = __builtin_amdgcn_readfirstlane(tp->down);
    const BatchDomain<T>& D = dom[d];
    if (s > 0 && !wait_domain(done, d, D.ntiles * s, err, spin_limit, &s_flag)) break;
    const int p = (parity + (int)s) & 1;
    // waves of a narrow strip with no needed lane only keep the barriers
    if (down)
      step2_tile<T, EOS, BX, BIG, true, true, 2>(D.f[p], D.f[p ^ 1], D.g, D.c, x0, y0, lds);
    else
      step2_tile<T, EOS, BX, BIG, false, true, 2>(D.f[p], D.f[p ^ 1], D.g, D.c, x0, y0, lds);
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

__global__ void k_batch_reset(unsigned* done, int n, unsigned* head, int ngroups, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) done[i] = 0u;
  if (i < ngroups) head[i] = 0u;
  if (i == 0) *err = 0;
}

// After a persistent launch: every domain must have counted all its tiles of
// every pair unless a wait aborted; otherwise no workgroup served its group.
template <typename T>
__global__ void k_batch_check(const BatchDomain<T>* __restrict__ dom, const unsigned* done, int n,
                              int npairs, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && done[i] != dom[i].ntiles * (unsigned)npairs && *err == 0) atomicOr(err, 2);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
template <typename T, int EOS, int BX>
static const void* persistent_fn() {
  return reinterpret_cast<const void*>(&k_batch_persistent<T, EOS, BX, false>);
}

template <typename T, int EOS>
static hipError_t occupancy_e(int bx, int* per_cu) {
  switch (bx) {
    case 128: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, persistent_fn<T, EOS, 128>(), 128, 0);
    case 256: return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, persistent_fn<T, EOS, 256>(), 256, 0);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t occupancy_t(int eos, int bx, int* per_cu) {
  switch (eos) {
    case LBM_EOS_IDEAL: return occupancy_e<T, LBM_EOS_IDEAL>(bx, per_cu);
    case LBM_EOS_CS: return occupancy_e<T, LBM_EOS_CS>(bx, per_cu);
    case LBM_EOS_VDW: return occupancy_e<T, LBM_EOS_VDW>(bx, per_cu);
    case LBM_EOS_PR: return occupancy_e<T, LBM_EOS_PR>(bx, per_cu);
  }
  return hipErrorInvalidValue;
}

hipError_t batch_occupancy(lbm_precision prec, int eos, int tile_x, int* per_cu) {
  if (prec == LBM_FP32) return occupancy_t<float>(eos, tile_x, per_cu);
  return occupancy_t<double>(eos, tile_x, per_cu);
}

template <typename T, int EOS, int BX>
static hipError_t launch_p(const BatchRun& r, hipStream_t s) {
  hipLaunchKernelGGL((k_batch_persistent<T, EOS, BX, false>), dim3(r.grid), dim3(BX), 0, s,
                     static_cast<const BatchDomain<T>*>(r.dom), static_cast<const BatchTile*>(r.tiles),
                     r.group_begin, r.ngroups, r.head, r.done, r.err, r.nsteps, r.parity, r.spin_limit);
  return hipGetLastError();
}

template <typename T, int EOS>
static hipError_t launch_pe(int bx, const BatchRun& r, hipStream_t s) {
  switch (bx) {
    case 128: return launch_p<T, EOS, 128>(r, s);
    case 256: return launch_p<T, EOS, 256>(r, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_pt(int eos, int bx, const BatchRun& r, hipStream_t s) {
  switch (eos) {
    case LBM_EOS_IDEAL: return launch_pe<T, LBM_EOS_IDEAL>(bx, r, s);
    case LBM_EOS_CS: return launch_pe<T, LBM_EOS_CS>(bx, r, s);
    case LBM_EOS_VDW: return launch_pe<T, LBM_EOS_VDW>(bx, r, s);
    case LBM_EOS_PR: return launch_pe<T, LBM_EOS_PR>(bx, r, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_persistent(lbm_precision prec, int eos, int tile_x, const BatchRun& r,
                                   hipStream_t s) {
  if (prec == LBM_FP32) return launch_pt<float>(eos, tile_x, r, s);
  return launch_pt<double>(eos, tile_x, r, s);
}

hipError_t launch_batch_reset(const BatchRun& r, int ndomains, hipStream_t s) {
  const int n = ndomains > r.ngroups ? ndomains : r.ngroups;
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

}  // namespace lbm
