// Test fixture (not part of the library): the shape of the persistent batch
// kernel's earlier barrier wait, in which thread 0 alone polled a counter in a
// loop inside a thread-0 section while the workgroup's other lanes and waves
// waited at the barrier after it.  The loop's exit then depends on which
// lanes are still active, which the compiler expresses as an exec mask that
// the loop narrows (s_andn2_b64 exec, exec, ...).  The CPU test that compiles
// this file checks that its gfx950 assembly shows that pattern, and that the
// library's persistent kernel shows none.
#include <hip/hip_runtime.h>

__device__ __forceinline__ unsigned poll(unsigned* p) {
  unsigned v = 0xFFFFFFFFu;
  __hip_atomic_compare_exchange_strong(p, &v, 0xFFFFFFFFu, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

__global__ void k_thread0_wait(unsigned* done, int* err, unsigned target, long long spin_limit,
                               unsigned* out) {
  __shared__ int s_flag;
  if (threadIdx.x == 0) {
    int ok = 1;
    long long it = 0;
    while (poll(done) < target) {
      if (poll(reinterpret_cast<unsigned*>(err)) != 0u) { ok = 0; break; }
      if (++it > spin_limit) {
        __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    s_flag = ok;
  }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = __builtin_amdgcn_readfirstlane(s_flag);
}
