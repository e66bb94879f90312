// Test fixture (not part of the library, never launched): a barrier inside a
// lane-dependent branch.  The compiler masks the branch with exec and skips
// it for a wave whose mask is empty, barrier included, so such a wave would
// pass one barrier fewer than the others.  The CPU test that compiles this
// file checks that its barrier-reachability check on the gfx950 assembly
// reports this barrier, and none in the library's two-step kernels.
#include <hip/hip_runtime.h>

__global__ void k_barrier_in_branch(const float* in, float* out, int n) {
  __shared__ float s[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float v = i < n ? in[i] : 0.f;
  if (v > 0.5f) {  // data-dependent, hence divergent
    s[threadIdx.x] = v;
    __syncthreads();
    v += s[(threadIdx.x + 1) & 255];
  }
  if (i < n) out[i] = v;
}
