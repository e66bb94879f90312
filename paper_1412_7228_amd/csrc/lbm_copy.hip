// The measured HBM ceiling that the step kernels are compared against: a plain
// device copy written for gfx950, one 16-byte load and one 16-byte store per
// lane, one launch over the whole range (consecutive lanes on consecutive
// 16-byte words, so every wave moves 1 KiB in and 1 KiB out per access).
#include <hip/hip_runtime.h>

#include "lbm.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_copy16(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

extern "C" lbm_status lbm_copy_bytes(void* dst, const void* src, size_t bytes, void* hip_stream) {
  if (!dst || !src || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
    return LBM_EINVAL;
  const long long n = (long long)(bytes / 16);
  if (n == 0) return LBM_OK;
  const long long blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return LBM_EINVAL;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     static_cast<const v4f*>(src), static_cast<v4f*>(dst), n);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}
