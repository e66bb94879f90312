// Single-lattice time step: one launch of k_step per step, or one launch of
// k_step2 per two steps.
#include "lbm_tile.h"
#include "lbm_tile2.h"

namespace lbm {

// One time step over the whole lattice: workgroup -> tile with the strips of
// a row block consecutive (so x-neighbours share an XCD), row blocks
// alternating their march direction.
template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX) k_step(const T* __restrict__ fa, T* __restrict__ fb,
                                              const Geometry geo, const DevC<T> c) {
  __shared__ typename V2<T>::t ring[4][BX + 2];
  const int lb = xcd_remap(blockIdx.x, geo.nblocks);
  const int rb = lb / geo.nstrips;
  const int strip = lb - rb * geo.nstrips;
  step_tile<T, EOS, BX, BIG>(fa, fb, geo, c, strip * BX, geo.y_begin + rb * geo.tile_y, (rb & 1) != 0,
                             ring);
}

template <typename T, int EOS, bool BIG>
static hipError_t launch_step_b(const Geometry& g, const DevC<T>& c, const void* fa, void* fb,
                                hipStream_t s) {
  const T* a = static_cast<const T*>(fa);
  T* b = static_cast<T*>(fb);
  switch (g.tile_x) {
    case 64:
      hipLaunchKernelGGL((k_step<T, EOS, 64, BIG>), dim3(g.nblocks), dim3(64), 0, s, a, b, g, c);
      break;
    case 128:
      hipLaunchKernelGGL((k_step<T, EOS, 128, BIG>), dim3(g.nblocks), dim3(128), 0, s, a, b, g, c);
      break;
    case 256:
      hipLaunchKernelGGL((k_step<T, EOS, 256, BIG>), dim3(g.nblocks), dim3(256), 0, s, a, b, g, c);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EOS>
static hipError_t launch_step_t(const Geometry& g, const DevC<T>& c, const void* fa, void* fb,
                                hipStream_t s) {
  const unsigned long long bytes = (unsigned long long)g.ny * g.row * sizeof(T);
  if (bytes < (1ull << 32)) return launch_step_b<T, EOS, false>(g, c, fa, fb, s);
  return launch_step_b<T, EOS, true>(g, c, fa, fb, s);
}

template <typename T>
static hipError_t launch_step_p(const Geometry& g, const ModelConsts& m, const void* fa, void* fb,
                                hipStream_t s) {
  const DevC<T> c = make_devc<T>(m);
  switch (m.eos) {
    case LBM_EOS_IDEAL: return launch_step_t<T, LBM_EOS_IDEAL>(g, c, fa, fb, s);
    case LBM_EOS_CS: return launch_step_t<T, LBM_EOS_CS>(g, c, fa, fb, s);
    case LBM_EOS_VDW: return launch_step_t<T, LBM_EOS_VDW>(g, c, fa, fb, s);
    case LBM_EOS_PR: return launch_step_t<T, LBM_EOS_PR>(g, c, fa, fb, s);
    default: return hipErrorInvalidValue;
  }
}

// Rows gathered ahead by the two-step kernel (AHEAD of step2_tile): FP32 one
// row, which fits five waves per SIMD (96 VGPRs); FP64 two rows (two waves per
// SIMD either way).  Measured on the row-interleaved layout, alternating
// builds: FP32 one row ahead at five waves is 0.3% faster than two rows ahead
// at four on 4096^2 at steps 200-2200, 2.7% at steps 5-25, and 10% on a
// 4096 x 520 slab in 128 x 8 tiles; FP64 two rows ahead 1% faster than one.
template <typename T>
constexpr int step2_ahead() { return sizeof(T) == 4 ? 1 : 2; }

// Two fused steps over the whole lattice; the same workgroup-to-tile order.
template <typename T, int EOS, int BX, bool BIG>
__global__ void __launch_bounds__(BX, sizeof(T) == 4 ? 5 : 1) k_step2(const T* __restrict__ fa, T* __restrict__ fb,
                                               const Geometry geo, const DevC<T> c) {
  __shared__ Tile2Lds<T, BX> lds;
  static_assert(tile2_width<BX>() == BX - kStep2Halo, "strip width");
  const int lb = xcd_remap(blockIdx.x, geo.nblocks);
  const int rb = lb / geo.nstrips;
  const int strip = lb - rb * geo.nstrips;
  const int xs = strip * tile2_width<BX>(), y0 = geo.y_begin + rb * geo.tile_y;
  if (rb & 1)
    step2_tile<T, EOS, BX, BIG, true, false, step2_ahead<T>()>(fa, fb, geo, c, xs, y0, lds);
  else
    step2_tile<T, EOS, BX, BIG, false, false, step2_ahead<T>()>(fa, fb, geo, c, xs, y0, lds);
}

template <typename T, int EOS, bool BIG>
static hipError_t launch_step2_b(const Geometry& g, const DevC<T>& c, const void* fa, void* fb,
                                 hipStream_t s) {
  const T* a = static_cast<const T*>(fa);
  T* b = static_cast<T*>(fb);
  switch (g.tile_x) {
    case 128:
      hipLaunchKernelGGL((k_step2<T, EOS, 128, BIG>), dim3(g.nblocks), dim3(128), 0, s, a, b, g, c);
      break;
    case 256:
      hipLaunchKernelGGL((k_step2<T, EOS, 256, BIG>), dim3(g.nblocks), dim3(256), 0, s, a, b, g, c);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int EOS>
static hipError_t launch_step2_t(const Geometry& g, const DevC<T>& c, const void* fa, void* fb,
                                 hipStream_t s) {
  const unsigned long long bytes = (unsigned long long)g.ny * g.row * sizeof(T);
  if (bytes < (1ull << 32)) return launch_step2_b<T, EOS, false>(g, c, fa, fb, s);
  return launch_step2_b<T, EOS, true>(g, c, fa, fb, s);
}

template <typename T>
static hipError_t launch_step2_p(const Geometry& g, const ModelConsts& m, const void* fa, void* fb,
                                 hipStream_t s) {
  const DevC<T> c = make_devc<T>(m);
  switch (m.eos) {
    case LBM_EOS_IDEAL: return launch_step2_t<T, LBM_EOS_IDEAL>(g, c, fa, fb, s);
    case LBM_EOS_CS: return launch_step2_t<T, LBM_EOS_CS>(g, c, fa, fb, s);
    case LBM_EOS_VDW: return launch_step2_t<T, LBM_EOS_VDW>(g, c, fa, fb, s);
    case LBM_EOS_PR: return launch_step2_t<T, LBM_EOS_PR>(g, c, fa, fb, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_step2(lbm_precision prec, const Geometry& g, const ModelConsts& m, const void* fa,
                        void* fb, hipStream_t s) {
  if (prec == LBM_FP32) return launch_step2_p<float>(g, m, fa, fb, s);
  return launch_step2_p<double>(g, m, fa, fb, s);
}

template <typename T, int EOS>
static hipError_t occupancy_e(int bx, bool big, int* per_cu) {
#define LBM_OCC(B)                                                                              \
  if (bx == B)                                                                                  \
    return big ? hipOccupancyMaxActiveBlocksPerMultiprocessor(                                  \
                     per_cu, reinterpret_cast<const void*>(&k_step<T, EOS, B, true>), B, 0)     \
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(                                  \
                     per_cu, reinterpret_cast<const void*>(&k_step<T, EOS, B, false>), B, 0);
  LBM_OCC(64) LBM_OCC(128) LBM_OCC(256)
#undef LBM_OCC
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t occupancy_t(int eos, int bx, bool big, int* per_cu) {
  switch (eos) {
    case LBM_EOS_IDEAL: return occupancy_e<T, LBM_EOS_IDEAL>(bx, big, per_cu);
    case LBM_EOS_CS: return occupancy_e<T, LBM_EOS_CS>(bx, big, per_cu);
    case LBM_EOS_VDW: return occupancy_e<T, LBM_EOS_VDW>(bx, big, per_cu);
    case LBM_EOS_PR: return occupancy_e<T, LBM_EOS_PR>(bx, big, per_cu);
  }
  return hipErrorInvalidValue;
}

hipError_t step_occupancy(lbm_precision prec, const Geometry& g, int eos, int* per_cu) {
  const size_t es = prec == LBM_FP32 ? 4 : 8;
  const bool big = (unsigned long long)g.ny * g.row * es >= (1ull << 32);
  if (prec == LBM_FP32) return occupancy_t<float>(eos, g.tile_x, big, per_cu);
  return occupancy_t<double>(eos, g.tile_x, big, per_cu);
}

hipError_t launch_step(lbm_precision prec, const Geometry& g, const ModelConsts& m, const void* fa,
                       void* fb, hipStream_t s) {
  if (prec == LBM_FP32) return launch_step_p<float>(g, m, fa, fb, s);
  return launch_step_p<double>(g, m, fa, fb, s);
}

// ---------------------------------------------------------------------------
// Initial state: f_a = W_a rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2], stored at
// the unstreamed position of each distribution (state_index).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_init_eq(const double* __restrict__ rho, const double* __restrict__ ux,
                          const double* __restrict__ uy, T* __restrict__ f, const Geometry geo) {
  const long long n = (long long)geo.nx * geo.ny;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int y = (int)(c / geo.nx), x = (int)(c - (long long)y * geo.nx);
  const double r = rho[c];
  const double u = ux ? ux[c] : 0.0, v = uy ? uy[c] : 0.0;
  const double uu = 1.5 * (u * u + v * v);
  const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const double eu = EX[a] * u + EY[a] * v;
    f[state_index(geo, a, x, y)] = T(W[a] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - uu));
  }
}

hipError_t launch_init_equilibrium(lbm_precision prec, const Geometry& g, const double* rho,
                                   const double* ux, const double* uy, void* f, hipStream_t s) {
  const long long n = (long long)g.nx * g.ny;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  if (prec == LBM_FP32)
    hipLaunchKernelGGL(k_init_eq<float>, grid, block, 0, s, rho, ux, uy, static_cast<float*>(f), g);
  else
    hipLaunchKernelGGL(k_init_eq<double>, grid, block, 0, s, rho, ux, uy, static_cast<double*>(f), g);
  return hipGetLastError();
}

}  // namespace lbm
