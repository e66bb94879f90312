// Fused time step of the pseudo-potential MRT lattice Boltzmann model on gfx950.
//
// One kernel does the whole step (density/psi pass, Kupershtokh force,
// pressure-tensor term, MRT collision, streaming) with A/B buffers:
//
//  * Pull streaming: cell x gathers f_a(x - e_a) from buffer A and writes its
//    post-collision f*_a(x) to buffer B at x, so every load and every store of
//    a wavefront is a contiguous (at most one element off) run of one plane.
//  * A workgroup of tile_x threads owns a strip of tile_x columns and marches
//    up tile_y rows.  For each row it gathers f, forms rho, U and psi (Eq. 10)
//    and puts (U, psi) into a 4-row ring in LDS; after one barrier the row
//    below has its full 3x3 stencil and is collided and stored.  The strip's
//    two edge columns of (U, psi) are recomputed by two lanes; the first and
//    last row of a tile are recomputed (not stored), so no intermediate field
//    ever goes to HBM: 9 loads + 9 stores per cell per step.
//  * Row offsets are uniform across the workgroup (scalar registers); only the
//    column index is per lane.
#include "lbm_device.h"

namespace lbm {

// f_a(x - e_a) for the 9 velocities, gathered at row r and column x.
// ro_* are the row offsets (elements) of rows r (rr), r - 1 (rm) and r + 1 (rp).
template <typename T>
__device__ __forceinline__ void gather(const T* __restrict__ fa, long long P, long long rr,
                                       long long rm, long long rp, int x, int xm, int xp,
                                       T (&g)[9]) {
  g[0] = fa[0 * P + rr + x];
  g[1] = fa[1 * P + rr + xm];  // e_1 = ( 1, 0)
  g[2] = fa[2 * P + rm + x];   // e_2 = ( 0, 1)
  g[3] = fa[3 * P + rr + xp];  // e_3 = (-1, 0)
  g[4] = fa[4 * P + rp + x];   // e_4 = ( 0,-1)
  g[5] = fa[5 * P + rm + xm];  // e_5 = ( 1, 1)
  g[6] = fa[6 * P + rm + xp];  // e_6 = (-1, 1)
  g[7] = fa[7 * P + rp + xp];  // e_7 = (-1,-1)
  g[8] = fa[8 * P + rp + xm];  // e_8 = ( 1,-1)
}

template <typename T>
__device__ __forceinline__ T density(const T (&g)[9]) {
  return g[0] + ((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
}

template <typename T, int EOS, int BX>
__global__ void __launch_bounds__(BX) k_step(const T* __restrict__ fa, T* __restrict__ fb,
                                              const Geometry geo, const DevC<T> c) {
  using T2 = typename V2<T>::t;
  __shared__ T2 ring[4][BX + 2];

  const int nx = geo.nx, ny = geo.ny;
  const long long P = geo.plane;
  const long long pitch = geo.pitch;
  const int lb = xcd_remap(blockIdx.x, geo.nblocks);
  const int strip = lb / geo.nrowblocks;
  const int rb = lb - strip * geo.nrowblocks;
  const int x0 = strip * BX, y0 = rb * geo.tile_y;
  const int W = min(BX, nx - x0), H = min(geo.tile_y, ny - y0);
  const int tx = threadIdx.x;
  const bool active = tx < W;
  const int x = x0 + (active ? tx : W - 1);  // idle lanes gather a valid column
  const int xm = (x == 0) ? nx - 1 : x - 1;
  const int xp = (x == nx - 1) ? 0 : x + 1;
  // lanes 0 and 1 also produce the strip's left / right edge column
  const bool edge = tx < 2;
  const int hx = (tx == 0) ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + W == nx ? 0 : x0 + W);
  const int hxm = (hx == 0) ? nx - 1 : hx - 1;
  const int hxp = (hx == nx - 1) ? 0 : hx + 1;
  const int hslot = (tx == 0) ? 0 : W + 1;

  T fc[9];
  T rho_c = T(0);
#pragma unroll 1
  for (int i = 0; i < H + 2; ++i) {
    const int r = y0 - 1 + i;
    const long long rr = wrap_(r, ny) * pitch;
    const long long rm = wrap_(r - 1, ny) * pitch;
    const long long rp = wrap_(r + 1, ny) * pitch;
    T g[9];
    gather(fa, P, rr, rm, rp, x, xm, xp, g);
    const T rho = density(g);
    const T U = eos_U<EOS>(rho, c);
    const int slot = i & 3;
    if (active) ring[slot][tx + 1] = T2{U, psi_of(U, c)};
    if (edge) {
      T h[9];
      gather(fa, P, rr, rm, rp, hx, hxm, hxp, h);
      const T Uh = eos_U<EOS>(density(h), c);
      ring[slot][hslot] = T2{Uh, psi_of(Uh, c)};
    }
    __syncthreads();
    if (i >= 2 && active) {
      // stencil of row r - 1: south = row r - 2, north = row r
      const int ss = (i - 2) & 3, sc = (i - 1) & 3, sn = slot;
      T Un[9], Pn[9];
      T2 v;
      v = ring[sc][tx + 1]; Un[0] = v.x; Pn[0] = v.y;
      v = ring[sc][tx + 2]; Un[1] = v.x; Pn[1] = v.y;  // ( 1, 0)
      v = ring[sn][tx + 1]; Un[2] = v.x; Pn[2] = v.y;  // ( 0, 1)
      v = ring[sc][tx];     Un[3] = v.x; Pn[3] = v.y;  // (-1, 0)
      v = ring[ss][tx + 1]; Un[4] = v.x; Pn[4] = v.y;  // ( 0,-1)
      v = ring[sn][tx + 2]; Un[5] = v.x; Pn[5] = v.y;  // ( 1, 1)
      v = ring[sn][tx];     Un[6] = v.x; Pn[6] = v.y;  // (-1, 1)
      v = ring[ss][tx];     Un[7] = v.x; Pn[7] = v.y;  // (-1,-1)
      v = ring[ss][tx + 2]; Un[8] = v.x; Pn[8] = v.y;  // ( 1,-1)
      T out[9];
      collide_cell(fc, rho_c, Un, Pn, c, out);
      T* dst = fb + (long long)(r - 1) * pitch + x;
#pragma unroll
      for (int a = 0; a < 9; ++a) dst[a * P] = out[a];
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) fc[a] = g[a];
    rho_c = rho;
  }
}

template <typename T, int EOS>
static hipError_t launch_step_t(const Geometry& g, const DevC<T>& c, const void* fa, void* fb,
                                hipStream_t s) {
  const T* a = static_cast<const T*>(fa);
  T* b = static_cast<T*>(fb);
  switch (g.tile_x) {
    case 64:
      hipLaunchKernelGGL((k_step<T, EOS, 64>), dim3(g.nblocks), dim3(64), 0, s, a, b, g, c);
      break;
    case 128:
      hipLaunchKernelGGL((k_step<T, EOS, 128>), dim3(g.nblocks), dim3(128), 0, s, a, b, g, c);
      break;
    case 256:
      hipLaunchKernelGGL((k_step<T, EOS, 256>), dim3(g.nblocks), dim3(256), 0, s, a, b, g, c);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
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

hipError_t launch_step(lbm_precision prec, const Geometry& g, const ModelConsts& m, const void* fa,
                       void* fb, hipStream_t s) {
  if (prec == LBM_FP32) return launch_step_p<float>(g, m, fa, fb, s);
  return launch_step_p<double>(g, m, fa, fb, s);
}

// ---------------------------------------------------------------------------
// Initial state: f_a = W_a rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2]
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
  T* dst = f + (long long)y * geo.pitch + x;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const double eu = EX[a] * u + EY[a] * v;
    dst[a * geo.plane] = T(W[a] * r * (1.0 + 3.0 * eu + 4.5 * eu * eu - uu));
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
