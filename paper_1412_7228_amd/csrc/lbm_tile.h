// The fused time step of one tile of a lattice on gfx950, shared by the
// single-lattice kernel (lbm_step.hip) and the batched persistent engine
// (lbm_batch.hip).
//
//  * Pull streaming: cell x gathers f_a(x - e_a) from buffer A and writes its
//    post-collision f*_a(x) to buffer B at x, so every load and every store of
//    a wavefront is a contiguous (at most one element off) run of one plane.
//  * A workgroup of tile_x threads owns a strip of tile_x columns and marches
//    along tile_y rows.  For each row it gathers f, forms rho, U and psi (Eq. 10)
//    and puts (U, psi) into a 4-row ring in LDS; after one barrier the previous
//    row has its full 3x3 stencil and is collided and stored.  The strip's two
//    edge columns of (U, psi) are recomputed by two lanes; the first and last
//    row of a tile are recomputed (not stored), so no intermediate field ever
//    goes to HBM: 9 loads + 9 stores per cell per step.
//  * Row offsets are uniform across the workgroup (scalar registers); only the
//    column index is per lane.
#pragma once

#include "lbm_device.h"

namespace lbm {

template <typename T>
__device__ __forceinline__ T density(const T (&g)[9]) {
  return g[0] + ((g[1] + g[3]) + (g[2] + g[4])) + ((g[5] + g[7]) + (g[6] + g[8]));
}

// Buffer resource of one distribution plane (gfx9 raw buffer, 32-bit
// offsets).  Loads through it take the row offset in a scalar register and
// the column offset in a vector register, so no per-lane 64-bit address
// arithmetic is needed; an offset past the plane reads 0 instead of faulting.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ T ld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
  }
}

template <typename T>
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, T v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
  }
}

// The distribution buffers as seen by the step kernel.  A buffer below 4 GiB
// is one resource and the plane offset goes into the scalar offset; a larger
// one gets one resource per plane.
template <bool BIG>
struct Planes {
  __amdgpu_buffer_rsrc_t r[BIG ? 9 : 1];
  unsigned plane_bytes;
  __device__ __forceinline__ void init(const void* base, unsigned long long plane_b) {
    if constexpr (BIG) {
#pragma unroll
      for (int a = 0; a < 9; ++a)
        r[a] = plane_rsrc(static_cast<const char*>(base) + a * plane_b, (unsigned)plane_b);
    } else {
      r[0] = plane_rsrc(base, (unsigned)(9 * plane_b));
    }
    plane_bytes = (unsigned)plane_b;
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int a) const { return r[BIG ? a : 0]; }
  __device__ __forceinline__ unsigned soff(int a, unsigned row) const {
    return BIG ? row : a * plane_bytes + row;
  }
};

// f_a(x - e_a) for the 9 velocities, gathered at row r.  rr, rm, rp are the
// byte offsets of rows r, r - 1, r + 1 within a plane (uniform); ox, oxm, oxp
// the byte offsets of columns x, x - 1, x + 1 (per lane).
template <typename T, bool BIG>
__device__ __forceinline__ void gather(const Planes<BIG>& pa, unsigned rr, unsigned rm,
                                       unsigned rp, unsigned ox, unsigned oxm, unsigned oxp,
                                       T (&g)[9]) {
  g[0] = ld<T>(pa.rsrc(0), ox, pa.soff(0, rr));
  g[1] = ld<T>(pa.rsrc(1), oxm, pa.soff(1, rr));  // e_1 = ( 1, 0)
  g[2] = ld<T>(pa.rsrc(2), ox, pa.soff(2, rm));   // e_2 = ( 0, 1)
  g[3] = ld<T>(pa.rsrc(3), oxp, pa.soff(3, rr));  // e_3 = (-1, 0)
  g[4] = ld<T>(pa.rsrc(4), ox, pa.soff(4, rp));   // e_4 = ( 0,-1)
  g[5] = ld<T>(pa.rsrc(5), oxm, pa.soff(5, rm));  // e_5 = ( 1, 1)
  g[6] = ld<T>(pa.rsrc(6), oxp, pa.soff(6, rm));  // e_6 = (-1, 1)
  g[7] = ld<T>(pa.rsrc(7), oxp, pa.soff(7, rp));  // e_7 = (-1,-1)
  g[8] = ld<T>(pa.rsrc(8), oxm, pa.soff(8, rp));  // e_8 = ( 1,-1)
}

// One tile: columns [x0, x0 + tile_x) x rows [y0, y0 + tile_y) (clipped to the
// lattice and to the launch's rows [y_begin, y_end)), marched upwards (down = false) or downwards.  Neighbouring row
// blocks march in opposite directions, so the rows they share as halos are
// gathered by both at about the same time and the second gather hits L2.
// The gathers of the next row are issued before the current row's collision
// so their latency overlaps the arithmetic.
template <typename T, int EOS, int BX, bool BIG>
__device__ __forceinline__ void step_tile(const T* __restrict__ fa, T* __restrict__ fb,
                                          const Geometry& geo, const DevC<T>& c, int x0, int y0,
                                          bool down, typename V2<T>::t (*ring)[BX + 2]) {
  using T2 = typename V2<T>::t;
  const int nx = geo.nx, ny = geo.ny;
  const int W = min(BX, nx - x0), H = min(geo.tile_y, geo.y_end - y0);
  const int tx = threadIdx.x;
  const bool active = tx < W;
  const int x = x0 + (active ? tx : W - 1);  // idle lanes gather a valid column
  const unsigned sz = sizeof(T);
  const unsigned ox = x * sz;
  const unsigned oxm = ((x == 0) ? nx - 1 : x - 1) * sz;
  const unsigned oxp = ((x == nx - 1) ? 0 : x + 1) * sz;
  // lanes 0 and 1 also produce the strip's left / right edge column
  const bool edge = tx < 2;
  const int hx = (tx == 0) ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + W == nx ? 0 : x0 + W);
  const unsigned ohx = hx * sz;
  const unsigned ohxm = ((hx == 0) ? nx - 1 : hx - 1) * sz;
  const unsigned ohxp = ((hx == nx - 1) ? 0 : hx + 1) * sz;
  const int hslot = (tx == 0) ? 0 : W + 1;

  const unsigned row_bytes = (unsigned)(geo.pitch * sz);
  Planes<BIG> pa, pb;
  pa.init(fa, (unsigned long long)geo.plane * sz);
  pb.init(fb, (unsigned long long)geo.plane * sz);

  const int dr = down ? -1 : 1;
  const int r0 = down ? y0 + H : y0 - 1;
  const int n = H + 2;
  // the row offsets of row r: rr (r), rm (r - 1), rp (r + 1)
  auto gather_row = [&](int r, T(&g)[9], T(&h)[9]) {
    const unsigned rr = wrap_(r, ny) * row_bytes;
    const unsigned rm = wrap_(r - 1, ny) * row_bytes;
    const unsigned rp = wrap_(r + 1, ny) * row_bytes;
    gather(pa, rr, rm, rp, ox, oxm, oxp, g);
    if (edge) gather(pa, rr, rm, rp, ohx, ohxm, ohxp, h);
  };

  T gn[9], hn[9];
  gather_row(r0, gn, hn);
  T fc[9];
  T rho_c = T(0);
#pragma unroll 1
  for (int i = 0; i < n; ++i) {
    const int r = r0 + dr * i;
    T g[9], h[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      g[a] = gn[a];
      h[a] = hn[a];
    }
    if (i + 1 < n) gather_row(r + dr, gn, hn);
    const T rho = density(g);
    const T U = eos_U<EOS>(rho, c);
    const int slot = i & 3;
    if (active) ring[slot][tx + 1] = T2{U, psi_of(U, c)};
    if (edge) {
      const T Uh = eos_U<EOS>(density(h), c);
      ring[slot][hslot] = T2{Uh, psi_of(Uh, c)};
    }
    __syncthreads();
    if (i >= 2 && active) {
      // collide row r - dr; its stencil rows are r - 2 dr, r - dr (centre) and r
      const int s_far = (i - 2) & 3, sc = (i - 1) & 3;
      const int sn = down ? s_far : slot;  // north = row + 1
      const int ss = down ? slot : s_far;  // south = row - 1
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
      const unsigned ro = (unsigned)(r - dr) * row_bytes;
#pragma unroll
      for (int a = 0; a < 9; ++a) st<T>(pb.rsrc(a), ox, pb.soff(a, ro), out[a]);
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) fc[a] = g[a];
    rho_c = rho;
  }
}

}  // namespace lbm
