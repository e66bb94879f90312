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

// The distribution buffers as seen by the step kernels.  Rows are
// interleaved: lattice row y holds the nine planes' rows back to back (row
// stride row_bytes, plane a at a * plane_bytes within it).  A buffer below
// 4 GiB is one resource, with the row and plane offsets in the scalar
// offset; a larger one gets a resource per lattice row, made when the row is
// addressed (a row of nine planes stays below 4 GiB).
template <bool BIG>
struct Planes {
  __amdgpu_buffer_rsrc_t r;  // the whole buffer (below 4 GiB)
  const char* base;
  unsigned plane_bytes, row_bytes;
  struct Row {
    __amdgpu_buffer_rsrc_t rs;
    unsigned off;  // scalar byte offset of plane 0 of the row
  };
  __device__ __forceinline__ void init(const void* b, unsigned plane_b, unsigned row_b,
                                       unsigned long long total_b) {
    base = static_cast<const char*>(b);
    plane_bytes = plane_b;
    row_bytes = row_b;
    if constexpr (!BIG) r = plane_rsrc(b, (unsigned)total_b);
  }
  // lattice row y, 0 <= y < ny
  __device__ __forceinline__ Row row(int y) const {
    if constexpr (BIG) {
      return Row{plane_rsrc(base + (unsigned long long)(unsigned)y * row_bytes, row_bytes), 0u};
    } else {
      return Row{r, (unsigned)y * row_bytes};
    }
  }
};

// f_a(x - e_a) for the 9 velocities, gathered at lattice row yr.  ym, yp are
// rows yr - 1 and yr + 1 after the periodic wrap (uniform); ox, oxm, oxp the
// byte offsets of columns x, x - 1, x + 1 (per lane).
template <typename T, bool BIG>
__device__ __forceinline__ void gather(const Planes<BIG>& pa, int yr, int ym, int yp,
                                       unsigned ox, unsigned oxm, unsigned oxp, T (&g)[9]) {
  const auto R = pa.row(yr), M = pa.row(ym), P = pa.row(yp);
  const unsigned pb = pa.plane_bytes;
  g[0] = ld<T>(R.rs, ox, R.off);
  g[1] = ld<T>(R.rs, oxm, R.off + pb);      // e_1 = ( 1, 0)
  g[2] = ld<T>(M.rs, ox, M.off + 2 * pb);   // e_2 = ( 0, 1)
  g[3] = ld<T>(R.rs, oxp, R.off + 3 * pb);  // e_3 = (-1, 0)
  g[4] = ld<T>(P.rs, ox, P.off + 4 * pb);   // e_4 = ( 0,-1)
  g[5] = ld<T>(M.rs, oxm, M.off + 5 * pb);  // e_5 = ( 1, 1)
  g[6] = ld<T>(M.rs, oxp, M.off + 6 * pb);  // e_6 = (-1, 1)
  g[7] = ld<T>(P.rs, oxp, P.off + 7 * pb);  // e_7 = (-1,-1)
  g[8] = ld<T>(P.rs, oxm, P.off + 8 * pb);  // e_8 = ( 1,-1)
}

// The nine post-collision values of one cell, stored at lattice row y.
template <typename T, bool BIG>
__device__ __forceinline__ void store_row(const Planes<BIG>& pb, int y, unsigned ox,
                                          const T (&out)[9]) {
  const auto W = pb.row(y);
#pragma unroll
  for (int a = 0; a < 9; ++a) st<T>(W.rs, ox, W.off + a * pb.plane_bytes, out[a]);
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

  Planes<BIG> pa, pb;
  const unsigned long long total = (unsigned long long)geo.ny * geo.row * sz;
  pa.init(fa, geo.pitch * sz, (unsigned)(geo.row * sz), total);
  pb.init(fb, geo.pitch * sz, (unsigned)(geo.row * sz), total);

  const int dr = down ? -1 : 1;
  const int r0 = down ? y0 + H : y0 - 1;
  const int n = H + 2;
  // the row offsets of row r: rr (r), rm (r - 1), rp (r + 1)
  auto gather_row = [&](int r, T(&g)[9], T(&h)[9]) {
    const int yr = wrap_(r, ny), ym = wrap_(r - 1, ny), yp = wrap_(r + 1, ny);
    gather(pa, yr, ym, yp, ox, oxm, oxp, g);
    if (edge) gather(pa, yr, ym, yp, ohx, ohxm, ohxp, h);
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
      store_row(pb, r - dr, ox, out);
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) fc[a] = g[a];
    rho_c = rho;
  }
}

}  // namespace lbm
