// Two fused time steps of one tile (temporal blocking), for the single-lattice
// kernel.  A pass reads the state once and writes it once for two steps, so it
// moves half the HBM bytes of two single-step passes at about twice the
// arithmetic per pass; the per-cell arithmetic is step_tile's, operation for
// operation, so both paths give bitwise the same states.
//
// A workgroup of BX lanes covers the BX consecutive columns u = xs - 3 + lane
// (periodic wrap in x) and marches along the rows of its row block.  Per row
// the pipeline runs four stages, each separated by a barrier:
//
//   A  gather f (pulled) of row r, form rho, U, psi        -> LDS ring 1
//   B  collide row r - 1 of the first step                  -> LDS ring F (9 planes)
//   C  pull the second step's f of row r - 2 out of ring F,
//      form rho, U, psi                                     -> LDS ring 2
//   D  collide row r - 3 of the second step                 -> HBM
//
// (rows counted along the march direction).  Stage B is valid on lanes
// 1..BX-2, C on 2..BX-3 and D on 3..BX-4, so a strip stores BX - 6 columns;
// the first step runs on 4 extra rows and the second on 2 extra rows at the
// ends of the row block.  Rings 1 and 2 hold 3 rows of (U, psi), ring F
// 3 rows of the first step's post-collision populations; three barriers per
// row make 3 slots enough.  Lanes outside a stage's valid range compute on
// whatever their neighbours hold (nothing of theirs is stored or read by a
// valid lane), so control flow stays uniform.
#pragma once

#include "lbm_tile.h"

namespace lbm {

template <typename T, int BX>
struct Tile2Lds {
  typename V2<T>::t ring1[3][BX + 2];
  typename V2<T>::t ring2[3][BX + 2];
  T F[3][9][BX + 2];
};

// Columns one pass stores per strip.
template <int BX>
constexpr int tile2_width() { return BX - 6; }

template <typename T, int EOS, int BX, bool BIG>
__device__ __forceinline__ void step2_tile(const T* __restrict__ fa, T* __restrict__ fb,
                                           const Geometry& geo, const DevC<T>& c, int xs, int y0,
                                           bool down, Tile2Lds<T, BX>& L) {
  using T2 = typename V2<T>::t;
  const int nx = geo.nx, ny = geo.ny;
  const int H = min(geo.tile_y, ny - y0);
  const int tx = threadIdx.x;
  const int u = xs - 3 + tx;            // this lane's column before the periodic wrap (>= -3)
  const int x = (u + nx) % nx;          // nx >= 3
  const unsigned sz = sizeof(T);
  const unsigned ox = x * sz;
  const unsigned oxm = ((x == 0) ? nx - 1 : x - 1) * sz;
  const unsigned oxp = ((x == nx - 1) ? 0 : x + 1) * sz;
  const bool store = tx >= 3 && tx < BX - 3 && u < min(xs + tile2_width<BX>(), nx);

  const unsigned row_bytes = (unsigned)(geo.pitch * sz);
  Planes<BIG> pa, pb;
  pa.init(fa, (unsigned long long)geo.plane * sz);
  pb.init(fb, (unsigned long long)geo.plane * sz);

  const int dr = down ? -1 : 1;
  const int r0 = down ? y0 + H + 2 : y0 - 3;
  const int n = H + 6;
  auto gather_row = [&](int r, T(&g)[9]) {
    const unsigned rr = wrap_(r, ny) * row_bytes;
    const unsigned rm = wrap_(r - 1, ny) * row_bytes;
    const unsigned rp = wrap_(r + 1, ny) * row_bytes;
    gather(pa, rr, rm, rp, ox, oxm, oxp, g);
  };
  // slots of the stencil rows: centre row c, the row at + 1 (north) and - 1
  // (south) in lattice y, given the slot of the newest (r) and oldest row
  auto load_stencil = [&](const T2 (*ring)[BX + 2], int s_new, int s_mid, int s_old, T(&Un)[9],
                          T(&Pn)[9]) {
    const int sn = down ? s_old : s_new;
    const int ss = down ? s_new : s_old;
    const int l = tx + 1;
    T2 v;
    v = ring[s_mid][l];     Un[0] = v.x; Pn[0] = v.y;
    v = ring[s_mid][l + 1]; Un[1] = v.x; Pn[1] = v.y;  // ( 1, 0)
    v = ring[sn][l];        Un[2] = v.x; Pn[2] = v.y;  // ( 0, 1)
    v = ring[s_mid][l - 1]; Un[3] = v.x; Pn[3] = v.y;  // (-1, 0)
    v = ring[ss][l];        Un[4] = v.x; Pn[4] = v.y;  // ( 0,-1)
    v = ring[sn][l + 1];    Un[5] = v.x; Pn[5] = v.y;  // ( 1, 1)
    v = ring[sn][l - 1];    Un[6] = v.x; Pn[6] = v.y;  // (-1, 1)
    v = ring[ss][l - 1];    Un[7] = v.x; Pn[7] = v.y;  // (-1,-1)
    v = ring[ss][l + 1];    Un[8] = v.x; Pn[8] = v.y;  // ( 1,-1)
  };

  T gn[9];
  gather_row(r0, gn);
  T fc1[9], fc2[9];
  T rho_c1 = T(0), rho_c2 = T(0);
#pragma unroll 1
  for (int i = 0; i < n; ++i) {
    // ---- A: first-step density of row r
    T g[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) g[a] = gn[a];
    if (i + 1 < n) gather_row(r0 + dr * (i + 1), gn);
    const T rho1 = density(g);
    {
      const T U = eos_U<EOS>(rho1, c);
      L.ring1[i % 3][tx + 1] = T2{U, psi_of(U, c)};
    }
    __syncthreads();
    // ---- B: first-step collision of row r - dr -> ring F slot (i - 1) % 3
    if (i >= 2) {
      T Un[9], Pn[9], out[9];
      load_stencil(L.ring1, i % 3, (i - 1) % 3, (i - 2) % 3, Un, Pn);
      collide_cell(fc1, rho_c1, Un, Pn, c, out);
      const int sf = (i - 1) % 3;
#pragma unroll
      for (int a = 0; a < 9; ++a) L.F[sf][a][tx + 1] = out[a];
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) fc1[a] = g[a];
    rho_c1 = rho1;
    __syncthreads();
    // ---- C: second-step density of row q = r - 2 dr, pulled out of ring F:
    // f_a(x, q) = f*_a(x - e_ax, q - e_ay); row q + k dr sits in slot (i - 2 + k) % 3
    if (i >= 4) {
      const int s_up = (i - 2 + 3 + dr) % 3;  // row q + 1 (lattice y): k = dr
      const int s_q = (i - 2) % 3;
      const int s_dn = (i - 2 + 3 - dr) % 3;  // row q - 1: k = -dr
      const int l = tx + 1;
      T f2[9];
      f2[0] = L.F[s_q][0][l];
      f2[1] = L.F[s_q][1][l - 1];       // e = ( 1, 0)
      f2[2] = L.F[s_dn][2][l];          // e = ( 0, 1)
      f2[3] = L.F[s_q][3][l + 1];       // e = (-1, 0)
      f2[4] = L.F[s_up][4][l];          // e = ( 0,-1)
      f2[5] = L.F[s_dn][5][l - 1];      // e = ( 1, 1)
      f2[6] = L.F[s_dn][6][l + 1];      // e = (-1, 1)
      f2[7] = L.F[s_up][7][l + 1];      // e = (-1,-1)
      f2[8] = L.F[s_up][8][l - 1];      // e = ( 1,-1)
      const T rho2 = density(f2);
      const T U = eos_U<EOS>(rho2, c);
      L.ring2[i % 3][l] = T2{U, psi_of(U, c)};
      __syncthreads();
      // ---- D: second-step collision of row q - dr -> HBM
      if (i >= 6) {
        T Un[9], Pn[9], out[9];
        load_stencil(L.ring2, i % 3, (i - 1) % 3, (i - 2) % 3, Un, Pn);
        collide_cell(fc2, rho_c2, Un, Pn, c, out);
        if (store) {
          const unsigned ro = (unsigned)(r0 + dr * (i - 3)) * row_bytes;
#pragma unroll
          for (int a = 0; a < 9; ++a) st<T>(pb.rsrc(a), ox, pb.soff(a, ro), out[a]);
        }
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) fc2[a] = f2[a];
      rho_c2 = rho2;
    } else {
      __syncthreads();
    }
  }
}

}  // namespace lbm
