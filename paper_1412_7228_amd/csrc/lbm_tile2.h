// Two fused time steps of one tile (temporal blocking), for the single-lattice
// kernel and the batched engine.  A pass reads the state once and writes it
// once for two steps, so it moves half the HBM bytes of two single-step
// passes at about twice the arithmetic per pass; the per-cell arithmetic is
// step_tile's, operation for operation, so both paths give bitwise the same
// states.
//
// A workgroup of BX lanes covers the BX consecutive columns u = xs - 3 + lane
// (periodic wrap in x) and marches along the rows of its row block.  Per row
// the pipeline runs four stages, each closed by a barrier:
//
//   A  gather f (pulled) of row r, form rho, U, psi        -> LDS ring 1
//   B  collide row r - 1 of the first step                  -> LDS ring F
//   C  pull the second step's f of row r - 2 out of ring F,
//      form rho, U, psi                                     -> LDS ring 2
//   D  collide row r - 3 of the second step                 -> HBM
//
// (rows counted along the march direction).  Stage B is valid on lanes
// 1..BX-2, C on 2..BX-3 and D on 3..BX-4, so a strip stores BX - 6 columns;
// the first step runs on 4 extra rows and the second on 2 extra rows at the
// ends of the row block.  Rings 1 and 2 hold 3 rows of (U, psi).  Ring F keeps
// each post-collision plane only as long as the second step needs it: the
// three planes pulled from the row ahead (in the march direction) live one
// iteration, the three pulled from the same row two, the three pulled from
// the row behind three.  Lanes outside a stage's valid range compute on
// whatever their neighbours hold (nothing of theirs is stored or read by a
// valid lane), so control flow stays uniform.
//
// With SKIP, a wave none of whose lanes is needed (a strip narrower than the
// workgroup, as narrow lattices and the last strip of a wide one are: W
// stored columns need the first W + 6 lanes) runs only the barriers, as many
// as the others pass (three per row), and nothing else.  The decision is
// wave-uniform and taken once, so the stages of the busy waves stay one
// straight-line block each.  It pays where a workgroup's freed issue slots go
// to other work at once (the persistent batch kernel); in per-step launches
// the idle waves computing their wrapped duplicate columns measure faster.
//
// AHEAD is how many rows ahead of the first step's row the gathers run: 1, or
// 2 with a third register set (nine more VGPRs, so four waves per SIMD in
// FP32 instead of five).  The second hides more of the loads' latency, the
// first keeps more waves; each kernel takes the one that measures faster for
// it (the launches state which).
#pragma once

#include "lbm_tile.h"

namespace lbm {

template <typename T, int BX>
struct Tile2Lds {
  typename V2<T>::t ring1[3][BX + 2];
  typename V2<T>::t ring2[3][BX + 2];
  T Fa[1][3][BX + 2];  // planes pulled from the row ahead
  T Fs[2][3][BX + 2];  // planes 0, 1, 3 (same row)
  T Fb[3][3][BX + 2];  // planes pulled from the row behind
};

// Columns one pass stores per strip.
template <int BX>
constexpr int tile2_width() { return BX - 6; }

template <typename T, int EOS, int BX, bool BIG, bool DOWN, bool SKIP = false, int AHEAD = 1>
__device__ __forceinline__ void step2_tile(const T* __restrict__ fa, T* __restrict__ fb,
                                           const Geometry& geo, const DevC<T>& c, int xs, int y0,
                                           Tile2Lds<T, BX>& L) {
  using T2 = typename V2<T>::t;
  const int nx = geo.nx, ny = geo.ny;
  const int H = min(geo.tile_y, geo.y_end - y0);  // rows past y_end belong to no tile
  const int tx = threadIdx.x;
  const int u = xs - 3 + tx;            // this lane's column before the periodic wrap (>= -3)
  const int x = (u + nx) % nx;          // nx >= 3
  const unsigned sz = sizeof(T);
  const unsigned ox = x * sz;
  const unsigned oxm = ((x == 0) ? nx - 1 : x - 1) * sz;
  const unsigned oxp = ((x == nx - 1) ? 0 : x + 1) * sz;
  const bool store = tx >= 3 && tx < BX - 3 && u < min(xs + tile2_width<BX>(), nx);

  Planes<BIG> pa, pb;
  const unsigned long long total = (unsigned long long)geo.ny * geo.row * sz;
  pa.init(fa, geo.pitch * sz, (unsigned)(geo.row * sz), total);
  pb.init(fb, geo.pitch * sz, (unsigned)(geo.row * sz), total);

  constexpr int dr = DOWN ? -1 : 1;
  const int r0 = DOWN ? y0 + H + 2 : y0 - 3;
  const int n = H + 6;
  // Planes pulled from the row ahead in the march direction (lattice y + dr):
  // those with e_y = -dr; from the row behind: e_y = +dr.  Column shifts are
  // -e_x: planes 2 and 4 none, 5 and 8 from x - 1, 6 and 7 from x + 1.
  constexpr int AH0 = DOWN ? 2 : 4, AH1 = DOWN ? 5 : 8, AH2 = DOWN ? 6 : 7;  // shifts 0, -1, +1
  constexpr int BH0 = DOWN ? 4 : 2, BH1 = DOWN ? 8 : 5, BH2 = DOWN ? 7 : 6;  // shifts 0, -1, +1

  // rows y0 - 4 .. y0 + H + 3 are gathered: more than one period away from the
  // lattice when ny < 4, so the wrap is a full modulo (uniform, scalar ALU)
  auto wrap_row = [&](int v) {
    const int m = v % ny;
    return m < 0 ? m + ny : m;
  };
  auto gather_row = [&](int r, T(&g)[9]) {
    gather(pa, wrap_row(r), wrap_row(r - 1), wrap_row(r + 1), ox, oxm, oxp, g);
  };
  // stencil of the centre row (slot s_mid) from the rows before (s_old) and
  // after (s_new) it in the march direction
  auto load_stencil = [&](const T2 (*ring)[BX + 2], int s_new, int s_mid, int s_old, T(&Un)[9],
                          T(&Pn)[9]) {
    const int sn = DOWN ? s_old : s_new;  // lattice y + 1
    const int ss = DOWN ? s_new : s_old;  // lattice y - 1
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

  // Register sets rotate between two roles per iteration (the loop body is
  // written twice with the roles swapped), so no populations are copied:
  // stage 1 uses P / Q as the current and the previous row (after B has
  // collided the previous row, the next row is gathered into its registers),
  // stage 2 uses R / S as the row just pulled out of ring F and the row it
  // collides.
  T P[9], Q[9], R[9], S[9];
  T rP = T(0), rQ = T(0), rR = T(0), rS = T(0);
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    Q[a] = T(0);
    R[a] = T(0);
    S[a] = T(0);
  }
  if constexpr (SKIP) {
    const int W = min(tile2_width<BX>(), nx - xs);  // stored columns of this strip
    if ((__builtin_amdgcn_readfirstlane(tx) & ~63) >= W + 6) {  // wave-uniform
#pragma unroll 1
      for (int i = 0; i < n; ++i) {
        __syncthreads();
        __syncthreads();
        __syncthreads();
      }
      return;
    }
  }
  gather_row(r0, P);
  const int l = tx + 1;

  auto iteration = [&](int i, T(&cur)[9], T& rcur, T(&prev)[9], T& rprev, T(&f2)[9], T& r2,
                       T(&fc2)[9], T& rc2) {
    // ---- A: first-step density of row r = r0 + dr i
    rcur = density(cur);
    {
      const T U = eos_U<EOS>(rcur, c);
      L.ring1[i % 3][l] = T2{U, psi_of(U, c)};
    }
    __syncthreads();
    // ---- B: first-step collision of row r - dr (written "in iteration i")
    if (i >= 2) {
      T Un[9], Pn[9], out[9];
      load_stencil(L.ring1, i % 3, (i - 1) % 3, (i - 2) % 3, Un, Pn);
      collide_cell(prev, rprev, Un, Pn, c, out);
      const int sb = (i - 1) % 3, ss = (i - 1) & 1;
      L.Fa[0][0][l] = out[AH0];
      L.Fa[0][1][l] = out[AH1];
      L.Fa[0][2][l] = out[AH2];
      L.Fs[ss][0][l] = out[0];
      L.Fs[ss][1][l] = out[1];
      L.Fs[ss][2][l] = out[3];
      L.Fb[sb][0][l] = out[BH0];
      L.Fb[sb][1][l] = out[BH1];
      L.Fb[sb][2][l] = out[BH2];
    }
    // the previous row is done: its registers take the next row
    if (i + AHEAD < n) gather_row(r0 + dr * (i + AHEAD), prev);
    __syncthreads();
    // ---- C: second-step density of row q = r - 2 dr: f_a(x, q) = f*_a(x - e_ax, q - e_ay).
    // Row q + dr was written in iteration i (Fa), q in i - 1 (Fs slot i & 1),
    // q - dr in i - 2 (Fb slot i % 3).
    if (i >= 4) {
      const int ss = i & 1, sb = i % 3;
      f2[AH0] = L.Fa[0][0][l];
      f2[AH1] = L.Fa[0][1][l - 1];
      f2[AH2] = L.Fa[0][2][l + 1];
      f2[0] = L.Fs[ss][0][l];
      f2[1] = L.Fs[ss][1][l - 1];      // e = ( 1, 0)
      f2[3] = L.Fs[ss][2][l + 1];      // e = (-1, 0)
      f2[BH0] = L.Fb[sb][0][l];
      f2[BH1] = L.Fb[sb][1][l - 1];
      f2[BH2] = L.Fb[sb][2][l + 1];
      r2 = density(f2);
      const T U = eos_U<EOS>(r2, c);
      L.ring2[i % 3][l] = T2{U, psi_of(U, c)};
    }
    __syncthreads();
    // ---- D: second-step collision of row q - dr -> HBM
    if (i >= 6) {
      T Un[9], Pn[9], out[9];
      load_stencil(L.ring2, i % 3, (i - 1) % 3, (i - 2) % 3, Un, Pn);
      collide_cell(fc2, rc2, Un, Pn, c, out);
      if (store) store_row(pb, r0 + dr * (i - 3), ox, out);
    }
  };

  static_assert(AHEAD == 1 || AHEAD == 2, "rows gathered ahead: 1 or 2");
  if constexpr (AHEAD == 1) {
#pragma unroll 1
    for (int i = 0; i < n; i += 2) {
      iteration(i, P, rP, Q, rQ, R, rR, S, rS);
      if (i + 1 < n) iteration(i + 1, Q, rQ, P, rP, S, rS, R, rR);
    }
  } else {
    // a third register set for the first step's rows: three roles rotate
    // (current, previous, two ahead) against the second step's two, so the
    // loop body is written six times
    T X[9];
    T rX = T(0);
#pragma unroll
    for (int a = 0; a < 9; ++a) X[a] = T(0);
    gather_row(r0 + dr, Q);  // row 1 (row 0 is in P; n >= 7)
#pragma unroll 1
    for (int i = 0; i < n; i += 6) {
      iteration(i, P, rP, X, rX, R, rR, S, rS);
      if (i + 1 < n) iteration(i + 1, Q, rQ, P, rP, S, rS, R, rR);
      if (i + 2 < n) iteration(i + 2, X, rX, Q, rQ, R, rR, S, rS);
      if (i + 3 < n) iteration(i + 3, P, rP, X, rX, S, rS, R, rR);
      if (i + 4 < n) iteration(i + 4, Q, rQ, P, rP, R, rR, S, rS);
      if (i + 5 < n) iteration(i + 5, X, rX, Q, rQ, S, rS, R, rR);
    }
  }
}

}  // namespace lbm
