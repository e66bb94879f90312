// Device-side building blocks of the pseudo-potential MRT lattice Boltzmann
// step for gfx950: the equations of state, the pseudo-potential, and the
// per-cell force + pressure-tensor term + MRT collision.  Included by the
// step kernels (one lattice, and the batched persistent engine) so that both
// run the same arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_internal.h"

namespace lbm {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };

// Working-precision reciprocal and square root.  FP32 uses the hardware
// v_rcp_f32 / v_sqrt_f32 (1 ulp).  FP64 refines the hardware estimates by
// Newton-Raphson steps to within about one ulp, for the positive normal
// arguments the update produces: the reciprocal by r <- r + r (1 - x r),
// twice; the square root from y ~ 1/sqrt(x) by one coupled step on
// s ~ sqrt(x), h ~ y/2 and two corrections s <- s + h (x - s^2).
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  const double e = __builtin_fma(-s, h, 0.5);
  s = __builtin_fma(s, e, s);
  h = __builtin_fma(h, e, h);
  s = __builtin_fma(__builtin_fma(-s, s, x), h, s);
  s = __builtin_fma(__builtin_fma(-s, s, x), h, s);
  return x == 0.0 ? 0.0 : s;  // the estimate of 1/sqrt(0) is infinite
}

// Constants of one step in working precision T.  Derived combinations are
// formed on the host in FP64 and rounded once.
template <typename T>
struct DevC {
  T KRT;     // K R T
  T Ka;      // K a          (PR: K a alpha(T))
  T b;       // b            (CS: b/4)
  T b2;      // PR: b^2
  T twoOverG;
  T fU, fP;  // force: F = fU * g(U) + fP * psi * g(psi), g = 12 sum_a w_a phi(x+e_a) e_a
  T kP, kB;  // Q: Qxx = kP psi (S_psi/12 - psi) + kB (S_U/12 - U), etc.
  T s_e, s_eps, s_q, s_nu;
  T h_e, h_eps, h_q, h_nu;  // 1 - s/2
  T c_e;                    // 1.5 s_e   (first non-zero entry of C, Eq. 26)
  int var_nu;               // density-dependent shear viscosity
  T nu_g, dnu, rho_g, inv_drho;
};

template <typename T>
inline DevC<T> make_devc(const ModelConsts& m) {
  DevC<T> c;
  c.KRT = T(m.K * m.R * m.T);
  c.Ka = T(m.eos == LBM_EOS_PR ? m.K * m.aalpha : m.K * m.a);
  c.b = T(m.eos == LBM_EOS_CS ? m.b / 4.0 : m.b);
  c.b2 = T(m.b * m.b);
  c.twoOverG = T(2.0 / m.G);
  c.fU = T(-m.A / 12.0);
  c.fP = T(-(1.0 - m.A) * m.G / 12.0);
  c.kP = T(m.kappa * (1.0 - m.A) * m.G / 2.0);
  c.kB = T(m.kappa * m.A / 2.0);
  c.s_e = T(m.s_e);
  c.s_eps = T(m.s_eps);
  c.s_q = T(m.s_q);
  c.s_nu = T(m.s_nu);
  c.h_e = T(1.0 - 0.5 * m.s_e);
  c.h_eps = T(1.0 - 0.5 * m.s_eps);
  c.h_q = T(1.0 - 0.5 * m.s_q);
  c.h_nu = T(1.0 - 0.5 * m.s_nu);
  c.c_e = T(1.5 * m.s_e);
  c.var_nu = m.nu_gas > 0.0 ? 1 : 0;
  c.nu_g = T(m.nu_gas);
  c.dnu = T(m.nu_liquid - m.nu_gas);
  c.rho_g = T(m.rho_gas);
  c.inv_drho = T(m.nu_gas > 0.0 ? 1.0 / (m.rho_liquid - m.rho_gas) : 0.0);
  return c;
}

// U = K p_EOS(rho) - rho/3  (Eq. 10 with c = 1, c_s^2 = 1/3).
template <int EOS, typename T>
__device__ __forceinline__ T eos_U(T rho, const DevC<T>& c) {
  const T third = T(1) / T(3);
  if constexpr (EOS == LBM_EOS_CS) {
    // Carnahan-Starling, n = b rho / 4
    const T n = c.b * rho;
    const T om = T(1) - n;
    const T num = T(1) + n * (T(1) + n * (T(1) - n));
    const T den = om * om * om;
    return rho * (c.KRT * num * rcp_(den) - c.Ka * rho) - rho * third;
  } else if constexpr (EOS == LBM_EOS_VDW) {
    // Eq. (21)
    return rho * (c.KRT * rcp_(T(1) - c.b * rho) - c.Ka * rho) - rho * third;
  } else if constexpr (EOS == LBM_EOS_PR) {
    // Eq. (29); Ka already holds K a alpha(T)
    const T q = T(1) + rho * (T(2) * c.b - c.b2 * rho);
    return rho * (c.KRT * rcp_(T(1) - c.b * rho) - c.Ka * rho * rcp_(q)) - rho * third;
  } else {
    return T(0) * rho;  // ideal gas: no interaction
  }
}

// psi = sqrt(2U/G), set to 0 where U > 0 (G < 0).
template <typename T>
__device__ __forceinline__ T psi_of(T U, const DevC<T>& c) {
  const T s = c.twoOverG * U;
  return sqrt_(s > T(0) ? s : T(0));
}

// One cell: g[9] the distributions at x after streaming (time t), rho their
// sum, Un/Pn the values of U and psi at x + e_a (index a, a = 0 is x itself).
// Writes the post-collision distributions f*_a(x) to out[9].
template <typename T>
__device__ __forceinline__ void collide_cell(const T (&g)[9], T rho, const T (&Un)[9],
                                             const T (&Pn)[9], const DevC<T>& c, T (&out)[9]) {
  // ---- Kupershtokh force, Eq. (9): 12 sum_a w_a phi(x+e_a) e_a, w = 1/3, 1/12
  const T gUx = T(4) * (Un[1] - Un[3]) + ((Un[5] - Un[7]) + (Un[8] - Un[6]));
  const T gUy = T(4) * (Un[2] - Un[4]) + ((Un[5] - Un[7]) + (Un[6] - Un[8]));
  const T gPx = T(4) * (Pn[1] - Pn[3]) + ((Pn[5] - Pn[7]) + (Pn[8] - Pn[6]));
  const T gPy = T(4) * (Pn[2] - Pn[4]) + ((Pn[5] - Pn[7]) + (Pn[6] - Pn[8]));
  const T psic = Pn[0], Uc = Un[0];
  const T fpp = c.fP * psic;
  const T Fx = c.fU * gUx + fpp * gPx;
  const T Fy = c.fU * gUy + fpp * gPy;

  // ---- pressure-tensor modification, Eq. (23) with the factor G/2
  const T t12 = T(1) / T(12);
  const T dP = (Pn[5] + Pn[7]) + (Pn[6] + Pn[8]);
  const T dU = (Un[5] + Un[7]) + (Un[6] + Un[8]);
  const T ka = c.kP * psic;
  const T Qxx = ka * ((T(4) * (Pn[1] + Pn[3]) + dP) * t12 - psic) +
                c.kB * ((T(4) * (Un[1] + Un[3]) + dU) * t12 - Uc);
  const T Qyy = ka * ((T(4) * (Pn[2] + Pn[4]) + dP) * t12 - psic) +
                c.kB * ((T(4) * (Un[2] + Un[4]) + dU) * t12 - Uc);
  const T Qxy = (ka * ((Pn[5] + Pn[7]) - (Pn[6] + Pn[8])) +
                 c.kB * ((Un[5] + Un[7]) - (Un[6] + Un[8]))) * t12;

  // ---- moments m = M f, order (rho, e, eps, jx, qx, jy, qy, pxx, pxy)
  const T a13 = g[1] + g[3], a24 = g[2] + g[4];
  const T d13 = g[1] - g[3], d24 = g[2] - g[4];
  const T sd = (g[5] + g[7]) + (g[6] + g[8]);
  const T dx = (g[5] - g[7]) + (g[8] - g[6]);
  const T dy = (g[5] - g[7]) + (g[6] - g[8]);
  const T s14 = a13 + a24;
  const T e = T(2) * sd - s14 - T(4) * g[0];
  const T eps = T(4) * g[0] - T(2) * s14 + sd;
  const T jx = d13 + dx, jy = d24 + dy;
  const T qx = dx - T(2) * d13, qy = dy - T(2) * d24;
  const T pxx = a13 - a24;
  const T pxy = (g[5] + g[7]) - (g[6] + g[8]);

  // ---- shear rate: constant, or from the density-dependent viscosity
  T s_nu = c.s_nu, h_nu = c.h_nu;
  if (c.var_nu) {
    T fr = (rho - c.rho_g) * c.inv_drho;
    fr = fr < T(0) ? T(0) : (fr > T(1) ? T(1) : fr);
    s_nu = rcp_(T(3) * (c.nu_g + fr * c.dnu) + T(0.5));
    h_nu = T(1) - T(0.5) * s_nu;
  }

  // ---- velocity v = (j + F/2)/rho and the collision of Eq. (25)
  const T mx = jx + T(0.5) * Fx, my = jy + T(0.5) * Fy;  // rho v
  const T ir = rcp_(rho);
  const T vx = mx * ir, vy = my * ir;
  const T v2 = vx * vx + vy * vy;
  const T vF = vx * Fx + vy * Fy;
  const T es = e - c.s_e * (e - rho * (T(3) * v2 - T(2))) + c.h_e * (T(6) * vF) + c.c_e * (Qxx + Qyy);
  const T epss = eps - c.s_eps * (eps - rho * (T(1) - T(3) * v2)) - c.h_eps * (T(6) * vF);
  const T jxs = jx + Fx, jys = jy + Fy;
  const T qxs = qx - c.s_q * (qx + mx) - c.h_q * Fx;
  const T qys = qy - c.s_q * (qy + my) - c.h_q * Fy;
  const T pxxs = pxx - s_nu * (pxx - (mx * vx - my * vy)) +
                 h_nu * (T(2) * (vx * Fx - vy * Fy)) - s_nu * (Qxx - Qyy);
  const T pxys = pxy - s_nu * (pxy - mx * vy) + h_nu * (vx * Fy + vy * Fx) - s_nu * Qxy;

  // ---- f* = M^{-1} m*, M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
  const T r9 = rho * (T(1) / T(9));
  const T a0 = r9 - es * (T(1) / T(36)) - epss * (T(1) / T(18));
  const T b0 = r9 + es * (T(1) / T(18)) + epss * (T(1) / T(36));
  const T Xa = (jxs - qxs) * (T(1) / T(6));
  const T Ya = (jys - qys) * (T(1) / T(6));
  const T Xd = jxs * (T(1) / T(6)) + qxs * t12;
  const T Yd = jys * (T(1) / T(6)) + qys * t12;
  const T Pq = pxxs * T(0.25), Rq = pxys * T(0.25);
  out[1] = a0 + Xa + Pq;
  out[2] = a0 + Ya - Pq;
  out[3] = a0 - Xa + Pq;
  out[4] = a0 - Ya - Pq;
  out[5] = b0 + (Xd + Yd) + Rq;
  out[6] = b0 + (Yd - Xd) - Rq;
  out[7] = b0 - (Xd + Yd) + Rq;
  out[8] = b0 + (Xd - Yd) - Rq;
  // f*_0 from the mass balance of the cell, so that neither the rounded
  // constants of M^{-1} nor the rounding of sums of nearly equal populations
  // create or destroy mass.  FP32 writes it as f*_0 = g_0 + sum_a (g_a - f*_a):
  // the changes g_a - f*_a are small next to the populations (exact where they
  // are within a factor 2 of each other), so the nine stored values sum to the
  // arriving density up to about one rounding of f*_0, without bias (a plain
  // FP32 rho - sum f*_a drifts by ~1e-9 of the mass per step).
  if constexpr (sizeof(T) == 4) {
    const T d1 = g[1] - out[1], d2 = g[2] - out[2], d3 = g[3] - out[3], d4 = g[4] - out[4];
    const T d5 = g[5] - out[5], d6 = g[6] - out[6], d7 = g[7] - out[7], d8 = g[8] - out[8];
    out[0] = g[0] + (((d1 + d3) + (d2 + d4)) + ((d5 + d7) + (d6 + d8)));
  } else {
    out[0] = rho - (((out[1] + out[2]) + (out[3] + out[4])) + ((out[5] + out[6]) + (out[7] + out[8])));
  }
}

// Workgroup -> tile order: the hardware deals workgroups round-robin over the
// 8 XCDs; renumber so that each XCD receives a contiguous run of tiles
// (neighbouring row blocks of a strip share their halo rows in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int full = n & ~7;
  if (b >= full) return b;
  const int per = full >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int wrap_(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// The buffers hold the post-collision distributions of the previous step,
// not yet streamed (the step kernel streams by pulling).  The distribution
// f_a(x, y) of the current state therefore sits at (x - e_a, y - e_a) of
// plane a.  Element index of f_a(x, y) (rows interleaved, plane a's part of
// lattice row y starting at y * row + a * pitch):
__device__ __forceinline__ long long state_index(const Geometry& g, int a, int x, int y) {
  const int ex = (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0);
  const int ey = (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0);
  return (long long)wrap_(y - ey, g.ny) * g.row + (long long)a * g.pitch + wrap_(x - ex, g.nx);
}

}  // namespace lbm
