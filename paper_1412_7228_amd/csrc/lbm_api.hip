// Host side of liblbm: the C ABI declared in include/lbm.h.
//
// Owns parameter validation, the critical temperature of each EOS, the
// device buffers, the launch shape and the FP64 observables.  Every device
// operation is enqueued on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_internal.h"

using namespace lbm;

namespace {

thread_local std::string g_last_error;

lbm_status fail(lbm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lbm_status fail(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s: %s (%s:%d)",    \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                         \
  } while (0)

constexpr uint64_t kStateMagic = 0x4c424d5053543032ull;  // "LBMPST02": rows interleaved

struct StateHeader {
  uint64_t magic;
  int32_t nx, ny, pitch, precision;
  int64_t step;
  uint64_t params_hash;
  uint64_t payload_bytes;
};

// ---------------------------------------------------------------------------
// Equations of state on the host (FP64), for the critical point and the
// Laplace pressures.  Same definitions as the device code.
// ---------------------------------------------------------------------------
double eos_pressure(int eos, double a_alpha, double b, double R, double K, double T, double a,
                    double rho) {
  switch (eos) {
    case LBM_EOS_CS: {
      const double n = b * rho / 4.0, om = 1.0 - n;
      return K * (rho * R * T * (1.0 + n + n * n - n * n * n) / (om * om * om) - a * rho * rho);
    }
    case LBM_EOS_VDW:
      return K * (rho * R * T / (1.0 - b * rho) - a * rho * rho);
    case LBM_EOS_PR:
      return K * (rho * R * T / (1.0 - b * rho) -
                  a_alpha * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho));
    default:
      return rho / 3.0;
  }
}

double pr_alpha(double omega, double T_over_Tc) {
  const double k = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
  const double s = 1.0 + k * (1.0 - std::sqrt(T_over_Tc));
  return s * s;
}

// dp/drho of the K = 1 pressure at temperature T, written out for each EOS
// (Peng-Robinson with alpha = 1: at the critical point alpha(Tc) = 1).
double eos_slope(int eos, double a, double b, double R, double T, double rho) {
  switch (eos) {
    case LBM_EOS_CS: {
      const double n = b * rho / 4.0, om = 1.0 - n;
      const double h1 = (1.0 + 4.0 * n + 4.0 * n * n - 4.0 * n * n * n + n * n * n * n) / (om * om * om * om);
      return R * T * h1 - 2.0 * a * rho;
    }
    case LBM_EOS_VDW: {
      const double d = 1.0 - b * rho;
      return R * T / (d * d) - 2.0 * a * rho;
    }
    case LBM_EOS_PR: {
      const double d = 1.0 - b * rho;
      const double q = 1.0 + 2.0 * b * rho - b * b * rho * rho;
      const double q1 = 2.0 * b - 2.0 * b * b * rho;
      return R * T / (d * d) - a * (2.0 * rho * q - rho * rho * q1) / (q * q);
    }
    default:
      return 1.0 / 3.0;
  }
}

double max_density(int eos, double b) { return eos == LBM_EOS_CS ? 4.0 / b : 1.0 / b; }

// Smallest dp/drho over (0, rho_max) at temperature T (golden-section
// search; dp/drho falls from R T at rho -> 0 into the van der Waals loop and
// rises again towards the excluded-volume limit).
double min_slope(int eos, double a, double b, double R, double T, double* at) {
  double lo = 1e-6 * max_density(eos, b), hi = 0.9 * max_density(eos, b);
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
  double fc = eos_slope(eos, a, b, R, T, c), fd = eos_slope(eos, a, b, R, T, d);
  for (int it = 0; it < 200 && (hi - lo) > 1e-14 * hi; ++it) {
    if (fc < fd) {
      hi = d; d = c; fd = fc; c = hi - gr * (hi - lo); fc = eos_slope(eos, a, b, R, T, c);
    } else {
      lo = c; c = d; fc = fd; d = lo + gr * (hi - lo); fd = eos_slope(eos, a, b, R, T, d);
    }
  }
  if (at) *at = 0.5 * (lo + hi);
  return std::min(fc, fd);
}

// Critical temperature: the T at which the smallest dp/drho is zero (the
// critical isotherm's inflection point with zero slope).  vdW has the closed form 8a/(27bR).
lbm_status critical_temperature(const lbm_params& p, double* Tc) {
  if (p.eos == LBM_EOS_VDW) {
    *Tc = 8.0 * p.a / (27.0 * p.b * p.R);
    return LBM_OK;
  }
  if (p.eos != LBM_EOS_CS && p.eos != LBM_EOS_PR)
    return fail(LBM_EINVAL, "critical temperature: EOS %d has none", p.eos);
  double lo = 1e-4 * p.a / (p.b * p.R), hi = 2.0 * p.a / (p.b * p.R);
  if (min_slope(p.eos, p.a, p.b, p.R, lo, nullptr) >= 0.0 ||
      min_slope(p.eos, p.a, p.b, p.R, hi, nullptr) <= 0.0)
    return fail(LBM_EINVAL, "critical temperature: no sign change of dp/drho");
  for (int it = 0; it < 200 && (hi - lo) > 4e-16 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (min_slope(p.eos, p.a, p.b, p.R, mid, nullptr) < 0.0) lo = mid; else hi = mid;
  }
  *Tc = 0.5 * (lo + hi);
  return LBM_OK;
}

// Maxwell construction at T: coexisting (rho_v, rho_l) with equal pressure
// and equal area  int_{rho_v}^{rho_l} (p - P)/rho^2 drho = 0.
double eos_p1(const lbm_params& p, double aalpha, double T, double rho) {
  return eos_pressure(p.eos, aalpha, p.b, p.R, 1.0, T, p.a, rho);
}

double eos_dp1(const lbm_params& p, double aalpha, double T, double rho) {
  // slope at temperature T (PR with alpha(T) through a -> a alpha)
  return eos_slope(p.eos, p.eos == LBM_EOS_PR ? aalpha : p.a, p.b, p.R, T, rho);
}

template <typename F>
double bisect(F f, double lo, double hi, int iters = 200) {
  double flo = f(lo);
  for (int it = 0; it < iters && hi - lo > 1e-16 * std::fabs(hi); ++it) {
    const double mid = 0.5 * (lo + hi);
    const double fm = f(mid);
    if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
  }
  return 0.5 * (lo + hi);
}

// Gauss-Legendre with 16 points on each of n equal panels of [a, b].
template <typename F>
double integrate(F f, double a, double b, int n = 64) {
  static const double xg[8] = {0.0950125098376374, 0.2816035507792589, 0.4580167776572274,
                               0.6178762444026438, 0.7554044083550030, 0.8656312023878318,
                               0.9445750230732326, 0.9894009349916499};
  static const double wg[8] = {0.1894506104550685, 0.1826034150449236, 0.1691565193950025,
                               0.1495959888165767, 0.1246289712555339, 0.0951585116824928,
                               0.0622535239386479, 0.0271524594117541};
  double s = 0.0;
  const double h = (b - a) / n;
  for (int k = 0; k < n; ++k) {
    const double c = a + (k + 0.5) * h, r = 0.5 * h;
    for (int i = 0; i < 8; ++i) s += wg[i] * r * (f(c - r * xg[i]) + f(c + r * xg[i]));
  }
  return s;
}

lbm_status coexistence(const lbm_params& p, double* rv, double* rl) {
  double Tc = 0.0;
  lbm_status st = critical_temperature(p, &Tc);
  if (st != LBM_OK) return st;
  if (!(p.T_over_Tc > 0.0 && p.T_over_Tc < 1.0))
    return fail(LBM_EINVAL, "coexistence needs 0 < T/Tc < 1 (got %g)", p.T_over_Tc);
  const double T = p.T_over_Tc * Tc;
  const double aalpha = p.eos == LBM_EOS_PR ? p.a * pr_alpha(p.omega_pr, p.T_over_Tc) : p.a;
  // spinodal densities around the minimum of dp/drho
  double rmin = 0.0;
  {
    double lo = 1e-6 * max_density(p.eos, p.b), hi = 0.9 * max_density(p.eos, p.b);
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
    double fc = eos_dp1(p, aalpha, T, c), fd = eos_dp1(p, aalpha, T, d);
    for (int it = 0; it < 200 && (hi - lo) > 1e-14 * hi; ++it) {
      if (fc < fd) { hi = d; d = c; fd = fc; c = hi - gr * (hi - lo); fc = eos_dp1(p, aalpha, T, c); }
      else { lo = c; c = d; fc = fd; d = lo + gr * (hi - lo); fd = eos_dp1(p, aalpha, T, d); }
    }
    rmin = 0.5 * (lo + hi);
    if (!(eos_dp1(p, aalpha, T, rmin) < 0.0)) return fail(LBM_EINVAL, "no two-phase region at T/Tc = %g", p.T_over_Tc);
  }
  const double top = 0.999 * max_density(p.eos, p.b);
  auto slope = [&](double r) { return eos_dp1(p, aalpha, T, r); };
  const double s_lo = bisect(slope, 1e-9 * top, rmin);
  const double s_hi = bisect(slope, rmin, top);
  const double p_max = eos_p1(p, aalpha, T, s_lo), p_min = std::max(eos_p1(p, aalpha, T, s_hi), 0.0);
  auto branches = [&](double P, double* v, double* l) {
    // the vapour branch starts below the ideal-gas density P/(R T)
    *v = bisect([&](double r) { return eos_p1(p, aalpha, T, r) - P; }, 1e-3 * P / (p.R * T), s_lo);
    *l = bisect([&](double r) { return eos_p1(p, aalpha, T, r) - P; }, s_hi, top);
  };
  // in s = ln(rho): int (p - P)/rho^2 drho = int (p - P)/rho ds, smooth near a dilute vapour
  auto area = [&](double P) {
    double v, l;
    branches(P, &v, &l);
    return integrate([&](double sv) {
      const double r = std::exp(sv);
      return (eos_p1(p, aalpha, T, r) - P) / r;
    }, std::log(v), std::log(l), 256);
  };
  // the area falls as P rises; bracket [p_min, p_max]
  const double plo = p_min > 0.0 ? p_min * (1.0 + 1e-12) : 1e-12 * p_max, phi = p_max * (1.0 - 1e-12);
  if (!(area(plo) > 0.0 && area(phi) < 0.0)) return fail(LBM_EINVAL, "Maxwell construction: no bracket");
  const double Ps = bisect(area, plo, phi, 120);
  branches(Ps, rv, rl);
  return LBM_OK;
}

lbm_status model_of(const lbm_params& p, ModelConsts* m) {
  m->eos = p.eos;
  m->K = p.K; m->R = p.R; m->a = p.a; m->b = p.b;
  m->G = p.eos == LBM_EOS_IDEAL ? -1.0 : p.G;
  m->A = p.A; m->kappa = p.kappa;
  m->s_e = p.s_e; m->s_eps = p.s_eps; m->s_q = p.s_q; m->s_nu = p.s_nu;
  m->nu_gas = p.nu_gas; m->nu_liquid = p.nu_liquid; m->rho_gas = p.rho_gas; m->rho_liquid = p.rho_liquid;
  m->T = 0.0;
  m->aalpha = p.a;
  if (p.eos != LBM_EOS_IDEAL) {
    double Tc = 0.0;
    lbm_status st = critical_temperature(p, &Tc);
    if (st != LBM_OK) return st;
    m->T = p.T_over_Tc * Tc;
    if (p.eos == LBM_EOS_PR) m->aalpha = p.a * pr_alpha(p.omega_pr, p.T_over_Tc);
  }
  return LBM_OK;
}

lbm_status validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 3 || p->ny < 3) return fail(LBM_EINVAL, "lattice %d x %d: each side must be >= 3", p->nx, p->ny);
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
    return fail(LBM_EINVAL, "unknown precision %d", p->precision);
  // one distribution plane's worth (ny * pitch elements) must stay below
  // 4 GiB: it bounds the cell count for the 32-bit cell indices of the
  // kernels; and one lattice row of the nine planes (9 * pitch elements) must
  // too: the kernels address a row with 32-bit offsets
  const unsigned es = p->precision == LBM_FP32 ? 4u : 8u;
  const unsigned long long pitch = (unsigned long long)(p->nx + 63) / 64 * 64;
  const unsigned long long plane_bytes = (unsigned long long)p->ny * pitch * es;
  if (plane_bytes >= (1ull << 32))
    return fail(LBM_EINVAL, "lattice %d x %d too large: one plane is %llu bytes (limit 4 GiB)",
                p->nx, p->ny, plane_bytes);
  if (9ull * pitch * es >= (1ull << 32))
    return fail(LBM_EINVAL, "lattice %d x %d too wide: one row of the nine planes is %llu bytes (limit 4 GiB)",
                p->nx, p->ny, 9ull * pitch * es);
  if (p->eos < LBM_EOS_IDEAL || p->eos > LBM_EOS_PR) return fail(LBM_EINVAL, "unknown EOS %d", p->eos);
  const double rates[4] = {p->s_e, p->s_eps, p->s_q, p->s_nu};
  for (double s : rates)
    if (!(s > 0.0 && s < 2.0)) return fail(LBM_EINVAL, "relaxation rate %g outside (0, 2)", s);
  if (!std::isfinite(p->A) || !std::isfinite(p->kappa)) return fail(LBM_EINVAL, "A or kappa not finite");
  if (p->nu_gas != 0.0) {
    if (!(p->nu_gas > 0.0 && p->nu_liquid > 0.0 && p->rho_liquid > p->rho_gas && p->rho_gas >= 0.0))
      return fail(LBM_EINVAL, "variable viscosity needs nu_gas, nu_liquid > 0 and rho_liquid > rho_gas >= 0");
  }
  if (p->eos != LBM_EOS_IDEAL) {
    if (!(p->G < 0.0)) return fail(LBM_EINVAL, "G must be negative (got %g)", p->G);
    if (!(p->a > 0.0 && p->b > 0.0 && p->R > 0.0 && p->K > 0.0))
      return fail(LBM_EINVAL, "EOS constants a, b, R, K must be positive");
    if (!(p->T_over_Tc > 0.0)) return fail(LBM_EINVAL, "T/Tc must be positive");
  }
  return LBM_OK;
}

uint64_t params_hash(const lbm_params& p) {
  // FNV-1a over the parameter bytes
  const unsigned char* b = reinterpret_cast<const unsigned char*>(&p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < sizeof p; ++i) h = (h ^ b[i]) * 1099511628211ull;
  return h;
}

int pitch_of(const lbm_params& p) { return (p.nx + 63) / 64 * 64; }

// Elements of one distribution buffer: ny lattice rows, each the nine planes'
// rows of pitch elements back to back (lbm.h).
size_t state_elems(const lbm_params& p) { return (size_t)p.ny * 9 * pitch_of(p); }

size_t elem_size(const lbm_params& p) { return p.precision == LBM_FP32 ? 4 : 8; }

}  // namespace

struct lbm_ctx {
  lbm_params p;
  ModelConsts m;
  Geometry g;   // single-step kernel (and the lattice's layout for read-out)
  Geometry g2;  // two-step kernel
  int fuse;     // steps per pass: 1 or 2
  size_t buf_bytes;
  void* buf[2];
  bool own_buf;
  int cur;
  hipStream_t stream;
  bool own_stream;
  int64_t step;
  bool initialized;
  int pending;  // steps of a row-range launch whose destination is not yet current (0: none)
  // graphs of runs of two-step launches (captured on cap_stream, launched on stream)
  hipStream_t cap_stream;
  struct GraphEntry {
    hipGraphExec_t exec;
    int launches, parity, version;
  } graphs[4];
  int ngraphs, version;  // version: bumped whenever the launch geometry changes
  // FP64 scratch for fields and observables (allocated on first use)
  double* work;      // 4 * nx*ny: rho, U, psi, out
  double* partials;  // obs_partials_count * kNumRed
  double* red;       // kNumRed + 2
};

namespace {

// Tiles of a launch: strips of `width` stored columns (tile_x for one step per
// pass, tile_x - 6 for two) and row blocks of tile_y rows.
Geometry make_geometry(const lbm_params& p, int tile_x, int tile_y, int width) {
  Geometry g{};
  g.nx = p.nx;
  g.ny = p.ny;
  g.pitch = pitch_of(p);
  g.row = 9ll * g.pitch;
  g.tile_x = tile_x;
  g.tile_y = tile_y;
  g.nstrips = (g.nx + width - 1) / width;
  g.nrowblocks = (g.ny + tile_y - 1) / tile_y;
  g.nblocks = g.nstrips * g.nrowblocks;
  g.y_begin = 0;
  g.y_end = g.ny;
  return g;
}

void set_geometry(lbm_ctx* c, int tile_x, int tile_y) {
  c->g = make_geometry(c->p, tile_x, tile_y, tile_x);
}

void set_geometry2(lbm_ctx* c, int tile_x, int tile_y) {
  c->g2 = make_geometry(c->p, tile_x, tile_y, tile_x - kStep2Halo);
}

// Default launch shape: strips as wide as the lattice allows (up to 256
// columns); rows per workgroup a power of two from 64 down to 8, the largest
// that still gives at least 4 workgroups per CU.  (Measured on the 4096^2
// lattice: 64 and 16 rows are equally fast; grids that are not a multiple of
// the CU count leave some CUs a block more than others.)
void default_launch(const lbm_params& p, int* tx, int* ty) {
  *tx = p.nx >= 256 ? 256 : (p.nx >= 128 ? 128 : 64);
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const long long strips = (p.nx + *tx - 1) / *tx;
  int rows = 64;
  while (rows > 8 && strips * ((p.ny + rows - 1) / rows) < 4ll * cus) rows /= 2;
  *ty = std::min(rows, p.ny);
}

// Default shape of the two-step launch: 256-lane strips (250 stored columns)
// with 16 rows (FP32) or 24 rows (FP64) per workgroup, fewer (down to 8) while
// that leaves under 4 workgroups per CU.  A lattice too small to give 256-lane
// strips 8 workgroups per CU even then (a slab of a larger lattice, 2048^2 and
// below) takes 128-lane strips, rows down to 8 for 8 workgroups per CU: more,
// smaller workgroups finish the grid sooner there (measured, alternating the
// two shapes: 4096 x 520, 128 x 8 is 3% faster than 256 x 8; 2048^2 and
// 4096 x 1024, 128 x 16 is 1.5% faster than 256 x 16; 1024^2, 128 x 8 is 6%
// faster).  On 4096^2 the 256-lane FP32 shapes of 12 to 28 rows are within 1.5%
// of each other (16 rows fastest).  FP64 lattices at least 250 columns wide take
// the whole-wave rule below instead.
void default_launch2(const lbm_params& p, int* tx, int* ty) {
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const int start = p.precision == LBM_FP32 ? 16 : 24;
  auto blocks = [&](int w, int rows) {
    return (long long)((p.nx + w - kStep2Halo - 1) / (w - kStep2Halo)) * ((p.ny + rows - 1) / rows);
  };
  auto rows_for = [&](int w, long long target) {
    int rows = start;
    while (rows > 8 && blocks(w, rows) < target) rows -= 4;
    return rows;
  };
  int w = 128, rows = 0;
  if (p.nx >= 250) {
    rows = rows_for(256, 4ll * cus);
    if (blocks(256, rows) >= 8ll * cus) w = 256;
  }
  if (w == 128) rows = rows_for(128, p.nx >= 250 ? 8ll * cus : 4ll * cus);
  if (p.precision == LBM_FP64 && p.nx >= 250) {
    // FP64: two 256-lane workgroups fit on a CU (62 KB of LDS each), so the grid
    // runs in few, long waves and a partly filled last wave costs much: take the
    // smallest whole number of waves whose row blocks are at most 72 rows tall
    // (and at least 8).  Measured against the shapes above: 4096^2, 256 x 69
    // (two waves) 3.5% faster than 256 x 24, while 256 x 64 (2.1 waves) is 8%
    // slower; 8192^2, 256 x 67 +4%; 2048^2, 256 x 37 (one wave) +10%;
    // 4096 x 520, 256 x 18 +14%.
    const long long slots = 2ll * cus;
    const long long ns = (p.nx + 256 - kStep2Halo - 1) / (256 - kStep2Halo);
    for (int k = 1; k <= 64; ++k) {
      const long long rb = k * slots / ns;
      if (rb < 1) continue;
      const long long t = (p.ny + rb - 1) / rb;
      if (t > 72) continue;
      if (t >= 8) {
        w = 256;
        rows = (int)t;
      }
      break;
    }
  }
  *tx = w;
  *ty = std::min(rows, p.ny);
}

// Allocates whichever scratch buffer is still missing (after a failed
// allocation the others stay, and the next call completes the set).
lbm_status ensure_scratch(lbm_ctx* c) {
  const size_t n = (size_t)c->p.nx * c->p.ny;
  if (!c->work) HIP_TRY(hipMalloc(&c->work, 4 * n * sizeof(double)));
  if (!c->partials) HIP_TRY(hipMalloc(&c->partials, (size_t)obs_partials_count(c->g) * kNumRed * sizeof(double)));
  if (!c->red) HIP_TRY(hipMalloc(&c->red, (kNumRed + 2) * sizeof(double)));
  return LBM_OK;
}

lbm_status make_ctx(const lbm_params* p, void* stream, void* ba, void* bb, size_t bytes,
                    lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation failed");
  c->p = *p;
  st = model_of(*p, &c->m);
  if (st != LBM_OK) { delete c; return st; }
  int tx, ty;
  default_launch(*p, &tx, &ty);
  set_geometry(c, tx, ty);
  default_launch2(*p, &tx, &ty);
  set_geometry2(c, tx, ty);
  c->fuse = 2;
  c->buf_bytes = state_elems(*p) * elem_size(*p);
  c->step = 0;
  c->cur = 0;
  c->stream = static_cast<hipStream_t>(stream);  // NULL is the HIP null stream
  c->own_stream = false;
  const size_t need = c->buf_bytes;  // read before any lbm_destroy(c) below
  if (ba) {
    if (!bb || bytes < need || ((uintptr_t)ba & 255) || ((uintptr_t)bb & 255)) {
      lbm_destroy(c);
      return fail(LBM_EINVAL, "caller buffers: need two 256-byte aligned buffers of %zu bytes", need);
    }
    c->buf[0] = ba; c->buf[1] = bb; c->own_buf = false;
  } else {
    c->own_buf = true;
    for (int i = 0; i < 2; ++i) {
      hipError_t e = hipMalloc(&c->buf[i], c->buf_bytes);
      if (e != hipSuccess) {
        lbm_destroy(c);
        return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "hipMalloc(%zu): %s", need,
                    hipGetErrorString(e));
      }
    }
  }
  // zero both buffers so the pitch padding and the gaps between planes are defined
  for (int i = 0; i < 2; ++i) {
    hipError_t e = hipMemsetAsync(c->buf[i], 0, c->buf_bytes, c->stream);
    if (e != hipSuccess) { lbm_destroy(c); return fail(LBM_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(e)); }
  }
  *out = c;
  return LBM_OK;
}

lbm_status copy_to_device(lbm_ctx* c, double* dst, const double* src, size_t n) {
  HIP_TRY(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
  return LBM_OK;
}

lbm_status check_density(const double* rho, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!(rho[i] > 0.0) || !std::isfinite(rho[i]))
      return fail(LBM_ENONFINITE, "initial density %g at cell %zu", rho[i], i);
  return LBM_OK;
}

// The host part of the observables: h[0..kNumRed) the device reduction
// (mass, momentum, density extremes, max |v|^2, fault counts), h[kNumRed] and
// h[kNumRed + 1] rho at (nx/2, ny/2) and at (0, 0); pressures and the Laplace
// quantities of Eq. 22 follow on the host in FP64.
lbm_status finish_observables(const lbm_params& p, const ModelConsts& m, const double* h,
                              int64_t step, lbm_obs* o) {
  const size_t n = (size_t)p.nx * p.ny;
  o->step = step;
  o->mass = h[0];
  o->mom_x = h[1];
  o->mom_y = h[2];
  o->rho_min = h[3];
  o->rho_max = h[4];
  o->max_u = std::sqrt(h[5]);
  o->n_domain = (int64_t)h[6];
  o->n_nonfinite = (int64_t)h[7];
  o->rho_in = h[kNumRed];
  o->rho_out = h[kNumRed + 1];
  o->p_in = eos_pressure(p.eos, m.aalpha, p.b, p.R, p.K, m.T, p.a, o->rho_in);
  o->p_out = eos_pressure(p.eos, m.aalpha, p.b, p.R, p.K, m.T, p.a, o->rho_out);
  o->dp = o->p_in - o->p_out;
  const double excess = o->mass - (double)n * o->rho_out;
  o->R_e = std::sqrt(excess / (o->rho_in - o->rho_out) / M_PI);
  o->sigma = o->dp * o->R_e;
  if (o->n_nonfinite > 0) return fail(LBM_ENONFINITE, "%lld cells with non-finite or non-positive density", (long long)o->n_nonfinite);
  if (o->n_domain > 0) return fail(LBM_EDOMAIN, "%lld cells with U > 0", (long long)o->n_domain);
  return LBM_OK;
}

// FP64 observables of one state (shared by lattices and batch domains).
lbm_status observe(const lbm_params& p, const ModelConsts& m, const Geometry& g, const void* f,
                   int64_t step, double* work, double* partials, double* red, hipStream_t stream,
                   lbm_obs* o) {
  const lbm_precision prec = (lbm_precision)p.precision;
  HIP_TRY(launch_density_fields(prec, g, m, f, work, stream));
  HIP_TRY(launch_observables(prec, g, m, f, work, partials, red, stream));
  const size_t i_in = (size_t)(p.ny / 2) * p.nx + p.nx / 2;
  HIP_TRY(hipMemcpyAsync(red + kNumRed, work + i_in, sizeof(double), hipMemcpyDeviceToDevice, stream));
  HIP_TRY(hipMemcpyAsync(red + kNumRed + 1, work, sizeof(double), hipMemcpyDeviceToDevice, stream));
  double h[kNumRed + 2];
  HIP_TRY(hipMemcpyAsync(h, red, sizeof h, hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return finish_observables(p, m, h, step, o);
}

lbm_status read_field(const lbm_params& p, const ModelConsts& m, const Geometry& g, const void* f,
                      int32_t which, double* work, hipStream_t stream, double* out) {
  if (which < LBM_FIELD_RHO || which > LBM_FIELD_F0 + 8) return fail(LBM_EINVAL, "unknown field %d", which);
  const lbm_precision prec = (lbm_precision)p.precision;
  const size_t n = (size_t)p.nx * p.ny;
  double* src = work;
  if (which >= LBM_FIELD_F0) {
    src = work + 3 * n;
    HIP_TRY(launch_plane_to_f64(prec, g, f, which - LBM_FIELD_F0, src, stream));
  } else {
    HIP_TRY(launch_density_fields(prec, g, m, f, work, stream));
    if (which != LBM_FIELD_RHO) {
      src = work + 3 * n;
      HIP_TRY(launch_velocity_field(prec, g, m, f, work, which == LBM_FIELD_UX ? 0 : 1, src, stream));
    }
  }
  HIP_TRY(hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return LBM_OK;
}

// Runs of two-step launches go as replays of one captured graph of this many
// launches; the rest of a call (fewer launches) is launched one by one, so a
// caller who repeats a step count never captures inside its loop.
constexpr int kGraphLaunches = 64;

// The graph of k two-step launches starting from buffer c->cur (cached per k,
// starting buffer and launch geometry; at most four kept).
lbm_status step2_graph(lbm_ctx* c, int k, hipGraphExec_t* out) {
  for (int i = 0; i < c->ngraphs; ++i) {
    const auto& g = c->graphs[i];
    if (g.launches == k && g.parity == c->cur && g.version == c->version) {
      *out = g.exec;
      return LBM_OK;
    }
  }
  if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  int cur = c->cur;
  for (int i = 0; i < k && e == hipSuccess; ++i, cur = 1 - cur)
    e = launch_step2((lbm_precision)c->p.precision, c->g2, c->m, c->buf[cur], c->buf[1 - cur], c->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(c->cap_stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(LBM_EDEVICE, "step graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  // keep the newest four: drop the oldest when full
  if (c->ngraphs == 4) {
    (void)hipGraphExecDestroy(c->graphs[0].exec);
    for (int i = 1; i < 4; ++i) c->graphs[i - 1] = c->graphs[i];
    c->ngraphs = 3;
  }
  c->graphs[c->ngraphs++] = {exec, k, c->cur, c->version};
  *out = exec;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_params_default(lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  std::memset(p, 0, sizeof *p);
  p->nx = 64; p->ny = 64;
  p->eos = LBM_EOS_CS;
  p->precision = LBM_FP64;
  p->a = 1.0; p->b = 4.0; p->R = 1.0; p->omega_pr = 0.344; p->K = 1.0;
  p->T_over_Tc = 0.8;
  p->A = -0.5; p->kappa = 0.0; p->G = -1.0;
  p->s_e = 1.0; p->s_eps = 1.0; p->s_q = 8.0 / 7.0; p->s_nu = 1.0;
  return LBM_OK;
}

lbm_status lbm_critical_temperature(const lbm_params* p, double* Tc) {
  if (!p || !Tc) return fail(LBM_EINVAL, "NULL argument");
  if (p->eos == LBM_EOS_IDEAL) return fail(LBM_EINVAL, "ideal gas has no critical point");
  if (!(p->a > 0.0 && p->b > 0.0 && p->R > 0.0)) return fail(LBM_EINVAL, "EOS constants must be positive");
  return critical_temperature(*p, Tc);
}

lbm_status lbm_coexistence(const lbm_params* p, double* rho_v, double* rho_l) {
  if (!p || !rho_v || !rho_l) return fail(LBM_EINVAL, "NULL argument");
  if (p->eos == LBM_EOS_IDEAL) return fail(LBM_EINVAL, "ideal gas has no coexistence");
  if (!(p->a > 0.0 && p->b > 0.0 && p->R > 0.0)) return fail(LBM_EINVAL, "EOS constants must be positive");
  return coexistence(*p, rho_v, rho_l);
}

lbm_status lbm_laplace_fit(const double* dp, const double* R_e, int32_t n, double* sigma, double* spread) {
  if (!dp || !R_e || !sigma) return fail(LBM_EINVAL, "NULL argument");
  if (n < 1) return fail(LBM_EINVAL, "Laplace fit needs at least one drop (n = %d)", n);
  double sxy = 0.0, sxx = 0.0, smin = HUGE_VAL, smax = -HUGE_VAL, ssum = 0.0;
  for (int32_t i = 0; i < n; ++i) {
    if (!(R_e[i] > 0.0) || !std::isfinite(R_e[i]) || !std::isfinite(dp[i]))
      return fail(LBM_EINVAL, "Laplace fit: drop %d has R_e = %g, dp = %g", i, R_e[i], dp[i]);
    const double x = 1.0 / R_e[i];
    sxy += dp[i] * x;
    sxx += x * x;
    const double s = dp[i] * R_e[i];
    smin = std::min(smin, s);
    smax = std::max(smax, s);
    ssum += s;
  }
  *sigma = sxy / sxx;
  if (spread) *spread = (smax - smin) / std::fabs(ssum / n);
  return LBM_OK;
}

size_t lbm_buffer_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  return state_elems(*p) * elem_size(*p);
}

lbm_status lbm_create(const lbm_params* p, void* hip_stream, lbm_ctx** out) {
  return make_ctx(p, hip_stream, nullptr, nullptr, 0, out);
}

lbm_status lbm_create_ext(const lbm_params* p, void* hip_stream, void* buf_a, void* buf_b,
                          size_t buf_bytes, lbm_ctx** out) {
  if (!buf_a || !buf_b) return fail(LBM_EINVAL, "caller buffers are NULL");
  return make_ctx(p, hip_stream, buf_a, buf_b, buf_bytes, out);
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->own_buf)
    for (int i = 0; i < 2; ++i)
      if (c->buf[i]) (void)hipFree(c->buf[i]);
  if (c->work) (void)hipFree(c->work);
  if (c->partials) (void)hipFree(c->partials);
  if (c->red) (void)hipFree(c->red);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  for (int i = 0; i < c->ngraphs; ++i) (void)hipGraphExecDestroy(c->graphs[i].exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

lbm_status lbm_set_launch(lbm_ctx* c, const lbm_launch* l) {
  if (!c || !l) return fail(LBM_EINVAL, "NULL argument");
  if (c->pending) return fail(LBM_ESTATE, "lbm_set_launch while a row-range launch is open");
  // steps_per_pass 0: two, unless the tile asked for is too narrow for them
  const int fuse = l->steps_per_pass != 0 ? l->steps_per_pass : (l->tile_x == 64 ? 1 : 2);
  if (fuse != 1 && fuse != 2) return fail(LBM_EINVAL, "steps_per_pass %d not in {1, 2}", l->steps_per_pass);
  int tx = l->tile_x, ty = l->tile_y;
  int dtx, dty, dtx2, dty2;
  default_launch(c->p, &dtx, &dty);
  default_launch2(c->p, &dtx2, &dty2);
  if (fuse == 1) {
    if (tx == 0) tx = dtx;
    if (ty == 0) ty = dty;
    if (tx != 64 && tx != 128 && tx != 256) return fail(LBM_EINVAL, "tile_x %d not in {64,128,256}", tx);
  } else {
    if (tx == 0) tx = dtx2;
    if (ty == 0) ty = dty2;
    if (tx != 128 && tx != 256)
      return fail(LBM_EINVAL, "tile_x %d not in {128,256} for two steps per pass", tx);
  }
  if (ty < 1) return fail(LBM_EINVAL, "tile_y %d < 1", ty);
  ty = std::min(ty, c->p.ny);
  if (fuse == 1) {
    set_geometry(c, tx, ty);
  } else {
    // the single step that ends an odd count keeps the default shape
    set_geometry(c, dtx, dty);
    set_geometry2(c, tx, ty);
  }
  c->fuse = fuse;
  ++c->version;  // cached graphs hold the old shape
  return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_ctx* c, lbm_launch* l) {
  if (!c || !l) return fail(LBM_EINVAL, "NULL argument");
  const Geometry& g = c->fuse == 2 ? c->g2 : c->g;
  l->tile_x = g.tile_x;
  l->tile_y = g.tile_y;
  l->steps_per_pass = c->fuse;
  return LBM_OK;
}

lbm_status lbm_init_field(lbm_ctx* c, const double* rho, const double* ux, const double* uy) {
  if (!c || !rho) return fail(LBM_EINVAL, "NULL argument");
  const size_t n = (size_t)c->p.nx * c->p.ny;
  lbm_status st = check_density(rho, n);
  if (st != LBM_OK) return st;
  st = ensure_scratch(c);
  if (st != LBM_OK) return st;
  double* d_rho = c->work;
  double* d_ux = ux ? c->work + n : nullptr;
  double* d_uy = uy ? c->work + 2 * n : nullptr;
  if ((st = copy_to_device(c, d_rho, rho, n)) != LBM_OK) return st;
  if (ux && (st = copy_to_device(c, d_ux, ux, n)) != LBM_OK) return st;
  if (uy && (st = copy_to_device(c, d_uy, uy, n)) != LBM_OK) return st;
  c->cur = 0;
  HIP_TRY(launch_init_equilibrium((lbm_precision)c->p.precision, c->g, d_rho, d_ux, d_uy,
                                  c->buf[c->cur], c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // host arrays may go away after return
  c->step = 0;
  c->pending = 0;
  c->initialized = true;
  return LBM_OK;
}

lbm_status lbm_set_distributions(lbm_ctx* c, const double* f) {
  if (!c || !f) return fail(LBM_EINVAL, "NULL argument");
  lbm_status st = ensure_scratch(c);
  if (st != LBM_OK) return st;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  c->cur = 0;
  for (int a = 0; a < 9; ++a) {
    if ((st = copy_to_device(c, c->work, f + a * n, n)) != LBM_OK) return st;
    HIP_TRY(launch_f64_to_plane((lbm_precision)c->p.precision, c->g, c->work, a, c->buf[c->cur],
                                c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = 0;
  c->pending = 0;
  c->initialized = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (!c->initialized) return fail(LBM_ESTATE, "lbm_step before lbm_init_field");
  if (c->pending) return fail(LBM_ESTATE, "lbm_step while a row-range launch is open");
  int64_t left = n;
  // two steps per launch: the buffer written holds the state after both; runs of
  // 64 launches go as replays of a captured graph (small lattices are launch-bound)
  if (c->fuse == 2) {
    while (left >= 2 * kGraphLaunches) {
      const int k = kGraphLaunches;
      hipGraphExec_t exec = nullptr;
      lbm_status st = step2_graph(c, k, &exec);
      if (st != LBM_OK) return st;
      HIP_TRY(hipGraphLaunch(exec, c->stream));
      if (k & 1) c->cur = 1 - c->cur;
      left -= 2 * (int64_t)k;
    }
    for (; left >= 2; left -= 2) {
      HIP_TRY(launch_step2((lbm_precision)c->p.precision, c->g2, c->m, c->buf[c->cur],
                           c->buf[1 - c->cur], c->stream));
      c->cur = 1 - c->cur;
    }
  }
  for (; left > 0; --left) {
    HIP_TRY(launch_step((lbm_precision)c->p.precision, c->g, c->m, c->buf[c->cur],
                        c->buf[1 - c->cur], c->stream));
    c->cur = 1 - c->cur;
  }
  c->step += n;
  return LBM_OK;
}

lbm_status lbm_step_rows(lbm_ctx* c, int32_t n, int32_t y_begin, int32_t rows, int32_t flags) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (!c->initialized) return fail(LBM_ESTATE, "lbm_step_rows before lbm_init_field");
  if (flags & ~LBM_ROWS_MORE) return fail(LBM_EINVAL, "lbm_step_rows: unknown flags 0x%x", flags);
  if (n != 1 && !(n == 2 && c->fuse == 2))
    return fail(LBM_EINVAL, "lbm_step_rows: n = %d; one launch does 1 step, or 2 with two steps per pass", n);
  if (c->pending && n != c->pending)
    return fail(LBM_EINVAL, "lbm_step_rows: n = %d while a %d-step launch is open", n, c->pending);
  if (rows < 1 || y_begin < 0 || (int64_t)y_begin + rows > c->p.ny)
    return fail(LBM_EINVAL, "lbm_step_rows: rows [%d, %lld) outside [0, %d)", y_begin,
                (long long)y_begin + rows, c->p.ny);
  Geometry g = n == 2 ? c->g2 : c->g;
  g.y_begin = y_begin;
  g.y_end = y_begin + rows;
  g.nrowblocks = (rows + g.tile_y - 1) / g.tile_y;
  g.nblocks = g.nstrips * g.nrowblocks;
  const lbm_precision prec = (lbm_precision)c->p.precision;
  if (n == 2)
    HIP_TRY(launch_step2(prec, g, c->m, c->buf[c->cur], c->buf[1 - c->cur], c->stream));
  else
    HIP_TRY(launch_step(prec, g, c->m, c->buf[c->cur], c->buf[1 - c->cur], c->stream));
  if (flags & LBM_ROWS_MORE) {
    c->pending = n;  // more ranges of the same steps follow: the source stays current
    return LBM_OK;
  }
  c->pending = 0;
  c->cur = 1 - c->cur;
  c->step += n;
  return LBM_OK;
}

lbm_status lbm_observables(lbm_ctx* c, lbm_obs* o) {
  if (!c || !o) return fail(LBM_EINVAL, "NULL argument");
  if (!c->initialized) return fail(LBM_ESTATE, "observables before lbm_init_field");
  lbm_status st = ensure_scratch(c);
  if (st != LBM_OK) return st;
  return observe(c->p, c->m, c->g, c->buf[c->cur], c->step, c->work, c->partials, c->red, c->stream, o);
}

lbm_status lbm_observables_noalloc(lbm_ctx* c, lbm_obs* o) {
  if (!c || !o) return fail(LBM_EINVAL, "NULL argument");
  const long long cells = (long long)c->p.nx * c->p.ny;
  if (cells > noalloc_max_cells())
    return fail(LBM_EINVAL, "lbm_observables_noalloc: %lld cells exceed its scratch (at most %lld cells)",
                cells, noalloc_max_cells());
  if (!c->initialized) return fail(LBM_ESTATE, "observables before lbm_init_field");
  // one call at a time in this process: every call on a device shares its scratch array
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  double* scratch = nullptr;
  HIP_TRY(noalloc_scratch(&scratch));
  double* red = scratch + (size_t)obs_partials_count(c->g) * kNumRed;
  HIP_TRY(launch_observables_direct((lbm_precision)c->p.precision, c->g, c->m, c->buf[c->cur], scratch,
                                    red, c->stream));
  double h[kNumRed + 2];
  HIP_TRY(hipMemcpyAsync(h, red, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return finish_observables(c->p, c->m, h, c->step, o);
}

int64_t lbm_noalloc_max_cells(void) { return noalloc_max_cells(); }

lbm_status lbm_get_field(lbm_ctx* c, int32_t which, double* out) {
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  if (!c->initialized) return fail(LBM_ESTATE, "field before lbm_init_field");
  lbm_status st = ensure_scratch(c);
  if (st != LBM_OK) return st;
  return read_field(c->p, c->m, c->g, c->buf[c->cur], which, c->work, c->stream, out);
}

lbm_status lbm_save_state(lbm_ctx* c, void* buf, size_t* len) {
  if (!c || !len) return fail(LBM_EINVAL, "NULL argument");
  const size_t need = sizeof(StateHeader) + c->buf_bytes;
  if (!buf) { *len = need; return LBM_OK; }
  if (*len < need) return fail(LBM_EINVAL, "state buffer of %zu bytes, need %zu", *len, need);
  if (!c->initialized) return fail(LBM_ESTATE, "save before lbm_init_field");
  if (c->pending) return fail(LBM_ESTATE, "save while a row-range launch is open");
  StateHeader h{kStateMagic, c->p.nx, c->p.ny, c->g.pitch, c->p.precision, c->step,
                params_hash(c->p), c->buf_bytes};
  std::memcpy(buf, &h, sizeof h);
  HIP_TRY(hipMemcpyAsync(static_cast<char*>(buf) + sizeof h, c->buf[c->cur], c->buf_bytes,
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *len = need;
  return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return fail(LBM_EINVAL, "NULL argument");
  StateHeader h;
  if (len < sizeof h) return fail(LBM_EINVAL, "state blob too short");
  std::memcpy(&h, buf, sizeof h);
  if (h.magic != kStateMagic) return fail(LBM_EINVAL, "not a state blob");
  if (h.nx != c->p.nx || h.ny != c->p.ny || h.precision != c->p.precision ||
      h.pitch != c->g.pitch || h.params_hash != params_hash(c->p) || h.payload_bytes != c->buf_bytes ||
      len < sizeof h + c->buf_bytes)
    return fail(LBM_EINVAL, "state blob does not match this context's parameters");
  c->cur = 0;
  HIP_TRY(hipMemcpyAsync(c->buf[0], static_cast<const char*>(buf) + sizeof h, c->buf_bytes,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->step = h.step;
  c->pending = 0;
  c->initialized = true;
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_state_info(const lbm_ctx* c, int64_t* step, const void** f_cur, int32_t* pitch) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (step) *step = c->step;
  if (f_cur) *f_cur = c->buf[c->cur];
  if (pitch) *pitch = c->g.pitch;
  return LBM_OK;
}

const char* lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_ENONFINITE: return "non-finite or non-positive density";
    case LBM_EDOMAIN: return "U > 0: pseudo-potential not real";
    case LBM_ESTATE: return "call out of order";
  }
  return "unknown status";
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ===========================================================================
// Batched engine (host side)
// ===========================================================================
struct lbm_batch {
  int n = 0;
  std::vector<lbm_params> p;
  std::vector<ModelConsts> m;
  std::vector<Geometry> g;
  std::vector<size_t> off[2];
  std::vector<unsigned> ntiles;   // single-step tiles of each domain
  std::vector<unsigned> ntiles2;  // two-step tiles of each domain
  std::vector<bool> inited;
  lbm_precision prec = LBM_FP64;
  int eos = 0;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t stream = nullptr;
  int mode = LBM_BATCH_PER_STEP;
  int tile_x = 256, tile_y = 16;
  int fuse = 2;                 // per-step mode: steps per launch (1 or 2)
  void* d_tiles2 = nullptr;     // two-step tile list (fuse == 2)
  int ntile2_total = 0;
  long long spin_limit = 1ll << 20;
  int per_cu = 0, cus = 0;
  // device layout
  void* d_dom = nullptr;
  void* d_tiles = nullptr;
  int* d_group_begin = nullptr;
  int nxcd = 1;               // XCDs of the device: one domain group each (persistent mode)
  int max_group_tiles = 1;    // two-step tiles of the largest group (bounds the pairs of one launch)
  unsigned* d_head = nullptr;
  unsigned* d_done = nullptr;
  int* d_err = nullptr;
  int ntile_total = 0, grid = 0;
  // state
  int parity = 0;
  int64_t step = 0;
  bool layout_ok = false;  // the device tile lists match mode / tile / fuse
  // graph cache
  hipGraphExec_t exec = nullptr;
  int exec_mode = -1, exec_steps = 0, exec_parity = -1, exec_fuse = 0;
  // FP64 scratch for observables / fields
  double* work = nullptr;
  double* partials = nullptr;
  double* red = nullptr;
};

namespace {

// The persistent launch mode (lbm_persistent.hip).  An earlier form of its
// kernel, with a wait loop run by one lane, never finished on the GPU; this
// switch turns the mode off again should the present form fail its GPU tests.
constexpr bool kPersistentEnabled = true;

void batch_free_layout(lbm_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  b->exec_mode = -1;
  for (void* q : {b->d_dom, b->d_tiles, b->d_tiles2, (void*)b->d_group_begin})
    if (q) (void)hipFree(q);
  b->d_dom = b->d_tiles = b->d_tiles2 = nullptr;
  b->d_group_begin = nullptr;
}

// Tiles of every domain and the device copies.  The single-step tile list
// (tile_x x tile_y tiles, domain by domain) serves one-step launches; the
// two-step list (strips of tile_x - 6 stored columns, the same row blocks)
// serves two-step launches, domain by domain in the per-step mode.  In the
// persistent mode the two-step list is stored group by group: the domains go
// to one group per XCD (longest processing time first onto the least loaded
// group), each domain's tiles together, so that a group's queue finishes one
// domain's pair of steps before the next.
lbm_status batch_layout(lbm_batch* b) {
  b->layout_ok = false;  // until every list below is on the device
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_free_layout(b);
  HIP_TRY(hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));
  struct T4 { int d, x0, y0, down; };
  std::vector<T4> tiles, tiles2;
  std::vector<long long> dcost(b->n, 0);
  b->ntiles.assign(b->n, 0);
  b->ntiles2.assign(b->n, 0);
  const int w2 = b->tile_x - kStep2Halo;
  for (int d = 0; d < b->n; ++d) {
    Geometry& g = b->g[d];
    g.tile_x = b->tile_x;
    g.tile_y = std::min(b->tile_y, g.ny);
    g.nstrips = (g.nx + g.tile_x - 1) / g.tile_x;
    g.nrowblocks = (g.ny + g.tile_y - 1) / g.tile_y;
    g.nblocks = g.nstrips * g.nrowblocks;
    for (int rb = 0; rb < g.nrowblocks; ++rb)
      for (int sx = 0; sx < g.nstrips; ++sx) tiles.push_back({d, sx * g.tile_x, rb * g.tile_y, rb & 1});
    b->ntiles[d] = (unsigned)g.nblocks;
    if (b->fuse == 2) {
      const int ns = (g.nx + w2 - 1) / w2;
      for (int rb = 0; rb < g.nrowblocks; ++rb)
        for (int sx = 0; sx < ns; ++sx) {
          const long long w = std::min(w2, g.nx - sx * w2), h = std::min(g.tile_y, g.ny - rb * g.tile_y);
          tiles2.push_back({d, sx * w2, rb * g.tile_y, rb & 1});
          dcost[d] += (w + kStep2Halo) * (h + 6);  // cells a pass computes, halo included
        }
      b->ntiles2[d] = (unsigned)(ns * g.nrowblocks);
    }
  }
  b->ntile_total = (int)tiles.size();
  b->ntile2_total = (int)tiles2.size();
  std::vector<int> group_begin;
  if (b->mode == LBM_BATCH_PERSISTENT) {
    HIP_TRY(batch_occupancy(b->prec, b->eos, b->tile_x, &b->per_cu));
    if (b->per_cu < 1) return fail(LBM_EDEVICE, "persistent batch kernel cannot be resident");
    b->grid = b->per_cu * b->cus;
    const int ng = b->nxcd;
    std::vector<int> order(b->n);
    for (int d = 0; d < b->n; ++d) order[d] = d;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return dcost[a] > dcost[c]; });
    std::vector<long long> load(ng, 0);
    std::vector<std::vector<int>> members(ng);
    for (int d : order) {
      const int gi = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      members[gi].push_back(d);
      load[gi] += dcost[d];
    }
    std::vector<int> first(b->n + 1, 0);  // two-step tiles were generated domain by domain
    for (int d = 0; d < b->n; ++d) first[d + 1] = first[d] + (int)b->ntiles2[d];
    std::vector<T4> sorted;
    group_begin.push_back(0);
    for (int gi = 0; gi < ng; ++gi) {
      for (int d : members[gi])
        for (int t = first[d]; t < first[d + 1]; ++t) sorted.push_back(tiles2[t]);
      group_begin.push_back((int)sorted.size());
    }
    b->max_group_tiles = 1;
    for (int gi = 0; gi < ng; ++gi)
      b->max_group_tiles = std::max(b->max_group_tiles, group_begin[gi + 1] - group_begin[gi]);
    tiles2.swap(sorted);
  } else {
    b->grid = b->ntile_total;
    group_begin.assign(2, 0);
  }
  const size_t db = batch_domain_bytes(b->prec), tb = batch_tile_bytes();
  std::vector<unsigned char> hd(db * b->n), ht(tb * tiles.size()), ht2(tb * tiles2.size());
  // the persistent barrier counts a domain's two-step tiles
  for (int d = 0; d < b->n; ++d)
    batch_fill_domain(b->prec, b->g[d], b->m[d], static_cast<char*>(b->arena) + b->off[0][d],
                      static_cast<char*>(b->arena) + b->off[1][d], b->fuse == 2 ? b->ntiles2[d] : b->ntiles[d],
                      hd.data() + d * db);
  for (size_t t = 0; t < tiles.size(); ++t)
    batch_fill_tile(tiles[t].d, tiles[t].x0, tiles[t].y0, tiles[t].down, ht.data() + t * tb);
  for (size_t t = 0; t < tiles2.size(); ++t)
    batch_fill_tile(tiles2[t].d, tiles2[t].x0, tiles2[t].y0, tiles2[t].down, ht2.data() + t * tb);
  HIP_TRY(hipMalloc(&b->d_dom, hd.size()));
  HIP_TRY(hipMalloc(&b->d_tiles, ht.size()));
  HIP_TRY(hipMalloc(&b->d_group_begin, group_begin.size() * sizeof(int)));
  HIP_TRY(hipMemcpyAsync(b->d_dom, hd.data(), hd.size(), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_tiles, ht.data(), ht.size(), hipMemcpyHostToDevice, b->stream));
  if (!ht2.empty()) {
    HIP_TRY(hipMalloc(&b->d_tiles2, ht2.size()));
    HIP_TRY(hipMemcpyAsync(b->d_tiles2, ht2.data(), ht2.size(), hipMemcpyHostToDevice, b->stream));
  }
  HIP_TRY(hipMemcpyAsync(b->d_group_begin, group_begin.data(), group_begin.size() * sizeof(int),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->layout_ok = true;
  return LBM_OK;
}

BatchRun batch_run(const lbm_batch* b, int nsteps, int parity) {
  BatchRun r{};
  r.dom = b->d_dom;
  r.tiles = b->d_tiles;
  r.group_begin = b->d_group_begin;
  r.ngroups = b->nxcd;
  r.head = b->d_head;
  r.done = b->d_done;
  r.err = b->d_err;
  r.grid = b->grid;
  r.nsteps = nsteps;
  r.parity = parity;
  r.spin_limit = b->spin_limit;
  return r;
}

// Buffer swaps that n steps take: one per step, or one per pair of steps and
// one for an odd last step.
int batch_launches(const lbm_batch* b, int n) {
  return b->fuse == 2 ? n / 2 + n % 2 : n;
}

// Enqueues n steps: persistent = queue/counter reset, one launch of n / 2
// pairs and the completion check; per-step = one launch per step (or per two
// steps) with alternating buffers; either way an odd last step is one
// single-step launch.
hipError_t batch_enqueue(lbm_batch* b, int n) {
  hipError_t e = hipSuccess;
  int launch = 0, left = n;
  if (b->mode == LBM_BATCH_PERSISTENT) {
    const int pairs = n / 2;
    if (pairs > 0) {
      BatchRun r = batch_run(b, pairs, b->parity);
      r.tiles = b->d_tiles2;
      e = launch_batch_reset(r, b->n, b->stream);
      if (e == hipSuccess) e = launch_batch_persistent(b->prec, b->eos, b->tile_x, r, b->stream);
      if (e == hipSuccess) e = launch_batch_check(b->prec, r, b->n, b->stream);
    }
    launch = pairs;
    left = n - 2 * pairs;
  } else if (b->fuse == 2) {
    for (; left >= 2 && e == hipSuccess; left -= 2, ++launch) {
      BatchRun r = batch_run(b, 2, (b->parity + launch) & 1);
      r.tiles = b->d_tiles2;
      r.grid = b->ntile2_total;
      e = launch_batch_step2(b->prec, b->eos, b->tile_x, r, b->stream);
    }
  }
  for (; left > 0 && e == hipSuccess; --left, ++launch) {
    BatchRun r = batch_run(b, 1, (b->parity + launch) & 1);
    r.grid = b->ntile_total;
    e = launch_batch(b->prec, b->eos, b->tile_x, r, b->stream);
  }
  return e;
}

// The same n steps captured once as a graph (re-captured when the mode, the
// step count or the buffer parity changes).
lbm_status batch_graph(lbm_batch* b, int n) {
  if (b->exec && b->exec_mode == b->mode && b->exec_steps == n && b->exec_parity == b->parity &&
      b->exec_fuse == b->fuse)
    return LBM_OK;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  b->exec = nullptr;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = batch_enqueue(b, n);
  hipError_t e2 = hipStreamEndCapture(b->stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(LBM_EDEVICE, "batch graph capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  b->exec_mode = b->mode;
  b->exec_steps = n;
  b->exec_parity = b->parity;
  b->exec_fuse = b->fuse;
  return LBM_OK;
}

lbm_status batch_scratch(lbm_batch* b) {
  if (b->work && b->partials && b->red) return LBM_OK;
  size_t cells = 0;
  int parts = 0;
  for (int d = 0; d < b->n; ++d) {
    cells = std::max(cells, (size_t)b->p[d].nx * b->p[d].ny);
    parts = std::max(parts, obs_partials_count(b->g[d]));
  }
  if (!b->work) HIP_TRY(hipMalloc(&b->work, 4 * cells * sizeof(double)));
  if (!b->partials) HIP_TRY(hipMalloc(&b->partials, (size_t)parts * kNumRed * sizeof(double)));
  if (!b->red) HIP_TRY(hipMalloc(&b->red, (kNumRed + 2) * sizeof(double)));
  return LBM_OK;
}

lbm_status batch_check_error(lbm_batch* b) {
  HIP_TRY(hipStreamSynchronize(b->stream));
  int err = 0;
  HIP_TRY(hipMemcpyAsync(&err, b->d_err, sizeof err, hipMemcpyDeviceToHost, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  if (err) {
    // reported once; the state of an aborted launch is not a whole step
    HIP_TRY(hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (err & 1)
      return fail(LBM_EDEVICE, "persistent batch launch aborted: a domain barrier wait exceeded the spin limit");
    return fail(LBM_EDEVICE, "persistent batch launch incomplete: no workgroup ran on the XCD of some domain group");
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(const lbm_params* params, int32_t n, void* hip_stream, lbm_batch** out) {
  if (!params || !out || n < 1) return fail(LBM_EINVAL, "batch: NULL argument or n < 1");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    lbm_status st = validate(&params[i]);
    if (st != LBM_OK) return fail(st, "batch domain %d: %s", i, g_last_error.c_str());
    if (params[i].eos != params[0].eos || params[i].precision != params[0].precision)
      return fail(LBM_EINVAL, "batch domain %d: every domain must share the EOS kind and precision", i);
  }
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->prec = (lbm_precision)params[0].precision;
  b->eos = params[0].eos;
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->p.assign(params, params + n);
  b->m.resize(n);
  b->g.resize(n);
  b->off[0].resize(n);
  b->off[1].resize(n);
  b->inited.assign(n, false);
  const size_t es = elem_size(params[0]);
  size_t total = 0;
  for (int d = 0; d < n; ++d) {
    lbm_status st = model_of(params[d], &b->m[d]);
    if (st != LBM_OK) { lbm_batch_destroy(b); return st; }
    Geometry& g = b->g[d];
    g.nx = params[d].nx;
    g.ny = params[d].ny;
    g.y_begin = 0;
    g.y_end = g.ny;
    g.pitch = pitch_of(params[d]);
    g.row = 9ll * g.pitch;
    const size_t bytes = (state_elems(params[d]) * es + 255) / 256 * 256;
    if (state_elems(params[d]) * es >= (1ull << 32)) {
      lbm_batch_destroy(b);
      return fail(LBM_EINVAL, "batch domain %d: a distribution buffer must stay below 4 GiB", d);
    }
    b->off[0][d] = total;
    b->off[1][d] = total + bytes;
    total += 2 * bytes;
  }
  b->arena_bytes = total;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipMalloc(&b->arena, total);
  if (e == hipSuccess) e = hipMemsetAsync(b->arena, 0, total, b->stream);
  if (e == hipSuccess) {
    // one domain group per XCD; a device that does not report XCDs is one group
    int nx = 0;
    if (hipDeviceGetAttribute(&nx, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess && nx >= 1 && nx <= 16)
      b->nxcd = nx;
    (void)hipGetLastError();
  }
  if (e == hipSuccess) e = hipMalloc(&b->d_head, 16 * sizeof(unsigned));
  if (e == hipSuccess) e = hipMalloc(&b->d_done, n * sizeof(unsigned));
  if (e == hipSuccess) e = hipMalloc(&b->d_err, sizeof(int));
  if (e == hipSuccess) e = hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream);
  if (e != hipSuccess) {
    lbm_batch_destroy(b);
    return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "batch allocation: %s", hipGetErrorString(e));
  }
  lbm_status st = batch_layout(b);
  if (st != LBM_OK) { lbm_batch_destroy(b); return st; }
  *out = b;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  batch_free_layout(b);
  for (void* q : {b->arena, (void*)b->d_head, (void*)b->d_done, (void*)b->d_err, (void*)b->work, (void*)b->partials, (void*)b->red})
    if (q) (void)hipFree(q);
  delete b;
}

lbm_status lbm_batch_set_launch(lbm_batch* b, const lbm_batch_launch* l) {
  if (!b || !l) return fail(LBM_EINVAL, "NULL argument");
  if (l->mode != LBM_BATCH_PERSISTENT && l->mode != LBM_BATCH_PER_STEP)
    return fail(LBM_EINVAL, "unknown batch mode %d", l->mode);
  if (l->mode == LBM_BATCH_PERSISTENT && !kPersistentEnabled)
    return fail(LBM_EINVAL, "persistent batch mode is switched off in this version of the library (its kernel has not "
                            "passed on a GPU); use LBM_BATCH_PER_STEP");
  // steps_per_pass 0: two, unless a 64-wide tile asks for one
  const int fuse = l->steps_per_pass ? l->steps_per_pass : (l->tile_x != 64 ? 2 : 1);
  if (fuse != 1 && fuse != 2) return fail(LBM_EINVAL, "steps_per_pass %d not in {1, 2}", fuse);
  if (fuse != 2 && l->mode == LBM_BATCH_PERSISTENT)
    return fail(LBM_EINVAL, "the persistent mode runs two steps per pass");
  // default row blocks: 16 rows for per-step launches; 24 for the persistent
  // launch, where a taller tile spends fewer queue and barrier round trips per row
  const int ty_default = fuse != 2 ? 32 : (l->mode == LBM_BATCH_PERSISTENT ? 24 : 16);
  const int tx = l->tile_x ? l->tile_x : (fuse == 2 ? 256 : 64), ty = l->tile_y ? l->tile_y : ty_default;
  if (tx != 64 && tx != 128 && tx != 256) return fail(LBM_EINVAL, "tile_x %d not in {64,128,256}", tx);
  if (fuse == 2 && tx == 64) return fail(LBM_EINVAL, "tile_x 64 too narrow for two steps per launch");
  if (ty < 1) return fail(LBM_EINVAL, "tile_y %d < 1", ty);
  if (l->spin_limit < 0) return fail(LBM_EINVAL, "negative spin limit");
  b->mode = l->mode;
  b->fuse = fuse;
  b->tile_x = tx;
  b->tile_y = ty;
  b->spin_limit = l->spin_limit ? l->spin_limit : (1ll << 20);
  if (l->spin_limit == 0 && l->force_spin_limit) b->spin_limit = 0;
  return batch_layout(b);
}

lbm_status lbm_batch_get_launch(const lbm_batch* b, lbm_batch_launch* l) {
  if (!b || !l) return fail(LBM_EINVAL, "NULL argument");
  l->mode = b->mode;
  l->tile_x = b->tile_x;
  l->tile_y = b->tile_y;
  l->spin_limit = b->spin_limit;
  l->force_spin_limit = 0;
  l->grid = b->grid;
  l->ntiles = b->ntile_total;
  l->resident_per_cu = b->per_cu;
  l->steps_per_pass = b->fuse;
  if (b->fuse == 2) {
    l->grid = b->mode == LBM_BATCH_PERSISTENT ? b->grid : b->ntile2_total;
    l->ntiles = b->ntile2_total;
  }
  return LBM_OK;
}

lbm_status lbm_batch_init_field(lbm_batch* b, int32_t i, const double* rho, const double* ux,
                                const double* uy) {
  if (!b || !rho) return fail(LBM_EINVAL, "NULL argument");
  if (i < 0 || i >= b->n) return fail(LBM_EINVAL, "domain %d out of range", i);
  const size_t n = (size_t)b->p[i].nx * b->p[i].ny;
  lbm_status st = check_density(rho, n);
  if (st != LBM_OK) return st;
  if ((st = batch_scratch(b)) != LBM_OK) return st;
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipMemcpyAsync(b->work, rho, n * sizeof(double), hipMemcpyHostToDevice, b->stream));
  if (ux) HIP_TRY(hipMemcpyAsync(b->work + n, ux, n * sizeof(double), hipMemcpyHostToDevice, b->stream));
  if (uy) HIP_TRY(hipMemcpyAsync(b->work + 2 * n, uy, n * sizeof(double), hipMemcpyHostToDevice, b->stream));
  void* f = static_cast<char*>(b->arena) + b->off[b->parity][i];
  HIP_TRY(launch_init_equilibrium(b->prec, b->g[i], b->work, ux ? b->work + n : nullptr,
                                  uy ? b->work + 2 * n : nullptr, f, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->inited[i] = true;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t n) {
  if (!b) return fail(LBM_EINVAL, "NULL batch");
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  for (int d = 0; d < b->n; ++d)
    if (!b->inited[d]) return fail(LBM_ESTATE, "batch domain %d not initialised", d);
  if (!b->layout_ok)
    return fail(LBM_ESTATE, "batch has no launch layout (the last lbm_batch_set_launch failed); set it again");
  // persistent mode: the whole call is one launch (plus a single step for an
  // odd count), chunked only where a group's queue (tiles x pairs) would pass
  // 2^31; per-step mode: one graph per call of up to 32,768 steps (the 20,000
  // steps of a droplet study are one graph launch of 10,000 kernel nodes;
  // capturing and instantiating it takes about 20 ms and its replay runs as
  // fast as shorter graphs)
  const int64_t chunk = b->mode == LBM_BATCH_PERSISTENT
                            ? 2 * std::max<int64_t>(1, ((1ll << 31) - 1) / b->max_group_tiles)
                            : 32768;
  int64_t left = n;
  while (left > 0) {
    const int k = (int)std::min(left, chunk);
    if (b->stream) {
      // graphs cannot be captured on the legacy null stream: only on a real stream
      lbm_status st = batch_graph(b, k);
      if (st != LBM_OK) return st;
      HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    } else {
      HIP_TRY(batch_enqueue(b, k));
    }
    b->parity = (b->parity + batch_launches(b, k)) & 1;
    left -= k;
  }
  b->step += n;
  return LBM_OK;
}

lbm_status lbm_batch_sync(lbm_batch* b) {
  if (!b) return fail(LBM_EINVAL, "NULL batch");
  return batch_check_error(b);
}

lbm_status lbm_batch_observables(lbm_batch* b, lbm_obs* out) {
  if (!b || !out) return fail(LBM_EINVAL, "NULL argument");
  lbm_status st = batch_check_error(b);
  if (st != LBM_OK) return st;
  if ((st = batch_scratch(b)) != LBM_OK) return st;
  lbm_status worst = LBM_OK;
  for (int d = 0; d < b->n; ++d) {
    const void* f = static_cast<char*>(b->arena) + b->off[b->parity][d];
    st = observe(b->p[d], b->m[d], b->g[d], f, b->step, b->work, b->partials, b->red, b->stream, &out[d]);
    if (st == LBM_EDEVICE || st == LBM_ENOMEM) return st;
    if (st != LBM_OK && worst == LBM_OK) worst = st;
  }
  if (worst != LBM_OK) return fail(worst, "at least one batch domain holds non-finite densities or U > 0 cells");
  return LBM_OK;
}

lbm_status lbm_batch_get_field(lbm_batch* b, int32_t i, int32_t which, double* out) {
  if (!b || !out) return fail(LBM_EINVAL, "NULL argument");
  if (i < 0 || i >= b->n) return fail(LBM_EINVAL, "domain %d out of range", i);
  lbm_status st = batch_check_error(b);
  if (st != LBM_OK) return st;
  if ((st = batch_scratch(b)) != LBM_OK) return st;
  const void* f = static_cast<char*>(b->arena) + b->off[b->parity][i];
  return read_field(b->p[i], b->m[i], b->g[i], f, which, b->work, b->stream, out);
}

}  // extern "C"

// ===========================================================================
// Surrogate network (host side)
// ===========================================================================
struct lbm_mlp {
  int max_batch = 0;
  hipStream_t stream = nullptr;
  float *p = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *gpart = nullptr;
  unsigned short* wb = nullptr;
  float *x = nullptr, *y = nullptr, *dy = nullptr, *acts = nullptr, *dx = nullptr;
  float *xd = nullptr, *td = nullptr;  // the training set of lbm_mlp_set_data (never reused as scratch)
  float* loss = nullptr;
  int loss_cap = 0;
  int ndata = 0;
  int64_t adam_t = 0;
};

namespace {

lbm_status mlp_check_n(const lbm_mlp* m, int32_t n) {
  if (n < 1 || n > m->max_batch) return fail(LBM_EINVAL, "batch of %d samples outside [1, %d]", n, m->max_batch);
  return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_mlp_param_count(void) { return mlp_param_count(); }

lbm_status lbm_mlp_create(int32_t max_batch, void* hip_stream, lbm_mlp** out) {
  if (!out || max_batch < 1 || max_batch > (1 << 20)) return fail(LBM_EINVAL, "max_batch must be in [1, 2^20]");
  *out = nullptr;
  lbm_mlp* m = new (std::nothrow) lbm_mlp();
  if (!m) return fail(LBM_ENOMEM, "host allocation failed");
  m->max_batch = max_batch;
  m->stream = static_cast<hipStream_t>(hip_stream);
  const size_t np = mlp_param_count();
  const int nwg = (max_batch + mlp_rows_per_block() - 1) / mlp_rows_per_block();
  hipError_t e = hipSuccess;
  auto alloc = [&](void** q, size_t bytes) { if (e == hipSuccess) e = hipMalloc(q, bytes); };
  alloc((void**)&m->p, np * 4);
  alloc((void**)&m->m, np * 4);
  alloc((void**)&m->v, np * 4);
  alloc((void**)&m->grad, np * 4);
  alloc((void**)&m->gpart, (size_t)nwg * np * 4);
  alloc((void**)&m->wb, np * 2);
  alloc((void**)&m->x, (size_t)max_batch * 3 * 4);
  alloc((void**)&m->xd, (size_t)max_batch * 3 * 4);
  alloc((void**)&m->td, (size_t)max_batch * 3 * 4);
  alloc((void**)&m->y, (size_t)max_batch * 3 * 4);
  alloc((void**)&m->dy, (size_t)max_batch * 3 * 4);
  alloc((void**)&m->dx, (size_t)max_batch * 3 * 4);
  alloc((void**)&m->acts, (size_t)max_batch * 3 * 128 * 4);
  if (e == hipSuccess) e = hipMemsetAsync(m->p, 0, np * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->m, 0, np * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->v, 0, np * 4, m->stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->wb, 0, np * 2, m->stream);
  if (e != hipSuccess) {
    lbm_mlp_destroy(m);
    return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "mlp allocation: %s", hipGetErrorString(e));
  }
  *out = m;
  return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp* m) {
  if (!m) return;
  (void)hipStreamSynchronize(m->stream);
  for (void* q : {(void*)m->p, (void*)m->m, (void*)m->v, (void*)m->grad, (void*)m->gpart, (void*)m->wb,
                  (void*)m->x, (void*)m->xd, (void*)m->td, (void*)m->y, (void*)m->dy, (void*)m->dx, (void*)m->acts,
                  (void*)m->loss})
    if (q) (void)hipFree(q);
  delete m;
}

lbm_status lbm_mlp_set_params(lbm_mlp* m, const float* params) {
  if (!m || !params) return fail(LBM_EINVAL, "NULL argument");
  const size_t np = mlp_param_count();
  HIP_TRY(hipMemcpyAsync(m->p, params, np * 4, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemsetAsync(m->m, 0, np * 4, m->stream));
  HIP_TRY(hipMemsetAsync(m->v, 0, np * 4, m->stream));
  HIP_TRY(launch_mlp_round(m->p, m->wb, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  m->adam_t = 0;
  return LBM_OK;
}

lbm_status lbm_mlp_get_params(lbm_mlp* m, float* params) {
  if (!m || !params) return fail(LBM_EINVAL, "NULL argument");
  HIP_TRY(hipMemcpyAsync(params, m->p, (size_t)mlp_param_count() * 4, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_forward(lbm_mlp* m, const float* x, int32_t n, float* y) {
  if (!m || !x || !y) return fail(LBM_EINVAL, "NULL argument");
  lbm_status st = mlp_check_n(m, n);
  if (st != LBM_OK) return st;
  HIP_TRY(hipMemcpyAsync(m->x, x, (size_t)n * 12, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(launch_mlp_forward(m->x, n, m->p, m->wb, nullptr, m->y, m->stream));
  HIP_TRY(hipMemcpyAsync(y, m->y, (size_t)n * 12, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_backward(lbm_mlp* m, const float* x, const float* dy, int32_t n, float* grad,
                            float* dx) {
  if (!m || !x || !dy) return fail(LBM_EINVAL, "NULL argument");
  lbm_status st = mlp_check_n(m, n);
  if (st != LBM_OK) return st;
  HIP_TRY(hipMemcpyAsync(m->x, x, (size_t)n * 12, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemcpyAsync(m->dy, dy, (size_t)n * 12, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(launch_mlp_forward(m->x, n, m->p, m->wb, m->acts, m->y, m->stream));
  HIP_TRY(launch_mlp_backward(m->x, m->acts, m->dy, n, m->wb, m->gpart, m->grad, m->dx, m->stream));
  if (grad) HIP_TRY(hipMemcpyAsync(grad, m->grad, (size_t)mlp_param_count() * 4, hipMemcpyDeviceToHost, m->stream));
  if (dx) HIP_TRY(hipMemcpyAsync(dx, m->dx, (size_t)n * 12, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

lbm_status lbm_mlp_set_data(lbm_mlp* m, const float* x, const float* t, int32_t n) {
  if (!m || !x || !t) return fail(LBM_EINVAL, "NULL argument");
  lbm_status st = mlp_check_n(m, n);
  if (st != LBM_OK) return st;
  HIP_TRY(hipMemcpyAsync(m->xd, x, (size_t)n * 12, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipMemcpyAsync(m->td, t, (size_t)n * 12, hipMemcpyHostToDevice, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  m->ndata = n;
  return LBM_OK;
}

lbm_status lbm_mlp_train(lbm_mlp* m, int32_t iters, float lr, float* loss_out) {
  if (!m) return fail(LBM_EINVAL, "NULL argument");
  if (m->ndata < 1) return fail(LBM_ESTATE, "lbm_mlp_train before lbm_mlp_set_data");
  if (iters < 0 || !(lr > 0.f)) return fail(LBM_EINVAL, "iters must be >= 0 and lr > 0");
  if (iters > m->loss_cap) {
    // forget the old buffer before anything can fail, so no later call uses it
    float* old = m->loss;
    m->loss = nullptr;
    m->loss_cap = 0;
    if (old) HIP_TRY(hipFree(old));
    HIP_TRY(hipMalloc(&m->loss, (size_t)iters * 4));
    m->loss_cap = iters;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int it = 0; it < iters; ++it) {
    ++m->adam_t;
    const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
    HIP_TRY(launch_mlp_forward(m->xd, m->ndata, m->p, m->wb, m->acts, m->y, m->stream));
    HIP_TRY(launch_mlp_mse(m->y, m->td, m->ndata, m->dy, m->loss + it, m->stream));
    HIP_TRY(launch_mlp_backward(m->xd, m->acts, m->dy, m->ndata, m->wb, m->gpart, m->grad, nullptr, m->stream));
    HIP_TRY(launch_mlp_adam(m->p, m->m, m->v, m->grad, m->wb, lr, b1, b2, eps, c1, c2, m->stream));
  }
  if (loss_out && iters > 0)
    HIP_TRY(hipMemcpyAsync(loss_out, m->loss, (size_t)iters * 4, hipMemcpyDeviceToHost, m->stream));
  HIP_TRY(hipStreamSynchronize(m->stream));
  return LBM_OK;
}

}  // extern "C"
