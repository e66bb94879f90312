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
#include <string>

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

constexpr uint64_t kStateMagic = 0x4c424d5053543031ull;  // "LBMPST01"

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

// 64-point Gauss-Legendre on [a, b] split into n panels.
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

lbm_status validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 3 || p->ny < 3) return fail(LBM_EINVAL, "lattice %d x %d: each side must be >= 3", p->nx, p->ny);
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32)
    return fail(LBM_EINVAL, "unknown precision %d", p->precision);
  // one distribution plane must stay below 4 GiB (32-bit buffer offsets)
  const unsigned long long plane_bytes = (unsigned long long)p->ny * ((p->nx + 63) / 64 * 64) *
                                         (p->precision == LBM_FP32 ? 4u : 8u);
  if (plane_bytes >= (1ull << 32))
    return fail(LBM_EINVAL, "lattice %d x %d too large: one plane is %llu bytes (limit 4 GiB)",
                p->nx, p->ny, plane_bytes);
  if (p->eos < LBM_EOS_IDEAL || p->eos > LBM_EOS_PR) return fail(LBM_EINVAL, "unknown EOS %d", p->eos);
  const double rates[4] = {p->s_e, p->s_eps, p->s_q, p->s_nu};
  for (double s : rates)
    if (!(s > 0.0 && s < 2.0)) return fail(LBM_EINVAL, "relaxation rate %g outside (0, 2)", s);
  if (!std::isfinite(p->A) || !std::isfinite(p->kappa)) return fail(LBM_EINVAL, "A or kappa not finite");
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

size_t elem_size(const lbm_params& p) { return p.precision == LBM_FP32 ? 4 : 8; }

}  // namespace

struct lbm_ctx {
  lbm_params p;
  ModelConsts m;
  Geometry g;
  size_t buf_bytes;
  void* buf[2];
  bool own_buf;
  int cur;
  hipStream_t stream;
  bool own_stream;
  int64_t step;
  bool initialized;
  // FP64 scratch for fields and observables (allocated on first use)
  double* work;      // 4 * nx*ny: rho, U, psi, out
  double* partials;  // obs_partials_count * kNumRed
  double* red;       // kNumRed + 2
};

namespace {

void set_geometry(lbm_ctx* c, int tile_x, int tile_y) {
  Geometry& g = c->g;
  g.nx = c->p.nx;
  g.ny = c->p.ny;
  g.pitch = pitch_of(c->p);
  g.plane = (long long)g.ny * g.pitch;
  g.tile_x = tile_x;
  g.tile_y = tile_y;
  g.nstrips = (g.nx + tile_x - 1) / tile_x;
  g.nrowblocks = (g.ny + tile_y - 1) / tile_y;
  g.nblocks = g.nstrips * g.nrowblocks;
}

// Default launch shape: strips as wide as the lattice allows (up to 256
// columns), row blocks sized so that the grid holds about 2048 workgroups
// (8 per CU), never fewer than 16 rows.
void default_launch(const lbm_params& p, int* tx, int* ty) {
  *tx = p.nx >= 256 ? 256 : (p.nx >= 128 ? 128 : 64);
  const int strips = (p.nx + *tx - 1) / *tx;
  const int want_rb = std::max(1, 2048 / strips);
  int rows = (p.ny + want_rb - 1) / want_rb;
  rows = std::max(rows, std::min(16, p.ny));
  *ty = rows;
}

lbm_status ensure_scratch(lbm_ctx* c) {
  if (c->work) return LBM_OK;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  HIP_TRY(hipMalloc(&c->work, 4 * n * sizeof(double)));
  HIP_TRY(hipMalloc(&c->partials, (size_t)obs_partials_count(c->g) * kNumRed * sizeof(double)));
  HIP_TRY(hipMalloc(&c->red, (kNumRed + 2) * sizeof(double)));
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
  ModelConsts& m = c->m;
  m.eos = p->eos;
  m.K = p->K; m.R = p->R; m.a = p->a; m.b = p->b;
  m.G = p->eos == LBM_EOS_IDEAL ? -1.0 : p->G;
  m.A = p->A; m.kappa = p->kappa;
  m.s_e = p->s_e; m.s_eps = p->s_eps; m.s_q = p->s_q; m.s_nu = p->s_nu;
  m.T = 0.0;
  m.aalpha = p->a;
  if (p->eos != LBM_EOS_IDEAL) {
    double Tc = 0.0;
    st = critical_temperature(*p, &Tc);
    if (st != LBM_OK) { delete c; return st; }
    m.T = p->T_over_Tc * Tc;
    if (p->eos == LBM_EOS_PR) m.aalpha = p->a * pr_alpha(p->omega_pr, p->T_over_Tc);
  }
  int tx, ty;
  default_launch(*p, &tx, &ty);
  set_geometry(c, tx, ty);
  c->buf_bytes = 9 * (size_t)c->g.plane * elem_size(*p);
  c->step = 0;
  c->cur = 0;
  c->stream = static_cast<hipStream_t>(stream);  // NULL is the HIP null stream
  c->own_stream = false;
  if (ba) {
    if (!bb || bytes < c->buf_bytes || ((uintptr_t)ba & 255) || ((uintptr_t)bb & 255)) {
      lbm_destroy(c);
      return fail(LBM_EINVAL, "caller buffers: need two 256-byte aligned buffers of %zu bytes",
                  c->buf_bytes);
    }
    c->buf[0] = ba; c->buf[1] = bb; c->own_buf = false;
  } else {
    c->own_buf = true;
    for (int i = 0; i < 2; ++i) {
      hipError_t e = hipMalloc(&c->buf[i], c->buf_bytes);
      if (e != hipSuccess) {
        lbm_destroy(c);
        return fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "hipMalloc(%zu): %s",
                    c->buf_bytes, hipGetErrorString(e));
      }
    }
  }
  // zero both buffers so the pitch padding is defined
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

size_t lbm_buffer_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  return 9 * (size_t)p->ny * pitch_of(*p) * elem_size(*p);
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
  delete c;
}

lbm_status lbm_set_launch(lbm_ctx* c, const lbm_launch* l) {
  if (!c || !l) return fail(LBM_EINVAL, "NULL argument");
  int tx = l->tile_x, ty = l->tile_y;
  int dtx, dty;
  default_launch(c->p, &dtx, &dty);
  if (tx == 0) tx = dtx;
  if (ty == 0) ty = dty;
  if (tx != 64 && tx != 128 && tx != 256) return fail(LBM_EINVAL, "tile_x %d not in {64,128,256}", tx);
  if (ty < 1) return fail(LBM_EINVAL, "tile_y %d < 1", ty);
  ty = std::min(ty, c->p.ny);
  set_geometry(c, tx, ty);
  return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_ctx* c, lbm_launch* l) {
  if (!c || !l) return fail(LBM_EINVAL, "NULL argument");
  l->tile_x = c->g.tile_x;
  l->tile_y = c->g.tile_y;
  return LBM_OK;
}

lbm_status lbm_init_field(lbm_ctx* c, const double* rho, const double* ux, const double* uy) {
  if (!c || !rho) return fail(LBM_EINVAL, "NULL argument");
  const size_t n = (size_t)c->p.nx * c->p.ny;
  for (size_t i = 0; i < n; ++i)
    if (!(rho[i] > 0.0) || !std::isfinite(rho[i]))
      return fail(LBM_ENONFINITE, "initial density %g at cell %zu", rho[i], i);
  lbm_status st = ensure_scratch(c);
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
  c->initialized = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_EINVAL, "NULL context");
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (!c->initialized) return fail(LBM_ESTATE, "lbm_step before lbm_init_field");
  for (int64_t i = 0; i < n; ++i) {
    HIP_TRY(launch_step((lbm_precision)c->p.precision, c->g, c->m, c->buf[c->cur],
                        c->buf[1 - c->cur], c->stream));
    c->cur = 1 - c->cur;
  }
  c->step += n;
  return LBM_OK;
}

lbm_status lbm_observables(lbm_ctx* c, lbm_obs* o) {
  if (!c || !o) return fail(LBM_EINVAL, "NULL argument");
  if (!c->initialized) return fail(LBM_ESTATE, "observables before lbm_init_field");
  lbm_status st = ensure_scratch(c);
  if (st != LBM_OK) return st;
  const lbm_precision prec = (lbm_precision)c->p.precision;
  const void* f = c->buf[c->cur];
  HIP_TRY(launch_density_fields(prec, c->g, c->m, f, c->work, c->stream));
  HIP_TRY(launch_observables(prec, c->g, c->m, f, c->work, c->partials, c->red, c->stream));
  const size_t n = (size_t)c->p.nx * c->p.ny;
  const size_t i_in = (size_t)(c->p.ny / 2) * c->p.nx + c->p.nx / 2;
  HIP_TRY(hipMemcpyAsync(c->red + kNumRed, c->work + i_in, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->red + kNumRed + 1, c->work, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double h[kNumRed + 2];
  HIP_TRY(hipMemcpyAsync(h, c->red, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const lbm_params& p = c->p;
  const ModelConsts& m = c->m;
  o->step = c->step;
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

lbm_status lbm_get_field(lbm_ctx* c, int32_t which, double* out) {
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  if (which < LBM_FIELD_RHO || which > LBM_FIELD_F0 + 8) return fail(LBM_EINVAL, "unknown field %d", which);
  if (!c->initialized) return fail(LBM_ESTATE, "field before lbm_init_field");
  lbm_status st = ensure_scratch(c);
  if (st != LBM_OK) return st;
  const lbm_precision prec = (lbm_precision)c->p.precision;
  const size_t n = (size_t)c->p.nx * c->p.ny;
  const void* f = c->buf[c->cur];
  double* src = c->work;
  if (which >= LBM_FIELD_F0) {
    src = c->work + 3 * n;
    HIP_TRY(launch_plane_to_f64(prec, c->g, f, which - LBM_FIELD_F0, src, c->stream));
  } else {
    HIP_TRY(launch_density_fields(prec, c->g, c->m, f, c->work, c->stream));
    if (which != LBM_FIELD_RHO) {
      src = c->work + 3 * n;
      HIP_TRY(launch_velocity_field(prec, c->g, c->m, f, c->work, which == LBM_FIELD_UX ? 0 : 1, src, c->stream));
    }
  }
  HIP_TRY(hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_save_state(lbm_ctx* c, void* buf, size_t* len) {
  if (!c || !len) return fail(LBM_EINVAL, "NULL argument");
  const size_t need = sizeof(StateHeader) + c->buf_bytes;
  if (!buf) { *len = need; return LBM_OK; }
  if (*len < need) return fail(LBM_EINVAL, "state buffer of %zu bytes, need %zu", *len, need);
  if (!c->initialized) return fail(LBM_ESTATE, "save before lbm_init_field");
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
