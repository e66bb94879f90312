/*
 * Plain FP64 CPU oracle of one time step of the D2Q9 pseudo-potential MRT
 * lattice Boltzmann model with Kupershtokh's hybrid force and the
 * pressure-tensor modification that tunes surface tension.
 *
 * TEST INFRASTRUCTURE ONLY.  It is the slow, obviously correct definition that
 * the GPU library is checked against.  It shares no source, header or table
 * with the GPU library; only the tests, the entry point's smoke check and the
 * CPU-baseline leg of the benchmark load it.
 *
 * Each step follows the paper's order and notation:
 *   1. density pass: rho = sum_a f_a, U = K p_EOS(rho) - rho/3 (Eq. 10 with
 *      c = 1, c_s^2 = 1/3), psi = sqrt(2U/G) with G < 0; psi is clamped to 0
 *      where U > 0 (counted as a domain fault);
 *   2. Kupershtokh force, Eq. (9), with omega_a = w(|e_a|^2), w(1) = 1/3,
 *      w(2) = 1/12 (Sec. 2, text under Eq. 7);
 *   3. pressure-tensor modification Q, Eq. (23), with the factor G/2 that
 *      Eq. (24)'s leading order requires;
 *   4. velocity v = (sum_a f_a e_a + F/2)/rho;
 *   5. moments m = M f, with the rows of M the D2Q9 polynomials in the order
 *      of Eq. (4): (rho, e, eps, jx, qx, jy, qy, pxx, pxy);
 *   6. collision in moment space, Eq. (25):
 *        m* = m - Lambda (m - m_eq) + (I - Lambda/2) S + C,
 *      m_eq from Eq. (4), S from Eq. (6) with its last entry read as
 *      vx Fy + vy Fx, C from Eq. (26) with its p_xx entry read as
 *      -s_nu (Qxx - Qyy);
 *   7. f* = M^{-1} m*, then streaming f_a(x + e_a, t+1) = f*_a(x, t) (Eq. 1)
 *      with periodic wrap in x and y (Sec. 3.1.1).
 *
 * Storage here is cell-major: f[(y*nx + x)*9 + a].
 * Build: gcc -O2 -fopenmp -fPIC -shared -o liboracle.so lbm_oracle.c -lm
 * OpenMP only splits rows among threads; every cell's arithmetic is the same
 * whatever the thread count, so results are bitwise independent of it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* lattice velocities e_0..e_8 */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

enum { ORC_IDEAL = 0, ORC_CS = 1, ORC_VDW = 2, ORC_PR = 3 };

typedef struct {
  int32_t nx, ny, eos, nthreads;
  double a, b, R, omega_pr, K;
  double T;      /* absolute temperature */
  double Tc;     /* critical temperature (PR alpha(T) only) */
  double A, kappa, G;
  double s_rho, s_e, s_eps, s_j, s_q, s_nu;
  /* nu_gas > 0: shear rate from nu(rho), linear in rho between rho_gas and
   * rho_liquid (clamped), s_nu = 1 / (3 nu + 1/2) (Sec. 4.2) */
  double nu_gas, nu_liquid, rho_gas, rho_liquid;
} orc_params;

/* -------------------------------------------------------------------------
 * Equation of state: K * p_EOS(rho).
 * vdW Eq. (21); PR Eq. (29); Carnahan-Starling p = rho R T (1+n+n^2-n^3)/(1-n)^3 - a rho^2,
 * n = b rho / 4; IDEAL p = rho/3 (so U = 0 and the interaction vanishes).
 * ---------------------------------------------------------------------- */
double orc_pressure(const orc_params *p, double rho) {
  double T = p->T;
  switch (p->eos) {
    case ORC_VDW:
      return p->K * (rho * p->R * T / (1.0 - p->b * rho) - p->a * rho * rho);
    case ORC_CS: {
      double n = p->b * rho / 4.0;
      double num = 1.0 + n + n * n - n * n * n;
      double den = (1.0 - n) * (1.0 - n) * (1.0 - n);
      return p->K * (rho * p->R * T * num / den - p->a * rho * rho);
    }
    case ORC_PR: {
      double w = p->omega_pr;
      double k = 0.37464 + 1.54226 * w - 0.26992 * w * w;
      double s = 1.0 + k * (1.0 - sqrt(T / p->Tc));
      double alpha = s * s;
      double b = p->b;
      return p->K * (rho * p->R * T / (1.0 - b * rho) -
                     p->a * alpha * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho));
    }
    default:
      return rho / 3.0;
  }
}

/* -------------------------------------------------------------------------
 * The transform M (rows = D2Q9 moment polynomials evaluated on e_a) and its
 * inverse M^{-1} = M^T diag(1 / |row|^2), which holds because the rows are
 * mutually orthogonal.
 * ---------------------------------------------------------------------- */
void orc_moment_matrix(double M[81], double Minv[81]) {
  for (int a = 0; a < 9; ++a) {
    double ex = EX[a], ey = EY[a];
    double c2 = ex * ex + ey * ey;
    M[0 * 9 + a] = 1.0;
    M[1 * 9 + a] = -4.0 + 3.0 * c2;
    M[2 * 9 + a] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
    M[3 * 9 + a] = ex;
    M[4 * 9 + a] = (3.0 * c2 - 5.0) * ex;
    M[5 * 9 + a] = ey;
    M[6 * 9 + a] = (3.0 * c2 - 5.0) * ey;
    M[7 * 9 + a] = ex * ex - ey * ey;
    M[8 * 9 + a] = ex * ey;
  }
  for (int k = 0; k < 9; ++k) {
    double nrm = 0.0;
    for (int a = 0; a < 9; ++a) nrm += M[k * 9 + a] * M[k * 9 + a];
    for (int a = 0; a < 9; ++a) Minv[a * 9 + k] = M[k * 9 + a] / nrm;
  }
}

/* -------------------------------------------------------------------------
 * Step 1: density pass over the whole lattice.
 * Returns the number of cells with U > 0 (psi clamped) in *n_domain and of
 * cells with rho <= 0 or a non-finite rho in *n_bad.
 * ---------------------------------------------------------------------- */
static void density_pass(const orc_params *p, const double *f, double *rho, double *U,
                         double *psi, int64_t *n_domain, int64_t *n_bad) {
  const int64_t ncell = (int64_t)p->nx * p->ny;
  int64_t nd = 0, nb = 0;
  for (int64_t c = 0; c < ncell; ++c) {
    double r = 0.0;
    for (int a = 0; a < 9; ++a) r += f[c * 9 + a];
    double u = orc_pressure(p, r) - r / 3.0;
    double s = 2.0 * u / p->G;
    rho[c] = r;
    U[c] = u;
    psi[c] = sqrt(s > 0.0 ? s : 0.0);
    if (!(u <= 0.0)) ++nd;
    if (!(r > 0.0) || !isfinite(r)) ++nb;
  }
  if (n_domain) *n_domain = nd;
  if (n_bad) *n_bad = nb;
}

static inline int64_t wrap_index(const orc_params *p, int x, int y) {
  x %= p->nx;
  if (x < 0) x += p->nx;
  y %= p->ny;
  if (y < 0) y += p->ny;
  return (int64_t)y * p->nx + x;
}

/* Interaction weights omega_a = w(|e_a|^2). */
static double omega_w(int a) {
  int c2 = EX[a] * EX[a] + EY[a] * EY[a];
  if (c2 == 1) return 1.0 / 3.0;
  if (c2 == 2) return 1.0 / 12.0;
  return 0.0;
}

/* -------------------------------------------------------------------------
 * Steps 2-3 at one cell: force (Eq. 9) and tensor Q (Eq. 23 times G/2).
 * ---------------------------------------------------------------------- */
static void interaction_at(const orc_params *p, const double *U, const double *psi, int x, int y,
                           double *Fx, double *Fy, double *Qxx, double *Qyy, double *Qxy) {
  const int64_t c = (int64_t)y * p->nx + x;
  double sUx = 0.0, sUy = 0.0, sPx = 0.0, sPy = 0.0;
  double qxx = 0.0, qyy = 0.0, qxy = 0.0;
  for (int a = 0; a < 9; ++a) {
    int64_t n = wrap_index(p, x + EX[a], y + EY[a]);
    double w = omega_w(a);
    sUx += w * U[n] * EX[a];
    sUy += w * U[n] * EY[a];
    sPx += w * psi[n] * EX[a];
    sPy += w * psi[n] * EY[a];
    double bracket = (1.0 - p->A) * (p->G / 2.0) * psi[c] * (psi[n] - psi[c]) +
                     (p->A / 2.0) * (U[n] - U[c]);
    qxx += w * bracket * EX[a] * EX[a];
    qyy += w * bracket * EY[a] * EY[a];
    qxy += w * bracket * EX[a] * EY[a];
  }
  *Fx = -p->A * sUx - (1.0 - p->A) * p->G * psi[c] * sPx;
  *Fy = -p->A * sUy - (1.0 - p->A) * p->G * psi[c] * sPy;
  *Qxx = p->kappa * qxx;
  *Qyy = p->kappa * qyy;
  *Qxy = p->kappa * qxy;
}

/* -------------------------------------------------------------------------
 * Steps 4-7 at one cell (without the streaming): f_in[9] -> f_out[9].
 * ---------------------------------------------------------------------- */
static void collide(const orc_params *p, const double *M, const double *Minv, const double f[9],
                    double Fx, double Fy, double Qxx, double Qyy, double Qxy, double out[9]) {
  double rho = 0.0, jx = 0.0, jy = 0.0;
  for (int a = 0; a < 9; ++a) {
    rho += f[a];
    jx += f[a] * EX[a];
    jy += f[a] * EY[a];
  }
  double vx = (jx + 0.5 * Fx) / rho;
  double vy = (jy + 0.5 * Fy) / rho;
  double v2 = vx * vx + vy * vy;
  double m[9];
  for (int k = 0; k < 9; ++k) {
    m[k] = 0.0;
    for (int a = 0; a < 9; ++a) m[k] += M[k * 9 + a] * f[a];
  }
  double meq[9] = {rho,           rho * (-2.0 + 3.0 * v2), rho * (1.0 - 3.0 * v2),
                   rho * vx,      -rho * vx,               rho * vy,
                   -rho * vy,     rho * (vx * vx - vy * vy), rho * vx * vy};
  double vF = vx * Fx + vy * Fy;
  double S[9] = {0.0, 6.0 * vF, -6.0 * vF, Fx, -Fx, Fy, -Fy,
                 2.0 * (vx * Fx - vy * Fy), vx * Fy + vy * Fx};
  double s_nu = p->s_nu;
  if (p->nu_gas > 0.0) {
    double frac = (rho - p->rho_gas) / (p->rho_liquid - p->rho_gas);
    if (frac < 0.0) frac = 0.0;
    if (frac > 1.0) frac = 1.0;
    double nu = p->nu_gas + frac * (p->nu_liquid - p->nu_gas);
    s_nu = 1.0 / (3.0 * nu + 0.5);
  }
  double s[9] = {p->s_rho, p->s_e, p->s_eps, p->s_j, p->s_q, p->s_j, p->s_q, s_nu, s_nu};
  double C[9] = {0.0, 1.5 * p->s_e * (Qxx + Qyy), 0.0, 0.0, 0.0, 0.0, 0.0,
                 -s_nu * (Qxx - Qyy), -s_nu * Qxy};
  double ms[9];
  for (int k = 0; k < 9; ++k)
    ms[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * S[k] + C[k];
  for (int a = 0; a < 9; ++a) {
    out[a] = 0.0;
    for (int k = 0; k < 9; ++k) out[a] += Minv[a * 9 + k] * ms[k];
  }
}

void orc_collide_cell(const orc_params *p, const double f[9], double Fx, double Fy, double Qxx,
                      double Qyy, double Qxy, double out[9]) {
  double M[81], Minv[81];
  orc_moment_matrix(M, Minv);
  collide(p, M, Minv, f, Fx, Fy, Qxx, Qyy, Qxy, out);
}

static int thread_count(const orc_params *p) { return p->nthreads > 0 ? p->nthreads : 1; }

/* -------------------------------------------------------------------------
 * One full step on the lattice: f_in (time n) -> f_out (time n+1).
 * work must hold 3*nx*ny doubles.  Returns the fault counts of the density pass.
 * ---------------------------------------------------------------------- */
void orc_step(const orc_params *p, const double *f_in, double *f_out, double *work,
              int64_t *n_domain, int64_t *n_bad) {
  const int64_t ncell = (int64_t)p->nx * p->ny;
  double *rho = work, *U = work + ncell, *psi = work + 2 * ncell;
  double M[81], Minv[81];
  orc_moment_matrix(M, Minv);
  density_pass(p, f_in, rho, U, psi, n_domain, n_bad);
#pragma omp parallel for schedule(static) num_threads(thread_count(p))
  for (int y = 0; y < p->ny; ++y) {
    for (int x = 0; x < p->nx; ++x) {
      const int64_t c = (int64_t)y * p->nx + x;
      double Fx, Fy, Qxx, Qyy, Qxy, post[9];
      interaction_at(p, U, psi, x, y, &Fx, &Fy, &Qxx, &Qyy, &Qxy);
      collide(p, M, Minv, f_in + c * 9, Fx, Fy, Qxx, Qyy, Qxy, post);
      for (int a = 0; a < 9; ++a) f_out[wrap_index(p, x + EX[a], y + EY[a]) * 9 + a] = post[a];
    }
  }
}

/* n steps in place on f (cell-major); scratch is 9*nx*ny + 3*nx*ny doubles.
 * Fault counts are summed over the steps. */
void orc_run(const orc_params *p, double *f, int64_t nsteps, double *scratch, int64_t *n_domain,
             int64_t *n_bad) {
  const int64_t ncell = (int64_t)p->nx * p->ny;
  double *g = scratch, *work = scratch + 9 * ncell;
  int64_t nd_sum = 0, nb_sum = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    int64_t nd = 0, nb = 0;
    orc_step(p, f, g, work, &nd, &nb);
    memcpy(f, g, sizeof(double) * 9 * ncell);
    nd_sum += nd;
    nb_sum += nb;
  }
  if (n_domain) *n_domain = nd_sum;
  if (n_bad) *n_bad = nb_sum;
}

/* f_a = W_a rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2], the second-order
 * equilibrium whose moments are Eq. (4). u arrays may be NULL (zero). */
void orc_init_equilibrium(const orc_params *p, const double *rho, const double *ux,
                          const double *uy, double *f) {
  const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const int64_t ncell = (int64_t)p->nx * p->ny;
  for (int64_t c = 0; c < ncell; ++c) {
    double u = ux ? ux[c] : 0.0, v = uy ? uy[c] : 0.0;
    for (int a = 0; a < 9; ++a) {
      double eu = EX[a] * u + EY[a] * v;
      f[c * 9 + a] = W[a] * rho[c] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * (u * u + v * v));
    }
  }
}

/* Interaction fields of a density field: U, psi, F and Q per cell. */
void orc_interaction(const orc_params *p, const double *rho, double *U, double *psi, double *Fx,
                     double *Fy, double *Qxx, double *Qyy, double *Qxy) {
  const int64_t ncell = (int64_t)p->nx * p->ny;
  for (int64_t c = 0; c < ncell; ++c) {
    double u = orc_pressure(p, rho[c]) - rho[c] / 3.0;
    double s = 2.0 * u / p->G;
    U[c] = u;
    psi[c] = sqrt(s > 0.0 ? s : 0.0);
  }
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      const int64_t c = (int64_t)y * p->nx + x;
      interaction_at(p, U, psi, x, y, &Fx[c], &Fy[c], &Qxx[c], &Qyy[c], &Qxy[c]);
    }
}

/* Macroscopic fields of a state: rho, v = (sum f e + F/2)/rho, and F. */
void orc_fields(const orc_params *p, const double *f, double *rho, double *ux, double *uy,
                double *Fx, double *Fy) {
  const int64_t ncell = (int64_t)p->nx * p->ny;
  double *U = (double *)malloc(sizeof(double) * ncell * 5);
  double *psi = U + ncell, *Qxx = U + 2 * ncell, *Qyy = U + 3 * ncell, *Qxy = U + 4 * ncell;
  for (int64_t c = 0; c < ncell; ++c) {
    double r = 0.0;
    for (int a = 0; a < 9; ++a) r += f[c * 9 + a];
    rho[c] = r;
  }
  orc_interaction(p, rho, U, psi, Fx, Fy, Qxx, Qyy, Qxy);
  for (int64_t c = 0; c < ncell; ++c) {
    double jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
      jx += f[c * 9 + a] * EX[a];
      jy += f[c * 9 + a] * EY[a];
    }
    ux[c] = (jx + 0.5 * Fx[c]) / rho[c];
    uy[c] = (jy + 0.5 * Fy[c]) / rho[c];
  }
  free(U);
}

/*
 * Observables of a state (Sec. 3.1.1, Eq. 22), in plain sequential sums:
 * out[0] mass = sum rho, out[1..2] momentum sum (j + F/2), out[3..4] rho min/max,
 * out[5] rho_in = rho at (nx/2, ny/2), out[6] rho_out = rho at (0, 0),
 * out[7..8] p_in, p_out = K p_EOS, out[9] dp = p_in - p_out,
 * out[10] R_e = sqrt(sum (rho - rho_out) / (rho_in - rho_out) / pi),
 * out[11] sigma = dp * R_e (Laplace law), out[12] max |v|,
 * out[13] count of U > 0, out[14] count of rho <= 0 or non-finite.
 */
void orc_observables(const orc_params *p, const double *f, double out[15]) {
  const int64_t ncell = (int64_t)p->nx * p->ny;
  double *rho = (double *)malloc(sizeof(double) * ncell * 5);
  double *ux = rho + ncell, *uy = rho + 2 * ncell, *Fx = rho + 3 * ncell, *Fy = rho + 4 * ncell;
  orc_fields(p, f, rho, ux, uy, Fx, Fy);
  double mass = 0.0, mx = 0.0, my = 0.0, rmin = INFINITY, rmax = -INFINITY, umax = 0.0;
  int64_t nd = 0, nb = 0;
  for (int64_t c = 0; c < ncell; ++c) {
    mass += rho[c];
    mx += rho[c] * ux[c];
    my += rho[c] * uy[c];
    if (rho[c] < rmin) rmin = rho[c];
    if (rho[c] > rmax) rmax = rho[c];
    double sp = sqrt(ux[c] * ux[c] + uy[c] * uy[c]);
    if (sp > umax) umax = sp;
    double u = orc_pressure(p, rho[c]) - rho[c] / 3.0;
    if (!(u <= 0.0)) ++nd;
    if (!(rho[c] > 0.0) || !isfinite(rho[c])) ++nb;
  }
  double rin = rho[(int64_t)(p->ny / 2) * p->nx + p->nx / 2];
  double rout = rho[0];
  double pin = orc_pressure(p, rin), pout = orc_pressure(p, rout);
  double excess = 0.0;
  for (int64_t c = 0; c < ncell; ++c) excess += rho[c] - rout;
  double Re = sqrt(excess / (rin - rout) / M_PI);
  out[0] = mass;
  out[1] = mx;
  out[2] = my;
  out[3] = rmin;
  out[4] = rmax;
  out[5] = rin;
  out[6] = rout;
  out[7] = pin;
  out[8] = pout;
  out[9] = pin - pout;
  out[10] = Re;
  out[11] = (pin - pout) * Re;
  out[12] = umax;
  out[13] = (double)nd;
  out[14] = (double)nb;
  free(rho);
}
