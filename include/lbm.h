/*
 * lbm.h -- C ABI of liblbm, the MI355X (gfx950) implementation of one time
 * step of the D2Q9 pseudo-potential multiple-relaxation-time lattice
 * Boltzmann model with Kupershtokh's hybrid interaction force and the
 * pressure-tensor modification that tunes surface tension independently of
 * the coexistence densities (Hu, Li & Uddin, arXiv 1412.7228).
 *
 * One step (Sec. 2 Eq. 1-10, Sec. 3.2.1 Eq. 23-26):
 *   rho = sum_a f_a;  U = K p_EOS(rho; T) - rho/3;  psi = sqrt(2U/G)      (Eq. 10)
 *   F = -A sum_a w_a U(x+e_a) e_a - (1-A) G psi(x) sum_a w_a psi(x+e_a) e_a  (Eq. 9)
 *   Q = kappa sum_a w_a [(1-A)(G/2) psi (psi(x+e_a)-psi) + (A/2)(U(x+e_a)-U)] e_a e_a (Eq. 23)
 *   v = (sum_a f_a e_a + F/2) / rho
 *   m* = m - Lambda (m - m_eq(rho, v)) + (I - Lambda/2) S(v, F) + C(Q)      (Eq. 25)
 *   f_a(x + e_a, t+1) = (M^{-1} m*)_a(x, t)                                  (Eq. 1)
 * with w = 1/3 (axis) and 1/12 (diagonal) (Sec. 2, under Eq. 7), m_eq of
 * Eq. (4), S of Eq. (6) and C of Eq. (26), on a lattice periodic in x and y
 * (Sec. 3.1.1).  The readings of the printed equations that this library
 * implements: the last entry of S is vx Fy + vy Fx; the p_xx entry of C is
 * -s_nu (Qxx - Qyy); Q carries the factor G/2 that Eq. (24) implies; psi is
 * set to 0 where U > 0 (such cells are counted as domain faults).
 *
 * Conventions for every function:
 *  - Return value: lbm_status, LBM_OK = 0, negative on error.  No function
 *    aborts or prints; lbm_last_error() gives a message for the calling thread.
 *  - Host arrays are double precision, nx*ny values, row-major [y][x]
 *    (x fastest); they are read or written during the call and stay owned by
 *    the caller.
 *  - Device state: two distribution buffers (A/B), each ny lattice rows of
 *    9 * pitch elements (pitch = nx rounded up to 64): row y holds the rows
 *    of the nine distribution planes back to back, so element (a, y, x) is at
 *    (9 * y + a) * pitch + x (plane stride pitch, row stride 9 * pitch; a
 *    row's update reads three such runs instead of 27 separate plane rows).
 *    Element type double (LBM_FP64) or float (LBM_FP32), plane index a = 0..8 in the
 *    velocity order e_0=(0,0), e_1=(1,0), e_2=(0,1), e_3=(-1,0), e_4=(0,-1),
 *    e_5=(1,1), e_6=(-1,1), e_7=(-1,-1), e_8=(1,-1).  A buffer holds the
 *    post-collision distributions of the previous step before streaming (the
 *    step kernel streams by pulling), so f_a(x, y) of the current state is
 *    the element (x - e_ax, y - e_ay) (periodic) of plane a.  Every host-side
 *    value (fields, distributions, observables, initial data) is the streamed
 *    state f(x, t) of Eq. (1).
 *  - All device work is enqueued on the context's HIP stream; lbm_step is
 *    asynchronous, every read-back call synchronises that stream.
 *  - A context is used by one host thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* an argument or parameter is out of range            */
  LBM_ENOMEM = -2,     /* a device or host allocation failed                  */
  LBM_EDEVICE = -3,    /* a HIP runtime call failed                           */
  LBM_ENONFINITE = -4, /* a density that is not finite or not positive        */
  LBM_EDOMAIN = -5,    /* U > 0 somewhere: psi = sqrt(2U/G) is not real       */
  LBM_ESTATE = -6      /* call out of order (e.g. step before init)           */
} lbm_status;

typedef enum {
  LBM_EOS_IDEAL = 0, /* p = rho/3, so U = 0: no interaction force, no Q            */
  LBM_EOS_CS = 1,    /* Carnahan-Starling: rho R T (1+n+n^2-n^3)/(1-n)^3 - a rho^2, n = b rho/4 */
  LBM_EOS_VDW = 2,   /* van der Waals, Eq. (21): rho R T/(1 - b rho) - a rho^2      */
  LBM_EOS_PR = 3     /* Peng-Robinson, Eq. (29), acentric factor omega_pr          */
} lbm_eos;

typedef enum { LBM_FP64 = 0, LBM_FP32 = 1 } lbm_precision;

typedef enum {
  LBM_FIELD_RHO = 0, /* density                                  */
  LBM_FIELD_UX = 1,  /* velocity (sum f e + F/2)/rho, x component */
  LBM_FIELD_UY = 2,  /* y component                               */
  LBM_FIELD_F0 = 3   /* distribution f_a is LBM_FIELD_F0 + a, a = 0..8 */
} lbm_field;

/* Distribution planes of the D2Q9 state: element (a, y, x) of a buffer is at
 * (LBM_Q * y + a) * pitch + x. */
#define LBM_Q 9

/* Problem statement: lattice size (Sec. 3.1.1), EOS and temperature
 * (Eq. 21, Eq. 29), mixing parameter A (Eq. 9), pressure-tensor
 * coefficient kappa (Eq. 23), relaxation rates (Eq. 2). */
typedef struct {
  int32_t nx, ny;     /* periodic lattice, each >= 3; ny * pitch elements (one
                         plane's worth) and 9 * pitch elements (one lattice row of
                         the nine planes) must each stay below 4 GiB                */
  int32_t eos;        /* lbm_eos                                                    */
  int32_t precision;  /* lbm_precision: element type of the distributions           */
  double a, b, R;     /* EOS constants (b*rho must stay below 1 for vdW/PR, 4 for CS) */
  double omega_pr;    /* Peng-Robinson acentric factor                              */
  double K;           /* multiplies the whole EOS pressure (Eq. 21), > 0            */
  double T_over_Tc;   /* temperature in units of the EOS's critical temperature     */
  double A;           /* Kupershtokh mixing parameter, Eq. (9)                      */
  double kappa;       /* pressure-tensor coefficient, Eq. (23)                      */
  double G;           /* interaction strength, < 0; results do not depend on it     */
  double s_e, s_eps, s_q, s_nu; /* MRT rates 1/tau of Eq. (2), each in (0, 2);
                                   s_rho and s_j do not enter (conserved moments)   */
  /* Density-dependent shear viscosity (Sec. 4.2 gives gas and liquid values):
   * with nu_gas > 0, each cell uses s_nu = 1 / (3 nu + 1/2) with
   * nu = nu_gas + f (nu_liquid - nu_gas), f = (rho - rho_gas) / (rho_liquid - rho_gas)
   * clamped to [0, 1], in place of the constant s_nu (also in the C source).
   * nu_gas = 0 (default) keeps the constant s_nu. */
  double nu_gas, nu_liquid, rho_gas, rho_liquid;
} lbm_params;

/* FP64 observables of the current state (Sec. 3.1.1, Eq. 22).
 * rho_in is rho at (nx/2, ny/2), rho_out at (0, 0); p = K p_EOS(rho);
 * dp = p_in - p_out; R_e = sqrt(sum(rho - rho_out) / (rho_in - rho_out) / pi)
 * (equimolar radius); sigma = dp * R_e (Laplace law); max_u = max |v|. */
typedef struct {
  int64_t step;
  double mass, mom_x, mom_y, rho_min, rho_max, rho_in, rho_out;
  double p_in, p_out, dp, R_e, sigma, max_u;
  int64_t n_nonfinite; /* cells with a non-finite or non-positive density */
  int64_t n_domain;    /* cells with U > 0                                */
} lbm_obs;

/* Launch shape of the fused step kernel: a workgroup owns a strip of
 * tile_x columns and marches over tile_y rows.
 *   steps_per_pass = 1: one time step per launch; tile_x in {64, 128, 256}.
 *   steps_per_pass = 2: two time steps per launch (each pass reads and writes
 *     the state once; bitwise the same states as single steps); tile_x in
 *     {128, 256}, of which tile_x - 6 columns are stored per strip.  An odd
 *     step count ends with one single-step launch of the default shape.
 * tile_y >= 1.  0 in a tile field selects the library default for the
 * lattice; steps_per_pass 0 selects 2, or 1 with tile_x = 64.  New contexts
 * start with two steps per pass and the default two-step shape: 256-lane
 * strips of 16 rows (FP32) where they give at least 8 workgroups per CU,
 * else 128-lane strips of 16 down to 8 rows; FP64 lattices at least 250
 * columns wide take 256-lane row blocks (8 to 72 rows) that fill a whole
 * number of waves of the device (two such workgroups per CU). */
typedef struct {
  int32_t tile_x, tile_y;
  int32_t steps_per_pass;
} lbm_launch;

typedef struct lbm_ctx lbm_ctx;

/* Fills *p with: 64 x 64, CS (a=1, b=4, R=1), K=1, T/Tc=0.8, A=-0.5,
 * kappa=0, G=-1, s_e=s_eps=s_nu=1, s_q=8/7, constant viscosity, FP64.
 * Returns LBM_EINVAL on NULL. */
lbm_status lbm_params_default(lbm_params* p);

/* Critical temperature of the EOS in *p (K does not change it); *Tc receives it.
 * LBM_EINVAL for an unknown EOS, IDEAL or non-positive constants. */
lbm_status lbm_critical_temperature(const lbm_params* p, double* Tc);

/* Maxwell equal-area coexistence densities of the EOS in *p at T_over_Tc
 * (0 < T/Tc < 1; K does not change them), for initial fields.  The model's
 * own steady densities deviate from these by the A-dependent amount of
 * Eq. (17).  LBM_EINVAL for IDEAL, T/Tc outside (0, 1) or no bracket. */
lbm_status lbm_coexistence(const lbm_params* p, double* rho_v, double* rho_l);

/* Laplace law over several drops (Eq. 22; the test of Sec. 3.1.1 and Sec. 4.1):
 * the least-squares slope through the origin of dp against 1/R_e,
 *   *sigma = sum(dp_i / R_i) / sum(1 / R_i^2),
 * and, if spread is not NULL, the relative spread of dp_i R_i over the drops,
 *   *spread = (max - min) / |mean|.
 * dp, R_e: n host doubles each (the lbm_obs fields of the same names), read
 * only, owned by the caller.  Host arithmetic in FP64; no device use.
 * LBM_EINVAL on NULL dp, R_e or sigma, n < 1, or a drop with R_e <= 0 or a
 * non-finite dp or R_e (outputs then unchanged). */
lbm_status lbm_laplace_fit(const double* dp, const double* R_e, int32_t n, double* sigma, double* spread);

/* Bytes of one distribution buffer for these parameters (0 if invalid). */
size_t lbm_buffer_bytes(const lbm_params* p);

/* Creates a context: validates *p, allocates both distribution buffers
 * (hipMalloc) and small scratch.  hip_stream is the hipStream_t on which all
 * of the context's device work is enqueued; NULL is the HIP null stream.  The
 * stream stays owned by the caller.  *out receives the context.
 * Errors: LBM_EINVAL (parameters), LBM_ENOMEM, LBM_EDEVICE. */
lbm_status lbm_create(const lbm_params* p, void* hip_stream, lbm_ctx** out);

/* As lbm_create, but the caller provides the two distribution buffers
 * (device pointers, each at least lbm_buffer_bytes(p) bytes, 256-byte
 * aligned); they stay owned by the caller and must outlive the context. */
lbm_status lbm_create_ext(const lbm_params* p, void* hip_stream, void* buf_a, void* buf_b,
                          size_t buf_bytes, lbm_ctx** out);

/* Releases everything the context owns (not caller buffers).  NULL is a no-op. */
void lbm_destroy(lbm_ctx* ctx);

/* Sets the launch shape of later steps (see lbm_launch). LBM_EINVAL if invalid. */
lbm_status lbm_set_launch(lbm_ctx* ctx, const lbm_launch* launch);
lbm_status lbm_get_launch(const lbm_ctx* ctx, lbm_launch* launch);

/* Initial state f_a = W_a rho [1 + 3 e.u + 4.5 (e.u)^2 - 1.5 u^2] (moments
 * of Eq. 4), W = 4/9, 1/9, 1/36.  rho is required, ux/uy may be NULL (zero).
 * Resets the step counter.  LBM_ENONFINITE if a density is not finite or <= 0. */
lbm_status lbm_init_field(lbm_ctx* ctx, const double* rho, const double* ux, const double* uy);

/* Sets the distributions directly from a host array f[a][y][x] (9*nx*ny
 * doubles, owned by the caller; copied before return), rounded to the context
 * precision.  Resets the step counter.  LBM_EINVAL on NULL. */
lbm_status lbm_set_distributions(lbm_ctx* ctx, const double* f);

/* Enqueues n >= 0 time steps of the update above (Eq. 1 with the force of
 * Eq. 9, the term of Eq. 23 and the collision of Eq. 25, Sec. 2 and
 * Sec. 3.2.1) on the context stream and returns.  With two
 * steps per pass, each run of 64 two-step launches is a replay of a HIP graph
 * captured on a stream of the context's own (kernels only; cached per starting
 * buffer and launch shape) and the remaining launches go one by one; the
 * states are bitwise those of the launches issued one by one.  LBM_EINVAL for
 * n < 0; LBM_ESTATE before the state is initialised or while a row-range
 * launch (lbm_step_rows) is open; numerical faults surface at the next
 * lbm_observables. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* Flag of lbm_step_rows: more row ranges of the same steps follow. */
enum { LBM_ROWS_MORE = 1 };

/* One launch of the same time step (Eqs. 1, 9, 23, 25) that updates only the
 * rows [y_begin, y_begin + rows) of the lattice: n = 1 step, or n = 2 steps
 * when the context runs two steps per pass (lbm_launch.steps_per_pass).  The
 * launch reads the current state's rows within 2n of the range (periodic in
 * y, as lbm_step) and writes the range into the other buffer, which then
 * becomes current and the step count advances by n; rows outside the range
 * keep whatever that buffer held (the state of an earlier launch).
 * flags = LBM_ROWS_MORE: the launch is one range of several for the same n
 * steps; the source buffer stays current, and the call without the flag that
 * ends the sequence makes the destination current.  While such a sequence is
 * open, lbm_step, lbm_set_launch and lbm_save_state return LBM_ESTATE and
 * another n returns LBM_EINVAL (init, set_distributions and load_state end it).
 * The paper's lattice is one periodic domain; this entry point is what a
 * y-slab decomposition of it needs: a slab of h rows is a context of h + 4n
 * rows whose first and last 2n rows are ghost rows, updated with
 * (n, 2n, h, 0) and refreshed from the neighbouring slabs' current buffers
 * (lbm_state_info) before the next call; or, to overlap that refresh, first
 * the rows that read no ghost row, (n, 4n, h - 4n, LBM_ROWS_MORE), then the
 * two ranges next to the ghost rows once they have arrived.  LBM_EINVAL for
 * n outside {1, 2}, n = 2 with one step per pass, rows < 1, a range outside
 * [0, ny) or unknown flags; LBM_ESTATE before the state is initialised. */
lbm_status lbm_step_rows(lbm_ctx* ctx, int32_t n, int32_t y_begin, int32_t rows, int32_t flags);

/* Computes the observables in FP64 on the device (deterministic reduction
 * order), synchronises and fills *out.  Returns LBM_ENONFINITE or
 * LBM_EDOMAIN (after filling *out) if the state holds such cells. */
lbm_status lbm_observables(lbm_ctx* ctx, lbm_obs* out);

/* lbm_observables for callers that cannot allocate device memory (code run
 * between HIP graph captures, tight serving loops, harnesses that forbid
 * hipMalloc): the same FP64 observables, bitwise, with nothing allocated by
 * the call or lazily for it.  It keeps no per-cell field arrays (each cell's
 * neighbourhood is recomputed from the distributions) and puts its partial
 * sums in a file-scope device array of the library: 4 MiB on each GPU it runs
 * on, held until the process ends, shared by every context on that GPU and
 * keeping the last call's contents (every call overwrites what it reads).
 * Calls that overlapped on one GPU would race on that array; the library
 * serialises its own calls with a process-wide lock held until the call's
 * stream has finished with the array.  Synchronises the context stream.
 * Errors: LBM_EINVAL on NULL or for a lattice of more than
 * lbm_noalloc_max_cells() cells (checked first), LBM_ESTATE before the state
 * is initialised, LBM_EDEVICE if a HIP call fails; LBM_ENONFINITE and
 * LBM_EDOMAIN as lbm_observables (after filling *out). */
lbm_status lbm_observables_noalloc(lbm_ctx* ctx, lbm_obs* out);
/* Largest lattice (nx * ny) that lbm_observables_noalloc accepts: 2^28. */
int64_t lbm_noalloc_max_cells(void);

/* Copies one field (lbm_field) of the current state to host out[y][x] in FP64
 * (nx*ny doubles, owned by the caller); synchronises the context stream.
 * LBM_EINVAL for an unknown field or NULL, LBM_ESTATE before the state is
 * initialised. */
lbm_status lbm_get_field(lbm_ctx* ctx, int32_t which, double* out);

/* Checkpoint: *len receives the byte size when buf is NULL; otherwise buf
 * (of *len bytes, host memory owned by the caller) receives a header (sizes,
 * precision, step, parameter hash) followed by the raw distribution buffer
 * (LBM_EINVAL if *len is too small, LBM_ESTATE before the state is
 * initialised or while a row-range launch is open).  lbm_load_state restores
 * such a blob into a context with the same parameters (LBM_EINVAL otherwise);
 * both synchronise the context stream.  A saved and reloaded run continues
 * bitwise as if uninterrupted. */
lbm_status lbm_save_state(lbm_ctx* ctx, void* buf, size_t* len);
lbm_status lbm_load_state(lbm_ctx* ctx, const void* buf, size_t len);

/* Waits for the context stream (LBM_EDEVICE if a HIP call failed). */
lbm_status lbm_sync(lbm_ctx* ctx);

/* Current step count, the device pointer of the buffer that holds the
 * current state and its plane row pitch in elements (for callers that time
 * or inspect the device state; layout [ny][9][pitch]: element (a, y, x) at
 * (9 * y + a) * pitch + x, post-collision values before streaming).  Each
 * output may be NULL.  The buffer stays owned by the context (or the
 * caller, after lbm_create_ext) and stops being current at the next step. */
lbm_status lbm_state_info(const lbm_ctx* ctx, int64_t* step, const void** f_cur, int32_t* pitch);

/* ---------------------------------------------------------------------------
 * Batched engine: n independent periodic lattices (e.g. Laplace-test droplets
 * of uneven sizes and parameters) advanced together.  Every domain runs the
 * same per-tile step as lbm_step.  All domains share the EOS kind and the
 * precision; lattice size and all other parameters are per domain.
 * ------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

typedef enum {
  LBM_BATCH_PERSISTENT = 0, /* one launch advances all domains by the n / 2 pairs of steps
                               of a call (two-step passes; an odd n ends with one
                               single-step launch).  The domains are split into one group
                               per XCD; the workgroups on an XCD take that group's tiles
                               pair by pair from a queue, and a tile waits for its
                               domain's previous pair at a per-domain barrier (bounded
                               wait; a wait past the spin limit aborts the launch, which
                               lbm_batch_sync reports).  Bitwise the states of the
                               per-step mode with the same tiles */
  LBM_BATCH_PER_STEP = 1    /* one launch per step (or per two fused steps) over all
                               tiles, the launches of a call captured in a HIP graph */
} lbm_batch_mode;

typedef struct {
  int32_t mode;             /* lbm_batch_mode                                         */
  int32_t tile_x, tile_y;   /* tile of every domain; 0 = default (256 x 16 with two
                               steps per launch, 256 x 24 in the persistent mode,
                               64 x 32 with one step per launch)                      */
  int64_t spin_limit;       /* persistent mode: polls before a barrier wait gives up;
                               0 = default (2^20, about a second)                      */
  int32_t force_spin_limit; /* non-zero with spin_limit 0: use 0 (test of the abort path) */
  /* filled by lbm_batch_get_launch: */
  int32_t grid;             /* workgroups per launch                                  */
  int32_t ntiles;           /* tiles over all domains                                 */
  int32_t resident_per_cu;  /* persistent mode: workgroups one CU holds at once       */
  /* input again: */
  int32_t steps_per_pass;   /* 1, or 2 = two fused steps per pass as in lbm_launch
                               (tile_x in {128, 256}; an odd count ends with one
                               single-step launch); 0 = 2 unless tile_x is 64.  The
                               persistent mode needs 2                                  */
} lbm_batch_launch;

/* Creates a batch of n domains with parameters params[0..n).  Allocates one
 * arena for all distribution buffers.  hip_stream as in lbm_create; on a
 * non-NULL stream the steps of one lbm_batch_step call are enqueued as one
 * HIP graph launch (the persistent mode's counter reset + launch, or all the
 * per-step launches of up to 32,768 steps; the graph is cached for the next
 * call with the same step count), on the null stream as plain launches.
 * LBM_EINVAL if a domain's parameters are invalid or the EOS kinds or
 * precisions differ. Default launch: LBM_BATCH_PER_STEP with two steps per
 * launch, 256 x 16 tiles. */
lbm_status lbm_batch_create(const lbm_params* params, int32_t n, void* hip_stream, lbm_batch** out);
void lbm_batch_destroy(lbm_batch* b);

/* Chooses the launch mode and tile shape (re-plans the tiles and, in
 * persistent mode, their grouping by XCD and a grid no larger than the GPU
 * holds at once).  LBM_EINVAL for an invalid choice, e.g. the persistent mode
 * with one step per pass or 64-lane tiles (the batch then keeps its previous
 * launch); LBM_ENOMEM or LBM_EDEVICE if the new tile lists cannot be placed on
 * the device, after which lbm_batch_step refuses to run until a later call
 * succeeds. */
lbm_status lbm_batch_set_launch(lbm_batch* b, const lbm_batch_launch* launch);
lbm_status lbm_batch_get_launch(const lbm_batch* b, lbm_batch_launch* launch);

/* Initial state of domain i, as lbm_init_field (host arrays of that domain's size). */
lbm_status lbm_batch_init_field(lbm_batch* b, int32_t i, const double* rho, const double* ux,
                                const double* uy);

/* Enqueues n steps of every domain (asynchronous).  LBM_EINVAL for n < 0;
 * LBM_ESTATE if a domain is not initialised or the batch has no launch layout
 * (a failed lbm_batch_set_launch). */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* Waits for the batch; LBM_EDEVICE if a persistent launch aborted (a barrier
 * wait exceeded the spin limit; the state is then not a whole step). */
lbm_status lbm_batch_sync(lbm_batch* b);

/* Observables of every domain into out[0..n) (as lbm_observables); returns the
 * first fault status after filling all entries. */
lbm_status lbm_batch_observables(lbm_batch* b, lbm_obs* out);

/* One field of domain i, as lbm_get_field. */
lbm_status lbm_batch_get_field(lbm_batch* b, int32_t i, int32_t which, double* out);

/* ---------------------------------------------------------------------------
 * Surrogate network: (A, kappa, T/Tc) -> (sigma, rho_l, rho_v), each
 * normalised by the caller.  3 -> 128 -> 128 -> 128 -> 3, tanh on the hidden
 * layers, linear output; 33,923 parameters in one flat FP32 vector in the
 * order W1 [128x3], b1, W2 [128x128], b2, W3 [128x128], b3, W4 [3x128], b4
 * (W is [out, in], row-major).  The weights are used rounded to bfloat16
 * (nearest, ties to even) from the FP32 master copy; biases, activations and
 * accumulation are FP32.  Training is full-batch Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) on the mean squared error over the 3 outputs.  Host
 * arrays are float, n x 3, row-major.
 * ------------------------------------------------------------------------- */
typedef struct lbm_mlp lbm_mlp;

int32_t lbm_mlp_param_count(void);
/* max_batch: largest n of any later call (<= 2^20).  Parameters start at 0. */
lbm_status lbm_mlp_create(int32_t max_batch, void* hip_stream, lbm_mlp** out);
void lbm_mlp_destroy(lbm_mlp* m);
/* Sets the FP32 master parameters (and their bfloat16 copy); resets Adam. */
lbm_status lbm_mlp_set_params(lbm_mlp* m, const float* params);
lbm_status lbm_mlp_get_params(lbm_mlp* m, float* params);
/* y[n x 3] = network(x[n x 3]). */
lbm_status lbm_mlp_forward(lbm_mlp* m, const float* x, int32_t n, float* y);
/* Gradients of sum(dy * y) with respect to the parameters (grad, 33,923
 * values; weight entries with respect to the rounded weights) and to the
 * inputs (dx, n x 3).  Either output may be NULL. */
lbm_status lbm_mlp_backward(lbm_mlp* m, const float* x, const float* dy, int32_t n, float* grad,
                            float* dx);
/* Training set (n <= max_batch) kept on the device in buffers of its own:
 * lbm_mlp_forward and lbm_mlp_backward between training calls leave it as set. */
lbm_status lbm_mlp_set_data(lbm_mlp* m, const float* x, const float* t, int32_t n);
/* iters full-batch Adam steps with learning rate lr; loss_out (iters values,
 * may be NULL) receives the loss before each step. */
lbm_status lbm_mlp_train(lbm_mlp* m, int32_t iters, float lr, float* loss_out);

/* Measurement helper (not part of the method): copies `bytes` bytes from src
 * to dst, both device pointers, 16-byte aligned, bytes a multiple of 16, with
 * one plain copy kernel (one 16-byte load and store per lane), enqueued on
 * hip_stream (NULL: the null stream), asynchronous.  Its bandwidth is the
 * practical HBM ceiling that the step kernels' rooflines are read against.
 * LBM_EINVAL for NULL, misaligned or ragged arguments; LBM_EDEVICE if the
 * launch fails.  The buffers stay owned by the caller and must not overlap. */
lbm_status lbm_copy_bytes(void* dst, const void* src, size_t bytes, void* hip_stream);

const char* lbm_strerror(lbm_status s);
/* Message of the last error on the calling thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
