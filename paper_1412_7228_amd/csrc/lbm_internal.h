// Internal interface between the host C ABI (lbm_api.hip) and the gfx950
// kernels (lbm_step.hip, lbm_fields.hip).  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm.h"

namespace lbm {

// Lattice geometry and the launch shape of the fused step kernel.  The state
// is row-interleaved: lattice row y holds the nine planes' rows back to back,
// so element (a, y, x) is at (9 y + a) * pitch + x.
struct Geometry {
  int nx, ny, pitch;       // elements; pitch = one plane's row (nx rounded up to 64)
  long long row;           // 9 * pitch: elements from one lattice row to the next
  int tile_x, tile_y;      // strip width (= workgroup size) and rows per workgroup
  int nstrips, nrowblocks; // ceil(nx / tile_x), ceil((y_end - y_begin) / tile_y)
  int nblocks;             // nstrips * nrowblocks
  int y_begin, y_end;      // rows a launch updates: [y_begin, y_end), normally [0, ny)
};

// Every model constant the step needs, in FP64; the launcher rounds them to
// the working precision.  Names follow the paper: K (Eq. 21), A (Eq. 9),
// kappa (Eq. 23), G (Eq. 7), s_* the MRT rates (Eq. 2).
struct ModelConsts {
  int eos;                  // lbm_eos
  double K, R, T, a, b;     // EOS
  double aalpha;            // Peng-Robinson a * alpha(T)
  double G, A, kappa;
  double s_e, s_eps, s_q, s_nu;
  double nu_gas, nu_liquid, rho_gas, rho_liquid;  // nu_gas > 0: density-dependent s_nu
};

// Fused density/psi + force + Q + MRT collision + streaming, one time step:
// reads f(t) from `fa`, writes f(t+1) to `fb` (separate buffers).
hipError_t launch_step(lbm_precision prec, const Geometry& g, const ModelConsts& m, const void* fa,
                       void* fb, hipStream_t s);

// Workgroups of the step kernel (for g.tile_x) that one CU holds at once.
// Two fused steps per launch (lbm_step.hip): g.tile_x in {128, 256}, strips of
// g.tile_x - 6 stored columns (g.nstrips counts them).
hipError_t launch_step2(lbm_precision prec, const Geometry& g, const ModelConsts& m, const void* fa,
                        void* fb, hipStream_t s);
constexpr int kStep2Halo = 6;
hipError_t step_occupancy(lbm_precision prec, const Geometry& g, int eos, int* per_cu);

// f = equilibrium(rho, u) from device FP64 arrays [ny][nx] (ux/uy may be null).
hipError_t launch_init_equilibrium(lbm_precision prec, const Geometry& g, const double* rho,
                                   const double* ux, const double* uy, void* f, hipStream_t s);

// f plane `a` (pitched, working precision) <-> unpadded FP64 [ny][nx].
hipError_t launch_plane_to_f64(lbm_precision prec, const Geometry& g, const void* f, int a,
                               double* out, hipStream_t s);
hipError_t launch_f64_to_plane(lbm_precision prec, const Geometry& g, const double* in, int a,
                               void* f, hipStream_t s);

// FP64 macroscopic fields of a state: rho, U, psi into `work` (3 * nx*ny doubles).
hipError_t launch_density_fields(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                                 const void* f, double* work, hipStream_t s);

// Velocity component (0 = x, 1 = y) into out[ny][nx]; needs the work arrays above.
hipError_t launch_velocity_field(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                                 const void* f, const double* work, int comp, double* out,
                                 hipStream_t s);

// Deterministic FP64 reduction of the observables: fills red[0..kNumRed).
// `partials` must hold obs_partials_count(g) * kNumRed doubles.
constexpr int kNumRed = 8;  // mass, mom_x, mom_y, rho_min, rho_max, max|v|, n_domain, n_bad
int obs_partials_count(const Geometry& g);
hipError_t launch_observables(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                              const void* f, const double* work, double* partials, double* red,
                              hipStream_t s);
// The same reduction from the distributions alone (no field arrays), plus rho
// at (nx/2, ny/2) and (0, 0) in red[kNumRed], red[kNumRed + 1]; bitwise the
// results of launch_density_fields + launch_observables.
hipError_t launch_observables_direct(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                                     const void* f, double* partials, double* red, hipStream_t s);
// The device address of the file-scope scratch array of the current device
// (kNumRed * (noalloc_max_cells() / 4096) + kNumRed + 2 doubles), resolved
// once per device; and the largest lattice (cells) whose partials fit in it.
hipError_t noalloc_scratch(double** out);
long long noalloc_max_cells();

// Batched engine (lbm_batch.hip).  Descriptors and tiles are opaque records
// filled on the host and copied to the device.
size_t batch_domain_bytes(lbm_precision prec);
size_t batch_tile_bytes();
void batch_fill_domain(lbm_precision prec, const Geometry& g, const ModelConsts& m, void* fa,
                       void* fb, unsigned ntiles, void* out);
void batch_fill_tile(int domain, int x0, int y0, int down, void* out);
// Persistent mode (lbm_persistent.hip): one launch of npairs two-step passes
// over the two-step tiles, grouped by XCD.  The tiles of XCD group g are
// tiles[group_begin[g] .. group_begin[g+1]), head[g] is that group's queue
// position, done[d] counts the finished tiles of domain d, err collects
// aborts (1: a wait passed the spin limit; 2: a domain missed tiles).
struct BatchRun {
  const void* dom;
  const void* tiles;
  const int* group_begin;
  int ngroups;
  unsigned* head;
  unsigned* done;
  int* err;
  int grid, nsteps, parity;  // nsteps: steps (per-step kernels) or pairs of steps (persistent)
  long long spin_limit;
};
// Workgroups of the persistent kernel (tile_x in {128, 256}) that one CU holds at once.
hipError_t batch_occupancy(lbm_precision prec, int eos, int tile_x, int* per_cu);
hipError_t launch_batch_persistent(lbm_precision prec, int eos, int tile_x, const BatchRun& r,
                                   hipStream_t s);
hipError_t launch_batch_reset(const BatchRun& r, int ndomains, hipStream_t s);
hipError_t launch_batch_check(lbm_precision prec, const BatchRun& r, int ndomains, hipStream_t s);
// Per-step mode (lbm_batch.hip): one single-step launch over the tile list.
hipError_t launch_batch(lbm_precision prec, int eos, int tile_x, const BatchRun& r, hipStream_t s);
// Per-step mode, two fused steps per launch over the two-step tile list.
hipError_t launch_batch_step2(lbm_precision prec, int eos, int tile_x, const BatchRun& r,
                              hipStream_t s);

// Surrogate network (lbm_mlp.hip).
int mlp_param_count();
int mlp_rows_per_block();
hipError_t launch_mlp_forward(const float* x, int B, const float* master, const unsigned short* wb,
                              float* acts, float* y, hipStream_t s);
hipError_t launch_mlp_backward(const float* x, const float* acts, const float* dy, int B,
                               const unsigned short* wb, float* gpart, float* grad, float* dx,
                               hipStream_t s);
hipError_t launch_mlp_mse(const float* y, const float* t, int B, float* dy, float* loss, hipStream_t s);
hipError_t launch_mlp_adam(float* p, float* m, float* v, const float* g, unsigned short* wb, float lr,
                           float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_mlp_round(const float* p, unsigned short* wb, hipStream_t s);

}  // namespace lbm
