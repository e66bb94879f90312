// FP64 read-out of a state: density/psi fields, velocity, distribution planes,
// and the deterministic reduction of the observables (mass, momentum,
// extremes, faults) used by the Laplace-law measurement (Eq. 22).
// Off the hot path: these run only when the caller asks for observables or fields.
#include <mutex>

#include "lbm_device.h"

namespace lbm {

constexpr int kRedThreads = 256;
constexpr int kRedCellsPerThread = 16;

// rho = sum_a f_a(x) of the current (streamed) state, U and psi in FP64.
template <typename T, int EOS>
__global__ void k_density_fields(const T* __restrict__ f, const Geometry geo, const DevC<double> c,
                                 double* __restrict__ work) {
  const long long n = (long long)geo.nx * geo.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / geo.nx), x = (int)(i - (long long)y * geo.nx);
  double r = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) r += (double)f[state_index(geo, a, x, y)];
  const double U = eos_U<EOS>(r, c);
  work[i] = r;
  work[n + i] = U;
  work[2 * n + i] = psi_of(U, c);
}

// Force of Eq. (9) at a cell from U and psi at the cell (index 0) and at its
// eight neighbours x + e_a (index a), and the momentum j of the cell's
// distributions g (the weights 1/3, 1/12 applied as 12 sum_a w_a phi e_a).
__device__ inline void force_momentum_core(const double (&Un)[9], const double (&Pn)[9],
                                           const DevC<double>& c, const double (&g)[9], double& Fx,
                                           double& Fy, double& jx, double& jy) {
  const double gUx = 4.0 * (Un[1] - Un[3]) + ((Un[5] - Un[7]) + (Un[8] - Un[6]));
  const double gUy = 4.0 * (Un[2] - Un[4]) + ((Un[5] - Un[7]) + (Un[6] - Un[8]));
  const double gPx = 4.0 * (Pn[1] - Pn[3]) + ((Pn[5] - Pn[7]) + (Pn[8] - Pn[6]));
  const double gPy = 4.0 * (Pn[2] - Pn[4]) + ((Pn[5] - Pn[7]) + (Pn[6] - Pn[8]));
  const double fpp = c.fP * Pn[0];
  Fx = c.fU * gUx + fpp * gPx;
  Fy = c.fU * gUy + fpp * gPy;
  jx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
  jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
}

// Offsets e_a of the lattice velocities, in the order of the distributions.
__device__ __forceinline__ int ex_of(int a) { return (a == 1 || a == 5 || a == 8) ? 1 : ((a == 3 || a == 6 || a == 7) ? -1 : 0); }
__device__ __forceinline__ int ey_of(int a) { return (a == 2 || a == 5 || a == 6) ? 1 : ((a == 4 || a == 7 || a == 8) ? -1 : 0); }

// rho = sum_a f_a(x, y) of the current (streamed) state in FP64, summed in
// plane order (the order every read-out uses).
template <typename T>
__device__ inline double cell_density(const T* __restrict__ f, const Geometry& geo, int x, int y) {
  double r = 0.0;
#pragma unroll
  for (int a = 0; a < 9; ++a) r += (double)f[state_index(geo, a, x, y)];
  return r;
}

template <typename T>
__device__ inline void cell_distributions(const T* __restrict__ f, const Geometry& geo, int x, int y,
                                          double (&g)[9]) {
#pragma unroll
  for (int a = 0; a < 9; ++a) g[a] = (double)f[state_index(geo, a, x, y)];
}

// Force and momentum at (x, y) from the FP64 U/psi fields of k_density_fields.
template <typename T>
__device__ inline void force_and_momentum(const T* __restrict__ f, const Geometry& geo,
                                          const DevC<double>& c, const double* __restrict__ work,
                                          int x, int y, double& Fx, double& Fy, double& jx,
                                          double& jy) {
  const long long n = (long long)geo.nx * geo.ny;
  const double* U = work + n;
  const double* psi = work + 2 * n;
  double Un[9], Pn[9], g[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const long long i = (long long)wrap_(y + ey_of(a), geo.ny) * geo.nx + wrap_(x + ex_of(a), geo.nx);
    Un[a] = U[i];
    Pn[a] = psi[i];
  }
  cell_distributions(f, geo, x, y, g);
  force_momentum_core(Un, Pn, c, g, Fx, Fy, jx, jy);
}

// The same from the distributions alone: rho, U and psi of the cell and its
// eight neighbours recomputed from f (no field arrays).  Returns rho and U of
// the cell itself in r0, U0.
template <typename T, int EOS>
__device__ inline void force_and_momentum_direct(const T* __restrict__ f, const Geometry& geo,
                                                 const DevC<double>& c, int x, int y, double& Fx,
                                                 double& Fy, double& jx, double& jy, double& r0,
                                                 double& U0) {
  double Un[9], Pn[9], g[9];
  for (int a = 0; a < 9; ++a) {
    const double r = cell_density(f, geo, wrap_(x + ex_of(a), geo.nx), wrap_(y + ey_of(a), geo.ny));
    Un[a] = eos_U<EOS>(r, c);
    Pn[a] = psi_of(Un[a], c);
    if (a == 0) r0 = r;
  }
  U0 = Un[0];
  cell_distributions(f, geo, x, y, g);
  force_momentum_core(Un, Pn, c, g, Fx, Fy, jx, jy);
}

template <typename T>
__global__ void k_velocity(const T* __restrict__ f, const Geometry geo, const DevC<double> c,
                           const double* __restrict__ work, int comp, double* __restrict__ out) {
  const long long n = (long long)geo.nx * geo.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / geo.nx), x = (int)(i - (long long)y * geo.nx);
  double Fx, Fy, jx, jy;
  force_and_momentum(f, geo, c, work, x, y, Fx, Fy, jx, jy);
  out[i] = (comp == 0 ? jx + 0.5 * Fx : jy + 0.5 * Fy) / work[i];
}

// One cell's contribution to the observables: mass, momentum (j + F/2),
// density extremes, max |v|^2, and the fault counts.
__device__ inline void accumulate_cell(double (&acc)[kNumRed], double r, double U, double Fx,
                                       double Fy, double jx, double jy) {
  const double mx = jx + 0.5 * Fx, my = jy + 0.5 * Fy;
  acc[0] += r;
  acc[1] += mx;
  acc[2] += my;
  acc[3] = fmin(acc[3], r);
  acc[4] = fmax(acc[4], r);
  const double vx = mx / r, vy = my / r;
  const double v2 = vx * vx + vy * vy;
  if (v2 == v2) acc[5] = fmax(acc[5], v2);
  acc[6] += (U <= 0.0) ? 0.0 : 1.0;                  // U > 0 (or NaN)
  acc[7] += (r > 0.0 && isfinite(r)) ? 0.0 : 1.0;    // rho <= 0 or not finite
}

// Tree reduction of the block's accumulators in a fixed order; thread q <
// kNumRed writes entry q of the block's result to out[q].
__device__ inline void block_reduce_store(const double (&acc)[kNumRed], double (&sh)[kNumRed][kRedThreads],
                                          double* __restrict__ out) {
#pragma unroll
  for (int q = 0; q < kNumRed; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int stride = kRedThreads / 2; stride > 0; stride >>= 1) {
    if ((int)threadIdx.x < stride) {
      const int o = threadIdx.x + stride;
      sh[0][threadIdx.x] += sh[0][o];
      sh[1][threadIdx.x] += sh[1][o];
      sh[2][threadIdx.x] += sh[2][o];
      sh[3][threadIdx.x] = fmin(sh[3][threadIdx.x], sh[3][o]);
      sh[4][threadIdx.x] = fmax(sh[4][threadIdx.x], sh[4][o]);
      sh[5][threadIdx.x] = fmax(sh[5][threadIdx.x], sh[5][o]);
      sh[6][threadIdx.x] += sh[6][o];
      sh[7][threadIdx.x] += sh[7][o];
    }
    __syncthreads();
  }
  if (threadIdx.x < kNumRed) out[threadIdx.x] = sh[threadIdx.x][0];
}

// Per-block partial reductions in a fixed order (cells i = base + k * 256 + lane).
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
    k_obs_partial(const T* __restrict__ f, const Geometry geo, const DevC<double> c,
                  const double* __restrict__ work, double* __restrict__ partials) {
  __shared__ double sh[kNumRed][kRedThreads];
  const long long n = (long long)geo.nx * geo.ny;
  const long long base = (long long)blockIdx.x * kRedThreads * kRedCellsPerThread;
  double acc[kNumRed] = {0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
  for (int k = 0; k < kRedCellsPerThread; ++k) {
    const long long i = base + (long long)k * kRedThreads + threadIdx.x;
    if (i >= n) break;
    const int y = (int)(i / geo.nx), x = (int)(i - (long long)y * geo.nx);
    double Fx, Fy, jx, jy;
    force_and_momentum(f, geo, c, work, x, y, Fx, Fy, jx, jy);
    accumulate_cell(acc, work[i], work[n + i], Fx, Fy, jx, jy);
  }
  block_reduce_store(acc, sh, partials + (long long)blockIdx.x * kNumRed);
}

// The same partials with no field arrays: each cell recomputes rho, U, psi of
// its neighbourhood from f.  Same cells per block, same order, same
// arithmetic, so the partials are bitwise those of k_obs_partial.
template <typename T, int EOS>
__global__ void __launch_bounds__(kRedThreads)
    k_obs_partial_direct(const T* __restrict__ f, const Geometry geo, const DevC<double> c,
                         double* __restrict__ partials) {
  __shared__ double sh[kNumRed][kRedThreads];
  const long long n = (long long)geo.nx * geo.ny;
  const long long base = (long long)blockIdx.x * kRedThreads * kRedCellsPerThread;
  double acc[kNumRed] = {0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
  for (int k = 0; k < kRedCellsPerThread; ++k) {
    const long long i = base + (long long)k * kRedThreads + threadIdx.x;
    if (i >= n) break;
    const int y = (int)(i / geo.nx), x = (int)(i - (long long)y * geo.nx);
    double Fx, Fy, jx, jy, r, U;
    force_and_momentum_direct<T, EOS>(f, geo, c, x, y, Fx, Fy, jx, jy, r, U);
    accumulate_cell(acc, r, U, Fx, Fy, jx, jy);
  }
  block_reduce_store(acc, sh, partials + (long long)blockIdx.x * kNumRed);
}

// rho at the two sample cells of the Laplace measurement, (nx/2, ny/2) and (0, 0).
template <typename T>
__global__ void k_sample_densities(const T* __restrict__ f, const Geometry geo, double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = cell_density(f, geo, geo.nx / 2, geo.ny / 2);
  if (threadIdx.x == 1) out[1] = cell_density(f, geo, 0, 0);
}

__global__ void __launch_bounds__(kRedThreads)
    k_obs_final(const double* __restrict__ partials, int nparts, double* __restrict__ red) {
  __shared__ double sh[kNumRed][kRedThreads];
  double acc[kNumRed] = {0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nparts; b += kRedThreads) {
    const double* p = partials + (long long)b * kNumRed;
    acc[0] += p[0];
    acc[1] += p[1];
    acc[2] += p[2];
    acc[3] = fmin(acc[3], p[3]);
    acc[4] = fmax(acc[4], p[4]);
    acc[5] = fmax(acc[5], p[5]);
    acc[6] += p[6];
    acc[7] += p[7];
  }
  block_reduce_store(acc, sh, red);
}

template <typename T>
__global__ void k_plane_to_f64(const T* __restrict__ f, const Geometry geo, int a,
                               double* __restrict__ out) {
  const long long n = (long long)geo.nx * geo.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / geo.nx), x = (int)(i - (long long)y * geo.nx);
  out[i] = (double)f[state_index(geo, a, x, y)];
}

template <typename T>
__global__ void k_f64_to_plane(const double* __restrict__ in, const Geometry geo, int a,
                               T* __restrict__ f) {
  const long long n = (long long)geo.nx * geo.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int y = (int)(i / geo.nx), x = (int)(i - (long long)y * geo.nx);
  f[state_index(geo, a, x, y)] = T(in[i]);
}

static dim3 cells_grid(const Geometry& g) {
  const long long n = (long long)g.nx * g.ny;
  return dim3((unsigned)((n + 255) / 256));
}

int obs_partials_count(const Geometry& g) {
  const long long n = (long long)g.nx * g.ny;
  const long long per = (long long)kRedThreads * kRedCellsPerThread;
  return (int)((n + per - 1) / per);
}

hipError_t launch_plane_to_f64(lbm_precision prec, const Geometry& g, const void* f, int a,
                               double* out, hipStream_t s) {
  if (prec == LBM_FP32)
    hipLaunchKernelGGL(k_plane_to_f64<float>, cells_grid(g), dim3(256), 0, s,
                       static_cast<const float*>(f), g, a, out);
  else
    hipLaunchKernelGGL(k_plane_to_f64<double>, cells_grid(g), dim3(256), 0, s,
                       static_cast<const double*>(f), g, a, out);
  return hipGetLastError();
}

hipError_t launch_f64_to_plane(lbm_precision prec, const Geometry& g, const double* in, int a,
                               void* f, hipStream_t s) {
  if (prec == LBM_FP32)
    hipLaunchKernelGGL(k_f64_to_plane<float>, cells_grid(g), dim3(256), 0, s, in, g, a,
                       static_cast<float*>(f));
  else
    hipLaunchKernelGGL(k_f64_to_plane<double>, cells_grid(g), dim3(256), 0, s, in, g, a,
                       static_cast<double*>(f));
  return hipGetLastError();
}

template <typename T, int EOS>
static void density_t(const Geometry& g, const DevC<double>& c, const void* f, double* work,
                      hipStream_t s) {
  hipLaunchKernelGGL((k_density_fields<T, EOS>), cells_grid(g), dim3(256), 0, s,
                     static_cast<const T*>(f), g, c, work);
}

template <typename T>
static hipError_t density_p(const Geometry& g, const ModelConsts& m, const void* f, double* work,
                            hipStream_t s) {
  const DevC<double> c = make_devc<double>(m);
  switch (m.eos) {
    case LBM_EOS_IDEAL: density_t<T, LBM_EOS_IDEAL>(g, c, f, work, s); break;
    case LBM_EOS_CS: density_t<T, LBM_EOS_CS>(g, c, f, work, s); break;
    case LBM_EOS_VDW: density_t<T, LBM_EOS_VDW>(g, c, f, work, s); break;
    case LBM_EOS_PR: density_t<T, LBM_EOS_PR>(g, c, f, work, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_density_fields(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                                 const void* f, double* work, hipStream_t s) {
  if (prec == LBM_FP32) return density_p<float>(g, m, f, work, s);
  return density_p<double>(g, m, f, work, s);
}

hipError_t launch_velocity_field(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                                 const void* f, const double* work, int comp, double* out,
                                 hipStream_t s) {
  const DevC<double> c = make_devc<double>(m);
  if (prec == LBM_FP32)
    hipLaunchKernelGGL(k_velocity<float>, cells_grid(g), dim3(256), 0, s,
                       static_cast<const float*>(f), g, c, work, comp, out);
  else
    hipLaunchKernelGGL(k_velocity<double>, cells_grid(g), dim3(256), 0, s,
                       static_cast<const double*>(f), g, c, work, comp, out);
  return hipGetLastError();
}

hipError_t launch_observables(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                              const void* f, const double* work, double* partials, double* red,
                              hipStream_t s) {
  const DevC<double> c = make_devc<double>(m);
  const int np = obs_partials_count(g);
  if (prec == LBM_FP32)
    hipLaunchKernelGGL(k_obs_partial<float>, dim3(np), dim3(kRedThreads), 0, s,
                       static_cast<const float*>(f), g, c, work, partials);
  else
    hipLaunchKernelGGL(k_obs_partial<double>, dim3(np), dim3(kRedThreads), 0, s,
                       static_cast<const double*>(f), g, c, work, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(kRedThreads), 0, s, partials, np, red);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Observables with no allocation: the partial sums live in one file-scope
// device array, resolved per device by hipGetSymbolAddress at a call's set-up.
// ---------------------------------------------------------------------------
constexpr int kNoAllocMaxPartials = 65536;  // blocks of 4096 cells: 2^28 cells
constexpr size_t kNoAllocScratchDoubles = (size_t)kNoAllocMaxPartials * kNumRed + kNumRed + 2;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

long long noalloc_max_cells() {
  return (long long)kNoAllocMaxPartials * kRedThreads * kRedCellsPerThread;
}

hipError_t noalloc_scratch(double** out) {
  static std::mutex mu;
  static double* per_device[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!per_device[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    per_device[dev] = static_cast<double*>(ptr);
  }
  *out = per_device[dev];
  return hipSuccess;
}

template <typename T>
static hipError_t observables_direct_t(const Geometry& g, const ModelConsts& m, const T* f,
                                       double* partials, double* red, hipStream_t s) {
  const DevC<double> c = make_devc<double>(m);
  const int np = obs_partials_count(g);
  switch (m.eos) {
    case LBM_EOS_IDEAL: hipLaunchKernelGGL((k_obs_partial_direct<T, LBM_EOS_IDEAL>), dim3(np), dim3(kRedThreads), 0, s, f, g, c, partials); break;
    case LBM_EOS_CS: hipLaunchKernelGGL((k_obs_partial_direct<T, LBM_EOS_CS>), dim3(np), dim3(kRedThreads), 0, s, f, g, c, partials); break;
    case LBM_EOS_VDW: hipLaunchKernelGGL((k_obs_partial_direct<T, LBM_EOS_VDW>), dim3(np), dim3(kRedThreads), 0, s, f, g, c, partials); break;
    case LBM_EOS_PR: hipLaunchKernelGGL((k_obs_partial_direct<T, LBM_EOS_PR>), dim3(np), dim3(kRedThreads), 0, s, f, g, c, partials); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(kRedThreads), 0, s, partials, np, red);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_sample_densities<T>, dim3(1), dim3(64), 0, s, f, g, red + kNumRed);
  return hipGetLastError();
}

hipError_t launch_observables_direct(lbm_precision prec, const Geometry& g, const ModelConsts& m,
                                     const void* f, double* partials, double* red, hipStream_t s) {
  if (prec == LBM_FP32)
    return observables_direct_t<float>(g, m, static_cast<const float*>(f), partials, red, s);
  return observables_direct_t<double>(g, m, static_cast<const double*>(f), partials, red, s);
}

}  // namespace lbm
