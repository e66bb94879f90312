// FP64 read-out of a state: density/psi fields, velocity, distribution planes,
// and the deterministic reduction of the observables (mass, momentum,
// extremes, faults) used by the Laplace-law measurement (Eq. 22).
// Off the hot path: these run only when the caller asks for observables or fields.
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

// Force of Eq. (9) at (x, y) from the FP64 U/psi fields, and the momentum j.
template <typename T>
__device__ inline void force_and_momentum(const T* __restrict__ f, const Geometry& geo,
                                          const DevC<double>& c, const double* __restrict__ work,
                                          int x, int y, double& Fx, double& Fy, double& jx,
                                          double& jy) {
  const long long n = (long long)geo.nx * geo.ny;
  const double* U = work + n;
  const double* psi = work + 2 * n;
  const int xm = x == 0 ? geo.nx - 1 : x - 1, xp = x == geo.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? geo.ny - 1 : y - 1, yp = y == geo.ny - 1 ? 0 : y + 1;
  const long long rc = (long long)y * geo.nx, rm = (long long)ym * geo.nx, rp = (long long)yp * geo.nx;
  const double gUx = 4.0 * (U[rc + xp] - U[rc + xm]) + ((U[rp + xp] - U[rm + xm]) + (U[rm + xp] - U[rp + xm]));
  const double gUy = 4.0 * (U[rp + x] - U[rm + x]) + ((U[rp + xp] - U[rm + xm]) + (U[rp + xm] - U[rm + xp]));
  const double gPx = 4.0 * (psi[rc + xp] - psi[rc + xm]) + ((psi[rp + xp] - psi[rm + xm]) + (psi[rm + xp] - psi[rp + xm]));
  const double gPy = 4.0 * (psi[rp + x] - psi[rm + x]) + ((psi[rp + xp] - psi[rm + xm]) + (psi[rp + xm] - psi[rm + xp]));
  const double fpp = c.fP * psi[rc + x];
  Fx = c.fU * gUx + fpp * gPx;
  Fy = c.fU * gUy + fpp * gPy;
  double g[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) g[a] = (double)f[state_index(geo, a, x, y)];
  jx = (g[1] - g[3]) + ((g[5] - g[7]) + (g[8] - g[6]));
  jy = (g[2] - g[4]) + ((g[5] - g[7]) + (g[6] - g[8]));
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

// Per-block partial reductions in a fixed order.
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
    const double r = work[i];
    const double mx = jx + 0.5 * Fx, my = jy + 0.5 * Fy;
    acc[0] += r;
    acc[1] += mx;
    acc[2] += my;
    acc[3] = fmin(acc[3], r);
    acc[4] = fmax(acc[4], r);
    const double vx = mx / r, vy = my / r;
    const double v2 = vx * vx + vy * vy;
    if (v2 == v2) acc[5] = fmax(acc[5], v2);
    acc[6] += (work[n + i] <= 0.0) ? 0.0 : 1.0;          // U > 0 (or NaN)
    acc[7] += (r > 0.0 && isfinite(r)) ? 0.0 : 1.0;       // rho <= 0 or not finite
  }
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
  if (threadIdx.x < kNumRed) partials[(long long)blockIdx.x * kNumRed + threadIdx.x] = sh[threadIdx.x][0];
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
  if (threadIdx.x < kNumRed) red[threadIdx.x] = sh[threadIdx.x][0];
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

}  // namespace lbm
