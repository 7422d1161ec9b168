// Euler-Maruyama step of the Langevin thermostat (Sec. 3), one thread per ion (gfx950).
//
//   r <- r + v dt
//   v <- v + (F - gamma v) dt / m + sqrt(2 gamma / beta) dW / m,   dW ~ N(0, dt) per component
//
// or, with the symplectic ordering (a reading for dynamics: the printed ordering gains
// energy on every stiff oscillation by 1 + (omega dt)^2 per step), the same velocity
// update first and r <- r + v_new dt.
//
// x and y wrap into the periodic cell; z is reflected specularly into [zlo, zhi] as often
// as it takes to land inside (v_z changes sign once per reflection), a stand-in for the
// wall force field: with W = zhi - zlo, k = floor((z - zlo) / W) reflections and
// t = (z - zlo) - k W, z becomes zlo + t for even k and zhi - t for odd k, clamped into
// [zlo, zhi] against rounding.  The deviates come from
// Philox4x64-10 with key (seed, 1) and counter (ion, step, 3, 0) -- the sampler uses key
// (seed, 0) -- through Box-Muller on the four words mapped into (0, 1).  FP64.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace srbe {

namespace {

__global__ __launch_bounds__(256) void k_langevin(int64_t n, double* __restrict__ xyz, double* __restrict__ vel,
                                                   const double* __restrict__ F, const double* __restrict__ mass,
                                                   double gamma, double noise, double dt, double Lx, double Ly,
                                                   double zlo, double zhi, uint64_t seed, uint64_t step,
                                                   const uint64_t* __restrict__ step_dev, int symplectic) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  U64x4 c;
  c.v[0] = (uint64_t)i;
  c.v[1] = step_dev ? *step_dev - 1 : step;
  c.v[2] = 3;
  c.v[3] = 0;
  const U64x4 w = philox4x64_10(c, seed, 1);
  const double U0 = u01_open(w.v[0]), U1 = u01_open(w.v[1]), U2 = u01_open(w.v[2]), U3 = u01_open(w.v[3]);
  const double r0 = sqrt(-2.0 * log(U0)), r2 = sqrt(-2.0 * log(U2));
  const double z[3] = {r0 * cos(2.0 * M_PI * U1), r0 * sin(2.0 * M_PI * U1), r2 * cos(2.0 * M_PI * U3)};
  const double sdt = sqrt(dt), m = mass[i];
  double r[3], v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double x = xyz[d * n + i], u = vel[d * n + i];
    v[d] = u + (F[d * n + i] - gamma * u) * dt / m + noise * (sdt * z[d]) / m;
    r[d] = x + (symplectic ? v[d] : u) * dt;
  }
  r[0] -= Lx * floor(r[0] / Lx);
  r[1] -= Ly * floor(r[1] / Ly);
  if (r[2] < zlo || r[2] > zhi) {
    const double W = zhi - zlo;
    const double k = floor((r[2] - zlo) / W);
    const double t = fmin(fmax((r[2] - zlo) - k * W, 0.0), W);
    const bool odd = fmod(k, 2.0) != 0.0;
    r[2] = fmin(fmax(odd ? zhi - t : zlo + t, zlo), zhi);
    if (odd) v[2] = -v[2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    xyz[d * n + i] = r[d];
    vel[d * n + i] = v[d];
  }
}

}  // namespace

void launch_langevin(int64_t n, double* xyz, double* vel, const double* F, const double* mass, double gamma,
                     double beta, double dt, double Lx, double Ly, double zlo, double zhi, uint64_t seed,
                     uint64_t step, hipStream_t s, const uint64_t* step_dev, int symplectic) {
  if (n == 0) return;
  const double noise = sqrt(2.0 * gamma / beta);  // 0 for beta = infinity
  hipLaunchKernelGGL(k_langevin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, xyz, vel, F, mass, gamma,
                     noise, dt, Lx, Ly, zlo, zhi, seed, step, step_dev, symplectic);
}

}  // namespace srbe
