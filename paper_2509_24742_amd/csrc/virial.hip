// Electrostatic virial (pressure) tensor of a step's estimator (gfx950), FP64.
//
// W = -dE/d(epsilon) under an affine strain of every position and of the box, at
// fixed charges (the paper gives forces but no virial; this is the reading used):
//   - Fourier part: sum over the step's modes (the deterministic kz modes and the
//     sample, with the step's weights w) of 1/2 w |S|^2 [I - 2 (1 + k^2/(4 alpha^2))
//     k k^T / k^2], S = S1 + S2 (fractional coordinates, hence S, do not change under
//     the strain; k and V do), from the coefficients w S the step left;
//   - real part (Eq. (13)): -sum over pairs within rc of q_a q_b K'(r) r r^T / r,
//     ion-ion, ion-Gaussian and Gaussian-Gaussian kernels, each pair once (ion-ion
//     and Gaussian-Gaussian pairs are visited from both ends with half weight);
//   - slab term (Eq. (17)): (2 pi / V) M_z^2 diag(1, 1, -1).
// Components [xx, yy, zz, xy, xz, yz], times ke.  One thread per ion and per electrode
// over the step's cell lists (positions from the FP64 input, minimum image in x, y);
// each block leaves its six sums in part, and k_virial_final adds them in block order,
// with the Fourier and slab parts, per replica.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace srbe {

namespace {

#define VIR_INV_SQRT_PI 0.5641895835477563

// d/dr [erfc(a r) / r]
__device__ __forceinline__ double vir_derfc(double a, double r) {
  const double ar = a * r;
  return -erfc(ar) / (r * r) - 2.0 * a * VIR_INV_SQRT_PI * exp(-ar * ar) / r;
}

__device__ __forceinline__ void add_pair(double (&v)[6], double c, double dx, double dy, double dz) {
  v[0] += c * dx * dx;
  v[1] += c * dy * dy;
  v[2] += c * dz * dz;
  v[3] += c * dx * dy;
  v[4] += c * dx * dz;
  v[5] += c * dy * dz;
}

template <int NV>
__device__ __forceinline__ void vir_block_sum(double (&v)[NV], double (*sh)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int u = 0; u < NV; ++u) {
    double x = v[u];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) sh[u][w] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int u = 0; u < NV; ++u) v[u] = (sh[u][0] + sh[u][1]) + (sh[u][2] + sh[u][3]);
}

// Block (r, t): t < ftiles: ions [256 t, 256 t + 256) of replica r; else electrodes.
__global__ __launch_bounds__(256) void k_virial_real(Geom g, StepBufs b, int ftiles, int etiles,
                                                     double* __restrict__ part) {
  __shared__ double sh[6][4];
  const int nb = ftiles + etiles;
  const int r = blockIdx.x / nb, t = blockIdx.x - r * nb;
  const int n = g.n_ele;
  const int64_t N = b.N;
  const double* __restrict__ X = b.ion_xyz;
  const double* __restrict__ E = b.ele_xyz;
  const double* __restrict__ Q = b.Q_out + (size_t)r * n;
  const double rc2 = g.rc * g.rc, a = g.alpha, ai = 1.0 / g.eta, ag = 1.0 / (sqrt(2.0) * g.eta);
  const int64_t b0 = b.off[r], b1 = b.off[r + 1];
  const int* cs = b.cstart + (size_t)r * (g.ncell + 1);
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  auto pair = [&](double xa, double ya, double za, double xb, double yb, double zb, double qq, double ab,
                  double half) {
    double dx = xa - xb, dy = ya - yb;
    const double dz = za - zb;
    dx -= g.Lx * rint(dx * g.invLx);
    dy -= g.Ly * rint(dy * g.invLy);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 >= rc2) return;
    const double rr = sqrt(r2);
    const double dk = ab > 0.0 ? vir_derfc(a, rr) - vir_derfc(ab, rr) : vir_derfc(a, rr);
    add_pair(v, -half * qq * dk / rr, dx, dy, dz);
  };
  if (t < ftiles) {
    const int64_t i = b0 + (int64_t)t * 256 + threadIdx.x;
    if (i < b1) {
      const double xi = X[i], yi = X[N + i], zi = X[2 * N + i], qi = b.ion_q[i];
      const unsigned key = b.keys[i];
      const int c = b.bigsort.count ? (int)key : (int)(key >> 13);
      for (int u = 0; u < kRunMax; ++u) {  // ions: half weight, each pair is seen from both ends
        const int2 run = b.ion_runs[(size_t)kRunMax * c + u];
        if (run.x < 0) break;
        for (int64_t k = b0 + cs[run.x]; k < b0 + cs[run.y]; ++k) {
          const int j = b.perm[k];
          if (j == i) continue;
          pair(xi, yi, zi, X[j], X[N + j], X[2 * N + j], qi * b.ion_q[j], 0.0, 0.5);
        }
      }
      for (int u = 0; u < kRunMax; ++u) {  // electrodes: full weight, seen from the ion only
        const int4 run = b.ele_rr[(size_t)kRunMax * c + u];
        if (run.x < 0) break;
        for (int e = run.x; e < run.y; ++e) {
          const int j = b.ele_perm[e];
          pair(xi, yi, zi, E[j], E[n + j], E[2 * n + j], qi * Q[j], ai, 1.0);
        }
      }
    }
  } else {
    const int j = (t - ftiles) * 256 + threadIdx.x;
    if (j < n) {
      const double xj = E[j], yj = E[n + j], zj = E[2 * n + j], qj = Q[j];
      const int c = b.ele_scell[b.ele_iperm[j]];
      for (int u = 0; u < kRunMax; ++u) {  // other electrodes: half weight
        const int4 run = b.ele_rr[(size_t)kRunMax * c + u];
        if (run.x < 0) break;
        for (int e = run.x; e < run.y; ++e) {
          const int k = b.ele_perm[e];
          if (k == j) continue;
          pair(xj, yj, zj, E[k], E[n + k], E[2 * n + k], qj * Q[k], ag, 0.5);
        }
      }
    }
  }
  vir_block_sum<6>(v, sh);
  if (threadIdx.x == 0)
    for (int u = 0; u < 6; ++u) part[((size_t)r * nb + t) * 6 + u] = v[u];
}

// Block r: the Fourier part over the replica's modes, the block partials of the real
// part in block order, the slab part; W_out[6 r ..].
__global__ __launch_bounds__(256) void k_virial_final(Geom g, StepBufs b, int nb, const double* __restrict__ part,
                                                      const double* __restrict__ Mz_e, double* __restrict__ W) {
  __shared__ double sh[6][4];
  const int r = blockIdx.x;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double TWO_PI_ = 6.283185307179586;
  for (int k = threadIdx.x; k < g.K; k += 256) {
    const size_t idx = (size_t)r * g.K + k;
    const double w = b.w[idx];  // the step's weights carry ke
    if (!(w > 0.0)) continue;  // a rejected given mode (flagged by the step) has weight 0
    const double2 c = b.coef[idx];
    const int4 m = b.modes[idx];
    const double kx = TWO_PI_ * m.x * g.invLx, ky = TWO_PI_ * m.y * g.invLy, kz = TWO_PI_ * m.z * g.invLz;
    const double k2 = kx * kx + ky * ky + kz * kz;
    const double e = 0.5 * (c.x * c.x + c.y * c.y) / w;  // 1/2 w |S|^2 with S = coef / w (ke in w)
    const double f = 2.0 * (1.0 + k2 / (4.0 * g.alpha * g.alpha)) / k2;
    v[0] += e - e * f * kx * kx;
    v[1] += e - e * f * ky * ky;
    v[2] += e - e * f * kz * kz;
    v[3] -= e * f * kx * ky;
    v[4] -= e * f * kx * kz;
    v[5] -= e * f * ky * kz;
  }
  vir_block_sum<6>(v, sh);
  if (threadIdx.x == 0) {
    double rs[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (b.real)
      for (int t = 0; t < nb; ++t)
        for (int u = 0; u < 6; ++u) rs[u] += part[((size_t)r * nb + t) * 6 + u];
    const double Mz = b.scal[4 * r + 2] + Mz_e[r];
    const double slab = (2.0 * M_PI / g.V) * Mz * Mz;
    const double sl[6] = {slab, slab, -slab, 0.0, 0.0, 0.0};
    for (int u = 0; u < 6; ++u) W[6 * r + u] = v[u] + g.ke * (rs[u] + sl[u]);
  }
}

// sum_j Q_j Z_j per replica (the electrodes' dipole of the slab term), in electrode order.
__global__ __launch_bounds__(256) void k_virial_mz(Geom g, StepBufs b, double* __restrict__ Mz_e) {
  __shared__ double sh[1][4];
  const int r = blockIdx.x, n = g.n_ele;
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < n; j += 256) v[0] += b.Q_out[(size_t)r * n + j] * b.ele_xyz[2 * n + j];
  vir_block_sum<1>(v, sh);
  if (threadIdx.x == 0) Mz_e[r] = v[0];
}

}  // namespace

size_t virial_scratch_doubles(const Geom& g, const StepBufs& b) {
  const int ftiles = (std::max(b.max_nrep, 0) + 255) / 256, etiles = (g.n_ele + 255) / 256;
  return (size_t)b.R * (ftiles + etiles) * 6 + (size_t)b.R;
}

void launch_virial(const Geom& g, const StepBufs& b, double* scratch, double* W, hipStream_t s) {
  const int ftiles = (std::max(b.max_nrep, 0) + 255) / 256, etiles = (g.n_ele + 255) / 256;
  const int nb = ftiles + etiles;
  double* part = scratch;
  double* Mz_e = scratch + (size_t)b.R * nb * 6;
  if (b.real && nb > 0) hipLaunchKernelGGL(k_virial_real, dim3((unsigned)b.R * nb), dim3(256), 0, s, g, b, ftiles, etiles, part);
  hipLaunchKernelGGL(k_virial_mz, dim3(b.R), dim3(256), 0, s, g, b, Mz_e);
  hipLaunchKernelGGL(k_virial_final, dim3(b.R), dim3(256), 0, s, g, b, nb, part, Mz_e, W);
}

}  // namespace srbe
