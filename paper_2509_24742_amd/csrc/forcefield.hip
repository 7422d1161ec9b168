// Short-range force field for SRBE-driven dynamics (gfx950), FP64.
//
// The paper's dynamics use a coarse-grained force field it does not give; this stand-in
// keeps ions apart, between the walls and in their molecules, so that the Langevin
// dynamics of Sec. 3 can run on the SRBE forces:
//   - WCA repulsion between sites of different molecules, 4 eps [(s/r)^12 - (s/r)^6] + eps
//     for r < 2^(1/6) s;
//   - two 9-3 walls, eps_w [(2/15)(s_w/d)^9 - (s_w/d)^3] cut and shifted at the minimum
//     d_min = (2/5)^(1/6) s_w, at z = zlo (acting upward) and z = zhi (downward);
//   - harmonic bonds (k/2)(r - r0)^2 to up to two partner sites per site.
// One thread per ion, over the cell lists of the handle's last step (the same neighbour
// runs as the real-space pass; the WCA range must not exceed rc), positions from the
// step's FP64 input (minimum image in x, y).  Every pair term is computed from both
// ends and added in neighbour-run order, so the result is bitwise repeatable.  The
// forces are added to F; the per-ion energy (half of each pair and bond term, all of its
// wall terms) is written to e_ion if given.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace srbe {

namespace {

__global__ __launch_bounds__(256) void k_ff_forces(Geom g, StepBufs b, FFParams ff, const int* __restrict__ mol,
                                                    const int* __restrict__ bond, const double* __restrict__ bond_r0,
                                                    double* __restrict__ F, double* __restrict__ e_ion, int ftiles) {
  const int r = blockIdx.x / ftiles, tile = blockIdx.x - r * ftiles;
  const int64_t b0 = b.off[r], b1 = b.off[r + 1];
  const int64_t i = b0 + (int64_t)tile * 256 + threadIdx.x;
  if (i >= b1) return;
  const int64_t N = b.N;
  const double* __restrict__ X = b.ion_xyz;
  const double xi = X[i], yi = X[N + i], zi = X[2 * N + i];
  const int mi = mol[i];
  // the ion's cell: the multi-block sort keeps it as the key, the one-block sort in its high bits
  const unsigned key = b.keys[i];
  const int c = b.bigsort.count ? (int)key : (int)(key >> 13);
  const int* cs = b.cstart + (size_t)r * (g.ncell + 1);
  const double s6 = ff.wca_sigma * ff.wca_sigma * ff.wca_sigma * ff.wca_sigma * ff.wca_sigma * ff.wca_sigma;
  const double rw2 = cbrt(2.0 * s6);  // (2^(1/6) s)^2 = (2 s^6)^(1/3)
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  for (int u = 0; u < kRunMax; ++u) {
    const int2 run = b.ion_runs[(size_t)kRunMax * c + u];
    if (run.x < 0) break;
    for (int64_t k = b0 + cs[run.x]; k < b0 + cs[run.y]; ++k) {
      const int j = b.perm[k];
      if (j == i || mol[j] == mi) continue;
      double dx = xi - X[j], dy = yi - X[N + j];
      const double dz = zi - X[2 * N + j];
      dx -= g.Lx * rint(dx * g.invLx);
      dy -= g.Ly * rint(dy * g.invLy);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 >= rw2) continue;
      const double ir2 = 1.0 / r2, sr6 = s6 * ir2 * ir2 * ir2;
      // -dU/dr / r = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2
      const double f = 24.0 * ff.wca_eps * (2.0 * sr6 * sr6 - sr6) * ir2;
      fx += f * dx;
      fy += f * dy;
      fz += f * dz;
      e += 0.5 * (4.0 * ff.wca_eps * (sr6 * sr6 - sr6) + ff.wca_eps);
    }
  }
  // walls
  const double dmin = pow(0.4, 1.0 / 6.0) * ff.wall_sigma;
  const double sw3 = ff.wall_sigma * ff.wall_sigma * ff.wall_sigma, sw9 = sw3 * sw3 * sw3;
  const double umin = ff.wall_eps * ((2.0 / 15.0) * sw9 / (dmin * dmin * dmin * dmin * dmin * dmin * dmin * dmin * dmin) -
                                     sw3 / (dmin * dmin * dmin));
  auto wall = [&](double d, double& dudd) {
    if (!(d < dmin)) {
      dudd = 0.0;
      return 0.0;
    }
    const double id = 1.0 / d, id3 = id * id * id, id9 = id3 * id3 * id3;
    dudd = ff.wall_eps * (-(18.0 / 15.0) * sw9 * id9 * id + 3.0 * sw3 * id3 * id);
    return ff.wall_eps * ((2.0 / 15.0) * sw9 * id9 - sw3 * id3) - umin;
  };
  double dlo, dhi;
  e += wall(zi - ff.wall_zlo, dlo);
  e += wall(ff.wall_zhi - zi, dhi);
  fz += -dlo + dhi;
  // bonds
  for (int u = 0; u < 2; ++u) {
    const int j = bond[2 * i + u];
    if (j < 0) continue;
    double dx = xi - X[j], dy = yi - X[N + j];
    const double dz = zi - X[2 * N + j];
    dx -= g.Lx * rint(dx * g.invLx);
    dy -= g.Ly * rint(dy * g.invLy);
    const double rr = sqrt(dx * dx + dy * dy + dz * dz), r0 = bond_r0[2 * i + u];
    const double f = -ff.bond_k * (rr - r0) / rr;
    fx += f * dx;
    fy += f * dy;
    fz += f * dz;
    e += 0.25 * ff.bond_k * (rr - r0) * (rr - r0);
  }
  F[i] += fx;
  F[N + i] += fy;
  F[2 * N + i] += fz;
  if (e_ion) e_ion[i] = e;
}

}  // namespace

void launch_ff_forces(const Geom& g, const StepBufs& b, const FFParams& ff, const int* mol, const int* bond,
                      const double* bond_r0, double* F, double* e_ion, hipStream_t s) {
  if (b.max_nrep == 0) return;
  const int ftiles = (b.max_nrep + 255) / 256;
  hipLaunchKernelGGL(k_ff_forces, dim3((unsigned)ftiles * b.R), dim3(256), 0, s, g, b, ff, mol, bond, bond_r0, F,
                     e_ion, ftiles);
}

}  // namespace srbe
