// Forces on the electrode atoms from the estimator of a step (gfx950).
//
// F_j = -Q_j grad Phi*(R_j): the electrode feels the field of every charge through the
// same sampled modes, with its own charge Q_j in place of an ion's q_i.
//   - k-space and slab parts (Eq. (25) and the slab force): the ion force pass run over
//     electrode records that carry Q_j (k_ele_force_records builds them, replica by
//     replica, with offsets r n_ele);
//   - real space (Eq. (13)): the ions around R_j through the ion-Gaussian kernel and
//     the other electrodes through the Gaussian-Gaussian kernel, over the cell lists of
//     the step, in FP64 for both precisions (k_ele_real_forces, one thread per
//     electrode and replica, its cell's neighbour runs in sorted order).
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels.h"

namespace srbe {

namespace {

#define SQRT_PI_INV 0.5641895835477563

// d/dr [erfc(a r) / r]
__device__ __forceinline__ double derfc_over_r(double a, double r) {
  const double ar = a * r;
  return -erfc(ar) / (r * r) - 2.0 * a * SQRT_PI_INV * exp(-ar * ar) / r;
}

__global__ __launch_bounds__(256) void k_ele_force_records(Geom g, StepBufs b, int fp32, int64_t* __restrict__ eoff,
                                                            uint4* __restrict__ r32, double4* __restrict__ r64) {
  const int n = g.n_ele;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t <= b.R) eoff[t] = t * n;
  if (t >= (int64_t)b.R * n) return;
  const int j = (int)(t % n);
  const double Q = b.Q_out[t];
  if (fp32) {
    const uint4 p = b.ele_fx[j];
    r32[t] = make_uint4(p.x, p.y, p.z, __float_as_uint((float)Q));
  } else {
    const double4 p = b.ele_d4[j];
    r64[t] = make_double4(p.x, p.y, p.z, Q);
  }
}

__global__ __launch_bounds__(256) void k_ele_real_forces(Geom g, StepBufs b, int fp32, double* __restrict__ F) {
  const int n = g.n_ele;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t NE = (int64_t)b.R * n;
  if (t >= NE) return;
  const int r = (int)(t / n), j = (int)(t - (int64_t)r * n);
  const int sp = b.ele_iperm[j];
  const int c = b.ele_scell[sp];
  const double4 pe = b.ele_d4[j];
  const double Qj = b.Q_out[t];
  const int64_t b0 = b.off[r];
  const int* cs = b.cstart + (size_t)r * (g.ncell + 1);
  const double rc2 = g.rc * g.rc, a = g.alpha, ai = 1.0 / g.eta, ag = 1.0 / (sqrt(2.0) * g.eta);
  double gx = 0.0, gy = 0.0, gz = 0.0;
  auto add = [&](double sx, double sy, double sz, double q, double ab) {
    double dx = pe.x - sx, dy = pe.y - sy;
    dx -= rint(dx);
    dy -= rint(dy);
    dx *= g.Lx;
    dy *= g.Ly;
    const double dz = (pe.z - sz) * g.Lz;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const double rr = sqrt(r2);
      const double s = q * (derfc_over_r(a, rr) - derfc_over_r(ab, rr)) / rr;
      gx += s * dx;
      gy += s * dy;
      gz += s * dz;
    }
  };
  // the ions of the neighbour runs (ion-Gaussian kernel)
  const int2* runs = b.ion_runs + (size_t)kRunMax * c;
  for (int u = 0; u < kRunMax; ++u) {
    const int2 rc = runs[u];
    if (rc.x < 0) break;
    for (int64_t k = b0 + cs[rc.x]; k < b0 + cs[rc.y]; ++k) {
      if (fp32) {
        const uint4 p = b.sfx[k];
        add((double)p.x * 0x1.0p-32, (double)p.y * 0x1.0p-32, (double)p.z * 0x1.0p-32, b.ion_q[b.perm[k]], ai);
      } else {
        const double4 p = b.sd4[k];
        add(p.x, p.y, p.z, p.w, ai);
      }
    }
  }
  // the other electrodes of the neighbour runs (Gaussian-Gaussian kernel)
  const int4* er = b.ele_rr + (size_t)kRunMax * c;
  for (int u = 0; u < kRunMax; ++u) {
    const int4 e = er[u];
    if (e.x < 0) break;
    for (int pos = e.x; pos < e.y; ++pos) {
      if (pos == sp) continue;
      const double4 p = b.ele_sd4[pos];
      add(p.x, p.y, p.z, b.Q_out[(size_t)r * n + b.ele_perm[pos]], ag);
    }
  }
  const double f = -g.ke * Qj;
  F[t] += f * gx;
  F[NE + t] += f * gy;
  F[2 * NE + t] += f * gz;
}

}  // namespace

void launch_electrode_forces(const Geom& g, const StepBufs& b, int fp32, double* F, int64_t* eoff, void* recs,
                             hipStream_t s) {
  const int64_t NE = (int64_t)b.R * g.n_ele;
  const unsigned blocks = (unsigned)((std::max<int64_t>(NE, (int64_t)b.R + 1) + 255) / 256);
  hipLaunchKernelGGL(k_ele_force_records, dim3(blocks), dim3(256), 0, s, g, b, fp32, eoff,
                     fp32 ? (uint4*)recs : nullptr, fp32 ? nullptr : (double4*)recs);
  StepBufs be = b;
  be.off = eoff;
  be.N = NE;
  be.max_nrep = g.n_ele;
  be.ion_fx = fp32 ? (uint4*)recs : nullptr;
  be.ion_d4 = fp32 ? nullptr : (double4*)recs;
  be.F_out = F;
  launch_ion_force(g, be, fp32, s);
  if (b.real) hipLaunchKernelGGL(k_ele_real_forces, dim3((unsigned)((NE + 255) / 256)), dim3(256), 0, s, g, b, fp32, F);
}

}  // namespace srbe
