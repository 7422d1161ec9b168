// Launch wrappers of the SRBE kernels (host-visible, internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace srbe {

// One mode of a replica for the FP32 potential/force passes (32 bytes, read by
// scalar loads: every lane of a wave walks the same mode list).
struct ModeRec32 {
  int mx, my, mz;
  float cre, cim;  // coefficient w_k S(k) (complex)
  float kx, ky, kz;
};

// Per-step device pointers and sizes.
struct StepBufs {
  int R;                    // replicas
  int64_t N;                // ions over all replicas
  int max_nrep;             // largest ion count of one replica
  const int64_t* off;       // [R+1] CSR offsets (device)
  const double* ion_xyz;    // SoA 3N
  const double* ion_q;      // N
  const double* dpsi;       // R
  const uint64_t* seed;     // R
  uint64_t step;
  const int32_t* kset_in;   // R*P*3 or null
  // electrodes (device, fixed)
  const double* ele_xyz;    // SoA 3*n_ele
  const double* ele_frac;   // SoA 3*n_ele fractional coordinates
  const uint4* ele_fx;      // AoS fixed point
  const double* ele_d;      // n_ele
  // workspace
  double* scal;             // R*4: sum q, sum |q|, sum q z, sum q^2
  int4* modes;              // R*K
  double* w;                // R*K
  double* ion_frac;         // SoA 3N (FP64 path)
  uint4* ion_fx;            // N (FP32 path)
  double2* part;            // R*nchunk*K
  int nchunk_ion, nchunk_ele;
  double2* S1;              // R*K
  double2* coef;            // R*K
  ModeRec32* rec;           // R*K (FP32 path)
  double* bstar;            // R*n_ele
  double* V;                // R*n_ele (dpsi d + b*), GEMM right-hand side, ld n_ele
  double* Qext;             // R*(n_ele+1) GEMM output (Q then psibar), ld n_ele+1
  float* Qf;                // R*n_ele FP32 copy of Q (FP32 path)
  double* rsum;             // R*8 per-replica reductions after the charge solve
  double* phi;              // N real-space ion-ion potential per ion
  unsigned* status;
  // outputs
  double* Q_out;
  double* F_out;
  double* psibar_out;
  double* energy_out;
  int32_t* kset_out;
  int32_t* nacc_out;
  const double* Q_in;
};

void launch_replica_scalars(const Geom& g, const StepBufs& b, hipStream_t s);
void launch_sample(const Geom& g, const StepBufs& b, hipStream_t s);
void launch_prep(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_sf_ions(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_sf_finalize(const Geom& g, const StepBufs& b, int stage, int fp32, hipStream_t s);
void launch_ele_potential(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_post_charges(const Geom& g, const StepBufs& b, int fixedQ, hipStream_t s);
void launch_sf_ele(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_ion_force(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_energy(const Geom& g, const StepBufs& b, int fixedQ, hipStream_t s);

// setup kernels
void launch_ele_phase_block(const double* ele_xyz, int n_ele, const int* m, const double* sqrtw, int nk, int ld,
                            double* E, const Geom& g, hipStream_t s);
void launch_ele_realspace_matrix(const Geom& g, const double* ele_xyz, int n_ele, double* A, hipStream_t s);
void launch_ele_fixed(const Geom& g, const double* ele_xyz, int n_ele, double* frac, uint4* fx, hipStream_t s);
void launch_symmetrize_lower(double* A, int n, int ld, hipStream_t s);
void launch_rowsum(const double* A, int n, int ld, double* out, hipStream_t s);
void launch_build_sext(const double* Ainv, int n, const double* g, double eg, double* Sext, hipStream_t s);
void launch_check_finite(const double* a, size_t n, unsigned* status, hipStream_t s);

}  // namespace srbe
