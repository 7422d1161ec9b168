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

// Workspace of the multi-block cell sort (count null: the one-block sort is used).
struct BigSort {
  int* count;     // R*(ncell+1) cell counts, then per-cell cursors
  int* prov;      // N provisional cell order (indices within the replica)
  double* tsum;   // R*ntile*4 charge sums per tile of 256 particles (ions)
  int* ctot;      // R*nchunk totals, then offsets, of the chunks of 1024 cells
  int ntile;      // tiles of 256 particles per replica
  int nchunk;     // chunks of 1024 cells: (ncell + 1024) / 1024 <= 1024
};

// Charge solve over two electrode lattices (SRBE_FLAG_LATTICE_SOLVE; nx 0: not used).
// Sites (w, iy, ix) of wall w; modes (p, q) with p along x.
struct LatticeSolve {
  int nx, ny;               // sites per wall along x and y (<= 768 each: LDS of the column launch)
  const int* site;          // 2*ny*nx electrode index of site (w, iy, ix)
  const double2* tw_x;      // nx: exp(-2 pi i j / nx)
  const double2* tw_y;      // ny: exp(-2 pi i j / ny)
  const double2* linv;      // ny*nx*4: Lambda(p, q)^-1 (00, 01, 10, 11) at (q nx + p) 4
  double c0, c1;            // A^-1 e on wall 0 and wall 1 (constant on each)
  double etc;               // e^T A^-1 e
  double2* T;               // workspace R*2*ny*nx: transforms along x
  double2* U;               // workspace R*2*ny*nx: solved modes, inverted along y
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
  const uint64_t* step_dev; // graph replays: the step is read from here (null: use step)
  uint64_t* step_adv;       // graph replays: the step counter the last kernel advances (else null)
  const int32_t* kset_in;   // R*P*3 or null
  const double* logq;       // sampler table of log q_d(m), |m| <= qmax[d] (per handle)
  // electrodes (device, fixed): original order and cell-sorted order
  const double* ele_xyz;    // SoA 3*n_ele
  const double* ele_d;      // n_ele
  const uint4* ele_fx;      // n_ele fixed point (original order)
  const double4* ele_d4;    // n_ele fractional coordinates (original order), w = 0
  const int* ele_perm;      // sorted position -> electrode index
  const int* ele_iperm;     // electrode index -> sorted position
  const int* ele_scell;     // cell of each sorted electrode
  const int* ele_cstart;    // ncell + 1
  const double2* ele_czr;   // ncell: z-extent of the electrodes of each cell
  const int2* ion_runs;     // ncell x kRunMax neighbour runs [c0, c1), merged across z; c0 = -1 ends
  const int4* ele_rr;       // ncell x kRunMax electrode runs (one z-layer each): sorted range [x, y),
                            // z-extent as float bits (z, w); x = -1 ends a cell's list
  const int2* reach;        // cell ranges [c0, c1) whose ions can be within rc of an electrode
  int nreach;
  const unsigned char* reach_cell;  // ncell flags: 1 for the cells of those ranges
  const int4* ele_chunks;   // (cell, first, end) runs of <= 64 cell-sorted electrodes of one cell
  int n_ele_chunks;
  const uint4* ele_sfx;     // sorted fixed point
  const double4* ele_sd4;   // sorted fractional coordinates
  // workspace
  double* scal;             // R*4: sum q, sum |q|, sum q z, sum q^2
  int4* modes;              // R*K
  double* w;                // R*K
  uint4* ion_fx;            // N fixed point + FP32 charge, original order (FP32 path)
  double4* ion_d4;          // N fractional coordinates + charge, original order (FP64 path)
  unsigned* keys;           // N cell sort keys, input order: cell << 13 | index within the replica
                            // (one-block sort), or the cell (multi-block sort)
  int* perm;                // N sorted position (within the replica's range) -> global ion index
  int* scell;               // N cell of each sorted ion
  int* cstart;              // R*(ncell+1) cell starts, relative to the replica's first ion
  uint4* sfx;               // N sorted fixed point (FP32 path)
  double4* sd4;             // N sorted fractional coordinates (FP64 path)
  double2* part;            // R*nchunk*K partial structure factors
  int nchunk_ion, nchunk_ele, ktiles;
  double2* S1;              // R*K
  double2* coef;            // R*K
  ModeRec32* rec;           // R*K (FP32 path)
  double* bN;               // R*n_ele real-space electrode potential from the ions
  double* bstar;            // R*n_ele
  double* V;                // R*ldcp(n_ele) (dpsi d + b*), GEMM right-hand side, V[r ldcp(n) + j]
  double* Qext;             // ksplit*R*(n_ele+1) GEMM partials over k-ranges (Q then psibar),
                            // Qext[(h R + r)(n+1) + i], summed in h order after the GEMM
  int ksplit;
  int ii_ipw;               // ion-ion pass: consecutive sorted ions per wave
  int ie_nbx;               // ion-electrode pass: blocks per replica
  int kw;                   // potential and force passes: waves per 64-particle block (2, 4, 8)
  int unroll;               // their FP32 mode-loop unroll depth (2, 4, 8)
  int esplit;               // electrode-potential real-space pass: waves per electrode chunk (1, 2, 4)
  int gemm_depth;           // charge-solve GEMM: contraction block of 16 gemm_depth (1 or 2)
  int real;                 // 1: the real-space terms are part of the step; 0: k-space only
  int bf16;                 // FP32 path with the structure factors' products from BF16 hi/lo halves
  float* Qf;                // R*n_ele FP32 copy of Q, original order (FP32 path)
  float* Qsf;               // R*n_ele FP32 Q in sorted electrode order (FP32 path)
  double* Qsd;              // R*n_ele FP64 Q in sorted electrode order (FP64 path)
  double* rsum;             // R*kRsumStride per-replica sums after the charge solve (kRsumParts partials)
  double* phi;              // N real-space ion-ion potential per ion
  double* Fii;              // 3N ion-ion real-space force sums (SoA, input order), before the ke q_i factor
  double* Fie;              // 3N ion-electrode real-space force sums, written for ions of reach cells only
  unsigned* status;
  BigSort bigsort;          // multi-block cell sort workspace (count null: one-block sort)
  LatticeSolve lat;         // lattice charge solve (lat.nx 0: the dense GEMM)
  double* eparts;           // R*etiles partial sums of q phi over tiles of kEnergyTile ions
  int etiles;               // tiles per replica (0: the energy sums the ions itself)
  int estride;              // energy_out values per replica: 1 (E*) or 5 (E* and its parts)
  double* epair;            // R*epair_nb partial sums of the electrode-electrode real-space
                            // energy (parts only), one per block of 256 electrodes
  int epair_nb;
  // outputs
  double* Q_out;
  double* F_out;
  double* psibar_out;
  double* energy_out;
  int32_t* kset_out;
  int32_t* nacc_out;
  const double* Q_in;
  const double* Sext;       // the dense charge solve's S_ext (null: lattice solve or fixed charges)
};

// Multi-system launches: one launch runs a phase of the step for every system of a
// batch (systems of different geometry, each with its own replicas).  Block L of the
// launch belongs to system s with start[s] <= L < start[s + 1] and runs that system's
// block L - start[s] with its descriptor d[s] (the Geom and StepBufs a single-system
// launch would take) and its integer arguments iarg[kMultiArgs s ..].
struct SysDesc {
  Geom g;
  StepBufs b;
};
constexpr int kMultiArgs = 4;
struct MultiLaunch {
  const SysDesc* d;   // nsys
  const int* start;   // nsys + 1
  const int* iarg;    // nsys x kMultiArgs
  int nsys;
  uint64_t* step_adv; // the final phase's first block advances this counter (graph replays), or null
};

// The system of block L (wave-uniform binary search over the block starts).
__device__ __forceinline__ int multi_system(const MultiLaunch& m, int L) {
  int lo = 0, hi = m.nsys;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (m.start[mid] <= L) lo = mid; else hi = mid;
  }
  return lo;
}

// Phases of the multi-system launches (launch_multi).
enum MultiPhase {
  MP_FRONT = 0,        // iarg: nsamp (sampler blocks before the one-block sorts)
  MP_BS_ZERO,          // multi-block sort: clear the counts (blocks of 256 counts)
  MP_BS_COUNT, MP_BS_SCAN_CHUNKS, MP_BS_SCAN_TOTALS, MP_BS_SCAN_OFFSETS, MP_BS_SCATTER, MP_BS_RANK,
  MP_STAGE_IONS,       // iarg: nsf, nre, esplit
  MP_SF_FINALIZE,      // iarg: stage
  MP_ELEPOT,           // iarg: electrode tiles of 64
  MP_CP_GEMM,          // iarg: row tiles, replica tiles
  MP_POST_CHARGES,     // iarg: fixedQ
  MP_STAGE_ELE,        // iarg: nsf, nie
  MP_ION_FORCE,        // iarg: ion tiles of 64
  MP_REAL_II,          // iarg: tiles
  MP_ENERGY_PARTS,
  MP_FINAL,            // iarg: ne, fixedQ, first ion, ions
};
// Launch one phase for the systems of m (nblocks = m's start[nsys]); fp32, W (waves per
// block of the potential and force passes), U (their unroll) and KB (GEMM contraction
// block) select the kernel and must be the same for every system.
void launch_multi(int phase, int fp32, int W, int U, int KB, const MultiLaunch& m, int nblocks, size_t lds,
                  hipStream_t s);
// The lattice solve's three launches (step 0, 1, 2) for the lattice systems of m; grid of
// one system's step: lattice_grid.
void launch_multi_lattice(int step, const MultiLaunch& m, int nblocks, size_t lds, hipStream_t s);
void lattice_grid(const StepBufs& b, int step, int& blocks, size_t& lds);
size_t sample_lds_bytes(int P);

// Parts of the fused launches (bit masks).  A step runs each fused launch whole; with
// phase timing on, each part is launched on its own so that it can be timed.
enum { FRONT_SAMPLE = 1, FRONT_SORT = 2 };
enum { STAGE_SF = 1, STAGE_REAL = 2 };

void launch_front(const Geom& g, const StepBufs& b, int fp32, int parts, hipStream_t s);
void launch_set_step(uint64_t* step_dev, uint64_t v, hipStream_t s);
void launch_logq_table(const Geom& g, double* T, hipStream_t s);
void launch_stage_ions(const Geom& g, const StepBufs& b, int fp32, int parts, hipStream_t s);
void launch_sf_finalize(const Geom& g, const StepBufs& b, int fp32, int stage, hipStream_t s);
void launch_ele_potential(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
int cp_gemm_ksplit(int n_ele, int R);
int ele_split(int units);
// nothing is launched if Sext is null (fixed charges)
void launch_cp_gemm(const Geom& g, const StepBufs& b, const double* Sext, hipStream_t s);
// the lattice charge solve: (Q; psibar) of every replica into Qext (one k-range)
void launch_lattice_solve(const Geom& g, const StepBufs& b, hipStream_t s);
// the short-range force field of the dynamics (srbe_ff in srbe.h)
struct FFParams {
  double wca_eps, wca_sigma, wall_eps, wall_sigma, wall_zlo, wall_zhi, bond_k;
};
// adds the force field's forces to F (SoA 3N) over the cell lists of the step b; e_ion: N or null
void launch_ff_forces(const Geom& g, const StepBufs& b, const FFParams& ff, const int* mol, const int* bond,
                      const double* bond_r0, double* F, double* e_ion, hipStream_t s);
// one Euler-Maruyama step of the Langevin thermostat for n ions (SoA, in place); with
// step_dev set, the step index is *step_dev - 1 (a captured dynamics step reads the
// counter its SRBE step has just advanced)
void launch_langevin(int64_t n, double* xyz, double* vel, const double* F, const double* mass, double gamma,
                     double beta, double dt, double Lx, double Ly, double zlo, double zhi, uint64_t seed,
                     uint64_t step, hipStream_t s, const uint64_t* step_dev = nullptr, int symplectic = 0);
// forces on the electrodes from the state b of a finished step: F (SoA, 3 R n_ele);
// eoff: R + 1 int64 scratch, recs: R n_ele records (uint4 FP32 / double4 FP64) scratch
void launch_electrode_forces(const Geom& g, const StepBufs& b, int fp32, double* F, int64_t* eoff, void* recs,
                             hipStream_t s);
void launch_post_charges(const Geom& g, const StepBufs& b, int fixedQ, int fp32, hipStream_t s);
void launch_ele_pair_energy(const Geom& g, const StepBufs& b, hipStream_t s);
size_t virial_scratch_doubles(const Geom& g, const StepBufs& b);
void launch_virial(const Geom& g, const StepBufs& b, double* scratch, double* W, hipStream_t s);
void launch_stage_ele(const Geom& g, const StepBufs& b, int fp32, int parts, hipStream_t s);
void launch_ion_force(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_real_ii(const Geom& g, const StepBufs& b, int fp32, hipStream_t s);
void launch_final(const Geom& g, const StepBufs& b, int fixedQ, hipStream_t s);

// setup kernels
// bs.count null: the one-block sort (n_ele <= kMaxBinParticles and ncell <= kMaxCells)
void launch_bin_electrodes(const Geom& g, const int64_t* off2, const double* ele_xyz, int n_ele, unsigned* keys,
                           uint4* fx, double4* d4, int* perm, int* scell, int* cstart, uint4* sfx, double4* sd4,
                           unsigned* status, const BigSort& bs, hipStream_t s);
// true if a batch whose largest replica holds max_particles needs the multi-block sort
bool use_big_sort(const Geom& g, int64_t max_particles);
void launch_cell_zrange(const Geom& g, const int* cstart, const double* ele_xyz, const int* perm, double2* zr,
                        hipStream_t s);
void launch_ele_phase_block(const double* ele_xyz, int n_ele, const int* m, const double* sqrtw, int nk, int ld,
                            double* E, const Geom& g, hipStream_t s);
void launch_ele_realspace_matrix(const Geom& g, const double* ele_xyz, int n_ele, double* A, hipStream_t s);
void launch_symmetrize_lower(double* A, int n, int ld, hipStream_t s);
void launch_rowsum(const double* A, int n, int ld, double* out, hipStream_t s);
void launch_build_sext(const double* Ainv, int n, const double* g, double eg, double* Sext, hipStream_t s);
void launch_check_finite(const double* a, size_t n, unsigned* status, hipStream_t s);

}  // namespace srbe
