/*
 * srbe.h -- C ABI of the SRBE constant-potential step on AMD MI355X (gfx950).
 *
 * The library implements the per-timestep electrostatics of the symmetry-
 * preserving random batch Ewald (SRBE) method for electrode/electrolyte slabs
 * (Gao, Zhou, Zhang, Xu, arXiv 2509.24742):
 *
 *   - structure factors S(k) = sum_j q_j exp(i k.r_j) (Eq. (15)) over the
 *     deterministic modes I = {(0,0,2 pi m/Lz): 1 <= |m| <= M} and a random batch
 *     of P modes drawn from exp(-k^2/(4 alpha^2))/G on the remaining lattice
 *     (Eqs. (26)-(29));
 *   - the electrode vector b* (Eq. (24) plus the exact slab and real-space terms of
 *     Eq. (19)) and the constant-potential charges Q = J A^-1 (dpsi d + b*) with
 *     the average potential psibar (Eqs. (9)-(11));
 *   - the ion forces F* (Eq. (25) plus slab and real-space terms) and the energy.
 *
 * Conventions shared by every call
 *   Units are the caller's; every Coulomb term carries params.coulomb_k
 *   (1.43996454784 eV nm / e^2 for nm, e, V, eV).  Positions are structure-of-
 *   arrays: x[0..n), y[0..n), z[0..n) contiguous in one buffer of 3n doubles.
 *   The box is [0,Lx) x [0,Ly) x [0,H], periodic in x and y; z is padded to
 *   Lz = lambda H with the slab correction of Eq. (17).
 *   "host" pointers are read during the call and not retained; "device" pointers
 *   are HIP device memory owned by the caller, read or written asynchronously on
 *   the stream passed to the call, and not retained after the work completes.
 *   A handle is not thread-safe; distinct handles are independent.  A handle
 *   lives on the HIP device that was current when it was created.
 *
 * Errors
 *   Every int-returning call returns SRBE_OK (0) or a negative code below.
 *   Argument checks run synchronously before anything is enqueued.  Checks that
 *   need device data (neutrality, z range, non-finite values) are made by the
 *   kernels; they set a device status word that srbe_sync_status() reports.
 */
#ifndef SRBE_H
#define SRBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRBE_OK 0
#define SRBE_EINVAL (-1)     /* invalid argument                                  */
#define SRBE_ENONNEUTRAL (-2) /* ions of a replica are not neutral               */
#define SRBE_ERANGE (-3)     /* a particle lies outside [0,H] in z, or non-finite  */
#define SRBE_ENOTSPD (-4)    /* electrode matrix A is not positive definite        */
#define SRBE_ENOMEM (-5)     /* device allocation failed                           */
#define SRBE_EHIP (-6)       /* HIP runtime or ROCm library error                  */
#define SRBE_ENUMERIC (-7)   /* non-finite value produced on the device            */

#define SRBE_FP64 0 /* every pass in FP64                                              */
#define SRBE_FP32 1 /* structure factors, potentials and forces in FP32 with exact
                       integer phases and FP64 carries; CP solve and energy in FP64   */
#define SRBE_BF16 2 /* SRBE_FP32 with every product q cos, q sin of the structure
                       factors (Eq. (15)) formed from BF16 hi/lo halves, q_hi c_hi +
                       q_hi c_lo + q_lo c_hi with FP32 accumulation: the arithmetic of a
                       BF16 matrix-core structure factor, for an error report (single
                       systems and srbe_step / srbe_graph_create only)                */

#define SRBE_FLAG_NO_CP 1 /* skip the electrode matrix: only fixed-charge steps      */
#define SRBE_FLAG_KSPACE_ONLY 2 /* leave out the real-space erfc terms (see below)   */
#define SRBE_FLAG_LATTICE_SOLVE 4 /* electrodes on two rectangular lattices: solve the
                                     charges in lattice Fourier space (see below)     */
#define SRBE_FLAG_ENERGY_PARTS 8 /* energy_out holds E* and its four parts per replica
                                    (see srbe_step)                                   */
#define SRBE_FLAG_IID_SAMPLER 16 /* draw the P modes i.i.d. by rejection sampling instead
                                    of by the Metropolis chain (see srbe_sample)      */

typedef struct srbe_params {
  double Lx, Ly, H;   /* box (length); electrodes and ions have 0 <= z <= H           */
  double lambda;      /* zero-padding ratio, Lz = lambda * H; lambda >= 1 and
                         (lambda - 1) * H > rc                                        */
  double alpha;       /* Ewald splitting parameter (1/length), Eq. (12)               */
  double eta;         /* width of the electrode Gaussians (a length), Eq. (1)         */
  double rc;          /* real-space cutoff, 0 < rc <= min(Lx, Ly) / 2                 */
  double coulomb_k;   /* Coulomb constant multiplying every electrostatic term        */
  double kspace_tol;  /* the reciprocal sum of A keeps every k with
                         exp(-k^2/(4 alpha^2)) >= kspace_tol (0 < tol < 1)            */
  int32_t M;          /* deterministic modes m_z = 1..M (M >= 0)                      */
  int32_t P;          /* random batch size, 0 <= P <= 2048                            */
  int32_t flags;      /* SRBE_FLAG_*                                                  */
  int32_t reserved;   /* must be 0                                                    */
} srbe_params;

typedef struct srbe_system srbe_system;

/*
 * srbe_create -- set up one electrode geometry (Sec. 2, Eqs. (18), (9)-(11)).
 *
 * ele_xyz  host, 3*n_ele doubles (SoA), electrode positions R_j.
 * ele_side host, n_ele int8: -1 for the negative, +1 for the positive electrode
 *          (d_j = side_j / 2 in Eq. (7)).
 * Builds A (Eq. (18); its slab entry is taken as (4 pi / V) Z_i Z_j, the Hessian of
 * the slab term of Eq. (17)), factorises it, and keeps S = J A^-1 and
 * -e^T A^-1 / (e^T A^-1 e) on the device.  Also evaluates G of Eq. (27).
 * With SRBE_FLAG_NO_CP set, A is not built and n_ele may be large; steps must
 * then pass Q_in.  With SRBE_FLAG_KSPACE_ONLY set, steps leave out the short-range
 * erfc terms of Eq. (13) -- the real-space part of b (Eq. (19)), the real-space
 * forces and the ion-ion real-space energy -- and skip their passes: for use beside
 * a pair code that computes them, and to attribute errors to the two parts (A, if
 * built, stays complete).
 * With SRBE_FLAG_LATTICE_SOLVE set, the electrodes must form two walls (two distinct
 * z), each a complete nx x ny rectangular lattice of spacing (Lx/nx, Ly/ny) with the
 * same nx, ny (at most 768 each) on both walls and any in-plane offset per wall, and
 * rc < min(Lx, Ly)/2.
 * A (Eq. (18)) is then block-circulant over the lattice: it is never formed, and the
 * charge update of Eqs. (9)-(11) runs per in-plane lattice mode (p, q) as a 2 x 2
 * solve between discrete Fourier transforms over the walls, with O(n_ele) memory.
 * Results equal the dense solve's to rounding, except where sites lie exactly rc
 * apart: the dense build decides each such pair from rounded coordinate differences
 * (A is then not exactly block-circulant), the lattice solve from the lattice
 * displacement.  Not a lattice: SRBE_EINVAL.
 * On success *out receives the handle; on failure *out is NULL.
 * Errors: SRBE_EINVAL, SRBE_ENOTSPD (A not positive definite, e.g. two electrodes
 * at one position), SRBE_ENOMEM, SRBE_EHIP.
 */
int srbe_create(const srbe_params* params, int32_t n_ele, const double* ele_xyz,
                const int8_t* ele_side, srbe_system** out);

/* srbe_destroy -- free the handle and its device memory (synchronises the device). */
void srbe_destroy(srbe_system* h);

/* srbe_last_error -- message of the last failure on this handle ("" if none). */
const char* srbe_last_error(const srbe_system* h);

/* srbe_error_string -- static description of an error code. */
const char* srbe_error_string(int code);

/*
 * srbe_step -- one SRBE step for n_rep replicas sharing the handle's electrodes
 * (Algorithm 1: sample P modes, compute b* by Eq. (24), update Q by Eq. (10),
 * compute the forces of Eq. (25) and the real-space forces; no integration).
 *
 * precision   SRBE_FP64, SRBE_FP32 or SRBE_BF16.
 * n_rep       number of replicas, 1 <= n_rep <= 65535.
 * ion_offsets host, n_rep+1 int64, CSR offsets: replica r owns ions
 *             [ion_offsets[r], ion_offsets[r+1]); ion_offsets[0] == 0.
 * ion_xyz     device, 3*N doubles SoA (N = ion_offsets[n_rep]).
 * ion_q       device, N doubles.  Each replica's ions must be neutral.
 * dpsi        device, n_rep doubles: potential difference Delta psi per replica.
 * seed        device, n_rep uint64: sampler seed per replica.
 * step        step index; with the seed it fixes the sample (counter-based RNG).
 * kset_in     device, n_rep*P*3 int32 (m_x, m_y, m_z per sampled mode), or NULL to
 *             sample on the device.  Each given mode must lie in L_k \ I.
 * Q_in        device, n_rep*n_ele doubles, or NULL.  Non-NULL: fixed electrode
 *             charges (the CP solve is skipped; Q_out receives a copy).
 * Q_out       device, n_rep*n_ele doubles: electrode charges.
 * F_out       device, 3*N doubles SoA: total force on every ion.
 * b_out       device, n_rep*n_ele doubles (b* per replica) or NULL.
 * psibar_out  device, n_rep doubles or NULL (NaN in fixed-charge steps).
 * energy_out  device, n_rep doubles or NULL: E* = 1/2 Q^T A Q - b*^T Q + c*, with
 *             c* the ion-ion energy using the same estimator (requires the CP
 *             solve; NaN in fixed-charge steps).  With SRBE_FLAG_ENERGY_PARTS set at
 *             creation: 5 doubles per replica, [total E*, real, fourier, self, slab],
 *             split as U_c is in Eqs. (13), (16), (17): real = every erfc pair term
 *             (ion-ion, ion-electrode, electrode-electrode; 0 with KSPACE_ONLY), self
 *             and slab = the two terms of Eq. (17) over ions and electrodes, fourier =
 *             the rest (the only part the sample changes; its mean over samples is the
 *             complete Fourier energy of Eq. (16)).  The electrode-electrode pair sum
 *             adds one pass over the electrodes' neighbours per step.  Not allowed in a
 *             batch of systems (srbe_batch_create refuses such handles).
 * kset_out    device, n_rep*P*3 int32 or NULL: the modes used.
 * stream      hipStream_t on which all work is enqueued (NULL = default stream).
 * Errors: SRBE_EINVAL (synchronous); device-data errors via srbe_sync_status.
 */
int srbe_step(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
              const double* ion_xyz, const double* ion_q, const double* dpsi, const uint64_t* seed,
              uint64_t step, const int32_t* kset_in, const double* Q_in, double* Q_out, double* F_out,
              double* b_out, double* psibar_out, double* energy_out, int32_t* kset_out, void* stream);

/*
 * srbe_step_noalloc -- srbe_step without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks, kernels and results as srbe_step (bitwise equal).
 * The step's workspace and its copy of ion_offsets live in a fixed device array of
 * 64 MiB inside the library, one per GPU, held until the process ends; a step needing
 * more (about 100 bytes per ion plus per-replica and per-mode terms: some 28 MB for 64
 * paper-shaped cells) is refused with SRBE_EINVAL (srbe_last_error gives the size)
 * before anything is enqueued.  Every call on one GPU, from any handle, shares that
 * array, so calls whose work overlaps in time on one GPU (other streams, other threads)
 * race and give wrong results: order them on one stream or synchronise between them.
 * ion_offsets is copied to the device by an asynchronous copy on stream (pageable host
 * memory is read before the call returns; pinned memory must stay unchanged until the
 * stream reaches the copy).  srbe_electrode_forces cannot follow this call (its state
 * is in the shared array).  No per-phase timing.  Calls no hipMalloc or hipFree.
 * Errors: as srbe_step.
 */
int srbe_step_noalloc(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                      const double* ion_xyz, const double* ion_q, const double* dpsi, const uint64_t* seed,
                      uint64_t step, const int32_t* kset_in, const double* Q_in, double* Q_out, double* F_out,
                      double* b_out, double* psibar_out, double* energy_out, int32_t* kset_out, void* stream);

/*
 * Captured steps.  srbe_graph_create records one srbe_step with fixed arguments
 * (the same meaning and checks as srbe_step, all device pointers kept by the
 * graph) into a HIP graph with its own workspace; srbe_graph_launch replays it on
 * any stream as one launch.  The sample of a replay is fixed by (seed, step) as in
 * srbe_step, where step comes from a device counter: first_step for the first
 * replay, advanced by one at the end of every replay, and reset by
 * srbe_graph_set_step (enqueued on the given stream).  The buffers passed at
 * creation must stay allocated, and their contents are read and written at each
 * replay.  Replays on one graph must not overlap in time (they share the
 * workspace); the graph must be destroyed before its handle.  Errors:
 * SRBE_EINVAL, SRBE_ENOMEM, SRBE_EHIP; device-data errors via srbe_sync_status.
 */
typedef struct srbe_graph srbe_graph;
int srbe_graph_create(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                      const double* ion_xyz, const double* ion_q, const double* dpsi, const uint64_t* seed,
                      uint64_t first_step, const int32_t* kset_in, const double* Q_in, double* Q_out,
                      double* F_out, double* b_out, double* psibar_out, double* energy_out, int32_t* kset_out,
                      srbe_graph** out);
int srbe_graph_launch(srbe_graph* g, void* stream);
int srbe_graph_set_step(srbe_graph* g, uint64_t step, void* stream);
void srbe_graph_destroy(srbe_graph* g);

/*
 * Batches of systems of different geometry (Sec. 2-3 for each system; the same step as
 * srbe_step).  srbe_batch_create groups existing handles (each its own box, electrodes,
 * alpha, M, P, precision-independent set-up); a batch step then runs every replica of
 * every system through the step with ONE launch per phase for all systems together (each
 * launch's blocks look up their system in a per-system table of geometry and buffers),
 * instead of one launch per phase and system.  Results equal srbe_step's for each system
 * to rounding order (the same kernels and per-system launch shapes).
 *
 * srbe_batch_create -- systems: host array of n_systems handles (1..4096, all on one
 * device, none created with SRBE_FLAG_ENERGY_PARTS), not owned: they must outlive the
 * batch and its graphs.
 * srbe_batch_step -- n_rep replicas, replica r belonging to system system_of_replica[r]
 * (host int32, non-decreasing, so each system's replicas are consecutive).
 * ion_offsets host n_rep + 1 int64 CSR over all replicas (ion_offsets[0] = 0); ion_xyz
 * (device 3N SoA), ion_q (N), F_out (3N SoA) as in srbe_step over the whole batch.
 * Per replica: dpsi, seed (device, n_rep; seed may be NULL only if no system has P > 0),
 * psibar_out (device, n_rep, required), energy_out (device, n_rep, or NULL).  Electrode
 * arrays are CSR over replicas: replica r's n_ele(system) entries start at the sum of
 * the n_ele of the replicas before it -- Q_out (required), Q_in (fixed charges, or NULL
 * for the constant-potential solve), b_out (or NULL).  Launch shapes: each system's
 * stored parameters for its (precision, replica count, largest replica), else its
 * defaults, with 4 waves and unroll 4 in the potential and force passes and 16-wide
 * GEMM blocks for all; in FP32 the defaults' real-space work splits and structure-factor
 * chunks are sized from the whole batch (each system its share of the batch's ions),
 * so FP32 sums may run in another order than in a single-system step.  The modes are sampled on the device (no kset_in / kset_out).  Asynchronous
 * on stream; device faults land in each system's status word (srbe_batch_sync_status).
 * Errors: SRBE_EINVAL, SRBE_ENOMEM, SRBE_EHIP (srbe_batch_last_error gives a message).
 * srbe_batch_graph_* -- the batch step captured with fixed arguments, as srbe_graph_*.
 * srbe_batch_sync_status -- srbe_sync_status of every system (the first fault found).
 */
typedef struct srbe_batch srbe_batch;
typedef struct srbe_batch_graph srbe_batch_graph;
int srbe_batch_create(srbe_system* const* systems, int32_t n_systems, srbe_batch** out);
void srbe_batch_destroy(srbe_batch* b);
const char* srbe_batch_last_error(const srbe_batch* b);
int srbe_batch_sync_status(srbe_batch* b);
int srbe_batch_step(srbe_batch* b, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                    const int32_t* system_of_replica, const double* ion_xyz, const double* ion_q, const double* dpsi,
                    const uint64_t* seed, uint64_t step, const double* Q_in, double* Q_out, double* F_out,
                    double* b_out, double* psibar_out, double* energy_out, void* stream);
int srbe_batch_graph_create(srbe_batch* b, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                            const int32_t* system_of_replica, const double* ion_xyz, const double* ion_q,
                            const double* dpsi, const uint64_t* seed, uint64_t first_step, const double* Q_in,
                            double* Q_out, double* F_out, double* b_out, double* psibar_out, double* energy_out,
                            srbe_batch_graph** out);
int srbe_batch_graph_launch(srbe_batch_graph* g, void* stream);
int srbe_batch_graph_set_step(srbe_batch_graph* g, uint64_t step, void* stream);
void srbe_batch_graph_destroy(srbe_batch_graph* g);

/*
 * srbe_electrode_forces -- forces on the electrode atoms from the estimator of the last
 * srbe_step on this handle: F_j = -Q_j grad Phi*(R_j), with the same sampled modes,
 * charges and positions.  Its parts:
 *   - the Fourier force of Eq. (25) with Q_j in place of q_i, and the slab force;
 *   - the real-space forces of Eq. (13) from the ions (ion-Gaussian kernel) and from
 *     the other electrodes (Gaussian-Gaussian kernel), in FP64 for both precisions.
 * The Fourier part runs in the step's precision.  With the ion forces it conserves
 * momentum per sample: the sum of all forces vanishes.
 * n_rep       the replica count of that step (checked).
 * F_ele_out   device, 3*n_rep*n_ele doubles SoA (x of every replica's electrodes, then y,
 *             then z); replica-major, electrodes in srbe_create order.
 * Must follow an srbe_step (eagerly, not a graph replay) on the same stream, whose
 * input, Q_out and F_out buffers are still valid, with no other srbe_step on the handle
 * in between.  Allocates and frees scratch, and blocks until done.
 * Errors: SRBE_EINVAL (no preceding step, another n_rep, NULL output), SRBE_ENOMEM,
 * SRBE_EHIP.
 */
int srbe_electrode_forces(srbe_system* h, int32_t n_rep, double* F_ele_out, void* stream);

/*
 * srbe_virial -- the electrostatic virial tensor W = -dE/d(epsilon) of the last
 * srbe_step's estimator on this handle, for the pressure tensor
 * P = (sum_i m_i v_i v_i^T + W + W_short-range) / V (kinetic and short-range parts are the
 * caller's).  The paper gives forces (Eqs. (21), (25)) but no virial; this is the
 * derivative under an affine strain of every position and of the box, at fixed
 * charges, with the kernels' alpha and Gaussian width fixed:
 *   - Fourier part: over the step's modes and weights (deterministic kz modes and the
 *     sample, as in Eq. (24)), sum 1/2 w |S|^2 [I - 2 (1 + k^2/(4 alpha^2)) k k^T / k^2]
 *     with S = S1 + S2 of the step (unbiased for the complete Fourier virial);
 *   - real part (Eq. (13)): -sum over pairs within rc of q_a q_b K'(r) r r^T / r over
 *     ion-ion, ion-Gaussian and Gaussian-Gaussian pairs (none with KSPACE_ONLY);
 *   - slab term of Eq. (17): (2 pi / V) M_z^2 diag(1, 1, -1), M_z = sum q z + sum Q Z.
 * FP64 throughout, in both precisions (the Fourier part from the step's FP64 S).
 * n_rep       the replica count of that step (checked).
 * W_out       device, 6*n_rep doubles: [xx, yy, zz, xy, xz, yz] per replica, times
 *             coulomb_k (energy units).
 * Must follow an srbe_step (eagerly, not a graph replay) on the same stream, whose
 * input and Q_out buffers are still valid, with no other srbe_step on the handle in
 * between.  Allocates and frees scratch, and blocks until done.
 * Errors: SRBE_EINVAL (no preceding step, another n_rep, NULL output), SRBE_ENOMEM,
 * SRBE_EHIP.
 */
int srbe_virial(srbe_system* h, int32_t n_rep, double* W_out, void* stream);

/*
 * srbe_langevin_update -- one Euler-Maruyama step of the Langevin thermostat (Sec. 3)
 * for n ions, in place, from the forces of a step:
 *   r <- r + v dt;  v <- v + (F - gamma v) dt / m + sqrt(2 gamma / beta) dW / m,
 * dW ~ N(0, dt) per component.  x and y wrap into [0, Lx) and [0, Ly); z is reflected
 * specularly into [zlo, zhi] as many times as it takes to land inside (zlo < zhi), v_z
 * changing sign once per reflection (a stand-in for the wall force field; ion-ion
 * repulsion is not modelled here: dynamics need a short-range force field added to F).
 * xyz, vel  device, 3n doubles SoA each, updated in place.
 * F         device, 3n doubles SoA (e.g. F_out of srbe_step).
 * mass      device, n doubles.
 * gamma >= 0 friction, beta > 0 inverse temperature (infinity: no noise), dt > 0.
 * Deviates: Philox4x64-10, key (seed, 1), counter (ion index, step, 3, 0), uniforms
 * ((w >> 12) + 1/2) 2^-52, Box-Muller (z_x, z_y from words 0, 1; z_z from 2, 3).
 * Enqueued on stream; no handle.  Errors: SRBE_EINVAL (arguments), SRBE_EHIP.
 */
int srbe_langevin_update(int64_t n, double* xyz, double* vel, const double* F, const double* mass, double gamma,
                         double beta, double dt, double Lx, double Ly, double zlo, double zhi, uint64_t seed,
                         uint64_t step, void* stream);

/*
 * Dynamics.  The paper's coarse-grained force field is not given; srbe_ff is a stand-in
 * that keeps ions apart, between the walls and in their molecules so that SRBE-driven
 * Langevin dynamics (Sec. 3) can run (charging curves):
 *   - WCA between sites of different molecules: 4 eps [(s/r)^12 - (s/r)^6] + eps for
 *     r < 2^(1/6) s (which must not exceed rc);
 *   - 9-3 walls at z = wall_zlo (acting upward) and z = wall_zhi (downward):
 *     eps_w [(2/15)(s_w/d)^9 - (s_w/d)^3], cut and shifted at its minimum d = (2/5)^(1/6) s_w;
 *   - harmonic bonds (bond_k / 2)(r - r0)^2 between listed sites.
 */
typedef struct srbe_ff {
  double wca_eps, wca_sigma;   /* energy, length                          */
  double wall_eps, wall_sigma; /* energy, length                          */
  double wall_zlo, wall_zhi;   /* wall planes                             */
  double bond_k;               /* energy / length^2                       */
} srbe_ff;

/*
 * srbe_ff_forces -- adds the force field's forces to F (device 3N SoA, e.g. F_out of the
 * step) for the ions of the last srbe_step on this handle (eager, same n_rep; its inputs
 * still valid and unchanged), over that step's cell lists.  mol: device N int32, molecule
 * of each ion (no WCA within a molecule); bond: device 2N int32, up to two bonded partner
 * ions per ion (global ion index, -1 for none; list each bond at both ends); bond_r0:
 * device 2N doubles, their rest lengths.  e_ion: device N doubles or NULL, each ion's
 * energy (half of its pair and bond terms, all of its wall terms).  FP64, deterministic.
 * Errors: SRBE_EINVAL (no preceding step, other n_rep, NULL arrays, WCA range above rc).
 */
int srbe_ff_forces(srbe_system* h, int32_t n_rep, const srbe_ff* ff, const int32_t* mol, const int32_t* bond,
                   const double* bond_r0, double* F, double* e_ion, void* stream);

/*
 * srbe_md_graph_create -- one step of SRBE-driven Langevin dynamics captured as a graph
 * (replayed with srbe_graph_launch, its step counter reset by srbe_graph_set_step,
 * destroyed with srbe_graph_destroy): the SRBE step of srbe_graph_create (sampling with
 * the counter's step, b*, the charge solve, the forces of Eq. (25) and real space) into
 * Q_out, F_out, psibar_out, energy_out; then F_out += the force field's forces
 * (srbe_ff_forces); then the Euler-Maruyama update of srbe_langevin_update of ion_xyz and
 * vel in place with the counter's step (noise key md->noise_seed; md->symplectic = 1 moves
 * the positions with the updated velocity, r + v_new dt, the symplectic ordering of the
 * same update: the printed r + v dt gains energy on stiff contacts, 0 keeps it).  Each replay advances
 * the dynamics by dt; F_out and Q_out hold the forces and charges at the positions before
 * the update.  Arguments as for srbe_graph_create, srbe_ff_forces and srbe_langevin_update
 * (mass: device N doubles).  Errors: as those calls.
 */
typedef struct srbe_md {
  srbe_ff ff;
  double gamma, beta, dt; /* Langevin friction, inverse temperature, time step        */
  double zlo, zhi;        /* reflecting bounds of z (a safety net behind the walls)   */
  uint64_t noise_seed;
  int32_t symplectic;     /* 1: r <- r + v_new dt; 0: r <- r + v dt (as printed)     */
  int32_t reserved;       /* must be 0                                                */
} srbe_md;
int srbe_md_graph_create(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                         double* ion_xyz, double* vel, const double* ion_q, const double* mass, const int32_t* mol,
                         const int32_t* bond, const double* bond_r0, const double* dpsi, const uint64_t* seed,
                         uint64_t first_step, const srbe_md* md, double* Q_out, double* F_out, double* psibar_out,
                         double* energy_out, srbe_graph** out);

/*
 * srbe_sample -- only the sampler of a step (Sec. 3, Eqs. (26)-(29)): writes the
 * n_rep*P*3 int32 modes the step with the same (seed, step) would use.
 * seed device n_rep uint64; kset_out device; n_accepted_out device n_rep int32 or NULL:
 * the Metropolis chain's accepted proposals.  Returns SRBE_EINVAL on bad arguments.
 * The chain: the proposal of Eq. (28) per axis, acceptance by Eq. (29), a fresh chain
 * per (seed, step) started at the first valid proposal of a 64-try start sequence.
 * With SRBE_FLAG_IID_SAMPLER the P modes are instead independent draws from the same
 * target by rejection sampling: attempt a (counter (a, step, 3, 0) for its proposal,
 * (a, step, 4, 0) for its uniform) is accepted when its mode lies outside I and the
 * origin and log U < log r(m) - log r(0), r the ratio of Eq. (29); the sample is the
 * accepted proposals in attempt order (n_accepted_out: the attempts used).  After
 * 65536 attempts the rest of the sample is (1, 0, 0) and the step flags SRBE_ENUMERIC
 * (only when most of the proposal's mass lies on I or the origin).
 */
int srbe_sample(srbe_system* h, int32_t n_rep, const uint64_t* seed, uint64_t step, int32_t* kset_out,
                int32_t* n_accepted_out, void* stream);

/*
 * srbe_sync_status -- wait for the handle's work and report device-side faults:
 * SRBE_ENONNEUTRAL, SRBE_ERANGE, SRBE_ENUMERIC, SRBE_EHIP, or SRBE_OK.  Clears the
 * status word.
 */
int srbe_sync_status(srbe_system* h);

/*
 * Per-phase timing (tracing).  When enabled, every later srbe_step records a HIP
 * event before and after each of its phases on the stream that runs it (the two
 * real-space force phases run on an internal stream beside the others, so they
 * overlap them).  Phases that a normal step runs together in one launch (the sampler beside
 * the cell sort; each structure-factor pass beside a real-space pass) are then
 * launched one after the other, with the same device code and results, so that each
 * can be timed.  srbe_profile_read waits for the events and returns, per phase, the
 * summed duration in milliseconds and the number of launches since the last read
 * (then resets).  Phases, in order: sample, cellsort (particle records and their
 * sort by cell), sf_ions, real_ele, real_ii, ele_potential, cp_gemm, post_charges,
 * sf_ele, real_ie, ion_force (the k-space and slab force), energy (the energy and the
 * real-space sums added to the forces), sf_ions_finalize and sf_ele_finalize (the
 * launches that add the structure-factor partial sums; sf_ions and sf_ele time the
 * partial-sum launches alone); the remaining slots are unused ("").
 * srbe_phase_name(i) returns the name of phase i.  Captured steps (srbe_graph_*)
 * record no phase events.  srbe_profile_enable(h, n) with n > 1 launches every phase
 * but energy (whose launch adds to F) n times in a row between its two events (the
 * phases are idempotent: the step's results are unchanged), so that the events' own
 * cost is spread over n launches; the counts read back are launches, so total ms /
 * launches is the time of one launch.  n = 1 times single launches; n = 0 disables.
 */
#define SRBE_N_PHASES 16
int srbe_profile_enable(srbe_system* h, int32_t enable);
int srbe_profile_read(srbe_system* h, double* ms_out /*host [SRBE_N_PHASES]*/,
                      int64_t* launches_out /*host [SRBE_N_PHASES]*/);
const char* srbe_phase_name(int32_t phase);

/*
 * Launch-parameter tuning (the step's tile shapes; not a computation of the paper).
 * Parameters, by index:
 *   SRBE_TUNE_SF_BLOCKS   structure-factor passes (Eq. (15), ions and electrodes):
 *                         target number of partial-sum blocks of 256 modes, which
 *                         sets the particles each block sums (1 .. 2^20)
 *   SRBE_TUNE_WAVES       electrode-potential (Eq. (24)) and ion k-space force
 *                         (Eq. (25)) passes: waves per 64-particle block, each wave
 *                         taking an equal share of the modes (2, 4 or 8)
 *   SRBE_TUNE_UNROLL      the unroll depth of their FP32 mode loops (2, 4 or 8)
 *   SRBE_TUNE_II_IONS     ion-ion real-space pass (Eq. (13)): consecutive cell-sorted
 *                         ions per wave (1 .. 1024)
 *   SRBE_TUNE_IE_BLOCKS   ion-electrode real-space pass: blocks per replica (1 .. 65536)
 *   SRBE_TUNE_ELE_SPLIT   electrode-potential real-space pass: waves per chunk of 64
 *                         electrodes (1, 2 or 4)
 *   SRBE_TUNE_GEMM_SPLIT  charge-solve GEMM (Eqs. (9)-(11)): ranges the contraction is
 *                         split into, each a block per output tile (1 .. 16)
 *   SRBE_TUNE_GEMM_DEPTH  its contraction block, in units of 16 indices (1 or 2): the
 *                         loads of one block are in flight while the previous one
 *                         is multiplied
 * A step (srbe_step, srbe_graph_create) uses the parameters stored in the handle
 * for its shape -- precision, n_rep and the largest replica's ion count -- else
 * defaults derived from the device's compute-unit count.  Results depend on the
 * parameters only through the order of floating-point sums (each setting is
 * bitwise repeatable).
 *
 * srbe_tune -- times captured steps (graph replays, `iters` timed after a warm-up,
 * iters >= 1) of the given inputs on `stream`, varying one parameter at a time over
 * its candidates starting from the defaults (coordinate descent, one pass), keeps
 * the fastest, stores it for the shape and writes it to params_out (host int32
 * [SRBE_TUNE_NPARAM], may be NULL).  ms_out (host double[2], may be NULL) receives
 * the ms per step of the defaults and of the stored parameters.  Inputs as for
 * srbe_step (sampled modes; seed required when P > 0); the outputs go to buffers the
 * call allocates and frees.  Blocks until done.  Errors: SRBE_EINVAL (arguments),
 * SRBE_ENOMEM, SRBE_EHIP, or a device fault of a timed step (then nothing is stored).
 * Live timing is currently switched off: processes that ran it (tens of graph
 * create / replay / destroy cycles) have aborted with host heap corruption whose
 * cause is not yet found.  The call checks its arguments and then returns
 * SRBE_EINVAL (srbe_last_error says so) without device work; choose parameters with
 * srbe_set_tuning, e.g. from a table of earlier timings.
 *
 * srbe_get_tuning -- the parameters a step of this shape would use (host int32
 * [SRBE_TUNE_NPARAM]).  ion_offsets: host, n_rep + 1.
 * srbe_set_tuning -- stores the given parameters (host int32 [SRBE_TUNE_NPARAM]) for
 * the shape, or with params NULL drops the stored entry (back to the defaults).
 * SRBE_EINVAL, with srbe_last_error naming the parameter, for a value outside its
 * range.  Graphs already created keep the parameters they were captured with.
 */
#define SRBE_TUNE_SF_BLOCKS 0
#define SRBE_TUNE_WAVES 1
#define SRBE_TUNE_UNROLL 2
#define SRBE_TUNE_II_IONS 3
#define SRBE_TUNE_IE_BLOCKS 4
#define SRBE_TUNE_ELE_SPLIT 5
#define SRBE_TUNE_GEMM_SPLIT 6
#define SRBE_TUNE_GEMM_DEPTH 7
#define SRBE_TUNE_NPARAM 8
int srbe_tune(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets, const double* ion_xyz,
              const double* ion_q, const double* dpsi, const uint64_t* seed, int32_t iters, int32_t* params_out,
              double* ms_out, void* stream);
int srbe_get_tuning(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                    int32_t* params_out);
int srbe_set_tuning(srbe_system* h, int32_t precision, int32_t n_rep, const int64_t* ion_offsets,
                    const int32_t* params);

/* srbe_normaliser -- G of Eq. (27) for the handle's parameters (host double). */
double srbe_normaliser(const srbe_system* h);

/* srbe_n_ele -- number of electrode atoms of the handle. */
int32_t srbe_n_ele(const srbe_system* h);

#ifdef __cplusplus
}
#endif

#endif /* SRBE_H */
