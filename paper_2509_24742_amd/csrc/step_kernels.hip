// Per-step kernels of the SRBE constant-potential step (gfx950).
//
// One step (Algorithm 1 of the paper, integration excluded) for R replicas sharing
// one electrode geometry:
//   [sample | records + cell sort] -> [sf(ions) | real_ele] -> sf finalize
//   -> ele_potential -> [FP64 GEMM: (Q; psibar) = S_ext (dpsi d + b*)] -> post_charges
//   -> [sf(electrodes) | real_ie] -> sf finalize -> ion_force -> energy,
// with the ion-ion real-space pass beside the chain from the cell sort to the force
// pass ([a | b]: one launch whose blocks run both parts).  Structure-factor partial
// sums are added in chunk order by a finalize pass; real-space neighbours are
// visited in a fixed (cell, index) order.  There are no floating-point atomics, so
// two runs on the same inputs give bitwise-identical results.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "kernels.h"

namespace srbe {

static inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

#define TWO_PI 6.283185307179586
#define INV_SQRT_PI 0.5641895835477563

// Sum over the 64 lanes of a wave by an xor butterfly: every lane ends with the same
// value, added in the same order on every run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Deterministic sum over a block of NT threads of NV doubles; result valid in thread 0.
template <int NT, int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[NT / 64]) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int a = 0; a < NV; ++a) {
    const double s = wave_sum(v[a]);
    if (lane == 0) sh[a][wv] = s;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      double s = 0.0;
      for (int u = 0; u < NT / 64; ++u) s += sh[a][u];
      v[a] = s;
    }
  }
  __syncthreads();
}

// ============================================================ particle records
// One block of 1024 threads per replica (the set-up binning of the electrodes uses
// the same code).  Per particle, in input order: the fractional coordinates
// s = (x/Lx, y/Ly, z/Lz), x and y wrapped into [0, 1), as 32-bit fixed point with
// the FP32 charge (REC bit 0) and/or in FP64 with the FP64 charge (REC bit 1); the
// range check (z in [0, H], finite coordinates and charge); the cell sort key
// (cell << 13 | index within the replica); and the replica's charge sums.  Then the
// sort by cell: cell counts (LDS integer atomics), their exclusive scan (the cell
// starts), a provisional slot per particle from a per-cell cursor, and, since the
// provisional order inside a cell depends on timing, each particle's final position
// inside its cell is the number of the cell's keys below its own.  So every cell
// lists its particles in index order, independent of timing.  Finally the records
// in cell order.
struct SortArgs {
  const int64_t* off;
  const double* xyz;  // SoA 3N
  const double* q;    // N charges (ions; may be null when a replica batch has no ions); unused for electrodes
  int64_t N;
  unsigned* keys;
  uint4* fx;
  double4* d4;
  double* scal;       // R*4 charge sums (q only)
  int* perm;
  int* scell;
  int* cstart;
  uint4* sfx;
  double4* sd4;
  unsigned* status;
};

// Records of particle i in input order, its range check and its charge sums
// (v: sum q, sum |q|, sum q z, sum q^2); returns its cell.
template <int REC>
__device__ __forceinline__ int particle_record(const Geom& g, const SortArgs& a, int64_t i, double (&v)[4]) {
  constexpr bool kIons = REC != 3;
  const int64_t N = a.N;
  const double x = a.xyz[i], y = a.xyz[N + i], z = a.xyz[2 * N + i];
  const double qi = kIons ? a.q[i] : 0.0;
  if (!isfinite(qi) || !isfinite(x) || !isfinite(y) || !(z >= 0.0 && z <= g.H)) atomicOr(a.status, ST_RANGE);
  const double sx = wrap_frac(x, g.invLx), sy = wrap_frac(y, g.invLy), sz = wrap_frac(z, g.invLz);
  if (REC & 1) a.fx[i] = make_uint4(to_fixed(sx), to_fixed(sy), to_fixed(sz), __float_as_uint((float)qi));
  if (REC & 2) a.d4[i] = make_double4(sx, sy, sz, qi);
  v[0] += qi;
  v[1] += fabs(qi);
  v[2] += qi * z;
  v[3] += qi * qi;
  return cell_index(g, sx, sy, z);
}

template <int REC>
__device__ __forceinline__ void sort_block(const Geom& g, int r, const SortArgs& a) {
  // REC 1 or 2: ions (charges given, the replica's sums written, also for a replica
  // without ions, whose charge pointer may be null); REC 3: the electrodes
  constexpr bool kIons = REC != 3;
  __shared__ unsigned prov[kMaxBinParticles];
  __shared__ int cnt[kMaxCells + 1];
  __shared__ int scan[2][kMaxCells + 1];
  __shared__ double red[4][16];
  const int t = threadIdx.x;
  const int64_t b0 = a.off[r];
  const int n = (int)(a.off[r + 1] - b0);
  for (int c = t; c <= g.ncell; c += 1024) cnt[c] = 0;
  __syncthreads();
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = t; k < n; k += 1024) {
    const int64_t i = b0 + k;
    const unsigned key = ((unsigned)particle_record<REC>(g, a, i, v) << 13) | (unsigned)k;
    a.keys[i] = key;
    atomicAdd(&cnt[key >> 13], 1);
  }
  if (kIons) {
    block_sum<1024, 4>(v, red);
    if (t == 0) {
      a.scal[4 * r + 0] = v[0];
      a.scal[4 * r + 1] = v[1];
      a.scal[4 * r + 2] = v[2];
      a.scal[4 * r + 3] = v[3];
      if (fabs(v[0]) > 1e-10 * v[1]) atomicOr(a.status, ST_NONNEUTRAL);
    }
  } else {
    __syncthreads();
  }
  // exclusive scan of the cell counts (Hillis-Steele over ncell + 1 entries)
  for (int c = t; c <= g.ncell; c += 1024) scan[0][c] = c == 0 ? 0 : cnt[c - 1];
  __syncthreads();
  int src = 0;
  for (int o = 1; o <= g.ncell; o <<= 1) {
    for (int c = t; c <= g.ncell; c += 1024) scan[src ^ 1][c] = scan[src][c] + (c >= o ? scan[src][c - o] : 0);
    __syncthreads();
    src ^= 1;
  }
  const int* start = scan[src];
  int* cs = a.cstart + (size_t)r * (g.ncell + 1);
  for (int c = t; c <= g.ncell; c += 1024) {
    cs[c] = start[c];
    cnt[c] = start[c];  // per-cell cursor
  }
  __syncthreads();
  // provisional slots (timing-dependent order inside a cell); each thread reads back
  // the keys it wrote itself
  for (int k = t; k < n; k += 1024) {
    const unsigned key = a.keys[b0 + k];
    prov[atomicAdd(&cnt[key >> 13], 1)] = key;
  }
  __syncthreads();
  // final position inside the cell: the number of the cell's keys below this one.
  // The records read here were written by other threads of this block before the
  // barriers above.
  for (int sidx = t; sidx < n; sidx += 1024) {
    const unsigned key = prov[sidx];
    const int c = (int)(key >> 13);
    const int lo = start[c], hi = start[c + 1];
    int rank = 0;
    for (int u = lo; u < hi; ++u) rank += prov[u] < key;
    const int pos = lo + rank;
    const int64_t i = b0 + (int)(key & 0x1FFFu);
    a.perm[b0 + pos] = (int)i;
    a.scell[b0 + pos] = c;
    if (REC & 1) a.sfx[b0 + pos] = a.fx[i];
    if (REC & 2) a.sd4[b0 + pos] = a.d4[i];
  }
}

// Multi-block cell sort, for replicas of more than kMaxBinParticles particles or grids
// of more than kMaxCells cells.  It gives sort_block's order (cells in index order,
// each cell's particles in index order) from five launches over tiles of 256
// particles (and three over chunks of 1024 cells): the cell counts are cleared;
// each particle's records and cell, the counts by integer atomics in device memory
// and each tile's charge sums; the exclusive scan of the counts (the cell starts; the
// counts become per-cell cursors) with the tile sums added in tile order; a
// provisional slot per particle from its cell's cursor (the order inside a cell
// depends on timing); and the final position inside the cell, the number of the
// cell's entries with a smaller index, with the records in cell order.  The time of
// the last pass grows with the square of the largest cell's count.
__global__ __launch_bounds__(256) void k_zero_int(int* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0;
}

// Each big-sort launch's body takes its block index lb (a multi-system launch passes the
// block's index within its system).
template <int REC>
__device__ __forceinline__ void bigsort_count_body(const Geom& g, const SortArgs& a, const BigSort& bs, int lb) {
  __shared__ double red[4][4];
  const int r = lb / bs.ntile, tile = lb - r * bs.ntile;
  const int64_t b0 = a.off[r];
  const int n = (int)(a.off[r + 1] - b0);
  const int k = tile * 256 + (int)threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  if (k < n) {
    const int c = particle_record<REC>(g, a, b0 + k, v);
    a.keys[b0 + k] = (unsigned)c;
    atomicAdd(&bs.count[(size_t)r * (g.ncell + 1) + c], 1);
  }
  if constexpr (REC != 3) {
    block_sum<256, 4>(v, red);
    if (threadIdx.x == 0)
      for (int u = 0; u < 4; ++u) bs.tsum[((size_t)r * bs.ntile + tile) * 4 + u] = v[u];
  }
}

template <int REC>
__global__ __launch_bounds__(256) void k_bigsort_count(Geom g, SortArgs a, BigSort bs) {
  bigsort_count_body<REC>(g, a, bs, blockIdx.x);
}

// Exclusive scan of the cell counts in three launches, so that the counts (just
// written by device-scope atomics) are read by many CUs at once rather than by one:
// each block of 1024 cells scans its chunk and records the chunk's total; per
// replica one block adds the tile charge sums in tile order and scans the chunk
// totals into chunk offsets; then each cell start gets its chunk's offset and the
// counts become per-cell cursors.
__device__ __forceinline__ int block_exclusive_scan_1024(int x, int& total, int* wtot) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wtot[wv] = incl;
  __syncthreads();
  int below = 0;
  total = 0;
  for (int u = 0; u < 16; ++u) {
    below += u < wv ? wtot[u] : 0;
    total += wtot[u];
  }
  return below + incl - x;
}

__device__ __forceinline__ void bigsort_scan_chunks_body(const Geom& g, const SortArgs& a, const BigSort& bs, int lb) {
  __shared__ int wtot[16];
  const int r = lb / bs.nchunk, ch = lb - r * bs.nchunk;
  const int c = ch * 1024 + (int)threadIdx.x;
  const int* cnt = bs.count + (size_t)r * (g.ncell + 1);
  int total;
  const int excl = block_exclusive_scan_1024(c < g.ncell ? cnt[c] : 0, total, wtot);
  if (c <= g.ncell) a.cstart[(size_t)r * (g.ncell + 1) + c] = excl;
  if (threadIdx.x == 0) bs.ctot[(size_t)r * bs.nchunk + ch] = total;
}

__global__ __launch_bounds__(1024) void k_bigsort_scan_chunks(Geom g, SortArgs a, BigSort bs) {
  bigsort_scan_chunks_body(g, a, bs, blockIdx.x);
}

template <int REC>
__device__ __forceinline__ void bigsort_scan_totals_body(const Geom& g, const SortArgs& a, const BigSort& bs, int lb) {
  __shared__ double red[4][16];
  __shared__ int wtot[16];
  const int r = lb, t = threadIdx.x;
  if constexpr (REC != 3) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int u = t; u < bs.ntile; u += 1024)
      for (int q = 0; q < 4; ++q) v[q] += bs.tsum[((size_t)r * bs.ntile + u) * 4 + q];
    block_sum<1024, 4>(v, red);
    if (t == 0) {
      for (int q = 0; q < 4; ++q) a.scal[4 * r + q] = v[q];
      if (fabs(v[0]) > 1e-10 * v[1]) atomicOr(a.status, ST_NONNEUTRAL);
    }
  }
  int* ct = bs.ctot + (size_t)r * bs.nchunk;  // nchunk <= 1024: one round
  int total;
  const int excl = block_exclusive_scan_1024(t < bs.nchunk ? ct[t] : 0, total, wtot);
  if (t < bs.nchunk) ct[t] = excl;
}

template <int REC>
__global__ __launch_bounds__(1024) void k_bigsort_scan_totals(Geom g, SortArgs a, BigSort bs) {
  bigsort_scan_totals_body<REC>(g, a, bs, blockIdx.x);
}

__device__ __forceinline__ void bigsort_scan_offsets_body(const Geom& g, const SortArgs& a, const BigSort& bs, int lb) {
  const int r = lb / bs.nchunk, ch = lb - r * bs.nchunk;
  const int c = ch * 1024 + (int)threadIdx.x;
  if (c > g.ncell) return;
  const size_t at = (size_t)r * (g.ncell + 1) + c;
  const int start = a.cstart[at] + bs.ctot[(size_t)r * bs.nchunk + ch];
  a.cstart[at] = start;
  bs.count[at] = start;  // cursor
}

__global__ __launch_bounds__(1024) void k_bigsort_scan_offsets(Geom g, SortArgs a, BigSort bs) {
  bigsort_scan_offsets_body(g, a, bs, blockIdx.x);
}

template <int REC>
__device__ __forceinline__ void bigsort_scatter_body(const Geom& g, const SortArgs& a, const BigSort& bs, int lb) {
  const int r = lb / bs.ntile, tile = lb - r * bs.ntile;
  const int64_t b0 = a.off[r];
  const int n = (int)(a.off[r + 1] - b0);
  const int k = tile * 256 + (int)threadIdx.x;
  if (k >= n) return;
  const int c = (int)a.keys[b0 + k];
  bs.prov[b0 + atomicAdd(&bs.count[(size_t)r * (g.ncell + 1) + c], 1)] = k;
}

template <int REC>
__global__ __launch_bounds__(256) void k_bigsort_scatter(Geom g, SortArgs a, BigSort bs) {
  bigsort_scatter_body<REC>(g, a, bs, blockIdx.x);
}

template <int REC>
__device__ __forceinline__ void bigsort_rank_body(const Geom& g, const SortArgs& a, const BigSort& bs, int lb) {
  const int r = lb / bs.ntile, tile = lb - r * bs.ntile;
  const int64_t b0 = a.off[r];
  const int n = (int)(a.off[r + 1] - b0);
  const int p = tile * 256 + (int)threadIdx.x;
  if (p >= n) return;
  const int* __restrict__ prov = bs.prov + b0;
  const int k = prov[p];
  const int c = (int)a.keys[b0 + k];
  const int* cs = a.cstart + (size_t)r * (g.ncell + 1);
  const int lo = cs[c], hi = cs[c + 1];
  int rank = 0;
  for (int u = lo; u < hi; ++u) rank += prov[u] < k;
  const int pos = lo + rank;
  const int64_t i = b0 + k;
  a.perm[b0 + pos] = (int)i;
  a.scell[b0 + pos] = c;
  if (REC & 1) a.sfx[b0 + pos] = a.fx[i];
  if (REC & 2) a.sd4[b0 + pos] = a.d4[i];
}

template <int REC>
__global__ __launch_bounds__(256) void k_bigsort_rank(Geom g, SortArgs a, BigSort bs) {
  bigsort_rank_body<REC>(g, a, bs, blockIdx.x);
}

template <int REC>
static void launch_big_sort(const Geom& g, const SortArgs& sa, const BigSort& bs, int R, hipStream_t s) {
  const int64_t ncount = (int64_t)R * (g.ncell + 1);
  hipLaunchKernelGGL(k_zero_int, dim3(std::min(4096, cdiv64(ncount, 256))), dim3(256), 0, s, bs.count, ncount);
  const dim3 tiles((unsigned)R * bs.ntile);
  hipLaunchKernelGGL(k_bigsort_count<REC>, tiles, dim3(256), 0, s, g, sa, bs);
  const dim3 chunks((unsigned)R * bs.nchunk);
  hipLaunchKernelGGL(k_bigsort_scan_chunks, chunks, dim3(1024), 0, s, g, sa, bs);
  hipLaunchKernelGGL(k_bigsort_scan_totals<REC>, dim3(R), dim3(1024), 0, s, g, sa, bs);
  hipLaunchKernelGGL(k_bigsort_scan_offsets, chunks, dim3(1024), 0, s, g, sa, bs);
  hipLaunchKernelGGL(k_bigsort_scatter<REC>, tiles, dim3(256), 0, s, g, sa, bs);
  hipLaunchKernelGGL(k_bigsort_rank<REC>, tiles, dim3(256), 0, s, g, sa, bs);
}

bool use_big_sort(const Geom& g, int64_t max_particles) {
  return max_particles > kMaxBinParticles || g.ncell > kMaxCells;
}

// ============================================================ sampler
// Metropolis sampler of Sec. 3 (Eqs. (26)-(29)).  Proposal per axis
// u = sigma_d z, sigma_d = alpha L_d / (sqrt(2) pi) (the variance of the density in
// Eq. (28)), m = floor(u + 1/2); target exp(-k^2/(4 alpha^2)) on L_k \ I; acceptance
// min{1, r(y)/r(x)} with r(m) = exp(-k^2/(4 alpha^2)) / prod_d q_d(m_d), decided as
// d >= 0 or log U < d, d = log r(y) - log r(x).  Chain: initial state = first
// valid proposal of a start sequence (64 tries, else (1,0,0)); then P iterations,
// each contributing its current state.  Random numbers: Philox4x64-10, key
// (seed, 0), counter (index, step, purpose, 0), purpose 0 = proposal, 1 =
// acceptance, 2 = start; uniforms ((w >> 12) + 1/2) 2^-52; Box-Muller
// z_x = sqrt(-2 ln U0) cos(2 pi U1), z_y = sqrt(-2 ln U0) sin(2 pi U1),
// z_z = sqrt(-2 ln U2) cos(2 pi U3).
#pragma clang fp contract(off)
__device__ double q_axis(int m, double alpha, double L) {
  const double a = fabs((double)m);
  const double c = M_PI / (alpha * L);
  return 0.5 * (erfc(c * (a - 0.5)) - erfc(c * (a + 0.5)));
}

__device__ void proposal(const Geom& g, uint64_t seed, uint64_t step, uint64_t purpose, uint64_t idx, int& mx,
                         int& my, int& mz) {
  U64x4 c;
  c.v[0] = idx;
  c.v[1] = step;
  c.v[2] = purpose;
  c.v[3] = 0;
  const U64x4 w = philox4x64_10(c, seed, 0);
  const double U0 = u01_open(w.v[0]), U1 = u01_open(w.v[1]), U2 = u01_open(w.v[2]), U3 = u01_open(w.v[3]);
  const double r0 = sqrt(-2.0 * log(U0));
  const double r2 = sqrt(-2.0 * log(U2));
  const double zx = r0 * cos(TWO_PI * U1);
  const double zy = r0 * sin(TWO_PI * U1);
  const double zz = r2 * cos(TWO_PI * U3);
  mx = (int)floor(g.sig[0] * zx + 0.5);
  my = (int)floor(g.sig[1] * zy + 0.5);
  mz = (int)floor(g.sig[2] * zz + 0.5);
}

// log q_d(m) for |m| <= qmax[d] from the table built at set-up by k_logq_table
// with the same expression (so the value is the same bits), else computed here.
__device__ double log_ratio_tab(const Geom& g, const double* __restrict__ T, int mx, int my, int mz) {
  const double kx = TWO_PI * (double)mx / g.Lx;
  const double ky = TWO_PI * (double)my / g.Ly;
  const double kz = TWO_PI * (double)mz / g.Lz;
  const double k2 = kx * kx + ky * ky + kz * kz;
  const int ax = abs(mx), ay = abs(my), az = abs(mz);
  const double l0 = ax <= g.qmax[0] ? T[ax] : log(q_axis(mx, g.alpha, g.Lx));
  const double l1 = ay <= g.qmax[1] ? T[g.qmax[0] + 1 + ay] : log(q_axis(my, g.alpha, g.Ly));
  const double l2 = az <= g.qmax[2] ? T[g.qmax[0] + g.qmax[1] + 2 + az] : log(q_axis(mz, g.alpha, g.Lz));
  const double lq = l0 + l1 + l2;
  return -k2 / (4.0 * (g.alpha * g.alpha)) - lq;
}

__global__ __launch_bounds__(256) void k_logq_table(Geom g, double* __restrict__ T) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n0 = g.qmax[0] + 1, n1 = g.qmax[1] + 1, n2 = g.qmax[2] + 1;
  if (i >= n0 + n1 + n2) return;
  if (i < n0)
    T[i] = log(q_axis(i, g.alpha, g.Lx));
  else if (i < n0 + n1)
    T[i] = log(q_axis(i - n0, g.alpha, g.Ly));
  else
    T[i] = log(q_axis(i - n0 - n1, g.alpha, g.Lz));
}

__device__ __forceinline__ bool valid_mode(const Geom& g, int mx, int my, int mz) {
  return !(mx == 0 && my == 0 && abs(mz) <= g.M);
}

__device__ double sampled_weight(const Geom& g, int mx, int my, int mz) {
  const double kx = TWO_PI * (double)mx / g.Lx;
  const double ky = TWO_PI * (double)my / g.Ly;
  const double kz = TWO_PI * (double)mz / g.Lz;
  const double k2 = kx * kx + ky * ky + kz * kz;
  return g.ke * (g.G / (double)g.P) * 4.0 * M_PI / (g.V * k2);
}
#pragma clang fp contract(fast)

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// The i.i.d. option: rejection sampling with the same proposal and target.  Attempt a
// draws its proposal from counter (a, step, 3, 0) as above and its uniform from word 0
// of counter (a, step, 4, 0); it is accepted when the proposal lies in L_k \ I and
// log U < log r(y) - log r(0), r the ratio of Eq. (29) (exp(-m^2/(2 sigma^2)) / q_d(m)
// is largest at m = 0 on every axis, so r(0) bounds r).  The accepted proposals in
// attempt order are the sample.  The block makes NT attempts per round, each thread
// one, and places the accepted ones by a block-wide count; after kIidMaxRounds rounds
// the rest of the sample is (1, 0, 0) and the status word flags a numeric error.
constexpr int kIidMaxRounds = 64;

#pragma clang fp contract(off)
template <int NT>
__device__ void sample_iid(const Geom& g, int r, const StepBufs& b, uint64_t seed, uint64_t step) {
  __shared__ int wcount[NT / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int P = g.P, M = g.M, K = g.K;
  const double l0 = log_ratio_tab(g, b.logq, 0, 0, 0);
  int filled = 0;  // block-uniform
  for (int round = 0; round < kIidMaxRounds && filled < P; ++round) {
    const uint64_t a = (uint64_t)round * NT + t;
    int mx, my, mz;
    proposal(g, seed, step, 3, a, mx, my, mz);
    U64x4 c;
    c.v[0] = a;
    c.v[1] = step;
    c.v[2] = 4;
    c.v[3] = 0;
    const U64x4 wa = philox4x64_10(c, seed, 0);
    bool ok = valid_mode(g, mx, my, mz);
    if (ok) ok = log(u01_open(wa.v[0])) < log_ratio_tab(g, b.logq, mx, my, mz) - l0;
    const uint64_t m = __ballot(ok);
    if (lane == 0) wcount[w] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int u = 0; u < NT / 64; ++u) {
      before += u < w ? wcount[u] : 0;
      total += wcount[u];
    }
    const int slot = filled + before + __popcll(m & ((1ull << lane) - 1));
    if (ok && slot < P) {
      b.modes[(size_t)r * K + M + slot] = make_int4(mx, my, mz, 0);
      b.w[(size_t)r * K + M + slot] = sampled_weight(g, mx, my, mz);
      if (b.kset_out) {
        int32_t* o = b.kset_out + ((size_t)r * P + slot) * 3;
        o[0] = mx;
        o[1] = my;
        o[2] = mz;
      }
      if (slot == P - 1 && b.nacc_out) b.nacc_out[r] = (int)(a + 1);
    }
    filled += total;
    __syncthreads();  // wcount is rewritten by the next round
  }
  for (int l = filled + t; l < P; l += NT) {
    b.modes[(size_t)r * K + M + l] = make_int4(1, 0, 0, 0);
    b.w[(size_t)r * K + M + l] = sampled_weight(g, 1, 0, 0);
    if (b.kset_out) {
      int32_t* o = b.kset_out + ((size_t)r * P + l) * 3;
      o[0] = 1;
      o[1] = 0;
      o[2] = 0;
    }
  }
  if (t == 0 && filled < P) {
    atomicOr(b.status, ST_NUMERIC);
    if (b.nacc_out) b.nacc_out[r] = kIidMaxRounds * NT;
  }
}
#pragma clang fp contract(fast)

// One block of NT threads per replica: wave 0 draws the 64 start tries while the
// other waves draw the P proposals; then wave 0 runs the chain.
template <int NT>
__device__ __forceinline__ void sample_block(const Geom& g, int r, const StepBufs& b) {
  extern __shared__ unsigned char smem[];
  const uint64_t* __restrict__ seeds = b.seed;
  const int32_t* __restrict__ kset_in = b.kset_in;
  const double* __restrict__ logq = b.logq;
  int4* __restrict__ modes = b.modes;
  double* __restrict__ wout = b.w;
  int32_t* __restrict__ kset_out = b.kset_out;
  int32_t* __restrict__ nacc_out = b.nacc_out;
  unsigned* status = b.status;
  const uint64_t step = b.step_dev ? *b.step_dev : b.step;  // graph replays take the step from device memory
  const int P = g.P, M = g.M, K = g.K;
  const int t = threadIdx.x;
  // deterministic modes (0, 0, m), m = 1..M, weight doubled for the pair +-m
  for (int m = 1 + t; m <= M; m += NT) {
    const double kz = TWO_PI * (double)m / g.Lz;
    const double k2 = kz * kz;
    modes[(size_t)r * K + (m - 1)] = make_int4(0, 0, m, 0);
    wout[(size_t)r * K + (m - 1)] = g.ke * 2.0 * 4.0 * M_PI * exp(-k2 / (4.0 * g.alpha * g.alpha)) / (g.V * k2);
  }
  if (P == 0) {
    if (t == 0 && nacc_out) nacc_out[r] = 0;
    return;
  }
  if (kset_in) {
    for (int l = t; l < P; l += NT) {
      const int32_t* m = kset_in + ((size_t)r * P + l) * 3;
      const int mx = m[0], my = m[1], mz = m[2];
      if (!valid_mode(g, mx, my, mz)) atomicOr(status, ST_BADKSET);
      modes[(size_t)r * K + M + l] = make_int4(mx, my, mz, 0);
      wout[(size_t)r * K + M + l] = valid_mode(g, mx, my, mz) ? sampled_weight(g, mx, my, mz) : 0.0;
      if (kset_out) {
        int32_t* o = kset_out + ((size_t)r * P + l) * 3;
        o[0] = mx;
        o[1] = my;
        o[2] = mz;
      }
    }
    if (t == 0 && nacc_out) nacc_out[r] = -1;
    return;
  }
  const uint64_t seed = seeds[r];
  if (g.iid) {
    sample_iid<NT>(g, r, b, seed, step);
    return;
  }
  // LDS: ly[P], lu[P] (double), state[P] (int), ym[P][3] (int16).  An invalid
  // proposal (target probability zero) has ly = NaN, which fails both accept tests.
  double* ly = reinterpret_cast<double*>(smem);
  double* lu = ly + P;
  int* state = reinterpret_cast<int*>(lu + P);
  short* ym = reinterpret_cast<short*>(state + P);
  __shared__ int first_valid;
  __shared__ int start_m[3];
  if (t == 0) first_valid = 1 << 30;
  __syncthreads();
  int sx = 0, sy = 0, sz = 0;
  if (t < 64) {
    proposal(g, seed, step, 2, (uint64_t)t, sx, sy, sz);
    if (valid_mode(g, sx, sy, sz)) atomicMin(&first_valid, t);
  }
  for (int l = t - 64; l >= 0 && l < P; l += NT - 64) {
    int mx, my, mz;
    proposal(g, seed, step, 0, (uint64_t)l, mx, my, mz);
    U64x4 c;
    c.v[0] = (uint64_t)l;
    c.v[1] = step;
    c.v[2] = 1;
    c.v[3] = 0;
    const U64x4 wa = philox4x64_10(c, seed, 0);
    const bool v = valid_mode(g, mx, my, mz);
    if (abs(mx) > 32767 || abs(my) > 32767 || abs(mz) > 32767) atomicOr(status, ST_NUMERIC);
    ym[3 * l + 0] = (short)mx;
    ym[3 * l + 1] = (short)my;
    ym[3 * l + 2] = (short)mz;
    ly[l] = v ? log_ratio_tab(g, logq, mx, my, mz) : (double)NAN;
    lu[l] = log(u01_open(wa.v[0]));
  }
  __syncthreads();
  if (t < 64 && t == first_valid) {
    start_m[0] = sx;
    start_m[1] = sy;
    start_m[2] = sz;
  }
  if (t == 0 && first_valid == (1 << 30)) {
    start_m[0] = 1;
    start_m[1] = 0;
    start_m[2] = 0;
  }
  __syncthreads();
  // the chain, one wave, 64 decisions at a time.  Lane j first decides as if
  // proposal j-1 was accepted (the state's log ratio then being ly[j-1]); every
  // decision up to the first rejection is then final (each used the state the
  // sequential chain has at that point), the rejected one too, and the remaining
  // lanes decide again from the known state.  Each final decision is the
  // sequential one, d = ly[j] - lx with the same operands.  With acceptance near
  // 1 a chunk takes one or two passes.
  if (t < 64) {
    double lx = log_ratio_tab(g, logq, start_m[0], start_m[1], start_m[2]);
    int cur = -1, nacc = 0;
    for (int base = 0; base < P; base += 64) {
      const int l = base + t;
      const int cnt = min(64, P - base);
      const double myly = l < P ? ly[l] : (double)NAN;
      const double mylu = l < P ? lu[l] : 0.0;
      const double prevly = __shfl_up(myly, 1, 64);
      bool acc = false;
      int done = 0;
      while (done < cnt) {
        const double prev = t == done ? lx : prevly;
        const double d = myly - prev;
        const bool a = d >= 0.0 || mylu < d;
        const uint64_t rej = __ballot(!a && t >= done && t < cnt);
        const int jstar = rej ? __ffsll((unsigned long long)rej) - 1 : cnt;
        if (t >= done && t < jstar) acc = true;
        if (jstar > done) lx = readlane_f64(myly, jstar - 1);
        done = jstar + 1;
      }
      const uint64_t am = __ballot(acc);
      nacc += __popcll(am);
      const uint64_t upto = t == 63 ? ~0ull : ((2ull << t) - 1);
      const uint64_t below = am & upto;
      const int mine = below ? base + 63 - __clzll(below) : cur;
      if (l < P) state[l] = mine;
      if (am) cur = base + 63 - __clzll(am);
    }
    if (t == 0 && nacc_out) nacc_out[r] = nacc;
  }
  __syncthreads();
  for (int l = t; l < P; l += NT) {
    const int s_ = state[l];
    const int mx = s_ < 0 ? start_m[0] : ym[3 * s_ + 0];
    const int my = s_ < 0 ? start_m[1] : ym[3 * s_ + 1];
    const int mz = s_ < 0 ? start_m[2] : ym[3 * s_ + 2];
    modes[(size_t)r * K + M + l] = make_int4(mx, my, mz, 0);
    wout[(size_t)r * K + M + l] = sampled_weight(g, mx, my, mz);
    if (kset_out) {
      int32_t* o = kset_out + ((size_t)r * P + l) * 3;
      o[0] = mx;
      o[1] = my;
      o[2] = mz;
    }
  }
}

size_t sample_lds_bytes(int P) { return (size_t)P * (8 + 8 + 4 + 6) + 16; }

// The step's first launch: blocks [0, nsamp) sample the replicas' modes, blocks
// [nsamp, nsamp + nsort) make and sort the replicas' particle records (the two are
// independent; one launch runs them side by side).
template <int REC>
__device__ __forceinline__ void front_body(const Geom& g, const StepBufs& b, const SortArgs& sa, int nsamp, int lb) {
  if (lb < nsamp)
    sample_block<1024>(g, lb, b);
  else
    sort_block<REC>(g, lb - nsamp, sa);
}

template <int REC>
__global__ __launch_bounds__(1024) void k_front(Geom g, StepBufs b, SortArgs sa, int nsamp) {
  front_body<REC>(g, b, sa, nsamp, blockIdx.x);
}

__host__ __device__ inline SortArgs ion_sort_args(const StepBufs& b) {
  return SortArgs{b.off,  b.ion_xyz, b.ion_q, b.N,    b.keys,  b.ion_fx, b.ion_d4,
                  b.scal, b.perm,    b.scell, b.cstart, b.sfx, b.sd4,    b.status};
}

void launch_front(const Geom& g, const StepBufs& b, int fp32, int parts, hipStream_t s) {
  const int nsamp = (parts & FRONT_SAMPLE) ? b.R : 0;
  const bool sort = (parts & FRONT_SORT) != 0, big = sort && b.bigsort.count != nullptr;
  const int nsort = sort && !big ? b.R : 0;
  const SortArgs sa = ion_sort_args(b);
  if (nsamp + nsort > 0) {
    const size_t lds = nsamp ? sample_lds_bytes(g.P) : 0;
    if (fp32)
      hipLaunchKernelGGL(k_front<1>, dim3(nsamp + nsort), dim3(1024), lds, s, g, b, sa, nsamp);
    else
      hipLaunchKernelGGL(k_front<2>, dim3(nsamp + nsort), dim3(1024), lds, s, g, b, sa, nsamp);
  }
  if (big) {
    if (fp32)
      launch_big_sort<1>(g, sa, b.bigsort, b.R, s);
    else
      launch_big_sort<2>(g, sa, b.bigsort, b.R, s);
  }
}

// Electrodes are binned once per handle with the same code (both record formats).
// off2: device {0, n_ele}; keys: n_ele scratch words; status: device word.
void launch_bin_electrodes(const Geom& g, const int64_t* off2, const double* ele_xyz, int n_ele, unsigned* keys,
                           uint4* fx, double4* d4, int* perm, int* scell, int* cstart, uint4* sfx, double4* sd4,
                           unsigned* status, const BigSort& bs, hipStream_t s) {
  const SortArgs sa{off2, ele_xyz, nullptr, (int64_t)n_ele, keys, fx, d4, nullptr, perm, scell, cstart, sfx, sd4,
                    status};
  if (bs.count) {
    launch_big_sort<3>(g, sa, bs, 1, s);
    return;
  }
  StepBufs none{};
  hipLaunchKernelGGL(k_front<3>, dim3(1), dim3(1024), 0, s, g, none, sa, 0);
}

void launch_logq_table(const Geom& g, double* T, hipStream_t s) {
  const int n = g.qmax[0] + g.qmax[1] + g.qmax[2] + 3;
  hipLaunchKernelGGL(k_logq_table, dim3(cdiv64(n, 256)), dim3(256), 0, s, g, T);
}

// Step counter of a captured step: set from the host, advanced by the replay's
// last kernel.
__global__ void k_set_step(uint64_t* step_dev, uint64_t v) { *step_dev = v; }

void launch_set_step(uint64_t* step_dev, uint64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, step_dev, v);
}

// ============================================================ structure factors
// S(k) = sum_j q_j exp(i k.r_j), Eq. (15).  One thread per mode; the particle loop
// is uniform across the wave, so particle records arrive by scalar loads.  Grid:
// (mode tiles of 256, particle chunks, replicas); each block writes partial sums
// and k_sf_finalize adds them in chunk order and writes S, the coefficients w S
// and (FP32) the mode records.  stage 1: ions, S1.  stage 2: electrodes with the
// new charges, S = S1 + S2.  (A last-arriving-block reduction would need an
// agent-scope release fence per block, which writes back L2 and costs far more
// than the extra launch on a multi-XCD device.)
// S (and the coefficients, mode records) of mode k of replica r from its sums (sr, si)
// over the particles of this stage.
__device__ __forceinline__ void finalize_mode(const Geom& g, int r, int k, double sr, double si,
                                              const int4* modes, const double* w, double2* S1, double2* coef,
                                              ModeRec32* rec, int stage, unsigned* status) {
  const size_t idx = (size_t)r * g.K + k;
  if (stage == 1) {
    S1[idx] = make_double2(sr, si);
  } else {
    const double2 s1 = S1[idx];
    sr += s1.x;
    si += s1.y;
  }
  if (!isfinite(sr) || !isfinite(si)) atomicOr(status, ST_NUMERIC);
  const double wk = w[idx];
  coef[idx] = make_double2(wk * sr, wk * si);
  if (rec) {
    const int4 m = modes[idx];
    ModeRec32 o;
    o.mx = m.x;
    o.my = m.y;
    o.mz = m.z;
    o.cre = (float)(wk * sr);
    o.cim = (float)(wk * si);
    o.kx = (float)(TWO_PI * (double)m.x * g.invLx);
    o.ky = (float)(TWO_PI * (double)m.y * g.invLy);
    o.kz = (float)(TWO_PI * (double)m.z * g.invLz);
    rec[idx] = o;
  }
}

__device__ __forceinline__ void finalize_tile(const Geom& g, int r, int k, const double2* part, int nchunk,
                                              const int4* modes, const double* w, double2* S1, double2* coef,
                                              ModeRec32* rec, int stage, unsigned* status) {
  if (k >= g.K) return;
  // chunks 16 at a time, all requested before the first add, added in chunk order
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < nchunk; c += 16) {
    double2 p[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      p[u] = c + u < nchunk ? part[((size_t)r * nchunk + c + u) * g.K + k] : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (c + u < nchunk) {
        sr += p[u].x;
        si += p[u].y;
      }
  }
  finalize_mode(g, r, k, sr, si, modes, w, S1, coef, rec, stage, status);
}

// Sum over particles [j0, j1) of q_j exp(i 2 pi m.s_j) for one mode (FP64 fractions).
template <bool ION>
__device__ __forceinline__ double2 sf64_sum(const double4* __restrict__ pts, const double* __restrict__ qq, int4 m,
                                            int j0, int j1) {
  const double mx = m.x, my = m.y, mz = m.z;
  double sr = 0.0, si = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double4 p = pts[j];
    double t = fma(mx, p.x, fma(my, p.y, mz * p.z));
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    const double qj = ION ? p.w : qq[j];
    sr = fma(qj, cs, sr);
    si = fma(qj, sn, si);
  }
  return make_double2(sr, si);
}

// FP32: exact integer phase m.u mod 2^32 (u = 32-bit fixed-point fractions), the
// hardware sin/cos of the phase in revolutions, FP32 sums over blocks of 64
// particles carried in FP64.
//
// BF16 (the hi/lo variant, an error report): each factor x of a product q cos, q sin
// is split into x_hi = bf16(x) and x_lo = bf16(x - x_hi), and the product is taken as
// q_hi c_hi + q_hi c_lo + q_lo c_hi with FP32 accumulation -- the arithmetic of a
// structure factor on BF16 matrix cores (three BF16 products of hi/lo halves, FP32
// accumulate; each BF16 x BF16 product is exact in FP32), carried out on the VALU.
__device__ __forceinline__ float bf16_round(float x) {
  // round to nearest even at 8 mantissa bits (finite x)
  const uint32_t u = __float_as_uint(x);
  return __uint_as_float((u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u);
}

template <bool BF16>
__device__ __forceinline__ void sf32_term(float qj, float x, float& ar, float& ai) {
  const float c = __builtin_amdgcn_cosf(x), s = __builtin_amdgcn_sinf(x);
  if constexpr (BF16) {
    const float qh = bf16_round(qj), ql = bf16_round(qj - qh);
    const float ch = bf16_round(c), cl = bf16_round(c - ch);
    const float sh = bf16_round(s), sl = bf16_round(s - sh);
    ar = fmaf(qh, ch, ar);
    ar = fmaf(qh, cl, ar);
    ar = fmaf(ql, ch, ar);
    ai = fmaf(qh, sh, ai);
    ai = fmaf(qh, sl, ai);
    ai = fmaf(ql, sh, ai);
  } else {
    ar = fmaf(qj, c, ar);
    ai = fmaf(qj, s, ai);
  }
}

template <bool ION, bool BF16 = false>
__device__ __forceinline__ double2 sf32_sum(const uint4* __restrict__ pts, const float* __restrict__ qq, int4 m,
                                            int j0, int j1) {
  const uint32_t mx = (uint32_t)m.x, my = (uint32_t)m.y, mz = (uint32_t)m.z;
  double dr = 0.0, di = 0.0;
  for (int jb = j0; jb < j1; jb += 64) {
    const int je = min(j1, jb + 64);
    float ar = 0.f, ai = 0.f;
    int j = jb;
    for (; j + 4 <= je; j += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint4 p = pts[j + u];
        const float qj = ION ? __uint_as_float(p.w) : qq[j + u];
        const uint32_t ph = mx * p.x + my * p.y + mz * p.z;
        sf32_term<BF16>(qj, (float)(int32_t)ph * 0x1.0p-32f, ar, ai);
      }
    }
    for (; j < je; ++j) {
      const uint4 p = pts[j];
      const float qj = ION ? __uint_as_float(p.w) : qq[j];
      const uint32_t ph = mx * p.x + my * p.y + mz * p.z;
      sf32_term<BF16>(qj, (float)(int32_t)ph * 0x1.0p-32f, ar, ai);
    }
    dr += (double)ar;
    di += (double)ai;
  }
  return make_double2(dr, di);
}

// Block (tile, chunk, r) of the partial sums: modes [256 tile, 256 tile + 256) over
// the particle chunk.
template <bool ION>
__device__ __forceinline__ void sf64_block(const Geom& g, const int64_t* __restrict__ off,
                                           const double4* __restrict__ pts, const double* __restrict__ qe,
                                           const int4* __restrict__ modes, double2* __restrict__ part, int nchunk,
                                           int tile, int ch, int r) {
  const int k = tile * 256 + threadIdx.x;
  const int b = ION ? (int)off[r] : 0;
  const int e = ION ? (int)off[r + 1] : g.n_ele;
  const int chunk = (e - b + nchunk - 1) / nchunk;
  const int j0 = b + ch * chunk;
  const int j1 = min(e, j0 + chunk);
  const double* qq = ION ? nullptr : qe + (size_t)r * g.n_ele;
  if (k < g.K) part[((size_t)r * nchunk + ch) * g.K + k] = sf64_sum<ION>(pts, qq, modes[(size_t)r * g.K + k], j0, j1);
}

template <bool ION, bool BF16 = false>
__device__ __forceinline__ void sf32_block(const Geom& g, const int64_t* __restrict__ off,
                                           const uint4* __restrict__ pts, const float* __restrict__ qe,
                                           const int4* __restrict__ modes, double2* __restrict__ part, int nchunk,
                                           int tile, int ch, int r) {
  const int k = tile * 256 + threadIdx.x;
  const int b = ION ? (int)off[r] : 0;
  const int e = ION ? (int)off[r + 1] : g.n_ele;
  const int chunk = (e - b + nchunk - 1) / nchunk;
  const int j0 = b + ch * chunk;
  const int j1 = min(e, j0 + chunk);
  const float* qq = ION ? nullptr : qe + (size_t)r * g.n_ele;
  if (k < g.K)
    part[((size_t)r * nchunk + ch) * g.K + k] = sf32_sum<ION, BF16>(pts, qq, modes[(size_t)r * g.K + k], j0, j1);
}

// Partial-sum block lb of stage 1 (ions, ION) or 2 (electrodes with the new charges),
// lb = (r nchunk + chunk) ktiles + tile.
template <bool FP32, bool ION>
__device__ __forceinline__ void sf_block(const Geom& g, const StepBufs& b, int lb) {
  const int nchunk = ION ? b.nchunk_ion : b.nchunk_ele;
  const int tile = lb % b.ktiles, ch = (lb / b.ktiles) % nchunk, r = lb / (b.ktiles * nchunk);
  if constexpr (FP32) {
    if (b.bf16) {
      if constexpr (ION)
        sf32_block<true, true>(g, b.off, b.ion_fx, nullptr, b.modes, b.part, nchunk, tile, ch, r);
      else
        sf32_block<false, true>(g, b.off, b.ele_fx, b.Qf, b.modes, b.part, nchunk, tile, ch, r);
    } else {
      if constexpr (ION)
        sf32_block<true>(g, b.off, b.ion_fx, nullptr, b.modes, b.part, nchunk, tile, ch, r);
      else
        sf32_block<false>(g, b.off, b.ele_fx, b.Qf, b.modes, b.part, nchunk, tile, ch, r);
    }
  } else {
    if constexpr (ION)
      sf64_block<true>(g, b.off, b.ion_d4, nullptr, b.modes, b.part, nchunk, tile, ch, r);
    else
      sf64_block<false>(g, b.off, b.ele_d4, b.Q_out, b.modes, b.part, nchunk, tile, ch, r);
  }
}

__device__ __forceinline__ void sf_finalize_body(const Geom& g, const StepBufs& b, int stage, int lb) {
  const int r = lb / b.ktiles, tile = lb - r * b.ktiles;
  finalize_tile(g, r, tile * 256 + threadIdx.x, b.part, stage == 1 ? b.nchunk_ion : b.nchunk_ele, b.modes, b.w,
                b.S1, b.coef, b.rec, stage, b.status);
}

__global__ __launch_bounds__(256) void k_sf_finalize(Geom g, const double2* __restrict__ part, int nchunk,
                                                     const int4* __restrict__ modes, const double* __restrict__ w,
                                                     double2* __restrict__ S1, double2* __restrict__ coef,
                                                     ModeRec32* __restrict__ rec, int stage, unsigned* status) {
  finalize_tile(g, blockIdx.y, blockIdx.x * 256 + threadIdx.x, part, nchunk, modes, w, S1, coef, rec, stage, status);
}

// The same for many chunks per mode (large replicas, where one thread per mode would
// walk hundreds of dependent load rounds): block (tile of 16 modes, r) of 256 threads,
// thread (slice s, mode m) adding the chunks [s nchunk / 16, (s + 1) nchunk / 16) of its
// mode in chunk order, then the first 16 threads the 16 slice sums in slice order.
// Small blocks, since the launch usually runs beside the ion-ion pass, whose waves hold
// most of the wave slots: a block of 16 waves waited there for a compute unit to drain.
constexpr int kWideFinalizeChunks = 64;  // above this many chunks per mode

__global__ __launch_bounds__(256) void k_sf_finalize_wide(Geom g, const double2* __restrict__ part, int nchunk,
                                                          const int4* __restrict__ modes,
                                                          const double* __restrict__ w, double2* __restrict__ S1,
                                                          double2* __restrict__ coef, ModeRec32* __restrict__ rec,
                                                          int stage, unsigned* status) {
  __shared__ double2 ws[16][16];
  const int m = threadIdx.x & 15, sl = threadIdx.x >> 4;
  const int r = blockIdx.y, k = blockIdx.x * 16 + m;
  const int c0 = (int)((int64_t)sl * nchunk / 16), c1 = (int)((int64_t)(sl + 1) * nchunk / 16);
  double sr = 0.0, si = 0.0;
  if (k < g.K) {
    for (int c = c0; c < c1; c += 16) {
      double2 p[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        p[u] = c + u < c1 ? part[((size_t)r * nchunk + c + u) * g.K + k] : make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c + u < c1) {
          sr += p[u].x;
          si += p[u].y;
        }
    }
  }
  ws[sl][m] = make_double2(sr, si);
  __syncthreads();
  if (sl == 0 && k < g.K) {
    sr = ws[0][m].x;
    si = ws[0][m].y;
#pragma unroll
    for (int u = 1; u < 16; ++u) {
      sr += ws[u][m].x;
      si += ws[u][m].y;
    }
    finalize_mode(g, r, k, sr, si, modes, w, S1, coef, rec, stage, status);
  }
}

void launch_sf_finalize(const Geom& g, const StepBufs& b, int fp32, int stage, hipStream_t s) {
  if (g.K == 0) return;
  const int nchunk = stage == 1 ? b.nchunk_ion : b.nchunk_ele;
  if (nchunk > kWideFinalizeChunks)
    hipLaunchKernelGGL(k_sf_finalize_wide, dim3((g.K + 15) / 16, b.R), dim3(256), 0, s, g, b.part, nchunk, b.modes,
                       b.w, b.S1, b.coef, fp32 ? b.rec : nullptr, stage, b.status);
  else
    hipLaunchKernelGGL(k_sf_finalize, dim3(b.ktiles, b.R), dim3(256), 0, s, g, b.part, nchunk, b.modes, b.w, b.S1,
                       b.coef, fp32 ? b.rec : nullptr, stage, b.status);
}

// ============================================================ real-space kernels
// FP64 erfc(x) for x >= 0, with E = exp(-x^2) beside it for the derivative: erfc(x) =
// E t p(u), t = 1 / (1 + x/2), u = (2 t - 1 - t0) / (1 - t0) with t0 = t(27), p of degree
// 20 fitted to erfcx(x) / t on [0, 27] (coefficients from fit_erfc.py beside this file;
// relative error 1.3e-14 in FP64, plus that of exp(-x^2) from the rounded x^2, ~1e-16 x^2).
// Beyond x = 27, E and so the result are below the smallest FP64 subnormal.
__device__ __forceinline__ double erfc_e64(double x, double& E) {
  E = exp(-x * x);
  const double t = 1.0 / fma(0.5, x, 1.0);
  const double u = fma(t, 29.0 / 13.5, -15.5 / 13.5);
  double p = 5.18322347079050235e-09;
  p = fma(p, u, 9.15908983234418801e-09);
  p = fma(p, u, -5.96955725824229679e-08);
  p = fma(p, u, -1.83108728307537812e-08);
  p = fma(p, u, 3.12694522697253297e-07);
  p = fma(p, u, -3.29070948319133605e-07);
  p = fma(p, u, -7.35054674846839475e-07);
  p = fma(p, u, 2.72720061601437206e-06);
  p = fma(p, u, -1.71507364475183724e-06);
  p = fma(p, u, -1.05829830498160832e-05);
  p = fma(p, u, 2.76972235614982518e-05);
  p = fma(p, u, 1.44669835925712893e-05);
  p = fma(p, u, -1.85052166647616797e-04);
  p = fma(p, u, 1.42801899132745516e-04);
  p = fma(p, u, 1.10927368016556236e-03);
  p = fma(p, u, -1.79400388641047948e-03);
  p = fma(p, u, -8.83472414082498228e-03);
  p = fma(p, u, 1.21948287907252696e-02);
  p = fma(p, u, 1.24119759473117527e-01);
  p = fma(p, u, 3.38058442287577476e-01);
  p = fma(p, u, 5.35156895807327726e-01);
  return E * t * p;
}

// Eq. (13): ion-ion erfc(alpha r)/r and ion-Gaussian [erfc(alpha r) - erfc(r/eta)]/r.
__device__ __forceinline__ void erfc_over_r(double a, double r, double& f, double& df) {
  double E;
  const double e = erfc_e64(a * r, E);
  const double inv = 1.0 / r;
  f = e * inv;
  df = -e * inv * inv - 2.0 * a * INV_SQRT_PI * E * inv;
}

// FP32 pair kernel: with x = a r, f = erfc(x) / r and h = -(1/r) d/dr [erfc(x) / r]
// = (f + (2a / sqrt(pi)) exp(-x^2)) / r^2.  erfc(x) = exp(-x^2) t p(t) with
// t = 1 / (1 + x/2), p of degree 9 fitted to the scaled complementary error function
// (coefficients from fit_erfc.py beside this file; relative error 3.3e-7 in FP32 on
// x in [0, 10], beyond which erfc underflows FP32).  One exp serves both terms.
__device__ __forceinline__ void erfc_pair_f(float a, float r, float rinv, float& f, float& h) {
  const float x = a * r;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float p = 1.228336431e-02f;
  p = fmaf(p, t, -1.232539415e-01f);
  p = fmaf(p, t, 4.289312065e-01f);
  p = fmaf(p, t, -6.700319052e-01f);
  p = fmaf(p, t, 4.212864637e-01f);
  p = fmaf(p, t, -9.832625091e-02f);
  p = fmaf(p, t, 2.255454361e-01f);
  p = fmaf(p, t, 2.386439592e-01f);
  p = fmaf(p, t, 2.828571498e-01f);
  p = fmaf(p, t, 2.820644975e-01f);
  const float e = __builtin_amdgcn_exp2f(-x * x * 1.4426950408889634f);  // exp(-x^2)
  f = e * t * p * rinv;
  h = fmaf(2.0f * (float)INV_SQRT_PI * a, e, f) * (rinv * rinv);
}

// Wave totals through DPP: within each 16-lane row, pairs (quad_perm 1,0,3,2),
// quads (quad_perm 2,3,0,1), halves (row_half_mirror) and rows (row_mirror); then
// the four row sums, read from lanes 0, 16, 32, 48, are added in row order.  The
// result is wave-uniform and the same on every run.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float wave_total(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return ((r0 + r1) + r2) + r3;
}

__device__ __forceinline__ double wave_total(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16), r2 = readlane_f64(v, 32),
               r3 = readlane_f64(v, 48);
  return ((r0 + r1) + r2) + r3;
}

// base + the number of lanes below this one with their bit set in m.
__device__ __forceinline__ unsigned lanes_below(uint64_t m, unsigned base = 0u) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, base));
}

// The wave totals of four per-lane values, added in a fixed order.  Pairs of lanes
// exchange two values each (even lanes keep the sums of v0 and v2, odd lanes of v1 and
// v3), then pairs of pairs (lane l keeps value l mod 4); two rotations by 4 and 8 lanes
// inside each 16-lane row add the row's four lanes of each value; the four rows'
// totals pass through a 16-float wave-private LDS scratch, and lane m < 4 adds them in
// row order.  Every lane returns the same four totals.
__device__ __forceinline__ void wave_total4(float v0, float v1, float v2, float v3, float* scratch, float& t0,
                                            float& t1, float& t2, float& t3) {
  const int lane = threadIdx.x & 63;
  const bool odd = lane & 1, b1 = (lane & 2) != 0;
  const float x = (odd ? v1 : v0) + dpp_f<0xB1>(odd ? v0 : v1);
  const float y = (odd ? v3 : v2) + dpp_f<0xB1>(odd ? v2 : v3);
  float z = (b1 ? y : x) + dpp_f<0x4E>(b1 ? x : y);
  z += dpp_f<0x124>(z);  // row_ror:4
  z += dpp_f<0x128>(z);  // row_ror:8
  if ((lane & 15) < 4) scratch[(lane >> 4) * 4 + (lane & 15)] = z;
  __builtin_amdgcn_wave_barrier();
  float t = 0.f;
  if (lane < 4) t = ((scratch[lane] + scratch[4 + lane]) + scratch[8 + lane]) + scratch[12 + lane];
  __builtin_amdgcn_wave_barrier();
  t0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 0));
  t1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 1));
  t2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 2));
  t3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t), 3));
}

// Neighbour scan of ONE particle by a whole wave.  The candidates are the records of
// the particle's neighbour runs: lane s holds run s as a record range [rb, re) (see
// resolve_runs; an empty range is skipped), and the scan takes the runs from the
// lanes in order.  A wave round tests 64 candidates, one per lane (coalesced loads):
// inside a run a round is 64 consecutive records; the remainder of a run is topped
// up with the heads of the following runs (up to kSegMax pieces), so short runs do
// not leave lanes idle.  load(j) reads record j; test(record, j, entry) fills the
// pair entry and says whether the pair is within range (evaluated branch-free:
// every lane of a round holds a valid j).  The hits of a round are appended in
// candidate order to a wave-private LDS ring (positions from a ballot and a lane
// prefix count).  head and tail count the entries evaluated and queued;
// whenever 64 entries are queued, eval_block(head, head + 64) evaluates them, one per
// lane.  Entries left queued at the end stay in the ring: the caller evaluates them
// later, possibly together with the next particle's (so a wave that scans several
// particles in turn evaluates full blocks of 64 except at its very end).  The ring
// holds at most 63 + 64 entries, so kRing = 128 never overflows.  All control flow
// is wave-uniform; the evaluation order of the entries is fixed, so the result does
// not depend on timing.
constexpr int kRing = 128;
constexpr int kRingAlloc = kRing + 16;  // ring + scratch for the wave's final reductions
constexpr int kSegMax = 4;

// LDS of a block's four scanning waves: a ring of kRingAlloc entries each.
template <bool FP32>
constexpr int ring_bytes() {
  return 4 * kRingAlloc * (FP32 ? (int)sizeof(float4) : (int)sizeof(double4));
}

// A home cell's candidate list (ion-ion pass): when a cell's neighbours form several runs,
// the wave writes the record indices of all of them, in run order, into a list of up to
// kListCap 16-bit offsets from the first run's start, so that its ions' scans take full
// rounds of 64 list entries instead of topping up rounds from short runs.
constexpr int kListCap = 1024;
constexpr int kListBytes = 4 * kListCap * (int)sizeof(uint16_t);

static_assert(kRunMax < 64, "one lane per run, and a terminator lane");

// Lane s turns run s of a -1-terminated run list into a record range [rb, re) with
// range(s, run, rb, re) (empty when the run can be skipped); the ranges of all runs
// are loaded at once rather than as one dependent chain per run.
template <class RangeF>
__device__ __forceinline__ void resolve_runs(const int2* __restrict__ runs, RangeF range, int& rb, int& re) {
  const int lane = threadIdx.x & 63;
  rb = 0;
  re = 0;
  const int2 rc = lane < kRunMax ? runs[lane] : make_int2(-1, -1);
  const uint64_t term = __ballot(rc.x < 0);  // non-zero: the lanes >= kRunMax count as terminators
  const uint64_t listed = (1ull << __builtin_ctzll(term)) - 1;  // the runs before the first terminator
  if ((listed >> lane) & 1) range(lane, rc, rb, re);
}

template <class Entry, class LoadF, class RowF, class TestF, class EvalF>
__device__ __forceinline__ void wave_scan(int rb, int re, Entry* __restrict__ ring, unsigned& head, unsigned& tail,
                                          LoadF load, RowF load_row, TestF test, EvalF eval_block) {
  const int lane = threadIdx.x & 63;
  uint64_t live = __ballot(rb < re);
  int pos = 0, end = 0;
  auto next_run = [&]() {
    if (pos < end) return true;
    if (!live) return false;
    const int s = __builtin_ctzll(live);
    live &= live - 1;
    pos = __builtin_amdgcn_readlane(rb, s);
    end = __builtin_amdgcn_readlane(re, s);
    return true;
  };
  auto round = [&](const auto& rec, int j, bool valid) {
    Entry ent;
    const bool hit = test(rec, j, ent) & valid;
    const uint64_t m = __ballot(hit);
    if (hit) ring[lanes_below(m, tail) & (kRing - 1)] = ent;
    tail += (unsigned)__popcll(m);
    if (tail - head >= 64) {
      __builtin_amdgcn_wave_barrier();
      eval_block(head, head + 64);
      head += 64;
    }
  };
  while (next_run()) {
    if (end - pos >= 64) {
      // full rounds inside the run in groups of three, three record buffers in
      // rotation: the records of the next two rounds are in flight while the
      // current round is tested, and each buffer is reloaded in place after use,
      // unconditionally, so no in-flight register is copied or merged.  load_row(j0)
      // reads record j0 + lane from a wave-uniform base, so a round's load needs no
      // per-lane address arithmetic.  Requests past the run (at most kScanPad
      // records, inside the arrays' padding) are not used.
      const int p0 = pos, nfull = (end - pos) >> 6;
      auto ld = [&](int t) { return load_row(p0 + 64 * t); };
      auto A = ld(0), B = ld(1), C = ld(2);
      int t = 0;
      for (; t + 3 <= nfull; t += 3) {
        round(A, p0 + 64 * t + lane, true);
        A = ld(t + 3);
        round(B, p0 + 64 * (t + 1) + lane, true);
        B = ld(t + 4);
        round(C, p0 + 64 * (t + 2) + lane, true);
        C = ld(t + 5);
      }
      if (t < nfull) round(A, p0 + 64 * t + lane, true);
      if (t + 1 < nfull) round(B, p0 + 64 * (t + 1) + lane, true);
      pos = p0 + 64 * nfull;
    }
    if (pos >= end) continue;
    // the run's remainder (< 64 records), topped up from the following runs:
    // lanes [from[u], from[u+1]) take records lane + base[u]
    int base[kSegMax], from[kSegMax];
    int filled = end - pos;
    base[0] = pos;
    from[0] = 0;
    pos = end;
#pragma unroll
    for (int u = 1; u < kSegMax; ++u) {
      base[u] = 0;
      from[u] = 64;
      if (filled < 64 && next_run()) {
        const int take = min(64 - filled, end - pos);
        base[u] = pos - filled;
        from[u] = filled;
        filled += take;
        pos += take;
      }
    }
    int j = lane + base[0];
#pragma unroll
    for (int u = 1; u < kSegMax; ++u)
      if (lane >= from[u]) j = lane + base[u];
    const bool valid = lane < filled;
    const int jj = valid ? j : base[0];  // lane 0 always holds a valid record
    round(load(jj), jj, valid);
  }
}

// The same scan over a candidate list (see kListCap): candidate q is record base + list[q],
// q < total.  Rounds of 64 list entries, the records of the next two rounds in flight (a
// request past the list's end repeats its last record and is not used).  The candidates
// come in the order wave_scan takes them, so the hits reach the ring in the same order
// and the results are the same bit for bit.
template <class Entry, class LoadF, class TestF, class EvalF>
__device__ __forceinline__ void wave_scan_list(const uint16_t* __restrict__ list, int total, int base,
                                               Entry* __restrict__ ring, unsigned& head, unsigned& tail,
                                               LoadF load, TestF test, EvalF eval_block) {
  const int lane = threadIdx.x & 63;
  auto round = [&](const auto& rec, int j, bool valid) {
    Entry ent;
    const bool hit = test(rec, j, ent) & valid;
    const uint64_t m = __ballot(hit);
    if (hit) ring[lanes_below(m, tail) & (kRing - 1)] = ent;
    tail += (unsigned)__popcll(m);
    if (tail - head >= 64) {
      __builtin_amdgcn_wave_barrier();
      eval_block(head, head + 64);
      head += 64;
    }
  };
  const int nr = (total + 63) >> 6;
  auto jof = [&](int t) { return base + (int)list[min(64 * t + lane, total - 1)]; };
  int jA = jof(0), jB = jof(1), jC = jof(2);
  auto A = load(jA), B = load(jB), C = load(jC);
  int t = 0;
  for (; t + 3 <= nr; t += 3) {
    round(A, jA, 64 * t + lane < total);
    jA = jof(t + 3);
    A = load(jA);
    round(B, jB, 64 * (t + 1) + lane < total);
    jB = jof(t + 4);
    B = load(jB);
    round(C, jC, 64 * (t + 2) + lane < total);
    jC = jof(t + 5);
    C = load(jC);
  }
  if (t < nr) round(A, jA, 64 * t + lane < total);
  if (t + 1 < nr) round(B, jB, 64 * (t + 1) + lane < total);
}

// Builds the candidate list of a home cell from its runs (lane s: run s as [rb, re)) when
// there are at least two and they fit (at most kListCap records, spanning under 2^16);
// returns false otherwise.  total and base: the list's length and offset base.  keep(j)
// drops record j from the list when false: the caller passes a test that is false only
// for records no ion of the home cell can reach, so the list still holds every partner,
// in the same order.
template <class KeepF>
__device__ __forceinline__ bool build_list(int rb, int re, uint16_t* __restrict__ list, int& total, int& base,
                                           KeepF keep) {
  const int lane = threadIdx.x & 63;
  const uint64_t live = __ballot(rb < re);
  if (__popcll(live) < 2) return false;
  base = __builtin_amdgcn_readlane(rb, __builtin_ctzll(live));
  const int last = __builtin_amdgcn_readlane(re, 63 - __builtin_clzll(live));
  int n = 0;
  for (uint64_t m = live; m; m &= m - 1) {
    const int s = __builtin_ctzll(m);
    n += __builtin_amdgcn_readlane(re, s) - __builtin_amdgcn_readlane(rb, s);
  }
  if (n > kListCap || last - base > 65535) return false;
  int at = 0;
  for (uint64_t m = live; m; m &= m - 1) {
    const int s = __builtin_ctzll(m);
    const int b0 = __builtin_amdgcn_readlane(rb, s), len = __builtin_amdgcn_readlane(re, s) - b0;
#pragma unroll 1
    for (int t0 = 0; t0 < len; t0 += 64) {
      const int t = t0 + lane;
      const bool k = t < len && keep(b0 + t);
      const uint64_t km = __ballot(k);
      if (k) list[at + lanes_below(km, 0)] = (uint16_t)(b0 - base + t);
      at += __popcll(km);
    }
  }
  total = at;
  __builtin_amdgcn_wave_barrier();
  return true;
}

// The electrode-potential pass can split each chunk's candidate records over esplit
// waves (1, 2 or 4; a contiguous share of every neighbour run each), so that a small
// batch, which would leave most of the chip idle, runs esplit times as many waves
// over shorter chains; the shares' sums are added in wave order through LDS.
int ele_split(int units) { return units >= 2048 ? 1 : units >= 1024 ? 2 : 4; }

// Real-space potential of the ions at each electrode (real-space part of Eq. (19)):
// bN_j = ke sum_i q_i [erfc(alpha r) - erfc(r/eta)]/r over ions with r < rc.  One
// lane per electrode: a wave takes up to 64 cell-sorted electrodes of one cell (the
// chunk list is built at set-up), so its lanes share the cell's neighbour runs and
// walk the same ion records in lockstep.  The records are uniform across the wave
// (scalar loads, in groups requested one group ahead); each lane tests its own
// distance and the pair
// terms run only for the lanes in range.  Each lane adds its terms in record
// order.  In FP32 the erfc(r/eta) term is not evaluated beyond eta_skip, where it
// is below 2^-30 of the kept term.
template <bool FP32>
__device__ __forceinline__ void real_ele_wave(const Geom& g, const StepBufs& bb, int chunk, int r, int q,
                                              int esplit, bool live_wave, double* __restrict__ part_sums) {
  const int64_t* __restrict__ off = bb.off;
  const int* __restrict__ cstart = bb.cstart;
  const uint4* __restrict__ sfx = bb.sfx;
  const double4* __restrict__ sd4 = bb.sd4;
  const int* __restrict__ ele_perm = bb.ele_perm;
  const int2* __restrict__ ion_runs = bb.ion_runs;
  const uint4* __restrict__ ele_sfx = bb.ele_sfx;
  const double4* __restrict__ ele_sd4 = bb.ele_sd4;
  double* __restrict__ bN = bb.bN;
  const int4 ch = bb.ele_chunks[chunk];  // (cell, first, end) of this wave's electrodes
  const int e = ch.y + (int)(threadIdx.x & 63);
  const bool live = e < ch.z;
  const int ec = live ? e : ch.y;
  const int b0 = (int)off[r];
  const int* cs = cstart + (size_t)r * (g.ncell + 1);
  const int2* runs = ion_runs + kRunMax * ch.x;
  double sum;
  if constexpr (FP32) {
    const uint4 pe = ele_sfx[ec];
    const float lx = (float)(g.Lx * 0x1.0p-32), ly = (float)(g.Ly * 0x1.0p-32), lz = (float)(g.Lz * 0x1.0p-32);
    const float a1 = (float)g.alpha, a2 = (float)(1.0 / g.eta), rc2 = (float)(g.rc * g.rc);
    float acc = 0.f;
    auto pair = [&](const uint4& p) {
      const float dx = (float)(int32_t)(pe.x - p.x) * lx;
      const float dy = (float)(int32_t)(pe.y - p.y) * ly;
      const float dz = (float)(int32_t)(pe.z - p.z) * lz;
      const float r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2) {
        const float rinv = __builtin_amdgcn_rsqf(r2), rr = r2 * rinv;
        float f1, h1, f2 = 0.f, h2;
        erfc_pair_f(a1, rr, rinv, f1, h1);
        if (rr < g.eta_skip) erfc_pair_f(a2, rr, rinv, f2, h2);
        acc = fmaf(__uint_as_float(p.w), f1 - f2, acc);
      }
    };
    for (int si = 0; si < kRunMax; ++si) {
      const int2 rc = runs[si];
      if (rc.x < 0) break;
      const int jb = b0 + cs[rc.x], jl = b0 + cs[rc.y] - jb;
      const int je = jb + (jl * (q + 1)) / esplit;  // this wave's share of the run
      int j = jb + (jl * q) / esplit;
      // groups of four records in two buffers: the next group is in flight while the
      // current one is used (loads past the run are clamped to its last record)
      if (j + 4 <= je) {
        uint4 A[4], B[4];
        auto ld = [&](uint4(&X)[4], int j0) {
#pragma unroll
          for (int u = 0; u < 4; ++u) X[u] = sfx[min(j0 + u, je - 1)];
        };
        ld(A, j);
        ld(B, j + 4);
        for (;;) {
#pragma unroll
          for (int u = 0; u < 4; ++u) pair(A[u]);
          j += 4;
          if (j + 4 > je) break;
          ld(A, j + 4);
#pragma unroll
          for (int u = 0; u < 4; ++u) pair(B[u]);
          j += 4;
          if (j + 4 > je) break;
          ld(B, j + 4);
        }
      }
      for (; j < je; ++j) pair(sfx[j]);
    }
    sum = (double)acc;
  } else {
    const double4 pe = ele_sd4[ec];
    const double a = g.alpha, ai = 1.0 / g.eta, rc2 = g.rc * g.rc;
    double acc = 0.0;
    auto pair = [&](const double4& p) {
      double sx = pe.x - p.x, sy = pe.y - p.y;
      sx -= rint(sx);
      sy -= rint(sy);
      const double dx = sx * g.Lx, dy = sy * g.Ly, dz = (pe.z - p.z) * g.Lz;
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2) {
        const double rr = sqrt(r2);
        double f1, d1, f2, d2;
        erfc_over_r(a, rr, f1, d1);
        erfc_over_r(ai, rr, f2, d2);
        acc += p.w * (f1 - f2);
      }
    };
    for (int si = 0; si < kRunMax; ++si) {
      const int2 rc = runs[si];
      if (rc.x < 0) break;
      const int jb = b0 + cs[rc.x], jl = b0 + cs[rc.y] - jb;
      const int je = jb + (jl * (q + 1)) / esplit;  // this wave's share of the run
      int j = jb + (jl * q) / esplit;
      if (j + 2 <= je) {
        double4 cur[2], nxt[2];
        cur[0] = sd4[j];
        cur[1] = sd4[j + 1];
        for (; j + 4 <= je; j += 2) {
          nxt[0] = sd4[j + 2];
          nxt[1] = sd4[j + 3];
          pair(cur[0]);
          pair(cur[1]);
          cur[0] = nxt[0];
          cur[1] = nxt[1];
        }
        pair(cur[0]);
        pair(cur[1]);
        j += 2;
      }
      for (; j < je; ++j) pair(sd4[j]);
    }
    sum = acc;
  }
  // the esplit waves' sums of each electrode, added in wave order
  const int w = threadIdx.x >> 6;
  part_sums[w * 64 + (threadIdx.x & 63)] = sum;
  __syncthreads();
  if (q == 0 && live && live_wave) {
    double t = part_sums[w * 64 + (threadIdx.x & 63)];
    for (int u = 1; u < esplit; ++u) t += part_sums[(w + u) * 64 + (threadIdx.x & 63)];
    bN[(size_t)r * g.n_ele + ele_perm[e]] = g.ke * t;
  }
}

// k-space stage 1 beside the electrode-side real-space pass (both follow the sort and
// the sampler): blocks [0, nre) are real-space blocks (4 / esplit electrode chunks
// each, a chunk's esplit waves taking a share of its candidates each; chunk unit
// u = r n_chunks + chunk), blocks [nre, nre + nsf) are structure-factor partial
// blocks.  The real-space waves are latency-bound, so they are dispatched first and
// the arithmetic-bound partial blocks fill the issue slots they leave.
template <bool FP32>
__device__ __forceinline__ void stage_ions_body(const Geom& g, const StepBufs& b, int nsf, int nre, int esplit,
                                                int bid) {
  __shared__ double part_sums[4 * 64];
  if (bid < nre) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int units = b.n_ele_chunks * b.R;
    const int u = bid * (4 / esplit) + w / esplit;  // chunk unit of this wave: u = r n_chunks + chunk
    const bool live_wave = u < units;
    const int uu = live_wave ? u : units - 1;       // a past-the-end wave repeats the last unit, unstored
    real_ele_wave<FP32>(g, b, uu % b.n_ele_chunks, uu / b.n_ele_chunks, w % esplit, esplit, live_wave, part_sums);
  } else {
    sf_block<FP32, true>(g, b, bid - nre);
  }
}

template <bool FP32>
__global__ __launch_bounds__(256) void k_stage_ions(Geom g, StepBufs b, int nsf, int nre, int esplit) {
  stage_ions_body<FP32>(g, b, nsf, nre, esplit, blockIdx.x);
}

void launch_stage_ions(const Geom& g, const StepBufs& b, int fp32, int parts, hipStream_t s) {
  const int units = b.n_ele_chunks * b.R, esplit = b.esplit;
  const int nsf = (parts & STAGE_SF && g.K > 0) ? b.ktiles * b.nchunk_ion * b.R : 0;
  const int nre = (parts & STAGE_REAL && g.n_ele > 0) ? (units * esplit + 3) / 4 : 0;
  if (nsf + nre == 0) return;
  if (fp32)
    hipLaunchKernelGGL(k_stage_ions<true>, dim3(nsf + nre), dim3(256), 0, s, g, b, nsf, nre, esplit);
  else
    hipLaunchKernelGGL(k_stage_ions<false>, dim3(nsf + nre), dim3(256), 0, s, g, b, nsf, nre, esplit);
}

// The force and potential passes: 64 particles per block, the mode list split
// into W parts, one per wave (so each wave still walks a uniform mode list: the
// wave index is made explicitly uniform so that the mode records are read with
// scalar loads), and the W partial results added in wave order through LDS.  W and
// the unroll depth U of the FP32 mode loops are chosen per workload by the tuner.
template <int W>
__device__ __forceinline__ void mode_part(int K, int& lo, int& hi) {
  const int q = (K + W - 1) / W;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  lo = min(K, w * q);
  hi = min(K, lo + q);
}

// Runs fn(W, U) with W in {2, 4, 8} waves per block and U in {2, 4, 8} as
// compile-time constants (other values fall back to 4).
template <typename Fn>
void with_wu(int w, int u, Fn&& fn) {
  auto pick_u = [&](auto W) {
    switch (u) {
      case 2: fn(W, std::integral_constant<int, 2>{}); break;
      case 8: fn(W, std::integral_constant<int, 8>{}); break;
      default: fn(W, std::integral_constant<int, 4>{}); break;
    }
  };
  switch (w) {
    case 2: pick_u(std::integral_constant<int, 2>{}); break;
    case 8: pick_u(std::integral_constant<int, 8>{}); break;
    default: pick_u(std::integral_constant<int, 4>{}); break;
  }
}

// ============================================================ electrode potential b*
// b*_j = -sum_k Re(coef_k exp(-i k.R_j))           (Eq. (24), coef = w S1)
//        - (4 pi ke / V) Z_j sum_i q_i z_i          (slab term, minus sign)
//        - bN_j                                     (real space; left out if bN is null)
// and V_j = b*_j + dpsi d_j, the right-hand side of the charge solve (rows of
// ldcp(n) doubles per replica for the GEMM below).
template <int W>
__device__ __forceinline__ void elepot_write(const Geom& g, int r, int j, double acc_part, double (*sh)[64],
                                             const double* ele_xyz, const double* ele_d, const double* scal,
                                             const double* dpsi, const double* bN, double* bstar, double* V) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  sh[w][lane] = acc_part;
  __syncthreads();
  if (w == 0 && j >= g.n_ele && j < ldcp(g.n_ele)) V[(size_t)r * ldcp(g.n_ele) + j] = 0.0;  // padding
  if (w == 0 && j < g.n_ele) {
    double acc = sh[0][lane];
#pragma unroll
    for (int u = 1; u < W; ++u) acc += sh[u][lane];
    const int n = g.n_ele;
    const double Z = ele_xyz[2 * n + j];
    const size_t idx = (size_t)r * n + j;
    const double b = -acc - (4.0 * M_PI * g.ke / g.V) * Z * scal[4 * r + 2] - (bN ? bN[idx] : 0.0);
    bstar[idx] = b;
    V[(size_t)r * ldcp(n) + j] = b + dpsi[r] * ele_d[j];
  }
}

// Block (tile, r): electrodes 64 tile .. 64 tile + 63 of replica r.
template <int W>
__device__ __forceinline__ void elepot64_body(const Geom& g, const StepBufs& b, int tile, int r) {
  const double* __restrict__ ele_xyz = b.ele_xyz;
  const double4* __restrict__ ele_d4 = b.ele_d4;
  const double* __restrict__ ele_d = b.ele_d;
  const int4* __restrict__ modes = b.modes;
  const double2* __restrict__ coef = b.coef;
  const double* __restrict__ scal = b.scal;
  const double* __restrict__ dpsi = b.dpsi;
  const double* __restrict__ bN = b.real ? b.bN : nullptr;
  double* __restrict__ bstar = b.bstar;
  double* __restrict__ V = b.V;
  __shared__ double sh[W][64];
  const int j = tile * 64 + (threadIdx.x & 63);
  const double4 p = j < g.n_ele ? ele_d4[j] : make_double4(0, 0, 0, 0);
  int lo, hi;
  mode_part<W>(g.K, lo, hi);
  double acc = 0.0;
  const int4* mr = modes + (size_t)r * g.K;
  const double2* cr = coef + (size_t)r * g.K;
  for (int k = lo; k < hi; ++k) {
    const int4 m = mr[k];
    double t = fma((double)m.x, p.x, fma((double)m.y, p.y, (double)m.z * p.z));
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    const double2 c = cr[k];
    acc = fma(c.x, cs, fma(c.y, sn, acc));
  }
  elepot_write<W>(g, r, j, acc, sh, ele_xyz, ele_d, scal, dpsi, bN, bstar, V);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_elepot64(Geom g, StepBufs b) {
  elepot64_body<W>(g, b, blockIdx.x, blockIdx.y);
}

template <int W, int U>
__device__ __forceinline__ void elepot32_body(const Geom& g, const StepBufs& b, int tile, int r) {
  const uint4* __restrict__ ele_fx = b.ele_fx;
  const double* __restrict__ ele_xyz = b.ele_xyz;
  const double* __restrict__ ele_d = b.ele_d;
  const ModeRec32* __restrict__ rec = b.rec;
  const double* __restrict__ scal = b.scal;
  const double* __restrict__ dpsi = b.dpsi;
  const double* __restrict__ bN = b.real ? b.bN : nullptr;
  double* __restrict__ bstar = b.bstar;
  double* __restrict__ V = b.V;
  __shared__ double sh[W][64];
  const int j = tile * 64 + (threadIdx.x & 63);
  const uint4 pe = j < g.n_ele ? ele_fx[j] : make_uint4(0, 0, 0, 0);
  int lo, hi;
  mode_part<W>(g.K, lo, hi);
  const ModeRec32* mr = rec + (size_t)r * g.K;
  double acc = 0.0;
  for (int kb = lo; kb < hi; kb += 64) {
    const int ke_ = min(hi, kb + 64);
    float a = 0.f;
    int k = kb;
    for (; k + U <= ke_; k += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const ModeRec32 m = mr[k + u];
        const uint32_t ph = (uint32_t)m.mx * pe.x + (uint32_t)m.my * pe.y + (uint32_t)m.mz * pe.z;
        const float x = (float)(int32_t)ph * 0x1.0p-32f;
        a = fmaf(m.cre, __builtin_amdgcn_cosf(x), a);
        a = fmaf(m.cim, __builtin_amdgcn_sinf(x), a);
      }
    }
    for (; k < ke_; ++k) {
      const ModeRec32 m = mr[k];
      const uint32_t ph = (uint32_t)m.mx * pe.x + (uint32_t)m.my * pe.y + (uint32_t)m.mz * pe.z;
      const float x = (float)(int32_t)ph * 0x1.0p-32f;
      a = fmaf(m.cre, __builtin_amdgcn_cosf(x), a);
      a = fmaf(m.cim, __builtin_amdgcn_sinf(x), a);
    }
    acc += (double)a;
  }
  elepot_write<W>(g, r, j, acc, sh, ele_xyz, ele_d, scal, dpsi, bN, bstar, V);
}

template <int W, int U>
__global__ __launch_bounds__(64 * W) void k_elepot32(Geom g, StepBufs b) {
  elepot32_body<W, U>(g, b, blockIdx.x, blockIdx.y);
}

void launch_ele_potential(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  const dim3 grid(cdiv64(g.n_ele, 64), b.R);
  with_wu(b.kw, fp32 ? b.unroll : 4, [&](auto W, auto U) {
    constexpr int w = decltype(W)::value, u = decltype(U)::value;
    if (fp32)
      hipLaunchKernelGGL((k_elepot32<w, u>), grid, dim3(64 * w), 0, s, g, b);
    else if constexpr (u == 4)  // the FP64 loop has no unroll parameter
      hipLaunchKernelGGL((k_elepot64<w>), grid, dim3(64 * w), 0, s, g, b);
  });
}

// ============================================================ charge solve
// [Q; psibar] = S_ext V (Eqs. (9)-(11)).  S_ext: (n+1) rows of ld = ldcp(n) doubles
// (row-major; the n x n block is symmetric); V: one row of ld doubles per replica;
// both zero-padded to ld, a multiple of 32.  A block computes a 64-row x 64-replica
// tile over one k-range: per KB-k block (KB = 16 or 32, chosen by the tuner) the two
// 64 x KB operand tiles are loaded by all 256 threads (coalesced 16-byte loads,
// KB / 4 doubles per thread and operand) into LDS (double buffered, rows padded by
// 2 doubles against bank conflicts), the next block's tiles travelling from HBM
// while the current one is multiplied: the wider block keeps twice the bytes in
// flight for twice the multiply time.  Each wave owns 16 rows: FP64 MFMA
// v_mfma_f64_16x16x4f64, lane l supplying A[l%16][k(l)] and B[k(l)][l%16], the
// result register v of lane l being row l/16 + 4 v, column l%16.  The contraction
// index k(l) may be any assignment of the 4 k values to the 4 lane groups as long
// as A and B use the same one: here a lane holds 4 consecutive k of its row (two
// 16-byte LDS reads) per 16 k and MFMA step u takes the u-th of them.  Rows past n
// and replicas past R read row 0 / replica 0 (valid memory) and are not stored.
// The k range is split into ksplit ranges (grid z), sized so that the grid fits the
// CUs in one pass; each range writes its own partial, summed in order after the
// GEMM.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));  // register staging (an array of
                                                             // HIP's double2 is kept in scratch)

template <int KB>
constexpr int gemm_ld() { return KB + 2; }  // LDS row stride of an operand tile (doubles)
template <int KB>
constexpr int gemm_lds_bytes() { return 2 * 2 * 64 * gemm_ld<KB>() * (int)sizeof(double); }

// Tile (rt, cg) of k-range h of ks.  lds_raw: gemm_lds_bytes<KB>() bytes,
// [buffer][A or B][64 rows x KB k, padded].
template <int KB>
__device__ __forceinline__ void cp_gemm_tile(int n, int R, const double* __restrict__ S, const double* __restrict__ V,
                                             double* __restrict__ Qpart, int rt, int cg, int h, int ks, void* lds_raw) {
  constexpr int LD = gemm_ld<KB>(), NL = KB / 8;  // NL: 16-byte loads per thread and operand
  double(*lds)[2][64 * LD] = reinterpret_cast<double(*)[2][64 * LD]>(lds_raw);
  const int ld = ldcp(n);
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nb = ld / KB;
  const int kb0 = (int)((int64_t)nb * h / ks), kb1 = (int)((int64_t)nb * (h + 1) / ks);
  // tile loader: thread t moves KB / 4 consecutive k of row t / 4 of each tile
  const int lrow = t >> 2, lk = (KB / 4) * (t & 3);
  const int arow = rt * 64 + lrow, brow = cg * 64 + lrow;
  const double* Ag = S + (size_t)(arow <= n ? arow : 0) * ld + lk;
  const double* Bg = V + (size_t)(brow < R ? brow : 0) * ld + lk;
  f64x2 ra[NL], rb[NL];
  auto gload = [&](int kb) {
    const int k0 = kb * KB;
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      ra[u] = *(const f64x2*)(Ag + k0 + 2 * u);
      rb[u] = *(const f64x2*)(Bg + k0 + 2 * u);
    }
  };
  auto lstore = [&](int buf) {
    double* A = &lds[buf][0][lrow * LD + lk];
    double* B = &lds[buf][1][lrow * LD + lk];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      *(f64x2*)(A + 2 * u) = ra[u];
      *(f64x2*)(B + 2 * u) = rb[u];
    }
  };
  f64x4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int kq = 4 * (lane >> 4);
  if (kb0 < kb1) {
    gload(kb0);
    lstore(0);
    __syncthreads();
    for (int kb = kb0; kb < kb1; ++kb) {
      const int buf = (kb - kb0) & 1;
      if (kb + 1 < kb1) gload(kb + 1);
#pragma unroll
      for (int sub = 0; sub < KB / 16; ++sub) {
        const double* A = &lds[buf][0][(w * 16 + (lane & 15)) * LD + 16 * sub + kq];
        const double2 a01 = *(const double2*)A, a23 = *(const double2*)(A + 2);
        double2 b01[4], b23[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double* B = &lds[buf][1][(c * 16 + (lane & 15)) * LD + 16 * sub + kq];
          b01[c] = *(const double2*)B;
          b23[c] = *(const double2*)(B + 2);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.x, b01[c].x, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a01.y, b01[c].y, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.x, b23[c].x, acc[c], 0, 0, 0);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a23.y, b23[c].y, acc[c], 0, 0, 0);
      }
      if (kb + 1 < kb1) lstore(buf ^ 1);
      __syncthreads();
    }
  }
  // this wave's 16 rows x 64 replicas of the partial
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rt * 64 + w * 16 + (lane >> 4) + 4 * v, r = cg * 64 + c * 16 + (lane & 15);
      if (row <= n && r < R) Qpart[((size_t)h * R + r) * (n + 1) + row] = acc[c][v];
    }
}

// The GEMM's tiles, one block each (rt fastest, then cg, then the k-range).
template <int KB>
__global__ __launch_bounds__(256) void k_cp_gemm(Geom g, StepBufs b, const double* __restrict__ S, int nrt, int ncg) {
  __shared__ __align__(16) unsigned char lds[gemm_lds_bytes<KB>()];
  const int bid = blockIdx.x;
  cp_gemm_tile<KB>(g.n_ele, b.R, S, b.V, b.Qext, bid % nrt, (bid / nrt) % ncg, bid / (nrt * ncg), b.ksplit, lds);
}

// k-ranges: as many as keep the grid within one block per CU of a 256-CU device
// (at most 16, at least 1).
int cp_gemm_ksplit(int n_ele, int R) {
  const int tiles = ((n_ele + 1 + 63) / 64) * ((R + 63) / 64);
  return std::max(1, std::min(kMaxGemmSplit, 256 / std::max(tiles, 1)));
}

void launch_cp_gemm(const Geom& g, const StepBufs& b, const double* Sext, hipStream_t s) {
  const int n = g.n_ele;
  const int nrt = (n + 1 + 63) / 64, ncg = (b.R + 63) / 64, ntile = nrt * ncg * b.ksplit;
  if (!Sext || ntile == 0) return;
  if (b.gemm_depth == 2)
    hipLaunchKernelGGL(k_cp_gemm<32>, dim3(ntile), dim3(256), 0, s, g, b, Sext, nrt, ncg);
  else
    hipLaunchKernelGGL(k_cp_gemm<16>, dim3(ntile), dim3(256), 0, s, g, b, Sext, nrt, ncg);
}

// ============================================================ after the charge solve
// Per replica: copy Q (and psibar) out of the GEMM result (or the fixed charges);
// the copies of Q the later passes read (FP32 original order and cell-sorted
// order); sums of Q Z (slab term), d.Q and b*.Q (energy), and Q^2 and bN.Q (its parts).
__device__ __forceinline__ double rsum_total(const double* rsum, int r, int q) {
  const double* rs = rsum + (size_t)r * kRsumStride + q;
  double t = rs[0];
#pragma unroll
  for (int p = 1; p < kRsumParts; ++p) t += rs[kRsumSlots * p];
  return t;
}

// Q_j of replica r from the GEMM partials, added in k-range order.  All partials are
// requested before the first add (ksplit <= kMaxGemmSplit), so that one thread waits
// out one memory latency rather than ksplit of them.
__device__ __forceinline__ double solved_q(const double* __restrict__ Qext, int ksplit, int R, int r, int n, int j) {
  double p[kMaxGemmSplit];
#pragma unroll
  for (int h = 0; h < kMaxGemmSplit; ++h) p[h] = h < ksplit ? Qext[((size_t)h * R + r) * (n + 1) + j] : 0.0;
  double q = p[0];
#pragma unroll
  for (int h = 1; h < kMaxGemmSplit; ++h)
    if (h < ksplit) q += p[h];
  return q;
}

// Block (r, pc): electrodes [j0, j1) of replica r, at most one per thread; their
// positions in the cell-sorted order come from the set-up's inverse permutation, so
// every load is independent of every other.
__device__ __forceinline__ void post_charges_body(const Geom& g, const StepBufs& b, int fixedQ, int fp32, int r,
                                                  int pc) {
  const double* __restrict__ Qext = b.Qext;
  const int ksplit = b.ksplit;
  const double* __restrict__ Q_in = fixedQ ? b.Q_in : nullptr;
  const double* __restrict__ ele_xyz = b.ele_xyz;
  const double* __restrict__ ele_d = b.ele_d;
  const int* __restrict__ ele_iperm = b.ele_iperm;
  const double* __restrict__ bstar = b.bstar;
  double* __restrict__ Q_out = b.Q_out;
  float* __restrict__ Qf = fp32 ? b.Qf : nullptr;
  float* __restrict__ Qsf = fp32 ? b.Qsf : nullptr;
  double* __restrict__ Qsd = fp32 ? nullptr : b.Qsd;
  double* __restrict__ psibar = b.psibar_out;
  double* __restrict__ rsum = b.rsum;
  unsigned* status = b.status;
  const double* __restrict__ bN = b.real ? b.bN : nullptr;
  __shared__ double sh[5][4];
  const int R = b.R;
  const int n = g.n_ele;
  const int j0 = (int)((int64_t)n * pc / kRsumParts), j1 = (int)((int64_t)n * (pc + 1) / kRsumParts);
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int bad = 0;
  for (int j = j0 + threadIdx.x; j < j1; j += 256) {
    const int k = ele_iperm[j];
    const double Qj = Q_in ? Q_in[(size_t)r * n + j] : solved_q(Qext, ksplit, R, r, n, j);
    if (!isfinite(Qj)) bad = 1;
    Q_out[(size_t)r * n + j] = Qj;
    if (Qf) Qf[(size_t)r * n + j] = (float)Qj;
    if (Qsf) Qsf[(size_t)r * n + k] = (float)Qj;
    if (Qsd) Qsd[(size_t)r * n + k] = Qj;
    v[0] += Qj * ele_xyz[2 * n + j];
    v[1] += Qj * ele_d[j];
    v[2] += Qj * bstar[(size_t)r * n + j];
    v[3] += Qj * Qj;
    if (bN) v[4] += Qj * bN[(size_t)r * n + j];
  }
  if (bad) atomicOr(status, ST_NUMERIC);
  block_sum<256, 5>(v, sh);
  if (threadIdx.x == 0) {
    double* rs = rsum + (size_t)r * kRsumStride + kRsumSlots * pc;
#pragma unroll
    for (int q = 0; q < 5; ++q) rs[q] = v[q];
    if (psibar && pc == 0) psibar[r] = Q_in ? (double)NAN : solved_q(Qext, ksplit, R, r, n, n);
  }
}

__global__ __launch_bounds__(256) void k_post_charges(Geom g, StepBufs b, int fixedQ, int fp32) {
  post_charges_body(g, b, fixedQ, fp32, blockIdx.x, blockIdx.y);
}

void launch_post_charges(const Geom& g, const StepBufs& b, int fixedQ, int fp32, hipStream_t s) {
  hipLaunchKernelGGL(k_post_charges, dim3(b.R, kRsumParts), dim3(256), 0, s, g, b, fixedQ, fp32);
}

// Electrode-electrode real-space energy (the Gaussian-Gaussian term of Eq. (13)),
// 1/2 ke sum_j Q_j sum_{k != j, r < rc} Q_k [erfc(alpha r) - erfc(r / (sqrt 2 eta))] / r,
// for the energy's parts only (E* itself takes 1/2 Q^T A Q from the solve's identity).
// Block (x, r): electrodes j of [256 x, 256 x + 256) of replica r, one per thread, over
// the electrode runs of j's cell (every electrode within rc of the cell), minimum image
// in x, y, FP64 throughout.  Each block leaves its sum (fixed tree order) in epair.
__global__ __launch_bounds__(256) void k_ele_pair_energy(Geom g, StepBufs b) {
  __shared__ double sh[1][4];
  const int r = blockIdx.y, n = g.n_ele;
  const int j = blockIdx.x * 256 + threadIdx.x;
  double v[1] = {0.0};
  if (j < n) {
    const double* __restrict__ X = b.ele_xyz;
    const double* __restrict__ Q = b.Q_out + (size_t)r * n;
    const double xj = X[j], yj = X[n + j], zj = X[2 * n + j];
    const int c = b.ele_scell[b.ele_iperm[j]];
    const double a = g.alpha, bg = 1.0 / (sqrt(2.0) * g.eta), rc2 = g.rc * g.rc;
    double t = 0.0;
    for (int u = 0; u < kRunMax; ++u) {
      const int4 run = b.ele_rr[(size_t)kRunMax * c + u];
      if (run.x < 0) break;
      for (int e = run.x; e < run.y; ++e) {
        const int k = b.ele_perm[e];
        if (k == j) continue;
        double dx = xj - X[k], dy = yj - X[n + k];
        const double dz = zj - X[2 * n + k];
        dx -= g.Lx * rint(dx * g.invLx);
        dy -= g.Ly * rint(dy * g.invLy);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= rc2) continue;
        const double rr = sqrt(r2);
        t += Q[k] * (erfc(a * rr) - erfc(bg * rr)) / rr;
      }
    }
    v[0] = 0.5 * g.ke * Q[j] * t;
  }
  block_sum<256, 1>(v, sh);
  if (threadIdx.x == 0) b.epair[(size_t)r * gridDim.x + blockIdx.x] = v[0];
}

void launch_ele_pair_energy(const Geom& g, const StepBufs& b, hipStream_t s) {
  if (!b.epair || g.n_ele == 0) return;
  hipLaunchKernelGGL(k_ele_pair_energy, dim3(b.epair_nb, b.R), dim3(256), 0, s, g, b);
}

// ============================================================ ion forces, reciprocal part
// F_i = -q_i sum_k k Im(coef_k exp(-i k.r_i))   (Eq. (25), coef = w (S1 + S2))
//       - (4 pi ke / V) q_i M_z e_z             (slab force, M_z = sum q z + sum Q Z)
// The real-space sums are added by the step's last launch (k_final).
template <int W>
__device__ __forceinline__ void ionforce_write(const Geom& g, int r, int64_t i, bool live, double qi, double gx,
                                               double gy, double gz, double (*sh)[3][64], const double* scal,
                                               const double* rsum, int64_t N, double* F) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  sh[w][0][lane] = gx;
  sh[w][1][lane] = gy;
  sh[w][2][lane] = gz;
  __syncthreads();
  if (w == 0 && live) {
    double gsum[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      gsum[d] = sh[0][d][lane];
#pragma unroll
      for (int u = 1; u < W; ++u) gsum[d] += sh[u][d][lane];
    }
    F[i] = -qi * gsum[0];
    F[N + i] = -qi * gsum[1];
    F[2 * N + i] = -qi * gsum[2] - (4.0 * M_PI * g.ke / g.V) * qi * (scal[4 * r + 2] + rsum_total(rsum, r, 0));
  }
}

// Block (bx, r): ions 64 bx .. 64 bx + 63 of replica r.
template <int W>
__device__ __forceinline__ void ionforce64_block(const Geom& g, const StepBufs& b, int bx, int r) {
  const int64_t* __restrict__ off = b.off;
  const double4* __restrict__ ion_d4 = b.ion_d4;
  const int64_t N = b.N;
  const int4* __restrict__ modes = b.modes;
  const double2* __restrict__ coef = b.coef;
  const double* __restrict__ scal = b.scal;
  const double* __restrict__ rsum = b.rsum;
  double* __restrict__ F = b.F_out;
  __shared__ double sh[W][3][64];
  const int64_t b0 = off[r], b1 = off[r + 1];
  const int64_t i = b0 + (int64_t)bx * 64 + (threadIdx.x & 63);
  if (b0 + (int64_t)bx * 64 >= b1) return;  // whole block past this replica's ions
  const bool live = i < b1;
  const double4 p = live ? ion_d4[i] : make_double4(0, 0, 0, 0);
  int lo, hi;
  mode_part<W>(g.K, lo, hi);
  double gx = 0.0, gy = 0.0, gz = 0.0;
  const int4* mr = modes + (size_t)r * g.K;
  const double2* cr = coef + (size_t)r * g.K;
  for (int k = lo; k < hi; ++k) {
    const int4 m = mr[k];
    double t = fma((double)m.x, p.x, fma((double)m.y, p.y, (double)m.z * p.z));
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    const double2 c = cr[k];
    const double im = fma(c.y, cs, -c.x * sn);
    gx = fma(TWO_PI * (double)m.x * g.invLx, im, gx);
    gy = fma(TWO_PI * (double)m.y * g.invLy, im, gy);
    gz = fma(TWO_PI * (double)m.z * g.invLz, im, gz);
  }
  ionforce_write<W>(g, r, i, live, p.w, gx, gy, gz, sh, scal, rsum, N, F);
}

template <int W, int U>
__device__ __forceinline__ void ionforce32_block(const Geom& g, const StepBufs& b, int bx, int r) {
  const int64_t* __restrict__ off = b.off;
  const uint4* __restrict__ ion_fx = b.ion_fx;
  const int64_t N = b.N;
  const ModeRec32* __restrict__ rec = b.rec;
  const double* __restrict__ scal = b.scal;
  const double* __restrict__ rsum = b.rsum;
  double* __restrict__ F = b.F_out;
  __shared__ double sh[W][3][64];
  const int64_t b0 = off[r], b1 = off[r + 1];
  const int64_t i = b0 + (int64_t)bx * 64 + (threadIdx.x & 63);
  if (b0 + (int64_t)bx * 64 >= b1) return;  // whole block past this replica's ions
  const bool live = i < b1;
  const uint4 pi_ = live ? ion_fx[i] : make_uint4(0, 0, 0, 0);
  int lo, hi;
  mode_part<W>(g.K, lo, hi);
  const ModeRec32* mr = rec + (size_t)r * g.K;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  // deterministic modes k = (0, 0, kz) in this part: only the z component
  {
    float az = 0.f;
    for (int k = lo; k < min(hi, g.M); ++k) {
      const ModeRec32 m = mr[k];
      const uint32_t ph = (uint32_t)m.mz * pi_.z;
      const float x = (float)(int32_t)ph * 0x1.0p-32f;
      const float im = m.cim * __builtin_amdgcn_cosf(x) - m.cre * __builtin_amdgcn_sinf(x);
      az = fmaf(m.kz, im, az);
    }
    gz += (double)az;
  }
  for (int kb = max(lo, g.M); kb < hi; kb += 64) {
    const int ke_ = min(hi, kb + 64);
    float ax = 0.f, ay = 0.f, az = 0.f;
    int k = kb;
    for (; k + U <= ke_; k += U) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const ModeRec32 m = mr[k + u];
        const uint32_t ph = (uint32_t)m.mx * pi_.x + (uint32_t)m.my * pi_.y + (uint32_t)m.mz * pi_.z;
        const float x = (float)(int32_t)ph * 0x1.0p-32f;
        const float im = m.cim * __builtin_amdgcn_cosf(x) - m.cre * __builtin_amdgcn_sinf(x);
        ax = fmaf(m.kx, im, ax);
        ay = fmaf(m.ky, im, ay);
        az = fmaf(m.kz, im, az);
      }
    }
    for (; k < ke_; ++k) {
      const ModeRec32 m = mr[k];
      const uint32_t ph = (uint32_t)m.mx * pi_.x + (uint32_t)m.my * pi_.y + (uint32_t)m.mz * pi_.z;
      const float x = (float)(int32_t)ph * 0x1.0p-32f;
      const float im = m.cim * __builtin_amdgcn_cosf(x) - m.cre * __builtin_amdgcn_sinf(x);
      ax = fmaf(m.kx, im, ax);
      ay = fmaf(m.ky, im, ay);
      az = fmaf(m.kz, im, az);
    }
    gx += (double)ax;
    gy += (double)ay;
    gz += (double)az;
  }
  ionforce_write<W>(g, r, i, live, (double)__uint_as_float(pi_.w), gx, gy, gz, sh, scal, rsum, N, F);
}


// ============================================================ ion forces, real space
// F_i += -ke q_i sum_j q_j K_ii'(r) r^ - ke q_i sum_e Q_e K_ig'(r) r^ over the
// neighbouring cells (r < rc), phi_i = ke sum_j q_j K_ii(r) (for the energy).
// A wave scans several consecutive cell-sorted ions in turn (see wave_scan), one
// ion at a time, and carries its hit ring from one ion to the next: an evaluation
// block may hold the previous ion's last entries and the current ion's first ones,
// and each lane adds a term to the previous or the current ion's sums by the
// entry's position (entries below `bound` are the previous ion's).  An ion's sums
// are final once its last entry has been evaluated.  Two kernels: the ion-ion part,
// which does not depend on the electrode charges and runs beside the k-space and
// charge-solve passes, leaves its sums in Fii (input order); the ion-electrode part,
// after the charge solve, visits only the ions of the cells that can reach an
// electrode (reach ranges built at set-up) and leaves its sums in Fie (written for
// exactly those ions); the k-space force pass then adds ke q_i (Fii + Fie) to F,
// reading Fie only for ions of reach cells.  An electrode run (one z-layer) whose
// z-extent lies farther than rc from the ion cannot hold a partner and is skipped.

// The previous and the current ion's per-lane sums (NV values each) and the ring
// position where the previous ion's entries end.
template <class T, int NV>
struct CarriedSums {
  T p[NV], c[NV];
  unsigned bound = 0;
  __device__ __forceinline__ CarriedSums() {
#pragma unroll
    for (int v = 0; v < NV; ++v) p[v] = c[v] = T(0);
  }
  // adds term[v] * mul[v] to the previous ion's sums if entry e is one of its own,
  // else to the current ion's (the other side gets an exact zero)
  __device__ __forceinline__ void add(unsigned e, const T (&term)[NV], const T (&mul)[NV]) {
    const bool prev = e < bound;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const T tp = prev ? term[v] : T(0), tc = prev ? T(0) : term[v];
      p[v] = fma(tp, mul[v], p[v]);
      c[v] = fma(tc, mul[v], c[v]);
    }
  }
  __device__ __forceinline__ void rotate(unsigned tail) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      p[v] = c[v];
      c[v] = T(0);
    }
    bound = tail;
  }
};

// Ion-ion pass, block (bx, r): waves 4 bx .. 4 bx + 3 of replica r, each taking
// bb.ii_ipw consecutive sorted ions.  lds: ring_bytes<FP32>() + kListBytes bytes.
// CULL: the home cells' candidate lists leave out the records out of reach of the
// cell (grids whose cells have several neighbour runs; the test's registers would
// cost the one-run grids a wave per SIMD).
template <bool FP32, bool CULL>
__device__ __forceinline__ void real_ii_block(const Geom& g, const StepBufs& bb, int bx, int r, void* lds) {
  const int64_t* __restrict__ off = bb.off;
  const int64_t N = bb.N;
  const int* __restrict__ cstart = bb.cstart;
  const int* __restrict__ perm = bb.perm;
  const int* __restrict__ scell = bb.scell;
  const int2* __restrict__ ion_runs = bb.ion_runs;
  const uint4* __restrict__ sfx = bb.sfx;
  const double4* __restrict__ sd4 = bb.sd4;
  double* __restrict__ Fii = bb.Fii;
  double* __restrict__ phi = bb.phi;
  using Entry = typename std::conditional<FP32, float4, double4>::type;
  using T = typename std::conditional<FP32, float, double>::type;
  const int b0 = (int)off[r], b1 = (int)off[r + 1];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ipw = bb.ii_ipw;
  const int kbeg = b0 + (bx * 4 + w) * ipw;
  if (kbeg >= b1) return;  // whole wave
  const int kend = min(b1, kbeg + ipw);
  Entry* ring = reinterpret_cast<Entry*>(lds) + w * kRingAlloc;
  uint16_t* list = reinterpret_cast<uint16_t*>(reinterpret_cast<unsigned char*>(lds) + ring_bytes<FP32>()) +
                   w * kListCap;
  const int* cs = cstart + (size_t)r * (g.ncell + 1);
  auto ion_range = [&](int, int2 rc, int& b, int& e) {
    b = b0 + cs[rc.x];
    e = b0 + cs[rc.y];
  };
  unsigned head = 0, tail = 0;
  CarriedSums<T, 4> acc;  // x, y, z force sums and the potential
  const float a1 = (float)g.alpha;
  auto eval_block = [&](unsigned e0, unsigned lim) {
    const unsigned e = e0 + lane;
    if (e >= lim) return;
    const Entry en = ring[e & (kRing - 1)];
    if constexpr (FP32) {
      const float r2 = en.x * en.x + en.y * en.y + en.z * en.z;
      const float rinv = __builtin_amdgcn_rsqf(r2), rr = r2 * rinv;
      float f, h;
      erfc_pair_f(a1, rr, rinv, f, h);
      const float s_ = en.w * h;
      acc.add(e, {s_, s_, s_, en.w}, {en.x, en.y, en.z, f});
    } else {
      const double rr = sqrt(en.x * en.x + en.y * en.y + en.z * en.z);
      double f, df;
      erfc_over_r(g.alpha, rr, f, df);
      const double s_ = -en.w * df / rr;
      acc.add(e, {s_, s_, s_, en.w}, {en.x, en.y, en.z, f});
    }
  };
  auto finish = [&](int k, const T (&a)[4]) {
    double fx, fy, fz, ph;
    if constexpr (FP32) {
      float t0, t1, t2, t3;
      wave_total4(a[0], a[1], a[2], a[3], reinterpret_cast<float*>(ring + kRing), t0, t1, t2, t3);
      fx = t0, fy = t1, fz = t2, ph = t3;
    } else {
      fx = wave_total(a[0]), fy = wave_total(a[1]), fz = wave_total(a[2]), ph = wave_total(a[3]);
    }
    if (lane == 0) {
      const int i = perm[k];
      Fii[i] = fx;
      Fii[N + i] = fy;
      Fii[2 * N + i] = fz;
      phi[i] = g.ke * ph;
    }
  };
  int home = -1, rb = 0, re = 0, ltotal = 0, lbase = 0;
  bool use_list = false;
  for (int k = kbeg; k < kend; ++k) {
    const int hk = __builtin_amdgcn_readfirstlane(scell[k]);
    if (hk != home) {
      home = hk;
      resolve_runs(ion_runs + kRunMax * home, ion_range, rb, re);
      if constexpr (!CULL) {
        use_list = build_list(rb, re, list, ltotal, lbase, [](int) { return true; });
      } else {
      // the list keeps the records within rc (with a margin) of the home cell's box
      // [c / n_d, (c + 1) / n_d) per axis (z: of the slab height H), a bound on the
      // distance of every ion of the cell; about a quarter of an rc-cell neighbourhood
      // lies farther
      const int cx = home % g.ncx, cy = (home / g.ncx) % g.ncy, cz = home / (g.ncx * g.ncy);
      const double zc = (cz + 0.5) * g.H / g.ncz * g.invLz, hz = 0.5 * g.H / g.ncz * g.invLz;
      if constexpr (FP32) {
        // fixed point: centre and half-width in units of 2^-32 of the box, the half-width
        // widened by 2^8 units for the records' rounding; lengths squared with a 1e-3 margin
        // (wave-uniform: kept in scalar registers, so the carried sums keep the vector ones)
        auto su = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
        const uint32_t Xc = su((uint32_t)((cx + 0.5) / g.ncx * 0x1.0p32)), Yc = su((uint32_t)((cy + 0.5) / g.ncy * 0x1.0p32));
        const uint32_t Zc = su((uint32_t)(zc * 0x1.0p32));
        const uint32_t Hx = su((uint32_t)(0x1.0p31 / g.ncx) + 256u), Hy = su((uint32_t)(0x1.0p31 / g.ncy) + 256u);
        const uint32_t Hz = su((uint32_t)(hz * 0x1.0p32) + 256u);
        const float lx = (float)(g.Lx * 0x1.0p-32), ly = (float)(g.Ly * 0x1.0p-32), lz = (float)(g.Lz * 0x1.0p-32);
        const float cut2 = (float)(g.rc * g.rc * 1.001);
        auto gap = [](uint32_t a, uint32_t c, uint32_t h, float l) {
          const int32_t d = (int32_t)(a - c);
          const uint32_t ad = d < 0 ? 0u - (uint32_t)d : (uint32_t)d;
          return (float)(ad > h ? ad - h : 0u) * l;
        };
        use_list = build_list(rb, re, list, ltotal, lbase, [&](int j) {
          const uint4 q = sfx[j];
          const float ex = gap(q.x, Xc, Hx, lx), ey = gap(q.y, Yc, Hy, ly), ez = gap(q.z, Zc, Hz, lz);
          return ex * ex + ey * ey + ez * ez <= cut2;
        });
      } else {
        auto sd = [](double v) {  // wave-uniform, into scalar registers
          return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                                  __builtin_amdgcn_readfirstlane(__double2loint(v)));
        };
        const double xc = sd((cx + 0.5) / g.ncx), yc = sd((cy + 0.5) / g.ncy), zcs = sd(zc);
        const double hx = sd(0.5 / g.ncx * (1.0 + 1e-9)), hy = sd(0.5 / g.ncy * (1.0 + 1e-9)), hzz = sd(hz * (1.0 + 1e-9));
        const double cut2 = g.rc * g.rc * (1.0 + 1e-9);
        use_list = build_list(rb, re, list, ltotal, lbase, [&](int j) {
          const double4 q = sd4[j];
          double dx = q.x - xc, dy = q.y - yc;
          dx -= rint(dx);
          dy -= rint(dy);
          const double ex = fmax(fabs(dx) - hx, 0.0) * g.Lx, ey = fmax(fabs(dy) - hy, 0.0) * g.Ly;
          const double ez = fmax(fabs(q.z - zcs) - hzz, 0.0) * g.Lz;
          return ex * ex + ey * ey + ez * ez <= cut2;
        });
      }
      }
    }
    if constexpr (FP32) {
      const uint4 pi_ = sfx[k];
      const float lx = (float)(g.Lx * 0x1.0p-32), ly = (float)(g.Ly * 0x1.0p-32), lz = (float)(g.Lz * 0x1.0p-32);
      // the pair test 0 < r^2 < rc^2 as one unsigned compare of the bit patterns (r^2
      // is not negative); r = 0 is the ion itself (two ions at one point have no
      // finite pair term)
      const unsigned rc2m1 = __float_as_uint((float)(g.rc * g.rc)) - 1u;
      auto load = [&](int j) { return sfx[j]; };
      auto test = [&](const uint4& p, int, float4& ent) {
        ent.x = (float)(int32_t)(pi_.x - p.x) * lx;
        ent.y = (float)(int32_t)(pi_.y - p.y) * ly;
        ent.z = (float)(int32_t)(pi_.z - p.z) * lz;
        ent.w = __uint_as_float(p.w);
        return __float_as_uint(ent.x * ent.x + ent.y * ent.y + ent.z * ent.z) - 1u < rc2m1;
      };
      if (use_list)
        wave_scan_list(list, ltotal, lbase, ring, head, tail, load, test, eval_block);
      else
        wave_scan(rb, re, ring, head, tail, load, [&](int j0) { return (sfx + j0)[lane]; }, test, eval_block);
    } else {
      const double4 pi_ = sd4[k];
      const double rc2 = g.rc * g.rc;
      auto load = [&](int j) { return sd4[j]; };
      auto test = [&](const double4& p, int j, double4& ent) {
        double sx = pi_.x - p.x, sy = pi_.y - p.y;
        sx -= rint(sx);
        sy -= rint(sy);
        ent.x = sx * g.Lx;
        ent.y = sy * g.Ly;
        ent.z = (pi_.z - p.z) * g.Lz;
        ent.w = p.w;
        return (ent.x * ent.x + ent.y * ent.y + ent.z * ent.z < rc2) & (j != k);
      };
      if (use_list)
        wave_scan_list(list, ltotal, lbase, ring, head, tail, load, test, eval_block);
      else
        wave_scan(rb, re, ring, head, tail, load, [&](int j0) { return (sd4 + j0)[lane]; }, test, eval_block);
    }
    if (k > kbeg) {  // the previous ion is complete once its last entries are evaluated
      if (head < acc.bound) {
        __builtin_amdgcn_wave_barrier();
        eval_block(head, tail);
        head = tail;
      }
      finish(k - 1, acc.p);
    }
    acc.rotate(tail);
  }
  __builtin_amdgcn_wave_barrier();
  eval_block(head, tail);
  finish(kend - 1, acc.p);
}

// Blocks are dealt to the 8 XCDs in turn by launch index (launch block L runs on XCD
// L mod 8), and each XCD has its own L2.  With 8 or more replicas, one replica's
// blocks all run on one XCD, so its records are fetched into one L2 only: block L
// takes block bx of replica r = L mod 8 + 8 m.  With fewer replicas that would leave
// XCDs idle; instead the (replica, block) items in order are cut into 8 contiguous
// ranges, one per XCD, so each L2 holds the records of a slab of consecutive cells
// (plus the stencil's reach) rather than of the whole system.  A wave's work depends
// only on (r, bx), so the mapping does not change results.
template <bool FP32, bool CULL>
__device__ __forceinline__ void real_ii_body(const Geom& g, const StepBufs& b, int tiles, int L) {
  __shared__ __align__(16) unsigned char lds[ring_bytes<FP32>() + kListBytes];
  const int j = L >> 3;
  int r, bx;
  if (b.R >= 8) {
    const int m = j / tiles;
    r = (L & 7) + 8 * m;
    bx = j - m * tiles;
  } else {
    const int items = b.R * tiles, per = (items + 7) >> 3;
    const int item = (L & 7) * per + j;
    if (item >= items) return;
    r = item / tiles;
    bx = item - r * tiles;
  }
  if (r >= b.R) return;
  real_ii_block<FP32, CULL>(g, b, bx, r, lds);
}

// (8 waves per SIMD in FP32, 3 in FP64: the culling variant spills a few registers
// rather than give up a wave)
template <bool FP32, bool CULL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FP32 ? 8 : 3))) void k_real_ii(Geom g, StepBufs b,
                                                                                                     int tiles) {
  real_ii_body<FP32, CULL>(g, b, tiles, blockIdx.x);
}

static int real_ii_tiles(const StepBufs& b) { return cdiv64(std::max(b.max_nrep, 1), 4 * b.ii_ipw); }

// Partial sums of q_i phi_i over tiles of kEnergyTile ions of each replica (large
// replicas), so the energy's ion sum is spread over many CUs: block (r, t).
__device__ __forceinline__ void energy_partials_body(const StepBufs& b, int lb) {
  __shared__ double sh[1][4];
  const int r = lb / b.etiles, t = lb - r * b.etiles;
  const int64_t i0 = b.off[r] + (int64_t)t * kEnergyTile, i1 = min(b.off[r + 1], i0 + kEnergyTile);
  double v[1] = {0.0};
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) v[0] += b.ion_q[i] * b.phi[i];
  block_sum<256, 1>(v, sh);
  if (threadIdx.x == 0) b.eparts[(size_t)r * b.etiles + t] = v[0];
}

__global__ __launch_bounds__(256) void k_energy_partials(StepBufs b) { energy_partials_body(b, blockIdx.x); }

void launch_real_ii(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  if (b.max_nrep == 0) return;
  const int tiles = real_ii_tiles(b);
  const dim3 grid(b.R >= 8 ? 8 * ((b.R + 7) / 8) * tiles : 8 * ((b.R * tiles + 7) / 8));
  const bool cull = g.ncx > 3 || g.ncy > 3;  // else every cell's neighbours are one run: no lists
  if (fp32 && cull)
    hipLaunchKernelGGL((k_real_ii<true, true>), grid, dim3(256), 0, s, g, b, tiles);
  else if (fp32)
    hipLaunchKernelGGL((k_real_ii<true, false>), grid, dim3(256), 0, s, g, b, tiles);
  else if (cull)
    hipLaunchKernelGGL((k_real_ii<false, true>), grid, dim3(256), 0, s, g, b, tiles);
  else
    hipLaunchKernelGGL((k_real_ii<false, false>), grid, dim3(256), 0, s, g, b, tiles);
  if (b.etiles) hipLaunchKernelGGL(k_energy_partials, dim3((unsigned)b.R * b.etiles), dim3(256), 0, s, b);
}

// Block bx of the nbx blocks that one replica's reach ranges are split over; the
// block's waves take the replica's ions in turn, one ion per visit.  The pass is
// latency-bound, so each wave loads the next ion's cell and record while it scans the
// current one, and an ion's electrode runs come from a set-up table of sorted ranges
// with their z-extent (one 16-byte load per run, all runs at once).  A run whose
// z-extent lies farther than rc from the ion cannot hold a partner and is skipped
// (the extent is stored in FP32; the margin below covers its rounding).
template <bool FP32>
__device__ __forceinline__ void real_ie_block(const Geom& g, const StepBufs& bb, int bx, int nbx, int r) {
  const int64_t* __restrict__ off = bb.off;
  const int64_t N = bb.N;
  const int* __restrict__ cstart = bb.cstart;
  const int2* __restrict__ reach = bb.reach;
  const int nreach = bb.nreach;
  const int* __restrict__ perm = bb.perm;
  const int* __restrict__ scell = bb.scell;
  const int4* __restrict__ ele_rr = bb.ele_rr;
  const uint4* __restrict__ sfx = bb.sfx;
  const double4* __restrict__ sd4 = bb.sd4;
  const uint4* __restrict__ ele_sfx = bb.ele_sfx;
  const double4* __restrict__ ele_sd4 = bb.ele_sd4;
  const float* __restrict__ Qsf = bb.Qsf;
  const double* __restrict__ Qsd = bb.Qsd;
  double* __restrict__ Fie = bb.Fie;
  using Entry = typename std::conditional<FP32, float4, double4>::type;
  using T = typename std::conditional<FP32, float, double>::type;
  using Rec = typename std::conditional<FP32, uint4, double4>::type;
  __shared__ Entry ring_all[4][kRingAlloc];
  const int b0 = (int)off[r];
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int gw = bx * 4 + w, stride = nbx * 4, first = gw;
  Entry* ring = ring_all[w];
  const int* cs = cstart + (size_t)r * (g.ncell + 1);
  const int n = g.n_ele;
  const double zlim = g.rc + 1e-5;  // skip margin: FP32 z-extents (~1e-6 nm) and fixed-point z (~1e-8 of the box)
  const float a1 = (float)g.alpha, a2 = (float)(1.0 / g.eta);
  unsigned head = 0, tail = 0;
  CarriedSums<T, 3> acc;
  auto eval_block = [&](unsigned e0, unsigned lim) {
    const unsigned e = e0 + lane;
    if (e >= lim) return;
    const Entry en = ring[e & (kRing - 1)];
    if constexpr (FP32) {
      const float r2 = en.x * en.x + en.y * en.y + en.z * en.z;
      const float rinv = __builtin_amdgcn_rsqf(r2), rr = r2 * rinv;
      float f1, h1, f2, h2 = 0.f;
      erfc_pair_f(a1, rr, rinv, f1, h1);
      if (rr < g.eta_skip) erfc_pair_f(a2, rr, rinv, f2, h2);
      const float s_ = en.w * (h1 - h2);
      acc.add(e, {s_, s_, s_}, {en.x, en.y, en.z});
    } else {
      const double rr = sqrt(en.x * en.x + en.y * en.y + en.z * en.z);
      double f1, d1, f2, d2;
      erfc_over_r(g.alpha, rr, f1, d1);
      erfc_over_r(1.0 / g.eta, rr, f2, d2);
      const double s_ = -en.w * (d1 - d2) / rr;
      acc.add(e, {s_, s_, s_}, {en.x, en.y, en.z});
    }
  };
  auto finish = [&](int k, const T (&a)[3]) {
    double fx, fy, fz;
    if constexpr (FP32) {
      float t0, t1, t2, t3;
      wave_total4(a[0], a[1], a[2], 0.f, reinterpret_cast<float*>(ring + kRing), t0, t1, t2, t3);
      fx = t0, fy = t1, fz = t2;
    } else {
      fx = wave_total(a[0]), fy = wave_total(a[1]), fz = wave_total(a[2]);
    }
    if (lane == 0) {
      const int i = perm[k];
      Fie[i] = fx;
      Fie[N + i] = fy;
      Fie[2 * N + i] = fz;
    }
  };
  // the wave's ions: positions first, first + stride, ... of each reach range in turn
  int qr = -1, k = 0, kstop = 0;
  auto advance = [&]() {
    k += stride;
    while (k >= kstop) {
      if (++qr >= nreach) return false;
      const int2 cr = reach[qr];
      k = b0 + cs[cr.x] + first;
      kstop = b0 + cs[cr.y];
    }
    return true;
  };
  k = -stride;  // so that the first advance lands on the first ion
  bool have = advance();
  int home = 0;
  Rec pi_{};
  if (have) {
    home = __builtin_amdgcn_readfirstlane(scell[k]);
    if constexpr (FP32) pi_ = sfx[k]; else pi_ = sd4[k];
  }
  int kprev = -1;
  while (have) {
    const int kc = k;
    const int hc = home;
    const Rec pc = pi_;
    have = advance();
    if (have) {  // the next ion's cell and record travel while this one is scanned
      home = __builtin_amdgcn_readfirstlane(scell[k]);
      if constexpr (FP32) pi_ = sfx[k]; else pi_ = sd4[k];
    }
    int rb = 0, re = 0;
    {
      const int4 t = lane < kRunMax ? ele_rr[kRunMax * hc + lane] : make_int4(-1, -1, 0, 0);
      const uint64_t term = __ballot(t.x < 0);  // non-zero: the lanes >= kRunMax count as terminators
      const uint64_t listed = (1ull << __builtin_ctzll(term)) - 1;
      double zi;
      if constexpr (FP32) zi = (double)pc.z * (g.Lz * 0x1.0p-32); else zi = pc.z * g.Lz;
      if ((listed >> lane) & 1) {
        const double zlo = (double)__int_as_float(t.z), zhi = (double)__int_as_float(t.w);
        rb = t.x;
        re = (zlo - zi >= zlim || zi - zhi >= zlim) ? t.x : t.y;
      }
    }
    if constexpr (FP32) {
      const float lx = (float)(g.Lx * 0x1.0p-32), ly = (float)(g.Ly * 0x1.0p-32), lz = (float)(g.Lz * 0x1.0p-32),
                  rc2 = (float)(g.rc * g.rc);
      const float* Qr = Qsf + (size_t)r * n;
      wave_scan(rb, re, ring, head, tail,
                [&](int j) {
                  uint4 p = ele_sfx[j];
                  p.w = __float_as_uint(Qr[j]);
                  return p;
                },
                [&](int j0) {
                  uint4 p = (ele_sfx + j0)[lane];
                  p.w = __float_as_uint((Qr + j0)[lane]);
                  return p;
                },
                [&](const uint4& p, int, float4& ent) {
                  ent.x = (float)(int32_t)(pc.x - p.x) * lx;
                  ent.y = (float)(int32_t)(pc.y - p.y) * ly;
                  ent.z = (float)(int32_t)(pc.z - p.z) * lz;
                  ent.w = __uint_as_float(p.w);
                  return ent.x * ent.x + ent.y * ent.y + ent.z * ent.z < rc2;
                },
                eval_block);
    } else {
      const double rc2 = g.rc * g.rc;
      const double* Qr = Qsd + (size_t)r * n;
      wave_scan(rb, re, ring, head, tail,
                [&](int j) {
                  double4 p = ele_sd4[j];
                  p.w = Qr[j];
                  return p;
                },
                [&](int j0) {
                  double4 p = (ele_sd4 + j0)[lane];
                  p.w = (Qr + j0)[lane];
                  return p;
                },
                [&](const double4& p, int, double4& ent) {
                  double sx = pc.x - p.x, sy = pc.y - p.y;
                  sx -= rint(sx);
                  sy -= rint(sy);
                  ent.x = sx * g.Lx;
                  ent.y = sy * g.Ly;
                  ent.z = (pc.z - p.z) * g.Lz;
                  ent.w = p.w;
                  return ent.x * ent.x + ent.y * ent.y + ent.z * ent.z < rc2;
                },
                eval_block);
    }
    if (kprev >= 0) {  // the previous ion is complete once its last entries are evaluated
      if (head < acc.bound) {
        __builtin_amdgcn_wave_barrier();
        eval_block(head, tail);
        head = tail;
      }
      finish(kprev, acc.p);
    }
    acc.rotate(tail);
    kprev = kc;
  }
  if (kprev >= 0) {
    __builtin_amdgcn_wave_barrier();
    eval_block(head, tail);
    finish(kprev, acc.p);
  }
}

// The ion-electrode real-space pass needs the new charges and is latency-bound; it
// shares its kernel with the electrode structure-factor partials:
//   k_stage_ele: [real_ie | electrode structure-factor partial blocks]
// The real-space blocks (b.ie_nbx per replica walking its reach ranges) come first in
// the grid: being latency-bound they start their chains at once, and the
// arithmetic-bound blocks fill the issue slots they leave.
template <bool FP32>
__device__ __forceinline__ void stage_ele_body(const Geom& g, const StepBufs& b, int nsf, int nie, int bid) {
  if (bid < nie)
    real_ie_block<FP32>(g, b, bid % b.ie_nbx, b.ie_nbx, bid / b.ie_nbx);
  else
    sf_block<FP32, false>(g, b, bid - nie);
}

template <bool FP32>
__global__ __launch_bounds__(256) void k_stage_ele(Geom g, StepBufs b, int nsf, int nie) {
  stage_ele_body<FP32>(g, b, nsf, nie, blockIdx.x);
}

template <bool FP32, int W, int U>
__device__ __forceinline__ void ion_force_body(const Geom& g, const StepBufs& b, int ftiles, int u) {
  if constexpr (FP32)
    ionforce32_block<W, U>(g, b, u % ftiles, u / ftiles);
  else
    ionforce64_block<W>(g, b, u % ftiles, u / ftiles);
}

template <bool FP32, int W, int U>
__global__ __launch_bounds__(64 * W) void k_ion_force(Geom g, StepBufs b, int ftiles) {
  ion_force_body<FP32, W, U>(g, b, ftiles, blockIdx.x);
}

void launch_stage_ele(const Geom& g, const StepBufs& b, int fp32, int parts, hipStream_t s) {
  const int nsf = (parts & STAGE_SF && g.K > 0) ? b.ktiles * b.nchunk_ele * b.R : 0;
  const int nie = (parts & STAGE_REAL && b.max_nrep > 0 && b.nreach > 0) ? b.ie_nbx * b.R : 0;
  if (nsf + nie == 0) return;
  if (fp32)
    hipLaunchKernelGGL(k_stage_ele<true>, dim3(nsf + nie), dim3(256), 0, s, g, b, nsf, nie);
  else
    hipLaunchKernelGGL(k_stage_ele<false>, dim3(nsf + nie), dim3(256), 0, s, g, b, nsf, nie);
}

void launch_ion_force(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  if (b.max_nrep == 0) return;
  const int ftiles = cdiv64(b.max_nrep, 64);
  with_wu(b.kw, fp32 ? b.unroll : 4, [&](auto W, auto U) {
    constexpr int w = decltype(W)::value, u = decltype(U)::value;
    if (fp32)
      hipLaunchKernelGGL((k_ion_force<true, w, u>), dim3(ftiles * b.R), dim3(64 * w), 0, s, g, b, ftiles);
    else if constexpr (u == 4)  // the FP64 loop has no unroll parameter
      hipLaunchKernelGGL((k_ion_force<false, w, 4>), dim3(ftiles * b.R), dim3(64 * w), 0, s, g, b, ftiles);
  });
}

// z-extent (min, max of Z) of the electrodes of every cell; empty cells get an
// empty interval.
__global__ __launch_bounds__(256) void k_cell_zrange(Geom g, const int* __restrict__ cstart,
                                                     const double* __restrict__ ele_xyz,
                                                     const int* __restrict__ perm, double2* __restrict__ zr) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= g.ncell) return;
  double lo = INFINITY, hi = -INFINITY;
  for (int k = cstart[c]; k < cstart[c + 1]; ++k) {
    const double z = ele_xyz[2 * g.n_ele + perm[k]];
    lo = fmin(lo, z);
    hi = fmax(hi, z);
  }
  zr[c] = make_double2(lo, hi);
}

void launch_cell_zrange(const Geom& g, const int* cstart, const double* ele_xyz, const int* perm, double2* zr,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_cell_zrange, dim3(cdiv64(g.ncell, 256)), dim3(256), 0, s, g, cstart, ele_xyz, perm, zr);
}

// ============================================================ energy
// E* = 1/2 dpsi d.Q - 1/2 b*.Q + c*,  c* = 1/2 sum_i q_i phi_i + 1/2 sum_k w_k |S1_k|^2
//      - ke alpha/sqrt(pi) sum q^2 + ke (2 pi / V) (sum q z)^2
// (1/2 Q^T A Q - b*^T Q + c* at the constrained charges, where Q^T A Q = b*.Q + dpsi d.Q).
// Its parts (estride 5), as U_c is split in Eqs. (13), (16), (17):
//   real  = 1/2 q.phi + Q.bN + (electrode-electrode real space, epair)
//   self  = ke [(1/(sqrt(2 pi) eta) - alpha/sqrt(pi)) sum Q^2 - alpha/sqrt(pi) sum q^2]
//   slab  = ke (2 pi / V) (sum q z + sum Q Z)^2
//   fourier = E* - real - self - slab (the only part the sample changes).
__device__ __forceinline__ void energy_block(const Geom& g, int r, const StepBufs& b, int fixedQ) {
  __shared__ double sh[3][4];
  const int64_t* __restrict__ off = b.off;
  const double* __restrict__ ion_q = b.ion_q;
  const double* __restrict__ phi = b.phi;
  const double* __restrict__ scal = b.scal;
  const double* __restrict__ rsum = b.rsum;
  double v[3] = {0.0, 0.0, 0.0};
  const int es = b.estride;
  if (fixedQ) {  // no energy without the charge solve: nothing to sum
    if (threadIdx.x < es) b.energy_out[(size_t)es * r + threadIdx.x] = (double)NAN;
    return;
  }
  if (b.real) {  // the ion-ion real-space energy (left out in k-space-only steps)
    if (b.etiles) {  // large replicas: the tiles' partial sums, in tile order
      for (int t = threadIdx.x; t < b.etiles; t += 256) v[0] += b.eparts[(size_t)r * b.etiles + t];
    } else {
#pragma unroll 8
      for (int64_t i = off[r] + threadIdx.x; i < off[r + 1]; i += 256) v[0] += ion_q[i] * phi[i];
    }
  }
  for (int k = threadIdx.x; k < g.K; k += 256) {
    const double2 s = b.S1[(size_t)r * g.K + k];
    v[1] += b.w[(size_t)r * g.K + k] * (s.x * s.x + s.y * s.y);
  }
  if (b.epair)
    for (int t = threadIdx.x; t < b.epair_nb; t += 256) v[2] += b.epair[(size_t)r * b.epair_nb + t];
  block_sum<256, 3>(v, sh);
  if (threadIdx.x == 0) {
    const double self_i = -g.ke * g.alpha * INV_SQRT_PI * scal[4 * r + 3];
    const double c = 0.5 * v[0] + 0.5 * v[1] + self_i + g.ke * (2.0 * M_PI / g.V) * scal[4 * r + 2] * scal[4 * r + 2];
    const double E = 0.5 * b.dpsi[r] * rsum_total(rsum, r, 1) - 0.5 * rsum_total(rsum, r, 2) + c;
    if (!isfinite(E)) atomicOr(b.status, ST_NUMERIC);
    double* out = b.energy_out + (size_t)es * r;
    out[0] = E;
    if (es == 5) {
      const double real = b.real ? 0.5 * v[0] + rsum_total(rsum, r, 4) + v[2] : 0.0;
      const double cg = 1.0 / (sqrt(2.0 * M_PI) * g.eta) - g.alpha * INV_SQRT_PI;
      const double self = g.ke * cg * rsum_total(rsum, r, 3) + self_i;
      const double Mz = scal[4 * r + 2] + rsum_total(rsum, r, 0);
      const double slab = g.ke * (2.0 * M_PI / g.V) * Mz * Mz;
      out[1] = real;
      out[2] = E - real - self - slab;
      out[3] = self;
      out[4] = slab;
    }
  }
}

// The step's last launch, after every pass: blocks [0, ne) assemble E* per replica,
// blocks [ne, ne + nf) add the real-space sums to the forces,
//   F_i += ke q_i (Fii_i + Fie_i)   (Fie only for ions of reach cells),
// and block 0 advances a replayed graph's step counter.
// (a multi-system launch passes the index of the ion's first entry, ion0, of the system,
// whose ions are [ion0, ion0 + nion); a single system has ion0 = 0 and nion = N)
__device__ __forceinline__ void final_body(const Geom& g, const StepBufs& b, int ne, int fixedQ, int64_t ion0,
                                           int64_t nion, int lb) {
  if ((int)lb < ne) {
    energy_block(g, lb, b, fixedQ);
    return;
  }
  const int64_t N = b.N;
  const int64_t i = ion0 + (int64_t)(lb - ne) * 256 + threadIdx.x;
  if (i >= ion0 + nion) return;
  if (!b.real || i >= N) return;
  const double kq = g.ke * b.ion_q[i];
  double rx = b.Fii[i], ry = b.Fii[N + i], rz = b.Fii[2 * N + i];
  // Fie is read for every ion (in bounds; stale for ions outside the reach cells) so
  // that its loads do not wait for the flag, which then selects it
  const double ex = b.Fie[i], ey = b.Fie[N + i], ez = b.Fie[2 * N + i];
  // the ion's cell: the multi-block sort keeps it as the key, the one-block sort in
  // the key's high bits
  const unsigned key = b.keys[i];
  if (b.reach_cell[b.bigsort.count ? key : key >> 13]) {
    rx += ex;
    ry += ey;
    rz += ez;
  }
  double* F = b.F_out;
  F[i] += kq * rx;
  F[N + i] += kq * ry;
  F[2 * N + i] += kq * rz;
}

__global__ __launch_bounds__(256) void k_final(Geom g, StepBufs b, int ne, int fixedQ) {
  if (b.step_adv && blockIdx.x == 0 && threadIdx.x == 0) *b.step_adv += 1;
  final_body(g, b, ne, fixedQ, 0, b.N, blockIdx.x);
}

// ============================================================ multi-system launches
// One launch per phase for every system of a batch (MultiLaunch in kernels.h): each block
// finds its system, then runs that system's block of the phase with the system's Geom
// and StepBufs (read from the descriptor table) exactly as the single-system kernel would.
template <int PH, int V1, int W>
constexpr int multi_threads() {
  return (PH == MP_FRONT || PH == MP_BS_SCAN_CHUNKS || PH == MP_BS_SCAN_TOTALS || PH == MP_BS_SCAN_OFFSETS) ? 1024
         : (PH == MP_ELEPOT || PH == MP_ION_FORCE)                                                         ? 64 * W
                                                                                                           : 256;
}

// PH: the phase; V1: FP32 (1) or FP64 (0) path (the front and sort phases: record kind
// REC = 1 or 2); W, U: waves and unroll of the potential and force passes; KB: GEMM block.
template <int PH, int V1, int W, int U, int KB>
__global__ __launch_bounds__((multi_threads<PH, V1, W>())) void k_multi(MultiLaunch m) {
  const int s = multi_system(m, blockIdx.x), lb = blockIdx.x - m.start[s];
  const Geom& g = m.d[s].g;
  const StepBufs& b = m.d[s].b;
  const int* ia = m.iarg + (size_t)kMultiArgs * s;
  constexpr bool FP32 = V1 == 1;
  if constexpr (PH == MP_FRONT) {
    front_body<V1>(g, b, ion_sort_args(b), ia[0], lb);
  } else if constexpr (PH == MP_BS_ZERO) {
    const int64_t i = (int64_t)lb * 256 + threadIdx.x;
    if (i < (int64_t)b.R * (g.ncell + 1)) b.bigsort.count[i] = 0;
  } else if constexpr (PH == MP_BS_COUNT) {
    bigsort_count_body<V1>(g, ion_sort_args(b), b.bigsort, lb);
  } else if constexpr (PH == MP_BS_SCAN_CHUNKS) {
    bigsort_scan_chunks_body(g, ion_sort_args(b), b.bigsort, lb);
  } else if constexpr (PH == MP_BS_SCAN_TOTALS) {
    bigsort_scan_totals_body<V1>(g, ion_sort_args(b), b.bigsort, lb);
  } else if constexpr (PH == MP_BS_SCAN_OFFSETS) {
    bigsort_scan_offsets_body(g, ion_sort_args(b), b.bigsort, lb);
  } else if constexpr (PH == MP_BS_SCATTER) {
    bigsort_scatter_body<V1>(g, ion_sort_args(b), b.bigsort, lb);
  } else if constexpr (PH == MP_BS_RANK) {
    bigsort_rank_body<V1>(g, ion_sort_args(b), b.bigsort, lb);
  } else if constexpr (PH == MP_STAGE_IONS) {
    stage_ions_body<FP32>(g, b, ia[0], ia[1], ia[2], lb);
  } else if constexpr (PH == MP_SF_FINALIZE) {
    sf_finalize_body(g, b, ia[0], lb);
  } else if constexpr (PH == MP_ELEPOT) {
    if constexpr (FP32)
      elepot32_body<W, U>(g, b, lb % ia[0], lb / ia[0]);
    else
      elepot64_body<W>(g, b, lb % ia[0], lb / ia[0]);
  } else if constexpr (PH == MP_CP_GEMM) {
    __shared__ __align__(16) unsigned char lds[gemm_lds_bytes<KB>()];
    cp_gemm_tile<KB>(g.n_ele, b.R, b.Sext, b.V, b.Qext, lb % ia[0], (lb / ia[0]) % ia[1], lb / (ia[0] * ia[1]),
                     b.ksplit, lds);
  } else if constexpr (PH == MP_POST_CHARGES) {
    post_charges_body(g, b, ia[0], V1, lb % b.R, lb / b.R);
  } else if constexpr (PH == MP_STAGE_ELE) {
    stage_ele_body<FP32>(g, b, ia[0], ia[1], lb);
  } else if constexpr (PH == MP_ION_FORCE) {
    ion_force_body<FP32, W, U>(g, b, ia[0], lb);
  } else if constexpr (PH == MP_REAL_II) {
    real_ii_body<FP32, true>(g, b, ia[0], lb);
  } else if constexpr (PH == MP_ENERGY_PARTS) {
    energy_partials_body(b, lb);
  } else if constexpr (PH == MP_FINAL) {
    if (m.step_adv && blockIdx.x == 0 && threadIdx.x == 0) *m.step_adv += 1;
    final_body(g, b, ia[0], ia[1], ia[2], ia[3], lb);
  }
}

template <bool FP32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_multi_real_ii(MultiLaunch m) {
  const int s = multi_system(m, blockIdx.x);
  const Geom g = m.d[s].g;  // copies: only the fields the pass reads are loaded
  const StepBufs b = m.d[s].b;
  real_ii_body<FP32, true>(g, b, m.iarg[(size_t)kMultiArgs * s], blockIdx.x - m.start[s]);
}

template <int PH, int V1, int W, int U, int KB>
static void multi_go(const MultiLaunch& m, int nblocks, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((k_multi<PH, V1, W, U, KB>), dim3(nblocks), dim3(multi_threads<PH, V1, W>()), lds, s, m);
}

// phases whose kernel depends only on the path: v = 1 is the FP32 path (record kind 1),
// v = 0 the FP64 path (record kind 2 for the front and sort phases)
template <int PH>
static void multi_v(int v, const MultiLaunch& m, int nblocks, size_t lds, hipStream_t s) {
  constexpr int kFp64 = PH <= MP_BS_RANK ? 2 : 0;
  if (v == 1)
    multi_go<PH, 1, 4, 4, 16>(m, nblocks, lds, s);
  else
    multi_go<PH, kFp64, 4, 4, 16>(m, nblocks, lds, s);
}

void launch_multi(int phase, int fp32, int W, int U, int KB, const MultiLaunch& m, int nblocks, size_t lds,
                  hipStream_t s) {
  if (nblocks == 0) return;
  switch (phase) {
    case MP_FRONT: multi_v<MP_FRONT>(fp32, m, nblocks, lds, s); break;
    case MP_BS_ZERO: multi_go<MP_BS_ZERO, 1, 4, 4, 16>(m, nblocks, lds, s); break;
    case MP_BS_COUNT: multi_v<MP_BS_COUNT>(fp32, m, nblocks, lds, s); break;
    case MP_BS_SCAN_CHUNKS: multi_go<MP_BS_SCAN_CHUNKS, 1, 4, 4, 16>(m, nblocks, lds, s); break;
    case MP_BS_SCAN_TOTALS: multi_v<MP_BS_SCAN_TOTALS>(fp32, m, nblocks, lds, s); break;
    case MP_BS_SCAN_OFFSETS: multi_go<MP_BS_SCAN_OFFSETS, 1, 4, 4, 16>(m, nblocks, lds, s); break;
    case MP_BS_SCATTER: multi_v<MP_BS_SCATTER>(fp32, m, nblocks, lds, s); break;
    case MP_BS_RANK: multi_v<MP_BS_RANK>(fp32, m, nblocks, lds, s); break;
    case MP_STAGE_IONS: multi_v<MP_STAGE_IONS>(fp32, m, nblocks, lds, s); break;
    case MP_SF_FINALIZE: multi_go<MP_SF_FINALIZE, 1, 4, 4, 16>(m, nblocks, lds, s); break;
    case MP_ELEPOT:
    case MP_ION_FORCE:
      with_wu(W, fp32 ? U : 4, [&](auto Wc, auto Uc) {
        constexpr int w = decltype(Wc)::value, u = decltype(Uc)::value;
        if (phase == MP_ELEPOT) {
          if (fp32) multi_go<MP_ELEPOT, 1, w, u, 16>(m, nblocks, lds, s);
          else if constexpr (u == 4) multi_go<MP_ELEPOT, 0, w, 4, 16>(m, nblocks, lds, s);
        } else {
          if (fp32) multi_go<MP_ION_FORCE, 1, w, u, 16>(m, nblocks, lds, s);
          else if constexpr (u == 4) multi_go<MP_ION_FORCE, 0, w, 4, 16>(m, nblocks, lds, s);
        }
      });
      break;
    case MP_CP_GEMM:
      if (KB == 32) multi_go<MP_CP_GEMM, 1, 4, 4, 32>(m, nblocks, lds, s);
      else multi_go<MP_CP_GEMM, 1, 4, 4, 16>(m, nblocks, lds, s);
      break;
    case MP_POST_CHARGES: multi_v<MP_POST_CHARGES>(fp32, m, nblocks, lds, s); break;
    case MP_STAGE_ELE: multi_v<MP_STAGE_ELE>(fp32, m, nblocks, lds, s); break;
    case MP_REAL_II:
      // a kernel of its own: the FP64 pass then gets the registers of the single-system one
      if (fp32)
        hipLaunchKernelGGL(k_multi_real_ii<true>, dim3(nblocks), dim3(256), lds, s, m);
      else
        hipLaunchKernelGGL(k_multi_real_ii<false>, dim3(nblocks), dim3(256), lds, s, m);
      break;
    case MP_ENERGY_PARTS: multi_go<MP_ENERGY_PARTS, 1, 4, 4, 16>(m, nblocks, lds, s); break;
    case MP_FINAL: multi_go<MP_FINAL, 1, 4, 4, 16>(m, nblocks, lds, s); break;
    default: break;
  }
}

void launch_final(const Geom& g, const StepBufs& b, int fixedQ, hipStream_t s) {
  const int ne = b.energy_out ? b.R : 0;
  int nf = b.real ? cdiv64(b.N, 256) : 0;
  if (ne + nf == 0 && b.step_adv) nf = 1;  // a replayed graph's step counter still advances
  if (ne + nf == 0) return;
  hipLaunchKernelGGL(k_final, dim3(ne + nf), dim3(256), 0, s, g, b, ne, fixedQ);
}

}  // namespace srbe
