// Device-side helpers shared by the SRBE kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srbe {

// Device status bits (OR-ed into a per-handle word, read by srbe_sync_status).
enum : unsigned {
  ST_NONNEUTRAL = 1u,  // a replica's ion charges do not sum to zero
  ST_RANGE = 2u,       // z outside [0, H] or a non-finite coordinate/charge
  ST_NUMERIC = 4u,     // non-finite value produced
  ST_BADKSET = 8u,     // a caller-given mode lies in I or is the origin
};

// Per-handle constants, passed by value to every kernel.
struct Geom {
  double Lx, Ly, H, Lz, V;
  double invLx, invLy, invLz;
  double alpha, eta, rc, ke;
  double G;        // normaliser of Eq. (27)
  double sig[3];   // proposal standard deviation per axis (in units of m)
  int qmax[3];     // log q_d(m) is tabulated for |m| <= qmax[d]
  int M, P, K;     // K = M + P modes per replica
  int iid;         // 1: the sample is drawn i.i.d. by rejection instead of by the Metropolis chain
  int n_ele;
  // real-space cell grid: ncx x ncy cells over the periodic x, y extent, ncz over
  // z in [0, H]; cells are wider than rc in x, y and than rc / nzs in z, so all pairs
  // closer than rc lie within one cell in x, y and nzs cells in z of each other
  int ncx, ncy, ncz, ncell;
  int nzs;          // the z-stencil reaches nzs cells up and down (cells are >= rc / nzs thick)
  float eta_skip;   // FP32 path: beyond this distance erfc(r/eta)/r and its derivative are below
                    // 2^-30 of the alpha terms at rc and are not evaluated
};

// Leading dimension of the charge-solve operands (S_ext rows, right-hand sides):
// n rounded up to a multiple of 32 doubles (the GEMM's widest contraction block),
// the padding held at zero.
__host__ __device__ inline int ldcp(int n) { return (n + 31) & ~31; }

constexpr int kMaxBinParticles = 8192;  // particles per replica the one-block cell sort handles
constexpr int kMaxCells = 2048;         // cells the one-block cell sort handles
constexpr int kMaxGridCells = 1 << 18;  // cells of the real-space grid (coarsened beyond)
static_assert((kMaxGridCells + 1024) / 1024 <= 1024, "the sort scans the chunk totals in one block round");
// Neighbour runs per cell: the cells within reach of a cell, sorted, as runs of
// consecutive cell indices (whose particles are adjacent in the cell-sorted order).
// At most 7 z-layers (nzs <= 3) x 3 rows x 2 pieces (a periodic wrap splits a row).
constexpr int kRunMax = 42;
// Entries past the end of every record array that the neighbour scan reads (its
// full rounds request the records of up to three rounds ahead, which may reach 191
// entries past the run's end; the values read there are never used).  Such arrays
// are allocated with this many extra entries.
constexpr int kScanPad = 192;
// Per-replica sums after the charge solve (slot 0: sum Q Z, 1: sum Q d, 2: sum Q b*,
// 3: sum Q^2, 4: sum Q bN) are kept as kRsumParts partial sums, one per block of the
// pass that writes them, at rsum[r kRsumStride + kRsumSlots part + slot], and always
// added in part order.
// Resident waves per SIMD of the real-space passes (their register use allows this
// many; the grids are sized from it).
constexpr int kRealWavesPerSimd32 = 7;
constexpr int kRealWavesPerSimd64 = 3;
constexpr int kRsumParts = 16;
// Most k-ranges the charge-solve GEMM may be split into (the copy-out adds at most
// this many partials, all requested at once).
constexpr int kMaxGemmSplit = 16;
constexpr int kRsumSlots = 8;
constexpr int kRsumStride = kRsumSlots * kRsumParts;
// Replicas above kEnergyLarge ions have the energy's ion sum q phi taken in partial
// sums over tiles of kEnergyTile ions by many blocks (added in tile order).
constexpr int kEnergyLarge = 8192;
constexpr int kEnergyTile = 4096;

// Cell of a position (x, y wrapped by the caller into fractions sx, sy in [0,1)).
__device__ __forceinline__ int cell_index(const Geom& g, double sx, double sy, double z) {
  int cx = (int)(sx * g.ncx);
  int cy = (int)(sy * g.ncy);
  int cz = (int)(z / g.H * g.ncz);
  cx = cx < 0 ? 0 : (cx >= g.ncx ? g.ncx - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= g.ncy ? g.ncy - 1 : cy);
  cz = cz < 0 ? 0 : (cz >= g.ncz ? g.ncz - 1 : cz);
  return (cz * g.ncy + cy) * g.ncx + cx;
}

// ------------------------------------------------------------------ Philox4x64-10
// Salmon, Moraes, Dror, Shaw, SC'11: per round two 64x64->128 products, the
// output (hi1^c1^k0, lo1, hi0^c3^k1, lo0), and a Weyl key bump between rounds.
struct U64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c.v[0], hi0 = __umul64hi(M0, c.v[0]);
    const uint64_t lo1 = M1 * c.v[2], hi1 = __umul64hi(M1, c.v[2]);
    U64x4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
  }
  return c;
}

// (0,1) uniform with 52 random bits: ((w >> 12) + 1/2) 2^-52, exact in FP64.
__device__ __forceinline__ double u01_open(uint64_t w) {
  return (static_cast<double>(w >> 12) + 0.5) * 0x1.0p-52;
}

// ------------------------------------------------------------------ fixed point
// Fractional coordinate s in [0,1) -> 32-bit fixed point (s * 2^32 mod 2^32).
__device__ __forceinline__ uint32_t to_fixed(double s) {
  double t = s * 4294967296.0;
  uint64_t u = static_cast<uint64_t>(t);
  return static_cast<uint32_t>(u);
}

// Wrap x into [0, L) given 1/L.
__device__ __forceinline__ double wrap_frac(double x, double invL) {
  double s = x * invL;
  s -= floor(s);
  if (s >= 1.0) s -= 1.0;
  return s;
}

}  // namespace srbe
