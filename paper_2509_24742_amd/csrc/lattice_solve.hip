// Charge update of Eqs. (9)-(11) for electrodes on two rectangular lattices (gfx950).
//
// When both electrode walls are complete nx x ny lattices of spacing (Lx/nx, Ly/ny),
// every term of A (Eq. (18)) depends on a pair of sites only through their walls and
// the lattice displacement between them taken modulo the lattice: A is
// block-circulant.  The 2-D discrete Fourier transform over a wall,
//   X(p, q) = sum_{ix, iy} x(ix, iy) exp(-2 pi i (p ix / nx + q iy / ny)),
// therefore turns A x = v into one 2 x 2 system per mode (p, q) between the two walls'
// transforms, Lambda(p, q) X(p, q) = V(p, q), with Lambda(p, q) the transform of the
// first row of each wall-pair block (built at set-up, inverted there).  A^-1 e is
// constant on each wall (c_w), so the constrained solution
//   Q = A^-1 (v + psibar e),  psibar = -e^T A^-1 v / e^T A^-1 e
// only changes the (0, 0) mode: e^T A^-1 v = U_0(0, 0) + U_1(0, 0) for U = Lambda^-1 V,
// and adding psibar e adds psibar nx ny c_w to U_w(0, 0).  Three launches per step:
//   1. per (replica, wall, row iy): the transform along x of v = dpsi d + b*, a row at a
//      time through LDS;
//   2. per (replica, column p): the transform along y of both walls' columns, the
//      2 x 2 solves of the column's modes, the constraint at (0, 0), and the inverse
//      transform along y, all in LDS;
//   3. per (replica, wall, row iy): the inverse transform along x and 1/(nx ny); the
//      real part is the charge, written with psibar to the same (Q; psibar) rows the
//      dense GEMM fills.
// Products of indices are reduced modulo the length before the twiddle-table lookup,
// so every phase is exact.  All sums run in a fixed order: results are bitwise
// repeatable.  FP64 throughout.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace srbe {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // a conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

constexpr int kLatThreads = 256;

// Every launch stages its twiddle table in LDS beside the data, so the sums' loads
// are LDS reads rather than a chain of dependent global loads.

// Launch 1: block (r, w, iy); the row of v and the x twiddles in LDS, thread p sums
// over ix.  LDS: nx doubles + nx double2.
// (each launch's body takes its block index b; a multi-system launch passes the block's
// index within its system)
__device__ __forceinline__ void lat_fwd_x_body(const LatticeSolve& L, const double* __restrict__ V, int ldv, int b) {
  extern __shared__ double2 lds_fx[];
  const int nx = L.nx, ny = L.ny;
  double2* tw = lds_fx;
  double* row = reinterpret_cast<double*>(lds_fx + nx);
  const int r = b / (2 * ny), wy = b - r * 2 * ny;  // wy = w ny + iy
  const int* site = L.site + (size_t)wy * nx;
  for (int ix = threadIdx.x; ix < nx; ix += kLatThreads) {
    row[ix] = V[(size_t)r * ldv + site[ix]];
    tw[ix] = L.tw_x[ix];
  }
  __syncthreads();
  double2* T = L.T + ((size_t)r * 2 * ny + wy) * nx;
  for (int p = threadIdx.x; p < nx; p += kLatThreads) {
    double2 acc = make_double2(0.0, 0.0);
    int ph = 0;  // p ix mod nx
#pragma unroll 8
    for (int ix = 0; ix < nx; ++ix) {
      const double2 t = tw[ph];
      acc.x += row[ix] * t.x;
      acc.y += row[ix] * t.y;
      ph += p;
      if (ph >= nx) ph -= nx;
    }
    T[p] = acc;
  }
}

__global__ __launch_bounds__(kLatThreads) void k_lat_fwd_x(LatticeSolve L, const double* __restrict__ V, int ldv) {
  lat_fwd_x_body(L, V, ldv, blockIdx.x);
}

// Launch 2: block (r, p); both walls' column p and the y twiddles through LDS.
// LDS: 5 ny double2 ([2][ny] input column, [2][ny] solved modes, ny twiddles).
__device__ __forceinline__ void lat_column_body(const LatticeSolve& L, double* __restrict__ Qext, int n, int b) {
  extern __shared__ double2 col[];
  const int nx = L.nx, ny = L.ny;
  const int r = b / nx, p = b - r * nx;
  double2* cin = col;
  double2* cu = col + 2 * ny;
  double2* tw = col + 4 * ny;
  for (int u = threadIdx.x; u < 2 * ny; u += kLatThreads) cin[u] = L.T[((size_t)r * 2 * ny + u) * nx + p];
  for (int u = threadIdx.x; u < ny; u += kLatThreads) tw[u] = L.tw_y[u];
  __syncthreads();
  for (int q = threadIdx.x; q < ny; q += kLatThreads) {
    double2 v0 = make_double2(0.0, 0.0), v1 = make_double2(0.0, 0.0);
    int ph = 0;  // q iy mod ny
#pragma unroll 4
    for (int iy = 0; iy < ny; ++iy) {
      const double2 t = tw[ph];
      const double2 a0 = cmul(cin[iy], t), a1 = cmul(cin[ny + iy], t);
      v0.x += a0.x;
      v0.y += a0.y;
      v1.x += a1.x;
      v1.y += a1.y;
      ph += q;
      if (ph >= ny) ph -= ny;
    }
    const double2* li = L.linv + ((size_t)q * nx + p) * 4;
    const double2 m00 = cmul(li[0], v0), m01 = cmul(li[1], v1), m10 = cmul(li[2], v0), m11 = cmul(li[3], v1);
    double2 u0 = make_double2(m00.x + m01.x, m00.y + m01.y);
    double2 u1 = make_double2(m10.x + m11.x, m10.y + m11.y);
    if (p == 0 && q == 0) {
      // e^T A^-1 v = U_0(0,0) + U_1(0,0) (real); the constraint adds psibar nx ny c_w
      const double psibar = -(u0.x + u1.x) / L.etc;
      u0.x += psibar * (double)nx * ny * L.c0;
      u1.x += psibar * (double)nx * ny * L.c1;
      Qext[(size_t)r * (n + 1) + n] = psibar;
    }
    cu[q] = u0;
    cu[ny + q] = u1;
  }
  __syncthreads();
  for (int iy = threadIdx.x; iy < ny; iy += kLatThreads) {
    double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
    int ph = 0;
#pragma unroll 4
    for (int q = 0; q < ny; ++q) {
      const double2 t = tw[ph];
      const double2 a0 = cmulc(cu[q], t), a1 = cmulc(cu[ny + q], t);
      s0.x += a0.x;
      s0.y += a0.y;
      s1.x += a1.x;
      s1.y += a1.y;
      ph += iy;
      if (ph >= ny) ph -= ny;
    }
    L.U[((size_t)r * 2 * ny + iy) * nx + p] = s0;
    L.U[((size_t)r * 2 * ny + ny + iy) * nx + p] = s1;
  }
}

__global__ __launch_bounds__(kLatThreads) void k_lat_column(LatticeSolve L, double* __restrict__ Qext, int n) {
  lat_column_body(L, Qext, n, blockIdx.x);
}

// Launch 3: block (r, w, iy); the row of half-inverted modes and the x twiddles in
// LDS, thread ix sums over p and writes the charge of its site.  LDS: 2 nx double2.
__device__ __forceinline__ void lat_inv_x_body(const LatticeSolve& L, double* __restrict__ Qext, int n, int b) {
  extern __shared__ double2 rowc[];
  const int nx = L.nx, ny = L.ny;
  double2* tw = rowc + nx;
  const int r = b / (2 * ny), wy = b - r * 2 * ny;
  const double2* U = L.U + ((size_t)r * 2 * ny + wy) * nx;
  for (int p = threadIdx.x; p < nx; p += kLatThreads) {
    rowc[p] = U[p];
    tw[p] = L.tw_x[p];
  }
  __syncthreads();
  const int* site = L.site + (size_t)wy * nx;
  const double scale = 1.0 / ((double)nx * ny);
  for (int ix = threadIdx.x; ix < nx; ix += kLatThreads) {
    double acc = 0.0;
    int ph = 0;
#pragma unroll 8
    for (int p = 0; p < nx; ++p) {
      const double2 t = tw[ph];
      acc += rowc[p].x * t.x + rowc[p].y * t.y;  // Re(U conj(t))
      ph += ix;
      if (ph >= nx) ph -= nx;
    }
    Qext[(size_t)r * (n + 1) + site[ix]] = acc * scale;
  }
}

__global__ __launch_bounds__(kLatThreads) void k_lat_inv_x(LatticeSolve L, double* __restrict__ Qext, int n) {
  lat_inv_x_body(L, Qext, n, blockIdx.x);
}

// The three launches for every lattice system of a batch at once (see MultiLaunch).
template <int STEP>
__global__ __launch_bounds__(kLatThreads) void k_multi_lattice(MultiLaunch m) {
  const int s = multi_system(m, blockIdx.x), lb = blockIdx.x - m.start[s];
  const StepBufs& b = m.d[s].b;
  const int n = m.d[s].g.n_ele;
  if constexpr (STEP == 0)
    lat_fwd_x_body(b.lat, b.V, ldcp(n), lb);
  else if constexpr (STEP == 1)
    lat_column_body(b.lat, b.Qext, n, lb);
  else
    lat_inv_x_body(b.lat, b.Qext, n, lb);
}

}  // namespace

void lattice_grid(const StepBufs& b, int step, int& blocks, size_t& lds) {
  const LatticeSolve& L = b.lat;
  blocks = step == 1 ? b.R * L.nx : b.R * 2 * L.ny;
  lds = step == 0 ? (size_t)L.nx * (sizeof(double) + sizeof(double2))
        : step == 1 ? (size_t)5 * L.ny * sizeof(double2)
                    : (size_t)2 * L.nx * sizeof(double2);
}

void launch_multi_lattice(int step, const MultiLaunch& m, int nblocks, size_t lds, hipStream_t s) {
  if (nblocks == 0) return;
  if (step == 0)
    hipLaunchKernelGGL(k_multi_lattice<0>, dim3(nblocks), dim3(kLatThreads), lds, s, m);
  else if (step == 1)
    hipLaunchKernelGGL(k_multi_lattice<1>, dim3(nblocks), dim3(kLatThreads), lds, s, m);
  else
    hipLaunchKernelGGL(k_multi_lattice<2>, dim3(nblocks), dim3(kLatThreads), lds, s, m);
}

void launch_lattice_solve(const Geom& g, const StepBufs& b, hipStream_t s) {
  const LatticeSolve& L = b.lat;
  const int R = b.R, n = g.n_ele;
  hipLaunchKernelGGL(k_lat_fwd_x, dim3((unsigned)R * 2 * L.ny), dim3(kLatThreads),
                     (size_t)L.nx * (sizeof(double) + sizeof(double2)), s, L, (const double*)b.V, ldcp(n));
  hipLaunchKernelGGL(k_lat_column, dim3((unsigned)R * L.nx), dim3(kLatThreads), (size_t)5 * L.ny * sizeof(double2),
                     s, L, b.Qext, n);
  hipLaunchKernelGGL(k_lat_inv_x, dim3((unsigned)R * 2 * L.ny), dim3(kLatThreads), (size_t)2 * L.nx * sizeof(double2),
                     s, L, b.Qext, n);
}

}  // namespace srbe
