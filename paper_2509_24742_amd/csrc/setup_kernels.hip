// Setup kernels: the electrode matrix A of Eq. (18) and the projected inverse
// S = J A^-1 of Eqs. (10)-(11).  A is constant (the electrodes do not move), so this
// runs once per geometry.
#include <math.h>

#include "kernels.h"

namespace srbe {

static inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

#define TWO_PI 6.283185307179586

// E[:, c] = sqrt(w_c) cos(k_c.R), E[:, nk + c] = sqrt(w_c) sin(k_c.R), column-major
// n_ele x 2nk with leading dimension ld.  Then A_F = E E^T: the reciprocal sum
// sum_k w_k cos(k.(R_i - R_j)) by the angle-difference identity.
__global__ __launch_bounds__(256) void k_ele_phase_block(const double* __restrict__ xyz, int n,
                                                         const int* __restrict__ m, const double* __restrict__ sqrtw,
                                                         int nk, int ld, double* __restrict__ E, Geom g) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (j >= n || c >= nk) return;
  const double sx = xyz[j] * g.invLx, sy = xyz[n + j] * g.invLy, sz = xyz[2 * n + j] * g.invLz;
  double t = fma((double)m[3 * c], sx, fma((double)m[3 * c + 1], sy, (double)m[3 * c + 2] * sz));
  t -= rint(t);
  double sn, cs;
  sincospi(2.0 * t, &sn, &cs);
  const double w = sqrtw[c];
  E[(size_t)c * ld + j] = w * cs;
  E[(size_t)(nk + c) * ld + j] = w * sn;
}

void launch_ele_phase_block(const double* ele_xyz, int n_ele, const int* m, const double* sqrtw, int nk, int ld,
                            double* E, const Geom& g, hipStream_t s) {
  hipLaunchKernelGGL(k_ele_phase_block, dim3(cdiv(n_ele, 256), nk), dim3(256), 0, s, ele_xyz, n_ele, m, sqrtw, nk, ld,
                     E, g);
}

// Real-space Gaussian-Gaussian images (Eq. (18), second term), the self entry
// 2 delta_ij (1/(sqrt(2 pi) eta) - alpha/sqrt(pi)) and the slab entry
// (4 pi / V) Z_i Z_j, all times ke, added to A (column-major, n x n).
__global__ __launch_bounds__(256) void k_ele_realspace_matrix(Geom g, const double* __restrict__ xyz, int n,
                                                              double* __restrict__ A) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  const double a = g.alpha, b = 1.0 / (sqrt(2.0) * g.eta), rc2 = g.rc * g.rc;
  double dx0 = xyz[i] - xyz[j], dy0 = xyz[n + i] - xyz[n + j];
  const double dz = xyz[2 * n + i] - xyz[2 * n + j];
  // every image closer than rc (rc <= L/2, so the nearest image suffices)
  dx0 -= g.Lx * rint(dx0 * g.invLx);
  dy0 -= g.Ly * rint(dy0 * g.invLy);
  double v = 0.0;
  const double r2 = dx0 * dx0 + dy0 * dy0 + dz * dz;
  if (i != j && r2 < rc2) {
    const double r = sqrt(r2);
    v += (erfc(a * r) - erfc(b * r)) / r;
  }
  if (i == j) v += 2.0 * (1.0 / (sqrt(2.0 * M_PI) * g.eta) - a / sqrt(M_PI));
  v += (4.0 * M_PI / g.V) * xyz[2 * n + i] * xyz[2 * n + j];
  A[(size_t)j * n + i] += g.ke * v;
}

void launch_ele_realspace_matrix(const Geom& g, const double* ele_xyz, int n_ele, double* A, hipStream_t s) {
  hipLaunchKernelGGL(k_ele_realspace_matrix, dim3(cdiv(n_ele, 256), n_ele), dim3(256), 0, s, g, ele_xyz, n_ele, A);
}

// Copy the lower triangle onto the upper one.
__global__ __launch_bounds__(256) void k_symmetrize_lower(double* A, int n, int ld) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n || i >= j) return;  // (i, j) with i < j is in the upper triangle
  A[(size_t)j * ld + i] = A[(size_t)i * ld + j];
}

void launch_symmetrize_lower(double* A, int n, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetrize_lower, dim3(cdiv(n, 256), n), dim3(256), 0, s, A, n, ld);
}

// out_i = sum_j A_ij (A symmetric, so column sums are read contiguously).
__global__ __launch_bounds__(256) void k_rowsum(const double* __restrict__ A, int n, int ld, double* __restrict__ out) {
  __shared__ double sh[256];
  const int col = blockIdx.x;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) v += A[(size_t)col * ld + i];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[col] = sh[0];
}

void launch_rowsum(const double* A, int n, int ld, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_rowsum, dim3(n), dim3(256), 0, s, A, n, ld, out);
}

// S_ext, (n+1) rows of ldcp(n) doubles, row-major: rows 0..n-1 hold
// S = A^-1 - g g^T / (e^T g) (= J A^-1, Eq. (10), symmetric); row n holds
// -g^T / (e^T g), so that row n times (dpsi d + b) is psibar of Eq. (9).  Columns
// n .. ldcp(n)-1 are zero.
__global__ __launch_bounds__(256) void k_build_sext(const double* __restrict__ Ainv, int n,
                                                    const double* __restrict__ gv, double eg,
                                                    double* __restrict__ Sext) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  const int ld = ldcp(n);
  if (j >= ld) return;
  double v = 0.0;
  if (j < n) v = i < n ? Ainv[(size_t)j * n + i] - gv[i] * gv[j] / eg : -gv[j] / eg;
  Sext[(size_t)i * ld + j] = v;
}

void launch_build_sext(const double* Ainv, int n, const double* gv, double eg, double* Sext, hipStream_t s) {
  hipLaunchKernelGGL(k_build_sext, dim3(cdiv(ldcp(n), 256), n + 1), dim3(256), 0, s, Ainv, n, gv, eg, Sext);
}

__global__ __launch_bounds__(256) void k_check_finite(const double* __restrict__ a, size_t n, unsigned* status) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n && !isfinite(a[i])) atomicOr(status, ST_NUMERIC);
}

void launch_check_finite(const double* a, size_t n, unsigned* status, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_check_finite, dim3(cdiv((int64_t)n, 256)), dim3(256), 0, s, a, n, status);
}

}  // namespace srbe
