// Per-step kernels of the SRBE constant-potential step (gfx950).
//
// Pipeline of one step (Algorithm 1 of the paper, integration excluded), all on
// one stream, for R replicas sharing one electrode geometry:
//   replica_scalars -> sample -> prep -> sf(ions) -> finalize(1) -> ele_potential
//   -> [FP64 GEMM: (Q; psibar) = S_ext V] -> post_charges -> sf(electrodes)
//   -> finalize(2) -> ion_force -> energy
// Every reduction has a fixed order (no floating-point atomics), so two runs on
// the same inputs give bitwise-identical results.
#include <math.h>

#include "kernels.h"

namespace srbe {

static inline int cdiv64(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

#define TWO_PI 6.283185307179586
#define INV_SQRT_PI 0.5641895835477563

// Deterministic block reduction of NV doubles over a 256-thread block; result in
// thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[256]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int a = 0; a < NV; ++a) sh[a][t] = v[a];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
#pragma unroll
      for (int a = 0; a < NV; ++a) sh[a][t] += sh[a][t + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = sh[a][0];
  __syncthreads();
}

// ============================================================ replica scalars
// sum q (neutrality), sum |q|, sum q z (slab term of Eq. (17)), sum q^2 (self term);
// flags z outside [0, H] and non-finite inputs.
__global__ __launch_bounds__(256) void k_replica_scalars(Geom g, const int64_t* __restrict__ off,
                                                         const double* __restrict__ xyz,
                                                         const double* __restrict__ q, int64_t N,
                                                         double* __restrict__ scal, unsigned* status) {
  __shared__ double sh[4][256];
  const int r = blockIdx.x;
  const int64_t b = off[r], e = off[r + 1];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  int bad = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    const double qi = q[i], x = xyz[i], y = xyz[N + i], z = xyz[2 * N + i];
    if (!isfinite(qi) || !isfinite(x) || !isfinite(y) || !(z >= 0.0 && z <= g.H)) bad = 1;
    v[0] += qi;
    v[1] += fabs(qi);
    v[2] += qi * z;
    v[3] += qi * qi;
  }
  if (bad) atomicOr(status, ST_RANGE);
  block_sum<4>(v, sh);
  if (threadIdx.x == 0) {
    scal[4 * r + 0] = v[0];
    scal[4 * r + 1] = v[1];
    scal[4 * r + 2] = v[2];
    scal[4 * r + 3] = v[3];
    if (fabs(v[0]) > 1e-10 * v[1]) atomicOr(status, ST_NONNEUTRAL);
  }
}

void launch_replica_scalars(const Geom& g, const StepBufs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_replica_scalars, dim3(b.R), dim3(256), 0, s, g, b.off, b.ion_xyz, b.ion_q, b.N, b.scal,
                     b.status);
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

__device__ double log_ratio(const Geom& g, int mx, int my, int mz) {
  const double kx = TWO_PI * (double)mx / g.Lx;
  const double ky = TWO_PI * (double)my / g.Ly;
  const double kz = TWO_PI * (double)mz / g.Lz;
  const double k2 = kx * kx + ky * ky + kz * kz;
  const double lq = log(q_axis(mx, g.alpha, g.Lx)) + log(q_axis(my, g.alpha, g.Ly)) + log(q_axis(mz, g.alpha, g.Lz));
  return -k2 / (4.0 * (g.alpha * g.alpha)) - lq;
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

__global__ __launch_bounds__(256) void k_sample(Geom g, const uint64_t* __restrict__ seeds, uint64_t step,
                                                const int32_t* __restrict__ kset_in, int4* __restrict__ modes,
                                                double* __restrict__ wout, int32_t* __restrict__ kset_out,
                                                int32_t* __restrict__ nacc_out, unsigned* status) {
  extern __shared__ unsigned char smem[];
  const int r = blockIdx.x;
  const int P = g.P, M = g.M, K = g.K;
  const int t = threadIdx.x;
  // deterministic modes (0, 0, m), m = 1..M, weight doubled for the pair +-m
  for (int m = 1 + t; m <= M; m += 256) {
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
    for (int l = t; l < P; l += 256) {
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
  // LDS layout: ly[P] (double), lu[P] (double), ym[P][3] (int), ok[P] (char)
  double* ly = reinterpret_cast<double*>(smem);
  double* lu = ly + P;
  int* ym = reinterpret_cast<int*>(lu + P);
  unsigned char* ok = reinterpret_cast<unsigned char*>(ym + 3 * P);
  __shared__ int first_valid;
  __shared__ int start_m[3];
  if (t == 0) first_valid = 1 << 30;
  __syncthreads();
  int sx = 0, sy = 0, sz = 0;
  if (t < 64) {
    proposal(g, seed, step, 2, (uint64_t)t, sx, sy, sz);
    if (valid_mode(g, sx, sy, sz)) atomicMin(&first_valid, t);
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
  for (int l = t; l < P; l += 256) {
    int mx, my, mz;
    proposal(g, seed, step, 0, (uint64_t)l, mx, my, mz);
    U64x4 c;
    c.v[0] = (uint64_t)l;
    c.v[1] = step;
    c.v[2] = 1;
    c.v[3] = 0;
    const U64x4 wa = philox4x64_10(c, seed, 0);
    const bool v = valid_mode(g, mx, my, mz);
    ym[3 * l + 0] = mx;
    ym[3 * l + 1] = my;
    ym[3 * l + 2] = mz;
    ok[l] = v ? 1 : 0;
    ly[l] = v ? log_ratio(g, mx, my, mz) : 0.0;
    lu[l] = log(u01_open(wa.v[0]));
  }
  __syncthreads();
  if (t == 0) {
    int cx = start_m[0], cy = start_m[1], cz = start_m[2];
    double lx = log_ratio(g, cx, cy, cz);
    int nacc = 0;
    for (int l = 0; l < P; ++l) {
      if (ok[l]) {
        const double d = ly[l] - lx;
        if (d >= 0.0 || lu[l] < d) {
          cx = ym[3 * l + 0];
          cy = ym[3 * l + 1];
          cz = ym[3 * l + 2];
          lx = ly[l];
          ++nacc;
        }
      }
      ym[3 * l + 0] = cx;
      ym[3 * l + 1] = cy;
      ym[3 * l + 2] = cz;
    }
    if (nacc_out) nacc_out[r] = nacc;
  }
  __syncthreads();
  for (int l = t; l < P; l += 256) {
    const int mx = ym[3 * l + 0], my = ym[3 * l + 1], mz = ym[3 * l + 2];
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

size_t sample_lds_bytes(int P) { return (size_t)P * (8 + 8 + 12 + 1) + 16; }

void launch_sample(const Geom& g, const StepBufs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_sample, dim3(b.R), dim3(256), sample_lds_bytes(g.P), s, g, b.seed, b.step, b.kset_in, b.modes,
                     b.w, b.kset_out, b.nacc_out, b.status);
}

// ============================================================ prep
// FP64 path: fractional coordinates s = x/L wrapped into [0,1).  FP32 path: the
// same as 32-bit fixed point (s 2^32 mod 2^32) with the charge as FP32, one
// 16-byte record per ion.  With fixed point, k.r in revolutions is the exact
// wrap-around integer m_x u_x + m_y u_y + m_z u_z mod 2^32.
__global__ __launch_bounds__(256) void k_prep(Geom g, const double* __restrict__ xyz, const double* __restrict__ q,
                                              int64_t N, double* __restrict__ frac, uint4* __restrict__ fx, int fp32) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= N) return;
  const double sx = wrap_frac(xyz[i], g.invLx);
  const double sy = wrap_frac(xyz[N + i], g.invLy);
  const double sz = wrap_frac(xyz[2 * N + i], g.invLz);
  if (fp32) {
    fx[i] = make_uint4(to_fixed(sx), to_fixed(sy), to_fixed(sz), __float_as_uint((float)q[i]));
  } else {
    frac[i] = sx;
    frac[N + i] = sy;
    frac[2 * N + i] = sz;
  }
}

void launch_prep(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  if (b.N == 0) return;
  hipLaunchKernelGGL(k_prep, dim3(cdiv64(b.N, 256)), dim3(256), 0, s, g, b.ion_xyz, b.ion_q, b.N, b.ion_frac, b.ion_fx,
                     fp32);
}

// ============================================================ structure factors
// S(k) = sum_j q_j exp(i k.r_j), Eq. (15).  One thread per mode, the particle loop
// is uniform across the wave (particle data arrive by scalar loads).  Grid:
// (mode tiles of 256, particle chunks, replicas); partial sums per chunk are
// combined in a fixed order by k_sf_finalize.
template <bool ION>
__global__ __launch_bounds__(256) void k_sf64(Geom g, const int64_t* __restrict__ off, int n_fixed,
                                              const double* __restrict__ fr, int64_t nstride,
                                              const double* __restrict__ q, const int4* __restrict__ modes,
                                              double2* __restrict__ part, int nchunk) {
  const int r = blockIdx.z;
  const int k = blockIdx.x * 256 + threadIdx.x;
  int64_t b, e;
  if (ION) {
    b = off[r];
    e = off[r + 1];
  } else {
    b = 0;
    e = n_fixed;
  }
  const int64_t chunk = (e - b + nchunk - 1) / nchunk;
  const int64_t j0 = b + (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(e, j0 + chunk);
  const double* qq = ION ? q : q + (size_t)r * n_fixed;
  if (k >= g.K) return;
  const int4 m = modes[(size_t)r * g.K + k];
  const double mx = m.x, my = m.y, mz = m.z;
  double sr = 0.0, si = 0.0;
  for (int64_t j = j0; j < j1; ++j) {
    double t = fma(mx, fr[j], fma(my, fr[nstride + j], mz * fr[2 * nstride + j]));
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    const double qj = ION ? qq[j] : qq[j];
    sr = fma(qj, cs, sr);
    si = fma(qj, sn, si);
  }
  part[((size_t)r * nchunk + blockIdx.y) * g.K + k] = make_double2(sr, si);
}

// FP32: exact integer phase, hardware sin/cos of the phase in revolutions, FP32
// sums over blocks of 64 particles carried in FP64.
template <bool ION>
__global__ __launch_bounds__(256) void k_sf32(Geom g, const int64_t* __restrict__ off, int n_fixed,
                                              const uint4* __restrict__ pts, const float* __restrict__ qe,
                                              const int4* __restrict__ modes, double2* __restrict__ part, int nchunk) {
  const int r = blockIdx.z;
  const int k = blockIdx.x * 256 + threadIdx.x;
  int64_t b, e;
  if (ION) {
    b = off[r];
    e = off[r + 1];
  } else {
    b = 0;
    e = n_fixed;
  }
  const int64_t chunk = (e - b + nchunk - 1) / nchunk;
  const int64_t j0 = b + (int64_t)blockIdx.y * chunk;
  const int64_t j1 = min(e, j0 + chunk);
  if (k >= g.K) return;
  const float* qq = ION ? nullptr : qe + (size_t)r * n_fixed;
  const int4 m = modes[(size_t)r * g.K + k];
  const uint32_t mx = (uint32_t)m.x, my = (uint32_t)m.y, mz = (uint32_t)m.z;
  double dr = 0.0, di = 0.0;
  for (int64_t jb = j0; jb < j1; jb += 64) {
    const int64_t je = min(j1, jb + 64);
    float ar = 0.f, ai = 0.f;
    for (int64_t j = jb; j < je; ++j) {
      const uint4 p = pts[j];
      const float qj = ION ? __uint_as_float(p.w) : qq[j];
      const uint32_t ph = mx * p.x + my * p.y + mz * p.z;
      const float x = (float)(int32_t)ph * 0x1.0p-32f;
      const float sn = __builtin_amdgcn_sinf(x);
      const float cs = __builtin_amdgcn_cosf(x);
      ar = fmaf(qj, cs, ar);
      ai = fmaf(qj, sn, ai);
    }
    dr += (double)ar;
    di += (double)ai;
  }
  part[((size_t)r * nchunk + blockIdx.y) * g.K + k] = make_double2(dr, di);
}

void launch_sf_ions(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  if (g.K == 0) return;
  dim3 grid(cdiv64(g.K, 256), b.nchunk_ion, b.R);
  if (fp32)
    hipLaunchKernelGGL(k_sf32<true>, grid, dim3(256), 0, s, g, b.off, 0, b.ion_fx, (const float*)nullptr, b.modes,
                       b.part, b.nchunk_ion);
  else
    hipLaunchKernelGGL(k_sf64<true>, grid, dim3(256), 0, s, g, b.off, 0, b.ion_frac, b.N, b.ion_q, b.modes, b.part,
                       b.nchunk_ion);
}

void launch_sf_ele(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  if (g.K == 0) return;
  dim3 grid(cdiv64(g.K, 256), b.nchunk_ele, b.R);
  if (fp32)
    hipLaunchKernelGGL(k_sf32<false>, grid, dim3(256), 0, s, g, b.off, g.n_ele, b.ele_fx, b.Qf, b.modes, b.part,
                       b.nchunk_ele);
  else
    hipLaunchKernelGGL(k_sf64<false>, grid, dim3(256), 0, s, g, b.off, g.n_ele, b.ele_frac, (int64_t)g.n_ele, b.Q_out,
                       b.modes, b.part, b.nchunk_ele);
}

// stage 1: S1 = sum of partials; coef = w S1.  stage 2: S = S1 + sum of partials
// (electrodes); coef = w S.  The FP32 path also fills the mode records.
__global__ __launch_bounds__(256) void k_sf_finalize(Geom g, const double2* __restrict__ part, int nchunk,
                                                     const int4* __restrict__ modes, const double* __restrict__ w,
                                                     double2* __restrict__ S1, double2* __restrict__ coef,
                                                     ModeRec32* __restrict__ rec, int stage, unsigned* status) {
  const int r = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= g.K) return;
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const double2 p = part[((size_t)r * nchunk + c) * g.K + k];
    sr += p.x;
    si += p.y;
  }
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

void launch_sf_finalize(const Geom& g, const StepBufs& b, int stage, int fp32, hipStream_t s) {
  if (g.K == 0) return;
  const int nchunk = stage == 1 ? b.nchunk_ion : b.nchunk_ele;
  hipLaunchKernelGGL(k_sf_finalize, dim3(cdiv64(g.K, 256), b.R), dim3(256), 0, s, g, b.part, nchunk, b.modes, b.w,
                     b.S1, b.coef, fp32 ? b.rec : nullptr, stage, b.status);
}

// ============================================================ real-space kernels
// Eq. (13): ion-ion erfc(alpha r)/r and ion-Gaussian [erfc(alpha r) - erfc(r/eta)]/r.
__device__ __forceinline__ void erfc_over_r(double a, double r, double& f, double& df) {
  const double e = erfc(a * r);
  const double inv = 1.0 / r;
  f = e * inv;
  df = -e * inv * inv - 2.0 * a * INV_SQRT_PI * exp(-(a * r) * (a * r)) * inv;
}

__device__ __forceinline__ void erfc_over_r_f(float a, float r, float& f, float& df) {
  const float e = erfcf(a * r);
  const float inv = 1.0f / r;
  f = e * inv;
  df = -e * inv * inv - 2.0f * a * (float)INV_SQRT_PI * __expf(-(a * r) * (a * r)) * inv;
}

// ============================================================ electrode potential b*
// b*_j = -sum_k Re(coef_k exp(-i k.R_j))                     (Eq. (24), coef = w S1)
//        - (4 pi ke / V) Z_j sum_i q_i z_i                    (slab term, minus sign)
//        - ke sum_i q_i [erfc(alpha r) - erfc(r/eta)]/r        (real space, r < rc)
// and V_j = b*_j + dpsi d_j, the right-hand side of the charge solve.
__global__ __launch_bounds__(256) void k_elepot64(Geom g, const int64_t* __restrict__ off,
                                                  const double* __restrict__ ion_xyz, const double* __restrict__ ion_q,
                                                  int64_t N, const double* __restrict__ ele_xyz,
                                                  const double* __restrict__ ele_frac, const double* __restrict__ ele_d,
                                                  const int4* __restrict__ modes, const double2* __restrict__ coef,
                                                  const double* __restrict__ scal, const double* __restrict__ dpsi,
                                                  double* __restrict__ bstar, double* __restrict__ V) {
  const int r = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int n = g.n_ele;
  if (j >= n) return;
  const double sx = ele_frac[j], sy = ele_frac[n + j], sz = ele_frac[2 * n + j];
  double acc = 0.0;
  const int4* mr = modes + (size_t)r * g.K;
  const double2* cr = coef + (size_t)r * g.K;
  for (int k = 0; k < g.K; ++k) {
    const int4 m = mr[k];
    double t = fma((double)m.x, sx, fma((double)m.y, sy, (double)m.z * sz));
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    const double2 c = cr[k];
    acc = fma(c.x, cs, fma(c.y, sn, acc));
  }
  const double X = ele_xyz[j], Y = ele_xyz[n + j], Z = ele_xyz[2 * n + j];
  double b = -acc - (4.0 * M_PI * g.ke / g.V) * Z * scal[4 * r + 2];
  double real = 0.0;
  const double a = g.alpha, ai = 1.0 / g.eta, rc2 = g.rc * g.rc;
  for (int64_t i = off[r]; i < off[r + 1]; ++i) {
    double dx = X - ion_xyz[i], dy = Y - ion_xyz[N + i];
    const double dz = Z - ion_xyz[2 * N + i];
    dx -= g.Lx * rint(dx * g.invLx);
    dy -= g.Ly * rint(dy * g.invLy);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const double rr = sqrt(r2);
      double f1, d1, f2, d2;
      erfc_over_r(a, rr, f1, d1);
      erfc_over_r(ai, rr, f2, d2);
      real += ion_q[i] * (f1 - f2);
    }
  }
  b -= g.ke * real;
  bstar[(size_t)r * n + j] = b;
  V[(size_t)r * n + j] = b + dpsi[r] * ele_d[j];
}

__global__ __launch_bounds__(256) void k_elepot32(Geom g, const int64_t* __restrict__ off,
                                                  const uint4* __restrict__ ion_fx, const uint4* __restrict__ ele_fx,
                                                  const double* __restrict__ ele_xyz, const double* __restrict__ ele_d,
                                                  const ModeRec32* __restrict__ rec, const double* __restrict__ scal,
                                                  const double* __restrict__ dpsi, double* __restrict__ bstar,
                                                  double* __restrict__ V) {
  const int r = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int n = g.n_ele;
  if (j >= n) return;
  const uint4 pe = ele_fx[j];
  const ModeRec32* mr = rec + (size_t)r * g.K;
  double acc = 0.0;
  for (int kb = 0; kb < g.K; kb += 64) {
    const int ke_ = min(g.K, kb + 64);
    float a = 0.f;
    for (int k = kb; k < ke_; ++k) {
      const ModeRec32 m = mr[k];
      const uint32_t ph = (uint32_t)m.mx * pe.x + (uint32_t)m.my * pe.y + (uint32_t)m.mz * pe.z;
      const float x = (float)(int32_t)ph * 0x1.0p-32f;
      a = fmaf(m.cre, __builtin_amdgcn_cosf(x), a);
      a = fmaf(m.cim, __builtin_amdgcn_sinf(x), a);
    }
    acc += (double)a;
  }
  const double Z = ele_xyz[2 * n + j];
  double b = -acc - (4.0 * M_PI * g.ke / g.V) * Z * scal[4 * r + 2];
  // real space in FP32 from fixed-point differences (exact periodic wrap in x, y)
  const float lx = (float)(g.Lx * 0x1.0p-32), ly = (float)(g.Ly * 0x1.0p-32), lz = (float)(g.Lz * 0x1.0p-32);
  const float a1 = (float)g.alpha, a2 = (float)(1.0 / g.eta), rc2 = (float)(g.rc * g.rc);
  float real = 0.f;
  for (int64_t i = off[r]; i < off[r + 1]; ++i) {
    const uint4 p = ion_fx[i];
    const float dx = (float)(int32_t)(pe.x - p.x) * lx;
    const float dy = (float)(int32_t)(pe.y - p.y) * ly;
    const float dz = (float)(int32_t)(pe.z - p.z) * lz;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const float rr = sqrtf(r2);
      float f1, d1, f2, d2;
      erfc_over_r_f(a1, rr, f1, d1);
      erfc_over_r_f(a2, rr, f2, d2);
      real = fmaf(__uint_as_float(p.w), f1 - f2, real);
    }
  }
  b -= g.ke * (double)real;
  bstar[(size_t)r * n + j] = b;
  V[(size_t)r * n + j] = b + dpsi[r] * ele_d[j];
}

void launch_ele_potential(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  dim3 grid(cdiv64(g.n_ele, 256), b.R);
  if (fp32)
    hipLaunchKernelGGL(k_elepot32, grid, dim3(256), 0, s, g, b.off, b.ion_fx, b.ele_fx, b.ele_xyz, b.ele_d, b.rec,
                       b.scal, b.dpsi, b.bstar, b.V);
  else
    hipLaunchKernelGGL(k_elepot64, grid, dim3(256), 0, s, g, b.off, b.ion_xyz, b.ion_q, b.N, b.ele_xyz, b.ele_frac,
                       b.ele_d, b.modes, b.coef, b.scal, b.dpsi, b.bstar, b.V);
}

// ============================================================ after the charge solve
// Per replica: copy Q (and psibar) out of the GEMM result (or the fixed charges),
// an FP32 copy of Q for the FP32 passes, and sum Q Z (slab term), d.Q, b*.Q
// (energy).
__global__ __launch_bounds__(256) void k_post_charges(Geom g, const double* __restrict__ Qext,
                                                      const double* __restrict__ Q_in, const double* __restrict__ ele_xyz,
                                                      const double* __restrict__ ele_d,
                                                      const double* __restrict__ bstar, double* __restrict__ Q_out,
                                                      float* __restrict__ Qf, double* __restrict__ psibar,
                                                      double* __restrict__ rsum, unsigned* status) {
  __shared__ double sh[3][256];
  const int r = blockIdx.x;
  const int n = g.n_ele;
  double v[3] = {0.0, 0.0, 0.0};
  int bad = 0;
  for (int j = threadIdx.x; j < n; j += 256) {
    const double Qj = Q_in ? Q_in[(size_t)r * n + j] : Qext[(size_t)r * (n + 1) + j];
    if (!isfinite(Qj)) bad = 1;
    Q_out[(size_t)r * n + j] = Qj;
    if (Qf) Qf[(size_t)r * n + j] = (float)Qj;
    v[0] += Qj * ele_xyz[2 * n + j];
    v[1] += Qj * ele_d[j];
    v[2] += Qj * bstar[(size_t)r * n + j];
  }
  if (bad) atomicOr(status, ST_NUMERIC);
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    rsum[8 * r + 0] = v[0];
    rsum[8 * r + 1] = v[1];
    rsum[8 * r + 2] = v[2];
    if (psibar) psibar[r] = Q_in ? (double)NAN : Qext[(size_t)r * (n + 1) + n];
  }
}

void launch_post_charges(const Geom& g, const StepBufs& b, int fixedQ, hipStream_t s) {
  hipLaunchKernelGGL(k_post_charges, dim3(b.R), dim3(256), 0, s, g, b.Qext, fixedQ ? b.Q_in : nullptr, b.ele_xyz,
                     b.ele_d, b.bstar, b.Q_out, b.Qf, b.psibar_out, b.rsum, b.status);
}

// ============================================================ ion forces
// F_i = -q_i sum_k k Im(coef_k exp(-i k.r_i))     (Eq. (25), coef = w (S1 + S2))
//       - (4 pi ke / V) q_i M_z e_z               (slab force, M_z = sum q z + sum Q Z)
//       - ke q_i sum_j q_j K_ii'(r) r^/ - ke q_i sum_e Q_e K_ig'(r) r^   (real space)
// phi_i = ke sum_j q_j K_ii(r) (ion-ion real-space potential, for the energy).
__global__ __launch_bounds__(256) void k_ionforce64(Geom g, const int64_t* __restrict__ off,
                                                    const double* __restrict__ ion_xyz,
                                                    const double* __restrict__ ion_q,
                                                    const double* __restrict__ ion_frac, int64_t N,
                                                    const double* __restrict__ ele_xyz, const double* __restrict__ Q,
                                                    const int4* __restrict__ modes, const double2* __restrict__ coef,
                                                    const double* __restrict__ scal, const double* __restrict__ rsum,
                                                    double* __restrict__ F, double* __restrict__ phi) {
  const int r = blockIdx.y;
  const int64_t b0 = off[r], b1 = off[r + 1];
  const int64_t i = b0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= b1) return;
  const double sx = ion_frac[i], sy = ion_frac[N + i], sz = ion_frac[2 * N + i];
  double gx = 0.0, gy = 0.0, gz = 0.0;
  const int4* mr = modes + (size_t)r * g.K;
  const double2* cr = coef + (size_t)r * g.K;
  for (int k = 0; k < g.K; ++k) {
    const int4 m = mr[k];
    double t = fma((double)m.x, sx, fma((double)m.y, sy, (double)m.z * sz));
    t -= rint(t);
    double sn, cs;
    sincospi(2.0 * t, &sn, &cs);
    const double2 c = cr[k];
    const double im = fma(c.y, cs, -c.x * sn);
    gx = fma(TWO_PI * (double)m.x * g.invLx, im, gx);
    gy = fma(TWO_PI * (double)m.y * g.invLy, im, gy);
    gz = fma(TWO_PI * (double)m.z * g.invLz, im, gz);
  }
  const double qi = ion_q[i];
  double Fx = -qi * gx, Fy = -qi * gy, Fz = -qi * gz;
  Fz -= (4.0 * M_PI * g.ke / g.V) * qi * (scal[4 * r + 2] + rsum[8 * r + 0]);
  const double X = ion_xyz[i], Y = ion_xyz[N + i], Z = ion_xyz[2 * N + i];
  const double a = g.alpha, ai = 1.0 / g.eta, rc2 = g.rc * g.rc;
  double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
  for (int64_t j = b0; j < b1; ++j) {
    if (j == i) continue;
    double dx = X - ion_xyz[j], dy = Y - ion_xyz[N + j];
    const double dz = Z - ion_xyz[2 * N + j];
    dx -= g.Lx * rint(dx * g.invLx);
    dy -= g.Ly * rint(dy * g.invLy);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const double rr = sqrt(r2);
      double f, df;
      erfc_over_r(a, rr, f, df);
      const double qj = ion_q[j];
      ph += qj * f;
      const double s = -qj * df / rr;
      fx += s * dx;
      fy += s * dy;
      fz += s * dz;
    }
  }
  const int n = g.n_ele;
  const double* Qr = Q + (size_t)r * n;
  for (int e = 0; e < n; ++e) {
    double dx = X - ele_xyz[e], dy = Y - ele_xyz[n + e];
    const double dz = Z - ele_xyz[2 * n + e];
    dx -= g.Lx * rint(dx * g.invLx);
    dy -= g.Ly * rint(dy * g.invLy);
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const double rr = sqrt(r2);
      double f1, d1, f2, d2;
      erfc_over_r(a, rr, f1, d1);
      erfc_over_r(ai, rr, f2, d2);
      const double s = -Qr[e] * (d1 - d2) / rr;
      fx += s * dx;
      fy += s * dy;
      fz += s * dz;
    }
  }
  const double kq = g.ke * qi;
  F[i] = Fx + kq * fx;
  F[N + i] = Fy + kq * fy;
  F[2 * N + i] = Fz + kq * fz;
  phi[i] = g.ke * ph;
}

__global__ __launch_bounds__(256) void k_ionforce32(Geom g, const int64_t* __restrict__ off,
                                                    const uint4* __restrict__ ion_fx, int64_t N,
                                                    const uint4* __restrict__ ele_fx, const float* __restrict__ Qf,
                                                    const ModeRec32* __restrict__ rec,
                                                    const double* __restrict__ scal, const double* __restrict__ rsum,
                                                    double* __restrict__ F, double* __restrict__ phi) {
  const int r = blockIdx.y;
  const int64_t b0 = off[r], b1 = off[r + 1];
  const int64_t i = b0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= b1) return;
  const uint4 pi_ = ion_fx[i];
  const ModeRec32* mr = rec + (size_t)r * g.K;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  // deterministic modes: k = (0, 0, kz); only the z component
  {
    float az = 0.f;
    for (int k = 0; k < g.M; ++k) {
      const ModeRec32 m = mr[k];
      const uint32_t ph = (uint32_t)m.mz * pi_.z;
      const float x = (float)(int32_t)ph * 0x1.0p-32f;
      const float im = m.cim * __builtin_amdgcn_cosf(x) - m.cre * __builtin_amdgcn_sinf(x);
      az = fmaf(m.kz, im, az);
    }
    gz += (double)az;
  }
  for (int kb = g.M; kb < g.K; kb += 64) {
    const int ke_ = min(g.K, kb + 64);
    float ax = 0.f, ay = 0.f, az = 0.f;
    for (int k = kb; k < ke_; ++k) {
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
  const double qi = (double)__uint_as_float(pi_.w);
  double Fx = -qi * gx, Fy = -qi * gy, Fz = -qi * gz;
  Fz -= (4.0 * M_PI * g.ke / g.V) * qi * (scal[4 * r + 2] + rsum[8 * r + 0]);
  const float lx = (float)(g.Lx * 0x1.0p-32), ly = (float)(g.Ly * 0x1.0p-32), lz = (float)(g.Lz * 0x1.0p-32);
  const float a1 = (float)g.alpha, a2 = (float)(1.0 / g.eta), rc2 = (float)(g.rc * g.rc);
  float fx = 0.f, fy = 0.f, fz = 0.f, ph = 0.f;
  for (int64_t j = b0; j < b1; ++j) {
    const uint4 p = ion_fx[j];
    const float dx = (float)(int32_t)(pi_.x - p.x) * lx;
    const float dy = (float)(int32_t)(pi_.y - p.y) * ly;
    const float dz = (float)(int32_t)(pi_.z - p.z) * lz;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2 && j != i) {
      const float rr = sqrtf(r2);
      float f, df;
      erfc_over_r_f(a1, rr, f, df);
      const float qj = __uint_as_float(p.w);
      ph = fmaf(qj, f, ph);
      const float s = -qj * df / rr;
      fx = fmaf(s, dx, fx);
      fy = fmaf(s, dy, fy);
      fz = fmaf(s, dz, fz);
    }
  }
  const int n = g.n_ele;
  const float* Qr = Qf + (size_t)r * n;
  for (int e = 0; e < n; ++e) {
    const uint4 p = ele_fx[e];
    const float dx = (float)(int32_t)(pi_.x - p.x) * lx;
    const float dy = (float)(int32_t)(pi_.y - p.y) * ly;
    const float dz = (float)(int32_t)(pi_.z - p.z) * lz;
    const float r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const float rr = sqrtf(r2);
      float f1, d1, f2, d2;
      erfc_over_r_f(a1, rr, f1, d1);
      erfc_over_r_f(a2, rr, f2, d2);
      const float s = -Qr[e] * (d1 - d2) / rr;
      fx = fmaf(s, dx, fx);
      fy = fmaf(s, dy, fy);
      fz = fmaf(s, dz, fz);
    }
  }
  const double kq = g.ke * qi;
  F[i] = Fx + kq * (double)fx;
  F[N + i] = Fy + kq * (double)fy;
  F[2 * N + i] = Fz + kq * (double)fz;
  phi[i] = g.ke * (double)ph;
}

void launch_ion_force(const Geom& g, const StepBufs& b, int fp32, hipStream_t s) {
  if (b.max_nrep == 0) return;
  dim3 grid(cdiv64(b.max_nrep, 256), b.R);
  if (fp32)
    hipLaunchKernelGGL(k_ionforce32, grid, dim3(256), 0, s, g, b.off, b.ion_fx, b.N, b.ele_fx, b.Qf, b.rec, b.scal,
                       b.rsum, b.F_out, b.phi);
  else
    hipLaunchKernelGGL(k_ionforce64, grid, dim3(256), 0, s, g, b.off, b.ion_xyz, b.ion_q, b.ion_frac, b.N, b.ele_xyz,
                       b.Q_out, b.modes, b.coef, b.scal, b.rsum, b.F_out, b.phi);
}

// ============================================================ energy
// E* = 1/2 dpsi d.Q - 1/2 b*.Q + c*,  c* = 1/2 sum_i q_i phi_i + 1/2 sum_k w_k |S1_k|^2
//      - ke alpha/sqrt(pi) sum q^2 + ke (2 pi / V) (sum q z)^2
// (1/2 Q^T A Q - b*^T Q + c* at the constrained charges, where Q^T A Q = b*.Q + dpsi d.Q).
__global__ __launch_bounds__(256) void k_energy(Geom g, const int64_t* __restrict__ off,
                                                const double* __restrict__ ion_q, const double* __restrict__ phi,
                                                const double2* __restrict__ S1, const double* __restrict__ w,
                                                const double* __restrict__ scal, const double* __restrict__ rsum,
                                                const double* __restrict__ dpsi, double* __restrict__ energy,
                                                int fixedQ, unsigned* status) {
  __shared__ double sh[2][256];
  const int r = blockIdx.x;
  double v[2] = {0.0, 0.0};
  for (int64_t i = off[r] + threadIdx.x; i < off[r + 1]; i += 256) v[0] += ion_q[i] * phi[i];
  for (int k = threadIdx.x; k < g.K; k += 256) {
    const double2 s = S1[(size_t)r * g.K + k];
    v[1] += w[(size_t)r * g.K + k] * (s.x * s.x + s.y * s.y);
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0) {
    const double c = 0.5 * v[0] + 0.5 * v[1] - g.ke * g.alpha * INV_SQRT_PI * scal[4 * r + 3] +
                     g.ke * (2.0 * M_PI / g.V) * scal[4 * r + 2] * scal[4 * r + 2];
    const double E = 0.5 * dpsi[r] * rsum[8 * r + 1] - 0.5 * rsum[8 * r + 2] + c;
    if (!fixedQ && !isfinite(E)) atomicOr(status, ST_NUMERIC);
    energy[r] = fixedQ ? (double)NAN : E;
  }
}

void launch_energy(const Geom& g, const StepBufs& b, int fixedQ, hipStream_t s) {
  if (!b.energy_out) return;
  hipLaunchKernelGGL(k_energy, dim3(b.R), dim3(256), 0, s, g, b.off, b.ion_q, b.phi, b.S1, b.w, b.scal, b.rsum,
                     b.dpsi, b.energy_out, fixedQ, b.status);
}

}  // namespace srbe
