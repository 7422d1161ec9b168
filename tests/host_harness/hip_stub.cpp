// Host stubs of the HIP runtime, rocBLAS/rocSOLVER and the library's launch functions,
// so that srbe_api.hip's host code (set-up, steps, graph capture, tuner) can run on the
// CPU under AddressSanitizer.  "Device" memory is host heap memory.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "kernels.h"

static int g_capturing = 0;
static hipStream_t g_cap_stream = nullptr;
static double g_clock = 0.0;
static long g_graph_live = 0, g_exec_live = 0, g_events_live = 0, g_streams_live = 0, g_allocs_live = 0;

extern "C" {
hipError_t hipMalloc(void** p, size_t n) { *p = aligned_alloc(256, ((n ? n : 1) + 255) / 256 * 256); ++g_allocs_live; return hipSuccess; }
hipError_t hipFree(void* p) { if (p) { free(p); --g_allocs_live; } return hipSuccess; }
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void* p, hipStream_t) { return hipFree(p); }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { if (n) memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) { if (n) memcpy(d, s, n); return hipSuccess; }
hipError_t hipMemset(void* d, int v, size_t n) { memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub"; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = (hipStream_t) new char[32]; ++g_streams_live; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete[] (char*)s; --g_streams_live; return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t e, unsigned) { volatile char c = ((char*)e)[0]; (void)c; return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t) new char[64](); ++g_events_live; return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { delete[] (char*)e; --g_events_live; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { g_clock += 0.01; memcpy((char*)e, &g_clock, sizeof(double)); return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t e) { volatile char c = ((char*)e)[0]; (void)c; return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  double ta, tb; memcpy(&ta, a, 8); memcpy(&tb, b, 8); *ms = (float)(tb - ta + 0.001 * (rand() % 100)); return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  if (g_capturing) { fprintf(stderr, "nested capture\n"); abort(); }
  g_capturing = 1; g_cap_stream = s; return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  if (!g_capturing || s != g_cap_stream) { fprintf(stderr, "end capture on another stream\n"); abort(); }
  g_capturing = 0; *g = (hipGraph_t) new char[128](); ++g_graph_live; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  volatile char c = ((char*)g)[0]; (void)c; *x = (hipGraphExec_t) new char[128](); ++g_exec_live; return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t) { volatile char c = ((char*)x)[127]; (void)c; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { delete[] (char*)x; --g_exec_live; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete[] (char*)g; --g_graph_live; return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = (void*)sym; return hipSuccess; }
void** __hipRegisterFatBinary(const void*) { static void* h[4]; return h; }
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, char*, char*, const char*, int, size_t, int, int) {}
rocblas_status rocblas_create_handle(rocblas_handle* h) { *h = (rocblas_handle) new char[16]; return rocblas_status_success; }
rocblas_status rocblas_destroy_handle(rocblas_handle h) { delete[] (char*)h; return rocblas_status_success; }
rocblas_status rocblas_set_stream(rocblas_handle, hipStream_t) { return rocblas_status_success; }
const char* rocblas_status_to_string(rocblas_status) { return "stub"; }
rocblas_status rocblas_dsyrk(rocblas_handle, rocblas_fill, rocblas_operation, rocblas_int n, rocblas_int k,
                             const double*, const double*, rocblas_int, const double*, double* C, rocblas_int ldc) {
  for (int j = 0; j < n; ++j) C[(size_t)j * ldc + j] += 1.0;  // keep A positive definite
  (void)k; return rocblas_status_success; }
rocblas_status rocsolver_dpotrf(rocblas_handle, rocblas_fill, rocblas_int, double*, rocblas_int, rocblas_int* info) {
  *info = 0; return rocblas_status_success; }
rocblas_status rocsolver_dpotri(rocblas_handle, rocblas_fill, rocblas_int, double*, rocblas_int, rocblas_int* info) {
  *info = 0; return rocblas_status_success; }
}

namespace srbe {
void lattice_grid(const StepBufs&, int, int& blocks, size_t& lds) { blocks = 1; lds = 0; }
size_t sample_lds_bytes(int P) { return (size_t)P * 26 + 16; }
int cp_gemm_ksplit(int, int) { return 7; }
int ele_split(int) { return 1; }
bool use_big_sort(const Geom&, int64_t) { return false; }
size_t virial_scratch_doubles(const Geom&, const StepBufs&) { return 1; }
void launch_multi(int, int, int, int, int, const MultiLaunch&, int, size_t, hipStream_t) {}
void launch_multi_lattice(int, const MultiLaunch&, int, size_t, hipStream_t) {}
void launch_front(const Geom&, const StepBufs&, int, int, hipStream_t) {}
void launch_set_step(uint64_t* p, uint64_t v, hipStream_t) { *p = v; }
void launch_logq_table(const Geom&, double*, hipStream_t) {}
void launch_stage_ions(const Geom&, const StepBufs&, int, int, hipStream_t) {}
void launch_sf_finalize(const Geom&, const StepBufs&, int, int, hipStream_t) {}
void launch_ele_potential(const Geom&, const StepBufs&, int, hipStream_t) {}
void launch_cp_gemm(const Geom&, const StepBufs&, const double*, hipStream_t) {}
void launch_lattice_solve(const Geom&, const StepBufs&, hipStream_t) {}
void launch_ff_forces(const Geom&, const StepBufs&, const FFParams&, const int*, const int*, const double*, double*,
                      double*, hipStream_t) {}
void launch_langevin(int64_t, double*, double*, const double*, const double*, double, double, double, double, double,
                     double, double, uint64_t, uint64_t, hipStream_t, const uint64_t*, int) {}
void launch_electrode_forces(const Geom&, const StepBufs&, int, double*, int64_t*, void*, hipStream_t) {}
void launch_post_charges(const Geom&, const StepBufs&, int, int, hipStream_t) {}
void launch_ele_pair_energy(const Geom&, const StepBufs&, hipStream_t) {}
void launch_virial(const Geom&, const StepBufs&, double*, double*, hipStream_t) {}
void launch_stage_ele(const Geom&, const StepBufs&, int, int, hipStream_t) {}
void launch_ion_force(const Geom&, const StepBufs&, int, hipStream_t) {}
void launch_real_ii(const Geom&, const StepBufs&, int, hipStream_t) {}
void launch_final(const Geom&, const StepBufs&, int, hipStream_t) {}
// set-up: every electrode in cell 0, identity order
void launch_bin_electrodes(const Geom& g, const int64_t*, const double* ele_xyz, int n, unsigned*, uint4* fx,
                           double4* d4, int* perm, int* scell, int* cstart, uint4* sfx, double4* sd4, unsigned*,
                           const BigSort&, hipStream_t) {
  for (int k = 0; k < n; ++k) {
    perm[k] = k; scell[k] = 0;
    fx[k] = make_uint4(0, 0, 0, 0); sfx[k] = fx[k];
    d4[k] = make_double4(ele_xyz[k] / g.Lx, ele_xyz[n + k] / g.Ly, ele_xyz[2 * n + k] / g.Lz, 0.0); sd4[k] = d4[k];
  }
  cstart[0] = 0;
  for (int c = 1; c <= g.ncell; ++c) cstart[c] = n;
}
void launch_cell_zrange(const Geom& g, const int* cstart, const double* ele_xyz, const int* perm, double2* zr,
                        hipStream_t) {
  const int n = cstart[g.ncell];
  for (int c = 0; c < g.ncell; ++c) zr[c] = make_double2(1e300, -1e300);
  for (int k = 0; k < n; ++k) {
    const double z = ele_xyz[2 * n + perm[k]];
    zr[0].x = std::min(zr[0].x, z); zr[0].y = std::max(zr[0].y, z);
  }
}
void launch_ele_phase_block(const double*, int, const int*, const double*, int, int, double*, const Geom&, hipStream_t) {}
void launch_ele_realspace_matrix(const Geom&, const double*, int, double*, hipStream_t) {}
void launch_symmetrize_lower(double*, int, int, hipStream_t) {}
void launch_rowsum(const double* A, int n, int ld, double* out, hipStream_t) {
  for (int i = 0; i < n; ++i) out[i] = 1.0 + 0 * A[(size_t)i * ld];
}
void launch_build_sext(const double*, int, const double*, double, double*, hipStream_t) {}
void launch_check_finite(const double*, size_t, unsigned*, hipStream_t) {}
}  // namespace srbe

long stub_live(int which) {
  switch (which) {
    case 0: return g_graph_live;
    case 1: return g_exec_live;
    case 2: return g_events_live;
    case 3: return g_streams_live;
    default: return g_allocs_live;
  }
}
