// Drives the library's host code as the tuning tests and the bench did: eager steps in
// both precisions, interleaved with srbe_tune calls (about 70 capture -> instantiate ->
// replay -> destroy cycles each) and srbe_graph_create / destroy, on two handles.
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "srbe.h"
long stub_live(int which);

static srbe_system* make_handle(int P) {
  const int nw = 12, n = 2 * nw * nw;
  std::vector<double> xyz(3 * n);
  std::vector<int8_t> side(n);
  for (int w = 0; w < 2; ++w)
    for (int i = 0; i < nw; ++i)
      for (int j = 0; j < nw; ++j) {
        const int k = w * nw * nw + i * nw + j;
        xyz[k] = 0.2 * i; xyz[n + k] = 0.2 * j; xyz[2 * n + k] = w ? 8.0 : 0.0;
        side[k] = w ? 1 : -1;
      }
  srbe_params p{2.4, 2.4, 8.0, 3.0, 3.0, 1.0 / 19.79, 1.19, 1.43996454784, 1e-16, 10, P, 0, 0};
  srbe_system* h = nullptr;
  const int rc = srbe_create(&p, n, xyz.data(), side.data(), &h);
  if (rc) { fprintf(stderr, "create %d\n", rc); exit(1); }
  return h;
}

int main() {
  srbe_system* hs[2] = {make_handle(100), make_handle(37)};
  const int R = 3, nper = 200, N = R * nper;
  std::vector<int64_t> off(R + 1);
  for (int r = 0; r <= R; ++r) off[r] = (int64_t)r * nper;
  double *xyz, *q, *dpsi, *Q, *F, *b, *psi, *E;
  uint64_t* seed;
  xyz = (double*)malloc(3 * N * 8); q = (double*)malloc(N * 8); dpsi = (double*)malloc(R * 8);
  seed = (uint64_t*)malloc(R * 8);
  Q = (double*)malloc(R * 288 * 8); F = (double*)malloc(3 * N * 8); b = (double*)malloc(R * 288 * 8);
  psi = (double*)malloc(R * 8); E = (double*)malloc(R * 8);
  for (int i = 0; i < 3 * N; ++i) xyz[i] = 1.0;
  for (int i = 0; i < N; ++i) q[i] = (i & 1) ? 0.78 : -0.78;
  for (int r = 0; r < R; ++r) { dpsi[r] = 2.0; seed[r] = 7 + r; }
  int total = 0;
  for (int round = 0; round < 6; ++round)
    for (int hi = 0; hi < 2; ++hi) {
      srbe_system* h = hs[hi];
      for (int prec = 0; prec < 2; ++prec) {
        for (int s = 0; s < 3; ++s)
          if (srbe_step(h, prec, R, off.data(), xyz, q, dpsi, seed, s, nullptr, nullptr, Q, F, b, psi, E, nullptr,
                        nullptr)) { fprintf(stderr, "step: %s\n", srbe_last_error(h)); return 1; }
        int32_t params[SRBE_TUNE_NPARAM];
        double ms[2];
        const int rc = srbe_tune(h, prec, R, off.data(), xyz, q, dpsi, seed, 3, params, ms, nullptr);
        if (rc) { fprintf(stderr, "tune: %d %s\n", rc, srbe_last_error(h)); return 1; }
        srbe_graph* g = nullptr;
        if (srbe_graph_create(h, prec, R, off.data(), xyz, q, dpsi, seed, 0, nullptr, nullptr, Q, F, b, psi, E,
                              nullptr, &g)) { fprintf(stderr, "graph: %s\n", srbe_last_error(h)); return 1; }
        for (int k = 0; k < 4; ++k) srbe_graph_launch(g, nullptr);
        srbe_graph_destroy(g);
        // phase timing on for a few eager steps, then read and off (as the bench does)
        srbe_profile_enable(h, 10);
        for (int s = 0; s < 2 + round; ++s)
          if (srbe_step(h, prec, R, off.data(), xyz, q, dpsi, seed, 100 + s, nullptr, nullptr, Q, F, b, psi, E,
                        nullptr, nullptr)) { fprintf(stderr, "prof step: %s\n", srbe_last_error(h)); return 1; }
        double pms[SRBE_N_PHASES];
        int64_t pn[SRBE_N_PHASES];
        if (srbe_profile_read(h, pms, pn)) { fprintf(stderr, "profile read\n"); return 1; }
        srbe_profile_enable(h, 0);
        ++total;
        printf("round %d handle %d precision %d: tuned ms %.3f -> %.3f, params %d %d %d %d %d %d %d %d\n", round, hi,
               prec, ms[0], ms[1], params[0], params[1], params[2], params[3], params[4], params[5], params[6],
               params[7]);
      }
    }
  srbe_destroy(hs[0]);
  srbe_destroy(hs[1]);
  free(xyz); free(q); free(dpsi); free(seed); free(Q); free(F); free(b); free(psi); free(E);
  printf("%d tune calls; live after destroy: graphs %ld execs %ld events %ld streams %ld allocations %ld\n", total,
         stub_live(0), stub_live(1), stub_live(2), stub_live(3), stub_live(4));
  return 0;
}
