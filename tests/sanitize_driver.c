/* Memory-safety driver for the oracle (test code, CPU only).
 *
 * Built together with oracle/eik_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py, it runs every
 * oracle entry point on seeded random problems -- degenerate shapes (1 x 1,
 * one row, one column), obstacles, unreachable pockets, several exit nodes
 * with duplicates, cells of every side from 1 to beyond the grid -- and
 * checks the relations that must hold between them (every exact method
 * equal to Fast Marching, the approximate ones above it).  Any sanitizer
 * report aborts the process; a failed relation exits with status 1. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "eik_oracle.h"

static uint64_t rs = 0x9e3779b97f4a7c15ull;
static uint64_t rnd(void) {  /* xorshift64* */
  rs ^= rs >> 12;
  rs ^= rs << 25;
  rs ^= rs >> 27;
  return rs * 0x2545f4914f6cdd1dull;
}
static double unif(void) { return (double)(rnd() >> 11) / 9007199254740992.0; }
static int irange(int lo, int hi) { return lo + (int)(rnd() % (uint64_t)(hi - lo + 1)); }

static int fails = 0;
#define CHECK(c, ...)                 \
  do {                                \
    if (!(c)) {                       \
      fprintf(stderr, __VA_ARGS__);   \
      fprintf(stderr, "\n");          \
      fails++;                        \
    }                                 \
  } while (0)

static double maxrel(const double* a, const double* b, long n) {
  double m = 0.0;
  for (long k = 0; k < n; ++k) {
    if (isinf(a[k]) || isinf(b[k])) {
      if (a[k] != b[k]) return INFINITY;
      continue;
    }
    double d = fabs(a[k] - b[k]) / (fabs(b[k]) > 1e-300 ? fabs(b[k]) : 1e-300);
    if (d > m) m = d;
  }
  return m;
}

static void run2d(int nx, int ny) {
  long n = (long)nx * ny;
  double* F = malloc(sizeof(double) * n);
  uint8_t* M = malloc(n);
  int ns = irange(1, 4);
  int64_t src[5];
  double q[5];
  for (long k = 0; k < n; ++k) {
    F[k] = 0.25 + 1.75 * unif();
    M[k] = unif() > 0.2;
  }
  for (int s = 0; s < ns; ++s) {
    src[s] = (int64_t)(rnd() % (uint64_t)n);
    M[src[s]] = 1;
    q[s] = 0.1 * unif();
  }
  src[ns] = src[0];  /* a duplicate exit node: the smaller cost counts */
  q[ns] = q[0] + 0.05;
  ns++;
  orc_problem p = {nx, ny, 1.0 / (nx > ny ? nx : ny), F, M, ns, src, q};
  double *U = malloc(sizeof(double) * n), *V = malloc(sizeof(double) * n);
  double* r = malloc(sizeof(double) * n);
  int64_t* ord = malloc(sizeof(int64_t) * n);
  int64_t na = 0;
  int32_t it = 0;
  CHECK(orc_fmm(&p, U, ord, &na) == 0, "fmm %dx%d", nx, ny);
  CHECK(orc_residual(&p, U, r) <= 1e-13, "residual %dx%d", nx, ny);
  if (n <= 900) {
    CHECK(orc_jacobi(&p, V, &it) == 0 && maxrel(V, U, n) <= 1e-12, "jacobi %dx%d", nx, ny);
  }
  CHECK(orc_fsm(&p, V, &it) == 0 && maxrel(V, U, n) <= 1e-12, "fsm %dx%d", nx, ny);
  CHECK(orc_lsm(&p, V, &it) == 0 && maxrel(V, U, n) <= 1e-12, "lsm %dx%d", nx, ny);
  uint8_t* unl = malloc(n);
  double mx = 0;
  int64_t cnt = 0;
  orc_sweep_init(&p, V, unl);
  for (int s = 0; s < 6; ++s) orc_fsm_sweep(&p, V, s, &mx, &cnt);
  orc_sweep_init(&p, V, unl);
  for (int s = 0; s < 6; ++s) orc_lsm_sweep(&p, V, unl, s, &mx, &cnt);
  int sides[] = {1, 2, 3, 4, 7, 16, 64, 1000};
  for (int t = 0; t < 8; ++t) {
    int s = sides[t];
    orc_cell_stats st;
    CHECK(orc_hcm(&p, s, 0, V, &st) == 0 && maxrel(V, U, n) <= 1e-12, "hcm %dx%d s=%d", nx, ny, s);
    CHECK(orc_hcm(&p, s, 1, V, &st) == 0, "fhcm %dx%d s=%d", nx, ny, s);
    for (long k = 0; k < n; ++k) CHECK(V[k] >= U[k] * (1 - 1e-14), "fhcm below exact");
    int32_t kx = orc_tiling(nx, s, NULL), ky = orc_tiling(ny, s, NULL);
    int64_t* order = malloc(sizeof(int64_t) * kx * ky);
    double* cu = malloc(sizeof(double) * kx * ky);
    CHECK(orc_fmsm(&p, s, V, order, cu, &st) == 0, "fmsm %dx%d s=%d", nx, ny, s);
    for (long k = 0; k < n; ++k) CHECK(V[k] >= U[k] * (1 - 1e-14), "fmsm below exact");
    free(order);
    free(cu);
  }
  for (int sd = 0; sd < 16; ++sd) (void)orc_fmsm_dirs(sd);
  free(F); free(M); free(U); free(V); free(r); free(ord); free(unl);
}

static void run3d(int nx, int ny, int nz) {
  long n = (long)nx * ny * nz;
  double* F = malloc(sizeof(double) * n);
  uint8_t* M = malloc(n);
  int ns = irange(1, 3);
  int64_t src[3];
  for (long k = 0; k < n; ++k) {
    F[k] = 0.5 + unif();
    M[k] = unif() > 0.15;
  }
  for (int s = 0; s < ns; ++s) {
    src[s] = (int64_t)(rnd() % (uint64_t)n);
    M[src[s]] = 1;
  }
  orc3_problem p = {nx, ny, nz, 0.1, F, M, ns, src, NULL};
  double *U = malloc(sizeof(double) * n), *V = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
  int64_t* ord = malloc(sizeof(int64_t) * n);
  int64_t na;
  int32_t it;
  CHECK(orc3_fmm(&p, U, ord, &na) == 0, "fmm3");
  CHECK(orc3_residual(&p, U, r) <= 1e-13, "residual3");
  CHECK(orc3_fsm(&p, V, &it) == 0 && maxrel(V, U, n) <= 1e-12, "fsm3");
  if (n <= 4000) CHECK(orc3_jacobi(&p, V, &it) == 0 && maxrel(V, U, n) <= 1e-12, "jacobi3");
  int sides[] = {1, 2, 3, 8, 100};
  for (int t = 0; t < 5; ++t) {
    int s = sides[t];
    long J = (long)((nx + s - 1) / s) * ((ny + s - 1) / s) * ((nz + s - 1) / s);
    int64_t* order = malloc(sizeof(int64_t) * J);
    double* cu = malloc(sizeof(double) * J);
    orc_cell_stats st;
    CHECK(orc3_fmsm(&p, s, V, order, cu, &st) == 0, "fmsm3 s=%d", s);
    for (long k = 0; k < n; ++k) CHECK(V[k] >= U[k] * (1 - 1e-14), "fmsm3 below exact");
    free(order);
    free(cu);
  }
  for (int f = 0; f < 64; ++f) (void)orc3_fmsm_orderings(f, f & 7);
  free(F); free(M); free(U); free(V); free(r); free(ord);
}

int main(int argc, char** argv) {
  int rounds = argc > 1 ? atoi(argv[1]) : 40;
  run2d(1, 1);
  run2d(1, 17);
  run2d(23, 1);
  run2d(2, 2);
  for (int k = 0; k < rounds; ++k) run2d(irange(1, 40), irange(1, 40));
  run3d(1, 1, 1);
  run3d(1, 9, 1);
  for (int k = 0; k < rounds / 4; ++k) run3d(irange(1, 14), irange(1, 14), irange(1, 14));
  (void)orc_update(INFINITY, INFINITY, 0.1);
  (void)orc3_update(1.0, INFINITY, INFINITY, 0.1);
  printf("%s: %d failed checks\n", fails ? "FAIL" : "ok", fails);
  return fails ? 1 : 0;
}
