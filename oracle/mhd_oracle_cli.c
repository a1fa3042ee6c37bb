/*
 * mhd_oracle_cli.c -- command-line front end of the CPU oracle (TEST
 * INFRASTRUCTURE ONLY: parity references at full size, CPU baselines).
 *
 *   mhd_oracle --in STATE --out STATE --steps N [--t-stop T] [--threads K]
 *              [--rk 2|3] [--solver hlld|hll] [--recon prim|char]
 *              [--limiter minmod|mc|vanleer] [--emf contact|e0|arith|uct_hll]
 *              [--pfloor P] [--report REPORT.json]
 *
 * STATE is one box in the boundary layout of the library (C order [z][y][x],
 * x fastest, FP64): the 8-byte tag "MHDSTAT1", int32 n[3], double lo[3],
 * hi[3], int32 bc[3], double gamma, cfl, t, then rho, m_x, m_y, m_z, E
 * (nz*ny*nx each) and the face fields B_x (nz*ny*(nx+1)), B_y
 * (nz*(ny+1)*nx), B_z ((nz+1)*ny*nx), all little-endian.  The report holds
 * the step count, the final time, the next time step, the event counters,
 * max|div B|, the wall time of the steps and the thread count.
 */
#include "mhd_oracle.h"

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

static void die(const char *m) {
  fprintf(stderr, "mhd_oracle: %s\n", m);
  exit(2);
}

static void rd(void *p, size_t sz, size_t n, FILE *f) {
  if (fread(p, sz, n, f) != n) die("short read");
}

static void wr(const void *p, size_t sz, size_t n, FILE *f) {
  if (fwrite(p, sz, n, f) != n) die("short write");
}

static int pick(const char *v, const char *const names[], int count, const char *what) {
  for (int i = 0; i < count; i++)
    if (!strcmp(v, names[i])) return i;
  fprintf(stderr, "mhd_oracle: bad %s '%s'\n", what, v);
  exit(2);
}

int main(int argc, char **argv) {
  const char *in = NULL, *out = NULL, *report = NULL;
  long steps = -1;
  double t_stop = 0.0, pfloor = 1e-10;
  int threads = 0, rk = 2, solver = ORC_HLLD, rec = ORC_REC_PRIM, lim = ORC_LIM_MINMOD,
      emf = ORC_EMF_CONTACT;
  static const char *const solvers[] = {"hlld", "hll"};
  static const char *const recs[] = {"prim", "char"};
  static const char *const lims[] = {"minmod", "mc", "vanleer"};
  static const char *const emfs[] = {"contact", "e0", "arith", "uct_hll"};
  for (int i = 1; i < argc; i++) {
    const char *a = argv[i];
    if (i + 1 >= argc) die("missing value");
    const char *v = argv[++i];
    if (!strcmp(a, "--in")) in = v;
    else if (!strcmp(a, "--out")) out = v;
    else if (!strcmp(a, "--report")) report = v;
    else if (!strcmp(a, "--steps")) steps = atol(v);
    else if (!strcmp(a, "--t-stop")) t_stop = atof(v);
    else if (!strcmp(a, "--threads")) threads = atoi(v);
    else if (!strcmp(a, "--rk")) rk = atoi(v);
    else if (!strcmp(a, "--pfloor")) pfloor = atof(v);
    else if (!strcmp(a, "--solver")) solver = pick(v, solvers, 2, "solver");
    else if (!strcmp(a, "--recon")) rec = pick(v, recs, 2, "recon");
    else if (!strcmp(a, "--limiter")) lim = pick(v, lims, 3, "limiter");
    else if (!strcmp(a, "--emf")) emf = pick(v, emfs, 4, "emf");
    else die("unknown option");
  }
  if (!in || !out || steps < 0) die("--in, --out and --steps are required");
  FILE *f = fopen(in, "rb");
  if (!f) die("cannot open --in");
  char tag[8];
  int32_t n[3], bc[3];
  double lo[3], hi[3], gamma, cfl, t;
  rd(tag, 1, 8, f);
  if (memcmp(tag, "MHDSTAT1", 8)) die("not a state file");
  rd(n, 4, 3, f);
  rd(lo, 8, 3, f);
  rd(hi, 8, 3, f);
  rd(bc, 4, 3, f);
  rd(&gamma, 8, 1, f);
  rd(&cfl, 8, 1, f);
  rd(&t, 8, 1, f);
  int ni[3] = {n[0], n[1], n[2]}, bci[3] = {bc[0], bc[1], bc[2]};
  orc_box *b = orc_box_new(ni, lo, hi, bci, gamma, cfl, pfloor);
  if (!b) die("bad box");
  if (orc_set_rk(b, rk) || orc_set_solver(b, solver) || orc_set_recon(b, rec) ||
      orc_set_limiter(b, lim) || orc_set_emf(b, emf))
    die("bad scheme option");
  size_t N = (size_t)n[0] * n[1] * n[2];
  size_t F[3] = {(size_t)n[2] * n[1] * (n[0] + 1), (size_t)n[2] * (n[1] + 1) * n[0],
                 (size_t)(n[2] + 1) * n[1] * n[0]};
  double *cons[5], *bface[3];
  for (int q = 0; q < 5; q++) {
    cons[q] = malloc(N * sizeof(double));
    if (!cons[q]) die("out of memory");
    rd(cons[q], 8, N, f);
  }
  for (int d = 0; d < 3; d++) {
    bface[d] = malloc(F[d] * sizeof(double));
    if (!bface[d]) die("out of memory");
    rd(bface[d], 8, F[d], f);
  }
  fclose(f);
  if (orc_set_state(b, (const double *const *)cons, (const double *const *)bface, t))
    die("periodic face mismatch");
  int used = orc_threads(threads);
  struct timespec t0, t1;
  clock_gettime(CLOCK_MONOTONIC, &t0);
  orc_step(b, (int)steps, t_stop);
  clock_gettime(CLOCK_MONOTONIC, &t1);
  double sec = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
  orc_get_state(b, cons, bface, &t);
  f = fopen(out, "wb");
  if (!f) die("cannot open --out");
  wr("MHDSTAT1", 1, 8, f);
  wr(n, 4, 3, f);
  wr(lo, 8, 3, f);
  wr(hi, 8, 3, f);
  wr(bc, 4, 3, f);
  wr(&gamma, 8, 1, f);
  wr(&cfl, 8, 1, f);
  wr(&t, 8, 1, f);
  for (int q = 0; q < 5; q++) wr(cons[q], 8, N, f);
  for (int d = 0; d < 3; d++) wr(bface[d], 8, F[d], f);
  if (fclose(f)) die("write failed");
  if (report) {
    long long c[3];
    orc_counters(b, c);
    FILE *r = fopen(report, "w");
    if (!r) die("cannot open --report");
    fprintf(r,
            "{\"steps\": %ld, \"t\": %.17g, \"dt_next\": %.17g, \"counters\": {\"floor\": %lld, "
            "\"hll\": %lld, \"bad\": %lld}, \"divb_max\": %.17g, \"seconds\": %.6f, "
            "\"mcell_updates_per_s\": %.6f, \"threads\": %d}\n",
            steps, t, orc_dt(b), c[0], c[1], c[2], orc_divb_max(b), sec,
            sec > 0 ? (double)N * (double)steps / sec / 1e6 : 0.0, used);
    fclose(r);
  }
  for (int q = 0; q < 5; q++) free(cons[q]);
  for (int d = 0; d < 3; d++) free(bface[d]);
  orc_box_free(b);
  return 0;
}
