"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code, gcc): a small C driver links oracle.c built with both sanitizers and
calls every entry point the tests use on seeded instances -- both losses, the
three storage types of X, fixed-zero / fixed-one sets, kbar = 0, an infeasible
node, M = +inf, empty and one-coordinate problems, every iteration variant,
warm starts and traces.  Any invalid access, leak or undefined operation
aborts the driver.  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double orc_g(const double *, const int8_t *, int64_t, int32_t);
int orc_in_dom(const double *, const int8_t *, int64_t, int32_t, double, double);
double orc_gstar(const double *, const int8_t *, int64_t, int32_t, double);
void orc_prox_gstar(const double *, const int8_t *, int64_t, double, int32_t, double, double *);
void orc_prox_g(const double *, const int8_t *, int64_t, double, int32_t, double, double *);
void orc_matvec(const void *, int, int64_t, int64_t, const double *, double *);
void orc_rmatvec(const void *, int, int64_t, int64_t, const double *, double *);
double orc_power_norm2(const void *, int, int64_t, int64_t, int64_t, double);
double orc_primal(const void *, int, const double *, int64_t, int64_t, int, double, double, int32_t,
                  const int8_t *, const double *);
double orc_dual(const void *, int, const double *, int64_t, int64_t, int, double, double, int32_t,
                const int8_t *, const double *);
int orc_solve(const void *, int, const double *, int64_t, int64_t, int, double, double, int32_t,
              const int8_t *, double, double, double, int64_t, double, const double *, double *,
              double *, double *, double *, int64_t, int, double *, int64_t *, int64_t);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static double urand(void) {  /* xorshift64*, uniform in [0, 1) */
  state ^= state >> 12; state ^= state << 25; state ^= state >> 27;
  return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) / 9007199254740992.0;
}
static double nrand(void) { return sqrt(-2.0 * log(1.0 - urand())) * cos(6.283185307179586 * urand()); }

static void *make_x(int xdt, int64_t n, int64_t p) {
  const int64_t m = n * p > 0 ? n * p : 1;
  if (xdt == 0) { double *x = malloc(sizeof(double) * m); for (int64_t i = 0; i < n * p; i++) x[i] = nrand(); return x; }
  if (xdt == 1) { float *x = malloc(sizeof(float) * m); for (int64_t i = 0; i < n * p; i++) x[i] = (float)nrand(); return x; }
  uint16_t *x = malloc(sizeof(uint16_t) * m);
  for (int64_t i = 0; i < n * p; i++) { float f = (float)nrand(); uint32_t b; memcpy(&b, &f, 4); x[i] = (uint16_t)(b >> 16); }
  return x;
}

static int run_case(int64_t n, int64_t p, int loss, int xdt, int32_t k, double M, int n0, int n1, int method) {
  void *X = make_x(xdt, n, p);
  double *y = malloc(sizeof(double) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) y[i] = loss ? (urand() < 0.5 ? -1.0 : 1.0) : nrand();
  int8_t *st = calloc(p > 0 ? p : 1, 1);
  for (int i = 0; i < n0 && i < p; i++) st[i] = 1;
  for (int i = 0; i < n1 && n0 + i < p; i++) st[n0 + i] = 2;
  double *v = malloc(sizeof(double) * (p > 0 ? p : 1)), *out = malloc(sizeof(double) * (p > 0 ? p : 1));
  for (int64_t j = 0; j < p; j++) v[j] = 3.0 * nrand();
  orc_prox_g(v, st, p, 0.7, k, M, out);
  orc_prox_gstar(v, st, p, 0.7, k, M, out);
  volatile double g = orc_g(out, st, p, k) + orc_gstar(v, st, p, k, M);
  (void)g;
  (void)orc_in_dom(out, st, p, k, M, 1e-9);
  double *u = malloc(sizeof(double) * (n > 0 ? n : 1)), *h = malloc(sizeof(double) * (p > 0 ? p : 1));
  orc_matvec(X, xdt, n, p, v, u);
  orc_rmatvec(X, xdt, n, p, u, h);
  double L = (loss ? 0.25 : 2.0) * orc_power_norm2(X, xdt, n, p, 200, 1e-10) * 1.01 + 1e-12;
  double *beta = malloc(sizeof(double) * (p > 0 ? p : 1)), *zeta = malloc(sizeof(double) * (n > 0 ? n : 1));
  double res[8], tr[64], ptr[64];
  int64_t rst[16];
  int rc = orc_solve(X, xdt, y, n, p, loss, 0.5, M, k, st, L, 1e-7, exp(3.0), 300, NAN, NULL, beta, zeta, res,
                     tr, 64, method, ptr, rst, 16);
  /* warm start from the solution, with a cutoff */
  rc |= orc_solve(X, xdt, y, n, p, loss, 0.5, M, k, st, L, 1e-7, exp(3.0), 50, res[1], beta, out, zeta, res,
                  NULL, 0, method, NULL, NULL, 0);
  volatile double pd = orc_primal(X, xdt, y, n, p, loss, 0.5, M, k, st, out) +
                       orc_dual(X, xdt, y, n, p, loss, 0.5, M, k, st, zeta);
  (void)pd;
  free(X); free(y); free(st); free(v); free(out); free(u); free(h); free(beta); free(zeta);
  return rc < 0 ? 1 : 0;
}

int main(void) {
  int bad = 0;
  const double Ms[3] = {2.0, 0.5, INFINITY};
  for (int xdt = 0; xdt < 3; xdt++)
    for (int loss = 0; loss < 2; loss++)
      for (int method = 0; method < 4; method++) {
        bad |= run_case(40, 13, loss, xdt, 3, Ms[method % 3], 2, 1, method);  /* J0, J1 */
        bad |= run_case(25, 30, loss, xdt, 2, Ms[(method + 1) % 3], 0, 2, method); /* kbar = 0 */
      }
  bad |= run_case(30, 8, 0, 0, 2, 2.0, 0, 3, 0);   /* |J1| > k: infeasible */
  bad |= run_case(12, 1, 0, 0, 1, 2.0, 0, 0, 0);   /* one coordinate */
  bad |= run_case(12, 5, 1, 1, 9, 2.0, 0, 0, 0);   /* k >= p */
  bad |= run_case(9, 6, 0, 2, 3, 2.0, 6, 0, 0);    /* every coordinate fixed to zero */
  printf("sanitized oracle driver done: %d\n", bad);
  return bad;
}
"""


def test_oracle_runs_clean_under_address_and_undefined_behavior_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wno-unknown-pragmas",
           "-o", str(exe), ORACLE_C, str(drv), "-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    if b.returncode != 0 and "asan" in (b.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not installed: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized oracle driver done: 0" in r.stdout
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
