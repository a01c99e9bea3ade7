"""The plain-C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, CPU
only) and driven through every public routine on small 2D and 3D grids, for each coarse
operator, smoother and transfer: no memory or undefined-behaviour error may be reported.
The driver is a small C program written here; the oracle source is compiled unchanged."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "mg_oracle.h"

static double *grid(int dim, int n) { return calloc((size_t)(dim == 2 ? n * n : n * n * n), sizeof(double)); }

static int run(int dim, int n, int order, int coarse, int smoother, int restrict_op, int prolong, int gamma) {
  or_config c = {dim, n, order, coarse, restrict_op, prolong, 2, 1, gamma, 9, 0.8, smoother};
  if (smoother == OR_SMOOTH_RBJ) c.omega = 1.1;
  if (smoother == OR_SMOOTH_RBGS) c.omega = 1.15;
  or_mg *m = or_mg_create(&c);
  if (!m) return 1;
  long np = dim == 2 ? (long)n * n : (long)n * n * n;
  double *f = grid(dim, n), *u = grid(dim, n), *t = grid(dim, n), *d = grid(dim, n);
  for (long p = 0; p < np; ++p) f[p] = (double)((p * 7919) % 101) - 50.0;
  /* zero boundary */
  for (long p = 0; p < np; ++p) {
    long i = p % n, j = (p / n) % n, k = dim == 3 ? p / ((long)n * n) : 1;
    if (i == 0 || i == n - 1 || j == 0 || j == n - 1 || (dim == 3 && (k == 0 || k == n - 1))) f[p] = 0.0;
  }
  double hist[8];
  or_mg_solve(m, u, f, 0.0, 3, hist);
  double s[13 * 13 * 13];
  int nl = 0;
  int R = or_mg_level_stencil(m, 0, &nl, s);
  or_apply(dim, n, R, s, u, t);
  or_residual(dim, n, R, s, f, u, d);
  or_jacobi(dim, n, R, s, 0.8, f, u, t);
  or_jacobi_colour(dim, n, R, s, 1.1, 1, f, u, t);
  or_gs_colour(dim, n, R, s, 1.1, 2, f, u, t);
  int nc = (n - 1) / 2 + 1;
  double *fc = grid(dim, nc);
  or_restrict(dim, n, restrict_op, d, fc);
  or_prolong_add(dim, n, prolong, fc, u);
  double a = or_norm(dim, n, d) + or_residual_norm_ld(dim, n, R, s, f, u);
  for (int l = 1; l < or_mg_levels(m); ++l) or_mg_level_stencil(m, l, &nl, s);
  double *g = grid(dim, 9), *v = grid(dim, 9);
  for (long p = 0; p < (dim == 2 ? 81 : 729); ++p) g[p] = 0.0;
  g[dim == 2 ? 40 : 364] = 1.0;
  or_mg_coarsest_solve(m, g, v);
  or_mg_destroy(m);
  free(f); free(u); free(t); free(d); free(fc); free(g); free(v);
  return a != a;  /* NaN check */
}

int main(void) {
  int bad = 0;
  for (int coarse = 0; coarse <= 3; ++coarse)
    for (int sm = 0; sm <= 2; ++sm) {
      bad |= run(2, 33, 4, coarse, sm, 1, 3, 1 + (coarse & 1));
      bad |= run(2, 17, 6, coarse, sm, 1, 1, 1);
      bad |= run(3, 17, 4, coarse, sm == 2 ? 1 : sm, 1, 3, 1 + (sm & 1));
    }
  bad |= run(2, 33, 4, 0, 0, 3, 3, 1);
  bad |= run(3, 17, 2, 2, 1, 3, 3, 2);
  or_set_num_threads(1);
  bad |= run(3, 17, 4, 1, 0, 1, 3, 2);
  printf("sanitized oracle driver done: %d\n", bad);
  return bad;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    oracle_dir = os.path.join(ROOT, "oracle")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I" + oracle_dir,
           str(src), os.path.join(oracle_dir, "mg_oracle.c"), "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               OMP_NUM_THREADS="2")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "sanitized oracle driver done: 0" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr[-4000:]
