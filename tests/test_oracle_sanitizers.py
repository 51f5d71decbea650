"""The oracle's C built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and driven through every thermal model and side kind:
no out-of-bounds access, leak or undefined behaviour may be reported."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include "lbpo.h"
int main(void) {
  const int nx = 24, ny = 20, n = nx * ny;
  double *rho = malloc(n * sizeof(double)), *ux = calloc(n, sizeof(double)),
         *uy = calloc(n, sizeof(double)), *T = malloc(n * sizeof(double));
  double *f = malloc(9 * n * sizeof(double)), *g = malloc(9 * n * sizeof(double)),
         *ph = malloc(n * sizeof(double)), *tv = malloc(2 * n * sizeof(double));
  for (int model = 0; model < 4; ++model)
    for (int bc = 0; bc < 3; ++bc) {
      lbpo_config c = {0};
      c.a = 3.0 / 49.0; c.b = 2.0 / 21.0; c.R = 1.0; c.omega = 0.344;
      c.cv = 5.0; c.lambda0 = 2.0 / 3.0; c.chi = 0.06; c.G = -1.0;
      c.sigma = 0.105; c.gy = -1e-4;
      for (int k = 0; k < 9; ++k) { c.s_f[k] = 1.1; c.s_g[k] = 1.0; }
      c.nx = nx; c.ny = ny; c.thermal_model = model;
      c.lambda_mode = model == 2 ? 1 : 0;
      for (int s = 0; s < 4; ++s) { c.bc[s] = bc; c.T_bc[s] = 0.1; }
      c.hot_x0 = 8; c.hot_x1 = 12; c.T_hot = 0.105;
      c.rho_v = 0.38; c.rho_l = 6.5;
      for (int i = 0; i < n; ++i) {
        int x = i % nx, y = i / nx;
        double r = sqrt((x - 12.0) * (x - 12.0) + (y - 10.0) * (y - 10.0));
        rho[i] = 3.44 - 3.06 * tanh(0.4 * (r - 5.0));
        T[i] = 0.0940689;
      }
      lbpo_handle *h;
      if (lbpo_create(&c, &h) != LBPO_OK) return 2;
      if (lbpo_init_fields(h, rho, ux, uy, T) != LBPO_OK) return 3;
      if (lbpo_step(h, 25) != LBPO_OK) return 4;
      lbpo_diag d;
      if (lbpo_get_diag(h, &d) != LBPO_OK) return 5;
      int32_t pv; double ra; int64_t st;
      if (lbpo_get_state(h, f, g, ph, &pv, &ra, &st) != LBPO_OK) return 6;
      if (lbpo_get_tv_prev(h, tv) != LBPO_OK) return 7;
      if (lbpo_set_state(h, f, g, ph, pv, ra, st) != LBPO_OK) return 8;
      if (lbpo_set_tv_prev(h, tv) != LBPO_OK) return 9;
      if (lbpo_step(h, 5) != LBPO_OK) return 10;
      if (lbpo_get_rho_u_T(h, rho, ux, uy, T) != LBPO_OK) return 11;
      for (int i = 0; i < n; ++i) { ux[i] = 0.0; uy[i] = 0.0; }
      lbpo_destroy(h);
      for (int i = 0; i < n; ++i) T[i] = 0.0940689;
    }
  free(rho); free(ux); free(uy); free(T); free(f); free(g); free(ph); free(tv);
  puts("ok");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "drv.c")
        exe = os.path.join(d, "drv")
        with open(drv, "w") as fh:
            fh.write(DRIVER)
        subprocess.check_call(
            ["gcc", "-O1", "-g", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             "-I", ORACLE, drv, os.path.join(ORACLE, "lbpo.c"), "-lm",
             "-o", exe])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        env.pop("LD_PRELOAD", None)
        r = subprocess.run([exe], capture_output=True, text=True, env=env,
                           timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.strip() == "ok"
        assert "runtime error" not in r.stderr, r.stderr
