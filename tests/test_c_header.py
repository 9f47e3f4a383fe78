"""The boundary is a C ABI: a C99 program that includes rpa.h, links the
library and calls its host-side entry points (no GPU needed)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2609_16408_amd")

PROGRAM = r"""
#include <stdio.h>
#include <math.h>
#include "rpa.h"

int main(void) {
  double om[8], w[8];
  if (rpa_frequency_rule(8, om, w) != RPA_OK) return 1;
  /* mapped Gauss-Legendre rule: sum_k w_k / (1 + omega_k)^2 = 1 exactly */
  double s = 0.0;
  for (int k = 0; k < 8; ++k) s += w[k] / ((1.0 + om[k]) * (1.0 + om[k]));
  if (fabs(s - 1.0) > 1e-13) return 2;
  if (rpa_frequency_rule(0, om, w) != RPA_E_ARG) return 3;
  rpa_setup_params p = {0};
  p.n[0] = 5; p.n[1] = 12; p.n[2] = 12;
  p.L[0] = p.L[1] = p.L[2] = 10.0;
  p.fd_radius = 6;
  p.n_occ = 2;
  rpa_handle h = 0;
  if (rpa_setup(&p, 0, &h) != RPA_E_ARG || h != 0) return 4;
  if (interpolate(0, RPA_INTERP_TRILINEAR, 2, 1, 0, 0, 0) != RPA_E_ARG) return 5;
  printf("ok %.15f %s\n", s, rpa_last_error(0));
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_program_uses_the_abi(tmp_path):
    lib = os.path.join(PKG, "librpa_mi355x.so")
    if not os.path.exists(lib):
        pytest.skip("library not built")
    src = tmp_path / "use_rpa.c"
    src.write_text(PROGRAM)
    exe = tmp_path / "use_rpa"
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
           "-L", PKG, "-lrpa_mi355x", "-Wl,-rpath," + PKG, "-Wl,-rpath,/opt/rocm/lib", "-lm",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.startswith("ok 1.0000000000000")
