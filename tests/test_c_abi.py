"""The boundary is a C ABI: include/pim.h compiles as strict C11 and a C
program linked against libpim.so runs the host-only entry points (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2604_17109_amd")

C_PROGRAM = r"""
#include <math.h>
#include <stdio.h>
#include <string.h>
#include "pim.h"

int main(void) {
  if (pim_abi_version() != 2) return 1;
  pim_params p;
  memset(&p, 0, sizeof p);
  p.n = 4;
  p.j_scale = 0.5;
  p.xi = 0.5;
  p.levels = 4;
  p.noise = PIM_NOISE_GAUSS;
  p.noise_bits = 8;
  int32_t th[3], um[8];
  if (pim_compile_step(&p, 1.0, 0.3, th, um) != PIM_OK) return 2;
  if (!(th[0] <= th[1] && th[1] <= th[2])) return 3;   /* thresholds are non-decreasing */
  pim_instance* inst = NULL;
  signed char J[16] = {0};
  if (pim_create((const int8_t*)J, NULL, NULL, NULL, &inst) != PIM_ERR_INVALID) return 4;
  if (strstr(pim_last_error(), "params") == NULL) return 5;
  if (inst != NULL) return 6;
  double Jr[4] = {0.0, 1.0, 1.0, 0.0}, Jq[4], scale;
  if (pim_quantize(Jr, 2, PIM_PREC_FP8, Jq, &scale) != PIM_OK) return 7;
  if (fabs(Jq[1] - 1.0) > 1e-6 || Jq[0] != 0.0) return 8;  /* scale is binary32: max |J| / 448 */
  printf("c abi ok\n");
  return 0;
}
"""


def test_header_is_c11_and_host_entry_points_run(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler on this host")
    if not os.path.exists(os.path.join(LIBDIR, "libpim.so")):
        pytest.skip("libpim.so is not built")
    src = tmp_path / "abi.c"
    src.write_text(C_PROGRAM)
    exe = tmp_path / "abi"
    r = subprocess.run([cc, "-std=c11", "-Wall", "-Wextra", "-Werror", f"-I{ROOT}/include", str(src), "-o", str(exe),
                        f"-L{LIBDIR}", "-lpim", f"-Wl,-rpath,{LIBDIR}", "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "c abi ok" in r.stdout, (r.returncode, r.stdout, r.stderr)
