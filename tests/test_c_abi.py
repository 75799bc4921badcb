"""The C ABI used from C: a C99 program (no Python, no torch) includes amrx.h, links libamrx.so
and runs the host-only calls: create, add patches, finalize, error codes and text, clustering."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB_DIR = os.path.join(ROOT, "paper_1112_1710_amd")

SRC = r"""
#include <stdio.h>
#include <string.h>
#include "amrx.h"

int main(void) {
  amrx_desc d;
  memset(&d, 0, sizeof d);
  d.root_n[0] = d.root_n[1] = d.root_n[2] = 16;
  d.max_level = 1;
  d.ratio = 2;
  d.nghost = 4;
  d.gamma = 5.0 / 3.0;
  d.cfl = 0.4;
  d.precision = AMRX_FP32;
  d.stream = NULL;
  amrx_hier* h = NULL;
  if (hier_create(&d, &h) != AMRX_OK) return 1;
  int lo0[3] = {0, 0, 0}, hi0[3] = {16, 16, 16}, lo1[3] = {8, 8, 8}, hi1[3] = {20, 20, 18}, id = -1;
  if (patch_add(h, 0, lo0, hi0, &id) != AMRX_OK || id != 0) return 2;
  if (patch_add(h, 1, lo1, hi1, &id) != AMRX_OK || id != 1) return 3;
  int bad_lo[3] = {0, 0, 0}, bad_hi[3] = {4, 4, 4};  /* touches the root boundary: breaks nesting */
  if (patch_add(h, 1, bad_lo, bad_hi, &id) != AMRX_ENEST) return 4;
  if (strlen(hier_last_error(h)) == 0) return 5;
  size_t sb = 0, cb = 0;
  if (hier_finalize(h, &sb, &cb) != AMRX_OK || sb == 0 || cb == 0) return 6;
  if (hier_finalize(h, &sb, &cb) != AMRX_ESTATE) return 7;
  unsigned char f[4 * 4 * 8];
  memset(f, 0, sizeof f);
  f[0] = f[sizeof f - 1] = 1;
  int boxes[6 * 8], nb = 0;
  if (amrx_cluster(f, 8, 4, 4, 2, 0.7, boxes, 8, &nb) != AMRX_OK || nb < 1) return 8;
  if (hier_destroy(h) != AMRX_OK) return 9;
  printf("ok %zu %zu %d\n", sb, cb, nb);
  return 0;
}
"""


def test_c_program_drives_the_host_calls(tmp_path):
    lib = os.path.join(LIB_DIR, "libamrx.so")
    if not os.path.exists(lib):
        pytest.skip("libamrx.so not built")
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(SRC)
    exe = tmp_path / "abi"
    build = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                            os.path.join(ROOT, "include"), str(src), "-L", LIB_DIR, "-lamrx",
                            "-Wl,-rpath," + LIB_DIR, "-o", str(exe)], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr)
    assert run.stdout.startswith("ok ")
