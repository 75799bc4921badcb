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


GPU_SRC = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <hip/hip_runtime_api.h>
#include "amrx.h"

/* uniform state (rho, mx, my, mz, E, bx, by, bz) */
static const double U0[8] = {1.25, 0.25, -0.5, 0.125, 2.0, 0.5, 0.75, -0.25};

static int fill(amrx_hier* h, char* state, int pid) {
  size_t off[8];
  int dims[3], which;
  if (patch_current(h, pid, &which) != AMRX_OK || patch_layout(h, pid, which, off, dims) != AMRX_OK) return 1;
  const size_t n = (size_t)dims[0] * dims[1] * dims[2];
  double* buf = (double*)malloc(n * sizeof(double));
  for (int m = 0; m < 8; ++m) {
    for (size_t i = 0; i < n; ++i) buf[i] = U0[m];
    if (hipMemcpy(state + off[m], buf, n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) return 2;
  }
  free(buf);
  return 0;
}

/* largest relative deviation from U0 over the interior cells and the interior face closures */
static double deviation(amrx_hier* h, char* state, int pid, const int n[3]) {
  size_t off[8];
  int dims[3], which;
  if (patch_current(h, pid, &which) != AMRX_OK || patch_layout(h, pid, which, off, dims) != AMRX_OK) return 1e300;
  const size_t len = (size_t)dims[0] * dims[1] * dims[2];
  double* buf = (double*)malloc(len * sizeof(double));
  double worst = 0.0;
  for (int m = 0; m < 8; ++m) {
    if (hipMemcpy(buf, state + off[m], len * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return 1e300;
    int top[3] = {4 + n[0], 4 + n[1], 4 + n[2]};
    if (m >= 5) top[m - 5] += 1;
    for (int k = 4; k < top[2]; ++k)
      for (int j = 4; j < top[1]; ++j)
        for (int i = 4; i < top[0]; ++i) {
          const double x = buf[((size_t)k * dims[1] + j) * dims[0] + i];
          const double d = fabs(x - U0[m]) / (fabs(U0[m]) + 1e-300);
          if (!(d <= worst)) worst = d;
        }
  }
  free(buf);
  return worst;
}

int main(void) {
  amrx_desc d;
  memset(&d, 0, sizeof d);
  d.root_n[0] = d.root_n[1] = d.root_n[2] = 16;
  d.max_level = 1;
  d.ratio = 2;
  d.nghost = 4;
  d.gamma = 5.0 / 3.0;
  d.cfl = 0.4;
  d.precision = AMRX_FP64;
  amrx_hier* h = NULL;
  if (hier_create(&d, &h) != AMRX_OK) return 1;
  int lo0[3] = {0, 0, 0}, hi0[3] = {16, 16, 16}, lo1[3] = {8, 8, 8}, hi1[3] = {20, 20, 18}, id;
  if (patch_add(h, 0, lo0, hi0, &id) != AMRX_OK || patch_add(h, 1, lo1, hi1, &id) != AMRX_OK) return 2;
  size_t sb = 0, cb = 0;
  if (hier_finalize(h, &sb, &cb) != AMRX_OK) return 3;
  void *state = NULL, *scratch = NULL;
  if (hipMalloc(&state, sb) != hipSuccess || hipMalloc(&scratch, cb) != hipSuccess) return 4;
  if (hier_bind(h, state, sb, scratch, cb) != AMRX_OK) { fprintf(stderr, "%s\n", hier_last_error(h)); return 5; }
  if (fill(h, (char*)state, 0) || fill(h, (char*)state, 1)) return 6;
  double dt0 = 0.0;
  if (hier_step(h, AMRX_BATCHED, &dt0) != AMRX_OK) { fprintf(stderr, "%s\n", hier_last_error(h)); return 7; }
  if (hipDeviceSynchronize() != hipSuccess) return 8;
  /* closed form: dt0 = C dx0 / sum_d (|v_d| + c_f,d), the same on every level (dt_l = 2^-l dt0) */
  const double g = d.gamma, r = U0[0];
  const double v[3] = {U0[1] / r, U0[2] / r, U0[3] / r}, b[3] = {U0[5], U0[6], U0[7]};
  const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  const double p = (g - 1.0) * (U0[4] - 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 0.5 * b2);
  const double a2 = g * p / r;
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double t = a2 + b2 / r;
    s += fabs(v[a]) + sqrt(0.5 * (t + sqrt(t * t - 4.0 * a2 * b[a] * b[a] / r)));
  }
  const double want = d.cfl * (1.0 / 16.0) / s;
  const int n0[3] = {16, 16, 16}, n1[3] = {12, 12, 10};
  const double e0 = deviation(h, (char*)state, 0, n0), e1 = deviation(h, (char*)state, 1, n1);
  printf("dt0 %.17g want %.17g dev %.3g %.3g\n", dt0, want, e0, e1);
  if (!(fabs(dt0 - want) <= 1e-12 * want)) return 9;
  if (!(e0 <= 1e-13 && e1 <= 1e-13)) return 10;
  hier_destroy(h);
  hipFree(state);
  hipFree(scratch);
  printf("ok\n");
  return 0;
}
"""


def _build_gpu_program(tmp_path):
    lib = os.path.join(LIB_DIR, "libamrx.so")
    if not os.path.exists(lib):
        pytest.skip("libamrx.so not built")
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "step.c"
    src.write_text(GPU_SRC)
    exe = tmp_path / "step"
    # the HIP runtime's C interface, as hipcc would select it for this platform
    build = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                            "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), str(src),
                            "-L", LIB_DIR, "-lamrx", "-L", "/opt/rocm/lib", "-lamdhip64", "-lm",
                            "-Wl,-rpath," + LIB_DIR + ":/opt/rocm/lib", "-o", str(exe)],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    return exe


def test_c_step_program_builds(tmp_path):
    """The C program that runs a root step (below, on the GPU) compiles and links on the host."""
    _build_gpu_program(tmp_path)


@pytest.mark.gpu
def test_c_program_runs_a_root_step(tmp_path):
    """From C alone (hipMalloc'd arenas, no Python or torch in the process): a uniform state stays uniform
    through a two-level root step and dt0 has its closed form."""
    exe = _build_gpu_program(tmp_path)
    print("C root step program", flush=True)
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(run.stdout, flush=True)
    assert run.returncode == 0, (run.returncode, run.stdout, run.stderr)
    assert run.stdout.strip().endswith("ok")
