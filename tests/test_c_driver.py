"""A C program that uses the library through its header alone (no Python, no torch).

The program reads the patch descriptors, the physics record and the U arena from
binary files, allocates U and dt with the HIP runtime, and runs `steps` RK2 steps
with amr_cfl_dt + amr_hydro_rk2_step, printing each dt as a hexadecimal float and
writing U back.  The CPU test compiles and links it against the public header and
the built library; the GPU test runs it on 12 uneven patches in FP64 and compares
the result with the oracle stepped with the same time steps (per cell, 1e-12 of
each variable's largest magnitude, and the dts bit for bit).
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from paper_0910_5547_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_0910_5547_amd")

DRIVER = r'''
#include <stdio.h>
#include <stdlib.h>
#include "amr_hydro.h"

#define CHECK(call)                                                                 \
  do {                                                                              \
    amr_status st_ = (call);                                                        \
    if (st_ != AMR_OK) {                                                            \
      fprintf(stderr, "%s failed: %d\n", #call, (int)st_);                          \
      return 2;                                                                     \
    }                                                                               \
  } while (0)

static void* slurp(const char* path, size_t* bytes) {
  FILE* f = fopen(path, "rb");
  if (!f) return NULL;
  fseek(f, 0, SEEK_END);
  *bytes = (size_t)ftell(f);
  fseek(f, 0, SEEK_SET);
  void* p = malloc(*bytes);
  if (p && fread(p, 1, *bytes, f) != *bytes) {
    free(p);
    p = NULL;
  }
  fclose(f);
  return p;
}

/* usage: driver desc.bin phys.bin U.bin steps cfl out.bin */
int main(int argc, char** argv) {
  if (argc != 7) return 1;
  size_t nd = 0, np = 0, nu = 0;
  amr_patch_desc* desc = (amr_patch_desc*)slurp(argv[1], &nd);
  amr_physics* phys = (amr_physics*)slurp(argv[2], &np);
  double* U = (double*)slurp(argv[3], &nu);
  const int steps = atoi(argv[4]);
  const double cfl = atof(argv[5]);
  if (!desc || !phys || !U || np != sizeof(amr_physics) || nd % sizeof(amr_patch_desc)) return 1;
  const int npatch = (int)(nd / sizeof(amr_patch_desc));

  hipStream_t s;
  if (hipStreamCreate(&s) != hipSuccess) return 3;
  amr_table* t = NULL;
  CHECK(amr_patch_table_create(desc, npatch, phys, s, &t));
  if ((size_t)amr_table_arena_elems(t) * sizeof(double) > nu) return 4;
  double *Ud = NULL, *dt_dev = NULL;
  if (hipMalloc((void**)&Ud, nu) != hipSuccess || hipMalloc((void**)&dt_dev, sizeof(double)) != hipSuccess) return 3;
  if (hipMemcpy(Ud, U, nu, hipMemcpyHostToDevice) != hipSuccess) return 3;
  for (int k = 0; k < steps; ++k) {
    double dt = 0.0;
    CHECK(amr_cfl_dt(t, Ud, cfl, -1, dt_dev, &dt, s));
    printf("dt %a\n", dt);
    CHECK(amr_hydro_rk2_step(t, Ud, dt_dev, -1, 0, s));
  }
  CHECK(amr_table_status(t, s));
  if (hipMemcpy(U, Ud, nu, hipMemcpyDeviceToHost) != hipSuccess) return 3;
  FILE* f = fopen(argv[6], "wb");
  if (!f || fwrite(U, 1, nu, f) != nu) return 5;
  fclose(f);
  CHECK(amr_patch_table_destroy(t));
  (void)hipFree(Ud);
  (void)hipFree(dt_dev);
  (void)hipStreamDestroy(s);
  free(desc);
  free(phys);
  free(U);
  return 0;
}
'''


def _build(tmp_path):
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe), "-L", PKG, "-lamrhydro",
                    "-Wl,-rpath," + PKG, "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
                   check=True)
    return exe


def test_c_driver_builds_against_the_header_and_library(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libamrhydro.so")):
        pytest.skip("library not built")
    exe = _build(tmp_path)
    assert exe.exists()
    # argument errors are caught before any HIP call
    assert subprocess.run([str(exe)], capture_output=True).returncode == 1


@pytest.mark.gpu
def test_c_driver_matches_the_oracle(tmp_path):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle as O
    from paper_0910_5547_amd import amr as A
    from tests.gpu_util import active_all, log, rel_err
    exe = _build(tmp_path)
    ps, U = W.uneven_patches(npatch=12, seed=31)
    descs = A.descriptors(ps)
    ph = A.physics(ps, precision=A.AMR_PREC_FP64)
    (tmp_path / "desc.bin").write_bytes(bytes(descs))
    (tmp_path / "phys.bin").write_bytes(bytes(ph))
    U.astype(np.float64).tofile(tmp_path / "U.bin")
    steps = 5
    log(f"case C driver, 12 patches x {steps} steps")
    out = subprocess.run([str(exe), str(tmp_path / "desc.bin"), str(tmp_path / "phys.bin"), str(tmp_path / "U.bin"),
                          str(steps), "0.8", str(tmp_path / "out.bin")], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    dts = [float.fromhex(line.split()[1]) for line in out.stdout.splitlines() if line.startswith("dt ")]
    assert len(dts) == steps
    Ug = np.fromfile(tmp_path / "out.bin", dtype=np.float64)
    assert Ug.shape == U.shape
    o = O.Oracle(ps)
    Uo = U.copy()
    for dt in dts:
        assert o.cfl_dt(Uo, 0.8) == dt
        assert o.rk2_step(Uo, dt) == 0
    g, r = active_all(ps, Ug), active_all(ps, Uo)
    e = rel_err(g, r)
    log(f"C driver: max rel err {max(e):.1e}, bitwise={np.array_equal(g, r)}")
    assert max(e) <= 1e-12
