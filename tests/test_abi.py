"""C-ABI checks that need no GPU: libgd.so loads, exports every function
include/gd.h declares, and rejects invalid input on the host before any
device work (error contract of include/gd.h)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1807_00699_amd import gd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gd.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gd_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gd.LIB_PATH):
        from paper_1807_00699_amd import build
        build.build()
    return gd.load()


def test_header_declarations_match_binding():
    assert set(_declared_functions()) == set(gd.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", gd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for name in _declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_struct_layouts_match_header(lib):
    # sizes as the C compiler lays them out (x86-64 SysV)
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "gd.h"
int main(void){printf("%zu %zu %zu %zu %zu %zu\n", sizeof(gd_params), offsetof(gd_params, stream),
 sizeof(gd_run_stats), offsetof(gd_run_stats, kernel_config), offsetof(gd_params, noise_seed),
 offsetof(gd_params, h_q));return 0;}
'''
    exe = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"gd_layout_{os.getpid()}")
    subprocess.run(["gcc", "-x", "c", "-I", os.path.join(ROOT, "include"), "-o", exe, "-"],
                   input=src, text=True, check=True)
    vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    os.remove(exe)
    assert vals == [C.sizeof(gd.gd_params), gd.gd_params.stream.offset,
                    C.sizeof(gd.gd_run_stats), gd.gd_run_stats.kernel_config.offset,
                    gd.gd_params.noise_seed.offset, gd.gd_params.h_q.offset]


def test_defaults_and_error_strings(lib):
    p = gd.default_params()
    assert p.struct_size == C.sizeof(gd.gd_params)
    assert (p.dt, p.eps, p.rho_th, p.gamma_c, p.j_scale) == (0.05, 0.1, 1.0, 0.0, 0.0)
    assert lib.gd_error_string(gd.GD_E_NOT_SYMMETRIC) == b"J is not symmetric"
    assert lib.gd_error_string(12345) == b"unknown error"


def _create(J, model=0, **kw):
    p = gd.default_params(**kw)
    h = C.c_void_p(123)
    Jc = np.ascontiguousarray(J, np.float32)
    rc = gd.load().gd_create(C.byref(h), Jc.shape[0], Jc.ctypes.data_as(C.c_void_p), None, model,
                             C.byref(p))
    return rc, h


def test_host_validation_errors(lib):
    J = np.zeros((4, 4), np.float32)
    J[0, 1] = 1.0                      # asymmetric
    rc, h = _create(J)
    assert rc == gd.GD_E_NOT_SYMMETRIC and h.value is None
    assert b"J[0][1]" in lib.gd_last_error()
    J = np.zeros((4, 4), np.float32)
    J[2, 3] = J[3, 2] = np.nan
    assert _create(J)[0] == gd.GD_E_NONFINITE
    assert _create(np.zeros((4, 4)), dt=0.0)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), integrator=7)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), precision=9)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), noise_D=-1.0)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), h_q=float("nan"))[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), variant=2)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), eps_hat=-1.0)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), variant=1, integrator=1)[0] == gd.GD_E_UNSUPPORTED
    assert _create(np.zeros((4, 4)), variant=1, precision=1)[0] == gd.GD_E_UNSUPPORTED
    for q in (0, 1, 9):
        assert _create(np.zeros((4, 4)), model=gd.GD_POTTS, q=q, h_q=0.5)[0] == gd.GD_E_INVALID_ARG
    assert _create(np.zeros((4, 4)), model=gd.GD_POTTS, q=3)[0] == gd.GD_E_INVALID_ARG
    bad = gd.default_params()
    bad.struct_size = 8
    h = C.c_void_p()
    z = np.zeros((4, 4), np.float32)
    assert lib.gd_create(C.byref(h), 4, z.ctypes.data_as(C.c_void_p), None, 0, C.byref(bad)) == gd.GD_E_INVALID_ARG
    assert lib.gd_create(C.byref(h), 0, z.ctypes.data_as(C.c_void_p), None, 0, None) == gd.GD_E_INVALID_ARG
    # size limits: 1 <= n <= 65536 (checked before J is read)
    assert lib.gd_create(C.byref(h), 65537, z.ctypes.data_as(C.c_void_p), None, 0, None) == gd.GD_E_INVALID_ARG
    assert lib.gd_create(C.byref(h), -3, z.ctypes.data_as(C.c_void_p), None, 0, None) == gd.GD_E_INVALID_ARG
    assert lib.gd_create(C.byref(h), 4, None, None, 0, None) == gd.GD_E_INVALID_ARG
    assert lib.gd_create(C.byref(h), 4, z.ctypes.data_as(C.c_void_p), None, 5, None) == gd.GD_E_INVALID_ARG
    # calls on a NULL handle fail cleanly
    assert lib.gd_run(None, 1, 1) == gd.GD_E_INVALID_ARG
    assert lib.gd_energy(None, None, None) == gd.GD_E_INVALID_ARG
    lib.gd_destroy(None)
