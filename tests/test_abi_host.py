"""Host-side checks of the C ABI: the library loads, exports what include/isam.h declares,
and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1905_06058_amd as P
import phantoms as ph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        from paper_1905_06058_amd import build
        build.build()
    return P.load_library()


def header_symbols():
    text = open(os.path.join(ROOT, "include", "isam.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isam_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = header_symbols()
    assert "isam_plan" in names and "isam_fista" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTS) == names


def test_strerror_is_static_and_total(lib):
    for code in [0, -1, -2, -3, -4, -5, -6, -7, 99, -100]:
        s = lib.isam_strerror(code)
        assert isinstance(s, bytes) and len(s) > 0


def _geom(**kw):
    return P.Geometry.of(ph.workload("tiny").optics, **kw)


def _plan_rc(lib, g):
    h = ctypes.c_void_p()
    rc = lib.isam_plan(ctypes.byref(g) if g is not None else None, None, ctypes.byref(h))
    if rc == 0:
        lib.isam_destroy(h)
    return rc


@pytest.mark.parametrize("kw,code", [
    (dict(nk=255), -1),            # odd
    (dict(nk=8), -1),              # fewer than 2J samples
    (dict(J=5), -1),
    (dict(J=8), -3),
    (dict(osf=3), -3),
    (dict(nx=0), -1),
    (dict(nx=96), -3),             # no lateral kernels built for this length
    (dict(nx=576), -3),            # odd factor 9
    (dict(nx=384), -5),            # 3 x 128: valid, but no device here
    (dict(nk=8192), -3),
    (dict(nx=4096), -3),
    (dict(ny=2), -5),              # a volume: valid, but no device here
    (dict(ny=3), -3),
    (dict(ny=2, dy=0.0), -1),
    (dict(dx=0.0), -1),
    (dict(dlambda=-1e-9), -1),
    (dict(a2=float("nan")), -1),
    (dict(z_focus=float("inf")), -1),
    (dict(kb_beta=1.0), -1),        # scaling undefined at the outer rows
])
def test_plan_rejects_bad_geometry(lib, kw, code):
    assert _plan_rc(lib, _geom(**kw)) == code


def test_plan_null_arguments(lib):
    g = _geom()
    assert lib.isam_plan(None, None, ctypes.byref(ctypes.c_void_p())) == -1
    assert lib.isam_plan(ctypes.byref(g), None, None) == -1


def test_entry_points_reject_null_plan(lib):
    buf = ctypes.create_string_buffer(64)
    assert lib.isam_forward(None, buf, buf, None) == -1
    assert lib.isam_adjoint(None, buf, buf, None) == -1
    assert lib.isam_normal(None, buf, buf, None) == -1
    L = ctypes.c_double()
    assert lib.isam_lipschitz(None, 10, 0, None, ctypes.byref(L), None) == -1
    assert lib.isam_lambda_max(None, buf, None, ctypes.byref(L), None) == -1
    assert lib.isam_fista(None, buf, 0.1, None, 1, 0.0, 1.0, 0, buf, None, None) == -1
    assert lib.isam_set_calibration(None, 0.0, 0.0, 0.0, None) == -1
    assert lib.isam_calibration_grad(None, buf, buf, ctypes.byref(L), None) == -1
    assert lib.isam_plan_dims(None, None, None, None) == -1
    lib.isam_destroy(None)
    h = ctypes.c_void_p()
    assert lib.isam_batch_plan(None, 1, None, ctypes.byref(h)) == -1
    assert lib.isam_batch_plan(ctypes.byref(_geom()), 0, None, ctypes.byref(h)) == -1
    assert lib.isam_batch_forward(None, buf, buf, None) == -1
    assert lib.isam_batch_adjoint(None, buf, buf, None) == -1
    assert lib.isam_batch_tune(None, 1, None) == -1
    assert lib.isam_batch_set_tiles(None, 256, 4, 4) == -1
    assert lib.isam_batch_set_schedule(None, 0) == -1
    sched = ctypes.c_int()
    assert lib.isam_batch_schedule(None, ctypes.byref(sched)) == -1
    assert lib.isam_batch_offsets(None, None) == -1
    lib.isam_batch_destroy(None)


def test_batch_plan_without_device_reports_enodev(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    gs = (P.Geometry * 2)(_geom(), _geom(nx=384))
    h = ctypes.c_void_p()
    assert lib.isam_batch_plan(gs, 2, None, ctypes.byref(h)) == -5
    assert not h.value


def test_valid_geometry_without_device_reports_enodev(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _plan_rc(lib, _geom()) == -5


C_CONSUMER = r"""
#include <stdio.h>
#include <string.h>
#include "isam.h"
int main(void) {
    isam_geometry g;
    isam_plan_t p = 0;
    memset(&g, 0, sizeof g);                      /* nx = 0: rejected before any device call */
    if (isam_plan(&g, 0, &p) != ISAM_EINVAL || p != 0) return 1;
    if (isam_forward(0, 0, 0, 0) != ISAM_EINVAL) return 2;
    if (isam_strerror(ISAM_OK) == 0 || isam_strerror(ISAM_EINVAL)[0] == 0) return 3;
    printf("%s\n", isam_strerror(ISAM_EINVAL));
    return 0;
}
"""


def test_header_is_plain_c_and_links(lib, tmp_path):
    """include/isam.h is ISO C99 (no C++ in the signatures); a C program links libisam.so
    and gets argument errors back without a device."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "consumer.c"
    src.write_text(C_CONSUMER)
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(P.LIB_PATH)
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                        os.path.join(ROOT, "include"), str(src), "-L", libdir, "-lisam",
                        "-Wl,-rpath," + libdir, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.strip()
