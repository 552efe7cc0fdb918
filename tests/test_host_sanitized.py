"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The HIP sources are compiled with the sanitizers on their host side only (each -fsanitize=
behind -Xarch_host; the gfx950 device code is unchanged) into a library in a temporary
directory, and a C program linked against it drives every entry point's argument checks:
invalid geometries of every kind, NULL and aliasing arguments, error strings, and (with no
device visible here) the device-probing paths of plan and batch creation.  The program must
exit 0 with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include <string.h>
#include "isam.h"

static isam_geometry base(void) {
    isam_geometry g;
    memset(&g, 0, sizeof g);
    g.nx = 64; g.ny = 1; g.nk = 256; g.dx = 4e-6; g.dy = 4e-6;
    g.lambda_c = 1300e-9; g.dlambda = 170e-9; g.waist = 8e-6; g.z_focus = 3e-4;
    g.a2 = 1e-9; g.a3 = 1e-16; g.J = 6; g.osf = 2; g.kb_beta = 0.0;
    return g;
}

#define EXPECT(call, code) do { int rc_ = (call); if (rc_ != (code)) { \
    printf("line %d: %s gave %d, expected %d\n", __LINE__, #call, rc_, (code)); return 1; } } while (0)

int main(void) {
    isam_plan_t p = 0;
    isam_geometry g;
    char buf[256];
    double d = 0.0;
    int64_t off[4];
    int i;
    for (i = -10; i <= 3; ++i) if (!isam_strerror(i) || !isam_strerror(i)[0]) return 2;
    g = base(); g.nx = 0; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.nk = 255; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.J = 5; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.J = 8; EXPECT(isam_plan(&g, 0, &p), ISAM_EUNSUPPORTED);
    g = base(); g.osf = 3; EXPECT(isam_plan(&g, 0, &p), ISAM_EUNSUPPORTED);
    g = base(); g.nx = 96; EXPECT(isam_plan(&g, 0, &p), ISAM_EUNSUPPORTED);
    g = base(); g.nk = 8192; EXPECT(isam_plan(&g, 0, &p), ISAM_EUNSUPPORTED);
    g = base(); g.ny = 3; EXPECT(isam_plan(&g, 0, &p), ISAM_EUNSUPPORTED);
    g = base(); g.ny = 2; g.dy = 0.0; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.dlambda = -1.0; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.a2 = 1.0 / 0.0; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.kb_beta = 1.0; EXPECT(isam_plan(&g, 0, &p), ISAM_EINVAL);
    g = base(); g.nx = 2048; g.ny = 2048; g.nk = 4096; EXPECT(isam_plan(&g, 0, &p), ISAM_EUNSUPPORTED);
    EXPECT(isam_plan(0, 0, &p), ISAM_EINVAL);
    g = base(); EXPECT(isam_plan(&g, 0, 0), ISAM_EINVAL);
    g = base(); EXPECT(isam_plan(&g, 0, &p), ISAM_ENODEV);
    if (p) return 3;
    g = base(); g.nx = 384; g.ny = 4; EXPECT(isam_plan(&g, 0, &p), ISAM_ENODEV);
    EXPECT(isam_forward(0, buf, (float*)buf, 0), ISAM_EINVAL);
    EXPECT(isam_adjoint(0, (const float*)buf, buf, 0), ISAM_EINVAL);
    EXPECT(isam_normal(0, buf, buf, 0), ISAM_EINVAL);
    EXPECT(isam_direct(0, (const float*)buf, buf, 0), ISAM_EINVAL);
    EXPECT(isam_lipschitz(0, 10, 0, 0, &d, 0), ISAM_EINVAL);
    EXPECT(isam_lambda_max(0, (const float*)buf, 0, &d, 0), ISAM_EINVAL);
    EXPECT(isam_calibration_grad(0, buf, (const float*)buf, &d, 0), ISAM_EINVAL);
    EXPECT(isam_fista(0, (const float*)buf, 0.1f, 0, 10, 0.f, 1.0, 0, buf, 0, 0), ISAM_EINVAL);
    EXPECT(isam_fista_ex(0, (const float*)buf, 0.1f, 0, 10, 0.f, 1.0, 0, 0, 0, 0, buf, 0, 0), ISAM_EINVAL);
    EXPECT(isam_fista_state_bytes(0, off), ISAM_EINVAL);
    EXPECT(isam_set_calibration(0, 0.0, 0.0, 0.0, 0), ISAM_EINVAL);
    EXPECT(isam_timing(0, 1, 0, 0), ISAM_EINVAL);
    EXPECT(isam_plan_dims(0, 0, 0, 0), ISAM_EINVAL);
    isam_destroy(0);
    {
        isam_geometry gs[2];
        isam_batch_t b = 0;
        gs[0] = base(); gs[1] = base(); gs[1].nx = 384;
        EXPECT(isam_batch_plan(0, 1, 0, &b), ISAM_EINVAL);
        EXPECT(isam_batch_plan(gs, 0, 0, &b), ISAM_EINVAL);
        EXPECT(isam_batch_plan(gs, 2, 0, &b), ISAM_ENODEV);
        if (b) return 4;
        EXPECT(isam_batch_forward(0, buf, (float*)buf, 0), ISAM_EINVAL);
        EXPECT(isam_batch_adjoint(0, (const float*)buf, buf, 0), ISAM_EINVAL);
        EXPECT(isam_batch_offsets(0, off), ISAM_EINVAL);
        EXPECT(isam_batch_tune(0, 1, 0), ISAM_EINVAL);
        EXPECT(isam_batch_set_tiles(0, 256, 4, 4), ISAM_EINVAL);
        isam_batch_destroy(0);
    }
    puts("ok");
    return 0;
}
"""


def test_host_code_under_asan_and_ubsan(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("drives the no-device paths; run where no GPU is visible")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("needs hipcc and a C compiler")
    from paper_1905_06058_amd import build
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    lib = build.build(out=str(tmp_path / "libisam.so"), objdir=str(tmp_path / "obj"), extra=san,
                      link_extra=["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"])
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    clang = "/opt/rocm/llvm/bin/clang"
    r = subprocess.run([clang, "-std=c99", "-Wall", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                        "-I", os.path.join(ROOT, "include"), str(src), str(lib),
                        "-Wl,-rpath," + str(tmp_path), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert r.returncode == 0 and "ok" in r.stdout, report[-4000:]
