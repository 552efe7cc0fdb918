"""GPU: isam_direct_static, the direct image of Eq. 9 without a plan and without allocating
(its tables live in the library's static device array), against isam_direct on a plan of
the same geometry: two calls in a row, the second smaller, then the size limit."""
import ctypes
import math

import numpy as np
import pytest

import phantoms as ph
from _util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06058_amd as pkg
    pkg.load_library()
    return pkg


def test_direct_static_matches_plan_direct_twice(P):
    import torch
    cases = [(4, 64, 2048, 40, 8), (1, 16, 256, 12, -3)]       # (ny, nx, nk, edge phases in pi)
    for ny, nx, nk, e2, e3 in cases:
        o = ph.custom_optics(nx, nk, edge_phase2=e2 * math.pi, edge_phase3=e3 * math.pi)
        g = P.Geometry.of(o, ny=ny, dy=o.dx)
        rng = np.random.default_rng(nx + nk)
        shape = (ny, nx, nk) if ny > 1 else (nx, nk)
        y = to_dev(rng.standard_normal(shape))
        got = P.direct_static(g, y)
        torch.cuda.synchronize()
        with P.Plan(g) as plan:
            want = plan.direct(y)
        print(f"{shape}: rel l2 {rel(to_host(got), to_host(want)):.2e}, bitwise {torch.equal(got, want)}")
        assert rel(to_host(got), to_host(want)) < 1e-5


def test_direct_static_limits(P):
    o = ph.custom_optics(8, 8192)
    g = P.Geometry.of(o)
    import torch
    y = torch.zeros((8, 8192), dtype=torch.float32, device="cuda")
    out = torch.empty((8, 8192), dtype=torch.complex64, device="cuda")
    lib = P.load_library()
    rc = lib.isam_direct_static(ctypes.byref(g), y.data_ptr(), out.data_ptr(), None)
    assert rc == -3                       # nk above the static tables' 4096
    g2 = P.Geometry.of(ph.custom_optics(8, 96))
    assert lib.isam_direct_static(ctypes.byref(g2), y.data_ptr(), out.data_ptr(), None) == -3
    assert lib.isam_direct_static(None, y.data_ptr(), out.data_ptr(), None) == -1
