"""GPU: volumes (3-D ISAM, two lateral axes) through the C ABI.

Small volumes are compared with the FP64 oracle's volume operator (mode N) at the
operator bar (1e-5 relative l2) and FISTA bar (1e-4).  At the full 256 x 256 x 2048 size
the checks are properties: the adjoint identity, and a volume constant along y, which
must act like the B-scan plan on every y row.
"""
import math

import numpy as np
import pytest

import oracle as O
import phantoms as ph
from _util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL_OP = 1e-5


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06058_amd as pkg
    pkg.load_library()
    return pkg


def vol_optics(nx, ny, nk, dy=None, focus=None):
    o = ph.custom_optics(nx, nk, edge_phase2=12 * math.pi, edge_phase3=3 * math.pi,
                         focus_rows=nk // 8 if focus is None else focus)
    return o, (dy if dy is not None else o.dx)


@pytest.mark.parametrize("ny,nx,nk", [(4, 8, 64), (8, 16, 32), (2, 32, 64), (16, 4, 128), (8, 8, 256)])
def test_volume_forward_adjoint_match_oracle(P, ny, nx, nk):
    o, dy = vol_optics(nx, ny, nk, dy=5e-6, focus=-11.5)
    g = O.Geometry.of(o, ny=ny, dy=dy)
    V = O.VolumeOperator(g, "N")
    rng = np.random.default_rng(ny * 100 + nx + nk)
    eta = ph.complex_gaussian(rng, (ny, nx, nk))
    r = rng.standard_normal((ny, nx, nk))
    with P.Plan(P.Geometry.of(o, ny=ny, dy=dy)) as plan:
        s = to_host(plan.forward(to_dev(eta)))
        a = to_host(plan.adjoint(to_dev(r)))
    assert rel(s, V.A(eta)) < TOL_OP
    assert rel(a, V.AH(r)) < TOL_OP


def test_volume_calibration_grad_matches_oracle(P):
    ny, nx, nk = 4, 16, 64
    o, dy = vol_optics(nx, ny, nk, dy=5e-6, focus=9)
    g = O.Geometry.of(o, ny=ny, dy=dy)
    rng = np.random.default_rng(6)
    eta = ph.complex_gaussian(rng, (ny, nx, nk))
    G = rng.standard_normal((ny, nx, nk))
    ref = O.VolumeOperator(g, "N").calibration_gradient(eta, G)
    with P.Plan(P.Geometry.of(o, ny=ny, dy=dy)) as plan:
        got = plan.calibration_grad(to_dev(eta), to_dev(G))
    for i in range(3):
        assert abs(got[i] - ref[i]) <= 2e-4 * abs(ref[i]), (i, got[i], ref[i])


def test_volume_fista_matches_oracle(P):
    ny, nx, nk = 8, 16, 64
    o, dy = vol_optics(nx, ny, nk, dy=4e-6)
    g = O.Geometry.of(o, ny=ny, dy=dy)
    V = O.VolumeOperator(g, "N")
    rng = np.random.default_rng(5)
    eta = np.stack([ph.layers(rng, nx, nk, 1) + ph.point_scatterers(rng, nx, nk, 4) for _ in range(ny)])
    y = ph.add_noise(V.A(eta), 25.0, 5)
    with P.Plan(P.Geometry.of(o, ny=ny, dy=dy)) as plan:
        L = plan.lipschitz(iters=50, seed=0)
        lam = 0.05 * plan.lambda_max(to_dev(y))
        res = plan.fista(to_dev(y), lam, 40, L=L)
        z = to_host(res.eta)
    ref = O.fista(V, y, lam, L, 40)
    assert rel(z, ref.z) < 1e-4
    assert abs(res.resid2 - ref.resid2[-1]) < 1e-4 * ref.resid2[-1]


def test_full_volume_adjoint_identity_and_y_constant_rows(P):
    """256 x 256 x 2048: <A x, y> = <x, A^H y>, and a y-constant object acts as the B-scan."""
    import torch
    ny, nx, nk = 256, 256, 2048
    o, dy = vol_optics(nx, ny, nk)
    gen = torch.Generator(device="cuda").manual_seed(1)
    with P.Plan(P.Geometry.of(o, ny=ny, dy=dy)) as vol, P.Plan(P.Geometry.of(o)) as bscan:
        x = torch.randn((ny, nx, nk), dtype=torch.complex64, device="cuda", generator=gen)
        y = torch.randn((ny, nx, nk), dtype=torch.float32, device="cuda", generator=gen)
        ax = vol.forward(x)
        ahy = vol.adjoint(y)
        lhs = float((ax.double() * y.double()).sum())
        rhs = float((x.conj() * ahy).real.double().sum())
        scale = float(ax.double().norm() * y.double().norm())
        assert abs(lhs - rhs) <= 1e-6 * scale
        x0 = torch.randn((nx, nk), dtype=torch.complex64, device="cuda", generator=gen)
        sv = vol.forward(x0.expand(ny, nx, nk).contiguous())
        s1 = bscan.forward(x0)
        for row in (0, 1, 97, 255):
            assert rel(to_host(sv[row]), to_host(s1)) < 1e-6, row


def test_full_volume_fista_runs_and_descends(P):
    import torch
    ny, nx, nk = 256, 256, 2048
    o, dy = vol_optics(nx, ny, nk)
    gen = torch.Generator(device="cuda").manual_seed(2)
    with P.Plan(P.Geometry.of(o, ny=ny, dy=dy)) as vol:
        x = torch.zeros((ny, nx, nk), dtype=torch.complex64, device="cuda")
        idx = torch.randint(0, ny * nx * nk, (20000,), device="cuda", generator=gen)
        x.view(-1)[idx] = torch.randn(20000, dtype=torch.complex64, device="cuda", generator=gen)
        y = vol.forward(x)
        lam = 0.05 * vol.lambda_max(y)
        r5 = vol.fista(y, lam, 5, L=1.01)
        r20 = vol.fista(y, lam, 20, L=1.01)
        assert r5.status == 0 and r20.status == 0
        assert math.isfinite(r20.resid2) and r20.resid2 < r5.resid2
