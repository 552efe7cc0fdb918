"""GPU: calibration gradient, the differentiable forward operator and calibration fitting.

The gradient of <g, A eta> with respect to (a2, a3, z_focus) (Eq. 7, 13) from the HIP
library is compared with the FP64 oracle's gradient and with FP64 central finite
differences of the oracle's forward operator.  Per-point terms and block sums are FP32,
so each component is held to 1e-4 relative, plus 1e-6 of the sum of the terms' magnitudes
(the scale of FP32 cancellation in the sum).
"""
import math

import numpy as np
import pytest

import oracle as O
import phantoms as ph
from _util import rel, to_dev, to_host

pytestmark = pytest.mark.gpu

NAMES = ("a2", "a3", "z_focus")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_06058_amd as pkg
    pkg.load_library()
    return pkg


def grad_tolerance(g, eta, G, columns=None):
    """Per-component bound: 1e-4 |grad| + 1e-6 sum |terms| (terms of the oracle's sum)."""
    X = O.resampled_spectrum(g, eta, "N", columns)
    Gs = np.fft.fft(G, axis=0, norm="ortho")
    base = np.conj(Gs) * 1j * O.modulation(g) * X
    mag = np.array([np.abs(np.real(base * D)).sum() for D in O.calibration_derivatives(g)])
    return mag


def check_grad(got, ref, mag):
    got, ref = np.asarray(got), np.asarray(ref)
    for i, name in enumerate(NAMES):
        assert abs(got[i] - ref[i]) <= 1e-4 * abs(ref[i]) + 1e-6 * mag[i], (name, got[i], ref[i])


def test_set_calibration_matches_fresh_plan_and_oracle(P):
    o = ph.workload("tiny").optics
    o2 = ph.custom_optics(o.nx, o.nk, edge_phase2=14 * math.pi, edge_phase3=-3 * math.pi, focus_rows=-21.5)
    rng = np.random.default_rng(11)
    eta = ph.complex_gaussian(rng, (o.nx, o.nk))
    with P.Plan(P.Geometry.of(o)) as plan, P.Plan(P.Geometry.of(o2)) as fresh:
        plan.set_calibration(o2.a2, o2.a3, o2.z_focus)
        s = plan.forward(to_dev(eta))
        s2 = fresh.forward(to_dev(eta))
        assert bool((s == s2).all())
    assert rel(to_host(s), O.forward_nufft(O.Geometry.of(o2), eta)) < 1e-5


def test_calibration_grad_matches_oracle_tiny(P):
    w = ph.workload("tiny")
    g = O.Geometry.of(w.optics)
    eta = ph.phantom(w)
    G = np.random.default_rng(3).standard_normal((g.nx, g.nk))
    with P.Plan(P.Geometry.of(w.optics)) as plan:
        got = plan.calibration_grad(to_dev(eta), to_dev(G))
    check_grad(got, O.calibration_gradient(g, eta, G, "N"), grad_tolerance(g, eta, G))


def test_calibration_grad_matches_fp64_central_differences(P):
    """Central differences of the FP64 oracle's <G, A_theta eta> (mode N)."""
    o = ph.custom_optics(16, 128, edge_phase2=20 * math.pi, edge_phase3=4 * math.pi, focus_rows=19)
    g = O.Geometry.of(o)
    rng = np.random.default_rng(8)
    eta = ph.complex_gaussian(rng, (g.nx, g.nk))
    G = rng.standard_normal((g.nx, g.nk))
    fd = []
    for name in NAMES:
        v = getattr(g, name)
        h = 1e-5 * abs(v)
        fp = np.sum(G * O.forward_nufft(g.with_(**{name: v + h}), eta))
        fm = np.sum(G * O.forward_nufft(g.with_(**{name: v - h}), eta))
        fd.append((fp - fm) / (2 * h))
    with P.Plan(P.Geometry.of(o)) as plan:
        got = plan.calibration_grad(to_dev(eta), to_dev(G))
    check_grad(got, fd, grad_tolerance(g, eta, G))


def test_calibration_grad_on_lateral_band_calib_size(P):
    """512 x 2048: an object whose lateral spectrum sits on a few columns (incl. the highest |q|)."""
    o = ph.workload("calib").optics
    g = O.Geometry.of(o)
    rng = np.random.default_rng(21)
    ls = [0, 5, 131, 255, 256, 400]
    spec = np.zeros((o.nx, o.nk), np.complex128)
    for l in ls:
        spec[l] = ph.complex_gaussian(rng, o.nk)
    eta = np.fft.ifft(spec, axis=0, norm="ortho")
    G = rng.standard_normal((o.nx, o.nk))
    with P.Plan(P.Geometry.of(o)) as plan:
        got = plan.calibration_grad(to_dev(eta), to_dev(G))
    ref = O.calibration_gradient(g, eta, G, "N", columns=ls)
    check_grad(got, ref, grad_tolerance(g, eta, G, columns=ls))


def test_autograd_function_uses_adjoint_and_calibration_grad(P):
    import torch
    from paper_1905_06058_amd.autograd import isam_forward
    w = ph.workload("tiny")
    o = w.optics
    rng = np.random.default_rng(5)
    G = to_dev(rng.standard_normal((o.nx, o.nk)))
    with P.Plan(P.Geometry.of(o)) as plan:
        eta = to_dev(ph.phantom(w)).requires_grad_(True)
        theta = torch.tensor([o.a2, o.a3, o.z_focus], dtype=torch.float64, requires_grad=True)
        s = isam_forward(plan, eta, theta)
        assert bool((s == plan.forward(eta.detach())).all())
        (G * s).sum().backward()
        assert bool((eta.grad == plan.adjoint(G)).all())
        ref = plan.calibration_grad(eta.detach(), G)
        assert np.array_equal(theta.grad.numpy(), np.array(ref))


@pytest.mark.parametrize("signs", [(1, -1, 1), (-1, 1, -1)])
def test_fit_calibration_from_thirty_percent_perturbation(P, signs):
    """Known object, noisy spectra (SNR 25 dB), start at +/-30 % on each parameter."""
    import torch
    from paper_1905_06058_amd.autograd import fit_calibration, natural_units
    w = ph.workload("calib")
    o = w.optics
    eta_np = ph.phantom(w)
    with P.Plan(P.Geometry.of(o)) as plan:
        eta = to_dev(eta_np)
        s = to_host(plan.forward(eta))
        y = to_dev(ph.add_noise(s, w.snr_db, w.seed))
        true = np.array([o.a2, o.a3, o.z_focus])
        start = true * (1 + 0.3 * np.array(signs))
        res = fit_calibration(plan, eta, y, tuple(start))
    relerr = np.abs(np.array(res.theta) - true) / np.abs(true)
    assert relerr.max() < 1e-3, (relerr, res.history)
    half, dz = natural_units(P.Geometry.of(o))
    assert abs(res.natural[2] - o.z_focus / dz) < 0.5           # within half a depth row
    assert torch.isfinite(torch.tensor(res.loss))
