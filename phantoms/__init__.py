"""Seeded synthetic inputs for the full-range ISAM operator and its FISTA solve.

This module is shared by the FP64 oracle's tests and by the GPU path's tests and
benchmark.  It holds the workload recipes (optics, sizes, seeds) and the random
objects and noise drawn from them, and nothing of the method's arithmetic: no
Stolt mapping, no NUFFT, no operator.  Noise is added to a clean signal that the
caller computes with whichever implementation it is testing.

Workloads stand in for the paper's SD-OCT B-scans (1024 A-scans x 2048 spectral
samples, Sec. "Materials and measurements"); the paper's measured datasets are
not available, so every object here is a seeded synthetic phantom.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace

import numpy as np

__all__ = [
    "Optics", "Workload", "workload", "WORKLOADS", "point_scatterers", "layers",
    "phantom", "add_noise", "complex_gaussian", "real_gaussian", "depth_weights",
]


@dataclass(frozen=True)
class Optics:
    """Plain optical and sampling parameters of one B-scan (SI units).

    Sampling is uniform in wavenumber; ``z_focus`` is the focal depth measured
    from zero delay; ``a2`` and ``a3`` are the quadratic and cubic coefficients
    of the dispersion polynomial (Eq. 7, a1 = 0, k0 = centre wavenumber).
    """
    nx: int
    nk: int
    dx: float
    lambda_c: float
    dlambda: float
    waist: float
    z_focus: float
    a2: float
    a3: float
    J: int = 6
    osf: int = 2
    kb_beta: float = 0.0          # 0 selects 2.34 * J

    def as_dict(self) -> dict:
        return asdict(self)


def _band(lambda_c: float, dlambda: float) -> float:
    """Linearised wavenumber bandwidth of a source of centre lambda_c and width dlambda."""
    return 2.0 * math.pi * dlambda / lambda_c ** 2


def _recipe_optics(nx: int, nk: int, *, edge_phase2: float, edge_phase3: float,
                   focus_rows: float, lambda_c=1300e-9, dlambda=170e-9,
                   dx=4e-6, waist=8e-6) -> Optics:
    """Optics of the synthetic workloads.

    The recipe states dispersion as the phase the quadratic (cubic) term reaches
    at the band edge, |k - k_c| = band/2, and focus as a number of depth rows of
    the full-range grid (row pitch pi / band).  This converts those recipe units
    into the physical coefficients the operator takes.
    """
    band = _band(lambda_c, dlambda)
    half = band / 2.0
    dz = math.pi / band
    return Optics(nx=nx, nk=nk, dx=dx, lambda_c=lambda_c, dlambda=dlambda, waist=waist,
                  z_focus=focus_rows * dz, a2=edge_phase2 / half ** 2,
                  a3=edge_phase3 / half ** 3)


@dataclass(frozen=True)
class Workload:
    name: str
    optics: Optics
    n_points: int
    n_layers: int
    snr_db: float
    iters: int
    lam_frac: float
    seed: int


def workload(name: str) -> Workload:
    """Named synthetic workloads.

    ``tiny``     64 A-scans x 256 samples, 40 scatterers, 20 pi quadratic
                 dispersion, focus +64 rows, SNR 30 dB, 100 FISTA iterations.
    ``bscan``    1024 A-scans x 2048 samples (the paper's acquisition shape),
                 5 layers + 2000 scatterers, 40 pi / 8 pi dispersion, focus
                 +512 rows, SNR 25 dB, 200 FISTA iterations.
    ``calib``    512 x 2048 B-scan used for calibration fitting.
    ``medium``   256 x 1024, a mid-size case the oracle still runs in seconds.
    """
    if name == "tiny":
        o = _recipe_optics(64, 256, edge_phase2=20 * math.pi, edge_phase3=0.0, focus_rows=64)
        return Workload(name, o, n_points=40, n_layers=0, snr_db=30.0, iters=100,
                        lam_frac=0.05, seed=0)
    if name == "bscan":
        o = _recipe_optics(1024, 2048, edge_phase2=40 * math.pi, edge_phase3=8 * math.pi,
                           focus_rows=512)
        return Workload(name, o, n_points=2000, n_layers=5, snr_db=25.0, iters=200,
                        lam_frac=0.05, seed=1)
    if name == "calib":
        o = _recipe_optics(512, 2048, edge_phase2=40 * math.pi, edge_phase3=8 * math.pi,
                           focus_rows=512)
        return Workload(name, o, n_points=1000, n_layers=5, snr_db=25.0, iters=50,
                        lam_frac=0.05, seed=2)
    if name == "medium":
        o = _recipe_optics(256, 1024, edge_phase2=40 * math.pi, edge_phase3=8 * math.pi,
                           focus_rows=256)
        return Workload(name, o, n_points=250, n_layers=3, snr_db=25.0, iters=60,
                        lam_frac=0.05, seed=4)
    raise KeyError(name)


WORKLOADS = ("tiny", "medium", "calib", "bscan")


def custom_optics(nx: int, nk: int, *, edge_phase2=40 * math.pi, edge_phase3=8 * math.pi,
                  focus_rows=None, **kw) -> Optics:
    """Same optics recipe at an arbitrary grid size (focus defaults to +nk/4 rows)."""
    if focus_rows is None:
        focus_rows = nk // 4
    return _recipe_optics(nx, nk, edge_phase2=edge_phase2, edge_phase3=edge_phase3,
                          focus_rows=focus_rows, **kw)


def complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """Circular complex Gaussian CN(0, 1) samples, complex128."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def real_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape)


def point_scatterers(rng: np.random.Generator, nx: int, nk: int, n: int) -> np.ndarray:
    """``n`` point scatterers at distinct grid positions, CN(0,1) amplitudes.

    Depth index i = m + nk/2 holds delay row m in [-nk/2, nk/2).  Rows
    m = -nk/2 (unpaired with a mirror) and m = 0 (zero delay) are avoided; half
    of the points sit at negative delay and half at positive delay.
    """
    eta = np.zeros((nx, nk), np.complex128)
    if n == 0:
        return eta
    half = nk // 2
    rows = half - 1                       # rows per side: m in [-nk/2+1, -1] and [1, nk/2-1]
    n_neg = n // 2
    n_pos = n - n_neg
    sel_neg = rng.choice(nx * rows, size=n_neg, replace=False)
    sel_pos = rng.choice(nx * rows, size=n_pos, replace=False)
    amps = complex_gaussian(rng, n)
    p = np.concatenate([sel_neg // rows, sel_pos // rows])
    i = np.concatenate([1 + sel_neg % rows, half + 1 + sel_pos % rows])
    eta[p, i] = amps
    return eta


def layers(rng: np.random.Generator, nx: int, nk: int, n_layers: int) -> np.ndarray:
    """Smooth layered interfaces on both sides of zero delay.

    Layer l follows m_l(p) = round(c_l + A_l sin(2 pi p / P_l + theta_l)) with
    c_l ~ U(-0.8, 0.8) nk/2, A_l ~ U[10, 60] rows, P_l ~ U[0.5, 2] nx,
    theta_l ~ U[0, 2 pi); reflectivity r_l ~ U[0.3, 1] times a per-pixel random
    phase.  Rows are clipped to [-nk/2 + 1, nk/2 - 1].
    """
    eta = np.zeros((nx, nk), np.complex128)
    half = nk // 2
    p = np.arange(nx)
    for _ in range(n_layers):
        c = rng.uniform(-0.8, 0.8) * half
        amp = rng.uniform(10, 60)
        per = rng.uniform(0.5, 2.0) * nx
        th = rng.uniform(0, 2 * math.pi)
        refl = rng.uniform(0.3, 1.0)
        m = np.rint(c + amp * np.sin(2 * math.pi * p / per + th)).astype(np.int64)
        m = np.clip(m, -half + 1, half - 1)
        ph = np.exp(2j * math.pi * rng.uniform(0, 1, nx))
        eta[p, m + half] += refl * ph
    return eta


def phantom(w: Workload) -> np.ndarray:
    """Object of a named workload: layers plus point scatterers, complex128 [nx][nk]."""
    rng = np.random.default_rng(w.seed)
    o = w.optics
    eta = layers(rng, o.nx, o.nk, w.n_layers)
    eta += point_scatterers(rng, o.nx, o.nk, w.n_points)
    return eta


def add_noise(s_clean: np.ndarray, snr_db: float, seed: int) -> np.ndarray:
    """White Gaussian noise on real spectra at the stated SNR.

    sigma^2 = ||s_clean||^2 / (numel * 10^(SNR/10)).
    """
    s_clean = np.asarray(s_clean, np.float64)
    rng = np.random.default_rng(seed + 7919)
    sigma = math.sqrt(float(np.sum(s_clean ** 2)) / (s_clean.size * 10 ** (snr_db / 10)))
    return s_clean + sigma * rng.standard_normal(s_clean.shape)


def depth_weights(nx: int, nk: int) -> np.ndarray:
    """Depth-increasing l1 weights: 0.5 at the most negative delay row to 1 at the last row."""
    w = np.linspace(0.5, 1.0, nk)
    return np.broadcast_to(w, (nx, nk)).copy()
