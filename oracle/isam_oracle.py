"""Plain FP64 CPU oracle of the full-range ISAM operator and its FISTA solve.

TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this module.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and shares no code with it.

What is computed, in the paper's notation (arXiv 1905.06058):

* object eta in C^{Nx x Nz}, depth row m in [-Nz/2, Nz/2) stored at index
  i = m + Nz/2 (Nz = Nk, Sec. "Background");
* measured real spectra s_d in R^{Nx x Nk};
* forward model s = Re(K^ eta) with K^ = diag(e^{j phi}) K (Eq. 5, 7, 8, 13);
* K = F_<->^{-1} diag(b) N F_<-> (Eq. 16): lateral FFT, a per-column Stolt
  resampling of the depth spectrum at beta = -sqrt(4k^2 - q^2) (Eq. 3), the
  beam filter b, the lateral inverse FFT;
* its adjoint back-projection K^H s = N'(F_<->(s)) (Eq. 17);
* FISTA on 1/2 ||Re(K^ eta) - s_d||^2 + lambda w^T |eta| (Eq. 12, Alg. 1) with
  the weighted complex soft threshold (Eq. 14) and the relative-residual stop
  (Eq. 15).

Two operator modes:

``E`` (exact): the Stolt resampling written as the direct nonuniform DFT
    X[l][n] = Nz^{-1/2} sum_m eta_hat[l][m] exp(+i kz[l][n] z_m).
``N`` (NUFFT): the same sum evaluated the way the paper does it, through a
    min-max interpolating NUFFT (Fessler & Sutton 2003): Kaiser-Bessel scaling,
    2x oversampled FFT, J-tap interpolation whose weights solve, per point, the
    least-squares problem that defines the min-max interpolator.

Where the paper leaves a passage open (sign conventions, normalisations, beam
filter and focus model, step size), the function that depends on it states the
reading it takes; each function names the passage it follows.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ProcessPoolExecutor
from dataclasses import dataclass, fields
import multiprocessing

import numpy as np
import scipy.fft
import scipy.linalg
import scipy.sparse
from threadpoolctl import threadpool_limits

__all__ = [
    "Geometry", "grids", "beam_filter", "dispersion_phase", "axial_wavenumber",
    "modulation", "kb_scaling", "stolt_points", "minmax_system", "minmax_weights",
    "minmax_error", "forward", "adjoint", "forward_exact", "adjoint_exact",
    "forward_nufft", "adjoint_nufft", "soft_threshold", "lipschitz", "lambda_max",
    "fista", "dense_matrix", "Operator", "resampled_spectrum", "calibration_derivatives",
    "calibration_gradient", "volume_q2", "VolumeOperator", "direct_image", "default_workers",
    "set_fft_workers",
]

# Threads of the library FFTs (scipy.fft's `workers`); 1 unless a caller asks for more.
_FFT_WORKERS = 1


def set_fft_workers(n: int) -> int:
    """Set the thread count of the oracle's FFTs; returns the previous value."""
    global _FFT_WORKERS
    prev, _FFT_WORKERS = _FFT_WORKERS, max(1, int(n))
    return prev


# --------------------------------------------------------------------------- geometry

@dataclass(frozen=True)
class Geometry:
    """Sampling and optics of one B-scan, SI units (rad/m, m)."""
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
    kb_beta: float = 0.0
    ny: int = 1              # lateral rows of a volume (1: a B-scan)
    dy: float = 0.0          # their pitch (0: same as dx)

    @classmethod
    def of(cls, obj, **overrides) -> "Geometry":
        """Copy the geometry fields from any object carrying them (e.g. an optics record)."""
        vals = {f.name: getattr(obj, f.name) for f in fields(cls) if hasattr(obj, f.name)}
        vals.update(overrides)
        return cls(**vals)

    def with_(self, **kw) -> "Geometry":
        vals = {f.name: getattr(self, f.name) for f in fields(self)}
        vals.update(kw)
        return Geometry(**vals)


@dataclass(frozen=True)
class Grids:
    kc: float          # centre wavenumber 2 pi / lambda_c (the k0 of Eq. 7)
    band: float        # wavenumber bandwidth 2 pi dlambda / lambda_c^2
    dk: float          # wavenumber step
    k: np.ndarray      # (nk,) k_n = kc + (n - nk/2) dk
    dz: float          # depth step pi / band
    m: np.ndarray      # (nz,) delay rows -nz/2 .. nz/2-1
    z: np.ndarray      # (nz,) z_m = m dz
    l: np.ndarray      # (nx,) lateral frequency index in FFT order
    q: np.ndarray      # (nx,) q_l = 2 pi l / (nx dx)
    K: int             # oversampled depth-FFT length osf * nz
    beta: float        # Kaiser-Bessel shape parameter


def grids(g: Geometry) -> Grids:
    """Sampling grids (Sec. "Background": N = Nx Nz with Nz the spectrometer length).

    Uniform sampling in k over the band; the full-range depth grid has Nz = Nk
    rows of pitch pi/band on both sides of zero delay; the lateral frequencies
    are those of an Nx-point DFT over the scan pitch dx (periodic lateral
    boundary).
    """
    kc = 2 * math.pi / g.lambda_c
    band = 2 * math.pi * g.dlambda / g.lambda_c ** 2
    dk = band / g.nk
    k = kc + (np.arange(g.nk) - g.nk / 2) * dk
    dz = math.pi / band
    nz = g.nk
    m = np.arange(-nz // 2, nz // 2)
    z = m * dz
    l = np.fft.fftfreq(g.nx, d=1.0 / g.nx)
    q = 2 * math.pi * l / (g.nx * g.dx)
    beta = g.kb_beta if g.kb_beta > 0 else 2.34 * g.J
    return Grids(kc, band, dk, k, dz, m, z, l, q, g.osf * nz, beta)


def beam_filter(g: Geometry) -> np.ndarray:
    """Beam / lens filter B(q, k) of Eq. 3 (the b of Eq. 16), shape (nx, nk).

    Gaussian beam of waist w0: two-way angular spectrum exp(-q^2 w0^2 / 8) on
    propagating components (q^2 < 4 k^2), zero on evanescent ones.
    """
    G = grids(g)
    q2 = (G.q ** 2)[:, None]
    prop = q2 < 4 * G.k[None, :] ** 2
    return np.where(prop, np.exp(-q2 * g.waist ** 2 / 8.0), 0.0)


def dispersion_phase(g: Geometry) -> np.ndarray:
    """phi(k_n) = a2 (k - k0)^2 + a3 (k - k0)^3 (Eq. 7 with a1 = 0, k0 = kc)."""
    G = grids(g)
    d = G.k - G.kc
    return g.a2 * d ** 2 + g.a3 * d ** 3


def axial_wavenumber(g: Geometry):
    """kz[l][n] = sqrt(4 k_n^2 - q_l^2), the Stolt-mapped axial frequency (Eq. 3).

    Eq. 3 evaluates the object spectrum at beta = -kz; with the forward
    transform exp(-i beta z) the resampled depth kernel is exp(+i kz z).
    Returns (kz, propagating mask); kz is 0 on evanescent points.
    """
    G = grids(g)
    arg = 4 * G.k[None, :] ** 2 - (G.q ** 2)[:, None]
    prop = arg > 0
    kz = np.sqrt(np.where(prop, arg, 0.0))
    return kz, prop


def modulation(g: Geometry) -> np.ndarray:
    """Pointwise factor c[l][n] multiplying the resampled spectrum.

    c = B(q, k) e^{j phi(k)} e^{j (2k - kz) z_f}: the beam filter (Eq. 3/16),
    the dispersion phase (Eq. 13) and the focal-plane reference of the Stolt
    map (the depth origin of the resampling moved to the focal plane).
    """
    G = grids(g)
    kz, prop = axial_wavenumber(g)
    B = beam_filter(g)
    phi = dispersion_phase(g)[None, :]
    focus = (2 * G.k[None, :] - kz) * g.z_focus
    c = B * np.exp(1j * phi) * np.exp(1j * focus)
    return np.where(prop, c, 0.0)


def _lateral_fft(x):
    """Unitary lateral DFT, exp(-2 pi i l p / Nx) / sqrt(Nx) (the F_<-> of Eq. 2)."""
    return scipy.fft.fft(x, axis=0, norm="ortho", workers=_FFT_WORKERS)


def _lateral_ifft(x):
    return scipy.fft.ifft(x, axis=0, norm="ortho", workers=_FFT_WORKERS)


# --------------------------------------------------------------------------- mode E

def forward_exact(g: Geometry, eta: np.ndarray) -> np.ndarray:
    """s = Re(K^ eta) with the Stolt resampling as a direct nonuniform DFT (Eq. 3-5, 13, 16)."""
    G = grids(g)
    eta_hat = _lateral_fft(np.asarray(eta, np.complex128))
    kz, _ = axial_wavenumber(g)
    c = modulation(g)
    X = np.empty((g.nx, g.nk), np.complex128)
    for l in range(g.nx):
        E = np.exp(1j * kz[l][:, None] * G.z[None, :])        # (nk, nz)
        X[l] = E @ eta_hat[l] / math.sqrt(g.nk)
    return np.real(_lateral_ifft(c * X))


def adjoint_exact(g: Geometry, r: np.ndarray) -> np.ndarray:
    """K^^H r for real r (Eq. 17), the adjoint of forward_exact under Re(u^H v)."""
    G = grids(g)
    R = _lateral_fft(np.asarray(r, np.float64).astype(np.complex128))
    kz, _ = axial_wavenumber(g)
    Xp = np.conj(modulation(g)) * R
    eta_hat = np.empty((g.nx, g.nk), np.complex128)
    for l in range(g.nx):
        E = np.exp(1j * kz[l][:, None] * G.z[None, :])
        eta_hat[l] = np.conj(E).T @ Xp[l] / math.sqrt(g.nk)
    return _lateral_ifft(eta_hat)


# --------------------------------------------------------------------------- mode N

def kb_scaling(g: Geometry) -> np.ndarray:
    """Scaling factors s_m = 1 / Psi(m / K) of the NUFFT (Jackson et al. 1991).

    Psi(u) = sinh(sqrt(beta^2 - (pi J u)^2)) / sqrt(beta^2 - (pi J u)^2) is the
    Fourier transform of a Kaiser-Bessel window of width J; its reciprocal
    pre-compensates the interpolation over the object rows m in [-Nz/2, Nz/2).
    Normalised to s_0 = 1 (a constant factor cancels in the least squares).
    """
    G = grids(g)
    u = G.m / G.K
    a = np.sqrt(G.beta ** 2 - (math.pi * g.J * u) ** 2)
    psi0 = math.sinh(G.beta) / G.beta
    return psi0 * a / np.sinh(a)


def stolt_points(g: Geometry):
    """Stolt points on the oversampled depth-frequency grid (Eq. 3).

    omega = kz dz is the phase step per depth row of exp(+i kz z_m);
    t = (omega mod 2 pi) K / (2 pi) locates it on the K-point grid; the J
    neighbours are g0+1 .. g0+J with g0 = floor(t) - J/2 and tau = t - floor(t).
    Returns (t, g0, tau), each (nx, nk); g0 is not yet reduced mod K.
    """
    G = grids(g)
    kz, _ = axial_wavenumber(g)
    omega = kz * G.dz
    t = np.mod(omega, 2 * math.pi) * G.K / (2 * math.pi)
    fl = np.floor(t)
    return t, fl.astype(np.int64) - g.J // 2, t - fl


def minmax_system(g: Geometry):
    """The least-squares system that defines the min-max interpolator.

    C[m][j] = s_m exp(2 pi i j m / K), j = 1..J (the J grid neighbours after
    scaling); the target for a point at fractional offset tau is
    b_m(tau) = exp(2 pi i (tau + J/2) m / K).  Both are relative to the common
    unimodular factor exp(2 pi i g0 m / K), which cancels (Fessler & Sutton 2003).
    """
    G = grids(g)
    s = kb_scaling(g)
    j = np.arange(1, g.J + 1)
    C = s[:, None] * np.exp(2j * math.pi * np.outer(G.m, j) / G.K)
    return C, G.m, G.K


def _targets(g, tau, m, K):
    return np.exp(2j * math.pi * np.outer(m, np.asarray(tau) + g.J / 2) / K)   # (nz, npts)


def minmax_weights(g: Geometry, tau: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """Min-max interpolation weights u(tau) = argmin_u ||b(tau) - C u||_2, exact per point.

    Solved with the reduced QR of C (a library least-squares route).  Returns
    an array of shape tau.shape + (J,).
    """
    C, m, K = minmax_system(g)
    Q, Rm = np.linalg.qr(C)
    flat = np.asarray(tau, np.float64).ravel()
    out = np.empty((flat.size, g.J), np.complex128)
    for a in range(0, flat.size, chunk):
        b = _targets(g, flat[a:a + chunk], m, K)
        out[a:a + chunk] = scipy.linalg.solve_triangular(Rm, Q.conj().T @ b).T
    return out.reshape(np.shape(tau) + (g.J,))


def minmax_error(g: Geometry, tau: np.ndarray) -> np.ndarray:
    """Worst-case error per unit ||eta_hat column||: ||b(tau) - C u(tau)||_2 / sqrt(Nz)."""
    C, m, K = minmax_system(g)
    tau = np.atleast_1d(np.asarray(tau, np.float64))
    u = minmax_weights(g, tau)
    b = _targets(g, tau, m, K)
    res = b - C @ u.T
    return np.linalg.norm(res, axis=0) / math.sqrt(g.nk)


def _oversampled_spectrum(g: Geometry, eta_hat_rows: np.ndarray) -> np.ndarray:
    """Y[g] = sum_m s_m eta_hat[m] exp(+2 pi i g m / K) for each given lateral row.

    Row m is placed at index (m mod K) of a zero-padded length-K buffer.
    """
    G = grids(g)
    s = kb_scaling(g)
    rows = np.atleast_2d(eta_hat_rows)
    buf = np.zeros((rows.shape[0], G.K), np.complex128)
    buf[:, np.mod(G.m, G.K)] = rows * s[None, :]
    return G.K * scipy.fft.ifft(buf, axis=1, workers=_FFT_WORKERS)


def _interp_matrix(g: Geometry, l: int, rows=None, tables=None) -> scipy.sparse.csr_matrix:
    """Sparse interpolation matrix P_l (len(rows) x K) of column l: u_j(tau_n) at (g0_n + j) mod K."""
    G = grids(g)
    t, g0, tau = tables if tables is not None else stolt_points(g)
    n = np.arange(g.nk) if rows is None else np.asarray(rows)
    u = minmax_weights(g, tau[l, n])                                   # (len(n), J)
    cols = np.mod(g0[l, n][:, None] + np.arange(1, g.J + 1)[None, :], G.K)
    ridx = np.repeat(np.arange(n.size), g.J)
    return scipy.sparse.csr_matrix((u.ravel(), (ridx, cols.ravel())), shape=(n.size, G.K))


def _check_support(spec, columns, what):
    if columns is None:
        return
    mask = np.ones(spec.shape[0], bool)
    mask[list(columns)] = False
    if mask.any():
        off = np.abs(spec[mask]).max()
        scale = max(np.abs(spec).max(), 1e-300)
        if off > 1e-12 * scale:
            raise ValueError(f"{what}: lateral spectrum is not confined to the given columns")


def forward_nufft(g: Geometry, eta: np.ndarray, columns=None, rows=None, P=None) -> np.ndarray:
    """s = Re(K^ eta) with the Stolt resampling done by the min-max NUFFT (Eq. 16).

    X_hat[l][n] = Nz^{-1/2} sum_j u_j(tau_ln) Y[l][(g0_ln + j) mod K].
    ``columns``: lateral frequencies l on which eta's lateral spectrum is
    supported (checked); others are skipped.  ``rows``: compute only these
    spectral samples n (the lateral inverse FFT is still exact for them).
    ``P``: optional cache {l: P_l} of interpolation matrices for all rows.
    """
    eta_hat = _lateral_fft(np.asarray(eta, np.complex128))
    _check_support(eta_hat, columns, "forward_nufft")
    cols = range(g.nx) if columns is None else sorted(set(columns))
    nsel = np.arange(g.nk) if rows is None else np.asarray(rows)
    c = modulation(g)[:, nsel]
    tables = stolt_points(g)
    X = np.zeros((g.nx, nsel.size), np.complex128)
    for l in cols:
        Y = _oversampled_spectrum(g, eta_hat[l])[0]
        if P is not None and rows is None:
            Pl = P[l]
        else:
            Pl = _interp_matrix(g, l, nsel, tables)
        X[l] = Pl @ Y / math.sqrt(g.nk)
    return np.real(_lateral_ifft(c * X))


def adjoint_nufft(g: Geometry, r: np.ndarray, columns=None, P=None) -> np.ndarray:
    """K^^H r for real r through the adjoint NUFFT N' (Eq. 17).

    Y'[l] = P_l^H (conj(c) R)[l];  eta_hat'[l][m] = Nz^{-1/2} s_m sum_g Y'[l][g] exp(-2 pi i g m / K).
    ``columns``: lateral frequencies on which r's lateral spectrum is supported.
    """
    G = grids(g)
    R = _lateral_fft(np.asarray(r, np.float64).astype(np.complex128))
    _check_support(R, columns, "adjoint_nufft")
    cols = range(g.nx) if columns is None else sorted(set(columns))
    Xp = np.conj(modulation(g)) * R
    s = kb_scaling(g)
    tables = stolt_points(g)
    eta_hat = np.zeros((g.nx, g.nk), np.complex128)
    for l in cols:
        Pl = P[l] if P is not None else _interp_matrix(g, l, None, tables)
        Yp = Pl.conj().T @ Xp[l]
        full = scipy.fft.fft(Yp)                     # sum_g Y'[g] exp(-2 pi i g m / K) at index m mod K
        eta_hat[l] = s * full[np.mod(G.m, G.K)] / math.sqrt(g.nk)
    return _lateral_ifft(eta_hat)


def default_workers() -> int:
    """Worker processes for building interpolation matrices: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:          # pragma: no cover - platforms without affinity
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _interp_chunk(g: Geometry, q2, cols):
    """Interpolation matrices of the given columns (a unit of work for a worker process).

    q2 None: the B-scan columns l of g (stolt_points); otherwise the per-column lateral
    frequencies of a volume (_column_model).  Same arithmetic as a serial build.
    """
    # the small dense products of the per-point least squares run fastest on one BLAS thread
    # (and then round alike in every process)
    with threadpool_limits(limits=1):
        if q2 is None:
            tables = stolt_points(g)
        else:
            tables = _column_model(g, q2)[2]
        return [_interp_matrix(g, l, None, tables) for l in cols]


def _interp_matrices(g: Geometry, ncols: int, q2=None, workers: int = 1) -> list:
    """P_l for l < ncols, built serially or split over `workers` spawned processes.

    Only the order of construction changes with `workers`; every matrix is produced by
    _interp_matrix from the same tables, so the result is identical.
    """
    if workers <= 1 or ncols < 2 * workers:
        return _interp_chunk(g, q2, range(ncols))
    chunks = [list(range(ncols))[i::workers] for i in range(workers)]
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        parts = list(ex.map(_interp_chunk, [g] * workers, [q2] * workers, chunks))
    out = [None] * ncols
    for ch, mats in zip(chunks, parts):
        for l, m in zip(ch, mats):
            out[l] = m
    return out


class Operator:
    """A = Re o K^ and A^H with cached interpolation matrices (mode N) for repeated use.

    ``workers`` > 1 builds the matrices in that many processes (large grids only; the
    matrices, and hence every result, are the same as with one).
    """

    def __init__(self, g: Geometry, mode: str = "N", workers: int = 1):
        self.g = g
        self.mode = mode
        self.P = None
        if mode == "N":
            mats = _interp_matrices(g, g.nx, None, workers)
            self.P = {l: mats[l] for l in range(g.nx)}
        elif mode != "E":
            raise ValueError(mode)

    def A(self, eta):
        if self.mode == "E":
            return forward_exact(self.g, eta)
        return forward_nufft(self.g, eta, P=self.P)

    def AH(self, r):
        if self.mode == "E":
            return adjoint_exact(self.g, r)
        return adjoint_nufft(self.g, r, P=self.P)


def forward(g: Geometry, eta, mode: str = "N"):
    return forward_exact(g, eta) if mode == "E" else forward_nufft(g, eta)


def adjoint(g: Geometry, r, mode: str = "N"):
    return adjoint_exact(g, r) if mode == "E" else adjoint_nufft(g, r)


def dense_matrix(g: Geometry, mode: str = "E") -> np.ndarray:
    """The real-linear map A as a dense (Nx Nk) x (2 Nx Nk) real matrix (tiny grids only).

    Column 2i is A applied to the i-th unit vector, column 2i+1 to j times it.
    """
    op = Operator(g, mode)
    n = g.nx * g.nk
    M = np.empty((n, 2 * n))
    for i in range(n):
        e = np.zeros(n, np.complex128)
        e[i] = 1.0
        M[:, 2 * i] = op.A(e.reshape(g.nx, g.nk)).ravel()
        e[i] = 1j
        M[:, 2 * i + 1] = op.A(e.reshape(g.nx, g.nk)).ravel()
    return M


# --------------------------------------------------------------------------- volumes

def volume_q2(g: Geometry) -> np.ndarray:
    """q^2 = qx^2 + qy^2 of every lateral-frequency column of a volume, shape (ny, nx).

    The 3-D form of the model (Sec. "Background": N = Nx Ny Nz): the lateral DFT runs
    over both lateral axes (FFT order on each), and the Stolt map of Eq. 3 uses the
    total lateral frequency.
    """
    dy = g.dy if g.dy > 0 else g.dx
    qx = 2 * math.pi * np.fft.fftfreq(g.nx, d=1.0 / g.nx) / (g.nx * g.dx)
    qy = 2 * math.pi * np.fft.fftfreq(g.ny, d=1.0 / g.ny) / (g.ny * dy)
    return qy[:, None] ** 2 + qx[None, :] ** 2


def _column_model(g: Geometry, q2: np.ndarray):
    """Per-column pieces for arbitrary lateral frequencies (q2: one value per column).

    Returns kz (propagating part, else 0), the modulation c of Eq. 13/16 (beam filter,
    dispersion, focal reference) and the Stolt points (t, g0, tau) on the K-point grid;
    arrays of shape (len(q2), nk).  These are the B-scan definitions of beam_filter,
    modulation and stolt_points with q_l^2 replaced by the column's q^2.
    """
    G = grids(g)
    q2 = np.asarray(q2, np.float64)
    arg = 4 * G.k[None, :] ** 2 - q2[:, None]
    prop = arg > 0
    kz = np.sqrt(np.where(prop, arg, 0.0))
    B = np.where(prop, np.exp(-q2[:, None] * g.waist ** 2 / 8.0), 0.0)
    c = B * np.exp(1j * dispersion_phase(g)[None, :]) * np.exp(1j * (2 * G.k[None, :] - kz) * g.z_focus)
    c = np.where(prop, c, 0.0)
    t = np.mod(kz * G.dz, 2 * math.pi) * G.K / (2 * math.pi)
    fl = np.floor(t)
    return kz, c, (t, fl.astype(np.int64) - g.J // 2, t - fl)


class VolumeOperator:
    """A = Re o K^ and A^H for a volume eta[ny][nx][nz] (complex) -> s[ny][nx][nk] (real).

    Eq. 16 with a two-dimensional unitary lateral DFT; each (qy, qx) column gets the
    B-scan's resampling (mode E: direct nonuniform DFT; mode N: min-max NUFFT) and
    modulation with q^2 = qx^2 + qy^2.
    """

    def __init__(self, g: Geometry, mode: str = "N", workers: int = 1):
        if mode not in ("E", "N"):
            raise ValueError(mode)
        self.g, self.mode = g, mode
        self.q2 = volume_q2(g).ravel()                     # column index ly * nx + lx
        self.kz, self.c, tables = _column_model(g, self.q2)
        self.P = None
        if mode == "N":
            self.P = _interp_matrices(g, self.q2.size, self.q2, workers)

    def _resample(self, eta_hat_cols):
        G = grids(self.g)
        X = np.empty_like(eta_hat_cols)
        for i in range(eta_hat_cols.shape[0]):
            if self.mode == "E":
                X[i] = np.exp(1j * self.kz[i][:, None] * G.z[None, :]) @ eta_hat_cols[i]
            else:
                X[i] = self.P[i] @ _oversampled_spectrum(self.g, eta_hat_cols[i])[0]
        return X / math.sqrt(self.g.nk)

    def A(self, eta):
        g = self.g
        eta_hat = scipy.fft.fft2(np.asarray(eta, np.complex128), axes=(0, 1), norm="ortho",
                                 workers=_FFT_WORKERS)
        X = self._resample(eta_hat.reshape(g.ny * g.nx, g.nk))
        return np.real(scipy.fft.ifft2((self.c * X).reshape(g.ny, g.nx, g.nk), axes=(0, 1), norm="ortho",
                                       workers=_FFT_WORKERS))

    def AH(self, r):
        g = self.g
        G = grids(g)
        R = scipy.fft.fft2(np.asarray(r, np.float64).astype(np.complex128), axes=(0, 1), norm="ortho",
                           workers=_FFT_WORKERS)
        Xp = np.conj(self.c) * R.reshape(g.ny * g.nx, g.nk)
        s = kb_scaling(g)
        out = np.empty_like(Xp)
        for i in range(Xp.shape[0]):
            if self.mode == "E":
                out[i] = np.conj(np.exp(1j * self.kz[i][:, None] * G.z[None, :])).T @ Xp[i]
            else:
                full = scipy.fft.fft(self.P[i].conj().T @ Xp[i])
                out[i] = s * full[np.mod(G.m, G.K)]
        out /= math.sqrt(g.nk)
        return scipy.fft.ifft2(out.reshape(g.ny, g.nx, g.nk), axes=(0, 1), norm="ortho",
                               workers=_FFT_WORKERS)

    def calibration_gradient(self, eta, grad_s) -> np.ndarray:
        """Gradient of <grad_s, A eta> with respect to (a2, a3, z_focus) for a volume.

        As for a B-scan (calibration_gradient): d/dtheta = Re sum conj(F grad_s) (i D_theta c X)
        with F the two-dimensional unitary lateral DFT and D = ((k-k0)^2, (k-k0)^3, 2k - kz).
        """
        g = self.g
        G = grids(g)
        eta_hat = scipy.fft.fft2(np.asarray(eta, np.complex128), axes=(0, 1), norm="ortho",
                                 workers=_FFT_WORKERS)
        X = self._resample(eta_hat.reshape(g.ny * g.nx, g.nk))
        Gs = scipy.fft.fft2(np.asarray(grad_s, np.float64).astype(np.complex128), axes=(0, 1), norm="ortho",
                            workers=_FFT_WORKERS)
        base = np.conj(Gs.reshape(g.ny * g.nx, g.nk)) * 1j * self.c * X
        d = (G.k - G.kc)[None, :]
        derivs = (np.broadcast_to(d ** 2, base.shape), np.broadcast_to(d ** 3, base.shape), 2 * G.k[None, :] - self.kz)
        return np.array([float(np.sum(np.real(base * D))) for D in derivs])


# --------------------------------------------------------------------------- calibration

def resampled_spectrum(g: Geometry, eta: np.ndarray, mode: str = "N", columns=None, P=None) -> np.ndarray:
    """X[l][n] = Nz^{-1/2} sum_m eta_hat[l][m] exp(+i kz[l][n] z_m), before the modulation c.

    Mode E evaluates the sum directly (Eq. 3); mode N through the min-max NUFFT
    (Eq. 16).  ``columns`` restricts the work to lateral frequencies on which
    eta's lateral spectrum is supported (checked); X is zero elsewhere.
    """
    G = grids(g)
    eta_hat = _lateral_fft(np.asarray(eta, np.complex128))
    _check_support(eta_hat, columns, "resampled_spectrum")
    cols = range(g.nx) if columns is None else sorted(set(columns))
    kz, _ = axial_wavenumber(g)
    tables = stolt_points(g) if mode == "N" else None
    X = np.zeros((g.nx, g.nk), np.complex128)
    for l in cols:
        if mode == "E":
            E = np.exp(1j * kz[l][:, None] * G.z[None, :])
            X[l] = E @ eta_hat[l] / math.sqrt(g.nk)
        elif mode == "N":
            Pl = P[l] if P is not None else _interp_matrix(g, l, None, tables)
            X[l] = Pl @ _oversampled_spectrum(g, eta_hat[l])[0] / math.sqrt(g.nk)
        else:
            raise ValueError(mode)
    return X


def calibration_derivatives(g: Geometry):
    """D_theta with dc/dtheta = i D_theta c for theta = (a2, a3, z_focus).

    From c = B e^{i phi} e^{i (2k - kz) z_f} and phi = a2 (k-k0)^2 + a3 (k-k0)^3
    (Eq. 7, 13): D = ((k-k0)^2, (k-k0)^3, 2k - kz), each of shape (nx, nk).
    """
    G = grids(g)
    kz, _ = axial_wavenumber(g)
    d = np.broadcast_to((G.k - G.kc)[None, :], (g.nx, g.nk))
    return d ** 2, d ** 3, 2 * G.k[None, :] - kz


def calibration_gradient(g: Geometry, eta: np.ndarray, grad_s: np.ndarray, mode: str = "N",
                         columns=None, P=None) -> np.ndarray:
    """Gradient of <grad_s, A eta> with respect to theta = (a2, a3, z_focus).

    A eta = Re(F^{-1}(c X)) with F the unitary lateral DFT; for real grad_s,
    <grad_s, Re F^{-1} Y> = Re sum conj(F grad_s) Y, hence
    d/dtheta = Re sum conj(F grad_s) (i D_theta c X).
    """
    X = resampled_spectrum(g, eta, mode, columns, P)
    Gs = _lateral_fft(np.asarray(grad_s, np.float64).astype(np.complex128))
    cX = modulation(g) * X
    base = np.conj(Gs) * 1j * cX
    return np.array([float(np.sum(np.real(base * D))) for D in calibration_derivatives(g)])


# --------------------------------------------------------------------------- baseline image

def direct_image(g: Geometry, y: np.ndarray) -> np.ndarray:
    """The "direct IFFT" image of Eq. 9 (Sec. "Methods under test"): dispersion compensation
    e^{-j phi} on each measured A-scan, then the inverse transform along the spectral axis.

    eta_d[p][m] = Nz^{-1/2} sum_n y[p][n] e^{-j phi(k_n)} e^{-2 j k_n z_m}, on the full-range
    depth grid of the operator (rows m in [-Nz/2, Nz/2) at index m + Nz/2).  It is the adjoint
    of the one-A-scan model with no lateral coupling (no Stolt map, beam filter or focus), so by
    Eq. 9 it holds half the object plus the doubly dispersed conjugate mirror.  The kernel
    e^{-2 j k_n z_m} is the one of the operator; a plain IFFT over the sample index differs from
    it by a unimodular phase per depth row and by its normalisation.
    Written as the direct sum (a dense matrix product), the definition.
    """
    G = grids(g)
    y = np.asarray(y, np.float64)
    Yd = y * np.exp(-1j * dispersion_phase(g))[None, :]
    E = np.exp(-2j * np.outer(G.k, G.z))                     # (nk, nz)
    return (Yd @ E) / math.sqrt(g.nk)


# --------------------------------------------------------------------------- solver

def soft_threshold(u: np.ndarray, theta) -> np.ndarray:
    """Weighted complex soft threshold of Eq. 14 with threshold theta_i (= lambda w_i times the step).

    T(u) = u max(|u| - theta, 0) / (max(|u| - theta, 0) + theta); theta = 0 is
    the identity (the quotient is read as 1 there).
    """
    u = np.asarray(u, np.complex128)
    theta = np.broadcast_to(np.asarray(theta, np.float64), u.shape)
    shrink = np.maximum(np.abs(u) - theta, 0.0)
    den = shrink + theta
    factor = np.divide(shrink, den, out=np.ones_like(shrink), where=den > 0)
    factor = np.where(theta == 0, 1.0, factor)
    return u * factor


def lipschitz(op, shape, iters: int = 50, seed: int = 0, safety: float = 1.01) -> float:
    """Step-size constant L >= ||A||^2 by power iteration on A^H A.

    The paper's fixed step 1/N (Alg. 1) depends on an unstated normalisation;
    L from power iteration is the normalisation-free equivalent.  ``op`` has
    methods A and AH.  Returns safety * the final Rayleigh quotient.
    """
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)
    x /= np.linalg.norm(x)
    ray = 0.0
    for _ in range(iters):
        Ax = op.A(x)
        ray = float(np.sum(Ax * Ax))          # ||A x||^2 with ||x|| = 1
        y = op.AH(Ax)
        x = y / np.linalg.norm(y)
    return safety * ray


def lambda_max(op, y: np.ndarray, w=None) -> float:
    """Smallest lambda for which eta = 0 minimises Eq. 12: max_i |(A^H y)_i| / w_i."""
    g = np.abs(op.AH(y))
    if w is not None:
        g = g / np.asarray(w, np.float64)
    return float(g.max())


@dataclass
class FistaResult:
    z: np.ndarray
    iters: int
    rel_res: list
    resid2: list
    l1: list


def fista(op, y: np.ndarray, lam: float, L: float, iters: int, w=None, tol: float = 0.0,
          add_residual: bool = False, eps: float = 1e-12, state=None) -> FistaResult:
    """MBIR full-range ISAM by FISTA (Alg. 1, Eq. 14, Eq. 15).

    Step 1/L in place of the paper's 1/N; threshold lambda w_i / L.
    eta^1 = z^0 = 0, t^1 = 1.  Per iteration k:
        g^k   = (1/L) A^H(A eta^k - y)
        z^k   = T(eta^k - g^k) with theta_i = lambda w_i / L
        r_r   = ||z^k - eta^k|| / (max(||g^k||, ||z^k - eta^k + g^k||) + eps)
        stop if tol > 0 and r_r < tol
        t^{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
        eta^{k+1} = z^k + ((t^k - 1)/t^{k+1}) (z^k - z^{k-1})
    Returns z^k, optionally plus (1/L) A^H(y - A z^k) (the optional residual step).
    ``state`` = (eta, z_prev, t, k0) resumes a run.
    """
    y = np.asarray(y, np.float64)
    shape = y.shape
    step = 1.0 / L
    w = np.ones(shape) if w is None else np.asarray(w, np.float64)
    theta = lam * w * step
    if state is None:
        eta = np.zeros(shape, np.complex128)
        z_prev = np.zeros(shape, np.complex128)
        t = 1.0
    else:
        eta, z_prev, t = state[0].copy(), state[1].copy(), state[2]
    rr_hist, res_hist, l1_hist = [], [], []
    z = z_prev
    k = 0
    for k in range(1, iters + 1):
        r = op.A(eta) - y
        gk = step * op.AH(r)
        z = soft_threshold(eta - gk, theta)
        d = z - eta
        rr = np.linalg.norm(d) / (max(np.linalg.norm(gk), np.linalg.norm(d + gk)) + eps)
        rr_hist.append(rr)
        res_hist.append(float(np.sum(r * r)))
        l1_hist.append(float(np.sum(w * np.abs(z))))
        if tol > 0 and rr < tol:
            break
        t_next = (1 + math.sqrt(1 + 4 * t * t)) / 2
        eta = z + ((t - 1) / t_next) * (z - z_prev)
        z_prev = z
        t = t_next
    out = z
    if add_residual:
        out = z + step * op.AH(y - op.A(z))
    res = FistaResult(out, k, rr_hist, res_hist, l1_hist)
    res.state = (eta, z_prev, t)
    return res
