"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test ties one part of the oracle to a closed form, a special case that
reduces to a library routine, an identity, brute force on a tiny grid, or the
method's own error bound, so that a dropped term, a wrong sign or index, or a
transposed operand fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import phantoms as ph


def tiny_geom(nx=4, nk=16, **kw):
    o = ph.custom_optics(nx, nk, **kw)
    return O.Geometry.of(o)


def rand_obj(rng, nx, nk, clear_edge=True):
    x = ph.complex_gaussian(rng, (nx, nk))
    if clear_edge:
        x[:, 0] = 0.0          # row m = -nz/2 has no mirror partner
    return x


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ------------------------------------------------------------------ special cases of the model

@pytest.mark.parametrize("nk", [16, 64])
def test_in_focus_limit_single_ascan_is_dispersed_fft(nk):
    """Nx = 1 (only q = 0): the Stolt map is the identity and A is a dispersed DFT per A-scan.

    With k_c / dk = P an integer, exp(+i 2 k_n z_m) = exp(2 pi i (n + P - nk/2) m / nk),
    so A eta = Re(e^{i phi} sqrt(nk) ifft(ifftshift(eta))[(n + P - nk/2) mod nk]) (numpy FFT).
    """
    lam = 1300e-9
    g = O.Geometry(nx=1, nk=nk, dx=4e-6, lambda_c=lam, dlambda=lam / 7.5, waist=8e-6,
                   z_focus=3e-4, a2=3e-10, a3=1e-16)
    G = O.grids(g)
    P = G.kc / G.dk
    assert abs(P - round(P)) < 1e-6
    P = int(round(P))
    rng = np.random.default_rng(1)
    eta = rand_obj(rng, 1, nk, clear_edge=False)
    phi = O.dispersion_phase(g)
    idx = np.mod(np.arange(nk) + P - nk // 2, nk)
    X = math.sqrt(nk) * np.fft.ifft(np.fft.ifftshift(eta[0]))[idx]
    want = np.real(np.exp(1j * phi) * X)
    got = O.forward_exact(g, eta)[0]
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # adjoint of the same special case: place e^{-i phi} r at (n + P - nk/2) mod nk, forward FFT
    r = rng.standard_normal((1, nk))
    v = np.zeros(nk, np.complex128)
    v[idx] = np.exp(-1j * phi) * r[0]
    want_a = np.fft.fftshift(np.fft.fft(v)) / math.sqrt(nk)
    got_a = O.adjoint_exact(g, r)[0]
    assert np.abs(got_a - want_a).max() < 1e-12 * np.abs(want_a).max()


def test_focal_row_object_has_no_stolt_warp():
    """An object confined to the focal row images without defocus.

    With z_f = m_f dz on the grid, c X = B e^{i phi} e^{i 2 k z_f} eta_hat[l][m_f] / sqrt(nz):
    the kz dependence of exp(i kz z_f) and of the focal reference cancel exactly.
    """
    g = tiny_geom(8, 32, focus_rows=5)
    G = O.grids(g)
    mf = 5
    rng = np.random.default_rng(2)
    eta = np.zeros((g.nx, g.nk), np.complex128)
    eta[:, mf + g.nk // 2] = ph.complex_gaussian(rng, g.nx)
    eta_hat_row = np.fft.fft(eta[:, mf + g.nk // 2], norm="ortho")
    B = O.beam_filter(g)
    phi = O.dispersion_phase(g)
    Xt = B * np.exp(1j * phi)[None, :] * np.exp(2j * G.k * mf * G.dz)[None, :] \
        * eta_hat_row[:, None] / math.sqrt(g.nk)
    want = np.real(np.fft.ifft(Xt, axis=0, norm="ortho"))
    got = O.forward_exact(g, eta)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()
    # mode N agrees within its interpolation bound (relative 1e-5)
    assert rel(O.forward_nufft(g, eta), want) < 1e-5


@pytest.mark.parametrize("mode", ["E", "N"])
def test_mirror_symmetry(mode):
    """Conjugate mirror M eta[p][m] = conj(eta[p][-m]): A_{zf,a}(M eta) = A_{-zf,-a}(eta) (Eq. 6, 8).

    At zero dispersion and focus the two coincide: the full-range ambiguity that the
    dispersion encoding breaks.
    """
    g = tiny_geom(8, 32, focus_rows=4)
    rng = np.random.default_rng(3)
    eta = rand_obj(rng, g.nx, g.nk)
    mir = np.zeros_like(eta)
    mir[:, 1:] = np.conj(eta[:, :0:-1])
    gm = g.with_(z_focus=-g.z_focus, a2=-g.a2, a3=-g.a3)
    lhs = O.forward(g, mir, mode)
    rhs = O.forward(gm, eta, mode)
    tol = 1e-12 if mode == "E" else 2e-5
    assert rel(lhs, rhs) < tol
    g0 = g.with_(z_focus=0.0, a2=0.0, a3=0.0)
    assert rel(O.forward(g0, mir, mode), O.forward(g0, eta, mode)) < tol
    # with dispersion the mirror images differ at O(1)
    assert rel(O.forward(g, mir, mode), O.forward(g, eta, mode)) > 0.1


def test_beam_filter_is_the_two_way_gaussian_angular_spectrum():
    """B(q) of Eq. 3 for a Gaussian beam of waist w0: the field at the focus is exp(-x^2/w0^2)
    one way, exp(-2 x^2 / w0^2) for illumination times collection.  Its Fourier transform,
    normalised at q = 0, is exp(-q^2 w0^2 / 8).  Here that transform is taken numerically: the
    unitary DFT (numpy) of the sampled two-way field on a lateral grid much wider than the beam
    and finely sampled (aliasing below e^-300), at the oracle's own lateral frequencies."""
    w0 = 8e-6
    g = O.Geometry(nx=512, nk=16, dx=0.5e-6, lambda_c=1300e-9, dlambda=170e-9, waist=w0,
                   z_focus=0.0, a2=0.0, a3=0.0)
    x = g.dx * np.fft.fftfreq(g.nx, d=1.0 / g.nx)             # periodic grid centred on x = 0
    field2 = np.exp(-2 * x ** 2 / w0 ** 2)
    F = np.fft.fft(field2)
    want = np.real(F / F[0])
    B = O.beam_filter(g)
    assert np.all(B == B[:, :1])                               # no k dependence for a fixed waist
    assert np.abs(B[:, 0] - want).max() < 1e-12
    assert B[g.nx // 8, 0] < 0.5                               # the filter is not trivially flat here


def test_dispersion_phase_at_band_centre_and_edges():
    """Eq. 7 with k0 the centre wavenumber 2 pi / lambda_c: the workloads state dispersion as
    the phase the quadratic (cubic) term reaches at the band edge |k - k0| = band / 2.  Sample 0
    sits at k0 - band/2 and sample nk/2 at k0 (uniform sampling in k over the band), so
    phi[0] = E2 - E3 and phi[nk/2] = 0, and the even and odd parts about the centre sample follow
    the two edge phases at every offset."""
    nk = 64
    E2, E3 = 40 * math.pi, 8 * math.pi
    g = O.Geometry.of(ph.custom_optics(8, nk, edge_phase2=E2, edge_phase3=E3))
    phi = O.dispersion_phase(g)
    assert abs(phi[0] - (E2 - E3)) < 1e-9
    assert abs(phi[nk // 2]) < 1e-12
    j = np.arange(1, nk // 2)
    u = 2 * j / nk                                             # |k - k0| / (band / 2)
    even = (phi[nk // 2 + j] + phi[nk // 2 - j]) / 2
    odd = (phi[nk // 2 + j] - phi[nk // 2 - j]) / 2
    assert np.abs(even - E2 * u ** 2).max() < 1e-9
    assert np.abs(odd - E3 * u ** 3).max() < 1e-9


# ------------------------------------------------------------------ adjoint

@pytest.mark.parametrize("mode", ["E", "N"])
def test_adjoint_dot_product(mode):
    """sum (A x) y = Re <x, A^H y> for the real-linear A (Eq. 12, 17)."""
    g = tiny_geom(8, 32)
    rng = np.random.default_rng(4)
    x = rand_obj(rng, g.nx, g.nk, clear_edge=False)
    y = rng.standard_normal((g.nx, g.nk))
    Ax = O.forward(g, x, mode)
    AHy = O.adjoint(g, y, mode)
    lhs = np.sum(Ax * y)
    rhs = np.real(np.vdot(x, AHy))
    assert abs(lhs - rhs) < 1e-13 * np.linalg.norm(Ax) * np.linalg.norm(y)


@pytest.mark.parametrize("mode", ["E", "N"])
def test_dense_adjoint_is_transpose(mode):
    """Brute force on a tiny grid: A^H applied to unit spectra gives the rows of the dense matrix."""
    g = tiny_geom(4, 16)
    M = O.dense_matrix(g, mode)
    n = g.nx * g.nk
    for i in range(0, n, 7):
        e = np.zeros(n)
        e[i] = 1.0
        a = O.adjoint(g, e.reshape(g.nx, g.nk), mode).ravel()
        col = np.empty(2 * n)
        col[0::2] = a.real
        col[1::2] = a.imag
        assert np.abs(col - M[i]).max() < 1e-13


# ------------------------------------------------------------------ NUFFT (mode N)

def test_stolt_points_reproduce_the_phase_step():
    """t = (omega mod 2 pi) K / 2 pi: exp(i omega) = exp(2 pi i t / K), t = g0 + J/2 + tau, tau in [0,1)."""
    g = O.Geometry.of(ph.workload("tiny").optics)
    G = O.grids(g)
    kz, _ = O.axial_wavenumber(g)
    t, g0, tau = O.stolt_points(g)
    assert np.all((tau >= 0) & (tau < 1))
    assert np.array_equal(g0 + g.J // 2 + tau, t)
    assert np.abs(np.exp(1j * kz * G.dz) - np.exp(2j * math.pi * t / G.K)).max() < 1e-12


def test_minmax_weights_match_library_least_squares():
    """Weights of the min-max interpolator vs an SVD-based least-squares solve (LAPACK gelsd)."""
    g = O.Geometry.of(ph.workload("tiny").optics)
    C, m, K = O.minmax_system(g)
    taus = np.array([0.0, 0.125, 0.37, 0.5, 0.93])
    u = O.minmax_weights(g, taus)
    for i, tau in enumerate(taus):
        b = np.exp(2j * math.pi * m * (tau + g.J / 2) / K)
        ref = scipy.linalg.lstsq(C, b, lapack_driver="gelsd")[0]
        assert np.abs(u[i] - ref).max() < 1e-9 * np.abs(ref).max()


def test_minmax_error_level_and_convergence_in_J():
    """The min-max worst-case error with J = 6, 2x oversampling and KB scaling is a few 1e-6,
    and falls by orders of magnitude at J = 8 (Fessler & Sutton 2003)."""
    g = O.Geometry.of(ph.workload("tiny").optics)
    taus = np.linspace(0, 1, 101)
    e6 = O.minmax_error(g, taus)
    assert 1e-7 < e6.max() < 1e-5
    e8 = O.minmax_error(g.with_(J=8, kb_beta=0.0), taus)
    assert e8.max() < e6.max() / 30


def test_nufft_obeys_minmax_bound_against_brute_force_nudft():
    """Per point |X_hat - X| <= E(tau) ||eta_hat column|| where X is the brute-force nonuniform DFT."""
    g = O.Geometry.of(ph.workload("tiny").optics)
    G = O.grids(g)
    rng = np.random.default_rng(5)
    eta_hat = ph.complex_gaussian(rng, (g.nx, g.nk))
    kz, _ = O.axial_wavenumber(g)
    t, g0, tau = O.stolt_points(g)
    Ebound = O.minmax_error(g, tau.ravel()).reshape(tau.shape)
    worst = 0.0
    for l in [0, 1, g.nx // 2, g.nx - 3]:
        X = np.exp(1j * kz[l][:, None] * G.z[None, :]) @ eta_hat[l] / math.sqrt(g.nk)
        Y = O.isam_oracle._oversampled_spectrum(g, eta_hat[l])[0]
        Pl = O.isam_oracle._interp_matrix(g, l)
        Xh = Pl @ Y / math.sqrt(g.nk)
        col = np.linalg.norm(eta_hat[l])
        ratio = np.abs(Xh - X) / (Ebound[l] * col)
        worst = max(worst, ratio.max())
    assert worst <= 1.0 + 1e-6


def test_mode_n_close_to_mode_e_on_phantom():
    w = ph.workload("tiny")
    g = O.Geometry.of(w.optics)
    eta = ph.phantom(w)
    sE = O.forward_exact(g, eta)
    sN = O.forward_nufft(g, eta)
    assert rel(sN, sE) < 1e-5
    y = ph.add_noise(sE, w.snr_db, w.seed)
    assert rel(O.adjoint_nufft(g, y), O.adjoint_exact(g, y)) < 1e-5


def test_sampled_rows_and_columns_agree_with_full():
    """The oracle's restricted evaluations (used for large-grid sampling) agree with the full one."""
    g = tiny_geom(16, 64)
    rng = np.random.default_rng(6)
    spec = np.zeros((g.nx, g.nk), np.complex128)
    cols = [0, 3, g.nx - 3, g.nx // 2]
    spec[cols] = ph.complex_gaussian(rng, (len(cols), g.nk))
    eta = np.fft.ifft(spec, axis=0, norm="ortho")
    full = O.forward_nufft(g, eta)
    assert rel(O.forward_nufft(g, eta, columns=cols), full) < 1e-13
    rows = [0, 5, 31, 63]
    assert rel(O.forward_nufft(g, eta, rows=rows), full[:, rows]) < 1e-13
    rspec = np.zeros((g.nx, g.nk), np.complex128)
    rspec[3] = ph.complex_gaussian(rng, g.nk)
    rspec[g.nx - 3] = np.conj(rspec[3])
    r = np.real(np.fft.ifft(rspec, axis=0, norm="ortho"))
    assert rel(O.adjoint_nufft(g, r, columns=[3, g.nx - 3]), O.adjoint_nufft(g, r)) < 1e-13


# ------------------------------------------------------------------ norm and step

def test_operator_norm_from_svd_and_power_iteration():
    """||A||^2 from the SVD of the dense realified matrix; the oracle's power iteration finds it."""
    g = tiny_geom(4, 16)
    M = O.dense_matrix(g, "E")
    smax2 = scipy.linalg.svdvals(M)[0] ** 2
    assert abs(smax2 - 1.0) < 1e-10          # unitary lateral FFT and Nz^{-1/2} depth DFT, B(0,k) = 1
    op = O.Operator(g, "E")
    L = O.lipschitz(op, (g.nx, g.nk), iters=200, seed=0, safety=1.0)
    assert abs(L - smax2) < 1e-8
    MN = O.dense_matrix(g, "N")
    sN = scipy.linalg.svdvals(MN)[0] ** 2
    assert abs(sN - 1.0) < 1e-4
    # many singular values sit near 1, so the Rayleigh quotient approaches sN slowly from below
    LN = O.lipschitz(O.Operator(g, "N"), (g.nx, g.nk), iters=200, safety=1.0)
    assert -1e-12 <= sN - LN < 1e-5


# ------------------------------------------------------------------ prox and FISTA

@pytest.mark.parametrize("mode", ["E", "N"])
def test_calibration_gradient_matches_central_differences(mode):
    """d<G, A_theta eta>/dtheta against FP64 central differences of the forward operator."""
    g = tiny_geom(8, 64, edge_phase2=6 * math.pi, edge_phase3=2 * math.pi, focus_rows=9)
    rng = np.random.default_rng(3)
    eta = rand_obj(rng, g.nx, g.nk, clear_edge=False)
    G = rng.standard_normal((g.nx, g.nk))
    an = O.calibration_gradient(g, eta, G, mode)
    for i, name in enumerate(("a2", "a3", "z_focus")):
        v = getattr(g, name)
        h = 1e-5 * abs(v)
        fp = np.sum(G * O.forward(g.with_(**{name: v + h}), eta, mode))
        fm = np.sum(G * O.forward(g.with_(**{name: v - h}), eta, mode))
        assert abs(an[i] - (fp - fm) / (2 * h)) < 1e-6 * abs(an[i]), name


def test_focus_does_not_act_on_a_single_ascan():
    """With one A-scan only q = 0 exists, where the Stolt map is the identity (kz = 2k):
    the focal depth changes nothing and its gradient vanishes."""
    g = tiny_geom(1, 64, edge_phase2=6 * math.pi, focus_rows=9)
    rng = np.random.default_rng(4)
    eta = rand_obj(rng, 1, 64, clear_edge=False)
    s0 = O.forward_exact(g, eta)
    s1 = O.forward_exact(g.with_(z_focus=3 * g.z_focus), eta)
    assert np.max(np.abs(s0 - s1)) < 1e-12 * np.max(np.abs(s0))
    G = rng.standard_normal((1, 64))
    grad = O.calibration_gradient(g, eta, G, "E")
    assert grad[2] == 0.0 and grad[0] != 0.0


# --------------------------------------------------------------- volumes

def _vol(nx, ny, nk, dy=None, **kw):
    o = ph.custom_optics(nx, nk, edge_phase2=6 * math.pi, edge_phase3=2 * math.pi, focus_rows=5, **kw)
    return O.Geometry.of(o, ny=ny, dy=dy if dy is not None else o.dx), o


@pytest.mark.parametrize("mode", ["E", "N"])
def test_volume_constant_along_y_is_the_bscan_operator(mode):
    """Only qy = 0 columns: every y row of A eta equals the B-scan operator of that row."""
    g, o = _vol(8, 4, 32, dy=5e-6)
    rng = np.random.default_rng(11)
    x0 = rand_obj(rng, 8, 32, clear_edge=False)
    sv = O.VolumeOperator(g, mode).A(np.broadcast_to(x0, (4, 8, 32)))
    s1 = O.forward(O.Geometry.of(o), x0, mode)
    assert np.abs(sv - s1[None]).max() < 1e-12 * np.abs(s1).max()


@pytest.mark.parametrize("mode", ["E", "N"])
def test_volume_constant_along_x_is_the_bscan_operator_along_y(mode):
    """Only qx = 0 columns: the volume acts along y as a B-scan of ny A-scans at pitch dy."""
    g, o = _vol(4, 8, 32, dy=3e-6)
    rng = np.random.default_rng(12)
    x0 = rand_obj(rng, 8, 32, clear_edge=False)              # [y][z]
    sv = O.VolumeOperator(g, mode).A(np.broadcast_to(x0[:, None, :], (8, 4, 32)))
    gy = O.Geometry.of(o, nx=8, dx=3e-6)
    s1 = O.forward(gy, x0, mode)
    assert np.abs(sv - s1[:, None, :]).max() < 1e-12 * np.abs(s1).max()


@pytest.mark.parametrize("mode", ["E", "N"])
def test_volume_adjoint_and_transpose_symmetry(mode):
    g, _ = _vol(8, 8, 32)
    V = O.VolumeOperator(g, mode)
    rng = np.random.default_rng(13)
    x = ph.complex_gaussian(rng, (8, 8, 32))
    y = rng.standard_normal((8, 8, 32))
    Ax = V.A(x)
    assert abs(np.sum(Ax * y) - np.real(np.vdot(x, V.AH(y)))) < 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
    # square lateral grid, equal pitches: swapping x and y commutes with A
    sw = V.A(np.swapaxes(x, 0, 1))
    assert np.abs(sw - np.swapaxes(Ax, 0, 1)).max() < 1e-12 * np.abs(Ax).max()


@pytest.mark.parametrize("mode", ["E", "N"])
def test_volume_calibration_gradient_matches_central_differences(mode):
    g, _ = _vol(8, 4, 32, dy=5e-6)
    rng = np.random.default_rng(15)
    x = ph.complex_gaussian(rng, (4, 8, 32))
    G = rng.standard_normal((4, 8, 32))
    an = O.VolumeOperator(g, mode).calibration_gradient(x, G)
    for i, name in enumerate(("a2", "a3", "z_focus")):
        v = getattr(g, name)
        h = 1e-5 * abs(v)
        fp = np.sum(G * O.VolumeOperator(g.with_(**{name: v + h}), mode).A(x))
        fm = np.sum(G * O.VolumeOperator(g.with_(**{name: v - h}), mode).A(x))
        assert abs(an[i] - (fp - fm) / (2 * h)) < 1e-6 * abs(an[i]), name


def test_volume_nufft_close_to_exact():
    g, _ = _vol(8, 4, 64, dy=5e-6)
    rng = np.random.default_rng(14)
    x = ph.complex_gaussian(rng, (4, 8, 64))
    e = O.VolumeOperator(g, "E").A(x)
    n = O.VolumeOperator(g, "N").A(x)
    assert 0 < rel(n, e) < 1e-5


def test_soft_threshold_closed_form_and_edges():
    """Eq. 14 equals u - theta u/|u| for |u| > theta and 0 otherwise; theta = 0 is the identity."""
    rng = np.random.default_rng(7)
    u = ph.complex_gaussian(rng, 1000) * 3
    theta = rng.uniform(0, 2, 1000)
    want = np.where(np.abs(u) > theta, u - theta * u / np.abs(u), 0)
    assert np.abs(O.soft_threshold(u, theta) - want).max() < 1e-14
    assert O.soft_threshold(np.array([0j]), 0.5)[0] == 0
    assert O.soft_threshold(np.array([0.5 + 0j]), 0.5)[0] == 0
    v = np.array([1 + 2j, 0j])
    assert np.array_equal(O.soft_threshold(v, 0.0), v)


class DenseOp:
    """A and A^H from a dense realified matrix (fast stand-in for tiny FISTA runs)."""

    def __init__(self, M, shape):
        self.M, self.shape = M, shape

    def A(self, x):
        v = np.empty(2 * x.size)
        v[0::2] = x.real.ravel()
        v[1::2] = x.imag.ravel()
        return (self.M @ v).reshape(self.shape)

    def AH(self, r):
        v = self.M.T @ r.ravel()
        return (v[0::2] + 1j * v[1::2]).reshape(self.shape)


def _tiny_problem():
    g = tiny_geom(4, 16)
    M = O.dense_matrix(g, "E")
    op = DenseOp(M, (g.nx, g.nk))
    rng = np.random.default_rng(8)
    x = np.zeros((g.nx, g.nk), np.complex128)
    idx = rng.choice(g.nx * g.nk, 6, replace=False)
    x.ravel()[idx] = ph.complex_gaussian(rng, 6)
    y = op.A(x) + 0.01 * rng.standard_normal((g.nx, g.nk))
    return g, op, y


def test_dense_op_matches_operator():
    g, op, y = _tiny_problem()
    rng = np.random.default_rng(9)
    x = rand_obj(rng, g.nx, g.nk, clear_edge=False)
    assert rel(op.A(x), O.forward_exact(g, x)) < 1e-13
    assert rel(op.AH(y), O.adjoint_exact(g, y)) < 1e-13


def test_fista_zero_solution_above_lambda_max():
    g, op, y = _tiny_problem()
    lmax = O.lambda_max(op, y)
    res = O.fista(op, y, lam=lmax * 1.0001, L=1.0, iters=5)
    assert np.all(res.z == 0)
    res = O.fista(op, y, lam=lmax * 0.9, L=1.0, iters=5)
    assert np.any(res.z != 0)


def test_weighted_lambda_max_is_the_zero_threshold():
    """Eq. 12 with depth weights: eta = 0 is optimal iff lambda w_i >= |(A^H y)_i| for every
    i, so weighted FISTA from zero stays at zero just above the weighted lambda_max and moves
    just below it (the first step is (1/L) A^H y against thresholds lambda w_i / L)."""
    g, op, y = _tiny_problem()
    w = ph.depth_weights(g.nx, g.nk)
    lw = O.lambda_max(op, y, w)
    assert np.all(O.fista(op, y, lam=lw * 1.0001, L=1.0, iters=3, w=w).z == 0)
    assert np.any(O.fista(op, y, lam=lw * 0.999, L=1.0, iters=1, w=w).z != 0)
    # and it is not the unweighted value (the weights rise from 0.5 to 1 with depth)
    assert abs(lw - O.lambda_max(op, y)) > 1e-3 * lw


def test_fista_reaches_kkt_point_and_obeys_rate_bound():
    """Optimality of the limit by the l1 KKT conditions; the O(1/k^2) rate of Beck & Teboulle 2009."""
    g, op, y = _tiny_problem()
    lam = 0.1 * O.lambda_max(op, y)
    L = 1.0 + 1e-9
    long = O.fista(op, y, lam, L, iters=20000)
    z = long.z
    grad = op.AH(op.A(z) - y)
    nz = np.abs(z) > 1e-10
    kkt_nz = np.abs(grad[nz] + lam * z[nz] / np.abs(z[nz])).max()
    kkt_z = max(0.0, (np.abs(grad[~nz]) - lam).max()) if (~nz).any() else 0.0
    assert kkt_nz < 1e-8 and kkt_z < 1e-8

    def F(v):
        r = op.A(v) - y
        return 0.5 * np.sum(r * r) + lam * np.sum(np.abs(v))

    Fstar = F(z)
    short = O.fista(op, y, lam, L, iters=1)
    for k in [1, 5, 20, 100]:
        zk = O.fista(op, y, lam, L, iters=k).z
        bound = 2 * L * np.sum(np.abs(z) ** 2) / (k + 1) ** 2
        assert F(zk) - Fstar <= bound + 1e-12
    assert short.iters == 1


def test_fista_energy_of_beck_teboulle_is_nonincreasing():
    """Beck & Teboulle 2009, Lemma 4.1: with v_k = F(z^k) - F* and
    u_k = t_k z^k - (t_k - 1) z^{k-1} - x*, the energy (2/L) t_k^2 v_k + ||u_k||^2 never rises
    along the iterates of Alg. 1 (t_1 = 1, z^0 = 0).  A wrong momentum weight breaks it."""
    g, op, y = _tiny_problem()
    lam = 0.1 * O.lambda_max(op, y)
    L = 1.0 + 1e-9
    xs = O.fista(op, y, lam, L, iters=20000).z

    def F(v):
        r = op.A(v) - y
        return 0.5 * np.sum(r * r) + lam * np.sum(np.abs(v))

    Fs = F(xs)
    K = 60
    t = [1.0]
    while len(t) < K:
        t.append((1 + math.sqrt(1 + 4 * t[-1] ** 2)) / 2)
    zs = [np.zeros_like(xs)] + [O.fista(op, y, lam, L, iters=k).z for k in range(1, K + 1)]
    E = []
    for k in range(1, K + 1):
        tk = t[k - 1]
        u = tk * zs[k] - (tk - 1) * zs[k - 1] - xs
        E.append(2 / L * tk ** 2 * (F(zs[k]) - Fs) + np.sum(np.abs(u) ** 2))
    E = np.asarray(E)
    assert np.all(np.diff(E) <= 1e-9 * E[0])
    assert E[-1] < 0.5 * E[0]


def test_fista_scalar_example_worked_by_hand():
    """Alg. 1 on one complex unknown with A x = Re x, y = 1, L = 2 (step 1/2), lambda = 0.

    From eta^1 = z^0 = 0, t^1 = 1: z^k = eta^k - (Re eta^k - 1)/2, t^{k+1} = (1 + sqrt(1 + 4 t_k^2))/2,
    eta^{k+1} = z^k + ((t^k - 1)/t^{k+1})(z^k - z^{k-1}).  By hand: z^1 = 1/2; the first momentum
    weight is 0, so z^2 = 3/4; t^2 = (1 + sqrt 5)/2, t^3 = (1 + sqrt(7 + 2 sqrt 5))/2, and
    eta^3 = 3/4 + (t^2 - 1)/t^3 / 4, z^3 = 1/2 + eta^3 / 2 = 0.91021919...; then z^4.
    The weights (t^k - 1)/t^k or t^k/t^{k+1} give 0.92274575... and 1.10144513... at k = 3."""
    op = DenseOp(np.array([[1.0, 0.0]]), (1, 1))
    y = np.array([[1.0]])
    t2 = (1 + math.sqrt(5)) / 2
    t3 = (1 + math.sqrt(7 + 2 * math.sqrt(5))) / 2
    z3 = 0.5 + (0.75 + 0.25 * (t2 - 1) / t3) / 2
    assert abs(z3 - 0.9102191906406651) < 1e-15
    want = [0.5, 0.75, z3, 0.9898805870005736]
    for k, zk in enumerate(want, start=1):
        res = O.fista(op, y, lam=0.0, L=2.0, iters=k)
        assert abs(res.z[0, 0] - zk) < 1e-14, k
        assert res.z[0, 0].imag == 0.0


def test_fista_relative_residual_stop_and_resume():
    g, op, y = _tiny_problem()
    lam = 0.1 * O.lambda_max(op, y)
    full = O.fista(op, y, lam, 1.0, iters=60)
    a = O.fista(op, y, lam, 1.0, iters=25)
    b = O.fista(op, y, lam, 1.0, iters=35, state=a.state)
    assert np.array_equal(b.z, full.z)
    stop = O.fista(op, y, lam, 1.0, iters=5000, tol=1e-3)
    assert stop.iters < 5000 and stop.rel_res[-1] < 1e-3
    assert all(r >= 1e-3 for r in stop.rel_res[:-1])


def test_residual_add_back_is_one_gradient_step():
    g, op, y = _tiny_problem()
    lam = 0.2 * O.lambda_max(op, y)
    plain = O.fista(op, y, lam, 1.0, iters=30)
    added = O.fista(op, y, lam, 1.0, iters=30, add_residual=True)
    assert rel(added.z, plain.z + op.AH(y - op.A(plain.z))) < 1e-14


# ------------------------------------------------------------------ direct image (Eq. 9)

def test_direct_image_is_the_per_ascan_in_focus_adjoint():
    """With one A-scan only q = 0 exists (kz = 2k, no beam filter or focal term), so the
    operator's adjoint is the dispersion-compensated transform of Eq. 9: the direct image of
    every A-scan equals the one-A-scan adjoint of that A-scan, and A-scans do not mix."""
    g = tiny_geom(6, 32, focus_rows=5)
    rng = np.random.default_rng(31)
    y = rng.standard_normal((g.nx, g.nk))
    d = O.direct_image(g, y)
    g1 = g.with_(nx=1)
    for p in range(g.nx):
        a = O.adjoint_exact(g1, y[p:p + 1])[0]
        assert np.abs(d[p] - a).max() < 1e-12 * np.abs(a).max()


def test_direct_image_against_numpy_fft():
    """With k_c / dk = P an integer, e^{-2 i k_n z_m} = e^{-2 pi i (n + P - nk/2) m / nk}: the direct
    image is numpy's forward FFT of y e^{-i phi} over the sample index, times a per-row phase."""
    nk = 64
    lam = 1300e-9
    g = O.Geometry(nx=3, nk=nk, dx=4e-6, lambda_c=lam, dlambda=lam / 7.5, waist=8e-6,
                   z_focus=0.0, a2=3e-10, a3=1e-16)
    G = O.grids(g)
    P = int(round(G.kc / G.dk))
    assert abs(G.kc / G.dk - P) < 1e-6
    rng = np.random.default_rng(32)
    y = rng.standard_normal((g.nx, nk))
    v = y * np.exp(-1j * O.dispersion_phase(g))[None, :]
    m = np.arange(-nk // 2, nk // 2)
    want = np.fft.fft(v, axis=1)[:, np.mod(m, nk)] * np.exp(-2j * math.pi * (P - nk // 2) * m / nk)[None, :]
    want /= math.sqrt(nk)
    got = O.direct_image(g, y)
    assert np.abs(got - want).max() < 1e-11 * np.abs(want).max()


def test_direct_image_holds_half_the_object_and_its_mirror():
    """Eq. 9 with no dispersion: the real measurement carries the object and its conjugate
    mirror with weight 1/2 each, and the direct image returns exactly that sum,
    (eta + M eta) / 2 with (M eta)[m] = conj(eta[-m]) (row -nz/2 has no mirror)."""
    nk = 32
    g = tiny_geom(1, nk, edge_phase2=0.0, edge_phase3=0.0, focus_rows=0)
    rng = np.random.default_rng(33)
    eta = rand_obj(rng, 1, nk)
    mir = np.zeros_like(eta)
    mir[:, 1:] = np.conj(eta[:, :0:-1])
    s = O.forward_exact(g, eta)
    got = O.direct_image(g, s)
    assert np.abs(got - (eta + mir) / 2).max() < 1e-12


# ------------------------------------------------------------------ inputs

def test_phantoms_are_seeded_and_full_range():
    w = ph.workload("tiny")
    a, b = ph.phantom(w), ph.phantom(w)
    assert np.array_equal(a, b)
    nk = w.optics.nk
    nzr = np.nonzero(a)
    assert np.count_nonzero(a) == 40
    assert np.all(nzr[1] != 0) and np.all(nzr[1] != nk // 2)
    assert np.sum(nzr[1] < nk // 2) == 20
    wb = ph.workload("bscan")
    o = wb.optics
    G = O.grids(O.Geometry.of(o))
    assert abs(o.z_focus / G.dz - 512) < 1e-9
    edge = G.band / 2
    assert abs(o.a2 * edge ** 2 - 40 * math.pi) < 1e-9
    assert abs(o.a3 * edge ** 3 - 8 * math.pi) < 1e-9
