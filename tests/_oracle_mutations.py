"""Planted mistakes in the FP64 oracle (test infrastructure): each entry replaces one oracle
function with a plausibly wrong version, so that the pins in test_oracle_pins.py can be shown
to catch it.  Used only by test_oracle_mutations.py, in a separate process per mistake."""
import math

import numpy as np

import oracle
import oracle.isam_oracle as OI


def _patch(name, fn):
    setattr(OI, name, fn)
    setattr(oracle, name, fn)


def _wrap(name, make):
    orig = getattr(OI, name)
    _patch(name, make(orig))


MUTATIONS = {
    # Eq. 7: dispersion phase with the wrong sign
    "dispersion_sign": lambda: _wrap("dispersion_phase", lambda f: lambda g: -f(g)),
    # Eq. 16: beam filter dropped (1 on propagating components)
    "beam_dropped": lambda: _wrap("beam_filter", lambda f: lambda g: (f(g) > 0).astype(float)),
    # Eq. 3: kz = sqrt(4 k^2 + q^2) instead of sqrt(4 k^2 - q^2)
    "kz_sign": lambda: _patch("axial_wavenumber", _kz_plus),
    # Eq. 2: lateral DFT not unitary
    "lateral_norm": lambda: _patch("_lateral_fft", lambda x: np.fft.fft(x, axis=0)),
    # Kaiser-Bessel scaling inverted
    "kb_inverse": lambda: _wrap("kb_scaling", lambda f: lambda g: 1.0 / f(g)),
    # min-max weights conjugated
    "weights_conj": lambda: _wrap("minmax_weights", lambda f: lambda g, tau, chunk=4096: np.conj(f(g, tau, chunk))),
    # Eq. 14: threshold halved
    "prox_threshold": lambda: _wrap("soft_threshold", lambda f: lambda u, theta: f(u, np.asarray(theta) / 2)),
    # Stolt neighbours shifted by one grid cell
    "stolt_offset": lambda: _wrap("stolt_points", lambda f: lambda g: _shift_g0(f(g))),
    # focal reference with the wrong sign
    "focus_sign": lambda: _patch("modulation", _modulation_focus_flipped),
    # adjoint without the conjugate of the modulation
    "adjoint_no_conj": lambda: _patch("adjoint_exact", _adjoint_no_conj),
    # depth pitch 2 pi / band instead of pi / band
    "depth_pitch": lambda: _wrap("grids", lambda f: lambda g: _double_dz(f(g))),
    # lambda_max without the weights
    "lambda_max_unweighted": lambda: _wrap("lambda_max", lambda f: lambda op, y, w=None: f(op, y)),
    # calibration derivative of the focal reference with the wrong sign of kz
    "calib_focus_term": lambda: _wrap("calibration_derivatives", lambda f: lambda g: _flip_kz_term(g, f(g))),
    # volume: the y lateral frequency dropped from q^2
    "volume_qy_dropped": lambda: _wrap("volume_q2", lambda f: lambda g: _drop_qy(g)),
    # min-max target offset by one grid cell (J/2 - 1 instead of J/2)
    "minmax_target_offset": lambda: _patch("_targets", _targets_off_by_one),
    # oversampled depth spectrum with the rows placed one index off
    "oversampled_placement": lambda: _patch("_oversampled_spectrum", _oversampled_shifted),
    # adjoint NUFFT with the interpolation matrix transposed but not conjugated
    "adjoint_nufft_no_conj": lambda: _patch("adjoint_nufft", _adjoint_nufft_no_conj),
    # FISTA momentum weight t_k / t_{k+1} instead of (t_k - 1) / t_{k+1}
    "fista_momentum": lambda: _patch("fista", lambda *a, **k: _fista_momentum(lambda t, tn: t / tn, *a, **k)),
    # the milder momentum slip (t_k - 1) / t_k, a convergent but different sequence
    "fista_momentum_mild": lambda: _patch("fista", lambda *a, **k: _fista_momentum(lambda t, tn: (t - 1) / t, *a, **k)),
    # beam filter of width w0^2 / 4 in the exponent instead of w0^2 / 8
    "beam_width": lambda: _wrap("beam_filter", lambda f: lambda g: f(g) ** 2),
    # dispersion polynomial expanded about k0 + dk instead of the centre wavenumber
    "dispersion_k0_shift": lambda: _patch("dispersion_phase", _dispersion_k0_shift),
    # direct image without the dispersion compensation (e^{+j phi})
    "direct_no_compensation": lambda: _patch("direct_image", _direct_wrong_sign_phi),
    # direct image with the conjugate depth kernel
    "direct_kernel_conj": lambda: _patch("direct_image", _direct_conj_kernel),
}


def _dispersion_k0_shift(g):
    G = OI.grids(g)
    d = G.k - (G.kc + G.dk)
    return g.a2 * d ** 2 + g.a3 * d ** 3


def _direct_wrong_sign_phi(g, y):
    G = OI.grids(g)
    Yd = np.asarray(y, np.float64) * np.exp(1j * OI.dispersion_phase(g))[None, :]
    return (Yd @ np.exp(-2j * np.outer(G.k, G.z))) / math.sqrt(g.nk)


def _direct_conj_kernel(g, y):
    G = OI.grids(g)
    Yd = np.asarray(y, np.float64) * np.exp(-1j * OI.dispersion_phase(g))[None, :]
    return (Yd @ np.exp(2j * np.outer(G.k, G.z))) / math.sqrt(g.nk)


def _fista_momentum(weight, op, y, lam, L, iters, w=None, tol=0.0, add_residual=False, eps=1e-12, state=None):
    y = np.asarray(y, np.float64)
    step = 1.0 / L
    w = np.ones(y.shape) if w is None else np.asarray(w, np.float64)
    theta = lam * w * step
    if state is None:
        eta = np.zeros(y.shape, np.complex128)
        z_prev = np.zeros(y.shape, np.complex128)
        t = 1.0
    else:
        eta, z_prev, t = state[0].copy(), state[1].copy(), state[2]
    rr_hist, res_hist, l1_hist = [], [], []
    z = z_prev
    k = 0
    for k in range(1, iters + 1):
        r = op.A(eta) - y
        gk = step * op.AH(r)
        z = OI.soft_threshold(eta - gk, theta)
        d = z - eta
        rr = np.linalg.norm(d) / (max(np.linalg.norm(gk), np.linalg.norm(d + gk)) + eps)
        rr_hist.append(rr)
        res_hist.append(float(np.sum(r * r)))
        l1_hist.append(float(np.sum(w * np.abs(z))))
        if tol > 0 and rr < tol:
            break
        t_next = (1 + math.sqrt(1 + 4 * t * t)) / 2
        eta = z + weight(t, t_next) * (z - z_prev)
        z_prev = z
        t = t_next
    out = z
    if add_residual:
        out = z + step * op.AH(y - op.A(z))
    res = OI.FistaResult(out, k, rr_hist, res_hist, l1_hist)
    res.state = (eta, z_prev, t)
    return res


def _adjoint_nufft_no_conj(g, r, columns=None, P=None):
    G = OI.grids(g)
    R = OI._lateral_fft(np.asarray(r, np.float64).astype(np.complex128))
    Xp = np.conj(OI.modulation(g)) * R
    s = OI.kb_scaling(g)
    tables = OI.stolt_points(g)
    eta_hat = np.zeros((g.nx, g.nk), np.complex128)
    for l in range(g.nx):
        Pl = P[l] if P is not None else OI._interp_matrix(g, l, None, tables)
        full = np.fft.fft(Pl.T @ Xp[l])
        eta_hat[l] = s * full[np.mod(G.m, G.K)] / math.sqrt(g.nk)
    return OI._lateral_ifft(eta_hat)


def _targets_off_by_one(g, tau, m, K):
    return np.exp(2j * math.pi * np.outer(m, np.asarray(tau) + g.J / 2 - 1) / K)


def _oversampled_shifted(g, eta_hat_rows):
    G = OI.grids(g)
    s = OI.kb_scaling(g)
    rows = np.atleast_2d(eta_hat_rows)
    buf = np.zeros((rows.shape[0], G.K), np.complex128)
    buf[:, np.mod(G.m + 1, G.K)] = rows * s[None, :]
    return G.K * np.fft.ifft(buf, axis=1)


def _flip_kz_term(g, D):
    G = OI.grids(g)
    kz, _ = OI.axial_wavenumber(g)
    return D[0], D[1], 2 * G.k[None, :] + kz


def _drop_qy(g):
    qx = 2 * math.pi * np.fft.fftfreq(g.nx, d=1.0 / g.nx) / (g.nx * g.dx)
    return np.broadcast_to(qx[None, :] ** 2, (g.ny, g.nx)).copy()


def _kz_plus(g):
    G = OI.grids(g)
    arg = 4 * G.k[None, :] ** 2 + (G.q ** 2)[:, None]
    return np.sqrt(arg), np.ones(arg.shape, bool)


def _shift_g0(res):
    t, g0, tau = res
    return t, g0 + 1, tau


def _modulation_focus_flipped(g):
    G = OI.grids(g)
    kz, prop = OI.axial_wavenumber(g)
    c = OI.beam_filter(g) * np.exp(1j * OI.dispersion_phase(g)[None, :]) * \
        np.exp(-1j * (2 * G.k[None, :] - kz) * g.z_focus)
    return np.where(prop, c, 0.0)


def _adjoint_no_conj(g, r):
    G = OI.grids(g)
    R = OI._lateral_fft(np.asarray(r, np.float64).astype(np.complex128))
    kz, _ = OI.axial_wavenumber(g)
    Xp = OI.modulation(g) * R
    eta_hat = np.empty((g.nx, g.nk), np.complex128)
    for l in range(g.nx):
        E = np.exp(1j * kz[l][:, None] * G.z[None, :])
        eta_hat[l] = np.conj(E).T @ Xp[l] / math.sqrt(g.nk)
    return OI._lateral_ifft(eta_hat)


def _double_dz(G):
    return OI.Grids(G.kc, G.band, G.dk, G.k, 2 * G.dz, G.m, 2 * G.z, G.l, G.q, G.K, G.beta)


def apply(name):
    MUTATIONS[name]()
