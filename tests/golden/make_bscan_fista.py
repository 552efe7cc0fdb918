"""Writes bscan_fista.npz: the FP64 oracle's FISTA iterates on the 1024 x 2048 B-scan workload.

Calls only oracle/ and phantoms/ (test infrastructure; never the HIP library).  The workload
is phantoms.workload("bscan") (seed 1): 5 layers + 2000 scatterers, 40 pi / 8 pi dispersion,
focus +512 rows, 25 dB SNR.  The measured spectra y are the oracle's mode-N forward of the
phantom plus seeded noise, rounded to float32 (the precision the GPU receives), and every
oracle step below runs on exactly those float32 values held in float64.

Stored: L (power iteration, 50 steps, seed 0, x 1.01), lambda = 0.05 lambda_max, sum(y^2) and
a strided sample of y (to check that a test regenerates the same y), and the iterates z^k of
Alg. 1 at k in CHECKPOINTS as sparse (index, complex64 value) pairs, with the oracle's
||A eta^k - y||^2 history.

Run:  python tests/golden/make_bscan_fista.py   (a few minutes on 8 cores)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O      # noqa: E402
import phantoms as ph   # noqa: E402

CHECKPOINTS = (1, 10, 50, 100, 200)
OUT = os.path.join(HERE, "bscan_fista.npz")


def bscan_data(op, w):
    """The workload's float32 spectra as float64, from the oracle's forward operator."""
    s = op.A(ph.phantom(w))
    return ph.add_noise(s, w.snr_db, w.seed).astype(np.float32).astype(np.float64)


def main():
    w = ph.workload("bscan")
    g = O.Geometry.of(w.optics)
    t0 = time.perf_counter()
    op = O.Operator(g, "N", workers=O.default_workers())
    print(f"operator built in {time.perf_counter() - t0:.1f} s", flush=True)
    y = bscan_data(op, w)
    L = O.lipschitz(op, y.shape, iters=50, seed=0)
    lam = w.lam_frac * O.lambda_max(op, y)
    print(f"L = {L!r}  lambda = {lam!r}", flush=True)
    out = {"L": np.float64(L), "lam": np.float64(lam), "y_sumsq": np.float64(np.sum(y * y)),
           "y_sample": y.ravel()[::4099].copy(), "checkpoints": np.array(CHECKPOINTS, np.int32)}
    state, done, resid2 = None, 0, []
    for k in CHECKPOINTS:
        res = O.fista(op, y, lam, L, k - done, state=state)
        state, done = res.state, k
        resid2 += res.resid2
        z = res.z.ravel()
        idx = np.flatnonzero(z)
        out[f"idx_{k}"] = idx.astype(np.int32)
        out[f"val_{k}"] = z[idx].astype(np.complex64)
        out[f"norm_{k}"] = np.float64(np.linalg.norm(z))
        print(f"k = {k}: {idx.size} nonzeros, ||z|| = {np.linalg.norm(z):.6e}, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
    out["resid2"] = np.array(resid2)
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
