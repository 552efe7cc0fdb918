#!/usr/bin/env python3
"""Throughput of the MI355X full-range ISAM hot path on the 1024 x 2048 B-scan.

A step is one FISTA iteration of the MBIR solve (Alg. 1): forward operator
A = Re(K^ .), residual, adjoint A^H, gradient step, weighted soft threshold and
momentum, on a synthetic 1024 A-scan x 2048-sample B-scan (5 layers + 2000 point
scatterers on both sides of zero delay, 40 pi / 8 pi dispersion, 25 dB SNR).
The same run also times A.A^H operator pairs (isam_forward + isam_adjoint).

Prints one JSON line.  Inputs are resident in device memory before timing starts.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
# FP32 vector peaks: the published figure (packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2
# flops x 2.4 GHz), and the rate without packed-FP32 instructions, which the kernels are compiled without
ALU_PEAK_TFS = 157.3
ALU_PEAK_UNPACKED_TFS = 78.6
METRIC = "A^H·A op pairs/s + FISTA iter/s, 1024×2048 B-scan FP32 vs plain; %HBM peak"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ["paper_1905_06058_amd/csrc/" + f for f in
                  ("common.hpp", "fft.hpp", "plan.hpp", "lateral.hpp", "lateral.hip", "lateral_real.hip",
                   "lateral_fista.hip", "nufft.hip", "solver.hip", "batch.hip", "direct.hip")]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="timed FISTA iterations")
    ap.add_argument("--warmup", type=int, default=200, help="untimed FISTA iterations before timing")
    ap.add_argument("--pairs", type=int, default=200, help="timed A.A^H pairs")
    ap.add_argument("--workload", default="bscan")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-reps", type=int, default=5, help="timed oracle iterations (median reported)")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-volume", action="store_true", help="skip the 256x256x2048 volume leg")
    ap.add_argument("--volume-iters", type=int, default=50, help="FISTA iterations of the volume leg")
    ap.add_argument("--batch-iters", type=int, default=50, help="FISTA iterations of the uneven-batch leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 64 MiB device copy (calibrates memory-traffic counters)")
    return ap.parse_args()


def progress(msg: str) -> None:
    """One line per finished leg on stderr (the JSON result line goes to stdout)."""
    print(f"bench.py: {msg}", file=sys.stderr, flush=True)


def sources_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pass_bytes(nx: int, nk: int, weighted: bool) -> dict:
    """Algorithmic HBM bytes per launch of each pass: inputs read once, outputs written once.
    The NUFFT passes and the update pass in their FISTA form: the forward also reads F(y),
    the adjoint also reads eta_hat (it writes the gradient step eta_hat - g_hat / L), and the
    update pass reads that step and z^{k-1} and writes z^k and the next eta_hat."""
    full = nx * nk
    half = (nx // 2 + 1) * nk
    c, f = 8, 4
    return {
        "lateral_fft_fwd": 2 * c * full,
        "nufft_fwd": c * full + 2 * c * half,
        "lateral_c2r": c * half + f * full,
        "lateral_r2c": f * full + c * half,
        "nufft_adj": c * half + 2 * c * full,
        "lateral_fft_inv": 2 * c * full,
        "fista_update": 4 * c * full + (f * full if weighted else 0),
        "direct": f * full + c * full,
    }


def pass_flops(nx: int, nk: int, J: int = 6) -> dict:
    """Algorithmic FP32 flops per launch: 5 N log2 N per complex FFT of length N, and per
    Stolt sample of a column J complex multiply-adds (8 flops) and the modulation product
    (6), plus the J weights (cubic complex Horner, 12 flops each) once per partner pair l,
    nx - l, which share q^2 and hence the weights: 6 J per column sample.  The adjoint in its
    FISTA form adds the gradient step (two multiply-adds, 4 flops, per output point)."""
    K = 2 * nk
    fft_col = 5 * K * math.log2(K)
    per_sample = 6 * J + 8 * J + 6
    lat = 5 * nx * math.log2(max(nx, 2)) * nk
    return {
        "nufft_fwd": nx * (fft_col + per_sample * nk),
        "nufft_adj": nx * (fft_col + per_sample * nk) + 4 * nx * nk,
        "fista_update": 2 * lat,
        "lateral_fft_fwd": lat, "lateral_fft_inv": lat, "lateral_c2r": lat / 2, "lateral_r2c": lat / 2,
    }


def _median_iteration(O, op, y, lam, L, reps):
    """One warm-up FISTA iteration of the oracle, then `reps` single iterations continuing the
    same solve (resumed from the saved state); returns the median seconds per iteration."""
    res = O.fista(op, y, lam, L, 1)
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        res = O.fista(op, y, lam, L, 1, state=res.state)
        times.append(time.perf_counter() - t0)
    return float(sorted(times)[len(times) // 2])


def cpu_baseline(w, reps: int, P, torch) -> dict:
    """The FP64 oracle (mode N) timed on this host: FISTA iterations on the full workload with
    one core and with every core this process may use, and one A.A^H pair of the 256 x 256 x
    2048 volume extrapolated from a 16 x 16 slab of columns; with the accuracy of the GPU
    path against it (accuracy_leg)."""
    import numpy as np
    import oracle as O
    import phantoms as ph
    from threadpoolctl import threadpool_limits

    ncores = len(os.sched_getaffinity(0))
    g = O.Geometry.of(w.optics)
    tb = time.perf_counter()
    op = O.Operator(g, "N", workers=O.default_workers())
    build_s = time.perf_counter() - tb
    progress(f"oracle interpolation matrices built in {build_s:.1f} s")
    y = ph.add_noise(op.A(ph.phantom(w)), w.snr_db, w.seed)
    lam = w.lam_frac * O.lambda_max(op, y)
    L = 1.01
    with threadpool_limits(limits=1):
        prev = O.set_fft_workers(1)
        t1 = _median_iteration(O, op, y, lam, L, reps)
    progress(f"oracle single-core iteration {t1:.2f} s")
    O.set_fft_workers(ncores)
    tn = _median_iteration(O, op, y, lam, L, reps)
    progress(f"oracle {ncores}-core iteration {tn:.2f} s")
    # volume: one pair on a 16 x 16 x 2048 slab (256 of the 65536 columns), all cores
    vo = ph.custom_optics(16, w.optics.nk, edge_phase2=40 * math.pi, edge_phase3=8 * math.pi,
                          focus_rows=w.optics.nk // 4)
    gv = O.Geometry.of(vo, ny=16, dy=vo.dx)
    V = O.VolumeOperator(gv, "N", workers=O.default_workers())
    rng = np.random.default_rng(5)
    xv = ph.complex_gaussian(rng, (16, 16, w.optics.nk))
    V.AH(V.A(xv))
    tv = []
    for _ in range(3):
        t0 = time.perf_counter()
        V.AH(V.A(xv))
        tv.append(time.perf_counter() - t0)
    O.set_fft_workers(prev)
    pair_slab = sorted(tv)[1]
    scale = (256 * 256) / (16 * 16)
    accuracy = accuracy_leg(P, torch, w, op, y)
    progress(f"accuracy against the oracle: {accuracy}")
    return {
        "value": round(1.0 / tn, 4),
        "unit": "iter/s",
        "cores": ncores,
        "kind": "oracle",
        "sample": (f"FP64 oracle (min-max NUFFT mode, cached interpolation matrices) on the full "
                   f"{g.nx}x{g.nk} workload: 1 warm-up then {reps} FISTA iterations of one solve, median; "
                   f"scipy.fft with {ncores} workers (scipy.sparse products are single-threaded); "
                   f"matrices built beforehand in {build_s:.1f} s ({O.default_workers()} processes, not timed)"),
        "single_core": {"value": round(1.0 / t1, 4), "unit": "iter/s", "cores": 1,
                        "s_per_iter": round(t1, 4)},
        "all_cores_s_per_iter": round(tn, 4),
        "volume_pair_extrapolated": {
            "value": round(1.0 / (pair_slab * scale), 6), "unit": "pairs/s", "cores": ncores,
            "sample": (f"one A.A^H pair on a 16x16x2048 slab of the 256x256x2048 volume ({pair_slab:.2f} s, "
                       f"median of 3), extrapolated linearly in columns (x{scale:.0f}); the 2-D lateral "
                       "FFT's log factor is not scaled, so this overstates the oracle's rate")},
        "accuracy": accuracy,
    }


def accuracy_leg(P, torch, w, op, y) -> dict:
    """Accuracy reported beside the timings: the GPU's A and A^H against the oracle (mode N)
    on the workload, the adjoint dot test, the FISTA image after 200 iterations against the
    oracle's stored iterate (same spectra, L and lambda), and on the 64 x 256 workload the
    largest ratio of the oracle's NUFFT error to the min-max bound (mode N against mode E)."""
    import numpy as np
    import oracle as O
    import phantoms as ph

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    out = {}
    eta = ph.phantom(w)
    with P.Plan(P.Geometry.of(w.optics)) as plan:
        s = plan.forward(torch.from_numpy(eta).to(torch.complex64).cuda()).double().cpu().numpy()
        yd = torch.from_numpy(y).float().cuda()
        a = plan.adjoint(yd).cpu().numpy().astype(np.complex128)
        out["A_rel_l2"] = rel(s, op.A(eta))
        out["AH_rel_l2"] = rel(a, op.AH(y))
        rng = np.random.default_rng(9)
        x = torch.from_numpy(ph.complex_gaussian(rng, eta.shape)).to(torch.complex64).cuda()
        r = torch.from_numpy(rng.standard_normal(eta.shape)).float().cuda()
        Ax = plan.forward(x).double()
        AHr = plan.adjoint(r).to(torch.complex128)
        lhs = float((Ax * r.double()).sum())
        rhs = float(torch.real(torch.vdot(x.to(torch.complex128).ravel(), AHr.ravel())))
        out["dot_test"] = abs(lhs - rhs) / (float(Ax.norm()) * float(r.double().norm()))
        golden = os.path.join(ROOT, "tests", "golden", "bscan_fista.npz")
        if w.name == "bscan" and os.path.exists(golden):
            gd = np.load(golden)
            y32 = torch.from_numpy(y.astype(np.float32)).cuda()
            res = plan.fista(y32, float(gd["lam"]), 200, L=float(gd["L"]))
            z = res.eta.cpu().numpy().astype(np.complex128).ravel()
            ref = np.zeros_like(z)
            ref[gd["idx_200"]] = gd["val_200"]
            out["fista_z200_rel_l2"] = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    # mode N against mode E on the 64 x 256 workload: the per-point error over the bound
    t = ph.workload("tiny")
    g = O.Geometry.of(t.optics)
    G = O.grids(g)
    eh = np.fft.fft(ph.phantom(t), axis=0, norm="ortho")
    kz, _ = O.axial_wavenumber(g)
    tt, g0, tau = O.stolt_points(g)
    Eb = O.minmax_error(g, tau.ravel()).reshape(tau.shape)
    worst = 0.0
    for l in range(g.nx):
        col = np.linalg.norm(eh[l])
        X = np.exp(1j * kz[l][:, None] * G.z[None, :]) @ eh[l] / math.sqrt(g.nk)
        Y = O.isam_oracle._oversampled_spectrum(g, eh[l])[0]
        Xh = O.isam_oracle._interp_matrix(g, l, None, (tt, g0, tau)) @ Y / math.sqrt(g.nk)
        worst = max(worst, float((np.abs(Xh - X) / (Eb[l] * col)).max()))
    out["tiny_nufft_bound_utilisation"] = worst
    return out


def batch_leg(P, torch, iters: int, nscans: int = 64, nx_choices=tuple(range(256, 1025, 128)),
              nk_choices=(1024, 2048), label: str = "") -> dict:
    """B-scans of uneven size (by default 64 of them, nx from {256, 384, ..., 1024}, nk from
    {1024, 2048}), own phantom and dispersion each: one batch (tuned tiles and FISTA schedule)
    against the same scans run one after another through their own plans (one launch per pass
    per scan, one stream).  Both FISTA schedules are timed: grouped launches (captured iteration
    graph, and eager) and each scan's own solve spread over the batch's streams."""
    import numpy as np
    import phantoms as ph
    rng = np.random.default_rng(3)
    opts = []
    for _ in range(nscans):
        nx = int(rng.choice(np.array(nx_choices)))
        nk = int(rng.choice(np.array(nk_choices)))
        opts.append(ph.custom_optics(nx, nk, edge_phase2=float(rng.uniform(10, 40)) * math.pi,
                                     edge_phase3=float(rng.uniform(-8, 8)) * math.pi,
                                     focus_rows=float(rng.uniform(-nk / 4, nk / 4))))
    b = P.Batch([P.Geometry.of(o) for o in opts])
    tiles = b.tune(reps=5)
    y = torch.empty(b.total, dtype=torch.float32, device="cuda")
    for i, o in enumerate(opts):
        eta = ph.layers(rng, o.nx, o.nk, 3) + ph.point_scatterers(rng, o.nx, o.nk, o.nx // 2)
        s = b.plan(i).forward(torch.from_numpy(eta).to(torch.complex64).cuda())
        b.scan(y, i).copy_(s + 0.05 * s.abs().max() * torch.randn_like(s))
    plans = [b.plan(i) for i in range(b.n)]
    L = [p.lipschitz(iters=20, seed=0) for p in plans]
    lam = [0.05 * p.lambda_max(b.scan(y, i).contiguous()) for i, p in enumerate(plans)]
    ys = [b.scan(y, i).contiguous() for i in range(b.n)]
    outs = [torch.empty((p.nx, p.nk), dtype=torch.complex64, device="cuda") for p in plans]
    out = torch.empty(b.total, dtype=torch.complex64, device="cuda")

    def timed(fn, reps=1):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    tuned = b.schedule()

    def fista_time(sched, graph=True):
        b.set_schedule(sched)
        return timed(lambda: b.fista(y, lam, iters, L=L, out=out, graph=graph), 3)

    t_grouped = fista_time("grouped")
    t_eager = fista_time("grouped", graph=False)
    t_streams = fista_time("streams")
    b.set_schedule(tuned)
    t_batch = t_grouped if tuned == "grouped" else t_streams
    t_scan = timed(lambda: [p.fista(ys[i], lam[i], iters, L=L[i], out=outs[i]) for i, p in enumerate(plans)], 3)
    x = torch.randn(b.total, dtype=torch.complex64, device="cuda")
    sb = torch.empty(b.total, dtype=torch.float32, device="cuda")
    xs = [b.scan(x, i).contiguous() for i in range(b.n)]
    ss = [torch.empty((p.nx, p.nk), dtype=torch.float32, device="cuda") for p in plans]

    def pairs_batch():
        for _ in range(10):
            b.forward(x, out=sb)
            b.adjoint(sb, out=x)

    def pairs_scan():
        for _ in range(10):
            for i, p in enumerate(plans):
                p.forward(xs[i], out=ss[i])
                p.adjoint(ss[i], out=xs[i])

    tp_batch = timed(pairs_batch, 2) / 10
    tp_scan = timed(pairs_scan, 2) / 10
    pts = b.total
    b.close()
    return {
        "workload": label or (f"{nscans} uneven B-scans, nx from {list(nx_choices)}, nk from {list(nk_choices)}, "
                              "own phantom, dispersion and focus each; synthetic"),
        "scans": nscans, "points": pts, "fista_iters": iters,
        "tiles": {str(k): v for k, v in tiles.items()},
        "schedule": tuned,
        "batched_fista_iter_per_s": round(iters / t_batch, 2),
        "grouped_fista_iter_per_s": round(iters / t_grouped, 2),
        "batched_eager_fista_iter_per_s": round(iters / t_eager, 2),
        "streams_fista_iter_per_s": round(iters / t_streams, 2),
        "per_scan_fista_iter_per_s": round(iters / t_scan, 2),
        "fista_speedup": round(t_scan / t_batch, 3),
        "batched_pairs_per_s": round(1.0 / tp_batch, 2),
        "per_scan_pairs_per_s": round(1.0 / tp_scan, 2),
        "pairs_speedup": round(tp_scan / tp_batch, 3),
        "note": f"an iteration or pair covers all {nscans} scans; whole calls are timed (set-up and output included)",
    }


def volume_leg(P, torch, iters: int) -> dict:
    """256 x 256 A-scans x 2048 samples (a 1.07 GB complex64 object): 20000 scatterers plus
    3 curved layers, FISTA for `iters` iterations; per-pass kernel times from isam_timing."""
    import numpy as np
    import phantoms as ph
    ny = nx = 256
    nk = 2048
    o = ph.custom_optics(nx, nk, edge_phase2=40 * math.pi, edge_phase3=8 * math.pi, focus_rows=nk // 4)
    plan = P.Plan(P.Geometry.of(o, ny=ny, dy=o.dx))
    rng = np.random.default_rng(5)
    eta = torch.zeros((ny, nx, nk), dtype=torch.complex64, device="cuda")
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for j in range(3):                                     # curved layers: depth row = smooth surface
        depth = (nk // 2 + (j - 1) * nk // 6 + 40 * np.sin(2 * np.pi * (xx / nx + j / 3))
                 + 30 * np.cos(2 * np.pi * yy / ny)).astype(np.int64)
        amp = 0.5 + 0.5 * rng.random((ny, nx))
        flat = (yy * nx + xx) * nk + np.clip(depth, 0, nk - 1)
        eta.view(-1)[torch.from_numpy(flat.ravel()).cuda()] += torch.from_numpy(amp.ravel()).to(torch.complex64).cuda()
    pts = torch.from_numpy(rng.integers(0, ny * nx * nk, 20000)).cuda()
    amps = torch.from_numpy(ph.complex_gaussian(rng, 20000)).to(torch.complex64).cuda()
    eta.view(-1)[pts] += amps
    s = plan.forward(eta)
    y = s + 0.05 * float(s.abs().max()) * torch.randn_like(s)
    del eta, s
    L = plan.lipschitz(iters=30, seed=0)
    lam = 0.05 * plan.lambda_max(y)
    out = torch.empty((ny, nx, nk), dtype=torch.complex64, device="cuda")
    plan.fista(y, lam, 2, L=L, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.fista(y, lam, iters, L=L, out=out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    plan.timing(True)
    plan.fista(y, lam, iters, L=L, out=out)
    passes = plan.timing(False)
    n = ny * nx * nk
    half = ny * (nx // 2 + 1) * nk
    # algorithmic bytes per iteration: y transforms (2 x 2 full complex passes), NUFFT forward
    # (read 1 full + 1 half, write 1 half), adjoint (read 1 half, write 1 full), update (5 full)
    ibytes = 8 * (4 * n + (n + 2 * half) + (half + n) + 5 * n)
    plan.close()
    per_pass = {k: {"avg_us": round(1e3 * ms / c, 2), "launches": c} for k, (ms, c) in passes.items() if c}
    return {
        "workload": "volume 256x256x2048 (ny x nx x nk), 20000 scatterers + 3 curved layers, synthetic",
        "fista_iters": iters, "status": res.status,
        "fista_iter_per_s": round(iters / dt, 2),
        "ms_per_iter": round(1e3 * dt / iters, 3),
        "algorithmic_bytes_per_iter": ibytes,
        "hbm_GBps": round(ibytes * iters / dt / 1e9, 1),
        "hbm_frac": round(ibytes * iters / dt / 1e9 / HBM_PEAK_GBS, 4),
        "passes": per_pass,
    }


def main() -> int:
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {args.gpus} is not supported "
              "(independent B-scans would shard across GPUs without communication)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import paper_1905_06058_amd as P
    import phantoms as ph

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    if args.copy_probe:
        src = torch.ones(16 << 20, dtype=torch.float32, device="cuda")    # 64 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = ph.workload(args.workload)
    o = w.optics
    nx, nk = o.nx, o.nk
    plan = P.Plan(P.Geometry.of(o))
    eta_true = torch.from_numpy(ph.phantom(w)).to(torch.complex64).cuda()
    s_clean = plan.forward(eta_true)
    y = torch.from_numpy(ph.add_noise(s_clean.double().cpu().numpy(), w.snr_db, w.seed)).float().cuda()
    L = plan.lipschitz(iters=50, seed=0)
    lam = w.lam_frac * plan.lambda_max(y)
    out = torch.empty((nx, nk), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()

    # ---- operator pairs A.A^H (isam_forward then isam_adjoint), before the FISTA timing so
    # that the timed solve is not the first sustained work on the GPU
    x = torch.randn((nx, nk), dtype=torch.complex64, device="cuda")
    sbuf = torch.empty((nx, nk), dtype=torch.float32, device="cuda")
    for _ in range(20):
        plan.forward(x, out=sbuf)
        plan.adjoint(sbuf, out=x)
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for _ in range(args.pairs):
        plan.forward(x, out=sbuf)
        plan.adjoint(sbuf, out=x)
    torch.cuda.synchronize()
    pair_s = (time.perf_counter() - tp) / max(args.pairs, 1)
    # the composed normal operator A^H A (isam_normal): the real spectra are not materialised,
    # since F(Re F^{-1} X) is the Hermitian part of X
    xn = torch.empty_like(x)
    for _ in range(20):
        plan.normal(x, out=xn)
    torch.cuda.synchronize()
    tn = time.perf_counter()
    for _ in range(args.pairs):
        plan.normal(x, out=xn)
    torch.cuda.synchronize()
    normal_s = (time.perf_counter() - tn) / max(args.pairs, 1)
    # the direct image of Eq. 9 (per A-scan dispersion compensation and transform)
    dimg = torch.empty((nx, nk), dtype=torch.complex64, device="cuda")
    for _ in range(20):
        plan.direct(y, out=dimg)
    torch.cuda.synchronize()
    td = time.perf_counter()
    for _ in range(args.pairs):
        plan.direct(y, out=dimg)
    torch.cuda.synchronize()
    direct_s = (time.perf_counter() - td) / max(args.pairs, 1)

    progress(f"operator legs done: {1.0 / pair_s:.0f} pairs/s, {1.0 / normal_s:.0f} normal/s, "
             f"{1.0 / direct_s:.0f} direct images/s")

    # ---- FISTA variants, ahead of the headline timing: iterations with the Eq. 15 norms
    # formed every iteration (a tolerance that never holds; at least 200, so that the rate is
    # not dominated by a call's fixed costs), and the paper's tol = 1e-3 solve (Sec.
    # "Parameters") run to its stop.  Sustained solver work right before the headline run also
    # brings the GPU's clocks to their level under load.  A two-iteration call first takes the
    # process's one-time costs of the solver's first launches.
    plan.fista(y, lam, 2, L=L, tol=1e-30, out=out)
    n15 = max(args.steps, 200)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r15 = plan.fista(y, lam, n15, L=L, tol=1e-30, out=out)
    torch.cuda.synchronize()
    wall15 = time.perf_counter() - t0
    t0 = time.perf_counter()
    rtol = plan.fista(y, lam, 5000, L=L, tol=1e-3, out=out)
    torch.cuda.synchronize()
    wall_tol = time.perf_counter() - t0

    # ---- FISTA: warm-up, then exactly `steps` iterations in one timed region
    if args.warmup > 0:
        plan.fista(y, lam, args.warmup, L=L, out=out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    res = plan.fista(y, lam, args.steps, L=L, out=out)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / max(args.steps, 1)
    if res.status != 0 or not math.isfinite(res.resid2):
        print(f"bench.py: FISTA status {res.status}", file=sys.stderr)
        return 1

    progress(f"FISTA {args.steps / wall:.0f} iter/s; with Eq. 15 norms {n15 / wall15:.0f} iter/s; "
             f"tol 1e-3 stop after {rtol.iters} iterations")

    # ---- per-pass kernel durations (HIP events on the launch stream) over a second FISTA run
    plan.timing(True)
    plan.fista(y, lam, args.steps, L=L, out=out)
    passes = plan.timing(False)
    plan.timing(True)
    for _ in range(args.pairs):
        plan.forward(x, out=sbuf)
        plan.adjoint(sbuf, out=x)
    for _ in range(args.pairs):
        plan.direct(y, out=dimg)
    passes_pair = plan.timing(False)
    nbytes = pass_bytes(nx, nk, weighted=False)
    per_pass = {}
    # the FISTA run's launches first (the byte counts above are the NUFFT passes' FISTA
    # forms); the operator-pair run adds the lateral passes FISTA does not use
    for name, (ms, cnt) in list(passes.items()) + list(passes_pair.items()):
        if cnt and name not in per_pass:
            avg = ms / cnt
            per_pass[name] = {"avg_us": round(1e3 * avg, 3), "launches": int(cnt),
                              "GBps": round(nbytes[name] / (avg * 1e-3) / 1e9, 1)}
    fista_passes = {k: v for k, v in passes.items() if v[1] and k != "lateral_r2c"}
    dom = max(fista_passes, key=lambda k: fista_passes[k][0])
    dom_avg_s = fista_passes[dom][0] / fista_passes[dom][1] * 1e-3
    flops = pass_flops(nx, nk)
    achieved_gbs = nbytes[dom] / dom_avg_s / 1e9
    achieved_tfs = flops[dom] / dom_avg_s / 1e12

    traffic = None
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        k = rec.get("kernels", {}).get(dom)
        if k and rec.get("sources") == sources_digest() and rec.get("workload") == args.workload:
            traffic = k["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        traffic = None
    # The HBM roof is the one the operator targets; neither roof is near saturation for the
    # NUFFT kernels (their limit is instruction issue with barrier / LDS latency), so the ALU
    # view is given beside it against both FP32 figures.
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": nbytes[dom], "avg_launch_us": round(dom_avg_s * 1e6, 3),
                "alu_view": {"achieved": round(achieved_tfs, 2), "unit": "TFLOP/s",
                             "algorithmic_flops_per_launch": round(flops.get(dom, 0.0)),
                             "peak": ALU_PEAK_TFS, "frac": round(achieved_tfs / ALU_PEAK_TFS, 4),
                             "peak_unpacked": ALU_PEAK_UNPACKED_TFS,
                             "frac_unpacked": round(achieved_tfs / ALU_PEAK_UNPACKED_TFS, 4)}}
    if max(achieved_gbs / HBM_PEAK_GBS, achieved_tfs / ALU_PEAK_TFS) < 0.5:
        roofline["limiter"] = ("neither roof: instruction issue with barrier and LDS latency inside a "
                               "workgroup (one wave of workgroups fills the GPU at this size)")
    iter_bytes = sum(nbytes[k] for k in ("nufft_fwd", "nufft_adj", "fista_update"))

    progress("per-pass timings done")
    batched = None if args.no_batch else batch_leg(P, torch, args.batch_iters)
    if batched:
        progress(f"batch leg done: FISTA x{batched['fista_speedup']}")
    # many small scans, where one launch per pass per scan is dominated by launch latency
    batched_small = None if args.no_batch else batch_leg(
        P, torch, args.batch_iters, nscans=256, nx_choices=(64, 128, 192, 256), nk_choices=(256, 512))
    volume = None if args.no_volume else volume_leg(P, torch, args.volume_iters)
    if volume:
        progress(f"volume leg done: {volume['fista_iter_per_s']} iter/s")

    cpu = None
    accuracy = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_reps, P, torch)
        progress(f"cpu baseline done: {cpu['value']} iter/s on {cpu['cores']} cores")
        accuracy = cpu["accuracy"]

    line = {
        "metric": METRIC,
        "value": round(args.steps / wall, 2),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {nx}x{nk} full-range B-scan, {w.n_layers} layers + "
                               f"{w.n_points} scatterers, FISTA lambda={w.lam_frac}*lambda_max, tol=0",
                   "nx": nx, "nk": nk, "J": 6, "oversampling": 2},
        "fista_iter_per_s": round(args.steps / wall, 2),
        "fista_gpu_ms_per_iter": round(gpu_ms / max(args.steps, 1), 5),
        "pairs_per_s": round(1.0 / pair_s, 2),
        "ms_per_pair": round(1e3 * pair_s, 5),
        "normal_per_s": round(1.0 / normal_s, 2),
        "direct_images_per_s": round(1.0 / direct_s, 2),
        "fista_eq15_norms_iter_per_s": round(n15 / wall15, 2),
        "fista_tol_1e-3": {"iters": rtol.iters, "status": rtol.status, "rel_res": rtol.rel_res,
                           "seconds": round(wall_tol, 5), "iter_per_s": round(rtol.iters / wall_tol, 2)},
        "roofline": roofline,
        "iteration_hbm": {"algorithmic_bytes": iter_bytes,
                          "GBps": round(iter_bytes * args.steps / wall / 1e9, 1),
                          "frac": round(iter_bytes * args.steps / wall / 1e9 / HBM_PEAK_GBS, 4)},
        "passes": per_pass,
        "batched": batched,
        "batched_small_scans": batched_small,
        "volume": volume,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "gpu": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line))
    plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
