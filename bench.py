"""Benchmark: FFT fixed-point solvers for the 25% square array at 2048^2.

One step = one full iteration of the solver (x pass with the local map and
the fp64 reductions, finalize with the stop rules, Gamma pass with both
y-direction FFTs) on the 2048 x 2048 grid.  The headline value is the
voxel-iterations per second of the accelerated scheme (Eyre-Milton in H'',
[alpha, beta] = [1/4, 4]) with complex-fp32 fields and fp64 reductions.
The same line carries the sweep sigma1 in {10, 100, 1000, 0.01} x
{MS, EM, ACC_EM} x {fp64 to 1e-8, fp32 to 1e-6}: iterations and device time
to tolerance, sigma* and its error against eq. J47a, plus the roofline of
the dominant kernel and the CPU oracle timed on a bounded sample.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 2048
SIGMAS = (10.0, 100.0, 1000.0, 0.01)
SCHEMES = ("ms", "em", "acc_em")
HEADLINE = dict(scheme="acc_em", precision="fp32", sigma1=100.0)
HBM_PEAK_GBS = 8000.0
HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE_SUMMARY = "xpass_gamma_2048sq_acc_em_fp32.txt"
KERNEL_NAMES = {"xpass": "void scfft::xpass_r2c_kernel<float, 2048,",
                "gamma": "void scfft::line_p2_kernel<float, 2048,"}
PROFILE_SUMMARY_FP64 = "xpass_gamma_2048sq_acc_em_fp64.txt"
KERNEL_NAMES_FP64 = {"xpass": "void scfft::xpass_r2c_kernel<double, 2048,",
                     "gamma": "void scfft::line_p2_kernel<double, 2048,"}


def algorithmic_bytes(scheme: str, precision: str, d: int, frac1: float, n0: int,
                      real: bool = True):
    """Bytes one voxel moves through HBM in each kernel of one iteration.

    x pass: read + write of the iterate X (d components; real-field mode
    stores the half spectrum, (n0/2+1)/n0 complex values per voxel), read +
    write of the previous physical field (real in real-field mode), the phase
    byte, and for the H'' schemes read + write of the S, T slots at phase-1
    voxels (2 slots for EM in H'', 1 for MS in H'').  Gamma pass: read + write
    of X.  3D adds two plain y passes of the same size as the Gamma pass.
    """
    c = 4 if precision == "fp32" else 8          # bytes of one real value
    if real:
        xs = d * (n0 // 2 + 1) / n0 * 2 * c       # X per voxel (complex half spectrum)
        ep = d * c                                 # real-space field per voxel
    else:
        xs = d * 2 * c
        ep = d * 2 * c
    xp = 2 * xs + 2 * ep + 1
    slots = {"acc_em": 2, "acc_ms": 1}.get(scheme, 0)
    xp += 2 * slots * ep * frac1
    gp = 2 * xs
    return {"xpass": xp, "gamma": gp, "y": gp if d == 3 else 0.0}


def _row(r, **kw):
    d = {"status": r["status"], "iterations": r["iterations"], "time_ms": round(r["elapsed_ms"], 3),
         "sigma_star": complex(r["sigma_star"]).real}
    d.update(kw)
    return d


def batch_inputs(scfft, inputs, torch):
    """The 16 random-disk structures (seeds 0-15, grids 256..1024) on the
    device, their contour intervals and the 128 conductivities each."""
    chis, alphas, betas, sig = [], [], [], []
    t_est = 0.0
    for seed, n in enumerate(inputs.BATCH_GRIDS):
        chi_np, _ = inputs.random_disks(n, seed=seed)
        chi = torch.as_tensor(chi_np).cuda()
        t0 = time.perf_counter()
        e = scfft.estimate_interval(chi, 100)
        t_est += time.perf_counter() - t0
        a_u = min(0.8 * e["alpha"], 0.8 / e["beta"], 0.0625)
        b_u = 1.0 / a_u
        z = inputs.contour_points(128, 0.6)
        chis.append(chi)
        alphas.append(a_u)
        betas.append(b_u)
        sig.append([scfft.sigma1_from_z(a_u, b_u, zz) for zz in z])
    return chis, alphas, betas, sig, t_est


def extra_configs(scfft, inputs, torch) -> dict:
    """3D cube array, mixed-grid batched contour sweep, adjoint gradients."""
    out = {}
    log = lambda *a: print("#", *a, file=sys.stderr, flush=True)   # noqa: E731

    # 64^2 square array, sigma1 = 10, basic scheme, fp64 to 1e-10 (smallest configuration)
    chi64 = torch.as_tensor(inputs.square_array(64)).cuda()
    r = scfft.solve(chi64, 10.0, (1.0, 0.0), "ms", precision="fp64", tol=1e-10, max_iter=1000,
                    check_every=16, fields=False, history=False)
    ex = float(np.sqrt((1 + 3 * 10.0) / (3 + 10.0)))
    out["square_64_ms"] = _row(r, rel_err_J47a=abs(r["sigma_star"] - ex) / ex,
                               workload="64^2 square array, sigma1 = 10, MS, fp64, tol 1e-10")
    log("64", out["square_64_ms"])

    # the paper's convergence setup: sigma1 = 0, [alpha, beta] = [1/4, 4], sigma* vs eq. J47a
    chi2k = torch.as_tensor(inputs.square_array(N)).cuda()
    ex0 = float(np.sqrt(1.0 / 3.0))
    hist = {}
    for scheme in ("ms", "acc_ms", "acc_em"):
        r = scfft.solve(chi2k, 0.0, (1.0, 0.0), scheme, precision="fp64", alpha=0.25, beta=4.0,
                        tol=-1, max_iter=40, stag_window=0, div_factor=0, fields=False,
                        history=True)
        err = np.abs(r["sigma_history"] - ex0) / ex0
        hist[scheme] = {f"n{k}": float(err[k]) for k in (1, 5, 10, 20, 30, 40)}
    hist["em"] = "undefined at sigma1 = 0 (sigma0 = sqrt(sigma1) = 0)"
    out["sigma1_zero_convergence"] = {
        "workload": "2048^2 square array, sigma1 = 0, fp64, relative error of sigma*_n vs eq. J47a",
        "rel_err": hist}
    log("sigma1=0", hist)

    # Lanczos support estimate of the square array at 2048^2 (fp64, 60 steps)
    t0 = time.perf_counter()
    lz = scfft.estimate_interval_lanczos(chi2k, (1.0, 0.0), steps=60)
    out["lanczos_2048"] = {"interval": lz, "time_ms": round(1e3 * (time.perf_counter() - t0), 3),
                           "workload": "2048^2 square array, e0 = e1, 60 Lanczos steps (fp64); "
                                       "continuum support [1/4, 3/4]"}
    log("lanczos 2048", out["lanczos_2048"])

    # series coefficients of eqs. J5-J7 from one run, sigma* for many sigma1
    a_, b_ = 0.25, 4.0
    s_real = np.logspace(-3, 4, 2048)
    zc = 0.3 * np.exp(2j * np.pi * (np.arange(2048) + 0.5) / 2048)
    s_cplx = np.array([complex(scfft.sigma1_from_z(a_, b_, z)) for z in zc])
    s_all = np.concatenate([s_real, s_cplx])
    ser = {"workload": "2048^2 square array, e0 = e1, [alpha, beta] = [1/4, 4]: c_0..c_40 from one "
                       "run, then sigma* at 4096 sigma1 (2048 on [1e-3, 1e4], 2048 on |z| = 0.3)"}
    for prec in ("fp64", "fp32"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = scfft.series_coefficients(chi2k, (1.0, 0.0), alpha=a_, beta=b_, nterms=40,
                                      precision=prec)
        t_run = time.perf_counter() - t0
        t0 = time.perf_counter()
        vals = scfft.series_evaluate(c, s_all, alpha=a_, beta=b_)
        pade = scfft.series_evaluate(c[:25], s_all, alpha=a_, beta=b_, pade_m=12)
        t_eval = time.perf_counter() - t0
        exact = np.sqrt((1 + 3 * s_all) / (3 + s_all))       # eq. J47a (principal branch)
        direct = {}
        for s in SIGMAS:
            r = scfft.solve(chi2k, s, (1.0, 0.0), "acc_em", precision=prec, alpha=a_, beta=b_,
                            tol=1e-12 if prec == "fp64" else 1e-6, max_iter=500, fields=False,
                            history=False)
            v = scfft.series_evaluate(c, [s], alpha=a_, beta=b_)[0]
            direct[str(s)] = {"series_vs_solve": float(abs(v - r["sigma_star"]) / abs(r["sigma_star"])),
                              "solve_ms": round(r["elapsed_ms"], 3), "solve_iters": r["iterations"]}
        ser[prec] = {"coeff_run_ms": round(1e3 * t_run, 3), "eval_ms_4096": round(1e3 * t_eval, 3),
                     "sigma1_per_s": len(s_all) / (t_run + t_eval),
                     "max_rel_err_vs_J47a": float(np.max(np.abs(vals - exact) / np.abs(exact))),
                     "pade_12_12_max_rel_err_vs_J47a": float(np.max(np.abs(pade - exact) / np.abs(exact))),
                     "direct": direct}
        log("series", prec, ser[prec])
    out["series_2048"] = ser
    del chi2k

    # 3D cubic array of cubes at ~25% on 256^3, sigma1 = 100, interval by power iteration
    n3 = 256
    chi3 = torch.as_tensor(inputs.cube_array(n3)).cuda()
    t0 = time.perf_counter()
    est = scfft.estimate_interval(chi3, 100)
    t_est = time.perf_counter() - t0
    a_u = min(est["alpha"], 1.0 / est["beta"])        # alpha*beta = 1 (stability reading)
    b_u = 1.0 / a_u
    rows = []
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-8)):
        for scheme in SCHEMES:
            r = scfft.solve(chi3, 100.0, (1.0, 0.0, 0.0), scheme, precision=prec, alpha=a_u,
                            beta=b_u, tol=tol, max_iter=2000, check_every=8, fields=False,
                            history=False, raise_on_error=False)
            rows.append(_row(r, precision=prec, scheme=scheme, tol=tol,
                             voxel_iters_per_s=n3 ** 3 * r["iterations"] / (r["elapsed_ms"] * 1e-3)
                             if r["elapsed_ms"] > 0 else None))
            log("3d", rows[-1])
    # Lanczos support estimate (60 fp64 steps) and an accelerated solve with its interval
    t0 = time.perf_counter()
    lz = scfft.estimate_interval_lanczos(chi3, (1.0, 0.0, 0.0), steps=60)
    t_lz = time.perf_counter() - t0
    r = scfft.solve(chi3, 100.0, (1.0, 0.0, 0.0), "acc_em", precision="fp32",
                    alpha=lz["alpha_used"], beta=lz["beta_used"], tol=1e-6, max_iter=2000,
                    check_every=8, fields=False, history=False, raise_on_error=False)
    lz_row = {"interval": lz, "estimate_s": round(t_lz, 3),
              "acc_em_fp32": _row(r, tol=1e-6)}
    log("3d lanczos", lz_row)
    out["cube_256"] = {"interval_raw": est, "interval_used": [a_u, b_u],
                       "estimate_s": round(t_est, 3), "runs": rows, "lanczos": lz_row,
                       "workload": "3D cubic array of cubes (side 161 of 256, f = 0.24875), "
                                   "sigma1 = 100, e0 = e1"}
    del chi3
    scfft.release()

    # batched sweep: 16 disk microstructures on mixed grids x 128 contour conductivities
    grids = inputs.BATCH_GRIDS
    chis, alphas, betas, sig, t_est = batch_inputs(scfft, inputs, torch)
    scfft.release()
    vox = sum(n * n for n in grids) * 128
    res = {}
    sstar = {}
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-8)):
        # untimed: the first batch call on these grids tunes, plans and
        # captures them (every solve stops at its first residual here)
        scfft.solve_batch(chis, np.array(sig), scheme="acc_em", alphas=alphas, betas=betas,
                          precision=prec, tol=1e300, max_iter=400, check_every=8)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rs = scfft.solve_batch(chis, np.array(sig), scheme="acc_em", alphas=alphas, betas=betas,
                               precision=prec, tol=tol, max_iter=400, check_every=8)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        its = np.array([r["iterations"] for r in rs])
        stats = np.array([r["status"] for r in rs])
        sstar[prec] = np.array([complex(r["sigma_star"]) for r in rs])
        # every solve is iterated until the slowest of the batch stops; the
        # voxel-iterations counted here are the useful ones (up to each stop)
        useful = sum(n * n * int(its[i * 128:(i + 1) * 128].sum()) for i, n in enumerate(grids))
        hist = {scfft.status_string(int(k)): int((stats == k).sum()) for k in np.unique(stats)}
        flagged = [(int(i) // 128, int(i) % 128) for i in np.nonzero(stats != 0)[0][:8]]
        res[prec] = {"wall_s": round(wall, 3), "useful_voxel_iters_per_s": useful / wall,
                     "device_ms": round(rs[0]["elapsed_ms"], 3),
                     "iterations_min_mean_max": [int(its.min()), float(its.mean()), int(its.max())],
                     "status_counts": hist,
                     "flagged_examples": [{"structure": a, "j": b, "sigma1": str(np.round(sig[a][b], 4)),
                                           "iterations": int(its[a * 128 + b]),
                                           "residual": rs[a * 128 + b]["residual"]} for a, b in flagged]}
        res[prec]["status_codes"] = stats
        log("batch", prec, {k: v for k, v in res[prec].items() if k != "status_codes"})
        scfft.release()
    # fp32 sigma* against the fp64 batch, for the solves that converged and
    # for those that stagnated at the fp32 floor
    st32 = res["fp32"].pop("status_codes")
    res["fp64"].pop("status_codes")
    rel = np.abs(sstar["fp32"] - sstar["fp64"]) / np.abs(sstar["fp64"])
    res["fp32_vs_fp64_sigma_rel_err"] = {
        "converged_max": float(rel[st32 == 0].max()) if np.any(st32 == 0) else None,
        "stagnated_max": float(rel[st32 != 0].max()) if np.any(st32 != 0) else None,
        "all_median": float(np.median(rel))}
    out["disk_batch"] = {"solves": len(rs), "voxels_per_batch_iteration": vox,
                         "interval_estimate_s": round(t_est, 3), "runs": res,
                         "workload": "16 periodic random-disk microstructures (seeds 0-15, radii "
                                     "U[0.03,0.08], f >= 0.30) on grids 256..1024 x 128 sigma1 on "
                                     "the |z''| = 0.6 contour, accelerated scheme, one batch"}
    del chis

    # adjoint gradients on a 1024^2 graded medium
    n5 = 1024
    rho = torch.as_tensor(inputs.density_field(n5, seed=5)).cuda()
    for prec, tol in (("fp32", 1e-6), ("fp64", 1e-10)):
        t0 = time.perf_counter()
        g = scfft.gradient(density=rho, sigma1=20.0, e0=(1.0, 0.0), precision=prec, tol=tol,
                           max_iter=3000)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out.setdefault("gradient_1024", {})[prec] = {
            "wall_s": round(wall, 3), "sigma_star": g["forward"]["sigma_star"].real,
            "dsigma_dsigma1": g["dsigma1"].real,
            "forward_iterations": g["forward"]["iterations"],
            "adjoint_iterations": g["adjoint"]["iterations"]}
        log("grad", prec, out["gradient_1024"][prec])
    h = 1e-3 * 20.0
    fp = scfft.solve(density=rho, sigma1=20.0 + h, e0=(1.0, 0.0), scheme="em", sigma0=np.sqrt(20.0),
                     tol=1e-12, max_iter=3000, fields=False, history=False)["sigma_star"].real
    fm = scfft.solve(density=rho, sigma1=20.0 - h, e0=(1.0, 0.0), scheme="em", sigma0=np.sqrt(20.0),
                     tol=1e-12, max_iter=3000, fields=False, history=False)["sigma_star"].real
    out["gradient_1024"]["central_fd_dsigma1_fp64"] = (fp - fm) / (2 * h)
    out["gradient_1024"]["workload"] = ("sigma = 1 + 19 rho(x), rho: seeded Gaussian-filtered noise "
                                        "(0.05 cell) clipped to [0,1], 1024^2, Eyre-Milton forward, "
                                        "transposed Eyre-Milton adjoint")
    scfft.release()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-iters", type=int, default=20)
    ap.add_argument("--profile-only", action="store_true",
                    help="only run the headline iteration with per-kernel timing (for rocprofv3)")
    ap.add_argument("--profile-workload", default="headline",
                    choices=["headline", "cube256_acc_em_fp32", "cube240_acc_em_fp32",
                             "square2048_acc_em_fp64",
                             "batch_fp32", "batch_fp64", "gradient1024_fp32",
                             "gradient1024_fp64"],
                    help="workload of --profile-only")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3D cube, batched-sweep and gradient workloads")
    args = ap.parse_args()
    if args.steps < 1:
        print(json.dumps({"error": "--steps must be at least 1"}), flush=True)
        return 2
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU slab decomposition is design-only)"}), flush=True)
        return 2

    import torch

    from paper_2001_08289_amd import inputs
    from paper_2001_08289_amd import scfft

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        return 1
    torch.cuda.set_device(0)
    chi_np = inputs.square_array(N)
    chi = torch.as_tensor(chi_np).cuda()
    frac1 = float(chi_np.mean())
    e0 = (1.0, 0.0)
    exact = {s: complex(np.sqrt((1 + 3 * s) / (3 + s))) for s in SIGMAS}   # eq. J47a

    hs = HEADLINE
    if args.profile_only:
        # calibration for the HBM byte counters: a 256 MiB fill (writes
        # only), then a 256 MiB sum (reads only)
        cal_x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        cal_x.fill_(1.0)
        float(cal_x.sum())
        torch.cuda.synchronize()
        del cal_x
        if args.profile_workload.startswith("batch"):
            # the 16 x 128 contour batch, a fixed number of iterations
            chis, alphas, betas, sig, _ = batch_inputs(scfft, inputs, torch)
            prec = args.profile_workload.split("_")[1]
            scfft.solve_batch(chis, np.array(sig), scheme="acc_em", alphas=alphas, betas=betas,
                              precision=prec, tol=-1.0, max_iter=args.profile_iters,
                              stag_window=0, div_factor=0.0, check_every=8)
            torch.cuda.synchronize()
            print(json.dumps({"workload": args.profile_workload, "iterations": args.profile_iters,
                              "grids": list(inputs.BATCH_GRIDS)}), flush=True)
            return 0
        if args.profile_workload.startswith("gradient"):
            # the graded 1024^2 medium: forward EM solve, transposed adjoint
            # solve and the gradient kernel, a fixed number of iterations each
            prec = args.profile_workload.split("_")[1]
            rho = torch.as_tensor(inputs.density_field(1024, seed=5)).cuda()
            scfft.gradient(density=rho, sigma1=20.0, e0=(1.0, 0.0), precision=prec, tol=-1.0,
                           max_iter=args.profile_iters, stag_window=0, div_factor=0.0)
            torch.cuda.synchronize()
            print(json.dumps({"workload": args.profile_workload,
                              "iterations": args.profile_iters}), flush=True)
            return 0
        if args.profile_workload.startswith("cube"):
            # cube array, sigma1 = 100, the 256^3 symmetrised power-iteration
            # interval; 240^3 runs the compile-time mixed-radix passes
            n3 = int(args.profile_workload[4:7])
            chi3 = torch.as_tensor(inputs.cube_array(n3)).cuda()
            prof = scfft.profile_passes(chi3, 100.0, (1.0, 0.0, 0.0), "acc_em", precision="fp32",
                                        alpha=0.1818, beta=5.5015, iters=args.profile_iters)
            grid = [n3, n3, n3]
        else:
            prec = "fp64" if args.profile_workload == "square2048_acc_em_fp64" else hs["precision"]
            prof = scfft.profile_passes(chi, hs["sigma1"], e0, hs["scheme"], precision=prec,
                                        alpha=0.25, beta=4.0, iters=args.profile_iters)
            grid = [N, N]
        print(json.dumps({"profile": prof, "workload": args.profile_workload, "grid": grid}),
              flush=True)
        return 0

    # ---------------------------------------------------------- headline
    common = dict(alpha=0.25, beta=4.0, tol=-1.0, stag_window=0, div_factor=0.0,
                  check_every=64, fields=False, history=False)
    # a solve with max_iter = m runs m + 1 passes (iterates 0..m): K steps
    # are one solve with max_iter = K - 1, replayed as one graph chunk.  The
    # W warm-up steps run as two solves (the first builds the plan and its
    # graphs, and the process's second solve call still pays a one-time host
    # cost of ~0.1 ms that the timed call should not)
    for w in (args.warmup - args.warmup // 2, args.warmup // 2):
        if w > 0:
            scfft.solve(chi, hs["sigma1"], e0, hs["scheme"], precision=hs["precision"],
                        max_iter=w - 1, **common)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = scfft.solve(chi, hs["sigma1"], e0, hs["scheme"], precision=hs["precision"],
                      max_iter=args.steps - 1, **common)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps
    value = N * N * args.steps / wall
    device_ms_per_step = res["elapsed_ms"] / args.steps
    print(f"# headline {hs}: {args.steps} steps in {wall:.4f} s ({ms_per_step:.4f} ms/step), "
          f"device loop {res['elapsed_ms']:.3f} ms ({device_ms_per_step:.4f} ms/step)",
          file=sys.stderr, flush=True)

    # ---------------------------------------------------------- roofline
    prof = scfft.profile_passes(chi, hs["sigma1"], e0, hs["scheme"], precision=hs["precision"],
                                alpha=0.25, beta=4.0, iters=args.profile_iters)
    ab = algorithmic_bytes(hs["scheme"], hs["precision"], 2, frac1, N, real=True)
    kern = {k: {"ms": round(prof[k], 5),
                "GB/s": round(ab[k] * N * N / (prof[k] * 1e-3) / 1e9, 1) if prof[k] > 0 else None}
            for k in ("xpass", "gamma")}
    dominant = max(("xpass", "gamma"), key=lambda k: prof[k])
    achieved = ab[dominant] * N * N / (prof[dominant] * 1e-3) / 1e9
    iter_bytes = (ab["xpass"] + ab["gamma"]) * N * N
    # measured HBM bytes per launch of the dominant kernel (rocprofv3 FETCH_SIZE +
    # WRITE_SIZE, calibrated), if the committed summary matches these kernels
    from paper_2001_08289_amd.profile_summary import read_traffic
    traffic = read_traffic(os.path.join(HERE, "profiles", PROFILE_SUMMARY),
                           KERNEL_NAMES[dominant])
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "bytes_per_launch": ab[dominant] * N * N,
                "per_kernel": kern,
                "iteration_GBps": round(iter_bytes / (ms_per_step * 1e-3) / 1e9, 1),
                "iteration_frac": round(iter_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "iteration_frac_kernel_time": round(
                    iter_bytes / ((prof["xpass"] + prof["gamma"]) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    print(f"# passes {prof}", file=sys.stderr, flush=True)
    # the autotuner's plan against the built-in rules (tuning off)
    plan_report = {"tuned": scfft.plan_info(chi, hs["sigma1"], e0, hs["scheme"],
                                            precision=hs["precision"], alpha=0.25, beta=4.0),
                   "tuned_pass_ms": {k: round(prof[k], 5) for k in ("xpass", "gamma")}}
    os.environ["SCFFT_TUNE"] = "0"
    scfft.release()
    rule = scfft.profile_passes(chi, hs["sigma1"], e0, hs["scheme"], precision=hs["precision"],
                                alpha=0.25, beta=4.0, iters=args.profile_iters)
    plan_report["rules"] = scfft.plan_info(chi, hs["sigma1"], e0, hs["scheme"],
                                           precision=hs["precision"], alpha=0.25, beta=4.0)
    plan_report["rules_pass_ms"] = {k: round(rule[k], 5) for k in ("xpass", "gamma")}
    del os.environ["SCFFT_TUNE"]
    scfft.release()
    # the same iteration in fp64 (the time-to-tolerance reference): both
    # kernels against the HBM roof, traffic from the committed fp64 summary
    prof64 = scfft.profile_passes(chi, hs["sigma1"], e0, hs["scheme"], precision="fp64",
                                  alpha=0.25, beta=4.0, iters=args.profile_iters)
    ab64 = algorithmic_bytes(hs["scheme"], "fp64", 2, frac1, N, real=True)
    roofline_fp64 = {}
    for k in ("xpass", "gamma"):
        gbs = ab64[k] * N * N / (prof64[k] * 1e-3) / 1e9
        roofline_fp64[k] = {
            "ms": round(prof64[k], 5), "bytes_per_launch": ab64[k] * N * N,
            "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": read_traffic(os.path.join(HERE, "profiles", PROFILE_SUMMARY_FP64),
                                    KERNEL_NAMES_FP64[k])}
    scfft.release()

    # ---------------------------------------------------------- sweep
    sweep = []
    if not args.no_sweep:
        for prec, tol in (("fp64", 1e-8), ("fp32", 1e-6)):
            for s1 in SIGMAS:
                for scheme in SCHEMES:
                    r = scfft.solve(chi, s1, e0, scheme, precision=prec, alpha=0.25, beta=4.0,
                                    tol=tol, max_iter=3000, check_every=8, fields=False,
                                    history=False, raise_on_error=False)
                    row = {"precision": prec, "sigma1": s1, "scheme": scheme, "tol": tol,
                           "status": r["status"], "iterations": r["iterations"],
                           "time_ms": round(r["elapsed_ms"], 3),
                           "sigma_star": r["sigma_star"].real,
                           "rel_err_J47a": abs(r["sigma_star"] - exact[s1]) / abs(exact[s1])}
                    sweep.append(row)
                    print(f"# {row}", file=sys.stderr, flush=True)

    def speedup(prec, s1):
        t = {r["scheme"]: r["time_ms"] for r in sweep if r["precision"] == prec and r["sigma1"] == s1
             and r["status"] == 0}
        if "acc_em" not in t:
            return None
        return {"vs_ms": round(t["ms"] / t["acc_em"], 3) if "ms" in t else None,
                "vs_em": round(t["em"] / t["acc_em"], 3) if "em" in t else None}

    accel = {f"{p}@{s}": speedup(p, s) for p in ("fp64", "fp32") for s in SIGMAS} if sweep else {}

    # fp32 at the fp64 run's iteration count: the precision's own cost and
    # error at equal work (the fp32 rows above stop at a 1e-6 increment)
    same_iters = []
    control = {}
    if not args.no_sweep:
        fp64_rows = {(r["sigma1"], r["scheme"]): r for r in sweep if r["precision"] == "fp64"}
        for (s1, scheme), r64 in fp64_rows.items():
            if r64["status"] != 0:
                continue
            r = scfft.solve(chi, s1, e0, scheme, precision="fp32", alpha=0.25, beta=4.0, tol=-1,
                            max_iter=r64["iterations"], stag_window=0, div_factor=0,
                            check_every=8, fields=False, history=False)
            same_iters.append({"sigma1": s1, "scheme": scheme, "iterations": r["iterations"],
                               "time_ms": round(r["elapsed_ms"], 3),
                               "fp64_time_ms": r64["time_ms"],
                               "rel_err_vs_fp64": abs(r["sigma_star"] - r64["sigma_star"]) /
                               abs(r64["sigma_star"])})
        # the literal symbol of eq. J11 (spectral) and the resistor network as
        # controls of the rotated default: 2048^2 to 1e-8 in fp64
        rows = []
        for symbol in ("spectral", "network"):
            for s1 in SIGMAS:
                for scheme in SCHEMES:
                    r = scfft.solve(chi, s1, e0, scheme, precision="fp64", alpha=0.25, beta=4.0,
                                    symbol=symbol, tol=1e-8, max_iter=4000, check_every=32,
                                    fields=False, history=False, raise_on_error=False)
                    rows.append({"symbol": symbol, "sigma1": s1, "scheme": scheme,
                                 "status": r["status"], "iterations": r["iterations"],
                                 "time_ms": round(r["elapsed_ms"], 3),
                                 "rel_err_J47a": abs(r["sigma_star"] - exact[s1]) / abs(exact[s1])})
                    print(f"# control {rows[-1]}", file=sys.stderr, flush=True)
            scfft.release()
        control["square_2048_fp64_tol1e-8"] = rows
        chi64 = torch.as_tensor(inputs.square_array(64)).cuda()
        ex10 = float(np.sqrt(31.0 / 13.0))
        c1 = {}
        for symbol in ("rotated", "spectral", "network"):
            r = scfft.solve(chi64, 10.0, e0, "ms", precision="fp64", symbol=symbol, tol=1e-10,
                            max_iter=4000, check_every=16, fields=False, history=False)
            c1[symbol] = {"iterations": r["iterations"], "sigma_star": r["sigma_star"].real,
                          "rel_err_J47a": abs(r["sigma_star"] - ex10) / ex10}
        control["square_64_ms_fp64_tol1e-10"] = c1
        scfft.release()

    # ---------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu:
        from oracle import solver as osolver
        # the oracle is single-threaded numpy (its own FFT, no BLAS calls)
        t0 = time.perf_counter()
        # two iterations (about 13 s): a bounded sample of the headline workload
        cpu_iters = 2
        osolver.solve(chi_np, hs["sigma1"], [1.0, 0.0], hs["scheme"], alpha=0.25, beta=4.0, tol=-1,
                      max_iter=cpu_iters, stag_window=0, div_factor=0)
        dt = time.perf_counter() - t0
        # the smallest configuration timed in full: 64^2, sigma1 = 10, MS, fp64, tol 1e-10
        chi_c1 = inputs.square_array(64)
        t0 = time.perf_counter()
        rc1 = osolver.solve(chi_c1, 10.0, [1.0, 0.0], "ms", tol=1e-10, max_iter=1000)
        dt1 = time.perf_counter() - t0
        cpu = {"value": cpu_iters * N * N / dt, "unit": "voxel-iters/s", "cores": 1,
               "kind": "oracle", "nproc": os.cpu_count(),
               "sample": f"{cpu_iters} iterations of the fp64 numpy oracle ({hs['scheme']}, "
                         f"2048^2, own FFT, set-up included), {dt:.1f} s",
               "square_64_ms_full": {"iterations": rc1["iterations"], "seconds": round(dt1, 4),
                                     "voxel_iters_per_s": 64 * 64 * (rc1["iterations"] + 1) / dt1,
                                     "sigma_star": rc1["sigma_star"].real}}

    extra = {} if args.no_extra else extra_configs(scfft, inputs, torch)

    out = {
        "metric": "voxel-iters/s + time to 1e-8 residual, accelerated vs basic, FP32 vs FP64",
        "value": value, "unit": "voxel-iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "passes_timed": res["iterations"] + 1,
        "device_loop_ms_per_step": device_ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "dtype_detail": "fp32 fields (real-space rows, complex half spectra), fp64 reductions and "
                        "scheme scalars",
        "data": "synthetic",
        "config": {"workload": "2D periodic square array of squares at 25% (centred square of side "
                               "N/2), 2048x2048, e0 = e1; headline: accelerated scheme (EM in H'', "
                               "[alpha,beta] = [1/4,4]) sigma1 = 100, complex-fp32 fields",
                   "grid": [N, N], "sweep_sigma1": list(SIGMAS), "schemes": list(SCHEMES),
                   "symbol": "rotated"},
        "roofline": roofline,
        "roofline_fp64": roofline_fp64,
        "cpu_baseline": cpu,
        "speedup_time_to_tol": accel,
        "fp32_at_fp64_iterations": same_iters,
        "symbol_controls": control,
        "plan": plan_report,
        "sweep": sweep,
        "extra_configs": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
