#!/usr/bin/env python3
"""H.psi band-application throughput of Chebyshev-filtered subspace iteration on one MI355X.

One step = one outer iteration of the method on the whole band block: the degree-m filter
T_m((S^-1 H - c)/r) X followed by Rayleigh-Ritz with residuals (Alg. 2), inputs resident in HBM.
value = nb * m * steps / wall time of the timed steps (FP64 path, the workload's own precision).

Also reported on the same line: the mixed-precision path (complex64 bands and FFTs, FP32-MFMA GEMMs, FP64
Rayleigh-Ritz) on the same workload with its accuracy against the FP64 path, per-kernel-class times from
HIP events in the timed region, the roofline of the dominant kernel class, and the FP64 CPU oracle timed
on the host cores over a bounded sample.

    python bench.py [--steps K] [--warmup W] [--config paw48] [--no-cpu] [--no-mixed]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H·ψ band-applications/s (FP32-MFMA vs FP64) at ≤1e-6 Ha; % HBM/MFMA roofline"
HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
GEMM_CLASSES = ("project", "backproject", "small", "rr_gram", "rr_rotate")
FFT_CLASSES = ("fft_col_inverse", "fft_plane", "fft_col_forward")
# kernel names as rocprofv3 reports them, per timer class and precision
KERNEL_NAMES = {  # kernel of each timer class, FP64 / mixed plan
    "backproject": ("k_gemm<double, double, double, double, 1, 2>", "k_gemm_h<double, float, 1, 2>"),
    "project": ("k_gemm<double, double, double, double, 0, 1>", "k_gemm_h<float, double, 0, 1>"),
    "fft_plane": ("k_plane<{n}, double>", "k_plane<{n}, float>"),
    "fft_col_inverse": ("k_col_inv<{n}, double>", "k_col_inv<{n}, float>"),
    "fft_col_forward": ("k_col_fwd<{n}, double>", "k_col_fwd<{n}, float>"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_path(cf, pb, prec, lam_plus, steps, warmup):
    """Warm up, then time `steps` outer iterations; returns timings, profile and the final state."""
    import torch

    plan = cf.plan_from_problem(pb, prec)
    dtype = torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128
    X = cf.to_device_block(pb.X0, dtype)
    m, nb = pb.cfg.m, pb.cfg.nb
    state = {"lam_minus": float(plan.rayleigh_quotients(X).max().item())}

    def step():
        c = 0.5 * (lam_plus + state["lam_minus"])
        r = 0.5 * (lam_plus - state["lam_minus"])
        plan.filter(X, m, c, r)
        ritz, res = plan.rayleigh_ritz(X)
        state["ritz"], state["res"] = ritz, res
        state["lam_minus"] = float(ritz.max().item())

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_read()
    plan.profile_enable(False)
    rr_stats = plan.rr_stats()

    # filter alone, event-timed on the current stream (same block, same interval)
    c = 0.5 * (lam_plus + state["lam_minus"])
    r = 0.5 * (lam_plus - state["lam_minus"])
    reps = max(3, min(steps, 10))
    filter_ms = time_filter(plan, X, m, c, r, reps)
    out = dict(plan=plan, X=X, seconds=t1 - t0, prof=prof, filter_ms=filter_ms, state=state, rr_stats=rr_stats,
               apps_per_s=nb * m * steps / (t1 - t0), filter_apps_per_s=nb * m / (filter_ms * 1e-3))
    if prec == cf.CHEB_MIXED:  # the same filter with the projector GEMMs on the FP32 MFMA instead of the split
        plan.set_split_gemm(False)
        out["filter_apps_per_s_fp32_mfma"] = nb * m / (time_filter(plan, X, m, c, r, reps) * 1e-3)
        plan.set_split_gemm(True)
    return out


def time_filter(plan, X, m, c, r, reps):
    """Mean event time (ms) of cheb_filter on a fresh copy of X; the copies are outside the timed events."""
    import torch

    Xf = X.clone()
    plan.filter(Xf, m, c, r)  # warm-up
    total = 0.0
    for _ in range(reps):
        Xf.copy_(X)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        plan.filter(Xf, m, c, r)
        ev1.record()
        torch.cuda.synchronize()
        total += ev0.elapsed_time(ev1)
    return total / reps


def roofline(prof, kind, n):
    """Roofline object for the kernel class with the largest event time (the dense eigensolver is a
    library call, not one of this library's kernels, and is left out)."""
    cands = {k: v for k, v in prof.items() if k != "rr_eig" and v["launches"] > 0}
    dom = max(cands, key=lambda k: cands[k]["ms"])
    d = cands[dom]
    per_launch_s = d["ms"] * 1e-3 / d["launches"]
    if dom in GEMM_CLASSES:
        achieved = d["flops"] / d["launches"] / per_launch_s / 1e12
        # the Rayleigh-Ritz Grams run on FP64 MFMA in both precisions
        peak = PEAK_TFLOPS["f64" if dom == "rr_gram" else kind]
        out = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s"}
    else:
        achieved = d["bytes"] / d["launches"] / per_launch_s / 1e9
        peak = HBM_PEAK_GBS
        out = {"bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["kernel_class"] = dom
    tmpl = KERNEL_NAMES.get(dom)
    out["kernel"] = tmpl[0 if kind == "f64" else 1].format(n=n) if tmpl else dom
    out["avg_launch_us"] = per_launch_s * 1e6
    out["algo_per_launch"] = (d["flops"] if dom in GEMM_CLASSES else d["bytes"]) / d["launches"]
    out["traffic"] = load_traffic(out["kernel"])
    return out


def load_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, if it covers this
    kernel and the kernel source it was taken on is unchanged; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(kernel)
        if not ent:
            return None
        import hashlib

        src = os.path.join(ROOT, "paper_1406_4350_amd", "csrc", ent["source"])
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        return ent["bytes_per_launch"] if h == ent["source_sha256"] else None
    except Exception:
        return None


def cpu_baseline(pb, target_s=15.0):
    """The FP64 oracle's matrix-free filter on the host cores, on a sample of bands of the same workload."""
    import numpy as np

    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    from oracle import matfree

    cores = len(os.sched_getaffinity(0))
    import contextlib

    ctx = threadpool_limits(limits=cores) if threadpool_limits else contextlib.nullcontext()
    with ctx:
        ops = matfree.Operators.from_problem(pb, workers=cores)
        m = pb.cfg.m
        # calibrate, after a warm-up call (FFT plans, thread pools), on 16 bands with one application of S^-1 H
        ops.apply_A(pb.X0[:, :4])
        Xc = pb.X0[:, :min(16, pb.cfg.nb)]
        t0 = time.perf_counter()
        ops.apply_A(Xc)
        per_app = (time.perf_counter() - t0) / Xc.shape[1]
        nbs = int(max(4, min(pb.cfg.nb, target_s / max(per_app * m, 1e-9))))
        Xs = np.asfortranarray(pb.X0[:, :nbs])
        # the whole block may take less than the target: repeat the same filter until the target is reached
        reps, dt = 0, 0.0
        while reps == 0 or dt < 0.8 * target_s:
            t0 = time.perf_counter()
            matfree.chebyshev_filter(ops, Xs, m, 1.0, 2.0)
            dt += time.perf_counter() - t0
            reps += 1
    return {"value": reps * nbs * m / dt, "unit": "band-applications/s", "cores": cores, "kind": "oracle",
            "sample": f"{reps} x one degree-{m} filter of {nbs} of {pb.cfg.nb} bands (FP64 matrix-free oracle, "
                      f"numpy/scipy FFT with {cores} workers), {dt:.1f} s"}


def mixed_accuracy(cf, pb, r64, rmx, lam_plus, extra=30):
    """Mixed-precision eigenpairs against converged FP64 ones. The FP64 run is continued for `extra` more
    iterations to serve as the reference; a mixed band meets the target when its residual, re-evaluated with
    the FP64 operators, is <= 1e-5 and its Ritz value is within 1e-6 Ha of the reference."""
    import numpy as np
    import torch

    plan = r64["plan"]
    X = r64["X"]
    lam_minus = float(r64["state"]["ritz"].max().item())
    for _ in range(extra):
        c, r = 0.5 * (lam_plus + lam_minus), 0.5 * (lam_plus - lam_minus)
        plan.filter(X, pb.cfg.m, c, r)
        ritz, res = plan.rayleigh_ritz(X)
        lam_minus = float(ritz.max().item())
    lam_ref, res_ref = ritz.cpu().numpy(), res.cpu().numpy()
    lamx = rmx["state"]["ritz"].cpu().numpy()
    U = rmx["X"].to(torch.complex128)
    HU = plan.apply_H(U)
    SU = plan.apply_S(U)
    lam_t = torch.from_numpy(lamx).to(U.device)
    res_x = torch.linalg.vector_norm(HU - SU * lam_t[:, None], dim=1).cpu().numpy()
    ref_ok = res_ref <= 1e-8
    conv = (res_x <= 1e-5) & ref_ok
    dlam = np.abs(lamx - lam_ref)
    ok = conv & (dlam <= 1e-6)
    return {"reference": f"FP64 path continued {extra} more iterations; {int(ref_ok.sum())} bands with residual <= 1e-8",
            "bands_converged_mixed": int(conv.sum()), "bands_meeting_target": int(ok.sum()),
            "max_abs_dlambda_converged_Ha": float(dlam[conv].max()) if conv.any() else None,
            "max_resid_fp64_eval_converged": float(res_x[conv].max()) if conv.any() else None}


def time_backward(cf, pb, lam_plus, reps=3):
    """Forward (filter + Rayleigh-Ritz) against forward + adjoint (cheb_filter_rr_backward), both precisions."""
    import torch

    out = {}
    m, nk = pb.cfg.m, min(pb.cfg.nk, pb.cfg.nb)
    for prec, name in ((cf.CHEB_FP64, "fp64"), (cf.CHEB_MIXED, "mixed")):
        plan = cf.plan_from_problem(pb, prec)
        dtype = torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128
        X0 = cf.to_device_block(pb.X0, dtype)
        lm = float(plan.rayleigh_quotients(X0).max().item())
        c, r = 0.5 * (lam_plus + lm), 0.5 * (lam_plus - lm)
        w = torch.from_numpy(pb.w[:nk])

        def fwd():
            Y = X0.clone()
            plan.filter(Y, m, c, r)
            plan.rayleigh_ritz(Y, with_residuals=False)

        def bwd():
            plan.filter_rr_backward(X0, m, c, r, w, 3)
        times = {}
        for key, fn in (("forward", fwd), ("forward_plus_adjoint", bwd)):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            times[key] = (time.perf_counter() - t0) / reps * 1e3
        times["adjoint_over_forward"] = (times["forward_plus_adjoint"] - times["forward"]) / times["forward"]
        out[name] = {k: round(v, 4) for k, v in times.items()}
        log(f"[bench] {name}: forward {times['forward']:.2f} ms, with adjoint {times['forward_plus_adjoint']:.2f} ms")
        plan.close()
    out["note"] = f"ms per call, nb={pb.cfg.nb}, m={m}, loss over the lowest {nk} Ritz values, checkpoints every 3 steps"
    return out


def locking_report(cf, pb, lam_plus, tol, iters):
    """Outer loop from the start block with the fixed degree m and with locking (Sec. 5.4, degrees from the
    Eq. 5 estimate): band-applications and wall time until the lowest 7/8 of the bands have residuals <= 2 tol
    (locked bands settle just below tol)."""
    import numpy as np
    import torch

    from paper_1406_4350_amd.driver import chebfsi

    nwant = pb.cfg.nb - pb.cfg.nb // 8
    out = {"tol": tol, "wanted_bands": nwant, "max_iters": iters}
    for name, lt in (("fixed_degree", None), ("locking", tol)):
        plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
        X = cf.to_device_block(pb.X0, torch.complex128)
        chebfsi(plan, X.clone(), pb.cfg.m, 1, lam_plus)  # warm-up: workspaces, code objects
        hist = chebfsi(plan, X, pb.cfg.m, iters, lam_plus, lock_tol=lt)[2]
        secs = np.cumsum([h["seconds"] for h in hist])
        apps = np.cumsum([h["band_applications"] for h in hist])
        hit = [i for i, h in enumerate(hist) if np.max(h["resid"][:nwant]) <= 2 * tol]
        k = hit[0] if hit else None
        out[name] = {"iterations": None if k is None else k + 1,
                     "band_applications": None if k is None else int(apps[k]),
                     "seconds": None if k is None else round(float(secs[k]), 4),
                     "locked_bands_last": int(hist[k]["locked"] or 0) if k is not None else None}
        log(f"[bench] {name}: reached after {out[name]['iterations']} iterations, "
            f"{out[name]['band_applications']} band-applications, {out[name]['seconds']} s")
        plan.close()
    f, l = out["fixed_degree"], out["locking"]
    if f["seconds"] and l["seconds"]:
        out["speedup"] = round(f["seconds"] / l["seconds"], 3)
        out["band_application_ratio"] = round(l["band_applications"] / f["band_applications"], 3)
    return out


def lobpcg_report(cf, pb, tol, iters):
    """LOBPCG (Sec. 3.1, the paper's comparison method) from the same start block, FP64: iterations, band
    applications of H (each also applies S) and wall time until the lowest 7/8 of the bands have residuals
    <= 2 tol, as for the Chebyshev runs of locking_report."""
    import numpy as np
    import torch

    from paper_1406_4350_amd.driver import lobpcg

    nwant = pb.cfg.nb - pb.cfg.nb // 8
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    lobpcg(plan, cf.to_device_block(pb.X0, torch.complex128), 1, tol)  # warm-up
    X = cf.to_device_block(pb.X0, torch.complex128)
    _, hist = lobpcg(plan, X, iters, tol)
    plan.close()
    secs = np.cumsum([h["seconds"] for h in hist])
    apps = np.cumsum([pb.cfg.nb] + [h["active"] for h in hist[1:]])
    # residuals reported at iteration k are those of the vectors after iteration k - 1
    hit = [i for i, h in enumerate(hist) if h["resid"] is not None and np.max(h["resid"][:nwant]) <= 2 * tol]
    k = hit[0] - 1 if hit else None
    out = {"tol": tol, "wanted_bands": nwant, "max_iters": iters,
           "iterations": k, "band_applications": None if k is None else int(apps[k]),
           "seconds": None if k is None else round(float(secs[k]), 4)}
    log(f"[bench] lobpcg: reached after {out['iterations']} iterations, {out['band_applications']} "
        f"band-applications, {out['seconds']} s")
    return out


def gamma_report(cf, name, steps, warmup):
    """The same workload at the Gamma point (real wavefunctions on the half sphere, two bands per complex
    transform): FP64 filter + Rayleigh-Ritz steps and the filter alone, FP64 and mixed."""
    import torch

    from paper_1406_4350_amd import workload as wl

    gp = wl.make_gamma_problem(name)
    probe = cf.plan_from_problem(gp, cf.CHEB_FP64)
    lam_plus = probe.upper_bound(torch.from_numpy(gp.v0), 10)
    probe.close()
    out = {"npw_half": gp.npw}
    for prec, name in ((cf.CHEB_FP64, "fp64"), (cf.CHEB_MIXED, "mixed")):
        r = run_path(cf, gp, prec, lam_plus, steps, warmup)
        out[name] = {"apps_per_s": r["apps_per_s"], "filter_apps_per_s": r["filter_apps_per_s"],
                     "ms_per_step": r["seconds"] * 1e3 / steps}
        log(f"[bench] gamma {name}: {r['apps_per_s']:.4g} band-apps/s, filter alone {r['filter_apps_per_s']:.4g}/s")
        r["plan"].close()
    return out


def device_report():
    """The device, the software and a measured device-to-device copy rate (read + write bytes / time) for
    context beside the 8 TB/s peak."""
    import torch

    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    gbps = 5 * 2 * src.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del src, dst
    return {"name": torch.cuda.get_device_name(0), "hip": torch.version.hip, "torch": torch.__version__,
            "copy_GBps": round(gbps, 1)}


def capacitance_report(cf, pb, lam_plus, iters):
    """FP64 filter with the capacitance solve applied directly and by `iters` corrections of the
    block-preconditioned iterative refinement of Sec. 5.1; relative difference of S^-1 X between the two."""
    import torch

    if pb.Q is None:
        return None
    plan = cf.plan_from_problem(pb, cf.CHEB_FP64)
    X = cf.to_device_block(pb.X0, torch.complex128)
    m, nb = pb.cfg.m, pb.cfg.nb
    lm = float(plan.rayleigh_quotients(X).max().item())
    c, r = 0.5 * (lam_plus + lm), 0.5 * (lam_plus - lm)
    out = {"corrections": iters}
    direct = plan.apply_Sinv(X).clone()
    out["direct_filter_apps_per_s"] = nb * m / (time_filter(plan, X, m, c, r, 5) * 1e-3)
    plan.set_capacitance_solver(iters)
    refined = plan.apply_Sinv(X)
    out["iterative_filter_apps_per_s"] = nb * m / (time_filter(plan, X, m, c, r, 5) * 1e-3)
    out["sinv_rel_diff"] = float(torch.linalg.norm(refined - direct) / torch.linalg.norm(direct))
    plan.set_capacitance_solver(0)
    plan.close()
    log(f"[bench] capacitance: direct {out['direct_filter_apps_per_s']:.4g}/s, {iters} corrections "
        f"{out['iterative_filter_apps_per_s']:.4g}/s, S^-1 difference {out['sinv_rel_diff']:.2e}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="paw48", help="workload name (paw48, paw64, paw96, paw128, nc16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--ref-iters", type=int, default=30,
                    help="extra FP64 iterations for the converged reference of the mixed accuracy check (0: skip)")
    ap.add_argument("--backward", action="store_true",
                    help="also time the adjoint of one filter + Rayleigh-Ritz pass against the forward pass")
    ap.add_argument("--lock-tol", type=float, default=1e-8,
                    help="residual tolerance of the locking comparison (0: skip it)")
    ap.add_argument("--lock-iters", type=int, default=40)
    ap.add_argument("--lobpcg-iters", type=int, default=60,
                    help="iteration cap of the LOBPCG comparison at the locking tolerance (0: skip)")
    ap.add_argument("--no-gamma", action="store_true", help="skip the Gamma-point form of the workload")
    ap.add_argument("--cap-iters", type=int, default=20,
                    help="corrections of the iterative capacitance solve to compare with the direct one (0: skip)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes three times (for scaling HBM "
                         "byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch

        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the filter shards by bands with no communication and the multi-GPU "
              "Rayleigh-Ritz exchange is not built; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    from paper_1406_4350_amd import chebfd as cf
    from paper_1406_4350_amd import workload as wl

    pb = wl.make_problem(args.config)
    cfg = pb.cfg
    log(f"[bench] workload {cfg.name}: n={cfg.n} npw={pb.npw} nb={cfg.nb} nproj={pb.nproj} m={cfg.m}")
    probe = cf.plan_from_problem(pb, cf.CHEB_FP64)
    lam_plus = probe.upper_bound(torch.from_numpy(pb.v0), 10)
    probe.close()
    log(f"[bench] lambda+ = {lam_plus:.6f} (10-step Lanczos)")

    r64 = run_path(cf, pb, cf.CHEB_FP64, lam_plus, args.steps, args.warmup)
    log(f"[bench] fp64: {r64['apps_per_s']:.4g} band-apps/s over {args.steps} steps, filter alone "
        f"{r64['filter_apps_per_s']:.4g}/s")
    out = {
        "metric": METRIC,
        "value": r64["apps_per_s"],
        "unit": "band-applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["seconds"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.n}^3 FFT box, sphere radius {cfg.radius} ({pb.npw} plane waves), "
                               f"{cfg.nb} bands, {cfg.natom} atoms x {pb.nproj // cfg.natom} projectors, "
                               f"{'PAW S via Woodbury' if cfg.overlap else 'S = I'}, degree m={cfg.m}, "
                               "one step = filter + Rayleigh-Ritz",
                   "npw": pb.npw, "nb": cfg.nb, "nproj": pb.nproj, "m": cfg.m, "n": cfg.n},
        "filter_only": {"fp64_apps_per_s": r64["filter_apps_per_s"], "fp64_ms": r64["filter_ms"]},
        "breakdown_ms_per_step": {k: v["ms"] / args.steps for k, v in r64["prof"].items()},
        "rr_solves_refined_library": r64["rr_stats"],
        "roofline": roofline(r64["prof"], "f64", cfg.n),
    }
    if not args.no_mixed:
        rmx = run_path(cf, pb, cf.CHEB_MIXED, lam_plus, args.steps, args.warmup)
        log(f"[bench] mixed: {rmx['apps_per_s']:.4g} band-apps/s, filter alone {rmx['filter_apps_per_s']:.4g}/s")
        out["mixed"] = {
            "value": rmx["apps_per_s"], "ratio_vs_fp64": rmx["apps_per_s"] / r64["apps_per_s"],
            "filter_apps_per_s": rmx["filter_apps_per_s"],
            "filter_ratio_vs_fp64": rmx["filter_apps_per_s"] / r64["filter_apps_per_s"],
            "filter_apps_per_s_fp32_mfma": rmx["filter_apps_per_s_fp32_mfma"],
            "dtype": "f32 (complex64 bands/FFTs/recurrence; projector GEMMs on FP16 hi/lo split MFMA with FP32 "
                     "accumulation); FP64 projector space and Rayleigh-Ritz",
            "accuracy": mixed_accuracy(cf, pb, r64, rmx, lam_plus, args.ref_iters) if args.ref_iters > 0 else None,
            "breakdown_ms_per_step": {k: v["ms"] / args.steps for k, v in rmx["prof"].items()},
            "rr_solves_refined_library": rmx["rr_stats"],
            "roofline": roofline(rmx["prof"], "f32", cfg.n),
        }
    if args.lock_tol > 0:
        out["locking"] = locking_report(cf, pb, lam_plus, args.lock_tol, args.lock_iters)
    if args.lobpcg_iters > 0 and args.lock_tol > 0:
        out["lobpcg"] = lobpcg_report(cf, pb, args.lock_tol, args.lobpcg_iters)
    if not args.no_gamma:
        out["gamma_point"] = gamma_report(cf, args.config, args.steps, args.warmup)
    if args.cap_iters > 0:
        out["capacitance_solve"] = capacitance_report(cf, pb, lam_plus, args.cap_iters)
    if args.backward:
        out["differentiation"] = time_backward(cf, pb, lam_plus)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(pb)
    out["device"] = device_report()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
