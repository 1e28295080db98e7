#!/usr/bin/env python3
"""H.psi band-application throughput of Chebyshev-filtered subspace iteration on one MI355X.

One step = one outer iteration of the method on the whole band block: the degree-m filter
T_m((S^-1 H - c)/r) X followed by Rayleigh-Ritz with residuals (Alg. 2), inputs resident in HBM.
value = nb * m * steps / wall time of the timed steps (FP64 path, the workload's own precision).

The default workload is paw128 (128^3 box, 137 065 plane waves, 2048 bands, 256 atoms x 13 projectors,
degree 12), the shape of the paper's 256-atom Ti crystal. Also reported on the same line: the mixed-precision
path (complex64 bands and FFTs, FP16-split MFMA projector GEMMs, FP64 Rayleigh-Ritz) on the same workload with its
accuracy over the lowest floor(0.8 nb) bands against the FP64 path run to convergence, per-kernel-class times
from HIP events in the timed region, the roofline of the dominant kernel and of every kernel class, the cost of
the adjoint against the forward pass (paw64 by default), and the FP64 CPU oracle timed on the host cores over a
bounded sample.

    python bench.py [--steps K] [--warmup W] [--config paw128] [--no-cpu] [--no-mixed] [--extras]
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
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "f16x3": 2500.0}
# vector ALU peaks (FMA = 2 flops): FP64 78.6; FP32 157.3 with packed FP32 instructions, which the build disables,
# so the FP32 kernels here issue at most half of it
VECTOR_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
MIXED_RESYNC_DEFAULT = 3  # a mixed plan recomputes the carried projections every 3rd filter step unless set
GEMM_CLASSES = ("project", "backproject", "small", "rr_gram", "rr_rotate")
FFT_CLASSES = ("fft_col_inverse", "fft_plane", "fft_col_forward")
# kernel names as rocprofv3 reports them, per timer class and precision
KERNEL_NAMES = {  # kernel of each timer class, FP64 / mixed plan
    "backproject": ("k_gemm<double, double, double, double, 1, 2>", "k_gemm_h<double, float, 1, 2>"),
    "project": ("k_gemm<double, double, double, double, 0, 1>", "k_gemm_h<double, double, 0, 1>"),
    "fft_plane": ("k_plane<{n}, double>", "k_plane<{n}, float>"),
    "fft_col_inverse": ("k_col_inv<{n}, double>", "k_col_inv<{n}, float>"),
    "fft_col_forward": ("k_col_fwd<{n}, double>", "k_col_fwd<{n}, float>"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_path(cf, pb, prec, lam_plus, steps, warmup, resync=None):
    """Warm up, then time `steps` outer iterations; returns timings, profile and the final state."""
    import torch

    plan = cf.plan_from_problem(pb, prec)
    if resync is not None:
        plan.set_projection_resync(resync)
    dtype = torch.complex64 if prec == cf.CHEB_MIXED else torch.complex128
    X = cf.to_device_block(pb.X0, dtype)
    m, nb = pb.cfg.m, pb.cfg.nb
    from paper_1406_4350_amd.driver import chebyshev_magnitude

    rq = plan.rayleigh_quotients(X)
    state = {"lam_minus": float(rq.max().item()), "lam_low": float(rq.min().item()), "stability": 0.0}
    # Rayleigh-Ritz hands the projections P^H X and (K + V) X of its rotated block to the next filter
    # (cheb_rayleigh_ritz_carry, cheb_filter_carry), so a step computes the projections once and transforms the
    # block m times (the filter's steps 2 .. m and Rayleigh-Ritz)
    pc = plan.projections(nb) if plan.nproj > 0 else None
    hx = torch.empty_like(X)
    state["carried"] = False

    def step():
        c = 0.5 * (lam_plus + state["lam_minus"])
        r = 0.5 * (lam_plus - state["lam_minus"])
        # amplification of the lowest band by this filter (Sec. 5.3: must stay far below 1/eps)
        state["stability"] = max(state["stability"], chebyshev_magnitude(m, (state["lam_low"] - c) / r))
        plan.filter(X, m, c, r, p_in=pc if state["carried"] else None, hx_in=hx if state["carried"] else None)
        ritz, res = plan.rayleigh_ritz(X, p_out=pc, hx_out=hx)
        state["carried"] = True
        state["ritz"], state["res"] = ritz, res
        state["lam_minus"] = float(ritz.max().item())
        state["lam_low"] = min(state["lam_low"], float(ritz.min().item()))

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
    reps = max(2, min(steps, 3))
    filter_ms = time_filter(plan, X, m, c, r, reps, pc, hx)
    out = dict(plan=plan, X=X, seconds=t1 - t0, prof=prof, filter_ms=filter_ms, state=state, rr_stats=rr_stats,
               apps_per_s=nb * m * steps / (t1 - t0), filter_apps_per_s=nb * m / (filter_ms * 1e-3), resync=resync)
    return out


def time_filter(plan, X, m, c, r, reps, pc=None, hx=None):
    """Mean event time (ms) of the filter on a fresh copy of X, as the bench step calls it (starting from the
    projections pc and (K + V) X hx that Rayleigh-Ritz returned for X, when given); the copies are outside the
    timed events."""
    import torch

    Xf = X.clone()
    kw = {"p_in": pc, "hx_in": hx}
    plan.filter(Xf, m, c, r, **kw)  # warm-up
    total = 0.0
    for _ in range(reps):
        Xf.copy_(X)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        plan.filter(Xf, m, c, r, **kw)
        ev1.record()
        torch.cuda.synchronize()
        total += ev0.elapsed_time(ev1)
    return total / reps


def class_roofline(name, d, kind, n):
    """Roofline numbers of one kernel class from its event timers: GEMM classes against the MFMA peak of the
    arithmetic they run on (FP64 for the FP64 path, the projector-space products and the Rayleigh-Ritz Grams in
    both paths, FP16 for the split projector GEMMs of mixed plans, where each useful product takes three FP16
    MFMAs), FFT classes against the HBM peak, and the plane pass (whose timers also count its transform
    arithmetic) against the vector ALU peak where that fraction is the larger. Achieved = algorithmic flops (8 per
    complex multiply-add; 5 n log2 n per length-n transform) or bytes per launch / average launch time."""
    per_launch_s = d["ms"] * 1e-3 / d["launches"]
    alu = False
    if name in GEMM_CLASSES:
        achieved = d["flops"] / d["launches"] / per_launch_s / 1e12
        dt = "f16x3" if (kind == "f32" and name in ("project", "backproject")) else "f64"
        peak = PEAK_TFLOPS[dt]
        out = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "mfma_dtype": dt}
        # flops the matrix cores execute per algorithmic flop: the FP64 tiles take 3 real products per complex
        # product (6 of the 8 counted flops), the FP16 split products 3 FP16 products per useful one
        out["executed_frac"] = achieved * (0.75 if dt == "f64" else 3.0) / peak
    else:
        achieved = d["bytes"] / d["launches"] / per_launch_s / 1e9
        out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        if d.get("flops", 0.0) > 0.0:
            # FFT arithmetic (5 n log2 n flops per length-n transform) against the vector ALU peak of the
            # precision; the class is bound by whichever roofline it comes closer to
            a_alu = d["flops"] / d["launches"] / per_launch_s / 1e12
            p_alu = VECTOR_PEAK_TFLOPS[kind]
            hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}
            if a_alu / p_alu > hbm["frac"]:
                alu = True
                out = {"bound": "alu", "achieved": a_alu, "peak": p_alu, "unit": "TFLOP/s", "hbm": hbm}
    out["frac"] = out["achieved"] / out["peak"]
    tmpl = KERNEL_NAMES.get(name)
    out["kernel"] = tmpl[0 if kind == "f64" else 1].format(n=n) if tmpl else name
    if name == "fft_plane" and kind == "f64" and n == 128:
        out["kernel"] = "k_plane_half"  # the FP64 128^3 plane pass runs in two halves of the y residues
    out["avg_launch_us"] = per_launch_s * 1e6
    out["algo_per_launch"] = (d["flops"] if (name in GEMM_CLASSES or alu) else d["bytes"]) / d["launches"]
    out["launches"] = d["launches"]
    out["ms_total"] = d["ms"]
    return out


def roofline(prof, kind, n):
    """Roofline object for the kernel class with the largest event time (the dense eigensolver is a library call,
    not one of this library's kernels, and is left out), plus the same numbers for every class."""
    cands = {k: v for k, v in prof.items() if k != "rr_eig" and v["launches"] > 0}
    dom = max(cands, key=lambda k: cands[k]["ms"])
    out = class_roofline(dom, cands[dom], kind, n)
    out["kernel_class"] = dom
    out["traffic"] = load_traffic(out["kernel"], n)
    out["by_class"] = {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                           for kk, vv in class_roofline(k, v, kind, n).items()} for k, v in cands.items()}
    return out


def load_traffic(kernel, n):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, if it covers this
    kernel at this box size and the kernel source it was taken on is unchanged; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        ent = data.get(kernel)
        if not ent or int(ent.get("n", n)) != int(n):
            return None
        import hashlib

        src = os.path.join(ROOT, "paper_1406_4350_amd", "csrc", ent["source"])
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        return ent["bytes_per_launch"] if h == ent["source_sha256"] else None
    except Exception:
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(pb, target_s=15.0):
    """The FP64 oracle's matrix-free filter on the host cores, on a sample of bands of the same workload: about
    target_s seconds of filtering (the operator set-up, a P^H P product of the projectors, is not timed)."""
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
        t_setup = time.perf_counter()
        ops = matfree.Operators.from_problem(pb, workers=cores, band_chunk=16)
        t_setup = time.perf_counter() - t_setup
        m = pb.cfg.m
        # calibrate, after a warm-up call (FFT plans, thread pools), on 8 bands with one application of S^-1 H
        ops.apply_A(pb.X0[:, :4])
        Xc = pb.X0[:, :min(8, pb.cfg.nb)]
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
            "cpu": cpu_model(),
            "sample": f"{reps} x one degree-{m} filter of {nbs} of {pb.cfg.nb} bands of the same workload (FP64 "
                      f"matrix-free oracle, numpy/scipy FFT and BLAS with {cores} threads), {dt:.1f} s timed; "
                      f"operator set-up {t_setup:.1f} s untimed"}


def continue_run(plan, X, m, lam_plus, ritz, res, k, tol, max_iters):
    """More outer iterations on X until the lowest k residuals are <= tol (at most max_iters)."""
    it = 0
    while it < max_iters and (tol is None or float(res[:k].max()) > tol):
        lam_minus = float(ritz.max())
        plan.filter(X, m, 0.5 * (lam_plus + lam_minus), 0.5 * (lam_plus - lam_minus))
        ritz, res = plan.rayleigh_ritz(X)
        it += 1
    return ritz, res, it


def mixed_accuracy(cf, pb, r64, rmx, lam_plus, max_extra, done):
    """Mixed-precision eigenpairs against converged FP64 ones over the lowest floor(0.8 nb) bands. The FP64 run is
    continued until those bands have residuals <= 1e-8 (at most max_extra more iterations) and serves as the
    reference; the mixed run is continued to the same number of iterations. A band meets the target when its
    mixed Ritz value is within 1e-6 Ha of the reference and the residual of its complex64 Ritz vector, re-evaluated
    with the FP64 operators, is <= 1e-5."""
    import numpy as np
    import torch

    m, k = pb.cfg.m, int(0.8 * pb.cfg.nb)
    st = r64["state"]
    ritz, res, extra = continue_run(r64["plan"], r64["X"], m, lam_plus, st["ritz"], st["res"], k, 1e-8, max_extra)
    lam_ref, res_ref = ritz.cpu().numpy(), res.cpu().numpy()
    sx = rmx["state"]
    ritz_x, _, extra_x = continue_run(rmx["plan"], rmx["X"], m, lam_plus, sx["ritz"], sx["res"], k, None, extra)
    lamx = ritz_x.cpu().numpy()
    plan = r64["plan"]
    U = rmx["X"].to(torch.complex128)
    HU = plan.apply_H(U)
    SU = plan.apply_S(U)
    lam_t = torch.from_numpy(lamx).to(U.device)
    res_x = torch.linalg.vector_norm(HU - SU * lam_t[:, None], dim=1).cpu().numpy()
    del U, HU, SU
    dlam = np.abs(lamx - lam_ref)[:k]
    ok = (dlam <= 1e-6) & (res_x[:k] <= 1e-5)
    return {"checked_bands": k, "iterations": done + extra,
            "fp64_reference": f"FP64 path run {done + extra} outer iterations; lowest {k} residuals <= "
                              f"{float(res_ref[:k].max()):.2e}",
            "max_abs_dlambda_Ha": float(dlam.max()), "max_resid_fp64_eval": float(res_x[:k].max()),
            "median_resid_fp64_eval": float(np.median(res_x[:k])),
            "bands_meeting_target": int(ok.sum()), "target_met": bool(ok.all()),
            "projection_resync_period": rmx.get("resync") if rmx.get("resync") is not None else MIXED_RESYNC_DEFAULT}


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
    """LOBPCG (Sec. 2.3, the paper's comparison method) from the same start block, FP64: iterations, band
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
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="paw128", help="workload name (paw128, paw96, paw64, paw48, nc16)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--ref-iters", type=int, default=25,
                    help="at most this many more FP64 iterations for the converged reference of the mixed accuracy "
                         "check (0: skip the check)")
    ap.add_argument("--resync", type=int, default=None,
                    help="projection resynchronisation period of the mixed plan (default: the library's)")
    ap.add_argument("--backward-config", default="paw64",
                    help="workload of the adjoint cost leg ('none' to skip)")
    ap.add_argument("--extras", action="store_true",
                    help="also run the locking, LOBPCG, Gamma-point and iterative capacitance legs on --extras-config")
    ap.add_argument("--extras-config", default="paw48")
    ap.add_argument("--lock-tol", type=float, default=1e-8)
    ap.add_argument("--lock-iters", type=int, default=40)
    ap.add_argument("--lobpcg-iters", type=int, default=60)
    ap.add_argument("--cap-iters", type=int, default=20)
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

    t_start = time.perf_counter()
    pb = wl.make_problem(args.config)
    cfg = pb.cfg
    log(f"[bench] workload {cfg.name}: n={cfg.n} npw={pb.npw} nb={cfg.nb} nproj={pb.nproj} m={cfg.m} "
        f"({time.perf_counter() - t_start:.1f} s to draw)")
    probe = cf.plan_from_problem(pb, cf.CHEB_FP64)
    lam_plus = probe.upper_bound(torch.from_numpy(pb.v0), 10)
    probe.close()
    del probe
    log(f"[bench] lambda+ = {lam_plus:.6f} (10-step Lanczos)")

    r64 = run_path(cf, pb, cf.CHEB_FP64, lam_plus, args.steps, args.warmup)
    log(f"[bench] fp64: {r64['apps_per_s']:.4g} band-apps/s over {args.steps} steps ({r64['seconds']:.1f} s), filter "
        f"alone {r64['filter_apps_per_s']:.4g}/s")
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
        "stability_T_m_lowest_band": r64["state"]["stability"],
        "roofline": roofline(r64["prof"], "f64", cfg.n),
    }
    if not args.no_mixed:
        rmx = run_path(cf, pb, cf.CHEB_MIXED, lam_plus, args.steps, args.warmup, resync=args.resync)
        log(f"[bench] mixed: {rmx['apps_per_s']:.4g} band-apps/s, filter alone {rmx['filter_apps_per_s']:.4g}/s")
        out["mixed"] = {
            "value": rmx["apps_per_s"], "ratio_vs_fp64": rmx["apps_per_s"] / r64["apps_per_s"],
            "filter_apps_per_s": rmx["filter_apps_per_s"],
            "filter_ratio_vs_fp64": rmx["filter_apps_per_s"] / r64["filter_apps_per_s"],
            "ms_per_step": rmx["seconds"] * 1e3 / args.steps,
            "dtype": "f32 (complex64 bands/FFTs/recurrence; projector GEMMs on FP16 hi/lo split MFMA with FP32 "
                     "accumulation); FP64 projector space and Rayleigh-Ritz",
            "breakdown_ms_per_step": {k: v["ms"] / args.steps for k, v in rmx["prof"].items()},
            "rr_solves_refined_library": rmx["rr_stats"],
            "roofline": roofline(rmx["prof"], "f32", cfg.n),
        }
        if args.ref_iters > 0:
            acc = mixed_accuracy(cf, pb, r64, rmx, lam_plus, args.ref_iters, args.warmup + args.steps)
            out["mixed"]["accuracy"] = acc
            log(f"[bench] mixed accuracy over the lowest {acc['checked_bands']} bands after {acc['iterations']} "
                f"iterations: max |d lambda| {acc['max_abs_dlambda_Ha']:.2e} Ha, max FP64-evaluated residual "
                f"{acc['max_resid_fp64_eval']:.2e}, target met: {acc['target_met']}")
        rmx["plan"].close()
        del rmx
    r64["plan"].close()
    del r64
    torch.cuda.empty_cache()
    if args.backward_config != "none":
        pbb = wl.make_problem(args.backward_config)
        pr = cf.plan_from_problem(pbb, cf.CHEB_FP64)
        lpb = pr.upper_bound(torch.from_numpy(pbb.v0), 10)
        pr.close()
        out["differentiation"] = time_backward(cf, pbb, lpb)
        out["differentiation"]["workload"] = args.backward_config
    if args.extras:
        pe = wl.make_problem(args.extras_config)
        pr = cf.plan_from_problem(pe, cf.CHEB_FP64)
        lpe = pr.upper_bound(torch.from_numpy(pe.v0), 10)
        pr.close()
        ex = {"workload": args.extras_config}
        if args.lock_tol > 0:
            ex["locking"] = locking_report(cf, pe, lpe, args.lock_tol, args.lock_iters)
            if args.lobpcg_iters > 0:
                ex["lobpcg"] = lobpcg_report(cf, pe, args.lock_tol, args.lobpcg_iters)
        ex["gamma_point"] = gamma_report(cf, args.extras_config, args.steps, args.warmup)
        if args.cap_iters > 0:
            ex["capacitance_solve"] = capacitance_report(cf, pe, lpe, args.cap_iters)
        out["extras"] = ex
    if not args.no_cpu:
        log("[bench] timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(pb)
        log(f"[bench] cpu oracle: {out['cpu_baseline']['value']:.4g} band-apps/s")
    out["device"] = device_report()
    out["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
