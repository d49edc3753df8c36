"""Benchmark of the semi-implicit Fourier-spectral (FS) phase-field step on
one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]

Headline: FS grid-point updates per second on 2D 1024 x 1024 with c + 4 eta
(F = 5 fields), FP32, seeded synthetic initial state, the inputs resident in
HBM before the timed region.  One "step" is one FS time step of the whole
grid (free-energy derivatives, forward transforms, k-space solve, inverse
transforms).  Exactly K steps are timed between two device
synchronisations.

Also reported on the same JSON line:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average launch time (HIP events on the library's stream),
                against 8 TB/s HBM
  cpu_baseline  the FP64 CPU oracle on a bounded sample of the same workload
  extras        FP64 path, 3D 256^3 FS (FP32, FP64), explicit FD step,
                adjoint step cost, and the paper's own FS-vs-FD figures
"""

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "FS grid-pt updates/s, 2D 1024² & 3D 256³, FP32 vs FP64; % HBM roofline"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(cfg, prec, kind):
    """Algorithmic HBM bytes of one launch of a 2D pass over the whole grid,
    from the per-stage figures of the unfused method, in which each stage of
    Algorithm 1 reads its inputs and writes its outputs once (an FFT counts
    one read and one write of the F fields), with s bytes per real value:

        derivative  2 F s    forward FFT  2 F s    k-space update  3 F s
        inverse FFT 2 F s    (whole step: 9 F s per grid point)

    Row pass: the derivative plus the x halves of both FFTs, 4 F s per point.
    Column pass: the update plus the y halves of both FFTs, 5 F s per point.
    """
    F = 1 + cfg["p"]
    P = cfg["n"][0] * cfg["n"][1] * (cfg["n"][2] if cfg["ndim"] == 3 else 1)
    s = 4 if prec == "f32" else 8
    per_point = {"row": 4, "col": 5, "step": 9}[kind]
    return per_point * F * s * P


def compulsory_bytes(cfg, prec, kind):
    """Bytes one launch of the fused 2D pass must move at the least, each of
    its own inputs read once and each output written once.

    Row pass: reads the F state x-spectra, writes the F right-hand-side
    x-spectra (df/dc and eta_i - dt L df/deta_i).  Column pass: reads those F
    plus the carried spectrum of c, writes the F new state x-spectra plus the
    carried spectrum.  An x-spectrum field holds (Nx/2 + 1) complex values
    per row.
    """
    F = 1 + cfg["p"]
    nx, ny = cfg["n"][0], cfg["n"][1]
    nz = cfg["n"][2] if cfg["ndim"] == 3 else 1
    s = 4 if prec == "f32" else 8
    spec = (nx // 2 + 1) * ny * nz * 2 * s  # one x-spectrum field
    if kind == "row":
        return 2 * F * spec
    if kind == "col":
        return (2 * F + 2) * spec
    raise ValueError(kind)


def rel_l2(got, ref, floor=1e-30):
    """Per-field relative L2 error ||got - ref|| / ||ref|| (None where the
    reference norm is below floor * sqrt(P): relaxed order parameters)."""
    import numpy as np
    out = []
    for f in range(ref.shape[0]):
        nb = float(np.linalg.norm(ref[f]))
        out.append(None if nb < floor * np.sqrt(ref[f].size)
                   else float(np.linalg.norm(got[f] - ref[f])) / nb)
    return out


def max_err(errs):
    vals = [e for e in errs if e is not None]
    return max(vals) if vals else None


def pass_rates(solver, cfg, prec, reps):
    """Average launch time of each steady-state 2D pass (pf_time_pass, HIP
    events on the library's stream) and the rates on its algorithmic and
    compulsory bytes."""
    from paper_2306_04322_amd import pfspec as PF
    out = {}
    for name, pid in (("row", 0), ("col", 1)):
        ms = PF.pf_time_pass(solver.h, pid, reps)
        a = algorithmic_bytes(cfg, prec, name)
        c = compulsory_bytes(cfg, prec, name)
        out[name] = {"avg_launch_us": round(ms * 1e3, 3),
                     "algorithmic_bytes_per_launch": a,
                     "achieved_GBs": round(a / (ms * 1e-3) / 1e9, 1),
                     "frac": round(a / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "compulsory_bytes_per_launch": c,
                     "compulsory_GBs": round(c / (ms * 1e-3) / 1e9, 1)}
    return out


def energy_passes(solver, cfg, prec, reps=20):
    """Device time per launch of the kernels of one pf_energy call (HIP events
    around each launch, pf_profile_*), for both gradient forms, with the rate
    on each kernel's compulsory bytes.  Spectral form: the row pass reads the
    F real fields and writes their F x-spectra, the column pass reads those
    (its outputs are per-work-group partial sums).  FD form: one kernel
    reading the F real fields.  Each call ends in a host readback, so every
    pass starts on an idle GPU."""
    from paper_2306_04322_amd import pfspec as PF
    F = 1 + cfg["p"]
    nx, ny = cfg["n"][0], cfg["n"][1]
    nz = cfg["n"][2] if cfg["ndim"] == 3 else 1
    s = 4 if prec == "f32" else 8
    real = F * nx * ny * nz * s
    spec = F * (nx // 2 + 1) * ny * nz * 2 * s
    out = {}
    for scheme, kernels in (("fs", (("row", PF.PROF_ROW, real + spec), ("col", PF.PROF_COL, spec))),
                            ("fd", (("fd", PF.PROF_FD, real),))):
        PF.pf_profile_enable(solver.h, True)
        for _ in range(reps):
            solver.energy(scheme)
        rec = {}
        for name, cls, nb in kernels + (("reduce", PF.PROF_RED, 0),):
            n, ms = PF.pf_profile_read(solver.h, cls)
            us = 1e3 * ms / max(1, n)
            rec[name] = {"launches": n, "avg_launch_us": round(us, 2)}
            if nb:
                rec[name].update({"compulsory_bytes_per_launch": nb,
                                  "compulsory_GBs": round(nb / (us * 1e-6) / 1e9, 1),
                                  "frac": round(nb / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
        PF.pf_profile_enable(solver.h, False)
        out[scheme] = rec
    return out


def passes_3d(solver, prec, dt, steps=10):
    """Per-pass times of the 3D 256^3 FS step and the rates on each pass's
    compulsory bytes (F = 5 x-spectra in and out; the z update one more each
    way for the carried c spectrum).  Row pass and z update: pf_time_pass
    (steady-state pass launched back to back between two events); the two y
    passes: the per-launch events of `steps` steps (pf_profile_*) less the z
    updates among them."""
    from paper_2306_04322_amd import pfspec as PF
    s = 4 if prec == "f32" else 8
    half = 256 * 256 * 129 * 2 * s
    row_us = 1e3 * PF.pf_time_pass(solver.h, 0, 20)
    z_us = 1e3 * PF.pf_time_pass(solver.h, 1, 20)
    PF.pf_profile_enable(solver.h, True)
    solver.step_fs(dt, steps)
    n_col, ms_col = PF.pf_profile_read(solver.h, PF.PROF_COL)
    PF.pf_profile_enable(solver.h, False)
    y_us = (1e3 * ms_col - steps * z_us) / max(1, n_col - steps)
    out = {}
    for name, us, nb in (("row", row_us, 10 * half), ("y_forward_or_inverse", y_us, 10 * half),
                         ("z_update", z_us, 12 * half)):
        out[name] = {"avg_launch_us": round(us, 2), "compulsory_bytes_per_launch": nb,
                     "compulsory_GBs": round(nb / (us * 1e-6) / 1e9, 1)}
    return out


def time_fs(solver, dt, steps, warmup, torch):
    if warmup:
        solver.step_fs(dt, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step_fs(dt, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10):
    """Device copy rate in GB/s (bytes read + bytes written per second) of a
    buffer four times the size of the last-level cache, with torch's copy
    kernel timed by events on torch's current stream."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def kernel_profile(solver, dt, steps, torch):
    from paper_2306_04322_amd import pfspec as P
    P.pf_profile_enable(solver.h, True)
    solver.step_fs(dt, steps)
    out = {}
    for name, cls in (("row", P.PROF_ROW), ("col", P.PROF_COL), ("reduce", P.PROF_RED)):
        n, ms = P.pf_profile_read(solver.h, cls)
        out[name] = (n, ms)
    P.pf_profile_enable(solver.h, False)
    return out


def cpu_baseline(cfg, u0, dt, budget_s=20.0):
    """FP64 oracle on the same workload, as many whole steps as fit the
    budget (at least one), timed on one host core.  Returns the record and
    the oracle's fields after those steps (for the error check)."""
    import numpy as np
    from oracle import fs as ofs
    P = int(np.prod(u0.shape[1:]))
    steps = 0
    u = u0
    # the calling thread runs the oracle pinned to one of the host cores it
    # may use; the affinity is restored afterwards
    allowed = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {allowed[0]})
    try:
        r0 = resource.getrusage(resource.RUSAGE_THREAD)
        t0 = time.perf_counter()
        while True:
            u = ofs.fs_run(u, cfg, dt, 1)
            steps += 1
            el = time.perf_counter() - t0
            if el >= budget_s or steps >= 50:
                break
        r1 = resource.getrusage(resource.RUSAGE_THREAD)
    finally:
        os.sched_setaffinity(0, set(allowed))
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    cores = max(1, int(round(cpu / el)))
    rec = {"value": P * steps / el, "unit": "grid-pt updates/s", "cores": cores,
           "kind": "oracle",
           "sample": "%d FS step(s) of the 2D 1024x1024, F=5 workload (FP64 NumPy oracle, own "
                     "radix-2 FFT), %.1f s wall, %.1f s CPU, thread pinned to core %d of %d "
                     "allowed (%d on the host)" % (steps, el, cpu, allowed[0], len(allowed),
                                                 os.cpu_count())}
    return rec, u, steps


def traffic_from_profile(kind):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if the
    kernel source is unchanged since they were taken."""
    path = os.path.join(ROOT, "profiles", "fs2d_1024_f32_row_col_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2306_04322_amd.build import fs_kernel_digest
        if rec.get("kernel_digest") != fs_kernel_digest():
            return None
        return rec.get(kind, {}).get("bytes_per_launch")
    except Exception:
        return None


def run_fields(cfg, prec, u0, dt, steps, torch):
    """Fields after `steps` FS steps from u0 on the GPU (one call)."""
    from paper_2306_04322_amd.pfspec import Solver
    s = Solver(cfg, prec)
    s.set_fields(u0)
    s.step_fs(dt, steps)
    u = s.get_fields()
    del s
    torch.cuda.empty_cache()
    return u


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="headline and roofline only")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (the FS step is benchmarked on a single "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2306_04322_amd import inputs as I
    from paper_2306_04322_amd.pfspec import Solver

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    cfg, w = I.workload_config("W2")
    dt = w["dt_fs"]
    # the FP32 run starts from the FP32-rounded state; every comparison below
    # starts from the same values
    u0 = I.workload_ic(cfg, w).astype(np.float32).astype(np.float64)
    P = cfg["n"][0] * cfg["n"][1]
    s32 = Solver(cfg, "f32")
    s32.set_fields(u0)
    # each steady-state pass timed on its own, back to back between two HIP
    # events on the library's stream (pf_time_pass); the passes read and
    # write the workspace only, after untimed steps have filled it (and
    # brought the GPU out of idle).  Run before the headline, so that the
    # headline, like every later measurement, starts on a GPU that has been
    # busy rather than idle.
    s32.step_fs(dt, 100)
    reps = max(50, min(args.steps, 500))
    rates = pass_rates(s32, cfg, "f32", reps)

    log("2D 1024^2 F=5 FP32: warmup", args.warmup, "timed", args.steps)
    s32.set_fields(u0)
    t = time_fs(s32, dt, args.steps, args.warmup, torch)
    value = P * args.steps / t
    ms = 1e3 * t / args.steps
    log("fp32 %.3f ms/step, %.3e pt-upd/s" % (ms, value))
    u32 = s32.get_fields()
    dom = "row" if rates["row"]["avg_launch_us"] >= rates["col"]["avg_launch_us"] else "col"
    oth = "col" if dom == "row" else "row"
    rd = rates[dom]
    roof = {"bound": "hbm", "achieved": rd["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": rd["frac"], "traffic": traffic_from_profile(dom),
            "kernel": ("rowpass_kernel<float,1024,4,X_FWD_DERIV,FE_PAPER> (row pass)" if dom == "row"
                       else "col_kernel<float,1024,COL_UPDATE> (column pass)"),
            "algorithmic_bytes_per_launch": rd["algorithmic_bytes_per_launch"],
            "algorithmic_bytes_rule": ("%d F s per grid point (F = 5 fields, s = 4 bytes): the "
                                       "method's per-stage bytes for the stages this pass performs"
                                       % (4 if dom == "row" else 5)),
            "avg_launch_us": rd["avg_launch_us"],
            "launches_timed": reps,
            "compulsory_bytes_per_launch": rd["compulsory_bytes_per_launch"],
            "compulsory_GBs": rd["compulsory_GBs"],
            "other_kernel": dict(name=oth, **rates[oth]),
            "cache": "the 1024^2 FP32 working set (about 80 MB) fits the 256 MB last-level "
                     "cache, so these rates are partly served from that cache; "
                     "extras.fs_2d_2048_* and fs_2d_4096_* are 2D cases whose working sets "
                     "(about 0.3 and 1.2 GB in FP32) exceed it"}
    cbw = copy_bandwidth(torch, dev)
    roof["copy_GBs"] = round(cbw, 1)
    roof["frac_of_copy"] = round(rd["achieved_GBs"] / cbw, 4)
    log("roofline", roof)
    del s32
    torch.cuda.empty_cache()

    # errors of the timed run: the FP32 fields against the FP64 GPU path over
    # the same steps from the same state
    n_all = args.warmup + args.steps
    u64 = run_fields(cfg, "f64", u0, dt, n_all, torch)
    e32 = rel_l2(u32, u64)
    errors = {"f32_vs_f64_gpu": {"steps": n_all, "rel_l2_per_field": e32, "max": max_err(e32)}}
    log("fp32 vs fp64 GPU after %d steps: %s" % (n_all, e32))
    # the same comparison where all five fields stay non-trivial: the Eq. (4)-(5)
    # state on the same grid (dx = 1), dt = 0.01, 200 steps, both precisions from
    # the FP32-rounded state
    cfgp = I.make_config(2, 1024, 1.0, 4, I.PAPER_FE)
    up = np.asarray(I.paper_ic_2d(cfgp), dtype=np.float32).astype(np.float64)
    ep = rel_l2(run_fields(cfgp, "f32", up, 0.01, 200, torch), run_fields(cfgp, "f64", up, 0.01, 200, torch))
    errors["f32_vs_f64_gpu_eq4_5_state"] = {"steps": 200, "dt": 0.01, "rel_l2_per_field": ep,
                                            "max": max_err(ep)}
    log("fp32 vs fp64 GPU, Eq. (4)-(5) state, 200 steps: %s" % ep)

    out = {"metric": METRIC, "value": value, "unit": "grid-pt updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "FS step, 2D 1024x1024 periodic, dx=1, c + 4 eta (F=5), paper "
                                  "f_chem, seeded uniform IC c=0.5+0.05U(-1,1), eta=0.1U(0,1), dt=0.1",
                      "grid": [1024, 1024], "fields": 5, "dt": dt, "precision": "f32",
                      "dt_note": "the configured dt = 0.5 exceeds the FS linear stability bound "
                                 "of this free energy (dt <= 0.2) and blows up at step 3; dt = 0.1 "
                                 "is used, and the step's cost does not depend on dt"},
           "roofline": roof,
           # whole step against the method's 9 F s bytes per grid point
           "step_roofline_9Fs": {"bytes_per_point": 9 * 5 * 4,
                                 "achieved_GBs": round(value * 9 * 5 * 4 / 1e9, 1),
                                 "frac": round(value * 9 * 5 * 4 / (HBM_PEAK_GBS * 1e9), 4)},
           "errors": errors}

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = {"read": a.numel() * 4, "write": a.numel() * 4}
        del a, b

    if not args.no_extras:
        extras = {}
        # the paper's timing protocol: six repetitions of a batch of steps,
        # mean and minimum time per step (FP32 headline workload)
        sb = Solver(cfg, "f32")
        sb.set_fields(u0)
        sb.step_fs(dt, 50)
        reps_ms = []
        for _ in range(6):
            tb = time_fs(sb, dt, 200, 0, torch)
            reps_ms.append(1e3 * tb / 200)
        extras["fs_2d_1024_f32_6x200"] = {"mean_ms_per_step": sum(reps_ms) / 6,
                                          "median_ms_per_step": float(np.median(reps_ms)),
                                          "min_ms_per_step": min(reps_ms),
                                          "max_ms_per_step": max(reps_ms)}
        del sb
        s64 = Solver(cfg, "f64")
        s64.set_fields(u0)
        n64 = args.steps
        t64 = time_fs(s64, dt, n64, args.warmup, torch)
        v64 = P * n64 / t64
        reps64 = []
        for _ in range(6):
            tb = time_fs(s64, dt, 200, 0, torch)
            reps64.append(1e3 * tb / 200)
        extras["fs_2d_1024_f64"] = {"value": v64, "ms_per_step": 1e3 * t64 / n64,
                                    "fp32_over_fp64": value / v64,
                                    "mean_ms_per_step_6x200": sum(reps64) / 6,
                                    "median_ms_per_step_6x200": float(np.median(reps64)),
                                    "fp32_over_fp64_6x200": (sum(reps64) / 6)
                                    / extras["fs_2d_1024_f32_6x200"]["mean_ms_per_step"],
                                    # the same on the medians of the six batches (one
                                    # disturbed batch moves the means)
                                    "fp32_over_fp64_6x200_median": float(np.median(reps64))
                                    / extras["fs_2d_1024_f32_6x200"]["median_ms_per_step"],
                                    "passes": pass_rates(s64, cfg, "f64", reps)}
        log("fp64 %.3f ms/step; fp32/fp64 = %.2f" % (1e3 * t64 / n64, value / v64))
        del s64
        torch.cuda.empty_cache()
        # 2D cases whose working sets exceed the 256 MB last-level cache:
        # 2048^2 (about 0.3 GB in FP32; the same row and column kernel forms
        # as 1024^2) and 4096^2 (about 1.2 GB; long-row forms)
        for nL, steps in ((2048, (200, 100)), (4096, (100, 50))):
            cfgL = I.make_config(2, nL, 1.0, 4, I.PAPER_FE)
            uL = I.random_ic(cfgL, seed=0).astype(np.float32).astype(np.float64)
            PL = nL * nL
            for prec, nS in zip(("f32", "f64"), steps):
                sL = Solver(cfgL, prec)
                sL.set_fields(uL)
                tL = time_fs(sL, dt, nS, 10, torch)
                rec = {"value": PL * nS / tL, "ms_per_step": 1e3 * tL / nS,
                       "step_frac_9Fs": round(PL * nS / tL * 9 * 5 * (4 if prec == "f32" else 8)
                                              / (HBM_PEAK_GBS * 1e9), 4),
                       "passes": pass_rates(sL, cfgL, prec, 50)}
                extras["fs_2d_%d_%s" % (nL, prec)] = rec
                log("2D %d^2 %s %.3f ms/step" % (nL, prec, rec["ms_per_step"]))
                del sL
                torch.cuda.empty_cache()
            extras["fs_2d_%d_f32_over_f64" % nL] = (extras["fs_2d_%d_f32" % nL]["value"]
                                                    / extras["fs_2d_%d_f64" % nL]["value"])
        # explicit FD on the same grid and state (stable dt of the FD scheme)
        sfd = Solver(cfg, "f32")
        sfd.set_fields(u0)
        sfd.step_fd(w["dt_fd"], 100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sfd.step_fd(w["dt_fd"], 2000)
        torch.cuda.synchronize()
        tfd = (time.perf_counter() - t0) / 2000
        extras["fd_2d_1024_f32"] = {"value": P / tfd, "ms_per_step": 1e3 * tfd,
                                    "fs_over_fd_time_per_step": (t / args.steps) / tfd}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(20):
            sfd.energy("fs")
        extras["energy_2d_1024_f32_ms"] = 1e3 * (time.perf_counter() - t0) / 20
        extras["energy_2d_1024_f32_passes"] = energy_passes(sfd, cfg, "f32")
        del sfd
        torch.cuda.empty_cache()
        # 3D 256^3, c + 4 eta
        cfg3, w3 = I.workload_config("W3")
        u3 = I.workload_ic(cfg3, w3)
        P3 = 256 ** 3
        for prec, n3 in (("f32", 200), ("f64", 100)):
            s3 = Solver(cfg3, prec)
            s3.set_fields(u3)
            t3 = time_fs(s3, w3["dt_fs"], n3, 10, torch)
            extras["fs_3d_256_" + prec] = {
                "value": P3 * n3 / t3, "ms_per_step": 1e3 * t3 / n3,
                "step_frac_9Fs": round(P3 * n3 / t3 * 9 * 5 * (4 if prec == "f32" else 8)
                                       / (HBM_PEAK_GBS * 1e9), 4),
                "passes": passes_3d(s3, prec, w3["dt_fs"])}
            log("3D %s %.3f ms/step" % (prec, 1e3 * t3 / n3))
            if prec == "f32":
                s3.step_fd(w3["dt_fd"], 10)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s3.step_fd(w3["dt_fd"], 100)
                torch.cuda.synchronize()
                tf3 = (time.perf_counter() - t0) / 100
                extras["fd_3d_256_f32"] = {"value": P3 / tf3, "ms_per_step": 1e3 * tf3}
            del s3
            torch.cuda.empty_cache()
        extras["fs_3d_256_f32_over_f64"] = (extras["fs_3d_256_f32"]["value"]
                                            / extras["fs_3d_256_f64"]["value"])
        # adjoint cost: 2D 512^2, c + 2 eta, FP32, K = 50
        cfg4, w4 = I.workload_config("W4")
        u4 = I.workload_ic(cfg4, w4)
        s4 = Solver(cfg4, "f32")
        s4.set_fields(u4)
        K = w4["K"]
        ck = s4.fields.clone()
        tf = time_fs(s4, w4["dt_fs"], K, 10, torch) / K
        seg = s4.segment_store(K)
        lam0 = torch.randn_like(ck)
        lam = lam0.clone()
        s4.adjoint_fs(w4["dt_fs"], K, ck, lam, seg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps_a = 5
        for _ in range(reps_a):
            lam.copy_(lam0)
            s4.adjoint_fs(w4["dt_fs"], K, ck, lam, seg)
        torch.cuda.synchronize()
        ta = (time.perf_counter() - t0) / (reps_a * K)
        extras["adjoint_2d_512_f32"] = {"forward_ms_per_step": 1e3 * tf,
                                        "adjoint_ms_per_step_incl_recompute": 1e3 * ta,
                                        "adjoint_over_forward": ta / tf}
        del s4, seg, lam, ck
        torch.cuda.empty_cache()
        # 3D adjoint: 128^3, c + 4 eta, FP32, segments of K = 100 steps; device
        # memory of a forward-only run against the adjoint's segment store
        cfg5, w5 = I.workload_config("W5")
        u5 = I.workload_ic(cfg5, w5)
        torch.cuda.reset_peak_memory_stats()
        base_mem = torch.cuda.memory_allocated()
        s5 = Solver(cfg5, "f32")
        s5.set_fields(u5)
        K5 = w5["K"]
        tf5 = time_fs(s5, w5["dt_fs"], K5, 10, torch) / K5
        fwd_peak = torch.cuda.max_memory_allocated() - base_mem
        ck5 = s5.fields.clone()
        seg5 = s5.segment_store(K5)
        lam5 = torch.randn_like(ck5)
        s5.adjoint_fs(w5["dt_fs"], K5, ck5, lam5, seg5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s5.adjoint_fs(w5["dt_fs"], K5, ck5, lam5, seg5)
        torch.cuda.synchronize()
        ta5 = (time.perf_counter() - t0) / K5
        adj_peak = torch.cuda.max_memory_allocated() - base_mem
        nseg = w5["steps"] // K5
        field_bytes = ck5.numel() * ck5.element_size()
        extras["adjoint_3d_128_f32"] = {
            "forward_ms_per_step": 1e3 * tf5, "adjoint_ms_per_step_incl_recompute": 1e3 * ta5,
            "adjoint_over_forward": ta5 / tf5,
            "forward_only_device_bytes": int(fwd_peak),
            "one_segment_device_bytes": int(adj_peak),
            "full_run_device_bytes": int(adj_peak + (nseg - 1) * field_bytes),
            "steps": w5["steps"], "K": K5}
        del s5, seg5, lam5, ck5
        torch.cuda.empty_cache()
        extras["paper_reference"] = {
            "hardware": "GeForce RTX 2080 Ti (4352 CUDA cores, 11 GB), CUDA 10.1, FP64, "
                        "PyCUDA + scikit-cuda (cuFFT)",
            "fs_over_fd_time_per_step_per_point": {"2d": "5.2-6.5", "3d": "2.3-4.3"},
            "fs_256sq_dt1e-3_t1_to_100_wall_s": 46,
            "derived_fs_rate_256sq_pt_upd_per_s": 1.41e8,
            "fd_2048sq_wall": "32 days (derived 1.01e9 pt-upd/s)"}
        out["extras"] = extras

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        rec, uo, ko = cpu_baseline(cfg, u0, dt)
        out["cpu_baseline"] = rec
        # errors against the FP64 oracle over the steps it ran (whole fields)
        for prec in ("f64", "f32"):
            e = rel_l2(run_fields(cfg, prec, u0, dt, ko, torch), uo)
            errors[prec + "_gpu_vs_oracle"] = {"steps": ko, "rel_l2_per_field": e, "max": max_err(e)}
            log("%s GPU vs oracle after %d steps: %s" % (prec, ko, e))

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
