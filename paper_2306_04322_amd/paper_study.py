"""The paper's 2D accuracy/efficiency study on one MI355X, with this
library's kernels.

    python -m paper_2306_04322_amd.paper_study [--quick] [--out FILE]

Sec. 2.1: the Ostwald-ripening benchmark on a 200 x 200 periodic box,
f_chem with p = 4, initial fields Eq. (4), (5).  Those fields are not
periodic, so the paper first evolves them with finite differences on a fine
grid from t = 0 to t = 1 and uses the t = 1 fields as the initial condition
of every case.  Sec. 3.3 measures the error Eq. (22),
E_phi = sum (phi_0 - phi)^2 / sum phi_0^2, at t = 100 against an FS run on
the finest grid with the smallest time step, comparing c and
eta = sum_i eta_i.

This module reproduces that protocol with its own reference (the paper's
fields are not available):
  1. periodisation: FD (pf_step_fd) on an n_per x n_per grid (the finest
     grid, at most 1024^2), t = 0 -> 1;
  2. coarser grids take those fields at every k-th point; finer grids get
     their band-limited (Fourier) interpolation, an input-preparation step
     done once on the host;
  3. FS runs (pf_step_fs) t = 1 -> t_end for each grid and time step, FD
     runs where affordable, timed with device synchronisation;
  4. E_c, E_eta of each run against the finest/smallest-dt FS run, on the
     coarser run's grid points.
The full protocol (n up to 2048, t_end = 100, dt = 1e-4) takes several
minutes of GPU time; --quick shrinks it to seconds.
"""

import argparse
import json
import sys
import time

import numpy as np

from . import inputs as I

DOMAIN = 200.0


def paper_config(n, kmode="spectral"):
    """Sec. 2.1 benchmark on an n x n grid of the 200 x 200 box."""
    return I.make_config(2, n, DOMAIN / n, 4, I.PAPER_FE, kmode)


def fd_stable_dt(n, safety=0.7):
    """Linear FD bound for f_chem at eta = 0 (f_cc = 2 rho2, f_ee = 2 w), times
    `safety` (Table 1's steps are 0.72-0.79 of it)."""
    dx = DOMAIN / n
    q = 8.0 / dx ** 2
    M, kc, L, ke = 5.0, 3.0, 5.0, 3.0
    ch = 2.0 / (M * q * (4.0 + kc * q))
    ac = 2.0 / (L * (2.0 + ke * q))
    return safety * min(ch, ac)


def resample(u, n):
    """Fields on an n x n grid from fields on an m x m grid of the same box:
    every (m/n)-th point when coarser, Fourier zero-padding when finer."""
    m = u.shape[-1]
    if n <= m:
        k = m // n
        return np.ascontiguousarray(u[:, ::k, ::k])
    U = np.fft.fft2(u, axes=(-2, -1))
    out = np.zeros(u.shape[:-2] + (n, n), dtype=complex)
    h = m // 2
    out[..., :h, :h] = U[..., :h, :h]
    out[..., :h, -h:] = U[..., :h, -h:]
    out[..., -h:, :h] = U[..., -h:, :h]
    out[..., -h:, -h:] = U[..., -h:, -h:]
    return np.ascontiguousarray(np.real(np.fft.ifft2(out, axes=(-2, -1))) * (n * n) / (m * m))


def e_phi(ref, got):
    """Eq. (22): sum (phi_0 - phi)^2 / sum phi_0^2."""
    return float(np.sum((ref - got) ** 2) / np.sum(ref ** 2))


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def run(grids, dts, t0, t_end, fd_grids, prec="f64", n_per=1024, log=_log):
    import torch
    from .pfspec import Solver

    nfine = max(grids)
    n_per = min(n_per, nfine)
    cfg_f = paper_config(n_per)
    u_ic = I.paper_ic_2d(cfg_f)
    # 1. periodisation by FD, t = 0 -> t0
    s = Solver(cfg_f, prec)
    s.set_fields(u_ic)
    dtp = fd_stable_dt(n_per)
    nper = int(np.ceil(t0 / dtp))
    dtp = t0 / nper
    log("periodisation: FD %d^2, %d steps of %.3e" % (n_per, nper, dtp))
    torch.cuda.synchronize()
    t = time.perf_counter()
    s.step_fd(dtp, nper)
    torch.cuda.synchronize()
    tper = time.perf_counter() - t
    u1 = s.get_fields()
    del s
    results = {"periodisation": {"grid": n_per, "dt": dtp, "steps": nper, "wall_s": tper},
               "runs": []}

    def evolve(n, dt, scheme):
        u = resample(u1, n)
        cfg = paper_config(n)
        sv = Solver(cfg, prec)
        sv.set_fields(u)
        nsteps = int(round((t_end - t0) / dt))
        torch.cuda.synchronize()
        t = time.perf_counter()
        done, last = 0, t
        chunk = 20000
        while done < nsteps:
            k = min(chunk, nsteps - done)
            if scheme == "fs":
                sv.step_fs(dt, k)
            else:
                sv.step_fd(dt, k)
            done += k
            if time.perf_counter() - last > 30.0:
                torch.cuda.synchronize()
                last = time.perf_counter()
                log("  %s %d^2: %d / %d steps" % (scheme, n, done, nsteps))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        out = sv.get_fields()
        E = sv.energy(scheme)
        del sv
        return out, wall, nsteps, E

    ref_dt = min(dts)
    ref, wall, nst, E = evolve(nfine, ref_dt, "fs")
    log("reference FS %d^2 dt=%g: %d steps, %.1f s" % (nfine, ref_dt, nst, wall))
    results["reference"] = {"grid": nfine, "dt": ref_dt, "steps": nst, "wall_s": wall,
                            "energy": E.tolist()}
    cases = [(n, dt, "fs") for n in sorted(grids) for dt in sorted(dts)
             if not (n == nfine and dt == ref_dt)]
    cases += [(n, fd_stable_dt(n), "fd") for n in sorted(fd_grids)]
    for n, dt, scheme in cases:
        out, wall, nst, E = evolve(n, dt, scheme)
        k = nfine // n
        r = ref[:, ::k, ::k]
        ec = e_phi(r[0], out[0])
        ee = e_phi(np.sum(r[1:], axis=0), np.sum(out[1:], axis=0))
        rec = {"scheme": scheme, "grid": n, "dt": dt, "steps": nst, "wall_s": wall,
               "s_per_step_per_point": wall / nst / n ** 2, "E_c_percent": 100 * ec,
               "E_eta_percent": 100 * ee, "energy": E.tolist()}
        results["runs"].append(rec)
        log("%s %4d^2 dt=%.3e steps=%8d wall=%7.2fs E_c=%.3e%% E_eta=%.3e%%"
            % (scheme, n, dt, nst, wall, 100 * ec, 100 * ee))
    return results


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small grids and short times")
    ap.add_argument("--out", default=None)
    ap.add_argument("--prec", default="f64")
    args = ap.parse_args(argv)
    if args.quick:
        res = run([64, 128, 256], [1e-3, 5e-3], 1.0, 3.0, [64, 128], args.prec)
    else:
        res = run([128, 256, 512, 1024, 2048], [1e-4, 1e-3, 5e-3], 1.0, 100.0, [128, 256],
                  args.prec)
    txt = json.dumps(res, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(txt)
    else:
        print(txt)
    return 0


if __name__ == "__main__":
    sys.exit(main())
