"""Write the expected values of the full-size FS parity tests.

Runs the FP64 oracle (and nothing else of this repository but the seeded
input module) over the benchmark shapes and stores, for each trajectory,

  * the oracle's final fields on a fixed sample of grid lines (every x point
    of a few (y[, z]) lines, chosen to include both ends of each axis and
    interior lines), and
  * per field, the sum and the sum of squares of the whole final field
    (FP64), so that a test can also check whole-field aggregates;

together with a SHA-256 digest of the oracle sources and the input module,
which a CPU test compares with the current sources so that a stale file is
caught.  Trajectories (Algorithm 1; Eq. (12)-(15), (19)):

  w2     2D 1024^2, c + 4 eta, seeded uniform state, dt = 0.1, 200 steps
  paper  2D 1024^2, c + 4 eta, Eq. (4)-(5) state at dx = 1, dt = 0.01, 200 steps
  w3     3D 256^3,  c + 4 eta, seeded uniform state, dt = 0.1, 2 steps

Every run starts from the FP32-rounded initial state, so one trajectory
serves the FP32 and the FP64 GPU paths.

Usage (from the repository root; about 15 minutes on 8 host cores):
    python tests/golden/make_fullsize_golden.py [w2 paper w3]
"""

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import fs as ofs  # noqa: E402
from paper_2306_04322_amd import inputs as I  # noqa: E402

WORKERS = 5

# (y) lines of the 1024^2 grids and (z, y) lines of the 256^3 grid
ROWS_2D = (0, 1, 517, 1023)
LINES_3D = ((0, 0), (0, 255), (1, 128), (77, 3), (128, 128), (200, 31),
            (254, 200), (255, 255))


def source_digest():
    """SHA-256 over the oracle sources and the input module, in name order."""
    h = hashlib.sha256()
    paths = sorted(os.path.join(ROOT, "oracle", f)
                   for f in os.listdir(os.path.join(ROOT, "oracle")) if f.endswith(".py"))
    paths.append(os.path.join(ROOT, "paper_2306_04322_amd", "inputs.py"))
    for p in paths:
        h.update(os.path.relpath(p, ROOT).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def fp32_rounded(u):
    return np.asarray(u, dtype=np.float32).astype(np.float64)


def trajectory(name):
    """(cfg, dt, steps, initial state) of one stored trajectory."""
    if name == "w2":
        cfg, w = I.workload_config("W2")
        return cfg, w["dt_fs"], 200, fp32_rounded(I.workload_ic(cfg, w))
    if name == "paper":
        cfg = I.make_config(2, 1024, 1.0, 4, I.PAPER_FE)
        return cfg, 0.01, 200, fp32_rounded(I.paper_ic_2d(cfg))
    if name == "w3":
        cfg, w = I.workload_config("W3")
        return cfg, w["dt_fs"], 2, fp32_rounded(I.workload_ic(cfg, w))
    raise KeyError(name)


def sample(u, ndim):
    """The stored lines of the fields u (F, ...): (F, lines, Nx)."""
    if ndim == 2:
        return np.ascontiguousarray(u[:, list(ROWS_2D), :])
    return np.ascontiguousarray(np.stack([u[:, z, y, :] for z, y in LINES_3D], axis=1))


def path_of(name):
    return os.path.join(HERE, "fullsize_%s.npz" % name)


def write(name):
    cfg, dt, steps, u0 = trajectory(name)
    t0 = time.time()
    ref = ofs.fs_run(u0, cfg, dt, steps, workers=WORKERS)
    np.savez(path_of(name),
             digest=np.array(source_digest()),
             dt=np.array(dt), steps=np.array(steps),
             sample=sample(ref, cfg["ndim"]),
             field_sum=ref.reshape(ref.shape[0], -1).sum(axis=1),
             field_sumsq=(ref.reshape(ref.shape[0], -1) ** 2).sum(axis=1))
    print("%s: %d oracle steps in %.0f s -> %s" % (name, steps, time.time() - t0, path_of(name)),
          flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["w2", "paper", "w3"]):
        write(nm)
