"""GPU parity at the benchmark shapes over the acceptance horizon.

Acceptance (relative L2 error per field after 200 steps): <= 1e-10 for the
FP64 GPU path and <= 1e-4 for the FP32 path.  Both precisions start from the
FP32-rounded initial state, so one oracle trajectory serves both and the
error measures arithmetic only.  The GPU runs are split into a 5-step and a
195-step call, as the benchmark's warm-up and timed calls are; the kernels
are the ones the benchmark launches (same instantiations and launch shapes).

Fields whose reference norm falls below the floor of `parity_util.rel_l2`
are reported and not compared: on the seeded uniform initial state of the
throughput workload the order parameters vanish within a few steps at
dt = 0.1 (dt L d2f/deta2 = 1 at eta = 0), in the oracle and on the GPU alike.
The 1024^2 run of the Eq. (4)-(5) state keeps all five fields non-trivial.

The oracle runs its field transforms on several threads here (bit-identical
to the serial oracle); its 1024^2 trajectories take a few minutes of host
time."""

import numpy as np
import pytest

from oracle import fs as ofs
from paper_2306_04322_amd import inputs as I
from parity_util import announce, fp32_rounded, gpu_or_fail, max_rel, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}
WORKERS = 5


def _gpu_run(cfg, u0, prec, dt, chunks):
    gpu_or_fail()
    from paper_2306_04322_amd.pfspec import Solver
    s = Solver(cfg, prec)
    s.set_fields(u0)
    for k in chunks:
        s.step_fs(dt, k)
    return s


def _report(name, prec, got, ref):
    errs = rel_l2(got, ref)
    # the deviation of c from its mean, which carries the dynamics (the mean
    # itself is held exactly)
    dc = got[0] - np.mean(got[0])
    dr = ref[0] - np.mean(ref[0])
    fl = float(np.linalg.norm(dc - dr) / np.linalg.norm(dr))
    print("%s %s rel-L2 per field %s; c - mean(c): %.3e" % (name, prec, errs, fl))
    return errs, fl


@pytest.fixture(scope="module")
def w2_trajectory():
    """Throughput workload, 2D 1024^2, c + 4 eta: 200 oracle steps."""
    cfg, w = I.workload_config("W2")
    u0 = fp32_rounded(I.workload_ic(cfg, w))
    return cfg, w, u0, ofs.fs_run(u0, cfg, w["dt_fs"], 200, workers=WORKERS)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_w2_1024_200_steps(w2_trajectory, prec):
    cfg, w, u0, ref = w2_trajectory
    announce("fs full 1024^2 W2 200 steps", prec)
    got = _gpu_run(cfg, u0, prec, w["dt_fs"], (5, 195)).get_fields()
    errs, fl = _report("W2", prec, got, ref)
    assert errs[0] is not None
    assert max_rel(errs) <= TOL[prec]
    assert fl <= (1e-8 if prec == "f64" else 1e-3)


@pytest.fixture(scope="module")
def paper_ic_trajectory():
    """2D 1024^2, c + 4 eta, Eq. (4)-(5) initial fields at x_j = j (dx = 1),
    dt = 0.01: 200 oracle steps."""
    cfg = I.make_config(2, 1024, 1.0, 4, I.PAPER_FE)
    u0 = fp32_rounded(I.paper_ic_2d(cfg))
    return cfg, u0, ofs.fs_run(u0, cfg, 0.01, 200, workers=WORKERS)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_paper_ic_1024_200_steps(paper_ic_trajectory, prec):
    cfg, u0, ref = paper_ic_trajectory
    announce("fs full 1024^2 paper IC 200 steps", prec)
    got = _gpu_run(cfg, u0, prec, 0.01, (5, 195)).get_fields()
    errs, fl = _report("paper IC 1024^2", prec, got, ref)
    assert all(e is not None for e in errs)
    assert max_rel(errs) <= TOL[prec]


@pytest.fixture(scope="module")
def w3_trajectory():
    """3D throughput workload, 256^3, c + 4 eta, seeded uniform state: two
    oracle steps (every point)."""
    cfg, w = I.workload_config("W3")
    u0 = fp32_rounded(I.workload_ic(cfg, w))
    return cfg, w, u0, ofs.fs_run(u0, cfg, w["dt_fs"], 2, workers=WORKERS)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_w3_256_random_ic(w3_trajectory, prec):
    cfg, w, u0, ref = w3_trajectory
    announce("fs full 256^3 W3 2 steps", prec)
    s = _gpu_run(cfg, u0, prec, w["dt_fs"], (2,))
    got = s.get_fields()
    del s
    errs, fl = _report("W3", prec, got, ref)
    assert all(e is not None for e in errs)
    assert max_rel(errs) <= TOL[prec]
