"""The degenerate case of the method: a spatially uniform state.

Every spatial term vanishes on a uniform state:
- its spectrum is the k = 0 mode alone, where |xi|^2 = 0 (Eq. (16));
- its 5-/7-point Laplacian is zero.
So the FS step (Eq. (14), (15)) and the FD step (Sec. 2.2) reduce to the
same pointwise recurrence. c keeps its value: the k = 0 mode of c is held,
and the FD update adds dt M Lap_h(mu) = 0. Each eta_i follows explicit Euler
on the local equation, eta <- eta - dt L df/deta (Eq. (3) without the
gradient term). The fields must stay uniform.

The expected values come from the oracle's pointwise derivative in FP64,
iterated on one point. The test also compares the FS and FD kernels with
each other, and checks the energy: both gradient parts vanish (to rounding),
and the chemical part and the mass are dV P f(u) and dV P c."""

import numpy as np
import pytest

from oracle import freeenergy as ofe
from paper_2306_04322_amd import inputs as I
from parity_util import DISTINCT, announce, gpu_or_fail

pytestmark = pytest.mark.gpu

U0 = (0.45, 0.3, 0.1, 0.6, 0.05)  # c, eta_1..eta_4
DT, STEPS = 0.01, 20  # dt L max|f_etaeta| stays well below 2


def _expected(u0, cfg):
    u = np.array(u0, dtype=np.float64).reshape(-1, 1)
    for _ in range(STEPS):
        g = ofe.gradient(u, cfg["fe"])
        u[1:] = u[1:] - DT * cfg["L"] * g[1:]
    return u[:, 0]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ndim,n", [(2, (64, 32)), (3, (16, 8, 32)), (2, (1024, 1024)),
                                    (3, (256, 256, 256))])
def test_uniform_state_fs_fd(ndim, n, prec):
    torch = gpu_or_fail()
    from paper_2306_04322_amd.pfspec import Solver
    cfg = I.make_config(ndim, n, 1.0, 4, I.PAPER_FE, **DISTINCT)
    u0 = np.array(U0, dtype=np.float32 if prec == "f32" else np.float64).astype(np.float64)
    exp = _expected(u0, cfg)
    shape = (5,) + tuple(reversed(n))
    s = Solver(cfg, prec)
    dev = s.device
    ufield = torch.as_tensor(u0, device=dev).reshape((5,) + (1,) * ndim).expand(shape)
    eps = 1e-13 if prec == "f64" else 1e-5
    ulp = 4 * (np.finfo(np.float64).eps if prec == "f64" else np.finfo(np.float32).eps)

    def check(name):
        f = s.fields.double()
        for k in range(5):
            lo, hi = float(f[k].min()), float(f[k].max())
            assert hi - lo <= ulp * abs(exp[k]), (name, k, lo, hi)
            assert abs(hi - exp[k]) <= eps * abs(exp[k]), (name, k, hi, exp[k])
        # c is the held mean: a double sum of P equal values, exact for FP32
        # values, rounded for FP64 ones
        assert float(f[0].min()) == pytest.approx(u0[0], rel=1e-14 if prec == "f64" else ulp, abs=0.0)
        return f[(slice(None),) + (0,) * ndim].cpu().numpy()

    announce("uniform state FS", ndim, n, prec)
    s.set_fields(ufield)
    s.step_fs(DT, STEPS)
    torch.cuda.synchronize()
    fs = check("fs")

    announce("uniform state FD", ndim, n, prec)
    s.set_fields(ufield)
    s.step_fd(DT, STEPS)
    torch.cuda.synchronize()
    fd = check("fd")
    # the two kernels round differently; rounding of the early steps, at the
    # scale of the initial values, persists while the order parameters decay
    np.testing.assert_allclose(fs, fd, rtol=ulp * STEPS, atol=ulp * STEPS * float(np.max(np.abs(u0))))

    announce("uniform state energy", ndim, n, prec)
    s.set_fields(ufield)
    P = int(np.prod(n))
    chem = P * float(ofe.density(u0.reshape(-1, 1), cfg["fe"])[0])
    for sch in ("fs", "fd"):
        e = s.energy(sch)
        assert abs(e[2]) + abs(e[3]) <= 1e-10 * abs(e[1]), (sch, e)
        # (the FP32 path holds the free-energy coefficients in FP32)
        assert e[1] == pytest.approx(chem, rel=1e-6 if prec == "f32" else 1e-12), (sch, e)
        assert e[4] == pytest.approx(P * u0[0], rel=1e-12), (sch, e)
    del s
    torch.cuda.empty_cache()
