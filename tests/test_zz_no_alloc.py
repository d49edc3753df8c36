"""pf_step_fs_static, the FS step whose workspace is the library's static
device array (for callers that cannot allocate), against pf_step_fs with a
caller workspace: same kernels, same launch shapes, so the fields must agree
bit for bit.  Two calls in a row on the one array, the second on a smaller
grid (and the other precision), then the first configuration again."""

import numpy as np
import pytest

from paper_2306_04322_amd import inputs as I
from parity_util import announce, gpu_or_fail

pytestmark = pytest.mark.gpu


def _pair(cfg, prec, u0, dt, steps):
    """(fields after pf_step_fs, fields after pf_step_fs_static), both from
    u0, on one handle."""
    torch = gpu_or_fail()
    from paper_2306_04322_amd import pfspec as P
    s = P.Solver(cfg, prec)
    s.set_fields(u0)
    other = s.fields.clone()
    s.step_fs(dt, steps)
    announce("pf_step_fs_static", cfg["n"][:cfg["ndim"]], "p", cfg["p"], prec, steps, "steps")
    P.pf_step_fs_static(s.h, other.data_ptr(), dt, steps)
    torch.cuda.synchronize()
    ref = s.fields.detach().cpu().numpy()
    got = other.detach().cpu().numpy()
    del s
    return ref, got


def test_static_matches_bound_workspace_two_calls():
    # first call: 2D 512^2, c + 4 eta, FP32 (a workspace of about 15 MB)
    cfg1, w1 = I.workload_config("W2", n=512)
    u1 = I.workload_ic(cfg1, w1)
    ref, got = _pair(cfg1, "f32", u1, w1["dt_fs"], 12)
    assert np.array_equal(ref, got)
    # second call, smaller: 3D 32^3, c + 2 eta, FP64, distinct kinetics
    cfg2 = I.make_config(3, 32, 1.0, 2, I.PAPER_FE, M=5.0, kappa_c=3.0, L=4.0, kappa_eta=2.0)
    u2 = I.random_ic(cfg2, seed=3)
    ref, got = _pair(cfg2, "f64", u2, 0.05, 7)
    assert np.array_equal(ref, got)
    # and the first configuration once more on what the second left behind
    ref, got = _pair(cfg1, "f32", u1, w1["dt_fs"], 3)
    assert np.array_equal(ref, got)


def test_static_rejects_oversize_workspace():
    gpu_or_fail()
    from paper_2306_04322_amd import pfspec as P
    cfg = I.make_config(2, 2048, 1.0, 4, I.PAPER_FE)
    h = P.pf_create(P.make_config(cfg, "f64"))
    try:
        assert P.pf_workspace_bytes(h) > P.PF_STATIC_SCRATCH_BYTES
        with pytest.raises(P.PFError) as ei:
            P.pf_step_fs_static(h, 256, 0.1, 1)
        assert ei.value.status == P.PF_ERR_NOMEM
    finally:
        P.pf_destroy(h)
