"""Work enqueued on a caller's stream (pf_set_stream): FS steps, FD steps
and the energy on a second stream of default priority give bit for bit the
results of the same calls on the stream the handle was created with."""

import numpy as np
import pytest

from paper_2306_04322_amd import inputs as I
from parity_util import DISTINCT, announce, gpu_or_fail

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_side_stream_matches_creation_stream(prec):
    torch = gpu_or_fail()
    from paper_2306_04322_amd import pfspec as P
    from paper_2306_04322_amd.pfspec import Solver
    cfg = I.make_config(2, (256, 128), (1.0, 0.8), 3, I.PAPER_FE, **DISTINCT)
    u0 = I.random_ic(cfg, seed=4)
    announce("side stream", prec)

    ref = Solver(cfg, prec)
    ref.set_fields(u0)
    ref.step_fs(0.05, 30)
    e_ref = ref.energy("fs")
    ref.step_fd(0.001, 20)
    e_fd_ref = ref.energy("fd")
    u_ref = ref.get_fields()

    s = Solver(cfg, prec)
    s.set_fields(u0)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()  # default priority
    P.pf_set_stream(s.h, side.cuda_stream)
    s.step_fs(0.05, 30)
    e = s.energy("fs")  # synchronises the side stream
    s.step_fd(0.001, 20)
    e_fd = s.energy("fd")
    side.synchronize()
    u = s.get_fields()

    assert np.array_equal(u, u_ref)
    assert np.array_equal(e, e_ref) and np.array_equal(e_fd, e_fd_ref)
