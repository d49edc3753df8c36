"""Host-only checks of the C-ABI library (no GPU, no compute calls).

The library must load, export every entry point include/pfspec.h declares,
and reject malformed configurations in pf_create before any HIP call."""

import os
import re

import pytest

from paper_2306_04322_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "pfspec.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2306_04322_amd import pfspec as P
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(P._lib, n), n
        assert n in P.EXPORTED, n
    assert P.pf_version() >= 100


def test_status_strings():
    from paper_2306_04322_amd import pfspec as P
    assert P.pf_status_string(P.PF_OK) == "PF_OK"
    assert P.pf_status_string(P.PF_ERR_NONFINITE) == "PF_ERR_NONFINITE"


def test_struct_layout_matches_header():
    import ctypes
    from paper_2306_04322_amd import pfspec as P
    # int32 ndim, n[3]; double dx[3]; int32 p, prec, fe; double fe_coef[12];
    # double M, kappa_c, L, kappa_eta; int32 kmode; void* stream
    assert P.pf_config.dx.offset == 16
    assert P.pf_config.fe_coef.offset == 56
    assert P.pf_config.M.offset == 56 + 96
    assert P.pf_config.kmode.offset == 56 + 96 + 32
    assert P.pf_config.stream.offset == 56 + 96 + 32 + 8
    assert ctypes.sizeof(P.pf_config) == 56 + 96 + 32 + 16


@pytest.mark.parametrize("mut,msg", [
    (dict(ndim=4), "ndim"),
    (dict(n=(48, 64, 1)), "powers of two"),
    (dict(n=(4, 64, 1)), "powers of two"),
    (dict(n=(8192, 64, 1)), "powers of two"),
    (dict(p=0), "p must"),
    (dict(p=9), "p must"),
    (dict(dx=(0.0, 1.0, 1.0)), "dx"),
    (dict(dx=(float("nan"), 1.0, 1.0)), "dx"),
    (dict(M=-1.0), "M, kappa_c"),
    (dict(kappa_eta=0.0), "M, kappa_c"),
])
def test_create_rejects_bad_config(mut, msg):
    from paper_2306_04322_amd import pfspec as P
    cfg = I.make_config(2, 64, 1.0, 2, I.PAPER_FE)
    cfg.update(mut)
    if "n" in mut and cfg["ndim"] == 2:
        pass
    c = P.make_config(cfg) if mut.get("ndim", 2) in (2, 3) else None
    if c is None:
        c = P.make_config(I.make_config(2, 64, 1.0, 2, I.PAPER_FE))
        c.ndim = mut["ndim"]
    with pytest.raises(P.PFError) as ei:
        P.pf_create(c)
    assert ei.value.status == P.PF_ERR_INVALID
    assert msg in str(ei.value)


def test_create_rejects_3d_too_large_and_bad_enums():
    from paper_2306_04322_amd import pfspec as P
    c = P.make_config(I.make_config(3, (2048, 8, 8), 1.0, 2, I.PAPER_FE))
    with pytest.raises(P.PFError):
        P.pf_create(c)
    for field, val in (("prec", 7), ("fe", 5), ("kmode", 9)):
        c = P.make_config(I.make_config(2, 64, 1.0, 2, I.PAPER_FE))
        setattr(c, field, val)
        with pytest.raises(P.PFError) as ei:
            P.pf_create(c)
        assert ei.value.status == P.PF_ERR_INVALID


@pytest.mark.parametrize("prec,es", [("f32", 4), ("f64", 8)])
def test_workspace_and_segment_sizes(prec, es):
    from paper_2306_04322_amd import pfspec as P
    cfg = I.make_config(3, (32, 16, 8), 1.0, 4, I.PAPER_FE)
    h = P.pf_create(P.make_config(cfg, prec))
    try:
        ws = P.pf_workspace_bytes(h)
        F, Pn = 5, 32 * 16 * 8
        # two x-spectrum sets of F + 1 fields at least
        assert ws >= 2 * (F + 1) * 16 * 8 * 17 * 2 * es
        assert ws % 256 == 0
        assert P.pf_segment_bytes(h, 7) == 7 * F * Pn * es
        # calls that need a bound handle fail before touching the GPU
        for fn, args in ((P.pf_step_fs, (0.1, 1)), (P.pf_step_fd, (0.1, 1))):
            with pytest.raises(P.PFError) as ei:
                fn(h, *args)
            assert ei.value.status == P.PF_ERR_INVALID
        with pytest.raises(P.PFError):
            P.pf_energy(h, 0)
        with pytest.raises(P.PFError):
            P.pf_set_params(h, 1.0, -1.0, 1.0, 1.0)
        for pass_id, reps in ((0, 10), (1, 10), (2, 10), (0, 0)):
            with pytest.raises(P.PFError) as ei:
                P.pf_time_pass(h, pass_id, reps)
            assert ei.value.status == P.PF_ERR_INVALID
    finally:
        P.pf_destroy(h)


def test_static_step_rejects_before_any_hip_call():
    """pf_step_fs_static checks its arguments and the workspace size against
    the static array before touching the GPU (the pointer is never used)."""
    from paper_2306_04322_amd import pfspec as P
    big = I.make_config(2, 2048, 1.0, 4, I.PAPER_FE)
    h = P.pf_create(P.make_config(big, "f64"))
    try:
        assert P.pf_workspace_bytes(h) > P.PF_STATIC_SCRATCH_BYTES
        with pytest.raises(P.PFError) as ei:
            P.pf_step_fs_static(h, 256, 0.1, 1)
        assert ei.value.status == P.PF_ERR_NOMEM
        for args in ((0, 0.1, 1), (128, 0.1, 1), (256, 0.0, 1), (256, 0.1, -1)):
            with pytest.raises(P.PFError) as ei:
                P.pf_step_fs_static(h, *args)
            assert ei.value.status == P.PF_ERR_INVALID
    finally:
        P.pf_destroy(h)
