"""ctypes binding of libpfspec (include/pfspec.h).

The functions below carry the C names and only marshal arguments; every
step of the method runs in the HIP library.  `Solver` is a convenience
wrapper that lets PyTorch own the device memory (fields, workspace) and
stream.  Importing this module fails loudly when the library has not been
built (``python -m paper_2306_04322_amd.build``): there is no fallback.
"""

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpfspec.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError("libpfspec.so is not built (run: python -m paper_2306_04322_amd.build)")
_lib = ctypes.CDLL(_LIB_PATH)

PF_OK, PF_ERR_INVALID, PF_ERR_UNSUPPORTED, PF_ERR_NOMEM, PF_ERR_HIP, PF_ERR_NONFINITE = range(6)
PF_F32, PF_F64 = 0, 1
PF_FE_POLY, PF_FE_PAPER = 0, 1
PF_K_SPECTRAL, PF_K_FD2, PF_K_FD4 = 0, 1, 2
KMODES = {"spectral": PF_K_SPECTRAL, "fd2": PF_K_FD2, "fd4": PF_K_FD4}
PROF_ROW, PROF_COL, PROF_FD, PROF_RED, PROF_ADJ = range(5)
PF_STATIC_SCRATCH_BYTES = 64 << 20  # include/pfspec.h


class pf_config(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double * 3),
                ("p", ctypes.c_int32), ("prec", ctypes.c_int32), ("fe", ctypes.c_int32),
                ("fe_coef", ctypes.c_double * 12), ("M", ctypes.c_double),
                ("kappa_c", ctypes.c_double), ("L", ctypes.c_double),
                ("kappa_eta", ctypes.c_double), ("kmode", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


_H = ctypes.c_void_p
_P = ctypes.c_void_p
_sig = {
    "pf_create": (ctypes.c_int, [ctypes.POINTER(pf_config), ctypes.POINTER(_H)]),
    "pf_destroy": (None, [_H]),
    "pf_workspace_bytes": (ctypes.c_size_t, [_H]),
    "pf_segment_bytes": (ctypes.c_size_t, [_H, ctypes.c_int64]),
    "pf_bind": (ctypes.c_int, [_H, _P, _P, ctypes.c_size_t]),
    "pf_set_params": (ctypes.c_int, [_H, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double]),
    "pf_set_stream": (ctypes.c_int, [_H, _P]),
    "pf_step_fs": (ctypes.c_int, [_H, ctypes.c_double, ctypes.c_int64]),
    "pf_step_fd": (ctypes.c_int, [_H, ctypes.c_double, ctypes.c_int64]),
    "pf_step_fs_static": (ctypes.c_int, [_H, _P, ctypes.c_double, ctypes.c_int64]),
    "pf_energy": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "pf_adjoint_fs": (ctypes.c_int, [_H, ctypes.c_double, ctypes.c_int64, _P, _P,
                                     ctypes.POINTER(ctypes.c_double), _P]),
    "pf_profile_enable": (ctypes.c_int, [_H, ctypes.c_int32]),
    "pf_profile_read": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double)]),
    "pf_time_pass": (ctypes.c_int, [_H, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double)]),
    "pf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "pf_last_error": (ctypes.c_char_p, []),
    "pf_version": (ctypes.c_int32, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class PFError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = "%s: %s (%s)" % (where, pf_status_string(status), pf_last_error())
        super().__init__(msg)


def _check(st, where):
    if st != PF_OK:
        raise PFError(st, where)


def pf_time_pass(h, pass_id, reps):
    ms = ctypes.c_double()
    _check(_lib.pf_time_pass(h, pass_id, reps, ctypes.byref(ms)), "pf_time_pass")
    return float(ms.value)


def pf_status_string(status):
    return _lib.pf_status_string(status).decode()


def pf_last_error():
    return _lib.pf_last_error().decode()


def pf_version():
    return _lib.pf_version()


def fe_coef_array(fe):
    """Pack a free-energy dict into the fe_coef[12] order of pf_config."""
    if fe["kind"] == "paper":
        vals = [fe["rho2"], fe["c_alpha"], fe["c_beta"], fe["w"], fe["alpha"]]
        kind = PF_FE_PAPER
    elif fe["kind"] == "poly":
        vals = [fe["c_alpha"], fe["c_beta"], fe["c_m"], fe["A"], fe["B"], fe["D"], fe["gamma"],
                fe["delta"], fe["eps"]]
        kind = PF_FE_POLY
    else:
        raise ValueError("unknown free energy %r" % fe["kind"])
    return kind, vals + [0.0] * (12 - len(vals))


def make_config(cfg, precision="f64", stream=None):
    """pf_config from a configuration dict (keys ndim, n, dx, p, fe, M,
    kappa_c, L, kappa_eta, kmode)."""
    c = pf_config()
    c.ndim = cfg["ndim"]
    for d in range(3):
        c.n[d] = int(cfg["n"][d]) if d < cfg["ndim"] else 1
        c.dx[d] = float(cfg["dx"][d]) if d < cfg["ndim"] else 1.0
    c.p = cfg["p"]
    c.prec = PF_F32 if precision == "f32" else PF_F64
    kind, vals = fe_coef_array(cfg["fe"])
    c.fe = kind
    for i, v in enumerate(vals):
        c.fe_coef[i] = float(v)
    c.M, c.kappa_c, c.L, c.kappa_eta = (float(cfg["M"]), float(cfg["kappa_c"]),
                                        float(cfg["L"]), float(cfg["kappa_eta"]))
    c.kmode = KMODES[cfg.get("kmode", "spectral")]
    c.stream = stream
    return c


def pf_create(config):
    h = _H()
    _check(_lib.pf_create(ctypes.byref(config), ctypes.byref(h)), "pf_create")
    return h


def pf_destroy(h):
    _lib.pf_destroy(h)


def pf_workspace_bytes(h):
    return int(_lib.pf_workspace_bytes(h))


def pf_segment_bytes(h, k):
    return int(_lib.pf_segment_bytes(h, k))


def pf_bind(h, fields_ptr, workspace_ptr, workspace_bytes):
    _check(_lib.pf_bind(h, fields_ptr, workspace_ptr, workspace_bytes), "pf_bind")


def pf_set_params(h, M, kappa_c, L, kappa_eta):
    _check(_lib.pf_set_params(h, M, kappa_c, L, kappa_eta), "pf_set_params")


def pf_set_stream(h, stream):
    _check(_lib.pf_set_stream(h, stream), "pf_set_stream")


def pf_step_fs(h, dt, nsteps):
    _check(_lib.pf_step_fs(h, dt, nsteps), "pf_step_fs")


def pf_step_fs_static(h, fields_ptr, dt, nsteps):
    _check(_lib.pf_step_fs_static(h, fields_ptr, dt, nsteps), "pf_step_fs_static")


def pf_step_fd(h, dt, nsteps):
    _check(_lib.pf_step_fd(h, dt, nsteps), "pf_step_fd")


def pf_energy(h, scheme=0):
    out = (ctypes.c_double * 5)()
    _check(_lib.pf_energy(h, scheme, out), "pf_energy")
    return np.array(out[:])


def pf_adjoint_fs(h, dt, k, u_ckpt_ptr, lambda_ptr, seg_store_ptr, dparams=None):
    d = (ctypes.c_double * 4)(*(dparams if dparams is not None else [0.0] * 4))
    _check(_lib.pf_adjoint_fs(h, dt, k, u_ckpt_ptr, lambda_ptr, d, seg_store_ptr), "pf_adjoint_fs")
    return np.array(d[:])


def pf_profile_enable(h, enable=True):
    _check(_lib.pf_profile_enable(h, 1 if enable else 0), "pf_profile_enable")


def pf_profile_read(h, kernel_class):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(_lib.pf_profile_read(h, kernel_class, ctypes.byref(n), ctypes.byref(ms)), "pf_profile_read")
    return int(n.value), float(ms.value)


def field_shape(cfg):
    nd = cfg["ndim"]
    return (1 + cfg["p"],) + tuple(int(cfg["n"][d]) for d in reversed(range(nd)))


class Solver:
    """A bound libpfspec handle whose device buffers are PyTorch tensors.

    fields     torch tensor (F, [Nz,] Ny, Nx) on the device, float32/float64
    workspace  torch uint8 tensor of pf_workspace_bytes
    All work is enqueued on `stream` (default: torch's current stream).
    """

    def __init__(self, cfg, precision="f64", device="cuda", stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.precision = precision
        self.dtype = torch.float32 if precision == "f32" else torch.float64
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = field_shape(cfg)
        # the library's destroy entry, held here so that __del__ still has it
        # while the interpreter tears down module globals at exit
        self._destroy = _lib.pf_destroy
        self.h = pf_create(make_config(cfg, precision, self.stream.cuda_stream))
        self.fields = torch.zeros(self.shape, dtype=self.dtype, device=self.device)
        nb = pf_workspace_bytes(self.h)
        self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
        pf_bind(self.h, self.fields.data_ptr(), self.workspace.data_ptr(), nb)

    def __del__(self):
        h = getattr(self, "h", None)
        destroy = getattr(self, "_destroy", None)
        if h is not None and destroy is not None:
            try:
                self.torch.cuda.synchronize(self.device)
            except Exception:
                pass
            destroy(h)
            self.h = None

    def set_fields(self, u):
        t = self.torch.as_tensor(np.asarray(u) if not self.torch.is_tensor(u) else u)
        self.fields.copy_(t.reshape(self.shape).to(self.dtype))

    def get_fields(self):
        self.torch.cuda.synchronize(self.device)
        return self.fields.detach().to("cpu", self.torch.float64).numpy()

    def set_params(self, M, kappa_c, L, kappa_eta):
        pf_set_params(self.h, M, kappa_c, L, kappa_eta)

    def step_fs(self, dt, nsteps=1):
        pf_step_fs(self.h, dt, nsteps)

    def step_fd(self, dt, nsteps=1):
        pf_step_fd(self.h, dt, nsteps)

    def energy(self, scheme="fs"):
        return pf_energy(self.h, 0 if scheme == "fs" else 1)

    def segment_store(self, k):
        nb = pf_segment_bytes(self.h, k)
        return self.torch.empty(nb // self.fields.element_size(), dtype=self.dtype,
                                device=self.device)

    def adjoint_fs(self, dt, k, u_ckpt, lam, seg_store, dparams=None):
        """lam (device tensor, field layout) holds dJ/du^k on entry and
        dJ/du^0 on return; returns dparams += dJ/d(M, kappa_c, L, kappa_eta)."""
        return pf_adjoint_fs(self.h, dt, k, u_ckpt.data_ptr(), lam.data_ptr(),
                             seg_store.data_ptr(), dparams)
