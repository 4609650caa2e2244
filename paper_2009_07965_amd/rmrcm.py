"""Python binding of the C ABI in include/rmrcm.h.

Argument marshalling only: every step of the method runs in the HIP
library.  Functions keep the C names; ``Solver`` is a small convenience
class over them.  Arrays may be NumPy arrays (host) or torch tensors on the
GPU (device pointers are passed straight through, so inputs already in HBM
are not copied through the host).

If the shared library is missing the import fails loudly: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmrcm.so")

RMRCM_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESINGULAR",
          -5: "ENOTCONV", -6: "ESTATE", -7: "ENOTSUP", -8: "ETOOBIG"}
RMRCM_FP64, RMRCM_MIXED, RMRCM_MIXED_LEARNED = 0, 1, 2
RMRCM_BC_NEUMANN, RMRCM_BC_DIRICHLET = 0, 1


class rmrcm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double),
        ("sub_nx", ctypes.c_int32), ("sub_ny", ctypes.c_int32),
        ("seg", ctypes.c_int32),
        ("alpha", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("ir_tol", ctypes.c_double),
        ("ir_max_iter", ctypes.c_int32),
        ("gate_tol", ctypes.c_double),
        ("cnn_weights", ctypes.c_char_p),
        ("device", ctypes.c_int32),
        ("mem_cap", ctypes.c_uint64),
        ("seg_u", ctypes.c_int32), ("seg_p", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("lz", ctypes.c_double),
    ]


EXPORTS = [
    "rmrcm_default_params", "rmrcm_plan_bytes", "rmrcm_set_refinement", "rmrcm_downscale", "rmrcm_setup", "rmrcm_refactor", "rmrcm_sync", "rmrcm_solve", "rmrcm_step",
    "rmrcm_set_step_graph", "rmrcm_step_noalloc",
    "rmrcm_get_interface",
    "rmrcm_counts", "rmrcm_set_stream", "rmrcm_get_stats", "rmrcm_destroy",
    "rmrcm_strerror", "rmrcm_autotune", "rmrcm_batch_create", "rmrcm_batch_refactor",
    "rmrcm_batch_solve", "rmrcm_batch_sync", "rmrcm_batch_get_stats", "rmrcm_batch_destroy",
    "rmrcm_export_local", "rmrcm_get_gate", "rmrcm_cnn_create", "rmrcm_cnn_num_params", "rmrcm_cnn_set_stream",
    "rmrcm_cnn_set_params", "rmrcm_cnn_get_params", "rmrcm_cnn_forward", "rmrcm_cnn_loss_grad",
    "rmrcm_cnn_train_step", "rmrcm_cnn_save", "rmrcm_cnn_load", "rmrcm_cnn_destroy",
]


class RMRCMError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, STATUS.get(status, "?"), status))


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError("librmrcm.so not built (run paper_2009_07965_amd.build)")
    lib = ctypes.CDLL(path)
    vp, dp, i8p = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
    lib.rmrcm_default_params.argtypes = [ctypes.POINTER(rmrcm_params)]
    lib.rmrcm_default_params.restype = None
    lib.rmrcm_plan_bytes.argtypes = [ctypes.POINTER(rmrcm_params), ctypes.POINTER(ctypes.c_uint64)]
    lib.rmrcm_plan_bytes.restype = ctypes.c_int
    lib.rmrcm_downscale.argtypes = [vp, dp, dp, dp, dp, dp, dp]
    lib.rmrcm_downscale.restype = ctypes.c_int
    lib.rmrcm_set_refinement.argtypes = [vp, ctypes.c_double, ctypes.c_int32]
    lib.rmrcm_set_refinement.restype = ctypes.c_int
    lib.rmrcm_setup.argtypes = [ctypes.POINTER(rmrcm_params), dp, i8p, ctypes.POINTER(vp)]
    lib.rmrcm_setup.restype = ctypes.c_int
    lib.rmrcm_refactor.argtypes = [vp, dp]
    lib.rmrcm_refactor.restype = ctypes.c_int
    lib.rmrcm_sync.argtypes = [vp]
    lib.rmrcm_sync.restype = ctypes.c_int
    lib.rmrcm_solve.argtypes = [vp, dp, dp, dp, dp]
    lib.rmrcm_solve.restype = ctypes.c_int
    lib.rmrcm_step.argtypes = [vp, dp, dp, dp, dp, dp]
    lib.rmrcm_step.restype = ctypes.c_int
    lib.rmrcm_step_noalloc.argtypes = [ctypes.POINTER(rmrcm_params), dp, i8p, dp, dp, dp, dp, vp]
    lib.rmrcm_step_noalloc.restype = ctypes.c_int
    lib.rmrcm_set_step_graph.argtypes = [vp, ctypes.c_int]
    lib.rmrcm_set_step_graph.restype = ctypes.c_int
    lib.rmrcm_get_interface.argtypes = [vp, dp, dp]
    lib.rmrcm_get_interface.restype = ctypes.c_int
    lib.rmrcm_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.rmrcm_counts.restype = ctypes.c_int
    lib.rmrcm_set_stream.argtypes = [vp, vp]
    lib.rmrcm_set_stream.restype = ctypes.c_int
    lib.rmrcm_get_stats.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.rmrcm_get_stats.restype = ctypes.c_int
    lib.rmrcm_destroy.argtypes = [vp]
    lib.rmrcm_destroy.restype = None
    lib.rmrcm_strerror.argtypes = [ctypes.c_int]
    lib.rmrcm_strerror.restype = ctypes.c_char_p
    lib.rmrcm_autotune.argtypes = [vp]
    lib.rmrcm_autotune.restype = ctypes.c_int
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.rmrcm_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(rmrcm_params), pp, pp,
                                       ctypes.c_int32, ctypes.POINTER(vp)]
    lib.rmrcm_batch_create.restype = ctypes.c_int
    lib.rmrcm_batch_refactor.argtypes = [vp, pp]
    lib.rmrcm_batch_refactor.restype = ctypes.c_int
    lib.rmrcm_batch_solve.argtypes = [vp, pp, pp, pp, pp]
    lib.rmrcm_batch_solve.restype = ctypes.c_int
    lib.rmrcm_batch_sync.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.rmrcm_batch_sync.restype = ctypes.c_int
    lib.rmrcm_batch_get_stats.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.rmrcm_batch_get_stats.restype = ctypes.c_int
    lib.rmrcm_batch_destroy.argtypes = [vp]
    lib.rmrcm_batch_destroy.restype = None
    lib.rmrcm_export_local.argtypes = [vp, vp, vp, vp]
    lib.rmrcm_export_local.restype = ctypes.c_int
    lib.rmrcm_get_gate.argtypes = [vp, vp, vp]
    lib.rmrcm_get_gate.restype = ctypes.c_int
    i32 = ctypes.c_int32
    lib.rmrcm_cnn_create.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.POINTER(vp)]
    lib.rmrcm_cnn_create.restype = ctypes.c_int
    lib.rmrcm_cnn_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.rmrcm_cnn_num_params.restype = ctypes.c_int
    lib.rmrcm_cnn_set_stream.argtypes = [vp, vp]
    lib.rmrcm_cnn_set_stream.restype = ctypes.c_int
    lib.rmrcm_cnn_set_params.argtypes = [vp, vp]
    lib.rmrcm_cnn_set_params.restype = ctypes.c_int
    lib.rmrcm_cnn_get_params.argtypes = [vp, vp]
    lib.rmrcm_cnn_get_params.restype = ctypes.c_int
    lib.rmrcm_cnn_forward.argtypes = [vp, i32, vp, vp]
    lib.rmrcm_cnn_forward.restype = ctypes.c_int
    lib.rmrcm_cnn_loss_grad.argtypes = [vp, i32, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.rmrcm_cnn_loss_grad.restype = ctypes.c_int
    lib.rmrcm_cnn_train_step.argtypes = [vp, i32, vp, vp, ctypes.c_float,
                                         ctypes.POINTER(ctypes.c_double)]
    lib.rmrcm_cnn_train_step.restype = ctypes.c_int
    lib.rmrcm_cnn_save.argtypes = [vp, ctypes.c_char_p]
    lib.rmrcm_cnn_save.restype = ctypes.c_int
    lib.rmrcm_cnn_load.argtypes = [ctypes.c_char_p, i32, i32, ctypes.POINTER(vp)]
    lib.rmrcm_cnn_load.restype = ctypes.c_int
    lib.rmrcm_cnn_destroy.argtypes = [vp]
    lib.rmrcm_cnn_destroy.restype = None
    return lib


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _ptr(a, dtype):
    """Raw pointer of a NumPy array (host) or torch tensor (any device)."""
    if a is None:
        return None, None
    if hasattr(a, "data_ptr"):                      # torch tensor
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(a.data_ptr()), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return ctypes.c_void_p(arr.ctypes.data), arr


def _check(st, where):
    if st != RMRCM_OK:
        raise RMRCMError(st, where)


def rmrcm_default_params() -> rmrcm_params:
    p = rmrcm_params()
    lib().rmrcm_default_params(ctypes.byref(p))
    return p


def rmrcm_plan_bytes(params: rmrcm_params) -> int:
    b = ctypes.c_uint64()
    _check(lib().rmrcm_plan_bytes(ctypes.byref(params), ctypes.byref(b)), "rmrcm_plan_bytes")
    return b.value


def rmrcm_downscale(ctx, source, bc_value, pressure, flux, pressure_out, flux_out) -> None:
    sp_, k1 = _ptr(source, np.float64)
    bp, k2 = _ptr(bc_value, np.float64)
    pp, k3 = _ptr(pressure, np.float64)
    fp, k4 = _ptr(flux, np.float64)
    po, k5 = _ptr(pressure_out, np.float64)
    fo, k6 = _ptr(flux_out, np.float64)
    if isinstance(pressure_out, np.ndarray) and k5 is not pressure_out:
        raise ValueError("pressure_out must be a contiguous float64 array")
    if isinstance(flux_out, np.ndarray) and k6 is not flux_out:
        raise ValueError("flux_out must be a contiguous float64 array")
    _check(lib().rmrcm_downscale(ctx, sp_, bp, pp, fp, po, fo), "rmrcm_downscale")


def rmrcm_set_refinement(ctx, ir_tol: float, ir_max_iter: int) -> None:
    _check(lib().rmrcm_set_refinement(ctx, ir_tol, ir_max_iter), "rmrcm_set_refinement")


def rmrcm_setup(params: rmrcm_params, perm, bc_type):
    kp, _k = _ptr(perm, np.float64)
    tp, _t = _ptr(bc_type, np.int8)
    ctx = ctypes.c_void_p()
    st = lib().rmrcm_setup(ctypes.byref(params), kp, tp, ctypes.byref(ctx))
    _check(st, "rmrcm_setup")
    return ctx


def rmrcm_refactor(ctx, perm):
    kp, _k = _ptr(perm, np.float64)
    _check(lib().rmrcm_refactor(ctx, kp), "rmrcm_refactor")


def rmrcm_sync(ctx):
    _check(lib().rmrcm_sync(ctx), "rmrcm_sync")


def rmrcm_solve(ctx, source, bc_value, pressure, flux):
    sp, _s = _ptr(source, np.float64)
    bp, _b = _ptr(bc_value, np.float64)
    pp, _p = _ptr(pressure, np.float64)
    fp, _f = _ptr(flux, np.float64)
    _check(lib().rmrcm_solve(ctx, sp, bp, pp, fp), "rmrcm_solve")


def rmrcm_step(ctx, perm, source, bc_value, pressure, flux):
    kp, _k = _ptr(perm, np.float64)
    sp, _s = _ptr(source, np.float64)
    bp, _b = _ptr(bc_value, np.float64)
    pp, _p = _ptr(pressure, np.float64)
    fp, _f = _ptr(flux, np.float64)
    _check(lib().rmrcm_step(ctx, kp, sp, bp, pp, fp), "rmrcm_step")


def rmrcm_step_noalloc(params: rmrcm_params, perm, bc_type, source, bc_value, pressure, flux,
                       stream_handle=None):
    """The allocation-free FP64 step: device tensors for perm, source (or
    None), bc_value, pressure and flux; returns when they are written."""
    kp, _k = _ptr(perm, np.float64)
    tp, _t = _ptr(bc_type, np.int8)
    sp, _s = _ptr(source, np.float64)
    bp, _b = _ptr(bc_value, np.float64)
    pp, _p = _ptr(pressure, np.float64)
    fp, _f = _ptr(flux, np.float64)
    st = lib().rmrcm_step_noalloc(ctypes.byref(params), kp, tp, sp, bp, pp, fp,
                                  ctypes.c_void_p(stream_handle) if stream_handle else None)
    _check(st, "rmrcm_step_noalloc")


def rmrcm_get_interface(ctx, U, P):
    up, _u = _ptr(U, np.float64)
    pp, _p = _ptr(P, np.float64)
    _check(lib().rmrcm_get_interface(ctx, up, pp), "rmrcm_get_interface")


def rmrcm_counts(ctx):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rmrcm_counts(ctx, ctypes.byref(a), ctypes.byref(b)), "rmrcm_counts")
    return a.value, b.value


def rmrcm_set_step_graph(ctx, enabled):
    _check(lib().rmrcm_set_step_graph(ctx, 1 if enabled else 0), "rmrcm_set_step_graph")


def rmrcm_set_stream(ctx, stream_handle):
    _check(lib().rmrcm_set_stream(ctx, ctypes.c_void_p(stream_handle)), "rmrcm_set_stream")


def rmrcm_get_stats(ctx) -> dict:
    need = lib().rmrcm_get_stats(ctx, None, 0)
    if need < 0:
        raise RMRCMError(need, "rmrcm_get_stats")
    buf = ctypes.create_string_buffer(need)
    lib().rmrcm_get_stats(ctx, buf, need)
    return json.loads(buf.value.decode())


def rmrcm_destroy(ctx):
    lib().rmrcm_destroy(ctx)


def rmrcm_strerror(status: int) -> str:
    return lib().rmrcm_strerror(status).decode()


def rmrcm_autotune(ctx):
    _check(lib().rmrcm_autotune(ctx), "rmrcm_autotune")


def _ptr_array(items, dtype):
    """ctypes array of raw pointers (None allowed) plus the objects kept alive."""
    keep, raw = [], []
    for a in items:
        p, k = _ptr(a, dtype)
        keep.append(k)
        raw.append(p.value if p is not None else None)
    return (ctypes.c_void_p * len(raw))(*raw), keep


def rmrcm_export_local(ctx, features, basis=None):
    """features: device float32 tensor [nsub, 2, S, S]; basis: float64
    array/tensor [nsub, R, S*S] or None.  Returns the interior mask."""
    nsub = features.shape[0]
    interior = np.zeros(nsub, dtype=np.int32)
    fp, _f = _ptr(features, np.float32)
    bp, _b = _ptr(basis, np.float64)
    _check(lib().rmrcm_export_local(ctx, fp, bp, ctypes.c_void_p(interior.ctypes.data)),
           "rmrcm_export_local")
    return interior


def rmrcm_get_gate(ctx, nsub):
    """(residual [nsub] float64, accepted [nsub] int32) of the learned mode's
    residual gate at the last setup."""
    r = np.zeros(nsub)
    a = np.zeros(nsub, dtype=np.int32)
    _check(lib().rmrcm_get_gate(ctx, ctypes.c_void_p(r.ctypes.data), ctypes.c_void_p(a.ctypes.data)),
           "rmrcm_get_gate")
    return r, a


class Net:
    """The local-basis surrogate network (rmrcm_cnn_*): S x S patches, width
    C, L convolution layers, R outputs.  Inputs / outputs are device
    float32 tensors."""

    def __init__(self, S, C, L, R, max_batch=256, device=0, _handle=None):
        self.S, self.C, self.L, self.R, self.max_batch = S, C, L, R, max_batch
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib().rmrcm_cnn_create(S, C, L, R, max_batch, device, ctypes.byref(h)),
                   "rmrcm_cnn_create")
            _handle = h
        self.h = _handle
        n = ctypes.c_int64()
        _check(lib().rmrcm_cnn_num_params(self.h, ctypes.byref(n)), "rmrcm_cnn_num_params")
        self.num_params = n.value

    @classmethod
    def load(cls, path, max_batch=256, device=0):
        h = ctypes.c_void_p()
        _check(lib().rmrcm_cnn_load(path.encode(), max_batch, device, ctypes.byref(h)), "rmrcm_cnn_load")
        with open(path, "rb") as f:
            hdr = np.frombuffer(f.read(24)[8:24], dtype=np.int32)
        return cls(int(hdr[0]), int(hdr[1]), int(hdr[2]), int(hdr[3]), max_batch, device, _handle=h)

    def set_stream(self, handle):
        _check(lib().rmrcm_cnn_set_stream(self.h, ctypes.c_void_p(handle)), "rmrcm_cnn_set_stream")

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.size == self.num_params
        _check(lib().rmrcm_cnn_set_params(self.h, ctypes.c_void_p(a.ctypes.data)), "rmrcm_cnn_set_params")

    def get_params(self):
        a = np.zeros(self.num_params, dtype=np.float32)
        _check(lib().rmrcm_cnn_get_params(self.h, ctypes.c_void_p(a.ctypes.data)), "rmrcm_cnn_get_params")
        return a

    def forward(self, x, y):
        _check(lib().rmrcm_cnn_forward(self.h, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr())), "rmrcm_cnn_forward")

    def loss_grad(self, x, t):
        loss = ctypes.c_double()
        g = np.zeros(self.num_params, dtype=np.float32)
        _check(lib().rmrcm_cnn_loss_grad(self.h, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(t.data_ptr()), ctypes.byref(loss),
                                         ctypes.c_void_p(g.ctypes.data)), "rmrcm_cnn_loss_grad")
        return loss.value, g

    def train_step(self, x, t, lr, want_loss=False):
        loss = ctypes.c_double()
        _check(lib().rmrcm_cnn_train_step(self.h, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(t.data_ptr()), ctypes.c_float(lr),
                                          ctypes.byref(loss) if want_loss else None),
               "rmrcm_cnn_train_step")
        return loss.value if want_loss else None

    def save(self, path):
        _check(lib().rmrcm_cnn_save(self.h, path.encode()), "rmrcm_cnn_save")

    def close(self):
        if getattr(self, "h", None) is not None:
            lib().rmrcm_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """An ensemble of independent problems enqueued together (see
    rmrcm_batch_create): refactor / solve all members, then sync."""

    def __init__(self, problems, precision=RMRCM_FP64, autotune=True, device=0):
        self.problems = list(problems)
        n = len(self.problems)
        prms = (rmrcm_params * n)()
        for i, pr in enumerate(self.problems):
            p = rmrcm_default_params()
            p.nx, p.ny, p.lx, p.ly = pr.nx, pr.ny, pr.lx, pr.ly
            p.sub_nx, p.sub_ny, p.seg, p.alpha = pr.sub_nx, pr.sub_ny, pr.seg, pr.alpha
            p.precision, p.device = precision, device
            prms[i] = p
        kp, self._k = _ptr_array([pr.K for pr in self.problems], np.float64)
        tp, self._t = _ptr_array([pr.bc_type for pr in self.problems], np.int8)
        b = ctypes.c_void_p()
        _check(lib().rmrcm_batch_create(n, prms, ctypes.cast(kp, ctypes.POINTER(ctypes.c_void_p)),
                                        ctypes.cast(tp, ctypes.POINTER(ctypes.c_void_p)),
                                        1 if autotune else 0, ctypes.byref(b)),
               "rmrcm_batch_create")
        self.b = b
        self._keep = []

    def refactor(self, perms):
        kp, keep = _ptr_array(perms, np.float64)
        self._keep = [keep]
        _check(lib().rmrcm_batch_refactor(self.b, ctypes.cast(kp, ctypes.POINTER(ctypes.c_void_p))),
               "rmrcm_batch_refactor")

    def solve(self, sources, bc_values, pressures=None, fluxes=None, wait=True):
        """Enqueue every member's solve; with wait, sync and return the
        (pressure, flux) arrays."""
        if pressures is None:
            pressures = [np.zeros((pr.ny, pr.nx)) for pr in self.problems]
        if fluxes is None:
            fluxes = [np.zeros((4, pr.ny, pr.nx)) for pr in self.problems]
        sp, k1 = _ptr_array(sources, np.float64)
        bp, k2 = _ptr_array(bc_values, np.float64)
        pp, k3 = _ptr_array(pressures, np.float64)
        fp, k4 = _ptr_array(fluxes, np.float64)
        self._keep.append((k1, k2, k3, k4))
        cast = lambda a: ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p))  # noqa: E731
        _check(lib().rmrcm_batch_solve(self.b, cast(sp), cast(bp), cast(pp), cast(fp)),
               "rmrcm_batch_solve")
        if wait:
            self.sync()
        return pressures, fluxes

    def sync(self):
        st = (ctypes.c_int32 * len(self.problems))()
        r = lib().rmrcm_batch_sync(self.b, st)
        self._keep = []
        if r != RMRCM_OK:
            raise RMRCMError(r, "rmrcm_batch_sync (member statuses %s)" % list(st))
        return list(st)

    def stats(self) -> dict:
        need = lib().rmrcm_batch_get_stats(self.b, None, 0)
        buf = ctypes.create_string_buffer(need)
        lib().rmrcm_batch_get_stats(self.b, buf, need)
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "b", None) is not None:
            lib().rmrcm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """One setup (permeability + boundary-condition types), many solves."""

    def __init__(self, nx, ny, K, bc_type, sub_nx, sub_ny, seg, alpha=1.0,
                 lx=1.0, ly=1.0, precision=RMRCM_FP64, device=0, **extra):
        p = rmrcm_default_params()
        p.nx, p.ny, p.lx, p.ly = nx, ny, lx, ly
        p.sub_nx, p.sub_ny, p.seg, p.alpha = sub_nx, sub_ny, seg, alpha
        p.precision, p.device = precision, device
        for k, v in extra.items():
            setattr(p, k, v)
        self.params = p
        self.nx, self.ny = nx, ny
        # 3D problems (nz >= 1): arrays (nz, ny, nx), six flux blocks
        self.nz = p.nz
        self.shape = (p.nz, ny, nx) if p.nz > 0 else (ny, nx)
        self.nflux = 6 if p.nz > 0 else 4
        self.ctx = rmrcm_setup(p, K, bc_type)
        self.nseg, self.nlocal = rmrcm_counts(self.ctx)

    @classmethod
    def from_problem(cls, prob, **kw):
        for k in ("seg_u", "seg_p"):
            if getattr(prob, k, 0) and k not in kw:
                kw[k] = getattr(prob, k)
        if getattr(prob, "nz", 0) and "nz" not in kw:
            kw["nz"], kw["lz"] = prob.nz, prob.lz
        return cls(prob.nx, prob.ny, prob.K, prob.bc_type, prob.sub_nx, prob.sub_ny,
                   prob.seg, alpha=prob.alpha, lx=prob.lx, ly=prob.ly, **kw)

    def refactor(self, K, wait=True):
        """New permeability, same geometry.  wait=False leaves the work
        enqueued (errors then surface at the next sync or waiting solve)."""
        rmrcm_refactor(self.ctx, K)
        if wait:
            rmrcm_sync(self.ctx)

    def sync(self):
        rmrcm_sync(self.ctx)

    def solve(self, q, bc_value, pressure=None, flux=None):
        """Returns (pressure (ny, nx), flux (4, ny, nx)), in 3D (nz, ny, nx)
        and (6, nz, ny, nx); NumPy unless output tensors are given."""
        if pressure is None:
            pressure = np.zeros(self.shape)
        if flux is None:
            flux = np.zeros((self.nflux,) + self.shape)
        rmrcm_solve(self.ctx, q, bc_value, pressure, flux)
        return pressure, flux

    def downscale(self, q, bc_value, pressure, flux):
        """Single-valued, cell-conservative (pressure, flux) from an MRCM
        solution of this problem (rmrcm_downscale)."""
        po = np.zeros((self.ny, self.nx))
        fo = np.zeros((4, self.ny, self.nx))
        rmrcm_downscale(self.ctx, q, bc_value, pressure, flux, po, fo)
        return po, fo

    def step(self, K, q, bc_value, pressure=None, flux=None):
        """refactor(K) and solve(q, bc_value) as one unit (a replayed graph
        for FP64 contexts with device arrays); returns (pressure, flux)."""
        if pressure is None:
            pressure = np.zeros(self.shape)
        if flux is None:
            flux = np.zeros((self.nflux,) + self.shape)
        rmrcm_step(self.ctx, K, q, bc_value, pressure, flux)
        return pressure, flux

    def interface(self):
        U = np.zeros(self.nseg)
        P = np.zeros(self.nseg)
        rmrcm_get_interface(self.ctx, U, P)
        return U, P

    def set_stream(self, handle):
        rmrcm_set_stream(self.ctx, handle)

    def set_step_graph(self, enabled):
        """step() as a replayed graph (True, the default) or launch by launch
        with the phase timers recording it (False); same results."""
        rmrcm_set_step_graph(self.ctx, enabled)

    def autotune(self):
        rmrcm_autotune(self.ctx)

    def stats(self):
        return rmrcm_get_stats(self.ctx)

    def close(self):
        if self.ctx is not None:
            rmrcm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
