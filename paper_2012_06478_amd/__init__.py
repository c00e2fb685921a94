"""MI355X Monte Carlo diffusion walker (after Lee, Fieremans & Novikov, "Realistic
Microstructure Simulator", arXiv 2012.06478): Python binding of ``librms.so``.

This module only marshals arguments to the C ABI of ``include/rms.h``; every
step of the walk runs in the library's HIP kernels.  The functions carry the
C names: ``rms_create_substrate``, ``rms_destroy_substrate``, ``rms_run``,
``rms_abi_version``, ``rms_last_error``.  Importing works without a GPU (the
library loads); calls that touch the device need one.  If the library has not
been built, loading fails loudly: there is no other implementation behind
these names.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librms.so")

RMS_OK = 0
RMS_FP64 = 0
RMS_MIXED = 1
RMS_PERM_KAPPA = 0
RMS_PERM_BAXTER = 1
RMS_MAX_SHAPES = 4
RMS_MAX_SIGNALS = 960
RMS_MAX_LABELS = 4096
RMS_MAX_PERM_PROB = 0.1
RMS_DUMP_FIXED = 15
RMS_NOALLOC_MAX_BYTES = 256 * 1024 * 1024  # scratch array of rms_run_noalloc, per GPU
RMS_WALK_AUTO = -1
RMS_WALK_ONE_LAUNCH = 0
RMS_WALK_PERSISTENT = 1
RMS_WALK_PACKED = 2
RMS_OPT_WALK_KERNEL = 1
RMS_OPT_SEG_POLL_LIMIT = 2
RMS_OPT_SERVER_WALKERS = 3
RMS_E_WAIT_GAVE_UP = -10
ERROR_NAMES = {
    -1: "RMS_E_INVALID_ARG", -2: "RMS_E_LABEL_RANGE", -3: "RMS_E_STEP_TOO_LARGE",
    -4: "RMS_E_PROB_TOO_LARGE", -5: "RMS_E_UNBALANCED_WAVEFORM", -6: "RMS_E_OOM",
    -7: "RMS_E_DEVICE", -8: "RMS_E_BUSY", -9: "RMS_E_TIMEOUT", -10: "RMS_E_WAIT_GAVE_UP",
}
WALK_KERNELS = {RMS_WALK_ONE_LAUNCH: "one launch", RMS_WALK_PERSISTENT: "persistent",
                RMS_WALK_PACKED: "packed"}
DUMP_FIELDS = ["dx", "dy", "dz", "R", "label", "ix", "iy", "iz", "ox", "oy", "oz",
               "label0", "n_face", "n_hit", "n_perm"]


class RmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class _Params(C.Structure):
    _fields_ = [("n_labels", C.c_int), ("D", C.POINTER(C.c_double)),
                ("kappa", C.POINTER(C.c_double)), ("T2", C.POINTER(C.c_double)),
                ("rho", C.POINTER(C.c_double)), ("conc", C.POINTER(C.c_double)),
                ("lam", C.c_double), ("perm_model", C.c_int)]


class _Record(C.Structure):
    _fields_ = [("n_rec", C.c_int), ("steps", C.POINTER(C.c_int64)),
                ("sum_alpha", C.POINTER(C.c_double)), ("m2", C.POINTER(C.c_double)),
                ("m4", C.POINTER(C.c_double)), ("D_dir", C.POINTER(C.c_double)),
                ("K_dir", C.POINTER(C.c_double))]


class _Result(C.Structure):
    _fields_ = [("signal", C.POINTER(C.c_double)), ("m2", C.c_double * 6),
                ("m4", C.c_double * 15), ("D_dir", C.POINTER(C.c_double)),
                ("K_dir", C.POINTER(C.c_double)), ("sum_alpha", C.c_double),
                ("b_disc", C.POINTER(C.c_double)), ("n_face_events", C.c_int64),
                ("n_membrane_hits", C.c_int64), ("n_permeations", C.c_int64),
                ("max_perm_prob", C.c_double), ("max_step_over_voxel", C.c_double),
                ("wall_s", C.c_double), ("kernel_ms", C.c_double), ("queue_s", C.c_double),
                ("walker_dump", C.POINTER(C.c_double)), ("walk_kernel", C.c_int)]


class _Request(C.Structure):
    _fields_ = [("substrate", C.c_void_p), ("params", C.POINTER(_Params)), ("seed", C.c_uint64),
                ("n_walkers", C.c_int64), ("n_steps", C.c_int64), ("dt_ms", C.c_double),
                ("n_shapes", C.c_int), ("waveform", C.POINTER(C.c_double)), ("n_dirs", C.c_int),
                ("dirs", C.POINTER(C.c_double)), ("n_b", C.c_int),
                ("bvals", C.POINTER(C.c_double)), ("precision", C.c_int)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("pending", C.c_int64), ("active", C.c_int64), ("launches", C.c_int64),
                ("walker_steps", C.c_int64), ("busy_s", C.c_double),
                ("bytes_in_use", C.c_size_t), ("bytes_budget", C.c_size_t)]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    try:  # share torch's HIP runtime (same SONAME) so its streams are valid here
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = C.CDLL(LIB_PATH)
    dp, i64p, u8p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_uint8)
    lib.rms_abi_version.restype = C.c_int
    lib.rms_last_error.restype = C.c_char_p
    lib.rms_set_option.argtypes = [C.c_int, C.c_int64]
    lib.rms_set_option.restype = C.c_int
    lib.rms_create_substrate.argtypes = [C.c_void_p, C.c_int, i64p, C.c_double, C.c_int, dp, dp,
                                         dp, u8p, C.POINTER(C.c_void_p)]
    lib.rms_create_substrate.restype = C.c_int
    lib.rms_destroy_substrate.argtypes = [C.c_void_p]
    lib.rms_destroy_substrate.restype = None
    lib.rms_run.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_uint64, C.c_int64, C.c_int64,
                            C.c_double, C.c_int, dp, C.c_int, dp, C.c_int, dp, C.c_int,
                            C.c_void_p, C.POINTER(_Result)]
    lib.rms_run.restype = C.c_int
    lib.rms_run_noalloc.argtypes = lib.rms_run.argtypes
    lib.rms_run_noalloc.restype = C.c_int
    lib.rms_run_record.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_uint64, C.c_int64,
                                   C.c_int64, C.c_double, C.c_int, dp, C.c_int, dp, C.c_int, dp,
                                   C.c_int, C.c_void_p, C.POINTER(_Record), C.POINTER(_Result)]
    lib.rms_run_record.restype = C.c_int
    lib.rms_spherical_mean.argtypes = [C.c_int, C.c_int, dp, dp]
    lib.rms_spherical_mean.restype = C.c_int
    lib.rms_cumulant_fit.argtypes = [C.c_int, dp, C.c_int, dp, C.c_double, dp, dp]
    lib.rms_cumulant_fit.restype = C.c_int
    lib.rms_server_create.argtypes = [C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]
    lib.rms_server_create.restype = C.c_int
    lib.rms_server_submit.argtypes = [C.c_void_p, C.POINTER(_Request), C.POINTER(C.c_int64)]
    lib.rms_server_submit.restype = C.c_int
    lib.rms_server_poll.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int)]
    lib.rms_server_poll.restype = C.c_int
    lib.rms_server_wait.argtypes = [C.c_void_p, C.c_int64, C.c_double, C.POINTER(_Result)]
    lib.rms_server_wait.restype = C.c_int
    lib.rms_server_stats_get.argtypes = [C.c_void_p, C.POINTER(_ServerStats)]
    lib.rms_server_stats_get.restype = C.c_int
    lib.rms_server_destroy.argtypes = [C.c_void_p]
    lib.rms_server_destroy.restype = None
    _lib = lib
    return lib


def exported_symbols() -> list[str]:
    """Names the library exports through the C ABI (for load checks)."""
    lib = _load()
    names = ["rms_abi_version", "rms_last_error", "rms_set_option", "rms_create_substrate",
             "rms_destroy_substrate", "rms_run", "rms_run_noalloc", "rms_run_record",
             "rms_spherical_mean",
             "rms_cumulant_fit", "rms_server_create", "rms_server_submit",
             "rms_server_poll", "rms_server_wait", "rms_server_stats_get", "rms_server_destroy"]
    return [n for n in names if hasattr(lib, n)]


def rms_abi_version() -> int:
    return _load().rms_abi_version()


def rms_last_error() -> str:
    return _load().rms_last_error().decode()


def rms_set_option(option: int, value: int) -> None:
    """Process-wide option (``RMS_OPT_WALK_KERNEL``, ``RMS_OPT_SEG_POLL_LIMIT``,
    ``RMS_OPT_SERVER_WALKERS``)."""
    _check(_load().rms_set_option(int(option), int(value)))


def _check(rc: int):
    if rc != RMS_OK:
        raise RmsError(rc, rms_last_error())


def _dptr(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


class Substrate:
    """Handle of a device-resident substrate (``rms_substrate*``)."""

    def __init__(self, handle, labels_shape, n_labels, voxel_um):
        self.handle = handle
        self.shape = labels_shape
        self.n_labels = n_labels
        self.voxel_um = voxel_um

    def close(self):
        if self.handle:
            _load().rms_destroy_substrate(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rms_create_substrate(labels, voxel_um, D, kappa=None, T2=None, dead=None) -> Substrate:
    """``labels``: [nz, ny, nx] uint8/uint16 array (x fastest); D [n]; kappa
    [n, n] or None; T2 [n] or None; dead [n] bool or None."""
    lib = _load()
    lab = np.ascontiguousarray(labels)
    if lab.ndim != 3 or lab.dtype not in (np.uint8, np.uint16):
        raise TypeError("labels must be a 3d uint8 or uint16 array")
    dims = np.array(lab.shape[::-1], np.int64)
    Dv = np.ascontiguousarray(D, np.float64).reshape(-1)
    n = Dv.size
    kap = _sized(kappa, n * n, "kappa")
    t2 = _sized(T2, n, "T2")
    dd = None if dead is None else np.ascontiguousarray(dead, np.uint8).reshape(-1)
    if dd is not None and dd.size != n:
        raise ValueError(f"dead must have {n} entries (one per label), not {dd.size}")
    h = C.c_void_p()
    rc = lib.rms_create_substrate(lab.ctypes.data, lab.dtype.itemsize,
                                  dims.ctypes.data_as(C.POINTER(C.c_int64)), float(voxel_um), n,
                                  _dptr(Dv), _dptr(kap), _dptr(t2),
                                  None if dd is None else dd.ctypes.data_as(C.POINTER(C.c_uint8)),
                                  C.byref(h))
    _check(rc)
    return Substrate(h, lab.shape, n, voxel_um)


def rms_destroy_substrate(sub: Substrate) -> None:
    sub.close()


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream (HIP stream on ROCm)


def _sized(a, n, name):
    """a as a flat contiguous float64 array of exactly n entries (or None):
    the library reads n entries through the pointer."""
    if a is None:
        return None
    v = np.ascontiguousarray(a, np.float64).reshape(-1)
    if v.size != n:
        raise ValueError(f"{name} must have {n} entries, not {v.size}")
    return v


def _protocol(n_steps, waveform, dirs, bvals):
    W = (np.zeros((0, n_steps)) if waveform is None
         else np.ascontiguousarray(np.atleast_2d(waveform), np.float64))
    if W.ndim != 2 or (W.shape[0] > 0 and W.shape[1] != int(n_steps)):
        raise ValueError(f"waveform must be [n_shapes, n_steps] with n_steps = {int(n_steps)}, "
                         f"not {list(W.shape)}")
    d = None if dirs is None else np.ascontiguousarray(dirs, np.float64)
    if d is not None and (d.size % 3 != 0 or (d.ndim == 2 and d.shape[1] != 3)):
        raise ValueError(f"dirs must be [n_dirs, 3], not {list(d.shape)}")
    g = np.zeros((0, 3)) if d is None else d.reshape(-1, 3)
    b = np.zeros(0) if bvals is None else np.ascontiguousarray(bvals, np.float64).reshape(-1)
    return W, g, b


def _params(params, keep, n_labels=None):
    """rms_params from a dict; with n_labels (the substrate's), every array is
    checked to hold the entries the library reads."""
    if params is None:
        return None
    Dv = np.ascontiguousarray(params["D"], np.float64).reshape(-1)
    n = Dv.size
    if n_labels is not None and n != n_labels:
        raise ValueError(f"params D must have {n_labels} entries (one per label), not {n}")
    kap = _sized(params.get("kappa"), n * n, "params kappa")
    t2 = _sized(params.get("T2"), n, "params T2")
    rho = _sized(params.get("rho"), n * n, "params rho")
    conc = _sized(params.get("conc"), n, "params conc")
    keep += [Dv, kap, t2, rho, conc]
    return _Params(Dv.size, _dptr(Dv), _dptr(kap), _dptr(t2), _dptr(rho), _dptr(conc),
                   float(params.get("lam", 0.0)), int(params.get("perm_model", RMS_PERM_KAPPA)))


class _ResultBuffers:
    def __init__(self, ns, nb, nd):
        self.shape = (ns, nb, nd)
        self.sig = np.zeros(max(ns * nb * nd, 1) * 2)
        self.Dd = np.zeros(max(nd, 1))
        self.Kd = np.zeros(max(nd, 1))
        self.bd = np.zeros(max(ns, 1))
        self.res = _Result()
        self.res.signal = _dptr(self.sig)
        self.res.D_dir = _dptr(self.Dd)
        self.res.K_dir = _dptr(self.Kd)
        self.res.b_disc = _dptr(self.bd)
        self.res.walker_dump = None

    def to_dict(self):
        ns, nb, nd = self.shape
        res, sig = self.res, self.sig
        return dict(
            signal=(sig[0::2] + 1j * sig[1::2])[: ns * nb * nd].reshape(ns, nb, nd),
            m2=np.array(res.m2[:]), m4=np.array(res.m4[:]), D=self.Dd[:nd].copy(),
            K=self.Kd[:nd].copy(), sum_alpha=res.sum_alpha, b_disc=self.bd[:ns].copy(),
            n_face_events=res.n_face_events, n_membrane_hits=res.n_membrane_hits,
            n_permeations=res.n_permeations, max_perm_prob=res.max_perm_prob,
            max_step_over_voxel=res.max_step_over_voxel, wall_s=res.wall_s,
            kernel_ms=res.kernel_ms, queue_s=res.queue_s,
            walk_kernel=WALK_KERNELS.get(res.walk_kernel, str(res.walk_kernel)),
        )


def rms_run(sub: Substrate, *, seed, n_walkers, n_steps, dt, waveform=None, dirs=None,
            bvals=None, precision=RMS_FP64, params=None, stream=None, dump=False) -> dict:
    """Run the walk; returns a dict of numpy results (see ``include/rms.h``).

    ``params``: optional dict with ``D``, ``kappa``, ``T2`` overriding the
    substrate's tissue parameters, ``rho`` [n, n] making membranes
    absorbing (magnetization transfer), and ``conc`` [n], ``lam``,
    ``perm_model`` for unequal spin concentrations (App. C).  ``stream``: a torch.cuda.Stream or a raw
    hipStream_t (int); None runs on the null stream."""
    return _run_call(_load().rms_run, sub, seed, n_walkers, n_steps, dt, waveform, dirs, bvals,
                     precision, params, stream, dump)


def rms_run_noalloc(sub: Substrate, *, seed, n_walkers, n_steps, dt, waveform=None, dirs=None,
                    bvals=None, precision=RMS_FP64, params=None, stream=None,
                    dump=False) -> dict:
    """``rms_run`` on the library's device scratch array (no device
    allocation; runs up to ``RMS_NOALLOC_MAX_BYTES`` of buffers, and calls
    that overlap on one GPU race; see ``include/rms.h``)."""
    return _run_call(_load().rms_run_noalloc, sub, seed, n_walkers, n_steps, dt, waveform, dirs,
                     bvals, precision, params, stream, dump)


def _run_call(fn, sub, seed, n_walkers, n_steps, dt, waveform, dirs, bvals, precision, params,
              stream, dump) -> dict:
    W, g, b = _protocol(n_steps, waveform, dirs, bvals)
    keep = []
    pp = _params(params, keep, sub.n_labels)
    rb = _ResultBuffers(W.shape[0], b.size, g.shape[0])
    wd = np.zeros((int(n_walkers), RMS_DUMP_FIXED + 3 * W.shape[0])) if dump else None
    rb.res.walker_dump = _dptr(wd) if wd is not None else None
    rc = fn(sub.handle, None if pp is None else C.byref(pp), int(seed) & (2**64 - 1),
            int(n_walkers), int(n_steps), float(dt), W.shape[0], _dptr(W), g.shape[0],
            _dptr(g), b.size, _dptr(b), int(precision), _stream_handle(stream), C.byref(rb.res))
    _check(rc)
    out = rb.to_dict()
    if wd is not None:
        out["dump"] = wd
        out["phase"] = wd[:, RMS_DUMP_FIXED:].reshape(int(n_walkers), W.shape[0], 3)
    return out


def rms_run_record(sub: Substrate, *, seed, n_walkers, n_steps, dt, record_steps,
                   waveform=None, dirs=None, bvals=None, precision=RMS_FP64, params=None,
                   stream=None, dump=False) -> dict:
    """``rms_run`` plus the displacement moments after each of ``record_steps``
    (ascending, 1..n_steps): the result gains ``records`` with ``steps``,
    ``sum_alpha`` [n_rec], ``m2`` [n_rec, 6], ``m4`` [n_rec, 15], ``D`` and
    ``K`` [n_rec, n_dirs] (see ``rms_run_record`` in ``include/rms.h``)."""
    lib = _load()
    W, g, b = _protocol(n_steps, waveform, dirs, bvals)
    keep = []
    pp = _params(params, keep, sub.n_labels)
    rb = _ResultBuffers(W.shape[0], b.size, g.shape[0])
    wd = np.zeros((int(n_walkers), RMS_DUMP_FIXED + 3 * W.shape[0])) if dump else None
    rb.res.walker_dump = _dptr(wd) if wd is not None else None
    steps = np.ascontiguousarray(record_steps, np.int64).reshape(-1)
    nr, nd = steps.size, g.shape[0]
    sa, m2, m4 = np.zeros(max(nr, 1)), np.zeros((max(nr, 1), 6)), np.zeros((max(nr, 1), 15))
    Dd, Kd = np.zeros((max(nr, 1), max(nd, 1))), np.zeros((max(nr, 1), max(nd, 1)))
    rec = _Record(nr, steps.ctypes.data_as(C.POINTER(C.c_int64)), _dptr(sa), _dptr(m2),
                  _dptr(m4), _dptr(Dd), _dptr(Kd))
    rc = lib.rms_run_record(sub.handle, None if pp is None else C.byref(pp),
                            int(seed) & (2**64 - 1), int(n_walkers), int(n_steps), float(dt),
                            W.shape[0], _dptr(W), nd, _dptr(g), b.size, _dptr(b),
                            int(precision), _stream_handle(stream), C.byref(rec), C.byref(rb.res))
    _check(rc)
    out = rb.to_dict()
    out["records"] = dict(steps=steps.copy(), sum_alpha=sa[:nr].copy(), m2=m2[:nr].copy(),
                          m4=m4[:nr].copy(), D=Dd[:nr, :nd].copy(), K=Kd[:nr, :nd].copy())
    if wd is not None:
        out["dump"] = wd
        out["phase"] = wd[:, RMS_DUMP_FIXED:].reshape(int(n_walkers), W.shape[0], 3)
    return out


def _signal_array(signal):
    """[n_b, n_dirs] complex -> contiguous [n_b][n_dirs][2] doubles."""
    S = np.asarray(signal)
    if S.ndim != 2:
        raise ValueError("signal must be [n_b, n_dirs] (one shape)")
    A = np.empty(S.shape + (2,))
    A[..., 0], A[..., 1] = S.real, S.imag
    return np.ascontiguousarray(A)


def rms_spherical_mean(signal) -> np.ndarray:
    """Direction average of a [n_b, n_dirs] complex signal; returns [n_b]."""
    A = _signal_array(signal)
    out = np.zeros((A.shape[0], 2))
    _check(_load().rms_spherical_mean(A.shape[0], A.shape[1], _dptr(A), _dptr(out)))
    return out[:, 0] + 1j * out[:, 1]


def rms_cumulant_fit(signal, bvals, b_max: float):
    """Per direction D and K from ln Re S(b) = -bD + b^2 D^2 K / 6 over
    0 < b <= b_max; returns (D [n_dirs], K [n_dirs])."""
    A = _signal_array(signal)
    b = np.ascontiguousarray(bvals, np.float64)
    if b.size != A.shape[0]:
        raise ValueError("bvals must match the signal's b axis")
    D = np.zeros(A.shape[1])
    K = np.zeros(A.shape[1])
    _check(_load().rms_cumulant_fit(b.size, _dptr(b), A.shape[1], _dptr(A), float(b_max),
                                    _dptr(D), _dptr(K)))
    return D, K


# ------------------------------------------------------------------ server --

def rms_server_create(mem_budget_bytes: int = 0, slice_steps: int = 0):
    h = C.c_void_p()
    _check(_load().rms_server_create(int(mem_budget_bytes), int(slice_steps), C.byref(h)))
    return h


def rms_server_submit(srv, sub: Substrate, *, seed, n_walkers, n_steps, dt, waveform=None,
                      dirs=None, bvals=None, precision=RMS_FP64, params=None):
    """Queue a request; returns (ticket, shape of its signal array)."""
    lib = _load()
    W, g, b = _protocol(n_steps, waveform, dirs, bvals)
    keep = []
    pp = _params(params, keep, sub.n_labels)
    q = _Request(sub.handle, None if pp is None else C.pointer(pp), int(seed) & (2**64 - 1),
                 int(n_walkers), int(n_steps), float(dt), W.shape[0], _dptr(W), g.shape[0],
                 _dptr(g), b.size, _dptr(b), int(precision))
    t = C.c_int64()
    _check(lib.rms_server_submit(srv, C.byref(q), C.byref(t)))
    return t.value, (W.shape[0], b.size, g.shape[0])


def rms_server_poll(srv, ticket: int) -> bool:
    d = C.c_int()
    _check(_load().rms_server_poll(srv, int(ticket), C.byref(d)))
    return bool(d.value)


def rms_server_wait(srv, ticket: int, shape, timeout_s: float = -1.0) -> dict:
    rb = _ResultBuffers(*shape)
    _check(_load().rms_server_wait(srv, int(ticket), float(timeout_s), C.byref(rb.res)))
    return rb.to_dict()


def rms_server_stats_get(srv) -> dict:
    st = _ServerStats()
    _check(_load().rms_server_stats_get(srv, C.byref(st)))
    return {k: getattr(st, k) for k, _ in _ServerStats._fields_}


def rms_server_destroy(srv) -> None:
    _load().rms_server_destroy(srv)


__all__ = ["rms_abi_version", "rms_last_error", "rms_set_option", "rms_create_substrate", "rms_destroy_substrate",
           "rms_run", "rms_run_noalloc", "rms_run_record", "rms_spherical_mean",
           "rms_cumulant_fit",
           "rms_server_create", "rms_server_submit", "rms_server_poll",
           "rms_server_wait", "rms_server_stats_get", "rms_server_destroy", "Substrate", "RmsError", "RMS_FP64", "RMS_MIXED", "exported_symbols",
           "DUMP_FIELDS"]
