"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain FP64 CPU oracle.

The oracle (``rms_oracle.c``) is a slow, obviously-correct C implementation of
the Monte Carlo walk of Lee, Fieremans & Novikov, "Realistic Microstructure
Simulator" (arXiv 2012.06478), Sections 2.1-2.3.  Only ``tests/``, the smoke
check and the benchmark's CPU-baseline leg may import this package.  It shares
no code with the GPU library under ``paper_2012_06478_amd/`` and imports
nothing from it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rms_oracle.c")
_LIB = os.path.join(_HERE, "librmsoracle.so")

ERRORS = {
    -1: "invalid argument",
    -2: "label out of range",
    -3: "step too large (ds >= voxel size)",
    -4: "bad b value",
    -6: "out of memory",
    -9: "more than three face events in one step",
}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, '?')}")
        self.code = code


def build() -> str:
    """Compile the oracle with gcc (no contraction, so every operation is the
    plain IEEE double one written in the source)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    P = C.POINTER
    d_p, u32_p, u64_p, i64_p, u8_p = (P(C.c_double), P(C.c_uint32), P(C.c_uint64),
                                      P(C.c_int64), P(C.c_uint8))
    lib.rmso_philox4x32_10.argtypes = [u32_p, u32_p, u32_p]
    lib.rmso_philox4x32_10.restype = None
    lib.rmso_uniform.argtypes = [C.c_uint32]
    lib.rmso_uniform.restype = C.c_double
    lib.rmso_direction.argtypes = [C.c_uint32, C.c_uint32, d_p]
    lib.rmso_direction.restype = None
    lib.rmso_step_size.argtypes = [C.c_double, C.c_double]
    lib.rmso_step_size.restype = C.c_double
    lib.rmso_perm_prob.argtypes = [C.c_double] * 4
    lib.rmso_perm_prob.restype = C.c_double
    lib.rmso_tables.argtypes = [C.c_int, d_p, d_p, d_p, u8_p, C.c_double, C.c_double, d_p,
                                u64_p, d_p]
    lib.rmso_tables.restype = C.c_int
    lib.rmso_bscale.argtypes = [C.c_int, C.c_int64, C.c_double, d_p, C.c_int, d_p, d_p, d_p]
    lib.rmso_bscale.restype = C.c_int
    lib.rmso_single_step.argtypes = [C.c_void_p, C.c_int, i64_p, C.c_int, C.c_double,
                                     C.c_double, d_p, u64_p, d_p, i64_p, d_p, P(C.c_int), d_p,
                                     u32_p, d_p, d_p, i64_p]
    lib.rmso_single_step.restype = C.c_int
    lib.rmso_run.argtypes = [C.c_void_p, C.c_int, i64_p, C.c_double, C.c_int, d_p, d_p, d_p,
                             u8_p, C.c_uint64, C.c_int64, i64_p, C.c_int64, C.c_double, C.c_int,
                             d_p, C.c_int, d_p, C.c_int, d_p, C.c_int, d_p, d_p, d_p, d_p, d_p,
                             d_p, d_p, i64_p, d_p, C.c_int, i64_p, d_p, d_p, d_p, C.c_double,
                             C.c_int]
    lib.rmso_run.restype = C.c_int
    lib.rmso_mt_prob.argtypes = [C.c_double, C.c_double, C.c_double]
    lib.rmso_mt_prob.restype = C.c_double
    lib.rmso_conc_perm_probs.argtypes = [C.c_double] * 6 + [C.c_int, C.c_double, d_p, d_p]
    lib.rmso_conc_perm_probs.restype = None
    lib.rmso_conc_tables.argtypes = [C.c_int, d_p, d_p, u8_p, d_p, C.c_double, C.c_int,
                                     C.c_double, u64_p]
    lib.rmso_conc_tables.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib.rmso_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def uniform(w: int) -> float:
    return _load().rmso_uniform(int(w))


def direction(wa: int, wb: int) -> np.ndarray:
    v = np.zeros(3)
    _load().rmso_direction(int(wa), int(wb), _ptr(v, C.c_double))
    return v


def step_size(D: float, dt: float) -> float:
    return _load().rmso_step_size(D, dt)


def perm_prob(kappa: float, D1: float, D2: float, dt: float) -> float:
    return _load().rmso_perm_prob(kappa, D1, D2, dt)


def mt_prob(rho: float, D: float, dt: float) -> float:
    """Saturation probability at an absorbing membrane (end of section 2.1.3)."""
    return _load().rmso_mt_prob(rho, D, dt)


def conc_perm_probs(kappa, D1, D2, c1, c2, lam, model, dt):
    """(P_1->2, P_2->1) across a membrane with spin concentrations (App. C)."""
    a, b = C.c_double(), C.c_double()
    _load().rmso_conc_perm_probs(kappa, D1, D2, c1, c2, lam, model, dt, C.byref(a), C.byref(b))
    return a.value, b.value


def tables(D, kappa, T2, dead, dt, voxel_um):
    """sigma (voxel units), thresholds [n, n] (uint64), 1/T2 per label."""
    D = np.ascontiguousarray(D, np.float64)
    n = D.size
    kap = None if kappa is None else np.ascontiguousarray(kappa, np.float64).reshape(n * n)
    t2 = None if T2 is None else np.ascontiguousarray(T2, np.float64)
    dd = None if dead is None else np.ascontiguousarray(dead, np.uint8)
    sigma = np.zeros(n)
    thr = np.zeros(n * n, np.uint64)
    inv = np.zeros(n)
    rc = _load().rmso_tables(n, _ptr(D, C.c_double), _ptr(kap, C.c_double), _ptr(t2, C.c_double),
                             _ptr(dd, C.c_uint8), dt, voxel_um, _ptr(sigma, C.c_double),
                             _ptr(thr, C.c_uint64), _ptr(inv, C.c_double))
    if rc:
        raise OracleError(rc)
    return sigma, thr.reshape(n, n), inv


def conc_tables(D, kappa, dead, conc, lam, model, dt):
    """Permeation thresholds [n, n] (uint64, floor(P 2^32)) with spin
    concentrations (App. C, general case; model 1: Baxter's rule)."""
    D = np.ascontiguousarray(D, np.float64)
    n = D.size
    kap = None if kappa is None else np.ascontiguousarray(kappa, np.float64).reshape(n * n)
    dd = None if dead is None else np.ascontiguousarray(dead, np.uint8)
    cc = None if conc is None else np.ascontiguousarray(conc, np.float64)
    thr = np.zeros(n * n, np.uint64)
    rc = _load().rmso_conc_tables(n, _ptr(D, C.c_double), _ptr(kap, C.c_double),
                                  _ptr(dd, C.c_uint8), _ptr(cc, C.c_double), float(lam),
                                  int(model), dt, _ptr(thr, C.c_uint64))
    if rc:
        raise OracleError(rc)
    return thr.reshape(n, n)


def bscale(waveform, dt, bvals):
    W = np.ascontiguousarray(np.atleast_2d(waveform), np.float64)
    b = np.ascontiguousarray(bvals, np.float64)
    ns, nsteps = W.shape
    bd = np.zeros(ns)
    k = np.zeros(ns * b.size)
    rc = _load().rmso_bscale(ns, nsteps, dt, _ptr(W, C.c_double), b.size, _ptr(b, C.c_double),
                             _ptr(bd, C.c_double), _ptr(k, C.c_double))
    if rc:
        raise OracleError(rc)
    return bd, k.reshape(ns, b.size)


def single_step(labels, voxel_um, dt, sigma, thresh, inv_T2, vox, off, label, v, mwords=(0, 0, 0)):
    """One step from a hand-placed walker.  Returns a dict with the new state."""
    lab = np.ascontiguousarray(labels)
    lb = lab.dtype.itemsize
    dims = np.array(lab.shape[::-1], np.int64)  # array is [z][y][x], x fastest
    sg = np.ascontiguousarray(sigma, np.float64)
    th = np.ascontiguousarray(thresh, np.uint64).reshape(-1)
    it = np.ascontiguousarray(inv_T2, np.float64)
    vx = np.array(vox, np.int64)
    of = np.array(off, np.float64)
    lb_c = C.c_int(int(label))
    vv = np.array(v, np.float64)
    mw = np.array(mwords, np.uint32)
    dx = np.zeros(3)
    R = np.zeros(1)
    cnt = np.zeros(3, np.int64)
    rc = _load().rmso_single_step(lab.ctypes.data, lb, _ptr(dims, C.c_int64), sg.size, voxel_um,
                                  dt, _ptr(sg, C.c_double), _ptr(th, C.c_uint64),
                                  _ptr(it, C.c_double), _ptr(vx, C.c_int64), _ptr(of, C.c_double),
                                  C.byref(lb_c), _ptr(vv, C.c_double), _ptr(mw, C.c_uint32),
                                  _ptr(dx, C.c_double), _ptr(R, C.c_double),
                                  _ptr(cnt, C.c_int64))
    if rc < 0:
        raise OracleError(rc)
    return dict(vox=vx, off=of, label=lb_c.value, dx=dx, R=R[0], events=int(cnt[0]),
                hits=int(cnt[1]), perms=int(cnt[2]))


DUMP_FIELDS = ["dx", "dy", "dz", "R", "label", "ix", "iy", "iz", "ox", "oy", "oz",
               "label0", "n_face", "n_hit", "n_perm"]


def host_threads() -> int:
    """Worker threads for the oracle: the cores this process may run on, at
    most 16 (the host share of one GPU on the measurement machines)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def run(labels, voxel_um, D, kappa=None, T2=None, dead=None, *, seed, n_walkers, n_steps, dt,
        waveform=None, dirs=None, bvals=None, walker_ids=None, n_threads=None, dump=False,
        rec_steps=None, rho=None, conc=None, lam=0.0, perm_model=0):
    """Run the oracle.  ``labels`` is a [nz, ny, nx] uint8/uint16 array (x
    fastest in memory).  Returns a dict of numpy results.  ``rec_steps``
    (ascending steps in 1..n_steps) adds ``records``: sum_alpha, m2, m4, D, K
    after each of those steps (section 2.3, D(t) and K(t)).  ``rho`` [n, n]
    (surface relaxivity, um/ms, for a walker in label a meeting label b) makes
    those membranes absorbing (magnetization transfer, end of section 2.1.3):
    a saturated walker's R becomes infinite, its weight 0.  ``conc`` [n]
    (spin concentration per label), ``lam`` (the exponent of Eq.
    gen-perm-prob; negative: the minimiser) and ``perm_model`` (0: kappa, 1:
    Baxter's alternative) follow App. C's general case."""
    lib = _load()
    lab = np.ascontiguousarray(labels)
    if lab.dtype not in (np.uint8, np.uint16):
        raise TypeError("labels must be uint8 or uint16")
    dims = np.array(lab.shape[::-1], np.int64)
    D = np.ascontiguousarray(D, np.float64)
    n = D.size
    kap = None if kappa is None else np.ascontiguousarray(kappa, np.float64).reshape(n * n)
    t2 = None if T2 is None else np.ascontiguousarray(T2, np.float64)
    dd = None if dead is None else np.ascontiguousarray(dead, np.uint8)
    if waveform is None:
        W = np.zeros((0, n_steps))
    else:
        W = np.ascontiguousarray(np.atleast_2d(waveform), np.float64)
    ns = W.shape[0]
    g = np.zeros((0, 3)) if dirs is None else np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    b = np.zeros(0) if bvals is None else np.ascontiguousarray(bvals, np.float64)
    ids = None
    if walker_ids is not None:
        ids = np.ascontiguousarray(walker_ids, np.int64)
        n_walkers = ids.size
    nd, nb = g.shape[0], b.size
    sig = np.zeros(max(ns * nb * nd, 1) * 2)
    m2 = np.zeros(6)
    m4 = np.zeros(15)
    Dd = np.zeros(max(nd, 1))
    Kd = np.zeros(max(nd, 1))
    sa = np.zeros(1)
    bd = np.zeros(max(ns, 1))
    cnt = np.zeros(3, np.int64)
    K = 15 + 3 * ns
    wd = np.zeros((n_walkers, K)) if dump else None
    rh = None if rho is None else np.ascontiguousarray(rho, np.float64).reshape(n * n)
    cc = None if conc is None else np.ascontiguousarray(conc, np.float64)
    rs = None if rec_steps is None else np.ascontiguousarray(rec_steps, np.int64)
    nr = 0 if rs is None else rs.size
    ro = np.zeros(max(nr, 1) * (22 + 2 * nd))
    if n_threads is None:
        n_threads = host_threads()
    rc = lib.rmso_run(lab.ctypes.data, lab.dtype.itemsize, _ptr(dims, C.c_int64), voxel_um, n,
                      _ptr(D, C.c_double), _ptr(kap, C.c_double), _ptr(t2, C.c_double),
                      _ptr(dd, C.c_uint8), int(seed) & (2**64 - 1), int(n_walkers),
                      _ptr(ids, C.c_int64), int(n_steps), dt, ns, _ptr(W, C.c_double), nd,
                      _ptr(g, C.c_double), nb, _ptr(b, C.c_double), int(n_threads),
                      _ptr(sig, C.c_double), _ptr(m2, C.c_double), _ptr(m4, C.c_double),
                      _ptr(Dd, C.c_double), _ptr(Kd, C.c_double), _ptr(sa, C.c_double),
                      _ptr(bd, C.c_double), _ptr(cnt, C.c_int64),
                      None if wd is None else _ptr(wd, C.c_double), nr, _ptr(rs, C.c_int64),
                      _ptr(ro, C.c_double), _ptr(rh, C.c_double), _ptr(cc, C.c_double),
                      float(lam), int(perm_model))
    if rc:
        raise OracleError(rc)
    out = dict(
        signal=(sig[0::2] + 1j * sig[1::2])[: ns * nb * nd].reshape(ns, nb, nd),
        m2=m2, m4=m4, D=Dd[:nd], K=Kd[:nd], sum_alpha=sa[0], b_disc=bd[:ns],
        n_face_events=int(cnt[0]), n_membrane_hits=int(cnt[1]), n_permeations=int(cnt[2]),
    )
    if wd is not None:
        out["dump"] = wd
        out["phase"] = wd[:, 15:].reshape(n_walkers, ns, 3)
    if rs is not None:
        R = ro[: nr * (22 + 2 * nd)].reshape(nr, 22 + 2 * nd)
        out["records"] = dict(steps=rs.copy(), sum_alpha=R[:, 0].copy(), m2=R[:, 1:7].copy(),
                              m4=R[:, 7:22].copy(), D=R[:, 22:22 + nd].copy(),
                              K=R[:, 22 + nd:22 + 2 * nd].copy())
    return out
