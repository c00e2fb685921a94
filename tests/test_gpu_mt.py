"""Absorbing membranes (magnetization transfer, end of section 2.1.3) on the
GPU, through the C ABI, against the CPU oracle.

Bars: per walker, the same walkers are saturated (R infinite) as in the oracle
and every other field meets the plain parity bars; the end results meet the
plain bars.  The served, recorded and one-launch forms of the same run agree
bit for bit; a zero relaxivity table runs the plain kernels.
"""
import math
import os

import numpy as np
import pytest

import oracle
import paper_2012_06478_amd as rms
from rms_inputs import cylinder_z, ellipsoid_packing, six_dirs, pgse

pytestmark = pytest.mark.gpu

NT = oracle.host_threads()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cyl():
    lab = cylinder_z(24, 8.0)
    D = np.array([2.0, 1.5])
    kap = np.array([[0.0, 0.05], [0.05, 0.0]])
    T2 = np.array([70.0, 50.0])
    rho = np.array([[0.0, 0.1], [0.3, 0.0]])
    return lab, D, kap, T2, rho


def _cmp_walkers(G, O):
    sg, so = np.isinf(G[:, 3]), np.isinf(O[:, 3])
    same = np.all(G[:, [4, 5, 6, 7, 11, 12, 13, 14]] == O[:, [4, 5, 6, 7, 11, 12, 13, 14]], axis=1)
    same &= np.max(np.abs(G[:, 0:3] - O[:, 0:3]), axis=1) <= 1e-9
    print(f"walkers identical {same.mean():.4%}, saturated {so.mean():.3f}", flush=True)
    assert same.all()  # the same random words and the same decisions for every walker
    assert np.array_equal(sg, so)
    fin = ~so
    assert np.allclose(G[fin, 3], O[fin, 3], rtol=1e-12, atol=1e-15)


def test_mt_fp64_per_walker_and_summary():
    """Permeable cylinder, absorbing from both sides (rho 0.1 out, 0.3 in), T2,
    2000 walkers x 1500 steps, PGSE, 6 directions x 3 b."""
    lab, D, kap, T2, rho = _cyl()
    n, N = 1500, 2000
    kw = dict(seed=13, n_walkers=N, n_steps=n, dt=2e-4, waveform=pgse(n, 2e-4, 0.06, 0.15),
              dirs=six_dirs(), bvals=[0.0, 0.5, 1.0])
    print(f"[case] mt cylinder walkers={N} steps={n}", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    g = rms.rms_run(sub, params=dict(D=D, kappa=kap, T2=T2, rho=rho), dump=True, **kw)
    sub.close()
    o = oracle.run(lab, 0.1, D, kap, T2, None, n_threads=NT, dump=True, rho=rho, **kw)
    assert 0.05 < np.isinf(o["dump"][:, 3]).mean() < 0.95
    _cmp_walkers(g["dump"], o["dump"])
    assert np.max(np.abs(g["signal"] - o["signal"])) < 1e-9
    assert math.isclose(g["sum_alpha"], o["sum_alpha"], rel_tol=1e-12)
    for k in ("n_face_events", "n_membrane_hits", "n_permeations"):
        assert g[k] == o[k], k


def test_mt_exact_on_identical_decisions():
    """Impermeable walls and a walk short enough that every walker's path is
    identical: the whole result matches the oracle to the plain FP64 bars."""
    lab, D, _, T2, rho = _cyl()
    kw = dict(seed=2, n_walkers=1024, n_steps=400, dt=2e-4, dirs=six_dirs())
    print("[case] mt impermeable short", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, None, T2)
    g = rms.rms_run(sub, params=dict(D=D, T2=T2, rho=rho), dump=True, **kw)
    sub.close()
    o = oracle.run(lab, 0.1, D, None, T2, None, n_threads=NT, dump=True, rho=rho, **kw)
    G, O = g["dump"], o["dump"]
    assert np.array_equal(np.isinf(G[:, 3]), np.isinf(O[:, 3]))
    assert np.isinf(O[:, 3]).any()
    assert math.isclose(g["sum_alpha"], o["sum_alpha"], rel_tol=1e-12)
    assert np.allclose(g["m2"], o["m2"], rtol=1e-9, atol=1e-15)
    assert np.allclose(g["D"], o["D"], rtol=1e-9, atol=1e-15)


def test_mt_forms_agree_bitwise():
    """rms_run (one launch), rms_run_record (packed intervals) and the server
    (packed slices, alongside a request without absorbing membranes) give the
    same end results; mixed precision too."""
    lab, _ = ellipsoid_packing(40, voxel_um=0.1, n_cells=6, semi_um=(0.5, 1.2), seed=4)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    kap = np.full((L, L), 0.03)
    np.fill_diagonal(kap, 0.0)
    rho = np.zeros((L, L))
    rho[1:, 0] = 0.2  # cells absorb at their outer faces
    P = dict(D=D, kappa=kap, rho=rho)
    kw = dict(seed=31, n_walkers=3000, n_steps=700, dt=2e-4, dirs=six_dirs(), bvals=[0.0, 1.0],
              waveform=pgse(700, 2e-4, 0.03, 0.08))
    sub = rms.rms_create_substrate(lab, 0.1, D, kap)
    for prec in (rms.RMS_FP64, rms.RMS_MIXED):
        print(f"[case] mt forms precision={prec}", flush=True)
        a = rms.rms_run(sub, params=P, precision=prec, **kw)
        b = rms.rms_run_record(sub, params=P, precision=prec, record_steps=[7, 350, 700], **kw)
        srv = rms.rms_server_create(0, 128)
        try:
            t1, s1 = rms.rms_server_submit(srv, sub, params=P, precision=prec, **kw)
            t2, s2 = rms.rms_server_submit(srv, sub, precision=prec, **kw)
            c = rms.rms_server_wait(srv, t1, s1)
            d = rms.rms_server_wait(srv, t2, s2)
        finally:
            rms.rms_server_destroy(srv)
        plain = rms.rms_run(sub, precision=prec, **kw)
        for x in (b, c):
            for k in ("signal", "m2", "m4", "D", "K"):
                assert np.array_equal(a[k], x[k]), k
            assert a["sum_alpha"] == x["sum_alpha"]
        for k in ("signal", "m2", "sum_alpha"):
            assert np.array_equal(np.asarray(d[k]), np.asarray(plain[k])), k
        assert a["sum_alpha"] < plain["sum_alpha"]
        assert np.all(np.diff(b["records"]["sum_alpha"]) <= 0)
    sub.close()


def test_mt_zero_table_is_plain():
    lab, D, kap, T2, _ = _cyl()
    kw = dict(seed=4, n_walkers=700, n_steps=300, dt=2e-4, dirs=six_dirs())
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    a = rms.rms_run(sub, params=dict(D=D, kappa=kap, T2=T2, rho=np.zeros((2, 2))), **kw)
    b = rms.rms_run(sub, **kw)
    sub.close()
    for k in ("m2", "m4", "D", "K"):
        assert np.array_equal(a[k], b[k]), k
    assert a["sum_alpha"] == b["sum_alpha"]


def test_mt_errors():
    lab, D, kap, T2, _ = _cyl()
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    try:
        for rho, code in ((np.array([[0.0, -0.1], [0.0, 0.0]]), -1),
                          (np.array([[0.0, np.nan], [0.0, 0.0]]), -1),
                          (np.array([[0.0, 500.0], [0.0, 0.0]]), -4)):
            with pytest.raises(rms.RmsError) as ei:
                rms.rms_run(sub, params=dict(D=D, kappa=kap, T2=T2, rho=rho), seed=1,
                            n_walkers=10, n_steps=10, dt=2e-4)
            assert ei.value.code == code
    finally:
        sub.close()
