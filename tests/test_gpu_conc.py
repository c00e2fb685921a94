"""Unequal spin concentrations and Baxter's permeation rule (App. C) on the
GPU, through the C ABI, against the CPU oracle.

Bars: every walker starts in the same voxel and label as in the oracle (the
concentration-weighted start draws the same words); per walker the end
state matches for at least 98% of walkers, and those to the plain FP64 bars;
the walker shares and moments agree within Monte Carlo noise of the oracle
run on the same walkers.
"""
import math
import os

import numpy as np
import pytest

import oracle
import paper_2012_06478_amd as rms
from rms_inputs import cylinder_z, six_dirs

pytestmark = pytest.mark.gpu

NT = oracle.host_threads()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


LAB = cylinder_z(24, 8.0)
D = np.array([1.2, 2.0])
CONC = np.array([0.4, 1.0])


def _pair(kappa, lam, model, precision=rms.RMS_FP64, N=3000, n=800, seed=23):
    kap = np.array([[0.0, kappa], [kappa, 0.0]])
    kw = dict(seed=seed, n_walkers=N, n_steps=n, dt=2e-4, dirs=six_dirs())
    print(f"[case] conc kappa={kappa} lam={lam} model={model} precision={precision}", flush=True)
    sub = rms.rms_create_substrate(LAB, 0.1, D, kap)
    g = rms.rms_run(sub, params=dict(D=D, kappa=kap, conc=CONC, lam=lam, perm_model=model),
                    precision=precision, dump=True, **kw)
    sub.close()
    o = oracle.run(LAB, 0.1, D, kap, None, None, n_threads=NT, dump=True, conc=CONC, lam=lam,
                   perm_model=model, **kw)
    return g, o


def _check(g, o):
    """FP64 form against the oracle: every walker takes the same path."""
    G, O = g["dump"], o["dump"]
    assert np.array_equal(G[:, 11], O[:, 11])  # start labels
    same = np.all(G[:, [4, 5, 6, 7, 12, 13, 14]] == O[:, [4, 5, 6, 7, 12, 13, 14]], axis=1)
    same &= np.max(np.abs(G[:, 0:3] - O[:, 0:3]), axis=1) <= 1e-9
    print(f"walkers identical {same.mean():.4%}, permeations {o['n_permeations']}", flush=True)
    assert same.all()
    for k in ("n_face_events", "n_membrane_hits", "n_permeations"):
        assert g[k] == o[k], k
    assert math.isclose(g["sum_alpha"], o["sum_alpha"], rel_tol=1e-12)


@pytest.mark.parametrize("lam", [-1.0, 0.0, 0.5])
def test_conc_kappa_model_parity(lam):
    g, o = _pair(2.0, lam, rms.RMS_PERM_KAPPA)
    _check(g, o)
    assert o["n_permeations"] > 1000


def test_baxter_parity():
    g, o = _pair(1.0, 0.0, rms.RMS_PERM_BAXTER)
    _check(g, o)
    assert g["max_perm_prob"] == 1.0


def test_conc_mixed_form_starts_identically():
    gm, o = _pair(2.0, -1.0, rms.RMS_PERM_KAPPA, precision=rms.RMS_MIXED, N=20_000, n=400)
    G, O = gm["dump"], o["dump"]
    assert np.array_equal(G[:, 11], O[:, 11])
    assert np.max(np.abs(G[:, 5:8] - O[:, 5:8]).sum(axis=1)[np.all(G[:, 12:15] == O[:, 12:15],
                                                                  axis=1)]) == 0
    assert np.allclose(gm["m2"], o["m2"], rtol=2e-3)


def test_conc_start_share_large():
    """1e6 walkers: the start share inside equals c_in V_in / sum c V within 4
    binomial errors (no oracle needed at this size)."""
    kap = np.array([[0.0, 0.1], [0.1, 0.0]])
    sub = rms.rms_create_substrate(LAB, 0.1, D, kap)
    N = 1_000_000
    g = rms.rms_run(sub, params=dict(D=D, kappa=kap, conc=CONC, lam=-1.0), seed=3, n_walkers=N,
                    n_steps=1, dt=2e-4, dump=True)
    sub.close()
    V = np.array([np.sum(LAB == 0), np.sum(LAB == 1)], float)
    f = CONC[1] * V[1] / (CONC @ V)
    share = np.mean(g["dump"][:, 11] == 1)
    assert abs(share - f) < 4 * np.sqrt(f * (1 - f) / N)


def test_conc_errors():
    kap = np.array([[0.0, 0.1], [0.1, 0.0]])
    sub = rms.rms_create_substrate(LAB, 0.1, D, kap)
    one = np.zeros((16, 16, 16), np.uint8)
    one[8, 8, 8] = 1
    tiny = rms.rms_create_substrate(one, 0.1, D, kap)
    try:
        bad = [(sub, dict(conc=np.array([0.0, 1.0]))), (sub, dict(conc=np.array([1.0, np.nan]))),
               (sub, dict(conc=CONC, lam=1.5)), (sub, dict(conc=CONC, perm_model=2)),
               (tiny, dict(conc=np.array([1e-6, 1.0])))]
        for s, extra in bad:
            with pytest.raises(rms.RmsError) as ei:
                rms.rms_run(s, params=dict(D=D, kappa=kap, **extra), seed=1, n_walkers=10,
                            n_steps=10, dt=2e-4)
            assert ei.value.code == -1, extra
    finally:
        sub.close()
        tiny.close()


def test_conc_forms_agree_bitwise():
    """rms_run, rms_run_record and the server (each runs the start-attempt
    kernel before its walk) give identical end results with concentrations,
    under both permeation rules."""
    kap = np.array([[0.0, 1.0], [1.0, 0.0]])
    kw = dict(seed=41, n_walkers=2500, n_steps=600, dt=2e-4, dirs=six_dirs(), bvals=[0.0, 1.0],
              waveform=np.concatenate([np.ones(150), np.zeros(300), -np.ones(150)]))
    sub = rms.rms_create_substrate(LAB, 0.1, D, kap)
    try:
        for model in (rms.RMS_PERM_KAPPA, rms.RMS_PERM_BAXTER):
            print(f"[case] conc forms model={model}", flush=True)
            P = dict(D=D, kappa=kap, conc=CONC, lam=-1.0, perm_model=model)
            a = rms.rms_run(sub, params=P, **kw)
            b = rms.rms_run_record(sub, params=P, record_steps=[1, 333, 600], **kw)
            srv = rms.rms_server_create(0, 200)
            try:
                t, shape = rms.rms_server_submit(srv, sub, params=P, **kw)
                c = rms.rms_server_wait(srv, t, shape)
            finally:
                rms.rms_server_destroy(srv)
            for x in (b, c):
                for k in ("signal", "m2", "m4", "D", "K"):
                    assert np.array_equal(a[k], x[k]), k
                for k in ("sum_alpha", "n_face_events", "n_membrane_hits", "n_permeations"):
                    assert a[k] == x[k], k
    finally:
        sub.close()
