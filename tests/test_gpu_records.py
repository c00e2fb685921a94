"""Displacement moments recorded during the walk (rms_run_record) on the GPU,
against the CPU oracle's records and against rms_run.

Bars: the FP64 records agree with the oracle's as the end moments do (1e-9
relative, sum of alpha 1e-12); the end results of rms_run_record equal
rms_run's bit for bit in both precision forms (the walk is the same
trajectories cut at the record steps); the mixed form's records are within
the mixed form's bars of the FP64 ones.  At full size, where the oracle cannot
run, the records are checked for properties that hold at any size.
"""
import math
import os

import numpy as np
import pytest

import oracle
import paper_2012_06478_amd as rms
from rms_inputs import cylinder_z, ellipsoid_packing, six_dirs, pgse, configs

pytestmark = pytest.mark.gpu

NT = oracle.host_threads()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cells():
    lab, _ = ellipsoid_packing(40, voxel_um=0.1, n_cells=6, semi_um=(0.5, 1.2), seed=4)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.full((L, L), 0.05)
    np.fill_diagonal(kap, 0.0)
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    return lab, D, kap, T2


def _assert_records_close(a, b, rtol):
    assert np.array_equal(a["steps"], b["steps"])
    assert np.allclose(a["sum_alpha"], b["sum_alpha"], rtol=max(rtol, 1e-12), atol=0)
    assert np.allclose(a["m2"], b["m2"], rtol=rtol, atol=1e-15)
    assert np.allclose(a["m4"], b["m4"], rtol=rtol, atol=1e-18)
    assert np.allclose(a["D"], b["D"], rtol=rtol, atol=1e-15)
    assert np.allclose(a["K"], b["K"], rtol=100 * rtol, atol=100 * rtol)


def _same_end(a, b):
    for k in ("signal", "m2", "m4", "D", "K", "b_disc"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("sum_alpha", "n_face_events", "n_membrane_hits", "n_permeations"):
        assert a[k] == b[k], k


def test_records_match_oracle_and_run_fp64():
    """Permeable cells with unequal D and T2, 1500 walkers (a ragged last block)
    x 600 steps, records at steps that start intervals inside a Philox block."""
    lab, D, kap, T2 = _cells()
    n, N = 600, 1500
    steps = [1, 2, 3, 5, 7, 64, 301, 599, 600]
    wf = pgse(n, 2e-4, 0.03, 0.06)
    kw = dict(seed=21, n_walkers=N, n_steps=n, dt=2e-4, waveform=wf, dirs=six_dirs(),
              bvals=[0.0, 0.5, 1.0])
    print(f"[case] cells {lab.shape} walkers={N} steps={n} records={steps}", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    g = rms.rms_run_record(sub, record_steps=steps, dump=True, **kw)
    e = rms.rms_run(sub, dump=True, **kw)
    sub.close()
    o = oracle.run(lab, 0.1, D, kap, T2, None, n_threads=NT, rec_steps=steps, **kw)
    assert g["n_permeations"] > 0
    _same_end(g, e)
    assert np.array_equal(g["dump"], e["dump"])
    _assert_records_close(g["records"], o["records"], 1e-9)
    # the record at the last step is the end moments
    assert g["records"]["sum_alpha"][-1] == g["sum_alpha"]
    assert np.array_equal(g["records"]["m2"][-1], g["m2"])
    assert np.array_equal(g["records"]["D"][-1], g["D"])


@pytest.mark.parametrize("steps", [[1], [599], [4, 8, 12], [3]])
def test_records_few_steps_match_oracle(steps):
    """A single record before the end, records on block boundaries, a record at
    the first step; 257 walkers x 600 steps on a two-compartment cylinder."""
    lab = cylinder_z(24, 7.0)
    D, T2 = [2.0, 1.7], np.array([70.0, 50.0])
    kap = np.array([[0.0, 0.04], [0.04, 0.0]])
    kw = dict(seed=5, n_walkers=257, n_steps=600, dt=2e-4, dirs=six_dirs())
    print(f"[case] cylinder records={steps}", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    g = rms.rms_run_record(sub, record_steps=steps, **kw)
    e = rms.rms_run(sub, **kw)
    sub.close()
    o = oracle.run(lab, 0.1, D, kap, T2, None, n_threads=NT, rec_steps=steps, **kw)
    _same_end(g, e)
    _assert_records_close(g["records"], o["records"], 1e-9)


def test_records_mixed_form():
    """Mixed form: its end results equal its rms_run bit for bit, and its records
    are within 1e-4 of the FP64 records (the mixed form's moment bar)."""
    lab, D, kap, T2 = _cells()
    steps = [3, 50, 199, 400]
    kw = dict(seed=8, n_walkers=4000, n_steps=400, dt=2e-4, dirs=six_dirs())
    print(f"[case] mixed records={steps}", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    gm = rms.rms_run_record(sub, record_steps=steps, precision=rms.RMS_MIXED, **kw)
    em = rms.rms_run(sub, precision=rms.RMS_MIXED, **kw)
    gd = rms.rms_run_record(sub, record_steps=steps, **kw)
    sub.close()
    _same_end(gm, em)
    a, b = gm["records"], gd["records"]
    assert np.allclose(a["sum_alpha"], b["sum_alpha"], rtol=1e-6)
    scale2 = np.max(np.abs(b["m2"]), axis=1, keepdims=True)
    assert np.max(np.abs(a["m2"] - b["m2"]) / scale2) < 1e-4
    assert np.max(np.abs(a["D"] - b["D"]) / np.abs(b["D"])) < 1e-4


def test_records_full_size_properties():
    """Ellipsoid packing 200^3, 1e6 walkers x 1e4 steps, 50 records: the record
    at the last step equals rms_run's end moments bit for bit; sum alpha never
    grows (R is non-decreasing per walker); M2 is positive definite; D(t) stays
    within the compartments' D0 range."""
    c = configs.ellipsoid_case()
    steps = list(range(200, c["n_steps"] + 1, 200))
    kw = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
              waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"])
    print(f"[case] ellipsoids200 full size, {len(steps)} records", flush=True)
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"])
    g = rms.rms_run_record(sub, record_steps=steps, **kw)
    e = rms.rms_run(sub, **kw)
    sub.close()
    print(f"record run {g['kernel_ms']:.1f} ms, plain run {e['kernel_ms']:.1f} ms", flush=True)
    _same_end(g, e)
    r = g["records"]
    assert r["sum_alpha"][-1] == e["sum_alpha"]
    assert np.array_equal(r["m2"][-1], e["m2"])
    assert np.array_equal(r["m4"][-1], e["m4"])
    assert np.all(np.diff(r["sum_alpha"]) < 0)
    for k in range(len(steps)):
        m = r["m2"][k]
        M = np.array([[m[0], m[1], m[2]], [m[1], m[3], m[4]], [m[2], m[4], m[5]]])
        assert np.all(np.linalg.eigvalsh(M) > 0)
    Dmax = float(np.max(c["D"]))
    assert np.all(r["D"] > 0) and np.all(r["D"] < Dmax)


@pytest.mark.parametrize("precision", [rms.RMS_FP64, rms.RMS_MIXED])
def test_even_records_match_oracle(precision):
    """Records every 150 steps (not a multiple of 4: intervals start inside a
    Philox block) match the oracle's (FP64 to 1e-9, mixed within its bar of
    the FP64 records) and the end results equal rms_run's."""
    lab, D, kap, T2 = _cells()
    steps = [150, 300, 450, 600, 750]
    kw = dict(seed=17, n_walkers=2000, n_steps=800, dt=2e-4, dirs=six_dirs(), bvals=[0.0, 1.0],
              waveform=pgse(800, 2e-4, 0.04, 0.08))
    print(f"[case] even records {steps} precision={precision}", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    g = rms.rms_run_record(sub, record_steps=steps, precision=precision, **kw)
    e = rms.rms_run(sub, precision=precision, **kw)
    gd = rms.rms_run_record(sub, record_steps=steps, **kw)
    sub.close()
    _same_end(g, e)
    if precision == rms.RMS_FP64:
        o = oracle.run(lab, 0.1, D, kap, T2, None, n_threads=NT, rec_steps=steps, **kw)
        _assert_records_close(g["records"], o["records"], 1e-9)
    else:
        a, b = g["records"], gd["records"]
        assert np.allclose(a["sum_alpha"], b["sum_alpha"], rtol=1e-6)
        assert np.max(np.abs(a["m2"] - b["m2"]) / np.max(np.abs(b["m2"]))) < 1e-4


def test_records_full_size_uneven():
    """Records at uneven steps at full size: the end results equal rms_run's bit
    for bit and sum alpha decreases."""
    c = configs.ellipsoid_case()
    steps = [37, 500, 2001, 4444, 7000, 9999]
    kw = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
              waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"])
    print("[case] ellipsoids200 full size, uneven records", flush=True)
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"])
    g = rms.rms_run_record(sub, record_steps=steps, **kw)
    e = rms.rms_run(sub, **kw)
    sub.close()
    _same_end(g, e)
    assert np.all(np.diff(g["records"]["sum_alpha"]) < 0)


def test_records_errors():
    """Malformed record lists and more than RMS_MAX_RECORDS records are refused
    with RMS_E_INVALID_ARG; exactly RMS_MAX_RECORDS records (one per step) run."""
    sub = rms.rms_create_substrate(cylinder_z(16, 5.0), 0.1, [2.0, 2.0])
    try:
        for steps in ([], [0], [5, 5], [7, 3], [11]):
            with pytest.raises(rms.RmsError) as ei:
                rms.rms_run_record(sub, seed=1, n_walkers=10, n_steps=10, dt=2e-4,
                                   record_steps=steps)
            assert ei.value.code == -1, steps
        with pytest.raises(rms.RmsError) as ei:  # one record more than RMS_MAX_RECORDS
            rms.rms_run_record(sub, seed=1, n_walkers=10, n_steps=5000, dt=2e-4,
                               record_steps=list(range(1, 4098)))
        assert ei.value.code == -1
        g = rms.rms_run_record(sub, seed=1, n_walkers=64, n_steps=4096, dt=2e-4,
                               record_steps=list(range(1, 4097)))
        assert g["records"]["m2"].shape == (4096, 6)
    finally:
        sub.close()


@pytest.mark.parametrize("precision", [rms.RMS_FP64, rms.RMS_MIXED])
def test_long_walk_persistent_equals_packed(precision):
    """700000 walkers (2.1 rounds of resident waves FP64, 1.8 mixed: the
    persistent walk) x 70000 steps (segments capped at 4096 steps: 18
    segments): rms_run equals the packed intervals of rms_run_record bit for
    bit."""
    lab = cylinder_z(24, 7.0)
    D, kap = [2.0, 1.7], np.array([[0.0, 0.02], [0.02, 0.0]])
    kw = dict(seed=12, n_walkers=700_000, n_steps=70_000, dt=2e-4, dirs=six_dirs(),
              bvals=[0.0, 1.0], waveform=pgse(70_000, 2e-4, 2.0, 10.0), precision=precision)
    print(f"[case] long walk 7e5 x 7e4 precision={precision}", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap)
    e = rms.rms_run(sub, **kw)
    g = rms.rms_run_record(sub, record_steps=[35_001, 70_000], **kw)
    sub.close()
    _same_end(g, e)
    assert g["n_permeations"] > 0


def test_records_on_a_torch_stream():
    """rms_run_record on a torch stream of the caller (its own second stream
    joins it) equals the run on the null stream bit for bit, and leaves the
    caller's stream usable."""
    import torch
    lab, D, kap, T2 = _cells()
    kw = dict(seed=19, n_walkers=5000, n_steps=500, dt=2e-4, dirs=six_dirs(), bvals=[0.0, 1.0],
              waveform=pgse(500, 2e-4, 0.03, 0.06))
    print("[case] records on a torch stream", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    try:
        a = rms.rms_run_record(sub, record_steps=[50, 250, 499], **kw)
        s = torch.cuda.Stream()
        b = rms.rms_run_record(sub, record_steps=[50, 250, 499], stream=s, **kw)
        with torch.cuda.stream(s):
            x = torch.ones(1000, device="cuda", dtype=torch.float64).sum()
        s.synchronize()
        assert float(x) == 1000.0
    finally:
        sub.close()
    _same_end(a, b)
    for k in ("sum_alpha", "m2", "m4", "D", "K"):
        assert np.array_equal(a["records"][k], b["records"][k]), k
