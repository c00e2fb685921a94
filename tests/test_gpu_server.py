"""The served form (continuous batching) through the C ABI.

Each request's results must be the same alone, in a mix with other requests
that arrive while it runs, and as a plain rms_run with the same arguments:
trajectories depend only on (seed, walker, step) and each request is reduced
on its own in a fixed order, so the bar is bit-identity.
"""
import time

import numpy as np
import pytest

import oracle
import paper_2012_06478_amd as rms
from rms_inputs import cylinder_z, ellipsoid_packing, pgse, six_dirs, fibonacci_hemisphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def substrates():
    lab, _ = ellipsoid_packing(n=48, n_cells=12, semi_um=(0.6, 1.4), seed=9)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.2
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    cells = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    cyl = rms.rms_create_substrate(cylinder_z(16, 5.0), 0.1, [2.0, 2.0])
    yield dict(cells=cells, cyl=cyl)
    cells.close()
    cyl.close()


def _requests(subs):
    dt = 2e-4
    n1, n2, n3 = 1500, 900, 2000
    return [
        (subs["cells"], dict(seed=5, n_walkers=3000, n_steps=n1, dt=dt,
                             waveform=pgse(n1, dt, 0.05, 0.2), dirs=fibonacci_hemisphere(9),
                             bvals=[0.0, 1.0, 2.5], precision=rms.RMS_MIXED)),
        (subs["cyl"], dict(seed=6, n_walkers=700, n_steps=n2, dt=dt,
                           waveform=np.stack([pgse(n2, dt, 0.02, 0.1), pgse(n2, dt, 0.03, 0.12)]),
                           dirs=six_dirs(), bvals=[0.0, 0.5], precision=rms.RMS_FP64)),
        (subs["cells"], dict(seed=7, n_walkers=10_000, n_steps=n3, dt=dt,
                             waveform=pgse(n3, dt, 0.1, 0.25), dirs=six_dirs(),
                             bvals=[0.0, 0.3, 1.0], precision=rms.RMS_MIXED,
                             params=dict(D=np.full(13, 1.5), kappa=None, T2=None))),
        (subs["cyl"], dict(seed=8, n_walkers=257, n_steps=0, dt=dt, dirs=six_dirs(),
                           precision=rms.RMS_FP64)),
    ]


def _same(a, b):
    for k in ("signal", "m2", "m4", "D", "K", "b_disc"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("sum_alpha", "n_face_events", "n_membrane_hits", "n_permeations"):
        assert a[k] == b[k], k


def test_server_matches_rms_run(substrates):
    reqs = _requests(substrates)
    print("[case] server vs rms_run, slice 256", flush=True)
    srv = rms.rms_server_create(0, 256)
    try:
        tickets = [rms.rms_server_submit(srv, s, **kw) for s, kw in reqs]
        results = [rms.rms_server_wait(srv, t, shape, 120.0) for t, shape in tickets]
        st = rms.rms_server_stats_get(srv)
    finally:
        rms.rms_server_destroy(srv)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["launches"] >= 8  # sliced: 2000 steps / 256
    for (s, kw), got in zip(reqs, results):
        ref = rms.rms_run(s, **kw)
        _same(got, ref)
        assert got["wall_s"] >= got["queue_s"] >= 0.0


def test_served_requests_match_the_oracle(substrates):
    """An FP64 and a mixed-precision request served together with a third one,
    each against the oracle on the same inputs: FP64 summaries within 1e-9
    (signals) and 1e-10 (moments, relative) with equal event counts; the mixed
    form's signals within 1e-3."""
    lab, _ = ellipsoid_packing(n=48, n_cells=12, semi_um=(0.6, 1.4), seed=9)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.2
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    n, dt = 1500, 2e-4
    base = dict(n_walkers=20_000, n_steps=n, dt=dt, waveform=pgse(n, dt, 0.05, 0.2),
                dirs=fibonacci_hemisphere(9), bvals=[0.0, 0.5, 1.0, 2.5])
    reqs = [dict(seed=31, precision=rms.RMS_FP64, **base),
            dict(seed=32, precision=rms.RMS_MIXED, **base)]
    srv = rms.rms_server_create(0, 400)
    try:
        print("[case] served requests vs oracle", flush=True)
        other = rms.rms_server_submit(srv, substrates["cyl"], seed=3, n_walkers=5000,
                                      n_steps=1000, dt=dt, dirs=six_dirs())
        tickets = [rms.rms_server_submit(srv, substrates["cells"], **q) for q in reqs]
        got = [rms.rms_server_wait(srv, t, sh) for t, sh in tickets]
        rms.rms_server_wait(srv, *other)
    finally:
        rms.rms_server_destroy(srv)
    for q, g in zip(reqs, got):
        kw = {k: v for k, v in q.items() if k != "precision"}
        o = oracle.run(lab, 0.1, D, kap, T2, n_threads=oracle.host_threads(), **kw)
        dS = np.max(np.abs(g["signal"] - o["signal"]))
        rel2 = np.max(np.abs(g["m2"] - o["m2"])) / np.max(np.abs(o["m2"]))
        print(f"precision {q['precision']}: max |dS| {dS:.2e}, M2 rel {rel2:.2e}", flush=True)
        if q["precision"] == rms.RMS_FP64:
            assert dS <= 1e-9 and rel2 <= 1e-10
            assert np.max(np.abs(g["m4"] - o["m4"])) <= 1e-10 * np.max(np.abs(o["m4"]))
            # the oracle's one-by-one sum of the weights: (n - 1) 2^-53 relative at most
            tol = max(1e-12, q["n_walkers"] * 2.0 ** -53)
            assert abs(g["sum_alpha"] - o["sum_alpha"]) <= tol * o["sum_alpha"]
            for k in ("n_face_events", "n_membrane_hits", "n_permeations"):
                assert g[k] == o[k], k
        else:
            assert dS <= 1e-3 and rel2 <= 1e-3


def test_alone_equals_in_mix(substrates):
    reqs = _requests(substrates)
    probe_sub, probe_kw = reqs[0]
    print("[case] alone", flush=True)
    srv = rms.rms_server_create(0, 128)
    try:
        t, shape = rms.rms_server_submit(srv, probe_sub, **probe_kw)
        alone = rms.rms_server_wait(srv, t, shape, 120.0)
    finally:
        rms.rms_server_destroy(srv)
    print("[case] mix", flush=True)
    srv = rms.rms_server_create(0, 128)
    try:
        first = [rms.rms_server_submit(srv, s, **kw) for s, kw in reqs[1:3]]
        # let the first two start, then the probe arrives while they run
        t0 = time.time()
        while rms.rms_server_stats_get(srv)["launches"] < 2 and time.time() - t0 < 30:
            time.sleep(0.001)
        t, shape = rms.rms_server_submit(srv, probe_sub, **probe_kw)
        late = [rms.rms_server_submit(srv, s, **kw) for s, kw in reqs[2:]]
        mixed = rms.rms_server_wait(srv, t, shape, 120.0)
        for tt, sh in first + late:
            rms.rms_server_wait(srv, tt, sh, 120.0)
        st = rms.rms_server_stats_get(srv)
    finally:
        rms.rms_server_destroy(srv)
    assert st["completed"] == 5
    _same(alone, mixed)


def test_admission_by_memory(substrates):
    """A budget of 3 MB holds the two small requests together but the large
    one (about 2.7 MB of walker state and records) only once the first has
    finished: it waits in line, and every result is still exact."""
    reqs = _requests(substrates)[:3]
    budget = 3_000_000
    print("[case] admission", flush=True)
    srv = rms.rms_server_create(budget, 512)
    try:
        tickets = [rms.rms_server_submit(srv, s, **kw) for s, kw in reqs]
        results = [rms.rms_server_wait(srv, t, shape, 120.0) for t, shape in tickets]
        st = rms.rms_server_stats_get(srv)
    finally:
        rms.rms_server_destroy(srv)
    assert st["completed"] == 3 and st["bytes_in_use"] == 0 and st["bytes_budget"] == budget
    # the large request was admitted only after the first one completed
    assert results[2]["queue_s"] >= results[0]["wall_s"] - 0.05
    for (s, kw), got in zip(reqs, results):
        _same(got, rms.rms_run(s, **kw))


def test_admission_by_walker_slots(substrates):
    """With 4000 walker slots the 3000- and 700-walker requests share them and
    the 10 000-walker request (more than all the slots) runs alone, after both
    have finished; every result is still exact, and the option returns to
    automatic."""
    reqs = _requests(substrates)[:3]
    print("[case] admission by walker slots", flush=True)
    rms.rms_set_option(rms.RMS_OPT_SERVER_WALKERS, 4000)
    try:
        srv = rms.rms_server_create(0, 512)
    finally:
        rms.rms_set_option(rms.RMS_OPT_SERVER_WALKERS, 0)
    try:
        tickets = [rms.rms_server_submit(srv, s, **kw) for s, kw in reqs]
        results = [rms.rms_server_wait(srv, t, shape, 120.0) for t, shape in tickets]
        st = rms.rms_server_stats_get(srv)
    finally:
        rms.rms_server_destroy(srv)
    assert st["completed"] == 3 and st["bytes_in_use"] == 0
    done_first_two = max(results[0]["wall_s"], results[1]["wall_s"])
    assert results[2]["queue_s"] >= done_first_two - 0.05
    for (s, kw), got in zip(reqs, results):
        _same(got, rms.rms_run(s, **kw))
    with pytest.raises(rms.RmsError):
        rms.rms_set_option(rms.RMS_OPT_SERVER_WALKERS, -1)


def test_server_errors(substrates):
    srv = rms.rms_server_create(1_000_000, 0)
    try:
        s, kw = _requests(substrates)[2]
        with pytest.raises(rms.RmsError) as e:
            rms.rms_server_submit(srv, s, **kw)  # needs more than the budget
        assert e.value.code == -8
        with pytest.raises(rms.RmsError) as e:
            rms.rms_server_submit(srv, s, seed=1, n_walkers=10, n_steps=10, dt=1e-3)
        assert e.value.code == -3
        small = dict(seed=1, n_walkers=64, n_steps=4000, dt=2e-4)
        t, shape = rms.rms_server_submit(srv, substrates["cyl"], **small)
        try:
            r = rms.rms_server_wait(srv, t, shape, 0.0)  # may already be done
        except rms.RmsError as err:
            assert err.code == -9
            r = rms.rms_server_wait(srv, t, shape, 120.0)
        assert r["sum_alpha"] == 64.0
    finally:
        rms.rms_server_destroy(srv)
