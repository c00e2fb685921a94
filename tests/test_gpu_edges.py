"""Edge cases of rms_run against the oracle (through the C ABI): a walk of
zero steps (the start alone), a single walker, walks whose step count is not
a multiple of the four steps a membrane-word block serves, the largest
number of gradient shapes, runs with no shape or no direction, and walker
counts one either side of a block of 256 threads.  FP64 bars as in
test_gpu_parity.py: every integer field identical, displacements and phases
within 1e-9, signals within 1e-9; the mixed form within 1e-3 on signals."""
import numpy as np
import pytest

import oracle
import paper_2012_06478_amd as rms
from rms_inputs import ellipsoid_packing, cylinder_z, pgse, six_dirs, fibonacci_hemisphere

pytestmark = pytest.mark.gpu

NT = oracle.host_threads()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def cells():
    lab, _ = ellipsoid_packing(n=40, n_cells=8, semi_um=(0.6, 1.2), seed=12)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.3
    T2 = np.full(L, 70.0)
    T2[0] = 50.0
    return lab, D, kap, T2


def _pair(tissue, *, precision=rms.RMS_FP64, **run):
    lab, D, kap, T2 = tissue
    print(f"[case] walkers={run['n_walkers']} steps={run['n_steps']} precision={precision}",
          flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    try:
        g = rms.rms_run(sub, precision=precision, dump=True, **run)
    finally:
        sub.close()
    o = oracle.run(lab, 0.1, D, kap, T2, n_threads=NT, dump=True, **run)
    return g, o


def _same_walkers(g, o):
    G, O = g["dump"], o["dump"]
    assert G.shape == O.shape
    for col in (4, 5, 6, 7, 11, 12, 13, 14):
        assert np.array_equal(G[:, col], O[:, col]), rms.DUMP_FIELDS[col]
    assert np.max(np.abs(G[:, 0:3] - O[:, 0:3]), initial=0.0) <= 1e-9
    assert np.allclose(G[:, 3], O[:, 3], rtol=1e-9, atol=1e-15)
    if G.shape[1] > 15:
        scale = max(1.0, np.max(np.abs(O[:, 15:])))
        assert np.max(np.abs(G[:, 15:] - O[:, 15:])) <= 1e-9 * scale


def _same_summary(g, o, tol=1e-9):
    if o["signal"].size:
        assert np.max(np.abs(g["signal"] - o["signal"])) <= tol
    assert np.allclose(g["m2"], o["m2"], rtol=1e-9, atol=1e-18)
    for k in ("n_face_events", "n_membrane_hits", "n_permeations"):
        assert g[k] == o[k], k


def test_zero_steps_is_the_start(cells):
    """No step: every walker is at its start (zero displacement, the start
    voxel and offset the oracle draws, weight 1)."""
    g, o = _pair(cells, seed=3, n_walkers=777, n_steps=0, dt=2e-4)
    _same_walkers(g, o)
    assert np.all(g["dump"][:, 0:3] == 0.0) and np.all(g["dump"][:, 12:15] == 0.0)
    assert np.array_equal(g["dump"][:, 8:11], o["dump"][:, 8:11])
    assert np.all(g["m2"] == 0.0)
    assert g["sum_alpha"] == 777.0


@pytest.mark.parametrize("n_steps", [1, 2, 3, 5, 7, 1001])
def test_step_counts_off_the_word_blocks(cells, n_steps):
    """Step counts that end inside a direction block (odd) or a membrane-word
    block (not a multiple of four)."""
    short = {1: None, 2: [1.0, -1.0], 3: [1.0, 0.0, -1.0]}
    wf = (short[n_steps] if n_steps in short
          else pgse(n_steps, 2e-4, n_steps * 5e-5, n_steps * 1.5e-4))
    g, o = _pair(cells, seed=11, n_walkers=3000, n_steps=n_steps, dt=2e-4, dirs=six_dirs(),
                 bvals=[0.0, 0.5] if wf is not None else None, waveform=wf)
    _same_walkers(g, o)
    _same_summary(g, o)


def test_single_walker(cells):
    g, o = _pair(cells, seed=99, n_walkers=1, n_steps=5000, dt=2e-4,
                 waveform=pgse(5000, 2e-4, 0.2, 0.6), dirs=six_dirs(), bvals=[0.0, 1.0])
    _same_walkers(g, o)
    _same_summary(g, o)


def test_four_shapes_and_many_directions(cells):
    """RMS_MAX_SHAPES shapes, per-walker phase vectors of every shape."""
    n, dt = 1200, 2e-4
    assert rms.RMS_MAX_SHAPES == 4
    wf = np.stack([pgse(n, dt, 0.02, 0.1), -pgse(n, dt, 0.05, 0.15),
                   pgse(n, dt, 0.01, 0.2), pgse(n, dt, 0.03, 0.06, start=0.02)])
    g, o = _pair(cells, seed=5, n_walkers=2500, n_steps=n, dt=dt, waveform=wf,
                 dirs=fibonacci_hemisphere(40), bvals=[0.0, 0.3, 1.0, 3.0])
    _same_walkers(g, o)
    _same_summary(g, o)
    assert g["signal"].shape == (4, 4, 40)


def test_no_shape_and_no_direction(cells):
    """Moments only (no signal), and a run with neither shapes nor
    directions (sum of weights and counters)."""
    g, o = _pair(cells, seed=6, n_walkers=2000, n_steps=800, dt=2e-4, dirs=six_dirs())
    _same_walkers(g, o)
    _same_summary(g, o)
    assert g["signal"].size == 0 and np.allclose(g["D"], o["D"], rtol=1e-9)
    g, o = _pair(cells, seed=6, n_walkers=2000, n_steps=800, dt=2e-4)
    _same_walkers(g, o)
    assert g["D"].size == 0 and abs(g["sum_alpha"] - o["sum_alpha"]) <= 1e-12 * o["sum_alpha"]


@pytest.mark.parametrize("n_walkers", [255, 256, 257, 64 * 1024 + 1])
def test_walker_counts_around_blocks(cells, n_walkers):
    g, o = _pair(cells, seed=21, n_walkers=n_walkers, n_steps=300, dt=2e-4,
                 waveform=pgse(300, 2e-4, 0.01, 0.04), dirs=six_dirs(), bvals=[0.0, 1.0])
    _same_walkers(g, o)
    _same_summary(g, o)


def test_mixed_form_edges(cells):
    """The mixed form on the odd step count and the single walker: integer
    fields as the oracle's for nearly every walker, signals within 1e-3."""
    for n_walkers, n_steps in ((3000, 7), (1, 5000)):
        wf = pgse(n_steps, 2e-4, n_steps * 5e-5, n_steps * 1.5e-4) if n_steps > 4 else None
        g, o = _pair(cells, precision=rms.RMS_MIXED, seed=13, n_walkers=n_walkers,
                     n_steps=n_steps, dt=2e-4, waveform=wf, dirs=six_dirs(),
                     bvals=[0.0, 0.5] if wf is not None else None)
        same = np.all(g["dump"][:, [4, 5, 6, 7, 11]] == o["dump"][:, [4, 5, 6, 7, 11]], axis=1)
        assert same.mean() >= 0.99
        if o["signal"].size:
            assert np.max(np.abs(g["signal"] - o["signal"])) <= 1e-3
        assert np.max(np.abs(g["dump"][same, 0:3] - o["dump"][same, 0:3])) <= 1e-5


def test_walker_count_limit(cells):
    """Walker indices are 32-bit (2^32 - 1 marks an empty thread slot): a run
    of 2^32 - 1 walkers is refused before anything is allocated, and the next
    run on the same substrate is unaffected."""
    lab, D, kap, T2 = cells
    print("[case] walker count limit", flush=True)
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    try:
        with pytest.raises(rms.RmsError) as e:
            rms.rms_run(sub, seed=1, n_walkers=2**32 - 1, n_steps=10, dt=2e-4)
        assert e.value.code == -1 and "2^32 - 2" in str(e.value)
        r = rms.rms_run(sub, seed=1, n_walkers=300, n_steps=10, dt=2e-4)
        assert r["n_face_events"] > 0
    finally:
        sub.close()
