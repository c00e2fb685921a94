"""Parity of the HIP walker (through the C ABI) with the CPU oracle.

Bars (the acceptance bars of this implementation):
  - per walker: final displacement within 1e-5 um, every integer field (end
    label and voxel, start label, event counts) identical;
  - signals within 1e-3 absolute.
The FP64 form is also held to 1e-9 on both, which is what double precision
with a different operation order gives.
"""
import math
import os

import numpy as np
import pytest

import oracle
import paper_2012_06478_amd as rms
from rms_inputs import (uniform_volume, cylinder_z, slab_x, ellipsoid_packing, pgse, six_dirs,
                        fibonacci_hemisphere, configs)

pytestmark = pytest.mark.gpu

NT = oracle.host_threads()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both(labels, vox, D, kappa=None, T2=None, dead=None, *, seed, n_walkers, n_steps, dt,
          waveform=None, dirs=None, bvals=None, dump=True, precision=rms.RMS_FP64):
    print(f"[case] labels={labels.shape}/{labels.dtype} walkers={n_walkers} steps={n_steps} "
          f"seed={seed} precision={precision}", flush=True)
    sub = rms.rms_create_substrate(labels, vox, D, kappa, T2, dead)
    g = rms.rms_run(sub, seed=seed, n_walkers=n_walkers, n_steps=n_steps, dt=dt,
                    waveform=waveform, dirs=dirs, bvals=bvals, precision=precision, dump=dump)
    sub.close()
    o = oracle.run(labels, vox, D, kappa, T2, dead, seed=seed, n_walkers=n_walkers,
                   n_steps=n_steps, dt=dt, waveform=waveform, dirs=dirs, bvals=bvals,
                   n_threads=NT, dump=dump)
    return g, o


def _assert_walkers(g, o, pos_tol):
    G, O = g["dump"], o["dump"]
    assert G.shape == O.shape
    dpos = np.max(np.abs(G[:, 0:3] - O[:, 0:3]))
    print(f"max |dx_gpu - dx_oracle| = {dpos:.3e} um", flush=True)
    assert dpos <= pos_tol
    for col in (4, 5, 6, 7, 11, 12, 13, 14):  # labels, voxel, counters
        assert np.array_equal(G[:, col], O[:, col]), rms.DUMP_FIELDS[col]
    assert np.max(np.abs(G[:, 8:11] - O[:, 8:11])) <= 1e-7
    assert np.allclose(G[:, 3], O[:, 3], rtol=1e-9, atol=1e-15)
    if G.shape[1] > 15:
        scale = max(1.0, np.max(np.abs(O[:, 15:])))
        assert np.max(np.abs(G[:, 15:] - O[:, 15:])) <= 1e-9 * scale


def _assert_summary(g, o, sig_tol):
    ds = np.max(np.abs(g["signal"] - o["signal"])) if g["signal"].size else 0.0
    print(f"max |S_gpu - S_oracle| = {ds:.3e}", flush=True)
    assert ds <= sig_tol
    assert np.allclose(g["m2"], o["m2"], rtol=1e-9, atol=1e-15)
    assert np.allclose(g["m4"], o["m4"], rtol=1e-9, atol=1e-18)
    assert np.allclose(g["D"], o["D"], rtol=1e-9, atol=1e-15)
    assert np.allclose(g["K"], o["K"], rtol=1e-7, atol=1e-9)
    assert math.isclose(g["sum_alpha"], o["sum_alpha"], rel_tol=1e-12)
    for k in ("n_face_events", "n_membrane_hits", "n_permeations"):
        assert g[k] == o[k], k
    assert np.allclose(g["b_disc"], o["b_disc"], rtol=1e-12)


def test_cylinder_tiny_per_walker():
    """32^3 u8 impermeable cylinder, 1024 walkers x 1000 steps, PGSE in the
    compressed timing, 6 directions x 4 b."""
    c = configs.cylinder_case(n_walkers=1024, n_steps=1000)
    g, o = _both(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], seed=c["seed"],
                 n_walkers=1024, n_steps=1000, dt=c["dt"], waveform=c["waveform"],
                 dirs=c["dirs"], bvals=c["bvals"])
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)
    assert np.all(g["signal"][:, 0] == 1.0)  # b = 0 exactly 1


def test_permeable_cells_ragged():
    """Small ellipsoid packing, u16, unequal D, permeable membranes, T2 per
    compartment; a walker count that fills no block."""
    lab, _ = ellipsoid_packing(n=48, n_cells=12, semi_um=(0.6, 1.4), seed=9)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.2
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    n, dt = 3000, 2e-4
    wf = np.stack([pgse(n, dt, 0.1, 0.4), -pgse(n, dt, 0.05, 0.3)])
    g, o = _both(lab, 0.1, D, kap, T2, seed=77, n_walkers=2021, n_steps=n, dt=dt, waveform=wf,
                 dirs=fibonacci_hemisphere(7), bvals=[0.0, 0.7, 3.0])
    assert o["n_permeations"] > 100
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


def test_dead_space_and_odd_steps():
    lab = slab_x(24, 3, 5, 6, 17)
    dead = np.array([1, 0], np.uint8)
    g, o = _both(lab, 0.1, np.array([2.0, 1.5]), None, None, dead, seed=3, n_walkers=300,
                 n_steps=777, dt=2e-4, dirs=six_dirs())
    assert np.all(g["dump"][:, 4] == 1) and np.all(g["dump"][:, 11] == 1)
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


def test_dead_space_on_a_volume_scanned_by_several_threads():
    """A volume above 2^22 voxels: the host lists the voxels a walker may
    start in on several threads, over contiguous ranges joined in voxel order;
    every start (an index into that list) equals the oracle's."""
    lab = cylinder_z(200, radius_vox=60.0, nz=130)  # 5.2e6 voxels
    dead = np.array([1, 0], np.uint8)
    g, o = _both(lab, 0.1, np.array([2.0, 2.0]), None, None, dead, seed=11, n_walkers=4000,
                 n_steps=64, dt=2e-4, dirs=six_dirs())
    assert np.all(g["dump"][:, 11] == 1)
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


def test_uint8_labels_beyond_flag_room():
    """uint8 volume with 46 labels: more than the uint8 device entries leave
    room for next to the halo flags, so the device volume is widened to
    uint16; permeable membranes, unequal D."""
    lab16, _ = ellipsoid_packing(n=40, n_cells=45, semi_um=(0.4, 0.9), seed=21)
    lab = lab16.astype(np.uint8)
    L = int(lab.max()) + 1
    assert L > 33
    D = np.full(L, 1.7)
    D[0] = 2.4
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.3
    n, dt = 1500, 2e-4
    g, o = _both(lab, 0.1, D, kap, None, seed=5, n_walkers=1500, n_steps=n, dt=dt,
                 waveform=pgse(n, dt, 0.05, 0.2), dirs=six_dirs(), bvals=[0.0, 1.0])
    assert o["n_permeations"] > 50
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


@pytest.mark.parametrize("dtype", [np.uint8, np.uint16])
def test_thin_axes_periodic_wrap(dtype):
    """1 x 2 x 37 voxels of random labels with permeable membranes: about a
    third of the steps cross the volume's end along x or y, so the periodic
    wrap through the device halo is taken constantly (one-voxel axis: the
    voxel is its own neighbour)."""
    rng = np.random.default_rng(11)
    lab = rng.integers(0, 3, size=(37, 2, 1)).astype(dtype)
    D = np.array([2.0, 1.2, 2.6])
    kap = np.full((3, 3), 0.5)
    np.fill_diagonal(kap, 0.0)
    n, dt = 900, 2e-4
    g, o = _both(lab, 0.1, D, kap, None, seed=8, n_walkers=700, n_steps=n, dt=dt,
                 waveform=pgse(n, dt, 0.03, 0.1), dirs=six_dirs(), bvals=[0.0, 2.0])
    assert o["n_face_events"] > 0.5 * 700 * n and o["n_permeations"] > 500
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


@pytest.mark.parametrize("n_walkers,n_steps", [(1, 0), (1, 1), (65, 2), (257, 3)])
def test_degenerate_sizes(n_walkers, n_steps):
    lab = cylinder_z(8, 3.0)
    g, o = _both(lab, 0.1, np.array([2.0, 2.0]), seed=11, n_walkers=n_walkers,
                 n_steps=n_steps, dt=2e-4, dirs=six_dirs())
    _assert_walkers(g, o, 1e-12)
    _assert_summary(g, o, 1e-12)
    if n_steps == 0:
        assert np.all(g["dump"][:, 0:3] == 0.0)


@pytest.mark.parametrize("n_walkers", [1023, 1024, 1025, 3073, 4097])
def test_reduction_fold_boundaries(n_walkers):
    """Walker counts around the reduction's fold of up to four walkers per
    thread (1024 walkers a block): every walker is counted once, so the
    summary equals the oracle's to the plain FP64 bars."""
    lab = cylinder_z(16, 5.0)
    kap = np.array([[0.0, 0.1], [0.1, 0.0]])
    n, dt = 60, 2e-4
    g, o = _both(lab, 0.1, np.array([2.0, 1.6]), kap, np.array([70.0, 50.0]), seed=31,
                 n_walkers=n_walkers, n_steps=n, dt=dt, waveform=pgse(n, dt, 0.002, 0.006),
                 dirs=six_dirs(), bvals=[0.0, 1.0, 4.0])
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


def test_four_shapes_and_anisotropic_volume():
    lab = uniform_volume(5, 7, 3)
    lab[1, 2:5, 1:4] = 1
    n, dt = 400, 2e-4
    wf = np.stack([pgse(n, dt, 0.005 * k, 0.015 * k) for k in (1, 2, 3, 4)])
    kap = np.array([[0, 0.3], [0.3, 0]])
    g, o = _both(lab, 0.1, np.array([1.0, 2.9]), kap, None, seed=2**40 + 5, n_walkers=513,
                 n_steps=n, dt=dt, waveform=wf, dirs=six_dirs(), bvals=[0.0, 0.2])
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)


def test_maximum_labels_and_signals():
    """RMS_MAX_LABELS labels and RMS_MAX_SIGNALS signals: a 64^3 u16 volume of
    4096 cubes of 4^3 voxels (labels 0..4095), D from 1.5 to 2.5 by label,
    every pair permeable (kappa 0.05); 4 shapes x 8 b x 30 directions = 960
    signals; 512 walkers x 300 steps against the oracle per walker and in
    summary.  One label or one signal more is refused with RMS_E_INVALID_ARG."""
    assert rms.RMS_MAX_LABELS == 4096 and rms.RMS_MAX_SIGNALS == 960
    i = np.arange(64) // 4
    lab = (i[:, None, None] * 256 + i[None, :, None] * 16 + i[None, None, :]).astype(np.uint16)
    L = 4096
    D = 1.5 + np.arange(L) / (L - 1)
    kap = np.full((L, L), 0.05)
    np.fill_diagonal(kap, 0.0)
    n, dt = 300, 2e-4
    wf = np.stack([pgse(n, dt, 0.004 * k, 0.01 * k) for k in (1, 2, 3, 4)])
    bvals = [0.0, 0.1, 0.2, 0.5, 1.0, 1.5, 2.0, 3.0]
    dirs = fibonacci_hemisphere(30)
    g, o = _both(lab, 0.1, D, kap, None, seed=21, n_walkers=512, n_steps=n, dt=dt, waveform=wf,
                 dirs=dirs, bvals=bvals)
    assert g["signal"].shape == (4, 8, 30) and o["n_permeations"] > 0
    _assert_walkers(g, o, 1e-9)
    _assert_summary(g, o, 1e-9)
    with pytest.raises(rms.RmsError) as ei:
        rms.rms_create_substrate(np.full((2, 2, 2), 4096, np.uint16), 0.1, np.full(L + 1, 2.0))
    assert ei.value.code == -1
    sub = rms.rms_create_substrate(lab, 0.1, D, kap)
    try:
        with pytest.raises(rms.RmsError) as ei:
            rms.rms_run(sub, seed=1, n_walkers=64, n_steps=n, dt=dt, waveform=wf,
                        dirs=fibonacci_hemisphere(31), bvals=bvals)
        assert ei.value.code == -1
    finally:
        sub.close()


def test_ellipsoid_config_full_size_sampled():
    """The 200^3 u16 permeable packing at its full size (1e6 walkers x 1e4
    steps, 30 directions x 6 b), in the launch configuration the benchmark
    times: sampled walkers match the oracle one by one, and the whole-run
    results obey what holds at any size."""
    c = configs.ellipsoid_case()
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"])
    print("[case] ellipsoids 200^3 full size", flush=True)
    g = rms.rms_run(sub, seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"],
                    dt=c["dt"], waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"],
                    dump=True)
    sub.close()
    ids = np.unique(np.linspace(0, c["n_walkers"] - 1, 97).astype(np.int64))
    o = oracle.run(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], seed=c["seed"],
                   n_walkers=ids.size, walker_ids=ids, n_steps=c["n_steps"], dt=c["dt"],
                   waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], n_threads=NT,
                   dump=True)
    G = g["dump"][ids]
    O = o["dump"]
    dpos = np.max(np.abs(G[:, 0:3] - O[:, 0:3]))
    print(f"sampled max |dx| diff {dpos:.3e} um", flush=True)
    assert dpos <= 1e-5
    for col in (4, 5, 6, 7, 11, 12, 13, 14):
        assert np.array_equal(G[:, col], O[:, col])
    S = g["signal"]
    assert np.all(S[:, 0] == 1.0)
    assert np.all(np.abs(S) <= 1.0 + 1e-12)
    # the whole-run moments are the alpha-weighted means of the dumped walkers
    dump = g["dump"]
    alpha = np.exp(-dump[:, 3])
    m2xx = np.sum(alpha * dump[:, 0] ** 2) / np.sum(alpha)
    assert math.isclose(g["m2"][0], m2xx, rel_tol=1e-9)
    assert g["n_permeations"] == int(dump[:, 14].sum())
    assert g["n_membrane_hits"] == int(dump[:, 13].sum())
    assert 0 < g["max_perm_prob"] < 0.01


def test_ellipsoid_full_walker_count_whole_result_against_oracle():
    """The 200^3 packing with its full 1e6 walkers for 4096 steps: the launch
    takes the persistent walk (two segments) and the final reduction more than
    256 blocks.  Every walker matches the oracle's, and so does the whole
    result: all 180 signals, the moments, D and K per direction."""
    c = configs.ellipsoid_case(n_steps=4096)
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"])
    print("[case] ellipsoids 200^3, 1e6 walkers x 4096 steps, whole result", flush=True)
    run = dict(seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"], dt=c["dt"],
               waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], dump=True)
    g = rms.rms_run(sub, **run)
    sub.close()
    assert g["walk_kernel"] == "persistent"
    o = oracle.run(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], n_threads=NT, **run)
    _assert_walkers(g, o, 1e-9)
    dS = np.max(np.abs(g["signal"] - o["signal"]))
    print(f"max |S - S_oracle| {dS:.3e}", flush=True)
    assert dS <= 1e-9
    assert np.allclose(g["m2"], o["m2"], rtol=1e-10, atol=0)
    assert np.allclose(g["m4"], o["m4"], rtol=1e-10, atol=1e-30)
    assert np.allclose(g["D"], o["D"], rtol=1e-10)
    assert np.allclose(g["K"], o["K"], rtol=1e-8, atol=1e-12)
    # The oracle adds the walkers' weights one by one in walker order; most
    # walkers never leave their compartment and share one of two weights, so
    # its rounding errors add up in one direction.  The bound for a recursive
    # sum of n positive terms is (n - 1) u relative (u = 2^-53).
    assert math.isclose(g["sum_alpha"], o["sum_alpha"], rel_tol=c["n_walkers"] * 2.0 ** -53)
    for k in ("n_face_events", "n_membrane_hits", "n_permeations"):
        assert g[k] == o[k], k


def test_b0_exactly_one_and_free_pins_on_gpu():
    """Closed forms checked on the GPU output directly (independent of the
    oracle): free diffusion <dx^2> = 2 D t, face-event rate 3 ds / (2 l)."""
    D, dt, n, N = 2.0, 2e-4, 300, 200_000
    sub = rms.rms_create_substrate(uniform_volume(16), 0.1, [D])
    g = rms.rms_run(sub, seed=21, n_walkers=N, n_steps=n, dt=dt, dirs=six_dirs(), dump=True)
    sub.close()
    X = g["dump"][:, 0:3]
    for a in range(3):
        x2 = X[:, a] ** 2
        assert abs(x2.mean() - 2 * D * n * dt) < 4 * x2.std() / math.sqrt(N)
    rate = g["dump"][:, 12] / n
    sigma = math.sqrt(6 * D * dt) / 0.1
    assert abs(rate.mean() - 1.5 * sigma) < 4 * rate.std() / math.sqrt(N)


def test_errors_reported():
    lab = cylinder_z(8, 3.0)
    sub = rms.rms_create_substrate(lab, 0.1, [2.0, 2.0])
    with pytest.raises(rms.RmsError) as e:
        rms.rms_run(sub, seed=1, n_walkers=10, n_steps=10, dt=1e-3)  # ds = 0.11 um > voxel
    assert e.value.code == -3
    with pytest.raises(rms.RmsError) as e:
        rms.rms_run(sub, seed=1, n_walkers=0, n_steps=10, dt=2e-4)
    assert e.value.code == -1
    with pytest.raises(rms.RmsError) as e:
        rms.rms_run(sub, seed=1, n_walkers=10, n_steps=10, dt=2e-4, waveform=np.ones(10),
                    dirs=six_dirs(), bvals=[1.0])
    assert e.value.code == -5
    with pytest.raises(rms.RmsError) as e:
        rms.rms_run(sub, seed=1, n_walkers=10, n_steps=10, dt=2e-4,
                    params=dict(D=[2.0, 2.0], kappa=[[0, 1e4], [1e4, 0]]))
    assert e.value.code == -4
    with pytest.raises(rms.RmsError) as e:  # P about 0.16: above RMS_MAX_PERM_PROB
        rms.rms_run(sub, seed=1, n_walkers=10, n_steps=10, dt=2e-4,
                    params=dict(D=[2.0, 2.0], kappa=[[0, 12.0], [12.0, 0]]))
    assert e.value.code == -4 and "RMS_MAX_PERM_PROB" in rms.rms_last_error()
    r = rms.rms_run(sub, seed=1, n_walkers=10, n_steps=10, dt=2e-4,
                    params=dict(D=[2.0, 2.0], kappa=[[0, 5.0], [5.0, 0]]))
    assert 0.05 < r["max_perm_prob"] <= rms.RMS_MAX_PERM_PROB
    sub.close()


def _sampled(c, precision, n_sample, label):
    sub = rms.rms_create_substrate(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"])
    print(f"[case] {label} full size, precision={precision}", flush=True)
    g = rms.rms_run(sub, seed=c["seed"], n_walkers=c["n_walkers"], n_steps=c["n_steps"],
                    dt=c["dt"], waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"],
                    precision=precision, dump=True)
    sub.close()
    ids = np.unique(np.linspace(0, c["n_walkers"] - 1, n_sample).astype(np.int64))
    o = oracle.run(c["labels"], c["voxel_um"], c["D"], c["kappa"], c["T2"], seed=c["seed"],
                   n_walkers=ids.size, walker_ids=ids, n_steps=c["n_steps"], dt=c["dt"],
                   waveform=c["waveform"], dirs=c["dirs"], bvals=c["bvals"], n_threads=NT,
                   dump=True)
    return g, o, ids


def test_cylinder_config_full_size_sampled():
    """The 32^3 cylinder at its full PGSE timing (delta 2 ms, Delta 10 ms: 60 000
    steps of 2e-4 ms), 1e4 walkers: sampled walkers match the oracle, b = 0 is
    exactly 1, and in the z-prism the signal along z follows the free-diffusion
    product exactly in expectation."""
    c = configs.cylinder_case()
    g, o, ids = _sampled(c, rms.RMS_FP64, 48, "cylinder")
    G, O = g["dump"][ids], o["dump"]
    assert np.max(np.abs(G[:, 0:3] - O[:, 0:3])) <= 1e-5
    for col in (4, 5, 6, 7, 11, 12, 13, 14):
        assert np.array_equal(G[:, col], O[:, col])
    assert np.all(g["signal"][0, 0] == 1.0)
    # z: reflections never touch the z motion, so S_z is the free product formula
    Q = c["dt"] * np.cumsum(c["waveform"][0][::-1])[::-1]
    bs = c["dt"] * np.sum(Q ** 2)
    ds = math.sqrt(6 * 2.0 * c["dt"])
    N = c["n_walkers"]
    for j, b in enumerate(c["bvals"]):
        S = np.prod(np.sinc(math.sqrt(b / bs) * Q * ds / np.pi))
        assert abs(g["signal"][0, j, 2].real - S) < 4 / math.sqrt(N)
    # free along the prism axis: D_zz = D0 (relative standard error ~ sqrt(2/N))
    assert abs(g["D"][2] - 2.0) < 4 * 2.0 * math.sqrt(2.0 / N)
    assert g["D"][0] < 2.0 and g["D"][1] < 2.0  # hindered or restricted across it


@pytest.mark.parametrize("precision", [rms.RMS_FP64, rms.RMS_MIXED])
def test_axon_bundle_full_size_sampled(precision):
    """The 400 x 400 x 1000 beaded-axon bundle at full size (1e7 walkers x 2e4
    steps, PGSE and OGSE, 30 directions x 6 b): sampled walkers match the
    oracle one by one (the mixed form: at least 15 of 16), and |S| <= 1."""
    c = configs.axon_case()
    g, o, ids = _sampled(c, precision, 16, "axons")
    G, O = g["dump"][ids], o["dump"]
    same = np.all(G[:, [4, 5, 6, 7, 11, 12, 13, 14]] == O[:, [4, 5, 6, 7, 11, 12, 13, 14]], axis=1)
    same &= np.max(np.abs(G[:, 0:3] - O[:, 0:3]), axis=1) <= 1e-5
    print(f"identical sampled walkers {same.sum()}/{same.size}", flush=True)
    assert same.all() if precision == rms.RMS_FP64 else same.sum() >= same.size - 1
    assert np.all(g["signal"][:, 0] == 1.0)
    assert np.all(np.abs(g["signal"]) <= 1.0 + 1e-12)
    assert g["n_permeations"] > 0
