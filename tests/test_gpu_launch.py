"""Launch paths of the walk, through the C ABI.

- rms_result.walk_kernel names the kernel that ran: the persistent walk where
  the walkers fill between 1.5 and 4.5 rounds of resident waves, one launch
  elsewhere, packed launches for recorded runs;
- the one-launch and persistent kernels give the same results bit for bit
  (a walker's trajectory depends only on seed, walker and step), in both
  precision forms;
- a wave of the persistent walk that gives up its bounded wait for the
  previous segment of its walkers (forced from the host: a poll limit of 0
  with fewer walkers than one round of resident waves, so waves are handed
  items whose previous segment is still running) stops every wave: the run
  returns RMS_E_WAIT_GAVE_UP, every kernel exits, and the next run on the same
  substrate equals a clean run bit for bit.
"""
import numpy as np
import pytest

import paper_2012_06478_amd as rms
from rms_inputs import ellipsoid_packing, pgse, fibonacci_hemisphere

pytestmark = pytest.mark.gpu

KEYS = ("signal", "m2", "m4", "D", "K", "sum_alpha", "n_face_events", "n_membrane_hits",
        "n_permeations")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(autouse=True)
def _default_options():
    yield
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_AUTO)
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 1 << 20)


@pytest.fixture(scope="module")
def sub():
    lab, _ = ellipsoid_packing(n=64, n_cells=10, seed=5)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.05
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    s = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    yield s
    s.close()


def _run(sub, n_walkers, n_steps, precision=rms.RMS_FP64):
    print(f"[case] launch walkers={n_walkers} steps={n_steps} precision={precision}", flush=True)
    return rms.rms_run(sub, seed=9, n_walkers=n_walkers, n_steps=n_steps, dt=2e-4,
                       waveform=pgse(n_steps, 2e-4, n_steps * 5e-5, n_steps * 1.5e-4),
                       dirs=fibonacci_hemisphere(6), bvals=[0.0, 1.0], precision=precision)


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("precision", [rms.RMS_FP64, rms.RMS_MIXED])
def test_persistent_and_one_launch_agree_bitwise(sub, precision):
    auto = _run(sub, 1_000_000, 2100, precision)
    assert auto["walk_kernel"] == "persistent"
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_ONE_LAUNCH)
    one = _run(sub, 1_000_000, 2100, precision)
    assert one["walk_kernel"] == "one launch"
    _same(auto, one)
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_AUTO)
    small = _run(sub, 20_000, 4100, precision)
    assert small["walk_kernel"] == "one launch"
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_PERSISTENT)
    forced = _run(sub, 20_000, 4100, precision)
    assert forced["walk_kernel"] == "persistent"
    _same(small, forced)


def test_recorded_run_reports_packed_launches(sub):
    r = rms.rms_run_record(sub, seed=9, n_walkers=5000, n_steps=400, dt=2e-4,
                           record_steps=[100, 400], dirs=fibonacci_hemisphere(6), bvals=[0.0])
    assert r["walk_kernel"] == "packed"


def test_wait_that_gives_up_fails_the_run_and_nothing_else(sub):
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_PERSISTENT)
    clean = _run(sub, 20_000, 4100)
    assert clean["walk_kernel"] == "persistent"
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 0)
    with pytest.raises(rms.RmsError) as e:
        _run(sub, 20_000, 4100)
    assert e.value.code == rms.RMS_E_WAIT_GAVE_UP
    assert "gave up" in rms.rms_last_error() or "gave up" in str(e.value)
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 1 << 20)
    again = _run(sub, 20_000, 4100)
    _same(clean, again)
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_AUTO)
    _same(clean, _run(sub, 20_000, 4100))  # one launch
