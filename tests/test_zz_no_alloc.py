"""rms_run_noalloc through the C ABI: the same results as rms_run, bit for
bit, on two calls in a row on one GPU, the second with fewer walkers, fewer
steps and another protocol (the scratch array keeps the first call's
contents); a run larger than the scratch array is refused before any device
work, and the next call still works."""
import numpy as np
import pytest

import paper_2012_06478_amd as rms
from rms_inputs import configs, ellipsoid_packing, pgse, fibonacci_hemisphere, six_dirs

pytestmark = pytest.mark.gpu

KEYS = ("signal", "m2", "m4", "D", "K", "sum_alpha", "b_disc", "n_face_events",
        "n_membrane_hits", "n_permeations", "max_perm_prob", "max_step_over_voxel",
        "walk_kernel")


def _same(a, b):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_noalloc_equals_run_two_calls():
    import torch
    torch.cuda.set_device(0)
    lab, _ = ellipsoid_packing(n=64, n_cells=20, semi_um=(0.6, 1.6), seed=4)
    L = int(lab.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    kap = np.zeros((L, L))
    kap[0, 1:] = kap[1:, 0] = 0.05
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    sub = rms.rms_create_substrate(lab, 0.1, D, kap, T2)
    try:
        dt = 2e-4
        n1, n2 = 1000, 600
        # 7e5 walkers take the persistent walk (1.5 to 4.5 rounds of resident
        # waves) in both forms, with its control words in the scratch array
        big = dict(seed=21, n_walkers=700_000, n_steps=n1, dt=dt,
                   waveform=pgse(n1, dt, 0.05, 0.15), dirs=fibonacci_hemisphere(30),
                   bvals=[0.0, 0.5, 1.0, 2.0])
        small = dict(seed=22, n_walkers=5_003, n_steps=n2, dt=dt,
                     waveform=pgse(n2, dt, 0.02, 0.08), dirs=six_dirs(), bvals=[0.0, 1.0],
                     dump=True)
        for prec in (rms.RMS_FP64, rms.RMS_MIXED):
            print(f"[case] noalloc vs run, precision {prec}, 700000 walkers x {n1} steps",
                  flush=True)
            a = rms.rms_run_noalloc(sub, precision=prec, **big)
            b = rms.rms_run(sub, precision=prec, **big)
            assert a["walk_kernel"] == "persistent"
            _same(a, b)
            print(f"[case] noalloc vs run, precision {prec}, 5003 walkers x {n2} steps",
                  flush=True)
            c = rms.rms_run_noalloc(sub, precision=prec, **small)
            d = rms.rms_run(sub, precision=prec, **small)
            _same(c, d)
            assert np.array_equal(c["dump"], d["dump"])
        print("[case] noalloc refuses a run larger than its scratch array", flush=True)
        with pytest.raises(rms.RmsError) as ei:
            rms.rms_run_noalloc(sub, seed=1, n_walkers=4_000_000, n_steps=10, dt=dt)
        assert "RMS_NOALLOC_MAX_BYTES" in str(ei.value)
        e = rms.rms_run_noalloc(sub, **{k: v for k, v in small.items() if k != "dump"})
        f = rms.rms_run(sub, **{k: v for k, v in small.items() if k != "dump"})
        _same(e, f)
    finally:
        sub.close()
