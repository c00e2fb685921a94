"""Pins of the oracle's recorded moments (D(t) and K(t) at a list of steps,
section 2.3) against facts that do not come from the recording itself
(CPU only).

- The random streams are keyed by step, so the first r steps of a walk are the
  whole walk of a run of r steps: the record after step r must equal that
  run's end moments exactly (the end moments are pinned by the physics tests).
- Free diffusion: <dx_a^2> = 2 D t at every record, and after n steps the
  excess kurtosis is -6/(5n) (sum of n independent projections, each uniform
  on [-ds, ds]).
- Impermeable compartments with T2: alpha(t) = exp(-t/T2_c) for a walker in
  compartment c, so sum alpha(t) = sum_c N_c exp(-t/T2_c) to rounding; this
  fails if a record weighted by the end-of-walk R instead of R(t).
"""
import math
import os

import numpy as np
import pytest

import oracle
from rms_inputs import cylinder_z, uniform_volume, six_dirs

NT = oracle.host_threads()


def _run(labels, D, *, kappa=None, T2=None, n_walkers, n_steps, dt=2e-4, rec_steps=None,
         dump=False, seed=11):
    return oracle.run(labels, 0.1, np.asarray(D, float), kappa, T2, None, seed=seed,
                      n_walkers=n_walkers, n_steps=n_steps, dt=dt, dirs=six_dirs(),
                      n_threads=NT, rec_steps=rec_steps, dump=dump)


def test_records_equal_end_of_shorter_runs():
    """Permeable two-compartment cylinder with unequal D and T2: every record
    equals, bit for bit, the end result of the run that stops at its step."""
    lab = cylinder_z(32, 10.0)
    D, T2 = [2.0, 1.5], np.array([60.0, 80.0])
    kappa = np.array([[0.0, 0.05], [0.05, 0.0]])
    steps = [1, 2, 3, 5, 8, 13, 100, 250]
    N = 3000
    r = _run(lab, D, kappa=kappa, T2=T2, n_walkers=N, n_steps=250, rec_steps=steps)
    rec = r["records"]
    assert rec["steps"].tolist() == steps
    assert r["n_permeations"] > 0
    for k, s in enumerate(steps):
        e = _run(lab, D, kappa=kappa, T2=T2, n_walkers=N, n_steps=s)
        assert rec["sum_alpha"][k] == e["sum_alpha"]
        assert np.array_equal(rec["m2"][k], e["m2"])
        assert np.array_equal(rec["m4"][k], e["m4"])
        assert np.array_equal(rec["D"][k], e["D"])
        assert np.array_equal(rec["K"][k], e["K"])


def test_records_free_diffusion_moments_and_kurtosis():
    """Uniform volume: <dx_a^2> = 2 D t within 4 standard errors (estimated from
    the recorded fourth moment) and excess kurtosis -6/(5n) within 4 sqrt(24/N)
    (the normal-theory error of a kurtosis estimate, larger than the error for
    these platykurtic sums) after n = 1..6 and 40 steps."""
    D, dt, N = 2.0, 2e-4, 400_000
    steps = [1, 2, 3, 4, 5, 6, 40]
    r = _run(uniform_volume(8), [D], n_walkers=N, n_steps=40, dt=dt, rec_steps=steps)
    rec = r["records"]
    diag2 = [0, 3, 5]          # xx, yy, zz in the M2 order
    diag4 = [0, 10, 14]        # xxxx, yyyy, zzzz in the M4 order
    for k, n in enumerate(steps):
        t = n * dt
        assert rec["sum_alpha"][k] == N  # no T2: alpha = 1
        for a in range(3):
            m2, m4 = rec["m2"][k][diag2[a]], rec["m4"][k][diag4[a]]
            se = math.sqrt((m4 - m2 * m2) / N)
            assert abs(m2 - 2 * D * t) < 4 * se
        for d in range(6):
            assert abs(rec["K"][k][d] - (-6.0 / (5 * n))) < 4 * math.sqrt(24.0 / N)
            assert abs(rec["D"][k][d] - D) < 0.02 * D


def test_records_t2_weight_at_record_time():
    """kappa = 0, T2 = 60 / 80 ms: sum alpha(t) = sum_c N_c exp(-t / T2_c) at
    every record, with N_c the walkers that start in compartment c."""
    dt, N = 2e-4, 4000
    T2 = np.array([60.0, 80.0])
    steps = [1, 7, 64, 500, 1999, 2000]
    r = _run(cylinder_z(32, 10.0), [2.0, 2.0], T2=T2, n_walkers=N, n_steps=2000, dt=dt,
             rec_steps=steps, dump=True)
    lab0 = r["dump"][:, 11].astype(int)
    for k, s in enumerate(steps):
        t = s * dt
        want = sum(np.sum(lab0 == c) * math.exp(-t / T2[c]) for c in (0, 1))
        assert abs(r["records"]["sum_alpha"][k] - want) < 1e-12 * want


@pytest.mark.parametrize("steps", [[0], [3, 3], [5, 2], [11]])
def test_records_reject_bad_steps(steps):
    """Record steps must ascend strictly inside 1..n_steps."""
    with pytest.raises(oracle.OracleError):
        _run(uniform_volume(4), [2.0], n_walkers=10, n_steps=10, rec_steps=steps)
