"""Pins of the oracle's absorbing membranes (magnetization transfer, end of
section 2.1.3; weight of Eq. wt-mt), CPU only.

- P_MT uses the constant C_d of Eq. (perm-prob): P_MT(rho) / rho equals the
  small-kappa limit of the permeation probability per unit kappa.
- Given a walker's membrane hits, its saturation is a product of independent
  trials, so with impermeable membranes (a single P per walker) the expected
  number of saturated walkers is sum_w 1 - (1 - P)^hits_w exactly; the count
  must fall within 4 binomial standard errors.
- Saturation draws its own words: every trajectory, counter and label equals
  the run without absorbing membranes.
- Slab pore with absorbing walls and a uniform start: the remaining weight is
  the exact series of Carslaw & Jaeger (heat loss from a slab with a
  radiation boundary): sum_n 2 L^2 / (xi_n^2 (xi_n^2 + L^2 + L))
  exp(-xi_n^2 D t / h^2), xi_n tan xi_n = L = rho h / D, h the half-width; its
  decay rate tends to the mean-field rho S/V the paper quotes.
"""
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle
from rms_inputs import cylinder_z, six_dirs

NT = oracle.host_threads()


def test_mt_probability_uses_perm_prob_constant():
    for D, dt in ((2.0, 2e-4), (0.5, 4e-4), (3.0, 1e-4)):
        k = 1e-9
        per_kappa = oracle.perm_prob(k, D, D, dt) / k
        for rho in (1e-3, 0.02, 0.3):
            assert math.isclose(oracle.mt_prob(rho, D, dt) / rho, per_kappa, rel_tol=1e-6)


def _cyl_run(rho, N=20_000, n=3000, seed=3):
    lab = cylinder_z(24, 8.0)
    R = None if rho is None else np.array([[0.0, rho[0]], [rho[1], 0.0]])
    return oracle.run(lab, 0.1, np.array([2.0, 1.5]), None, None, None, seed=seed,
                      n_walkers=N, n_steps=n, dt=2e-4, dirs=six_dirs(), n_threads=NT,
                      dump=True, rho=R)


def test_mt_saturation_count_matches_hit_counts():
    """Impermeable cylinder; walls absorb from inside (rho 0.3) and outside
    (rho 0.1)."""
    r = _cyl_run((0.1, 0.3))
    d = r["dump"]
    lab0 = d[:, 11].astype(int)
    hits = d[:, 13]
    P = np.where(lab0 == 1, oracle.mt_prob(0.3, 1.5, 2e-4), oracle.mt_prob(0.1, 2.0, 2e-4))
    p_sat = 1.0 - (1.0 - P) ** hits
    sat = np.isinf(d[:, 3])
    assert 0.1 < sat.mean() < 0.9
    want, sd = p_sat.sum(), math.sqrt(np.sum(p_sat * (1 - p_sat)))
    assert abs(sat.sum() - want) < 4 * sd
    for c in (0, 1):  # each side's own probability
        m = lab0 == c
        assert abs(sat[m].sum() - p_sat[m].sum()) < 4 * math.sqrt(np.sum(p_sat[m] * (1 - p_sat[m])))
    assert math.isclose(r["sum_alpha"], float(np.sum(~sat)), rel_tol=0, abs_tol=0)


def test_mt_leaves_trajectories_unchanged():
    a = _cyl_run((0.1, 0.3), N=3000, n=800)
    b = _cyl_run(None, N=3000, n=800)
    da, db = a["dump"], b["dump"]
    keep = [c for c in range(da.shape[1]) if c != 3]
    assert np.array_equal(da[:, keep], db[:, keep])
    assert np.all(np.isinf(da[:, 3]) | (da[:, 3] == db[:, 3]))


def _slab_survival(t, D, rho, h, n_terms=60):
    L = rho * h / D
    tot = 0.0
    for k in range(n_terms):
        lo, hi = k * math.pi + 1e-12, k * math.pi + math.pi / 2 - 1e-12
        xi = brentq(lambda x: x * math.tan(x) - L, lo, hi)
        tot += 2 * L * L / (xi * xi * (xi * xi + L * L + L)) * math.exp(-xi * xi * D * t / (h * h))
    return tot


def test_mt_slab_pore_exact_series():
    """Pore of width 2 um (20 voxels) between dead walls, periodic along y and
    z; D = 2, rho = 0.2 um/ms on both walls (L = 0.1); records at 1, 2, 4 ms.
    Tolerance: 4 binomial standard errors plus 1% of the loss for the finite
    step (ds = 0.049 um against h = 1 um)."""
    nx, w = 24, 20
    lab = np.zeros((6, 6, nx), np.uint8)
    lab[:, :, w:] = 1  # dead wall
    D, rho, dt, N = 2.0, 0.2, 2e-4, 40_000
    steps = [5000, 10000, 20000]
    r = oracle.run(lab, 0.1, np.array([D, 1.0]), None, None, np.array([0, 1], np.uint8),
                   seed=9, n_walkers=N, n_steps=20000, dt=dt, dirs=six_dirs(), n_threads=NT,
                   rec_steps=steps, rho=np.array([[0.0, rho], [0.0, 0.0]]))
    h = w * 0.1 / 2
    for k, s in enumerate(steps):
        t = s * dt
        want = _slab_survival(t, D, rho, h)
        got = r["records"]["sum_alpha"][k] / N
        tol = 4 * math.sqrt(want * (1 - want) / N) + 0.01 * (1 - want)
        assert abs(got - want) < tol, (t, got, want)
    # the long-time decay rate approaches the mean-field rho S/V (S/V = 1/h)
    lam = -(math.log(_slab_survival(4.0, D, rho, h)) - math.log(_slab_survival(3.0, D, rho, h)))
    assert abs(lam - rho / h) < 0.05 * rho / h


@pytest.mark.parametrize("bad", [-0.1, float("inf"), float("nan")])
def test_mt_rejects_bad_rho(bad):
    with pytest.raises(oracle.OracleError):
        oracle.run(cylinder_z(8, 2.0), 0.1, np.array([2.0, 2.0]), seed=1, n_walkers=4,
                   n_steps=4, dt=2e-4, rho=np.array([[0.0, bad], [0.0, 0.0]]))
