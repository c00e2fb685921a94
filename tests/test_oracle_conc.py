"""Pins of the oracle's unequal spin concentrations (App. C, general case, and
the alternative permeation of Baxter et al.), CPU only.

- Eq. (gen-perm-prob) keeps P_1->2 / P_2->1 = c2 sqrt(D2) / (c1 sqrt(D1)) for
  every lambda, which is what holds the density ratio c1/c2 at equilibrium;
  Eq. (alt-perm-prob1-2) keeps the same ratio.
- alpha_lambda as printed is monotone in lambda, so its literal minimiser is
  an end of [0, 1]; the printed closed-form lambda is taken for the
  "minimising" option, keeps the probabilities finite as a concentration
  vanishes, and kappa0 / (1 - alpha_lambda) recovers the input kappa (Eq.
  gen-kappa-correction).
- Equal concentrations reduce to Eq. (perm-prob-general) exactly.
- A walk started with density proportional to c keeps the compartments'
  walker shares at c_i V_i / sum_j c_j V_j after several exchange times,
  with either permeation rule (4 binomial standard errors).
- The permeation flux at equilibrium, per unit membrane area and unit density
  of the side it leaves, is the effective permeability kappa' = P D / (ds C3)
  (Eq. perm-prob read backwards); with Baxter's rule P does not depend on the
  step, so kappa' scales as dt^(-1/2) (App. C), while under Eq.
  gen-perm-prob it stays near kappa.
"""
import math
import os

import numpy as np
import pytest

import oracle
from rms_inputs import cylinder_z, six_dirs

NT = oracle.host_threads()
C3 = 2.0 / 3.0


CASES = [(2.0, 1.2, 1.0, 0.4), (0.8, 2.5, 0.3, 1.0), (2.0, 2.0, 1.0, 2.0), (1.0, 3.0, 1.0, 1.0)]


@pytest.mark.parametrize("D1,D2,c1,c2", CASES)
@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, -1.0])
def test_probability_ratio_holds_equilibrium(D1, D2, c1, c2, lam):
    P12, P21 = oracle.conc_perm_probs(0.05, D1, D2, c1, c2, lam, 0, 2e-4)
    assert P12 > 0 and P21 > 0
    assert math.isclose(P12 / P21, c2 * math.sqrt(D2) / (c1 * math.sqrt(D1)), rel_tol=1e-12)


@pytest.mark.parametrize("D1,D2,c1,c2", CASES)
def test_baxter_probabilities(D1, D2, c1, c2):
    P12, P21 = oracle.conc_perm_probs(1.0, D1, D2, c1, c2, 0.0, 1, 2e-4)
    assert max(P12, P21) == 1.0
    assert math.isclose(P12 / P21, c2 * math.sqrt(D2) / (c1 * math.sqrt(D1)), rel_tol=1e-12)
    assert oracle.conc_perm_probs(0.0, D1, D2, c1, c2, 0.0, 1, 2e-4) == (0.0, 0.0)


def test_baxter_probability_one_permeates_on_every_word():
    """Baxter's rule gives probability 1 from the side of smaller c sqrt(D)
    (Eq. alt-perm-prob1-2): its threshold is 2^32, so even the largest 32-bit
    membrane word permeates; from the other side the largest word reflects."""
    D = np.array([1.0, 2.0])
    conc = np.array([1.0, 1.0])  # c sqrt(D): 1 (label 0) < sqrt 2 (label 1)
    kap = np.array([[0.0, 0.5], [0.5, 0.0]])
    thr = oracle.conc_tables(D, kap, None, conc, 0.0, 1, 2e-4)
    assert int(thr[0, 1]) == 2**32
    assert int(thr[1, 0]) == math.floor(math.sqrt(0.5) * 2**32)
    lab = np.zeros((2, 2, 2), np.uint8)
    lab[:, :, 1] = 1
    sigma, _, inv = oracle.tables(D, None, None, None, 2e-4, 0.1)
    top = 2**32 - 1
    r = oracle.single_step(lab, 0.1, 2e-4, sigma, thr, inv, [0, 0, 0], [0.99, 0.5, 0.5], 0,
                           [1.0, 0.0, 0.0], (top, 0, 0))
    assert r["hits"] == 1 and r["perms"] == 1 and r["label"] == 1
    r = oracle.single_step(lab, 0.1, 2e-4, sigma, thr, inv, [1, 0, 0], [0.01, 0.5, 0.5], 1,
                           [-1.0, 0.0, 0.0], (top, 0, 0))
    assert r["hits"] == 1 and r["perms"] == 0 and r["label"] == 1


@pytest.mark.parametrize("D1,D2,c1,c2", CASES)
def test_printed_lambda_and_kappa_correction(D1, D2, c1, c2):
    """alpha_lambda as printed is r^lambda times a constant (r = c2/c1), so on
    [0, 1] it is monotone and its minimum sits at an end; the printed closed
    form lambda = 1 / (1 + c2 sqrt(D2) / (c1 sqrt(D1))) is taken for the
    negative-lambda option (it keeps both probabilities finite as a
    concentration goes to 0, its stated purpose); the correction identity
    holds for it."""
    kappa, dt = 0.3, 2e-4
    grid = [sum(oracle.conc_perm_probs(kappa, D1, D2, c1, c2, l, 0, dt)) / 2
            for l in np.linspace(0.0, 1.0, 201)]
    d = np.diff(grid)
    assert np.all(d >= -1e-18) or np.all(d <= 1e-18)
    lam = 1.0 / (1.0 + c2 * math.sqrt(D2) / (c1 * math.sqrt(D1)))
    assert oracle.conc_perm_probs(kappa, D1, D2, c1, c2, -1.0, 0, dt) == \
        oracle.conc_perm_probs(kappa, D1, D2, c1, c2, lam, 0, dt)
    P12, P21 = oracle.conc_perm_probs(kappa, D1, D2, c1, c2, lam, 0, dt)
    ds1 = math.sqrt(6 * D1 * dt)
    k0 = P12 * D1 / (ds1 * C3 * (c2 / c1) ** lam)
    assert math.isclose(k0 / (1 - (P12 + P21) / 2), kappa, rel_tol=1e-12)


def test_printed_lambda_regular_as_concentration_vanishes():
    """With the printed lambda, P stays bounded as c1 -> 0 (for a fixed lambda
    in (0, 1] the probability out of side 1 grows without bound)."""
    prev = None
    for c1 in (1e-2, 1e-4, 1e-6, 1e-9):
        P12, P21 = oracle.conc_perm_probs(0.05, 2.0, 2.0, c1, 1.0, -1.0, 0, 2e-4)
        assert 0 < P12 < 2e-3 and 0 <= P21 < 2e-3
        if prev is not None:
            assert P21 <= prev
        prev = P21
    assert oracle.conc_perm_probs(0.05, 2.0, 2.0, 1e-9, 1.0, 0.5, 0, 2e-4)[0] == 1.0


def test_equal_concentrations_reduce_to_perm_prob_general():
    for D1, D2 in ((2.0, 1.2), (0.7, 2.4)):
        for lam in (0.0, 0.3, 1.0, -1.0):
            P12, P21 = oracle.conc_perm_probs(0.4, D1, D2, 1.7, 1.7, lam, 0, 2e-4)
            assert math.isclose(P12, oracle.perm_prob(0.4, D1, D2, 2e-4), rel_tol=1e-13)
            assert math.isclose(P21, oracle.perm_prob(0.4, D2, D1, 2e-4), rel_tol=1e-13)


@pytest.mark.parametrize("model,lam", [(0, -1.0), (0, 0.0), (1, 0.0)])
def test_walker_shares_stay_at_concentration_equilibrium(model, lam):
    """Cylinder of radius 1 um: inside c 1, D 2; outside c 0.4, D 1.2; kappa 2
    um/ms (exchange time about 0.25 ms); 40000 walkers for 5000 steps (1 ms)."""
    lab = cylinder_z(24, 10.0)
    D = np.array([1.2, 2.0])
    conc = np.array([0.4, 1.0])
    kap = np.array([[0.0, 2.0], [2.0, 0.0]])
    N = 40_000
    r = oracle.run(lab, 0.1, D, kap, None, None, seed=17, n_walkers=N, n_steps=5000, dt=2e-4,
                   dirs=six_dirs(), n_threads=NT, dump=True, conc=conc, lam=lam,
                   perm_model=model)
    V = np.array([np.sum(lab == 0), np.sum(lab == 1)], float)
    f_in = conc[1] * V[1] / (conc @ V)
    se = math.sqrt(f_in * (1 - f_in) / N)
    start_in = np.mean(r["dump"][:, 11] == 1)
    end_in = np.mean(r["dump"][:, 4] == 1)
    assert r["n_permeations"] > N  # every walker crosses about once or more
    assert abs(start_in - f_in) < 4 * se
    assert abs(end_in - f_in) < 4 * se * math.sqrt(2)


@pytest.mark.parametrize("conc", [[0.0, 1.0], [-1.0, 1.0], [np.inf, 1.0]])
def test_rejects_bad_concentrations(conc):
    with pytest.raises(oracle.OracleError):
        oracle.run(cylinder_z(8, 2.0), 0.1, np.array([2.0, 2.0]),
                   np.array([[0.0, 0.1], [0.1, 0.0]]), seed=1, n_walkers=4, n_steps=4,
                   dt=2e-4, conc=np.array(conc))


@pytest.mark.parametrize("model,kappa", [(1, 1.0), (0, 2.0)])
def test_permeation_flux_scaling_with_step(model, kappa):
    """Two slabs 1 um wide (labels 0 | 1, periodic along x: two membranes of
    0.4 x 0.4 um), D 2 on both sides, c 1 and 0.3; 20000 walkers started at the
    concentration equilibrium walk 0.4 ms at dt = 2e-4 and 8e-4 ms.  The
    permeation count equals sum over sides of kappa'_side N_side / V_side x A x
    T within 4 Poisson errors plus 0.5%; Baxter's count halves when dt grows
    four-fold (kappa' ~ dt^(-1/2)), the kappa rule's follows its P/ds."""
    w, ny, lp = 10, 4, 0.1
    lab = np.zeros((ny, ny, 2 * w), np.uint8)
    lab[:, :, w:] = 1
    D = np.array([2.0, 2.0])
    conc = np.array([1.0, 0.3])
    kap = np.array([[0.0, kappa], [kappa, 0.0]])
    N, T = 20_000, 0.4
    V = w * lp * (ny * lp) ** 2      # each slab's volume
    A = 2 * (ny * lp) ** 2           # both membranes
    got, want = [], []
    for dt in (2e-4, 8e-4):
        n = int(round(T / dt))
        r = oracle.run(lab, lp, D, kap, None, None, seed=11, n_walkers=N, n_steps=n, dt=dt,
                       dirs=six_dirs(), n_threads=NT, dump=True, conc=conc, perm_model=model)
        P01, P10 = oracle.conc_perm_probs(kappa, D[0], D[1], conc[0], conc[1], 0.0, model, dt)
        ds = math.sqrt(6 * D[0] * dt)
        n0 = int(np.sum(r["dump"][:, 11] == 0))
        flux = sum(P * D[0] / (ds * C3) * m / V for P, m in ((P01, n0), (P10, N - n0)))
        e = flux * A * n * dt
        assert abs(r["n_permeations"] - e) < 4 * math.sqrt(e) + 0.005 * e, (dt, r["n_permeations"], e)
        got.append(r["n_permeations"])
        want.append(e)
    if model == 1:
        assert math.isclose(want[0] / want[1], 2.0, rel_tol=1e-3)
    else:
        assert abs(want[0] / want[1] - 1.0) < 0.1
    assert abs(got[0] / got[1] - want[0] / want[1]) < 0.03 * want[0] / want[1]
