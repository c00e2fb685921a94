"""Statistical pins of the oracle's whole walk against closed forms and
independent references (CPU only).

Every expectation below is exact for the discrete walk or an exact solution
of the diffusion problem the walk approximates; tolerances are 4 Monte Carlo
standard errors (estimated from the same sample) unless stated otherwise.
"""
import math
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.stats import chi2

import oracle
from rms_inputs import uniform_volume, cylinder_z, slab_x, pgse, six_dirs

NT = oracle.host_threads()
INF = float("inf")


def _run(labels, D, *, kappa=None, T2=None, dead=None, seed=5, n_walkers, n_steps, dt=2e-4,
         waveform=None, dirs=None, bvals=None, dump=True, vox=0.1):
    return oracle.run(labels, vox, np.asarray(D, float), kappa, T2, dead, seed=seed,
                      n_walkers=n_walkers, n_steps=n_steps, dt=dt, waveform=waveform, dirs=dirs,
                      bvals=bvals, dump=dump, n_threads=NT)


def _kurtosis_and_se(x):
    """Excess kurtosis of a zero-mean sample and its delta-method standard
    error."""
    m2, m4, m6, m8 = (np.mean(x ** k) for k in (2, 4, 6, 8))
    K = m4 / m2 ** 2 - 3.0
    var = ((m8 - m4 ** 2) / m2 ** 4 - 4 * m4 * (m6 - m4 * m2) / m2 ** 5
           + 4 * m4 ** 2 * (m4 - m2 ** 2) / m2 ** 6) / x.size
    return K, math.sqrt(var)


# -------------------------------------------------------------- free space --

@pytest.mark.parametrize("n_steps,n_walkers", [(1, 200_000), (2, 200_000), (5, 100_000),
                                               (300, 40_000)])
def test_free_diffusion_moments(n_steps, n_walkers):
    """Uniform volume: each step's projection on any fixed axis is uniform on
    [-ds, ds], so <dx_a^2> = 2 D t exactly and the excess kurtosis after n
    steps is -6/(5n) (section 2.1.3 Eq. step-size; section 2.3)."""
    D, dt = 2.0, 2e-4
    r = _run(uniform_volume(8), [D], n_walkers=n_walkers, n_steps=n_steps, dt=dt,
             dirs=six_dirs())
    t = n_steps * dt
    X = r["dump"][:, 0:3]
    for a in range(3):
        x2 = X[:, a] ** 2
        assert abs(x2.mean() - 2 * D * t) < 4 * x2.std() / math.sqrt(x2.size)
    G = six_dirs()
    for d in range(6):
        p = X @ G[d]
        K, se = _kurtosis_and_se(p)
        assert abs(K - (-6.0 / (5 * n_steps))) < 4 * se
        assert abs(r["K"][d] - K) < 1e-9  # the oracle's own output is the same estimator
        assert abs(r["D"][d] - np.mean(p ** 2) / (2 * t)) < 1e-12 * D


def test_free_signal_exact_product():
    """Uniform volume: phi = sum_k q_k (g . dx_k) with independent uniform
    projections, so S = prod_k sin(q_k ds)/(q_k ds) exactly, with q_k = k Q_k
    and Q_k = dt sum_{i>=k} G_i (section 2.3, Eq. signal)."""
    D, dt, n = 2.0, 2e-4, 100
    G = pgse(n, dt, 20 * dt, 60 * dt)
    b = np.array([0.0, 0.001, 0.003, 0.006])
    N = 200_000
    r = _run(uniform_volume(8), [D], n_walkers=N, n_steps=n, dt=dt, waveform=G,
             dirs=six_dirs(), bvals=b)
    Q = dt * np.cumsum(G[::-1])[::-1]
    bs = dt * np.sum(Q ** 2)
    ds = math.sqrt(6 * D * dt)
    for j, bj in enumerate(b):
        q = math.sqrt(bj / bs) * Q * ds
        S = np.prod(np.sinc(q / np.pi))
        for d in range(6):
            got = r["signal"][0, j, d]
            assert abs(got.real - S) < 4 / math.sqrt(N)
            assert abs(got.imag) < 4 / math.sqrt(N)
    assert np.all(r["signal"][0, 0] == 1.0 + 0.0j)  # b = 0 is exactly 1 (section 2.3)
    assert abs(r["b_disc"][0] - bs) < 1e-15


def test_face_event_rate():
    """Uniform volume: along an axis a step crosses ds |v_a| / l_p faces on
    average, |v_a| being uniform on [0, 1]; three axes give 3 ds / (2 l_p)."""
    D, dt, n, N = 2.0, 2e-4, 500, 20_000
    r = _run(uniform_volume(8), [D], n_walkers=N, n_steps=n, dt=dt)
    per_walker = r["dump"][:, 12] / n
    sigma = math.sqrt(6 * D * dt) / 0.1
    assert abs(per_walker.mean() - 1.5 * sigma) < 4 * per_walker.std() / math.sqrt(N)
    assert r["n_membrane_hits"] == 0


# ---------------------------------------------------------------- membranes --

def _golden(name):
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_worked_values.txt")
    for line in open(path):
        if line.startswith(name + " "):
            return float(line.split()[1])
    raise KeyError(name)


def test_flat_membrane_hit_fraction():
    """Appendix C.1 after Eq. (flux1-2): at a flat membrane, a fraction
    (2 d C_d)^-1 = 1/4 of the walkers within ds of it meet it in a step.
    With two planes, both sides and uniform density: hits per walker-step
    = 4 (1/4) ds / L_x."""
    D, dt, n, N = 2.0, 2e-4, 500, 20_000
    nx = 20
    r = _run(slab_x(nx, 4, 4, 5, 15), [D, D], kappa=np.zeros((2, 2)), n_walkers=N,
             n_steps=n, dt=dt)
    sigma = math.sqrt(6 * D * dt) / 0.1
    want = 4 * _golden("hit_fraction_3d") * sigma / nx
    per_walker = r["dump"][:, 13] / n
    assert abs(per_walker.mean() - want) < 4 * per_walker.std() / math.sqrt(N)
    assert r["n_permeations"] == 0


def _chi2_uniform(pos, lo, hi, nbins):
    h, _ = np.histogram(pos, bins=nbins, range=(lo, hi))
    e = pos.size / nbins
    stat = np.sum((h - e) ** 2 / e)
    return chi2.sf(stat, nbins - 1)


@pytest.mark.parametrize("D1,D2,kappa", [(2.0, 2.0, 0.0), (1.0, 2.5, 0.5)])
def test_density_stays_uniform(D1, D2, kappa):
    """Elastic reflection keeps a uniform density at impermeable membranes
    (section 2.1.2), and the permeation probabilities of Eq.
    (perm-prob-general), whose ratio is sqrt(D2/D1), keep it uniform across a
    permeable membrane between compartments of unequal D (Appendix C.2)."""
    N, n = 100_000, 1500
    k = np.array([[0, kappa], [kappa, 0]])
    r = _run(slab_x(20, 2, 2, 5, 15), [D2, D1], kappa=k, n_walkers=N, n_steps=n)
    x = r["dump"][:, 5] + r["dump"][:, 8]
    assert _chi2_uniform(x, 0.0, 20.0, 80) > 1e-3
    frac = np.mean(r["dump"][:, 4] == 1)
    assert abs(frac - 0.5) < 4 * math.sqrt(0.25 / N)
    if kappa > 0:
        assert r["n_permeations"] > 0


def _slab_msd(a, D, t, terms=200):
    """<(x - x0)^2> in a slab of width a with reflecting walls and a uniform
    start: a^2/6 - (16 a^2/pi^4) sum_{n odd} exp(-n^2 pi^2 D t/a^2)/n^4."""
    n = np.arange(1, 2 * terms, 2)
    return a * a / 6 - 16 * a * a / np.pi ** 4 * np.sum(np.exp(-(n * np.pi) ** 2 * D * t / a ** 2)
                                                         / n ** 4)


def test_slab_restricted_diffusion_exact_series():
    """Impermeable slab of width a = 1 um: <dx^2>(t) follows the exact
    eigen-series for reflecting walls, approaching a^2/6 (D(t) ~ a^2/(12 t),
    Appendix A); the directions along the slab stay free."""
    D, dt, N = 2.0, 2e-4, 40_000
    lab = slab_x(20, 2, 2, 5, 15)
    dead = np.array([1, 0], np.uint8)
    for n in (250, 1000, 4000):
        r = _run(lab, [D, D], dead=dead, n_walkers=N, n_steps=n, dt=dt)
        X = r["dump"][:, 0:3]
        t = n * dt
        x2 = X[:, 0] ** 2
        assert abs(x2.mean() - _slab_msd(1.0, D, t)) < 4 * x2.std() / math.sqrt(N)
        y2 = X[:, 1] ** 2
        assert abs(y2.mean() - 2 * D * t) < 4 * y2.std() / math.sqrt(N)
        assert np.all(r["dump"][:, 4] == 1)  # never enters the dead label


def test_voxelized_cylinder_long_time_limit():
    """Long times in an impermeable voxelized cylinder: <dx^2> -> 2 Var(x)
    over the union of voxels, and the narrow-pulse signal across it tends to
    |<exp(i q x)>|^2 = |mean over voxels of exp(i q x_c)|^2 sinc^2(q l/2)."""
    D, dt, n, N, l = 2.0, 2e-4, 5000, 20_000, 0.1
    lab = cylinder_z(16, 5.0)
    dead = np.array([1, 0], np.uint8)
    G = np.zeros(n)
    G[0], G[-1] = -1.0, 1.0  # phase = q . (x_n - x_1)
    b = np.array([0.0, 2.0, 8.0])
    r = _run(lab, [D, D], dead=dead, n_walkers=N, n_steps=n, dt=dt, waveform=G,
             dirs=np.eye(3), bvals=b)
    yy, xx = np.nonzero(lab[0] == 1)
    xc = (xx + 0.5) * l
    var_x = np.mean((xc - xc.mean()) ** 2) + l * l / 12
    X = r["dump"][:, 0:3]
    x2 = X[:, 0] ** 2
    assert abs(x2.mean() - 2 * var_x) < 4 * x2.std() / math.sqrt(N)
    tq = (n - 1) * dt
    for j in (1, 2):
        q = math.sqrt(b[j] / tq)
        S = abs(np.mean(np.exp(1j * q * xc))) ** 2 * np.sinc(q * l / 2 / np.pi) ** 2
        assert abs(r["signal"][0, j, 0].real - S) < 4 / math.sqrt(N)


def test_t2_weights_impermeable():
    """Eq. (wt-relax) with kappa = 0: each walker keeps its compartment, so
    alpha = exp(-T/T2_c) exactly and sum(alpha) = sum_c N_c exp(-T/T2_c)."""
    dt, n, N = 2e-4, 2000, 5000
    T2 = np.array([60.0, 80.0])
    r = _run(cylinder_z(32, 10.0), [2.0, 2.0], T2=T2, n_walkers=N, n_steps=n, dt=dt)
    T = n * dt
    lab0 = r["dump"][:, 11].astype(int)
    assert np.all(lab0 == r["dump"][:, 4])
    assert np.allclose(r["dump"][:, 3], T / T2[lab0], rtol=1e-12, atol=0)
    want = sum(np.sum(lab0 == c) * math.exp(-T / T2[c]) for c in (0, 1))
    assert abs(r["sum_alpha"] - want) < 1e-12 * want


def test_prism_invariance_per_walker():
    """In a z-aligned prism the faces met are normal to x or y, so reflections
    never touch the z motion: per walker, dz and the z phase equal those of
    the same walker in free space (same seed, same start)."""
    dt, n, N = 2e-4, 2000, 2000
    G = pgse(n, dt, 0.05, 0.3)
    args = dict(n_walkers=N, n_steps=n, dt=dt, waveform=G, dirs=six_dirs(), bvals=[0.0, 1.0])
    a = _run(cylinder_z(32, 10.0), [2.0, 2.0], **args)
    b = _run(uniform_volume(32), [2.0], **args)
    assert a["n_membrane_hits"] > 0
    assert np.max(np.abs(a["dump"][:, 2] - b["dump"][:, 2])) < 1e-12
    assert np.max(np.abs(a["phase"][:, 0, 2] - b["phase"][:, 0, 2])) < 1e-12
    assert abs(a["signal"][0, 1, 2] - b["signal"][0, 1, 2]) < 1e-12


# ----------------------------------------------------- exchange, genuine kappa --

def _fd_tagged_fraction(L, x0, x1, D_in, D_out, kappa, times, h=0.005):
    """Independent reference: the tagged population that starts uniformly in
    the slab [x0, x1) of a periodic line of length L, evolved by the 1d
    diffusion equation with flux continuity and -D drho/dx = kappa (rho- -
    rho+) at both membranes (Appendix B, the boundary condition at a
    permeable membrane), on a finite-volume grid (series resistances
    h/(2D) + 1/kappa + h/(2D) across a membrane), solved exactly in time.
    Returns the fraction of the tagged population inside the slab."""
    m = int(round(L / h))
    xc = (np.arange(m) + 0.5) * h
    inside = (xc >= x0) & (xc < x1)
    Dc = np.where(inside, D_in, D_out)
    A = np.zeros((m, m))
    for i in range(m):
        j = (i + 1) % m
        if inside[i] == inside[j]:
            c = Dc[i] / h
        else:
            c = 1.0 / (h / (2 * Dc[i]) + 1.0 / kappa + h / (2 * Dc[j]))
        # flux c (rho_i - rho_j) from cell i to cell j; divide by h for density
        A[i, i] -= c / h
        A[i, j] += c / h
        A[j, j] -= c / h
        A[j, i] += c / h
    rho0 = inside.astype(float)
    out = []
    for t in times:
        rho = expm(A * t) @ rho0
        out.append(rho[inside].sum() / rho0.sum())
    return np.array(out)


@pytest.mark.parametrize("D_in,D_out", [(1.0, 1.0), (1.0, 2.0)])
def test_exchange_matches_diffusion_with_genuine_kappa(D_in, D_out):
    """Permeable slab (1 um) in a 2 um periodic cell, uniform start: the share
    of the walkers that started in the slab and are in it at time t follows
    the diffusion equation with the genuine permeability kappa, which is what
    Eq. (perm-prob-general) is built to give (Appendix C.1)."""
    kappa, dt, N = 0.5, 2e-4, 100_000
    lab = slab_x(20, 2, 2, 5, 15)
    k = np.array([[0, kappa], [kappa, 0]])
    steps = (500, 1500, 3000)
    ref = _fd_tagged_fraction(2.0, 0.5, 1.5, D_in, D_out, kappa, [s * dt for s in steps])
    for s, f_ref in zip(steps, ref):
        r = _run(lab, [D_out, D_in], kappa=k, n_walkers=N, n_steps=s, dt=dt)
        tag = r["dump"][:, 11] == 1
        f = np.mean(r["dump"][tag, 4] == 1)
        se = math.sqrt(f * (1 - f) / tag.sum())
        assert abs(f - f_ref) < 4 * se + 0.002, (s, f, f_ref)


def test_genuine_kappa_not_input_kappa_at_large_alpha():
    """Appendix C.1: the input kappa_0 of Eq. (perm-prob) yields the larger
    genuine permeability kappa = kappa_0 / (1 - alpha) (Eq. kappa-correction),
    alpha the mean permeation probability of the two sides (Eq.
    kappa-factor-prob); Eq. (perm-prob-general) is built so that the walk
    shows the kappa given.  With ds = 0.9 voxel and kappa such that P = 0.2,
    the share of the slab's walkers still in it follows the diffusion
    equation with kappa, and not with kappa_0 = (1 - alpha) kappa (outside
    the same tolerance at the first three times)."""
    D, sig = 0.5, 0.9
    ds = sig * 0.1
    dt = ds * ds / (6 * D)
    x = 0.25  # kappa ds C_3 / D; P = x / (1 + x) = 0.2 = alpha for equal D
    kappa = x * D / (ds * 2.0 / 3.0)
    alpha = x / (1 + x)
    N = 200_000
    lab = slab_x(20, 1, 1, 5, 15)
    k = np.array([[0, kappa], [kappa, 0]])
    steps = (20, 60, 150, 400)
    times = [s * dt for s in steps]
    ref = _fd_tagged_fraction(2.0, 0.5, 1.5, D, D, kappa, times)
    ref0 = _fd_tagged_fraction(2.0, 0.5, 1.5, D, D, (1 - alpha) * kappa, times)
    for i, (s, f_ref, f_ref0) in enumerate(zip(steps, ref, ref0)):
        r = _run(lab, [D, D], kappa=k, n_walkers=N, n_steps=s, dt=dt)
        assert abs(r["n_permeations"] / r["n_membrane_hits"] - alpha) < 0.01
        tag = r["dump"][:, 11] == 1
        f = np.mean(r["dump"][tag, 4] == 1)
        tol = 4 * math.sqrt(f * (1 - f) / tag.sum()) + 0.002
        assert abs(f - f_ref) < tol, (s, f, f_ref)
        if i < 3:  # and the walk is not the diffusion with kappa_0
            assert abs(f - f_ref0) > tol, (s, f, f_ref0)


def test_paper_permeability_validation_delta_source():
    """Appendix B, the elastic-collision permeability check: two planes at
    +-a/2 (a = 1 um), kappa = 0.1 um/ms, D_0 = 0.5 um^2/ms on both sides,
    dt = 4e-4 ms, walkers released at the middle (here: the walkers whose
    start lies within 0.1 um of it, picked from a uniform start by a run of 0
    steps), 1000 steps.  The permeability recovered from the density, as the
    kappa for which the diffusion equation with the membrane condition
    -D drho/dx = kappa (rho- - rho+) puts the same share of the walkers past
    the planes at 0.2 and 0.4 ms, lies within 3% of the kappa put in."""
    from scipy.optimize import brentq
    D, dt, kappa = 0.5, 4e-4, 0.1
    lab = slab_x(20, 1, 1, 5, 15)  # planes at x = 0.5 and 1.5 um, middle at 1.0
    k = np.array([[0, kappa], [kappa, 0]])
    ids = []
    for c in range(4):
        cand = np.arange(c * 1_000_000, (c + 1) * 1_000_000, dtype=np.int64)
        r = oracle.run(lab, 0.1, [D, D], k, seed=11, walker_ids=cand, n_walkers=cand.size,
                       n_steps=0, dt=dt, dump=True, n_threads=NT)
        x0 = (r["dump"][:, 5] + r["dump"][:, 8]) * 0.1
        ids.append(cand[np.abs(x0 - 1.0) < 0.1])
    ids = np.concatenate(ids)
    assert ids.size > 350_000

    h, L = 0.005, 2.0
    m = int(round(L / h))
    xc = (np.arange(m) + 0.5) * h
    inside = (xc >= 0.5) & (xc < 1.5)
    rho0 = (np.abs(xc - 1.0) < 0.1).astype(float)
    rho0 /= rho0.sum()

    def outside_share(kap, t):
        A = np.zeros((m, m))
        for i in range(m):
            j = (i + 1) % m
            c = D / h if inside[i] == inside[j] else 1.0 / (h / D + 1.0 / kap)
            A[i, i] -= c / h
            A[i, j] += c / h
            A[j, j] -= c / h
            A[j, i] += c / h
        return (expm(A * t) @ rho0)[~inside].sum()

    for n in (500, 1000):
        r = oracle.run(lab, 0.1, [D, D], k, seed=11, walker_ids=ids, n_walkers=ids.size,
                       n_steps=n, dt=dt, dump=True, n_threads=NT)
        F = np.mean(r["dump"][:, 4] == 0)
        k_hat = brentq(lambda kk: outside_share(kk, n * dt) - F, 0.02, 0.5)
        assert abs(k_hat - kappa) < 0.03 * kappa, (n, F, k_hat)


def _fd_signal_closed_pore(edges, Ds, kappa, intervals, h=0.005):
    """Independent reference for the complex signal: the pore [edges[0],
    edges[-1]) on a line, compartments between successive edges with
    diffusivities Ds, permeability kappa between neighbouring compartments
    and reflecting ends, discretised by finite volumes and solved exactly in
    time.  intervals is a list of (duration, q): during each, every move by
    dx carries the factor exp(-i q dx), so that a walker's weight is
    exp(-i sum_k q_k (x(t_k) - x(t_k-1))) (the multiple-propagator form of
    S = <exp(-i phi)>, section 2.3, Eq. signal); the start is uniform."""
    L = edges[-1] - edges[0]
    m = int(round(L / h))
    xc = edges[0] + (np.arange(m) + 0.5) * h
    comp = np.searchsorted(edges, xc, side="right") - 1
    Dc = np.asarray(Ds, float)[comp]
    rho = np.full(m, 1.0 / m, complex)
    for dur, q in intervals:
        A = np.zeros((m, m), complex)
        for i in range(m - 1):
            j = i + 1
            if comp[i] == comp[j]:
                c = Dc[i] / h
            else:
                c = 1.0 / (h / (2 * Dc[i]) + 1.0 / kappa + h / (2 * Dc[j]))
            A[i, i] -= c / h
            A[j, i] += c / h * np.exp(-1j * q * h)
            A[j, j] -= c / h
            A[i, j] += c / h * np.exp(1j * q * h)
        rho = expm(A * dur) @ rho
    return rho.sum()


def test_imaginary_signal_sign_multiple_propagator():
    """The sign convention S = <alpha exp(-i phi)> (section 2.3, Eq. signal),
    which only the imaginary part shows.  Im S vanishes when the pore is
    mirror-symmetric or the waveform odd under time reversal, so the pore here
    is a closed 1 um channel along x with two compartments (0.4 um at D = 2,
    0.6 um at D = 0.3 um^2/ms, kappa = 2 um/ms between them, dead walls), and
    the gradient three narrow pulses +1, -3, +2 at steps 1, 1501 and 2001.
    The phase is then -Q_1 (x_1501 - x_1) + Q_2 (x_2001 - x_1501) along x;
    the finite-volume multiple-propagator solution of the same problem gives
    S, imaginary part included; its conjugate, the other sign convention, is
    excluded by more than twice the tolerance."""
    dt, N = 2e-4, 200_000
    n1, n2, n3 = 1, 1501, 2001
    lab = np.zeros((1, 1, 11), np.uint8)
    lab[0, 0, 1:5] = 1   # x in [0.1, 0.5) um
    lab[0, 0, 5:11] = 2  # x in [0.5, 1.1) um
    D = np.array([1.0, 2.0, 0.3])
    kap = np.zeros((3, 3))
    kap[1, 2] = kap[2, 1] = 2.0
    dead = np.array([1, 0, 0], np.uint8)
    G = np.zeros(n3)
    G[n1 - 1], G[n2 - 1], G[n3 - 1] = 1.0, -3.0, 2.0
    Q = dt * np.cumsum(G[::-1])[::-1]
    b_unit = dt * np.sum(Q ** 2)
    for c in (2.0, 3.0):  # phase per um of displacement in the first interval
        scale = c / dt
        r = _run(lab, D, kappa=kap, dead=dead, n_walkers=N, n_steps=n3, dt=dt,
                 waveform=G[None], dirs=np.array([[1.0, 0.0, 0.0]]), bvals=[scale ** 2 * b_unit])
        phi = scale * r["phase"][:, 0, 0]
        w = np.exp(-1j * phi)
        se_re = w.real.std() / math.sqrt(N)
        se_im = w.imag.std() / math.sqrt(N)
        S_mc = r["signal"][0, 0, 0]
        assert abs(S_mc - w.mean()) < 1e-12
        S_ref = _fd_signal_closed_pore([0.1, 0.5, 1.1], [2.0, 0.3], 2.0,
                                       [((n2 - n1) * dt, -c), ((n3 - n2) * dt, 2 * c)])
        tol_im = 4 * se_im + 0.003
        assert abs(S_mc.real - S_ref.real) < 4 * se_re + 0.003, (c, S_mc, S_ref)
        assert abs(S_mc.imag - S_ref.imag) < tol_im, (c, S_mc, S_ref)
        # the other sign convention, <alpha exp(+i phi)>, misses by more than twice that
        assert abs(S_mc.imag + S_ref.imag) > 2 * tol_im, (c, S_mc, S_ref)


def test_t2_time_split_with_exchange():
    """Eq. (wt-relax) with exchange: R = sum_c t_c / T2_c, where t_c is the
    time spent in compartment c.  At equilibrium the expected share of time
    spent in c is its volume fraction, so <R> = T f_1 / T2_1 when only
    compartment 1 relaxes; with equal T2 everywhere R = T/T2 for every
    walker whatever its path."""
    dt, n, N = 2e-4, 1500, 40_000
    lab = slab_x(20, 2, 2, 5, 15)
    k = np.array([[0, 0.5], [0.5, 0]])
    r = _run(lab, [2.5, 1.0], kappa=k, T2=np.array([INF, 10.0]), n_walkers=N, n_steps=n, dt=dt)
    T = n * dt
    R = r["dump"][:, 3]
    assert r["n_permeations"] > 1000
    assert abs(R.mean() - T * 0.5 / 10.0) < 4 * R.std() / math.sqrt(N)
    r = _run(lab, [2.5, 1.0], kappa=k, T2=np.array([10.0, 10.0]), n_walkers=2000, n_steps=n,
             dt=dt)
    assert np.allclose(r["dump"][:, 3], T / 10.0, rtol=1e-12, atol=0)
