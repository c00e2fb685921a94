"""Pins of the oracle's whole walk in closed geometries (CPU only): the
short-time surface-to-volume law, the long-time limit in a voxelized sphere
and Karger's two-compartment exchange across a permeable sphere.

- Short times (Mitra et al.): D(t)/D0 = 1 - 4/(9 sqrt(pi)) (S/V) sqrt(D0 t)
  for the mean diffusivity trace(<dx dx>)/(6t).  A cube cell with faces on
  voxel faces has S/V = 6/L exactly; its corrections are exponentially small
  while sqrt(D0 t) << L, so the law is the expectation once sqrt(D0 t) spans
  a few steps ds.
- Long times in an impermeable voxelized sphere: the end point is uniform
  over the union of voxels and independent of the start, so per axis
  <dx^2> = 2 mu2 and <dx^4> = 2 mu4 + 6 mu2^2 with the central moments mu_k of
  that union (voxel centres plus a uniform offset), and the narrow-pulse
  signal is |<exp(i q x)>|^2.
- Exchange across a permeable sphere in the barrier-limited regime (kappa R
  / D << 1): the probability that a walker found inside at t = 0 is inside at
  t relaxes as p_eq + (1 - p_eq) exp(-t kappa S (1/V_in + 1/V_out)) (Karger's
  first-order exchange), S the area of the voxel faces between the labels and
  p_eq = V_in / V.  This holds because a face of area A passes kappa A rho per
  unit time (Eq. perm-prob with C_3 = 2/3).
"""
import math
import os

import numpy as np

import oracle
from rms_inputs import cube_cell, sphere_cell, six_dirs

NT = oracle.host_threads()
LP = 0.1  # voxel size, um


def _faces_between(inside):
    """Voxel faces between the inside and the outside of a periodic volume."""
    return int(sum(np.sum(inside != np.roll(inside, 1, axis=a)) for a in range(3)))


def test_short_time_surface_to_volume_law():
    """Impermeable cube of 40 voxels (4 um) in a 48^3 volume, D0 = 2,
    200000 walkers inside, moments recorded at 0.02-0.16 ms (sqrt(D0 t) =
    0.2-0.57 um, 4-12 steps ds).  Tolerance: 4 standard errors of D(t)
    (relative 0.82/sqrt(N) for a near-Gaussian displacement) plus 3% of the
    predicted reduction for the finite step."""
    lab = cube_cell(48, 4, 44)
    inside = lab == 1
    S = _faces_between(inside) * LP * LP
    V = inside.sum() * LP ** 3
    assert math.isclose(S / V, 6 / (40 * LP), rel_tol=1e-12)
    D0, dt, N = 2.0, 2e-4, 200_000
    steps = [100, 200, 400, 800]
    r = oracle.run(lab, LP, np.array([D0, D0]), None, None, np.array([1, 0], np.uint8), seed=5,
                   n_walkers=N, n_steps=steps[-1], dt=dt, dirs=six_dirs(), n_threads=NT,
                   rec_steps=steps)
    for k, s in enumerate(steps):
        t = s * dt
        m2 = r["records"]["m2"][k]
        got = (m2[0] + m2[3] + m2[5]) / (6 * t) / D0
        want = 1 - 4 / (9 * math.sqrt(math.pi)) * (S / V) * math.sqrt(D0 * t)
        tol = 4 * 0.82 / math.sqrt(N) + 0.03 * (1 - want)
        assert abs(got - want) < tol, (t, got, want)


def test_voxelized_sphere_long_time_limit():
    """Impermeable sphere of radius 10 voxels (1 um) in a 24^3 volume, D0 =
    2, 20000 walkers for 2 ms (the slowest mode decays by exp(-17)): per axis
    <dx^2> and <dx^4> against the moments of the union of voxels, and the
    narrow-pulse signal along x against |<exp(i q x)>|^2."""
    lab = sphere_cell(24, 10.0)
    inside = lab == 1
    D0, dt, n, N = 2.0, 2e-4, 10_000, 20_000
    G = np.zeros(n)
    G[0], G[-1] = -1.0, 1.0  # phase = q . (x_n - x_1)
    b = np.array([0.0, 1.0, 4.0])
    r = oracle.run(lab, LP, np.array([D0, D0]), None, None, np.array([1, 0], np.uint8), seed=9,
                   n_walkers=N, n_steps=n, dt=dt, waveform=G, dirs=np.eye(3), bvals=b,
                   n_threads=NT, dump=True)
    X = r["dump"][:, 0:3]
    idx = np.argwhere(inside)[:, ::-1]  # (x, y, z) voxel indices
    for a in range(3):
        c = (idx[:, a] + 0.5) * LP
        c = c - c.mean()
        mu2 = np.mean(c ** 2) + LP ** 2 / 12
        mu4 = np.mean(c ** 4) + 6 * np.mean(c ** 2) * LP ** 2 / 12 + LP ** 4 / 80
        x2, x4 = X[:, a] ** 2, X[:, a] ** 4
        assert abs(x2.mean() - 2 * mu2) < 4 * x2.std() / math.sqrt(N), a
        assert abs(x4.mean() - (2 * mu4 + 6 * mu2 ** 2)) < 4 * x4.std() / math.sqrt(N), a
    xc = (idx[:, 0] + 0.5) * LP
    tq = (n - 1) * dt
    for j in (1, 2):
        q = math.sqrt(b[j] / tq)
        want = abs(np.mean(np.exp(1j * q * xc))) ** 2 * np.sinc(q * LP / 2 / np.pi) ** 2
        assert abs(r["signal"][0, j, 0].real - want) < 4 / math.sqrt(N)


def test_karger_exchange_permeable_sphere():
    """Sphere of radius 10 voxels (1 um) in a 24^3 volume, D0 = 2 on both
    sides, kappa = 0.05 um/ms (kappa R / D = 0.025; exchange time 3.1 ms);
    20000 walkers started uniformly; the share of the walkers started inside
    that are inside at 1 and 3 ms.  Tolerance: 4 binomial standard errors plus
    2% of the part not yet relaxed (the barrier-limited model's error is of
    order kappa R / D)."""
    lab = sphere_cell(24, 10.0)
    inside = lab == 1
    S = _faces_between(inside) * LP * LP
    v_in, v_out = inside.sum() * LP ** 3, (~inside).sum() * LP ** 3
    rate = 0.05 * S * (1 / v_in + 1 / v_out)
    p_eq = v_in / (v_in + v_out)
    kap = np.array([[0.0, 0.05], [0.05, 0.0]])
    D0, dt, N = 2.0, 2e-4, 20_000
    for t in (1.0, 3.0):
        r = oracle.run(lab, LP, np.array([D0, D0]), kap, None, None, seed=7, n_walkers=N,
                       n_steps=int(round(t / dt)), dt=dt, dirs=six_dirs(), n_threads=NT,
                       dump=True)
        d = r["dump"]
        start_in = d[:, 11] == 1
        got = np.mean(d[start_in, 4] == 1)
        want = p_eq + (1 - p_eq) * math.exp(-rate * t)
        tol = 4 * math.sqrt(want * (1 - want) / start_in.sum()) + 0.02 * (want - p_eq)
        assert abs(got - want) < tol, (t, got, want)
