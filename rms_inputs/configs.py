"""The synthetic workloads, as plain dicts of inputs (no results).

Units: um, ms, um^2/ms (D), um/ms (kappa), ms/um^2 (b).  Each builder returns
a dict with ``labels`` ([nz, ny, nx] array), ``voxel_um``, ``D``, ``kappa``
([n, n]), ``T2``, ``dead`` (or None), ``seed``, ``n_walkers``, ``n_steps``,
``dt``, ``waveform`` ([n_shapes, n_steps]), ``dirs`` and ``bvals``.
"""
from __future__ import annotations

import numpy as np

from .protocols import pgse, ogse_cos, six_dirs, fibonacci_hemisphere
from .substrates import cylinder_z, ellipsoid_packing, axon_bundle

_INF = float("inf")


def _pair_matrix(n_labels: int, kappa: float) -> np.ndarray:
    """kappa on every face between label 0 and a cell; cells never touch."""
    k = np.zeros((n_labels, n_labels))
    k[0, 1:] = kappa
    k[1:, 0] = kappa
    return k


def cylinder_case(n_walkers: int = 10_000, n_steps: int = 60_000, seed: int = 1) -> dict:
    """32^3 u8 volume, 0.1 um voxels, one impermeable z-aligned cylinder of
    radius 10 voxels (label 1) in label 0, D0 = 2 in both, no T2.  PGSE with
    delta = 2 ms, Delta = 10 ms at dt = 2e-4 ms needs 60 000 steps; a shorter
    ``n_steps`` keeps the same shape compressed in time."""
    dt = 2e-4
    if n_steps >= 60_000:
        wf = pgse(n_steps, dt, 2.0, 10.0)
    else:
        T = n_steps * dt
        wf = pgse(n_steps, dt, T / 6.0, 5.0 * T / 6.0)
    return dict(name="cylinder32_u8", labels=cylinder_z(32, 10.0), voxel_um=0.1,
                D=np.array([2.0, 2.0]), kappa=np.zeros((2, 2)), T2=np.array([_INF, _INF]),
                dead=None, seed=seed, n_walkers=n_walkers, n_steps=n_steps, dt=dt,
                waveform=wf[None, :], dirs=six_dirs(), bvals=np.array([0.0, 0.5, 1.0, 2.0]))


def ellipsoid_case(n: int = 200, n_cells: int = 120, n_walkers: int = 1_000_000,
                   n_steps: int = 10_000, seed: int = 2, kappa: float = 0.02) -> dict:
    """200^3 u16 volume, 0.1 um voxels, ellipsoidal cells (semi-axes 1-4 um,
    random orientation) in extracellular label 0; D intra 2 / extra 2.5;
    kappa on every membrane; T2 80 (intra) / 60 (extra) ms; PGSE with
    delta = T/4 and Delta = 3T/4 over T = n_steps dt; 30 directions x 6 b."""
    labels, info = ellipsoid_packing(n=n, n_cells=n_cells, seed=seed)
    L = int(labels.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 2.5
    T2 = np.full(L, 80.0)
    T2[0] = 60.0
    dt = 2e-4
    T = n_steps * dt
    wf = pgse(n_steps, dt, T / 4.0, 3.0 * T / 4.0)
    return dict(name=f"ellipsoids{n}_u16", labels=labels, info=info, voxel_um=0.1, D=D,
                kappa=_pair_matrix(L, kappa), T2=T2, dead=None, seed=seed, n_walkers=n_walkers,
                n_steps=n_steps, dt=dt, waveform=wf[None, :], dirs=fibonacci_hemisphere(30),
                bvals=np.array([0.0, 0.2, 0.5, 1.0, 1.5, 2.0]))


def axon_case(nx: int = 400, ny: int = 400, nz: int = 1000, n_axons: int = 300,
              n_walkers: int = 10_000_000, n_steps: int = 20_000, seed: int = 3,
              kappa: float = 0.01) -> dict:
    """Beaded undulating tube bundle, D intra 2 / extra 1.8, kappa 0.01, no
    T2; PGSE (delta = T/4, Delta = 3T/4) and a cosine OGSE (two lobes of
    0.45 T, Delta = T/2, two periods per lobe); 30 directions x 6 b."""
    labels, info = axon_bundle(nx, ny, nz, n_axons=n_axons, seed=seed)
    L = int(labels.max()) + 1
    D = np.full(L, 2.0)
    D[0] = 1.8
    dt = 2e-4
    T = n_steps * dt
    wf = np.stack([pgse(n_steps, dt, T / 4.0, 3.0 * T / 4.0),
                   ogse_cos(n_steps, dt, 0.45 * T, 0.5 * T, 2)])
    return dict(name=f"axons{nx}x{ny}x{nz}_u16", labels=labels, info=info, voxel_um=0.1, D=D,
                kappa=_pair_matrix(L, kappa), T2=np.full(L, _INF), dead=None, seed=seed,
                n_walkers=n_walkers, n_steps=n_steps, dt=dt, waveform=wf,
                dirs=fibonacci_hemisphere(30), bvals=np.array([0.0, 0.2, 0.5, 1.0, 1.5, 2.0]))
