"""Synthetic label volumes, seeded and deterministic.

Every generator returns a C-contiguous array of shape [nz, ny, nx] (x fastest
in memory) of uint8 or uint16 labels.  Label 0 is the extracellular space (or
the background); cells are labelled 1, 2, ...  Voxel membership uses the
voxel-centre rule: voxel (i, j, k) belongs to a body when its centre
((i + 1/2), (j + 1/2), (k + 1/2)) voxel lengths lies inside it.  The volumes
are meant to be walked with periodic boundaries, so the packings wrap around.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_gen.c")
_LIB = os.path.join(_HERE, "_gen.so")
_lib = None


def build() -> str:
    """Compile the packing generators (plain C, gcc)."""
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", _LIB + ".tmp",
                           _SRC, "-lm"])
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
        d, i64, u64 = C.c_double, C.c_int64, C.c_uint64
        lib.gen_ellipsoids.argtypes = [i64, d, C.c_int, d, d, u64, C.c_int, d, C.c_void_p,
                                       C.c_void_p]
        lib.gen_axons.argtypes = [i64, i64, i64, d, C.c_int, u64, d, d, d, d, d, d, d, d, d,
                                  C.c_void_p, C.c_void_p]
        _lib = lib
    return _lib


def uniform_volume(nx: int, ny: int | None = None, nz: int | None = None,
                   label: int = 0, dtype=np.uint8) -> np.ndarray:
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    return np.full((nz, ny, nx), label, dtype=dtype)


def cylinder_z(n: int = 32, radius_vox: float = 10.0, nz: int | None = None,
               dtype=np.uint8) -> np.ndarray:
    """A z-aligned cylinder (label 1) of the given radius, centred in an n x n
    cross-section, in label 0."""
    nz = n if nz is None else nz
    c = (np.arange(n) + 0.5) - n / 2.0
    inside = (c[None, :] ** 2 + c[:, None] ** 2) <= radius_vox ** 2  # [y, x]
    lab = np.zeros((nz, n, n), dtype=dtype)
    lab[:, inside] = 1
    return lab


def slab_x(nx: int, ny: int, nz: int, x0: int, x1: int, dtype=np.uint8) -> np.ndarray:
    """Label 1 on the voxel columns x0 <= i < x1, label 0 elsewhere: two flat
    membranes normal to x at i = x0 and i = x1."""
    lab = np.zeros((nz, ny, nx), dtype=dtype)
    lab[:, :, x0:x1] = 1
    return lab


def cube_cell(n: int, lo: int, hi: int, dtype=np.uint8) -> np.ndarray:
    """Label 1 on the cube lo <= i, j, k < hi, label 0 elsewhere."""
    lab = np.zeros((n, n, n), dtype=dtype)
    lab[lo:hi, lo:hi, lo:hi] = 1
    return lab


def sphere_cell(n: int, radius_vox: float, dtype=np.uint8) -> np.ndarray:
    """A voxelized sphere (label 1) centred in an n^3 volume of label 0."""
    c = (np.arange(n) + 0.5) - n / 2.0
    r2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    return (r2 <= radius_vox ** 2).astype(dtype)


def ellipsoid_packing(n: int = 200, voxel_um: float = 0.1, n_cells: int = 120,
                      semi_um: tuple = (1.0, 4.0), seed: int = 2, max_tries: int = 10_000,
                      shrink: float = 0.9) -> tuple[np.ndarray, dict]:
    """Random sequential addition of randomly oriented ellipsoids (uint16).

    Cell c = 1..n_cells draws semi-axes uniform in ``semi_um`` and a uniform
    random rotation, then tries up to ``max_tries`` uniform voxel centres; a
    placement is accepted when none of its voxels is taken by an earlier cell
    or touches one through a face (so every cell is wrapped in extracellular
    label 0).  After ``max_tries`` failures the semi-axes shrink by
    ``shrink``.  Returns the labels and a dict with the achieved volume
    fraction and the final semi-axes.
    """
    lab = np.zeros((n, n, n), np.uint16)
    semi = np.zeros((n_cells, 3))
    rc = _load().gen_ellipsoids(n, voxel_um, n_cells, semi_um[0], semi_um[1], seed, max_tries,
                                shrink, lab.ctypes.data, semi.ctypes.data)
    if rc:
        raise RuntimeError(f"ellipsoid packing failed ({rc})")
    return lab, dict(volume_fraction=float((lab > 0).mean()), semi_axes_um=semi)


def axon_bundle(nx: int = 400, ny: int = 400, nz: int = 1000, voxel_um: float = 0.1,
                n_axons: int = 300, seed: int = 3, mu: float = -0.144, sigma: float = 0.334,
                bead_spacing_um: float = 4.0, bead_width_um: float = 0.5,
                bead_amp: float = 0.2, wavelength_um: tuple = (10.0, 30.0),
                slope: float = 0.039, max_tilt_deg: float = 15.0) -> tuple[np.ndarray, dict]:
    """A bundle of beaded, undulating tubes along z in extracellular label 0
    (uint16, periodic).

    Tube a = 1..n_axons: base radius lognormal(mu, sigma) um; Gaussian beads
    of relative height ``bead_amp`` and width ``bead_width_um`` at
    Poisson-spaced z (mean ``bead_spacing_um``); a one-harmonic undulation per
    transverse axis with wavelength uniform in ``wavelength_um`` and amplitude
    ``slope`` times the wavelength; an axis tilted from z by an angle uniform
    in [0, max_tilt_deg] with uniform azimuth.  Voxels are claimed first-come,
    and a tube never takes a voxel that shares a face with an earlier tube.
    """
    lab = np.zeros((nz, ny, nx), np.uint16)
    r0 = np.zeros(n_axons)
    rc = _load().gen_axons(nx, ny, nz, voxel_um, n_axons, seed, mu, sigma, bead_spacing_um,
                           bead_width_um, bead_amp, wavelength_um[0], wavelength_um[1], slope,
                           np.deg2rad(max_tilt_deg), lab.ctypes.data, r0.ctypes.data)
    if rc:
        raise RuntimeError(f"axon bundle failed ({rc})")
    return lab, dict(intra_fraction=float((lab > 0).mean()), r0_um=r0)
