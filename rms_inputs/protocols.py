"""Gradient waveforms and direction sets.

A waveform is an array of n_steps samples; sample i is the (dimensionless)
gradient shape during step i+1, i.e. on the time interval (i dt, (i+1) dt].
The library scales each shape so that its b value equals each requested b.
"""
from __future__ import annotations

import numpy as np


def pgse(n_steps: int, dt: float, delta: float, Delta: float, start: float = 0.0) -> np.ndarray:
    """Pulsed-gradient spin echo (effective gradient): +1 for delta ms from
    ``start``, -1 for delta ms from ``start + Delta``; zero elsewhere.  Each
    lobe covers round(delta/dt) whole steps, so the shape is exactly
    balanced."""
    g = np.zeros(n_steps)
    nd = int(round(delta / dt))
    i0 = int(round(start / dt))
    i1 = int(round((start + Delta) / dt))
    if nd <= 0 or i1 + nd > n_steps or i0 + nd > i1:
        raise ValueError("PGSE timing does not fit in the step count")
    g[i0:i0 + nd] = 1.0
    g[i1:i1 + nd] = -1.0
    return g


def ogse_cos(n_steps: int, dt: float, lobe: float, Delta: float, periods: int,
             start: float = 0.0) -> np.ndarray:
    """Cosine oscillating-gradient spin echo: a lobe of ``periods`` cosine
    periods lasting ``lobe`` ms, sampled at step midpoints, and a second lobe
    ``Delta`` ms later equal to minus the first (so the pair is balanced
    sample by sample)."""
    g = np.zeros(n_steps)
    nl = int(round(lobe / dt))
    i0 = int(round(start / dt))
    i1 = int(round((start + Delta) / dt))
    if nl <= 0 or i1 + nl > n_steps or i0 + nl > i1:
        raise ValueError("OGSE timing does not fit in the step count")
    t = (np.arange(nl) + 0.5) * dt
    lobe_shape = np.cos(2.0 * np.pi * periods * t / (nl * dt))
    g[i0:i0 + nl] = lobe_shape
    g[i1:i1 + nl] = -lobe_shape
    return g


def six_dirs() -> np.ndarray:
    s = 1.0 / np.sqrt(2.0)
    return np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [s, s, 0], [s, 0, s], [0, s, s]], float)


def fibonacci_hemisphere(n: int) -> np.ndarray:
    """n deterministic, nearly uniform unit vectors with z >= 0 (spherical
    Fibonacci lattice restricted to the upper hemisphere)."""
    k = np.arange(n) + 0.5
    z = 1.0 - k / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    golden = np.pi * (3.0 - np.sqrt(5.0))
    ph = golden * np.arange(n)
    return np.stack([r * np.cos(ph), r * np.sin(ph), z], axis=1)
