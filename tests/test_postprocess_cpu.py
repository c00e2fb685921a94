"""Host-only post-processing of signals (spherical mean, cumulant fit) in the
library, checked against closed forms (CPU; no device work)."""
import math

import numpy as np
import pytest

import paper_2012_06478_amd as rms
from rms_inputs import fibonacci_hemisphere

B = np.array([0.0, 0.2, 0.5, 1.0, 1.5, 2.0])


def test_cumulant_fit_exact_on_cumulant_signal():
    rng = np.random.default_rng(3)
    D = rng.uniform(0.3, 2.5, 7)
    K = rng.uniform(-0.5, 2.0, 7)
    S = np.exp(-np.outer(B, D) + np.outer(B ** 2, D ** 2 * K) / 6.0)
    Df, Kf = rms.rms_cumulant_fit(S.astype(complex), B, 2.0)
    assert np.allclose(Df, D, rtol=1e-10)
    assert np.allclose(Kf, K, rtol=1e-8, atol=1e-10)


def test_cumulant_fit_ignores_b_above_bmax():
    D, K = 1.1, 0.7
    S = np.exp(-B * D + B ** 2 * D * D * K / 6.0)[:, None].astype(complex)
    S[B > 1.0] = -5.0  # not a signal: must not be read
    Df, Kf = rms.rms_cumulant_fit(S, B, 1.0)
    assert math.isclose(Df[0], D, rel_tol=1e-10) and math.isclose(Kf[0], K, rel_tol=1e-8)


def test_cumulant_fit_errors():
    S = np.ones((6, 2), complex)
    with pytest.raises(rms.RmsError):
        rms.rms_cumulant_fit(S, B, 0.3)  # one b value in (0, 0.3]
    S[2, 1] = 0.0
    with pytest.raises(rms.RmsError):
        rms.rms_cumulant_fit(S, B, 2.0)


def test_spherical_mean_of_a_stick():
    """S = exp(-b D (g.z)^2) over a fine hemisphere: the mean tends to
    sqrt(pi / (4 b D)) erf(sqrt(b D))."""
    G = fibonacci_hemisphere(2000)
    D = 2.0
    b = np.array([0.1, 0.5, 1.0, 3.0])
    S = np.exp(-np.outer(b, D * G[:, 2] ** 2)).astype(complex)
    m = rms.rms_spherical_mean(S)
    want = np.sqrt(np.pi / (4 * b * D)) * np.array([math.erf(math.sqrt(x * D)) for x in b])
    assert np.allclose(m.real, want, atol=2e-3)
    assert np.all(m.imag == 0)


def test_spherical_mean_is_the_mean():
    rng = np.random.default_rng(1)
    S = rng.normal(size=(4, 9)) + 1j * rng.normal(size=(4, 9))
    assert np.allclose(rms.rms_spherical_mean(S), S.mean(axis=1), rtol=1e-14)
