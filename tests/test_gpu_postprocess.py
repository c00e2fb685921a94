"""Post-processing of a GPU run's signals: in free diffusion the cumulant fit
gives D = D0 and K = 0 (up to the finite-step excess kurtosis), matching the
moment-based D, and the spherical mean of an isotropic signal equals each
direction's signal within noise."""
import numpy as np
import pytest

import paper_2012_06478_amd as rms
from rms_inputs import uniform_volume, pgse, fibonacci_hemisphere

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_free_diffusion_cumulant_fit():
    n, dt, D0 = 2000, 2e-4, 2.0
    b = np.array([0.0, 0.1, 0.2, 0.3, 0.4, 0.5])
    G = fibonacci_hemisphere(30)
    print("[case] free diffusion 2e5 walkers x 2000 steps, cumulant fit", flush=True)
    sub = rms.rms_create_substrate(uniform_volume(16), 0.1, [D0])
    r = rms.rms_run(sub, seed=4, n_walkers=200_000, n_steps=n, dt=dt,
                    waveform=pgse(n, dt, n * dt / 4, 3 * n * dt / 4), dirs=G, bvals=b)
    sub.close()
    S = r["signal"][0]
    Df, Kf = rms.rms_cumulant_fit(S, b, 0.5)
    print(f"D fit {Df.mean():.4f} +- {Df.std():.4f}, K fit {Kf.mean():.3f} +- {Kf.std():.3f}",
          flush=True)
    assert np.all(np.abs(Df - D0) < 0.05 * D0)
    assert abs(Df.mean() - D0) < 0.01 * D0
    assert abs(Kf.mean()) < 0.15
    assert np.all(np.abs(r["D"] - D0) < 0.03 * D0)
    m = rms.rms_spherical_mean(S)
    assert np.allclose(m.real, np.exp(-b * D0), atol=0.01)
