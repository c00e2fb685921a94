"""The closed-geometry laws the oracle is pinned to, on the GPU through the C
ABI at walker counts the oracle cannot reach (properties that hold at any
size; the expectations and their derivations are those of the oracle's
pins): the short-time surface-to-volume law in a cube cell, the long-time
limit in a voxelized sphere and Karger's exchange across a permeable sphere.
With 1e6-1e7 walkers the Monte Carlo error is a few times smaller than the
allowances for the finite step and the barrier-limited model."""
import math

import numpy as np
import pytest

import paper_2012_06478_amd as rms
from rms_inputs import cube_cell, sphere_cell, six_dirs

pytestmark = pytest.mark.gpu

LP = 0.1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _faces_between(inside):
    return int(sum(np.sum(inside != np.roll(inside, 1, axis=a)) for a in range(3)))


@pytest.mark.parametrize("precision", [rms.RMS_FP64, rms.RMS_MIXED])
def test_short_time_surface_to_volume_law(precision):
    """Cube of 40 voxels in 48^3, D0 = 2, 1e7 walkers inside, moments at
    0.02-0.16 ms: D(t)/D0 against 1 - 4/(9 sqrt(pi)) (S/V) sqrt(D0 t) within 4
    standard errors plus 3% of the reduction."""
    lab = cube_cell(48, 4, 44)
    inside = lab == 1
    sv = _faces_between(inside) * LP * LP / (inside.sum() * LP ** 3)
    D0, dt, N = 2.0, 2e-4, 10_000_000
    steps = [100, 200, 400, 800]
    print(f"[case] cube S/V law precision={precision} walkers={N}", flush=True)
    sub = rms.rms_create_substrate(lab, LP, [D0, D0], None, None, np.array([1, 0], np.uint8))
    g = rms.rms_run_record(sub, seed=5, n_walkers=N, n_steps=steps[-1], dt=dt, dirs=six_dirs(),
                           record_steps=steps, precision=precision)
    sub.close()
    for k, s in enumerate(steps):
        t = s * dt
        m2 = g["records"]["m2"][k]
        got = (m2[0] + m2[3] + m2[5]) / (6 * t) / D0
        want = 1 - 4 / (9 * math.sqrt(math.pi)) * sv * math.sqrt(D0 * t)
        print(f"t {t:.2f} ms: D/D0 {got:.5f}, law {want:.5f}", flush=True)
        assert abs(got - want) < 4 * 0.82 / math.sqrt(N) + 0.03 * (1 - want), t


def test_voxelized_sphere_long_time_limit():
    """Impermeable sphere of radius 10 voxels in 24^3, 1e6 walkers for 2 ms:
    per axis <dx^2> = 2 mu2 and <dx^4> = 2 mu4 + 6 mu2^2 of the union of
    voxels (4 standard errors from the walker dump)."""
    lab = sphere_cell(24, 10.0)
    inside = lab == 1
    D0, dt, n, N = 2.0, 2e-4, 10_000, 1_000_000
    print(f"[case] sphere long-time walkers={N}", flush=True)
    sub = rms.rms_create_substrate(lab, LP, [D0, D0], None, None, np.array([1, 0], np.uint8))
    g = rms.rms_run(sub, seed=9, n_walkers=N, n_steps=n, dt=dt, dirs=six_dirs(), dump=True)
    sub.close()
    X = g["dump"][:, 0:3]
    idx = np.argwhere(inside)[:, ::-1]
    for a in range(3):
        c = (idx[:, a] + 0.5) * LP
        c = c - c.mean()
        mu2 = np.mean(c ** 2) + LP ** 2 / 12
        mu4 = np.mean(c ** 4) + 6 * np.mean(c ** 2) * LP ** 2 / 12 + LP ** 4 / 80
        x2, x4 = X[:, a] ** 2, X[:, a] ** 4
        assert abs(x2.mean() - 2 * mu2) < 4 * x2.std() / math.sqrt(N), a
        assert abs(x4.mean() - (2 * mu4 + 6 * mu2 ** 2)) < 4 * x4.std() / math.sqrt(N), a


def test_karger_exchange_permeable_sphere():
    """Sphere of radius 10 voxels in 24^3, kappa = 0.05 um/ms, 2e6 walkers:
    the share of walkers started inside that are inside at 1 and 3 ms against
    Karger's first-order exchange, within 4 binomial errors plus 2% of the
    part not yet relaxed."""
    lab = sphere_cell(24, 10.0)
    inside = lab == 1
    S = _faces_between(inside) * LP * LP
    v_in, v_out = inside.sum() * LP ** 3, (~inside).sum() * LP ** 3
    rate = 0.05 * S * (1 / v_in + 1 / v_out)
    p_eq = v_in / (v_in + v_out)
    kap = np.array([[0.0, 0.05], [0.05, 0.0]])
    D0, dt, N = 2.0, 2e-4, 2_000_000
    sub = rms.rms_create_substrate(lab, LP, [D0, D0], kap)
    try:
        for t in (1.0, 3.0):
            print(f"[case] Karger sphere t={t} ms walkers={N}", flush=True)
            g = rms.rms_run(sub, seed=7, n_walkers=N, n_steps=int(round(t / dt)), dt=dt,
                            dirs=six_dirs(), dump=True)
            d = g["dump"]
            start_in = d[:, 11] == 1
            got = np.mean(d[start_in, 4] == 1)
            want = p_eq + (1 - p_eq) * math.exp(-rate * t)
            print(f"inside share {got:.5f}, first-order exchange {want:.5f}", flush=True)
            tol = 4 * math.sqrt(want * (1 - want) / start_in.sum()) + 0.02 * (want - p_eq)
            assert abs(got - want) < tol, t
    finally:
        sub.close()
