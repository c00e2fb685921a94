"""Pins of the oracle's building blocks against facts fixed outside it:
published known-answer vectors, values the paper prints, closed forms and
hand-worked single steps.  CPU only."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_values():
    vals = {}
    with open(os.path.join(GOLDEN, "paper_worked_values.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, value, tol, cite = line.split()
            vals[name] = (float(value), float(tol), cite)
    return vals


# ---------------------------------------------------------------- Philox ----

def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(w[0:4], w[4:6])
        assert list(out) == w[6:10]


_ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct probe : rocrand_device::philox4x32_10_engine {
    uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }
};
int main() {
    probe p;
    unsigned a[6];
    while (std::scanf("%x %x %x %x %x %x", &a[0], &a[1], &a[2], &a[3], &a[4], &a[5]) == 6) {
        uint4 c; c.x = a[0]; c.y = a[1]; c.z = a[2]; c.w = a[3];
        uint2 k; k.x = a[4]; k.y = a[5];
        uint4 o = p.run(c, k);
        std::printf("%08x %08x %08x %08x\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand(tmp_path):
    """The oracle's Philox4x32-10 agrees with rocRAND's (an independent
    implementation, called as a library on the host) on random inputs."""
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(_ROCRAND_PROBE)
    try:
        subprocess.check_call(["hipcc", "-O1", "-o", str(exe), str(src)],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL, timeout=300)
    except (subprocess.CalledProcessError, subprocess.TimeoutExpired):
        pytest.skip("rocRAND host probe did not build")
    rng = np.random.default_rng(7)
    ins = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    text = "\n".join(" ".join("%08x" % v for v in row) for row in ins) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True,
                         timeout=60).stdout.split("\n")
    for row, line in zip(ins, out):
        ref = [int(x, 16) for x in line.split()]
        got = oracle.philox4x32_10(row[0:4], row[4:6])
        assert list(got) == ref


# ------------------------------------------------------ uniform, direction ---

def test_uniform_mapping_exact():
    assert oracle.uniform(0) == 2.0 ** -33
    assert oracle.uniform(2**32 - 1) == 1.0 - 2.0 ** -33
    assert oracle.uniform(2**31) == 0.5 + 2.0 ** -33


def test_direction_uniform_on_sphere():
    """Archimedes: every Cartesian component of a uniform unit vector is
    uniform on [-1, 1], so <v^2> = 1/3 and <v^4> = 1/5."""
    rng = np.random.default_rng(11)
    w = rng.integers(0, 2**32, size=(40000, 2), dtype=np.uint64)
    V = np.array([oracle.direction(int(a), int(b)) for a, b in w])
    n = V.shape[0]
    assert np.max(np.abs(np.linalg.norm(V, axis=1) - 1.0)) < 4e-16
    for a in range(3):
        m2 = np.mean(V[:, a] ** 2)
        m4 = np.mean(V[:, a] ** 4)
        # variances of v^2 and v^4 for v uniform on [-1, 1]
        s2 = math.sqrt((1 / 5 - 1 / 9) / n)
        s4 = math.sqrt((1 / 9 - 1 / 25) / n)
        assert abs(m2 - 1 / 3) < 4 * s2
        assert abs(m4 - 1 / 5) < 4 * s4
        # Kolmogorov-Smirnov distance to the uniform law on [-1, 1]
        x = np.sort(V[:, a])
        F = (x + 1.0) / 2.0
        ks = np.max(np.maximum(np.arange(1, n + 1) / n - F, F - np.arange(n) / n))
        assert ks < 1.63 / math.sqrt(n)  # p ~ 0.01


# ---------------------------------------------------------- step, P, b -------

def test_step_size_matches_paper():
    g = _golden_values()
    ds = oracle.step_size(g["step_D0"][0], g["step_dt"][0])
    assert abs(ds - g["step_ds"][0]) <= g["step_ds"][1]


def test_perm_prob_small_kappa_limit():
    """Eq. (perm-prob): P ~ kappa ds C_3 / D0 when P << 1."""
    g = _golden_values()
    C3 = g["C_3"][0]
    D, dt = 2.0, 2e-4
    ds = math.sqrt(6 * D * dt)
    for kappa in (1e-4, 1e-3, 1e-2):
        P = oracle.perm_prob(kappa, D, D, dt)
        lin = kappa * ds * C3 / D
        assert abs(P - lin) / lin < 2 * lin  # first-order correction is O(P)


def test_perm_prob_kappa_correction_identity():
    """Appendix C.1: with kappa0 = P12 D1 / (ds1 C_3) (Eq. perm-prob solved for
    the input permeability) and alpha = (P12 + P21)/2 (Eq. kappa-factor-prob),
    the genuine permeability is kappa0 / (1 - alpha) (Eq. kappa-correction)."""
    C3 = 2.0 / 3.0
    for (kappa, D1, D2, dt) in [(0.02, 2.0, 2.5, 2e-4), (0.1, 0.5, 0.5, 4e-4),
                                (1.0, 1.0, 3.0, 1e-3), (5.0, 2.0, 1.0, 5e-4)]:
        P12 = oracle.perm_prob(kappa, D1, D2, dt)
        P21 = oracle.perm_prob(kappa, D2, D1, dt)
        ds1 = math.sqrt(6 * D1 * dt)
        ds2 = math.sqrt(6 * D2 * dt)
        k0_12 = P12 * D1 / (ds1 * C3)
        k0_21 = P21 * D2 / (ds2 * C3)
        assert abs(k0_12 - k0_21) < 1e-12 * k0_12  # one input kappa0 for both sides
        alpha = 0.5 * (P12 + P21)
        assert abs(k0_12 / (1 - alpha) - kappa) < 1e-12 * kappa


def test_perm_prob_equilibrium_ratio():
    """Appendix C.2 with equal spin concentrations: P12/P21 = sqrt(D2/D1)
    keeps the equilibrium density."""
    for D1, D2 in [(1.0, 2.0), (2.0, 2.5), (0.3, 3.0)]:
        P12 = oracle.perm_prob(0.05, D1, D2, 2e-4)
        P21 = oracle.perm_prob(0.05, D2, D1, 2e-4)
        assert abs(P12 / P21 - math.sqrt(D2 / D1)) < 1e-13


def test_perm_prob_limits():
    assert oracle.perm_prob(0.0, 2.0, 2.0, 2e-4) == 0.0
    assert oracle.perm_prob(1e9, 2.0, 2.0, 2e-4) <= 1.0
    # the uncapped expression tends to 2 D2/(D1 sqrt(D2/D1) + D2) -> capped at 1 for D1 < D2
    assert oracle.perm_prob(1e12, 1.0, 4.0, 2e-4) == 1.0


def test_tables():
    D = np.array([2.5, 2.0, 2.0])
    kap = np.full((3, 3), 0.02)
    dead = np.array([0, 0, 1], np.uint8)
    sigma, thr, inv = oracle.tables(D, kap, np.array([60.0, 80.0, np.inf]), dead, 2e-4, 0.1)
    assert np.allclose(sigma[:2], np.sqrt(6 * D[:2] * 2e-4) / 0.1, rtol=0, atol=1e-15)
    assert np.all(np.diag(thr) == 2**32)
    P01 = oracle.perm_prob(0.02, 2.5, 2.0, 2e-4)
    assert thr[0, 1] == math.floor(P01 * 2**32)
    assert thr[0, 2] == 0 and thr[2, 0] == 0 and thr[1, 2] == 0
    assert inv[0] == 1 / 60.0 and inv[2] == 0.0
    with pytest.raises(oracle.OracleError) as e:
        oracle.tables(np.array([2.0]), None, None, None, 1e-3, 0.1)  # ds = 0.11 um > 0.1 um
    assert e.value.code == -3


def test_discrete_b_tends_to_pgse_formula():
    """Section 2.3: a PGSE of unit strength has b = delta^2 (Delta - delta/3);
    the discrete b of the sampled shape converges to it as dt -> 0."""
    from rms_inputs import pgse
    delta, Delta = 0.5, 1.5
    errs = []
    for dt in (1e-3, 2.5e-4):
        n = int(round(2.0 / dt))
        bd, k = oracle.bscale(pgse(n, dt, delta, Delta), dt, [0.0, 1.0])
        exact = delta ** 2 * (Delta - delta / 3)
        errs.append(abs(bd[0] - exact) / exact)
        assert k[0, 0] == 0.0 and abs(k[0, 1] ** 2 * bd[0] - 1.0) < 1e-12
    assert errs[1] < errs[0] and errs[1] < 1e-3


def test_zero_waveform_rejects_nonzero_b():
    with pytest.raises(oracle.OracleError):
        oracle.bscale(np.zeros(100), 1e-3, [1.0])


# ------------------------------------------------------------ single steps ---

def _tables(D, dt=2e-4, vox=0.1, kappa=None, n=None):
    D = np.atleast_1d(np.asarray(D, float))
    return oracle.tables(D, kappa, None, None, dt, vox)


def test_free_step_moves_exactly_ds():
    lab = np.zeros((4, 4, 4), np.uint8)
    sigma, thr, inv = _tables([2.0])
    rng = np.random.default_rng(3)
    for _ in range(200):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        off = rng.uniform(size=3)
        r = oracle.single_step(lab, 0.1, 2e-4, sigma, thr, inv, [1, 2, 3], off, 0, v)
        assert abs(np.linalg.norm(r["dx"]) - sigma[0] * 0.1) < 1e-15
        # the continuous position advanced by sigma * v with carries into the voxel index
        pos0 = np.array([1, 2, 3]) + off
        pos1 = r["vox"] + r["off"]
        d = (pos1 - pos0 + 2) % 4 - 2  # periodic minimum image
        assert np.allclose(d, sigma[0] * v, atol=1e-14)
        assert r["hits"] == 0


def _fold(x):
    """Specular reflection off the faces of [0, 1]."""
    if x < 0:
        return -x
    if x > 1:
        return 2 - x
    return x


def test_corner_reflector_single_voxel_cell():
    """Section 2.1.1 and the corner-reflector figure: inside a one-voxel cell
    with impermeable faces a step meets at most three faces and each one flips
    the normal component; the end point is the folded free end point."""
    lab = np.zeros((3, 3, 3), np.uint8)
    lab[1, 1, 1] = 1
    sigma, thr, inv = _tables([2.0, 2.0])
    s = sigma[1]
    cases = [
        ([0.9, 0.9, 0.9], [1, 1, 1], 3),
        ([0.05, 0.95, 0.5], [-1, 1, 0.2], 2),
        ([0.8, 0.5, 0.5], [1, 0, 0], 1),
        ([0.5, 0.5, 0.5], [1, 1, 1], 0),
        ([0.99, 0.02, 0.97], [0.3, -0.5, 1.0], 3),
    ]
    for off, v, n_ev in cases:
        v = np.array(v, float)
        v /= np.linalg.norm(v)
        r = oracle.single_step(lab, 0.1, 2e-4, sigma, thr, inv, [1, 1, 1], off, 1, v)
        want = np.array([_fold(o + s * c) for o, c in zip(off, v)])
        assert r["events"] == n_ev and r["hits"] == n_ev and r["perms"] == 0
        assert np.allclose(r["off"], want, atol=1e-14)
        assert list(r["vox"]) == [1, 1, 1] and r["label"] == 1
        assert np.allclose(r["dx"], (want - np.array(off)) * 0.1, atol=1e-15)


def test_membrane_pass_reflect_and_remaining_length():
    """A face between different labels: a membrane word below the threshold
    permeates, one at or above it reflects (section 2.1.3).  After permeating
    into a compartment of different D the rest of the step's duration is kept,
    so the remaining length scales by sqrt(D2/D1)."""
    lab = np.zeros((2, 2, 2), np.uint8)
    lab[:, :, 1] = 1  # x = 1 column is label 1
    D1, D2 = 1.0, 2.0
    dt = 2e-4
    sigma, _, inv = _tables([D1, D2], dt=dt)
    thr = np.array([[2**32, 1000], [1000, 2**32]], np.uint64)
    off = [1.0 - 0.1 * sigma[0], 0.5, 0.5]  # 10% of the step to the +x face
    v = [1.0, 0.0, 0.0]
    r = oracle.single_step(lab, 0.1, dt, sigma, thr, inv, [0, 0, 0], off, 0, v, (999, 0, 0))
    assert r["perms"] == 1 and r["label"] == 1 and list(r["vox"]) == [1, 0, 0]
    assert abs(r["off"][0] - 0.9 * sigma[1]) < 1e-14  # 90% of the duration at sigma_2
    r = oracle.single_step(lab, 0.1, dt, sigma, thr, inv, [0, 0, 0], off, 0, v, (1000, 0, 0))
    assert r["perms"] == 0 and r["label"] == 0 and list(r["vox"]) == [0, 0, 0]
    assert abs(r["off"][0] - (1.0 - 0.9 * sigma[0])) < 1e-14


def test_same_label_face_is_transparent():
    lab = np.full((2, 2, 2), 7, np.uint8)
    sigma, thr, inv = oracle.tables(np.full(8, 2.0), None, None, None, 2e-4, 0.1)
    r = oracle.single_step(lab, 0.1, 2e-4, sigma, thr, inv, [1, 1, 1], [0.99, 0.99, 0.99],
                           7, np.array([1, 1, 1]) / math.sqrt(3))
    assert r["events"] == 3 and r["hits"] == 0 and list(r["vox"]) == [0, 0, 0]  # wrapped


def test_dead_label_never_entered():
    lab = np.zeros((2, 2, 2), np.uint8)
    lab[:, :, 1] = 1
    sigma, thr, inv = oracle.tables(np.array([2.0, 2.0]), np.full((2, 2), 1e6), None,
                                    np.array([0, 1], np.uint8), 2e-4, 0.1)
    assert thr[0, 1] == 0
    r = oracle.single_step(lab, 0.1, 2e-4, sigma, thr, inv, [0, 0, 0], [0.99, 0.5, 0.5], 0,
                           [1.0, 0, 0], (0, 0, 0))
    assert r["label"] == 0 and r["hits"] == 1 and r["perms"] == 0
