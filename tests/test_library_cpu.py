"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects bad substrates before touching a device."""
import os
import re

import numpy as np
import pytest

import paper_2012_06478_amd as rms

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "rms.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rms_\w+)\s*\(", text, re.M)))


def test_header_symbols_exported():
    names = _declared_functions()
    assert "rms_run" in names and "rms_create_substrate" in names
    lib = rms._load()
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version_matches_header():
    text = open(os.path.join(ROOT, "include", "rms.h")).read()
    v = int(re.search(r"#define RMS_ABI_VERSION (\d+)", text).group(1))
    assert rms.rms_abi_version() == v


def test_label_range_rejected_before_device():
    lab = np.zeros((4, 4, 4), np.uint8)
    lab[0, 0, 0] = 3
    with pytest.raises(rms.RmsError) as e:
        rms.rms_create_substrate(lab, 0.1, [2.0, 2.0])
    assert e.value.code == -2
    assert "label 3" in rms.rms_last_error()


@pytest.mark.parametrize("bad", [dict(voxel_um=0.0), dict(D=[])])
def test_bad_substrate_arguments(bad):
    kw = dict(labels=np.zeros((2, 2, 2), np.uint8), voxel_um=0.1, D=[2.0])
    kw.update(bad)
    with pytest.raises(rms.RmsError) as e:
        rms.rms_create_substrate(**kw)
    assert e.value.code == -1


def test_binding_checks_array_sizes_before_the_library_reads_them():
    """The library reads n_shapes * n_steps waveform samples and n_labels (or
    n_labels^2) tissue values through raw pointers: the binding refuses arrays
    of other sizes before any call."""
    fake = rms.Substrate(None, (2, 2, 2), 2, 0.1)  # never reaches the library
    run = dict(seed=1, n_walkers=8, n_steps=10, dt=2e-4, dirs=[[1.0, 0, 0]], bvals=[0.0])
    with pytest.raises(ValueError, match="waveform"):
        rms.rms_run(fake, waveform=np.zeros((1, 9)), **run)
    with pytest.raises(ValueError, match="waveform"):
        rms.rms_run_record(fake, waveform=np.zeros((2, 11)), record_steps=[5], **run)
    with pytest.raises(ValueError, match="T2"):
        rms.rms_run(fake, params=dict(D=[2.0, 2.0], T2=[80.0]), **run)
    with pytest.raises(ValueError, match="kappa"):
        rms.rms_run(fake, params=dict(D=[2.0, 2.0], kappa=np.zeros(3)), **run)
    with pytest.raises(ValueError, match="rho"):
        rms.rms_run(fake, params=dict(D=[2.0, 2.0], rho=np.zeros((3, 3))), **run)
    with pytest.raises(ValueError, match="conc"):
        rms.rms_run(fake, params=dict(D=[2.0, 2.0], conc=[1.0, 1.0, 1.0]), **run)
    with pytest.raises(ValueError, match="D must have 2"):
        rms.rms_run(fake, params=dict(D=[2.0, 2.0, 2.0]), **run)
    with pytest.raises(ValueError, match="dirs"):
        rms.rms_run(fake, dirs=np.zeros((2, 2)), seed=1, n_walkers=8, n_steps=10, dt=2e-4)
    lab = np.zeros((2, 2, 2), np.uint8)
    with pytest.raises(ValueError, match="T2"):
        rms.rms_create_substrate(lab, 0.1, [2.0, 2.0], None, [80.0])
    with pytest.raises(ValueError, match="kappa"):
        rms.rms_create_substrate(lab, 0.1, [2.0, 2.0], np.zeros(2))
    with pytest.raises(ValueError, match="dead"):
        rms.rms_create_substrate(lab, 0.1, [2.0, 2.0], dead=[0, 0, 1])


def test_set_option_validates_without_a_device():
    with pytest.raises(rms.RmsError) as e:
        rms.rms_set_option(99, 0)
    assert e.value.code == -1
    with pytest.raises(rms.RmsError):
        rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, 7)
    with pytest.raises(rms.RmsError):
        rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, -1)
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_ONE_LAUNCH)
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 0)
    rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, rms.RMS_WALK_AUTO)
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 1 << 20)
    text = open(os.path.join(ROOT, "include", "rms.h")).read()
    for name in ("RMS_WALK_ONE_LAUNCH", "RMS_WALK_PERSISTENT", "RMS_WALK_PACKED",
                 "RMS_OPT_WALK_KERNEL", "RMS_OPT_SEG_POLL_LIMIT", "RMS_OPT_SERVER_WALKERS"):
        assert getattr(rms, name) == int(re.search(rf"#define {name} (\d+)", text).group(1))
    assert rms.ERROR_NAMES[rms.RMS_E_WAIT_GAVE_UP] == "RMS_E_WAIT_GAVE_UP"
    assert int(re.search(r"#define RMS_E_WAIT_GAVE_UP \((-\d+)\)", text).group(1)) == -10


def test_header_limits_match_binding():
    text = open(os.path.join(ROOT, "include", "rms.h")).read()
    for name in ("RMS_MAX_SHAPES", "RMS_MAX_SIGNALS", "RMS_MAX_LABELS", "RMS_DUMP_FIXED"):
        v = int(re.search(rf"#define {name} (\d+)", text).group(1))
        assert getattr(rms, name) == v
    v = float(re.search(r"#define RMS_MAX_PERM_PROB ([0-9.]+)", text).group(1))
    assert rms.RMS_MAX_PERM_PROB == v


_SINCOS_PROBE = r"""
#include "rms_host.h"
#include "rms_device.h"
#include <cmath>
#include <cstdio>
#include <random>
int main() {
    double2 tab[rms::kTrigSize + 1];
    rms::fill_trig_table(tab);
    std::mt19937_64 g(1);
    const uint32_t edge[] = {0u, 0x00ffffffu, 0x01000000u, 0x3fffffffu, 0x40000000u,
                             0x80000000u, 0xbfffffffu, 0xffffffffu};
    double maxe = 0.0;
    for (int i = 0; i < 2000000; ++i) {
        const uint32_t w = i < 8 ? edge[i] : static_cast<uint32_t>(g());
        double s, c;
        rms::dev::sincos_2pi_word(w, tab, tab[rms::kTrigSize], &s, &c,
                                  [](double a, double b, double k) { return std::fma(a, b, k); });
        const long double th = 2.0L * 3.14159265358979323846264338327950288L *
                               ((static_cast<long double>(w) + 0.5L) * 0x1p-32L);
        // the function returns 2 sin and 2 cos
        maxe = std::fmax(maxe, std::fabs(static_cast<double>(sinl(th) - 0.5L * s)));
        maxe = std::fmax(maxe, std::fabs(static_cast<double>(cosl(th) - 0.5L * c)));
    }
    std::printf("%.3e\n", maxe);
    return 0;
}
"""


def test_device_sincos_2pi_accuracy(tmp_path):
    """The double-precision walker's cos/sin of 2 pi u (angle table of 256
    entries holding twice the cosine and sine, short Taylor series of the
    remainder, angle-sum formulas) against long-double libm, on the host build
    of the same function with the library's own table."""
    import shutil
    import subprocess
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    src = tmp_path / "sc.cpp"
    exe = tmp_path / "sc"
    src.write_text(_SINCOS_PROBE)
    csrc = os.path.join(ROOT, "paper_2012_06478_amd", "csrc")
    subprocess.check_call(["hipcc", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", csrc, "-o", str(exe), str(src)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL, timeout=300)
    err = float(subprocess.run([str(exe)], capture_output=True, text=True, check=True,
                               timeout=120).stdout)
    print(f"max error {err:.3e}")
    assert err < 4e-16


_ORDER_PROBE = r"""
#include "rms_device.h"
#include <cmath>
#include <cstdio>
#include <random>
template <typename Real>
long check(std::mt19937_64& g, long n) {
    std::uniform_real_distribution<double> U(0.0, 1.0);
    long bad = 0;
    for (long i = 0; i < n; ++i) {
        Real gg[3], m[3];
        for (int a = 0; a < 3; ++a) {
            gg[a] = static_cast<Real>(i % 7 == 0 && a == 1 ? 0.0 : U(g));  // some gaps exactly 0
            m[a] = static_cast<Real>(U(g) + 1e-9);
        }
        int ax[3];
        rms::dev::event_order(gg, m, ax);
        bool perm = ax[0] != ax[1] && ax[0] != ax[2] && ax[1] != ax[2] &&
                    ax[0] >= 0 && ax[0] < 3 && ax[1] >= 0 && ax[1] < 3 && ax[2] >= 0 && ax[2] < 3;
        if (!perm) { ++bad; continue; }
        long double e[3];
        for (int a = 0; a < 3; ++a) e[a] = static_cast<long double>(gg[a]) / m[a];
        if (e[ax[0]] > e[ax[1]] || e[ax[1]] > e[ax[2]]) ++bad;
    }
    return bad;
}
// exact ties (zero gaps, equal ratios) must keep the lower axis first
template <typename Real>
long ties() {
    long bad = 0;
    const Real gs[4] = {Real(0), Real(0.25), Real(0.5), Real(0.75)};
    for (int mask = 0; mask < 64; ++mask) {
        Real gg[3], m[3];
        for (int a = 0; a < 3; ++a) {
            gg[a] = gs[(mask >> (2 * a)) & 3];
            m[a] = Real(0.5);  // equal |v|: equal gaps are exact ties
        }
        int ax[3];
        rms::dev::event_order(gg, m, ax);
        for (int k = 0; k < 2; ++k) {
            const Real ek = gg[ax[k]], en = gg[ax[k + 1]];
            if (ek > en || (ek == en && ax[k] > ax[k + 1])) ++bad;
        }
    }
    return bad;
}
int main() {
    std::mt19937_64 g(7);
    std::printf("%ld %ld %ld %ld\n", check<double>(g, 1000000), check<float>(g, 1000000),
                ties<double>(), ties<float>());
    return 0;
}
"""


def test_device_event_order(tmp_path):
    """The walker's division-free order of a step's face events (pairwise
    cross-multiplied comparisons indexing a permutation table) against sorting
    the path lengths gap / |v| in long double, and exact ties (zero gaps,
    equal ratios) kept in axis order, on the host build of the same function,
    for both precision forms."""
    import shutil
    import subprocess
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    src = tmp_path / "order.cpp"
    exe = tmp_path / "order"
    src.write_text(_ORDER_PROBE)
    csrc = os.path.join(ROOT, "paper_2012_06478_amd", "csrc")
    subprocess.check_call(["hipcc", "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", csrc, "-o", str(exe), str(src)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL, timeout=300)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True,
                         timeout=120).stdout.split()
    assert out == ["0", "0", "0", "0"], out


def test_label_range_names_the_first_bad_voxel_of_a_large_volume():
    """Volumes of more than 2^22 voxels are scanned by several host threads
    over contiguous ranges: the error still names the first bad voxel."""
    lab = np.zeros((130, 200, 200), np.uint16)  # 5.2e6 voxels, z slowest
    lab[120, 7, 9] = 900   # in a late range
    lab[40, 3, 5] = 700    # the first one in voxel order
    with pytest.raises(rms.RmsError) as e:
        rms.rms_create_substrate(lab, 0.1, [2.0, 2.0])
    assert e.value.code == -2
    first = (40 * 200 + 3) * 200 + 5
    assert f"voxel {first} has label 700" in rms.rms_last_error()


@pytest.mark.parametrize("option,value,needle", [
    (rms.RMS_OPT_WALK_KERNEL, 7, "RMS_OPT_WALK_KERNEL"),
    (rms.RMS_OPT_SERVER_WALKERS, -1, "RMS_OPT_SERVER_WALKERS"),
    (rms.RMS_OPT_SEG_POLL_LIMIT, -1, "RMS_OPT_SEG_POLL_LIMIT"),
    (rms.RMS_OPT_SEG_POLL_LIMIT, 1 << 32, "RMS_OPT_SEG_POLL_LIMIT"),
    (99, 0, "unknown option"),
])
def test_options_refuse_values_outside_their_range(option, value, needle):
    """Launch and server options are checked on the host; a refused value
    leaves the option as it was."""
    with pytest.raises(rms.RmsError) as e:
        rms.rms_set_option(option, value)
    assert e.value.code == -1
    assert needle in rms.rms_last_error()


def test_options_accept_their_documented_values():
    for v in (rms.RMS_WALK_ONE_LAUNCH, rms.RMS_WALK_PERSISTENT, rms.RMS_WALK_AUTO):
        rms.rms_set_option(rms.RMS_OPT_WALK_KERNEL, v)
    rms.rms_set_option(rms.RMS_OPT_SERVER_WALKERS, 123456)
    rms.rms_set_option(rms.RMS_OPT_SERVER_WALKERS, 0)          # automatic again
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 0xFFFFFFFE)
    rms.rms_set_option(rms.RMS_OPT_SEG_POLL_LIMIT, 1 << 20)    # the default
