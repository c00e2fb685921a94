"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host only): a small driver links rms_oracle.c built with both sanitizers and
runs walks that take every branch of the walk (membranes that permeate and
reflect, dead labels, absorbing membranes, spin concentrations with both
permeation rules, recorded moments, several threads); the run must end
cleanly with no sanitizer report.  Skipped if gcc cannot link the sanitizer
runtimes."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int rmso_run(const void*, int, const int64_t*, double, int, const double*, const double*,
             const double*, const uint8_t*, uint64_t, int64_t, const int64_t*, int64_t, double,
             int, const double*, int, const double*, int, const double*, int, double*, double*,
             double*, double*, double*, double*, double*, int64_t*, double*, int,
             const int64_t*, double*, const double*, const double*, double, int);
int main(void) {
    enum { N = 12 };
    static uint8_t lab[N * N * N];
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x) {
                const double r2 = (x - 5.5) * (x - 5.5) + (y - 5.5) * (y - 5.5);
                lab[(z * N + y) * N + x] = x == 0 ? 2 : (r2 <= 16.0 ? 1 : 0);
            }
    const int64_t dims[3] = {N, N, N};
    const double D[3] = {2.5, 2.0, 1.0};
    double kap[9] = {0, 0.4, 0, 0.4, 0, 0, 0, 0, 0};
    const double T2[3] = {60.0, 80.0, INFINITY};
    const uint8_t dead[3] = {0, 0, 1};
    double rho[9] = {0, 0.02, 0, 0.01, 0, 0, 0, 0, 0};
    const double conc[3] = {0.7, 1.0, 1.0};
    const int64_t n_steps = 400;
    double* wf = calloc(2 * n_steps, sizeof(double));
    for (int i = 0; i < 50; ++i) { wf[10 + i] = 1.0; wf[300 + i] = -1.0; wf[n_steps + 20 + i] = -1.0; wf[n_steps + 250 + i] = 1.0; }
    const double dirs[6] = {1, 0, 0, 0.3, 0.4, 0.5};
    const double bvals[2] = {0.0, 1.0};
    double sig[2 * 2 * 2 * 2], m2[6], m4[15], Dd[2], Kd[2], sa, bd[2], rec[3 * (22 + 4)];
    int64_t cnt[3];
    const int64_t rs[3] = {1, 200, 400};
    double* dump = malloc(sizeof(double) * 700 * (15 + 6));
    int rc = 0;
    for (int variant = 0; variant < 4; ++variant) {
        const double* r = variant == 1 || variant == 3 ? rho : NULL;
        const double* c = variant >= 2 ? conc : NULL;
        rc |= rmso_run(lab, 1, dims, 0.1, 3, D, kap, T2, dead, 7 + variant, 700, NULL, n_steps,
                       2e-4, 2, wf, 2, dirs, 2, bvals, 3, sig, m2, m4, Dd, Kd, &sa, bd, cnt,
                       dump, 3, rs, rec, r, c, variant == 3 ? -1.0 : 0.0, variant == 3);
        if (!(sa > 0.0)) rc |= 1;
    }
    printf("rc %d sum_alpha %.6f permeations %lld\n", rc, sa, (long long)cnt[2]);
    free(dump);
    free(wf);
    return rc != 0;
}
"""


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    src = tmp_path / "driver.c"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-pthread",
           str(src), os.path.join(ROOT, "oracle", "rms_oracle.c"), "-lm", "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer runtimes not available: " + r.stderr[-300:])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr[-3000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
    assert run.stdout.startswith("rc 0")
