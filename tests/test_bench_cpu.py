"""CPU checks of bench.py's contract: one GPU only, the walk kernel it names
for a workload, and the traffic figure tied to the profiled kernel sources."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _case(n_walkers, n_shapes=1, dtype=np.uint16):
    return dict(labels=np.zeros((4, 4, 4), dtype), n_walkers=n_walkers, n_steps=10,
                waveform=np.zeros((n_shapes, 10)))


def test_walk_kernel_name_takes_the_kind_the_library_reports():
    assert bench.walk_kernel_name(True, _case(1_000_000), "persistent").startswith(
        "walk_seg_kernel<WalkerF64T<uint16,1,false>>")
    assert bench.walk_kernel_name(True, _case(10_000, 1, np.uint8), "one launch") == (
        "walk_kernel<WalkerF64T<uint8,1,false>> (one launch)")
    assert "<uint16,2,false>" in bench.walk_kernel_name(False, _case(10_000_000, 2),
                                                        "one launch")


def test_default_workload_is_the_axon_bundle():
    src = open(os.path.join(ROOT, "bench.py")).read()
    assert 'choices=WORKLOADS, default="axons"' in src
    c = bench.WORKLOADS
    assert "axons" in c


def test_traffic_needs_the_profiled_sources():
    """The traffic figure is reported only while the walk sources hash to the
    value recorded with the counters."""
    sha = bench.kernel_sha()
    assert len(sha) == 16 and int(sha, 16) >= 0
    t = bench.traffic_from_profile("axons400x400x1000_u16", "fp64")
    assert t is None or t > 0


def test_committed_counters_match_the_walk_sources():
    """The committed counter summaries of the default workload (both forms)
    were taken on the current walk sources, so the bench line carries their
    traffic; a change to the walk sources needs the counters taken again."""
    for form in ("fp64", "mixed"):
        t = bench.traffic_from_profile("axons400x400x1000_u16", form)
        assert t is not None and t > 0, form
