"""Host checks of bench.py: the one-GPU guard and the lookup of HBM traffic in
the rocprofv3 summaries (taken only from a summary of the same workload made
on the current kernel sources)."""
import os
import subprocess
import sys

import bench
from paper_1611_02274_amd.build import kernel_source_digest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def _summary(path, workload, sha, nbytes):
    with open(path, "w") as fh:
        fh.write("# a summary\n\n| Kernel | Calls |\n|---|---|\n\n## Machine-readable\n\n")
        fh.write(f"traffic_workload: {workload}\nkernel_source_sha1: {sha}\n")
        fh.write(f"traffic_bytes_per_launch: {nbytes}\n")


def test_traffic_only_from_a_matching_summary(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    digest = kernel_source_digest()
    _summary(prof / "a_stale.md", "net53_rkc", "0" * 40, 111)
    _summary(prof / "b_other.md", "net13_rkc", digest, 222)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("net53_rkc") == (None, None)
    _summary(prof / "c_match.md", "net53_rkc", digest, 6063255426)
    assert bench.measured_traffic("net53_rkc") == (6063255426.0, "c_match.md")
    assert bench.measured_traffic("net13_rkc") == (222.0, "b_other.md")
    assert bench.measured_traffic("ragged") == (None, None)


def test_committed_summaries_are_machine_readable():
    """Every committed summary names its workload, the sources it was taken on
    and a positive byte count (or none for a timing-only summary)."""
    import glob
    paths = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert paths
    for path in paths:
        kv = {}
        with open(path) as fh:
            for line in fh:
                k, sep, v = line.strip().partition(":")
                if sep and k.startswith(("traffic_", "kernel_source")):
                    kv[k.strip()] = v.strip()
        assert kv.get("traffic_workload"), path
        assert len(kv.get("kernel_source_sha1", "")) == 40, path
        if "traffic_bytes_per_launch" in kv:
            assert float(kv["traffic_bytes_per_launch"]) > 0, path
