"""Host logic of bench.py, on the CPU: the one-GPU guard, and the rule that HBM counter figures
taken on other kernel sources are not reported (the traffic of a changed kernel is unknown)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("argv, env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT, capture_output=True,
                       text=True, timeout=120, env={**os.environ, **env})
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def _summary(tmp_path, sha, kernel="k"):
    blob = {"kernel": kernel, "source_sha256": sha, "traffic_bytes_per_launch": 123.0}
    p = tmp_path / "traffic.md"
    p.write_text("# traffic\n\n```json\n" + json.dumps(blob) + "\n```\n")
    return str(p)


def test_traffic_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    sha = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, sha))
    assert bench.load_traffic("k") == 123.0
    assert bench.load_traffic("other_kernel") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", _summary(tmp_path, "0" * 64))
    assert bench.load_traffic("k") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.load_traffic("k") is None


def test_source_hash_covers_every_kernel_source(tmp_path, monkeypatch):
    """One changed byte in any HIP source or header changes the hash."""
    src = os.path.join(ROOT, "paper_2511_08929_amd", "csrc")
    names = sorted(f for f in os.listdir(src) if f.endswith((".hip", ".hpp", ".h")))
    assert names
    fake = tmp_path / "paper_2511_08929_amd" / "csrc"
    fake.mkdir(parents=True)
    for f in names:
        (fake / f).write_bytes(open(os.path.join(src, f), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_source_hash()
    assert base == bench.kernel_source_hash()
    for f in (names[0], names[-1]):
        data = (fake / f).read_bytes()
        (fake / f).write_bytes(data + b" ")
        assert bench.kernel_source_hash() != base
        (fake / f).write_bytes(data)
    assert bench.kernel_source_hash() == base
