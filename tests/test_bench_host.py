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


def test_driver_argv_keeps_the_workload():
    """The driver's `--steps 20 --warmup 5` sets how many whole collisions are timed; the collision
    itself stays the 3000-step head-on workload."""
    a = bench.parse_args(["--gpus", "1", "--steps", "20", "--warmup", "5"])
    assert (a.steps, a.warmup, a.gpus) == (20, 5, 1)
    assert bench.COLLISION_STEPS == 3000 and not hasattr(a, "time_steps")
    d = bench.parse_args([])
    assert d.steps >= 1 and d.warmup >= 0 and d.n == 1_000_000
    assert not d.probe and not d.probe_grid and bench.parse_args(["--probe-grid"]).probe_grid


@pytest.mark.parametrize("argv", [["--steps", "0"], ["--warmup", "-1"]])
def test_bad_counts_are_refused(argv):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""


def _spec(k, s_mean=(0.0, 0.0, 0.0)):
    import numpy as np
    k = np.asarray(k, dtype=float)
    return dict(k=k, xi2=np.zeros_like(k), lin=np.zeros_like(k), s_mean=np.asarray(s_mean))


def test_spectrum_error_handles_empty_and_sparse_inputs():
    import numpy as np
    e = bench.spectrum_error(_spec([]), _spec([]))
    assert e["bins"] == 0 and e["spectrum_max_rel"] is None and e["photons"] == 0
    e = bench.spectrum_error(_spec([1.0, 2.0, 3.0]), _spec([1.0]))        # no bin reaches min_count
    assert e["bins"] == 0 and e["spectrum_max_rel"] is None
    rng = np.random.default_rng(0)
    k = 10 ** rng.uniform(0, 2, 200_000)
    e = bench.spectrum_error(_spec(k), _spec(k, (0.0, 0.001, 0.0)))
    assert e["bins"] > 0 and e["spectrum_max_rel"] == 0.0 and e["spin_mean_abs"] == 0.001


def test_extras_are_fail_soft_and_budgeted():
    out = {}

    def boom():
        raise RuntimeError("no")

    assert bench.run_extra(out, "x", 1e9, boom) is None
    assert "RuntimeError" in out["errors"]["x"]
    assert bench.run_extra(out, "y", -1.0, boom) is None
    assert out["skipped"][0].startswith("y: time budget")
    assert bench.run_extra(out, "z", 1e9, lambda v: v + 1, 1) == 2


def test_roofline_bound_follows_the_longer_ceiling(monkeypatch):
    """Algorithmic bytes / 8 TB/s against committed VALU instructions / one per CU per cycle."""
    kt = {"plan_photon": (100, 4.0), "plan_lepton": (100, 2.0), "plan_process": (100, 1.0)}
    ck = {"n_lepton_steps": 10 ** 8, "n_photon_steps": 3 * 10 ** 8, "n_photon_qed": 10 ** 8}
    monkeypatch.setattr(bench, "load_valu", lambda k: None)
    monkeypatch.setattr(bench, "load_traffic", lambda k: None)
    r = bench.roofline(kt, ck, 5000.0)
    assert r["kernel"] == "plan_photon" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    bpl = 3 * 10 ** 8 * 52 / 100
    assert abs(r["achieved"] - bpl / 40e-6 / 1e9) < 0.1 and r["frac"] == r["hbm"]["frac"]
    # VALU work whose minimum time exceeds the HBM minimum time makes the bound ALU
    t_hbm = bpl / 8e12
    monkeypatch.setattr(bench, "load_valu", lambda k: 2.0 * t_hbm * 256 * 2.4e9)
    r = bench.roofline(kt, ck, 5000.0)
    assert r["bound"] == "alu" and r["frac"] == r["alu"]["frac"] and r["hbm"]["frac"] > 0
    monkeypatch.setattr(bench, "load_valu", lambda k: 0.5 * t_hbm * 256 * 2.4e9)
    assert bench.roofline(kt, ck, 5000.0)["bound"] == "hbm"


def test_ensemble_stores_follow_initial_chi():
    """The ensemble members' stores grow with their initial chi (the cascading members get the
    most room), never below the floors, and the full-count rule needs less room per electron."""
    import numpy as np
    from types import SimpleNamespace

    def member(n, gamma0, a0):
        p = np.zeros((3, n)); p[0] = np.sqrt(gamma0 ** 2 - 1.0)
        return SimpleNamespace(n=n, p=p, a0=a0)

    eps = bench.synth.EPS_R
    hot = member(10_000, 9000.0, 200.0)          # chi0 = 2 gamma0 a0 eps_r ~ 10.9
    warm = member(10_000, 9000.0, 100.0)         # ~ 5.5
    cold = member(10_000, 1000.0, 50.0)          # ~ 0.3
    assert 2 * 9000.0 * 200.0 * eps > 6.5 and 5 < 2 * 9000.0 * 100.0 * eps < 6.5
    for rule in ("compact50", "compact10"):
        c_hot, c_warm, c_cold = (bench.ensemble_caps(m, rule) for m in (hot, warm, cold))
        assert c_hot["cap_g"] > c_warm["cap_g"] > c_cold["cap_g"] >= 100_000
        assert c_hot["cap_p"] >= 4 * hot.n and c_cold["cap_p"] >= 1000
        assert c_hot["cap_e"] == hot.n + c_hot["cap_p"]
    assert bench.ensemble_caps(hot, "compact10")["cap_g"] < bench.ensemble_caps(hot, "compact50")["cap_g"]
    tiny = member(10, 9000.0, 200.0)
    assert bench.ensemble_caps(tiny, "compact50") == dict(cap_e=1010, cap_p=1000, cap_g=100_000)
