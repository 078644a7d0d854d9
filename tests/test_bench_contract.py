"""CPU checks of the benchmark's contract: one GPU only, and HBM traffic reported only
from counter runs taken on the current kernel source."""
from __future__ import annotations

import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, env=e, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_source_digest_ignores_comments_and_blank_lines(tmp_path, monkeypatch):
    b = _bench()
    d = tmp_path / "paper_2204_05821_amd" / "csrc"
    d.mkdir(parents=True)
    src = "int a = 1;  // one\n\n__global__ void k() {}\n"
    (d / "kernels.h").write_text(src)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    base = b.source_digest()
    (d / "kernels.h").write_text("// header comment\n" + src.replace("// one", "// another comment") + "\n\n")
    assert b.source_digest() == base
    (d / "kernels.h").write_text(src.replace("1", "2"))
    assert b.source_digest() != base


def test_traffic_reported_only_for_matching_source(tmp_path, monkeypatch):
    b = _bench()
    (tmp_path / "profiles").mkdir()
    entry = {"bytes_per_launch": 7.0e10, "source_digest": "abc", "read": 6.6e10, "written": 0.4e10}
    (tmp_path / "profiles" / "pmc_traffic.json").write_text(json.dumps({"w": {"k_sig_range": entry}}))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "source_digest", lambda: "abc")
    assert b.measured_traffic("k_sig_range", "w") == pytest.approx(7.0e10)
    assert b.measured_traffic("k_lookup", "w") is None
    assert b.measured_traffic("k_sig_range", "other") is None
    monkeypatch.setattr(b, "source_digest", lambda: "def")
    assert b.measured_traffic("k_sig_range", "w") is None


def test_committed_counter_runs_are_well_formed():
    """Every committed per-kernel traffic figure names its digest and adds up."""
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as f:
        data = json.load(f)
    assert "rmat_rdf_s27_m1B_k10" in data
    for workload, kernels in data.items():
        assert "k_sig_range" in kernels, workload
        for name, e in kernels.items():
            assert len(e["source_digest"]) == 16
            assert e["bytes_per_launch"] > 0
            assert e["bytes_per_launch"] == pytest.approx(e["read"] + e["written"], rel=1e-9)
