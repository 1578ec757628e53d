"""Host logic of bench.py that runs without a GPU: the one-GPU refusal and the
gate that reports the measured HBM traffic only for the kernel sources it was
measured on."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.strip().startswith("{")


def _fake_tree(tmp_path, sources, recorded_hash):
    csrc = tmp_path / "paper_2507_01770_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name, text in sources.items():
        (csrc / name).write_bytes(text)
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"bytes_per_sweep": 12345, "source_hash": recorded_hash}
    (prof / "hbm_bytes_sep_abs_sin2_n10000.md").write_text("# HBM bytes\n\n```json\n" + json.dumps(rec) + "\n```\n")


def test_traffic_reported_only_for_the_measured_sources(tmp_path, monkeypatch):
    sources = {"a.hip": b"kernel one\n", "b.hpp": b"header\n"}
    h = hashlib.sha256(b"".join(sources[k] for k in sorted(sources))).hexdigest()[:16]
    _fake_tree(tmp_path, sources, h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic() == 12345
    (tmp_path / "paper_2507_01770_amd" / "csrc" / "a.hip").write_bytes(b"kernel two\n")
    assert bench.measured_traffic() is None


def test_traffic_absent_without_a_profile(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic() is None


def test_every_result_field_bench_reads_exists():
    # bench.py reads solve results through these names; each must be a Result field
    import dataclasses
    import re
    import paper_2507_01770_amd as ibb
    fields = {f.name for f in dataclasses.fields(ibb.Result)}
    text = open(os.path.join(ROOT, "bench.py")).read()
    used = set(re.findall(r"\b(?:r|rp|rp1|rq|rs1|res)\.([a-z_][a-z0-9_]*)\b", text))
    assert used, "no result fields found"
    assert used <= fields, sorted(used - fields)
