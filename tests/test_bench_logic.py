"""Host logic of bench.py: the roofline's traffic record (read from the
committed counter summary, and only while the level kernel's source is the
one the counters were taken with)."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _bench():
    import bench
    return bench


def test_traffic_record_matches_source_hash(tmp_path, monkeypatch):
    b = _bench()
    src = os.path.join(ROOT, "paper_2606_28865_amd", "csrc", "levels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    prof = tmp_path / "profiles"
    prof.mkdir()
    (tmp_path / "paper_2606_28865_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2606_28865_amd" / "csrc" / "levels.hip").write_bytes(open(src, "rb").read())
    text = f"# x\n\n- levels.hip sha256[:16]: `{sha}`\n- bytes per launch: 8.5e+07\n"
    (prof / "multibody_fp64_hbm_counters.md").write_text(text)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.level_sums_traffic() == 8.5e7
    # a different source: the record is stale
    (prof / "multibody_fp64_hbm_counters.md").write_text(text.replace(sha, "0" * 16))
    assert b.level_sums_traffic() is None
    # no record
    (prof / "multibody_fp64_hbm_counters.md").unlink()
    assert b.level_sums_traffic() is None


def test_committed_traffic_record_parses():
    b = _bench()
    path = os.path.join(ROOT, "profiles", "multibody_fp64_hbm_counters.md")
    assert os.path.exists(path)
    v = b.level_sums_traffic()
    assert v is None or v > 1e6
