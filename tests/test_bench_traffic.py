"""Host logic of bench.py's roofline traffic: a committed counter summary is
used only while the kernel sources it was taken with are unchanged."""
import hashlib
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _tree(tmp_path, wl, sources, recorded_sha=None):
    name, files = bench.TRAFFIC_FILES[wl]
    csrc = tmp_path / "paper_2003_06027_amd" / "csrc"
    csrc.mkdir(parents=True)
    h = hashlib.sha256()
    for f in files:
        (csrc / f).write_bytes(sources[f])
        h.update(sources[f])
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = recorded_sha or h.hexdigest()
    (prof / name).write_text(f"fetch_scale 2.0\nkernel_source_sha256 {sha}\n"
                             "step_forward 100 bytes  algorithmic 90 bytes  ratio 1.111\n"
                             "step_adjoint 300 bytes  algorithmic 280 bytes  ratio 1.071\n")
    return files


@pytest.mark.parametrize("wl", sorted(bench.TRAFFIC_FILES))
def test_traffic_read_while_sources_match(tmp_path, monkeypatch, wl):
    files = bench.TRAFFIC_FILES[wl][1]
    _tree(tmp_path, wl, {f: f"// {f}\n".encode() for f in files})
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("forward", wl) == 100
    assert bench.measured_traffic("adjoint", wl) == 300
    assert bench.measured_traffic("recompute", wl) is None      # no such line


@pytest.mark.parametrize("wl", sorted(bench.TRAFFIC_FILES))
def test_traffic_dropped_after_a_source_change(tmp_path, monkeypatch, wl):
    files = bench.TRAFFIC_FILES[wl][1]
    _tree(tmp_path, wl, {f: f"// {f}\n".encode() for f in files}, recorded_sha="0" * 64)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("forward", wl) is None


def test_committed_summaries_parse():
    for wl in bench.TRAFFIC_FILES:
        for ph in ("forward", "recompute", "adjoint"):
            v = bench.measured_traffic(ph, wl)
            assert v is None or v > 0
