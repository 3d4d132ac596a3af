"""Host-side logic of bench.py: the measured-traffic record is used only
while the step kernel's sources are the ones it was measured on."""
import json

import bench


def test_traffic_record_matches_current_sources():
    assert bench.measured_traffic() is None or bench.measured_traffic() > 0


def test_traffic_record_ignored_after_kernel_change(tmp_path, monkeypatch):
    prof = tmp_path / "p.md"
    rec = {"source_digest": "0" * 16, "bytes_per_launch": 123}
    prof.write_text("x\ntraffic-record: " + json.dumps(rec) + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(prof))
    assert bench.measured_traffic() is None
    rec["source_digest"] = bench.kernel_source_digest()
    prof.write_text("traffic-record: " + json.dumps(rec) + "\n")
    assert bench.measured_traffic() == 123.0


def test_gpus_above_one_exit(monkeypatch, capsys):
    import pytest
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().err


def test_algorithmic_figures_per_step():
    # the per-step figures the roofline divides by: sparse sweeps vs the
    # dense inverse of each component
    import bench
    info = {"total_branches": 100, "nnz_L": 40, "total_nodes": 30}
    assert bench.algorithmic_flops_per_step(info) == 10 * 100 + 4 * 40 + 30
    assert bench.algorithmic_flops_per_step(info, [10, 20]) == 10 * 100 + 2 * (100 + 400)
    assert bench.algorithmic_bytes_per_step(info, 5) == 64 * 100 + 8 * 5 + 24 * 40 + 8 * 30
    assert bench.algorithmic_bytes_per_step(info, 5, [10, 20]) == 64 * 100 + 8 * 5 + 8 * (100 + 400)
