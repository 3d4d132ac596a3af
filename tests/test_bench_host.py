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


def test_roofline_object_prices_the_method_bytes():
    # frac = the sparse method's bytes per time step x time steps (x passes)
    # / kernel seconds / 8 TB/s, whichever solver ran
    info = {"total_branches": 100, "nnz_L": 40, "total_nodes": 30}
    r = bench.roofline_object(info, 5, 1000, "k_split", 1e-3)
    per_step = 64 * 100 + 8 * 5 + 24 * 40 + 8 * 30
    assert r["algorithmic_bytes_per_time_step"] == per_step
    assert abs(r["achieved"] - per_step * 1000 / 1e-3 / 1e9) < 1e-9
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-15
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["traffic"] is None
    r2 = bench.roofline_object(info, 5, 1000, "k_adjoint", 1e-3, passes=2.0, extra_bytes_per_step=32)
    assert abs(r2["achieved"] - (per_step + 32) * 2000 / 1e-3 / 1e9) < 1e-9
    r3 = bench.roofline_object(info, 5, 1000, "k_split", 1e-3, traffic=4e6)
    assert abs(r3["traffic_gbs"] - 4.0) < 1e-12
