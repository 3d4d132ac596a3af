"""Host-side logic of the launch-shape autotuner."""
from paper_1903_01081_amd.tune import candidates


def test_candidates_cover_every_solver_and_shape():
    c = candidates(0)
    solvers = {s["solver"] for s in c}
    assert solvers == {"auto", "sparse", "dense", "compensation"}
    assert {s.get("block_size") for s in c if s["solver"] == "auto"} >= {0, 64, 256, 512}
    assert {s.get("dense_tail") for s in c if s["solver"] == "auto"} >= {64, 128}
    assert {s.get("split_cols") for s in c if s["solver"] == "dense"} == {16, 32}


def test_candidates_skip_split_widths_with_checkpoints():
    # the split dense solver runs forward only: with checkpoints only the
    # default dense shape is tried (the library rejects it if it would split)
    c = candidates(500)
    assert [s for s in c if s["solver"] == "dense"] == [dict(solver="dense")]


def test_packing_candidates_only_where_they_change_the_items():
    from paper_1903_01081_amd import netgen
    from paper_1903_01081_amd.tune import PACK_BUDGETS, _packing_changes_items
    assert any(s.get("pack_nodes", 0) in PACK_BUDGETS for s in candidates(0))
    big, cfg = netgen.config1(n_bus=400, n_steps=10)      # three 400-node phases
    small, cfg4 = netgen.config4(n_inst=4, n_steps=10)
    shape = dict(solver="auto", pack_nodes=256)
    assert not _packing_changes_items(big, cfg["dt"], 10, 0, shape)
    assert _packing_changes_items(small, cfg4["dt"], 10, 0, shape)
    assert _packing_changes_items(big, cfg["dt"], 10, 0, dict(solver="auto"))


def test_compensation_candidate_only_without_checkpoints():
    assert dict(solver="compensation") in candidates(0)
    assert all(s["solver"] != "compensation" for s in candidates(500))
