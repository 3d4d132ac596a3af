"""Host-side logic of the launch-shape autotuner."""
from paper_1903_01081_amd.tune import candidates


def test_candidates_cover_every_solver_and_shape():
    c = candidates(0)
    solvers = {s["solver"] for s in c}
    assert solvers == {"auto", "sparse", "dense"}
    assert {s.get("block_size") for s in c if s["solver"] == "auto"} >= {0, 64, 256, 512}
    assert {s.get("dense_tail") for s in c if s["solver"] == "auto"} >= {64, 128}
    assert {s.get("split_cols") for s in c if s["solver"] == "dense"} == {16, 32}


def test_candidates_skip_split_widths_with_checkpoints():
    # the split dense solver runs forward only: with checkpoints only the
    # default dense shape is tried (the library rejects it if it would split)
    c = candidates(500)
    assert [s for s in c if s["solver"] == "dense"] == [dict(solver="dense")]
