"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the network analysis of the library (validation, connected components,
ordering, symbolic LDL^T, sweep levels, dense-tail choice, the compensation
solver's plan) is built from its
sources with g++ -fsanitize=address,undefined, errors fatal, and run on the
seeded workloads' networks under every solver and launch-shape setting and
on invalid inputs (tests/host_asan/analysis_driver.cpp)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from paper_1903_01081_amd import netgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_batch(path, nets):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", len(nets)))
        for n in nets:
            B, V = int(n.n_branches), int(len(n.ev_step))
            has_ins = n.in_service0 is not None
            has_rec = n.rec_nodes is not None
            n_rec = int(len(n.rec_nodes)) if has_rec else int(n.n_nodes)
            f.write(struct.pack("<7i", int(n.n_nodes), B, 3 * int(n.n_lines), V, n_rec, int(has_ins), int(has_rec)))
            for a, t in ((n.k, np.int32), (n.m, np.int32), (n.kind, np.int32), (n.R, np.float64), (n.L, np.float64),
                         (n.C, np.float64), (n.E, np.float64), (n.omega, np.float64), (n.phase, np.float64),
                         (n.line, np.int32)):
                f.write(np.ascontiguousarray(a, t).tobytes())
            if has_ins:
                f.write(np.ascontiguousarray(n.in_service0, np.uint8).tobytes())
            f.write(np.ascontiguousarray(n.ev_step, np.int64).reshape(V).tobytes())
            f.write(np.ascontiguousarray(n.ev_branch, np.int32).reshape(V).tobytes())
            f.write(np.ascontiguousarray(n.ev_in_service, np.uint8).reshape(V).tobytes())
            if has_rec:
                f.write(np.ascontiguousarray(n.rec_nodes, np.int32).tobytes())


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("asan") / "analysis_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1903_01081_amd", "csrc"),
           os.path.join(ROOT, "paper_1903_01081_amd", "csrc", "analysis.cpp"),
           os.path.join(ROOT, "paper_1903_01081_amd", "csrc", "comp_plan.cpp"),
           os.path.join(ROOT, "tests", "host_asan", "analysis_driver.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


BATCHES = {
    "nine_bus": lambda: netgen.config0(n_steps=400)[0],
    "grid_events": lambda: [netgen.small_grid(5, 40, fault_step=30, remove_series=2, remove_step=60, n_mon=8)],
    "n1_sample": lambda: netgen.config2(n_scen=6)[0],
    "n1_events": lambda: netgen.config2(n_bus=20, n_scen=6, n_steps=400, event_step=100)[0],
    "uneven_sample": lambda: netgen.config4(n_inst=8, n_steps=400)[0],
    "grid1000": lambda: netgen.config1(n_steps=400)[0],
    "travelling_wave": lambda: [netgen.small_grid(7, 30, fault_step=30, travelling_wave_dt=20e-6),
                                netgen.small_grid(8, 12)],
}


@pytest.mark.parametrize("name", list(BATCHES))
def test_analysis_clean_under_sanitizers(driver, tmp_path, name):
    path = str(tmp_path / f"{name}.bin")
    write_batch(path, BATCHES[name]())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, path], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    ok = [ln.split(" ok ")[1] for ln in r.stdout.splitlines() if " ok " in ln and "pack_nodes" not in ln]
    assert ok, r.stdout
    # items and symbolic patterns do not depend on the solver or launch shape
    # (packing, which merges items, aside)
    sizes = {tuple(s.split()[:4]) for s in ok}
    assert len(sizes) == 1, sizes
    assert sum("pack_nodes" in ln and " ok " in ln for ln in r.stdout.splitlines()) == 3, r.stdout
    # the compensation plan: forward only; the N-1 batch plans
    assert "compensation K 50 error 1" in r.stdout, r.stdout
    if name == "n1_sample":
        # (its events lie past the driver's 400-step horizon: one topology)
        assert "compensation K 0 comp families 3 rank 0" in r.stdout, r.stdout
    if name == "n1_events":
        # a removed branch and a fault from step 100: two switched branches
        assert "compensation K 0 comp families 3 rank 2" in r.stdout, r.stdout
