"""The device EMF cosine (csrc/trig.h) checked against the C library on the
host: the same source compiled for the CPU."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def emf_cos(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("trig")
    src = d / "t.cpp"
    src.write_text('#include "trig.h"\nextern "C" void cos_many(const double* x, double* y, long n) '
                   '{ for (long i = 0; i < n; ++i) y[i] = emt::emf_cos(x[i]); }\n')
    so = d / "libt.so"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC",
                           "-I", os.path.join(ROOT, "paper_1903_01081_amd", "csrc"), str(src), "-o", str(so)],
                          stderr=subprocess.DEVNULL)
    lib = ctypes.CDLL(str(so))
    lib.cos_many.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long]

    def f(x):
        x = np.ascontiguousarray(x, np.float64)
        y = np.empty_like(x)
        lib.cos_many(x.ctypes.data, y.ctypes.data, x.size)
        return y
    return f


def test_cos_within_two_ulp(emf_cos):
    rng = np.random.default_rng(0)
    # the EMF arguments: omega t + phase for t up to seconds at 60 Hz, and beyond
    x = np.concatenate([rng.uniform(-7, 7, 200000), rng.uniform(-3e4, 3e4, 400000),
                        np.arange(0, 50001) * (2 * np.pi * 60 * 20e-6) + 0.3,
                        np.array([0.0, np.pi / 2, np.pi, 1e6, -1e6])])
    y = emf_cos(x)
    ref = np.cos(x)
    assert np.max(np.abs(y - ref)) <= 2.3e-16
    big = np.abs(ref) > 1e-3
    ulp = np.abs(y - ref)[big] / np.spacing(np.abs(ref[big]))
    assert ulp.max() <= 2.0


def test_cos_symmetry_and_period(emf_cos):
    x = np.linspace(0, 100, 10001)
    assert np.array_equal(emf_cos(x), emf_cos(-x))
    assert np.max(np.abs(emf_cos(x + 2 * np.pi) - emf_cos(x))) < 1e-14
