"""CPU builds under sanitizers: the library's host construction and
insertion (the code rg_build_from_knn and rg_insert run, multi-threaded)
with address + undefined-behaviour checks and with the thread checker, and
the oracle with address + undefined-behaviour checks.  Each must finish
without a report and reproduce the normal builds' results bit for bit."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import datagen
import paper_2408_08933_amd as rg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2408_08933_amd", "csrc")
CXX = shutil.which("g++")
CC = shutil.which("gcc")
pytestmark = pytest.mark.skipif(not CXX or not CC, reason="needs gcc and g++")

UBSAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-fsanitize=thread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           TSAN_OPTIONS="halt_on_error=1")


def _build_host(tmp, flags, name):
    exe = os.path.join(tmp, name)
    cmd = [CXX, "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", *flags,
           os.path.join(NATIVE, "sanitize_host_build.cpp"), os.path.join(CSRC, "host_build.cpp"), "-o", exe,
           "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


@pytest.fixture(scope="module")
def case(oracle_lib):
    g = datagen.Generator(1, n=1200, n_train=1200, n_test=40)
    X, T, Q = g.base(), g.train(), g.test()
    Nq, M, L = 16, 16, 100
    knn, _ = oracle_lib.knn(X, T, Nq)
    V = np.concatenate([g.in_distribution(20), Q[:20]])
    return X, T, Q, V, knn, Nq, M, L


def _write_host_input(path, X, T, V, knn, Nq, M, L, threads):
    with open(path, "wb") as f:
        np.array([X.shape[0], T.shape[0], V.shape[0]], np.int64).tofile(f)
        np.array([X.shape[1], Nq, M, L, threads], np.int32).tofile(f)
        for a, t in ((X, np.float32), (knn, np.uint32), (T, np.float32), (V, np.float32)):
            np.ascontiguousarray(a, dtype=t).tofile(f)


def _read_graph(f, n):
    off = np.fromfile(f, np.int64, n + 1)
    idx = np.fromfile(f, np.uint32, int(off[-1]))
    return off, idx


@pytest.mark.parametrize("kind", ["address+undefined", "thread"])
def test_host_construction_under_sanitizer(case, kind):
    X, T, Q, V, knn, Nq, M, L = case
    with tempfile.TemporaryDirectory() as tmp:
        exe = _build_host(tmp, UBSAN if kind != "thread" else TSAN, "hb")
        inp, out = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
        _write_host_input(inp, X, T, V, knn, Nq, M, L, threads=4)
        r = subprocess.run([exe, inp, out], capture_output=True, text=True, env=ENV, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
        # the same build and insertion through the library itself
        ix = rg.rg_build_from_knn(X, knn, Nq, M, L_build=L, keep_stages=True, train_host=T, threads=4)
        off0, idx0, entry0 = ix.graph()
        n = X.shape[0]
        with open(out, "rb") as f:
            entry = int(np.fromfile(f, np.uint32, 1)[0])
            np.fromfile(f, np.int64, 1)
            off, idx = _read_graph(f, n)
            assert entry == entry0 and np.array_equal(off, off0) and np.array_equal(idx, idx0)
            ix.insert(V, L=L)
            off1, idx1, _ = ix.graph()
            off2, idx2 = _read_graph(f, n + V.shape[0])
            assert np.array_equal(off2, off1) and np.array_equal(idx2, idx1)


def test_oracle_under_sanitizer(oracle_lib, case):
    X, T, Q, V, knn, Nq, M, L = case
    k = 10
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle")
        cmd = [CC, "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", *UBSAN,
               os.path.join(NATIVE, "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "roar_oracle.c"), "-o", exe,
               "-lm"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        inp, out = os.path.join(tmp, "in.bin"), os.path.join(tmp, "out.bin")
        with open(inp, "wb") as f:
            np.array([X.shape[0], T.shape[0], Q.shape[0]], np.int64).tofile(f)
            np.array([X.shape[1], Nq, M, L, k], np.int32).tofile(f)
            for a in (X, T, Q):
                np.ascontiguousarray(a, dtype=np.float32).tofile(f)
        env = dict(ENV, OMP_NUM_THREADS="4")
        r = subprocess.run([exe, inp, out], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
        G = oracle_lib.Graph(X, T, Nq, M, L)
        ids0, ds0, _, _, gaps0 = oracle_lib.search(X, G.offsets, G.indices, G.entry, Q, k, L)
        n, nq = X.shape[0], Q.shape[0]
        with open(out, "rb") as f:
            assert int(np.fromfile(f, np.uint32, 1)[0]) == G.entry
            assert int(np.fromfile(f, np.int64, 1)[0]) == G.repairs
            off, idx = _read_graph(f, n)
            assert np.array_equal(off, G.offsets) and np.array_equal(idx, G.indices)
            assert np.array_equal(np.fromfile(f, np.uint32, nq * k).reshape(nq, k), ids0)
            assert np.array_equal(np.fromfile(f, np.float64, nq * k).reshape(nq, k), ds0)
            assert np.array_equal(np.fromfile(f, np.float64, nq), gaps0)
