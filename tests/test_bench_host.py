"""Host logic of bench.py (CPU): the roofline's measured traffic is used
only for the kernel sources and the operating point the counters were
taken on, recall@k is the plain set definition, and the operating point is
the smallest swept L whose recall reaches the target."""
import importlib.util
import os
import shutil

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _tree(tmp_path):
    """A copy of the four kernel sources the traffic file is keyed on."""
    src = os.path.join(ROOT, "paper_2408_08933_amd", "csrc")
    dst = tmp_path / "paper_2408_08933_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in ("beam.hip", "queue_ops.h", "wave_ops.h", "rg_internal.h"):
        shutil.copy(os.path.join(src, f), dst / f)
    (tmp_path / "profiles").mkdir()
    return dst


def test_measured_traffic_keyed_on_sources_and_operating_point(tmp_path, monkeypatch):
    b = _bench()
    dst = _tree(tmp_path)
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    sha = b.search_sources_sha()
    (tmp_path / "profiles" / "search_fp32_w.traffic.txt").write_text(
        f"L=100\nk=10\nnq=1000\nsources_sha={sha}\nfetch_bytes_per_launch=3e9\nwrite_bytes_per_launch=1e9\n")
    rate, by = b.measured_traffic("w", 100, 10, 1000, 2.0)
    assert by == 4e9 and abs(rate - 4e9 / 2e-3 / 1e9) < 1e-9  # GB/s over the 2 ms launch
    # another operating point, another workload, or changed sources: no figure
    assert b.measured_traffic("w", 101, 10, 1000, 2.0) == (None, None)
    assert b.measured_traffic("w", 100, 100, 1000, 2.0) == (None, None)
    assert b.measured_traffic("w", 100, 10, 999, 2.0) == (None, None)
    assert b.measured_traffic("other", 100, 10, 1000, 2.0) == (None, None)
    with open(dst / "beam.hip", "a") as fh:
        fh.write("\n// changed\n")
    assert b.search_sources_sha() != sha
    assert b.measured_traffic("w", 100, 10, 1000, 2.0) == (None, None)


def test_recall_definition():
    b = _bench()
    ids = np.array([[1, 2, 3], [4, 5, 6]], np.uint32)
    gt = np.array([[3, 2, 9, 1], [7, 8, 9, 4]], np.uint32)
    # row 0: {1,2,3} vs {3,2,9} -> 2 of 3; row 1: {4,5,6} vs {7,8,9} -> 0
    assert abs(b.recall_at(ids, gt, 3) - 2 / 6) < 1e-12
    assert abs(b.recall_at(ids, gt, 1) - 0.0) < 1e-12


def test_sweep_takes_the_smallest_L_that_reaches_the_target(monkeypatch):
    b = _bench()

    class FakeLib:
        @staticmethod
        def rg_search(ix, Q, k, L):
            return L, None       # the "ids" carry L to the recall stand-in below

        @staticmethod
        def as_u32(x):
            return x

    class FakeTorch:
        class cuda:
            @staticmethod
            def synchronize():
                pass

    # recall rises with L and first reaches 0.90 at L = 805, between the
    # grid's 750 and 1000
    monkeypatch.setattr(b, "recall_at", lambda L, gt, k: 0.90 if L >= 805 else 0.90 * L / 805)
    L, curve = b.sweep(FakeLib, FakeTorch, None, None, None, 10, b.L_GRID, 0.90)
    got = dict(curve)
    assert L == 805 and got[805] >= 0.90 and got[804] < 0.90
    assert b.L_GRID[-1] <= 1024      # the longest queue rg_search takes
    # never reached: no operating point
    monkeypatch.setattr(b, "recall_at", lambda L, gt, k: 0.5)
    assert b.sweep(FakeLib, FakeTorch, None, None, None, 10, b.L_GRID, 0.90)[0] is None
