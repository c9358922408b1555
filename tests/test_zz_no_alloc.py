"""The allocation-free search entry point (rg_search_noalloc) against
rg_search: the same kernel family on a device scratch array instead of
allocated bitmaps, so the results must be identical, call after call."""
import sys

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
rg = pytest.importorskip("paper_2408_08933_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    g = datagen.Generator(2, n=20000, n_train=1, n_test=600, d=200)
    X, Q = g.base(), g.test()
    off, idx = datagen.random_graph(X.shape[0], 24, seed=9)
    ix = rg.rg_index_from_csr(torch.from_numpy(X).to(dev), off, idx, 0)
    return dev, ix, torch.from_numpy(Q).to(dev)


def run(fn, ix, Q, k, L):
    nq = Q.shape[0]
    dev = Q.device
    ids = torch.full((nq, k), -7, dtype=torch.int32, device=dev)
    ds = torch.full((nq, k), -7.0, dtype=torch.float32, device=dev)
    hops = torch.full((nq,), -7, dtype=torch.int32, device=dev)
    ev = torch.full((nq,), -7, dtype=torch.int32, device=dev)
    fn(ix, Q, k, L, ids, ds, hops, ev)
    torch.cuda.synchronize()
    return ids, ds, hops, ev


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_noalloc_equals_search_two_calls(setup, storage):
    dev, ix, Q = setup
    st = rg.RG_STORE_FP32 if storage == "fp32" else rg.RG_STORE_BF16
    rg.rg_index_set_storage(ix, st)
    try:
        # the second call is smaller, so it runs on what the first one left
        for nq, k, L in ((600, 10, 96), (37, 25, 40)):
            say(f"noalloc vs rg_search {storage} nq={nq} k={k} L={L}")
            a = run(rg.rg_search_into, ix, Q[:nq], k, L)
            b = run(rg.rg_search_noalloc_into, ix, Q[:nq], k, L)
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
            if storage == "fp32":   # both on the exact bitmap: the same rows scored
                assert torch.equal(a[3], b[3])
            else:                   # rg_search's LDS table may score forgotten rows again
                assert (a[3] >= b[3]).all()
    finally:
        rg.rg_index_set_storage(ix, rg.RG_STORE_FP32)


def test_noalloc_rejects_bad_arguments(setup):
    dev, ix, Q = setup
    for k, L in ((0, 10), (10, 0), (1025, 10), (10, 1025)):
        ids = torch.empty((4, max(k, 1)), dtype=torch.int32, device=dev)
        ds = torch.empty((4, max(k, 1)), dtype=torch.float32, device=dev)
        with pytest.raises(rg.RGError):
            rg.rg_search_noalloc_into(ix, Q[:4], k, L, ids, ds)
    # output buffers smaller than nq x k are refused before any launch
    ids = torch.empty((4, 10), dtype=torch.int32, device=dev)
    ds = torch.empty((4, 10), dtype=torch.float32, device=dev)
    with pytest.raises(ValueError):
        rg.rg_search_noalloc_into(ix, Q[:4], 11, 10, ids, ds)
