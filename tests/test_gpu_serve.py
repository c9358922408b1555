"""Serving form: continuous batching with mixed (k, L).  Each request's
result must be identical alone (rg_search) and in the mix, bit for bit."""
import sys
import time

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
    g = datagen.Generator(1, n=5000, n_train=5000, n_test=400)
    X, Tr, Q = g.base(), g.train(), g.test()
    say("serve: build n=5000 d=64")
    ix = rg.rg_build(torch.from_numpy(X).to(dev), torch.from_numpy(Tr).to(dev), 32, 32, L_build=200)
    return dev, X, Q, ix


def run_mix(srv, Q, ks, Ls, rate=None, timeout=120.0):
    n = len(ks)
    rng = np.random.default_rng(11)
    out = {}
    t0 = time.time()
    i = 0
    while len(out) < n:
        if i < n:
            rc = srv.submit(Q[i % len(Q)], int(ks[i]), int(Ls[i]), i)
            if rc == rg.RG_OK:
                i += 1
                if rate:
                    time.sleep(rng.exponential(1.0 / rate))
        for r in srv.poll():
            out[r["tag"]] = r
        assert time.time() - t0 < timeout, f"serving stalled: {len(out)}/{n} done"
        if i >= n:
            time.sleep(0.001)
    return out


def alone(dev, ix, q, k, L):
    ids, ds = rg.rg_search(ix, torch.from_numpy(q[None, :].copy()).to(dev), int(k), int(L))
    torch.cuda.synchronize()
    return rg.as_u32(ids)[0], ds.cpu().numpy()[0]


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp8"])
def test_alone_equals_mix(setup, storage):
    dev, X, Q, ix = setup
    if storage != "fp32":
        rg.rg_index_set_storage(ix, rg.RG_STORE_BF16 if storage == "bf16" else rg.RG_STORE_FP8E4M3)
    try:
        rng = np.random.default_rng(5)
        n = 240
        ks = rng.choice([1, 10, 100], n)
        Ls = rng.choice([32, 128, 512], n)
        srv = rg.Server(ix, max_slots=48, hops_per_step=8)
        say(f"serve {storage}: {n} mixed requests, 48 slots")
        res = run_mix(srv, Q, ks, Ls, rate=4000.0)
        st = srv.stats()
        srv.close()
        assert st["completed"] == n and st["steps"] > 1
        for i in range(n):
            r = res[i]
            assert r["status"] == 0 and r["k"] == ks[i]
            ai, ad = alone(dev, ix, Q[i % len(Q)], ks[i], Ls[i])
            assert np.array_equal(r["ids"], ai), f"request {i} ids differ alone vs mix"
            assert np.array_equal(r["dists"], ad), f"request {i} dists differ alone vs mix"
            assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        lat = np.array([res[i]["t_done"] - res[i]["t_submit"] for i in range(n)])
        say(f"  latency p50 {np.percentile(lat, 50) * 1e3:.2f} ms p99 {np.percentile(lat, 99) * 1e3:.2f} ms")
    finally:
        rg.rg_index_set_storage(ix, rg.RG_STORE_FP32)


def test_memory_bounded_admission(setup):
    dev, X, Q, ix = setup
    # with a 2^12-entry visited table one slot keeps ~29.0 KB at d=64 (query,
    # queue, table, a result record per in-flight step): a 90 KB pool admits
    # three requests at a time
    srv = rg.Server(ix, max_slots=1000, hbm_pool_bytes=90_000, hash_bits=12)
    assert srv.slots() == 3
    n = 40
    res = run_mix(srv, Q, np.full(n, 10), np.full(n, 64))
    srv.close()
    for i in range(n):
        ai, ad = alone(dev, ix, Q[i % len(Q)], 10, 64)
        assert np.array_equal(res[i]["ids"], ai)


def test_automatic_slot_count(setup):
    # max_slots = 0: twice the step workgroups the device holds at once
    dev, X, Q, ix = setup
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    srv = rg.Server(ix, max_slots=0, hops_per_step=8)
    slots = srv.slots()
    assert slots >= 2 * cus and slots % (2 * cus) == 0
    n = 30
    res = run_mix(srv, Q, np.full(n, 10), np.full(n, 64))
    srv.close()
    for i in range(n):
        ai, ad = alone(dev, ix, Q[i % len(Q)], 10, 64)
        assert np.array_equal(res[i]["ids"], ai)
    with pytest.raises(rg.RGError):
        rg.Server(ix, max_slots=-1)


def test_close_with_work_in_flight(setup):
    # closing a server while requests are queued and steps are in flight
    # finishes the admitted work, drops the queued requests and returns
    dev, X, Q, ix = setup
    srv = rg.Server(ix, max_slots=64, hops_per_step=4)
    n = 2000
    rng = np.random.default_rng(9)
    ks = rng.choice([1, 10, 100], n).astype(np.int32)
    Ls = rng.choice([32, 128, 512], n).astype(np.int32)
    qs = np.stack([Q[i % len(Q)] for i in range(n)]).astype(np.float32)
    assert srv.submit_batch(qs, ks, Ls, np.arange(n)) == n
    time.sleep(0.01)
    t = time.time()
    srv.close()
    assert time.time() - t < 30.0


def test_pool_too_small_is_rejected(setup):
    dev, X, Q, ix = setup
    with pytest.raises(rg.RGError):
        rg.Server(ix, hbm_pool_bytes=100)
    for hb in (7, 14):
        with pytest.raises(rg.RGError):
            rg.Server(ix, hash_bits=hb)
