"""Host logic of the request loop (hsym_serve_sim: the same scheduler on a
virtual clock, no device): admission order, memory budget, continuous
batching and latency accounting."""
import numpy as np

import paper_1609_01689_amd as hs


def trace(k, seed=5, rate=50.0):
    rng = np.random.default_rng(seed)
    arr = np.cumsum(rng.exponential(1.0 / rate, k))
    iters = rng.integers(5, 200, k)
    its = rng.uniform(1e-4, 2e-3, k)
    nbytes = rng.integers(1, 40, k) * (1 << 30)
    return arr, iters, its, nbytes


def test_every_request_finishes_after_it_arrives():
    arr, iters, its, nb = trace(300)
    res, rep = hs.hsym_serve_sim(arr, iters, its, nb, 0.002)
    assert all(r["status"] == hs.HSYM_OK for r in res)
    for r, a, it in zip(res, arr, iters):
        assert r["admit_s"] >= a
        assert r["finish_s"] > r["admit_s"]
        assert r["iters"] == it
    assert rep["wall_s"] == max(r["finish_s"] for r in res) - min(arr)


def test_admission_is_fifo_and_within_budget():
    arr, iters, its, nb = trace(400, seed=7, rate=500.0)
    budget = 100 << 30
    res, rep = hs.hsym_serve_sim(arr, iters, its, nb, 0.001, budget_bytes=budget, max_active=16)
    admits = np.array([r["admit_s"] for r in res])
    order = np.argsort(arr, kind="stable")
    assert np.all(np.diff(admits[order]) >= 0)          # admitted in arrival order
    assert rep["peak_reserved_bytes"] <= budget
    assert rep["max_active_seen"] <= 16
    # replay the reservations: at no admission instant do the requests in flight exceed the budget
    for i in range(len(res)):
        t = res[i]["admit_s"]
        held = sum(nb[j] for j in range(len(res)) if res[j]["admit_s"] <= t < res[j]["finish_s"])
        assert held <= budget


def test_oversized_request_is_rejected_not_blocking():
    arr = np.array([0.0, 0.0, 0.01])
    res, _ = hs.hsym_serve_sim(arr, [10, 10, 10], [0.01] * 3, [10, 1000, 10], 0.0, budget_bytes=100)
    assert [r["status"] for r in res] == [hs.HSYM_OK, hs.HSYM_E_OUT_OF_MEMORY, hs.HSYM_OK]
    assert res[2]["finish_s"] < 0.5


def test_short_request_overtakes_long_one():
    # continuous batching at iteration granularity: a short request that
    # arrives while a long one runs finishes first
    res, rep = hs.hsym_serve_sim([0.0, 0.05], [1000, 5], [0.001, 0.001], [1, 1], 0.0)
    assert res[1]["finish_s"] < res[0]["finish_s"]
    assert res[1]["latency_s"] < 0.02
    assert rep["max_active_seen"] == 2


def test_fifo_head_of_line_waits_for_memory():
    # the second request does not fit next to the first: it waits for it to
    # finish, and the third (which would fit) waits behind it
    res, _ = hs.hsym_serve_sim([0.0, 0.01, 0.02], [100, 10, 10], [0.001] * 3, [60, 60, 10], 0.0,
                               budget_bytes=100)
    assert res[1]["admit_s"] >= res[0]["finish_s"]
    assert res[2]["admit_s"] >= res[1]["admit_s"]


def test_bad_arguments_raise():
    import pytest
    with pytest.raises(hs.HsymError):
        hs.hsym_serve_sim([0.0], [0], [0.1], [1], 0.0)
