"""Serving loop (continuous batching of whole solves): admission by HBM
budget, concurrent requests on their own streams, and results that do not
depend on the mix."""
import time

import numpy as np
import pytest

import oracle
import paper_2601_16637_amd as sbd
import workload as wl


def small_stream(nreq=10, seed=7100):
    descs = wl.serving_stream(nreq=nreq, seed=seed, norb_range=(10, 16), ndet_range=(2e3, 2e5))
    return [wl.make_request(d) for d in descs]


def submit(server, W, **opts):
    return server.submit(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, W.h, W.eri, W.e_core,
                         W.nroots, **opts)


def estimate(W, **opts):
    return sbd.serve_estimate(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, W.h, W.eri,
                              W.e_core, W.nroots, **opts)


# ------------------------------------------------------------------ host only
def test_estimate_grows_with_size_and_precision():
    reqs = small_stream(6)
    est = [estimate(W) for W in reqs]
    assert all(e % (2 << 20) == 0 and e > 0 for e in est)
    nd = [W.alpha.size * W.beta.size for W in reqs]
    order = np.argsort(nd)
    assert est[order[-1]] >= est[order[0]]
    W = reqs[0]
    assert estimate(W, sigma_prec=sbd.FP32) >= estimate(W)          # FP32 staging on top
    assert estimate(W, max_space=40) > estimate(W, max_space=10)
    # the estimate covers the Davidson vectors at least
    N = W.alpha.size * W.beta.size
    assert estimate(W, max_space=20) >= 2 * 20 * N * 8
    # device-driven iterations add spare rows of V and W (8 each) and a second collapse scratch
    assert estimate(W, device_iterations=8) >= estimate(W) + 2 * 8 * N * 8


def test_estimate_rejects_bad_requests():
    W = small_stream(1)[0]
    with pytest.raises(sbd.SBDError):
        sbd.serve_estimate(0, 1, 1, W.alpha, W.beta, np.zeros(0), np.zeros(0), 0.0, 1)
    with pytest.raises(sbd.SBDError):
        sbd.serve_estimate(W.norb, W.n_alpha, W.n_beta, W.alpha, W.beta, W.h, W.eri, W.e_core, 9)


def test_server_rejects_bad_arguments():
    with pytest.raises(sbd.SBDError):
        sbd.Server(1024, 1)            # budget below one region
    with pytest.raises(sbd.SBDError):
        sbd.Server(1 << 30, 0)         # no workers


# ------------------------------------------------------------------ GPU
@pytest.mark.gpu
def test_serve_alone_vs_mix_identical():
    """Each request's energies are bitwise the same when it runs alone (one
    worker, one request at a time) and in a mix of four concurrent workers
    with FP64 and FP32 requests interleaved."""
    reqs = small_stream(10)
    precs = [sbd.FP64 if i % 2 == 0 else sbd.FP32 for i in range(len(reqs))]
    alone = []
    s1 = sbd.Server(8 << 30, 1)
    for W, p in zip(reqs, precs):
        t = submit(s1, W, sigma_prec=p)
        alone.append(s1.wait(t))
    s1.close()
    s4 = sbd.Server(8 << 30, 4)
    tickets = [submit(s4, W, sigma_prec=p) for W, p in zip(reqs, precs)]
    mix = [s4.wait(t) for t in tickets]
    s4.close()
    for W, a, m in zip(reqs, alone, mix):
        assert a["status"] == 0 and m["status"] == 0, (a["message"], m["message"])
        k = W.nroots
        assert np.array_equal(a["energies"][:k], m["energies"][:k])
        assert a["report"]["iterations"] == m["report"]["iterations"]
        assert m["ndet"] == W.alpha.size * W.beta.size
        assert 0 < m["peak_bytes"] <= m["region_bytes"]
    # the mix really ran concurrently: some requests' [admission, completion)
    # intervals overlap, and some request was admitted while another was running
    iv = sorted((m["admit_at_ms"], m["done_at_ms"]) for m in mix)
    overlaps = sum(1 for i in range(len(iv)) for j in range(i + 1, len(iv)) if iv[j][0] < iv[i][1])
    assert overlaps >= 1, iv
    assert any(a0 < b0 < a1 for (a0, a1) in iv for (b0, _) in iv), iv
    # alone, one worker: no two requests overlap
    iv1 = sorted((a["admit_at_ms"], a["done_at_ms"]) for a in alone)
    assert all(iv1[i + 1][0] >= iv1[i][1] for i in range(len(iv1) - 1))


@pytest.mark.gpu
def test_serve_energies_match_oracle():
    reqs = small_stream(4, seed=7300)
    s = sbd.Server(8 << 30, 2)
    tickets = [submit(s, W, tol_residual=1e-8) for W in reqs]
    res = [s.wait(t) for t in tickets]
    s.close()
    for W, r in zip(reqs, res):
        assert r["status"] == 0, r["message"]
        S = oracle.OracleSystem.from_workload(W)
        ro = oracle.davidson(S.sigma, S.diag(), W.nroots, tol=1e-9, max_space=24)
        assert np.abs(r["energies"][:W.nroots] - ro.energies).max() <= 1e-8


@pytest.mark.gpu
def test_serve_admission_respects_budget():
    """With a budget that fits only a few requests at once, everything still
    completes and the regions live at any instant never exceed the budget."""
    reqs = small_stream(12, seed=7500)
    est = [estimate(W) for W in reqs]
    budget = max(est) + min(est)
    s = sbd.Server(budget, 6)
    tickets = [submit(s, W) for W in reqs]
    res = [s.wait(t) for t in tickets]
    s.close()
    for r in res:
        assert r["status"] == 0, r["message"]
        assert r["region_bytes"] <= budget
    # at every admission instant, the regions of the requests then running fit the budget
    for r in res:
        t = r["admit_at_ms"]
        live = sum(q["region_bytes"] for q in res if q["admit_at_ms"] <= t < q["done_at_ms"])
        assert live <= budget
    # and the budget did force some requests to wait for memory
    assert max(r["queue_ms"] for r in res) > 0.0


@pytest.mark.gpu
@pytest.mark.parametrize("graph", [0, 1])
def test_serve_device_driven_iterations(graph):
    """Requests with device-driven iterations (and, optionally, the iteration
    replayed from a graph) fit the regions their estimate reserves and reach
    the host-driven requests' energies, in both precisions."""
    reqs = small_stream(8, seed=7400)
    precs = [sbd.FP64 if i % 2 == 0 else sbd.FP32 for i in range(len(reqs))]
    s = sbd.Server(16 << 30, 4)
    host = [submit(s, W, sigma_prec=p, tol_residual=1e-7) for W, p in zip(reqs, precs)]
    dev = [submit(s, W, sigma_prec=p, tol_residual=1e-7, device_iterations=8, use_graph=graph)
           for W, p in zip(reqs, precs)]
    rh = [s.wait(t) for t in host]
    rd = [s.wait(t) for t in dev]
    s.close()
    for W, a, b in zip(reqs, rh, rd):
        assert a["status"] == 0 and b["status"] == 0, (a["message"], b["message"])
        assert b["report"]["device_iterations"] > 0
        assert 0 < b["peak_bytes"] <= b["region_bytes"]
        k = W.nroots
        assert np.abs(a["energies"][:k] - b["energies"][:k]).max() <= 1e-9


@pytest.mark.gpu
def test_serve_rejects_request_larger_than_budget():
    W = small_stream(1)[0]
    s = sbd.Server(2 << 20, 1)
    with pytest.raises(sbd.SBDError) as ei:
        submit(s, W)
    assert ei.value.status == -5
    s.close()


@pytest.mark.gpu
def test_serve_small_request_passes_a_head_that_does_not_fit():
    """With the slab taken by a running request, a queued request too large for
    the remaining space does not hold back a smaller one that fits."""
    reqs = small_stream(12, seed=7600)
    by = sorted(reqs, key=lambda W: W.alpha.size * W.beta.size)
    small, big = by[0], by[-1]
    e_small, e_big = estimate(small), estimate(big)
    budget = e_big + e_small  # the big one running leaves room for one small one only
    s = sbd.Server(budget, 3)
    t_run = submit(s, big)
    t_head = submit(s, big)      # cannot fit while the first one runs
    t_small = submit(s, small)   # fits beside the running one
    r_small, r_run, r_head = s.wait(t_small), s.wait(t_run), s.wait(t_head)
    s.close()
    assert r_small["status"] == r_run["status"] == r_head["status"] == 0
    assert r_small["admit_at_ms"] < r_head["admit_at_ms"]


@pytest.mark.gpu
def test_serve_destroy_fails_queued_waiters():
    """Destroying a server while a thread waits on a queued request hands that
    thread an SBD_ERR_STATE result instead of leaving it blocked."""
    import threading
    reqs = small_stream(4, seed=7700)
    big = max(reqs, key=lambda W: W.alpha.size * W.beta.size)
    s = sbd.Server(estimate(big), 1)
    tickets = [submit(s, big) for _ in range(3)]
    got = {}

    def wait_last():
        got["r"] = s.wait(tickets[-1])

    th = threading.Thread(target=wait_last)
    th.start()
    time.sleep(0.2)  # the waiter is inside sbd_serve_wait by now
    s.close()
    th.join(timeout=60)
    assert not th.is_alive()
    assert got["r"]["status"] in (0, -8)
