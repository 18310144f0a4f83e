"""GPU test of the serving loop: a burst of TRQRCP / TUXV requests of uneven
sizes under an HBM budget that holds only a few of them at once.  Every result
must be bitwise identical to the same request computed alone through the
regular entry points, the arena must never exceed the budget, and requests
must actually overlap (several running at once)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _requests(n_req, seed):
    rng = synth.rng(seed)
    out = []
    for i in range(n_req):
        m = int(rng.integers(256, 700))
        n = int(rng.integers(256, 700))
        k = int(rng.choice([16, 32, 64]))
        op = int(rng.integers(0, 2))
        b = min(64, k)
        sig = synth.spectrum("pow10", min(m, n), scale=50.0)
        a = synth.low_rank(m, n, sig, seed + 10 * i, seed + 10 * i + 1).astype(np.float32)
        om = synth.omega(b + 8, m, seed + 10 * i + 2)
        out.append(dict(op=op, a=np.asfortranarray(a), om=np.asfortranarray(om), b=b, p=8, k=k))
    return out


def _alone(api, r):
    dev = torch.device("cuda", 0)
    A = api.colmajor(r["a"], dtype=torch.float32, device=dev)
    Om = api.colmajor(r["om"], device=dev)
    if r["op"] == 0:
        jp, Y, T, R = api.trqrcp_truncate(A, Om, r["b"], r["p"], r["k"])
        res = (jp, Y, T, R)
    else:
        U, X, V, jp = api.tuxv_svd(A, Om, r["b"], r["p"], r["k"])
        res = (jp, U, X, V)
    api.default_handle(0).sync()
    return [x.cpu().numpy() for x in res]


def test_serving_results_match_alone_and_respect_budget(api):
    reqs = _requests(14, 8000)
    alone = [_alone(api, r) for r in reqs]
    fp = []
    for r in reqs:
        m, n = r["a"].shape
        k = r["k"]
        fp.append(m * n * 4 + (r["b"] + 8) * m * 8 + n * 8 + (m * k + k * k + k * n) * 8)
    budget = int(2.5 * max(fp))
    srv = api.Server(budget, slots=4, max_m=700, max_n=700, max_k=64, max_ell=72)
    try:
        ids = [srv.submit(r["op"], r["a"], r["om"], r["b"], r["p"], r["k"]) for r in reqs]
        results = [srv.wait(i) for i in ids]
        st = srv.stats()
    finally:
        srv.stop()
    assert st["completed"] == len(reqs)
    assert st["peak_bytes"] <= budget
    assert st["peak_running"] >= 2, st
    for r, res, ref in zip(reqs, results, alone):
        assert res["state"] == 2 and res["status"] == 0 and res["device_error"] == 0
        jp, o0, o1, o2 = res["outputs"]
        assert np.array_equal(jp, ref[0])
        assert np.array_equal(o0, ref[1])
        assert np.array_equal(o1, ref[2])
        assert np.array_equal(o2, ref[3])
        assert res["latency_ms"] >= res["queue_ms"] >= 0.0


def test_serving_rejects_oversize(api):
    srv = api.Server(1 << 20, slots=2, max_m=700, max_n=700, max_k=64, max_ell=72)
    try:
        a = np.asfortranarray(synth.gaussian((600, 600), 1).astype(np.float32))
        om = np.asfortranarray(synth.omega(72, 600, 2))
        with pytest.raises(Exception):
            srv.submit(0, a, om, 64, 8, 64)           # needs more than 1 MiB
        big = np.asfortranarray(synth.gaussian((800, 300), 3).astype(np.float32))
        with pytest.raises(Exception):
            srv.submit(0, big, np.asfortranarray(synth.omega(72, 800, 4)), 64, 8, 32)   # m > max_m
    finally:
        srv.stop()
