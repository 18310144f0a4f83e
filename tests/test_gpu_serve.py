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


def _c5_request(op, m, n, k, seed):
    """A request shaped like the serving workload: FP32 A = U diag(10^(-i/50)) V^T
    (the part of the spectrum above 1e-9 drawn), b = min(64, k), p = 8."""
    r = min(m, n, 450)
    sig = 10.0 ** (-np.arange(r) / 50.0)
    a = synth.low_rank(m, n, sig, seed, seed + 1).astype(np.float32)
    b = min(64, k)
    om = synth.omega(b + 8, m, seed + 2)
    tol = float(np.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2)))   # optimal relative error
    return dict(op=op, a=np.asfortranarray(a), om=np.asfortranarray(om), b=b, p=8, k=k, tol=tol)


def _err_trqrcp(a, jpvt, Y, T, R):
    k = R.shape[0]
    qk = -(Y @ (T @ Y[:k].T))                  # first k columns of I - Y T Y^T
    qk[:k] += np.eye(k)
    return np.linalg.norm(a[:, jpvt] - qk @ R) / np.linalg.norm(a)


def test_serving_auto_precision_against_oracle(api):
    """Requests with RQ_AUTO and the accuracy they need (the optimal rank-k error
    of their spectrum): each runs in the arithmetic rq_serve_route picks, and every
    result is compared with the FP64 oracle on the same (FP32-rounded) input.
    Mixed results must be within 1.05x of the oracle's truncation error; FP64
    results must match it to parity tolerance (pivots on the certified prefix, R
    rows or sigma(X), error)."""
    import oracle
    from paper_2008_04447_amd import _lib
    shapes = [(0, 600, 500, 16), (1, 700, 400, 64), (0, 1800, 1700, 128), (1, 1700, 1650, 128),
              (1, 900, 800, 128), (0, 800, 700, 256), (1, 1000, 900, 256), (0, 300, 900, 32)]
    reqs = [_c5_request(op, m, n, k, 8100 + 10 * i) for i, (op, m, n, k) in enumerate(shapes)]
    srv = api.Server(2 << 30, slots=4, max_m=1800, max_n=1700, max_k=256, max_ell=72)
    try:
        ids = [srv.submit(r["op"], r["a"], r["om"], r["b"], r["p"], r["k"], tol=r["tol"],
                          sigma=True) for r in reqs]
        results = [srv.wait(i) for i in ids]
    finally:
        srv.stop()
    routes = set()
    for r, res in zip(reqs, results):
        assert res["state"] == 2 and res["status"] == 0 and res["device_error"] == 0
        m, n = r["a"].shape
        k = r["k"]
        want = api.serve_route(_lib.RQ_AUTO, m, n, k, r["tol"])
        assert res["prec_used"] == want
        routes.add(want)
        a = r["a"].astype(np.float64)
        jp, o0, o1, o2 = res["outputs"]
        if r["op"] == 0:
            ref = oracle.trqrcp(a, r["om"], r["b"], r["p"], k)
            e = _err_trqrcp(a, jp, o0, o1, o2)
            e_ref = _err_trqrcp(a, ref.jpvt, ref.y, ref.t, ref.r)
            trace, scale = ref.trace, ref.sample_scale
        else:
            ref = oracle.tuxv(a, r["om"], r["b"], r["p"], k)
            e = np.linalg.norm(a - o0 @ o1 @ o2.T) / np.linalg.norm(a)
            e_ref = np.linalg.norm(a - ref.u @ ref.x @ ref.v.T) / np.linalg.norm(a)
            trace, scale = ref.trq.trace, ref.trq.sample_scale
        print(f"op {r['op']} {m}x{n} k={k}: {'mixed' if want else 'fp64'} error {e:.4e} "
              f"oracle {e_ref:.4e} ratio {e / e_ref:.4f}")
        assert e <= 1.05 * e_ref
        if want == _lib.RQ_FP64:
            pre = trace.prefix(scale, 1e-10, 1e-13)
            ref_jp = ref.jpvt if r["op"] == 0 else ref.trq.jpvt
            np.testing.assert_array_equal(jp[:min(pre, k)], ref_jp[:min(pre, k)])
            if pre >= k:
                assert abs(e - e_ref) <= 1e-8 * e_ref
                if r["op"] == 1:
                    tol = 1e-10 * ref.sigma + 16 * k * np.finfo(float).eps * ref.sigma[0]
                    assert np.all(np.abs(res["sigma"] - ref.sigma) <= tol)
                else:
                    d = np.linalg.norm(o2 - ref.r, axis=1)
                    assert np.all(d <= 1e-10 * np.linalg.norm(ref.r, axis=1)
                                  + 1e-12 * np.linalg.norm(a))
    assert routes == {_lib.RQ_FP64, _lib.RQ_MIXED_BF16}
