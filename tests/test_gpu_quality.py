"""Synthetic analogue of the decomposition-quality experiment (Section 5.3,
Figure 4): truncation error against rank over several Gaussian Omega (b = 32,
p = 8) for RQRCP, TUXV, QRCP (Algorithm 2 on the GPU), presorted unpivoted QR
and the truncated SVD, on a matrix with strongly correlated neighbouring columns
(synth.smooth_columns).  Checked: the paper's qualitative claims that RQRCP's
error is consistent with QRCP's, that presorting without pivoting is much worse,
and that TUXV lies between the SVD and RQRCP in every run (a sandwich that holds
exactly: TUXV projects onto the row space RQRCP found); and for one Omega the
GPU's RQRCP and TUXV errors equal the FP64 oracle's."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _inplace_errors(qr, kmax, ranks, na):
    rf = np.triu(qr)
    rf[kmax:, kmax:] = qr[kmax:, kmax:]
    tail = np.cumsum(np.sum(rf * rf, axis=1)[::-1])[::-1]
    return np.array([np.sqrt(tail[k]) / na for k in ranks])


@pytest.mark.parametrize("kind,c", [("poly", 1.0), ("exp", 40.0)])
def test_quality_claims(api, kind, c):
    m, n, b, p, seeds = 700, 600, 32, 8, 8
    ranks = list(range(32, 161, 32))
    kmax = max(ranks)
    i = np.arange(min(m, n), dtype=np.float64)
    sig = (i + 1.0) ** -c if kind == "poly" else np.exp(-i / c)
    a = synth.smooth_columns(m, n, sig, 9100)
    na = np.linalg.norm(a)
    dev = torch.device("cuda", 0)
    A = api.colmajor(a, device=dev)
    sv = np.linalg.svd(a, compute_uv=False)
    tail = np.cumsum((sv ** 2)[::-1])[::-1]
    svd = np.array([np.sqrt(tail[k]) / na for k in ranks])
    X = api.colmajor(a, device=dev)
    api.qrcp_factor(X, kmax)
    api.default_handle(0).sync()
    qrcp = _inplace_errors(X.cpu().numpy(), kmax, ranks, na)
    order = np.argsort(-np.linalg.norm(a, axis=0))
    q, _ = np.linalg.qr(a[:, order[:kmax]])
    qr_sorted = np.array([np.linalg.norm(a - q[:, :k] @ (q[:, :k].T @ a)) / na for k in ranks])
    rq, tx = [], []
    for s in range(seeds):
        om = synth.omega(b + p, m, 9200 + s)
        Om = api.colmajor(om, device=dev)
        X.copy_(A)
        api.rqrcp_factor(X, Om, b, p, kmax)
        api.default_handle(0).sync()
        rq.append(_inplace_errors(X.cpu().numpy(), kmax, ranks, na))
        row = []
        for k in ranks:
            U, Xk, V, _ = api.tuxv_svd(A, Om, b, p, k)
            api.default_handle(0).sync()
            U, Xk, V = (t.cpu().numpy() for t in (U, Xk, V))
            row.append(np.linalg.norm(a - U @ Xk @ V.T) / na)
        tx.append(row)
        if s == 0:
            # the GPU curves for this Omega against the FP64 oracle's
            ref = oracle.rqrcp(a, om, b, p, k=kmax)
            np.testing.assert_allclose(rq[0], _inplace_errors(ref.qr, kmax, ranks, na), rtol=1e-8)
            t64 = oracle.tuxv(a, om, b, p, 64)
            e64 = np.linalg.norm(a - t64.u @ t64.x @ t64.v.T) / na
            assert abs(row[1] - e64) <= 1e-8 * e64
    rq, tx = np.array(rq), np.array(tx)
    med = np.median(rq, axis=0) / qrcp
    print(f"{kind} {c}: rqrcp/qrcp median {med.min():.3f}..{med.max():.3f}; "
          f"tuxv/svd {np.max(np.median(tx, 0) / svd):.3f}; qr presorted/qrcp "
          f"{np.min(qr_sorted / qrcp):.2f}; spread rqrcp {np.max(rq.max(0) / rq.min(0)):.4f} "
          f"tuxv {np.max(tx.max(0) / tx.min(0)):.4f}")
    assert np.all(tx <= rq * (1 + 1e-12)) and np.all(tx >= svd * (1 - 1e-12))
    assert np.all(med <= 1.15) and np.all(med >= 0.9)
    assert np.all(qr_sorted >= 1.2 * qrcp)
    assert np.all(np.median(tx, axis=0) <= 1.3 * svd)
