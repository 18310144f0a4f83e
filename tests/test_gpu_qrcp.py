"""GPU parity of the plain column-pivoted QR baseline (Algorithm 2) against the
FP64 Businger-Golub oracle (Algorithm 1; both choose the same pivots in exact
arithmetic).  The GPU downdates norms, so a decision is certified when the best
and runner-up trailing norms differ by more than 1e-6 relative (the downdate's
accuracy) plus 1e-13 of the largest initial norm."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import q_from_inplace

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL, ABS = 1e-6, 1e-13


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _run(api, a, k, nb):
    A = api.colmajor(a, device=torch.device("cuda", 0))
    jpvt, tau = api.qrcp_factor(A, k=k, nb=nb)
    api.default_handle(0).sync()
    return A.cpu().numpy(), jpvt.cpu().numpy(), tau.cpu().numpy()


def _apply_q(qr, tau, x):
    """H_1 ... H_k x with H_j = I - tau_j v_j v_j^T, v_j from the in-place tails."""
    x = np.array(x, dtype=np.float64)
    for j in range(len(tau) - 1, -1, -1):
        v = qr[j:, j].copy()
        v[0] = 1.0
        x[j:] -= tau[j] * np.outer(v, v @ x[j:])
    return x


def _check(a, k, qr, jpvt, tau, min_prefix):
    m, n = a.shape
    ref = oracle.qrcp(a, k=k)
    pre = ref.trace.prefix(ref.nu0_max, REL, ABS)
    assert pre >= min_prefix, f"certified prefix only {pre}"
    assert sorted(jpvt) == list(range(n))
    np.testing.assert_array_equal(jpvt[:pre], ref.jpvt[:pre])
    floor = 1e-12 * np.linalg.norm(a)
    rows = min(pre, k)
    d = np.linalg.norm(np.triu(qr[:rows]) - np.triu(ref.qr[:rows]), axis=1)
    nrm = np.linalg.norm(np.triu(ref.qr[:rows]), axis=1)
    bad = np.flatnonzero(d > 1e-10 * nrm + floor)
    assert bad.size == 0, f"R rows {bad[:5]}"
    r_full = np.triu(qr)
    r_full[k:, k:] = qr[k:, k:]
    if m <= 2000:
        q = q_from_inplace(qr, tau)
        assert np.linalg.norm(a[:, jpvt] - q @ r_full) / np.linalg.norm(a) <= 1e-13
        assert np.linalg.norm(q.T @ q - np.eye(m), 2) <= 1e-13
    else:
        # tall: apply the reflectors implicitly (an explicit m x m Q is too big)
        qr_r = _apply_q(qr, tau, r_full)
        assert np.linalg.norm(a[:, jpvt] - qr_r) / np.linalg.norm(a) <= 1e-13
        q_thin = _apply_q(qr, tau, np.eye(m, n))
        assert np.linalg.norm(q_thin.T @ q_thin - np.eye(n), 2) <= 1e-13
    rd = np.abs(np.diag(qr)[:k])
    assert np.all(rd[1:] <= rd[:-1] * (1 + 1e-8))          # non-increasing |R_jj|
    return pre


@pytest.mark.parametrize("m,n,k,nb", [
    (300, 240, None, 32),
    (257, 129, None, 16),
    (64, 90, None, 8),
    (500, 300, 200, 64),
    (40, 40, None, 1),
    (17000, 96, None, 32),      # 67 pivot workgroups: more records than one wave's lanes
])
def test_qrcp_matches_oracle(api, m, n, k, nb):
    k = min(m, n) if k is None else k
    sig = synth.spectrum("pow10", min(m, n), scale=min(m, n) / 6.0)
    a = synth.low_rank(m, n, sig, 5000 + m, 5001 + n)
    qr, jpvt, tau = _run(api, a, k, nb)
    _check(a, k, qr, jpvt, tau, min_prefix=min(k, 16))


def test_qrcp_known_pivots_full_parity(api):
    a, perm = synth.graded_known_pivots(200, 120, 5100, decay=4.0, eta=1e-3)
    qr, jpvt, tau = _run(api, a, 120, 32)
    np.testing.assert_array_equal(jpvt, perm)
    _check(a, 120, qr, jpvt, tau, min_prefix=120)


def test_qrcp_gaussian_1000(api):
    a = synth.gaussian((1000, 1000), 5200)
    qr, jpvt, tau = _run(api, a, 1000, 64)
    pre = _check(a, 1000, qr, jpvt, tau, min_prefix=16)
    print(f"certified prefix {pre}/1000")


def test_qrcp_deterministic(api):
    a = synth.gaussian((300, 280), 5300)
    r1 = _run(api, a, 280, 32)
    r2 = _run(api, a, 280, 32)
    for x, y in zip(r1, r2):
        assert np.array_equal(x, y)
