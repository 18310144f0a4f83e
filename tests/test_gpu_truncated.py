"""GPU parity of TRQRCP (Algorithm 5), single-sample RQRCP (Algorithm 3) and TUXV
(Algorithm 6) against the FP64 oracle.

Pivots must match the oracle exactly on the certified prefix (sample norms
recomputed exactly on both sides); Y, T and R to 1e-10 relative plus an
absolute floor of 1e-12 ||A||_F; TUXV's U, V orthonormal, U X V^T = A V V^T and
the singular values of X equal the oracle's where the pivots agree."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL, ABS = 1e-10, 1e-13


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _dev(api, x, dtype=None):
    return api.colmajor(x, dtype=dtype or torch.float64, device=torch.device("cuda", 0))


def _case(m, n, seed, scale):
    sig = synth.spectrum("pow10", min(m, n), scale=scale)
    return synth.low_rank(m, n, sig, seed, seed + 1)


@pytest.mark.parametrize("m,n,k,b,p", [
    (300, 240, 96, 32, 8),
    (257, 400, 100, 16, 8),
    (500, 300, 64, 64, 8),      # single block
    (200, 150, 20, 32, 8),      # k < b: single-sample case
    (130, 90, 90, 16, 4),       # k = min(m, n)
])
def test_trqrcp_matches_oracle(api, m, n, k, b, p):
    a = _case(m, n, 6000 + m, min(m, n) / 5.0)
    om = synth.omega(b + p, m, 6002 + n)
    jpvt, Y, T, R = api.trqrcp_truncate(_dev(api, a), _dev(api, om), b, p, k)
    api.default_handle(0).sync()
    jpvt, Y, T, R = (x.cpu().numpy() for x in (jpvt, Y, T, R))
    ref = oracle.trqrcp(a, om, b, p, k)
    pre = ref.trace.prefix(ref.sample_scale, REL, ABS)
    assert pre >= min(k, 16)
    assert sorted(jpvt) == list(range(n))
    np.testing.assert_array_equal(jpvt[:pre], ref.jpvt[:pre])
    floor = 1e-12 * np.linalg.norm(a)
    rows = min(pre, k)
    d = np.linalg.norm(R[:rows] - ref.r[:rows], axis=1)
    nrm = np.linalg.norm(ref.r[:rows], axis=1)
    assert np.all(d <= 1e-10 * nrm + floor)
    if pre >= k:
        np.testing.assert_allclose(Y, ref.y, atol=1e-9)
        np.testing.assert_allclose(T, ref.t, atol=1e-9 * max(1.0, np.abs(ref.t).max()))
    # on its own: Q = I - Y T Y^T is orthogonal and Q[:, :k] R reproduces A P's best part
    q = np.eye(m) - Y @ T @ Y.T
    assert np.linalg.norm(q.T @ q - np.eye(m), 2) <= 1e-13
    ap = a[:, jpvt]
    err_gpu = np.linalg.norm(ap - q[:, :k] @ R)
    ref_err = np.linalg.norm(a[:, ref.jpvt] - (np.eye(m) - ref.y @ ref.t @ ref.y.T)[:, :k] @ ref.r)
    assert err_gpu <= ref_err * (1 + 1e-8) + 1e-13 * np.linalg.norm(a)


@pytest.mark.parametrize("m,n,k,p", [
    (300, 240, 24, 8),
    (513, 200, 64, 16),         # b = k at the library's limit, ragged m
    (150, 400, 7, 5),           # n > m, k not a multiple of 4
])
def test_single_sample_rqrcp_matches_oracle(api, m, n, k, p):
    """Algorithm 3 (one sample of ell = k + p rows, k pivots) is TRQRCP with b = k."""
    a = _case(m, n, 6500 + m, min(m, n) / 5.0)
    om = synth.omega(k + p, m, 6502 + n)
    jpvt, Y, T, R = api.trqrcp_truncate(_dev(api, a), _dev(api, om), k, p, k)
    api.default_handle(0).sync()
    jpvt, Y, R = (x.cpu().numpy() for x in (jpvt, Y, R))
    w, tau, ref_jpvt, trace = oracle.single_sample_rqrcp(a, om, k)
    pre = trace.prefix(np.linalg.norm(om @ a, axis=0).max(), REL, ABS)
    assert pre >= min(k, 8)
    assert sorted(jpvt) == list(range(n))
    np.testing.assert_array_equal(jpvt[:pre], ref_jpvt[:pre])
    ref_r = np.triu(w[:k])
    floor = 1e-12 * np.linalg.norm(a)
    d = np.linalg.norm(R[:pre] - ref_r[:pre], axis=1)
    assert np.all(d <= 1e-10 * np.linalg.norm(ref_r[:pre], axis=1) + floor)
    if pre >= k:
        np.testing.assert_array_equal(jpvt, ref_jpvt)
        np.testing.assert_allclose(Y, np.tril(w[:, :k], -1) + np.eye(m, k), atol=1e-9)


@pytest.mark.parametrize("m,n,k,b,p", [
    (300, 240, 64, 32, 8),
    (400, 257, 100, 16, 8),
    (160, 300, 130, 64, 8),     # n > m, several 64-column QR panels
    (700, 500, 300, 64, 8),     # k > 256: Z1 = A V in two column chunks
])
def test_tuxv_matches_oracle(api, m, n, k, b, p):
    a = _case(m, n, 6100 + m, min(m, n) / 5.0)
    om = synth.omega(b + p, m, 6102 + n)
    U, X, V, jpvt = api.tuxv_svd(_dev(api, a), _dev(api, om), b, p, k)
    api.default_handle(0).sync()
    U, X, V, jpvt = (x.cpu().numpy() for x in (U, X, V, jpvt))
    ref = oracle.tuxv(a, om, b, p, k)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-13)
    assert np.allclose(X, np.triu(X))
    np.testing.assert_allclose(U @ X @ V.T, a @ V @ V.T, atol=1e-13 * np.abs(a).max())
    pre = ref.trq.trace.prefix(ref.trq.sample_scale, REL, ABS)
    sig = np.linalg.svd(X, compute_uv=False)
    e_gpu = np.linalg.norm(a - U @ X @ V.T)
    e_ref = np.linalg.norm(a - ref.u @ ref.x @ ref.v.T)
    if pre >= k:
        np.testing.assert_array_equal(jpvt[:k], ref.trq.jpvt[:k])
        np.testing.assert_allclose(sig, ref.sigma, rtol=1e-10, atol=1e-13 * sig[0])
        assert abs(e_gpu - e_ref) <= 1e-10 * e_ref + 1e-13 * np.linalg.norm(a)
    sv = np.linalg.svd(a, compute_uv=False)
    assert np.all(sig <= sv[:k] * (1 + 1e-10))
    assert e_gpu >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-10)


def test_tuxv_exact_rank_recovers_spectrum(api):
    m, n, k = 220, 180, 24
    sig = synth.spectrum("pow10", k, scale=8.0)
    a = synth.low_rank(m, n, sig, 6200, 6201)
    U, X, V, jpvt = api.tuxv_svd(_dev(api, a), _dev(api, synth.omega(24, m, 6202)), 16, 8, k)
    api.default_handle(0).sync()
    s = np.linalg.svd(X.cpu().numpy(), compute_uv=False)
    np.testing.assert_allclose(s, sig, rtol=1e-11)


@pytest.mark.parametrize("m,n,k,b,p,jmax", [
    (300, 200, 40, 16, 8, 2),     # k <= 64: U^T A in one chunk
    (300, 200, 40, 16, 8, 3),
    (400, 350, 100, 32, 8, 2),    # k > 64: U^T A in two chunks of rows
    (400, 350, 100, 32, 8, 3),
])
def test_tuxv_iterations_match_oracle(api, m, n, k, b, p, jmax):
    """Algorithm 6 with jmax alternations: closed forms, triangularity and the
    oracle's singular values and error."""
    a = _case(m, n, 6300 + m + jmax, min(m, n) / 5.0)
    om = synth.omega(b + p, m, 6302 + n)
    U, X, V, jpvt = api.tuxv_svd(_dev(api, a), _dev(api, om), b, p, k, jmax=jmax)
    api.default_handle(0).sync()
    U, X, V, jpvt = (x.cpu().numpy() for x in (U, X, V, jpvt))
    ref = oracle.tuxv(a, om, b, p, k, jmax=jmax)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-13)
    tri = np.triu(X) if jmax % 2 else np.tril(X)
    np.testing.assert_array_equal(X, tri)
    approx = U @ X @ V.T
    closed = a @ V @ V.T if jmax % 2 else U @ (U.T @ a)   # the last step's projection
    np.testing.assert_allclose(approx, closed, atol=1e-12 * np.abs(a).max())
    sig = np.linalg.svd(X, compute_uv=False)
    e_gpu = np.linalg.norm(a - approx)
    e_ref = np.linalg.norm(a - ref.u @ ref.x @ ref.v.T)
    pre = ref.trq.trace.prefix(ref.trq.sample_scale, REL, ABS)
    if pre >= k:
        np.testing.assert_allclose(sig, ref.sigma, rtol=1e-9, atol=1e-13 * sig[0])
        assert abs(e_gpu - e_ref) <= 1e-9 * e_ref + 1e-13 * np.linalg.norm(a)
    sv = np.linalg.svd(a, compute_uv=False)
    assert np.all(sig <= sv[:k] * (1 + 1e-10))
    assert e_gpu >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-10)


def test_tuxv_iterations_mixed_error_ratio(api):
    m, n, k, b, p, jmax = 1500, 600, 96, 32, 8, 2
    sig = synth.spectrum("poly", min(m, n), power=1.5)
    a64 = synth.low_rank(m, n, sig, 6400, 6401) + 1e-6 * synth.gaussian((m, n), 6402)
    a32 = a64.astype(np.float32)
    a = a32.astype(np.float64)
    om = synth.omega(b + p, m, 6403)
    A = api.colmajor(a32, dtype=torch.float32, device=torch.device("cuda", 0))
    U, X, V, _ = api.tuxv_svd(A, _dev(api, om), b, p, k, jmax=jmax)
    api.default_handle(0).sync()
    U, X, V = (x.cpu().numpy() for x in (U, X, V))
    ref = oracle.tuxv(a, om, b, p, k, jmax=jmax)
    e_mix = np.linalg.norm(a - U @ X @ V.T) / np.linalg.norm(a)
    e_ref = np.linalg.norm(a - ref.u @ ref.x @ ref.v.T) / np.linalg.norm(a)
    print(f"TUXV jmax={jmax} error mixed {e_mix:.6e} vs FP64 {e_ref:.6e}")
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    assert e_mix <= 1.05 * e_ref
