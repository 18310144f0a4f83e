"""GPU parity of RQRCP with repeated sampling (Section 3.4: the sample of block
J is a fresh sketch Omega^[J] A^[J] of the updated trailing matrix instead of
the sample update) against the FP64 oracle, to the bar of the RQRCP tests:
pivots equal on the certified prefix, R rows to 1e-10 relative there, and the
GPU factorization accurate on its own."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import q_from_inplace

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REL, ABS = 1e-10, 1e-13


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _host(t):
    return t.detach().cpu().numpy()


def _omegas(ell, m, nblk, seed):
    """Slice J is an ell x m Gaussian; block J uses its first m - J b columns."""
    full = [synth.omega(ell, m, seed + j) for j in range(nblk)]
    dev = torch.device("cuda", 0)
    om = torch.empty((nblk, m, ell), dtype=torch.float64, device=dev)
    for j, f in enumerate(full):
        om[j] = torch.from_numpy(np.ascontiguousarray(f.T)).to(dev)
    return full, om


def _run(api, a, b, p, k, seed):
    m, n = a.shape
    nblk = (k + b - 1) // b
    full, om = _omegas(b + p, m, nblk, seed)
    A = api.colmajor(a, device=torch.device("cuda", 0))
    jpvt, tau, T = api.rsrqrcp_factor(A, om, b, p, k)
    api.default_handle(0).sync()
    ref = oracle.rsrqrcp(a, lambda j, rows: full[j][:, :rows], b, p, k=k)
    return _host(A), _host(jpvt), _host(tau), _host(T), ref


@pytest.mark.parametrize("m,n,b,p,k", [
    (300, 240, 32, 8, None),     # several blocks, ragged last block
    (130, 200, 16, 8, 100),      # partial factorization, wide
    (257, 129, 8, 0, None),      # p = 0, odd sizes; late samples have fewer rows than ell
    (500, 300, 64, 8, 200),
])
def test_rsrqrcp_matches_oracle(api, m, n, b, p, k):
    k = min(m, n) if k is None else k
    sig = synth.spectrum("pow10", min(m, n), scale=min(m, n) / 6.0)
    a = synth.low_rank(m, n, sig, 4500 + m, 4501 + n)
    qr, jpvt, tau, T, ref = _run(api, a, b, p, k, 4502 + m + n)
    pre = ref.trace.prefix(ref.sample_scale, REL, ABS)
    assert pre >= min(k, 16), f"certified prefix only {pre}"
    assert sorted(jpvt) == list(range(n))
    np.testing.assert_array_equal(jpvt[:pre], ref.jpvt[:pre])
    rows = min(pre, k)
    floor = 1e-12 * np.linalg.norm(a)
    r_g, r_o = np.triu(qr[:k]), np.triu(ref.qr[:k])
    d = np.linalg.norm(r_g[:rows] - r_o[:rows], axis=1)
    nrm = np.linalg.norm(r_o[:rows], axis=1)
    assert np.all(d <= 1e-10 * nrm + floor)
    # the GPU factorization on its own
    q = q_from_inplace(qr, tau)
    r_full = np.triu(qr)
    r_full[k:, k:] = qr[k:, k:]
    assert np.linalg.norm(a[:, jpvt] - q @ r_full) / np.linalg.norm(a) <= 1e-13
    assert np.linalg.norm(q.T @ q - np.eye(m), 2) <= 1e-13
    col0 = 0
    while col0 < k:
        bj = min(b, k - col0)
        y = oracle.unit_lower(qr[col0:, col0:col0 + bj], bj)
        np.testing.assert_allclose(T[:bj, col0:col0 + bj], oracle.form_t(y, tau[col0:col0 + bj]),
                                   atol=1e-12)
        col0 += bj


def test_rsrqrcp_first_block_equals_rqrcp(api):
    """Block 0 of both variants samples Omega^[0] A: same pivots and panel."""
    m, n, b, p = 400, 300, 32, 8
    a = synth.gaussian((m, n), 4600)
    qr, jpvt, tau, T, _ = _run(api, a, b, p, 96, 4601)
    full, _ = _omegas(b + p, m, 1, 4601)
    A = api.colmajor(a, device=torch.device("cuda", 0))
    jp2, tau2, _, _ = api.rqrcp_factor(A, api.colmajor(full[0], device=torch.device("cuda", 0)), b, p, 96)
    api.default_handle(0).sync()
    np.testing.assert_array_equal(jpvt[:b], _host(jp2)[:b])
    np.testing.assert_array_equal(tau[:b], _host(tau2)[:b])


def test_rsrqrcp_zero_matrix_runs_clean(api):
    """Repeated sampling needs no R11^{-1}: the all-zero matrix whose sample
    update breaks down in RQRCP factors without a status bit, with no column
    moved and every tau zero."""
    m, n, b, p = 120, 90, 16, 8
    _, om = _omegas(b + p, m, (n + b - 1) // b, 4800)
    A = api.colmajor(np.zeros((m, n)), device=torch.device("cuda", 0))
    jpvt, tau, T = api.rsrqrcp_factor(A, om, b, p, n)
    api.default_handle(0).sync()
    np.testing.assert_array_equal(_host(jpvt), np.arange(n))
    assert np.all(_host(tau) == 0.0)
    assert np.all(_host(A) == 0.0)


def test_rsrqrcp_bad_stride_rejected(api):
    m, n, b, p = 64, 48, 16, 4
    a = synth.gaussian((m, n), 4700)
    A = api.colmajor(a, device=torch.device("cuda", 0))
    _, om = _omegas(b + p, m, 3, 4701)
    from paper_2008_04447_amd import _lib
    h = api.default_handle(0)
    jp = torch.empty(n, dtype=torch.int64, device="cuda")
    tau = torch.empty(n, dtype=torch.float64, device="cuda")
    rc = _lib.load().rsrqrcp_factor(h.ptr, m, n, n, b, p, A.data_ptr(), m, om.data_ptr(), b + p,
                                    (b + p) * m - 1, jp.data_ptr(), tau.data_ptr(), None, 0)
    assert rc == -11


def test_rsrqrcp_parity_workload_1000(api):
    """1000 x 1000, sigma_i = 10^(-i/100), b = 32, p = 8 (the parity workload)."""
    cfg = synth.workload(0)
    m, n, b, p = cfg["m"], cfg["n"], cfg["b"], cfg["p"]
    sig = synth.spectrum("pow10", n, scale=100.0)
    a = synth.low_rank(m, n, sig, synth.seed_for(0, "U"), synth.seed_for(0, "V"))
    qr, jpvt, tau, T, ref = _run(api, a, b, p, n, synth.seed_for(0, "Omega") + 100)
    pre = ref.trace.prefix(ref.sample_scale, REL, ABS)
    assert pre >= 32, f"certified prefix only {pre}"
    np.testing.assert_array_equal(jpvt[:pre], ref.jpvt[:pre])
    q = q_from_inplace(qr, tau)
    assert np.linalg.norm(a[:, jpvt] - q @ np.triu(qr)) / np.linalg.norm(a) <= 1e-13
    print(f"certified pivot prefix {pre}/{n}")
