"""Mixed-precision path (BF16 MFMA with FP32 accumulation for the sketch and the
bulk inner products; panel, norms and sample QRCP in FP64).

Entry-wise parity with the FP64 oracle is not expected (BF16 rounding can move
near-tie pivots), so these tests are graded as the target states them: the
truncation error of the mixed factorization must be within 1.05x of the FP64
oracle's on the same input, plus rounding bounds on the BF16 sketch itself."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U8 = 2.0 ** -8     # BF16 unit roundoff (8 significand bits incl. the implicit one)


@pytest.fixture(scope="module")
def api():
    from paper_2008_04447_amd import api as _api
    return _api


def _dev(api, x, dtype):
    return api.colmajor(x, dtype=dtype, device=torch.device("cuda", 0))


def _bf16(x):
    """Round to BF16 (nearest, ties to even) through FP32, returned as float64."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("ell,m,n", [(72, 2000, 1500), (40, 777, 300), (24, 64, 5000)])
def test_bf16_sketch_within_rounding_bound(api, ell, m, n):
    a = synth.gaussian((m, n), 7000 + m).astype(np.float32)
    om = synth.omega(ell, m, 7001 + n)
    B = api.sketch(_dev(api, om, torch.float64), _dev(api, a, torch.float32))
    api.default_handle(0).sync()
    ref = om @ a.astype(np.float64)
    bound = 2.5 * U8 * (np.abs(om) @ np.abs(a.astype(np.float64))) + m * 1.2e-7 * (np.abs(om) @ np.abs(a))
    err = np.abs(B.cpu().numpy() - ref)
    assert np.all(err <= bound)
    assert np.median(err / bound) < 0.2


def _trunc_err(a, jpvt, Y, T, R):
    m = a.shape[0]
    k = R.shape[0]
    q = np.eye(m) - Y @ T @ Y.T
    return np.linalg.norm(a[:, jpvt] - q[:, :k] @ R) / np.linalg.norm(a)


@pytest.mark.parametrize("m,n,k,b,p,scale", [
    (2000, 2000, 512, 64, 8, 200.0),     # the 20000^2 exp(-i/200) case at 1/10 scale
    (1200, 900, 128, 32, 8, 60.0),
])
def test_trqrcp_mixed_error_ratio(api, m, n, k, b, p, scale):
    sig = synth.spectrum("exp", min(m, n), scale=scale)
    a64 = synth.low_rank(m, n, sig, 7100 + m, 7101 + n)
    a32 = a64.astype(np.float32)
    om = synth.omega(b + p, m, 7102)
    jpvt, Y, T, R = api.trqrcp_truncate(_dev(api, a32, torch.float32), _dev(api, om, torch.float64),
                                        b, p, k)
    api.default_handle(0).sync()
    jpvt, Y, T, R = (x.cpu().numpy() for x in (jpvt, Y, T, R))
    assert sorted(jpvt) == list(range(n))
    assert np.isfinite(Y).all() and np.isfinite(T).all() and np.isfinite(R).all()
    q = np.eye(m) - Y @ T @ Y.T
    assert np.linalg.norm(q.T @ q - np.eye(m), 2) <= 1e-12
    ref = oracle.trqrcp(a32.astype(np.float64), om, b, p, k)
    e_mix = _trunc_err(a32.astype(np.float64), jpvt, Y, T, R)
    e_ref = _trunc_err(a32.astype(np.float64), ref.jpvt, ref.y, ref.t, ref.r)
    print(f"truncation error mixed {e_mix:.6e} vs FP64 oracle {e_ref:.6e}, ratio {e_mix / e_ref:.5f}")
    assert e_mix <= 1.05 * e_ref


# The 1.05 error-ratio target needs a truncation error well above the BF16
# rounding of A seen through k directions (about 2^-9 sqrt(k / n) relative), so
# the deep k = 300 case uses a flatter spectrum.
@pytest.mark.parametrize("m,n,k,b,p,power", [
    (2500, 800, 128, 64, 8, 1.5),     # aligned rows, K tail of 32 in Z1 = A V
    (1001, 333, 72, 32, 8, 1.5),      # odd m: element loads, clamped last row tile
    (1200, 700, 300, 64, 8, 1.0),     # k > 256: two column chunks of Z1
])
def test_tuxv_mixed_error_ratio_and_spectrum(api, m, n, k, b, p, power):
    sig = synth.spectrum("poly", min(m, n), power=power)
    a64 = synth.low_rank(m, n, sig, 7200 + m, 7201 + n) + 1e-6 * synth.gaussian((m, n), 7203 + k)
    a32 = a64.astype(np.float32)
    a = a32.astype(np.float64)
    om = synth.omega(b + p, m, 7202)
    U, X, V, jpvt = api.tuxv_svd(_dev(api, a32, torch.float32), _dev(api, om, torch.float64), b, p, k)
    api.default_handle(0).sync()
    U, X, V = (x.cpu().numpy() for x in (U, X, V))
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    ref = oracle.tuxv(a, om, b, p, k)
    e_mix = np.linalg.norm(a - U @ X @ V.T) / np.linalg.norm(a)
    e_ref = np.linalg.norm(a - ref.u @ ref.x @ ref.v.T) / np.linalg.norm(a)
    s_mix = np.linalg.svd(X, compute_uv=False)
    rel = np.abs(s_mix - ref.sigma) / ref.sigma
    print(f"TUXV error mixed {e_mix:.6e} vs FP64 {e_ref:.6e}; sigma rel err median {np.median(rel):.2e} "
          f"max {rel.max():.2e}")
    # X is the upper factor of the QR of Z1 = A V formed with BF16 operands and
    # FP32 accumulation, so U X matches bf16(A) bf16(V) to FP32 summation error.
    z1_ref = _bf16(a32) @ _bf16(V)
    scale = np.abs(_bf16(a32)) @ np.abs(_bf16(V))
    err = np.abs(U @ X - z1_ref)
    assert np.all(err <= 2.0 * n * 2.0 ** -24 * scale + 1e-12 * np.abs(z1_ref).max())
    assert e_mix <= 1.05 * e_ref
    assert np.median(rel[:32]) < 1e-2
