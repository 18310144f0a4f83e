"""CPU checks of the C ABI: the library loads, exports every function that
include/rqrcp.h declares, and rejects invalid arguments on the host before any
device work (LAPACK-style negative argument index)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rqrcp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:rq_status|const char\*|int32_t)\s+(\w+)\s*\(", text,
                                 flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2008_04447_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librqrcp.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for must in ["rq_create", "rq_destroy", "rq_sync_status", "rqrcp_factor", "qrcp_factor",
                 "trqrcp_truncate", "tuxv_svd", "rq_sketch", "rq_sample_qrcp"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2008_04447_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in exported, name
        assert name in _lib.SIGNATURES, name


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


def test_null_handle_is_argument_one(lib):
    assert lib.rq_destroy(None) == -1
    assert lib.rqrcp_factor(None, 4, 4, 4, 2, 2, None, 4, None, 4, None, None, None, 2, None) == -1


@pytest.mark.parametrize("args,code", [
    ((-1, 4, 4, 2, 2), -2),          # m < 0
    ((4, -1, 0, 2, 2), -3),          # n < 0
    ((4, 4, 5, 2, 2), -4),           # k > min(m, n)
    ((4, 4, 4, 0, 2), -5),           # b < 1
    ((4, 4, 4, 65, 0), -5),          # b > 64
    ((8, 4, 4, 2, -1), -6),          # p < 0
    ((100, 4, 4, 64, 40), -6),       # ell > 96
    ((4, 4, 4, 2, 4), -6),           # ell > m
])
def test_rqrcp_argument_validation(lib, args, code):
    m, n, k, b, p = args
    buf = ctypes.c_void_p(0x2000)
    rc = lib.rqrcp_factor(FAKE, m, n, k, b, p, buf, max(1, m), buf, max(1, b + p), buf, buf,
                          None, 0, None)
    assert rc == code


def test_rqrcp_leading_dimension_and_pointer_checks(lib):
    buf = ctypes.c_void_p(0x2000)
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, None, 10, buf, 4, buf, buf, None, 0, None) == -7
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, buf, 9, buf, 4, buf, buf, None, 0, None) == -8
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, buf, 10, None, 4, buf, buf, None, 0, None) == -9
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, buf, 10, buf, 3, buf, buf, None, 0, None) == -10
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, buf, 10, buf, 4, None, buf, None, 0, None) == -11
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, buf, 10, buf, 4, buf, None, None, 0, None) == -12
    assert lib.rqrcp_factor(FAKE, 10, 6, 6, 2, 2, buf, 10, buf, 4, buf, buf, buf, 1, None) == -14


def test_sketch_and_sample_qrcp_validation(lib):
    buf = ctypes.c_void_p(0x2000)
    assert lib.rq_sketch(FAKE, 7, 4, 10, 5, buf, 4, buf, 10, buf, 4) == -2
    assert lib.rq_sketch(FAKE, 0, 0, 10, 5, buf, 4, buf, 10, buf, 4) == -3
    assert lib.rq_sketch(FAKE, 0, 4, 10, 5, buf, 3, buf, 10, buf, 4) == -7
    assert lib.rq_sketch(FAKE, 0, 4, 10, 5, buf, 4, buf, 9, buf, 4) == -9
    assert lib.rq_sample_qrcp(FAKE, 8, 10, 9, buf, 8, buf) == -4
    assert lib.rq_sample_qrcp(FAKE, 8, 10, 4, buf, 7, buf) == -6


def test_rsrqrcp_argument_numbering(lib):
    """ostride is argument 11, so jpvt, tau, T, ldt report 12..15."""
    buf = ctypes.c_void_p(0x2000)
    args = (FAKE, 10, 6, 6, 2, 2, buf, 10)
    assert lib.rsrqrcp_factor(None, 10, 6, 6, 2, 2, buf, 10, buf, 4, 40, buf, buf, None, 0) == -1
    assert lib.rsrqrcp_factor(*args, None, 4, 40, buf, buf, None, 0) == -9
    assert lib.rsrqrcp_factor(*args, buf, 3, 40, buf, buf, None, 0) == -10
    assert lib.rsrqrcp_factor(*args, buf, 4, 39, buf, buf, None, 0) == -11
    assert lib.rsrqrcp_factor(*args, buf, 4, 40, None, buf, None, 0) == -12
    assert lib.rsrqrcp_factor(*args, buf, 4, 40, buf, None, None, 0) == -13
    assert lib.rsrqrcp_factor(*args, buf, 4, 40, buf, buf, buf, 1) == -15


def test_tuxv_iter_jmax_is_argument_20(lib):
    buf = ctypes.c_void_p(0x2000)
    args = (0, 10, 8, 4, 2, 2, buf, 10, buf, 4, buf, 10, buf, 4, buf, 8, buf, None)
    assert lib.tuxv_svd_iter(None, *args, 1) == -1
    assert lib.tuxv_svd_iter(FAKE, *args, 0) == -20


def test_singular_values_validation(lib):
    buf = ctypes.c_void_p(0x2000)
    assert lib.rq_singular_values(None, 4, buf, 4, buf) == -1
    assert lib.rq_singular_values(FAKE, -1, buf, 4, buf) == -2
    assert lib.rq_singular_values(FAKE, 4, None, 4, buf) == -3
    assert lib.rq_singular_values(FAKE, 4, buf, 3, buf) == -4
    assert lib.rq_singular_values(FAKE, 4, buf, 4, None) == -5
    assert lib.rq_singular_values(FAKE, 1025, buf, 1025, buf) == 1003
    # sigma of more than RQ_MAX_SVD values is refused before any work
    args = (0, 3000, 2000, 1025, 64, 8, buf, 3000, buf, 72, buf, 3000, buf, 1025, buf, 2000, buf)
    assert lib.tuxv_svd(FAKE, *args, buf) == 1003


def test_noalloc_argument_validation(lib):
    buf = ctypes.c_void_p(0x2000)
    assert lib.rq_sample_qrcp_noalloc(None, 8, 100, 4, buf, 8, buf) == -1
    assert lib.rq_sample_qrcp_noalloc(FAKE, 97, 100, 4, buf, 97, buf) == -2
    assert lib.rq_sample_qrcp_noalloc(FAKE, 8, 100, 9, buf, 8, buf) == -4
    assert lib.rq_sample_qrcp_noalloc(FAKE, 8, 100, 4, buf, 7, buf) == -6
    assert lib.rq_sample_qrcp_noalloc(FAKE, 8, 100, 4, buf, 8, None) == -7
    # beyond the static scratch: refused before the handle is used
    assert lib.rq_sample_qrcp_noalloc(FAKE, 8, 16385, 4, buf, 8, buf) == 1003


def _declared_params():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:rq_status|const char\*|int32_t)\s+(\w+)\s*\((.*?)\);", text,
                         flags=re.M | re.S):
        params = [" ".join(p.split()) for p in m.group(2).split(",") if p.strip()]
        out[m.group(1)] = [p.rsplit(" ", 1)[0] for p in params]
    return out


def _kind_of_c(t):
    if "*" in t or t in ("rq_handle", "rq_server"):
        return "ptr"
    return {"int64_t": "i64", "uint64_t": "u64", "int32_t": "i32", "int": "i32", "rq_prec": "i32",
            "uint32_t": "u32", "size_t": "u64", "double": "f64"}[t]


def _kind_of_ctypes(t):
    import ctypes
    if t in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(t, "_type_") and t.__name__.startswith("LP_"):
        return "ptr"
    return {ctypes.c_int64: "i64", ctypes.c_uint64: "u64", ctypes.c_int32: "i32",
            ctypes.c_uint32: "u32", ctypes.c_double: "f64"}[t]


def test_binding_signatures_match_the_header():
    """Every ctypes signature has the header's parameter count and kinds, so a
    change on one side cannot silently shift the arguments of the other."""
    from paper_2008_04447_amd import _lib
    decl = _declared_params()
    assert set(_lib.SIGNATURES) <= set(decl)
    for name, (_, argtypes) in _lib.SIGNATURES.items():
        want = [_kind_of_c(t.replace("const ", "")) for t in decl[name]]
        got = [_kind_of_ctypes(t) for t in argtypes]
        assert got == want, name


@pytest.mark.parametrize("cmd", [["gcc", "-std=c99", "-x", "c"], ["g++", "-std=c++17", "-x", "c++"]])
def test_header_compiles_standalone(cmd):
    """include/rqrcp.h is plain C: it compiles on its own as C99 and as C++."""
    import shutil
    if shutil.which(cmd[0]) is None:
        pytest.skip(f"{cmd[0]} not installed")
    r = subprocess.run(cmd[:1] + ["-fsyntax-only", "-Wall", "-Wextra", "-Werror"] + cmd[1:] + [HEADER],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr


def test_workspace_query_validation_and_values(lib):
    """rq_workspace_query touches no device: its argument checks and the sizes it
    reports are host logic (numbering h=1 op=2 prec=3 m=4 n=5 k=6 b=7 p=8 bytes=9)."""
    from paper_2008_04447_amd import _lib
    out = ctypes.c_size_t(0)
    q = lambda op, m, n, k, b, p, prec=0, o=ctypes.byref(out): lib.rq_workspace_query(
        FAKE, op, prec, m, n, k, b, p, o)
    assert lib.rq_workspace_query(None, _lib.RQ_OP_RQRCP, 0, 10, 10, 10, 2, 2, ctypes.byref(out)) == -1
    assert q(7, 10, 10, 10, 2, 2) == -2
    assert q(_lib.RQ_OP_RQRCP, 10, 10, 10, 2, 2, prec=5) == -3
    assert q(_lib.RQ_OP_RQRCP, -1, 10, 10, 2, 2) == -4
    assert q(_lib.RQ_OP_RQRCP, 10, 65537, 10, 2, 2) == -5
    assert q(_lib.RQ_OP_RQRCP, 10, 10, 11, 2, 2) == -6
    assert q(_lib.RQ_OP_RQRCP, 10, 10, 10, 65, 2) == -7
    assert q(_lib.RQ_OP_RQRCP, 10, 10, 10, 2, 9) == -8          # ell > m
    assert q(_lib.RQ_OP_RQRCP, 10, 10, 10, 2, 2, o=None) == -9
    sizes = {}
    for op in (_lib.RQ_OP_TRQRCP, _lib.RQ_OP_TUXV, _lib.RQ_OP_RQRCP, _lib.RQ_OP_RSRQRCP,
               _lib.RQ_OP_QRCP, _lib.RQ_OP_SKETCH, _lib.RQ_OP_SAMPLE_QRCP):
        assert q(op, 2000, 1500, 32, 32, 8) == 0, op
        sizes[op] = out.value
        assert out.value > 0, op
        assert q(op, 2000, 3000, 32, 32, 8) == 0
        assert out.value > sizes[op], op                      # grows with n
    # TUXV needs the TRQRCP work plus its own; the sample QRCP needs no records for 0 steps
    assert sizes[_lib.RQ_OP_TUXV] > sizes[_lib.RQ_OP_TRQRCP]
    assert q(_lib.RQ_OP_SAMPLE_QRCP, 0, 1500, 0, 32, 8) == 0 and out.value == 0
    # the 8000 x 8000 factorization (b = 64, p = 8) fits in well under 1 GB
    assert q(_lib.RQ_OP_RQRCP, 8000, 8000, 8000, 64, 8) == 0 and 0 < out.value < 1 << 30


def test_serve_route_rule(lib):
    """The per-request precision rule of the serving loop (host logic): BF16 when
    its rounding floor 1.5 * 2^-9 * sqrt(k / min(m, n)) is at most 0.3 tol."""
    from paper_2008_04447_amd import _lib
    route = lib.rq_serve_route
    assert route(_lib.RQ_FP64, 100, 100, 10, 0.0) == _lib.RQ_FP64
    assert route(_lib.RQ_MIXED_BF16, 100, 100, 10, 0.0) == _lib.RQ_MIXED_BF16
    assert route(_lib.RQ_AUTO, 100, 100, 10, 0.0) == -1          # tol required
    assert route(_lib.RQ_AUTO, 100, 100, 10, float("nan")) == -1
    assert route(7, 100, 100, 10, 0.1) == -1
    # sigma_i = 10^(-i/50): the optimal relative error at rank k is 10^(-k/50)
    tol = lambda k: 10.0 ** (-k / 50.0)
    assert route(_lib.RQ_AUTO, 2000, 2000, 16, tol(16)) == _lib.RQ_MIXED_BF16
    assert route(_lib.RQ_AUTO, 2000, 2000, 64, tol(64)) == _lib.RQ_MIXED_BF16
    assert route(_lib.RQ_AUTO, 2000, 2000, 128, tol(128)) == _lib.RQ_MIXED_BF16
    assert route(_lib.RQ_AUTO, 1000, 3000, 128, tol(128)) == _lib.RQ_FP64     # min(m, n) small
    assert route(_lib.RQ_AUTO, 4096, 4096, 256, tol(256)) == _lib.RQ_FP64
    f = lambda k, nn: 1.5 * 2.0 ** -9 * (k / nn) ** 0.5
    for k, nn in [(16, 256), (64, 700), (128, 1614), (128, 1613), (256, 4096)]:
        want = _lib.RQ_MIXED_BF16 if f(k, nn) <= 0.3 * tol(k) else _lib.RQ_FP64
        assert route(_lib.RQ_AUTO, nn, nn + 5, k, tol(k)) == want
