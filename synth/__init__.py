"""Seeded synthetic inputs for the RQRCP family (Duersch & Gu, arXiv:2008.04447).

This module only *draws* inputs: Gaussian compression matrices, Haar-orthogonal
factors, prescribed spectra and the graded known-pivot family.  It holds none of
the factorization arithmetic, so both the FP64 CPU oracle (under ``oracle/``) and
the HIP path may consume what it produces without sharing any method code.

The paper's own test matrices are "randomly generated" dense matrices (Section 5,
full and truncated timing experiments); its quality experiments use matrices
from a collection that is not available here, so the shapes and spectra below
stand in for them.

Conventions
-----------
* Every generator takes an explicit integer seed and uses numpy's PCG64, so the
  same seed gives the same bytes on any machine.
* Matrices are returned in Fortran (column-major) order, float64 unless stated.
* ``omega(ell, m, seed)`` is the i.i.d. N(0,1) compression matrix of the paper's
  sketch (Section 3, Gaussian projection); scale does not affect pivoting.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 200804470
_ROLES = {"U": 0, "V": 1, "Omega": 2, "noise": 3, "perm": 4, "G": 5}


def seed_for(config: int, role: str) -> int:
    """Seed of one input role ("U", "V", "Omega", "noise", ...) of workload ``config``."""
    return SEED_BASE + 1000 * int(config) + _ROLES[role]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. N(0,1) array in column-major order."""
    g = rng(seed).standard_normal(size=shape)
    return np.asfortranarray(g.astype(dtype, copy=False))


def omega(ell: int, m: int, seed: int) -> np.ndarray:
    """ell x m Gaussian compression matrix (column-major, float64)."""
    return gaussian((ell, m), seed)


def haar(n: int, r: int, seed: int) -> np.ndarray:
    """n x r matrix with Haar-distributed orthonormal columns.

    Mezzadri's recipe: QR of an n x r Gaussian, then flip each column so that the
    triangular factor has a positive diagonal (sign(0) taken as +1).  The library
    QR here only draws an input; it is not part of any method under test.
    """
    g = rng(seed).standard_normal(size=(n, r))
    q, rr = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return np.asfortranarray(q * d[None, :])


def spectrum(kind: str, r: int, **kw) -> np.ndarray:
    """Named singular-value profiles, index i = 0..r-1 (0-based, sigma_0 = 1).

    * ``"pow10"``  : 10^(-i / scale)          (scale=100 for the 1000^2 case)
    * ``"pow10x"`` : 10^(-decades * i / span)  (the 8000^2 graded case)
    * ``"exp"``    : exp(-i / scale)           (the 20000^2 truncated case)
    * ``"poly"``   : (i+1)^(-power)            (the 50000 x 8000 TUXV case)
    """
    i = np.arange(r, dtype=np.float64)
    if kind == "pow10":
        return 10.0 ** (-i / float(kw.get("scale", 100.0)))
    if kind == "pow10x":
        return 10.0 ** (-float(kw["decades"]) * i / float(kw["span"]))
    if kind == "exp":
        return np.exp(-i / float(kw.get("scale", 200.0)))
    if kind == "poly":
        return (i + 1.0) ** (-float(kw.get("power", 1.5)))
    raise ValueError(kind)


def low_rank(m: int, n: int, sigma: np.ndarray, seed_u: int, seed_v: int) -> np.ndarray:
    """A = U diag(sigma) V^T with Haar U (m x r), V (n x r), r = len(sigma)."""
    r = len(sigma)
    u = haar(m, r, seed_u)
    v = haar(n, r, seed_v)
    return np.asfortranarray((u * sigma[None, :]) @ v.T)


def graded_known_pivots(m: int, n: int, seed: int, decay: float = 4.0, eta: float = 1e-3,
                        ratio: float | None = None):
    """Well-separated family with a known QRCP pivot order.

    A = Q0 (D + eta * striu(G)) Pi^T, with Q0 Haar (m x n), D_jj = 10^(-decay*j/n)
    (or ratio^j when ``ratio`` is given), G Gaussian and Pi a seeded permutation.
    Returns (A, perm) where ``perm[j]`` is the original column placed at position j,
    i.e. A[:, perm] = Q0 (D + eta striu(G)).
    """
    q0 = haar(m, n, seed)
    j = np.arange(n, dtype=np.float64)
    d = (ratio ** j) if ratio is not None else 10.0 ** (-decay * j / n)
    g = rng(seed + 7).standard_normal(size=(n, n))
    t = np.diag(d) + eta * np.triu(g, 1) * d[None, :]
    perm = rng(seed + 11).permutation(n)
    core = q0 @ t                       # columns in pivot order
    a = np.empty((m, n))
    a[:, perm] = core
    return np.asfortranarray(a), perm


def dct_basis(n: int, r: int) -> np.ndarray:
    """n x r orthonormal DCT-II basis vectors: column i samples cos(pi i (j + 1/2) / n),
    so the first columns vary smoothly with the row index j."""
    from scipy.fft import idct
    return np.asfortranarray(idct(np.eye(n)[:, :r], axis=0, norm="ortho"))


def smooth_columns(m: int, n: int, sigma: np.ndarray, seed: int, device=None):
    """Matrix whose neighbouring columns are strongly correlated, like the images
    and discretized fields of the paper's quality experiment: A = U diag(sigma) V^T
    diag(env) with U Haar (m x r), V the first r DCT-II basis vectors of length n
    (smooth in the column index) and a seeded smooth column envelope
    env_j = 1 + 0.6 sin(6 pi j / n + phi).  Column norms then cluster, so ordering
    columns by norm alone picks near-duplicates.  With ``device`` the result is a
    column-major float64 torch tensor (U drawn with torch's seeded generator)."""
    r = len(sigma)
    v = dct_basis(n, r)
    phi = rng(seed + 3).uniform(0.0, 2.0 * np.pi)
    env = 1.0 + 0.6 * np.sin(6.0 * np.pi * np.arange(n) / n + phi)
    if device is None:
        u = haar(m, r, seed)
        return np.asfortranarray(((u * sigma[None, :]) @ v.T) * env[None, :])
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    x = torch.randn((m, r), generator=g, dtype=torch.float64, device=device)
    q, rr = torch.linalg.qr(x, mode="reduced")
    d = torch.sign(torch.diagonal(rr))
    d[d == 0] = 1.0
    u = q * d[None, :] * torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)[None, :]
    a = (u @ torch.from_numpy(np.ascontiguousarray(v.T)).to(device)) * \
        torch.from_numpy(env).to(device)[None, :]
    out = torch.empty((n, m), dtype=torch.float64, device=device).t()
    out.copy_(a)
    return out


def workload(config: int, small: bool = False):
    """Concrete input of one benchmark/parity configuration.

    config 0: 1000 x 1000, Haar U,V, sigma_i = 10^(-i/100), b=32, p=8.
    config 1: 8000 x 8000, i.i.d. N(0,1) (variant 'gauss') or Haar with
              sigma_i = 10^(-6 i/8000) (variant 'graded'), b=64, p=8.
    config 2: 20000 x 20000 FP32, Haar U,V, sigma_i = exp(-i/200), k=512, b=64, p=8.
    config 3: 50000 x 8000 FP32, sigma_i=(i+1)^-1.5 plus N(0, std 1e-6) noise, k=256.
    Returns a dict of sizes; matrices are produced by the helpers above on demand.
    """
    table = {
        0: dict(m=1000, n=1000, b=32, p=8, k=1000),
        1: dict(m=8000, n=8000, b=64, p=8, k=8000),
        2: dict(m=20000, n=20000, b=64, p=8, k=512),
        3: dict(m=50000, n=8000, b=64, p=8, k=256),
    }
    return dict(table[config])


def low_rank_device(m, n, sigma, seed, device, dtype_out=None):
    """Large low-rank inputs drawn on a GPU: A = U diag(sigma) V^T with Haar U
    (m x r) and V (n x r), r = len(sigma), built in float64 with torch's seeded
    device generator (Mezzadri's sign-corrected QR, as ``haar``).  Only the
    first r singular values are drawn, so callers pass the part of the spectrum
    that is visible at the output precision.  Returns a column-major tensor."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = len(sigma)
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)

    def haar_t(rows):
        x = torch.randn((rows, r), generator=g, dtype=torch.float64, device=device)
        q, rr = torch.linalg.qr(x, mode="reduced")
        d = torch.sign(torch.diagonal(rr))
        d[d == 0] = 1.0
        return q * d[None, :]

    u = haar_t(m)
    v = haar_t(n)
    a = (u * s[None, :]) @ v.T
    del u, v
    out = torch.empty((n, m), dtype=dtype_out or torch.float64, device=device).t()
    out.copy_(a)
    return out


def gaussian_device(m, n, seed, device, std=1.0):
    """i.i.d. N(0, std^2) m x n float64 tensor (column-major) from a seeded device generator."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return (torch.randn((n, m), generator=g, dtype=torch.float64, device=device) * std).t()
