"""Seeded synthetic matrix pairs for the GSVD tests and benchmark.

This module only draws random matrices; it contains none of the
Hari-Zimmermann arithmetic, so both the CPU oracle and the GPU library can be
fed from it without sharing any code of the method.

A pair is built with a prescribed generalized singular value decomposition
(Section 1 of the paper, the output contract F Z = U Sigma_F, G Z = V Sigma_G):

    F = U Sigma_F X,   G = V Sigma_G X,   Sigma_F^2 + Sigma_G^2 = I,

so that the generalized singular values of (F, G) are exactly
sigma_j = (Sigma_F)_jj / (Sigma_G)_jj and Z is X^{-1} up to a column scaling
and permutation.  The recipe (fixed draw order U, V, X, sigma):

* U (m_F x n), V (m_G x n): Householder QR (LAPACK geqrf/orgqr through
  numpy.linalg.qr) of a seeded N(0,1) matrix, columns signed so that
  diag(R) > 0.  Complex pairs draw (N + iN)/sqrt(2) entries.
* X (n x n): SVD of a seeded N(0,1) matrix, X0 = P S Q^*, then
  X = P diag(geomspace(1, 1/kappa, n)) Q^*, so kappa_2(X) = kappa exactly
  (up to rounding).
* sigma_j = 10^u, u ~ U(log10 lo, log10 hi); Sigma_F = sigma/sqrt(1+sigma^2),
  Sigma_G = 1/sqrt(1+sigma^2).

The paper's own datasets (Section 5.1.2) are not available; these pairs stand
in for them, with the shapes, condition numbers and value ranges of the
workloads listed in ``CONFIGS``.
"""

from __future__ import annotations

import dataclasses
import os

# numpy's QR and SVD run in OpenBLAS, which picks its kernels by CPU model;
# kernels of different families round differently, so the same seed would
# give pairs that differ in the last bits from one host to another.  One
# fixed family (AVX2 "Haswell", present on every x86-64 host used here)
# makes the pairs bitwise the same everywhere.  It takes effect only if
# numpy was not imported before this module; blas_coretype() tells.
os.environ.setdefault("OPENBLAS_CORETYPE", "Haswell")

import numpy as np  # noqa: E402

SEED_BASE = 190900101


@dataclasses.dataclass(frozen=True)
class PairSpec:
    m_f: int
    m_g: int
    n: int
    kappa: float
    sig_lo: float
    sig_hi: float
    is_complex: bool = False


# Workloads: a small unblocked case, the 4096x1024 real pair, a complex pair,
# the mixed-precision pair and the batched ensemble (drawn by make_batch).
CONFIGS = {
    1: PairSpec(64, 48, 32, 10.0, 1e-2, 1e2),
    2: PairSpec(4096, 4096, 1024, 1e2, 1e-3, 1e3),
    3: PairSpec(3072, 2048, 1024, 50.0, 1e-2, 1e2, is_complex=True),
    4: PairSpec(8192, 8192, 2048, 1e2, 1e-2, 1e2),
}
BATCH_CONFIG = dict(count=512, n_lo=16, n_hi=256, kappa_lo=1.0, kappa_hi=1e2,
                    sig_lo=1e-2, sig_hi=1e2)


def _gauss(rng: np.random.Generator, shape, is_complex: bool) -> np.ndarray:
    if is_complex:
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        return (re + 1j * im) / np.sqrt(2.0)
    return rng.standard_normal(shape)


def _orthonormal(rng, m: int, n: int, is_complex: bool) -> np.ndarray:
    a = _gauss(rng, (m, n), is_complex)
    q, r = np.linalg.qr(a)
    d = np.diag(r)
    ph = d / np.abs(d)
    return q * ph[np.newaxis, :]


def _conditioned(rng, n: int, kappa: float, is_complex: bool) -> np.ndarray:
    x0 = _gauss(rng, (n, n), is_complex)
    p, _, qh = np.linalg.svd(x0)
    s = np.geomspace(1.0, 1.0 / kappa, n) if n > 1 else np.ones(1)
    return (p * s[np.newaxis, :]) @ qh


# OpenBLAS splits a factorization's work by its thread count, which changes
# the rounding; the draws run with a fixed count (every host used has at
# least this many cores).
BLAS_THREADS = 4


def _blas_threads():
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(limits=BLAS_THREADS, user_api="blas")
    except ImportError:      # pragma: no cover - threadpoolctl is part of the image
        import contextlib
        return contextlib.nullcontext()


def make_pair(spec: PairSpec, rng: np.random.Generator):
    """Draw one pair.  Returns (F, G, sigma_desc) with F, G Fortran-ordered
    (column-major) and sigma the prescribed values sorted descending."""
    with _blas_threads():
        return _make_pair(spec, rng)


def _make_pair(spec: PairSpec, rng: np.random.Generator):
    u = _orthonormal(rng, spec.m_f, spec.n, spec.is_complex)
    v = _orthonormal(rng, spec.m_g, spec.n, spec.is_complex)
    x = _conditioned(rng, spec.n, spec.kappa, spec.is_complex)
    lo, hi = np.log10(spec.sig_lo), np.log10(spec.sig_hi)
    sigma = 10.0 ** rng.uniform(lo, hi, spec.n)
    sf = sigma / np.sqrt(1.0 + sigma * sigma)
    sg = 1.0 / np.sqrt(1.0 + sigma * sigma)
    f = np.asfortranarray((u * sf[np.newaxis, :]) @ x)
    g = np.asfortranarray((v * sg[np.newaxis, :]) @ x)
    return f, g, np.sort(sigma)[::-1].copy()


def config_pair(k: int, **override):
    """The seeded pair of workload ``k`` (1..4); fields of the PairSpec may be
    overridden to draw a smaller pair of the same kind."""
    spec = dataclasses.replace(CONFIGS[k], **override)
    return make_pair(spec, np.random.default_rng(SEED_BASE + k))


def custom_pair(m_f, m_g, n, *, kappa=10.0, sig_lo=1e-2, sig_hi=1e2,
                is_complex=False, seed=0):
    spec = PairSpec(m_f, m_g, n, kappa, sig_lo, sig_hi, is_complex)
    return make_pair(spec, np.random.default_rng(SEED_BASE + 1000 + seed))


def make_batch(count=None, seed=5, n_lo=None, n_hi=None):
    """The batched ensemble: ``count`` independent real pairs with
    n ~ U{n_lo..n_hi}, m_F, m_G ~ U{n..2n}, kappa ~ log-U[1, 1e2] and
    sigma log-uniform in [1e-2, 1e2], all from one generator."""
    c = dict(BATCH_CONFIG)
    count = c["count"] if count is None else count
    n_lo = c["n_lo"] if n_lo is None else n_lo
    n_hi = c["n_hi"] if n_hi is None else n_hi
    rng = np.random.default_rng(SEED_BASE + seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        m_f = int(rng.integers(n, 2 * n + 1))
        m_g = int(rng.integers(n, 2 * n + 1))
        kappa = 10.0 ** rng.uniform(np.log10(c["kappa_lo"]), np.log10(c["kappa_hi"]))
        spec = PairSpec(m_f, m_g, n, kappa, c["sig_lo"], c["sig_hi"])
        out.append(make_pair(spec, rng))
    return out


def blas_coretype():
    """The OpenBLAS kernel family numpy runs on in this process (None if it
    cannot be read); the seeded pairs are host-independent under
    "Haswell"."""
    try:
        import threadpoolctl
        for d in threadpoolctl.threadpool_info():
            if d.get("internal_api") == "openblas":
                return d.get("architecture")
    except Exception:
        pass
    return None
