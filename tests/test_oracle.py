"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests retypes the oracle's formulas: the 2x2 transformations are
checked through the congruence properties they must have (Section 2.1), whole
solves through the GSVD output contract (Section 1), the GEVD link, brute-force
generalized eigenvalues, high-precision singular values of F G^{-1}, the worked
example printed in Appendix G and the n = 1 closed form's defining properties.
"""

import json
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sl

import gsvd_inputs as gi
from contract import assert_contract
import oracle

EPS = np.finfo(np.float64).eps
GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers

def check_contract(F, G, r, tol_res=1e-13, tol_orth=1e-13):
    """Section 1: F Z = U Sigma_F, G Z = V Sigma_G, U^*U = V^*V = I,
    Sigma_F^2 + Sigma_G^2 = I, Sigma = Sigma_F / Sigma_G sorted descending,
    and the GEVD link F^*F Z = G^*G Z Sigma^2."""
    U, V, Z = r["U"], r["V"], r["Z"]
    sf, sg, s = r["sigma_f"], r["sigma_g"], r["sigma"]
    n = Z.shape[0]
    rf = np.linalg.norm(F @ Z - U * sf) / (np.linalg.norm(F) * np.linalg.norm(Z))
    rg = np.linalg.norm(G @ Z - V * sg) / (np.linalg.norm(G) * np.linalg.norm(Z))
    assert rf < tol_res and rg < tol_res, (rf, rg)
    assert np.linalg.norm(U.conj().T @ U - np.eye(n)) < tol_orth * n
    assert np.linalg.norm(V.conj().T @ V - np.eye(n)) < tol_orth * n
    assert np.max(np.abs(sf * sf + sg * sg - 1.0)) < 8 * EPS
    assert np.all(sf > 0) and np.all(sg > 0)
    np.testing.assert_allclose(s, sf / sg, rtol=8 * EPS)
    assert np.all(np.diff(s) <= 0), "sigma not sorted descending"
    A = F.conj().T @ F
    B = G.conj().T @ G
    lhs = A @ Z
    rhs = B @ Z * (s * s)
    gev = np.linalg.norm(lhs - rhs, axis=0) / (np.linalg.norm(A) * np.linalg.norm(Z, axis=0)
                                               * np.maximum(1.0, s * s))
    assert np.max(gev) < 1e-12, np.max(gev)


def rel_err(a, b):
    return np.max(np.abs(a - b) / np.abs(b))


# ------------------------------------------------------- 2x2 (Section 2.1)

def _spd(rng, cplx=False):
    a = rng.standard_normal((2, 2))
    if cplx:
        a = a + 1j * rng.standard_normal((2, 2))
    return a @ a.conj().T


def _check_2x2(A, B, Z, cplx=False):
    """Z^* B Z = I and Z^* A Z diagonal (Section 2.1), with diagonal entries
    equal to the generalized eigenvalues of the pencil (A, B)."""
    H = (lambda M: M.conj().T) if cplx else (lambda M: M.T)
    kB = np.linalg.cond(B)
    N = H(Z) @ B @ Z
    M = H(Z) @ A @ Z
    zn = np.linalg.norm(Z) ** 2
    assert np.max(np.abs(N - np.eye(2))) < 64 * EPS * kB, N
    assert abs(M[0, 1]) < 64 * EPS * np.linalg.norm(A) * zn, M
    assert abs(M[1, 0]) < 64 * EPS * np.linalg.norm(A) * zn, M
    lam = sl.eigh(A, B, eigvals_only=True)
    got = np.sort(np.real(np.diag(M)))
    assert np.allclose(got, lam, rtol=1e-10 * kB, atol=64 * EPS * np.linalg.norm(A) * zn), (got, lam)
    # 0 <= phi, psi < pi/2 means the scaled cosines on the diagonal are positive.
    assert np.real(Z[0, 0]) > 0 and np.real(Z[1, 1]) > 0
    if cplx:
        assert abs(np.imag(Z[0, 0])) == 0.0 and abs(np.imag(Z[1, 1])) == 0.0


def test_2x2_real_random():
    rng = np.random.default_rng(11)
    for _ in range(5000):
        A = _spd(rng)
        x = rng.uniform(-0.99, 0.99)
        Z, exc = oracle.real_2x2(A[0, 0], A[1, 1], A[0, 1], x)
        assert not exc
        _check_2x2(A, np.array([[1.0, x], [x, 1.0]]), Z)


@pytest.mark.parametrize("x", [0.6, -0.6, 0.0, 1e-9, -0.95])
def test_2x2_real_exception(x):
    # A' proportional to B' (Section 2.1.2, the exception), also for x < 0.
    a = 2.5
    A = a * np.array([[1.0, x], [x, 1.0]])
    Z, exc = oracle.real_2x2(A[0, 0], A[1, 1], A[0, 1], x)
    assert exc
    _check_2x2(A, np.array([[1.0, x], [x, 1.0]]), Z)


@pytest.mark.parametrize("case", ["equal_diag", "zero_b", "zero_a12", "diag_A"])
def test_2x2_real_special(case):
    x = 0.3
    if case == "equal_diag":
        A = np.array([[2.0, 0.7], [0.7, 2.0]])        # h = 0, cot(2 theta) = 0
    elif case == "zero_b":
        x = 0.0
        A = np.array([[3.0, 0.5], [0.5, 1.0]])        # an ordinary Jacobi rotation
    elif case == "zero_a12":
        A = np.array([[3.0, 0.0], [0.0, 1.0]])
    else:
        A = np.array([[1.0, 0.9 * 0.3], [0.9 * 0.3, 2.0]])
    Z, _ = oracle.real_2x2(A[0, 0], A[1, 1], A[0, 1], x)
    _check_2x2(A, np.array([[1.0, x], [x, 1.0]]), Z)


def test_2x2_real_zero_b_is_rotation():
    # With B' = I the transformation must be orthogonal (a Jacobi rotation).
    A = np.array([[3.0, 0.5], [0.5, 1.0]])
    Z, _ = oracle.real_2x2(3.0, 1.0, 0.5, 0.0)
    assert np.allclose(Z.T @ Z, np.eye(2), atol=4 * EPS)


def test_2x2_complex_random():
    rng = np.random.default_rng(12)
    for _ in range(3000):
        A = _spd(rng, True)
        b = complex(rng.uniform(-0.69, 0.69), rng.uniform(-0.69, 0.69))
        Z, exc = oracle.cplx_2x2(A[0, 0].real, A[1, 1].real, A[0, 1], b)
        assert not exc
        B = np.array([[1.0, b], [np.conj(b), 1.0]])
        _check_2x2(A, B, Z, cplx=True)


def test_2x2_complex_exception():
    # v = h = 0: arg(b) = arg(a12) and a11 = a22 (Section 2.1.1, the exception).
    b = 0.4 * np.exp(1j * 0.7)
    a12 = 1.3 * np.exp(1j * 0.7)
    A = np.array([[2.0, a12], [np.conj(a12), 2.0]])
    Z, exc = oracle.cplx_2x2(2.0, 2.0, a12, b)
    assert exc
    _check_2x2(A, np.array([[1.0, b], [np.conj(b), 1.0]]), Z, cplx=True)


@pytest.mark.parametrize("sgn", [1.0, -1.0])
def test_2x2_complex_h_zero(sgn):
    # h = 0 with v != 0 of either sign: tan(gamma) is infinite.
    b = 0.3 + 0.0j
    a12 = 0.8 + sgn * 0.5j
    A = np.array([[1.5, a12], [np.conj(a12), 1.5]])
    Z, exc = oracle.cplx_2x2(1.5, 1.5, a12, b)
    assert not exc
    _check_2x2(A, np.array([[1.0, b], [np.conj(b), 1.0]]), Z, cplx=True)


def test_2x2_complex_reduces_to_real():
    # Real data through the complex formulas diagonalizes the same pencil.
    rng = np.random.default_rng(13)
    for _ in range(500):
        A = _spd(rng)
        x = rng.uniform(-0.9, 0.9)
        Zc, _ = oracle.cplx_2x2(A[0, 0], A[1, 1], A[0, 1], x)
        _check_2x2(A.astype(complex), np.array([[1.0, x], [x, 1.0]], dtype=complex), Zc, cplx=True)


# -------------------------------------------------- orderings (Section 2.2)

@pytest.mark.parametrize("n", [2, 4, 6, 8, 32, 64])
def test_mm_ordering(n):
    t = oracle.ordering(oracle.ORD_MM, n)
    assert t.shape == (n, n // 2, 2)
    seen = {}
    for k, step in enumerate(t):
        idx = step.reshape(-1)
        assert sorted(idx.tolist()) == list(range(n)), "step is not a perfect matching"
        for p, q in step:
            assert p < q
            seen[(p, q)] = seen.get((p, q), 0) + 1
    assert len(seen) == n * (n - 1) // 2, "a pair is missing from the sweep"
    rep = sorted(pq for pq, c in seen.items() if c > 1)
    assert rep == [(p, p + n // 2) for p in range(n // 2)] or n == 2
    assert sum(seen.values()) == n * n // 2      # quasi-cyclic, s = n


@pytest.mark.parametrize("n", [2, 4, 6, 8, 32, 64])
def test_rr_ordering(n):
    t = oracle.ordering(oracle.ORD_RR, n)
    assert t.shape == (n - 1, n // 2, 2)
    pairs = set()
    for step in t:
        assert sorted(step.reshape(-1).tolist()) == list(range(n))
        for p, q in step:
            assert p < q
            pairs.add((p, q))
    assert len(pairs) == n * (n - 1) // 2           # cyclic, s = n - 1


def test_rowcyclic_ordering():
    t = oracle.ordering(oracle.ORD_ROWCYCLIC, 5)
    got = [tuple(p) for p in t[:, 0, :].tolist()]
    assert got == [(i, j) for i in range(5) for j in range(i + 1, 5)]


# ------------------------------------------------------- whole solves

def test_constructed_pair_config1():
    F, G, s = gi.config_pair(1)
    r = oracle.gsvd(F, G, tol=32 * EPS)
    assert r["converged"]
    assert rel_err(r["sigma"], s) < 1e-12
    check_contract(F, G, r)


@pytest.mark.parametrize("kind", [oracle.ORD_ROWCYCLIC, oracle.ORD_MM, oracle.ORD_RR])
@pytest.mark.parametrize("cplx", [False, True])
def test_constructed_pairs(kind, cplx):
    F, G, s = gi.custom_pair(60, 45, 28, kappa=30.0, is_complex=cplx, seed=7)
    r = oracle.gsvd(F, G, ordering=kind, threads=2)
    assert r["converged"] and r["status"] == 0
    assert rel_err(r["sigma"], s) < 1e-12
    check_contract(F, G, r)


@pytest.mark.parametrize("n", [3, 5, 17])
def test_odd_n(n):
    F, G, s = gi.custom_pair(n + 4, n + 1, n, seed=n)
    for kind in (oracle.ORD_ROWCYCLIC, oracle.ORD_MM, oracle.ORD_RR):
        r = oracle.gsvd(F, G, ordering=kind)
        assert rel_err(r["sigma"], s) < 1e-12
        check_contract(F, G, r)


def test_threads_do_not_change_result():
    F, G, _ = gi.custom_pair(70, 60, 32, seed=9)
    r1 = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=1)
    r4 = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=4)
    for k in ("U", "V", "Z", "sigma"):
        assert np.array_equal(r1[k], r4[k])


@pytest.mark.parametrize("cplx", [False, True])
def test_n1_closed_form(cplx):
    rng = np.random.default_rng(5)
    F = rng.standard_normal((7, 1)) + (1j * rng.standard_normal((7, 1)) if cplx else 0)
    G = rng.standard_normal((4, 1)) + (1j * rng.standard_normal((4, 1)) if cplx else 0)
    r = oracle.gsvd(F, G)
    check_contract(F, G, r)
    # The single generalized eigenvalue of (F^*F, G^*G) is sigma^2.
    lam = (np.vdot(F, F) / np.vdot(G, G)).real
    assert abs(r["sigma"][0] ** 2 - lam) < 4 * EPS * lam


@pytest.mark.parametrize("seed", range(6))
def test_bruteforce_tiny(seed):
    # sigma^2 are the generalized eigenvalues of (F^*F, G^*G) (Section 1);
    # safe to compute this way because B is well conditioned here.
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 9))
    cplx = bool(seed % 2)
    F = rng.standard_normal((n + 3, n))
    G = rng.standard_normal((n + 2, n)) + 2 * np.eye(n + 2, n)
    if cplx:
        F = F + 1j * rng.standard_normal(F.shape)
        G = G + 1j * rng.standard_normal(G.shape)
    A, B = F.conj().T @ F, G.conj().T @ G
    assert np.linalg.cond(B) < 1e3
    lam = sl.eigh(A, B, eigvals_only=True)[::-1]
    r = oracle.gsvd(F, G)
    assert rel_err(r["sigma"] ** 2, lam) < 1e-12
    check_contract(F, G, r)


def _mp_gsv(F, G, dps=40):
    mp.mp.dps = dps
    Fm = mp.matrix(F.tolist())
    Gm = mp.matrix(G.tolist())
    s = mp.svd_r(Fm * mp.inverse(Gm), compute_uv=False)
    return np.array(sorted((float(v) for v in s), reverse=True))


@pytest.mark.parametrize("kappa_g", [1e1, 1e4, 1e8, 1e12])
def test_square_graded_high_precision(kappa_g):
    # For square nonsingular G the generalized singular values are the
    # singular values of F G^{-1} (Appendix G, the 32-digit comparison),
    # and the GSVD keeps them relatively accurate as kappa(G) grows.
    rng = np.random.default_rng(int(np.log10(kappa_g)))
    n = 10
    F = rng.standard_normal((n, n))
    G = rng.standard_normal((n, n)) @ np.diag(np.geomspace(1.0, 1.0 / kappa_g, n))
    ref = _mp_gsv(F, G)
    r = oracle.gsvd(F, G)
    assert r["converged"]
    assert rel_err(r["sigma"], ref) < 1e-12, (r["sigma"], ref)


def test_appendix_g_example():
    with open(os.path.join(GOLD, "appendix_g.json")) as fh:
        gold = json.load(fh)
    F = np.array(gold["F"], dtype=float)
    G = np.array(gold["G_without_g11"], dtype=float)
    G[0, 0] = gold["g11"]
    r = oracle.gsvd(F, G)
    printed = np.array(gold["sigma_printed_desc"])
    # The printed values carry 16 significant digits.
    assert rel_err(r["sigma"], printed) < 2e-15
    lam = np.array(gold["lambda_exact_desc"])
    assert rel_err(r["sigma"] ** 2, lam) < 4e-15
    ref = _mp_gsv(F, G, dps=50)
    assert rel_err(r["sigma"], ref) < 4 * EPS


def test_no_sort_still_valid():
    F, G, s = gi.custom_pair(40, 40, 16, seed=21)
    r = oracle.gsvd(F, G, sort=False)
    assert rel_err(r["sigma"], s) < 1e-12
    check_contract(F, G, r)


def test_sweep_cap_reports_not_converged():
    F, G, _ = gi.custom_pair(40, 40, 16, seed=22)
    r = oracle.gsvd(F, G, max_sweeps=1)
    assert r["status"] == 1 and not r["converged"] and r["sweeps"] == 1


def test_bad_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.gsvd(np.ones((3, 4)), np.ones((5, 4)))      # m_F < n


# ---------------------------------------------------------------- variant 4
# Section 2.5: criterion C2 calls a transformation small when the unscaled
# cosines cos(phi) and cos(psi) are 1; C1 when the scaled ones (the diagonal
# of Zhat' = (1/t)[[cos phi, sin phi], [-sin psi, cos psi]]) are 1.

def test_2x2_cosines_are_those_of_the_printed_form():
    """The cosines the oracle reports are t times the diagonal of Zhat', and
    with t times the off-diagonal entries they form unit vectors (cos, sin):
    the relations of the printed form of Zhat' (real Section 2.1.2, complex
    Section 2.1.1)."""
    rng = np.random.default_rng(77)
    for _ in range(300):
        a = rng.standard_normal((2, 2))
        A = a @ a.T
        x = rng.uniform(-0.95, 0.95)
        Z, exc, cc = oracle.real_2x2(A[0, 0], A[1, 1], A[0, 1], x, cosines=True)
        assert not exc
        t = np.sqrt(1.0 - x * x)
        assert np.allclose(cc, t * np.diag(Z), rtol=1e-14, atol=0)
        assert abs(cc[0] ** 2 + (t * Z[0, 1]) ** 2 - 1.0) < 1e-14
        assert abs(cc[1] ** 2 + (t * Z[1, 0]) ** 2 - 1.0) < 1e-14
        b = complex(rng.uniform(-0.6, 0.6), rng.uniform(-0.6, 0.6))
        ac = complex(rng.standard_normal(), rng.standard_normal())
        aii, ajj = abs(ac) + rng.uniform(0.5, 2), abs(ac) + rng.uniform(0.5, 2)
        Zc, exc, ccc = oracle.cplx_2x2(aii, ajj, ac, b, cosines=True)
        tc = np.sqrt(1.0 - abs(b) ** 2)
        assert not exc
        assert np.allclose(ccc, tc * np.real(np.diag(Zc)), rtol=1e-14, atol=0)
        assert abs(ccc[0] ** 2 + abs(tc * Zc[0, 1]) ** 2 - 1.0) < 1e-13
        assert abs(ccc[1] ** 2 + abs(tc * Zc[1, 0]) ** 2 - 1.0) < 1e-13


def test_c1_and_c2_differ_when_t_is_below_one():
    """x = 2e-8 and a_ij = (a_ii + a_jj) x / 2 make D = 0 exactly, so tan(theta)
    = 0 and cos(phi) = cos(psi) = 1 - xi*eta rounds to 1 (C2: small), while t =
    sqrt(1 - x^2) rounds below 1, so the scaled cosines exceed 1 (C1: big)."""
    x = 2e-8
    aii, ajj = 2.0, 1.0
    aij = (aii + ajj) * x / 2.0
    Z, exc, cc = oracle.real_2x2(aii, ajj, aij, x, cosines=True)
    assert not exc
    assert cc[0] == 1.0 and cc[1] == 1.0
    assert Z[0, 0] != 1.0 and Z[1, 1] != 1.0


@pytest.mark.parametrize("cplx", [False, True])
def test_variant4_constructed_pairs(cplx):
    """Variant 4 (criterion C2) reaches the prescribed generalized singular
    values and the output contract, like variant 0."""
    F, G, s_true = gi.custom_pair(90, 70, 40, kappa=1e2, is_complex=cplx, seed=404)
    r4 = oracle.gsvd(F, G, variant=4)
    r0 = oracle.gsvd(F, G, variant=0)
    assert r4["converged"] and r4["status"] == 0
    assert rel_err(r4["sigma"], s_true) < 1e-12
    assert rel_err(r4["sigma"], r0["sigma"]) < 1e-13
    check_contract(F, G, r4)


def test_variant4_equals_variant0_for_orthonormal_g():
    """With G^T G = I every pivot B' is the identity up to rounding, t = 1
    exactly, the scaled and unscaled cosines coincide and both criteria give
    the same run, bit for bit."""
    rng = np.random.default_rng(405)
    F = rng.standard_normal((60, 24))
    G, _ = np.linalg.qr(rng.standard_normal((50, 24)))
    r0 = oracle.gsvd(F, G, variant=0)
    r4 = oracle.gsvd(F, G, variant=4)
    assert r0["sweeps"] == r4["sweeps"] and r0["rot_big"] == r4["rot_big"]
    for k in ("sigma", "U", "V", "Z"):
        assert np.array_equal(r0[k], r4[k])


def test_variant4_changes_the_classification():
    """On this seeded pair the two criteria classify some transformations
    differently (the counts of big transformations differ), so the variant
    argument reaches the classification."""
    F, G, _ = gi.custom_pair(120, 100, 48, kappa=1e2, seed=406)
    r0 = oracle.gsvd(F, G, variant=0, ordering=oracle.ORD_MM, threads=2)
    r4 = oracle.gsvd(F, G, variant=4, ordering=oracle.ORD_MM, threads=2)
    assert (r0["rot_big"], r0["sweeps"]) != (r4["rot_big"], r4["sweeps"])


def test_bad_variant_rejected():
    F, G, _ = gi.custom_pair(10, 10, 4, seed=407)
    with pytest.raises(ValueError):
        oracle.gsvd(F, G, variant=2)


# ---------------------------------------------------------------- QR shortening
# The shortened pair (R_F P2, R_G) has the Grams P^T F^T F P and P^T G^T G P
# (P = P1 P2), so its GSVD has the same sigma and, mapped back, the same
# normalised Z (unique up to column signs, or unit phases in the complex
# case, for distinct sigma); U = Q_F U''
# and V = Q_G V'' must satisfy the output contract on the original pair.

def _align_signs(Z, Zref):
    """Z with each column multiplied by the sign (real) or unit phase
    (complex) that brings it closest to the same column of Zref."""
    c = np.sum(Z.conj() * Zref, axis=0)
    return Z * (c / np.abs(c))


@pytest.mark.parametrize("shape", [(300, 200, 60), (64, 48, 32), (40, 40, 40), (90, 150, 17)])
@pytest.mark.parametrize("cplx", [False, True])
def test_qr_shortening_same_gsvd(shape, cplx):
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=50.0, is_complex=cplx, seed=600 + n)
    a = oracle.gsvd_qr(F, G, ordering=oracle.ORD_MM)
    b = oracle.gsvd(F, G, ordering=oracle.ORD_MM)
    assert a["status"] == 0 and a["converged"]
    assert np.max(np.abs(a["sigma"] - s_true) / s_true) < 1e-12
    assert np.max(np.abs(a["sigma"] - b["sigma"]) / b["sigma"]) < 1e-12
    assert_contract(F, G, a["U"], a["V"], a["Z"], a["sigma_f"], a["sigma_g"], a["sigma"])
    Zb = b["Z"]
    err = np.max(np.abs(_align_signs(a["Z"], Zb) - Zb)) / np.max(np.abs(Zb))
    assert err < 1e-10


def test_qr_shortening_pivot_order():
    """Column pivoting takes the column of largest norm first (for F, and for
    G P1, whose column norms are those of G); with columns of F scaled by
    distinct powers of 4 the whole first permutation is the norm order."""
    rng = np.random.default_rng(611)
    n = 8
    F = rng.standard_normal((30, n)) * 1e-6 + np.eye(30, n)
    F = F * (4.0 ** rng.permutation(n))
    G = rng.standard_normal((20, n)) * np.array([1, 9, 2, 3, 4, 5, 6, 7.0])
    r = oracle.gsvd_qr(F, G)
    assert list(r["p1"]) == list(np.argsort(-np.linalg.norm(F, axis=0)))
    assert r["q"][0] == np.argmax(np.linalg.norm(G, axis=0))
    assert sorted(r["q"]) == list(range(n))
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"])


# ------------------------------------------------ enhanced dot products (App. A)

def _rd_pairs():
    rng = np.random.default_rng(812)
    a = rng.standard_normal(3000) * 2.0 ** rng.integers(-40, 40, 3000)
    b = rng.standard_normal(3000) * 2.0 ** rng.integers(-40, 40, 3000)
    # products whose round-to-nearest value lies above the exact one
    extra_a = [1.0 + 2.0 ** -30, 3.0, -(1.0 + 2.0 ** -29), 0.1, 1e300]
    extra_b = [1.0 + 2.0 ** -30 - 2.0 ** -52, 0.1, 1.0 + 2.0 ** -31, -0.7, 1e-300]
    return list(zip(np.r_[a, extra_a], np.r_[b, extra_b]))


def test_mul_rd_is_the_rounded_down_product():
    """c is the largest double not above a*b and c + d == a*b exactly, so
    d >= 0 (exact rational arithmetic; round toward -infinity by definition)."""
    from fractions import Fraction
    for a, b in _rd_pairs():
        c, d = oracle.mul_rd(a, b)
        exact = Fraction(float(a)) * Fraction(float(b))
        assert Fraction(c) <= exact < Fraction(np.nextafter(c, np.inf))
        assert Fraction(c) + Fraction(d) == exact
        assert d >= 0.0


def test_edot_recovers_what_the_products_lose():
    """x = (1 + 2^-30, 1), y = (1 + 2^-30, -(1 + 2^-29)): x.y = 2^-60 exactly;
    every rounded product loses it and the ordinary dot product gives 0,
    the enhanced one adds the (non-negative) errors back and gets it."""
    x = np.array([1.0 + 2.0 ** -30, 1.0])
    y = np.array([1.0 + 2.0 ** -30, -(1.0 + 2.0 ** -29)])
    assert x[0] * y[0] + x[1] * y[1] == 0.0
    assert oracle.edot(x, y) == 2.0 ** -60


def test_edot_exact_on_integers_and_close_to_exact():
    from fractions import Fraction
    rng = np.random.default_rng(813)
    xi = rng.integers(-1000, 1000, 500).astype(float)
    yi = rng.integers(-1000, 1000, 500).astype(float)
    assert oracle.edot(xi, yi) == float(np.dot(xi.astype(np.int64), yi.astype(np.int64)))
    x = rng.standard_normal(400)
    y = rng.standard_normal(400)
    exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y))
    bound = 400 * np.finfo(float).eps * float(np.sum(np.abs(x * y)))
    assert abs(Fraction(oracle.edot(x, y)) - exact) <= Fraction(bound)


@pytest.mark.parametrize("v_enh,v_plain", [(1, 0), (5, 4)])
def test_enhanced_variants_same_gsvd(v_enh, v_plain):
    """Variants 1 and 5 differ from 0 and 4 only in how the pivot entries are
    summed: the same GSVD to rounding, the contract, but not the same bits."""
    F, G, s_true = gi.custom_pair(150, 120, 40, kappa=1e2, seed=814)
    e = oracle.gsvd(F, G, variant=v_enh, ordering=oracle.ORD_MM, threads=2)
    p = oracle.gsvd(F, G, variant=v_plain, ordering=oracle.ORD_MM, threads=2)
    assert e["status"] == 0 and e["converged"]
    assert np.max(np.abs(e["sigma"] - p["sigma"]) / p["sigma"]) < 1e-12
    assert np.max(np.abs(e["sigma"] - s_true) / s_true) < 1e-12
    assert_contract(F, G, e["U"], e["V"], e["Z"], e["sigma_f"], e["sigma_g"], e["sigma"])
    assert not np.array_equal(e["Z"], p["Z"])


def test_enh_abs2_complex_norm_procedure():
    """The simpler complex procedure of Appendix A: exact where the squares
    are, and within 1 ulp of the exact |z|^2 on random and crafted entries
    (dropping the error terms of the rounded-down squares costs up to 2
    ulp on the crafted ones)."""
    from fractions import Fraction
    assert oracle.enh_abs2(3 + 4j) == 25.0 and oracle.enh_abs2(-12 + 5j) == 169.0
    rng = np.random.default_rng(816)
    n = 4000
    zs = list(rng.standard_normal(n) * 2.0 ** rng.integers(-30, 30, n)
              + 1j * rng.standard_normal(n) * 2.0 ** rng.integers(-30, 30, n))
    zs += [complex(1.0 + k * 2.0 ** -40, 0.0) for k in range(1, 500)]
    zs += [complex(1.0 + k * 2.0 ** -40, 0.75 + k * 2.0 ** -41) for k in range(1, 500)]
    for z in zs:
        exact = Fraction(z.real) ** 2 + Fraction(z.imag) ** 2
        err = abs(Fraction(oracle.enh_abs2(z)) - exact)
        assert err <= Fraction(float(np.spacing(float(exact))))


@pytest.mark.parametrize("v_enh,v_plain", [(1, 0), (5, 4)])
def test_enhanced_variants_complex_same_gsvd(v_enh, v_plain):
    F, G, s_true = gi.custom_pair(120, 90, 32, kappa=1e2, is_complex=True, seed=817)
    e = oracle.gsvd(F, G, variant=v_enh, ordering=oracle.ORD_MM, threads=2)
    p = oracle.gsvd(F, G, variant=v_plain, ordering=oracle.ORD_MM, threads=2)
    assert e["status"] == 0 and e["converged"]
    assert np.max(np.abs(e["sigma"] - p["sigma"]) / p["sigma"]) < 1e-12
    assert np.max(np.abs(e["sigma"] - s_true) / s_true) < 1e-12
    assert_contract(F, G, e["U"], e["V"], e["Z"], e["sigma_f"], e["sigma_g"], e["sigma"])
    assert not np.array_equal(e["Z"], p["Z"])


# ------------------------------------------- per-step sorting (Section 3.5.3)

def test_real_sort_keys_are_the_transformed_diagonal():
    """The real sort keys a''_11, a''_22 must be the diagonal of Z'^T A' Z'
    (the squared norms the two columns of F get from the transformation),
    for random pencils, both signs of x, and the exception's matrix."""
    rng = np.random.default_rng(31)
    cases = []
    for _ in range(3000):
        A = _spd(rng)
        cases.append((A, rng.uniform(-0.99, 0.99)))
    for x in (0.6, -0.6, 0.0, -0.95):
        cases.append((2.5 * np.array([[1.0, x], [x, 1.0]]), x))   # the exception
    for A, x in cases:
        Z, _ = oracle.real_2x2(A[0, 0], A[1, 1], A[0, 1], x)
        k11, k22 = oracle.real_sort_keys(A[0, 0], A[1, 1], A[0, 1], Z)
        D = Z.T @ A @ Z
        scale = np.linalg.norm(A) * np.linalg.norm(Z) ** 2
        assert abs(k11 - D[0, 0]) < 16 * EPS * scale, (k11, D[0, 0])
        assert abs(k22 - D[1, 1]) < 16 * EPS * scale, (k22, D[1, 1])


def _random_step_pair(rng, m, n, cplx):
    F = rng.standard_normal((m, n))
    G = rng.standard_normal((m, n))
    if cplx:
        F = F + 1j * rng.standard_normal((m, n))
        G = G + 1j * rng.standard_normal((m, n))
    # prescaled as the sweeps see it: unit columns of G (Section 2)
    d = 1.0 / np.linalg.norm(G, axis=0)
    F, G = F * d, G * d
    # spread the column norms of F so the sort decision is clear-cut
    F = F * np.geomspace(1.0, 50.0, n)[rng.permutation(n)]
    Z = np.diag(d).astype(F.dtype)
    return F, G, Z


@pytest.mark.parametrize("cplx", [False, True])
def test_sorted_step_puts_the_larger_norm_first(cplx):
    """After a step with sorting, column i of F has the larger norm (Section
    3.5.3), and the step is the congruence [f_i f_j] Z' (up to the swap) of
    the columns it was given: checked against the transformed pair's own
    norms, in many random pairs where the transformation alone would leave
    the larger norm second about half of the time."""
    rng = np.random.default_rng(32 if cplx else 33)
    swapped = kept = 0
    for _ in range(400):
        F, G, Z = _random_step_pair(rng, 9, 4, cplx)
        i, j = sorted(rng.choice(4, 2, replace=False))
        F1, G1, Z1, nall, _ = oracle.step(F, G, Z, i, j, sort=True)
        assert nall == 1
        ni, nj = np.linalg.norm(F1[:, i]), np.linalg.norm(F1[:, j])
        assert ni >= nj * (1 - 1e-13), (ni, nj)
        # unsorted step: the same transformation without the swap
        F0, G0, Z0, _, _ = oracle.step(F, G, Z, i, j, sort=False)
        same = np.allclose(F1[:, [i, j]], F0[:, [i, j]], rtol=0, atol=0)
        flip = np.array_equal(F1[:, [i, j]], F0[:, [j, i]])
        assert same or flip
        swapped += flip and not same
        kept += same
        # untouched columns stay put; G and Z follow F's swap
        others = [c for c in range(4) if c not in (i, j)]
        assert np.array_equal(F1[:, others], F[:, others])
        order = [j, i] if (flip and not same) else [i, j]
        assert np.array_equal(G1[:, [i, j]], G0[:, order])
        assert np.array_equal(Z1[:, [i, j]], Z0[:, order])
    assert swapped > 50 and kept > 50, (swapped, kept)


@pytest.mark.parametrize("cplx", [False, True])
def test_sorted_skip_step_swaps_by_norm(cplx):
    """An orthogonal pair is not transformed, only sorted: column i gets the
    larger norm (Section 2.1, the skip test, with the sorting swap)."""
    rng = np.random.default_rng(34)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)) + (1j * rng.standard_normal((8, 8)) if cplx else 0))
    F = Q[:, :2] * np.array([1.0, 3.0])          # orthogonal, ||f_0|| < ||f_1||
    G = Q[:, 2:4]                                  # orthonormal: b_ij = 0
    Z = np.eye(2, dtype=F.dtype)
    F1, G1, Z1, nall, _ = oracle.step(F, G, Z, 0, 1, sort=True, tol=1e-8)
    assert nall == 0
    assert np.array_equal(F1, F[:, [1, 0]]) and np.array_equal(G1, G[:, [1, 0]])
    assert np.array_equal(Z1, Z[:, [1, 0]])
    F2, _, _, _, _ = oracle.step(F, G, Z, 0, 1, sort=False, tol=1e-8)
    assert np.array_equal(F2, F)
