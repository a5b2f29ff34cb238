"""GPU parity of the QR pivot factors (hz_dgsvd with pivot_qr = 1, Section
2.3 and Appendix E): the triangular factors of the block-column pairs come
from a tree of Householder factorizations instead of Cholesky factors of
their Grams.

Well-conditioned pairs: sigma within 1e-10 of the oracle's and the output
contract, as on the Gram path.  A pair whose F is too ill-conditioned for
its Grams (kappa(X) = 10, sigma down to 1e-9, so kappa(F D) is about 2e9,
D the prescaling): the Gram path stops with HZ_ECHOL, the QR path converges
and its sigma agree with the oracle's and the prescribed ones within
8 eps kappa(F D), the accuracy the one-sided method has on F D."""

import numpy as np
import pytest

import gsvd_inputs as gi
from contract import assert_contract, max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
SIG_TOL = 1e-10


def _hz():
    import paper_1909_00101_amd as hz
    return hz


def _run(F, G, **kw):
    r = _hz().gsvd(torch.from_numpy(np.asfortranarray(F)).cuda(),
                   torch.from_numpy(np.asfortranarray(G)).cuda(), **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


@pytest.mark.parametrize("shape,w", [((64, 48, 32), 8), ((300, 200, 100), 16),
                                     ((700, 650, 256), 32), ((129, 100, 64), 32),
                                     ((40, 40, 40), 16)])
def test_qr_factors_parity(shape, w):
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=1e2, seed=900 + n)
    print(f"pivot_qr parity {shape} w={w}", flush=True)
    r = _run(F, G, w=w, pivot_qr=1, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=4)
    print(f"  sweeps {r['sweeps']} err {max_rel(r['sigma'], o['sigma']):.2e}")
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


@pytest.mark.parametrize("shape,w", [((4700, 300, 128), 32), ((300, 4700, 96), 16)])
def test_qr_factors_three_tree_levels(shape, w):
    """The taller matrix takes three levels of the QR tree (4700 rows: 10
    nodes of 512 rows, then 2, then 1) while the other has one node from the
    start and is carried through the later levels as one triangle stacked on
    zeros (its factorization must come out unchanged)."""
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=1e2, seed=930 + n)
    print(f"pivot_qr three tree levels {shape} w={w}", flush=True)
    r = _run(F, G, w=w, pivot_qr=1, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=4)
    print(f"  sweeps {r['sweeps']} err {max_rel(r['sigma'], o['sigma']):.2e}")
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def _ill_pair(n):
    F, G, s_true = gi.custom_pair(3 * n, 2 * n, n, kappa=10.0, sig_lo=1e-9, sig_hi=1e2,
                                  seed=910 + n)
    d = 1.0 / np.linalg.norm(G, axis=0)
    return F, G, s_true, 8 * EPS * np.linalg.cond(F * d)


def _check_ill(F, G, s_true, bound, r):
    import oracle
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=4)
    print(f"  sweeps {r['sweeps']} err_oracle {max_rel(r['sigma'], o['sigma']):.2e} "
          f"err_truth {max_rel(r['sigma'], s_true):.2e} oracle_err {max_rel(o['sigma'], s_true):.2e}")
    assert o["status"] == 0
    assert max_rel(r["sigma"], s_true) < bound
    assert max_rel(r["sigma"], o["sigma"]) < bound
    # orthonormality of U and V holds to rounding
    n_ = r["Z"].shape[0]
    assert np.linalg.norm(r["U"].T @ r["U"] - np.eye(n_)) / n_ < 1e-12
    assert np.linalg.norm(r["V"].T @ r["V"] - np.eye(n_)) / n_ < 1e-12


def test_qr_factors_where_grams_fail():
    """n = 64, w = 32: the one block pair is all of F, its Gram is not
    positive definite in floating point and the Gram path stops with
    HZ_ECHOL; the QR path converges to the prescribed sigma."""
    hz = _hz()
    F, G, s_true, bound = _ill_pair(64)
    print(f"ill-conditioned F n=64 w=32: 8 eps kappa(FD) = {bound:.1e}", flush=True)
    with pytest.raises(hz.GsvdError) as ei:
        _run(F, G, w=32, ordering=hz.HZ_ORD_MM)
    assert ei.value.status == hz.HZ_ECHOL
    _check_ill(F, G, s_true, bound, _run(F, G, w=32, pivot_qr=1, ordering=hz.HZ_ORD_MM))


@pytest.mark.parametrize("n,w", [(128, 32), (96, 16)])
def test_qr_factors_ill_conditioned(n, w):
    """Block pairs that are column subsets of the ill-conditioned F: the QR
    path reaches the accuracy bound; the Gram path's error is printed for
    comparison."""
    hz = _hz()
    F, G, s_true, bound = _ill_pair(n)
    print(f"ill-conditioned F n={n} w={w}: 8 eps kappa(FD) = {bound:.1e}", flush=True)
    try:
        g = _run(F, G, w=w, ordering=hz.HZ_ORD_MM)
        print(f"  Gram path: status {g['status']} err_truth {max_rel(g['sigma'], s_true):.2e}")
    except hz.GsvdError as e:
        print(f"  Gram path: status {e.status}")
    _check_ill(F, G, s_true, bound, _run(F, G, w=w, pivot_qr=1, ordering=hz.HZ_ORD_MM))


def test_qr_factors_with_shortening():
    """pivot_qr on the square pair of the QR-shortened solve."""
    import oracle
    F, G, s_true = gi.custom_pair(900, 700, 128, kappa=1e2, seed=920)
    print("pivot_qr with qr_shorten", flush=True)
    r = _run(F, G, w=16, pivot_qr=1, qr_shorten=1)
    assert r["status"] == 0
    assert max_rel(r["sigma"], oracle.gsvd(F, G, threads=4)["sigma"]) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


@pytest.mark.parametrize("shape,w", [((64, 48, 32), 8), ((300, 200, 100), 16),
                                     ((129, 100, 64), 16), ((40, 40, 40), 8),
                                     ((4700, 260, 64), 16)])
def test_qr_factors_complex_parity(shape, w):
    """Complex pairs: Householder reflectors with complex tau and a real
    diagonal in R, which the complex inner solver takes as its factor (the
    4700-row F takes three levels of the QR tree)."""
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=50.0, is_complex=True, seed=930 + n)
    print(f"pivot_qr complex {shape} w={w}", flush=True)
    r = _run(F, G, w=w, pivot_qr=1, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=4)
    print(f"  sweeps {r['sweeps']} err {max_rel(r['sigma'], o['sigma']):.2e}")
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_qr_factors_complex_ill_conditioned():
    """A complex pair with F too ill-conditioned for its Grams (kappa(X) =
    10, sigma down to 1e-9; n = 32, w = 16: the one block pair is all of F):
    the QR path reaches 8 eps kappa(F D) against the prescribed sigma and the
    oracle; the Gram path's outcome is printed."""
    import oracle
    hz = _hz()
    n = 32
    F, G, s_true = gi.custom_pair(3 * n, 2 * n, n, kappa=10.0, sig_lo=1e-9, sig_hi=1e2,
                                  is_complex=True, seed=940)
    d = 1.0 / np.linalg.norm(G, axis=0)
    bound = 8 * EPS * np.linalg.cond(F * d)
    print(f"complex ill-conditioned F: 8 eps kappa(FD) = {bound:.1e}", flush=True)
    try:
        g = _run(F, G, w=16, ordering=hz.HZ_ORD_MM)
        print(f"  Gram path: status {g['status']} err_truth {max_rel(g['sigma'], s_true):.2e}")
    except hz.GsvdError as e:
        print(f"  Gram path: status {e.status}")
    r = _run(F, G, w=16, pivot_qr=1, ordering=hz.HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, ordering=oracle.ORD_MM, threads=4)
    print(f"  QR path: sweeps {r['sweeps']} err_truth {max_rel(r['sigma'], s_true):.2e} "
          f"err_oracle {max_rel(r['sigma'], o['sigma']):.2e}")
    assert max_rel(r["sigma"], s_true) < bound
    assert max_rel(r["sigma"], o["sigma"]) < bound
