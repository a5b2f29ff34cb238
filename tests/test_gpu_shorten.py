"""GPU parity of the QR-shortened real path (hz_dgsvd with qr_shorten = 1,
Section 2) against the oracle's shortened solve (scipy's column-pivoted
Householder QR around the unblocked oracle) and the plain oracle.

The GPU forms the pivoted QR from the Gram matrices (pivoted Cholesky plus
one Cholesky-QR refinement), so its R factors and the square pair it
iterates on agree with the oracle's only to rounding; the outputs that are
unique are compared directly: sigma (1e-10 relative, the bar of the plain
path) and Z, which with Sigma_F^2 + Sigma_G^2 = I is unique up to column
signs for distinct sigma (compared after aligning signs).  U and V are
checked through the output contract on the original pair.
"""

import ctypes

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
    hz = _hz()
    r = hz.gsvd(torch.from_numpy(np.asfortranarray(F)).cuda(),
                torch.from_numpy(np.asfortranarray(G)).cuda(), qr_shorten=1, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def _z_err(Z, Zref):
    c = np.sum(Z * Zref, axis=0)
    return float(np.max(np.abs(Z * np.sign(c) - Zref)) / np.max(np.abs(Zref)))


@pytest.mark.parametrize("shape,w", [((300, 200, 60), 8), ((150, 120, 40), 16),
                                     ((64, 48, 32), 8), ((90, 150, 17), 8),
                                     ((40, 40, 40), 16), ((400, 300, 100), 16),
                                     ((700, 650, 130), 32), ((5, 4, 2), 8)])
def test_shortened_parity(shape, w):
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=50.0, seed=700 + n)
    print(f"shortened parity {shape} w={w}", flush=True)
    r = _run(F, G, w=w, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd_qr(F, G, ordering=oracle.ORD_MM)
    p = oracle.gsvd(F, G, ordering=oracle.ORD_MM)
    print(f"  sweeps gpu={r['sweeps']} oracle_qr={o['sweeps']} plain={p['sweeps']} "
          f"err={max_rel(r['sigma'], o['sigma']):.2e} z={_z_err(r['Z'], o['Z']):.2e}")
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], p["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert _z_err(r["Z"], o["Z"]) < 1e-9
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_shortened_headline_shape():
    """F, G 4096 x 1024 with w = 32, modified modulus, tol = 1024 eps, the
    launch of the plain path's headline workload: sigma against the oracle's
    sigma for the same seeded pair (tests/golden/oracle_config2.json, written
    by tests/golden/make_golden.py from the oracle alone), against the known
    generalized singular values of the generator, and the contract."""
    import json
    import os
    gold = np.array(json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                                 "oracle_config2.json")))["sigma"])
    F, G, s_true = gi.config_pair(2)
    print("shortened 4096x1024 w=32", flush=True)
    r = _run(F, G, w=32, ordering=_hz().HZ_ORD_MM, tol=1024 * EPS)
    err = max_rel(r["sigma"], gold)
    print(f"  sweeps={r['sweeps']} err_vs_oracle={err:.2e} "
          f"err_vs_truth={max_rel(r['sigma'], s_true):.2e}")
    assert r["status"] == 0 and r["converged"]
    assert err < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_shortened_leading_dimensions():
    """Through the C ABI with ldf, ldg, ldz above the row counts: the padding
    rows are neither read into the factorization nor written."""
    import oracle
    hz = _hz()
    L = hz.lib()
    m_f, m_g, n = 130, 100, 36
    F, G, _ = gi.custom_pair(m_f, m_g, n, kappa=20.0, seed=720)
    ldf, ldg, ldz = m_f + 5, m_g + 3, n + 9
    fill = 777.0

    def padded(a, ld):
        b = np.full((ld, a.shape[1]), fill, order="F")
        b[:a.shape[0], :] = a
        return torch.from_numpy(b).cuda()

    dF, dG = padded(F, ldf), padded(G, ldg)
    dZ = torch.from_numpy(np.full((ldz, n), fill, order="F")).cuda()
    sig = torch.empty(n, dtype=torch.float64, device="cuda")
    sf, sg = torch.empty_like(sig), torch.empty_like(sig)
    p = hz.params(w=8, qr_shorten=1)
    info = hz.HzInfo()
    st = L.hz_dgsvd(ctypes.byref(p), m_f, m_g, n, ctypes.c_void_p(dF.data_ptr()), ldf,
                    ctypes.c_void_p(dG.data_ptr()), ldg, ctypes.c_void_p(dZ.data_ptr()), ldz,
                    ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(sf.data_ptr()),
                    ctypes.c_void_p(sg.data_ptr()), None, 0, ctypes.byref(info), None)
    torch.cuda.synchronize()
    assert st == 0 and info.converged
    Uf, Vf, Zf = dF.cpu().numpy(), dG.cpu().numpy(), dZ.cpu().numpy()
    assert np.all(Uf[m_f:] == fill) and np.all(Vf[m_g:] == fill) and np.all(Zf[n:] == fill)
    o = oracle.gsvd_qr(F, G)
    assert max_rel(sig.cpu().numpy(), o["sigma"]) < SIG_TOL
    assert_contract(F, G, Uf[:m_f], Vf[:m_g], Zf[:n], sf.cpu().numpy(), sg.cpu().numpy(),
                    sig.cpu().numpy(), tol_res=1e-12, tol_orth=1e-12)


def test_shortened_rank_deficient_f():
    """A zero column makes F rank deficient: the pivoted Cholesky of F^T F
    meets an exactly zero pivot at its last step and the solve returns
    HZ_ECHOL before any sweep, with failed_pair = -1."""
    hz = _hz()
    F, G, _ = gi.custom_pair(80, 70, 20, kappa=10.0, seed=730)
    F[:, 7] = 0.0
    print("shortened rank-deficient F", flush=True)
    with pytest.raises(hz.GsvdError) as ei:
        _run(F, G, w=8)
    assert ei.value.status == hz.HZ_ECHOL
    assert ei.value.info.failed_pair == -1 and ei.value.info.sweeps == 0


def test_shortened_mixed():
    """The mixed-precision solver on the shortened pair: FP32 sweeps and the
    FP64 restart run on (R_F P2, R_G); sigma against the oracle's, the
    contract on the original pair."""
    import oracle
    F, G, s_true = gi.custom_pair(1500, 1200, 256, kappa=1e2, seed=740)
    print("shortened mixed 1500x256", flush=True)
    r = _run(F, G, w=32, inner_max_sweeps=1, mixed=True)
    assert r["status"] == 0 and r["converged"]
    print(f"  sweeps fp32={r['sweeps_fp32']} fp64={r['sweeps']}")
    assert r["sweeps_fp32"] > 0
    assert max_rel(r["sigma"], oracle.gsvd(F, G, threads=4)["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def _z_err_phase(Z, Zref):
    c = np.sum(Z.conj() * Zref, axis=0)
    return float(np.max(np.abs(Z * (c / np.abs(c)) - Zref)) / np.max(np.abs(Zref)))


@pytest.mark.parametrize("shape,w", [((150, 120, 40), 8), ((300, 200, 100), 16),
                                     ((64, 48, 32), 16), ((21, 19, 3), 8)])
def test_shortened_complex_parity(shape, w):
    """Complex pairs: Hermitian Grams, the Hermitian pivoted Cholesky and the
    complex triangular solves; Z is unique up to unit phases of its columns."""
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=30.0, is_complex=True, seed=750 + n)
    print(f"shortened complex {shape} w={w}", flush=True)
    r = _run(F, G, w=w, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd_qr(F, G, ordering=oracle.ORD_MM)
    print(f"  sweeps {r['sweeps']} err {max_rel(r['sigma'], o['sigma']):.2e} "
          f"z {_z_err_phase(r['Z'], o['Z']):.2e}")
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert _z_err_phase(r["Z"], o["Z"]) < 1e-9
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_shortened_complex_workload_shape():
    """The complex 3072x1024 / 2048x1024 pair at w = 16."""
    F, G, s_true = gi.config_pair(3)
    print("shortened complex 3072x1024", flush=True)
    r = _run(F, G, w=16, ordering=_hz().HZ_ORD_MM, inner_max_sweeps=1,
             tol=1024 * EPS)
    print(f"  sweeps {r['sweeps']} err_vs_truth {max_rel(r['sigma'], s_true):.2e}")
    assert r["status"] == 0 and r["converged"]
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)
