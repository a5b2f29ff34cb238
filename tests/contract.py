"""Checks of the GSVD output contract (paper, Section 1), shared by the oracle
pins and the GPU parity tests.  Pure numpy; imports neither the oracle nor
the GPU library."""

import numpy as np

EPS = np.finfo(np.float64).eps


def contract_residuals(F, G, U, V, Z, sf, sg, s):
    """Normwise residuals of F Z = U Sigma_F, G Z = V Sigma_G, U^*U = I,
    V^*V = I, Sigma_F^2 + Sigma_G^2 = 1, sigma = Sigma_F/Sigma_G and of the
    GEVD link F^*F Z = G^*G Z Sigma^2 (columnwise, relative)."""
    n = Z.shape[0]
    out = {}
    out["fz"] = np.linalg.norm(F @ Z - U * sf) / (np.linalg.norm(F) * np.linalg.norm(Z))
    out["gz"] = np.linalg.norm(G @ Z - V * sg) / (np.linalg.norm(G) * np.linalg.norm(Z))
    out["uu"] = np.linalg.norm(U.conj().T @ U - np.eye(n)) / max(1, n)
    out["vv"] = np.linalg.norm(V.conj().T @ V - np.eye(n)) / max(1, n)
    out["pyth"] = np.max(np.abs(sf * sf + sg * sg - 1.0))
    out["ratio"] = np.max(np.abs(s - sf / sg) / s)
    A = F.conj().T @ F
    B = G.conj().T @ G
    gev = np.linalg.norm(A @ Z - B @ Z * (s * s), axis=0) / (
        np.linalg.norm(A) * np.linalg.norm(Z, axis=0) * np.maximum(1.0, s * s))
    out["gevd"] = np.max(gev)
    out["sorted"] = bool(np.all(np.diff(s) <= 0))
    return out


def assert_contract(F, G, U, V, Z, sf, sg, s, tol_res=1e-13, tol_orth=1e-13):
    r = contract_residuals(F, G, U, V, Z, sf, sg, s)
    assert r["fz"] < tol_res and r["gz"] < tol_res, r
    assert r["uu"] < tol_orth and r["vv"] < tol_orth, r
    assert r["pyth"] < 8 * EPS, r
    assert r["ratio"] < 8 * EPS, r
    assert r["gevd"] < 1e-12, r
    assert r["sorted"], r
    assert np.all(sf > 0) and np.all(sg > 0)
    return r


def max_rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b) / np.abs(b)))
