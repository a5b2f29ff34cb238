"""GPU parity of the complex128 path (hz_zgsvd through the C ABI) against the
CPU oracle: sigma within 1e-10 relative, the GSVD contract of the outputs
(U^H U = V^H V = I, F Z = U Sigma_F, G Z = V Sigma_G), bitwise reruns, the
device complex 2x2 transformation's congruence invariants (Section 2.1.1)."""

import hashlib
import json
import os

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


def _oracle(F, G, **kw):
    import oracle
    return oracle.gsvd(F, G, **kw)


def _run(F, G, **kw):
    hz = _hz()
    dF = torch.from_numpy(np.asfortranarray(F)).cuda()
    dG = torch.from_numpy(np.asfortranarray(G)).cuda()
    r = hz.gsvd(dF, dG, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def _check(F, G, r):
    return assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"],
                           r["sigma"], tol_res=1e-12, tol_orth=1e-12)


def test_device_complex_2x2_invariants():
    hz = _hz()
    rng = np.random.default_rng(41)
    rows, mats = [], []
    for _ in range(3000):
        a = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
        A = a @ a.conj().T
        b = complex(rng.uniform(-0.69, 0.69), rng.uniform(-0.69, 0.69))
        rows.append((A[0, 0].real, A[1, 1].real, A[0, 1].real, A[0, 1].imag, b.real, b.imag))
    # exception v = h = 0, h = 0 with v of both signs, b = 0, diagonal A
    e = np.exp(0.7j)
    rows += [(2.0, 2.0, (1.3 * e).real, (1.3 * e).imag, (0.4 * e).real, (0.4 * e).imag),
             (1.5, 1.5, 0.8, 0.5, 0.3, 0.0), (1.5, 1.5, 0.8, -0.5, 0.3, 0.0),
             (3.0, 1.0, 0.5, 0.2, 0.0, 0.0), (3.0, 1.0, 0.0, 0.0, 0.2, 0.1)]
    out = hz.eval_2x2(torch.tensor(rows, dtype=torch.float64, device="cuda")).cpu().numpy()
    for (aii, ajj, ar, ai, br, bi), z in zip(rows, out):
        A = np.array([[aii, ar + 1j * ai], [ar - 1j * ai, ajj]])
        B = np.array([[1.0, br + 1j * bi], [br - 1j * bi, 1.0]])
        Z = np.array([[z[0], z[3] + 1j * z[4]], [z[1] + 1j * z[2], z[5]]])
        N = Z.conj().T @ B @ Z
        M = Z.conj().T @ A @ Z
        kB = np.linalg.cond(B)
        zn = np.linalg.norm(Z) ** 2
        assert np.max(np.abs(N - np.eye(2))) < 64 * EPS * kB, (aii, ajj, ar, ai, br, bi, N)
        assert abs(M[0, 1]) < 64 * EPS * np.linalg.norm(A) * zn, (aii, ajj, ar, ai, br, bi, M)
        assert z[0] > 0 and z[5] > 0


@pytest.mark.parametrize("shape", [(40, 36, 24, 8), (70, 50, 37, 8), (200, 150, 96, 16),
                                   (300, 256, 160, 16), (64, 64, 2, 8)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("iord", [2, 3], ids=["innerRR", "ring"])
def test_complex_parity(shape, iord):
    m_f, m_g, n, w = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=50.0, is_complex=True, seed=n + 3)
    o = _oracle(F, G, ordering=1, threads=4)
    r = _run(F, G, w=w, inner_ordering=iord)
    err = max_rel(r["sigma"], o["sigma"])
    print(f"{shape}: sweeps={r['sweeps']} status={r['status']} err={err:.2e}")
    assert r["status"] == 0
    assert err < SIG_TOL
    assert max_rel(r["sigma"], s_true) < 1e-11
    _check(F, G, r)


def test_complex_n1():
    rng = np.random.default_rng(8)
    F = rng.standard_normal((6, 1)) + 1j * rng.standard_normal((6, 1))
    G = rng.standard_normal((4, 1)) + 1j * rng.standard_normal((4, 1))
    o = _oracle(F, G)
    r = _run(F, G)
    assert r["status"] == 0
    assert max_rel(r["sigma"], o["sigma"]) < 4 * EPS
    _check(F, G, r)


def test_complex_bo_and_rr():
    F, G, _ = gi.custom_pair(180, 160, 64, kappa=50.0, is_complex=True, seed=12)
    o = _oracle(F, G)
    for kw in (dict(inner_max_sweeps=1), dict(ordering=2), dict(inner_lanes=16),
               dict(inner_ordering=3, inner_max_sweeps=1),
               dict(inner_ordering=3, inner_lanes=16), dict(inner_ordering=3, variant=5)):
        r = _run(F, G, w=16, **kw)
        assert r["status"] == 0
        assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
        _check(F, G, r)


def test_complex_bitwise_reruns():
    F, G, _ = gi.custom_pair(256, 200, 96, kappa=50.0, is_complex=True, seed=13)
    dig = set()
    for _ in range(3):
        r = _run(F, G, w=16)
        h = hashlib.sha256()
        for k in ("U", "V", "Z", "sigma", "sigma_f", "sigma_g"):
            h.update(np.ascontiguousarray(r[k]).tobytes())
        dig.add(h.hexdigest())
    assert len(dig) == 1


def test_complex_rejects_w32():
    hz = _hz()
    F, G, _ = gi.custom_pair(80, 80, 64, is_complex=True, seed=14)
    with pytest.raises(ValueError):
        _run(F, G, w=32)


@pytest.mark.parametrize("iord", [2, 3], ids=["innerRR", "ring"])
def test_config3_full_size_vs_oracle_golden(iord):
    """The complex 3072x1024 / 2048x1024 workload (w = 16, tol = 1024 eps,
    round-robin or ring ordering inside the blocks) against the oracle's
    sigma for the same seeded pair."""
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_config3.json")
    gold = json.load(open(path))
    F, G, s_true = gi.config_pair(3)
    hz = _hz()
    dF = torch.from_numpy(F).cuda()
    dG = torch.from_numpy(G).cuda()
    r = hz.gsvd(dF, dG, w=16, tol=1024 * EPS, inner_max_sweeps=1, inner_ordering=iord)
    torch.cuda.synchronize()
    s = r["sigma"].cpu().numpy()
    err = max_rel(s, np.array(gold["sigma"]))
    print(f"config3: sweeps={r['sweeps']} err_vs_oracle={err:.2e} "
          f"err_vs_prescribed={max_rel(s, s_true):.2e}")
    assert r["status"] == 0
    assert err < SIG_TOL
    U, V, Z = r["U"], r["V"], r["Z"]
    sf, sg = r["sigma_f"], r["sigma_g"]
    n = Z.shape[0]
    fz = torch.linalg.norm(dF @ Z - U * sf) / (torch.linalg.norm(dF) * torch.linalg.norm(Z))
    gz = torch.linalg.norm(dG @ Z - V * sg) / (torch.linalg.norm(dG) * torch.linalg.norm(Z))
    eye = torch.eye(n, dtype=torch.complex128, device=U.device)
    uu = torch.linalg.norm(U.conj().T @ U - eye) / n
    vv = torch.linalg.norm(V.conj().T @ V - eye) / n
    assert float(fz) < 1e-12 and float(gz) < 1e-12, (float(fz), float(gz))
    assert float(uu) < 1e-12 and float(vv) < 1e-12, (float(uu), float(vv))


@pytest.mark.parametrize("w", [8, 16])
def test_complex_rank_deficient_reports_cholesky_failure(w):
    """Two equal columns of the complex G (one a complex multiple of the
    other would do as well): the Hermitian Cholesky of their pivot block
    meets a pivot at rounding level, which the lane holding it reports, and
    the solve stops with HZ_ECHOL."""
    hz = _hz()
    F, G, _ = gi.custom_pair(120, 90, 48, kappa=10.0, is_complex=True, seed=95)
    G[:, 13] = G[:, 12] * np.exp(0.3j)
    dF = torch.from_numpy(np.asfortranarray(F)).cuda()
    dG = torch.from_numpy(np.asfortranarray(G)).cuda()
    print(f"complex rank deficiency, w={w}", flush=True)
    with pytest.raises(hz.GsvdError) as e:
        hz.gsvd(dF, dG, w=w)
    assert e.value.status == hz.HZ_ECHOL
    assert e.value.info.failed_pair >= 0
