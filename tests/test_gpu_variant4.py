"""GPU parity of variant 4 (criterion C2 of Section 2.5: a transformation is
small when the unscaled cosines cos(phi), cos(psi) are exactly 1) for the
real, complex, mixed and batched solvers against the oracle run with the
same variant, and the special case that pins it independently: with
orthonormal G every pivot has t = 1, both criteria coincide and the GPU runs
of variants 0 and 4 agree bit for bit."""

import numpy as np
import pytest

import gsvd_inputs as gi
from contract import assert_contract, max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIG_TOL = 1e-10


def _hz():
    import paper_1909_00101_amd as hz
    return hz


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def _run(F, G, **kw):
    hz = _hz()
    r = hz.gsvd(_dev(F), _dev(G), **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


@pytest.mark.parametrize("w,cplx,mixed", [(8, False, False), (16, False, False),
                                          (32, False, False), (16, True, False),
                                          (16, False, True)],
                         ids=["real-w8", "real-w16", "real-w32", "complex-w16", "mixed-w16"])
def test_variant4_parity(w, cplx, mixed):
    import oracle
    F, G, s_true = gi.custom_pair(300, 260, 128, kappa=1e2, is_complex=cplx, seed=410 + w)
    o = oracle.gsvd(F, G, variant=4, threads=4)
    r = _run(F, G, w=w, variant=4, mixed=mixed)
    print(f"w={w} cplx={cplx} mixed={mixed}: sweeps={r['sweeps']} oracle={o['sweeps']} "
          f"err={max_rel(r['sigma'], o['sigma']):.2e}")
    assert r["status"] == 0 and r["converged"]
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < 1e-11
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_variant4_equals_variant0_for_orthonormal_g():
    rng = np.random.default_rng(420)
    F = rng.standard_normal((400, 96))
    G, _ = np.linalg.qr(rng.standard_normal((300, 96)))
    a = _run(F, G, w=16, variant=0)
    b = _run(F, G, w=16, variant=4)
    assert a["sweeps"] == b["sweeps"] and a["rot_big"] == b["rot_big"]
    for k in ("sigma", "U", "V", "Z"):
        assert np.array_equal(a[k], b[k])


def test_variant4_batched():
    import oracle
    hz = _hz()
    pairs = gi.make_batch(count=10, seed=430, n_lo=8, n_hi=96)
    st, outs = hz.gsvd_batched([(_dev(F), _dev(G)) for F, G, _ in pairs], variant=4)
    torch.cuda.synchronize()
    assert st == 0
    for (F, G, s_true), o in zip(pairs, outs):
        s = o["sigma"].cpu().numpy()
        assert max_rel(s, oracle.gsvd(F, G, variant=4)["sigma"]) < SIG_TOL
        assert max_rel(s, s_true) < 1e-11
