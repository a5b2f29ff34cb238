"""GPU parity of the enhanced-dot-product variants 1 and 5 (Table 1,
Appendix A): the inner solver forms the pointwise pivot entries from
products rounded toward -infinity and their non-negative errors, summed
apart.  Checked: the device's rounded-down product and error term bit for
bit against the oracle's (both are exact by definition), sigma against the
oracle's run of the same variant (real and complex pairs) (1e-10 relative, the bar of the plain
path) and the output contract, in the single-pair, batched, mixed and
dataflow forms; and that the variant reaches the kernel (the bits differ
from those of variants 0 and 4)."""

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
    r = _hz().gsvd(_dev(F), _dev(G), **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def test_device_mul_rd_bitwise():
    import oracle
    hz = _hz()
    rng = np.random.default_rng(820)
    a = rng.standard_normal(4000) * 2.0 ** rng.integers(-60, 60, 4000)
    b = rng.standard_normal(4000) * 2.0 ** rng.integers(-60, 60, 4000)
    a = np.r_[a, 1.0 + 2.0 ** -30, 3.0, -(1.0 + 2.0 ** -29), 0.1, 1e300, 2.0, -0.0]
    b = np.r_[b, 1.0 + 2.0 ** -30 - 2.0 ** -52, 0.1, 1.0 + 2.0 ** -31, -0.7, 1e-300, 0.5, 3.0]
    c, d = hz.eval_mul_rd(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    c, d = c.cpu().numpy(), d.cpu().numpy()
    ref = np.array([oracle.mul_rd(x, y) for x, y in zip(a, b)])
    assert np.array_equal(c.view(np.int64), ref[:, 0].view(np.int64))
    assert np.array_equal(d.view(np.int64), ref[:, 1].view(np.int64))
    assert np.all(d >= 0.0)


@pytest.mark.parametrize("variant", [1, 5])
@pytest.mark.parametrize("shape,w,lanes", [((64, 48, 32), 8, 0), ((300, 200, 100), 16, 8),
                                           ((400, 300, 128), 32, 16), ((400, 300, 128), 32, 4)])
def test_enhanced_parity(variant, shape, w, lanes):
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=1e2, seed=830 + n)
    print(f"enhanced variant {variant} {shape} w={w} lanes={lanes}", flush=True)
    r = _run(F, G, w=w, variant=variant, inner_lanes=lanes, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, variant=variant, ordering=oracle.ORD_MM, threads=4)
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)
    p = _run(F, G, w=w, variant=variant & 4, inner_lanes=lanes, ordering=_hz().HZ_ORD_MM)
    assert not np.array_equal(p["Z"], r["Z"])


def test_enhanced_batched():
    import oracle
    hz = _hz()
    pairs = gi.make_batch(count=12, seed=840, n_lo=8, n_hi=80)
    dev = [(_dev(F), _dev(G)) for F, G, _ in pairs]
    print("enhanced batched", flush=True)
    st, outs = hz.gsvd_batched(dev, variant=1)
    torch.cuda.synchronize()
    assert st == 0
    for (F, G, s), o in zip(pairs, outs):
        sig = o["sigma"].cpu().numpy()
        assert max_rel(sig, oracle.gsvd(F, G, variant=1)["sigma"]) < SIG_TOL
        assert max_rel(sig, s) < SIG_TOL


def test_enhanced_mixed():
    import oracle
    F, G, s_true = gi.custom_pair(700, 600, 256, kappa=1e2, seed=850)
    print("enhanced mixed", flush=True)
    r = _run(F, G, mixed=True, w=32, variant=5, inner_max_sweeps=1)
    assert r["status"] == 0 and r["converged"]
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    o = oracle.gsvd(F, G, variant=5, ordering=oracle.ORD_MM, threads=4)
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_enhanced_dataflow_matches_steps():
    """The dataflow schedule runs the same task arithmetic as the per-step
    kernels, so with variant 1 the two agree bit for bit."""
    hz = _hz()
    F, G, _ = gi.custom_pair(520, 400, 256, kappa=1e2, seed=860)
    print("enhanced dataflow", flush=True)
    a = _run(F, G, w=32, variant=1, inner_max_sweeps=1, schedule=hz.HZ_SCHED_DATAFLOW)
    b = _run(F, G, w=32, variant=1, inner_max_sweeps=1, schedule=hz.HZ_SCHED_STEPS)
    assert a["status"] == 0 and b["status"] == 0
    for k in ("sigma", "U", "V", "Z"):
        assert np.array_equal(a[k], b[k])


@pytest.mark.parametrize("variant", [1, 5])
@pytest.mark.parametrize("shape,w", [((120, 90, 32), 8), ((300, 200, 100), 16)])
def test_enhanced_complex_parity(variant, shape, w):
    """Complex pairs: the squared norms by the simpler procedure of Appendix
    A, the off-diagonal entries ordinary."""
    import oracle
    m_f, m_g, n = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=1e2, is_complex=True, seed=870 + n)
    print(f"enhanced complex variant {variant} {shape} w={w}", flush=True)
    r = _run(F, G, w=w, variant=variant, ordering=_hz().HZ_ORD_MM)
    assert r["status"] == 0 and r["converged"]
    o = oracle.gsvd(F, G, variant=variant, ordering=oracle.ORD_MM, threads=4)
    assert max_rel(r["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"], s_true) < SIG_TOL
    assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"], r["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)
    p = _run(F, G, w=w, variant=variant & 4, ordering=_hz().HZ_ORD_MM)
    assert not np.array_equal(p["Z"], r["Z"])
