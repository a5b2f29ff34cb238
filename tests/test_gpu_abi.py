"""GPU checks of the C ABI itself, called through ctypes without the Python
convenience layer: leading dimensions larger than the row counts (the
library must read F, G and write U, V, Z through ldf, ldg, ldz and leave the
padding rows alone), work = NULL (the library allocates its own
workspace), and small n bordered up to one block pair of the widest
width."""

import ctypes

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


def _padded(a, ld, fill):
    """Column-major device buffer with leading dimension ld holding a; the
    rows beyond a's are set to fill."""
    m, n = a.shape
    buf = np.full((ld, n), fill, dtype=a.dtype, order="F")
    buf[:m, :] = a
    return torch.from_numpy(buf).cuda()


@pytest.mark.parametrize("cplx", [False, True])
def test_leading_dimensions_and_null_workspace(cplx):
    import oracle
    hz = _hz()
    L = hz.lib()
    m_f, m_g, n = 150, 120, 40
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=30.0, is_complex=cplx, seed=501)
    ldf, ldg, ldz = m_f + 7, m_g + 13, n + 5
    fill = 12345.0
    dF, dG = _padded(F, ldf, fill), _padded(G, ldg, fill)
    dtype = torch.complex128 if cplx else torch.float64
    dZ = torch.from_numpy(np.full((ldz, n), fill, dtype=F.dtype, order="F")).cuda()
    # the buffers hold exactly ld * n elements of the solver's type
    for d, ld in ((dF, ldf), (dG, ldg), (dZ, ldz)):
        assert d.dtype == dtype and d.numel() == ld * n
    sig = torch.empty(n, dtype=torch.float64, device="cuda")
    sf, sg = torch.empty_like(sig), torch.empty_like(sig)
    p = hz.params(w=8)
    info = hz.HzInfo()
    fn = L.hz_zgsvd if cplx else L.hz_dgsvd
    st = fn(ctypes.byref(p), m_f, m_g, n, ctypes.c_void_p(dF.data_ptr()), ldf,
            ctypes.c_void_p(dG.data_ptr()), ldg, ctypes.c_void_p(dZ.data_ptr()), ldz,
            ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(sf.data_ptr()),
            ctypes.c_void_p(sg.data_ptr()), None, 0, ctypes.byref(info), None)
    torch.cuda.synchronize()
    assert st == 0 and info.converged
    Uf, Vf, Zf = dF.cpu().numpy(), dG.cpu().numpy(), dZ.cpu().numpy()
    # padding rows untouched
    assert np.all(Uf[m_f:, :] == fill) and np.all(Vf[m_g:, :] == fill)
    assert np.all(Zf[n:, :] == fill)
    U, V, Z = Uf[:m_f, :], Vf[:m_g, :], Zf[:n, :]
    s = sig.cpu().numpy()
    o = oracle.gsvd(F, G)
    assert max_rel(s, o["sigma"]) < SIG_TOL
    assert max_rel(s, s_true) < 1e-11
    assert_contract(F, G, U, V, Z, sf.cpu().numpy(), sg.cpu().numpy(), s,
                    tol_res=1e-12, tol_orth=1e-12)


@pytest.mark.parametrize("n", [2, 3, 5, 33])
def test_small_n_bordered_to_the_widest_block(n):
    """n far below 2w = 64: the pair is bordered to 64 columns (one pivot pair,
    two steps); the bordering columns must not leak into the outputs."""
    import oracle
    hz = _hz()
    F, G, s_true = gi.custom_pair(n + 40, n + 17, n, kappa=10.0, seed=510 + n)
    r = hz.gsvd(torch.from_numpy(np.asfortranarray(F)).cuda(),
                torch.from_numpy(np.asfortranarray(G)).cuda(), w=32)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}
    assert res["status"] == 0
    assert max_rel(res["sigma"], oracle.gsvd(F, G)["sigma"]) < SIG_TOL
    assert_contract(F, G, res["U"], res["V"], res["Z"], res["sigma_f"], res["sigma_g"],
                    res["sigma"], tol_res=1e-12, tol_orth=1e-12)


def test_misaligned_exact_workspace_is_not_overrun():
    """A caller workspace 8 bytes past a 256-byte boundary holding exactly
    the bytes the solve needs: the binding may not place the aligned
    workspace past its end.  Bytes after the view must stay untouched, and
    the solve must be bitwise the one with a fresh workspace."""
    hz = _hz()
    F, G, _ = gi.custom_pair(90, 70, 24, kappa=10.0, seed=520)
    dF = torch.from_numpy(np.asfortranarray(F)).cuda()
    dG = torch.from_numpy(np.asfortranarray(G)).cuda()
    p = hz.params(w=8)
    need = hz.lib().hz_dgsvd_work_size(ctypes.byref(p), 90, 70, 24)
    base = torch.full((need + 2048,), 0xA5, dtype=torch.uint8, device="cuda")
    off = (-base.data_ptr()) % 256 + 8
    view = base[off:off + need]
    ref = hz.gsvd(dF, dG, w=8)
    got = hz.gsvd(dF, dG, w=8, workspace=view)
    torch.cuda.synchronize()
    assert torch.all(base[off + need:] == 0xA5).item()
    for k in ("U", "V", "Z", "sigma", "sigma_f", "sigma_g"):
        assert torch.equal(ref[k], got[k]), k


def test_batched_null_workspace_equals_caller_workspace():
    """hz_dgsvd_batched with work = NULL (stream-ordered allocation inside
    the library) gives bitwise the results of the same call on a caller
    workspace; the pairs include n = 1."""
    hz = _hz()
    L = hz.lib()
    pairs = gi.make_batch(count=6, seed=530, n_lo=2, n_hi=70)
    rng = np.random.default_rng(531)
    pairs.append((rng.standard_normal((9, 1)), rng.standard_normal((4, 1)), None))

    def run(null_work):
        W = [(torch.from_numpy(np.asfortranarray(F)).cuda(),
              torch.from_numpy(np.asfortranarray(G)).cuda()) for F, G, _ in pairs]
        batch = len(W)
        ns = [f.shape[1] for f, _ in W]
        Zs = [torch.empty((n, n), dtype=torch.float64, device="cuda").t() for n in ns]
        sig = [torch.empty(n, dtype=torch.float64, device="cuda") for n in ns]
        sf = [torch.empty_like(x) for x in sig]
        sg = [torch.empty_like(x) for x in sig]
        i64 = lambda v: (ctypes.c_int64 * batch)(*v)
        ptrs = lambda ts: (ctypes.c_void_p * batch)(*[t.data_ptr() for t in ts])
        # leading dimension of a column-major buffer (a single column's stride
        # is arbitrary)
        ld = lambda t: t.shape[0] if t.shape[1] == 1 else t.stride(1)
        p = hz.params(w=16)
        mf, mg, nn = i64([f.shape[0] for f, _ in W]), i64([g.shape[0] for _, g in W]), i64(ns)
        nbytes = L.hz_dgsvd_batched_work_size(ctypes.byref(p), batch, mf, mg, nn)
        work = None if null_work else torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        wptr = None if null_work else ctypes.c_void_p((work.data_ptr() + 255) & ~255)
        infos = (hz.HzInfo * batch)()
        st = L.hz_dgsvd_batched(ctypes.byref(p), batch, mf, mg, nn, ptrs([f for f, _ in W]),
                                i64([ld(f) for f, _ in W]), ptrs([g for _, g in W]),
                                i64([ld(g) for _, g in W]), ptrs(Zs), i64(ns), ptrs(sig),
                                ptrs(sf), ptrs(sg), wptr, 0 if null_work else nbytes, infos,
                                None)
        torch.cuda.synchronize()
        return st, [infos[i].status for i in range(batch)], \
            [(f.cpu().numpy(), g.cpu().numpy(), z.cpu().numpy(), s.cpu().numpy())
             for (f, g), z, s in zip(W, Zs, sig)]

    st0, s0, a = run(False)
    st1, s1, b = run(True)
    assert st0 == st1 == 0 and s0 == s1
    for i, (ra, rb) in enumerate(zip(a, b)):
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y), i


def test_n1_null_workspace():
    """n = 1 with work = NULL: the closed form with the library's own status
    word, sigma = ||f|| / ||g||."""
    hz = _hz()
    L = hz.lib()
    rng = np.random.default_rng(540)
    F, G = rng.standard_normal((11, 1)), rng.standard_normal((6, 1))
    dF = torch.from_numpy(np.asfortranarray(F)).cuda()
    dG = torch.from_numpy(np.asfortranarray(G)).cuda()
    dZ = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    sig = torch.empty(1, dtype=torch.float64, device="cuda")
    sf, sg = torch.empty_like(sig), torch.empty_like(sig)
    info = hz.HzInfo()
    st = L.hz_dgsvd(None, 11, 6, 1, ctypes.c_void_p(dF.data_ptr()), 11,
                    ctypes.c_void_p(dG.data_ptr()), 6, ctypes.c_void_p(dZ.data_ptr()), 1,
                    ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(sf.data_ptr()),
                    ctypes.c_void_p(sg.data_ptr()), None, 0, ctypes.byref(info), None)
    torch.cuda.synchronize()
    assert st == 0 and info.converged
    want = np.linalg.norm(F) / np.linalg.norm(G)
    assert abs(sig.item() - want) <= 4 * np.finfo(np.float64).eps * want
