"""hz_dgsvd_noalloc, the entry point that allocates nothing, against
hz_dgsvd with the same parameters: two calls in a row on one process's
static scratch, the second on a smaller pair, each bitwise equal to
hz_dgsvd's result (the same kernels on the same inputs) and within the
parity tolerance of the CPU oracle; a solve whose workspace exceeds the
scratch is refused before anything is launched."""

import numpy as np
import pytest

import gsvd_inputs as gi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIG_TOL = 1e-10
EPS = np.finfo(np.float64).eps


def _hz():
    import paper_1909_00101_amd as hz
    return hz


def _noalloc(F, G, **kw):
    hz = _hz()
    U = torch.from_numpy(np.asfortranarray(F)).cuda()
    V = torch.from_numpy(np.asfortranarray(G)).cuda()
    n = F.shape[1]
    Z = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    sig = torch.empty(n, dtype=torch.float64, device="cuda")
    sf, sg = torch.empty_like(sig), torch.empty_like(sig)
    st, info = hz.gsvd_noalloc(U, V, Z, sig, sf, sg, **kw)
    torch.cuda.synchronize()
    return st, info, dict(U=U, V=V, Z=Z, sigma=sig, sigma_f=sf, sigma_g=sg)


# (m_f, m_g, n, kappa, seed, w): the second pair is smaller than the first,
# ragged in n (bordered up to a multiple of 2w) and in the row counts.
CALLS = [(520, 480, 300, 50.0, 7101, 32), (130, 129, 37, 20.0, 7102, 16)]


def test_noalloc_matches_hz_dgsvd_on_two_calls_in_a_row():
    import oracle
    hz = _hz()
    for m_f, m_g, n, kappa, seed, w in CALLS:
        print(f"noalloc call: {m_f}x{n} / {m_g}x{n}, w={w}, seed={seed}", flush=True)
        F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=kappa, seed=seed)
        kw = dict(w=w, inner_max_sweeps=1, tol=n * EPS)
        ref = hz.gsvd(torch.from_numpy(F).cuda(), torch.from_numpy(G).cuda(), **kw)
        torch.cuda.synchronize()
        st, info, out = _noalloc(F, G, **kw)
        assert st == ref["status"] == hz.HZ_OK
        assert info.sweeps == ref["sweeps"] and info.converged == 1
        assert info.rot_total == ref["rot_total"] and info.updates_skipped == ref["updates_skipped"]
        for k in ("U", "V", "Z", "sigma", "sigma_f", "sigma_g"):
            assert torch.equal(out[k], ref[k]), k
        orc = oracle.gsvd(F, G, tol=n * EPS)
        s = out["sigma"].cpu().numpy()
        err = float(np.max(np.abs(s - orc["sigma"]) / orc["sigma"]))
        assert err < SIG_TOL, err


def test_noalloc_refuses_a_solve_beyond_its_scratch():
    hz = _hz()
    L = hz.lib()
    import ctypes
    m, n = 8192, 2048
    p = hz.params(w=32)
    need = L.hz_dgsvd_work_size(ctypes.byref(p), m, m, n)
    assert need > hz.HZ_NOALLOC_SCRATCH_BYTES
    # full-size buffers, so that nothing could be out of bounds had it run
    U = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    V = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    Z = torch.zeros((n, n), dtype=torch.float64, device="cuda").t()
    sig = torch.zeros(n, dtype=torch.float64, device="cuda")
    sf, sg = torch.zeros_like(sig), torch.zeros_like(sig)
    st, _ = hz.gsvd_noalloc(U, V, Z, sig, sf, sg, w=32)
    torch.cuda.synchronize()
    assert st == hz.HZ_ENOSCRATCH
    assert float(sig.abs().sum()) == 0.0 and float(U.abs().sum()) == 0.0
