"""GPU checks of the autotuner (hz_dgsvd_tune, hz_dgsvd_batched_tune): it
leaves the input untouched, returns parameters with which the solver
converges to oracle parity, persists its choice in the cache file and
returns the cached choice on the next call without timing again."""

import numpy as np
import pytest

import gsvd_inputs as gi
from contract import max_rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIG_TOL = 1e-10


def _hz():
    import paper_1909_00101_amd as hz
    return hz


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def test_tune_single_pair(tmp_path):
    import oracle
    hz = _hz()
    F, G, _ = gi.custom_pair(600, 500, 256, kappa=1e2, seed=61)
    dF, dG = _dev(F), _dev(G)
    cache = str(tmp_path / "tune.txt")
    best, ms = hz.tune(dF, dG, cache=cache, w=16)
    torch.cuda.synchronize()
    assert np.array_equal(dF.cpu().numpy(), F) and np.array_equal(dG.cpu().numpy(), G)
    assert best["w"] == 16 and ms > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1
    again, ms2 = hz.tune(dF, dG, cache=cache, w=16)
    assert again == best and ms2 == pytest.approx(ms, rel=1e-5)
    assert len(open(cache).read().splitlines()) == 1
    r = hz.gsvd(dF, dG, **best)
    assert r["status"] == 0
    o = oracle.gsvd(F, G, threads=4)
    assert max_rel(r["sigma"].cpu().numpy(), o["sigma"]) < SIG_TOL


def test_tune_batched(tmp_path):
    import oracle
    hz = _hz()
    pairs = gi.make_batch(count=24, seed=71, n_lo=8, n_hi=96)
    dev = [(_dev(F), _dev(G)) for F, G, _ in pairs]
    cache = str(tmp_path / "tune.txt")
    best, ms = hz.tune_batched(dev, cache=cache)
    torch.cuda.synchronize()
    for (F, G, _), (dF, dG) in zip(pairs, dev):
        assert np.array_equal(dF.cpu().numpy(), F) and np.array_equal(dG.cpu().numpy(), G)
    again, _ = hz.tune_batched(dev, cache=cache)
    assert again == best
    st, outs = hz.gsvd_batched(dev, **best)
    assert st == 0
    for (F, G, _), o in zip(pairs[:6], outs[:6]):
        assert max_rel(o["sigma"].cpu().numpy(), oracle.gsvd(F, G)["sigma"]) < SIG_TOL


def test_tune_inner_ordering_and_shortened(tmp_path):
    """inner_ordering = 0 lets the tuner choose the ordering inside a block
    pair (stored in the cache line and returned again on a hit, under a key
    of its own); with qr_shorten = 1 the candidates are timed on the
    shortened pair, and the chosen parameters solve the tall pair to oracle
    parity."""
    import oracle
    hz = _hz()
    F, G, s_true = gi.custom_pair(900, 700, 128, kappa=1e2, seed=62)
    dF, dG = _dev(F), _dev(G)
    cache = str(tmp_path / "tune.txt")
    best, ms = hz.tune(dF, dG, cache=cache, w=16, inner_ordering=0)
    assert best["inner_ordering"] in (hz.HZ_ORD_MM, hz.HZ_ORD_RR, hz.HZ_ORD_RING) and ms > 0
    fields = open(cache).read().split()
    assert len(fields) == 9 and int(fields[8]) == best["inner_ordering"]
    again, _ = hz.tune(dF, dG, cache=cache, w=16, inner_ordering=0)
    assert again == best
    fixed, _ = hz.tune(dF, dG, cache=cache, w=16)          # inner ordering given: own key
    assert fixed["inner_ordering"] == hz.HZ_ORD_RR
    assert len(open(cache).read().splitlines()) == 2
    sbest, sms = hz.tune(dF, dG, cache=cache, qr_shorten=1, inner_ordering=0)
    assert sms > 0 and len(open(cache).read().splitlines()) == 3
    assert np.array_equal(dF.cpu().numpy(), F) and np.array_equal(dG.cpu().numpy(), G)
    r = hz.gsvd(dF, dG, qr_shorten=1, **sbest)
    assert r["status"] == 0
    assert max_rel(r["sigma"].cpu().numpy(), oracle.gsvd(F, G, threads=4)["sigma"]) < SIG_TOL
    assert max_rel(r["sigma"].cpu().numpy(), s_true) < SIG_TOL
