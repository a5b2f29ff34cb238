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
