"""GPU parity of the batched real FP64 path (hz_dgsvd_batched through the C
ABI): many independent pairs of uneven sizes in one call.

Bar, per pair: generalized singular values within 1e-10 relative of the CPU
oracle's (kappa(X) <= 1e2), the GSVD output contract of the GPU outputs, and
the pair's own status.  The batched kernels run the same device bodies as
the single-pair solver; with one Gram row split (gram_splits = 1) both sum
every Gram entry in the same order, so each pair's batched result must equal
its single-pair result bit for bit -- a check that catches any mixing of one
pair's data, tables or counters with another's.
"""

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


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def _run_batch(pairs, **kw):
    hz = _hz()
    st, outs = hz.gsvd_batched([(_dev(F), _dev(G)) for F, G, *_ in pairs], **kw)
    torch.cuda.synchronize()
    res = [{k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in o.items()}
           for o in outs]
    return st, res


def _run_single(F, G, **kw):
    hz = _hz()
    r = hz.gsvd(_dev(F), _dev(G), **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


def _check(F, G, r):
    return assert_contract(F, G, r["U"], r["V"], r["Z"], r["sigma_f"], r["sigma_g"],
                           r["sigma"], tol_res=1e-12, tol_orth=1e-12)


def _small_batch():
    pairs = gi.make_batch(count=20, seed=11, n_lo=2, n_hi=80)
    rng = np.random.default_rng(12)
    pairs.append((rng.standard_normal((7, 1)), rng.standard_normal((3, 1)), None))   # n = 1
    pairs.append(gi.custom_pair(64, 64, 2, kappa=3.0, seed=13))
    pairs.append(gi.custom_pair(300, 140, 130, kappa=1e2, seed=14))   # several row chunks
    return pairs


@pytest.mark.parametrize("w,lanes,iord", [(8, 0, 2), (16, 0, 2), (16, 4, 2), (8, 0, 3),
                                           (16, 8, 3), (16, 16, 3)])
def test_small_batch_vs_oracle(w, lanes, iord):
    pairs = _small_batch()
    st, res = _run_batch(pairs, w=w, inner_lanes=lanes, inner_ordering=iord)
    assert st == 0, [r["status"] for r in res]
    worst = 0.0
    for i, ((F, G, s_true), r) in enumerate(zip(pairs, res)):
        o = _oracle(F, G, threads=4)
        err = max_rel(r["sigma"], o["sigma"])
        worst = max(worst, err)
        assert r["status"] == 0 and r["converged"], (i, r["status"])
        assert err < SIG_TOL, (i, F.shape, G.shape, err)
        if s_true is not None:
            assert max_rel(r["sigma"], s_true) < 1e-11, i
        _check(F, G, r)
    print(f"w={w}: {len(pairs)} pairs, worst err vs oracle {worst:.2e}")


@pytest.mark.parametrize("w,iord,lanes,sched", [(8, 2, 8, 1), (16, 2, 16, 0), (32, 2, 16, 0),
                                                (16, 3, 16, 0), (32, 3, 8, 0), (16, 3, 8, 1)])
def test_batched_equals_single_pair_bitwise(w, iord, lanes, sched):
    """Every pair of a batch, per-step (sched 1) or persistent (default
    where w is 16 or 32), bitwise equal to the single-pair solver with the
    same block width, ordering and lanes (one Gram split)."""
    pairs = gi.make_batch(count=9, seed=21, n_lo=2, n_hi=100)
    st, res = _run_batch(pairs, w=w, inner_ordering=iord, inner_lanes=lanes, schedule=sched)
    assert st == 0
    for i, ((F, G, _), r) in enumerate(zip(pairs, res)):
        s = _run_single(F, G, w=w, gram_splits=1, inner_ordering=iord, inner_lanes=lanes)
        assert r["sweeps"] == s["sweeps"], (i, r["sweeps"], s["sweeps"])
        assert r["rot_total"] == s["rot_total"] and r["rot_big"] == s["rot_big"], i
        for k in ("sigma", "sigma_f", "sigma_g", "U", "V", "Z"):
            assert np.array_equal(r[k], s[k]), (i, k)


def test_failures_stay_with_their_pair():
    hz = _hz()
    pairs = [list(p) for p in gi.make_batch(count=5, seed=31, n_lo=20, n_hi=60)]
    pairs[2][0][3, 1] = np.nan                         # non-finite input
    pairs[3][1][:, 5] = pairs[3][1][:, 4]              # G rank deficient
    st, res = _run_batch(pairs, w=8)
    assert st == hz.HZ_ENONFINITE
    assert res[2]["status"] == hz.HZ_ENONFINITE
    assert res[3]["status"] == hz.HZ_ECHOL
    for i in (0, 1, 4):
        F, G, _ = pairs[i]
        assert res[i]["status"] == 0
        assert max_rel(res[i]["sigma"], _oracle(F, G)["sigma"]) < SIG_TOL
        _check(F, G, res[i])


def test_persistent_failures_stay_with_their_pair():
    """The persistent schedule: a non-finite pair and a rank-deficient pair
    stop with their own status while the other pairs of the launch converge
    to oracle parity."""
    hz = _hz()
    pairs = [list(p) for p in gi.make_batch(count=6, seed=32, n_lo=40, n_hi=120)]
    pairs[1][0][3, 1] = np.nan
    pairs[4][1][:, 5] = pairs[4][1][:, 4]
    st, res = _run_batch(pairs, w=16, schedule=3)
    assert st == hz.HZ_ENONFINITE
    assert res[1]["status"] == hz.HZ_ENONFINITE
    assert res[4]["status"] == hz.HZ_ECHOL
    for i in (0, 2, 3, 5):
        F, G, _ = pairs[i]
        assert res[i]["status"] == 0 and res[i]["converged"]
        assert max_rel(res[i]["sigma"], _oracle(F, G)["sigma"]) < SIG_TOL
        _check(F, G, res[i])


@pytest.mark.parametrize("w,sched", [(8, 1), (16, 3), (32, 3)])
def test_sweep_cap_per_pair(w, sched):
    hz = _hz()
    pairs = gi.make_batch(count=4, seed=41, n_lo=30, n_hi=60)
    st, res = _run_batch(pairs, w=w, max_sweeps=1, schedule=sched)
    assert st == hz.HZ_ENOCONV
    assert all(r["status"] == hz.HZ_ENOCONV and r["sweeps"] == 1 for r in res)
    st, res = _run_batch(pairs, w=w, max_sweeps=3, schedule=sched)
    assert all(r["sweeps"] == 3 or (r["status"] == 0 and r["sweeps"] < 3) for r in res)


@pytest.mark.parametrize("w,lanes,iord", [(16, 16, 2), (16, 16, 3), (32, 8, 3), (32, 16, 1)])
def test_persistent_equals_per_step_bitwise(w, lanes, iord):
    """One persistent launch for all sweeps gives bitwise the results, the
    sweep counts and the counters of the per-step schedule with its host
    check after every sweep."""
    pairs = gi.make_batch(count=24, seed=23, n_lo=2, n_hi=200)
    kw = dict(w=w, inner_lanes=lanes, inner_ordering=iord)
    st1, a = _run_batch(pairs, schedule=1, **kw)
    st3, b = _run_batch(pairs, schedule=3, **kw)
    assert st1 == st3 == 0
    for i, (ra, rb) in enumerate(zip(a, b)):
        assert ra["sweeps"] == rb["sweeps"], (i, ra["sweeps"], rb["sweeps"])
        assert ra["rot_total"] == rb["rot_total"] and ra["rot_big"] == rb["rot_big"], i
        assert ra["inner_sweeps"] == rb["inner_sweeps"], i
        for k in ("sigma", "sigma_f", "sigma_g", "U", "V", "Z"):
            assert np.array_equal(ra[k], rb[k]), (i, k)


def test_bitwise_reruns():
    pairs = gi.make_batch(count=16, seed=51, n_lo=16, n_hi=128)
    a = _run_batch(pairs)[1]
    b = _run_batch(pairs)[1]
    for ra, rb in zip(a, b):
        for k in ("sigma", "U", "V", "Z"):
            assert np.array_equal(ra[k], rb[k])


def test_full_batch_512_pairs():
    """The 512-pair ensemble (n ~ U{16..256}, m ~ U{n..2n}) with default
    parameters: every pair converges; the contract residuals of every pair
    are computed on the GPU; every pair's sigma is checked against its
    prescribed values, and a sample of pairs (the largest, the smallest and
    four more) against the oracle."""
    hz = _hz()
    pairs = gi.make_batch()
    dev = [(_dev(F), _dev(G)) for F, G, _ in pairs]
    st, outs = hz.gsvd_batched([(F.clone(), G.clone()) for F, G in dev])
    torch.cuda.synchronize()
    assert st == 0, sorted({o["status"] for o in outs})
    worst = dict(fz=0.0, uu=0.0, pyth=0.0, true=0.0)
    for (dF, dG), o, (_, _, s_true) in zip(dev, outs, pairs):
        U, V, Z, sf, sg = o["U"], o["V"], o["Z"], o["sigma_f"], o["sigma_g"]
        n = Z.shape[0]
        fz = torch.linalg.norm(dF @ Z - U * sf) / (torch.linalg.norm(dF) * torch.linalg.norm(Z))
        gz = torch.linalg.norm(dG @ Z - V * sg) / (torch.linalg.norm(dG) * torch.linalg.norm(Z))
        eye = torch.eye(n, dtype=torch.float64, device=U.device)
        uu = torch.linalg.norm(U.T @ U - eye) / n
        vv = torch.linalg.norm(V.T @ V - eye) / n
        worst["fz"] = max(worst["fz"], float(fz), float(gz))
        worst["uu"] = max(worst["uu"], float(uu), float(vv))
        worst["pyth"] = max(worst["pyth"], float(torch.max(torch.abs(sf * sf + sg * sg - 1))))
        worst["true"] = max(worst["true"], max_rel(o["sigma"].cpu().numpy(), s_true))
    print("512 pairs:", {k: f"{v:.2e}" for k, v in worst.items()},
          "sweeps", max(o["sweeps"] for o in outs))
    assert worst["fz"] < 1e-12 and worst["uu"] < 1e-12
    assert worst["pyth"] < 8 * EPS
    assert worst["true"] < 1e-10
    ns = [F.shape[1] for F, _, _ in pairs]
    sample = {int(np.argmax(ns)), int(np.argmin(ns)), 7, 100, 300, 511}
    for i in sorted(sample):
        F, G, _ = pairs[i]
        err = max_rel(outs[i]["sigma"].cpu().numpy(), _oracle(F, G, threads=8)["sigma"])
        assert err < SIG_TOL, (i, err)
