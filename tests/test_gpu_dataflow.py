"""GPU checks of the dataflow schedule of the real FP64 solver
(HZ_SCHED_DATAFLOW: one persistent launch per sweep, Gram / inner-solve /
update tasks taken from a dependency-ordered queue).  Every task's
arithmetic depends only on its (step, pair, split, tile), so the results
must equal the per-step schedule's bit for bit, sweep counts included; and
they must match the oracle to the parity bar."""

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


def _run(F, G, **kw):
    hz = _hz()
    r = hz.gsvd(torch.from_numpy(np.asfortranarray(F)).cuda(),
                torch.from_numpy(np.asfortranarray(G)).cuda(), **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in r.items()}


SHAPES = [
    # m_f, m_g, n, kappa, gram_splits, update_rows, inner_max_sweeps
    (700, 520, 256, 1e2, 4, 32, 30),
    (333, 200, 130, 30.0, 2, 16, 1),      # ragged: bordering to 192 columns, 3 pairs
    (1024, 900, 512, 1e2, 8, 64, 1),
    (64, 64, 64, 10.0, 1, 16, 30),        # one pair, one chunk
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s[:3])))
def test_dataflow_matches_steps_bitwise_and_oracle(shape):
    import oracle
    hz = _hz()
    m_f, m_g, n, kappa, gs, ur, ims = shape
    F, G, s_true = gi.custom_pair(m_f, m_g, n, kappa=kappa, seed=n + 7)
    kw = dict(w=32, gram_splits=gs, update_rows=ur, inner_max_sweeps=ims)
    a = _run(F, G, schedule=hz.HZ_SCHED_STEPS, **kw)
    b = _run(F, G, schedule=hz.HZ_SCHED_DATAFLOW, **kw)
    print(f"{shape}: sweeps steps={a['sweeps']} dataflow={b['sweeps']} status={b['status']}")
    assert a["status"] == 0 and b["status"] == 0
    assert a["sweeps"] == b["sweeps"] and a["rot_total"] == b["rot_total"]
    for k in ("sigma", "sigma_f", "sigma_g", "U", "V", "Z"):
        assert np.array_equal(a[k], b[k]), k
    o = oracle.gsvd(F, G, threads=4)
    assert max_rel(b["sigma"], o["sigma"]) < SIG_TOL
    assert max_rel(b["sigma"], s_true) < 1e-11
    assert_contract(F, G, b["U"], b["V"], b["Z"], b["sigma_f"], b["sigma_g"], b["sigma"],
                    tol_res=1e-12, tol_orth=1e-12)


def test_dataflow_bitwise_reruns():
    hz = _hz()
    F, G, _ = gi.custom_pair(1500, 1200, 384, kappa=1e2, seed=91)
    kw = dict(w=32, gram_splits=8, update_rows=64, inner_max_sweeps=1,
              schedule=hz.HZ_SCHED_DATAFLOW)
    r1, r2 = _run(F, G, **kw), _run(F, G, **kw)
    for k in ("sigma", "U", "V", "Z"):
        assert np.array_equal(r1[k], r2[k])


def test_dataflow_failure_flags():
    """Columns 0 and 1 of G both equal e_0: their prescale factor is exactly 1,
    their Gram entries exactly 1, so the second Cholesky pivot is exactly 0
    and the inner task must report HZ_ECHOL through the task queue."""
    hz = _hz()
    F, G, _ = gi.custom_pair(300, 300, 128, seed=92)
    G[:, 0] = 0.0
    G[0, 0] = 1.0
    G[:, 1] = G[:, 0]
    with pytest.raises(hz.GsvdError) as e:
        _run(F, G, w=32, schedule=hz.HZ_SCHED_DATAFLOW)
    assert e.value.status == hz.HZ_ECHOL
    assert e.value.info.failed_pair >= 0
