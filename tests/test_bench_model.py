"""The algorithmic work model behind bench.py's roofline figures, on the CPU.

The per-step figures are checked against counts written out by hand from
the kernels' definitions (the Gram reads F and G once and forms the lower
half of a symmetric 2w x 2w block per pivot pair; the update reads and
writes F, G and Z once and multiplies by a 2w x 2w matrix), on the 4096 x
1024 real pair (w = 32: 64 MiB and 0.55 GFLOP for the Gram, 144 MiB and
1.21 GFLOP for the update) and the complex 3072/2048 x 1024 pair (w = 16:
about 2.30 GFLOP and 272 MiB per step)."""

import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_model", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_real_headline_step(bench):
    gram, upd = bench.algorithmic(4096, 4096, 1024, 32)
    pairs, m = 16, 8192
    assert gram["bytes"] == 8 * 1024 * m == 64 * 2 ** 20
    # per pair: 2w (2w + 1) / 2 entries, each a length-m dot product (2 flops a term)
    assert gram["flops"] == pairs * (64 * 65 // 2) * 2 * m
    assert abs(gram["flops"] / 1e9 - 0.545) < 0.001
    assert upd["bytes"] == 2 * 8 * 1024 * (m + 1024) == 144 * 2 ** 20
    # per pair: rows of F, G, Z times a 64 x 64 matrix
    assert upd["flops"] == pairs * (m + 1024) * 64 * 64 * 2
    assert abs(upd["flops"] / 1e9 - 1.208) < 0.001


def test_complex_step(bench):
    gram, upd = bench.algorithmic(3072, 2048, 1024, 16, esz=16, cmul=4)
    f = gram["flops"] + upd["flops"]
    b = gram["bytes"] + upd["bytes"]
    assert abs(f / 1e9 - 2.30) < 0.01
    assert b == (80 + 192) * 2 ** 20


def test_bordering_and_solve_totals(bench):
    assert bench.nw_of(1024, 32) == 1024
    assert bench.nw_of(130, 32) == 192
    assert bench.nw_of(1, 8) == 16
    gram, upd = bench.algorithmic(4096, 4096, 1024, 32)
    f1, b1 = bench.solve_work(4096, 4096, 1024, 32, 1)
    steps = 1024 // 32
    assert f1 == steps * (gram["flops"] + upd["flops"])
    assert b1 == steps * (gram["bytes"] + upd["bytes"])
    # a skipped block update removes one pair's share of a step's update
    f2, b2 = bench.solve_work(4096, 4096, 1024, 32, 1, skipped=3)
    assert f1 - f2 == pytest.approx(3 * upd["flops"] / 16)
    assert b1 - b2 == pytest.approx(3 * upd["bytes"] / 16)
    # 19 sweeps are 19 times one
    f19, b19 = bench.solve_work(4096, 4096, 1024, 32, 19)
    assert f19 == pytest.approx(19 * f1) and b19 == pytest.approx(19 * b1)


def test_roof_fractions(bench):
    r = bench.roof_of(78.6e12, 8.0e12, 1.0)
    assert r["frac_mfma"] == pytest.approx(1.0) and r["frac_hbm"] == pytest.approx(1.0)
    r = bench.roof_of(7.86e12, 4.0e12, 2.0)
    assert r["tflops"] == pytest.approx(3.93) and r["frac_hbm"] == pytest.approx(0.25)
    assert bench.roof_of(1.0, 1.0, 0.0) is None


def test_inner_flops(bench):
    # one launch of 16 pivot pairs of order 64, each running one inner sweep
    # of 63 steps (16 sweeps counted over the pairs), 100 transformations:
    # two Cholesky factorizations per pair, 4 length-64 dot products per
    # column pair and step, and per transformation 6 columns of length 64,
    # each entry one multiply and one multiply-add (3 flops)
    w, pairs = 32, 16
    got = bench.inner_flops(w, 1, 16, 100, pairs, 63)
    chol = pairs * 2 * (2 * 64 ** 3 / 3)
    dots = 16 * 63 * w * (4 * 2 * 64)
    apply = 100 * 6 * 64 * 3
    assert got == pytest.approx(chol + dots + apply)
