"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/hzgsvd.h, validates arguments before any
device work, and builds orderings with the properties of Section 2.2."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hzgsvd.h")


@pytest.fixture(scope="module")
def hz():
    import paper_1909_00101_amd as hz
    if not os.path.exists(hz.LIB_PATH):
        hz.build()
    return hz


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w \*]*?\b(hz_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("hz_dgsvd", "hz_dgsvd_work_size", "hz_default_params", "hz_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol(hz):
    L = ctypes.CDLL(hz.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_defaults(hz):
    p = hz.params()
    assert (p.variant, p.ordering, p.inner_ordering, p.w) == (0, hz.HZ_ORD_MM, hz.HZ_ORD_RR, 0)
    assert (p.inner_max_sweeps, p.max_sweeps, p.sort) == (30, 30, 1)
    assert p.tol == 0.0 and p.mixed_switch == 1e-5


def test_strerror(hz):
    L = hz.lib()
    assert L.hz_strerror(0) == b"success"
    assert b"positive definite" in L.hz_strerror(2)
    assert L.hz_strerror(-3) == b"invalid argument"
    assert L.hz_version().startswith(b"hzgsvd")


def _call(hz, p, m_f, m_g, n, F=8, ldf=None, G=8, ldg=None, Z=8, ldz=None, s=8, sf=8, sg=8,
          work=None, wb=0):
    L = hz.lib()
    v = ctypes.c_void_p
    return L.hz_dgsvd(ctypes.byref(p) if p is not None else None, m_f, m_g, n,
                      v(F), ldf if ldf is not None else m_f, v(G), ldg if ldg is not None else m_g,
                      v(Z), ldz if ldz is not None else n, v(s), v(sf), v(sg), v(work), wb,
                      None, None)


@pytest.mark.parametrize("case,expect", [
    (dict(m_f=0, m_g=5, n=1), -2), (dict(m_f=5, m_g=0, n=1), -3),
    (dict(m_f=3, m_g=5, n=4), -4), (dict(m_f=5, m_g=3, n=4), -4), (dict(m_f=5, m_g=5, n=0), -4),
    (dict(m_f=5, m_g=5, n=2, F=0), -5), (dict(m_f=5, m_g=5, n=2, F=12), -5),
    (dict(m_f=5, m_g=5, n=2, ldf=4), -6), (dict(m_f=5, m_g=5, n=2, G=0), -7),
    (dict(m_f=5, m_g=5, n=2, ldg=2), -8), (dict(m_f=5, m_g=5, n=2, Z=0), -9),
    (dict(m_f=5, m_g=5, n=2, ldz=1), -10), (dict(m_f=5, m_g=5, n=2, s=0), -11),
    (dict(m_f=5, m_g=5, n=2, sf=0), -12), (dict(m_f=5, m_g=5, n=2, sg=4), -13),
    (dict(m_f=5, m_g=5, n=2, work=264), -14),
    (dict(m_f=500, m_g=500, n=200, work=256, wb=100), -15),
])
def test_argument_validation_before_device_work(hz, case, expect):
    # Every rejection happens on the host before any HIP call, so these run
    # without a GPU.
    assert _call(hz, hz.params(), **case) == expect


def test_bad_params_rejected(hz):
    for kw in (dict(variant=2), dict(variant=3), dict(w=12), dict(ordering=7),
               dict(inner_max_sweeps=0),
               dict(max_sweeps=0), dict(inner_ordering=0)):
        assert _call(hz, hz.params(**kw), 64, 64, 32) == -1


def test_work_size(hz):
    L = hz.lib()
    p = hz.params(w=32)
    a = L.hz_dgsvd_work_size(ctypes.byref(p), 4096, 4096, 1024)
    # at least the working copies of F, G, Z
    assert a >= 8 * (4096 * 1024 * 2 + 1024 * 1024)
    assert a < 2 * 8 * (4096 * 1024 * 2 + 1024 * 1024)
    assert L.hz_dgsvd_work_size(ctypes.byref(p), 10, 10, 11) == 0
    assert L.hz_dgsvd_work_size(None, 10, 10, 1) > 0


def _table(hz, kind, N):
    L = hz.lib()
    steps = L.hz_ordering(kind, N, None)
    t = (ctypes.c_int * (steps * N))()
    assert L.hz_ordering(kind, N, t) == steps
    return np.array(t).reshape(steps, N // 2, 2)


@pytest.mark.parametrize("N", [2, 4, 8, 16, 32, 64, 128])
def test_library_orderings(hz, N):
    mm = _table(hz, hz.HZ_ORD_MM, N)
    rr = _table(hz, hz.HZ_ORD_RR, N)
    assert mm.shape[0] == N and rr.shape[0] == N - 1
    for t, cyclic in ((mm, False), (rr, True)):
        seen = {}
        for step in t:
            assert sorted(step.reshape(-1).tolist()) == list(range(N))
            for p, q in step:
                assert p < q
                seen[(p, q)] = seen.get((p, q), 0) + 1
        assert len(seen) == N * (N - 1) // 2
        if cyclic:
            assert all(c == 1 for c in seen.values())
    assert hz.lib().hz_ordering(hz.HZ_ORD_MM, 7, None) == -1
    assert hz.lib().hz_ordering(5, 8, None) == -1


@pytest.mark.parametrize("N,lanes", [(16, 8), (32, 4), (32, 8), (32, 16), (64, 4), (64, 8),
                                     (64, 16)])
def test_ring_ordering(hz, N, lanes):
    """The inner solver's ring ordering: N - 1 steps of N/2 disjoint pairs
    (i < j) covering every pair once (a cyclic parallel ordering); within a
    level a lane group keeps its first column; and the schedule is free of
    races: where the solver does not synchronise its workgroup after a
    step, every column a group touches in the next step was last touched by
    a group of the same wave."""
    L = hz.lib()
    steps = L.hz_ring_ordering(N, lanes, None, None)
    assert steps == N - 1
    t = (ctypes.c_int * (steps * N))()
    sy = (ctypes.c_int * steps)()
    assert L.hz_ring_ordering(N, lanes, t, sy) == steps
    tab = np.array(t).reshape(steps, N // 2, 2)
    sync = list(sy)
    seen = set()
    for step in tab:
        assert sorted(step.reshape(-1).tolist()) == list(range(N))
        for i, j in step:
            assert i < j and (i, j) not in seen
            seen.add((i, j))
    assert len(seen) == N * (N - 1) // 2
    gw = 64 // lanes
    last = {}                      # column -> (wave of the group that last touched it, synced since)
    for k, step in enumerate(tab):
        for g, (i, j) in enumerate(step):
            for c in (i, j):
                if c in last:
                    wave, synced = last[c]
                    assert synced or wave == g // gw, (k, g, c)
        for g, (i, j) in enumerate(step):
            last[i] = (g // gw, False)
            last[j] = (g // gw, False)
        if sync[k]:
            last = {c: (wv, True) for c, (wv, _) in last.items()}
    assert sync[-1] == 1
    # the first column of a group stays for a whole level (levels of N/2, N/4, ... steps)
    k0, h = 0, N // 2
    while h >= 1:
        for g in range(N // 2):
            assert len({int(tab[k, g, 0]) for k in range(k0, k0 + h)}) == 1
        k0, h = k0 + h, h // 2
    assert L.hz_ring_ordering(48, 8, None, None) == -1
    assert L.hz_ring_ordering(16, 2, None, None) == -1


def test_product_path_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_1909_00101_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "hz_oracle" not in src, f
                assert "oracle/" not in src, f


def _bcall(hz, batch, mf, mg, n, ptr=8, ld=None, arrays=None, work=None, wb=0):
    """hz_dgsvd_batched with fake (aligned, never dereferenced) device
    pointers: only argument checks run, so no GPU is touched."""
    L = hz.lib()
    p = hz.params()
    i64 = lambda v: (ctypes.c_int64 * len(v))(*v) if v is not None else None
    pv = lambda: (ctypes.c_void_p * max(batch, 1))(*([ptr] * max(batch, 1)))
    a = dict(mf=i64(mf), mg=i64(mg), n=i64(n), F=pv(), ldf=i64(ld or mf), G=pv(),
             ldg=i64(ld or mg), Z=pv(), ldz=i64(ld or n), s=pv(), sf=pv(), sg=pv())
    if arrays:
        a.update(arrays)
    return L.hz_dgsvd_batched(ctypes.byref(p), batch, a["mf"], a["mg"], a["n"], a["F"],
                              a["ldf"], a["G"], a["ldg"], a["Z"], a["ldz"], a["s"], a["sf"],
                              a["sg"], work, wb, None, None)


def test_batched_argument_validation(hz):
    assert _bcall(hz, -1, [4], [4], [2]) == -2
    assert _bcall(hz, 70000, [4], [4], [2]) == -2
    assert _bcall(hz, 0, [4], [4], [2]) == 0          # empty batch: nothing to do
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], arrays=dict(mf=None)) == -3
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], arrays=dict(n=None)) == -5
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], arrays=dict(G=None)) == -8
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], arrays=dict(sg=None)) == -14
    # per-pair checks take the single-pair argument index + 1
    assert _bcall(hz, 2, [4, 0], [4, 4], [2, 2]) == -3     # m_f < 1
    assert _bcall(hz, 2, [4, 4], [4, 1], [2, 2]) == -5     # n > m_g
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], ptr=12) == -6   # misaligned F
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], arrays=dict(
        ldz=(ctypes.c_int64 * 2)(2, 1))) == -11
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], work=ctypes.c_void_p(8)) == -15
    assert _bcall(hz, 2, [4, 4], [4, 4], [2, 2], work=ctypes.c_void_p(256), wb=16) == -16


def test_batched_work_size(hz):
    L = hz.lib()
    i64 = lambda v: (ctypes.c_int64 * len(v))(*v)
    p = hz.params()
    one = [L.hz_dgsvd_work_size(ctypes.byref(hz.params(w=16)), m, g, k)
           for m, g, k in ((300, 256, 200), (90, 60, 40))]
    both = L.hz_dgsvd_batched_work_size(ctypes.byref(p), 2, i64([300, 90]), i64([256, 60]),
                                        i64([200, 40]))
    assert both > 0 and both % 256 == 0
    # at least the working copies of both pairs
    assert both > 8 * (320 + 256 + 256) * 224
    assert L.hz_dgsvd_batched_work_size(ctypes.byref(p), 1, i64([3]), i64([3]), i64([4])) == 0
    assert L.hz_dgsvd_batched_work_size(ctypes.byref(p), 0, None, None, None) == 256
    assert min(one) > 0


def test_tuner_argument_validation(hz):
    L = hz.lib()
    p = hz.params()
    best = hz.HzParams()
    v = ctypes.c_void_p(8)
    assert L.hz_dgsvd_tune(ctypes.byref(p), 0, 4, 2, v, 4, v, 4, None, ctypes.byref(best),
                           None, None) == -2
    assert L.hz_dgsvd_tune(ctypes.byref(p), 4, 4, 5, v, 4, v, 4, None, ctypes.byref(best),
                           None, None) == -4
    assert L.hz_dgsvd_tune(ctypes.byref(p), 4, 4, 2, v, 4, v, 4, None, None, None, None) == -10
    bad = hz.params(w=12)
    assert L.hz_dgsvd_tune(ctypes.byref(bad), 4, 4, 2, v, 4, v, 4, None, ctypes.byref(best),
                           None, None) == -1
    i64 = lambda vals: (ctypes.c_int64 * len(vals))(*vals)
    pv = (ctypes.c_void_p * 1)(8)
    assert L.hz_dgsvd_batched_tune(ctypes.byref(p), 0, i64([4]), i64([4]), i64([2]), pv,
                                   i64([4]), pv, i64([4]), None, ctypes.byref(best), None,
                                   None) == -2
    assert L.hz_dgsvd_batched_tune(ctypes.byref(p), 1, i64([4]), i64([4]), i64([2]), pv,
                                   i64([3]), pv, i64([4]), None, ctypes.byref(best), None,
                                   None) == -7
    assert L.hz_dgsvd_batched_tune(ctypes.byref(p), 1, i64([4]), i64([4]), i64([2]), pv,
                                   i64([4]), pv, i64([4]), None, None, None, None) == -11


@pytest.mark.parametrize("shape", [(4096, 4096, 1024, 8, 64), (700, 520, 256, 4, 32),
                                   (333, 200, 130, 2, 16), (64, 64, 64, 1, 16)],
                         ids=lambda s: "x".join(map(str, s[:3])))
def test_dataflow_task_list_is_a_dependency_order(hz, shape):
    """The persistent sweep kernel takes tasks in list order and waits for
    their inputs; it can only drain if every task comes after everything it
    waits for.  Checks that, that every task appears once, and that the
    parents of a pair are the previous step's pairs holding its blocks."""
    m_f, m_g, n, splits, urows = shape
    L = hz.lib()
    L.hz_dataflow_tasks.argtypes = [ctypes.POINTER(hz.HzParams), ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]
    p = hz.params(w=32, gram_splits=splits, update_rows=urows)
    info = np.zeros(4, dtype=np.int32)
    nt = L.hz_dataflow_tasks(ctypes.byref(p), m_f, m_g, n, None, None, info.ctypes.data)
    steps, npairs, S, T = (int(v) for v in info)
    assert nt == steps * npairs * (2 * S + 1 + T)
    tasks = np.zeros((nt, 4), dtype=np.int32)
    par = np.zeros((steps * npairs, 2), dtype=np.int32)
    assert L.hz_dataflow_tasks(ctypes.byref(p), m_f, m_g, n, tasks.ctypes.data,
                               par.ctypes.data, None) == nt
    seen = {}
    for i, (kind, k, l, sub) in enumerate(tasks.tolist()):
        key = (kind, k, l, sub)
        assert key not in seen
        seen[key] = i
    assert len(seen) == nt
    nblk = 2 * npairs
    tab = np.zeros(steps * npairs * 2, dtype=np.int32)
    L.hz_ordering(hz.HZ_ORD_MM, nblk, tab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    tab = tab.reshape(steps, npairs, 2)
    for k in range(1, steps):
        for l in range(npairs):
            a, b = par[k * npairs + l]
            assert set(tab[k, l]) <= set(tab[k - 1, a]) | set(tab[k - 1, b])
            assert tab[k, l, 0] in tab[k - 1, a] and tab[k, l, 1] in tab[k - 1, b]
    for (kind, k, l, sub), i in seen.items():
        if kind == 0 and k > 0:
            for q in par[k * npairs + l]:
                for t in range(T):
                    assert seen[(2, k - 1, int(q), t)] < i
        elif kind == 1:
            for s_ in range(2 * S):
                assert seen[(0, k, l, s_)] < i
        elif kind == 2:
            assert seen[(1, k, l, 0)] < i


def test_qr_shorten_sizes_and_rejections(hz):
    """The shortened solve needs Q_F, Q_G and the square solve's workspace;
    the real, complex and mixed solvers take it; the batched entry points,
    and n beyond the pivoted Cholesky's limit (also in the tuner), reject
    it, all on the host."""
    L = hz.lib()
    p = hz.params(w=32, qr_shorten=1)
    plain = L.hz_dgsvd_work_size(ctypes.byref(hz.params(w=32)), 1024, 1024, 1024)
    a = L.hz_dgsvd_work_size(ctypes.byref(p), 4096, 4096, 1024)
    assert a >= plain + 8 * 2 * 4096 * 1024
    assert L.hz_zgsvd_work_size(ctypes.byref(hz.params(w=16, qr_shorten=1)), 3072, 2048,
                                1024) > 16 * (3072 + 2048) * 1024
    assert L.hz_dgsvd_mixed_work_size(ctypes.byref(p), 4096, 4096, 1024) > a
    assert L.hz_dgsvd_work_size(ctypes.byref(p), 9000, 9000, 8193) == 0
    assert L.hz_dgsvd_work_size(ctypes.byref(hz.params(qr_shorten=2)), 64, 64, 32) == 0
    v = ctypes.c_void_p(256)
    assert _call(hz, hz.params(qr_shorten=2), 64, 64, 32) == -1
    assert _call(hz, p, 500, 500, 200, work=256, wb=a // 1000) == -15
    i64 = lambda vals: (ctypes.c_int64 * len(vals))(*vals)
    assert L.hz_dgsvd_batched_work_size(ctypes.byref(p), 1, i64([64]), i64([64]),
                                        i64([32])) == 0
    best = hz.HzParams()
    assert L.hz_dgsvd_tune(ctypes.byref(hz.params(qr_shorten=1)), 9000, 9000, 8193, v, 9000, v,
                           9000, None, ctypes.byref(best), None, None) == -1


def test_enhanced_variants_accepted(hz):
    """Variants 1 and 5 (enhanced dot products) are accepted by the real,
    mixed and complex solvers; variants 2, 3, 6, 7 are not built."""
    L = hz.lib()
    for variant in (1, 5):
        p = hz.params(variant=variant)
        assert L.hz_dgsvd_work_size(ctypes.byref(p), 64, 64, 32) > 0
        assert L.hz_dgsvd_mixed_work_size(ctypes.byref(p), 64, 64, 32) > 0
        assert L.hz_zgsvd_work_size(ctypes.byref(p), 64, 64, 32) > 0
    for variant in (2, 3, 6, 7):
        assert L.hz_zgsvd_work_size(ctypes.byref(hz.params(variant=variant)), 64, 64, 32) == 0


def test_pivot_qr_sizes_and_rejections(hz):
    """QR pivot factors (pivot_qr = 1) belong to the real and complex solvers
    with the per-step schedule: more workspace there (the QR tree levels);
    rejected on the host by the mixed and batched solvers and with the
    dataflow schedule."""
    L = hz.lib()
    v = ctypes.c_void_p(256)
    p = hz.params(pivot_qr=1, w=32)
    plain = L.hz_dgsvd_work_size(ctypes.byref(hz.params(w=32)), 4096, 4096, 1024)
    assert L.hz_dgsvd_work_size(ctypes.byref(p), 4096, 4096, 1024) > plain
    assert L.hz_zgsvd_work_size(ctypes.byref(hz.params(pivot_qr=1)), 64, 64, 32) > \
        L.hz_zgsvd_work_size(ctypes.byref(hz.params()), 64, 64, 32)
    assert L.hz_dgsvd_mixed_work_size(ctypes.byref(p), 64, 64, 32) == 0
    assert L.hz_dgsvd_work_size(ctypes.byref(hz.params(pivot_qr=1, w=32,
                                                       schedule=hz.HZ_SCHED_DATAFLOW)),
                                64, 64, 64) == 0
    assert L.hz_dgsvd_work_size(ctypes.byref(hz.params(pivot_qr=2)), 64, 64, 32) == 0
    assert L.hz_dgsvd_mixed(ctypes.byref(hz.params(pivot_qr=1)), 64, 64, 32, v, 64, v, 64, v,
                            32, v, v, v, None, 0, None, None) == -1
    i64 = lambda vals: (ctypes.c_int64 * len(vals))(*vals)
    assert L.hz_dgsvd_batched_work_size(ctypes.byref(p), 1, i64([64]), i64([64]),
                                        i64([32])) == 0


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 (or a WORLD_SIZE above 1)
    exits with a message before touching a device."""
    import subprocess
    import sys
    bench = os.path.join(ROOT, "bench.py")
    for args, env in (([bench, "--gpus", "2"], {}), ([bench], {"WORLD_SIZE": "2"})):
        e = dict(os.environ)
        e.update(env)
        r = subprocess.run([sys.executable, *args], capture_output=True, text=True, env=e,
                           timeout=120)
        assert r.returncode == 2, (r.returncode, r.stderr[-500:])
        assert "one GPU" in r.stderr


def test_product_path_fails_loudly_without_library():
    """With the HIP library absent, the binding raises instead of computing
    anything on the CPU (there is no fallback path)."""
    import subprocess
    import sys
    code = f"""
import sys
sys.path.insert(0, {ROOT!r})
import torch
import paper_1909_00101_amd as hz
hz.LIB_PATH = '/nonexistent/libhzgsvd.so'
hz._lib = None
try:
    hz.lib()
    print('LOADED')
except RuntimeError as e:
    print('lib raised')
F = torch.randn(8, 4, dtype=torch.float64)
G = torch.randn(8, 4, dtype=torch.float64)
try:
    hz.gsvd(F, G)
    print('RESULT')
except Exception as e:
    print('gsvd raised', type(e).__name__)
"""
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-800:]
    assert "lib raised" in r.stdout and "gsvd raised" in r.stdout, r.stdout
    assert "LOADED" not in r.stdout and "RESULT" not in r.stdout, r.stdout


def test_caller_workspace_is_used_only_when_aligned_space_suffices():
    """A caller workspace whose start is not 256-byte aligned loses up to 255
    bytes to the alignment: the binding must not hand the library a buffer
    shorter than the solve needs, and must tell it the usable size."""
    import torch
    import paper_1909_00101_amd as hz
    assert hz.aligned_span(256, 1000) == (256, 1000)
    assert hz.aligned_span(264, 1000) == (512, 752)
    assert hz.aligned_span(264, 100) == (512, 0)
    need = 4096
    base = torch.empty(need + 1024, dtype=torch.uint8)
    off = (-base.data_ptr()) % 256          # first 256-byte boundary inside base
    aligned = base[off:off + need]
    wptr, avail, keep = hz._workspace(aligned, need, "cpu")
    assert keep is aligned and wptr == aligned.data_ptr() and avail == need
    misaligned = base[off + 8:off + 8 + need]   # exactly `need` bytes, 8 past a boundary
    wptr, avail, keep = hz._workspace(misaligned, need, "cpu")
    assert keep is not misaligned and wptr % 256 == 0 and avail >= need
    assert wptr >= keep.data_ptr() and wptr + need <= keep.data_ptr() + keep.numel()
    roomy = base[off + 8:]                  # room to spare after aligning
    wptr, avail, keep = hz._workspace(roomy, need, "cpu")
    assert keep is roomy and wptr % 256 == 0
    assert wptr + avail == roomy.data_ptr() + roomy.numel() and avail >= need
