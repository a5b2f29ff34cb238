#!/usr/bin/env python3
"""Benchmark of the blocked one-sided implicit Hari-Zimmermann GSVD on MI355X.

Workload: the seeded real FP64 pair F, G of 4096 x 1024 (kappa(X) = 1e2,
generalized singular values log-uniform in [1e-3, 1e3]), block width w = 32,
modified-modulus outer ordering, relative-orthogonality threshold 1024 eps.
A step is one complete GSVD solve of that pair (prescale, sweeps of block
steps to convergence, extraction and sort), inputs resident in HBM; before
each solve the pair is restored from pristine device copies (two 32 MiB
device-to-device copies, inside the timed region, <0.1% of a solve).

Prints one JSON line: solves/s, the measured per-kernel split, the roofline
entry of the dominant kernel (algorithmic bytes or flops per launch over its
average launch time, measured with HIP events on the solve's stream) and the
CPU oracle timed on a bounded sample on the host.  Unless --no-forms is
given, the line also carries the mixed-precision form against plain FP64 on
the 8192 x 2048 pair and the batched form against a loop of single-pair
solves on the 512-pair ensemble (wall time of each, same parameters, with
the accuracy each reaches).
"""

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
METRIC = "GSVD solves/s + FP64 MFMA util, 4096x1024 pair; mixed/batched vs plain"


def algorithmic(m_f, m_g, n, w):
    """Algorithmic work per launch of each block-step kernel (one step =
    n/(2w) pivot pairs).  Gram: reads all of F and G once, 8 n (m_F+m_G)
    bytes; 2w(2w+1)(m_F+m_G) flops per pair using symmetry.  Update: reads
    and writes all of F, G, Z, 16 n (m_F+m_G+n) bytes; 2 (2w)^2 (m_F+m_G+n)
    flops per pair."""
    pairs = n // (2 * w)
    gram = dict(bytes=8.0 * n * (m_f + m_g), flops=pairs * 2.0 * w * (2 * w + 1) * (m_f + m_g))
    upd = dict(bytes=16.0 * n * (m_f + m_g + n),
               flops=pairs * 2.0 * (2 * w) ** 2 * (m_f + m_g + n))
    return gram, upd


def inner_flops(w, launches, inner_sweeps, rotations, npairs, isteps):
    """Algorithmic FP64 work of the inner solver per launch (one step of
    n/(2w) pivot pairs): two Cholesky factorizations of order 2w,
    (2w)^3/3 multiply-adds each; per inner sweep ``isteps`` steps (2w - 1
    for round robin, 2w for modified modulus) of w column pairs, each forming
    4 dot products of length 2w (16w flops); per applied transformation 6
    columns of length 2w updated (36w flops)."""
    W2 = 2 * w
    chol = npairs * launches * 2.0 * (2.0 * W2 ** 3 / 3.0)
    dots = inner_sweeps * isteps * w * 16.0 * w
    apply = rotations * 36.0 * w
    return (chol + dots + apply) / max(1, launches)


def cpu_baseline(F, G, tol, golden_sweeps):
    """Time one sweep of the CPU oracle (modified-modulus ordering, OpenMP over
    the disjoint pairs of each step, all host threads) on the same pair, and
    scale by the oracle's sweep count for this pair to solves/s."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    r = oracle.gsvd(F, G, ordering=oracle.ORD_MM, tol=tol, max_sweeps=1, threads=threads)
    dt = time.perf_counter() - t0
    sweeps = golden_sweeps
    return dict(value=1.0 / (dt * sweeps), unit="solves/s", cores=threads, kind="oracle",
                sample=f"one full sweep ({r['rot_all']} pointwise steps) of the unblocked "
                       f"oracle on the 4096x1024 pair took {dt:.2f} s on {threads} threads; "
                       f"scaled by the {sweeps} sweeps the oracle needs on this pair")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gsvd_real_4096x1024_w32_bo_traffic.txt")
KERNEL_SOURCES = ["paper_1909_00101_amd/csrc/hz_real.hip", "paper_1909_00101_amd/csrc/hz_kernels_real.h",
                  "paper_1909_00101_amd/csrc/hz_device.h"]


def measured_traffic():
    """HBM bytes per dispatch of each kernel of the 4096x1024 workload, from
    the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (each counter
    scaled by its reading for a 32 MiB device copy).  Empty when the kernel
    sources have changed since the counters were taken."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read()
                                for f in KERNEL_SOURCES)).hexdigest()[:16]
    out, sha = {}, None
    for line in open(TRAFFIC_FILE):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        if t[0] == "source_sha":
            sha = t[1]
        elif len(t) == 7:
            out[t[0]] = (float(t[5]) + float(t[6])) * 2.0 ** 20
    return out if sha == h else {}


def _timed(fn, reps):
    import torch
    best, out = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return best, out


def mixed_vs_plain(reps=2):
    """hz_dgsvd_mixed against hz_dgsvd on the seeded 8192 x 2048 pair (w = 32,
    one inner sweep, tol = n eps, the same launch parameters for both, the
    switch to FP64 at the default off-diagonal measure 1e-5), and both again
    on the QR-shortened pair (qr_shorten = 1); all restore the pair from
    device copies inside the timed call (two 128 MiB copies)."""
    import torch
    import gsvd_inputs as gi
    import paper_1909_00101_amd as hz
    spec = gi.CONFIGS[4]
    F, G, s_true = gi.config_pair(4)
    dev = torch.device("cuda:0")
    F0, G0 = torch.from_numpy(F).to(dev), torch.from_numpy(G).to(dev)
    Fw, Gw = F0.clone(), G0.clone()
    kw = dict(w=32, inner_max_sweeps=1, tol=spec.n * np.finfo(np.float64).eps, gram_splits=8,
              update_rows=64)
    res = {}
    for name, mixed, short in (("plain", False, 0), ("mixed", True, 0),
                               ("plain_shortened", False, 1), ("mixed_shortened", True, 1)):
        def run():
            Fw.copy_(F0)
            Gw.copy_(G0)
            return hz.gsvd(Fw, Gw, overwrite=True, mixed=mixed, qr_shorten=short, **kw)
        run()
        dt, r = _timed(run, reps)
        err = float(np.max(np.abs(r["sigma"].cpu().numpy() - s_true) / s_true))
        res[name] = dict(ms=round(dt * 1e3, 2), sweeps_fp64=r["sweeps"],
                         sweeps_fp32=r["sweeps_fp32"], max_rel_sigma_err=err, status=r["status"])
    del F0, G0, Fw, Gw
    torch.cuda.empty_cache()
    return dict(workload=f"seeded {spec.m_f}x{spec.n} real pair, kappa(X)=1e2, w=32, "
                         f"one inner sweep, tol=n*eps, 8 Gram splits, 64 update rows per wave",
                speedup=round(res["plain"]["ms"] / res["mixed"]["ms"], 3),
                speedup_shortened=round(res["plain"]["ms"] / res["plain_shortened"]["ms"], 3),
                speedup_mixed_shortened=round(res["plain"]["ms"] / res["mixed_shortened"]["ms"], 3),
                **res)


def complex_shortened_vs_plain(reps=2):
    """hz_zgsvd on the seeded complex 3072x1024 / 2048x1024 pair (kappa(X) =
    50, w = 16, modified-modulus outer and inner orderings, one inner sweep,
    tol = n eps) plain and QR-shortened; both restore the pair from device
    copies inside the timed call."""
    import torch
    import gsvd_inputs as gi
    import paper_1909_00101_amd as hz
    spec = gi.CONFIGS[3]
    F, G, s_true = gi.config_pair(3)
    dev = torch.device("cuda:0")
    F0, G0 = torch.from_numpy(F).to(dev), torch.from_numpy(G).to(dev)
    Fw, Gw = F0.clone(), G0.clone()
    kw = dict(w=16, ordering=hz.HZ_ORD_MM, inner_ordering=hz.HZ_ORD_MM, inner_max_sweeps=1,
              tol=spec.n * np.finfo(np.float64).eps)
    res = {}
    for name, short in (("plain", 0), ("shortened", 1)):
        def run():
            Fw.copy_(F0)
            Gw.copy_(G0)
            return hz.gsvd(Fw, Gw, overwrite=True, qr_shorten=short, **kw)
        run()
        dt, r = _timed(run, reps)
        err = float(np.max(np.abs(r["sigma"].cpu().numpy() - s_true) / s_true))
        res[name] = dict(ms=round(dt * 1e3, 2), sweeps=r["sweeps"], max_rel_sigma_err=err,
                         status=r["status"])
    del F0, G0, Fw, Gw
    torch.cuda.empty_cache()
    return dict(workload=f"seeded complex {spec.m_f}x{spec.n} / {spec.m_g}x{spec.n} pair, "
                         "kappa(X)=50, w=16, MM outer and inner orderings, one inner sweep, "
                         "tol=n*eps",
                speedup=round(res["plain"]["ms"] / res["shortened"]["ms"], 3), **res)


def batched_vs_plain(tune_cache=None, reps=3):
    """hz_dgsvd_batched on the 512-pair ensemble (n ~ U{16..256}, m ~ U{n..2n})
    against hz_dgsvd called on each pair in turn, both with the parameters
    the batched autotuner picks (or its defaults with one inner sweep); the
    pairs are restored from device copies in both."""
    import torch
    import gsvd_inputs as gi
    import paper_1909_00101_amd as hz
    pairs = gi.make_batch()
    dev = torch.device("cuda:0")
    D = [(torch.from_numpy(F).to(dev), torch.from_numpy(G).to(dev)) for F, G, _ in pairs]
    W = [(F.clone(), G.clone()) for F, G in D]
    S = [s for _, _, s in pairs]
    kw = dict(inner_max_sweeps=1)
    if tune_cache is not None:
        kw, _ = hz.tune_batched(D, cache=tune_cache)

    def restore():
        for (f0, g0), (f, g) in zip(D, W):
            f.copy_(f0)
            g.copy_(g0)

    def batched():
        restore()
        return hz.gsvd_batched(W, overwrite=True, **kw)

    def loop():
        restore()
        return [hz.gsvd(f, g, overwrite=True, **kw) for f, g in W]

    batched()
    tb, (st, outs) = _timed(batched, reps)
    eb = max(float(np.max(np.abs(o["sigma"].cpu().numpy() - s) / s)) for o, s in zip(outs, S))
    tl, louts = _timed(loop, 1)
    el = max(float(np.max(np.abs(o["sigma"].cpu().numpy() - s) / s)) for o, s in zip(louts, S))
    return dict(workload="512 seeded real pairs, n~U{16..256}, m_F,m_G~U{n..2n}, "
                         "kappa log-uniform in [1,1e2]", params=kw,
                batched_ms=round(tb * 1e3, 2), loop_ms=round(tl * 1e3, 2),
                speedup=round(tl / tb, 2), pairs_per_s=round(len(pairs) / tb, 1),
                status=st, max_sweeps=max(o["sweeps"] for o in outs),
                max_rel_sigma_err_batched=eb, max_rel_sigma_err_loop=el)


def qr_shortened_vs_plain(F0, G0, s_true, tol, plain_kw, tune_cache=None, reps=3):
    """The QR-shortened solve (hz_dgsvd with qr_shorten = 1: pivoted QR of F
    and G, sweeps on the square pair (R_F P2, R_G), then U = Q_F U'',
    V = Q_G V'', Z = P1 P2 Z'') against the plain solve of the headline pair,
    both timed here the same way (restore from device copies plus solve,
    fastest of ``reps``).  The plain solve uses the headline's parameters;
    the shortened one the autotuner's choice for the square pair (block
    width free), or w = 16 with one inner sweep without the tuner."""
    import torch
    import paper_1909_00101_amd as hz
    Fw, Gw = F0.clone(), G0.clone()
    skw = dict(w=16, inner_max_sweeps=1)
    if tune_cache is not None:
        skw, _ = hz.tune(F0, G0, cache=tune_cache, ordering=hz.HZ_ORD_MM, tol=tol, qr_shorten=1,
                         inner_ordering=0)
    skw = dict(skw, ordering=hz.HZ_ORD_MM, tol=tol, qr_shorten=1)
    res = {}
    for name, kw in (("plain", plain_kw), ("shortened", skw)):
        def run():
            Fw.copy_(F0)
            Gw.copy_(G0)
            return hz.gsvd(Fw, Gw, overwrite=True, **kw)
        run()
        dt, r = _timed(run, reps)
        err = float(np.max(np.abs(r["sigma"].cpu().numpy() - s_true) / s_true))
        res[name] = dict(ms=round(dt * 1e3, 2), sweeps=r["sweeps"], max_rel_sigma_err=err,
                         status=r["status"],
                         params={k: kw[k] for k in ("w", "inner_ordering", "inner_max_sweeps",
                                                    "inner_lanes", "gram_splits", "update_rows")
                                 if k in kw})
    del Fw, Gw
    torch.cuda.empty_cache()
    return dict(workload="the headline pair (seeded 4096x1024, kappa(X)=1e2), MM ordering, "
                         "tol=1024*eps", speedup=round(res["plain"]["ms"] / res["shortened"]["ms"], 3),
                **res)


def transfer_inclusive(F, G, Fw, Gw, work, kw, reps=3):
    """Solves timed with the host transfers the paper's timings include: F and
    G copied from pinned host memory into the device buffers, the solve, and
    U, V, Z, sigma, sigma_F, sigma_G copied back into pinned host memory."""
    import torch
    import paper_1909_00101_amd as hz

    def pinned_like(t):
        return torch.empty_strided(t.size(), t.stride(), dtype=t.dtype, pin_memory=True)

    Fh, Gh = pinned_like(Fw), pinned_like(Gw)
    Fh.copy_(torch.from_numpy(F))
    Gh.copy_(torch.from_numpy(G))
    keys = ("U", "V", "Z", "sigma", "sigma_f", "sigma_g")
    out_h = None

    def run():
        nonlocal out_h
        Fw.copy_(Fh, non_blocking=True)
        Gw.copy_(Gh, non_blocking=True)
        r = hz.gsvd(Fw, Gw, overwrite=True, workspace=work, **kw)
        if out_h is None:
            out_h = {k: pinned_like(r[k]) for k in keys}
        for k in keys:
            out_h[k].copy_(r[k], non_blocking=True)
        return r

    run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ms = float(np.median(ts)) * 1e3
    h2d = (Fh.numel() + Gh.numel()) * 8
    d2h = sum(t.numel() * t.element_size() for t in out_h.values())
    return dict(ms=round(ms, 2), solves_per_s=round(1e3 / ms, 3), reps=reps,
                h2d_MiB=round(h2d / 2**20, 1), d2h_MiB=round(d2h / 2**20, 1),
                note="pinned host buffers; not the headline value, which has the pair "
                     "resident in HBM")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--w", type=int, default=32)
    ap.add_argument("--inner-max-sweeps", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the QR-shortened, mixed-precision, complex and batched comparisons")
    ap.add_argument("--only-form", choices=("qr_shortened", "mixed", "complex", "batched"),
                    help="run only this comparison and print its JSON (for profiling)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use --w/--inner-max-sweeps and library defaults, no autotuner")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1909_00101_amd",
                                                         "tune_cache.txt"),
                    help="autotuner cache file (read, and appended to on a miss)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import gsvd_inputs as gi
    import paper_1909_00101_amd as hz

    spec = gi.CONFIGS[2]
    F, G, s_true = gi.config_pair(2)
    eps = np.finfo(np.float64).eps
    tol = spec.n * eps
    dev = torch.device("cuda:0")
    F0 = torch.from_numpy(F).to(dev)          # Fortran-ordered -> column-major storage
    G0 = torch.from_numpy(G).to(dev)
    Fw = F0.clone()
    Gw = G0.clone()
    kw = dict(w=args.w, ordering=hz.HZ_ORD_MM, tol=tol, inner_max_sweeps=args.inner_max_sweeps)
    tune_cache = None if args.no_tune else args.tune_cache
    if tune_cache is not None:
        # block width, outer ordering and tolerance are the workload's; the
        # tuner picks the ordering inside a block pair, the inner sweep cap,
        # Gram splits, update rows and inner lanes
        best, _ = hz.tune(F0, G0, cache=tune_cache, w=args.w, ordering=hz.HZ_ORD_MM, tol=tol,
                          inner_ordering=0)
        kw.update(best)
    if args.only_form:
        if args.only_form == "qr_shortened":
            res = qr_shortened_vs_plain(F0, G0, s_true, tol, kw, tune_cache)
        elif args.only_form == "mixed":
            res = mixed_vs_plain()
        elif args.only_form == "complex":
            res = complex_shortened_vs_plain()
        else:
            res = batched_vs_plain(tune_cache)
        print(json.dumps(dict(form=args.only_form, **res)))
        return
    p = hz.params(**kw)
    nbytes = hz.lib().hz_dgsvd_work_size(ctypes.byref(p), spec.m_f, spec.m_g, spec.n)
    work = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)

    def solve():
        Fw.copy_(F0)
        Gw.copy_(G0)
        return hz.gsvd(Fw, Gw, overwrite=True, workspace=work, **kw)

    for _ in range(args.warmup):
        r = solve()
    torch.cuda.synchronize()
    L = hz.lib()
    # untimed pass with events around every launch: the per-kernel split
    L.hz_profile_enable(1)
    solve()
    torch.cuda.synchronize()
    ms = (ctypes.c_double * 4)()
    cnt = (ctypes.c_int64 * 4)()
    L.hz_profile_read(ms, cnt, 4)
    kind_index = {"gram": 0, "inner": 1, "update": 2}
    dom = max(kind_index, key=lambda k: ms[kind_index[k]])
    split_ms = {k: (ms[i], cnt[i]) for k, i in kind_index.items()}
    split_pass = dict(split_ms)
    # timed region: events only around the dominant kernel's launches (events
    # around every launch would stretch the solve by about 10 %)
    L.hz_profile_enable(4 + kind_index[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweeps, isw, rots = [], 0, 0
    for _ in range(args.steps):
        r = solve()
        sweeps.append(r["sweeps"])
        isw += r["inner_sweeps"]
        rots += r["rot_total"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    L.hz_profile_read(ms, cnt, 4)
    L.hz_profile_enable(0)
    split_ms[dom] = (ms[kind_index[dom]], cnt[kind_index[dom]])
    err = float(np.max(np.abs(r["sigma"].cpu().numpy() - s_true) / s_true))

    gram, upd = algorithmic(spec.m_f, spec.m_g, spec.n, args.w)
    npairs = spec.n // (2 * args.w)
    launches_timed = sum(sweeps) * (spec.n // args.w)     # inner launches in the timed solves
    isteps = 2 * args.w if kw.get("inner_ordering") == hz.HZ_ORD_MM else 2 * args.w - 1
    inner = dict(flops=inner_flops(args.w, launches_timed, isw, rots, npairs, isteps),
                 bytes=None)
    kinds = {"gram": (*split_ms["gram"], gram), "inner": (*split_ms["inner"], inner),
             "update": (*split_ms["update"], upd)}
    split = {k: round(v[0] / max(1e-9, sum(x[0] for x in split_pass.values())), 4)
             for k, v in split_pass.items()}
    t_launch = kinds[dom][0] / max(1, kinds[dom][1]) * 1e-3
    work_d = kinds[dom][2]
    ridge = FP64_MFMA_PEAK_TFS * 1e12 / (HBM_PEAK_GBS * 1e9)
    if dom == "inner":
        # latency-bound FP64 VALU work on one workgroup per pivot pair
        achieved = work_d["flops"] / t_launch / 1e12
        # the solver uses one workgroup (one compute unit) per pivot pair:
        # frac_of_used_cus prices it against the FP64 vector peak of those
        cu_peak = FP64_MFMA_PEAK_TFS * npairs / 256
        roof = dict(bound="alu", achieved=round(achieved, 4), peak=FP64_MFMA_PEAK_TFS,
                    unit="TFLOP/s", frac=round(achieved / FP64_MFMA_PEAK_TFS, 5), traffic=None,
                    cus_used=npairs, frac_of_used_cus=round(achieved / cu_peak, 4))
        intensity = None
    else:
        intensity = work_d["flops"] / work_d["bytes"]
        if intensity < ridge:
            achieved = work_d["bytes"] / t_launch / 1e9
            roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                        unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None)
        else:
            achieved = work_d["flops"] / t_launch / 1e12
            roof = dict(bound="mfma", achieved=round(achieved, 2), peak=FP64_MFMA_PEAK_TFS,
                        unit="TFLOP/s", frac=round(achieved / FP64_MFMA_PEAK_TFS, 4),
                        traffic=None)
    lp = kw.get("inner_lanes") or (16 if args.w == 32 else 8)
    names = {"gram": [f"hz::k_gram<{2 * args.w}>", f"hz::k_gram_sum<{2 * args.w}>"],
             "inner": [f"hz::k_inner<{2 * args.w},{lp}>"],
             "update": [f"hz::k_update<{2 * args.w}>"]}
    traffic = measured_traffic()
    tr = {k: (sum(traffic[n] for n in v) if all(n in traffic for n in v) else None)
          for k, v in names.items()}
    roof["traffic"] = tr[dom]
    roof["kernel"] = "+".join(names[dom])
    roof["avg_launch_us"] = round(t_launch * 1e6, 2)
    if intensity is not None:
        roof["intensity_flop_per_byte"] = round(intensity, 2)
    per_kernel = {k: dict(avg_us=round(v[0] / max(1, v[1]) * 1e3, 2), launches=int(v[1]))
                  for k, v in kinds.items()}
    for k in kinds:
        per_kernel[k]["traffic_bytes"] = tr[k]
    for k in ("gram", "update"):
        wd = kinds[k][2]
        t = kinds[k][0] / max(1, kinds[k][1]) * 1e-3
        per_kernel[k]["GB_s"] = round(wd["bytes"] / t / 1e9, 1) if t > 0 else None
        per_kernel[k]["TFLOP_s"] = round(wd["flops"] / t / 1e12, 2) if t > 0 else None
    # whole-solve FP64 MFMA utilisation from algorithmic flops of the executed steps
    steps_per_sweep = spec.n // args.w
    mean_sweeps = float(np.mean(sweeps))
    solve_flops = mean_sweeps * steps_per_sweep * (gram["flops"] + upd["flops"])
    solves_per_s = args.steps / dt
    mfma_util = solve_flops * solves_per_s / (FP64_MFMA_PEAK_TFS * 1e12)

    out = dict(metric=METRIC, value=round(solves_per_s, 3), unit="solves/s", n_gpus=1,
               steps=args.steps, warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 3),
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
               data="synthetic",
               config=dict(workload="blocked real FP64 GSVD of a seeded 4096x1024 pair "
                                    "(kappa(X)=1e2, sigma log-uniform in [1e-3,1e3])",
                           m_f=spec.m_f, m_g=spec.m_g, n=spec.n, w=args.w, ordering="MM",
                           tol="1024*eps", parallelism="single GPU",
                           launch={k: kw[k] for k in ("inner_ordering", "inner_max_sweeps",
                                                      "inner_lanes", "gram_splits",
                                                      "update_rows") if k in kw}),
               sweeps=sweeps, max_rel_sigma_err_vs_prescribed=err,
               fp64_mfma_util_solve=round(mfma_util, 4),
               kernel_time_split=split, kernels=per_kernel, roofline=roof)
    if not args.no_forms:
        out["transfer_inclusive"] = transfer_inclusive(F, G, Fw, Gw, work, kw)
        out["forms"] = dict(
            qr_shortened=qr_shortened_vs_plain(F0, G0, s_true, tol, kw, tune_cache),
            mixed=mixed_vs_plain(), complex=complex_shortened_vs_plain(),
            batched=batched_vs_plain(tune_cache))
    if not args.no_cpu_baseline:
        golden = os.path.join(ROOT, "tests", "golden", "oracle_config2.json")
        gs = None
        if os.path.exists(golden):
            with open(golden) as fh:
                gs = json.load(fh)["sweeps"]
        out["cpu_baseline"] = cpu_baseline(F, G, tol, gs if gs else int(round(mean_sweeps)))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
