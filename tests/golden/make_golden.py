"""Write the oracle's generalized singular values for the large seeded
workloads to tests/golden/oracle_config<k>.json.

Calls only the CPU oracle (oracle/) on pairs drawn by gsvd_inputs; nothing
here comes from the GPU library.  Usage: python tests/golden/make_golden.py 2 3 4
"""
import json
import os
import sys
import time

os.environ.setdefault("OPENBLAS_CORETYPE", "Haswell")   # host-independent pairs

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gsvd_inputs as gi  # noqa: E402
import oracle  # noqa: E402

EPS = np.finfo(np.float64).eps


def main(configs):
    threads = len(os.sched_getaffinity(0))
    for k in configs:
        spec = gi.CONFIGS[k]
        F, G, s_true = gi.config_pair(k)
        tol = spec.n * EPS
        t0 = time.time()
        r = oracle.gsvd(F, G, ordering=oracle.ORD_MM, tol=tol, max_sweeps=30, threads=threads)
        dt = time.time() - t0
        rec = dict(
            source="oracle/hz_oracle.c (unblocked, variant 0, modified-modulus ordering, "
                   "column sorting) on gsvd_inputs.config_pair(%d)" % k,
            config=k, m_f=spec.m_f, m_g=spec.m_g, n=spec.n, complex=spec.is_complex,
            tol=tol, sweeps=r["sweeps"], converged=r["converged"], rot_all=r["rot_all"],
            rot_big=r["rot_big"], seconds=round(dt, 2), threads=threads,
            max_rel_err_vs_prescribed=float(np.max(np.abs(r["sigma"] - s_true) / s_true)),
            blas_coretype=gi.blas_coretype(),
            sigma=[float(x) for x in r["sigma"]],
        )
        path = os.path.join(HERE, "oracle_config%d.json" % k)
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=0)
        print(k, r["sweeps"], r["converged"], "%.1fs" % dt, rec["max_rel_err_vs_prescribed"])


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [2])
