"""CPU oracle for the one-sided implicit Hari-Zimmermann GSVD.

TEST INFRASTRUCTURE ONLY: this package may be imported by the tests, the smoke
check and the benchmark's CPU-baseline leg, never by the GPU library.  It
wraps ``hz_oracle.c`` (plain C, double / double complex, unblocked) through
ctypes.  The C file shares no code with the GPU path; see its header for the
algorithm, the paper passages it follows and the readings taken where the
paper is ambiguous.  :func:`gsvd_qr` adds the QR shortening of tall pairs
(Section 2) around it, with scipy's column-pivoted QR as a library step.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hz_oracle.c")
_LIB = os.path.join(_HERE, "libhzoracle.so")

ORD_ROWCYCLIC, ORD_MM, ORD_RR = 0, 1, 2
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE double, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        sig = [i64, i64, i64, dp, i64, dp, i64, dp, i64, dp, dp, dp,
               ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
               ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        for name in ("hzo_dgsvd", "hzo_zgsvd"):
            f = getattr(lib, name)
            f.argtypes = sig
            f.restype = ctypes.c_int
        lib.hzo_real_2x2.argtypes = [ctypes.c_double] * 4 + [dp, ctypes.POINTER(ctypes.c_int)]
        lib.hzo_real_2x2.restype = None
        lib.hzo_real_2x2_c.argtypes = [ctypes.c_double] * 4 + [dp, ctypes.POINTER(ctypes.c_int),
                                                               dp]
        lib.hzo_real_2x2_c.restype = None
        lib.hzo_cplx_2x2_v.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, dp,
                                       ctypes.POINTER(ctypes.c_int), dp]
        lib.hzo_cplx_2x2_v.restype = None
        lib.hzo_edot.argtypes = [ctypes.c_int64, dp, dp]
        lib.hzo_edot.restype = ctypes.c_double
        lib.hzo_mul_rd.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        lib.hzo_mul_rd.restype = None
        lib.hzo_enh_abs2.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.hzo_enh_abs2.restype = ctypes.c_double
        lib.hzo_ordering.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        lib.hzo_ordering.restype = ctypes.c_int
        lib.hzo_real_sort_keys.argtypes = [ctypes.c_double] * 3 + [dp, dp, dp]
        lib.hzo_real_sort_keys.restype = None
        for name in ("hzo_step_real", "hzo_step_cplx"):
            f = getattr(lib, name)
            f.argtypes = [i64, i64, i64, dp, i64, dp, i64, dp, i64, i64, i64, ctypes.c_double,
                          ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
            f.restype = None
        _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gsvd(F, G, *, ordering=ORD_ROWCYCLIC, tol=0.0, max_sweeps=30, sort=True, threads=0,
         variant=0):
    """GSVD of the pair (F, G) by the unblocked oracle.

    Returns a dict with U, V, Z (Fortran-ordered), sigma, sigma_f, sigma_g
    (descending in sigma), sweeps, rot_all, rot_big, converged, status.
    tol <= 0 selects sqrt(n)*eps.  variant 0 classifies small transformations
    by criterion C1, variant 4 by criterion C2 (Section 2.5, Table 1);
    variants 1 and 5 are 0 and 4 with the enhanced dot products of Appendix
    A (complex pairs: the squared norms only).
    F and G are copied, not modified.
    """
    lib = _load()
    is_c = np.iscomplexobj(F) or np.iscomplexobj(G)
    dt = np.complex128 if is_c else np.float64
    U = np.array(F, dtype=dt, order="F", copy=True)
    V = np.array(G, dtype=dt, order="F", copy=True)
    m_f, n = U.shape
    m_g, n2 = V.shape
    if n != n2:
        raise ValueError("F and G must have the same number of columns")
    Z = np.zeros((n, n), dtype=dt, order="F")
    s = np.zeros(n)
    sf = np.zeros(n)
    sg = np.zeros(n)
    info = np.zeros(4, dtype=np.int64)
    fn = lib.hzo_zgsvd if is_c else lib.hzo_dgsvd
    st = fn(m_f, m_g, n, _dptr(U), m_f, _dptr(V), m_g, _dptr(Z), n,
            _dptr(s), _dptr(sf), _dptr(sg), int(ordering), float(tol), int(max_sweeps),
            1 if sort else 0, int(variant), int(threads),
            info.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if st < 0:
        raise ValueError("oracle rejected the arguments")
    return dict(U=U, V=V, Z=Z, sigma=s, sigma_f=sf, sigma_g=sg, sweeps=int(info[0]),
                rot_all=int(info[1]), rot_big=int(info[2]), converged=bool(info[3]), status=st)


def gsvd_qr(F, G, **kw):
    """GSVD of (F, G) through the shortened pair of Section 2 (the paragraph
    before the prescaling): F P1 = Q_F R_F and (G P1) P2 = Q_G R_G by
    column-pivoted Householder QR (LAPACK geqp3, through scipy), the square
    pair F'' = R_F P2, G'' = R_G of order n is solved by :func:`gsvd` (same
    keyword arguments), and the factors of (F, G) are recovered as
    Z = P1 P2 Z'', U = Q_F U'', V = Q_G V''; sigma, sigma_f, sigma_g are those
    of the shortened pair.  The dict of :func:`gsvd` is returned with U, V, Z
    replaced and the permutations added as ``p1`` (F[:, p1] = Q_F R_F) and
    ``q`` (the combined column order, G[:, q] = Q_G R_G)."""
    import scipy.linalg
    Q_f, R_f, p1 = scipy.linalg.qr(np.asarray(F), mode="economic", pivoting=True)
    Q_g, R_g, p2 = scipy.linalg.qr(np.asarray(G)[:, p1], mode="economic", pivoting=True)
    r = gsvd(R_f[:, p2], R_g, **kw)
    q = p1[p2]
    Z = np.empty_like(r["Z"])
    Z[q, :] = r["Z"]
    r.update(U=np.asfortranarray(Q_f @ r["U"]), V=np.asfortranarray(Q_g @ r["V"]),
             Z=np.asfortranarray(Z), p1=p1, q=q)
    return r


def edot(x, y):
    """The enhanced dot product of Appendix A of two real vectors."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    return float(_load().hzo_edot(len(x), _dptr(x), _dptr(y)))


def enh_abs2(z):
    """|z|^2 by the simpler complex procedure of Appendix A."""
    return float(_load().hzo_enh_abs2(float(np.real(z)), float(np.imag(z))))


def mul_rd(a, b):
    """(c, d): a*b rounded toward -infinity and d = fma(a, b, -c)."""
    c = ctypes.c_double()
    d = ctypes.c_double()
    _load().hzo_mul_rd(float(a), float(b), ctypes.byref(c), ctypes.byref(d))
    return c.value, d.value


def real_2x2(aii, ajj, aij, x, cosines=False):
    """The oracle's real 2x2 transformation (Section 2.1.2) as a 2x2 array
    and the exception flag; with cosines=True also (cos phi, cos psi)."""
    lib = _load()
    z = np.zeros(4)
    cc = np.zeros(2)
    e = ctypes.c_int(0)
    lib.hzo_real_2x2_c(aii, ajj, aij, x, _dptr(z), ctypes.byref(e), _dptr(cc))
    if cosines:
        return z.reshape(2, 2, order="F"), bool(e.value), cc
    return z.reshape(2, 2, order="F"), bool(e.value)


def cplx_2x2(aii, ajj, aij, b, cosines=False):
    """The oracle's complex 2x2 transformation (Section 2.1.1) and the
    exception flag; with cosines=True also (cos phi, cos psi)."""
    lib = _load()
    a = np.array([complex(aij).real, complex(aij).imag])
    bb = np.array([complex(b).real, complex(b).imag])
    z = np.zeros(8)
    cc = np.zeros(2)
    e = ctypes.c_int(0)
    lib.hzo_cplx_2x2_v(aii, ajj, _dptr(a), _dptr(bb), _dptr(z), ctypes.byref(e), _dptr(cc))
    zc = z[0::2] + 1j * z[1::2]
    if cosines:
        return zc.reshape(2, 2, order="F"), bool(e.value), cc
    return zc.reshape(2, 2, order="F"), bool(e.value)


def ordering(kind: int, n: int) -> np.ndarray:
    """The oracle's ordering table: array (steps, pairs_per_step, 2)."""
    lib = _load()
    N = n + (n & 1)
    if kind == ORD_ROWCYCLIC:
        steps, pp = n * (n - 1) // 2, 1
    else:
        steps, pp = (N if kind == ORD_MM else N - 1), N // 2
    t = np.zeros(steps * pp * 2, dtype=np.int32)
    got = lib.hzo_ordering(kind, n, t.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    assert got == steps
    return t.reshape(steps, pp, 2)


def real_sort_keys(aii, ajj, aij, Z):
    """The oracle's sort keys of a real transformed pivot pair (Section
    3.5.3): (a''_11, a''_22) from the pivot entries and the 2x2 Z."""
    z = np.asfortranarray(np.asarray(Z, dtype=np.float64)).ravel(order="F")
    a11 = ctypes.c_double()
    a22 = ctypes.c_double()
    _load().hzo_real_sort_keys(float(aii), float(ajj), float(aij), _dptr(z),
                               ctypes.byref(a11), ctypes.byref(a22))
    return a11.value, a22.value


def step(F, G, Z, i, j, *, tol=0.0, sort=True, variant=0):
    """One pointwise step of the oracle (Section 2.1) on the pivot pair
    (i, j), i < j, of copies of F, G, Z; returns (F, G, Z, transformations,
    big transformations) after the step.  tol <= 0 selects sqrt(n)*eps."""
    lib = _load()
    is_c = np.iscomplexobj(F) or np.iscomplexobj(G) or np.iscomplexobj(Z)
    dt = np.complex128 if is_c else np.float64
    F = np.array(F, dtype=dt, order="F", copy=True)
    G = np.array(G, dtype=dt, order="F", copy=True)
    Z = np.array(Z, dtype=dt, order="F", copy=True)
    m_f, n = F.shape
    m_g = G.shape[0]
    if tol <= 0.0:
        tol = np.sqrt(n) * np.finfo(np.float64).eps
    c = np.zeros(2, dtype=np.int64)
    fn = lib.hzo_step_cplx if is_c else lib.hzo_step_real
    fn(m_f, m_g, n, _dptr(F), m_f, _dptr(G), m_g, _dptr(Z), n, int(i), int(j), float(tol),
       1 if sort else 0, int(variant), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return F, G, Z, int(c[0]), int(c[1])
