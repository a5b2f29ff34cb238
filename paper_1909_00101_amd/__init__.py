"""MI355X (gfx950) one-sided, blocked, implicit Hari-Zimmermann GSVD.

Thin ctypes binding of ``libhzgsvd.so`` (C ABI declared in
``include/hzgsvd.h``).  This module only marshals arguments: every step of
the solve runs in the library's HIP kernels.  PyTorch supplies device memory
and the current stream; there is no CPU fallback -- if the library is not
built, every call raises.

Matrices are column-major (Fortran order).  A torch tensor ``F`` of shape
(m, n) is passed as is when ``F.t().is_contiguous()`` (column-major storage),
otherwise a column-major copy is made.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libhzgsvd.so")
CSRC = os.path.join(_HERE, "csrc")
SOURCES = ["hz_api.hip", "hz_real.hip", "hz_cplx.hip", "hz_mixed.hip", "hz_batched.hip",
           "hz_dataflow.hip", "hz_shorten.hip", "hz_pivqr.hip"]

HZ_OK, HZ_ENOCONV, HZ_ECHOL, HZ_ENONFINITE, HZ_EHIP, HZ_ENOSCRATCH = 0, 1, 2, 3, 4, 5
HZ_NOALLOC_SCRATCH_BYTES = 128 << 20
HZ_ORD_MM, HZ_ORD_RR, HZ_ORD_RING = 1, 2, 3
HZ_SCHED_STEPS, HZ_SCHED_DATAFLOW, HZ_SCHED_PERSISTENT = 1, 2, 3

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-result"]


def build(verbose: bool = False) -> str:
    """Compile libhzgsvd.so for gfx950 with hipcc (always recompiles)."""
    objs = []
    bdir = os.path.join(_HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(_ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
        if verbose and r.stderr:
            print(r.stderr)
        objs.append(obj)
    tmp = LIB_PATH + ".tmp"
    r = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class HzParams(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("ordering", ctypes.c_int),
                ("inner_ordering", ctypes.c_int), ("w", ctypes.c_int),
                ("inner_max_sweeps", ctypes.c_int), ("max_sweeps", ctypes.c_int),
                ("tol", ctypes.c_double), ("sort", ctypes.c_int),
                ("mixed_switch", ctypes.c_double), ("max_fp32_sweeps", ctypes.c_int),
                ("inner_lanes", ctypes.c_int), ("gram_splits", ctypes.c_int),
                ("update_rows", ctypes.c_int), ("schedule", ctypes.c_int),
                ("qr_shorten", ctypes.c_int), ("pivot_qr", ctypes.c_int),
                ("timing", ctypes.c_int)]


class HzInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int), ("sweeps_fp32", ctypes.c_int),
                ("converged", ctypes.c_int), ("w", ctypes.c_int),
                ("failed_pair", ctypes.c_int64), ("rot_total", ctypes.c_uint64),
                ("rot_big", ctypes.c_uint64), ("last_offdiag", ctypes.c_double),
                ("inner_sweeps", ctypes.c_uint64), ("status", ctypes.c_int),
                ("n_offdiag", ctypes.c_int), ("fp32_offdiag", ctypes.c_double * 32),
                ("t_gram", ctypes.c_double), ("t_inner", ctypes.c_double),
                ("t_update", ctypes.c_double), ("t_other", ctypes.c_double),
                ("updates_skipped", ctypes.c_uint64), ("fp32_chol_restarts", ctypes.c_int)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        i64, vp, dp = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p
        L.hz_default_params.argtypes = [ctypes.POINTER(HzParams)]
        L.hz_default_params.restype = None
        L.hz_dgsvd_work_size.argtypes = [ctypes.POINTER(HzParams), i64, i64, i64]
        L.hz_dgsvd_work_size.restype = ctypes.c_size_t
        L.hz_dgsvd.argtypes = [ctypes.POINTER(HzParams), i64, i64, i64, dp, i64, dp, i64, dp,
                               i64, dp, dp, dp, vp, ctypes.c_size_t, ctypes.POINTER(HzInfo), vp]
        L.hz_dgsvd.restype = ctypes.c_int
        L.hz_zgsvd.argtypes = L.hz_dgsvd.argtypes
        L.hz_zgsvd.restype = ctypes.c_int
        L.hz_zgsvd_work_size.argtypes = L.hz_dgsvd_work_size.argtypes
        L.hz_zgsvd_work_size.restype = ctypes.c_size_t
        L.hz_dgsvd_noalloc.argtypes = [ctypes.POINTER(HzParams), i64, i64, i64, dp, i64, dp,
                                       i64, dp, i64, dp, dp, dp, ctypes.POINTER(HzInfo), vp]
        L.hz_dgsvd_noalloc.restype = ctypes.c_int
        L.hz_dgsvd_mixed.argtypes = L.hz_dgsvd.argtypes
        L.hz_dgsvd_mixed.restype = ctypes.c_int
        L.hz_dgsvd_mixed_work_size.argtypes = L.hz_dgsvd_work_size.argtypes
        L.hz_dgsvd_mixed_work_size.restype = ctypes.c_size_t
        L.hz_eval_2x2_z.argtypes = [i64, vp, vp, vp]
        L.hz_eval_2x2_z.restype = ctypes.c_int
        L.hz_strerror.argtypes = [ctypes.c_int]
        L.hz_strerror.restype = ctypes.c_char_p
        L.hz_eval_2x2.argtypes = [i64, vp, vp, vp]
        L.hz_eval_2x2.restype = ctypes.c_int
        L.hz_eval_mul_rd.argtypes = [i64, vp, vp, vp, vp, vp]
        L.hz_eval_mul_rd.restype = ctypes.c_int
        L.hz_ring_ordering.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]
        L.hz_ring_ordering.restype = ctypes.c_int
        L.hz_ordering.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.hz_ordering.restype = ctypes.c_int
        L.hz_profile_enable.argtypes = [ctypes.c_int]
        L.hz_profile_enable.restype = None
        L.hz_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        L.hz_profile_read.restype = ctypes.c_int
        L.hz_profile_read_phases.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        L.hz_profile_read_phases.restype = ctypes.c_int
        pa = ctypes.POINTER(ctypes.c_int64)
        L.hz_dgsvd_batched_work_size.argtypes = [ctypes.POINTER(HzParams), ctypes.c_int, pa, pa, pa]
        L.hz_dgsvd_batched_work_size.restype = ctypes.c_size_t
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.hz_dgsvd_batched.argtypes = [ctypes.POINTER(HzParams), ctypes.c_int, pa, pa, pa,
                                       pp, pa, pp, pa, pp, pa, pp, pp, pp, vp, ctypes.c_size_t,
                                       ctypes.POINTER(HzInfo), vp]
        L.hz_dgsvd_batched.restype = ctypes.c_int
        L.hz_dgsvd_tune.argtypes = [ctypes.POINTER(HzParams), i64, i64, i64, dp, i64, dp, i64,
                                    ctypes.c_char_p, ctypes.POINTER(HzParams),
                                    ctypes.POINTER(ctypes.c_double), vp]
        L.hz_dgsvd_tune.restype = ctypes.c_int
        L.hz_dgsvd_batched_tune.argtypes = [ctypes.POINTER(HzParams), ctypes.c_int, pa, pa, pa,
                                            pp, pa, pp, pa, ctypes.c_char_p,
                                            ctypes.POINTER(HzParams),
                                            ctypes.POINTER(ctypes.c_double), vp]
        L.hz_dgsvd_batched_tune.restype = ctypes.c_int
        L.hz_version.argtypes = []
        L.hz_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def params(**kw) -> HzParams:
    p = HzParams()
    lib().hz_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def eval_mul_rd(a, b):
    """The device's rounded-down products of two float64 CUDA tensors of the
    same length and their error terms (hz_eval_mul_rd): (c, d)."""
    import torch
    L = lib()
    a = a.contiguous()
    b = b.contiguous()
    if a.dtype != torch.float64 or b.dtype != torch.float64 or a.shape != b.shape:
        raise TypeError("a and b must be float64 tensors of one shape")
    c = torch.empty_like(a)
    d = torch.empty_like(a)
    st = L.hz_eval_mul_rd(a.numel(), _ptr(a), _ptr(b), _ptr(c), _ptr(d),
                          ctypes.c_void_p(torch.cuda.current_stream(a.device).cuda_stream))
    if st != 0:
        raise RuntimeError(f"hz_eval_mul_rd returned {st}")
    return c, d


def eval_2x2(inp):
    """Evaluate the device 2x2 transformation on a CUDA float64 tensor of rows
    (a_ii, a_jj, a_ij, b_ij) -> (Z11, Z21, Z12, Z22) (real, shape (k, 4)) or
    (a_ii, a_jj, Re a_ij, Im a_ij, Re b_ij, Im b_ij) -> (Z11, Re Z21, Im Z21,
    Re Z12, Im Z12, Z22) (complex, shape (k, 6))."""
    import torch
    inp = inp.contiguous()
    out = torch.empty_like(inp)
    stream = torch.cuda.current_stream(inp.device).cuda_stream
    fn = lib().hz_eval_2x2 if inp.shape[1] == 4 else lib().hz_eval_2x2_z
    st = fn(inp.shape[0], _ptr(inp), _ptr(out), ctypes.c_void_p(stream))
    if st != 0:
        raise RuntimeError(f"hz_eval_2x2 failed: {st}")
    return out


def _colmajor(t):
    return t if t.t().is_contiguous() else t.t().contiguous().t()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _ld(t):
    """Leading dimension of a column-major matrix view (torch normalises the
    stride of a size-1 dimension, so a single column reports its row count)."""
    return t.stride(1) if t.shape[1] > 1 else max(1, t.shape[0])


def aligned_span(ptr: int, size: int):
    """The 256-byte aligned start inside a buffer of ``size`` bytes at
    ``ptr`` and the bytes that remain from there (0 if none)."""
    start = (ptr + 255) & ~255
    return start, max(0, ptr + size - start)


def _workspace(workspace, nbytes, dev):
    """(aligned pointer, usable bytes, tensor kept alive) for a solve that
    needs ``nbytes``: the caller's buffer when at least ``nbytes`` remain
    after aligning its start to 256 bytes, else a fresh allocation.  The
    usable byte count, not ``nbytes``, is what the library is told, so its
    own size check sees the real extent of the buffer."""
    import torch
    if workspace is not None:
        wptr, avail = aligned_span(workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size())
        if avail >= nbytes:
            return wptr, avail, workspace
    workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    wptr, avail = aligned_span(workspace.data_ptr(), workspace.numel())
    return wptr, avail, workspace


class GsvdError(RuntimeError):
    def __init__(self, status, info):
        msg = lib().hz_strerror(status).decode()
        super().__init__(f"hz status {status}: {msg}")
        self.status = status
        self.info = info


def gsvd(F, G, *, overwrite=False, raise_on_noconv=False, workspace=None, mixed=False, **kw):
    """GSVD of (F, G) on the GPU.

    F (m_F x n) and G (m_G x n) are float64 or complex128 CUDA tensors
    (hz_dgsvd or hz_zgsvd).  Returns a dict
    with U, V (overwriting column-major copies of F, G unless ``overwrite``
    and the inputs are already column-major), Z, sigma, sigma_f, sigma_g
    (descending in sigma), the hz_info fields and the status code.
    Keyword arguments set hz_params fields (w, ordering, inner_max_sweeps,
    max_sweeps, tol, sort, ...).  ``mixed=True`` selects the mixed-precision
    real solver (hz_dgsvd_mixed).
    """
    import torch
    L = lib()
    cplx = F.dtype == torch.complex128
    if F.dtype not in (torch.float64, torch.complex128) or G.dtype != F.dtype:
        raise TypeError("F and G must both be float64 or both complex128")
    if not (F.is_cuda and G.is_cuda):
        raise ValueError("F and G must be CUDA (HIP) tensors")
    U = _colmajor(F) if overwrite else F.t().contiguous().t().clone() if F.t().is_contiguous() \
        else _colmajor(F)
    V = _colmajor(G) if overwrite else G.t().contiguous().t().clone() if G.t().is_contiguous() \
        else _colmajor(G)
    m_f, n = U.shape
    m_g = V.shape[0]
    dev = U.device
    Z = torch.empty((n, n), dtype=F.dtype, device=dev).t()
    sig = torch.empty(n, dtype=torch.float64, device=dev)
    sf = torch.empty_like(sig)
    sg = torch.empty_like(sig)
    p = params(**kw)
    if mixed and cplx:
        raise TypeError("the mixed-precision solver is real only")
    wsz = L.hz_zgsvd_work_size if cplx else (L.hz_dgsvd_mixed_work_size if mixed
                                             else L.hz_dgsvd_work_size)
    nbytes = wsz(ctypes.byref(p), m_f, m_g, n)
    if nbytes == 0:
        raise ValueError("invalid shape or parameters")
    wptr, wbytes, workspace = _workspace(workspace, nbytes, dev)
    info = HzInfo()
    stream = torch.cuda.current_stream(dev).cuda_stream
    fn = L.hz_zgsvd if cplx else (L.hz_dgsvd_mixed if mixed else L.hz_dgsvd)
    st = fn(ctypes.byref(p), m_f, m_g, n, _ptr(U), _ld(U), _ptr(V), _ld(V),
                    _ptr(Z), _ld(Z), _ptr(sig), _ptr(sf), _ptr(sg), ctypes.c_void_p(wptr),
                    wbytes, ctypes.byref(info), ctypes.c_void_p(stream))
    if st < 0:
        raise ValueError(f"{'hz_zgsvd' if cplx else 'hz_dgsvd'} rejected argument {-st}")
    if st in (HZ_ECHOL, HZ_ENONFINITE, HZ_EHIP) or (raise_on_noconv and st == HZ_ENOCONV):
        raise GsvdError(st, info)
    return dict(U=U, V=V, Z=Z, sigma=sig, sigma_f=sf, sigma_g=sg, status=st,
                sweeps=info.sweeps, converged=bool(info.converged), w=info.w,
                rot_total=info.rot_total, rot_big=info.rot_big,
                inner_sweeps=info.inner_sweeps, sweeps_fp32=info.sweeps_fp32,
                last_offdiag=info.last_offdiag,
                fp32_offdiag=[info.fp32_offdiag[i] for i in range(info.n_offdiag)],
                times_ms=dict(gram=info.t_gram, inner=info.t_inner, update=info.t_update,
                              other=info.t_other),
                updates_skipped=info.updates_skipped,
                fp32_chol_restarts=info.fp32_chol_restarts, info=info)


def gsvd_noalloc(U, V, Z, sigma, sigma_f, sigma_g, **kw):
    """hz_dgsvd_noalloc on caller-provided tensors: U and V hold F and G on
    entry (float64, column-major, CUDA) and are overwritten in place; Z
    (n x n, column-major), sigma, sigma_f, sigma_g (n) are outputs.  The
    library's static scratch is the workspace, so nothing is allocated.
    Returns (status, HzInfo)."""
    import torch
    for t in (U, V, Z):
        if t.dtype != torch.float64 or not t.is_cuda or not t.t().is_contiguous():
            raise TypeError("U, V, Z must be column-major float64 CUDA tensors")
    m_f, n = U.shape
    m_g = V.shape[0]
    p = params(**kw)
    info = HzInfo()
    stream = torch.cuda.current_stream(U.device).cuda_stream
    st = lib().hz_dgsvd_noalloc(ctypes.byref(p), m_f, m_g, n, _ptr(U), _ld(U), _ptr(V), _ld(V),
                                _ptr(Z), _ld(Z), _ptr(sigma), _ptr(sigma_f), _ptr(sigma_g),
                                ctypes.byref(info), ctypes.c_void_p(stream))
    return st, info


def _i64s(vals):
    return (ctypes.c_int64 * len(vals))(*vals)


def _ptrs(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def gsvd_batched(pairs, *, overwrite=False, workspace=None, **kw):
    """Batched GSVD of independent real pairs [(F_i, G_i), ...] of any sizes
    (float64 CUDA tensors on one device) with one call of hz_dgsvd_batched.
    Returns (status, [dict per pair]) where each dict holds U, V, Z, sigma,
    sigma_f, sigma_g and the pair's hz_info fields, including its own
    status.  Keyword arguments set hz_params fields."""
    import torch
    L = lib()
    batch = len(pairs)
    if batch == 0:
        return HZ_OK, []
    Us, Vs, Zs, sg_, sfs, sgs = [], [], [], [], [], []
    dev = pairs[0][0].device
    for F, G in pairs:
        if F.dtype != torch.float64 or G.dtype != torch.float64:
            raise TypeError("the batched solver takes float64 pairs")
        if not (F.is_cuda and G.is_cuda) or F.device != dev or G.device != dev:
            raise ValueError("all pairs must be CUDA (HIP) tensors on one device")
        U = _colmajor(F) if overwrite else F.t().contiguous().t().clone() \
            if F.t().is_contiguous() else _colmajor(F)
        V = _colmajor(G) if overwrite else G.t().contiguous().t().clone() \
            if G.t().is_contiguous() else _colmajor(G)
        n = U.shape[1]
        Us.append(U)
        Vs.append(V)
        Zs.append(torch.empty((n, n), dtype=torch.float64, device=dev).t())
        sg_.append(torch.empty(n, dtype=torch.float64, device=dev))
        sfs.append(torch.empty(n, dtype=torch.float64, device=dev))
        sgs.append(torch.empty(n, dtype=torch.float64, device=dev))
    mf = _i64s([u.shape[0] for u in Us])
    mg = _i64s([v.shape[0] for v in Vs])
    nn = _i64s([u.shape[1] for u in Us])
    p = params(**kw)
    nbytes = L.hz_dgsvd_batched_work_size(ctypes.byref(p), batch, mf, mg, nn)
    if nbytes == 0:
        raise ValueError("invalid shapes or parameters")
    wptr, wbytes, workspace = _workspace(workspace, nbytes, dev)
    infos = (HzInfo * batch)()
    stream = torch.cuda.current_stream(dev).cuda_stream
    st = L.hz_dgsvd_batched(ctypes.byref(p), batch, mf, mg, nn,
                            _ptrs(Us), _i64s([_ld(u) for u in Us]),
                            _ptrs(Vs), _i64s([_ld(v) for v in Vs]),
                            _ptrs(Zs), _i64s([_ld(z) for z in Zs]),
                            _ptrs(sg_), _ptrs(sfs), _ptrs(sgs), ctypes.c_void_p(wptr), wbytes,
                            infos, ctypes.c_void_p(stream))
    if st < 0:
        raise ValueError(f"hz_dgsvd_batched rejected argument {-st}")
    if st == HZ_EHIP:
        raise GsvdError(st, None)
    out = []
    for i in range(batch):
        f = infos[i]
        out.append(dict(U=Us[i], V=Vs[i], Z=Zs[i], sigma=sg_[i], sigma_f=sfs[i],
                        sigma_g=sgs[i], status=f.status, sweeps=f.sweeps,
                        converged=bool(f.converged), w=f.w, rot_total=f.rot_total,
                        rot_big=f.rot_big, inner_sweeps=f.inner_sweeps))
    return st, out


_TUNED = ("w", "inner_max_sweeps", "inner_lanes", "gram_splits", "update_rows", "ordering",
          "inner_ordering")


def tune(F, G, *, cache=None, **kw):
    """Autotune the single-pair real solver on (F, G) (float64 CUDA tensors,
    not modified) with hz_dgsvd_tune.  Fields given in ``kw`` stay fixed;
    returns (dict of the chosen parameters, milliseconds of the timed
    solve).  ``cache`` names the text file that persists the choice."""
    import torch
    L = lib()
    F = _colmajor(F)
    G = _colmajor(G)
    if F.dtype != torch.float64 or G.dtype != torch.float64:
        raise TypeError("the tuner takes float64 pairs")
    p = params(**kw)
    best = HzParams()
    ms = ctypes.c_double()
    stream = torch.cuda.current_stream(F.device).cuda_stream
    st = L.hz_dgsvd_tune(ctypes.byref(p), F.shape[0], G.shape[0], F.shape[1], _ptr(F), _ld(F),
                         _ptr(G), _ld(G), cache.encode() if cache else None, ctypes.byref(best),
                         ctypes.byref(ms), ctypes.c_void_p(stream))
    if st != 0:
        raise GsvdError(st, None) if st > 0 else ValueError(f"hz_dgsvd_tune rejected argument {-st}")
    return {k: getattr(best, k) for k in _TUNED}, ms.value


def tune_batched(pairs, *, cache=None, **kw):
    """Autotune the batched solver on [(F_i, G_i), ...] (not modified) with
    hz_dgsvd_batched_tune; returns (chosen parameters, milliseconds).  The
    ordering is tuned too unless given."""
    kw.setdefault("ordering", 0)
    import torch
    L = lib()
    Fs = [_colmajor(F) for F, _ in pairs]
    Gs = [_colmajor(G) for _, G in pairs]
    batch = len(pairs)
    p = params(**kw)
    best = HzParams()
    ms = ctypes.c_double()
    stream = torch.cuda.current_stream(Fs[0].device).cuda_stream
    st = L.hz_dgsvd_batched_tune(ctypes.byref(p), batch, _i64s([f.shape[0] for f in Fs]),
                                 _i64s([g.shape[0] for g in Gs]), _i64s([f.shape[1] for f in Fs]),
                                 _ptrs(Fs), _i64s([_ld(f) for f in Fs]), _ptrs(Gs),
                                 _i64s([_ld(g) for g in Gs]), cache.encode() if cache else None,
                                 ctypes.byref(best), ctypes.byref(ms), ctypes.c_void_p(stream))
    if st != 0:
        raise GsvdError(st, None) if st > 0 else ValueError(
            f"hz_dgsvd_batched_tune rejected argument {-st}")
    return {k: getattr(best, k) for k in _TUNED}, ms.value
