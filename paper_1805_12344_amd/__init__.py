"""Thin Python binding of libabip (the MI355X ABIP solver).

Each function mirrors one C entry point of ``include/abip.h`` with the same
name; it only marshals torch tensors (device memory) and the current HIP
stream into the call.  Every step of the solver runs in the HIP library; if
the library is missing this module raises on import of the binding -- there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabip.so")

# error codes / statuses / enums (include/abip.h)
ABIP_OK = 0
ABIP_E_INVALID, ABIP_E_DIM, ABIP_E_NONFINITE, ABIP_E_HIP, ABIP_E_OOM, ABIP_E_STATE = -1, -2, -3, -4, -5, -6
ABIP_UNSOLVED, ABIP_SOLVED, ABIP_PRIMAL_INFEASIBLE, ABIP_DUAL_INFEASIBLE, ABIP_MAX_ITERS = 0, 1, 2, 3, 4
ABIP_DENSE_ROWMAJOR, ABIP_CSR = 0, 1
ABIP_PREC_FP64, ABIP_PREC_FP32_POLISH = 0, 1
ABIP_RESTART_HEURISTIC, ABIP_RESTART_SQRT = 0, 1
ABIP_LIN_AUTO, ABIP_LIN_DIRECT, ABIP_LIN_CG, ABIP_LIN_TRSV = 0, 1, 2, 3
ABIP_ENGINE_AUTO, ABIP_ENGINE_WG, ABIP_ENGINE_GRID = 0, 1, 2

STATUS_NAMES = {0: "unsolved", 1: "solved", 2: "primal_infeasible", 3: "dual_infeasible", 4: "max_iters"}


class abip_settings(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("gamma", ctypes.c_double), ("max_admm_iters", ctypes.c_int64),
        ("restart_rule", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("lin_solver", ctypes.c_int32), ("engine", ctypes.c_int32),
        ("fp32_max_iters", ctypes.c_int64), ("cg_tol", ctypes.c_double),
        ("cg_max_iters", ctypes.c_int32), ("block_threads", ctypes.c_int32),
        ("adjoint_tol", ctypes.c_double), ("adjoint_max_iters", ctypes.c_int64),
        ("cg_rule", ctypes.c_int32), ("use_graph", ctypes.c_int32),
        ("lds_resident", ctypes.c_int32),
        ("bb", ctypes.c_int32), ("bb_max_redo", ctypes.c_int32), ("bb_eps_cor", ctypes.c_double),
        ("bb_eps_penalty", ctypes.c_double), ("scale_iters", ctypes.c_int32), ("sparse_gram", ctypes.c_int32),
        ("grid_mirror", ctypes.c_int32),
    ]


class abip_info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("admm_iters", ctypes.c_int64), ("admm_iters_fp64", ctypes.c_int64),
        ("ipm_iters", ctypes.c_int64), ("cg_iters", ctypes.c_int64),
        ("pres", ctypes.c_double), ("dres", ctypes.c_double), ("gap", ctypes.c_double),
        ("pobj", ctypes.c_double), ("dobj", ctypes.c_double), ("tau", ctypes.c_double),
        ("kappa", ctypes.c_double), ("theta", ctypes.c_double), ("mu", ctypes.c_double),
        ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
        ("colpass_fp32", ctypes.c_int64), ("colpass_fp64", ctypes.c_int64), ("kernel_ms", ctypes.c_double),
        ("ticks_colpass", ctypes.c_int64), ("ticks_ginv", ctypes.c_int64), ("ticks_total", ctypes.c_int64),
        ("ticks_check", ctypes.c_int64), ("ticks_update", ctypes.c_int64),
        ("colpass_lds_fp32", ctypes.c_int64), ("colpass_lds_fp64", ctypes.c_int64),
        ("ginv_hbm_fp32", ctypes.c_int64), ("ginv_hbm_fp64", ctypes.c_int64),
        ("lds_mode", ctypes.c_int32), ("fp32_exit_kkt", ctypes.c_double), ("err_vs_fp64", ctypes.c_double),
        ("beta", ctypes.c_double), ("bb_probe_iters", ctypes.c_int64), ("bb_estimates", ctypes.c_int32),
        ("gram_nnz", ctypes.c_int64), ("grid_mirror", ctypes.c_int32),
    ]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, "?")
        return d


class abip_matrix(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("format", ctypes.c_int32),
        ("val", ctypes.c_void_p), ("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p),
        ("nnz", ctypes.c_int64),
    ]


EXPORTS = [
    "abip_default_settings", "abip_setup", "abip_setup_batch", "abip_solve", "abip_solve_batch",
    "abip_backward", "abip_backward_batch", "abip_apply_iq", "abip_set_state", "abip_get_state",
    "abip_iterate", "abip_free", "abip_last_error", "abip_version", "abip_backward_stats",
    "abip_autotune", "abip_solve_noalloc", "abip_update_data",
    "abip_presolve", "abip_presolve_get", "abip_presolve_info", "abip_postsolve", "abip_presolve_free",
    "abip_get_scaling",
]


class ABIPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libabip error {code}: {msg}")
        self.code = code


def load_library(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"libabip.so not found at {path}; run paper_1805_12344_amd.build.build() first")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.abip_default_settings.argtypes = [ctypes.POINTER(abip_settings)]
    lib.abip_setup.argtypes = [ctypes.POINTER(P), ctypes.POINTER(abip_matrix), P, P,
                               ctypes.POINTER(abip_settings), P]
    lib.abip_setup_batch.argtypes = [ctypes.POINTER(P), ctypes.c_int32, ctypes.POINTER(abip_matrix),
                                     ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(abip_settings), P]
    lib.abip_solve.argtypes = [P, P, P, P, ctypes.POINTER(abip_info)]
    lib.abip_solve_batch.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(abip_info)]
    lib.abip_backward.argtypes = [P, P, P, P, P]
    lib.abip_backward_batch.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                        ctypes.POINTER(P)]
    lib.abip_apply_iq.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32]
    lib.abip_set_state.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double]
    lib.abip_get_state.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.POINTER(ctypes.c_double)]
    lib.abip_iterate.argtypes = [P, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.abip_free.argtypes = [P]
    lib.abip_backward_stats.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.abip_autotune.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.abip_update_data.argtypes = [P, ctypes.POINTER(abip_matrix), ctypes.POINTER(P), ctypes.POINTER(P)]
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.abip_presolve.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, ctypes.POINTER(P), i32p, i32p, i32p]
    lib.abip_presolve_get.argtypes = [P, P, P, P, ctypes.POINTER(ctypes.c_double)]
    lib.abip_presolve_info.argtypes = [P, i32p, P, P, P, P, P, i32p]
    lib.abip_postsolve.argtypes = [P, P, P, P, P, P]
    lib.abip_presolve_free.argtypes = [P]
    lib.abip_get_scaling.argtypes = [P, ctypes.c_int32, P, P]
    lib.abip_solve_noalloc.argtypes = [ctypes.POINTER(abip_matrix), P, P, P, P, P, ctypes.POINTER(abip_info),
                                       ctypes.POINTER(abip_settings), P]
    lib.abip_last_error.restype = ctypes.c_char_p
    lib.abip_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("abip_last_error", "abip_version"):
            getattr(lib, name).restype = ctypes.c_int
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc):
    if rc != ABIP_OK:
        raise ABIPError(rc, lib().abip_last_error().decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, shape=None):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    t = t.to(device="cuda", dtype=torch.float64).contiguous()
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def abip_default_settings(**overrides) -> abip_settings:
    s = abip_settings()
    _check(lib().abip_default_settings(ctypes.byref(s)))
    for k, v in overrides.items():
        if not hasattr(s, k):
            raise AttributeError(k)
        setattr(s, k, v)
    return s


class Work:
    """Owner of an ``abip_work*`` handle plus the device copies it was made from."""

    def __init__(self, handle, dims, keep):
        self.handle = handle
        self.dims = dims          # list of (m, n)
        self._keep = keep
        self.last_info = None
        self.nnz = None           # CSR handles: stored entries of A

    @property
    def B(self):
        return len(self.dims)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if self.handle is not None and self.handle.value:
            lib().abip_free(self.handle)
        self.handle = None


def _csr_parts(A):
    """(indptr, indices, data, (m, n)) of a scipy.sparse matrix or a dict with those keys."""
    if isinstance(A, dict):
        return A["indptr"], A["indices"], A["data"], tuple(A["shape"])
    if hasattr(A, "tocsr") and hasattr(A, "indptr"):
        A = A.tocsr()
        return A.indptr, A.indices, A.data, tuple(A.shape)
    return None


def abip_setup(A, b, c, settings: abip_settings | None = None) -> Work:
    """Set up one LP.  A: dense (array / tensor, m x n, row-major) or CSR
    (scipy.sparse matrix, or dict(indptr, indices, data, shape)); the CSR form
    runs the sparse CG engine."""
    parts = _csr_parts(A)
    if parts is not None:
        indptr, indices, data, (m, n) = parts
        rp = torch.as_tensor(indptr).to(device="cuda", dtype=torch.int32).contiguous()
        ci = torch.as_tensor(indices).to(device="cuda", dtype=torch.int32).contiguous()
        va = torch.as_tensor(data).to(device="cuda", dtype=torch.float64).contiguous()
        if rp.numel() != m + 1 or ci.numel() != va.numel():
            raise ValueError("CSR: indptr must have m+1 entries and indices/data the same length")
        b = _dev(b, (m,))
        c = _dev(c, (n,))
        mat = abip_matrix(m, n, ABIP_CSR, va.data_ptr() if va.numel() else None, rp.data_ptr(),
                          ci.data_ptr() if ci.numel() else None, int(va.numel()))
        h = ctypes.c_void_p()
        s = settings or abip_default_settings()
        _check(lib().abip_setup(ctypes.byref(h), ctypes.byref(mat), _ptr(b), _ptr(c), ctypes.byref(s), _stream()))
        w = Work(h, [(m, n)], (rp, ci, va, b, c, s))
        w.nnz = int(va.numel())
        return w
    A = _dev(A)
    m, n = A.shape
    b = _dev(b, (m,))
    c = _dev(c, (n,))
    mat = abip_matrix(m, n, ABIP_DENSE_ROWMAJOR, A.data_ptr(), None, None, 0)
    h = ctypes.c_void_p()
    s = settings or abip_default_settings()
    _check(lib().abip_setup(ctypes.byref(h), ctypes.byref(mat), _ptr(b), _ptr(c), ctypes.byref(s), _stream()))
    return Work(h, [(m, n)], (A, b, c, s))


def abip_setup_batch(As, bs, cs, settings: abip_settings | None = None) -> Work:
    B = len(As)
    As = [_dev(A) for A in As]
    bs = [_dev(b, (A.shape[0],)) for A, b in zip(As, bs)]
    cs = [_dev(c, (A.shape[1],)) for A, c in zip(As, cs)]
    mats = (abip_matrix * B)(*[abip_matrix(A.shape[0], A.shape[1], ABIP_DENSE_ROWMAJOR, A.data_ptr(),
                                           None, None, 0) for A in As])
    bp = (ctypes.c_void_p * B)(*[b.data_ptr() for b in bs])
    cp = (ctypes.c_void_p * B)(*[c.data_ptr() for c in cs])
    h = ctypes.c_void_p()
    s = settings or abip_default_settings()
    _check(lib().abip_setup_batch(ctypes.byref(h), B, mats, bp, cp, ctypes.byref(s), _stream()))
    return Work(h, [(A.shape[0], A.shape[1]) for A in As], (As, bs, cs, s))


def abip_update_data(w: Work, As, bs, cs):
    """Load new dense LPs of the same shapes into a handle (abip_update_data);
    As, bs, cs: lists of B arrays / tensors (one LP: single-element lists)."""
    B = w.B
    if len(As) != B or len(bs) != B or len(cs) != B:
        raise ValueError(f"expected {B} LPs")
    As = [_dev(A) for A in As]
    bs = [_dev(b, (A.shape[0],)) for A, b in zip(As, bs)]
    cs = [_dev(c, (A.shape[1],)) for A, c in zip(As, cs)]
    mats = (abip_matrix * B)(*[abip_matrix(A.shape[0], A.shape[1], ABIP_DENSE_ROWMAJOR, A.data_ptr(),
                                           None, None, 0) for A in As])
    bp = (ctypes.c_void_p * B)(*[b.data_ptr() for b in bs])
    cp = (ctypes.c_void_p * B)(*[c.data_ptr() for c in cs])
    _check(lib().abip_update_data(w.handle, mats, bp, cp))
    w._keep = (As, bs, cs, w._keep[3] if isinstance(w._keep, tuple) and len(w._keep) > 3 else None)


ABIP_PRESOLVE_REDUCED, ABIP_PRESOLVE_INFEASIBLE, ABIP_PRESOLVE_UNBOUNDED = 0, 1, 2


class Presolved:
    """A presolve record (abip_presolve) and what it produced, as host numpy
    arrays: status, A/b/c (the standard form, when REDUCED), obj_offset, where,
    rows_kept, cols_kept, row_kind, fixed (list of (column, value))."""

    def __init__(self, handle, m, n, status, m_std, n_std):
        self.handle, self.m, self.n, self.status = handle, m, n, status
        self.m_std, self.n_std = m_std, n_std

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.abip_presolve_free(self.handle)
            self.handle = None


def _host64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a.detach().cpu() if hasattr(a, "detach") else a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def abip_presolve(A, b, c, l=None, w=None) -> Presolved:
    """Section 4.5's presolve of min c^T x s.t. A x = b, l <= x <= w (host data)."""
    A = _host64(A)
    m, n = A.shape
    b, c = _host64(b, (m,)), _host64(c, (n,))
    lv = None if l is None else _host64(l, (n,))
    wv = None if w is None else _host64(w, (n,))
    h = ctypes.c_void_p()
    st, ms, ns = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().abip_presolve(m, n, ptr(A), ptr(b), ptr(c), ptr(lv), ptr(wv), ctypes.byref(h), ctypes.byref(st),
                               ctypes.byref(ms), ctypes.byref(ns)))
    p = Presolved(h, m, n, st.value, ms.value, ns.value)
    p.__dict__.update(abip_presolve_info(p))
    if p.status == ABIP_PRESOLVE_REDUCED:
        p.A, p.b, p.c, p.obj_offset = abip_presolve_get(p)
    return p


def abip_presolve_info(p: Presolved) -> dict:
    """where, rows_kept, cols_kept, row_kind, fixed [(column, value)] of a presolve."""
    m, n = p.m, p.n
    where = ctypes.c_int32()
    rows = np.zeros(m, dtype=np.int32)
    cols = np.zeros(n, dtype=np.int32)
    kind = np.zeros(m, dtype=np.int32)
    fc = np.zeros(n, dtype=np.int32)
    fv = np.zeros(n)
    nf = ctypes.c_int32()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().abip_presolve_info(p.handle, ctypes.byref(where), vp(rows), vp(cols), vp(kind), vp(fc), vp(fv),
                                    ctypes.byref(nf)))
    reduced = p.status == ABIP_PRESOLVE_REDUCED
    return dict(where=where.value, row_kind=kind, fixed=[(int(fc[t]), float(fv[t])) for t in range(nf.value)],
                rows_kept=rows[: int(np.sum(kind == -1))] if reduced else None,
                cols_kept=cols[: n - nf.value] if reduced else None)


def abip_presolve_get(p: Presolved):
    """(A_std, b_std, c_std, obj_offset) of a presolve that reduced the LP."""
    A = np.zeros((p.m_std, p.n_std))
    b = np.zeros(p.m_std)
    c = np.zeros(p.n_std)
    off = ctypes.c_double()
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().abip_presolve_get(p.handle, vp(A), vp(b), vp(c), ctypes.byref(off)))
    return A, b, c, off.value


def abip_presolve_free(p: Presolved):
    if p.handle:
        _check(lib().abip_presolve_free(p.handle))
        p.handle = None


def abip_postsolve(p: Presolved, x_std, y_std):
    """(x, y, r) of the original LP from a solution of the standard form (host arrays)."""
    xs = _host64(x_std, (p.n_std,))
    ys = _host64(y_std, (p.m_std,))
    x, y, r = np.zeros(p.n), np.zeros(p.m), np.zeros(p.n)
    _check(lib().abip_postsolve(p.handle, xs.ctypes.data_as(ctypes.c_void_p), ys.ctypes.data_as(ctypes.c_void_p),
                                x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p),
                                r.ctypes.data_as(ctypes.c_void_p)))
    return x, y, r


def abip_solve(w: Work):
    """Returns (x, y, s, info_dict) as new CUDA float64 tensors."""
    m, n = w.dims[0]
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    s = torch.empty(n, dtype=torch.float64, device="cuda")
    info = abip_info()
    _check(lib().abip_solve(w.handle, _ptr(x), _ptr(y), _ptr(s), ctypes.byref(info)))
    w.last_info = [info.as_dict()]
    return x, y, s, w.last_info[0]


def abip_solve_batch(w: Work):
    """Returns lists xs, ys, ss and a list of info dicts."""
    B = w.B
    xs = [torch.empty(n, dtype=torch.float64, device="cuda") for (m, n) in w.dims]
    ys = [torch.empty(m, dtype=torch.float64, device="cuda") for (m, n) in w.dims]
    ss = [torch.empty(n, dtype=torch.float64, device="cuda") for (m, n) in w.dims]
    infos = (abip_info * B)()
    xp = (ctypes.c_void_p * B)(*[t.data_ptr() for t in xs])
    yp = (ctypes.c_void_p * B)(*[t.data_ptr() for t in ys])
    sp = (ctypes.c_void_p * B)(*[t.data_ptr() for t in ss])
    _check(lib().abip_solve_batch(w.handle, xp, yp, sp, infos))
    w.last_info = [infos[k].as_dict() for k in range(B)]
    return xs, ys, ss, w.last_info


def abip_backward(w: Work, dL_dx, want_A: bool = False):
    m, n = w.dims[0]
    g = _dev(dL_dx, (n,))
    dc = torch.empty(n, dtype=torch.float64, device="cuda")
    db = torch.empty(m, dtype=torch.float64, device="cuda")
    dA = None
    if want_A:     # CSR handles: dL/dA on the stored entries, in their CSR order
        dA = torch.empty((m, n) if w.nnz is None else (w.nnz,), dtype=torch.float64, device="cuda")
    _check(lib().abip_backward(w.handle, _ptr(g), _ptr(dc), _ptr(db), _ptr(dA)))
    return dc, db, dA


def abip_backward_batch(w: Work, dL_dx, want_A: bool = False):
    B = w.B
    gs = [_dev(g, (n,)) for g, (m, n) in zip(dL_dx, w.dims)]
    dcs = [torch.empty(n, dtype=torch.float64, device="cuda") for (m, n) in w.dims]
    dbs = [torch.empty(m, dtype=torch.float64, device="cuda") for (m, n) in w.dims]
    dAs = [torch.empty((m, n), dtype=torch.float64, device="cuda") if want_A else None for (m, n) in w.dims]
    P = ctypes.c_void_p
    _check(lib().abip_backward_batch(w.handle, (P * B)(*[g.data_ptr() for g in gs]),
                                     (P * B)(*[t.data_ptr() for t in dcs]),
                                     (P * B)(*[t.data_ptr() for t in dbs]),
                                     (P * B)(*[(t.data_ptr() if t is not None else 0) for t in dAs])))
    return dcs, dbs, dAs


def abip_backward_stats(w: Work, k: int = 0):
    it = ctypes.c_int64()
    rr = ctypes.c_double()
    _check(lib().abip_backward_stats(w.handle, k, ctypes.byref(it), ctypes.byref(rr)))
    return it.value, rr.value


def abip_apply_iq(w: Work, k: int, win, use_fp32: bool = False, transpose: bool = False):
    m, n = w.dims[k]
    win = _dev(win, (m + n + 2,))
    out = torch.empty(m + n + 2, dtype=torch.float64, device="cuda")
    _check(lib().abip_apply_iq(w.handle, k, _ptr(win), _ptr(out), int(use_fp32) | (2 * int(transpose))))
    return out


def abip_set_state(w: Work, k: int, y, x, s, tau, kappa, theta, mu):
    m, n = w.dims[k]
    y, x, s = _dev(y, (m,)), _dev(x, (n,)), _dev(s, (n,))
    _check(lib().abip_set_state(w.handle, k, _ptr(y), _ptr(x), _ptr(s), float(tau), float(kappa),
                                float(theta), float(mu)))


def abip_get_state(w: Work, k: int):
    m, n = w.dims[k]
    y = torch.empty(m, dtype=torch.float64, device="cuda")
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    s = torch.empty(n, dtype=torch.float64, device="cuda")
    sc = (ctypes.c_double * 4)()
    _check(lib().abip_get_state(w.handle, k, _ptr(y), _ptr(x), _ptr(s), sc))
    return y, x, s, dict(tau=sc[0], kappa=sc[1], theta=sc[2], mu=sc[3])


def abip_get_scaling(w: Work, k: int = 0):
    """(D, E): LP k's row and column scaling factors (CUDA float64 tensors)."""
    m, n = w.dims[k]
    D = torch.empty(m, dtype=torch.float64, device="cuda")
    E = torch.empty(n, dtype=torch.float64, device="cuda")
    _check(lib().abip_get_scaling(w.handle, k, _ptr(D), _ptr(E)))
    return D, E


def abip_iterate(w: Work, k: int, iters: int, use_fp32: bool = False):
    _check(lib().abip_iterate(w.handle, k, int(iters), int(use_fp32)))


def abip_autotune(w: Work, iters: int = 50):
    """Try the engine's launch configurations for `iters` updates each; keep the fastest.
    Returns dict(chosen=..., ms=[time per candidate]): `chosen` is the kept
    candidate's index for the one-workgroup engine, its workgroup count for the
    grid and sparse engines (order and meaning as in abip_autotune)."""
    ms = (ctypes.c_double * 8)()
    nc = ctypes.c_int32()
    ch = ctypes.c_int32()
    _check(lib().abip_autotune(w.handle, int(iters), ms, 8, ctypes.byref(nc), ctypes.byref(ch)))
    return dict(chosen=ch.value, ms=[ms[i] for i in range(min(8, nc.value))])


def abip_solve_noalloc(A, b, c, settings: abip_settings | None = None, out=None):
    """One dense LP set up and solved without device allocations inside the
    library (abip_solve_noalloc).  Returns (x, y, s, info_dict); ``out`` may give
    preallocated (x, y, s) CUDA float64 tensors to write into."""
    A = _dev(A)
    m, n = A.shape
    b = _dev(b, (m,))
    c = _dev(c, (n,))
    if out is None:
        out = (torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(m, dtype=torch.float64, device="cuda"),
               torch.empty(n, dtype=torch.float64, device="cuda"))
    x, y, s = out
    mat = abip_matrix(m, n, ABIP_DENSE_ROWMAJOR, A.data_ptr(), None, None, 0)
    info = abip_info()
    st = settings or abip_default_settings()
    _check(lib().abip_solve_noalloc(ctypes.byref(mat), _ptr(b), _ptr(c), _ptr(x), _ptr(y), _ptr(s),
                                    ctypes.byref(info), ctypes.byref(st), _stream()))
    return x, y, s, info.as_dict()


def abip_free(w: Work):
    w.free()


def abip_version() -> str:
    return lib().abip_version().decode()


def abip_last_error() -> str:
    return lib().abip_last_error().decode()


class ABIPSolve(torch.autograd.Function):
    """x* = argmin {c^T x : A x = b, x >= 0} as a differentiable function of (A, b, c).

    forward: abip_setup + abip_solve (settings as given); backward: abip_backward,
    the adjoint of the converged HSD fixed point (reusing the cached factor).
    Inputs are float64 CUDA tensors; gradients are returned for A, b and c.
    """

    @staticmethod
    def forward(ctx, A, b, c, settings=None):
        w = abip_setup(A, b, c, settings)
        x, y, s, info = abip_solve(w)
        if info["status"] != ABIP_SOLVED:
            raise ABIPError(ABIP_E_STATE, f"solve ended with status {info['status_name']}")
        ctx.work = w
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        want_A = ctx.needs_input_grad[0]
        dc, db, dA = abip_backward(ctx.work, gx.contiguous().to(torch.float64), want_A=want_A)
        return dA, db, dc, None


def abip_solve_diff(A, b, c, settings=None):
    """Differentiable single-LP solve (see ABIPSolve)."""
    return ABIPSolve.apply(A, b, c, settings)
