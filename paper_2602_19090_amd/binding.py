"""ctypes binding of librefeig.so (the C ABI declared in include/refeig.h).

Argument marshalling only: every step of the refinement runs in the HIP
library. torch supplies device memory and the current HIP stream. Matrices
cross the ABI in column-major order; a column-major n x n matrix is held here
as a C-contiguous torch tensor T of shape (n, n) with T[j, i] = X[i, j] (row j
of T is eigenvector j). ``colmajor`` / ``from_colmajor`` convert numpy arrays.

Importing this module raises if the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# One HIP runtime per process: torch ships its own libamdhip64 (soname
# libamdhip64.so.7). Loading torch first makes the dynamic loader bind
# librefeig's libamdhip64.so.7 dependency to that copy instead of mapping a
# second runtime, which would not see the device.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librefeig.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                      "g.build()'` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

REFEIG_OK, REFEIG_NOT_CONVERGED = 0, 1
REFEIG_E_ARG, REFEIG_E_NONFINITE, REFEIG_E_GAP = -1, -2, -3
REFEIG_E_RANGE, REFEIG_E_NOMEM, REFEIG_E_HIP = -4, -5, -6
REFEIG_OZAKI_INT8, REFEIG_FP64_PLAIN = 0, 2
MAX_ITERS = 32


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("max_iter", ctypes.c_int), ("fixed_iters", ctypes.c_int),
                ("stop_rule", ctypes.c_int), ("delta_safety", ctypes.c_double),
                ("xi", ctypes.c_double), ("theta", ctypes.c_double), ("ka_max", ctypes.c_int),
                ("d_extra", ctypes.c_int), ("verbose", ctypes.c_int),
                ("kx_force", ctypes.c_int), ("schedule", ctypes.c_int),
                ("sparse_k", ctypes.c_int), ("vmode", ctypes.c_int), ("plan", ctypes.c_int),
                ("enqueue_only", ctypes.c_int),
                ("group_tau", ctypes.c_double),
                ("reserved_d", ctypes.c_double * 3)]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int),
                ("beta", ctypes.c_int * MAX_ITERS), ("kx", ctypes.c_int * MAX_ITERS),
                ("dv", ctypes.c_int * MAX_ITERS), ("dw", ctypes.c_int * MAX_ITERS),
                ("du", ctypes.c_int * MAX_ITERS), ("pairs", ctypes.c_int * MAX_ITERS),
                ("eps", ctypes.c_double * MAX_ITERS), ("ms_iter", ctypes.c_double * MAX_ITERS),
                ("ms_gemm", ctypes.c_double * MAX_ITERS),
                ("pairs_p", (ctypes.c_int * 3) * MAX_ITERS),
                ("pairs_f", (ctypes.c_double * 3) * MAX_ITERS),
                ("ms_p", (ctypes.c_double * 3) * MAX_ITERS),
                ("launches_p", (ctypes.c_int * 3) * MAX_ITERS),
                ("groups", ctypes.c_int * MAX_ITERS), ("delta_it", ctypes.c_double * MAX_ITERS),
                ("min_gap", ctypes.c_double),
                ("max_abs_lambda", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("vres", ctypes.c_int * MAX_ITERS),
                ("ms_phase", (ctypes.c_double * 5) * MAX_ITERS)]

    def as_dict(self):
        k = self.iters
        return {"status": self.status, "iters": k, "beta": list(self.beta[:k]),
                "kx": list(self.kx[:k]), "dv": list(self.dv[:k]), "dw": list(self.dw[:k]),
                "du": list(self.du[:k]), "pairs": list(self.pairs[:k]), "eps": list(self.eps[:k]),
                "ms_iter": list(self.ms_iter[:k]), "ms_gemm": list(self.ms_gemm[:k]),
                "pairs_p": [list(self.pairs_p[i]) for i in range(k)],
                "ms_p": [list(self.ms_p[i]) for i in range(k)],
                "pairs_f": [list(self.pairs_f[i]) for i in range(k)],
                "launches_p": [list(self.launches_p[i]) for i in range(k)],
                "groups": list(self.groups[:k]), "delta_it": list(self.delta_it[:k]),
                "min_gap": self.min_gap, "max_abs_lambda": self.max_abs_lambda,
                "ms_total": self.ms_total, "vres": list(self.vres[:k]),
                "ms_phase": [list(self.ms_phase[i]) for i in range(k)]}


_vp, _int, _dbl, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
_lib.refeig_default_opts.argtypes = [ctypes.POINTER(Opts)]
_lib.refeig_workspace_bytes.argtypes = [_int, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_lib.refine_eigvecs.argtypes = [_vp, _int, _vp, _int, _vp, _int, _dbl, ctypes.POINTER(Opts), _vp,
                                _sz, _vp, ctypes.POINTER(Report)]
_lib.refeig_strerror.restype = ctypes.c_char_p
_lib.refine_eigvecs_noalloc.argtypes = [_vp, _int, _vp, _int, _vp, _int, _dbl,
                                        ctypes.POINTER(Opts), _vp, ctypes.POINTER(Report)]
_lib.refeig_herm_workspace_bytes.argtypes = [_int, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_lib.refine_eigvecs_herm.argtypes = [_vp, _int, _vp, _int, _vp, _int, _dbl, ctypes.POINTER(Opts),
                                     _vp, _sz, _vp, ctypes.POINTER(Report)]
_lib.refeig_strerror.argtypes = [_int]
_lib.refeig_split_cols.argtypes = [_vp, _int, _int, _int, _int, _vp, _vp, _vp, _vp]
_lib.refeig_slice_gemm.argtypes = [_vp, _vp, _sz, _int, _int, _int, _int, _int, _vp, _vp]
_lib.refeig_split_cols_ex.argtypes = [_vp, _int, _int, _int, _int, _vp, _vp, _vp, _vp, _int, _vp,
                                      _vp]
_lib.refeig_residue_planes.argtypes = [_vp, _sz, _sz, _int, _int, _vp, _vp, _vp]
_lib.refeig_residue_gemm.argtypes = [_vp, _vp, _sz, _int, _int, _vp, _vp, _vp, _vp]
_lib.refeig_slice_gemm_fp8.argtypes = [_vp, _vp, _sz, _int, _int, _int, _int, _int, _vp, _vp]
_lib.refeig_digits_to_e4m3.argtypes = [_vp, _vp, _sz, _vp]
_lib.refeig_mfma_ceiling.argtypes = [_int, _dbl, _vp, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl),
                                     ctypes.POINTER(_dbl)]
_lib.refeig_server_create.argtypes = [_int, _sz, ctypes.POINTER(Opts), ctypes.POINTER(_vp)]
_lib.refeig_server_submit.argtypes = [_vp, _vp, _int, _vp, _int, _vp, _int, _dbl, _vp,
                                      ctypes.POINTER(_int)]
_lib.refeig_server_request_bytes.argtypes = [_int, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_lib.refeig_host_admission_sim.argtypes = [_int, _vp, _vp, _vp, _int, _sz, _vp, _vp]
_lib.refeig_read_report.argtypes = [_vp, _int, ctypes.POINTER(Opts), ctypes.POINTER(_int),
                                    ctypes.POINTER(Report)]
_lib.refeig_server_wait.argtypes = [_vp, _int, ctypes.POINTER(_int), ctypes.POINTER(Report),
                                    ctypes.POINTER(_dbl)]
_lib.refeig_server_destroy.argtypes = [_vp]

_lib.refeig_batched_workspace_bytes.argtypes = [_int, _vp, ctypes.POINTER(Opts),
                                                ctypes.POINTER(_sz)]
_lib.refine_eigvecs_batched.argtypes = [_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.POINTER(Opts), _vp, _sz, _vp, _vp]

_lib.refeig_batch_workspace_bytes.argtypes = [_int, _vp, ctypes.POINTER(Opts), ctypes.POINTER(_sz)]
_lib.refeig_batch_create.argtypes = [_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                     ctypes.POINTER(Opts), _vp, _sz, ctypes.POINTER(_vp)]
_lib.refeig_batch_launch.argtypes = [_vp, _vp]
_lib.refeig_batch_results.argtypes = [_vp, _vp, _vp]
_lib.refeig_batch_destroy.argtypes = [_vp]

_lib.refeig_tile_cache_lookup.argtypes = [ctypes.c_char_p, _int, ctypes.POINTER(_int)]
_lib.refeig_row_nonzeros.argtypes = [_vp, _int, _int, _vp, ctypes.POINTER(_int)]
_lib.refeig_host_beta.argtypes = [_int, _vp, _vp, _vp, _vp, _dbl, ctypes.POINTER(Opts),
                                  ctypes.POINTER(_int), ctypes.POINTER(_int)]
_lib.refeig_host_column_order.argtypes = [_int, _vp, _vp]
_lib.refeig_host_crt_plan.argtypes = [_int, _int, _int, ctypes.POINTER(_int), _vp, _vp, _vp, _vp,
                                      _vp, _vp]
_lib.refeig_host_group_ritz.argtypes = [_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]

EXPORTED = ["refeig_default_opts", "refeig_workspace_bytes", "refine_eigvecs", "refeig_strerror",
            "refine_eigvecs_noalloc",
            "refeig_herm_workspace_bytes", "refine_eigvecs_herm",
            "refeig_split_cols", "refeig_split_cols_ex", "refeig_slice_gemm",
            "refeig_residue_planes", "refeig_residue_gemm", "refeig_slice_gemm_fp8",
            "refeig_digits_to_e4m3", "refeig_batched_workspace_bytes",
            "refeig_server_create", "refeig_server_submit", "refeig_server_wait",
            "refeig_server_destroy", "refeig_server_request_bytes", "refeig_host_admission_sim",
            "refine_eigvecs_batched", "refeig_read_report", "refeig_host_beta",
            "refeig_batch_workspace_bytes", "refeig_batch_create", "refeig_batch_launch",
            "refeig_batch_results", "refeig_batch_destroy", "refeig_tile_cache_lookup",
            "refeig_host_column_order",
            "refeig_host_crt_plan", "refeig_host_group_ritz", "refeig_row_nonzeros",
            "refeig_mfma_ceiling"]


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def default_opts(**kw) -> Opts:
    o = Opts()
    _lib.refeig_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def strerror(status: int) -> str:
    return _lib.refeig_strerror(status).decode()


def workspace_bytes(n: int, opts: Opts | None = None) -> int:
    b = _sz()
    st = _lib.refeig_workspace_bytes(n, ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(b))
    if st != 0:
        raise ValueError(f"refeig_workspace_bytes({n}): {strerror(st)}")
    return b.value


def colmajor(M: np.ndarray, device="cuda"):
    """numpy (n, m) matrix -> C-contiguous torch tensor holding it column-major."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(M, dtype=np.float64).T)).to(device)


def from_colmajor(T) -> np.ndarray:
    return np.asfortranarray(T.detach().cpu().numpy().T)


def refine_eigvecs(A, X, D, target: float, opts: Opts | None = None, work=None, stream=None):
    """Refine X (column-major tensor, see module doc) and D in place. Returns (status, report)."""
    n = D.numel()
    assert A.dtype == X.dtype == D.dtype and A.is_cuda and X.is_cuda and D.is_cuda
    assert A.is_contiguous() and X.is_contiguous() and D.is_contiguous()
    assert tuple(A.shape) == (n, n) and tuple(X.shape) == (n, n)
    rep = Report()
    wb = work.numel() * work.element_size() if work is not None else 0
    st = _lib.refine_eigvecs(_ptr(A), n, _ptr(X), n, _ptr(D), n, float(target),
                             ctypes.byref(opts) if opts is not None else None, _ptr(work), wb,
                             _stream(stream), ctypes.byref(rep))
    return st, rep


def refine_eigvecs_noalloc(A, X, D, target: float, opts: Opts | None = None, stream=None):
    """refine_eigvecs through the entry point that allocates nothing (its workspace is the
    library's static device array; n <= REFEIG_NOALLOC_MAX_N). Returns (status, report)."""
    n = D.numel()
    assert A.dtype == X.dtype == D.dtype and A.is_cuda and X.is_cuda and D.is_cuda
    assert A.is_contiguous() and X.is_contiguous() and D.is_contiguous()
    assert tuple(A.shape) == (n, n) and tuple(X.shape) == (n, n)
    rep = Report()
    st = _lib.refine_eigvecs_noalloc(_ptr(A), n, _ptr(X), n, _ptr(D), n, float(target),
                                     ctypes.byref(opts) if opts is not None else None,
                                     _stream(stream), ctypes.byref(rep))
    return st, rep


def read_report(work, n: int, opts: Opts | None = None):
    """refeig_read_report: (status, report) of a solve enqueued with opts.enqueue_only on the
    workspace `work` (call after the stream has finished it)."""
    st, rep = _int(0), Report()
    r = _lib.refeig_read_report(_ptr(work), int(n), ctypes.byref(opts) if opts is not None else None,
                                ctypes.byref(st), ctypes.byref(rep))
    if r != 0:
        raise ValueError(strerror(r))
    return st.value, rep


def colmajor_complex(M: np.ndarray, device="cuda"):
    """numpy complex (n, m) matrix -> C-contiguous complex128 torch tensor holding it
    column-major (interleaved real and imaginary parts)."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(M, dtype=np.complex128).T)).to(device)


def herm_workspace_bytes(n: int, opts: Opts | None = None) -> int:
    out = _sz(0)
    st = _lib.refeig_herm_workspace_bytes(int(n), ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(out))
    if st != 0:
        raise ValueError(strerror(st))
    return out.value


def refine_eigvecs_herm(A, X, D, target: float, opts: Opts | None = None, work=None, stream=None):
    """Hermitian A: refine the complex X (complex128, column-major, see colmajor_complex) and
    the real D in place. Returns (status, report)."""
    import torch
    n = D.numel()
    assert A.dtype == X.dtype == torch.complex128 and D.dtype == torch.float64
    assert A.is_cuda and X.is_cuda and D.is_cuda
    assert A.is_contiguous() and X.is_contiguous() and D.is_contiguous()
    assert tuple(A.shape) == (n, n) and tuple(X.shape) == (n, n)
    rep = Report()
    wb = work.numel() * work.element_size() if work is not None else 0
    st = _lib.refine_eigvecs_herm(_ptr(A), n, _ptr(X), n, _ptr(D), n, float(target),
                                  ctypes.byref(opts) if opts is not None else None, _ptr(work), wb,
                                  _stream(stream), ctypes.byref(rep))
    return st, rep


def batched_workspace_bytes(ns, opts: Opts | None = None) -> int:
    arr = (ctypes.c_int * len(ns))(*[int(v) for v in ns])
    out = _sz(0)
    st = _lib.refeig_batched_workspace_bytes(len(ns), ctypes.cast(arr, _vp),
                                             ctypes.byref(opts) if opts is not None else None,
                                             ctypes.byref(out))
    if st != 0:
        raise ValueError(strerror(st))
    return out.value


def refine_eigvecs_batched(As, Xs, Ds, targets, opts: Opts | None = None, work=None, stream=None):
    """Batched refine_eigvecs over lists of (A, X, D) tensors (each as for refine_eigvecs).
    Returns (status, [report per problem])."""
    count = len(As)
    assert len(Xs) == len(Ds) == len(targets) == count
    ns = []
    for A, X, D in zip(As, Xs, Ds):
        n = D.numel()
        assert A.is_cuda and X.is_cuda and D.is_cuda and A.is_contiguous() and X.is_contiguous()
        assert tuple(A.shape) == (n, n) and tuple(X.shape) == (n, n)
        ns.append(n)
    ci = ctypes.c_int * count
    cp = ctypes.c_void_p * count
    n_a, ld_a = ci(*ns), ci(*ns)
    A_a, X_a, D_a = (cp(*[t.data_ptr() for t in ts]) for ts in (As, Xs, Ds))
    t_a = (ctypes.c_double * count)(*[float(t) for t in targets])
    reps = (Report * count)()
    wb = work.numel() * work.element_size() if work is not None else 0
    c = lambda a: ctypes.cast(a, _vp)
    st = _lib.refine_eigvecs_batched(count, c(n_a), c(A_a), c(ld_a), c(X_a), c(ld_a), c(D_a), c(t_a),
                                     ctypes.byref(opts) if opts is not None else None, _ptr(work),
                                     wb, _stream(stream), c(reps))
    return st, list(reps)


def batch_workspace_bytes(ns, opts: Opts | None = None) -> int:
    arr = (ctypes.c_int * len(ns))(*[int(v) for v in ns])
    out = _sz(0)
    st = _lib.refeig_batch_workspace_bytes(len(ns), ctypes.cast(arr, _vp),
                                           ctypes.byref(opts) if opts is not None else None,
                                           ctypes.byref(out))
    if st != 0:
        raise ValueError(strerror(st))
    return out.value


class Batch:
    """A grouped batch captured in a HIP graph (refeig_batch_*): created once over lists of
    (A, X, D) tensors (as refine_eigvecs_batched; fixed_iters > 0), replayed with launch(),
    results() -> (status, [status per problem], [report per problem]). The tensors and the
    workspace are kept alive by this object until close()."""

    def __init__(self, As, Xs, Ds, targets, opts: Opts, work=None):
        import torch
        count = len(As)
        assert len(Xs) == len(Ds) == len(targets) == count
        ns = [D.numel() for D in Ds]
        for A, X, n in zip(As, Xs, ns):
            assert A.is_cuda and X.is_cuda and A.is_contiguous() and X.is_contiguous()
            assert tuple(A.shape) == (n, n) and tuple(X.shape) == (n, n)
        if work is None:
            work = torch.empty(batch_workspace_bytes(ns, opts), dtype=torch.uint8, device="cuda")
        self._keep = (list(As), list(Xs), list(Ds), work)
        ci, cp = ctypes.c_int * count, ctypes.c_void_p * count
        self._n = ci(*ns)
        A_a, X_a, D_a = (cp(*[t.data_ptr() for t in ts]) for ts in (As, Xs, Ds))
        t_a = (ctypes.c_double * count)(*[float(t) for t in targets])
        c = lambda a: ctypes.cast(a, _vp)
        self._h = _vp()
        self.count = count
        st = _lib.refeig_batch_create(count, c(self._n), c(A_a), c(self._n), c(X_a), c(self._n),
                                      c(D_a), c(t_a), ctypes.byref(opts), _ptr(work),
                                      work.numel() * work.element_size(), ctypes.byref(self._h))
        if st != 0:
            raise ValueError(strerror(st))

    def launch(self, stream=None):
        st = _lib.refeig_batch_launch(self._h, _stream(stream))
        if st != 0:
            raise RuntimeError(strerror(st))

    def results(self):
        sts = (ctypes.c_int * self.count)()
        reps = (Report * self.count)()
        st = _lib.refeig_batch_results(self._h, ctypes.cast(sts, _vp), ctypes.cast(reps, _vp))
        return st, list(sts), list(reps)

    def close(self):
        if self._h:
            _lib.refeig_batch_destroy(self._h)
            self._h = _vp()
            self._keep = None


class Server:
    """The continuous-batching server (refeig_server_*) with admission by HBM footprint:
    a device arena of budget_bytes, `lanes` concurrent requests at most. submit() returns a
    ticket at once (the request waits for the work already enqueued on torch's current
    stream); wait(ticket) returns (status, report, t_done) with t_done on time.monotonic()'s
    clock. The tensors of a request are kept alive here until it is waited for."""

    def __init__(self, lanes: int, budget_bytes: int, opts: Opts | None = None):
        self._h = _vp()
        st = _lib.refeig_server_create(int(lanes), int(budget_bytes),
                                       ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(self._h))
        if st != 0:
            raise RuntimeError(strerror(st))
        self._keep = {}

    def submit(self, A, X, D, target: float, stream=None) -> int:
        n = D.numel()
        assert A.is_cuda and X.is_cuda and D.is_cuda and A.is_contiguous() and X.is_contiguous()
        assert tuple(A.shape) == (n, n) and tuple(X.shape) == (n, n)
        t = _int(0)
        st = _lib.refeig_server_submit(self._h, _ptr(A), n, _ptr(X), n, _ptr(D), n,
                                       float(target), _stream(stream), ctypes.byref(t))
        if st != 0:
            raise ValueError(strerror(st))
        self._keep[t.value] = (A, X, D)
        return t.value

    def wait(self, ticket: int):
        st, rep, td = _int(0), Report(), _dbl(0.0)
        r = _lib.refeig_server_wait(self._h, int(ticket), ctypes.byref(st), ctypes.byref(rep),
                                    ctypes.byref(td))
        if r != 0:
            raise ValueError(strerror(r))
        self._keep.pop(int(ticket), None)
        return st.value, rep, td.value

    def close(self):
        if self._h:
            _lib.refeig_server_destroy(self._h)
            self._h = _vp()
            self._keep.clear()


def server_request_bytes(n: int, opts: Opts | None = None) -> int:
    b = _sz()
    st = _lib.refeig_server_request_bytes(int(n), ctypes.byref(opts) if opts is not None else None,
                                          ctypes.byref(b))
    if st != 0:
        raise ValueError(strerror(st))
    return b.value


def host_admission_sim(t_arr, nbytes, dur, lanes: int, budget: int):
    """refeig_host_admission_sim: (status, t_start, offsets)."""
    t = np.ascontiguousarray(t_arr, dtype=np.float64)
    b = np.ascontiguousarray(nbytes, dtype=np.uint64)
    d = np.ascontiguousarray(dur, dtype=np.float64)
    ts = np.empty(len(t)); off = np.empty(len(t), dtype=np.uint64)
    st = _lib.refeig_host_admission_sim(len(t), _np_ptr(t), _np_ptr(b), _np_ptr(d), int(lanes),
                                        int(budget), _np_ptr(ts), _np_ptr(off))
    return st, ts, off


def tile_cache_lookup(arch: str, npad: int):
    """refeig_tile_cache_lookup: (cached, tile) for padded order npad on arch."""
    t = _int(0)
    st = _lib.refeig_tile_cache_lookup(arch.encode(), int(npad), ctypes.byref(t))
    if st < 0:
        raise ValueError(strerror(st))
    return st == 0, t.value


def row_nonzeros(A, stream=None) -> int:
    """refeig_row_nonzeros on a column-major device tensor A (n, n)."""
    n = A.shape[0]
    k = _int(0)
    st = _lib.refeig_row_nonzeros(_ptr(A), n, n, _stream(stream), ctypes.byref(k))
    if st != 0:
        raise RuntimeError(strerror(st))
    return k.value


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def host_beta(lam, e, c, mx, target, opts: Opts | None = None):
    """Host entry point refeig_host_beta: (status, beta, kx)."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    e = np.ascontiguousarray(e, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    mx = np.ascontiguousarray(mx, dtype=np.float64)
    b, k = _int(0), _int(0)
    st = _lib.refeig_host_beta(len(lam), _np_ptr(lam), _np_ptr(e), _np_ptr(c), _np_ptr(mx),
                               float(target), ctypes.byref(opts) if opts is not None else None,
                               ctypes.byref(b), ctypes.byref(k))
    return st, b.value, k.value


def host_crt_plan(npad: int, ka1: int, kx: int):
    """The residue-product plan of V (refeig_host_crt_plan): dict with moduli, wA, wX (N x 18),
    U (N x 3, y_q / m_q per modulus), L (N x 4, the 34-bit limbs of the same fractions) and
    M (3)."""
    N = _int(0)
    mods = np.zeros(28, dtype=np.int32)
    wA = np.zeros(28 * 18, dtype=np.int32)
    wX = np.zeros(28 * 18, dtype=np.int32)
    u = np.zeros(84)
    lim = np.zeros(112)
    M = np.zeros(3)
    st = _lib.refeig_host_crt_plan(int(npad), int(ka1), int(kx), ctypes.byref(N), _np_ptr(mods),
                                   _np_ptr(wA), _np_ptr(wX), _np_ptr(u), _np_ptr(lim), _np_ptr(M))
    if st != 0:
        raise ValueError(strerror(st))
    n = N.value
    return {"moduli": mods[:n].tolist(), "wA": wA.reshape(28, 18)[:n], "wX": wX.reshape(28, 18)[:n],
            "U": u.reshape(28, 3)[:n], "L": lim.reshape(28, 4)[:n], "M": M}


def host_column_order(lam):
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty(len(lam), dtype=np.int32)
    st = _lib.refeig_host_column_order(len(lam), _np_ptr(lam), _np_ptr(out))
    return st, out


def host_group_ritz(G_hi, G_lo, W, lam_hi, lam_lo):
    """Host entry point refeig_host_group_ritz: (status, Y, mu_hi, mu_lo)."""
    k = len(lam_hi)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (G_hi, G_lo, W, lam_hi, lam_lo)]
    Y = np.empty((k, k)); mh = np.empty(k); ml = np.empty(k)
    st = _lib.refeig_host_group_ritz(k, *[_np_ptr(a) for a in arrs], _np_ptr(Y), _np_ptr(mh),
                                     _np_ptr(ml))
    return st, Y, mh, ml


def rows_to_kblocked(P):
    """Planes (k, R, K), row m holding its K entries in order, rearranged into the
    K-blocked memory order the kernels use (same shape): element (m, kk) of a plane
    at ((kk // 64) * R + m) * 64 + kk % 64."""
    k, R, K = P.shape
    return P.reshape(k, R, K // 64, 64).permute(0, 2, 1, 3).contiguous().view(k, R, K)


def kblocked_to_rows(P):
    """Inverse of rows_to_kblocked (a view where possible)."""
    k, R, K = P.shape
    return P.reshape(k, K // 64, R, 64).permute(0, 2, 1, 3).reshape(k, R, K)


def split_cols(M, rows: int, cols: int, k: int, want_trunc=True, stream=None):
    """Debug entry point refeig_split_cols on a column-major tensor M (cols, rows).
    The planes come back K-blocked, shape (k, cols_pad, rows_pad)."""
    import torch
    rpad, cpad = -(-rows // 256) * 256, -(-cols // 256) * 256
    exps = torch.empty(cols, dtype=torch.int32, device=M.device)
    planes = torch.empty((k, cpad, rpad), dtype=torch.int8, device=M.device)
    trunc = torch.empty((cols, rows), dtype=torch.float64, device=M.device) if want_trunc else None
    st = _lib.refeig_split_cols(_ptr(M), rows, rows, cols, k, _ptr(exps), _ptr(planes), _ptr(trunc),
                                _stream(stream))
    return st, exps, planes, trunc


def digits_to_e4m3(D, stream=None):
    """refeig_digits_to_e4m3: FP8 E4M3 codes (uint8 tensor, same shape) of the int8 digits D,
    each in [-15, 15]."""
    import torch
    assert D.dtype == torch.int8 and D.is_contiguous()
    codes = torch.empty(D.shape, dtype=torch.uint8, device=D.device)
    st = _lib.refeig_digits_to_e4m3(_ptr(D), _ptr(codes), D.numel(), _stream(stream))
    return st, codes


def mfma_ceiling(variant: int, seconds: float = 1.0, stream=None):
    """refeig_mfma_ceiling: (status, ms, INT8 POP/s, shader clock GHz) of the matrix-core probe
    (variant 0: operands in registers, 1: from LDS, 2: LDS reads, writes and a barrier)."""
    ms, pops, ghz = _dbl(), _dbl(), _dbl()
    st = _lib.refeig_mfma_ceiling(variant, seconds, _stream(stream), ctypes.byref(ms),
                                  ctypes.byref(pops), ctypes.byref(ghz))
    return st, ms.value, pops.value, ghz.value


def slice_gemm_fp8(Lp8, Rp8, npad: int, kl: int, kr: int, d_min: int, ndiag: int, stream=None):
    """refeig_slice_gemm_fp8 (the FP8 ablation): as slice_gemm, with planes of E4M3 codes."""
    import torch
    assert Lp8.stride(0) == Rp8.stride(0) == npad * npad
    C = torch.empty((ndiag, npad, npad), dtype=torch.int32, device=Lp8.device)
    st = _lib.refeig_slice_gemm_fp8(_ptr(Lp8), _ptr(Rp8), npad * npad, npad, kl, kr, d_min, ndiag,
                                    _ptr(C), _stream(stream))
    return st, C


def slice_gemm(Lp, Rp, npad: int, kl: int, kr: int, d_min: int, ndiag: int, stream=None):
    """Debug entry point refeig_slice_gemm. Lp: (kl, npad, npad) int8, Rp: (kr, npad, npad),
    both K-blocked (see rows_to_kblocked)."""
    import torch
    assert Lp.stride(0) == Rp.stride(0) == npad * npad
    C = torch.empty((ndiag, npad, npad), dtype=torch.int32, device=Lp.device)
    st = _lib.refeig_slice_gemm(_ptr(Lp), _ptr(Rp), npad * npad, npad, kl, kr, d_min, ndiag,
                                _ptr(C), _stream(stream))
    return st, C


def split_cols_ex(M, rows: int, cols: int, k: int, colmap=None, kT: int = 0, stream=None):
    """Debug entry point refeig_split_cols_ex on a column-major tensor M (cols, rows): the
    planes of columns colmap[j] (host int array, or None), and kT planes in the transposed
    operand form. Returns (status, exps, planes (k, cols_pad, rows_pad), trunc,
    planesT (kT, rows_pad, cols_pad) or None), all K-blocked."""
    import torch
    rpad, cpad = -(-rows // 256) * 256, -(-cols // 256) * 256
    exps = torch.empty(cols, dtype=torch.int32, device=M.device)
    planes = torch.empty((k, cpad, rpad), dtype=torch.int8, device=M.device)
    trunc = torch.empty((cols, rows), dtype=torch.float64, device=M.device)
    planesT = torch.empty((kT, rpad, cpad), dtype=torch.int8, device=M.device) if kT > 0 else None
    cm = None if colmap is None else np.ascontiguousarray(colmap, dtype=np.int32)
    st = _lib.refeig_split_cols_ex(_ptr(M), rows, rows, cols, k,
                                   _np_ptr(cm) if cm is not None else None, _ptr(exps),
                                   _ptr(planes), _ptr(trunc), int(kT), _ptr(planesT),
                                   _stream(stream))
    return st, exps, planes, trunc, planesT


def residue_planes(planes, k: int, moduli, stream=None):
    """refeig_residue_planes: planes (>= k, ...) int8 tensor (plane stride = one plane);
    returns (status, res) with res (len(moduli), ...) int8, same plane shape."""
    import torch
    assert planes.dtype == torch.int8 and planes.is_contiguous()
    stride = planes[0].numel()
    m = np.ascontiguousarray(moduli, dtype=np.int32)
    res = torch.empty((len(m),) + tuple(planes.shape[1:]), dtype=torch.int8, device=planes.device)
    st = _lib.refeig_residue_planes(_ptr(planes), stride, stride, int(k), len(m), _np_ptr(m),
                                    _ptr(res), _stream(stream))
    return st, res


def residue_gemm(Lp, Rp, npad: int, moduli, vblk=None, out=None, stream=None):
    """refeig_residue_gemm: residue planes Lp (>= N, npad, npad) and Rp (K-blocked), N =
    len(moduli); vblk: host (npad / 256, 2) ints (slot count, level) or None. Returns (status,
    C) with C (N, npad, npad) int8 (out, when given, is written in place)."""
    import torch
    assert Lp.stride(0) == Rp.stride(0) == npad * npad
    m = np.ascontiguousarray(moduli, dtype=np.int32)
    C = out if out is not None else torch.empty((len(m), npad, npad), dtype=torch.int8,
                                                device=Lp.device)
    vb = None if vblk is None else np.ascontiguousarray(vblk, dtype=np.int32).reshape(-1)
    st = _lib.refeig_residue_gemm(_ptr(Lp), _ptr(Rp), npad * npad, npad, len(m), _np_ptr(m),
                                  _np_ptr(vb) if vb is not None else None, _ptr(C),
                                  _stream(stream))
    return st, C
