"""MI355X sGS-ADMM solver for the PSD-only SDPs of sparse moment relaxations.

Thin ctypes binding of ``libstrom.so`` (include/strom.h, include/strom_gen.h): every call
marshals arguments and forwards to the C ABI; every step of the ADMM iteration runs in the
library's HIP kernels.  PyTorch is used only for device memory and streams.  Importing this
package fails loudly when the native library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstrom.so")

F64, F32 = 0, 1
RUNNING, CONVERGED, MAXITER, DIVERGED = 0, 1, 2, 3
STATUS = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_HIP", -4: "E_FACTOR", -5: "E_AGAIN",
          -6: "E_NOTFOUND", -7: "E_STATE"}
EXPORTS = [
    "strom_default_opts", "strom_last_error", "strom_ctx_create", "strom_ctx_destroy",
    "strom_sdp_setup", "strom_sdp_destroy", "strom_admm_step", "strom_admm_enqueue",
    "strom_kkt_residuals", "strom_get_iterate", "strom_set_iterate", "strom_sdp_sizes",
    "strom_project_psd_batched", "strom_submit", "strom_poll", "strom_profile_iteration",
    "strom_eig_batched", "strom_dual_bound", "strom_dual_bound_noalloc", "strom_extract",
    "strom_batch_create", "strom_batch_step", "strom_batch_tune", "strom_batch_destroy",
    "strom_gen_build", "strom_gen_sizes", "strom_gen_export", "strom_gen_trace_bounds", "strom_gen_free",
]


class StromError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Opts(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("tau", C.c_double), ("eps_reg", C.c_double), ("tol", C.c_double),
                ("maxiter", C.c_int64), ("kkt_every", C.c_int32), ("proj_dtype", C.c_int32),
                ("polish_eta", C.c_double), ("sigma_every", C.c_int32), ("task_split", C.c_int32),
                ("block_rows", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("eta_p", C.c_double), ("eta_d", C.c_double), ("eta_g", C.c_double), ("pobj", C.c_double),
                ("dobj", C.c_double), ("sigma", C.c_double), ("iters", C.c_int64), ("state", C.c_int32),
                ("t_queue_s", C.c_double), ("t_setup_s", C.c_double), ("t_solve_s", C.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["eta"] = max(d["eta_p"], d["eta_d"], d["eta_g"])
        return d


class Problem_(C.Structure):
    _fields_ = [("nblocks", C.c_int32), ("block_sizes", C.c_void_p), ("m", C.c_int32), ("nnz", C.c_int64),
                ("A_rowptr", C.c_void_p), ("A_col", C.c_void_p), ("A_val", C.c_void_p), ("b", C.c_void_p),
                ("C_svec", C.c_void_p), ("X0_svec", C.c_void_p), ("S0_svec", C.c_void_p)]


class PhaseTimes(C.Structure):
    _fields_ = [("rhs_ms", C.c_double), ("solve_ms", C.c_double), ("xb_ms", C.c_double),
                ("project_ms", C.c_double), ("xupdate_ms", C.c_double), ("kkt_ms", C.c_double),
                ("iteration_ms", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.strom_default_opts.argtypes = [C.POINTER(Opts)]
    L.strom_last_error.restype = C.c_char_p
    L.strom_ctx_create.argtypes = [C.c_int, vp, C.c_size_t, C.POINTER(vp)]
    L.strom_ctx_destroy.argtypes = [vp]
    L.strom_sdp_setup.argtypes = [vp, C.POINTER(Problem_), C.POINTER(Opts), C.POINTER(vp)]
    L.strom_sdp_destroy.argtypes = [vp]
    L.strom_admm_step.argtypes = [vp, i32, C.POINTER(Info)]
    L.strom_admm_enqueue.argtypes = [vp, i32]
    L.strom_kkt_residuals.argtypes = [vp, C.POINTER(Info)]
    L.strom_get_iterate.argtypes = [vp, vp, vp, vp]
    L.strom_set_iterate.argtypes = [vp, vp, vp, vp]
    L.strom_sdp_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64)]
    L.strom_project_psd_batched.argtypes = [vp, i32, i32, vp, vp, vp, vp, C.c_int, vp]
    L.strom_eig_batched.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp, C.c_int, vp]
    L.strom_dual_bound.argtypes = [vp, vp, vp, vp]
    L.strom_dual_bound_noalloc.argtypes = [vp, vp, vp, vp]
    L.strom_scratch_bytes.restype = C.c_size_t
    L.strom_extract.argtypes = [vp, i32, vp, vp, vp]
    L.strom_batch_create.argtypes = [vp, i32, vp, C.POINTER(vp)]
    L.strom_batch_step.argtypes = [vp, i32, vp]
    L.strom_batch_tune.argtypes = [vp, i32, i32, vp, vp, vp, C.POINTER(i32)]
    L.strom_batch_destroy.argtypes = [vp]
    L.strom_submit.argtypes = [vp, C.POINTER(Problem_), C.POINTER(Opts), C.POINTER(C.c_uint64)]
    L.strom_poll.argtypes = [vp, C.c_uint64, C.POINTER(Info), vp, vp, vp]
    L.strom_profile_iteration.argtypes = [vp, i32, C.POINTER(PhaseTimes)]
    L.strom_gen_build.argtypes = [C.c_int, C.c_int, vp, C.c_int, C.POINTER(vp)]
    L.strom_gen_sizes.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64), C.POINTER(i64)]
    L.strom_gen_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.strom_gen_trace_bounds.argtypes = [vp, vp]
    L.strom_gen_free.argtypes = [vp]
    for name in EXPORTS:
        if name not in ("strom_default_opts", "strom_last_error", "strom_gen_free"):
            getattr(L, name).restype = C.c_int
    return L


_L = _load()


def lib():
    return _L


def _check(rc: int):
    if rc != 0:
        raise StromError(rc, _L.strom_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def default_opts(**kw) -> Opts:
    o = Opts()
    _L.strom_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "proj_dtype" and isinstance(v, str):
            v = F32 if v.lower() in ("f32", "fp32", "float32") else F64
        setattr(o, k, v)
    return o


class Problem:
    """Host copy of one SDP in the C ABI's layout (svec columns, CSR rows)."""

    def __init__(self, block_sizes, rowptr, col, val, b, C_svec, X0=None, S0=None, row_kind=None):
        self.block_sizes = np.ascontiguousarray(block_sizes, dtype=np.int32)
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.b = np.ascontiguousarray(b, dtype=np.float64)
        self.C = np.ascontiguousarray(C_svec, dtype=np.float64)
        self.X0 = None if X0 is None else np.ascontiguousarray(X0, dtype=np.float64)
        self.S0 = None if S0 is None else np.ascontiguousarray(S0, dtype=np.float64)
        self.row_kind = row_kind
        self.m = len(self.b)
        self.nsvec = len(self.C)
        self.nnz = len(self.col)
        _validate_problem(self)

    def _c(self) -> Problem_:
        p = Problem_()
        p.nblocks = len(self.block_sizes)
        p.block_sizes = _ptr(self.block_sizes)
        p.m = self.m
        p.nnz = self.nnz
        p.A_rowptr = _ptr(self.rowptr)
        p.A_col = _ptr(self.col)
        p.A_val = _ptr(self.val)
        p.b = _ptr(self.b)
        p.C_svec = _ptr(self.C)
        p.X0_svec = _ptr(self.X0)
        p.S0_svec = _ptr(self.S0)
        return p


def _bad(msg: str):
    raise StromError(-1, msg)


def _validate_problem(p) -> None:
    """Lengths the C ABI cannot see behind its raw pointers (E_INVAL on a mismatch)."""
    if p.block_sizes.ndim != 1 or len(p.block_sizes) == 0 or (p.block_sizes <= 0).any():
        _bad("block sizes must be a non-empty list of positive integers")
    n = int(np.sum(p.block_sizes.astype(np.int64) * (p.block_sizes.astype(np.int64) + 1) // 2))
    if p.nsvec != n:
        _bad(f"C has {p.nsvec} entries, the blocks' svec length is {n}")
    for name in ("X0", "S0"):
        v = getattr(p, name)
        if v is not None and len(v) != n:
            _bad(f"{name} has {len(v)} entries, the blocks' svec length is {n}")
    if len(p.rowptr) != p.m + 1:
        _bad(f"rowptr has {len(p.rowptr)} entries, expected m + 1 = {p.m + 1}")
    if len(p.val) != p.nnz or (p.m >= 0 and len(p.rowptr) and p.rowptr[-1] != p.nnz) or \
            (len(p.rowptr) and p.rowptr[0] != 0):
        _bad("rowptr, col and val do not describe one CSR matrix")


def _check_dense_blocks(n_dev, offset_dev, inp, out, max_n: int, device, out_dtype=None, elems=None) -> None:
    """Checks of the device arguments of the dense batched calls, done on the host before any
    launch: index dtypes, device, contiguity, matching float types, and every block inside the
    buffers (offset + n*n <= numel, n <= max_n).  `elems(n)` is the per-block extent (n*n)."""
    import torch
    elems = elems or (lambda n: n * n)
    if n_dev.dtype != torch.int32 or offset_dev.dtype != torch.int64:
        _bad("block sizes must be int32 and offsets int64")
    if n_dev.dim() != 1 or offset_dev.dim() != 1 or n_dev.numel() != offset_dev.numel():
        _bad("block sizes and offsets must be 1-D tensors of equal length")
    tensors = [n_dev, offset_dev, inp] + ([out] if out is not None else [])
    for t in tensors:
        if t.device != device:
            _bad(f"tensor on {t.device}, the context is on {device}")
        if not t.is_contiguous():
            _bad("tensors must be contiguous")
    if inp.dtype not in (torch.float32, torch.float64):
        _bad("matrices must be float32 or float64")
    if out is not None and out.dtype != (out_dtype or inp.dtype):
        _bad("output dtype differs from the input's")
    if n_dev.numel() == 0:
        return
    n = n_dev.to("cpu", torch.int64)
    o = offset_dev.to("cpu")
    if int(n.min()) <= 0 or int(n.max()) > max_n:
        _bad(f"block sizes must be in 1..max_n = {max_n}")
    if int(o.min()) < 0:
        _bad("negative block offset")
    end = int((o + elems(n)).max())
    if end > inp.numel() or (out is not None and end > out.numel()):
        _bad("a block reaches past the end of its buffer")


def generate(family: int, N: int, params) -> Problem:
    """Relaxation of one trajectory problem (strom_gen_build)."""
    prm = np.ascontiguousarray(params, dtype=np.float64)
    h = C.c_void_p()
    _check(_L.strom_gen_build(int(family), int(N), _ptr(prm), len(prm), C.byref(h)))
    try:
        nb, m, nnz, n = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        _check(_L.strom_gen_sizes(h, C.byref(nb), C.byref(m), C.byref(nnz), C.byref(n)))
        bs = np.zeros(nb.value, np.int32)
        rp = np.zeros(m.value + 1, np.int64)
        ci = np.zeros(nnz.value, np.int32)
        av = np.zeros(nnz.value, np.float64)
        b = np.zeros(m.value, np.float64)
        Cv = np.zeros(n.value, np.float64)
        kind = np.zeros(m.value, np.int32)
        _check(_L.strom_gen_export(h, _ptr(bs), _ptr(rp), _ptr(ci), _ptr(av), _ptr(b), _ptr(Cv), _ptr(kind)))
        rb = np.zeros(nb.value, np.float64)
        has_rb = _L.strom_gen_trace_bounds(h, _ptr(rb)) == 0
    finally:
        _L.strom_gen_free(h)
    prob = Problem(bs, rp, ci, av, b, Cv, row_kind=kind)
    prob.trace_bounds = rb if has_rb else None  # R_beta of the certificate, None if a variable is unbounded
    return prob


def _stream_handle(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class Context:
    """One device: stream, HBM budget and the serving queue (strom_ctx)."""

    def __init__(self, device: int = 0, stream=None, hbm_budget: int = 0):
        import weakref
        self._h = C.c_void_p()
        self._instances = weakref.WeakSet()
        self._batches = weakref.WeakSet()
        self._sizes = {}  # ticket -> (n_svec, m), so poll never hands a short buffer to the library
        self.device = None
        _check(_L.strom_ctx_create(int(device), _stream_handle(stream), C.c_size_t(hbm_budget), C.byref(self._h)))
        import torch
        self.device = torch.device("cuda", int(device))

    def close(self):
        """Destroy the context; instances still alive on it are destroyed first."""
        if self._h:
            for bat in list(self._batches):
                bat.close()
            for inst in list(self._instances):
                inst.close()
            _check(_L.strom_ctx_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, problem: Problem, opts: Opts | None = None) -> int:
        t = C.c_uint64()
        p = problem._c()
        _check(_L.strom_submit(self._h, C.byref(p), C.byref(opts) if opts is not None else None, C.byref(t)))
        self._sizes[t.value] = (problem.nsvec, problem.m)
        return t.value

    def poll(self, ticket: int, nsvec: int | None = None, m: int | None = None):
        """None while in flight, else (info dict, X, y, S).  The iterates are returned when sizes
        are passed (they must be the request's own n_svec and m); the buffers are always allocated
        from the sizes recorded at submit."""
        want = nsvec is not None or m is not None
        rec = self._sizes.get(int(ticket))
        if want and rec is not None and (nsvec not in (None, rec[0]) or m not in (None, rec[1])):
            _bad(f"request {ticket} has n_svec {rec[0]} and m {rec[1]}, not {nsvec} and {m}")
        info = Info()
        X = y = S = None
        if want and rec is not None:
            X, S, y = np.zeros(rec[0]), np.zeros(rec[0]), np.zeros(rec[1])
        elif want:
            _bad(f"unknown request {ticket}")
        rc = _L.strom_poll(self._h, C.c_uint64(ticket), C.byref(info), _ptr(X), _ptr(y), _ptr(S))
        if rc == -5:
            return None
        _check(rc)
        self._sizes.pop(int(ticket), None)
        return info.as_dict(), X, y, S

    def project_psd_batched(self, n_dev, offset_dev, inp, out, max_n: int, stream=None):
        """Project dense column-major blocks (torch device tensors) onto the PSD cone."""
        import torch
        _check_dense_blocks(n_dev, offset_dev, inp, out, int(max_n), self.device)
        dt = F32 if inp.dtype == torch.float32 else F64
        _check(_L.strom_project_psd_batched(self._h, int(n_dev.numel()), int(max_n), C.c_void_p(n_dev.data_ptr()),
                                            C.c_void_p(offset_dev.data_ptr()), C.c_void_p(inp.data_ptr()),
                                            C.c_void_p(out.data_ptr()), dt, _stream_handle(stream)))


    def eig_batched(self, n_dev, offset_dev, inp, woff_dev, w, v=None, max_n: int = 0, stream=None):
        """Eigenvalues (ascending, at woff_dev[k] of w) and optionally eigenvectors (columns at
        offset_dev[k] of v) of dense column-major blocks (torch device tensors)."""
        import torch
        _check_dense_blocks(n_dev, offset_dev, inp, v, int(max_n), self.device)
        _check_dense_blocks(n_dev, woff_dev, w, None, int(max_n), self.device, elems=lambda n: n)
        if w.dtype != inp.dtype:
            _bad("eigenvalue dtype differs from the input's")
        dt = F32 if inp.dtype == torch.float32 else F64
        _check(_L.strom_eig_batched(self._h, int(n_dev.numel()), int(max_n), C.c_void_p(n_dev.data_ptr()),
                                    C.c_void_p(offset_dev.data_ptr()), C.c_void_p(inp.data_ptr()),
                                    C.c_void_p(woff_dev.data_ptr()), C.c_void_p(w.data_ptr()),
                                    C.c_void_p(v.data_ptr() if v is not None else None), dt,
                                    _stream_handle(stream)))


class Instance:
    """One SDP on the device (strom_sdp)."""

    def __init__(self, ctx: Context, problem: Problem, opts: Opts | None = None):
        self.ctx = ctx
        self._h = C.c_void_p()
        p = problem._c()
        if not ctx._h:
            raise StromError(-7, "context is closed")
        _check(_L.strom_sdp_setup(ctx._h, C.byref(p), C.byref(opts) if opts is not None else None,
                                  C.byref(self._h)))
        ctx._instances.add(self)
        n, m, nl = C.c_int64(), C.c_int32(), C.c_int64()
        _check(_L.strom_sdp_sizes(self._h, C.byref(n), C.byref(m), C.byref(nl)))
        self.nsvec, self.m, self.nnzL = n.value, m.value, nl.value

    def close(self):
        if self._h:
            _check(_L.strom_sdp_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n_iter: int) -> dict:
        info = Info()
        _check(_L.strom_admm_step(self._h, int(n_iter), C.byref(info)))
        return info.as_dict()

    def enqueue(self, n_iter: int):
        _check(_L.strom_admm_enqueue(self._h, int(n_iter)))

    def dual_bound(self, R_beta, noalloc: bool = False):
        """(lb, lambda_min per block) of the certificate's lower bound at the current y;
        noalloc: through strom_dual_bound_noalloc (static work buffer, no device allocation)."""
        R = np.ascontiguousarray(R_beta, dtype=np.float64)
        lam = np.zeros(len(R))
        lb = C.c_double()
        fn = _L.strom_dual_bound_noalloc if noalloc else _L.strom_dual_bound
        _check(fn(self._h, R.ctypes.data_as(C.c_void_p), C.cast(C.byref(lb), C.c_void_p),
                  lam.ctypes.data_as(C.c_void_p)))
        return lb.value, lam

    def extract(self, blocks, sizes):
        """(largest two eigenvalues per listed block, top eigenvectors scaled to first entry 1)
        of the listed blocks of the current X; sizes: the listed blocks' sizes."""
        bl = np.ascontiguousarray(blocks, dtype=np.int32)
        lam = np.zeros(2 * len(bl))
        vt = np.zeros(int(np.sum(sizes)))
        _check(_L.strom_extract(self._h, len(bl), bl.ctypes.data_as(C.c_void_p), lam.ctypes.data_as(C.c_void_p),
                                vt.ctypes.data_as(C.c_void_p)))
        out, o = [], 0
        for n in sizes:
            out.append(vt[o:o + int(n)])
            o += int(n)
        return lam.reshape(-1, 2), out

    def kkt(self) -> dict:
        info = Info()
        _check(_L.strom_kkt_residuals(self._h, C.byref(info)))
        return info.as_dict()

    def get_iterate(self):
        X = np.zeros(self.nsvec)
        y = np.zeros(self.m)
        S = np.zeros(self.nsvec)
        _check(_L.strom_get_iterate(self._h, _ptr(X), _ptr(y), _ptr(S)))
        return X, y, S

    def set_iterate(self, X=None, y=None, S=None):
        X = None if X is None else np.ascontiguousarray(X, dtype=np.float64)
        y = None if y is None else np.ascontiguousarray(y, dtype=np.float64)
        S = None if S is None else np.ascontiguousarray(S, dtype=np.float64)
        for name, v, n in (("X", X, self.nsvec), ("y", y, self.m), ("S", S, self.nsvec)):
            if v is not None and len(v) != n:
                _bad(f"{name} has {len(v)} entries, the instance needs {n}")
        _check(_L.strom_set_iterate(self._h, _ptr(X), _ptr(y), _ptr(S)))

    def profile(self, reps: int = 10) -> dict:
        t = PhaseTimes()
        _check(_L.strom_profile_iteration(self._h, int(reps), C.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}


class Batch:
    """Instances of one context iterated together by merged launches (strom_batch_*); while the
    batch is open they are stepped only through it."""

    def __init__(self, ctx: Context, instances):
        self.ctx = ctx
        self.instances = list(instances)
        hs = (C.c_void_p * len(self.instances))(*[i._h.value for i in self.instances])
        self._h = C.c_void_p()
        _check(_L.strom_batch_create(ctx._h, len(self.instances), C.cast(hs, C.c_void_p), C.byref(self._h)))
        ctx._batches.add(self)

    def step(self, n_iter: int) -> list:
        infos = (Info * len(self.instances))()
        _check(_L.strom_batch_step(self._h, int(n_iter), C.cast(infos, C.c_void_p)))
        return [i.as_dict() for i in infos]

    def tune(self, reps: int = 3) -> list:
        """Autotune the merged projection; returns (n, threads FP64, threads FP32) per class."""
        cap = 64
        n, a, b = (np.zeros(cap, np.int32) for _ in range(3))
        k = C.c_int32()
        _check(_L.strom_batch_tune(self._h, int(reps), cap, _ptr(n), _ptr(a), _ptr(b), C.byref(k)))
        return [(int(n[c]), int(a[c]), int(b[c])) for c in range(min(cap, k.value))]

    def close(self):
        if self._h:
            _check(_L.strom_batch_destroy(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
