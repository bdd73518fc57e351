"""Plain FP64 CPU oracle of the sGS-ADMM moment-relaxation solver.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the product (``paper_2406_05846_amd``) never does, and
this package never imports the product.  It shares no code with the HIP path.

The C sources next to this file hold the arithmetic (see ``oracle.h`` for the map from each
file to the paper's sections); this module only marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = ["pop.c", "relax.c", "ldl.c", "jacobi.c", "admm.c", "cert.c"]

TOY1D, PENDULUM, CARTPOLE, PAPER_PENDULUM, CAR, FLYING, LANDING, BACKIN, PAPER_CARTPOLE = 0, 1, 2, 3, 4, 5, 6, 7, 8
ROW_NORM, ROW_MOMENT, ROW_LOCALIZING, ROW_EQUALITY, ROW_CONSENSUS = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fPIC", "-shared",
               "-Wall", "-Wno-unused-function", "-o", _SO] + \
              [os.path.join(_HERE, s) for s in _SRCS] + ["-lm"]
        subprocess.run(cmd, check=True)
    return _SO


class _Sdp(C.Structure):
    _fields_ = [
        ("nblocks", C.c_int32), ("bsize", C.POINTER(C.c_int32)), ("bkind", C.POINTER(C.c_int32)),
        ("bclique", C.POINTER(C.c_int32)), ("boff", C.POINTER(C.c_int64)), ("nsvec", C.c_int64),
        ("m", C.c_int32), ("nnz", C.c_int64), ("rowptr", C.POINTER(C.c_int64)),
        ("col", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double)), ("b", C.POINTER(C.c_double)),
        ("C", C.POINTER(C.c_double)), ("rowkind", C.POINTER(C.c_int32)),
        ("rowclique", C.POINTER(C.c_int32)), ("nclique_vars", C.c_int32), ("dx", C.c_int32),
        ("du", C.c_int32),
    ]


class _Ldl(C.Structure):
    _fields_ = [("m", C.c_int32), ("eps", C.c_double), ("Lp", C.POINTER(C.c_int64)),
                ("Li", C.POINTER(C.c_int32)), ("Lx", C.POINTER(C.c_double)),
                ("D", C.POINTER(C.c_double)), ("nnzL", C.c_int64)]


class _Opts(C.Structure):
    _fields_ = [("sigma0", C.c_double), ("tau", C.c_double), ("tol", C.c_double),
                ("maxiter", C.c_int64), ("sigma_every", C.c_int32), ("eps_rel", C.c_double),
                ("verbose", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("eta_p", C.c_double), ("eta_d", C.c_double), ("eta_g", C.c_double),
                ("eta", C.c_double), ("pobj", C.c_double), ("dobj", C.c_double),
                ("sigma", C.c_double), ("iters", C.c_int64), ("converged", C.c_int32),
                ("t_setup_s", C.c_double), ("t_solve_s", C.c_double), ("nnzL", C.c_int64)]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = C.CDLL(_SO)
        L.orc_relax.argtypes = [C.c_int, C.c_int, _dp, C.c_int, C.POINTER(C.POINTER(_Sdp))]
        L.orc_relax.restype = C.c_int
        L.orc_sdp_free.argtypes = [C.POINTER(_Sdp)]
        L.orc_lift.argtypes = [C.c_int, C.c_int, _dp, C.c_int, _dp, C.c_void_p]
        L.orc_lift.restype = C.c_double
        L.orc_rollout.argtypes = [C.c_int, C.c_int, _dp, C.c_int, _dp, _dp]
        L.orc_rollout.restype = C.c_double
        L.orc_lookahead.argtypes = [C.c_int]
        L.orc_lookahead.restype = C.c_int
        L.orc_lookahead_map.argtypes = [C.c_int, C.POINTER(C.c_int)]
        L.orc_lookahead_map.restype = C.c_int
        L.orc_ldl_factor.argtypes = [C.c_int32, C.c_int64, _i64, _i32, _dp, C.c_double,
                                     C.POINTER(C.POINTER(_Ldl))]
        L.orc_ldl_factor.restype = C.c_int
        L.orc_ldl_solve.argtypes = [C.POINTER(_Ldl), _dp]
        L.orc_ldl_free.argtypes = [C.POINTER(_Ldl)]
        L.orc_jacobi_eig.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_jacobi_eig.restype = C.c_int
        L.orc_project_psd.argtypes = [C.c_int, _dp, _dp]
        L.orc_project_psd.restype = C.c_int
        L.orc_default_opts.argtypes = [C.POINTER(_Opts)]
        L.orc_admm_solve.argtypes = [C.c_int32, _i32, C.c_int32, _i64, _i32, _dp, _dp, _dp,
                                     C.POINTER(_Opts), _dp, _dp, _dp, C.POINTER(_Info), C.c_void_p]
        L.orc_admm_solve.restype = C.c_int
        L.orc_project_svec.argtypes = [C.c_int32, _i32, _dp, _dp]
        L.orc_kkt.argtypes = [C.c_int32, _i32, C.c_int32, _i64, _i32, _dp, _dp, _dp, _dp, _dp, _dp,
                              C.POINTER(_Info)]
        L.orc_trace_bounds.argtypes = [C.c_int, C.c_int, _dp, C.c_int, _dp]
        L.orc_trace_bounds.restype = C.c_int
        L.orc_dual_bound.argtypes = [C.c_int32, _i32, C.c_int32, _i64, _i32, _dp, _dp, _dp, _dp, _dp,
                                     C.POINTER(C.c_double), _dp]
        L.orc_dual_bound.restype = C.c_int
        L.orc_extract.argtypes = [C.c_int32, _i32, _dp, C.c_int32, _i32, _dp, _dp]
        L.orc_extract.restype = C.c_int
        _lib = L
    return _lib


class SDP:
    """A PSD-only multi-block SDP in svec/CSR form (numpy copies of the oracle's arrays)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    @property
    def A(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.m, self.nsvec))


def _arr(ptr, n, dtype):
    return np.ctypeslib.as_array(ptr, shape=(int(n),)).astype(dtype, copy=True)


def relax(family: int, N: int, params) -> SDP:
    """Sparse second-order moment relaxation of a family instance (oracle's own generator)."""
    prm = np.ascontiguousarray(params, dtype=np.float64)
    out = C.POINTER(_Sdp)()
    rc = lib().orc_relax(int(family), int(N), prm, len(prm), C.byref(out))
    if rc != 0:
        raise ValueError(f"orc_relax failed: {rc}")
    s = out.contents
    nb, m, nnz, n = s.nblocks, s.m, s.nnz, s.nsvec
    res = SDP(nblocks=nb, bsize=_arr(s.bsize, nb, np.int32), bkind=_arr(s.bkind, nb, np.int32),
              bclique=_arr(s.bclique, nb, np.int32), boff=_arr(s.boff, nb, np.int64), nsvec=int(n),
              m=int(m), nnz=int(nnz), rowptr=_arr(s.rowptr, m + 1, np.int64),
              col=_arr(s.col, nnz, np.int32), val=_arr(s.val, nnz, np.float64),
              b=_arr(s.b, m, np.float64), C=_arr(s.C, n, np.float64),
              rowkind=_arr(s.rowkind, m, np.int32), rowclique=_arr(s.rowclique, m, np.int32),
              nclique_vars=s.nclique_vars, dx=s.dx, du=s.du, family=family, N=N,
              params=prm.copy())
    lib().orc_sdp_free(out)
    return res


def lift(family: int, N: int, params, z, want_X: bool = True):
    prm = np.ascontiguousarray(params, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    X = None
    ptr = None
    if want_X:
        n = relax(family, N, prm).nsvec
        X = np.zeros(n)
        ptr = X.ctypes.data_as(C.c_void_p)
    obj = lib().orc_lift(int(family), int(N), prm, len(prm), z, ptr)
    return X, obj


def lookahead_map(family: int):
    """Components of x_{k+2} that clique k of the family holds after (x_k, u_k, x_{k+1})."""
    lmap = (C.c_int * 21)()
    dl = lib().orc_lookahead_map(int(family), lmap)
    return [int(lmap[j]) for j in range(dl)]


def clique_vars(sdp: SDP, z, k: int):
    """The variables of clique k in a trajectory z of rollout(): z's window (x_k, u_k, x_{k+1}),
    then the lookahead components of x_{k+2} (past x_N: z's trailing values)."""
    step, base = sdp.dx + sdp.du, 2 * sdp.dx + sdp.du
    out = list(z[k * step: k * step + base])
    for j, c in enumerate(lookahead_map(sdp.family)):
        out.append(z[(k + 2) * step + c] if k + 2 <= sdp.N else z[sdp.N * step + sdp.dx + j])
    return np.array(out)


def rollout(family: int, N: int, params, u, dx: int, du: int):
    prm = np.ascontiguousarray(params, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    z = np.zeros((N + 1) * dx + N * du + lib().orc_lookahead(int(family)))
    obj = lib().orc_rollout(int(family), int(N), prm, len(prm), u, z)
    return z, obj


class LDL:
    def __init__(self, sdp: SDP, eps_rel: float = 1e-12):
        self._p = C.POINTER(_Ldl)()
        rc = lib().orc_ldl_factor(sdp.m, sdp.nsvec, sdp.rowptr, sdp.col, sdp.val, eps_rel,
                                  C.byref(self._p))
        if rc != 0:
            raise ValueError(f"orc_ldl_factor failed: {rc}")
        self.m = sdp.m
        self.eps = self._p.contents.eps
        self.nnzL = self._p.contents.nnzL

    def solve(self, r):
        x = np.ascontiguousarray(r, dtype=np.float64).copy()
        lib().orc_ldl_solve(self._p, x)
        return x

    def __del__(self):
        if getattr(self, "_p", None):
            lib().orc_ldl_free(self._p)
            self._p = None


def jacobi_eig(a):
    a = np.array(a, dtype=np.float64, order="F")
    n = a.shape[0]
    buf = np.ascontiguousarray(a.reshape(-1, order="F"))
    v = np.zeros(n * n)
    w = np.zeros(n)
    sweeps = lib().orc_jacobi_eig(n, buf, v, w)
    return w, v.reshape((n, n), order="F"), sweeps


def project_psd(a):
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    buf = np.ascontiguousarray(a.reshape(-1, order="F"))
    out = np.zeros(n * n)
    lib().orc_project_psd(n, buf, out)
    return out.reshape((n, n), order="F")


def project_svec(bsize, x):
    bsize = np.ascontiguousarray(bsize, dtype=np.int32)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    lib().orc_project_svec(len(bsize), bsize, x, out)
    return out


def default_opts(**kw) -> dict:
    o = _Opts()
    lib().orc_default_opts(C.byref(o))
    d = {f: getattr(o, f) for f, _ in _Opts._fields_}
    d.update(kw)
    return d


def admm_solve(sdp: SDP, X0=None, S0=None, history: bool = False, **kw):
    """Run Algorithm 1 to eta <= tol (or maxiter).  Returns a dict with X, y, S and info."""
    o = _Opts(**default_opts(**kw))
    n, m = sdp.nsvec, sdp.m
    X = np.zeros(n) if X0 is None else np.array(X0, dtype=np.float64)
    S = np.zeros(n) if S0 is None else np.array(S0, dtype=np.float64)
    y = np.zeros(m)
    info = _Info()
    hist = np.zeros(4 * max(1, int(o.maxiter))) if history else None
    rc = lib().orc_admm_solve(sdp.nblocks, sdp.bsize, m, sdp.rowptr, sdp.col, sdp.val, sdp.b, sdp.C,
                              C.byref(o), X, y, S, C.byref(info),
                              hist.ctypes.data_as(C.c_void_p) if history else None)
    if rc != 0:
        raise ValueError(f"orc_admm_solve failed: {rc}")
    res = {f: getattr(info, f) for f, _ in _Info._fields_}
    res.update(X=X, y=y, S=S)
    if history:
        res["history"] = hist[: 4 * int(info.iters)].reshape(-1, 4)
    return res


def kkt(sdp: SDP, X, y, S) -> dict:
    info = _Info()
    lib().orc_kkt(sdp.nblocks, sdp.bsize, sdp.m, sdp.rowptr, sdp.col, sdp.val, sdp.b, sdp.C,
                  np.ascontiguousarray(X, dtype=np.float64), np.ascontiguousarray(y, dtype=np.float64),
                  np.ascontiguousarray(S, dtype=np.float64), C.byref(info))
    return {f: getattr(info, f) for f, _ in _Info._fields_}


def trace_bounds(family: int, N: int, params):
    """R_beta per block of the certificate (relax.c), or None if a variable is unbounded."""
    prm = np.ascontiguousarray(params, dtype=np.float64)
    nb = relax(family, N, prm).nblocks
    out = np.zeros(nb)
    rc = lib().orc_trace_bounds(int(family), int(N), prm, len(prm), out)
    if rc == -2:
        return None
    if rc != 0:
        raise ValueError(f"orc_trace_bounds failed: {rc}")
    return out


def dual_bound(sdp: SDP, y, R_beta):
    """Certificate lower bound <b,y> + sum_beta R_beta min(0, lambda_min((C - A^*y)_beta))
    and lambda_min per block (cert.c)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    R = np.ascontiguousarray(R_beta, dtype=np.float64)
    lam = np.zeros(sdp.nblocks)
    lb = C.c_double()
    rc = lib().orc_dual_bound(sdp.nblocks, sdp.bsize, sdp.m, sdp.rowptr, sdp.col, sdp.val, sdp.b, sdp.C, y, R,
                              C.byref(lb), lam)
    if rc != 0:
        raise ValueError(f"orc_dual_bound failed: {rc}")
    return lb.value, lam


def extract(sdp: SDP, X, blocks):
    """Largest two eigenvalues and the top eigenvector (first entry 1) of the listed blocks of X."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    bl = np.ascontiguousarray(blocks, dtype=np.int32)
    sizes = [int(sdp.bsize[k]) for k in bl]
    lam = np.zeros(2 * len(bl))
    vt = np.zeros(sum(sizes))
    rc = lib().orc_extract(sdp.nblocks, sdp.bsize, X, len(bl), bl, lam, vt)
    if rc != 0:
        raise ValueError(f"orc_extract failed: {rc}")
    out, o = [], 0
    for n in sizes:
        out.append(vt[o:o + n])
        o += n
    return lam.reshape(-1, 2), out
