"""ctypes wrapper of the LAMG CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  The product path (the HIP library and its binding) never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lamg_oracle.cpp")
SAN_LIB = os.path.join(HERE, "liblamg_oracle_san.so")
LIB = os.environ.get("LAMG_ORACLE_LIB") or os.path.join(HERE, "liblamg_oracle.so")

L_FINEST, L_ELIM, L_AGG = 0, 1, 2


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle (serial, no FMA contraction, no fast-math).  With
    sanitize, an AddressSanitizer + UndefinedBehaviorSanitizer build into its
    own library (loaded by setting LAMG_ORACLE_LIB and preloading the ASan
    runtime; tests/test_oracle_sanitize.py)."""
    out = SAN_LIB if sanitize else LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        extra = (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
                 if sanitize else [])
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", *extra,
                               "-shared", "-fPIC", "-o", tmp, SRC])
        os.replace(tmp, out)
    return out


class Opts(C.Structure):
    _fields_ = [("gamma", C.c_double), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("tv_k_min", C.c_int), ("tv_k_max", C.c_int), ("tv_sweeps", C.c_int),
                ("q_max", C.c_double), ("mu", C.c_double), ("hub_factor", C.c_double),
                ("elim_max_degree", C.c_int), ("coarsest_max_n", C.c_int),
                ("weak_edge_ratio", C.c_double), ("elim_stop_frac", C.c_double),
                ("ec", C.c_int), ("tol", C.c_double), ("max_cycles", C.c_int),
                ("seed", C.c_uint64), ("stage1_quantile", C.c_double), ("relax_fast_ratio", C.c_double),
                ("coarsest_sweeps", C.c_int), ("dense_max", C.c_int), ("allow_negative", C.c_int),
                ("recomb_finest", C.c_int), ("recomb_norm", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        vp, i64, i32p, i64p, dp, fp, u8p = (C.c_void_p, C.c_int64, C.POINTER(C.c_int32),
                                            C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                            C.POINTER(C.c_float), C.POINTER(C.c_uint8))
        sig = {
            "ora_opts_default": (None, [C.POINTER(Opts)]),
            "ora_set_plain_rows": (None, [C.c_int]),
            "ora_recombine": (None, [i64, i64p, i32p, dp, dp, dp, dp, dp, C.c_int, C.c_int, dp, dp]),
            "ora_laplacian": (vp, [i64, i64, i32p, i32p, dp, C.POINTER(C.c_int)]),
            "ora_csr_nnz": (i64, [vp]), "ora_csr_n": (i64, [vp]),
            "ora_csr_export": (None, [vp, i64p, i32p, dp, dp]),
            "ora_csr_free": (None, [vp]),
            "ora_connected": (C.c_int, [i64, i64p, i32p]),
            "ora_colour": (None, [i64, i64p, i32p, C.c_uint64, C.c_int, i32p]),
            "ora_colour_jp": (C.c_int, [i64, i64p, i32p, C.c_uint64, C.c_int, i32p]),
            "ora_hash5": (C.c_uint64, [C.c_uint64] * 5),
            "ora_unit_pm1": (C.c_double, [C.c_uint64]),
            "ora_row_reduce": (C.c_double, [i64, dp]),
            "ora_gs": (None, [i64, i64p, i32p, dp, dp, dp, dp, C.c_int, C.c_int]),
            "ora_gs32": (None, [i64, i64p, i32p, fp, fp, fp, fp, C.c_int, C.c_int]),
            "ora_residual": (None, [i64, i64p, i32p, dp, dp, dp, dp, dp]),
            "ora_gs_multicolour": (None, [i64, i64p, i32p, dp, dp, i32p, dp, dp]),
            "ora_elim_select": (None, [i64, i64p, i32p, C.c_int, u8p]),
            "ora_schur": (vp, [i64, i64p, i32p, dp, dp, u8p, i32p]),
            "ora_galerkin": (vp, [i64, i64p, i32p, dp, dp, i32p, i64]),
            "ora_setup": (vp, [i64, i64, i32p, i32p, dp, C.POINTER(Opts), C.POINTER(C.c_int)]),
            "ora_setup_lgm": (vp, [i64, C.POINTER(Opts), C.POINTER(C.c_int)]),
            "ora_free": (None, [vp]),
            "ora_num_levels": (C.c_int, [vp]),
            "ora_level_dims": (None, [vp, C.c_int, i64p]),
            "ora_level_gamma": (C.c_double, [vp, C.c_int]),
            "ora_level_export": (None, [vp, C.c_int, i64p, i32p, dp, dp, i64p, i32p]),
            "ora_transfer_export": (None, [vp, C.c_int, i32p]),
            "ora_agg_export": (None, [vp, C.c_int, dp, dp, u8p, u8p, u8p, i32p, dp]),
            "ora_perm1": (None, [vp, i32p]),
            "ora_coarsest_n": (i64, [vp]),
            "ora_coarsest_relax": (C.c_int, [vp]),
            "ora_coarsest_solve": (None, [vp, dp, dp]),
            "ora_solve": (C.c_int, [vp, dp, dp, C.c_int, C.c_int, dp, dp]),
            "ora_cycle": (None, [vp, dp, dp]),
            "ora_visit_counts": (None, [vp, i64p]),
            "ora_adjoint": (C.c_int, [vp, i64, i32p, i32p, dp, dp, dp, dp, dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().ora_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Csr:
    def __init__(self, ptr, col, val, diag):
        self.ptr, self.col, self.val, self.diag = ptr, col, val, diag

    @property
    def n(self):
        return self.ptr.shape[0] - 1

    def dense(self) -> np.ndarray:
        n = self.n
        a = np.zeros((n, n))
        rows = np.repeat(np.arange(n), np.diff(self.ptr))
        a[rows, self.col] = -self.val
        a[np.arange(n), np.arange(n)] = self.diag
        return a


def laplacian(n, eu, ev, w) -> Csr:
    eu, ev, w = _i32(eu), _i32(ev), _f64(w)
    st = C.c_int(0)
    h = lib().ora_laplacian(n, eu.shape[0], _p(eu, C.c_int32), _p(ev, C.c_int32), _p(w, C.c_double), C.byref(st))
    if st.value:
        raise ValueError(f"oracle laplacian status {st.value}")
    return _export_csr_n(h, n)


def _export_csr_n(h, n) -> Csr:
    L = lib()
    nnz = L.ora_csr_nnz(h)
    ptr = np.zeros(n + 1, np.int64)
    col = np.zeros(nnz, np.int32)
    val = np.zeros(nnz)
    diag = np.zeros(n)
    L.ora_csr_export(h, _p(ptr, C.c_int64), _p(col, C.c_int32), _p(val, C.c_double), _p(diag, C.c_double))
    L.ora_csr_free(h)
    return Csr(ptr, col, val, diag)


def laplacian_status(n, eu, ev, w) -> int:
    eu, ev, w = _i32(eu), _i32(ev), _f64(w)
    st = C.c_int(0)
    h = lib().ora_laplacian(n, eu.shape[0], _p(eu, C.c_int32), _p(ev, C.c_int32), _p(w, C.c_double), C.byref(st))
    if h:
        lib().ora_csr_free(h)
    return st.value


def connected(A: Csr) -> bool:
    return bool(lib().ora_connected(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32)))


def colour(A: Csr, seed=0, level=0) -> np.ndarray:
    out = np.zeros(A.n, np.int32)
    lib().ora_colour(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), seed, level, _p(out, C.c_int32))
    return out


def colour_jp(A: Csr, seed=0, level=0):
    out = np.zeros(A.n, np.int32)
    r = lib().ora_colour_jp(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), seed, level, _p(out, C.c_int32))
    return out, r


def hash5(seed, stream, a, b, c) -> int:
    return int(lib().ora_hash5(seed, stream, a, b, c))


def unit_pm1(h) -> float:
    return float(lib().ora_unit_pm1(h))


def recombine(A: Csr, b, x, Xs, norm: int = 0):
    """Iterate recombination (eq. recomb) of the final iterate x with the
    saved iterates Xs ([n, th], th <= 2), minimising the residual 2-norm
    (norm 0, as printed) or the energy norm of the error (norm 1).
    Returns (y, alpha)."""
    Xs = np.ascontiguousarray(np.asarray(Xs, np.float64).reshape(A.n, -1))
    th = Xs.shape[1]
    y = np.zeros(A.n)
    alpha = np.zeros(th)
    lib().ora_recombine(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), _p(_f64(A.val), C.c_double),
                        _p(_f64(A.diag), C.c_double), _p(_f64(b), C.c_double), _p(_f64(x), C.c_double),
                        _p(Xs, C.c_double), th, int(norm), _p(y, C.c_double), _p(alpha, C.c_double))
    return y, alpha


def set_plain_rows(plain: bool):
    """Sum every row left to right (True) or in the fixed chunked order
    (False, the default that the GPU path shares)."""
    lib().ora_set_plain_rows(1 if plain else 0)


def row_reduce(terms) -> float:
    t = _f64(terms)
    return float(lib().ora_row_reduce(t.shape[0], _p(t, C.c_double)))


def gs(A: Csr, b, x, sweeps=1, k=1):
    x = _f64(x).copy()
    bb = _f64(b) if b is not None else None
    lib().ora_gs(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), _p(_f64(A.val), C.c_double),
                 _p(_f64(A.diag), C.c_double), _p(bb, C.c_double), _p(x, C.c_double), k, sweeps)
    return x


def gs32(A: Csr, val32, diag32, b, x, sweeps=1, k=1):
    x = np.ascontiguousarray(x, np.float32).copy()
    bb = np.ascontiguousarray(b, np.float32) if b is not None else None
    lib().ora_gs32(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32),
                   _p(np.ascontiguousarray(val32, np.float32), C.c_float),
                   _p(np.ascontiguousarray(diag32, np.float32), C.c_float),
                   _p(bb, C.c_float), _p(x, C.c_float), k, sweeps)
    return x


def residual(A: Csr, b, x):
    r = np.zeros(A.n)
    lib().ora_residual(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), _p(_f64(A.val), C.c_double),
                       _p(_f64(A.diag), C.c_double), _p(_f64(b), C.c_double), _p(_f64(x), C.c_double),
                       _p(r, C.c_double))
    return r


def gs_multicolour(A: Csr, colours, b, x):
    x = _f64(x).copy()
    lib().ora_gs_multicolour(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32),
                             _p(_f64(A.val), C.c_double), _p(_f64(A.diag), C.c_double),
                             _p(_i32(colours), C.c_int32), _p(_f64(b), C.c_double), _p(x, C.c_double))
    return x


def elim_select(A: Csr, maxdeg=4) -> np.ndarray:
    out = np.zeros(A.n, np.uint8)
    lib().ora_elim_select(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), maxdeg, _p(out, C.c_uint8))
    return out


def schur(A: Csr, inF):
    crank = np.zeros(A.n, np.int32)
    f = np.ascontiguousarray(inF, np.uint8)
    h = lib().ora_schur(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), _p(_f64(A.val), C.c_double),
                        _p(_f64(A.diag), C.c_double), _p(f, C.c_uint8), _p(crank, C.c_int32))
    return _export_csr_n(h, int(lib().ora_csr_n(h))), crank


def galerkin(A: Csr, agg, nc):
    h = lib().ora_galerkin(A.n, _p(_i64(A.ptr), C.c_int64), _p(_i32(A.col), C.c_int32), _p(_f64(A.val), C.c_double),
                           _p(_f64(A.diag), C.c_double), _p(_i32(agg), C.c_int32), nc)
    return _export_csr_n(h, nc)


class Level:
    pass


class Hierarchy:
    """An oracle hierarchy built from a COO edge list."""

    def __init__(self, n, eu, ev, w, **opts):
        self._eu, self._ev, self._w = _i32(eu), _i32(ev), _f64(w)
        self.opts = default_opts(**opts)
        st = C.c_int(0)
        self.h = lib().ora_setup(n, self._eu.shape[0], _p(self._eu, C.c_int32), _p(self._ev, C.c_int32),
                                 _p(self._w, C.c_double), C.byref(self.opts), C.byref(st))
        self.status = st.value
        if st.value:
            raise ValueError(f"oracle setup status {st.value}")
        self.n = n

    @classmethod
    def lgm(cls, side, **opts):
        """Lean geometric multigrid hierarchy of the side x side periodic
        Poisson grid (Section 5.3): red-black GS, 2 x 2 aggregation at every
        level, gamma at every level, flat mu = 2."""
        self = cls.__new__(cls)
        self.opts = default_opts(**opts)
        st = C.c_int(0)
        self.h = lib().ora_setup_lgm(side, C.byref(self.opts), C.byref(st))
        self.status = st.value
        if st.value:
            raise ValueError(f"oracle LGM setup status {st.value}")
        self.n = side * side
        return self

    def __del__(self):
        h = getattr(self, "h", None)
        if h and lib is not None:  # module globals may be gone at interpreter exit
            lib().ora_free(h)
            self.h = None

    @property
    def num_levels(self) -> int:
        return lib().ora_num_levels(self.h)

    def dims(self, l):
        d = np.zeros(8, np.int64)
        lib().ora_level_dims(self.h, l, _p(d, C.c_int64))
        return dict(n=int(d[0]), nnz=int(d[1]), type=int(d[2]), ncol=int(d[3]), nF=int(d[4]),
                    K=int(d[5]), stage=int(d[6]), gamma=float(lib().ora_level_gamma(self.h, l)))

    def level(self, l) -> Level:
        d = self.dims(l)
        n, nnz, ncol = d["n"], d["nnz"], d["ncol"]
        ptr = np.zeros(n + 1, np.int64)
        col = np.zeros(nnz, np.int32)
        val = np.zeros(nnz)
        diag = np.zeros(n)
        cptr = np.zeros(ncol + 1, np.int64)
        perm = np.zeros(n, np.int32)
        lib().ora_level_export(self.h, l, _p(ptr, C.c_int64), _p(col, C.c_int32), _p(val, C.c_double),
                               _p(diag, C.c_double), _p(cptr, C.c_int64), _p(perm, C.c_int32))
        L = Level()
        L.__dict__.update(d)
        L.A = Csr(ptr, col, val, diag)
        L.cptr, L.perm = cptr, perm
        if l > 0:
            nf = self.dims(l - 1)["n"]
            tr = np.zeros(nf, np.int32)
            lib().ora_transfer_export(self.h, l, _p(tr, C.c_int32))
            L.transfer = tr
        return L

    def agg_diag(self, l):
        d = self.dims(l)
        n, nnz, K = d["n"], d["nnz"], d["K"]
        tv = np.zeros(n * K)
        aff = np.zeros(nnz)
        ok = np.zeros(nnz, np.uint8)
        weak = np.zeros(nnz, np.uint8)
        hub = np.zeros(n, np.uint8)
        state = np.zeros(n, np.int32)
        scal = np.zeros(5)
        lib().ora_agg_export(self.h, l, _p(tv, C.c_double), _p(aff, C.c_double), _p(ok, C.c_uint8),
                             _p(weak, C.c_uint8), _p(hub, C.c_uint8), _p(state, C.c_int32), _p(scal, C.c_double))
        return dict(tv=tv.reshape(n, K), aff=aff, ok=ok, weak=weak, hub=hub, state=state,
                    delta1=scal[0], alpha1=scal[1], alpha2=scal[2], stage=int(scal[3]), rate=scal[4], K=K)

    def perm1(self):
        p = np.zeros(self.n, np.int32)
        lib().ora_perm1(self.h, _p(p, C.c_int32))
        return p

    @property
    def coarsest_relax(self) -> bool:
        return bool(lib().ora_coarsest_relax(self.h))

    def coarsest_solve(self, b):
        n = int(lib().ora_coarsest_n(self.h))
        x = np.zeros(n)
        lib().ora_coarsest_solve(self.h, _p(_f64(b), C.c_double), _p(x, C.c_double))
        return x

    def visit_counts(self):
        c = np.zeros(self.num_levels, np.int64)
        lib().ora_visit_counts(self.h, _p(c, C.c_int64))
        return c

    def solve(self, b, precision=0, x0=None):
        """Returns (x, info dict, residual history)."""
        x = _f64(x0).copy() if x0 is not None else np.zeros(self.n)
        info = np.zeros(4)
        hist = np.zeros(self.opts.max_cycles + 1)
        rc = lib().ora_solve(self.h, _p(_f64(b), C.c_double), _p(x, C.c_double), precision,
                             1 if x0 is not None else 0, _p(info, C.c_double), _p(hist, C.c_double))
        cyc = int(info[0])
        return x, dict(status=rc, cycles=cyc, rel_residual=info[1], acf=info[2], removed_mean=info[3]), hist[:cyc + 1]

    def cycle(self, b_perm, x_perm):
        x = _f64(x_perm).copy()
        lib().ora_cycle(self.h, _p(_f64(b_perm), C.c_double), _p(x, C.c_double))
        return x

    def adjoint(self, x, g):
        m = self._eu.shape[0]
        gb = np.zeros(self.n)
        gw = np.zeros(m)
        info = np.zeros(4)
        rc = lib().ora_adjoint(self.h, m, _p(self._eu, C.c_int32), _p(self._ev, C.c_int32), _p(_f64(x), C.c_double),
                               _p(_f64(g), C.c_double), _p(gb, C.c_double), _p(gw, C.c_double), _p(info, C.c_double))
        return gb, gw, rc
