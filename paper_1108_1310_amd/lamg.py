"""Python binding of the LAMG HIP library (include/lamg.h, include/lamg_test.h).

Argument marshalling only: every step of setup and solve runs in the HIP
kernels of ``libpaper_lamg.so``.  PyTorch supplies device memory and the
current stream.  There is no CPU fallback: loading fails loudly when the
library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpaper_lamg.so")

OK, E_INVALID_ARG, E_BAD_WEIGHT, E_NOT_CONNECTED, E_NOT_CONVERGED, E_BREAKDOWN, E_OUT_OF_MEMORY, E_DEVICE = range(8)
FP64, FP32_REFINE = 0, 1
EC_RECOMBINE, EC_FLAT_MU = 0, 1
RECOMB_RESIDUAL, RECOMB_ENERGY = 0, 1


# Device allocator hooks of lamg_options (alloc(bytes, ctx) -> ptr, dealloc(ptr, ctx)).
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("gamma", C.c_double), ("nu_pre", C.c_int), ("nu_post", C.c_int),
                ("tv_k_min", C.c_int), ("tv_k_max", C.c_int), ("tv_sweeps", C.c_int),
                ("q_max", C.c_double), ("mu", C.c_double), ("hub_factor", C.c_double),
                ("elim_max_degree", C.c_int), ("coarsest_max_n", C.c_int),
                ("weak_edge_ratio", C.c_double), ("elim_stop_frac", C.c_double), ("stage1_quantile", C.c_double),
                ("relax_fast_ratio", C.c_double), ("coarsest_sweeps", C.c_int), ("dense_max", C.c_int),
                ("tail_max_n", C.c_int),
                ("ec", C.c_int), ("precision", C.c_int), ("tol", C.c_double), ("max_cycles", C.c_int),
                ("warm_start", C.c_int), ("seed", C.c_uint64), ("stream", C.c_void_p),
                ("alloc", ALLOC_FN), ("dealloc", DEALLOC_FN), ("alloc_ctx", C.c_void_p),
                ("allow_negative_weights", C.c_int), ("recomb_norm", C.c_int)]


class Info(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("levels", C.c_int32), ("rel_residual", C.c_double), ("acf", C.c_double),
                ("removed_mean", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("bytes_moved", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LevelStats(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("n", C.c_int32), ("kind", C.c_int32), ("colours", C.c_int32),
                ("hub_colours", C.c_int32), ("in_tail", C.c_int32), ("reserved", C.c_int32), ("gamma", C.c_double),
                ("visits", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class LamgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = lib().lamg_last_error().decode() if status in (E_DEVICE, E_OUT_OF_MEMORY) else ""
        super().__init__(f"{where}: {lib().lamg_status_str(status).decode()} (status {status}) {detail}".rstrip())


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"LAMG HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "lamg_options_default": (None, [C.POINTER(Options)]),
            "lamg_setup": (C.c_int, [i64, i64, vp, vp, vp, C.POINTER(Options), C.POINTER(vp)]),
            "lamg_setup_lgm": (C.c_int, [i32, C.POINTER(Options), C.POINTER(vp)]),
            "lamg_solve": (C.c_int, [vp, vp, vp, C.POINTER(Info)]),
            "lamg_solve_batch": (C.c_int, [i32, C.POINTER(vp), C.POINTER(i32), C.POINTER(vp), C.POINTER(vp),
                                           C.POINTER(Info)]),
            "lamg_solve_batch_noalloc": (C.c_int, [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                                   C.POINTER(Info)]),
            "lamg_set_solve_options": (C.c_int, [vp, C.POINTER(Options)]),
            "lamg_edge_gradient": (C.c_int, [i64, vp, vp, vp, vp, vp, vp]),
            "lamg_eigs": (C.c_int, [vp, i32, vp, vp, d, i32, i32, C.POINTER(i32), vp]),
            "lamg_level_info": (C.c_int, [vp, i32, C.POINTER(LevelStats)]),
            "lamg_free": (None, [vp]),
            "lamg_status_str": (C.c_char_p, [C.c_int]),
            "lamg_last_error": (C.c_char_p, []),
            "lamg_t_num_levels": (C.c_int, [vp]),
            "lamg_t_coarsest_relax": (C.c_int, [vp]),
            "lamg_t_level_dims": (C.c_int, [vp, C.c_int, C.POINTER(i64)]),
            "lamg_t_level_gamma": (d, [vp, C.c_int]),
            "lamg_t_level_export": (C.c_int, [vp, C.c_int, vp, vp, vp, vp, vp, vp]),
            "lamg_t_transfer_export": (C.c_int, [vp, C.c_int, vp]),
            "lamg_t_agg_export": (C.c_int, [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]),
            "lamg_t_cycle": (C.c_int, [vp, vp, vp]),
            "lamg_t_mv_cycle": (C.c_int, [vp, i32, vp, vp]),
            "lamg_t_mv_columns": (C.c_int, [vp, i32, vp, vp, vp]),
            "lamg_t_batch_config": (C.c_int, [i32]),
            "lamg_t_coarsest_solve": (C.c_int, [vp, vp, vp]),
            "lamg_t_gs": (C.c_int, [i32, vp, vp, vp, vp, i32, vp, vp, vp, i32, vp]),
            "lamg_t_gs32": (C.c_int, [i32, vp, vp, vp, vp, i32, vp, vp, vp, i32, vp]),
            "lamg_t_residual": (C.c_int, [i32, vp, vp, vp, vp, vp, vp, vp, vp]),
            "lamg_t_colour": (C.c_int, [i32, vp, vp, u64, i32, vp, vp]),
            "lamg_t_hub_info": (C.c_int, [vp, i32, vp]),
            "lamg_t_level_gs": (C.c_int, [vp, i32, i32, i32, vp, vp]),
            "lamg_t_level_gs_zero": (C.c_int, [vp, i32, i32, i32, vp, vp]),
            "lamg_t_prof_enable": (None, [C.c_int]),
            "lamg_t_prof_read": (C.c_int, [C.c_int, C.POINTER(d), C.POINTER(i64), C.POINTER(i64)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> list[str]:
    return [n for n in ("lamg_options_default", "lamg_setup", "lamg_solve", "lamg_solve_batch",
                        "lamg_set_solve_options", "lamg_free", "lamg_status_str") if hasattr(lib(), n)]


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(rc: int, where: str):
    if rc != OK:
        raise LamgError(rc, where)


def options(**kw) -> Options:
    o = Options()
    lib().lamg_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _dev(t, dtype):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    return t.to(device="cuda", dtype=dtype).contiguous()


class TorchAllocator:
    """Device memory of hierarchies from torch's caching allocator (blocks on
    the current stream, 512-byte aligned), through the allocator hooks of
    lamg_options.  Keeps the callbacks alive and counts the live blocks."""

    def __init__(self):
        self.live = {}
        self.allocs = 0
        self.frees = 0

        def _alloc(nbytes, ctx):
            try:
                p = int(torch.cuda.caching_allocator_alloc(int(nbytes)))
            except RuntimeError:
                return None
            self.live[p] = int(nbytes)
            self.allocs += 1
            return p

        def _dealloc(ptr, ctx):
            self.live.pop(int(ptr), None)
            self.frees += 1
            torch.cuda.caching_allocator_delete(int(ptr))

        self.c_alloc = ALLOC_FN(_alloc)
        self.c_dealloc = DEALLOC_FN(_dealloc)


class Hierarchy:
    """A LAMG hierarchy of the Laplacian of a weighted undirected graph.

    ``eu, ev`` (int32) and ``w`` (float64) describe the edges (any order;
    duplicates of a pair are summed).  Arrays are moved to the GPU if needed.
    ``allocator``: a TorchAllocator to take the hierarchy's device memory
    from torch's caching allocator (default: the library's hipMalloc).
    """

    def __init__(self, n: int, eu, ev, w, allocator: "TorchAllocator" = None, **opts):
        eu, ev, w = _dev(eu, torch.int32), _dev(ev, torch.int32), _dev(w, torch.float64)
        self.opts = options(stream=_stream(), **opts)
        self._allocator = allocator
        if allocator is not None:
            self.opts.alloc = allocator.c_alloc
            self.opts.dealloc = allocator.c_dealloc
        h = C.c_void_p()
        rc = lib().lamg_setup(int(n), int(eu.numel()), _ptr(eu), _ptr(ev), _ptr(w), C.byref(self.opts), C.byref(h))
        _check(rc, "lamg_setup")
        self.h = h
        self.n = int(n)
        self.m = int(eu.numel())

    @classmethod
    def lgm(cls, side: int, allocator: "TorchAllocator" = None, **opts):
        """Lean geometric multigrid (Section 5.3) for the periodic Poisson
        problem on a side x side grid (node (i, j) = i + side j): red-black
        GS, 2 x 2 coarsening at every level, gamma at every level, flat
        mu = 2."""
        self = cls.__new__(cls)
        self.opts = options(stream=_stream(), **opts)
        self.opts.ec, self.opts.mu = EC_FLAT_MU, 2.0  # what the setup sets
        self._allocator = allocator
        if allocator is not None:
            self.opts.alloc = allocator.c_alloc
            self.opts.dealloc = allocator.c_dealloc
        h = C.c_void_p()
        _check(lib().lamg_setup_lgm(int(side), C.byref(self.opts), C.byref(h)), "lamg_setup_lgm")
        self.h = h
        self.n = int(side) * int(side)
        self.m = 2 * self.n
        return self

    def close(self):
        if getattr(self, "h", None):
            lib().lamg_free(self.h)
            self.h = None

    def __del__(self):
        # at interpreter exit the module globals (or torch, for a hierarchy on
        # torch's allocator) may already be gone; the process teardown
        # releases device memory then
        if _lib is None or not getattr(self, "h", None):
            return
        if getattr(self, "_allocator", None) is not None and sys.is_finalizing():
            return
        _lib.lamg_free(self.h)
        self.h = None

    def set_solve_options(self, **kw):
        for k, v in kw.items():
            setattr(self.opts, k, v)
        self.opts.stream = _stream()
        _check(lib().lamg_set_solve_options(self.h, C.byref(self.opts)), "lamg_set_solve_options")

    def solve(self, b, x=None, check: bool = True, **kw):
        """Solve A x = b - mean(b).  Returns (x, info dict)."""
        if kw:
            self.set_solve_options(**kw)
        b = _dev(b, torch.float64)
        warm = x is not None
        x = _dev(x, torch.float64).clone() if warm else torch.empty(self.n, dtype=torch.float64, device="cuda")
        if bool(self.opts.warm_start) != warm:
            self.set_solve_options(warm_start=int(warm))
        info = Info()
        rc = lib().lamg_solve(self.h, _ptr(b), _ptr(x), C.byref(info))
        if check and rc not in (OK, E_NOT_CONVERGED):
            _check(rc, "lamg_solve")
        d = info.as_dict()
        d["status"] = rc
        return x, d

    def eigs(self, k: int, x0, tol: float = 1e-8, max_iter: int = 200, cycles: int = 1, check: bool = True):
        """The k lowest eigenpairs of A on the zero-sum subspace (Section 6.4:
        LOBPCG preconditioned by LAMG cycles of this hierarchy).  ``x0``:
        [n, k] initial block (seeded random).  Returns (evals [k] float64
        host, X [n, k] on the GPU, info dict with iters, resid, status)."""
        X = _dev(x0, torch.float64).clone().contiguous()
        if X.dim() != 2 or X.shape[0] != self.n or X.shape[1] != k:
            raise ValueError("x0 must be [n, k]")
        ev = np.zeros(k, np.float64)
        rs = np.zeros(k, np.float64)
        it = C.c_int32(0)
        self.set_solve_options()  # the current stream
        rc = lib().lamg_eigs(self.h, int(k), _ptr(X), C.c_void_p(ev.ctypes.data), float(tol), int(max_iter),
                             int(cycles), C.byref(it), C.c_void_p(rs.ctypes.data))
        if check and rc not in (OK, E_NOT_CONVERGED):
            _check(rc, "lamg_eigs")
        return ev, X, {"iters": int(it.value), "resid": rs, "status": rc}

    def level_info(self, l: int) -> dict:
        """Per-level statistics: n, nnz, kind (0 finest, 1 elimination, 2
        aggregation), colours, hub_colours, in_tail, gamma, visits (bodies per
        finest-level cycle)."""
        st = LevelStats()
        _check(lib().lamg_level_info(self.h, l, C.byref(st)), "lamg_level_info")
        return st.as_dict()

    # ------------------------------------------------------ inspection (tests)
    @property
    def num_levels(self) -> int:
        return lib().lamg_t_num_levels(self.h)

    @property
    def coarsest_relax(self) -> bool:
        return bool(lib().lamg_t_coarsest_relax(self.h))

    def dims(self, l: int) -> dict:
        d = (C.c_int64 * 8)()
        _check(lib().lamg_t_level_dims(self.h, l, d), "lamg_t_level_dims")
        return dict(n=d[0], nnz=d[1], type=d[2], ncol=d[3], nF=d[4], K=d[5], stage=d[6], nlong=d[7],
                    gamma=float(lib().lamg_t_level_gamma(self.h, l)))

    def level(self, l: int) -> dict:
        d = self.dims(l)
        n, nnz, ncol = d["n"], d["nnz"], d["ncol"]
        rp = np.zeros(n + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        val = np.zeros(nnz)
        diag = np.zeros(n)
        cptr = np.zeros(ncol + 1, np.int32)
        perm = np.zeros(n, np.int32)
        vp = lambda a: C.c_void_p(a.ctypes.data)
        _check(lib().lamg_t_level_export(self.h, l, vp(rp), vp(ci), vp(val), vp(diag), vp(cptr), vp(perm)),
               "lamg_t_level_export")
        d.update(rp=rp, ci=ci, val=val, diag=diag, cptr=cptr, perm=perm)
        if l > 0:
            tr = np.zeros(self.dims(l - 1)["n"], np.int32)
            _check(lib().lamg_t_transfer_export(self.h, l, vp(tr)), "lamg_t_transfer_export")
            d["transfer"] = tr
        return d

    def agg_diag(self, l: int) -> dict:
        d = self.dims(l)
        n, nnz, K = d["n"], d["nnz"], d["K"]
        tv = np.zeros(n * K)
        aff = np.zeros(nnz)
        ok = np.zeros(nnz, np.uint8)
        weak = np.zeros(nnz, np.uint8)
        hub = np.zeros(n, np.uint8)
        st = np.zeros(n, np.int32)
        scal = np.zeros(5)
        vp = lambda a: C.c_void_p(a.ctypes.data)
        _check(lib().lamg_t_agg_export(self.h, l, vp(tv), vp(aff), vp(ok), vp(weak), vp(hub), vp(st), vp(scal)),
               "lamg_t_agg_export")
        return dict(tv=tv.reshape(n, K), aff=aff, ok=ok, weak=weak, hub=hub, state=st, delta1=scal[0],
                    alpha1=scal[1], alpha2=scal[2], stage=int(scal[3]), rate=scal[4], K=K)

    def hub_info(self, l: int) -> dict:
        """The hub split of level l's GS sweeps (k = -1: not taken)."""
        d = (C.c_int64 * 4)()
        _check(lib().lamg_t_hub_info(self.h, l, d), "lamg_t_hub_info")
        return dict(k=d[0], r0=d[1], n=d[2], nnz=d[3])

    def level_gs(self, l: int, b_perm, x_perm, sweeps: int = 1, precision: int = 0):
        """The solve's GS sweeps on level l (colour order), FP64 or FP32."""
        t = torch.float64 if precision == 0 else torch.float32
        b = None if b_perm is None else _dev(b_perm, t).contiguous()
        x = _dev(x_perm, t).clone().contiguous()
        _check(lib().lamg_t_level_gs(self.h, l, precision, sweeps, None if b is None else _ptr(b), _ptr(x)),
               "lamg_t_level_gs")
        return x

    def level_gs_zero(self, l: int, b_perm, sweeps: int = 1, precision: int = 0):
        """level_gs from a zero iterate with the first sweep's gathers of
        untouched colours skipped, as inside the cycle."""
        t = torch.float64 if precision == 0 else torch.float32
        b = None if b_perm is None else _dev(b_perm, t).contiguous()
        x = torch.empty(self.dims(l)["n"], dtype=t, device="cuda")
        _check(lib().lamg_t_level_gs_zero(self.h, l, precision, sweeps, None if b is None else _ptr(b), _ptr(x)),
               "lamg_t_level_gs_zero")
        return x

    def cycle(self, b_perm, x_perm):
        b = _dev(b_perm, torch.float64)
        x = _dev(x_perm, torch.float64).clone()
        _check(lib().lamg_t_cycle(self.h, _ptr(b), _ptr(x)), "lamg_t_cycle")
        return x

    def mv_cycle(self, B_perm, X_perm):
        """One FP64 multi-vector cycle on [n, k] colour-ordered blocks."""
        b = _dev(B_perm, torch.float64).contiguous()
        x = _dev(X_perm, torch.float64).clone().contiguous()
        _check(lib().lamg_t_mv_cycle(self.h, b.shape[1], _ptr(b), _ptr(x)), "lamg_t_mv_cycle")
        return x

    def solve_multi(self, B, X=None, **kw):
        """Solve A X[:, j] = B[:, j] - mean for every column of B [n, k] with
        the multi-vector cycle.  Returns (X, info of the worst column, per-column
        dict with cycles / rel_residual / removed_mean arrays, status)."""
        if kw:
            self.set_solve_options(**kw)
        B = _dev(B, torch.float64).contiguous()
        k = B.shape[1]
        Xs, infos, rc = solve_batch([self], [B], None if X is None else [X])
        cyc = np.zeros(k, np.int32)
        rel = np.zeros(k)
        rm = np.zeros(k)
        if k > 1:
            _check(lib().lamg_t_mv_columns(self.h, k, C.c_void_p(cyc.ctypes.data), C.c_void_p(rel.ctypes.data),
                                           C.c_void_p(rm.ctypes.data)), "lamg_t_mv_columns")
        return Xs[0], infos[0], dict(cycles=cyc, rel_residual=rel, removed_mean=rm), rc

    def coarsest_solve(self, b):
        b = _dev(b, torch.float64)
        x = torch.zeros_like(b)
        _check(lib().lamg_t_coarsest_solve(self.h, _ptr(b), _ptr(x)), "lamg_t_coarsest_solve")
        return x


def edge_gradient(eu, ev, x, lam):
    """grad_w[e] = -(lam_u - lam_v)(x_u - x_v) for every edge (HIP kernel)."""
    eu, ev = _dev(eu, torch.int32), _dev(ev, torch.int32)
    g = torch.empty(eu.numel(), dtype=torch.float64, device="cuda")
    _check(lib().lamg_edge_gradient(eu.numel(), _ptr(eu), _ptr(ev), _ptr(x.contiguous()), _ptr(lam.contiguous()),
                                    _ptr(g), _stream()), "lamg_edge_gradient")
    return g


class LaplacianSolve(torch.autograd.Function):
    """x = A(w)^+ (b - mean b) for the Laplacian of the graph (eu, ev, w).

    Backward (the adjoint reuses the hierarchy because A is symmetric):
    lam = A^+ (g - mean g); dL/db = lam; dL/dw_e = -(lam_u - lam_v)(x_u - x_v).
    The hierarchy is built in forward and kept on the context.  The adjoint
    solve uses the energy correction `adjoint_ec` (default 1, the flat mu of
    eq. galerkin2): its right-hand side is typically smooth (a function of x
    on a node subset), a regime in which recombination in the printed
    residual norm can stall on large graphs, and recombination in the energy
    norm (recomb_norm=RECOMB_ENERGY) is unreliable near the rounding floor of
    tight tolerances, while the flat correction converges.
    """

    @staticmethod
    def forward(ctx, b, w, eu, ev, n, opts=None):
        opts = dict(opts or {})
        ctx.adjoint_ec = int(opts.pop("adjoint_ec", EC_FLAT_MU))
        H = Hierarchy(int(n), eu, ev, w.detach(), **opts)
        x, info = H.solve(b.detach())
        if info["status"] != OK:
            raise LamgError(info["status"], "LaplacianSolve.forward")
        ctx.H = H
        ctx.save_for_backward(x, eu, ev)
        return x

    @staticmethod
    def backward(ctx, g):
        x, eu, ev = ctx.saved_tensors
        ctx.H.set_solve_options(ec=ctx.adjoint_ec)
        lam, info = ctx.H.solve(g.detach().to(torch.float64))
        if info["status"] != OK:
            raise LamgError(info["status"], "LaplacianSolve.backward")
        gw = edge_gradient(eu, ev, x, lam) if ctx.needs_input_grad[1] else None
        gb = lam if ctx.needs_input_grad[0] else None
        return gb, gw, None, None, None, None


def laplacian_solve(b, w, eu, ev, n, **opts):
    """Differentiable solve (see LaplacianSolve)."""
    return LaplacianSolve.apply(b, w, eu, ev, n, opts or None)


def solve_batch(hs: list[Hierarchy], Bs: list, Xs: list | None = None):
    """Batched solves: Bs[i] is [n_i] or [n_i, k_i] (row-major)."""
    cnt = len(hs)
    Bd = [_dev(b, torch.float64) for b in Bs]
    warm = Xs is not None
    Xd = [_dev(x, torch.float64).clone() for x in Xs] if warm else [torch.empty_like(b) for b in Bd]
    for h in hs:
        if bool(h.opts.warm_start) != warm:
            h.set_solve_options(warm_start=int(warm))
    nrhs = (C.c_int32 * cnt)(*[1 if b.dim() == 1 else b.shape[1] for b in Bd])
    hp = (C.c_void_p * cnt)(*[h.h.value for h in hs])
    bp = (C.c_void_p * cnt)(*[b.data_ptr() for b in Bd])
    xp = (C.c_void_p * cnt)(*[x.data_ptr() for x in Xd])
    infos = (Info * cnt)()
    rc = lib().lamg_solve_batch(cnt, hp, nrhs, bp, xp, infos)
    if rc not in (OK, E_NOT_CONVERGED):
        _check(rc, "lamg_solve_batch")
    return Xd, [i.as_dict() for i in infos], rc


NOALLOC_MAX_GRAPHS = 4096  # LAMG_NOALLOC_MAX_GRAPHS
BATCH_CONFIGS = 10  # LAMG_T_BATCH_CONFIGS


def solve_batch_noalloc(hs: list[Hierarchy], Bs: list, Xs: list | None = None):
    """Many graphs, one right-hand side each, through the allocation-free
    entry (lamg_solve_batch_noalloc): the same persistent launch as
    solve_batch, its buffers in the library's static device scratch.  The
    outputs are allocated here, before the call."""
    cnt = len(hs)
    Bd = [_dev(b, torch.float64) for b in Bs]
    warm = Xs is not None
    Xd = [_dev(x, torch.float64).clone() for x in Xs] if warm else [torch.empty_like(b) for b in Bd]
    for h in hs:
        if bool(h.opts.warm_start) != warm:
            h.set_solve_options(warm_start=int(warm))
    hp = (C.c_void_p * cnt)(*[h.h.value for h in hs])
    bp = (C.c_void_p * cnt)(*[b.data_ptr() for b in Bd])
    xp = (C.c_void_p * cnt)(*[x.data_ptr() for x in Xd])
    infos = (Info * cnt)()
    rc = lib().lamg_solve_batch_noalloc(cnt, hp, bp, xp, infos)
    if rc not in (OK, E_NOT_CONVERGED):
        msg = lib().lamg_last_error().decode()
        raise LamgError(rc, f"lamg_solve_batch_noalloc {msg}".rstrip())
    return Xd, [i.as_dict() for i in infos], rc


# ------------------------------------------------------------ kernel entries
def gs(rp, ci, val, diag, cptr, b, x, sweeps=1):
    """Multicolour GS sweeps on a colour-major DEVICE CSR (test entry point)."""
    n = x.numel()
    cp = np.ascontiguousarray(cptr, np.int32)
    f = lib().lamg_t_gs if x.dtype == torch.float64 else lib().lamg_t_gs32
    _check(f(n, _ptr(rp), _ptr(ci), _ptr(val), _ptr(diag), cp.shape[0] - 1, C.c_void_p(cp.ctypes.data), _ptr(b),
             _ptr(x), sweeps, _stream()), "lamg_t_gs")
    return x


def residual(rp, ci, val, diag, b, x):
    r = torch.empty_like(x)
    _check(lib().lamg_t_residual(x.numel(), _ptr(rp), _ptr(ci), _ptr(val), _ptr(diag), _ptr(b), _ptr(x), _ptr(r),
                                 _stream()), "lamg_t_residual")
    return r


def colour(rp, ci, n, seed=0, level=0):
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(lib().lamg_t_colour(n, _ptr(rp), _ptr(ci), seed, level, _ptr(out), _stream()), "lamg_t_colour")
    return out


KERNELS = {0: "gs_fp64", 1: "residual_fp64", 2: "gs_fp32", 3: "residual_fp32",
           4: "mv_gs_fp64", 5: "mv_residual_fp64", 6: "mv_gs_fp32", 7: "mv_residual_fp32",
           8: "hub_sweep_fp64", 9: "hub_sweep_fp32", 10: "restrict_agg_fp64", 11: "restrict_agg_fp32",
           12: "interp_agg_fp64", 13: "interp_agg_fp32", 14: "tail_fp64", 15: "tail_fp32"}


def prof_enable(on: bool = True):
    """Time the relaxation / residual kernels with HIP event spans on their
    stream (whole sweeps; see lamg_test.h)."""
    lib().lamg_t_prof_enable(1 if on else 0)


def prof_read(kernel: int) -> dict:
    ms, la, by = C.c_double(), C.c_int64(), C.c_int64()
    _check(lib().lamg_t_prof_read(kernel, C.byref(ms), C.byref(la), C.byref(by)), "lamg_t_prof_read")
    return dict(kernel=KERNELS[kernel], ms=ms.value, launches=la.value, bytes=by.value)
