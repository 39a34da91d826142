"""ctypes binding of libspx (include/spx.h): argument marshalling only.

Every step of the factorisation and solve runs in the HIP library; torch supplies the
device memory (through its caching allocator) and the stream.  If libspx.so is missing
the binding raises: there is no fallback path.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspx.so")

SPX_OK, SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_EAGAIN, SPX_EABORT, SPX_ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
ACC_R, ACC_RW, ACC_CW = 1, 2, 3
T_POTRF, T_TRSM, T_SYRK, T_GEMM, T_FTRSM, T_FGEMM, T_BTRSM, T_BGEMM, T_LOAD, T_STORE, T_INV = range(11)
TASK_NAMES = ["POTRF", "TRSM", "SYRK", "GEMM", "FTRSM", "FGEMM", "BTRSM", "BGEMM", "LOAD", "STORE", "INV"]
TILE_CANDIDATES = [32, 64, 128, 256, 512]
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
Q_SHARDED, Q_PRIORITY, Q_FIFO = 0, 1, 2
F_TRACE, F_SCALED, F_COMMUTE = 1, 2, 4
GEMM_COMMUTE = 1 << 16


class SpxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spx error {code}: {msg}")
        self.code = code


class NotPositiveDefinite(ArithmeticError):
    def __init__(self, info):
        super().__init__(f"leading minor of order {info} is not positive definite")
        self.info = info


class Access(ctypes.Structure):
    _fields_ = [("task", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("datum", ctypes.c_uint64)]


class Opts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("update_prec", ctypes.c_int32), ("queue_policy", ctypes.c_int32),
                ("num_wg", ctypes.c_int32), ("flags", ctypes.c_uint32), ("pad", ctypes.c_int32),
                ("shift", ctypes.c_double)]


class Refine(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("method", ctypes.c_int32),
                ("x_init", ctypes.c_int32), ("pad", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("method_used", ctypes.c_int32), ("eta_max", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("kernel_ms", ctypes.c_double), ("pack_ms", ctypes.c_double), ("idle_frac", ctypes.c_double),
                ("ntasks", ctypes.c_uint32), ("nparts", ctypes.c_uint32), ("num_wg", ctypes.c_uint32),
                ("tile", ctypes.c_uint32), ("device_allocs", ctypes.c_uint64)]


MODE_FP64, MODE_MIXED = 0, 1


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nrhs", ctypes.c_int64), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("where", ctypes.c_int32), ("tol", ctypes.c_double), ("tag", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("method_used", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("info", ctypes.c_int64), ("eta_max", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("tag", ctypes.c_uint64), ("batch_size", ctypes.c_int32),
                ("lane", ctypes.c_int32), ("t_ready", ctypes.c_double)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("num_wg", ctypes.c_int32),
                ("mixed_min_n", ctypes.c_int32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("bytes_in_use", ctypes.c_uint64), ("bytes_peak", ctypes.c_uint64),
                ("max_running", ctypes.c_uint64), ("busy_s", ctypes.c_double), ("pool_used_high", ctypes.c_uint64)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

# Every symbol include/spx.h declares, in declaration order.
EXPORTS = [
    "spx_last_error", "spx_ctx_create", "spx_ctx_destroy", "spx_graph_build", "spx_graph_info", "spx_graph_edges",
    "spx_graph_indegree", "spx_graph_to_dot", "spx_graph_destroy", "spx_cholesky_graph", "spx_gemm_graph",
    "spx_potrf_tiled",
    "spx_factor_info", "spx_factor_get_l", "spx_factor_destroy", "spx_gemm_tiled", "spx_run_graph", "spx_potrs", "spx_potrs_noalloc",
    "spx_backward_error",
    "spx_run_task", "spx_posv_batched", "spx_potrf_batched", "spx_potrs_batched", "spx_backward_error_batched",
    "spx_set_tile_table", "spx_tile_for",
    "spx_autotune_batched", "spx_server_create", "spx_submit", "spx_poll", "spx_server_now",
    "spx_server_get_stats", "spx_server_destroy", "spx_last_stats", "spx_ctx_set_flags", "spx_trace",
    "spx_trace_push",
]

_lib = None


def lib():
    """Loads libspx.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime; it must be the one libspx binds to (the library's
    # libamdhip64.so.7 dependency then resolves to the copy already loaded).  Loading
    # libspx first would bring in a second runtime that does not share torch's devices,
    # streams or memory.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "spx_last_error": (ctypes.c_char_p, []),
        "spx_ctx_create": (ctypes.c_int, [ctypes.c_int, vp, ALLOC_FN, FREE_FN, vp, P(vp)]),
        "spx_ctx_destroy": (None, [vp]),
        "spx_graph_build": (ctypes.c_int, [u32, P(Access), u64, P(i32), P(vp)]),
        "spx_graph_info": (ctypes.c_int, [vp, P(u32), P(u64)]),
        "spx_graph_edges": (ctypes.c_int, [vp, P(u32), P(u32), u64]),
        "spx_graph_indegree": (ctypes.c_int, [vp, P(u32), u32]),
        "spx_graph_to_dot": (ctypes.c_int, [vp, ctypes.c_char_p]),
        "spx_graph_destroy": (None, [vp]),
        "spx_run_graph": (ctypes.c_int, [vp, vp, u64, P(Opts)]),
        "spx_cholesky_graph": (ctypes.c_int, [i32, i32, P(vp), P(i32), u32]),
        "spx_gemm_graph": (ctypes.c_int, [i32, P(vp), P(i32), u32]),
        "spx_potrf_tiled": (ctypes.c_int, [vp, i64, vp, i64, P(Opts), P(vp), P(i64)]),
        "spx_factor_info": (ctypes.c_int, [vp, P(i64), P(i32), P(i64)]),
        "spx_factor_get_l": (ctypes.c_int, [vp, vp, vp, i64]),
        "spx_factor_destroy": (None, [vp]),
        "spx_gemm_tiled": (ctypes.c_int, [vp, i64, vp, i64, vp, i64, vp, i64, P(Opts)]),
        "spx_potrs": (ctypes.c_int, [vp, vp, i64, vp, i64, vp, i64, vp, i64, P(Refine), P(SolveStats)]),
        "spx_potrs_noalloc": (ctypes.c_int, [vp, vp, i64, vp, i64, vp, i64]),
        "spx_backward_error": (ctypes.c_int, [vp, i64, vp, i64, i64, vp, i64, vp, i64, P(ctypes.c_double)]),
        "spx_run_task": (ctypes.c_int, [vp, i32, i32, i32, i32, i32, i32, vp, vp, i32, P(i64)]),
        "spx_posv_batched": (ctypes.c_int, [vp, i32, P(i64), P(vp), P(i64), P(i64), P(vp), P(i64), P(vp), P(i64),
                                             P(Opts), P(i64), P(vp)]),
        "spx_potrf_batched": (ctypes.c_int, [vp, i32, P(i64), P(vp), P(i64), P(Opts), P(vp), P(i64)]),
        "spx_potrs_batched": (ctypes.c_int, [vp, i32, P(vp), P(i64), P(vp), P(i64), P(vp), P(i64), P(vp), P(i64),
                                              P(Refine), P(SolveStats)]),
        "spx_backward_error_batched": (ctypes.c_int, [vp, i32, P(i64), P(vp), P(i64), P(i64), P(vp), P(i64), P(vp),
                                                       P(i64), P(ctypes.c_double)]),
        "spx_set_tile_table": (ctypes.c_int, [vp, i32, i32, P(i64), P(i32)]),
        "spx_tile_for": (ctypes.c_int, [vp, i32, i64, P(i32)]),
        "spx_autotune_batched": (ctypes.c_int, [vp, i32, i32, P(i64), i32, i32, i32, P(i32), P(ctypes.c_double)]),
        "spx_server_create": (ctypes.c_int, [vp, ctypes.c_size_t, P(ServerOpts), P(vp)]),
        "spx_submit": (ctypes.c_int, [vp, P(Request), P(u64)]),
        "spx_poll": (ctypes.c_int, [vp, u64, P(Result)]),
        "spx_server_now": (ctypes.c_double, [vp]),
        "spx_server_get_stats": (ctypes.c_int, [vp, P(ServerStats)]),
        "spx_server_destroy": (None, [vp]),
        "spx_last_stats": (ctypes.c_int, [vp, P(Stats)]),
        "spx_ctx_set_flags": (ctypes.c_int, [vp, u32]),
        "spx_trace": (i64, [vp, P(u64), i64]),
        "spx_trace_push": (i64, [vp, P(u64), i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc):
    if rc < 0:
        raise SpxError(rc, lib().spx_last_error().decode(errors="replace"))
    return rc


# ------------------------------------------------------------------------------------------
# Graphs (host only)
# ------------------------------------------------------------------------------------------
class Graph:
    def __init__(self, handle, task_types=None):
        self._h = ctypes.c_void_p(handle)
        self.task_types = task_types

    @classmethod
    def build(cls, ntasks, accesses, priority=None):
        acc = (Access * max(len(accesses), 1))()
        for i, (t, m, d) in enumerate(accesses):
            acc[i].task, acc[i].mode, acc[i].datum = t, m, d
        pr = None
        if priority is not None:
            pr = (ctypes.c_int32 * ntasks)(*[int(p) for p in priority])
        h = ctypes.c_void_p()
        _check(lib().spx_graph_build(ntasks, acc, len(accesses), pr, ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def cholesky(cls, nt, with_solve=False, io=False, inverse=False, potrf_steps=1, commute=False):
        """The paper's program; io: with LOAD in front (and STORE at the end with the
        solve), as the batched calls run it; inverse: with the inversion tasks INV(k) after
        the factor and the substitution that uses them; potrf_steps > 1: each POTRF(k) as
        that many chained step tasks; commute: the updates as commutative writes."""
        h = ctypes.c_void_p()
        from math import comb
        T = nt + 2 * comb(nt, 2) + comb(nt, 3) + (2 * (nt + comb(nt, 2)) if with_solve else 0)
        if io:
            T += 2 if with_solve else 1
        if inverse:
            T += nt
        T += nt * (potrf_steps - 1)
        types = (ctypes.c_int32 * T)()
        flag = int(bool(with_solve)) | (2 if io else 0) | (4 if inverse else 0) | (8 if commute else 0) | (potrf_steps << 8)
        _check(lib().spx_cholesky_graph(nt, flag, ctypes.byref(h), types, T))
        return cls(h.value, np.array(types[:], dtype=np.int32))

    @classmethod
    def gemm(cls, nt, commute=False):
        """The tiled matrix product's program (spx_gemm_graph)."""
        h = ctypes.c_void_p()
        types = (ctypes.c_int32 * (nt ** 3))()
        _check(lib().spx_gemm_graph(nt | (GEMM_COMMUTE if commute else 0), ctypes.byref(h), types, nt ** 3))
        return cls(h.value, np.array(types[:], dtype=np.int32))

    def info(self):
        nt, ne = ctypes.c_uint32(), ctypes.c_uint64()
        _check(lib().spx_graph_info(self._h, ctypes.byref(nt), ctypes.byref(ne)))
        return nt.value, ne.value

    def edges(self):
        _, E = self.info()
        src = np.zeros(max(E, 1), np.uint32)
        dst = np.zeros(max(E, 1), np.uint32)
        _check(lib().spx_graph_edges(self._h, src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                     dst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), E))
        return np.stack([src[:E], dst[:E]], axis=1)

    def indegree(self):
        T, _ = self.info()
        d = np.zeros(max(T, 1), np.uint32)
        _check(lib().spx_graph_indegree(self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), T))
        return d[:T]

    def to_dot(self, path):
        _check(lib().spx_graph_to_dot(self._h, os.fsencode(path)))

    def close(self):
        if self._h:
            lib().spx_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------
# Device context, factor, solve
# ------------------------------------------------------------------------------------------
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A libspx context on one GPU, using torch's current stream and caching allocator."""

    def __init__(self, device=0, stream=None, torch_allocator=True):
        import torch

        self.torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        import weakref

        self._factors = weakref.WeakSet()
        if torch_allocator:
            dev = device

            def _alloc(nbytes, strm, user):
                return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(strm or 0) or stream)

            def _free(p, strm, user):
                torch.cuda.caching_allocator_delete(p)

            self._alloc_cb, self._free_cb = ALLOC_FN(_alloc), FREE_FN(_free)
        else:
            self._alloc_cb, self._free_cb = ALLOC_FN(), FREE_FN()
        h = ctypes.c_void_p()
        _check(lib().spx_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), self._alloc_cb, self._free_cb, None,
                                    ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h:
            for f in list(self._factors):  # a factor must not outlive its context
                f.close()
            lib().spx_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, t, name):
        torch = self.torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if t.stride(-1) != 1:
            raise ValueError(f"{name} must have unit stride along its last dimension")
        return t

    def potrf(self, A, tile=0, update_prec=PREC_FP64, queue_policy=Q_SHARDED, num_wg=0, flags=0, shift=None):
        """Factors the lower triangle of the SPD matrix A (n x n float64 on the device).
        shift (not None): factor D^-1/2 A D^-1/2 + shift I instead (a preconditioner)."""
        A = self._dev(A, "A")
        n = A.shape[0]
        if A.dim() != 2 or A.shape[1] != n:
            raise ValueError("A must be square")
        if shift is not None:
            flags |= F_SCALED
        o = Opts(tile, update_prec, queue_policy, num_wg, flags, 0, float(shift or 0.0))
        h = ctypes.c_void_p()
        info = ctypes.c_int64()
        _check(lib().spx_potrf_tiled(self._h, n, _ptr(A), A.stride(0), ctypes.byref(o), ctypes.byref(h),
                                     ctypes.byref(info)))
        if info.value:
            raise NotPositiveDefinite(info.value)
        return Factor(self, h.value)

    def potrs(self, F, B, X=None, A=None, tol=0.0, max_iter=0, method=0, return_stats=False, x_init=False):
        """Solves A X = B with the factor (B: n or n x nrhs float64 on the device)."""
        torch = self.torch
        B = self._dev(B, "B")
        vec = B.dim() == 1
        B2 = B.reshape(B.shape[0], -1)
        if X is None:
            X2 = torch.empty_like(B2)
        else:
            X2 = self._dev(X, "X").reshape(B2.shape)
        ref = None
        if method:
            ref = Refine(tol, max_iter, method, int(x_init), 0)
        st = SolveStats()
        a_ptr, lda = (None, 0) if A is None else (_ptr(self._dev(A, "A")), A.stride(0))
        _check(lib().spx_potrs(self._h, F._h, B2.shape[1], _ptr(B2), B2.stride(0), _ptr(X2), X2.stride(0), a_ptr, lda,
                               ctypes.byref(ref) if ref is not None else None, ctypes.byref(st)))
        out = X2.reshape(B.shape) if vec else X2
        if return_stats:
            return out, {"iters": st.iters, "method_used": st.method_used, "eta_max": st.eta_max}
        return out

    def run_graph(self, graph, spin_ticks, queue_policy=Q_SHARDED, num_wg=0, flags=0):
        """Runs every task of graph as an empty task of spin_ticks device clock ticks
        (100 MHz) with the graph's dependencies (spx_run_graph); returns the stats."""
        o = Opts(0, PREC_FP64, queue_policy, num_wg, flags, 0, 0.0)
        _check(lib().spx_run_graph(self._h, graph._h, int(spin_ticks), ctypes.byref(o)))
        return self.stats()

    def gemm(self, A, B, C, tile=0, queue_policy=Q_SHARDED, num_wg=0, flags=0):
        """C <- C + A B in place (spx_gemm_tiled); returns C."""
        for t, nm in ((A, "A"), (B, "B"), (C, "C")):
            self._dev(t, nm)
        n = A.shape[0]
        if A.shape != (n, n) or B.shape != (n, n) or C.shape != (n, n):
            raise ValueError("A, B and C must be n x n")
        o = Opts(tile, PREC_FP64, queue_policy, num_wg, flags, 0, 0.0)
        _check(lib().spx_gemm_tiled(self._h, n, _ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(C), C.stride(0),
                                    ctypes.byref(o)))
        return C

    def potrs_noalloc(self, F, B, X):
        """The allocation-free solve (spx_potrs_noalloc): X = A^{-1} B into the caller's X
        (same shape as B), with no device allocation; returns X."""
        n = F.n
        B2 = self._dev(B, "B").reshape(n, -1)
        X2 = self._dev(X, "X").reshape(n, -1)
        if X2.shape != B2.shape:
            raise ValueError("X must have the shape of B")
        _check(lib().spx_potrs_noalloc(self._h, F._h, B2.shape[1], _ptr(B2), B2.stride(0), _ptr(X2), X2.stride(0)))
        return X

    def backward_error(self, A, X, B):
        A = self._dev(A, "A")
        X2 = self._dev(X, "X").reshape(A.shape[0], -1)
        B2 = self._dev(B, "B").reshape(A.shape[0], -1)
        q = X2.shape[1]
        eta = (ctypes.c_double * q)()
        _check(lib().spx_backward_error(self._h, A.shape[0], _ptr(A), A.stride(0), q, _ptr(X2), X2.stride(0), _ptr(B2),
                                        B2.stride(0), eta))
        return np.array(eta[:])

    def run_task(self, type_, i, j, k, nt, b, tiles, rhs=None, nrhs=0):
        """Runs one task on packed tile storage (see spx_run_task); returns info."""
        tiles = self._dev(tiles, "tiles")
        r = None if rhs is None else _ptr(self._dev(rhs, "rhs"))
        info = ctypes.c_int64()
        _check(lib().spx_run_task(self._h, type_, i, j, k, nt, b, _ptr(tiles), r, nrhs, ctypes.byref(info)))
        return info.value

    # -------------------------------------------------------------- batched (one launch)
    def _batch_arrays(self, As, Bs=None, Xs=None):
        k = len(As)
        i64a = ctypes.c_int64 * k
        vpa = ctypes.c_void_p * k
        n = i64a(*[a.shape[0] for a in As])
        lda = i64a(*[a.stride(0) for a in As])
        pa = vpa(*[a.data_ptr() for a in As])
        for a in As:
            self._dev(a, "A")
            if a.dim() != 2 or a.shape[0] != a.shape[1]:
                raise ValueError("every A must be square")
        out = [n, pa, lda]
        if Bs is not None:
            out += [i64a(*[b.shape[1] for b in Bs]), vpa(*[b.data_ptr() for b in Bs]), i64a(*[b.stride(0) for b in Bs]),
                    vpa(*[x.data_ptr() for x in Xs]), i64a(*[x.stride(0) for x in Xs])]
        return out

    def posv_batched(self, As, Bs, tile=0, update_prec=PREC_FP64, queue_policy=Q_SHARDED, num_wg=0, flags=0,
                     Xs=None, keep=False):
        """Factors and solves every (A_i, B_i) in one launch; returns (Xs, info array), and
        with keep=True also the list of factors (None where info > 0).
        B_i: n_i x q_i float64 on the device (2-D)."""
        torch = self.torch
        if len(As) != len(Bs) or not As:
            raise ValueError("need equally many matrices and right-hand sides")
        Bs = [self._dev(b, "B") for b in Bs]
        if any(b.dim() != 2 or b.shape[0] != a.shape[0] for a, b in zip(As, Bs)):
            raise ValueError("B_i must be n_i x q_i")
        if Xs is None:
            Xs = [torch.empty_like(b) for b in Bs]
        n, pa, lda, q, pb, ldb, px, ldx = self._batch_arrays(As, Bs, Xs)
        info = (ctypes.c_int64 * len(As))()
        o = Opts(tile, update_prec, queue_policy, num_wg, flags)
        hs = (ctypes.c_void_p * len(As))() if keep else None
        _check(lib().spx_posv_batched(self._h, len(As), n, pa, lda, q, pb, ldb, px, ldx, ctypes.byref(o), info, hs))
        if keep:
            return Xs, np.array(info[:], dtype=np.int64), [Factor(self, h) if h else None for h in hs]
        return Xs, np.array(info[:], dtype=np.int64)

    def potrf_batched(self, As, tile=0, update_prec=PREC_FP64, queue_policy=Q_SHARDED, num_wg=0, flags=0):
        """Factors every A_i in one launch; returns (list of Factor or None, info array)."""
        if not As:
            raise ValueError("empty batch")
        n, pa, lda = self._batch_arrays(As)
        k = len(As)
        hs = (ctypes.c_void_p * k)()
        info = (ctypes.c_int64 * k)()
        o = Opts(tile, update_prec, queue_policy, num_wg, flags)
        _check(lib().spx_potrf_batched(self._h, k, n, pa, lda, ctypes.byref(o), hs, info))
        fs = [Factor(self, h) if h else None for h in hs]
        return fs, np.array(info[:], dtype=np.int64)

    def potrs_batched(self, Fs, Bs, As=None, tol=0.0, max_iter=0, method=0, Xs=None, x_init=False):
        """Solves with existing factors in batched launches (optionally refined against the
        original matrices As).  Returns (Xs, stats list)."""
        torch = self.torch
        k = len(Fs)
        if k == 0 or len(Bs) != k or (As is not None and len(As) != k):
            raise ValueError("need one right-hand side (and matrix) per factor")
        Bs = [self._dev(b, "B") for b in Bs]
        if Xs is None:
            Xs = [torch.empty_like(b) for b in Bs]
        i64a, vpa = ctypes.c_int64 * k, ctypes.c_void_p * k
        fh = vpa(*[f._h.value for f in Fs])
        q = i64a(*[b.shape[1] for b in Bs])
        pb, ldb = vpa(*[b.data_ptr() for b in Bs]), i64a(*[b.stride(0) for b in Bs])
        px, ldx = vpa(*[x.data_ptr() for x in Xs]), i64a(*[x.stride(0) for x in Xs])
        pa = lda = None
        if As is not None:
            pa, lda = vpa(*[self._dev(a, "A").data_ptr() for a in As]), i64a(*[a.stride(0) for a in As])
        ref = Refine(tol, max_iter, method, int(x_init), 0)
        st = (SolveStats * k)()
        _check(lib().spx_potrs_batched(self._h, k, fh, q, pb, ldb, px, ldx, pa, lda, ctypes.byref(ref), st))
        return Xs, [{"iters": s.iters, "method_used": s.method_used, "eta_max": s.eta_max} for s in st]

    def backward_error_batched(self, As, Xs, Bs):
        k = len(As)
        i64a, vpa = ctypes.c_int64 * k, ctypes.c_void_p * k
        eta = (ctypes.c_double * k)()
        _check(lib().spx_backward_error_batched(
            self._h, k, i64a(*[a.shape[0] for a in As]), vpa(*[a.data_ptr() for a in As]),
            i64a(*[a.stride(0) for a in As]), i64a(*[b.shape[1] for b in Bs]), vpa(*[x.data_ptr() for x in Xs]),
            i64a(*[x.stride(0) for x in Xs]), vpa(*[b.data_ptr() for b in Bs]), i64a(*[b.stride(0) for b in Bs]), eta))
        return np.array(eta[:])

    def set_tile_table(self, prec, table):
        """table: list of (n_max, tile), n_max increasing ([] clears)."""
        k = len(table)
        nm = (ctypes.c_int64 * max(k, 1))(*[int(a) for a, _ in table])
        tl = (ctypes.c_int32 * max(k, 1))(*[int(b) for _, b in table])
        _check(lib().spx_set_tile_table(self._h, prec, k, nm, tl))

    def tile_for(self, prec, n):
        t = ctypes.c_int32()
        _check(lib().spx_tile_for(self._h, prec, n, ctypes.byref(t)))
        return t.value

    def autotune_batched(self, sizes, prec=PREC_FP64, nrhs=4, copies=256, reps=2):
        """Times every candidate tile per probe size (see spx_autotune_batched); the result
        becomes the context's table.  Returns {"prec", "table": [(n_max, tile)], "ms": ...}."""
        k = len(sizes)
        sz = (ctypes.c_int64 * k)(*[int(s) for s in sizes])
        best = (ctypes.c_int32 * k)()
        ms = (ctypes.c_double * (5 * k))()
        _check(lib().spx_autotune_batched(self._h, prec, k, sz, nrhs, copies, reps, best, ms))
        return {"prec": prec, "nrhs": nrhs, "copies": copies,
                "table": [(int(s), int(b)) for s, b in zip(sizes, best)],
                "ms": {int(s): dict(zip(TILE_CANDIDATES, ms[5 * i:5 * i + 5])) for i, s in enumerate(sizes)}}

    def stats(self):
        s = Stats()
        _check(lib().spx_last_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def set_flags(self, flags):
        """Context-wide launch flags (F_TRACE: trace every later launch; 0: off)."""
        _check(lib().spx_ctx_set_flags(self._h, flags))

    def trace(self):
        n = _check(lib().spx_trace(self._h, None, 0))
        rec = np.zeros(max(n, 1) * 4, np.uint64)
        _check(lib().spx_trace(self._h, rec.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n))
        return rec[: 4 * n].reshape(n, 4)

    def trace_push(self):
        """Per task of the last traced launch: the device tick it was pushed (0: a root)."""
        n = _check(lib().spx_trace_push(self._h, None, 0))
        out = np.zeros(max(n, 1), np.uint64)
        _check(lib().spx_trace_push(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n))
        return out[:n]


class Factor:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self._h = ctypes.c_void_p(handle)
        ctx._factors.add(self)
        n, b, npad = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().spx_factor_info(self._h, ctypes.byref(n), ctypes.byref(b), ctypes.byref(npad)))
        self.n, self.tile, self.n_padded = n.value, b.value, npad.value

    def L(self):
        torch = self.ctx.torch
        out = torch.empty((self.n, self.n), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        _check(lib().spx_factor_get_l(self.ctx._h, self._h, _ptr(out), out.stride(0)))
        return out

    def close(self):
        if self._h and self.ctx._h:
            lib().spx_factor_destroy(self._h)
        self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (spx_server_*): submit SPD solve requests, poll for results.

    Tensors passed to submit() must stay alive and unmodified until the ticket is done;
    the server keeps a reference to them until poll() returns the result."""

    def __init__(self, ctx, hbm_budget_bytes, lanes=2, max_batch=0, num_wg=0, mixed_min_n=0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        o = ServerOpts(lanes, max_batch, num_wg, mixed_min_n)
        _check(lib().spx_server_create(ctx._h, int(hbm_budget_bytes), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, A, B, X, mode=MODE_FP64, tol=0.0, tag=0):
        """A: n x n, B and X: n x nrhs float64, all on the device, all on the host, or A and
        B on the device and X on the host (host tensors are best pinned).  Returns the ticket."""
        torch = self.ctx.torch
        ts = (A, B, X)
        if not all(isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1
                   for t in ts):
            raise TypeError("A, B, X must be 2-D float64 tensors with unit column stride")
        if A.is_cuda and B.is_cuda and not X.is_cuda:
            where = 2  # inputs on the device, the solution to host memory
        elif all(t.is_cuda == A.is_cuda for t in ts):
            where = 1 if A.is_cuda else 0
        else:
            raise ValueError("A, B, X: all on the device, all on the host, or A and B on the device and X on the host")
        r = Request(A.shape[0], B.shape[1], A.data_ptr(), B.data_ptr(), X.data_ptr(), A.stride(0), B.stride(0),
                    X.stride(0), mode, where, tol, tag)
        t = ctypes.c_uint64()
        _check(lib().spx_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = ts
        return t.value

    def poll(self, ticket):
        """None while running, else a dict with the result (the ticket is then released)."""
        r = Result()
        rc = lib().spx_poll(self._h, ticket, ctypes.byref(r))
        if rc == SPX_EAGAIN:
            return None
        _check(rc)
        self._keep.pop(ticket, None)
        return {k: getattr(r, k) for k, _ in Result._fields_}

    def wait(self, ticket, timeout=600.0):
        import time
        t0 = time.monotonic()
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() - t0 > timeout:
                raise TimeoutError(f"ticket {ticket} not done after {timeout} s")
            time.sleep(0.0002)

    def now(self):
        return lib().spx_server_now(self._h)

    def stats(self):
        s = ServerStats()
        _check(lib().spx_server_get_stats(self._h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().spx_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
