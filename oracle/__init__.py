"""Oracle for the tile-DAG Cholesky path: ctypes wrapper around liboracle.so.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg of
the benchmark import this package; the product library never does.

Every matrix argument is a numpy (n, n) float64 array holding a symmetric matrix in the
usual row-major view; only its lower triangle is read (LAPACK 'L' convention).  The C
side works on column-major storage; the conversion happens here.

Functions and the passages they follow (Specx, arXiv 2308.15964):
  dag_edges, cholesky_dag  - STF dependency inference (Sec. 2.1, Sec. 4.1, Sec. 4.7),
                             pairwise definition of RAW / WAR / WAW edges.
  cholesky                 - tiled Cholesky with POTRF / TRSM / SYRK / GEMM tasks in FP64
                             (Sec. 5.2), run by a sequential STF executor in a chosen
                             topological order, or by a thread pool; optional solve.
  gemm_program, gemm_dag, gemm, gemm_entries
                           - the tiled matrix product C + A B of the GEMM application
                             (Sec. 5.2), one task per tile triple, same executors.
  factor_residual, factor_residual_probe, factor_residual_vectors, backward_error,
  entry_check
                           - checks of a factor and a solution against the definitions
                             A = L L^T and A x = b, with compensated dot products.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

R, RW = 1, 2


class _Access(ctypes.Structure):
    _fields_ = [("task", ctypes.c_uint32), ("mode", ctypes.c_uint32), ("datum", ctypes.c_uint64)]


class _Task(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("i", ctypes.c_int32), ("j", ctypes.c_int32), ("k", ctypes.c_int32)]


TASK_NAMES = ["POTRF", "TRSM", "SYRK", "GEMM", "FTRSM", "FGEMM", "BTRSM", "BGEMM", "MGEMM"]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        i64, u64, u32, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_double)
        L.orc_dag_edges.restype = i64
        L.orc_dag_edges.argtypes = [u32, ctypes.POINTER(_Access), u64, ctypes.POINTER(u32),
                                    ctypes.POINTER(u32), u64, ctypes.POINTER(u64)]
        L.orc_cholesky_program.restype = i64
        L.orc_cholesky_program.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Task),
                                           ctypes.POINTER(_Access), ctypes.POINTER(u64)]
        L.orc_cholesky_dag.restype = i64
        L.orc_cholesky_dag.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(u32), ctypes.POINTER(u32),
                                       u64, ctypes.POINTER(u64), ctypes.POINTER(i64)]
        L.orc_cholesky.restype = i64
        L.orc_cholesky.argtypes = [i64, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int, u64, ctypes.c_int,
                                   ctypes.POINTER(i64), i64, ctypes.POINTER(u32), ctypes.POINTER(i64), ctypes.c_int]
        L.orc_run_task.restype = i64
        L.orc_run_task.argtypes = [ctypes.c_int] * 4 + [dp, i64, ctypes.c_int, dp, ctypes.c_int]
        L.orc_factor_residual.restype = ctypes.c_double
        L.orc_factor_residual.argtypes = [dp, dp, i64]
        L.orc_factor_residual_probe.restype = ctypes.c_double
        L.orc_factor_residual_probe.argtypes = [dp, dp, i64, ctypes.c_int, u64]
        L.orc_factor_residual_vectors.restype = ctypes.c_double
        L.orc_factor_residual_vectors.argtypes = [dp, dp, i64, dp, ctypes.c_int]
        L.orc_backward_error.restype = None
        L.orc_backward_error.argtypes = [dp, i64, dp, dp, i64, ctypes.c_int, ctypes.c_double, dp]
        L.orc_norm_inf_sym.restype = ctypes.c_double
        L.orc_norm_inf_sym.argtypes = [dp, i64]
        L.orc_factor_entry_check.restype = ctypes.c_double
        L.orc_factor_entry_check.argtypes = [dp, dp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), i64]
        L.orc_gemm_program.restype = i64
        L.orc_gemm_program.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Task), ctypes.POINTER(_Access),
                                       ctypes.POINTER(u64)]
        L.orc_gemm.restype = i64
        L.orc_gemm.argtypes = [i64, ctypes.c_int, dp, ctypes.c_int, u64, ctypes.c_int, ctypes.POINTER(i64),
                               ctypes.POINTER(u32), ctypes.POINTER(i64), ctypes.c_int]
        L.orc_gemm_dag.restype = i64
        L.orc_gemm_dag.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(u32), ctypes.POINTER(u32), u64,
                                   ctypes.POINTER(u64), ctypes.POINTER(i64)]
        L.orc_gemm_entries.restype = None
        L.orc_gemm_entries.argtypes = [dp, dp, dp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), i64, dp]
        L.orc_dot2.restype = ctypes.c_double
        L.orc_dot2.argtypes = [dp, dp, i64]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _lower_cm(A):
    """Lower triangle of the row-major view, stored column-major (a fresh copy)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    assert A.shape == (n, n)
    return np.asfortranarray(np.tril(A))


def _cm_to_lower(a_cm):
    return np.ascontiguousarray(np.tril(a_cm))


def dag_edges(ntasks, accesses):
    """accesses: sequence of (task, mode, datum).  Returns (edges (E,2) uint32 sorted by
    (src, dst), {'RAW','WAR','WAW': count})."""
    acc = (_Access * max(len(accesses), 1))()
    for i, (t, m, d) in enumerate(accesses):
        acc[i].task, acc[i].mode, acc[i].datum = t, m, d
    kinds = (ctypes.c_uint64 * 3)()
    E = lib().orc_dag_edges(ntasks, acc, len(accesses), None, None, 0, kinds)
    if E < 0:
        raise ValueError("invalid access list")
    src = np.zeros(max(E, 1), np.uint32)
    dst = np.zeros(max(E, 1), np.uint32)
    lib().orc_dag_edges(ntasks, acc, len(accesses), src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                        dst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), E, kinds)
    return np.stack([src[:E], dst[:E]], axis=1), {"RAW": kinds[0], "WAR": kinds[1], "WAW": kinds[2]}


def cholesky_program(nt, with_solve=False, commute=False):
    """The oracle's task program: ([(name, i, j, k)], [(task, mode, datum)]); commute: the
    updates are commutative writes."""
    na = ctypes.c_uint64()
    fl = int(bool(with_solve)) | (0x100 if commute else 0)
    T = lib().orc_cholesky_program(nt, fl, None, None, ctypes.byref(na))
    tasks = (_Task * max(T, 1))()
    acc = (_Access * max(na.value, 1))()
    lib().orc_cholesky_program(nt, fl, tasks, acc, ctypes.byref(na))
    return ([(TASK_NAMES[t.type], t.i, t.j, t.k) for t in tasks[:T]],
            [(a.task, a.mode, a.datum) for a in acc[: na.value]])


def cholesky_dag(nt, with_solve=False, commute=False):
    """Edges of the oracle's own right-looking Cholesky (+ solve) task program."""
    kinds = (ctypes.c_uint64 * 3)()
    T = ctypes.c_int64()
    fl = int(bool(with_solve)) | (0x100 if commute else 0)
    E = lib().orc_cholesky_dag(nt, fl, None, None, 0, kinds, ctypes.byref(T))
    src = np.zeros(max(E, 1), np.uint32)
    dst = np.zeros(max(E, 1), np.uint32)
    lib().orc_cholesky_dag(nt, fl, src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                           dst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), E, kinds, ctypes.byref(T))
    return T.value, np.stack([src[:E], dst[:E]], axis=1), {"RAW": kinds[0], "WAR": kinds[1], "WAW": kinds[2]}


ORDER_INSERTION, ORDER_RANDOM, ORDER_PRIORITY, ORDER_GIVEN = 0, 1, 2, 3


def cholesky(A, nb, B=None, order=ORDER_INSERTION, seed=0, nthreads=1, limit=0, drop_edge=None,
             return_order=False, commute=False, given=None):
    """Tile Cholesky (tile size nb, n % nb == 0) of the lower triangle of A, optionally
    followed by the solve of A X = B.  Returns (L, X or None, info[, order]); info is 0
    or the 1-based global column of the first non-positive pivot.  commute: the updates
    are commutative writes (sequential only).  order=ORDER_GIVEN runs the task order
    `given` (ValueError if it is not a valid order of the program's DAG)."""
    a = _lower_cm(A)
    n = a.shape[0]
    if n % nb:
        raise ValueError("n must be a multiple of nb")
    y = None
    nrhs = 0
    if B is not None:
        B = np.asarray(B, dtype=np.float64)
        vec = B.ndim == 1
        y = np.asfortranarray(B.reshape(n, -1).copy())
        nrhs = y.shape[1]
    from math import comb

    nt = n // nb
    T = nt + 2 * comb(nt, 2) + comb(nt, 3) + (2 * (nt + comb(nt, 2)) if nrhs else 0)
    ordbuf = np.full(T, -1, np.int64)
    if order == ORDER_GIVEN:
        ordbuf[:] = np.asarray(given, np.int64)
    nrun = ctypes.c_int64(0)
    de = None
    if drop_edge is not None:
        de = (ctypes.c_uint32 * 2)(int(drop_edge[0]), int(drop_edge[1]))
    info = lib().orc_cholesky(n, nb, _dp(a), _dp(y) if y is not None else None, nrhs, order, seed, nthreads,
                              ordbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), limit, de, ctypes.byref(nrun),
                              int(bool(commute)))
    if info == -2:
        raise ValueError("not a valid order of the program's DAG")
    if info < 0:
        raise RuntimeError("oracle failed")
    L = _cm_to_lower(a)
    X = None
    if y is not None:
        X = np.ascontiguousarray(y)
        if vec:
            X = X.reshape(n)
    out = (L, X, int(info))
    if return_order:
        out = out + (ordbuf[: nrun.value].copy(),)
    return out


def gemm_program(nt, commute=False):
    """The oracle's GEMM task program: ([(name, i, j, k)], [(task, mode, datum)])."""
    na = ctypes.c_uint64()
    T = lib().orc_gemm_program(nt, int(bool(commute)), None, None, ctypes.byref(na))
    tasks = (_Task * max(T, 1))()
    acc = (_Access * max(na.value, 1))()
    lib().orc_gemm_program(nt, int(bool(commute)), tasks, acc, ctypes.byref(na))
    return ([(TASK_NAMES[t.type], t.i, t.j, t.k) for t in tasks[:T]],
            [(a.task, a.mode, a.datum) for a in acc[: na.value]])


def gemm_dag(nt, commute=False):
    """Edges of the GEMM program by the pairwise definition: (T, edges, kinds)."""
    kinds = (ctypes.c_uint64 * 3)()
    T = ctypes.c_int64()
    E = lib().orc_gemm_dag(nt, int(bool(commute)), None, None, 0, kinds, ctypes.byref(T))
    src = np.zeros(max(E, 1), np.uint32)
    dst = np.zeros(max(E, 1), np.uint32)
    lib().orc_gemm_dag(nt, int(bool(commute)), src.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                       dst.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), E, kinds, ctypes.byref(T))
    return T.value, np.stack([src[:E], dst[:E]], axis=1), {"RAW": kinds[0], "WAR": kinds[1], "WAW": kinds[2]}


def gemm(A, B, C, nb, order=ORDER_INSERTION, seed=0, nthreads=1, drop_edge=None, return_order=False,
         commute=False, given=None):
    """C + A B (all n x n, n % nb == 0) by the tiled program.  Returns the new C (and the
    run order when asked).  commute / given as for cholesky."""
    A, B, C = (np.asarray(x, np.float64) for x in (A, B, C))
    n = A.shape[0]
    if n % nb:
        raise ValueError("n must be a multiple of nb")
    abc = np.asfortranarray(np.concatenate([A, B, C], axis=1))
    nt = n // nb
    ordbuf = np.full(nt ** 3, -1, np.int64)
    if order == ORDER_GIVEN:
        ordbuf[:] = np.asarray(given, np.int64)
    nrun = ctypes.c_int64(0)
    de = None if drop_edge is None else (ctypes.c_uint32 * 2)(int(drop_edge[0]), int(drop_edge[1]))
    rc = lib().orc_gemm(n, nb, _dp(abc), order, seed, nthreads, ordbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        de, ctypes.byref(nrun), int(bool(commute)))
    if rc == -2:
        raise ValueError("not a valid order of the program's DAG")
    if rc < 0:
        raise RuntimeError("oracle failed")
    out = np.ascontiguousarray(abc[:, 2 * n:])
    if return_order:
        return out, ordbuf[: nrun.value].copy()
    return out


def gemm_entries(A, B, C, ii, jj):
    """C(i,j) + sum over m ascending of A(i,m) B(m,j) for each sampled (i, j), plain FP64."""
    a, b, c = (np.asfortranarray(np.asarray(x, np.float64)) for x in (A, B, C))
    ii = np.ascontiguousarray(ii, np.int64)
    jj = np.ascontiguousarray(jj, np.int64)
    out = np.zeros(len(ii))
    lib().orc_gemm_entries(_dp(a), _dp(b), _dp(c), a.shape[0], ii.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                           jj.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(ii), _dp(out))
    return out


def run_task(name, i, j, k, M, nb, Y=None):
    """Runs one task of the program on copies of the dense matrix M (n x n, all entries
    used as stored: this is a kernel-level check, not the symmetric-input convention) and
    of Y (n x nrhs).  Returns (M', Y', info)."""
    a = np.asfortranarray(np.array(M, dtype=np.float64))
    n = a.shape[0]
    y = None if Y is None else np.asfortranarray(np.array(Y, dtype=np.float64).reshape(n, -1))
    info = lib().orc_run_task(TASK_NAMES.index(name), i, j, k, _dp(a), n, nb, _dp(y) if y is not None else None,
                              0 if y is None else y.shape[1])
    if info < 0:
        raise ValueError("bad task")
    return np.ascontiguousarray(a), None if y is None else np.ascontiguousarray(y), int(info)


def factor_residual(A, L):
    """||A - L L^T||_F / ||A||_F (exact up to compensated rounding; O(n^3))."""
    a, l = _lower_cm(A), _lower_cm(L)
    return lib().orc_factor_residual(_dp(a), _dp(l), a.shape[0])


def factor_residual_probe(A, L, nvec=8, seed=1234):
    """max_v ||(A - L L^T) v|| / ||A v|| over nvec seeded Gaussian v (O(n^2) each)."""
    a, l = _lower_cm(A), _lower_cm(L)
    return lib().orc_factor_residual_probe(_dp(a), _dp(l), a.shape[0], nvec, seed)


def factor_residual_vectors(A, L, V):
    """max over the columns v of V (n x q) of ||(A - L L^T) v|| / ||A v||, the
    arithmetic of factor_residual_probe on caller-chosen vectors."""
    a, l = _lower_cm(A), _lower_cm(L)
    n = a.shape[0]
    V = np.asfortranarray(np.asarray(V, np.float64).reshape(n, -1))
    return lib().orc_factor_residual_vectors(_dp(a), _dp(l), n, _dp(V), V.shape[1])


def norm_inf(A):
    a = _lower_cm(A)
    return lib().orc_norm_inf_sym(_dp(a), a.shape[0])


def backward_error(A, X, B, anorm=None):
    """Per-column eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)."""
    a = _lower_cm(A)
    n = a.shape[0]
    X = np.asfortranarray(np.asarray(X, np.float64).reshape(n, -1))
    B = np.asfortranarray(np.asarray(B, np.float64).reshape(n, -1))
    q = X.shape[1]
    eta = np.zeros(q)
    lib().orc_backward_error(_dp(a), n, _dp(X), _dp(B), n, q, -1.0 if anorm is None else float(anorm), _dp(eta))
    return eta


def entry_check(A, L, ii, jj):
    """max over sampled (i,j) of |A_ij - sum_{m<=j} L_im L_jm| / sqrt(A_ii A_jj)."""
    a, l = _lower_cm(A), _lower_cm(L)
    ii = np.ascontiguousarray(ii, np.int64)
    jj = np.ascontiguousarray(jj, np.int64)
    return lib().orc_factor_entry_check(_dp(a), _dp(l), a.shape[0], ii.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        jj.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(ii))


def dot2(x, y):
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    return lib().orc_dot2(_dp(x), _dp(y), len(x))
