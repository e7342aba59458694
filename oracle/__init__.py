"""CPU oracle for the pms reduction: TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library
(``paper_1708_04710_amd``) and never imports it.

What it computes (each function names the passage it follows):

* ``reduce_standard`` -- the standard reduction (Alg. "Standard reduction",
  Sec. 1), left to right with sorted sparse columns.  Its result low* is
  unique for the complex (Sec. 2.3), so it is the definition that every
  schedule, the parallel multi-scale one included, must reproduce exactly.
* ``reduce_twist`` -- the same with the twist order and clearing
  (Alg. "Standard reduction with a twist", Sec. 2.4); used as the CPU timing
  baseline and as a second, differently scheduled reference.
* ``build_vr_i32`` / ``build_vr_f32`` / ``build_vr_f64`` /
  ``build_lowerstar`` -- filtrations (Sec. 2.2) in a compatible order by the
  key (value, dimension, lexicographic vertex tuple), with the boundary
  matrix of eq. "def:boundary_matrix" as CSC.
* ``pairs`` / ``essential`` -- the partition of low* into Pos / Neg / Ess
  (Sec. 2.3, Lemma "Pairing").
* ``left_beta`` -- left(i) and beta_j (Def. "left", Def. "beta"), written
  out from their definitions; used to pin the bounds of Thm. "Properties of
  beta_j".

All indices are 0-based, with -1 where the paper writes 0 ("none").
The arithmetic lives in ``pms_oracle.c`` (plain C, compiled with
``-ffp-contract=off``); this module only marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pms_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK = 0
ORC_ERR_ARG = -1
ORC_ERR_NOT_COMPATIBLE = -2
ORC_ERR_OOM = -3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle's C source into ``liboracle.so`` (gcc, no GPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Filtration(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("col_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("rows", ctypes.POINTER(ctypes.c_int32)),
        ("dim", ctypes.POINTER(ctypes.c_int8)),
        ("value", ctypes.POINTER(ctypes.c_double)),
        ("verts", ctypes.POINTER(ctypes.c_int32)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_reduce_standard.argtypes = [ctypes.c_int64, P, P, P, P]
        lib.oracle_reduce_twist.argtypes = [ctypes.c_int64, P, P, P, P, P]
        lib.oracle_build_vr_i32.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.POINTER(_Filtration)]
        lib.oracle_build_vr_f32.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                            ctypes.c_int32, ctypes.POINTER(_Filtration)]
        lib.oracle_build_vr_f64.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                            ctypes.c_int32, ctypes.POINTER(_Filtration)]
        lib.oracle_build_lowerstar.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(_Filtration)]
        lib.oracle_filtration_free.argtypes = [ctypes.POINTER(_Filtration)]
        for f in (lib.oracle_reduce_standard, lib.oracle_reduce_twist, lib.oracle_build_vr_i32,
                  lib.oracle_build_vr_f32, lib.oracle_build_vr_f64, lib.oracle_build_lowerstar):
            f.restype = ctypes.c_int
        lib.oracle_filtration_free.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None


@dataclass
class Filtration:
    """A filtration in compatible order with its boundary matrix (CSC)."""
    col_ptr: np.ndarray  # int64 [m+1]
    rows: np.ndarray     # int32 [nnz], ascending per column
    dim: np.ndarray      # int8 [m]
    value: np.ndarray    # int64 / float32 / float64 [m]
    verts: np.ndarray    # int32 [m, 4], ascending vertex ids, -1 padded

    @property
    def m(self) -> int:
        return int(self.dim.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.rows.shape[0])


def _take(f: _Filtration, value_dtype) -> Filtration:
    m, nnz = int(f.m), int(f.nnz)
    lib = _load()
    try:
        col_ptr = np.ctypeslib.as_array(f.col_ptr, shape=(m + 1,)).copy()
        rows = (np.ctypeslib.as_array(f.rows, shape=(nnz,)).copy() if nnz
                else np.zeros(0, np.int32))
        if m:
            dim = np.ctypeslib.as_array(f.dim, shape=(m,)).copy()
            value = np.ctypeslib.as_array(f.value, shape=(m,)).copy()
            verts = np.ctypeslib.as_array(f.verts, shape=(m * 4,)).copy().reshape(m, 4)
        else:
            dim = np.zeros(0, np.int8)
            value = np.zeros(0, np.float64)
            verts = np.zeros((0, 4), np.int32)
    finally:
        lib.oracle_filtration_free(ctypes.byref(f))
    if value_dtype == np.int64:
        v = value.astype(np.int64)
        assert np.array_equal(v.astype(np.float64), value)
        value = v
    elif value_dtype == np.float32:
        v = value.astype(np.float32)
        assert np.array_equal(v.astype(np.float64), value)
        value = v
    return Filtration(col_ptr=col_ptr, rows=rows, dim=dim, value=value, verts=verts)


def build_vr_i32(pts: np.ndarray, thr_sqd: int = -1, maxdim: int = 2) -> Filtration:
    """Vietoris-Rips on integer points, exact int64 squared distances."""
    pts = np.ascontiguousarray(pts, dtype=np.int32)
    n, D = pts.shape
    f = _Filtration()
    rc = _load().oracle_build_vr_i32(_ptr(pts), n, D, int(thr_sqd), maxdim, ctypes.byref(f))
    if rc:
        raise OracleError(rc, "build_vr_i32")
    return _take(f, np.int64)


def build_vr_f32(pts: np.ndarray, thr_sqd: float = -1.0, maxdim: int = 2) -> Filtration:
    """Vietoris-Rips on FP32 points; squared distances rounded to FP32 step by step."""
    pts = np.ascontiguousarray(pts, dtype=np.float32)
    n, D = pts.shape
    f = _Filtration()
    rc = _load().oracle_build_vr_f32(_ptr(pts), n, D, float(thr_sqd), maxdim, ctypes.byref(f))
    if rc:
        raise OracleError(rc, "build_vr_f32")
    return _take(f, np.float32)


def build_vr_f64(pts: np.ndarray, thr_sqd: float = -1.0, maxdim: int = 2) -> Filtration:
    """Vietoris-Rips on FP64 points (reference pipeline for gradients)."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    n, D = pts.shape
    f = _Filtration()
    rc = _load().oracle_build_vr_f64(_ptr(pts), n, D, float(thr_sqd), maxdim, ctypes.byref(f))
    if rc:
        raise OracleError(rc, "build_vr_f64")
    return _take(f, np.float64)


def build_lowerstar(grid: np.ndarray) -> Filtration:
    """Lower-star filtration of the Freudenthal triangulation of a grid.

    ``grid`` has shape (nz, ny, nx); vertex id = x + nx*(y + ny*z)."""
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    if grid.ndim != 3:
        raise ValueError("grid must be 3-D (nz, ny, nx)")
    nz, ny, nx = grid.shape
    f = _Filtration()
    rc = _load().oracle_build_lowerstar(_ptr(grid), nx, ny, nz, ctypes.byref(f))
    if rc:
        raise OracleError(rc, "build_lowerstar")
    return _take(f, np.float32)


def reduce_standard(col_ptr: np.ndarray, rows: np.ndarray, with_stats: bool = False):
    """Standard reduction; returns low* (int32 [m], -1 = zero column)."""
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    m = col_ptr.shape[0] - 1
    low = np.empty(m, np.int32)
    stats = np.zeros(2, np.int64)
    rc = _load().oracle_reduce_standard(m, _ptr(col_ptr), _ptr(rows), _ptr(low), _ptr(stats))
    if rc:
        raise OracleError(rc, "reduce_standard")
    return (low, {"additions": int(stats[0]), "xors": int(stats[1])}) if with_stats else low


def reduce_twist(col_ptr: np.ndarray, rows: np.ndarray, dim: np.ndarray, with_stats: bool = False):
    """Standard reduction with a twist; same low* as ``reduce_standard``."""
    col_ptr = np.ascontiguousarray(col_ptr, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    dim = np.ascontiguousarray(dim, dtype=np.int8)
    m = col_ptr.shape[0] - 1
    low = np.empty(m, np.int32)
    stats = np.zeros(2, np.int64)
    rc = _load().oracle_reduce_twist(m, _ptr(col_ptr), _ptr(rows), _ptr(dim), _ptr(low), _ptr(stats))
    if rc:
        raise OracleError(rc, "reduce_twist")
    return (low, {"additions": int(stats[0]), "xors": int(stats[1])}) if with_stats else low


def pairs(low_star: np.ndarray):
    """Persistence pairs (birth index low*(j), death index j), ascending in j
    (Sec. 2.3: j in Neg is paired with the positive simplex low*(j))."""
    low_star = np.asarray(low_star)
    death = np.nonzero(low_star >= 0)[0].astype(np.int32)
    birth = low_star[death].astype(np.int32)
    return birth, death


def essential(low_star: np.ndarray) -> np.ndarray:
    """Ess = positive simplices that are no column's low* (Sec. 2.3), ascending."""
    low_star = np.asarray(low_star)
    m = low_star.shape[0]
    is_birth = np.zeros(m, bool)
    is_birth[low_star[low_star >= 0]] = True
    return np.nonzero((low_star < 0) & ~is_birth)[0].astype(np.int32)


def left_beta(col_ptr: np.ndarray, rows: np.ndarray):
    """left(i) = first column with a non-zero in row i (Def. "left");
    beta_j = largest row whose left is j (Def. "beta").  -1 for "none"."""
    col_ptr = np.asarray(col_ptr, np.int64)
    rows = np.asarray(rows, np.int32)
    m = col_ptr.shape[0] - 1
    left = np.full(m, -1, np.int64)
    for j in range(m):
        for r in rows[col_ptr[j]:col_ptr[j + 1]]:
            if left[r] < 0:
                left[r] = j
    beta = np.full(m, -1, np.int64)
    for i in range(m):
        if left[i] >= 0 and i > beta[left[i]]:
            beta[left[i]] = i
    return left.astype(np.int32), beta.astype(np.int32)
