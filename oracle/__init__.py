"""Plain serial CPU oracle for the Newman-Ziff first-spanning sweep on sc(5).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  The product library and its
Python binding never import it; the two share no code.  The oracle is the C
library ``libnzo.so`` built from ``nzo.c`` with gcc (see ``nzo.h`` for the
definitions it follows) plus the FP64 NumPy MLP in ``mlp.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nzo.c")
_LIB = os.path.join(_HERE, "libnzo.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libnzo.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i32, u32, u64, i64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
        P = ctypes.c_void_p
        L.nzo_zone_size.argtypes = [ctypes.c_int]
        L.nzo_zone_size.restype = ctypes.c_int
        L.nzo_offsets.argtypes = [u32, P]
        L.nzo_offsets.restype = ctypes.c_int
        L.nzo_philox4x32_10.argtypes = [P, P, P]
        L.nzo_philox4x32_10.restype = None
        L.nzo_key.argtypes = [u64, u64, u32, u32]
        L.nzo_key.restype = u64
        L.nzo_sort_keyed.argtypes = [P, i64, P]
        L.nzo_sort_keyed.restype = ctypes.c_int
        L.nzo_order.argtypes = [i32, u64, u64, P]
        L.nzo_order.restype = ctypes.c_int
        L.nzo_sweep_order.argtypes = [i32, u32, P, i64, P, P, P, ctypes.c_int, ctypes.c_int]
        L.nzo_sweep_order.restype = ctypes.c_int
        L.nzo_sweep.argtypes = [i32, u32, u64, u64, P, P]
        L.nzo_sweep.restype = ctypes.c_int
        L.nzo_sweep_many.argtypes = [i32, u32, u64, u64, i64, ctypes.c_int, P, P, P]
        L.nzo_sweep_many.restype = ctypes.c_int
        L.nzo_sweep_many_bc.argtypes = [i32, u32, ctypes.c_int, u64, u64, i64, ctypes.c_int, P, P, P]
        L.nzo_sweep_many_bc.restype = ctypes.c_int
        L.nzo_prefix_labels.argtypes = [i32, u32, P, i64, P]
        L.nzo_prefix_labels.restype = ctypes.c_int
        L.nzo_canonical.argtypes = [P, i64, P, i64, P]
        L.nzo_canonical.restype = ctypes.c_int
        L.nzo_convolve_window.argtypes = [P, i64, i64, i64, P, i64, P, P]
        L.nzo_sweep_order_bc.argtypes = [ctypes.c_int32, ctypes.c_uint32, ctypes.c_int, P, i64, P, P, P,
                                         ctypes.c_int, ctypes.c_int]
        L.nzo_sweep_order_bc.restype = ctypes.c_int
        L.nzo_convolve_window.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def zone_size(k: int) -> int:
    return lib().nzo_zone_size(k)


def offsets(mask: int) -> np.ndarray:
    """Offsets of D(mask) as an (z, 5) int32 array."""
    buf = np.zeros(892 * 5, dtype=np.int32)
    z = lib().nzo_offsets(mask, _ptr(buf))
    if z < 0:
        raise ValueError(f"bad zone mask {mask}")
    return buf[: 5 * z].reshape(z, 5).copy()


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().nzo_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def key(seed: int, sample: int, site: int, tag: int = 0) -> int:
    return int(lib().nzo_key(seed, sample, site, tag))


def sort_keyed(keys) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(len(k), dtype=np.uint32)
    _check(lib().nzo_sort_keyed(_ptr(k), len(k), _ptr(out)), "sort_keyed")
    return out


def order(L: int, seed: int, sample: int) -> np.ndarray:
    out = np.zeros(L**5, dtype=np.uint32)
    _check(lib().nzo_order(L, seed, sample, _ptr(out)), "order")
    return out


def sweep_order(L: int, mask: int, order_arr, smax: bool = False, check: bool = False,
                run_to_end: bool = False, periodic: bool = False):
    """Sweep over an explicit order; returns (nstar, mass[, smax array])."""
    o = np.ascontiguousarray(order_arr, dtype=np.uint32)
    ns = np.zeros(1, dtype=np.int32)
    ms = np.zeros(1, dtype=np.int32)
    sm = np.zeros(max(len(o), 1), dtype=np.int32) if smax else None
    rc = lib().nzo_sweep_order_bc(L, mask, int(periodic), _ptr(o), len(o), _ptr(ns), _ptr(ms),
                                  _ptr(sm) if smax else None, int(check), int(run_to_end))
    if rc == -2:
        raise AssertionError("oracle invariant violated")
    _check(rc, "sweep_order")
    if smax:
        return int(ns[0]), int(ms[0]), sm[: len(o)]
    return int(ns[0]), int(ms[0])


def sweep(L: int, mask: int, seed: int, sample: int):
    ns = np.zeros(1, dtype=np.int32)
    ms = np.zeros(1, dtype=np.int32)
    _check(lib().nzo_sweep(L, mask, seed, sample, _ptr(ns), _ptr(ms)), "sweep")
    return int(ns[0]), int(ms[0])


def sweep_many(L: int, mask: int, seed: int, sample0: int, count: int, nthreads: int = 1,
               times: bool = False, periodic: bool = False):
    """n* and mass of samples sample0 .. sample0+count-1; periodic: the first
    cluster that wraps around axis 0 (L >= 5)."""
    ns = np.zeros(count, dtype=np.int32)
    ms = np.zeros(count, dtype=np.int32)
    tm = np.zeros(3, dtype=np.float64)
    _check(lib().nzo_sweep_many_bc(L, mask, int(periodic), seed, sample0, count, nthreads, _ptr(ns), _ptr(ms),
                                   _ptr(tm)), "sweep_many")
    if times:
        return ns, ms, tm
    return ns, ms


def prefix_labels(L: int, mask: int, order_arr, n: int) -> np.ndarray:
    o = np.ascontiguousarray(order_arr, dtype=np.uint32)
    lab = np.zeros(L**5, dtype=np.int32)
    _check(lib().nzo_prefix_labels(L, mask, _ptr(o), n, _ptr(lab)), "prefix_labels")
    return lab


def convolve_window(Q, n_lo: int, N: int, p_grid):
    """(out, cover): binomial convolution of Q[n - n_lo], n in [n_lo, n_lo + len(Q))."""
    q = np.ascontiguousarray(Q, dtype=np.float64)
    p = np.ascontiguousarray(p_grid, dtype=np.float64)
    out = np.zeros(len(p), dtype=np.float64)
    cov = np.zeros(len(p), dtype=np.float64)
    _check(lib().nzo_convolve_window(_ptr(q), int(n_lo), int(n_lo + len(q)), int(N), _ptr(p), len(p), _ptr(out),
                                     _ptr(cov)), "convolve_window")
    return out, cov


def smax_window(L: int, mask: int, seed: int, sample0: int, nsamples: int, n_lo: int, n_hi: int,
                periodic: bool = False) -> np.ndarray:
    """Sum over samples sample0 .. of S_max(n), n in [n_lo, n_hi) (the largest
    cluster size after n occupied sites), from the serial sweep run past n*."""
    acc = np.zeros(n_hi - n_lo, dtype=np.int64)
    for s in range(sample0, sample0 + nsamples):
        o = order(L, seed, s)
        _, _, sm = sweep_order(L, mask, o[:n_hi], smax=True, run_to_end=True, periodic=periodic)
        acc += sm[n_lo - 1:n_hi - 1]
    return acc


def canonical(hist, p_grid) -> np.ndarray:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    p = np.ascontiguousarray(p_grid, dtype=np.float64)
    R = np.zeros(len(p), dtype=np.float64)
    _check(lib().nzo_canonical(_ptr(h), len(h), _ptr(p), len(p), _ptr(R)), "canonical")
    return R
