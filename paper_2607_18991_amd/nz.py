"""ctypes binding of libnz (include/nz.h).

Argument marshalling only: every step of the sweep runs in the HIP kernels of
libnz.so.  PyTorch supplies device memory and the stream.  Importing this module
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnz.so")

NZ_OK = 0
NZ_EINVAL = -1
NZ_EUNSUPPORTED = -2
NZ_ENOMEM = -3
NZ_EDEVICE = -4
NZ_EWORKSPACE = -5
NZ_FREE = 0
NZ_PERIODIC = 1
NZ_MLP_NPARAM = 8 * 64 + 64 + 64 * 64 + 64 + 64 * 2 + 2
NZ_MLP_NACT = 128

# every symbol include/nz.h declares
EXPORTS = (
    "nz_last_error", "nz_abi_version", "nz_coordination", "nz_sweep", "nz_canonical",
    "nz_batch_workspace_bytes", "nz_sweep_batch", "nz_last_batch_stats",
    "nz_mlp_forward", "nz_mlp_backward", "nz_mlp_adam", "nz_set_timing", "nz_last_batch_timing",
    "nz_mlp_loss", "nz_smax_window", "nz_convolve_window", "nz_sweep_batch_static", "nz_static_scratch_bytes",
    "nz_last_batch_job_stats", "nz_last_batch_cc_timing",
    "nz_mlp_size_stats", "nz_mlp_features", "nz_prefill_target", "nz_prefill_plan",
)


class NzJob(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("zone_mask", ctypes.c_uint32), ("boundary", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64), ("sample0", ctypes.c_int64),
        ("nsamples", ctypes.c_int64), ("n0", ctypes.c_int64), ("backoff", ctypes.c_int64),
        ("band_hi", ctypes.c_int64), ("prio", ctypes.c_double),
    ]


class NzTuning(ctypes.Structure):
    _fields_ = [("residency", ctypes.c_int32), ("wg_waves", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("bucket_log2", ctypes.c_int32),
                ("sweep_mode", ctypes.c_int32), ("summary", ctypes.c_int32), ("split_z", ctypes.c_int32)]


class NzError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnz error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    # PyTorch ships its own HIP runtime (same soname as the system one).  It
    # must be loaded first so that libnz binds to it: one HIP runtime per
    # process, and torch's device pointers and streams are valid in our calls.
    import torch  # noqa: F401

    L = ctypes.CDLL(LIB_PATH)
    P, i32, u32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64
    L.nz_last_error.restype = ctypes.c_char_p
    L.nz_last_error.argtypes = []
    L.nz_abi_version.restype = ctypes.c_int
    L.nz_coordination.argtypes = [u32]
    L.nz_coordination.restype = ctypes.c_int
    L.nz_sweep.argtypes = [i32, u32, i32, i64, u64, P, P]
    L.nz_sweep.restype = ctypes.c_int
    L.nz_canonical.argtypes = [P, i64, P, i64, P]
    L.nz_canonical.restype = ctypes.c_int
    L.nz_smax_window.argtypes = [i32, u32, i32, u64, i64, i64, i64, i64, i64, P]
    L.nz_smax_window.restype = ctypes.c_int
    L.nz_convolve_window.argtypes = [P, i64, i64, i64, P, i64, P, P]
    L.nz_convolve_window.restype = ctypes.c_int
    L.nz_batch_workspace_bytes.argtypes = [P, i32, P, ctypes.POINTER(ctypes.c_size_t)]
    L.nz_batch_workspace_bytes.restype = ctypes.c_int
    L.nz_sweep_batch.argtypes = [P, i32, P, ctypes.c_size_t, P, P, P, P, P]
    L.nz_sweep_batch.restype = ctypes.c_int
    L.nz_sweep_batch_static.argtypes = [P, i32, P, P, P, P, P]
    L.nz_sweep_batch_static.restype = ctypes.c_int
    L.nz_static_scratch_bytes.argtypes = []
    L.nz_static_scratch_bytes.restype = ctypes.c_size_t
    L.nz_last_batch_stats.argtypes = [P]
    L.nz_last_batch_stats.restype = ctypes.c_int
    L.nz_last_batch_job_stats.argtypes = [P, P, i32]
    L.nz_last_batch_job_stats.restype = ctypes.c_int
    L.nz_last_batch_cc_timing.argtypes = [P]
    L.nz_last_batch_cc_timing.restype = ctypes.c_int
    L.nz_mlp_size_stats.argtypes = [P, i32, P]
    L.nz_mlp_size_stats.restype = ctypes.c_int
    L.nz_mlp_features.argtypes = [P, P, i32, ctypes.c_double, ctypes.c_double, P]
    L.nz_mlp_features.restype = ctypes.c_int
    L.nz_prefill_target.argtypes = [P, i64, i32, P]
    L.nz_prefill_target.restype = ctypes.c_int
    L.nz_prefill_plan.argtypes = [P, P, i32, ctypes.c_double, ctypes.c_double, i32]
    L.nz_prefill_plan.restype = ctypes.c_int
    L.nz_set_timing.argtypes = [ctypes.c_int]
    L.nz_set_timing.restype = ctypes.c_int
    L.nz_last_batch_timing.argtypes = [P]
    L.nz_last_batch_timing.restype = ctypes.c_int
    L.nz_mlp_forward.argtypes = [P, P, P, P, i32, P]
    L.nz_mlp_forward.restype = ctypes.c_int
    L.nz_mlp_backward.argtypes = [P, P, P, P, P, i32, P]
    L.nz_mlp_backward.restype = ctypes.c_int
    L.nz_mlp_adam.argtypes = [P, P, P, P, P, P, i32, P]
    L.nz_mlp_adam.restype = ctypes.c_int
    L.nz_mlp_loss.argtypes = [P, P, P, P, P, i32, P]
    L.nz_mlp_loss.restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != NZ_OK:
        raise NzError(rc, lib().nz_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- host entry points
def nz_abi_version() -> int:
    return lib().nz_abi_version()


def nz_coordination(zone_mask: int) -> int:
    return lib().nz_coordination(zone_mask)


def nz_canonical(hist, p_grid) -> np.ndarray:
    h = np.ascontiguousarray(hist, dtype=np.uint64)
    p = np.ascontiguousarray(p_grid, dtype=np.float64)
    R = np.zeros(len(p), dtype=np.float64)
    _check(lib().nz_canonical(_np_ptr(h), len(h), _np_ptr(p), len(p), _np_ptr(R)))
    return R


def nz_smax_window(L: int, zone_mask: int, seed: int, sample0: int, nsamples: int, n_lo: int, n_hi: int,
                   n0: int = -1, boundary: int = NZ_FREE) -> np.ndarray:
    """Sum over the samples of S_max(n) for n in [n_lo, n_hi) (uint64 array)."""
    out = np.zeros(max(n_hi - n_lo, 1), dtype=np.uint64)
    _check(lib().nz_smax_window(L, zone_mask, boundary, seed, sample0, nsamples, n0, n_lo, n_hi, _np_ptr(out)))
    return out[: n_hi - n_lo]


def nz_convolve_window(Q, n_lo: int, N: int, p_grid):
    """(out, cover): binomial convolution of Q[n - n_lo] over n in [n_lo, n_lo + len(Q))."""
    q = np.ascontiguousarray(Q, dtype=np.float64)
    p = np.ascontiguousarray(p_grid, dtype=np.float64)
    out = np.zeros(max(len(p), 1), dtype=np.float64)
    cov = np.zeros(max(len(p), 1), dtype=np.float64)
    _check(lib().nz_convolve_window(_np_ptr(q), n_lo, n_lo + len(q), N, _np_ptr(p), len(p), _np_ptr(out),
                                    _np_ptr(cov)))
    return out[: len(p)], cov[: len(p)]


def nz_sweep(L: int, zone_mask: int, nsamples: int, seed: int, boundary: int = NZ_FREE):
    """Plain sweep of samples 0..nsamples-1; returns (nstar, mass) int32 arrays."""
    ns = np.zeros(max(nsamples, 1), dtype=np.int32)
    ms = np.zeros(max(nsamples, 1), dtype=np.int32)
    _check(lib().nz_sweep(L, zone_mask, boundary, nsamples, seed, _np_ptr(ns), _np_ptr(ms)))
    return ns[:nsamples], ms[:nsamples]


def make_jobs(jobs) -> ctypes.Array:
    """jobs: iterable of dicts with keys L, zone_mask, seed, nsamples and optional
    sample0, n0 (-1 plain), backoff, band_hi, prio, boundary."""
    jobs = list(jobs)
    arr = (NzJob * max(len(jobs), 1))()
    for k, j in enumerate(jobs):
        arr[k].L = int(j["L"])
        arr[k].zone_mask = int(j["zone_mask"])
        arr[k].boundary = int(j.get("boundary", NZ_FREE))
        arr[k].seed = int(j["seed"]) & (2**64 - 1)
        arr[k].sample0 = int(j.get("sample0", 0))
        arr[k].nsamples = int(j["nsamples"])
        arr[k].n0 = int(j.get("n0", -1))
        arr[k].backoff = int(j.get("backoff", 0))
        arr[k].band_hi = int(j.get("band_hi", 0))
        arr[k].prio = float(j.get("prio", 0.0))
    return arr, len(jobs)


def make_tuning(tune) -> NzTuning | None:
    if tune is None:
        return None
    t = NzTuning()
    t.residency = int(tune.get("residency", 0))
    t.wg_waves = int(tune.get("wg_waves", 0))
    t.waves_per_simd = int(tune.get("waves_per_simd", 0))
    t.bucket_log2 = int(tune.get("bucket_log2", 0))
    t.sweep_mode = int(tune.get("sweep_mode", 0))
    t.summary = int(tune.get("summary", 0))
    t.split_z = int(tune.get("split_z", 0))
    return t


def nz_batch_workspace_bytes(jobs, tune=None) -> int:
    arr, n = make_jobs(jobs)
    t = make_tuning(tune)
    out = ctypes.c_size_t(0)
    _check(lib().nz_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), n,
                                          ctypes.byref(t) if t is not None else None, ctypes.byref(out)))
    return int(out.value)


def nz_sweep_batch(jobs, ws, nstar, mass=None, tune=None, stream=None):
    """Device batch sweep.  ws, nstar, mass are torch CUDA tensors (uint8 workspace,
    int32 outputs).  Returns the per-job backoff counts as a numpy array."""
    arr, n = make_jobs(jobs)
    t = make_tuning(tune)
    back = np.zeros(max(n, 1), dtype=np.int32)
    _check(lib().nz_sweep_batch(ctypes.cast(arr, ctypes.c_void_p), n, ctypes.c_void_p(ws.data_ptr()),
                                ws.numel() * ws.element_size(), ctypes.c_void_p(nstar.data_ptr()),
                                ctypes.c_void_p(mass.data_ptr()) if mass is not None else None,
                                _np_ptr(back), ctypes.byref(t) if t is not None else None, _stream_ptr(stream)))
    return back[:n]


def nz_sweep_batch_static(jobs, nstar, mass=None, tune=None, stream=None):
    """nz_sweep_batch inside the library's own device buffer (no allocation).
    nstar, mass are torch CUDA int32 tensors.  Returns the per-job backoff
    counts as a numpy array."""
    arr, n = make_jobs(jobs)
    t = make_tuning(tune)
    back = np.zeros(max(n, 1), dtype=np.int32)
    _check(lib().nz_sweep_batch_static(ctypes.cast(arr, ctypes.c_void_p), n,
                                       ctypes.c_void_p(nstar.data_ptr()) if nstar is not None else None,
                                       ctypes.c_void_p(mass.data_ptr()) if mass is not None else None,
                                       _np_ptr(back), ctypes.byref(t) if t is not None else None,
                                       _stream_ptr(stream)))
    return back[:n]


def nz_static_scratch_bytes() -> int:
    return int(lib().nz_static_scratch_bytes())


def nz_last_batch_stats() -> dict:
    s = np.zeros(6, dtype=np.int64)
    _check(lib().nz_last_batch_stats(_np_ptr(s)))
    return {"chunks": int(s[0]), "band_redo": int(s[1]), "bucket_redo": int(s[2]), "backoffs": int(s[3]),
            "prefilled_sites": int(s[4]), "serial_steps": int(s[5])}


def nz_last_batch_job_stats(njobs: int):
    """(serial, prefilled) int64 arrays per job of the last batch."""
    a = np.zeros(max(njobs, 1), dtype=np.int64)
    b = np.zeros(max(njobs, 1), dtype=np.int64)
    _check(lib().nz_last_batch_job_stats(_np_ptr(a), _np_ptr(b), njobs))
    return a[:njobs], b[:njobs]


def nz_last_batch_cc_timing() -> dict:
    ms = np.zeros(5, dtype=np.float64)
    _check(lib().nz_last_batch_cc_timing(_np_ptr(ms)))
    return {"hook_ms": ms[0], "compress_ms": ms[1], "accum_ms": ms[2], "expand_ms": ms[3], "dispatches": int(ms[4])}


def nz_set_timing(enable: bool) -> None:
    _check(lib().nz_set_timing(int(bool(enable))))


def nz_last_batch_timing() -> dict:
    ms = np.zeros(6, dtype=np.float64)
    _check(lib().nz_last_batch_timing(_np_ptr(ms)))
    return {"keys_ms": ms[0], "cc_ms": ms[1], "sort_ms": ms[2], "sweep_ms": ms[3], "total_ms": ms[4],
            "sweep_launches": int(ms[5])}


# ---------------------------------------------------------------- learned-prefill planning (host)
def nz_mlp_size_stats(Ls):
    L = np.ascontiguousarray(Ls, dtype=np.int32)
    out = np.zeros(2, dtype=np.float64)
    _check(lib().nz_mlp_size_stats(_np_ptr(L), len(L), _np_ptr(out)))
    return float(out[0]), float(out[1])


def nz_mlp_features(masks, Ls, size_mean: float, size_std: float) -> np.ndarray:
    m = np.ascontiguousarray(masks, dtype=np.uint32)
    L = np.ascontiguousarray(Ls, dtype=np.int32)
    x = np.zeros((max(len(m), 1), 8), dtype=np.float32)
    _check(lib().nz_mlp_features(_np_ptr(m), _np_ptr(L), len(m), size_mean, size_std, _np_ptr(x)))
    return x[: len(m)]


def nz_prefill_target(nstar, L: int):
    """(samples used, mean, std, ln mean, ln std) of n*/N over the samples
    that span."""
    ns = np.ascontiguousarray(nstar, dtype=np.int32)
    out = np.zeros(5, dtype=np.float64)
    _check(lib().nz_prefill_target(_np_ptr(ns), len(ns), L, _np_ptr(out)))
    return int(out[0]), float(out[1]), float(out[2]), float(out[3]), float(out[4])


def nz_prefill_plan(y, jobs, k_sigma: float, band_sigma: float, plain: bool = False):
    """Copies of the job dicts with n0, backoff and band_hi from the MLP
    outputs y[j] = (ln mean, ln std)."""
    yy = np.ascontiguousarray(y, dtype=np.float32).reshape(-1, 2)
    jobs = [dict(j) for j in jobs]
    arr, n = make_jobs(jobs)
    _check(lib().nz_prefill_plan(_np_ptr(yy), ctypes.cast(arr, ctypes.c_void_p), n, k_sigma, band_sigma,
                                 int(bool(plain))))
    for k, j in enumerate(jobs):
        j["band_hi"] = int(arr[k].band_hi)
        j["n0"] = int(arr[k].n0)
        if not plain:
            j["backoff"] = int(arr[k].backoff)
    return jobs


# ---------------------------------------------------------------- MLP kernels
def nz_mlp_forward(params_bf16, x, y, act, stream=None):
    _check(lib().nz_mlp_forward(ctypes.c_void_p(params_bf16.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(act.data_ptr()), x.shape[0],
                                _stream_ptr(stream)))


def nz_mlp_backward(params_bf16, x, act, dy, grad, stream=None):
    _check(lib().nz_mlp_backward(ctypes.c_void_p(params_bf16.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(act.data_ptr()), ctypes.c_void_p(dy.data_ptr()),
                                 ctypes.c_void_p(grad.data_ptr()), x.shape[0], _stream_ptr(stream)))


def nz_mlp_adam(params_fp32, params_bf16, grad, m, v, hyper, step: int, stream=None):
    h = np.ascontiguousarray(hyper, dtype=np.float32)
    _check(lib().nz_mlp_adam(ctypes.c_void_p(params_fp32.data_ptr()), ctypes.c_void_p(params_bf16.data_ptr()),
                             ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                             ctypes.c_void_p(v.data_ptr()), _np_ptr(h), int(step), _stream_ptr(stream)))


def nz_mlp_loss(y, target, weight, dy, loss, stream=None):
    _check(lib().nz_mlp_loss(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                             ctypes.c_void_p(weight.data_ptr()), ctypes.c_void_p(dy.data_ptr()),
                             ctypes.c_void_p(loss.data_ptr()), y.shape[0], _stream_ptr(stream)))
