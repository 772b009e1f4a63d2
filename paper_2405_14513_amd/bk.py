"""ctypes binding of libbk.so (argument marshalling only).

Function names match the C ABI in include/bk.h.  Every numeric step runs in
the library's HIP kernels; this module only converts arguments, and raises
``BkError`` on a non-zero status.  Device memory and streams may come from
PyTorch: pass ``tensor.data_ptr()`` and ``torch.cuda.current_stream().cuda_stream``.
There is no fallback: if libbk.so is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

BK_F32 = 1
BK_F64 = 2

BK_OK = 0
BK_ERR_ARG = -1
BK_ERR_STATE = -2
BK_ERR_SIZE = -3
BK_ERR_OOM = -4
BK_ERR_HIP = -5

_STATUS = {
    BK_ERR_ARG: "BK_ERR_ARG",
    BK_ERR_STATE: "BK_ERR_STATE",
    BK_ERR_SIZE: "BK_ERR_SIZE",
    BK_ERR_OOM: "BK_ERR_OOM",
    BK_ERR_HIP: "BK_ERR_HIP",
}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbk.so")


class BkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class bk_binning(ctypes.Structure):
    _fields_ = [
        ("ng", ctypes.c_int),
        ("box_len", ctypes.c_double),
        ("n_k1", ctypes.c_int),
        ("k1_min", ctypes.c_double),
        ("k1_max", ctypes.c_double),
        ("n_mu", ctypes.c_int),
        ("n_t", ctypes.c_int),
        ("l_max", ctypes.c_int),
        ("m_max", ctypes.c_int),
        ("even_l_only", ctypes.c_int),
    ]


class bk_model(ctypes.Structure):
    _fields_ = [("amp", ctypes.c_double), ("n_s", ctypes.c_double), ("f_ng", ctypes.c_double), ("beta", ctypes.c_double)]


_lib = None

_SIGS = {
    "bk_plan_create": [ctypes.POINTER(bk_binning), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_void_p)],
    "bk_plan_create_multires": [ctypes.POINTER(bk_binning), ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
    "bk_plan_destroy": [ctypes.c_void_p],
    "bk_n_resolutions": [ctypes.c_void_p],
    "bk_query_resolution": [ctypes.c_void_p, ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 3,
    "bk_get_multipoles_res": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_get_triangle_counts_res": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.c_size_t],
    "bk_get_bin_means_res": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_load_grid": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p],
    "bk_estimate": [ctypes.c_void_p, ctypes.c_void_p],
    "bk_estimate_timed": [ctypes.c_void_p, ctypes.c_void_p],
    "bk_estimate_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_void_p],
    "bk_synchronize": [ctypes.c_void_p],
    "bk_query_sizes": [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 4,
    "bk_get_lm_list": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_size_t],
    "bk_get_multipoles": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_get_triangle_counts": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_size_t],
    "bk_get_bin_means": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_get_plan_info": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_get_stage_times": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_plan_autotune": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "bk_debug_get_buffer": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                            ctypes.POINTER(ctypes.c_size_t)],
    "bk_debug_mfma_probe": [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
    "bk_debug_read_range": [ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_size_t],
    "bk_debug_set_D": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p],
    "bk_group_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
    "bk_group_estimate": [ctypes.c_void_p, ctypes.c_void_p],
    "bk_group_destroy": [ctypes.c_void_p],
    "bk_count_triangles": [ctypes.POINTER(bk_binning), ctypes.POINTER(ctypes.c_int64), ctypes.c_size_t,
                           ctypes.POINTER(ctypes.c_int64)],
    "bk_discrete_prediction": [ctypes.POINTER(bk_binning), ctypes.POINTER(bk_model), ctypes.POINTER(ctypes.c_double),
                               ctypes.c_size_t],
    "bk_continuum_multipoles": [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.c_size_t],
}


def lib():
    """Load libbk.so once (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2405_14513_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        handle.bk_last_error.argtypes = []
        handle.bk_last_error.restype = ctypes.c_char_p
        _lib = handle
    return _lib


def bk_last_error() -> str:
    return lib().bk_last_error().decode()


def _check(status: int):
    if status != BK_OK:
        raise BkError(status, bk_last_error())


def make_binning(ng, n_k1, k1_min, k1_max, n_mu, n_t, box_len=0.0, l_max=6, m_max=6, even_l_only=1) -> bk_binning:
    return bk_binning(int(ng), float(box_len), int(n_k1), float(k1_min), float(k1_max), int(n_mu), int(n_t),
                      int(l_max), int(m_max), int(even_l_only))


def bk_plan_create(binning: bk_binning, prec: int = BK_F32, device: int = 0, max_batch: int = 1) -> int:
    out = ctypes.c_void_p()
    _check(lib().bk_plan_create(ctypes.byref(binning), int(prec), int(device), int(max_batch), ctypes.byref(out)))
    return out.value


def bk_plan_create_multires(binning: bk_binning, extra_bins, prec: int = BK_F32, device: int = 0,
                            max_batch: int = 1) -> int:
    """extra_bins: sequence of (n_k1, n_mu, n_t) for resolutions 1, 2, ..."""
    flat = [int(x) for d in extra_bins for x in d]
    arr = (ctypes.c_int * max(1, len(flat)))(*flat)
    out = ctypes.c_void_p()
    _check(lib().bk_plan_create_multires(ctypes.byref(binning), arr, len(flat) // 3, int(prec), int(device),
                                         int(max_batch), ctypes.byref(out)))
    return out.value


def bk_n_resolutions(plan: int) -> int:
    return int(lib().bk_n_resolutions(ctypes.c_void_p(plan)))


def bk_query_resolution(plan: int, res: int):
    v = [ctypes.c_int() for _ in range(3)]
    _check(lib().bk_query_resolution(ctypes.c_void_p(plan), int(res), *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def bk_get_multipoles_res(plan: int, res: int, batch: int) -> np.ndarray:
    n_lm = bk_query_sizes(plan)[0]
    n_k1, n_mu, n_t = bk_query_resolution(plan, res)
    out = np.empty(batch * n_lm * n_k1 * n_mu * n_t, dtype=np.float64)
    _check(lib().bk_get_multipoles_res(ctypes.c_void_p(plan), int(res),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
    return out.reshape(batch, n_lm, n_k1, n_mu, n_t)


def bk_get_triangle_counts_res(plan: int, res: int) -> np.ndarray:
    n_k1, n_mu, n_t = bk_query_resolution(plan, res)
    out = np.empty(n_k1 * n_mu * n_t, dtype=np.int64)
    _check(lib().bk_get_triangle_counts_res(ctypes.c_void_p(plan), int(res),
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), out.size))
    return out.reshape(n_k1, n_mu, n_t)


def bk_get_bin_means_res(plan: int, res: int) -> np.ndarray:
    n_k1, n_mu, n_t = bk_query_resolution(plan, res)
    out = np.empty(n_k1 * n_mu * n_t * 3, dtype=np.float64)
    _check(lib().bk_get_bin_means_res(ctypes.c_void_p(plan), int(res),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
    return out.reshape(n_k1, n_mu, n_t, 3)


def bk_plan_destroy(plan: int):
    _check(lib().bk_plan_destroy(ctypes.c_void_p(plan)))


def bk_load_grid(plan: int, ptr: int, dtype: int, batch: int, is_device_ptr: bool, stream: int = 0):
    _check(lib().bk_load_grid(ctypes.c_void_p(plan), ctypes.c_void_p(ptr), int(dtype), int(batch),
                              int(bool(is_device_ptr)), ctypes.c_void_p(stream)))


def bk_estimate(plan: int, stream: int = 0):
    _check(lib().bk_estimate(ctypes.c_void_p(plan), ctypes.c_void_p(stream)))


def bk_estimate_timed(plan: int, stream: int = 0):
    _check(lib().bk_estimate_timed(ctypes.c_void_p(plan), ctypes.c_void_p(stream)))


def bk_estimate_noalloc(plan: int, ptr: int, dtype: int, batch: int, out_ptr: int, stream: int = 0):
    """Estimate from device input `ptr` into device output `out_ptr` without allocating (static scratch)."""
    _check(lib().bk_estimate_noalloc(ctypes.c_void_p(plan), ctypes.c_void_p(ptr), int(dtype), int(batch),
                                     ctypes.c_void_p(out_ptr), ctypes.c_void_p(stream)))


def bk_synchronize(plan: int):
    _check(lib().bk_synchronize(ctypes.c_void_p(plan)))


def bk_query_sizes(plan: int):
    v = [ctypes.c_int() for _ in range(4)]
    _check(lib().bk_query_sizes(ctypes.c_void_p(plan), *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def bk_get_lm_list(plan: int):
    n_lm = bk_query_sizes(plan)[0]
    buf = (ctypes.c_int * (2 * n_lm))()
    _check(lib().bk_get_lm_list(ctypes.c_void_p(plan), buf, 2 * n_lm))
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(n_lm)]


def bk_get_multipoles(plan: int, batch: int, cap: int | None = None) -> np.ndarray:
    n_lm, n_k1, n_mu, n_t = bk_query_sizes(plan)
    n = batch * n_lm * n_k1 * n_mu * n_t
    out = np.empty(n if cap is None else cap, dtype=np.float64)
    _check(lib().bk_get_multipoles(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   out.size))
    return out[:n].reshape(batch, n_lm, n_k1, n_mu, n_t)


def bk_get_triangle_counts(plan: int) -> np.ndarray:
    _, n_k1, n_mu, n_t = bk_query_sizes(plan)
    out = np.empty(n_k1 * n_mu * n_t, dtype=np.int64)
    _check(lib().bk_get_triangle_counts(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        out.size))
    return out.reshape(n_k1, n_mu, n_t)


def bk_get_bin_means(plan: int) -> np.ndarray:
    _, n_k1, n_mu, n_t = bk_query_sizes(plan)
    out = np.empty(n_k1 * n_mu * n_t * 3, dtype=np.float64)
    _check(lib().bk_get_bin_means(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  out.size))
    return out.reshape(n_k1, n_mu, n_t, 3)


def bk_get_plan_info(plan: int) -> dict:
    out = np.empty(11, dtype=np.float64)
    _check(lib().bk_get_plan_info(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 11))
    keys = ["combinations", "work_items", "sides", "rings", "dense_terms", "useful_terms", "device_bytes",
            "plane_triples", "self_partnered", "grid_sides", "d_elems_per_field"]
    return dict(zip(keys, out.tolist()))


def bk_get_stage_times(plan: int) -> list:
    out = np.empty(4, dtype=np.float64)
    _check(lib().bk_get_stage_times(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4))
    return out.tolist()


def bk_get_stage_times_count(plan: int) -> list:
    """The four stage times and, fifth, the number of timed estimates averaged."""
    out = np.empty(5, dtype=np.float64)
    _check(lib().bk_get_stage_times(ctypes.c_void_p(plan), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 5))
    return out.tolist()


def bk_plan_autotune(plan: int, stream: int = 0) -> list:
    out = (ctypes.c_int * 3)()
    _check(lib().bk_plan_autotune(ctypes.c_void_p(plan), ctypes.c_void_p(stream), out))
    return list(out)


def bk_discrete_prediction(binning: bk_binning, amp: float, n_s: float, f_ng: float, beta: float) -> np.ndarray:
    step = 2 if binning.even_l_only else 1
    n_lm = sum(min(l, binning.m_max) + 1 for l in range(0, binning.l_max + 1, step))
    shape = (n_lm, binning.n_k1, binning.n_mu, binning.n_t)
    out = np.empty(int(np.prod(shape)), dtype=np.float64)
    model = bk_model(float(amp), float(n_s), float(f_ng), float(beta))
    _check(lib().bk_discrete_prediction(ctypes.byref(binning), ctypes.byref(model),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
    return out.reshape(shape)


def bk_continuum_multipoles(l_max: int, m_max: int, mu: float, t: float, beta: float) -> np.ndarray:
    n_lm = sum(min(l, m_max) + 1 for l in range(0, l_max + 1, 2))
    out = np.empty(n_lm, dtype=np.float64)
    _check(lib().bk_continuum_multipoles(int(l_max), int(m_max), float(mu), float(t), float(beta),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size))
    return out


def bk_count_triangles(binning: bk_binning):
    n = binning.n_k1 * binning.n_mu * binning.n_t
    out = np.empty(n, dtype=np.int64)
    ncomb = ctypes.c_int64()
    _check(lib().bk_count_triangles(ctypes.byref(binning), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n,
                                    ctypes.byref(ncomb)))
    return out.reshape(binning.n_k1, binning.n_mu, binning.n_t), ncomb.value


def bk_debug_get_buffer(plan: int, which: int, prec: int) -> np.ndarray:
    need = ctypes.c_size_t()
    _check(lib().bk_debug_get_buffer(ctypes.c_void_p(plan), int(which), None, 0, ctypes.byref(need)))
    if which in (2, 4, 5):
        out = np.empty(need.value // 4, dtype=np.int32)
    elif which == 3:
        out = np.empty(need.value, dtype=np.uint8)
    elif which == 6:
        out = np.empty(need.value // 8, dtype=np.float64)
    else:
        out = np.empty(need.value // (8 if prec == BK_F32 else 16), dtype=np.complex64 if prec == BK_F32 else np.complex128)
    _check(lib().bk_debug_get_buffer(ctypes.c_void_p(plan), int(which), ctypes.c_void_p(out.ctypes.data), out.nbytes,
                                     ctypes.byref(need)))
    return out


def bk_debug_get_buffer_size(plan: int, which: int) -> int:
    """Size in bytes of a test-support buffer (see bk_debug_get_buffer)."""
    need = ctypes.c_size_t()
    _check(lib().bk_debug_get_buffer(ctypes.c_void_p(plan), int(which), None, 0, ctypes.byref(need)))
    return need.value


def bk_debug_read_range(plan: int, which: int, prec: int, offset: int, count: int) -> np.ndarray:
    """`count` elements from element `offset` of buffer 0 or 1 (complex of the
    plan's precision) or 6 (float64)."""
    if which == 6:
        dt = np.dtype(np.float64)
    else:
        dt = np.dtype(np.complex64 if prec == BK_F32 else np.complex128)
    out = np.empty(int(count), dtype=dt)
    _check(lib().bk_debug_read_range(ctypes.c_void_p(plan), int(which), int(offset) * dt.itemsize,
                                     ctypes.c_void_p(out.ctypes.data), out.nbytes))
    return out


def bk_debug_set_D(plan: int, ptr: int, batch: int, is_device_ptr: bool, stream: int = 0):
    _check(lib().bk_debug_set_D(ctypes.c_void_p(plan), ctypes.c_void_p(ptr), int(batch), int(bool(is_device_ptr)),
                                ctypes.c_void_p(stream)))


def bk_debug_mfma_probe(prec: int) -> np.ndarray:
    out = np.empty(256, dtype=np.float64)
    _check(lib().bk_debug_mfma_probe(int(prec), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 256))
    return out.reshape(64, 4)


def bk_group_create(plans) -> int:
    arr = (ctypes.c_void_p * len(plans))(*plans)
    out = ctypes.c_void_p()
    _check(lib().bk_group_create(arr, len(plans), ctypes.byref(out)))
    return out.value


def bk_group_estimate(group: int, stream: int = 0):
    _check(lib().bk_group_estimate(ctypes.c_void_p(group), ctypes.c_void_p(stream)))


def bk_group_destroy(group: int):
    _check(lib().bk_group_destroy(ctypes.c_void_p(group)))


class Estimator:
    """A plan plus convenience methods taking torch tensors or numpy arrays."""

    def __init__(self, binning: bk_binning, prec: int = BK_F32, device: int = 0, max_batch: int = 1,
                 extra_bins=()):
        self.binning = binning
        self.prec = prec
        if extra_bins:
            self.plan = bk_plan_create_multires(binning, extra_bins, prec, device, max_batch)
        else:
            self.plan = bk_plan_create(binning, prec, device, max_batch)
        self.batch = 0

    def close(self):
        if self.plan:
            bk_plan_destroy(self.plan)
            self.plan = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, delta, stream: int = 0):
        """delta: torch tensor (CPU or GPU) or numpy array, shape [B, N, N, N] or [N, N, N]."""
        if isinstance(delta, np.ndarray):
            arr = np.ascontiguousarray(delta)
            if arr.dtype not in (np.float32, np.float64):
                raise TypeError("delta must be float32 or float64")
            batch = 1 if arr.ndim == 3 else arr.shape[0]
            dtype = BK_F32 if arr.dtype == np.float32 else BK_F64
            bk_load_grid(self.plan, arr.ctypes.data, dtype, batch, False, stream)
        else:
            import torch

            t = delta.contiguous()
            if t.dtype not in (torch.float32, torch.float64):
                raise TypeError("delta must be float32 or float64")
            batch = 1 if t.dim() == 3 else t.shape[0]
            dtype = BK_F32 if t.dtype == torch.float32 else BK_F64
            bk_load_grid(self.plan, t.data_ptr(), dtype, batch, t.is_cuda, stream)
            self._keep = t
        self.batch = batch

    def estimate(self, stream: int = 0):
        bk_estimate(self.plan, stream)

    def estimate_timed(self, stream: int = 0):
        bk_estimate_timed(self.plan, stream)

    def multipoles(self, res: int = 0) -> np.ndarray:
        return bk_get_multipoles_res(self.plan, res, self.batch)

    def counts(self, res: int = 0) -> np.ndarray:
        return bk_get_triangle_counts_res(self.plan, res)

    def bin_means(self, res: int = 0) -> np.ndarray:
        return bk_get_bin_means_res(self.plan, res)

    def lm_list(self):
        return bk_get_lm_list(self.plan)

    def info(self) -> dict:
        return bk_get_plan_info(self.plan)

    def stage_times(self) -> list:
        return bk_get_stage_times(self.plan)

    def autotune(self, stream: int = 0) -> list:
        return bk_plan_autotune(self.plan, stream)
