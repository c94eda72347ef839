"""ctypes binding of libtnc.so: the C ABI declared in include/tnc.h.

Argument marshalling only -- every computation happens in the library's HIP
kernels.  The functions keep the C names; ``Context``/``Network``/``Plan``
are thin owners of the handles that call them.  Loading fails loudly when
the library has not been built (``python -m paper_2606_01852_amd.build``).
Device pointers are passed as Python ints (e.g. ``tensor.data_ptr()``).
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnc.so")

OK, E_ARG, E_PATH, E_NOMEM, E_DEVICE, E_BUSY, E_UNSUPPORTED = range(7)
PREC_C64, PREC_BF16X3 = 0, 1
GEMM_4M, GEMM_3M = 0, 1
IN_C64, IN_C128 = 0, 1
OUT_C128, OUT_C64 = 0, 1
STATUS_NAMES = {0: "TNC_OK", 1: "TNC_E_ARG", 2: "TNC_E_PATH", 3: "TNC_E_NOMEM", 4: "TNC_E_DEVICE",
                5: "TNC_E_BUSY", 6: "TNC_E_UNSUPPORTED"}


class TncError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class PlanInfo(C.Structure):
    _fields_ = [("flops_per_slice", C.c_double), ("bytes_per_slice", C.c_double),
                ("transpose_bytes", C.c_double), ("n_slices", C.c_int64),
                ("max_intermediate", C.c_int64), ("peak_bytes", C.c_int64), ("max_chunk", C.c_int64),
                ("chunk_peak_bytes", C.c_int64), ("chunk_flops", C.c_double), ("n_steps", C.c_int32), ("n_permutes", C.c_int32),
                ("n_permuted_stores", C.c_int32), ("n_result", C.c_int32), ("n_cached_leaves", C.c_int32),
                ("n_inplace_leaves", C.c_int32), ("n_launches", C.c_int64)]


class StepInfo(C.Structure):
    _fields_ = [("A", C.c_int32), ("B", C.c_int32), ("C", C.c_int32), ("nH", C.c_int32), ("nM", C.c_int32),
                ("nN", C.c_int32), ("nK", C.c_int32), ("h", C.c_int64), ("m", C.c_int64), ("n", C.c_int64),
                ("k", C.c_int64), ("natural", C.c_int32), ("kernel", C.c_int32), ("variant", C.c_int32),
                ("swapped", C.c_int32), ("split", C.c_int32), ("hA", C.c_int64), ("hB", C.c_int64),
                ("presplit", C.c_int32), ("presplit_fused", C.c_int32)]


class DistHW(C.Structure):
    _fields_ = [("hbm_bytes_per_s", C.c_double), ("flops_per_s", C.c_double),
                ("net_bytes_per_s", C.c_double), ("latency_s", C.c_double)]


class DistStep(C.Structure):
    _fields_ = [("chain", C.c_int32), ("step", C.c_int32), ("state", C.c_int32), ("n_dist", C.c_int32),
                ("dist", C.c_int32 * 16), ("t_gemm_s", C.c_double), ("t_comm_s", C.c_double),
                ("out_bytes", C.c_double)]


_P = C.c_void_p
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)
_DP = C.POINTER(C.c_double)

_SIGS = {
    "tnc_last_error": (C.c_char_p, []),
    "tnc_version": (C.c_char_p, []),
    "tnc_device_count": (C.c_int, []),
    "tnc_ctx_create": (C.c_int, [C.c_int, _P, C.c_size_t, _P, C.POINTER(_P)]),
    "tnc_ctx_destroy": (C.c_int, [_P]),
    "tnc_ctx_sync": (C.c_int, [_P]),
    "tnc_ctx_set_gemm_variant": (C.c_int, [_P, C.c_int32]),
    "tnc_gemm_variant_count": (C.c_int, []),
    "tnc_net_create": (C.c_int, [_P, C.c_int32, _I32P, _I32P, C.c_int32, _I64P, C.c_int32, _I32P,
                                 C.POINTER(_P), C.c_int32, C.POINTER(_P)]),
    "tnc_net_set_tensor": (C.c_int, [_P, C.c_int32, _P, C.c_int32]),
    "tnc_net_set_tensor_device": (C.c_int, [_P, C.c_int32, _P]),
    "tnc_net_destroy": (C.c_int, [_P]),
    "tnc_plan_create": (C.c_int, [_P, C.c_int32, _I32P, C.c_int32, _I32P, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "tnc_plan_destroy": (C.c_int, [_P]),
    "tnc_plan_get_info": (C.c_int, [_P, C.POINTER(PlanInfo)]),
    "tnc_plan_get_step": (C.c_int, [_P, C.c_int32, C.POINTER(StepInfo)]),
    "tnc_plan_get_batch_step": (C.c_int, [_P, C.c_int32, C.POINTER(StepInfo)]),
    "tnc_plan_get_order": (C.c_int, [_P, C.c_int32, _I32P, C.c_int32, _I32P]),
    "tnc_plan_set_max_chunk": (C.c_int, [_P, C.c_int64]),
    "tnc_plan_set_graph": (C.c_int, [_P, C.c_int32]),
    "tnc_plan_set_grouping": (C.c_int, [_P, C.c_int32]),
    "tnc_plan_set_store_order": (C.c_int, [_P, C.c_int32]),
    "tnc_plan_autotune": (C.c_int, [_P]),
    "tnc_plan_distribute": (C.c_int, [_P, C.c_int32, C.c_double, C.POINTER(DistHW), C.POINTER(DistStep),
                                      C.c_int32, _I32P, _DP, _DP]),
    "tnc_device_calibrate": (C.c_int, [_P, C.POINTER(DistHW)]),
    "tnc_plan_set_profile": (C.c_int, [_P, C.c_int32]),
    "tnc_plan_get_profile": (C.c_int, [_P, C.c_int32, _DP, _I64P]),
    "tnc_contract": (C.c_int, [_P, C.c_int64, C.c_int64, _DP]),
    "tnc_contract_async": (C.c_int, [_P, C.c_int64, C.c_int64, _P, C.c_int32]),
    "tnc_plan_result_norm2": (C.c_int, [_P, _DP]),
    "tnc_permute": (C.c_int, [_P, _P, _P, C.c_int32, _I64P, _I32P]),
    "tnc_permute_noalloc": (C.c_int, [_P, _P, _P, C.c_int32, _I64P, _I32P]),
    "tnc_batched_cgemm": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, C.c_int64, _P, C.c_int64, _P,
                                    C.c_int64, _P, C.c_int32, C.c_int32]),
    "tnc_serve_start": (C.c_int, [_P, C.c_int32, C.c_int32]),
    "tnc_serve_stop": (C.c_int, [_P]),
    "tnc_serve_set_heavy": (C.c_int, [_P, C.c_double, C.c_int32]),
    "tnc_serve_set_fusion": (C.c_int, [_P, C.c_int32, C.c_double]),
    "tnc_serve_get_stats": (C.c_int, [_P, _I64P, _I64P, _I64P]),
    "tnc_submit": (C.c_int, [_P, _P, C.c_int64, C.c_int64, _DP, C.POINTER(C.c_uint64)]),
    "tnc_batcher_create": (C.c_int, [_P, C.c_int32, C.c_int32, _I32P, C.POINTER(_P)]),
    "tnc_batcher_destroy": (C.c_int, [_P]),
    "tnc_submit_row": (C.c_int, [_P, _P, C.POINTER(_P), C.c_int32, _DP, C.POINTER(C.c_uint64)]),
    "tnc_poll": (C.c_int, [_P, C.c_uint64, _I32P, _DP]),
    "tnc_wait": (C.c_int, [_P, C.c_uint64, _DP]),
}

_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """Load libtnc.so (raises if it has not been built).

    PyTorch, when installed, is imported first: its wheel carries its own
    HIP runtime, and the library must bind to the runtime already in the
    process (the one that owns the caller's tensors and streams) rather than
    load a second copy of it, which would not see the device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_01852_amd.build`")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return list(_SIGS)


def _check(status: int) -> None:
    if status != OK:
        raise TncError(status, lib().tnc_last_error().decode())


def _i32(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).reshape(-1))


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(C.POINTER(t)) if a.size else None


# ---------------------------------------------------------------- raw calls
def tnc_version() -> str:
    return lib().tnc_version().decode()


def tnc_device_count() -> int:
    return int(lib().tnc_device_count())


def tnc_ctx_create(device: int, arena: int = 0, arena_bytes: int = 0, stream: int = 0) -> int:
    out = _P()
    _check(lib().tnc_ctx_create(device, arena or None, arena_bytes, stream or None, C.byref(out)))
    return out.value


def tnc_ctx_destroy(ctx: int) -> None:
    _check(lib().tnc_ctx_destroy(ctx))


def tnc_ctx_sync(ctx: int) -> None:
    _check(lib().tnc_ctx_sync(ctx))


def tnc_ctx_set_gemm_variant(ctx: int, variant: int) -> None:
    _check(lib().tnc_ctx_set_gemm_variant(ctx, variant))


def tnc_gemm_variant_count() -> int:
    return int(lib().tnc_gemm_variant_count())


def tnc_net_create(ctx: int, labels: Sequence[Sequence[int]], extents: Sequence[int], open_labels: Sequence[int],
                   leaves: Optional[Sequence[np.ndarray]]) -> int:
    ranks = _i32([len(l) for l in labels])
    flat = _i32([x for l in labels for x in l])
    ext = np.ascontiguousarray(np.asarray(extents, dtype=np.int64))
    opn = _i32(open_labels)
    hold = None
    data = None
    kind = IN_C64
    if leaves is not None:
        hold = [np.ascontiguousarray(x, dtype=np.complex64) for x in leaves]
        data = (_P * len(hold))(*[h.ctypes.data for h in hold])
    out = _P()
    _check(lib().tnc_net_create(ctx, len(labels), _ptr(ranks, C.c_int32), _ptr(flat, C.c_int32), len(ext),
                                _ptr(ext, C.c_int64), len(opn), _ptr(opn, C.c_int32), data, kind, C.byref(out)))
    return out.value


def tnc_net_set_tensor(net: int, tensor: int, values: np.ndarray) -> None:
    v = np.ascontiguousarray(values, dtype=np.complex64)
    _check(lib().tnc_net_set_tensor(net, tensor, v.ctypes.data, IN_C64))


def tnc_net_set_tensor_device(net: int, tensor: int, dev_ptr: int) -> None:
    _check(lib().tnc_net_set_tensor_device(net, tensor, dev_ptr))


def tnc_net_destroy(net: int) -> None:
    _check(lib().tnc_net_destroy(net))


def tnc_plan_create(net: int, pairs: np.ndarray, sliced: Sequence[int] = (), prec: int = PREC_C64,
                    form: int = GEMM_4M) -> int:
    pr = _i32(pairs)
    sl = _i32(sliced)
    out = _P()
    _check(lib().tnc_plan_create(net, len(pr) // 2, _ptr(pr, C.c_int32), len(sl), _ptr(sl, C.c_int32), prec,
                                 form, C.byref(out)))
    return out.value


def tnc_plan_destroy(plan: int) -> None:
    _check(lib().tnc_plan_destroy(plan))


def tnc_plan_get_info(plan: int) -> PlanInfo:
    info = PlanInfo()
    _check(lib().tnc_plan_get_info(plan, C.byref(info)))
    return info


def tnc_plan_get_step(plan: int, step: int) -> StepInfo:
    s = StepInfo()
    _check(lib().tnc_plan_get_step(plan, step, C.byref(s)))
    return s


def tnc_plan_get_batch_step(plan: int, step: int) -> StepInfo:
    s = StepInfo()
    _check(lib().tnc_plan_get_batch_step(plan, step, C.byref(s)))
    return s


def tnc_plan_get_order(plan: int, tensor_id: int) -> list:
    rank = C.c_int32()
    _check(lib().tnc_plan_get_order(plan, tensor_id, None, 0, C.byref(rank)))
    buf = np.zeros(max(rank.value, 1), dtype=np.int32)
    _check(lib().tnc_plan_get_order(plan, tensor_id, _ptr(buf, C.c_int32), rank.value, C.byref(rank)))
    return [int(x) for x in buf[:rank.value]]


def tnc_plan_set_max_chunk(plan: int, max_chunk: int) -> None:
    _check(lib().tnc_plan_set_max_chunk(plan, max_chunk))


def tnc_device_calibrate(ctx: int) -> DistHW:
    """Measured FP32 MFMA rate (flops_per_s) and copy bandwidth
    (hbm_bytes_per_s) of the context's device."""
    hw = DistHW()
    _check(lib().tnc_device_calibrate(ctx, C.byref(hw)))
    return hw


def tnc_plan_distribute(plan: int, n_gpus: int, large_bytes: float, hbm: float, flops: float, net: float,
                        latency: float):
    """Returns (steps, total_s, redistributed_bytes); steps is a list of
    DistStep records."""
    hw = DistHW(hbm, flops, net, latency)
    n = C.c_int32()
    tot = C.c_double()
    moved = C.c_double()
    _check(lib().tnc_plan_distribute(plan, n_gpus, large_bytes, C.byref(hw), None, 0, C.byref(n), C.byref(tot),
                                     C.byref(moved)))
    arr = (DistStep * max(n.value, 1))()
    _check(lib().tnc_plan_distribute(plan, n_gpus, large_bytes, C.byref(hw), arr, n.value, C.byref(n),
                                     C.byref(tot), C.byref(moved)))
    return list(arr[:n.value]), tot.value, moved.value


def tnc_plan_autotune(plan: int) -> None:
    _check(lib().tnc_plan_autotune(plan))


def tnc_plan_set_graph(plan: int, enable: bool) -> None:
    _check(lib().tnc_plan_set_graph(plan, int(enable)))


def tnc_plan_set_grouping(plan: int, enable: bool) -> None:
    _check(lib().tnc_plan_set_grouping(plan, int(enable)))


def tnc_plan_set_store_order(plan: int, mode: int) -> None:
    _check(lib().tnc_plan_set_store_order(plan, int(mode)))


def tnc_plan_set_profile(plan: int, enable: bool) -> None:
    _check(lib().tnc_plan_set_profile(plan, int(enable)))


def tnc_plan_get_profile(plan: int, step: int):
    ms = C.c_double()
    n = C.c_int64()
    _check(lib().tnc_plan_get_profile(plan, step, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def tnc_contract(plan: int, first: int, count: int, n_result: int) -> np.ndarray:
    out = np.zeros(max(n_result, 1), dtype=np.complex128)
    _check(lib().tnc_contract(plan, first, count, out.ctypes.data_as(_DP)))
    return out[:n_result]


def tnc_contract_async(plan: int, first: int, count: int, out_dev: int, out_type: int = OUT_C128) -> None:
    _check(lib().tnc_contract_async(plan, first, count, out_dev, out_type))


def tnc_plan_result_norm2(plan: int) -> float:
    v = C.c_double()
    _check(lib().tnc_plan_result_norm2(plan, C.byref(v)))
    return v.value


def tnc_permute(ctx: int, in_dev: int, out_dev: int, extents: Sequence[int], perm: Sequence[int]) -> None:
    ext = np.ascontiguousarray(np.asarray(extents, dtype=np.int64))
    pm = _i32(perm)
    _check(lib().tnc_permute(ctx, in_dev, out_dev, len(ext), _ptr(ext, C.c_int64), _ptr(pm, C.c_int32)))


def tnc_permute_noalloc(ctx: int, in_dev: int, out_dev: int, extents: Sequence[int], perm: Sequence[int]) -> None:
    ext = np.ascontiguousarray(np.asarray(extents, dtype=np.int64))
    pm = _i32(perm)
    _check(lib().tnc_permute_noalloc(ctx, in_dev, out_dev, len(ext), _ptr(ext, C.c_int64), _ptr(pm, C.c_int32)))


def tnc_batched_cgemm(ctx: int, h: int, m: int, n: int, k: int, a_dev: int, stride_a: int, b_dev: int,
                      stride_b: int, c_dev: int, prec: int = PREC_C64, form: int = GEMM_4M) -> None:
    _check(lib().tnc_batched_cgemm(ctx, h, m, n, k, a_dev, stride_a, b_dev, stride_b, c_dev, prec, form))


def tnc_serve_start(ctx: int, max_inflight: int, queue_cap: int) -> None:
    _check(lib().tnc_serve_start(ctx, max_inflight, queue_cap))


def tnc_serve_set_heavy(ctx: int, heavy_flops: float, heavy_slots: int = 1) -> None:
    _check(lib().tnc_serve_set_heavy(ctx, float(heavy_flops), int(heavy_slots)))


FUSE_FLOPS_PER_LAUNCH = float(2 ** 30)   # the server's default fusion criterion
FUSE_ALL = 1e300                          # fuse every light request of one structure


def tnc_serve_set_fusion(ctx: int, max_requests: int, flops_per_launch: float = FUSE_FLOPS_PER_LAUNCH) -> None:
    _check(lib().tnc_serve_set_fusion(ctx, max_requests, flops_per_launch))


def tnc_serve_get_stats(ctx: int):
    """(jobs, fused jobs, requests run in fused jobs) since the server started."""
    j, fj, fr = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().tnc_serve_get_stats(ctx, C.byref(j), C.byref(fj), C.byref(fr)))
    return j.value, fj.value, fr.value


def tnc_serve_stop(ctx: int) -> None:
    _check(lib().tnc_serve_stop(ctx))


def tnc_submit(ctx: int, plan: int, first: int, count: int, out: np.ndarray) -> int:
    assert out.dtype == np.complex128 and out.flags.c_contiguous
    rid = C.c_uint64()
    _check(lib().tnc_submit(ctx, plan, first, count, out.ctypes.data_as(_DP), C.byref(rid)))
    return rid.value


def tnc_batcher_create(plan: int, batch_label: int, leaves) -> int:
    lv = np.ascontiguousarray(np.asarray(leaves, dtype=np.int32))
    h = _P()
    _check(lib().tnc_batcher_create(plan, int(batch_label), int(lv.size), lv.ctypes.data_as(_I32P), C.byref(h)))
    return h.value


def tnc_batcher_destroy(b: int) -> None:
    _check(lib().tnc_batcher_destroy(b))


def tnc_submit_row(ctx: int, b: int, rows, out: np.ndarray) -> int:
    """rows[i]: values of the batcher's i-th leaf for one batch row (the leaf
    without its batch mode), complex128; copied before the call returns."""
    assert out.dtype == np.complex128 and out.flags.c_contiguous
    arrs = [np.ascontiguousarray(np.asarray(r, dtype=np.complex128)) for r in rows]
    ptrs = (_P * max(1, len(arrs)))(*[a.ctypes.data for a in arrs])
    rid = C.c_uint64()
    _check(lib().tnc_submit_row(ctx, b, ptrs, IN_C128, out.ctypes.data_as(_DP), C.byref(rid)))
    return rid.value


def tnc_poll(ctx: int, rid: int):
    done = C.c_int32()
    lat = C.c_double()
    _check(lib().tnc_poll(ctx, rid, C.byref(done), C.byref(lat)))
    return bool(done.value), lat.value


def tnc_wait(ctx: int, rid: int) -> float:
    lat = C.c_double()
    _check(lib().tnc_wait(ctx, rid, C.byref(lat)))
    return lat.value


# ---------------------------------------------------------------- handle owners
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()


@atexit.register
def _close_live_contexts() -> None:
    # stop servers (their worker threads call the HIP runtime) while the
    # interpreter and the runtime are still alive
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """Owns a tnc_ctx.  ``device=-1`` plans on the host only."""

    def __init__(self, device: int = 0, arena_bytes: int = 0, arena_ptr: int = 0, stream: int = 0):
        self.device = device
        self.handle = tnc_ctx_create(device, arena_ptr, arena_bytes, stream)
        _live_contexts.add(self)

    def sync(self) -> None:
        tnc_ctx_sync(self.handle)

    def close(self) -> None:
        if self.handle:
            tnc_ctx_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Network:
    def __init__(self, ctx: Context, labels, extents, open_labels, leaves=None):
        self.ctx = ctx
        self.labels = [tuple(int(x) for x in l) for l in labels]
        self.handle = tnc_net_create(ctx.handle, self.labels, extents, open_labels,
                                     None if ctx.device < 0 else leaves)

    def set_tensor(self, t: int, values: np.ndarray) -> None:
        tnc_net_set_tensor(self.handle, t, values)

    def close(self) -> None:
        if self.handle:
            tnc_net_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batcher:
    """Row requests of `plan` batched over its batch label (see tnc_batcher_create)."""

    def __init__(self, plan: "Plan", batch_label: int, leaves):
        self.plan = plan
        self.leaves = [int(t) for t in leaves]
        self.handle = tnc_batcher_create(plan.handle, batch_label, self.leaves)

    def close(self) -> None:
        if self.handle:
            tnc_batcher_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    def __init__(self, net: Network, pairs, sliced=(), prec: int = PREC_C64, form: int = GEMM_4M):
        self.net = net
        self.handle = tnc_plan_create(net.handle, pairs, sliced, prec, form)
        self.info = tnc_plan_get_info(self.handle)

    def contract(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        count = self.info.n_slices - first if count is None else count
        return tnc_contract(self.handle, first, count, self.info.n_result)

    def step(self, s: int) -> StepInfo:
        return tnc_plan_get_step(self.handle, s)

    def order(self, tensor_id: int) -> list:
        return tnc_plan_get_order(self.handle, tensor_id)

    def close(self) -> None:
        if self.handle:
            tnc_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
