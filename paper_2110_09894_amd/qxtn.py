"""ctypes binding of libqxtn.so (argument marshalling only; all work runs in the HIP library).

Function names follow the C-ABI in include/qxtn.h.  Device buffers are passed
as torch tensors (their data_ptr), streams as torch.cuda.Stream or raw handles.
The library must have been built (``python -m paper_2110_09894_amd.build``);
importing this module without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqxtn.so")

QX_OK = 0
QX_ERR_INVALID_ARG = -1
QX_ERR_INVALID_NETWORK = -2
QX_ERR_INVALID_TREE = -3
QX_ERR_UNSUPPORTED = -4
QX_ERR_OUT_OF_BUDGET = -5
QX_ERR_HIP = -6
QX_ERR_DRY_RUN = -7

QX_C64 = 0
QX_SPLIT_BF16 = 1
QX_SPLIT_FP16 = 2
PRECISIONS = {"c64": QX_C64, "split_bf16": QX_SPLIT_BF16, "split_fp16": QX_SPLIT_FP16}

EXPORTED = ["qx_plan_create", "qx_plan_get_info", "qx_plan_get_op_info", "qx_plan_peak_bytes", "qx_contract",
            "qx_plan_destroy",
            "qx_last_error", "qx_plan_set_timing", "qx_plan_get_timing", "qx_permute_c64", "qx_cgemm",
            "qx_cgemm_noalloc"]
CGEMM_NOALLOC_SCRATCH_BYTES = 64 << 20

# matrix-core work-group tiles (qx_gemm_tile order); options take index + 1, 0 = automatic
TILES = ["128x128", "64x64", "128x64", "64x128", "256x128", "128x256", "128x128p3", "128x128p4", "thin"]


def _tile_opt(tile):
    if tile is None or tile == 0:
        return 0
    if isinstance(tile, str):
        return TILES.index(tile) + 1
    raise ValueError("tile must be None or one of " + ", ".join(TILES))

OPCLASSES = ["gemm", "simt", "dot", "permute", "slice_sum", "gather", "scale"]


class QxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qxtn status {status}: {msg}")
        self.status = status


class _Network(C.Structure):
    _fields_ = [("n_tensors", C.c_int32), ("index_ptr", C.POINTER(C.c_int64)),
                ("index_ids", C.POINTER(C.c_int64)), ("data_ptr", C.POINTER(C.c_int64)),
                ("data", C.POINTER(C.c_double)), ("n_qubits", C.c_int32),
                ("output_index", C.POINTER(C.c_int64))]


class _Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("max_bitstrings", C.c_int32),
                ("slice_batch_log2", C.c_int32), ("dry_run", C.c_int32),
                ("hbm_budget_bytes", C.c_int64), ("autotune", C.c_int32), ("eager", C.c_int32),
                ("open_qubits", C.c_uint64), ("gemm_tile", C.c_int32), ("reserved_", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("device_bytes", C.c_int64), ("arena_bytes", C.c_int64), ("n_leaves", C.c_int32),
                ("n_sliced", C.c_int32), ("slice_batch_log2", C.c_int32), ("width", C.c_int32),
                ("n_ops_const", C.c_int32), ("n_ops_call", C.c_int32), ("n_ops_block", C.c_int32),
                ("n_gemm_block", C.c_int32), ("flops_per_slice", C.c_double),
                ("flops_block", C.c_double), ("gemm_flops_block", C.c_double),
                ("flops_call", C.c_double), ("n_open", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OpInfo(C.Structure):
    _fields_ = [("phase", C.c_int32), ("op_class", C.c_int32), ("M", C.c_int64), ("N", C.c_int64),
                ("K", C.c_int64), ("batch", C.c_int64), ("tile", C.c_int32), ("batched", C.c_int32),
                ("flops", C.c_double), ("bytes", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["op_class"] = OPCLASSES[d["op_class"]]
        d["tile"] = TILES[d["tile"]] if d["tile"] >= 0 else None
        return d


class _OpTiming(C.Structure):
    _fields_ = [("launches", C.c_int64), ("seconds", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2110_09894_amd.build`")
        L = C.CDLL(_LIB_PATH)
        L.qx_plan_create.restype = C.c_int
        L.qx_plan_create.argtypes = [C.POINTER(_Network), C.POINTER(C.c_int32), C.POINTER(C.c_int64), C.c_int32,
                                     C.POINTER(_Options), C.c_void_p, C.POINTER(C.c_void_p)]
        L.qx_plan_get_info.restype = C.c_int
        L.qx_plan_get_info.argtypes = [C.c_void_p, C.POINTER(PlanInfo)]
        L.qx_plan_get_op_info.restype = C.c_int
        L.qx_plan_get_op_info.argtypes = [C.c_void_p, C.c_int32, C.POINTER(OpInfo)]
        L.qx_plan_peak_bytes.restype = C.c_int
        L.qx_plan_peak_bytes.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.qx_contract.restype = C.c_int
        L.qx_contract.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]
        L.qx_plan_destroy.restype = None
        L.qx_plan_destroy.argtypes = [C.c_void_p]
        L.qx_last_error.restype = C.c_char_p
        L.qx_last_error.argtypes = []
        L.qx_plan_set_timing.restype = C.c_int
        L.qx_plan_set_timing.argtypes = [C.c_void_p, C.c_int32]
        L.qx_plan_get_timing.restype = C.c_int
        L.qx_plan_get_timing.argtypes = [C.c_void_p, C.POINTER(_OpTiming), C.c_int32]
        L.qx_permute_c64.restype = C.c_int
        L.qx_permute_c64.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_int64, C.c_void_p]
        L.qx_cgemm.restype = C.c_int
        L.qx_cgemm.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p] + [C.c_int64] * 11 + [C.c_int32, C.c_int32,
                                                                                         C.c_void_p]
        L.qx_cgemm_noalloc.restype = C.c_int
        L.qx_cgemm_noalloc.argtypes = L.qx_cgemm.argtypes
        _lib = L
    return _lib


def last_error() -> str:
    return lib().qx_last_error().decode()


def _check(status):
    if status != QX_OK:
        raise QxError(status, last_error())


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(a, dtype):
    return a.ctypes.data_as(C.POINTER(dtype))


class Plan:
    """Owns a qx_plan handle (qx_plan_create / qx_plan_destroy)."""

    def __init__(self, network, tree, sliced=(), precision="c64", max_bitstrings=1, slice_batch_log2=-1,
                 dry_run=False, hbm_budget_bytes=0, autotune=False, eager=False, open_qubits=(), gemm_tile=None,
                 stream=None):
        index_ptr, index_ids, data_ptr, data, output_index = network.to_csr()
        self._keep = [np.ascontiguousarray(index_ptr, np.int64), np.ascontiguousarray(index_ids, np.int64),
                      np.ascontiguousarray(data_ptr, np.int64), np.ascontiguousarray(data, np.float64),
                      np.ascontiguousarray(output_index, np.int64)]
        ip, ii, dp, dd, oi = self._keep
        net = _Network(len(ip) - 1, _ptr(ip, C.c_int64), _ptr(ii, C.c_int64), _ptr(dp, C.c_int64),
                       _ptr(dd, C.c_double), len(oi), _ptr(oi, C.c_int64))
        tr = np.ascontiguousarray(np.asarray(tree, dtype=np.int32).reshape(-1))
        sl = np.ascontiguousarray(np.asarray(list(sliced), dtype=np.int64))
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        mask = 0
        for q in open_qubits:
            mask |= 1 << int(q)
        opt = _Options(prec, int(max_bitstrings), int(slice_batch_log2), int(bool(dry_run)), int(hbm_budget_bytes),
                       int(bool(autotune)), int(bool(eager)), mask, _tile_opt(gemm_tile), 0)
        h = C.c_void_p()
        _check(lib().qx_plan_create(C.byref(net), _ptr(tr, C.c_int32) if tr.size else None,
                                    _ptr(sl, C.c_int64) if sl.size else None, len(sl), C.byref(opt),
                                    _stream_handle(stream) if not dry_run else None, C.byref(h)))
        self.handle = h
        self.n_sliced = len(sl)
        self.n_qubits = len(oi)
        self.max_bitstrings = int(max_bitstrings)
        self.precision = prec
        self.n_open = bin(mask).count("1")
        self._keep = None

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().qx_plan_get_info(self.handle, C.byref(inf)))
        return inf.as_dict()

    def ops(self) -> list:
        """Every device op of the plan in launch order (qx_plan_get_op_info)."""
        inf = self.info()
        out = []
        for i in range(inf["n_ops_const"] + inf["n_ops_call"] + inf["n_ops_block"]):
            o = OpInfo()
            _check(lib().qx_plan_get_op_info(self.handle, i, C.byref(o)))
            out.append(o.as_dict())
        return out

    def peak_bytes(self, n_bitstrings=0, slice_batch_log2=-1) -> int:
        """Device bytes of this plan recompiled for another bitstring capacity / slice batch (host only)."""
        out = C.c_int64()
        _check(lib().qx_plan_peak_bytes(self.handle, int(n_bitstrings), int(slice_batch_log2), C.byref(out)))
        return out.value

    def contract(self, bitstrings, amplitudes, slice_range=None, stream=None):
        """amplitudes (float64 [B, 2^m, 2] contiguous, device; m open qubits, [B, 2] when none)
        += sum over slice_range of each slice's value."""
        lo, hi = slice_range if slice_range is not None else (0, 1 << self.n_sliced)
        B = int(bitstrings.shape[0])
        need = (B << self.n_open) * 2
        if amplitudes.numel() < need or not amplitudes.is_contiguous() or amplitudes.element_size() != 8:
            raise ValueError(f"amplitudes must be a contiguous float64 buffer of at least B * 2^{self.n_open} * 2 "
                             "elements")
        _check(lib().qx_contract(self.handle, C.c_void_p(bitstrings.data_ptr()), B, int(lo), int(hi),
                                 C.c_void_p(amplitudes.data_ptr()), _stream_handle(stream)))

    def set_timing(self, enable: bool):
        _check(lib().qx_plan_set_timing(self.handle, int(bool(enable))))

    def get_timing(self, reset=False) -> dict:
        arr = (_OpTiming * len(OPCLASSES))()
        _check(lib().qx_plan_get_timing(self.handle, arr, int(bool(reset))))
        return {name: {"launches": arr[i].launches, "seconds": arr[i].seconds, "flops": arr[i].flops,
                       "bytes": arr[i].bytes} for i, name in enumerate(OPCLASSES)}

    def destroy(self):
        if getattr(self, "handle", None) is not None:
            lib().qx_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def plan_create(network, tree, sliced=(), **kw) -> Plan:
    return Plan(network, tree, sliced, **kw)


def plan_get_info(plan: Plan) -> dict:
    return plan.info()


def contract(plan: Plan, bitstrings, amplitudes, slice_range=None, stream=None):
    plan.contract(bitstrings, amplitudes, slice_range, stream)


def plan_destroy(plan: Plan):
    plan.destroy()


def permute_c64(x, out, in_pos, items=1, stream=None):
    ip = np.ascontiguousarray(np.asarray(in_pos, dtype=np.int32))
    _check(lib().qx_permute_c64(C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), len(ip),
                                _ptr(ip, C.c_int32), int(items), _stream_handle(stream)))


def cgemm(a, b, c, M, N, K, a_ms, a_ks, b_ks, b_ns, stride_a=0, stride_b=0, stride_c=0, batch=1,
          precision="c64", tile=None, stream=None):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().qx_cgemm(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_void_p(c.data_ptr()),
                          M, N, K, a_ms, a_ks, b_ks, b_ns, stride_a, stride_b, stride_c, batch, prec,
                          _tile_opt(tile), _stream_handle(stream)))


def cgemm_noalloc(a, b, c, M, N, K, a_ms, a_ks, b_ks, b_ns, stride_a=0, stride_b=0, stride_c=0, batch=1,
                  precision="c64", tile=None, stream=None):
    """qx_cgemm_noalloc: the same product as ``cgemm`` without any device allocation (split-BF16 operand
    copies in the library's per-device scratch of CGEMM_NOALLOC_SCRATCH_BYTES)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().qx_cgemm_noalloc(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()), C.c_void_p(c.data_ptr()),
                                  M, N, K, a_ms, a_ks, b_ks, b_ns, stride_a, stride_b, stride_c, batch, prec,
                                  _tile_opt(tile), _stream_handle(stream)))
