"""Thin Python binding of the kvop C ABI (argument marshalling only).

Every function keeps the C name and forwards to libkvop.so; device buffers are passed as
torch tensors (their data pointers), host arrays as numpy arrays, and the stream is the
current torch stream unless given.  Every computation happens in the HIP library: if it
is not built, importing a function raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkvop.so")

KVOP_OK, KVOP_EINVAL, KVOP_ENOMEM, KVOP_EBADHANDLE, KVOP_EDEVICE = range(5)
KVOP_F32, KVOP_BF16 = 0, 1
KVOP_KV_F32, KVOP_KV_BF16, KVOP_KV_FP8 = 0, 1, 2
KVOP_FILTER, KVOP_MAP, KVOP_JOIN = 0, 1, 2
KVOP_FLAG_ANY_COUNT = 1
KVOP_FLAG_PADDED = 2
KVOP_MIXED_PERSISTENT, KVOP_MIXED_GRAPH = 1, 2
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EBADHANDLE", 4: "EDEVICE"}


class KvopError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class kvop_model_cfg(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("d_model", C.c_int32), ("n_heads", C.c_int32),
                ("n_kv_heads", C.c_int32), ("head_dim", C.c_int32), ("d_ffn", C.c_int32),
                ("vocab", C.c_int32), ("rms_eps", C.c_float), ("rope_theta", C.c_float)]


class kvop_op(C.Structure):
    _fields_ = [("kind", C.c_int32), ("suffix_host", C.POINTER(C.c_int32)), ("suffix_len", C.c_int32),
                ("yes_id", C.c_int32), ("no_id", C.c_int32), ("theta_pos", C.c_float),
                ("theta_neg", C.c_float), ("label_lo", C.c_int32), ("label_n", C.c_int32),
                ("n_gen", C.c_int32), ("flags", C.c_uint32)]


class kvop_stage(C.Structure):
    _fields_ = [("r", C.c_float), ("theta_pos", C.c_float), ("theta_neg", C.c_float), ("idx_dev", C.c_void_p),
                ("idx_offsets_host", C.POINTER(C.c_int64))]


class kvop_mixed_op(C.Structure):
    _fields_ = [("op", kvop_op), ("logits_out_dev", C.c_void_p), ("decision_out_dev", C.c_void_p),
                ("tokens_out_dev", C.c_void_p)]


_P = C.c_void_p
_SIGS = {
    "kvop_last_error": (C.c_char_p, []),
    "kvop_weights_numel": (C.c_int64, [C.POINTER(kvop_model_cfg)]),
    "kvop_model_create": (C.c_int, [C.POINTER(kvop_model_cfg), _P, C.c_int64, C.c_int, _P, C.POINTER(_P)]),
    "kvop_model_destroy": (C.c_int, [_P]),
    "kvop_pool_create": (C.c_int, [_P, C.c_int, C.c_uint64, C.POINTER(_P)]),
    "kvop_pool_destroy": (C.c_int, [_P]),
    "kvop_doc_bytes": (C.c_uint64, [_P, C.c_int64]),
    "kvop_pool_stats": (C.c_int, [_P, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_int32)]),
    "kvop_kv_build": (C.c_int, [_P, _P, _P, C.c_int32, _P, _P, _P]),
    "kvop_kv_build_scored": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, _P, _P, _P, _P]),
    "kvop_retained_count": (C.c_int32, [C.c_float, C.c_int64]),
    "kvop_ea_select": (C.c_int, [_P, _P, _P, C.c_int32, C.c_float, _P, _P, _P]),
    "kvop_kv_release": (C.c_int, [_P, _P, C.c_int32]),
    "kvop_op_eval": (C.c_int, [_P, C.POINTER(kvop_op), C.c_float, _P, _P, _P, C.c_int32, _P, _P, _P, _P]),
    "kvop_gemm_num_tiles": (C.c_int32, [C.c_int32]),
    "kvop_gemm_tile_name": (C.c_char_p, [C.c_int32, C.c_int32]),
    "kvop_debug_gemm_rope": (C.c_int, [C.c_int32, _P, _P, _P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       _P, _P, _P, C.c_int32, _P]),
    "kvop_debug_gemm": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, C.c_int32,
                                  C.c_int32, C.c_int64, C.c_int64, C.c_int64, _P]),
    "kvop_gemm_set_tile": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "kvop_gemm_pick_tile": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
    "kvop_debug_read_cache": (C.c_int, [_P, C.c_uint64, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    "kvop_cascade_eval": (C.c_int, [_P, C.POINTER(kvop_op), C.POINTER(kvop_stage), C.c_int32, _P, C.c_int32, _P, _P,
                                    _P, _P, _P]),
    "kvop_op_eval_select": (C.c_int, [_P, C.POINTER(kvop_op), C.c_float, _P, _P, _P, C.c_int32, _P, C.c_int32, _P,
                                      _P, _P]),
    "kvop_proxy_create": (C.c_int, [C.c_int32, C.c_int32, _P, C.POINTER(_P)]),
    "kvop_proxy_destroy": (C.c_int, [_P]),
    "kvop_proxy_fit_standardizer": (C.c_int, [_P, _P, C.c_int64, _P]),
    "kvop_proxy_set_standardizer": (C.c_int, [_P, _P, _P, _P]),
    "kvop_proxy_train_step": (C.c_int, [_P, _P, _P, _P, C.c_int32, C.c_float, _P, _P]),
    "kvop_proxy_grads": (C.c_int, [_P, _P, _P, _P, C.c_int32, _P, _P, _P]),
    "kvop_proxy_infer": (C.c_int, [_P, _P, C.c_int64, C.c_float, _P, _P, _P, _P]),
    "kvop_debug_stage": (C.c_int, [_P, _P, C.c_float, _P, _P, _P, C.c_int32, C.c_int32, _P, _P]),
    "kvop_proxy_infer_noalloc": (C.c_int, [_P, _P, C.c_int64, C.c_float, _P, _P, _P, _P]),
    "kvop_proxy_params": (C.c_int, [_P, _P, _P]),
    "kvop_set_wave_rows": (C.c_int, [C.c_int64]),
    "kvop_set_attention_kernel": (C.c_int, [C.c_int32]),
    "kvop_get_attention_kernel": (C.c_int32, []),
    "kvop_debug_fp8_to_bf16": (C.c_int, [_P, C.c_int32, _P, _P]),
    "kvop_autotune": (C.c_int, [_P, C.c_int64, C.c_int32, _P, _P, C.c_int32]),
    "kvop_tuning_export": (C.c_int32, [_P, C.c_int32]),
    "kvop_tuning_import": (C.c_int, [C.c_char_p]),
    "kvop_mixed_eval": (C.c_int, [_P, _P, C.c_int32, C.c_float, _P, _P, _P, _P, _P, C.c_int32, C.c_uint32, _P]),
    "kvop_profile_start": (C.c_int, []),
    "kvop_profile_stop": (C.c_int, [_P, _P, C.c_int32]),
    "kvop_profile_num_classes": (C.c_int32, []),
    "kvop_profile_launches": (C.c_int32, [C.c_int32, _P, C.c_int32]),
    "kvop_profile_class_name": (C.c_char_p, [C.c_int32]),
    "kvop_plan_optimize": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "kvop_plan_loss": (C.c_int, [_P, _P, C.c_double, C.c_double, _P, _P]),
    "kvop_plan_evaluate": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "kvop_plan_reorder": (C.c_int, [C.c_int32, _P, _P, _P, _P, C.c_double, _P, _P]),
    "kvop_beta_lower_bound": (C.c_int, [C.c_double, C.c_double, C.c_double, _P]),
}
_lib_handle = None


def lib():
    """Load libkvop.so (built in-tree by build_lib); raise if it is missing."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2602_04430_amd.build_lib`")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        _lib_handle = h
    return _lib_handle


def _check(status: int):
    if status != KVOP_OK:
        raise KvopError(status, lib().kvop_last_error().decode())


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t) -> C.c_void_p:
    return C.c_void_p(0 if t is None else int(t.data_ptr()))


def _host(a, dtype):
    arr = np.ascontiguousarray(np.asarray(a), dtype=dtype)
    return arr, arr.ctypes.data_as(C.c_void_p)


def make_cfg(shape) -> kvop_model_cfg:
    return kvop_model_cfg(shape.n_layers, shape.d_model, shape.n_heads, shape.n_kv_heads, shape.head_dim,
                          shape.d_ffn, shape.vocab, shape.rms_eps, shape.rope_theta)


def kvop_weights_numel(cfg: kvop_model_cfg) -> int:
    return int(lib().kvop_weights_numel(C.byref(cfg)))


def kvop_model_create(cfg: kvop_model_cfg, weights_dev, compute: int, stream=None) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().kvop_model_create(C.byref(cfg), _dptr(weights_dev), int(weights_dev.numel()), compute,
                                   _stream(stream), C.byref(out)))
    return out


def kvop_model_destroy(model) -> None:
    _check(lib().kvop_model_destroy(model))


def kvop_pool_create(model, kv_dtype: int, nbytes: int) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().kvop_pool_create(model, kv_dtype, int(nbytes), C.byref(out)))
    return out


def kvop_pool_destroy(pool) -> None:
    _check(lib().kvop_pool_destroy(pool))


def kvop_doc_bytes(pool, L: int) -> int:
    return int(lib().kvop_doc_bytes(pool, int(L)))


def kvop_pool_stats(pool):
    u, c, n = C.c_uint64(), C.c_uint64(), C.c_int32()
    _check(lib().kvop_pool_stats(pool, C.byref(u), C.byref(c), C.byref(n)))
    return int(u.value), int(c.value), int(n.value)


def kvop_kv_build(pool, tokens_dev, offsets: Sequence[int], pooled_dev=None, stream=None) -> np.ndarray:
    """Returns the uint64 handles of the built documents."""
    offs, po = _host(offsets, np.int64)
    n = len(offs) - 1
    handles = np.zeros(max(n, 0), np.uint64)
    _check(lib().kvop_kv_build(pool, _dptr(tokens_dev), po, n, _stream(stream),
                               handles.ctypes.data_as(C.c_void_p), _dptr(pooled_dev)))
    return handles


def kvop_kv_build_scored(pool, tokens_dev, offsets: Sequence[int], n_future: int, scores_dev, pooled_dev=None,
                         stream=None) -> np.ndarray:
    """kvop_kv_build that also writes every row's expected-attention score into scores_dev
    (FP32, indexed like tokens_dev from offsets[0]).  Returns the handles."""
    offs, po = _host(offsets, np.int64)
    n = len(offs) - 1
    handles = np.zeros(max(n, 0), np.uint64)
    _check(lib().kvop_kv_build_scored(pool, _dptr(tokens_dev), po, n, int(n_future), _stream(stream),
                                      handles.ctypes.data_as(C.c_void_p), _dptr(pooled_dev), _dptr(scores_dev)))
    return handles


def kvop_retained_count(r: float, L: int) -> int:
    return int(lib().kvop_retained_count(float(r), int(L)))


def kvop_ea_select(pool, scores_dev, offsets: Sequence[int], r: float, idx_dev, stream=None) -> np.ndarray:
    """Retained lists at retention r from expected-attention scores, written into idx_dev
    (int32, room for the total); returns the int64 list offsets (n + 1)."""
    offs, po = _host(offsets, np.int64)
    n = len(offs) - 1
    out = np.zeros(max(n, 0) + 1, np.int64)
    _check(lib().kvop_ea_select(pool, _dptr(scores_dev), po, n, float(r), _stream(stream), _dptr(idx_dev),
                                out.ctypes.data_as(C.c_void_p)))
    return out


def kvop_kv_release(pool, handles) -> None:
    h, hp = _host(handles, np.uint64)
    _check(lib().kvop_kv_release(pool, hp, len(h)))


def make_op(kind: int, suffix, yes_id: int = 1, no_id: int = 0, theta_pos: float = 0.0, theta_neg: float = 0.0,
            label_lo: int = 0, label_n: int = 0, n_gen: int = 1, flags: int = 0):
    suf = np.ascontiguousarray(np.asarray(suffix, np.int32))
    op = kvop_op(kind, suf.ctypes.data_as(C.POINTER(C.c_int32)), len(suf), yes_id, no_id, theta_pos, theta_neg,
                 label_lo, label_n, n_gen, flags)
    op._keep = suf  # keep the suffix alive with the descriptor
    return op


def kvop_op_eval(pool, op: kvop_op, r: float, idx_dev, idx_offsets: Sequence[int], handles, logits_dev,
                 decision_dev=None, tokens_dev=None, stream=None) -> None:
    offs, po = _host(idx_offsets, np.int64)
    h, hp = _host(handles, np.uint64)
    n_items = len(h) // (2 if op.kind == KVOP_JOIN else 1)
    _check(lib().kvop_op_eval(pool, C.byref(op), float(r), _dptr(idx_dev), po, hp, n_items, _stream(stream),
                              _dptr(logits_dev), _dptr(decision_dev), _dptr(tokens_dev)))


def kvop_debug_stage(pool, op: kvop_op, r: float, idx_dev, idx_offsets: Sequence[int], handles, layer: int,
                     hidden_dev, stream=None) -> None:
    """Residual stream of the suffix rows after `layer`: FP32 [n_items, S, d_model] into hidden_dev."""
    offs, po = _host(idx_offsets, np.int64)
    h, hp = _host(handles, np.uint64)
    n_items = len(h) // (2 if op.kind == KVOP_JOIN else 1)
    _check(lib().kvop_debug_stage(pool, C.byref(op), float(r), _dptr(idx_dev), po, hp, n_items, int(layer),
                                  _stream(stream), _dptr(hidden_dev)))


def kvop_gemm_num_tiles(dtype: int) -> int:
    return int(lib().kvop_gemm_num_tiles(dtype))


def kvop_gemm_tile_name(dtype: int, tile: int) -> str:
    return lib().kvop_gemm_tile_name(dtype, tile).decode()


def kvop_debug_gemm(dtype: int, out_dtype: int, epilogue: int, tile: int, A, B, Cm, M: int, N: int, K: int,
                    lda: int, ldb: int, ldc: int, stream=None) -> None:
    _check(lib().kvop_debug_gemm(dtype, out_dtype, epilogue, tile, _dptr(A), _dptr(B), _dptr(Cm), M, N, K, lda, ldb,
                                 ldc, _stream(stream)))


def kvop_debug_gemm_rope(tile: int, A, B, Cm, M: int, N: int, K: int, head_dim: int, rot_cols: int, pos, cos_t, sin_t,
                         fused: bool, stream=None) -> None:
    _check(lib().kvop_debug_gemm_rope(tile, _dptr(A), _dptr(B), _dptr(Cm), M, N, K, head_dim, rot_cols, _dptr(pos),
                                      _dptr(cos_t), _dptr(sin_t), int(bool(fused)), _stream(stream)))


def kvop_gemm_set_tile(dtype: int, epilogue: int, N: int, K: int, M: int, tile: int) -> None:
    _check(lib().kvop_gemm_set_tile(dtype, epilogue, N, K, M, tile))


def kvop_gemm_pick_tile(dtype: int, epilogue: int, M: int, N: int, K: int) -> int:
    return int(lib().kvop_gemm_pick_tile(dtype, epilogue, M, N, K))


def kvop_debug_read_cache(pool, handle, layer: int, kv_head: int, kv: int, out_dev, stream=None) -> None:
    _check(lib().kvop_debug_read_cache(pool, C.c_uint64(int(handle)), layer, kv_head, kv, _dptr(out_dev),
                                       _stream(stream)))


def kvop_profile_start() -> None:
    _check(lib().kvop_profile_start())


def kvop_profile_stop() -> dict:
    """{class name: (milliseconds, launches)} since kvop_profile_start (synchronises)."""
    n = int(lib().kvop_profile_num_classes())
    ms = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.int64)
    _check(lib().kvop_profile_stop(ms.ctypes.data_as(C.c_void_p), cnt.ctypes.data_as(C.c_void_p), n))
    return {lib().kvop_profile_class_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}


def kvop_profile_launches(name: str) -> list:
    """Per-launch milliseconds of one class since the last kvop_profile_start/stop."""
    names = [lib().kvop_profile_class_name(i).decode() for i in range(kvop_profile_num_classes())]
    cls = names.index(name)
    n = int(lib().kvop_profile_launches(cls, None, 0))
    out = np.zeros(max(n, 1), np.float64)
    lib().kvop_profile_launches(cls, out.ctypes.data_as(C.c_void_p), n)
    return out[:n].tolist()


def kvop_profile_num_classes() -> int:
    return int(lib().kvop_profile_num_classes())


def kvop_profile_class_name(i: int) -> str:
    return lib().kvop_profile_class_name(i).decode()


def kvop_op_eval_select(pool, op: kvop_op, r: float, idx_dev, idx_offsets, handles, select, logits_dev,
                        decision_dev=None, stream=None) -> None:
    offs, po = _host(idx_offsets, np.int64)
    h, hp = _host(handles, np.uint64)
    sel, sp = _host(select, np.int32)
    n_items = len(h) // (2 if op.kind == KVOP_JOIN else 1)
    _check(lib().kvop_op_eval_select(pool, C.byref(op), float(r), _dptr(idx_dev), po, hp, n_items, sp, len(sel),
                                     _stream(stream), _dptr(logits_dev), _dptr(decision_dev)))


def kvop_cascade_eval(pool, op: kvop_op, stages, handles, logits_dev, decision_dev, stage_dev,
                      stream=None) -> np.ndarray:
    """stages: sequence of (r, theta_pos, theta_neg, idx_dev, idx_offsets).  Returns the number
    of items each stage evaluated."""
    keep = []
    arr = (kvop_stage * len(stages))()
    for i, (r, tp, tn, idx_dev, offs) in enumerate(stages):
        o = np.ascontiguousarray(np.asarray(offs, np.int64))
        keep.append(o)
        arr[i] = kvop_stage(float(r), float(tp), float(tn), _dptr(idx_dev), o.ctypes.data_as(C.POINTER(C.c_int64)))
    h, hp = _host(handles, np.uint64)
    n_items = len(h) // (2 if op.kind == KVOP_JOIN else 1)
    processed = np.zeros(len(stages), np.int32)
    _check(lib().kvop_cascade_eval(pool, C.byref(op), arr, len(stages), hp, n_items, _stream(stream), _dptr(logits_dev),
                                   _dptr(decision_dev), _dptr(stage_dev), processed.ctypes.data_as(C.c_void_p)))
    return processed


def kvop_proxy_create(d_in: int, d_hidden: int, params_dev) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().kvop_proxy_create(d_in, d_hidden, _dptr(params_dev), C.byref(out)))
    return out


def kvop_proxy_destroy(proxy) -> None:
    _check(lib().kvop_proxy_destroy(proxy))


def kvop_proxy_fit_standardizer(proxy, feats_dev, stream=None) -> None:
    _check(lib().kvop_proxy_fit_standardizer(proxy, _dptr(feats_dev), int(feats_dev.shape[0]), _stream(stream)))


def kvop_proxy_set_standardizer(proxy, mean_dev, inv_std_dev, stream=None) -> None:
    _check(lib().kvop_proxy_set_standardizer(proxy, _dptr(mean_dev), _dptr(inv_std_dev), _stream(stream)))


def kvop_proxy_train_step(proxy, feats_dev, labels_dev, rows_dev, batch: int, lr: float, loss_dev=None,
                          stream=None) -> None:
    _check(lib().kvop_proxy_train_step(proxy, _dptr(feats_dev), _dptr(labels_dev), _dptr(rows_dev), batch, lr,
                                       _stream(stream), _dptr(loss_dev)))


def kvop_proxy_grads(proxy, feats_dev, labels_dev, rows_dev, batch: int, grads_dev, loss_dev=None,
                     stream=None) -> None:
    _check(lib().kvop_proxy_grads(proxy, _dptr(feats_dev), _dptr(labels_dev), _dptr(rows_dev), batch,
                                  _stream(stream), _dptr(grads_dev), _dptr(loss_dev)))


def kvop_proxy_infer(proxy, feats_dev, tau: float, cls_dev, conf_dev, answered_dev, stream=None) -> None:
    _check(lib().kvop_proxy_infer(proxy, _dptr(feats_dev), int(feats_dev.shape[0]), tau, _stream(stream),
                                  _dptr(cls_dev), _dptr(conf_dev), _dptr(answered_dev)))


def kvop_proxy_infer_noalloc(proxy, feats_dev, tau: float, cls_dev, conf_dev, answered_dev, stream=None) -> None:
    """kvop_proxy_infer without device allocation (fixed per-GPU scratch; bounded row count)."""
    _check(lib().kvop_proxy_infer_noalloc(proxy, _dptr(feats_dev), int(feats_dev.shape[0]), tau, _stream(stream),
                                          _dptr(cls_dev), _dptr(conf_dev), _dptr(answered_dev)))


def kvop_proxy_params(proxy, out_dev, stream=None) -> None:
    _check(lib().kvop_proxy_params(proxy, _dptr(out_dev), _stream(stream)))


def kvop_set_wave_rows(rows: int) -> None:
    _check(lib().kvop_set_wave_rows(int(rows)))


def kvop_set_attention_kernel(variant: int) -> None:
    _check(lib().kvop_set_attention_kernel(int(variant)))


def kvop_get_attention_kernel() -> int:
    return int(lib().kvop_get_attention_kernel())


def kvop_debug_fp8_to_bf16(codes_dev, out_dev, stream=None) -> None:
    _check(lib().kvop_debug_fp8_to_bf16(_dptr(codes_dev), int(codes_dev.numel()), _dptr(out_dev), _stream(stream)))


def kvop_mixed_eval(pool, ops, r: float, idx_dev, idx_offsets, handles, item_op, item_list, flags: int,
                    stream=None) -> None:
    """ops: list of (kvop_op, logits_dev, decision_dev or None, tokens_dev or None)."""
    arr = (kvop_mixed_op * len(ops))()
    keep = []
    for i, (op, lg, dec, tk) in enumerate(ops):
        arr[i].op = op
        keep.append(op._keep)
        arr[i].logits_out_dev = _dptr(lg)
        arr[i].decision_out_dev = _dptr(dec)
        arr[i].tokens_out_dev = _dptr(tk)
    offs, po = _host(idx_offsets, np.int64)
    h, hp = _host(handles, np.uint64)
    io, iop = _host(item_op, np.int32)
    il, ilp = _host(item_list, np.int64)
    _check(lib().kvop_mixed_eval(pool, C.cast(arr, C.c_void_p), len(ops), float(r), _dptr(idx_dev), po, hp, iop, ilp,
                                 len(io), int(flags), _stream(stream)))


def kvop_autotune(model, rows: int, reps: int = 3, stream=None) -> str:
    buf = C.create_string_buffer(1 << 16)
    _check(lib().kvop_autotune(model, int(rows), int(reps), _stream(stream), buf, len(buf)))
    return buf.value.decode()


def kvop_tuning_export() -> str:
    n = int(lib().kvop_tuning_export(None, 0))
    buf = C.create_string_buffer(n + 1)
    lib().kvop_tuning_export(buf, n + 1)
    return buf.value.decode()


def kvop_tuning_import(text: str) -> None:
    _check(lib().kvop_tuning_import(text.encode()))


# ----------------------------------------------------------------------------- plan optimizer (host)

class kvop_plan_problem(C.Structure):
    _fields_ = [("n_filters", C.c_int32), ("n_ops", C.c_void_p), ("cost", C.c_void_p), ("log_odds", C.c_void_p),
                ("gold", C.c_void_p), ("n_tuples", C.c_int32), ("target_recall", C.c_double),
                ("target_precision", C.c_double), ("alpha", C.c_double)]


class kvop_plan_opts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("lr", C.c_double), ("beta", C.c_double), ("tau0", C.c_double),
                ("tau_end", C.c_double), ("theta0", C.c_double)]


class kvop_plan_report(C.Structure):
    _fields_ = [("tp", C.c_double), ("fp", C.c_double), ("fn", C.c_double), ("recall_lb", C.c_double),
                ("precision_lb", C.c_double), ("cost_frac", C.c_double)]


class PlanProblem:
    """Host arrays of a kvop_plan_problem kept alive with the struct.
    log_odds: per filter [n_j, S]; cost: per filter [n_j]; gold: per filter [S] (0/1)."""

    def __init__(self, log_odds, cost, gold, target_recall, target_precision, alpha):
        self.n_ops = np.array([np.asarray(x).shape[0] for x in log_odds], np.int32)
        self.lo = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float32) for x in log_odds]), np.float32)
        self.cost = np.ascontiguousarray(np.concatenate([np.asarray(c, np.float64) for c in cost]), np.float64)
        self.gold = np.ascontiguousarray(np.stack([np.asarray(g, np.int8) for g in gold]), np.int8)
        self.n_total = int(self.n_ops.sum())
        self.s = kvop_plan_problem(len(self.n_ops), self.n_ops.ctypes.data, self.cost.ctypes.data,
                                   self.lo.ctypes.data, self.gold.ctypes.data, int(self.lo.shape[1]),
                                   float(target_recall), float(target_precision), float(alpha))


def _report(r: kvop_plan_report) -> dict:
    return {k: getattr(r, k) for k, _ in kvop_plan_report._fields_}


def kvop_plan_optimize(pb: PlanProblem, steps=300, lr=0.05, beta=10.0, tau0=1.0, tau_end=0.02, theta0=1.0) -> dict:
    o = kvop_plan_opts(int(steps), float(lr), float(beta), float(tau0), float(tau_end), float(theta0))
    n = pb.n_total
    params = np.zeros(3 * n, np.float64)
    sel = np.zeros(n, np.int8)
    tp, tn = np.zeros(n, np.float32), np.zeros(n, np.float32)
    trace = np.zeros(int(steps), np.float64)
    rep = kvop_plan_report()
    _check(lib().kvop_plan_optimize(C.byref(pb.s), C.byref(o), params.ctypes.data, sel.ctypes.data, tp.ctypes.data,
                                    tn.ctypes.data, trace.ctypes.data, C.byref(rep)))
    return {"params": params, "selected": sel, "theta_pos": tp, "theta_neg": tn, "trace": trace,
            "report": _report(rep)}


def kvop_plan_loss(pb: PlanProblem, params, tau: float, beta: float):
    p = np.ascontiguousarray(params, np.float64)
    g = np.zeros(3 * pb.n_total, np.float64)
    out = C.c_double()
    _check(lib().kvop_plan_loss(C.byref(pb.s), p.ctypes.data, float(tau), float(beta), C.byref(out), g.ctypes.data))
    return out.value, g


def kvop_plan_evaluate(pb: PlanProblem, selected, theta_pos, theta_neg) -> dict:
    sel = np.ascontiguousarray(selected, np.int8)
    tp, tn = np.ascontiguousarray(theta_pos, np.float32), np.ascontiguousarray(theta_neg, np.float32)
    n, S = pb.n_total, pb.lo.shape[1]
    inter, intra = np.zeros(n), np.zeros(n)
    proc, acc = np.zeros(n, np.int32), np.zeros(S, np.int8)
    rep = kvop_plan_report()
    _check(lib().kvop_plan_evaluate(C.byref(pb.s), sel.ctypes.data, tp.ctypes.data, tn.ctypes.data, C.byref(rep),
                                    inter.ctypes.data, intra.ctypes.data, proc.ctypes.data, acc.ctypes.data))
    return {"report": _report(rep), "sel_inter": inter, "sel_intra": intra, "processed": proc, "accept": acc}


def kvop_plan_reorder(impl, cost, sel_inter, sel_intra, n_tuples: float):
    im = np.ascontiguousarray(impl, np.int32)
    c, si, sa = (np.ascontiguousarray(x, np.float64) for x in (cost, sel_inter, sel_intra))
    order = np.zeros(len(im), np.int32)
    out = C.c_double()
    _check(lib().kvop_plan_reorder(len(im), im.ctypes.data, c.ctypes.data, si.ctypes.data, sa.ctypes.data,
                                   float(n_tuples), order.ctypes.data, C.byref(out)))
    return order, out.value


def kvop_beta_lower_bound(a: float, b: float, alpha: float) -> float:
    out = C.c_double()
    _check(lib().kvop_beta_lower_bound(float(a), float(b), float(alpha), C.byref(out)))
    return out.value
