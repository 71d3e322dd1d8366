"""Thin ctypes binding of libhicr.so (argument marshalling only).

Function names match the C ABI in include/hicr.h.  Every function returns the
C return code first, followed by any output values.  Device buffers are
passed as integer addresses (e.g. ``tensor.data_ptr()``); streams as integer
hipStream_t handles (e.g. ``torch.cuda.current_stream().cuda_stream``) or 0
for the context's own stream.

The library must have been built (``paper_2509_01425_amd.build``); there is no
fallback: importing this module on a machine without the built library
raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhicr.so")

OK = 0
EINVAL = -1
ERANGE = -2
EBADSLOT = -3
EUNSUPPORTED = -4
EAGAIN = -5
ENOMEM = -6
ETIMEDOUT = -7
EHAZARD = -8
EDEVICE = -9
EBUSY = -10

MEM_HBM = 0
MEM_HOST = 1

SCHED_FIXED = 0
SCHED_TUNED = 1
SCHED_LEARNED = 2
NUM_CLASSES = 12

DESC_DTYPE = np.dtype(
    [("dst_slot", "<u4"), ("src_slot", "<u4"), ("dst_off", "<u8"),
     ("src_off", "<u8"), ("size", "<u8")], align=True)


class hicr_sched(ctypes.Structure):
    _fields_ = [("chunk_bytes", ctypes.c_uint32), ("wgs_per_desc", ctypes.c_uint32),
                ("unroll", ctypes.c_uint32), ("mode", ctypes.c_uint32)]


CH_FIXED, CH_VAR = 0, 1
CH_SPSC, CH_MPSC_LOCK, CH_MPSC_NOLOCK = 0, 1, 2
CH_HOST, CH_DEVICE = 0, 1
CH_MAX_PRODUCERS = 64


class hicr_channel_cfg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("producers", ctypes.c_uint32), ("endpoints", ctypes.c_uint32),
                ("token_bytes", ctypes.c_uint64), ("capacity", ctypes.c_uint64),
                ("entries", ctypes.c_uint64), ("payload", ctypes.c_uint32),
                ("entries_slot", ctypes.c_uint32)]


class hicr_stream(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_void_p), ("producer", ctypes.c_uint32),
                ("src", ctypes.c_uint32), ("out", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("first_msg", ctypes.c_uint64), ("n_msgs", ctypes.c_uint64)]


class hicr_pump_io(ctypes.Structure):
    _fields_ = [("msg_src_off", ctypes.c_void_p), ("msg_size", ctypes.c_void_p),
                ("n_msgs", ctypes.c_uint64), ("trace_dev", ctypes.c_void_p),
                ("ts_dev", ctypes.c_void_p), ("timeout_ns", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


PUMP_DEVICE_TABLES = 0x1


REQ_COPY, REQ_BURST = 0, 1


class hicr_request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("channel", ctypes.c_uint32),
                ("first", ctypes.c_uint64), ("count", ctypes.c_uint64),
                ("hbm_bytes", ctypes.c_uint64), ("arrival_ns", ctypes.c_uint64)]


ON_COMPLETE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64)


class hicr_serve_cfg(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_uint32), ("src", ctypes.c_uint32),
                ("streams", ctypes.c_uint32), ("max_batch_reqs", ctypes.c_uint32),
                ("descs", ctypes.c_void_p), ("n_descs", ctypes.c_uint64),
                ("msg_src_off", ctypes.c_void_p), ("msg_size", ctypes.c_void_p),
                ("n_msgs", ctypes.c_uint64), ("channels", ctypes.c_void_p),
                ("n_channels", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("sched_or_null", ctypes.c_void_p), ("on_complete", ON_COMPLETE),
                ("user", ctypes.c_void_p), ("admit_ns", ctypes.c_void_p),
                ("done_ns", ctypes.c_void_p)]


class hicr_serve_stats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_uint64), ("peak_arena_bytes", ctypes.c_uint64),
                ("copy_launches", ctypes.c_uint64), ("pump_launches", ctypes.c_uint64),
                ("max_inflight_requests", ctypes.c_uint64), ("wall_ns", ctypes.c_uint64)]


class hicr_dev_ring(ctypes.Structure):
    _fields_ = [("payload", ctypes.c_uint64), ("P", ctypes.c_uint64), ("entries", ctypes.c_uint64),
                ("E", ctypes.c_uint64), ("coord", ctypes.c_uint64), ("producer", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class hicr_dobj_handle(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("size", ctypes.c_uint64), ("offset", ctypes.c_uint64),
                ("slot", ctypes.c_uint32), ("memspace", ctypes.c_uint32)]


_u32, _u64, _vp, _int = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
_pu32, _pu64, _pvp = ctypes.POINTER(_u32), ctypes.POINTER(_u64), ctypes.POINTER(_vp)

_SIGNATURES = {
    "hicr_sched_class": (_int, [_u32, ctypes.POINTER(hicr_sched)]),
    "hicr_ctx_create": (_int, [_int, _vp, _pvp]),
    "hicr_ctx_destroy": (_int, [_vp]),
    "hicr_strerror": (ctypes.c_char_p, [_int]),
    "hicr_last_error": (_int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "hicr_ctx_set_sched": (_int, [_vp, ctypes.POINTER(hicr_sched)]),
    "hicr_ctx_set_copy_grid": (_int, [_vp, _u32]),
    "hicr_ctx_set_pairs": (_int, [_vp, _u32]),
    "hicr_slot_register": (_int, [_vp, _vp, _u64, _u32, _pu32]),
    "hicr_slot_deregister": (_int, [_vp, _u32]),
    "hicr_slot_counters": (_int, [_vp, _u32, _pu64, _pu64]),
    "hicr_memcpy": (_int, [_vp, _u32, _u64, _u32, _u64, _u64]),
    "hicr_memcpy_batch": (_int, [_vp, _vp, _u64, ctypes.POINTER(hicr_sched), _vp, _pu64]),
    "hicr_memcpy_batch_noalloc": (_int, [_vp, _vp, _u64, ctypes.POINTER(hicr_sched), _vp,
                                         _pu64]),
    "hicr_fence": (_int, [_vp]),
    "hicr_fence_slot": (_int, [_vp, _u32, _u64, _u64, _u64]),
    "hicr_dobj_publish": (_int, [_vp, _u32, _u64, _u64, _pu64]),
    "hicr_dobj_get_handle": (_int, [_vp, _u64, ctypes.POINTER(hicr_dobj_handle)]),
    "hicr_dobj_get": (_int, [_vp, ctypes.POINTER(hicr_dobj_handle), _u32, _u64]),
    "hicr_dobj_unpublish": (_int, [_vp, _u64]),
    "hicr_plan_create": (_int, [_vp, _vp, _u64, ctypes.POINTER(hicr_sched), _u32, _pvp, _pu64]),
    "hicr_plan_launch": (_int, [_vp, _vp]),
    "hicr_plan_destroy": (_int, [_vp]),
    "hicr_channel_create": (_int, [_vp, ctypes.POINTER(hicr_channel_cfg), _pvp]),
    "hicr_channel_destroy": (_int, [_vp]),
    "hicr_channel_push": (_int, [_vp, _u32, _u32, _u64, _u64]),
    "hicr_channel_peek": (_int, [_vp, _u32, _u64, _pu64, _pu64, _pu32]),
    "hicr_channel_pop": (_int, [_vp, _u32, _u64]),
    "hicr_channel_depth": (_int, [_vp, _u32, _pu64, _pu64]),
    "hicr_channel_pump": (_int, [_vp, ctypes.POINTER(hicr_stream), _u32,
                                 ctypes.POINTER(hicr_pump_io), _vp]),
    "hicr_channel_abort": (_int, [_vp]),
    "hicr_channel_device_view": (_int, [_vp, _u32, ctypes.POINTER(hicr_dev_ring)]),
    "hicr_sched_features": (_int, [_vp, _u64, _vp]),
    "hicr_autotune": (_int, [_vp, _vp, _u64, _u32, _vp, _pu32]),
    "hicr_tune_add": (_int, [_vp, _vp, _u64, _u32]),
    "hicr_tune_clear": (_int, [_vp]),
    "hicr_tune_lookup": (_int, [_vp, _vp, _u64, _pu32]),
    "hicr_mlp_set_params": (_int, [_vp, _vp]),
    "hicr_mlp_get_params": (_int, [_vp, _vp]),
    "hicr_mlp_forward": (_int, [_vp, _vp, _u32, _vp]),
    "hicr_mlp_grad": (_int, [_vp, _vp, _vp, _u32, _vp, _vp]),
    "hicr_mlp_train_step": (_int, [_vp, _vp, _vp, _u32, ctypes.c_float, _vp]),
    "hicr_last_choice": (_int, [_vp, _pu32]),
    "hicr_pingpong": (_int, [_vp, _u32, _u32, _u32, _u32, _u32, _vp, _u32, _u32, _u32, _vp]),
    "hicr_serve": (_int, [_vp, _vp, _u64, ctypes.POINTER(hicr_serve_cfg),
                          ctypes.POINTER(hicr_serve_stats)]),
}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2509_01425_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


# ------------------------------------------------------------------ calls

def hicr_sched_class(cls: int):
    s = hicr_sched()
    rc = lib().hicr_sched_class(cls, ctypes.byref(s))
    return rc, s


def make_sched(chunk_bytes: int, wgs_per_desc: int, unroll: int, mode: int = SCHED_FIXED):
    return hicr_sched(chunk_bytes, wgs_per_desc, unroll, mode)


def hicr_ctx_create(device: int = 0, stream: int = 0):
    out = _vp()
    rc = lib().hicr_ctx_create(device, stream or None, ctypes.byref(out))
    return rc, out.value


def hicr_ctx_destroy(ctx) -> int:
    return lib().hicr_ctx_destroy(ctx)


def hicr_strerror(code: int) -> str:
    return lib().hicr_strerror(code).decode()


def hicr_last_error(ctx) -> str:
    buf = ctypes.create_string_buffer(512)
    lib().hicr_last_error(ctx, buf, 512)
    return buf.value.decode()


def hicr_ctx_set_sched(ctx, sched: hicr_sched) -> int:
    return lib().hicr_ctx_set_sched(ctx, ctypes.byref(sched))


def hicr_ctx_set_copy_grid(ctx, wgs_per_cu: int) -> int:
    return lib().hicr_ctx_set_copy_grid(ctx, wgs_per_cu)


def hicr_ctx_set_pairs(ctx, pair_mask: int) -> int:
    return lib().hicr_ctx_set_pairs(ctx, pair_mask)


def PAIR(dst_space: int, src_space: int) -> int:
    return 1 << (2 * dst_space + src_space)


PAIRS_ALL = 0xF


def hicr_slot_register(ctx, ptr: int, size: int, memspace: int = MEM_HBM):
    out = _u32()
    rc = lib().hicr_slot_register(ctx, ptr, size, memspace, ctypes.byref(out))
    return rc, out.value


def hicr_slot_deregister(ctx, slot: int) -> int:
    return lib().hicr_slot_deregister(ctx, slot)


def hicr_slot_counters(ctx, slot: int):
    s, r = _u64(), _u64()
    rc = lib().hicr_slot_counters(ctx, slot, ctypes.byref(s), ctypes.byref(r))
    return rc, s.value, r.value


def hicr_memcpy(ctx, dst: int, dst_off: int, src: int, src_off: int, size: int) -> int:
    return lib().hicr_memcpy(ctx, dst, dst_off, src, src_off, size)


def hicr_memcpy_batch(ctx, descs: np.ndarray, sched=None, stream: int = 0):
    d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
    bad = _u64(0)
    rc = lib().hicr_memcpy_batch(ctx, d.ctypes.data if d.size else None, d.size,
                                 ctypes.byref(sched) if sched is not None else None,
                                 stream or None, ctypes.byref(bad))
    return rc, bad.value


def hicr_memcpy_batch_noalloc(ctx, descs: np.ndarray, sched=None, stream: int = 0):
    d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
    bad = _u64(0)
    rc = lib().hicr_memcpy_batch_noalloc(ctx, d.ctypes.data if d.size else None, d.size,
                                         ctypes.byref(sched) if sched is not None else None,
                                         stream or None, ctypes.byref(bad))
    return rc, bad.value


def hicr_fence(ctx) -> int:
    return lib().hicr_fence(ctx)


def hicr_fence_slot(ctx, slot: int, exp_sent: int, exp_recv: int, timeout_ns: int) -> int:
    return lib().hicr_fence_slot(ctx, slot, exp_sent, exp_recv, timeout_ns)


PLAN_GRAPH = 1


def hicr_plan_create(ctx, descs: np.ndarray, sched=None, flags: int = 0):
    """Returns (rc, plan handle, bad index)."""
    d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
    out, bad = _vp(), _u64(0)
    rc = lib().hicr_plan_create(ctx, d.ctypes.data if d.size else None, d.size,
                                ctypes.byref(sched) if sched is not None else None, flags,
                                ctypes.byref(out), ctypes.byref(bad))
    return rc, out.value, bad.value


def hicr_plan_launch(plan, stream: int = 0) -> int:
    return lib().hicr_plan_launch(plan, stream or None)


def hicr_plan_destroy(plan) -> int:
    return lib().hicr_plan_destroy(plan)


def hicr_dobj_publish(ctx, slot: int, offset: int, size: int):
    out = _u64(0)
    rc = lib().hicr_dobj_publish(ctx, slot, offset, size, ctypes.byref(out))
    return rc, out.value


def hicr_dobj_get_handle(ctx, obj_id: int):
    h = hicr_dobj_handle()
    rc = lib().hicr_dobj_get_handle(ctx, obj_id, ctypes.byref(h))
    return rc, h


def hicr_dobj_get(ctx, handle: hicr_dobj_handle, dst: int, dst_off: int) -> int:
    return lib().hicr_dobj_get(ctx, ctypes.byref(handle), dst, dst_off)


def hicr_dobj_unpublish(ctx, obj_id: int) -> int:
    return lib().hicr_dobj_unpublish(ctx, obj_id)


# --------------------------------------------------------------- channels

def make_channel_cfg(kind, mode, producers, endpoints, payload, entries_slot,
                     token_bytes=0, capacity=0, entries=0):
    return hicr_channel_cfg(kind, mode, producers, endpoints, token_bytes, capacity, entries,
                            payload, entries_slot)


def hicr_channel_create(ctx, cfg: hicr_channel_cfg):
    out = _vp()
    rc = lib().hicr_channel_create(ctx, ctypes.byref(cfg), ctypes.byref(out))
    return rc, out.value


def hicr_channel_device_view(ch, ring: int = 0):
    v = hicr_dev_ring()
    rc = lib().hicr_channel_device_view(ch, ring, ctypes.byref(v))
    return rc, v


def hicr_channel_destroy(ch) -> int:
    return lib().hicr_channel_destroy(ch)


def hicr_channel_push(ch, producer: int, src: int, src_off: int, count: int) -> int:
    return lib().hicr_channel_push(ch, producer, src, src_off, count)


def hicr_channel_peek(ch, ring: int, i: int):
    off, size, prod = _u64(), _u64(), _u32()
    rc = lib().hicr_channel_peek(ch, ring, i, ctypes.byref(off), ctypes.byref(size),
                                 ctypes.byref(prod))
    return rc, off.value, size.value, prod.value


def hicr_channel_pop(ch, ring: int, n: int) -> int:
    return lib().hicr_channel_pop(ch, ring, n)


def hicr_channel_depth(ch, ring: int):
    m, b = _u64(), _u64()
    rc = lib().hicr_channel_depth(ch, ring, ctypes.byref(m), ctypes.byref(b))
    return rc, m.value, b.value


def hicr_channel_pump(ctx, streams, msg_src_off, msg_size, trace_dev: int = 0, ts_dev: int = 0,
                      timeout_ns: int = 0, stream: int = 0, n_msgs: int = None):
    """streams: sequence of (channel, producer, src_slot, out_slot, first_msg, n_msgs).
    msg_src_off / msg_size: host arrays, or device addresses (ints, with
    n_msgs given) for HICR_PUMP_DEVICE_TABLES."""
    arr = (hicr_stream * max(len(streams), 1))()
    for i, (ch, p, src, out, first, n) in enumerate(streams):
        arr[i] = hicr_stream(ch, p, src, out, 0, first, n)
    if isinstance(msg_src_off, int):
        io = hicr_pump_io(msg_src_off or None, msg_size or None, n_msgs, trace_dev or None,
                          ts_dev or None, timeout_ns, PUMP_DEVICE_TABLES, 0)
    else:
        off = np.ascontiguousarray(msg_src_off, dtype=np.uint64)
        size = np.ascontiguousarray(msg_size, dtype=np.uint64)
        io = hicr_pump_io(off.ctypes.data if off.size else None,
                          size.ctypes.data if size.size else None, off.size, trace_dev or None,
                          ts_dev or None, timeout_ns, 0, 0)
    return lib().hicr_channel_pump(ctx, arr, len(streams), ctypes.byref(io), stream or None)


def hicr_channel_abort(ctx) -> int:
    return lib().hicr_channel_abort(ctx)


# ------------------------------------------------------ schedule selection

MLP_PARAMS = 7052


def _descs(descs):
    return np.ascontiguousarray(descs, dtype=DESC_DTYPE)


def hicr_sched_features(descs: np.ndarray):
    d = _descs(descs)
    out = np.zeros(32, dtype=np.float32)
    rc = lib().hicr_sched_features(d.ctypes.data if d.size else None, d.size, out.ctypes.data)
    return rc, out


def hicr_autotune(ctx, descs: np.ndarray, reps: int = 3):
    d = _descs(descs)
    times = np.zeros(NUM_CLASSES, dtype=np.float32)
    best = _u32(0)
    rc = lib().hicr_autotune(ctx, d.ctypes.data if d.size else None, d.size, reps,
                             times.ctypes.data, ctypes.byref(best))
    return rc, times, best.value


def hicr_tune_lookup(ctx, descs: np.ndarray):
    d = _descs(descs)
    out = _u32(0)
    rc = lib().hicr_tune_lookup(ctx, d.ctypes.data if d.size else None, d.size, ctypes.byref(out))
    return rc, out.value


def hicr_tune_add(ctx, descs: np.ndarray, cls: int) -> int:
    d = _descs(descs)
    return lib().hicr_tune_add(ctx, d.ctypes.data if d.size else None, d.size, cls)


def hicr_tune_clear(ctx) -> int:
    return lib().hicr_tune_clear(ctx)


def hicr_mlp_set_params(ctx, params: np.ndarray) -> int:
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == MLP_PARAMS
    return lib().hicr_mlp_set_params(ctx, p.ctypes.data)


def hicr_mlp_get_params(ctx):
    out = np.zeros(MLP_PARAMS, dtype=np.float32)
    rc = lib().hicr_mlp_get_params(ctx, out.ctypes.data)
    return rc, out


def hicr_mlp_forward(ctx, x_dev: int, batch: int, logits_dev: int) -> int:
    return lib().hicr_mlp_forward(ctx, x_dev, batch, logits_dev)


def hicr_mlp_grad(ctx, x_dev: int, y_dev: int, batch: int, grad_dev: int, loss_dev: int = 0) -> int:
    return lib().hicr_mlp_grad(ctx, x_dev, y_dev, batch, grad_dev, loss_dev or None)


def hicr_mlp_train_step(ctx, x_dev: int, y_dev: int, batch: int, lr: float,
                        loss_dev: int = 0) -> int:
    return lib().hicr_mlp_train_step(ctx, x_dev, y_dev, batch, lr, loss_dev or None)


def hicr_last_choice(ctx):
    c = _u32(0)
    rc = lib().hicr_last_choice(ctx, ctypes.byref(c))
    return rc, c.value


# ------------------------------------------------------------------ serving

def hicr_serve(ctx, reqs: np.ndarray, arena: int, src: int, descs: np.ndarray,
               msg_src_off: np.ndarray, msg_size: np.ndarray, channels, streams: int = 2,
               max_batch_reqs: int = 64, sched=None, on_complete=None, admit_ns=None,
               done_ns=None):
    """reqs: structured array with the fields of hicr_request (40 bytes each).
    on_complete(request, arena_off) is called on this thread.  admit_ns /
    done_ns: optional uint64 numpy arrays of len(reqs), filled in place.
    Returns (rc, stats)."""
    assert reqs.dtype.itemsize == ctypes.sizeof(hicr_request)
    r = np.ascontiguousarray(reqs)
    d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
    mo = np.ascontiguousarray(msg_src_off, dtype=np.uint64)
    ms = np.ascontiguousarray(msg_size, dtype=np.uint64)
    ch = (ctypes.c_void_p * max(len(channels), 1))(*channels)
    cb = ON_COMPLETE(lambda user, q, off: on_complete(int(q), int(off))) if on_complete \
        else ON_COMPLETE()
    cfg = hicr_serve_cfg(arena, src, streams, max_batch_reqs,
                         d.ctypes.data if d.size else None, d.size,
                         mo.ctypes.data if mo.size else None, ms.ctypes.data if ms.size else None,
                         mo.size, ctypes.cast(ch, ctypes.c_void_p), len(channels), 0,
                         ctypes.addressof(sched) if sched is not None else None, cb, None,
                         admit_ns.ctypes.data if admit_ns is not None else None,
                         done_ns.ctypes.data if done_ns is not None else None)
    st = hicr_serve_stats()
    rc = lib().hicr_serve(ctx, r.ctypes.data if r.size else None, r.size, ctypes.byref(cfg),
                          ctypes.byref(st))
    return rc, st


def hicr_pingpong(ctx, src: int, dst: int, ring_a: int, ring_b: int, buf: int, sizes, reps: int,
                  wgs_per_endpoint: int = 0):
    sz = np.ascontiguousarray(sizes, dtype=np.uint64)
    out = np.zeros(sz.size * reps, dtype=np.uint64)
    rc = lib().hicr_pingpong(ctx, src, dst, ring_a, ring_b, buf, sz.ctypes.data, sz.size, reps,
                             wgs_per_endpoint, out.ctypes.data)
    return rc, out.reshape(sz.size, reps)
