"""CPU oracle for the HiCR communication-manager data path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2509_01425_amd``) and never imports it.

Contents:
  * ``Ctx``      -- slots, memcpy, batches, counters, fence (paper Sec. 3.1.3,
                    3.1.4), backed by ``liboracle.so`` (plain C byte loops);
  * ``FChan``    -- fixed-size SPSC ring (Sec. 4.3, Channels);
  * ``VChan``    -- variable-size ring; SPSC, and the shared ring of a locking
                    MPSC channel when producer tags are kept (Sec. 4.3);
  * ``mlp``      -- fp64 reference of the schedule-predicting network;
  * ``protocol`` -- step-level model of the ring protocol with an exhaustive
                    interleaving explorer;
  * ``protocol_kernels`` -- the same for the refinements the device kernels
                    run: batched publication and consumption, the team drain
                    of a locking ring, ping-pong's striped counters.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK = 0
EINVAL = -1
ERANGE = -2
EBADSLOT = -3
EUNSUPPORTED = -4
EAGAIN = -5
ENOMEM = -6
ETIMEDOUT = -7
EHAZARD = -8

MEM_HBM = 0
MEM_HOST = 1
# A context accepts HBM -> HBM transfers unless created with another pair
# matrix (bit 2 * dst_space + src_space; 0b1111 accepts every pair).
PAIR_HBM_HBM = 1 << (2 * MEM_HBM + MEM_HBM)

DESC_DTYPE = np.dtype(
    [("dst_slot", "<u4"), ("src_slot", "<u4"), ("dst_off", "<u8"),
     ("src_off", "<u8"), ("size", "<u8")], align=True)
assert DESC_DTYPE.itemsize == 32

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u32, u64, vp, i = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        pu32, pu64 = ctypes.POINTER(u32), ctypes.POINTER(u64)
        sig = {
            "or_ctx_create": (vp, [u32]),
            "or_ctx_destroy": (None, [vp]),
            "or_slot_register": (i, [vp, vp, u64, u32, pu32]),
            "or_slot_deregister": (i, [vp, u32]),
            "or_slot_counters": (i, [vp, u32, pu64, pu64]),
            "or_memcpy": (i, [vp, u32, u64, u32, u64, u64]),
            "or_memcpy_batch": (i, [vp, vp, u64, pu64]),
            "or_count_batch": (i, [vp, vp, u64, pu64]),
            "or_hazard_check": (i, [vp, vp, u64, pu64, pu64]),
            "or_fence": (i, [vp]),
            "or_fence_slot": (i, [vp, u32, u64, u64]),
            "or_copy_bytes": (None, [vp, vp, u64]),
            "or_fchan_init": (i, [vp, vp, u64, u64]),
            "or_fchan_push": (i, [vp, vp, u64]),
            "or_fchan_peek": (i, [vp, u64, pu64]),
            "or_fchan_pop": (i, [vp, u64]),
            "or_fchan_depth": (u64, [vp]),
            "or_vchan_init": (i, [vp, vp, u64, vp, vp, u64]),
            "or_vchan_push": (i, [vp, u32, vp, u64]),
            "or_vchan_peek": (i, [vp, u64, pu64, pu64, pu32]),
            "or_vchan_read": (i, [vp, u64, vp]),
            "or_vchan_pop": (i, [vp, u64]),
            "or_vchan_depth": (None, [vp, pu64, pu64]),
            "or_vchan_replay": (i, [vp, u32, vp, u64, vp, vp, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def copy_bytes(dst: np.ndarray, src: np.ndarray, n: int) -> None:
    lib().or_copy_bytes(_ptr(dst), _ptr(src), n)


class Ctx:
    """Slots, memcpy, counters and fence over host buffers."""

    def __init__(self, pair_mask: int = PAIR_HBM_HBM):
        self._c = lib().or_ctx_create(pair_mask)
        self._keep = []  # buffers registered as slots stay alive with the ctx

    def __del__(self):
        if getattr(self, "_c", None):
            lib().or_ctx_destroy(self._c)
            self._c = None

    def register(self, buf: np.ndarray, space: int = MEM_HBM, offset: int = 0, size=None):
        """Register ``buf[offset:offset+size]`` (bytes); returns (rc, slot)."""
        assert buf.dtype == np.uint8 and buf.flags.c_contiguous
        size = buf.size - offset if size is None else size
        out = ctypes.c_uint32(0)
        base = _ptr(buf) + offset if buf.size else 0
        rc = lib().or_slot_register(self._c, base, size, space, ctypes.byref(out))
        if rc == OK:
            self._keep.append(buf)
        return rc, out.value

    def register_raw(self, addr: int, size: int, space: int = MEM_HBM):
        out = ctypes.c_uint32(0)
        rc = lib().or_slot_register(self._c, addr, size, space, ctypes.byref(out))
        return rc, out.value

    def deregister(self, slot: int) -> int:
        return lib().or_slot_deregister(self._c, slot)

    def counters(self, slot: int):
        s, r = ctypes.c_uint64(), ctypes.c_uint64()
        rc = lib().or_slot_counters(self._c, slot, ctypes.byref(s), ctypes.byref(r))
        return rc, s.value, r.value

    def memcpy(self, dst, dst_off, src, src_off, size) -> int:
        return lib().or_memcpy(self._c, dst, dst_off, src, src_off, size)

    def memcpy_batch(self, descs: np.ndarray):
        d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
        bad = ctypes.c_uint64(0)
        rc = lib().or_memcpy_batch(self._c, _ptr(d) if d.size else None, d.size,
                                   ctypes.byref(bad))
        return rc, bad.value

    def count_batch(self, descs: np.ndarray):
        d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
        bad = ctypes.c_uint64(0)
        rc = lib().or_count_batch(self._c, _ptr(d) if d.size else None, d.size,
                                  ctypes.byref(bad))
        return rc, bad.value

    def hazard_check(self, descs: np.ndarray):
        d = np.ascontiguousarray(descs, dtype=DESC_DTYPE)
        a, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
        rc = lib().or_hazard_check(self._c, _ptr(d) if d.size else None, d.size,
                                   ctypes.byref(a), ctypes.byref(b))
        return rc, a.value, b.value

    def fence(self) -> int:
        return lib().or_fence(self._c)

    def fence_slot(self, slot, exp_sent, exp_recv) -> int:
        return lib().or_fence_slot(self._c, slot, exp_sent, exp_recv)


class _FChanC(ctypes.Structure):
    _fields_ = [("ring", ctypes.c_void_p), ("C", ctypes.c_uint64), ("T", ctypes.c_uint64),
                ("head", ctypes.c_uint64), ("tail", ctypes.c_uint64)]


class FChan:
    """Fixed-size SPSC ring of C tokens of T bytes."""

    def __init__(self, C: int, T: int):
        self.ring = np.zeros(max(C * T, 1), dtype=np.uint8)
        self._s = _FChanC()
        self.rc_init = lib().or_fchan_init(ctypes.byref(self._s), _ptr(self.ring), C, T)

    @property
    def head(self):
        return self._s.head

    @property
    def tail(self):
        return self._s.tail

    def push(self, src: np.ndarray, k: int) -> int:
        return lib().or_fchan_push(ctypes.byref(self._s), _ptr(src) if src.size else None, k)

    def peek(self, i: int):
        off = ctypes.c_uint64(0)
        rc = lib().or_fchan_peek(ctypes.byref(self._s), i, ctypes.byref(off))
        return rc, off.value

    def pop(self, n: int) -> int:
        return lib().or_fchan_pop(ctypes.byref(self._s), n)

    def depth(self) -> int:
        return lib().or_fchan_depth(ctypes.byref(self._s))


class _VChanC(ctypes.Structure):
    _fields_ = [("payload", ctypes.c_void_p), ("P", ctypes.c_uint64),
                ("sizes", ctypes.c_void_p), ("tags", ctypes.c_void_p), ("E", ctypes.c_uint64),
                ("hm", ctypes.c_uint64), ("tm", ctypes.c_uint64),
                ("hb", ctypes.c_uint64), ("tb", ctypes.c_uint64)]


class VChan:
    """Variable-size ring: P payload bytes, E size entries.  With
    ``tagged=True`` every entry also records its producer (the shared ring of
    a locking MPSC channel)."""

    def __init__(self, P: int, E: int, tagged: bool = False):
        self.payload = np.zeros(max(P, 1), dtype=np.uint8)
        self.sizes = np.zeros(max(E, 1), dtype=np.uint64)
        self.tags = np.zeros(max(E, 1), dtype=np.uint32) if tagged else None
        self._s = _VChanC()
        self.rc_init = lib().or_vchan_init(
            ctypes.byref(self._s), _ptr(self.payload), P, _ptr(self.sizes),
            _ptr(self.tags) if tagged else None, E)

    @property
    def state(self):
        s = self._s
        return s.hm, s.tm, s.hb, s.tb

    def push(self, src: np.ndarray, s: int, producer: int = 0) -> int:
        return lib().or_vchan_push(ctypes.byref(self._s), producer,
                                   _ptr(src) if src.size else None, s)

    def peek(self, i: int):
        off, size, prod = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint32(0)
        rc = lib().or_vchan_peek(ctypes.byref(self._s), i, ctypes.byref(off),
                                 ctypes.byref(size), ctypes.byref(prod))
        return rc, off.value, size.value, prod.value

    def read(self, i: int):
        rc, _, size, prod = self.peek(i)
        if rc != OK:
            return rc, None, None
        out = np.zeros(max(size, 1), dtype=np.uint8)
        rc = lib().or_vchan_read(ctypes.byref(self._s), i, _ptr(out))
        return rc, out[:size], prod

    def pop(self, n: int) -> int:
        return lib().or_vchan_pop(ctypes.byref(self._s), n)

    def depth(self):
        m, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
        lib().or_vchan_depth(ctypes.byref(self._s), ctypes.byref(m), ctypes.byref(b))
        return m.value, b.value


class MPSC:
    """Multiple-producer single-consumer channel (Sec. 4.3).

    ``locking=True``: one shared ring; producers take exclusive access in
    turn, so the ring holds one total order of all producers' messages.
    ``locking=False``: one dedicated ring per producer; the consumer reads
    each producer's ring in FIFO order.
    """

    def __init__(self, K: int, P: int, E: int, locking: bool):
        self.K, self.locking = K, locking
        if locking:
            self.rings = [VChan(P, E, tagged=True)]
        else:
            self.rings = [VChan(P, E) for _ in range(K)]

    def push(self, producer: int, src: np.ndarray, s: int) -> int:
        if not 0 <= producer < self.K:
            return EINVAL
        if self.locking:
            return self.rings[0].push(src, s, producer)
        return self.rings[producer].push(src, s, producer)

    def ring_for(self, producer: int) -> VChan:
        return self.rings[0] if self.locking else self.rings[producer]


def vchan_replay(P: int, E: int, order, blobs, offs, sizes, tagged: bool = False):
    """Outputs of one ring (P payload bytes, E entries) driven by one
    sequential schedule in C (``or_vchan_replay``): push t is producer
    order[t]'s next message (bytes blobs[p][offs[p][k] : + sizes[p][k]]); a
    push that finds the ring full first consumes the oldest message into the
    output of the producer its entry names, and the ring is drained at the
    end.  A producer named more often than it has messages gives EINVAL.
    Returns (rc, [output bytes of producer p]).  ``tagged`` keeps
    producer tags (the shared ring of a locking MPSC channel); untagged, every
    message goes to output 0."""
    K = len(blobs)
    ch = VChan(P, E, tagged=tagged)
    order = np.ascontiguousarray(order, dtype=np.uint32)
    blobs = [np.ascontiguousarray(b, dtype=np.uint8) for b in blobs]
    offs = [np.ascontiguousarray(o, dtype=np.uint64) for o in offs]
    sizes = [np.ascontiguousarray(z, dtype=np.uint64) for z in sizes]
    for b, o, z in zip(blobs, offs, sizes):
        if o.size != z.size or (o.size and int((o + z).max()) > b.size):
            raise ValueError("a message lies outside its producer's source bytes")
    if tagged:
        totals = [int(z.sum()) for z in sizes]
    else:
        totals = [int(sum(int(z.sum()) for z in sizes))] + [0] * (K - 1)
    outs = [np.zeros(max(t, 1), dtype=np.uint8) for t in totals]
    used = np.zeros(K, dtype=np.uint64)
    counts = np.array([z.size for z in sizes], dtype=np.uint64)
    arr = ctypes.c_void_p * K
    rc = lib().or_vchan_replay(
        ctypes.byref(ch._s), K, _ptr(order), order.size,
        arr(*[_ptr(b) for b in blobs]), arr(*[_ptr(o) for o in offs]),
        arr(*[_ptr(z) for z in sizes]), _ptr(counts), arr(*[_ptr(o) for o in outs]), _ptr(used))
    return rc, [o[:int(u)] for o, u in zip(outs, used)]
