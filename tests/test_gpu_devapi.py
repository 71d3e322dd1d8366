"""GPU parity of the device-side channel API (hicr_device.h): a producer and
a consumer workgroup of the caller's own kernel move seeded messages through
one ring; the consumer's output equals the oracle's FIFO ring output."""
import ctypes
import os

import numpy as np
import pytest

from tests.parity import oracle_fifo_outputs
from workloads import memcpy as wm
from workloads.content import content

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    L = ctypes.CDLL(os.path.join(HERE, "devapi", "libdevapi.so"))
    L.devapi_pipe_run.restype = ctypes.c_int
    L.devapi_pipe_run.argtypes = [ctypes.POINTER(H.hicr_dev_ring), ctypes.c_uint64, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                  ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    yield torch, H, wd, ctx, L
    assert H.hicr_ctx_destroy(ctx) == H.OK


def _channel(torch, H, ctx, mode, K, P, E):
    rings = K if mode == H.CH_MPSC_NOLOCK else 1
    pay = torch.zeros(rings * P, dtype=torch.uint8, device="cuda")
    ent = torch.zeros(rings * E, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    _, ps = H.hicr_slot_register(ctx, pay.data_ptr(), rings * P)
    _, es = H.hicr_slot_register(ctx, ent.data_ptr(), rings * E * 8)
    rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, mode, K, H.CH_DEVICE, ps, es,
                                                           capacity=P, entries=E))
    assert rc == H.OK, H.hicr_last_error(ctx)
    return ch, (pay, ent, ps, es)


def _run(torch, H, wd, L, view, sizes, seed, batch):
    g = np.random.default_rng(seed)
    src_n = int(sizes.sum()) + 4096
    src = torch.empty(src_n, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), src_n, seed)
    offs = (g.random(len(sizes)) * (src_n - sizes + 1)).astype(np.int64)
    out = torch.zeros(int(sizes.sum()) + 64, dtype=torch.uint8, device="cuda")
    off_d = torch.from_numpy(offs).cuda()
    size_d = torch.from_numpy(sizes.astype(np.int64)).cuda()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    eag = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    rc = L.devapi_pipe_run(ctypes.byref(view), src.data_ptr(), off_d.data_ptr(), size_d.data_ptr(),
                           len(sizes), out.data_ptr(), batch, 2 * 10**8, err.data_ptr(),
                           eag.data_ptr())
    assert rc == 0 and int(err.item()) == 0, (rc, int(err.item()))
    blob = content(seed, 0, src_n)
    return out.cpu().numpy(), [blob[o:o + s] for o, s in zip(offs, sizes)], int(eag.item())


@pytest.mark.parametrize("P,E,batch", [(4096, 8, 1), (4096, 8, 3), (1 << 16, 64, 8)])
def test_user_kernel_spsc_matches_oracle(env, P, E, batch):
    torch, H, wd, ctx, L = env
    _say("devapi spsc", P, E, batch)
    ch, keep = _channel(torch, H, ctx, H.CH_SPSC, 1, P, E)
    rc, view = H.hicr_channel_device_view(ch, 0)
    assert rc == H.OK and view.P == P and view.E == E
    g = np.random.default_rng(P + batch)
    sizes = wm.log_uniform(g, 1, P, 400).astype(np.int64)
    sizes[:4] = [0, P, 1, P - 1]
    got, msgs, eagain = _run(torch, H, wd, L, view, sizes, 90 + batch, batch)
    want = oracle_fifo_outputs(P, E, msgs)
    assert np.array_equal(got[:len(want)], want)
    assert not got[len(want):].any()
    if P == 4096:
        assert eagain > 0          # the small ring pushed back on the producer
    assert H.hicr_channel_destroy(ch) == H.OK


def test_user_kernel_nolock_subring_after_pump(env):
    """A non-locking MPSC channel pumped once by the library, then one of its
    sub-rings driven by user kernels: the producer resumes at the ring's
    published counters; afterwards the pump refuses the channel."""
    torch, H, wd, ctx, L = env
    P, E, K = 8192, 16, 3
    ch, keep = _channel(torch, H, ctx, H.CH_MPSC_NOLOCK, K, P, E)
    # pump 40 messages through producer 1's ring with the library first
    g = np.random.default_rng(7)
    n0 = 40
    sz0 = wm.log_uniform(g, 1, P, n0).astype(np.uint64)
    src = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), 1 << 20, 11)
    out0 = torch.zeros(int(sz0.sum()) + 64, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    _, ss = H.hicr_slot_register(ctx, src.data_ptr(), 1 << 20)
    _, os0 = H.hicr_slot_register(ctx, out0.data_ptr(), out0.numel())
    offs0 = (g.random(n0) * ((1 << 20) - sz0.astype(np.float64) + 1)).astype(np.uint64)
    streams = [(ch, 1, ss, os0, 0, n0)]
    assert H.hicr_channel_pump(ctx, streams, offs0, sz0) == H.OK, H.hicr_last_error(ctx)
    assert H.hicr_fence(ctx) == H.OK
    blob = content(11, 0, 1 << 20)
    msgs0 = [blob[int(o):int(o) + int(s)] for o, s in zip(offs0, sz0)]
    want0 = oracle_fifo_outputs(P, E, msgs0)
    assert np.array_equal(out0.cpu().numpy()[:len(want0)], want0)
    # then user kernels on the same ring
    rc, view = H.hicr_channel_device_view(ch, 1)
    assert rc == H.OK and view.producer == 1
    sizes = wm.log_uniform(g, 1, P, 200).astype(np.int64)
    got, msgs, _ = _run(torch, H, wd, L, view, sizes, 33, 2)
    want = oracle_fifo_outputs(P, E, msgs)
    assert np.array_equal(got[:len(want)], want)
    assert H.hicr_channel_pump(ctx, streams, offs0, sz0) == H.EINVAL
    assert H.hicr_channel_destroy(ch) == H.OK


def test_device_view_rejections(env):
    torch, H, wd, ctx, L = env
    ch, keep = _channel(torch, H, ctx, H.CH_MPSC_LOCK, 2, 4096, 8)
    assert H.hicr_channel_device_view(ch, 0)[0] == H.EUNSUPPORTED
    assert H.hicr_channel_destroy(ch) == H.OK
    ch, keep = _channel(torch, H, ctx, H.CH_SPSC, 1, 4096, 8)
    assert H.hicr_channel_device_view(ch, 1)[0] == H.EINVAL
    assert H.hicr_channel_destroy(ch) == H.OK
    buf = torch.zeros(8192, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    _, b = H.hicr_slot_register(ctx, buf.data_ptr(), 8192)
    rc, hch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, H.CH_SPSC, 1, H.CH_HOST, b, b,
                                                            capacity=4096, entries=8))
    assert rc == H.OK
    assert H.hicr_channel_device_view(hch, 0)[0] == H.EINVAL
    assert H.hicr_channel_destroy(hch) == H.OK
