"""GPU test of the two-endpoint ping-pong (the paper's Test Case 1 on one GPU):
after round trips of every size the pinger's buffer holds the echoed
message, byte for byte what the oracle's one-message channels deliver."""
import numpy as np
import pytest

import oracle
from workloads.content import content

pytestmark = pytest.mark.gpu


def test_pingpong_echo_and_times():
    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    smax = (1 << 22) + 37
    bufs = [torch.zeros(smax + 64, dtype=torch.uint8, device="cuda") for _ in range(5)]
    wd.fill(bufs[0].data_ptr(), smax, 5)
    torch.cuda.synchronize()
    slots = [H.hicr_slot_register(ctx, b.data_ptr(), smax + 64)[1] for b in bufs]
    sizes = [1, 15, 16, 17, 4096, 65537, 1 << 20, smax]
    for W in (0, 1, 7):
        print("pingpong W", W, flush=True)
        for s in sizes:
            bufs[1].zero_()
            torch.cuda.synchronize()
            rc, rtt = H.hicr_pingpong(ctx, *slots, [s], 3, W)
            assert rc == H.OK, H.hicr_last_error(ctx)
            assert (rtt > 0).all()
            # the oracle: the message through two one-message channels
            msg = content(5, 0, s)
            a, b = oracle.VChan(s, 1), oracle.VChan(s, 1)
            assert a.push(msg, s) == oracle.OK
            echoed = a.read(0)[1]
            assert a.pop(1) == oracle.OK and b.push(echoed, s) == oracle.OK
            want = b.read(0)[1]
            got = bufs[1][:s + 16].cpu().numpy()
            assert np.array_equal(got[:s], want) and not got[s:].any()
    assert H.hicr_pingpong(ctx, *slots, [smax + 65], 1, 0)[0] == H.ERANGE
    assert H.hicr_ctx_destroy(ctx) == H.OK


@pytest.mark.timeout(900)
def test_pingpong_two_gib_message():
    """The largest size the benchmark sweeps (2^31 bytes, the paper's ~2.14 GB
    end point): one round trip, the echo checked whole against the message
    carried by the oracle's two one-message rings."""
    import torch
    from paper_2509_01425_amd import hicr as H
    from tests.parity import pmap
    from workloads import device as wd
    s = 1 << 31
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    print("pingpong 2 GiB: alloc", flush=True)
    bufs = [torch.zeros(s + 64, dtype=torch.uint8, device="cuda") for _ in range(5)]
    wd.fill(bufs[0].data_ptr(), s, 6)
    torch.cuda.synchronize()
    slots = [H.hicr_slot_register(ctx, b.data_ptr(), s + 64)[1] for b in bufs]
    rc, rtt = H.hicr_pingpong(ctx, *slots, [s], 1, 0)
    assert rc == H.OK, H.hicr_last_error(ctx)
    assert (rtt > 0).all()
    print(f"pingpong 2 GiB: round trip {int(rtt[0, 0]) / 100:.0f} us", flush=True)
    step = 64 << 20
    msg = np.concatenate(pmap(lambda o: content(6, o, min(step, s - o)), range(0, s, step)))
    a, b = oracle.VChan(s, 1), oracle.VChan(s, 1)
    assert a.push(msg, s) == oracle.OK
    echoed = a.read(0)[1]
    del msg
    assert a.pop(1) == oracle.OK and b.push(echoed, s) == oracle.OK
    del echoed
    want = b.read(0)[1]
    got = bufs[1].cpu().numpy()
    assert np.array_equal(got[:s], want) and not got[s:].any()
    assert H.hicr_ctx_destroy(ctx) == H.OK
    del bufs
    torch.cuda.empty_cache()
