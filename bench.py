"""Benchmark: batched slot memcpy on one MI355X.

One step = one pass of the data path over one batch: host validation and
packing of 4,096 memcpy requests, upload, schedule, the fused copy launch
(piece scan, copy, completion counters) and the fence.  The workload is the
batched configuration: 8,192 slot windows over a 64 GiB + 64 MiB HBM pool,
4,096 requests per batch with sizes log-uniform in [256 B, 64 MiB], unaligned
offsets, disjoint destinations (~22 GB moved, ~44 GB read + written per
batch).  The pool is filled once with seeded bytes before timing; every step
uses a different seeded batch.

Printed: one JSON line with the whole-job throughput (algorithmic read +
write bytes / time), per-step p50/p99, the copy kernel's roofline (event-
timed on the stream it runs on) beside the box's reference copy, read and
write streams, HBM traffic from committed rocprofv3 counters when they still
match the kernel source; then the channel pumps (both MPSC modes), the
tiny batch's submit-to-fence latency (memcpy_batch and plan replays), the
serving loop (60 s of Poisson arrivals at 2,000 requests/s, 200 GB budget),
the learned schedule (a 2,000 + 200 batch version of the 20,000 + 1,000
configuration, which `--workload learned` runs whole), and the CPU oracle's
rates (one thread and every usable CPU, copy and channel paths) on bounded
samples of the same workloads.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--sched CLASS|tuned|learned]
       python bench.py --calibrate-copy   (plain-copy kernel for counter scaling)
       python bench.py --workload {channels,learned,serving,pingpong,tiny,halo,memspace,placement}
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "achieved HBM GB/s (R+W) for batched slot memcpy/channels vs peak; p99 latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "copy_kernel_batched_traffic.json")
COPY_SRC = os.path.join(ROOT, "paper_2509_01425_amd", "csrc", "copy.hip")


def _src_hash(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def traffic_per_launch():
    """HBM bytes per copy launch from the committed rocprofv3 counter summary,
    or None when the kernel source changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("kernel_source_sha256_16") != _src_hash(COPY_SRC):
        return None
    return t


def host_info():
    """The host the CPU baselines ran on: CPU model, logical CPUs, and the
    CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def _greedy_parts(sizes, parts):
    """Indices of `sizes` split over `parts` workers, longest first onto the
    least-loaded worker (the partition the all-core baseline uses)."""
    import heapq
    heap = [(0, k) for k in range(parts)]
    out = [[] for _ in range(parts)]
    for i in np.argsort(-sizes, kind="stable"):
        load, k = heapq.heappop(heap)
        out[k].append(int(i))
        heapq.heappush(heap, (load + int(sizes[i]), k))
    return [np.array(sorted(o), dtype=np.int64) for o in out if o]


def cpu_baseline(batch_descs, target_bytes=12 << 30):
    """Time the CPU oracle on a bounded sample of one batch: requests taken in
    a seeded random order until their sizes reach ``target_bytes``, remapped
    into a host pool (destinations then sources, each request at its original
    offset modulo 64).  Timed on one thread, then on every usable CPU with
    the requests split greedily by bytes (longest first), five passes, the
    median reported; each thread runs its share through its own oracle
    context (the oracle's C code runs without the interpreter lock)."""
    import concurrent.futures as cf
    import oracle
    g = np.random.default_rng(99)
    order = g.permutation(len(batch_descs))
    sizes = batch_descs["size"][order].astype(np.int64)
    k = int(np.searchsorted(np.cumsum(sizes), target_bytes)) + 1
    pick = batch_descs[order[:k]]
    sz = pick["size"].astype(np.int64)
    dmod = pick["dst_off"].astype(np.int64) % 64
    smod = pick["src_off"].astype(np.int64) % 64
    dpos = np.concatenate([[0], np.cumsum(sz + 128)[:-1]]) + dmod
    dst_len = int(dpos[-1] + sz[-1] + 64)
    spos = np.concatenate([[0], np.cumsum(sz + 128)[:-1]]) + smod
    src_len = int(spos[-1] + sz[-1] + 64)
    dst = np.zeros(dst_len, np.uint8)
    dst[:] = 1  # fault every page in before timing
    src = np.ones(src_len, np.uint8)
    moved = 2 * int(sz.sum())

    def run_part(idx):
        c = oracle.Ctx()
        _, a = c.register(dst)
        _, b = c.register(src)
        d = np.zeros(len(idx), dtype=oracle.DESC_DTYPE)
        d["dst_slot"], d["src_slot"] = a, b
        d["dst_off"], d["src_off"], d["size"] = dpos[idx], spos[idx], sz[idx]
        t0 = time.perf_counter()
        rc, _ = c.memcpy_batch(d)
        assert rc == oracle.OK
        return time.perf_counter() - t0

    dt1 = run_part(np.arange(k))
    threads = len(os.sched_getaffinity(0))
    parts = _greedy_parts(sz, threads)
    # the all-core pass is short: its median over `passes` runs is reported
    # (about 10-20 s of CPU work in all, with the one-thread pass)
    passes = 5
    dts = []
    with cf.ThreadPoolExecutor(max_workers=len(parts)) as ex:
        for _ in range(passes):
            t0 = time.perf_counter()
            list(ex.map(run_part, parts))
            dts.append(time.perf_counter() - t0)
    dtn = float(np.median(dts))
    return {"value": round(moved / dtn / 1e9, 3), "unit": "GB/s", "cores": len(parts),
            "kind": "oracle",
            "sample": f"{k} requests ({int(sz.sum())} bytes) of batch 0 remapped into a host "
                      f"pool, byte-loop oracle on {len(parts)} threads (greedy byte partition): "
                      f"median {dtn:.2f} s over {passes} passes; one thread: {dt1:.2f} s",
            "single_thread": {"value": round(moved / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1},
            "host": host_info()}


def cpu_channel_baseline(n_streams=32, seed=5):
    """The oracle's channel path on a sample of the channel configuration: the
    first n_streams SPSC streams (651 or 652 messages each, 16 B..256 KiB)
    each replayed through the oracle's 1 MiB / 64-entry ring, on one thread
    and on every usable CPU (one stream per task).  GB/s counts the same
    algorithmic bytes as the GPU pump (4 per payload byte + 16 per message)."""
    import concurrent.futures as cf
    import oracle
    from workloads import channels as wc
    from workloads.content import content
    plan = wc.plan()
    work = []
    for s in range(n_streams):
        b0, b1 = int(plan.msg_begin[s]), int(plan.msg_begin[s + 1])
        work.append((content(seed, s * plan.src_bytes, plan.src_bytes),
                     plan.msg_src_off[b0:b1], plan.msg_size[b0:b1]))
    payload = int(sum(int(z.sum()) for _, _, z in work))
    msgs = int(sum(len(z) for _, _, z in work))
    moved = 4 * payload + 16 * msgs

    def run(w):
        blob, o, z = w
        rc, _ = oracle.vchan_replay(plan.P, plan.E, np.zeros(len(z), np.uint32), [blob], [o], [z])
        assert rc == oracle.OK

    t0 = time.perf_counter()
    for w in work:
        run(w)
    dt1 = time.perf_counter() - t0
    threads = min(len(os.sched_getaffinity(0)), n_streams)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, work))
    dtn = time.perf_counter() - t0
    return {"value": round(moved / dtn / 1e9, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n_streams} SPSC streams, {msgs} messages, {payload} payload bytes of "
                      f"the channel configuration through the oracle's ring: {dtn:.2f} s on "
                      f"{threads} threads, {dt1:.2f} s on one",
            "single_thread": {"value": round(moved / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1}}


def copy_ceiling(torch, wd, pool, stream, n=4 << 30, reps=3):
    """What a plain 4 GiB stream reaches on this machine (context for the copy
    kernel's fraction of peak): the fastest reference copy shape over a grid
    sweep, the runtime's device-to-device hipMemcpyAsync, and read-only and
    write-only streams.  GB/s counts read + write bytes (read or write only
    for the one-sided streams); median of `reps` event-timed launches."""
    a, b = pool.data_ptr(), pool.data_ptr() + n
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    s = stream.cuda_stream

    def timed(kind, blocks):
        wd.ref_stream(kind, b, a, n, blocks, sink.data_ptr(), s)  # warm-up
        ms = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            wd.ref_stream(kind, b, a, n, blocks, sink.data_ptr(), s)
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    sweep = {bl: 2 * n / (timed(wd.REF_COPY, bl) * 1e-3) / 1e9 for bl in (256, 512, 768, 1024, 2048)}
    best = max(sweep, key=sweep.get)
    return {"best_copy_GBps": round(sweep[best], 1), "best_copy_blocks": best,
            "copy_sweep_GBps": {str(k): round(v, 1) for k, v in sweep.items()},
            "hipMemcpyAsync_d2d_GBps": round(2 * n / (timed(wd.REF_MEMCPY, 1) * 1e-3) / 1e9, 1),
            "read_only_GBps": round(n / (timed(wd.REF_READ, 2048) * 1e-3) / 1e9, 1),
            "write_only_GBps": round(n / (timed(wd.REF_WRITE, 1024) * 1e-3) / 1e9, 1),
            "bytes": n}


def calibrate_copy(n_bytes=4 << 30, reps=3):
    """Plain aligned copy of a known size, for scaling rocprofv3 counters."""
    import torch
    from workloads import device as wd
    buf = torch.empty(2 * n_bytes, dtype=torch.uint8, device="cuda")
    for _ in range(reps):
        wd.ref_copy(buf.data_ptr() + n_bytes, buf.data_ptr(), n_bytes, 1024)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "wl_ref_copy", "bytes_read": n_bytes,
                      "bytes_written": n_bytes, "launches": reps}), flush=True)


def channel_rig(torch, H, ctx, plan, mpsc_mode, seed, stream=0):
    """Allocate, fill and register everything a channel plan needs and create
    its device-endpoint channels; returns the pump's stream list and buffers."""
    from workloads import device as wd
    S = plan.n_streams
    src = torch.empty(S * plan.src_bytes, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), src.numel(), seed, 0, stream)
    sb = plan.stream_bytes().astype(np.int64)
    out_off = np.concatenate([[0], np.cumsum(sb)[:-1]]).astype(np.int64)
    out = torch.zeros(int(sb.sum()) + 64, dtype=torch.uint8, device="cuda")
    rings_per = [1] * plan.n_spsc + [1 if mpsc_mode == H.CH_MPSC_LOCK else plan.K] * plan.n_mpsc
    n_rings = sum(rings_per)
    payload = torch.empty(n_rings * plan.P, dtype=torch.uint8, device="cuda")
    entries = torch.zeros(n_rings * plan.E, dtype=torch.int64, device="cuda")
    chans = []
    r0 = 0
    for c, nr in enumerate(rings_per):
        _, ps = H.hicr_slot_register(ctx, payload.data_ptr() + r0 * plan.P, nr * plan.P)
        _, es = H.hicr_slot_register(ctx, entries.data_ptr() + r0 * plan.E * 8, nr * plan.E * 8)
        spsc = c < plan.n_spsc
        cfg = H.make_channel_cfg(H.CH_VAR, H.CH_SPSC if spsc else mpsc_mode,
                                 1 if spsc else plan.K, H.CH_DEVICE, ps, es,
                                 capacity=plan.P, entries=plan.E)
        rc, ch = H.hicr_channel_create(ctx, cfg)
        assert rc == H.OK, H.hicr_last_error(ctx)
        chans.append(ch)
        r0 += nr
    streams = []
    for s in range(S):
        rc, ss = H.hicr_slot_register(ctx, src.data_ptr() + s * plan.src_bytes, plan.src_bytes)
        assert rc == H.OK
        rc, os_ = H.hicr_slot_register(ctx, out.data_ptr() + int(out_off[s]), max(int(sb[s]), 1))
        assert rc == H.OK
        streams.append((chans[int(plan.stream_channel[s])], int(plan.stream_producer[s]), ss, os_,
                        int(plan.msg_begin[s]), int(plan.msg_begin[s + 1] - plan.msg_begin[s])))
    return {"streams": streams, "src": src, "out": out, "out_off": out_off, "stream_bytes": sb,
            "payload": payload, "entries": entries, "channels": chans}


def bench_channels(torch, H, mpsc_mode, steps=3, warmup=1, seed=5):
    """The channel configuration (1,024 SPSC + 64 MPSC x 8 producers, 1e6
    messages, 1 MiB / 64-entry rings) through one persistent pump per step.
    The message tables (source offset and size of every message) are inputs
    resident in device memory (HICR_PUMP_DEVICE_TABLES), uploaded once like
    the sources.  GB/s counts 4 bytes per payload byte (source read, ring
    write, ring read, output write) plus the 8-byte entry written and read per
    message."""
    from workloads import channels as wc
    plan = wc.plan()
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK
    rig = channel_rig(torch, H, ctx, plan, mpsc_mode, seed, stream.cuda_stream)
    ts = torch.zeros(2 * plan.n_msgs, dtype=torch.int64, device="cuda")
    offs = torch.from_numpy(plan.msg_src_off.astype(np.int64)).cuda()
    sizes = torch.from_numpy(plan.msg_size.astype(np.int64)).cuda()
    torch.cuda.synchronize()
    times = []
    for k in range(warmup + steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        rc = H.hicr_channel_pump(ctx, rig["streams"], offs.data_ptr(), sizes.data_ptr(), 0,
                                 ts.data_ptr(), timeout_ns=10 * 10**9, n_msgs=plan.n_msgs)
        e1.record(stream)
        assert rc == H.OK, H.hicr_last_error(ctx)
        assert H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
        e1.synchronize()
        if k >= warmup:
            times.append(e0.elapsed_time(e1))
    t = ts.cpu().numpy().reshape(2, -1).astype(np.int64)
    lat_us = (t[1] - t[0]) / 100.0
    payload = int(plan.msg_size.sum())
    moved = 4 * payload + 16 * plan.n_msgs
    ms = float(np.mean(times))
    for ch in rig["channels"]:
        H.hicr_channel_destroy(ch)
    H.hicr_ctx_destroy(ctx)
    del rig
    torch.cuda.empty_cache()
    return {"mpsc_mode": "locking" if mpsc_mode == H.CH_MPSC_LOCK else "non-locking",
            "value": round(moved / ms / 1e6, 1), "unit": "GB/s", "ms_per_pump": round(ms, 3),
            "frac_of_peak": round(moved / ms / 1e6 / HBM_PEAK_GBS, 4),
            "messages": plan.n_msgs, "payload_bytes": payload,
            "latency_p50_us": round(float(np.percentile(lat_us, 50)), 2),
            "latency_p99_us": round(float(np.percentile(lat_us, 99)), 2)}


def bench_learned(torch, H, n_train=20000, n_test=1000, reps=3, epochs=300, batch=256, lr=1e-3,
                  save=None):
    """The learned-schedule configuration.  Every batch of the training law
    (tiny-like or batched-like family, 8..4096 requests) is autotuned over the
    12 classes (median of `reps` timed runs); the network is trained on the
    GPU by the library's kernels on the first n_train batches (Adam, 300
    epochs of mini-batches of 256) and judged on the n_test held-out batches by measured
    copy time against the best fixed class of the training set, the untuned
    default class, the tuned table (nearest training batch) and the
    autotuner's per-batch best."""
    from workloads import memcpy as wm
    from workloads.mlp_init import he_uniform
    t_start = time.time()
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK
    from workloads import device as wd
    pool = torch.empty(wm.B_POOL, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), wm.B_POOL, 3, 0, stream.cuda_stream)
    bases, sizes = wm.batched_slots()
    slots = np.empty(len(bases), dtype=np.uint32)
    for k, (b, sz) in enumerate(zip(bases, sizes)):
        rc, slots[k] = H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(sz), H.MEM_HBM)
    torch.cuda.synchronize()
    N = n_train + n_test
    X = np.zeros((N, 32), np.float32)
    T = np.zeros((N, 12), np.float32)
    nbytes = np.zeros(N, np.float64)

    def batch_descs(b):
        d, _ = wm.family(b)
        d["dst_slot"] = slots[d["dst_slot"]]
        d["src_slot"] = slots[d["src_slot"]]
        return d

    for b in range(N):
        d = batch_descs(b)
        rc, times, _ = H.hicr_autotune(ctx, d, reps)
        assert rc == H.OK, H.hicr_last_error(ctx)
        X[b] = H.hicr_sched_features(d)[1]
        T[b] = times
        nbytes[b] = 2.0 * float(d["size"].sum())
        if b % 2000 == 0:
            print(f"autotune {b}/{N} ({time.time() - t_start:.0f} s)", file=sys.stderr, flush=True)
    y = np.argmin(T, axis=1).astype(np.int32)
    tr, te = slice(0, n_train), slice(n_train, N)
    # training on the GPU; the shuffles are seeded inputs
    assert H.hicr_mlp_set_params(ctx, he_uniform(0)) == H.OK
    xd = torch.from_numpy(X[tr]).cuda()
    yd = torch.from_numpy(y[tr]).cuda()
    g = np.random.default_rng(np.random.SeedSequence([0x48694352, 3, 99]))
    t0 = time.time()
    # the mini-batch gathers run on the library's stream, so each training
    # step reads a finished gather and a freed batch is reused only after it
    with torch.cuda.stream(stream):
        for ep in range(epochs):
            perm = torch.from_numpy(g.permutation(n_train)).cuda()
            for i in range(0, n_train - batch + 1, batch):
                idx = perm[i:i + batch]
                xb, yb = xd[idx].contiguous(), yd[idx].contiguous()
                assert H.hicr_mlp_train_step(ctx, xb.data_ptr(), yb.data_ptr(), batch, lr) == H.OK
        assert H.hicr_fence(ctx) == H.OK
        train_s = time.time() - t0
        logits = torch.zeros(n_test, 12, dtype=torch.float32, device="cuda")
        xt = torch.from_numpy(X[te]).cuda()
        assert H.hicr_mlp_forward(ctx, xt.data_ptr(), n_test, logits.data_ptr()) == H.OK
    pred = np.argmax(logits.cpu().numpy(), axis=1)
    fixed = int(np.argmin(T[tr].sum(axis=0)))
    default = 4
    # tuned table: nearest training feature (the same rule the library applies)
    for b in range(n_train):
        H.hicr_tune_add(ctx, batch_descs(b), int(y[b]))
    Xtr = X[tr]
    nn_cls = np.array([y[int(np.argmin(((Xtr - X[n_train + i]) ** 2).sum(1)))] for i in range(n_test)])
    Tt = T[te]
    rows = np.arange(n_test)

    def by_labels(choice):
        t = float(Tt[rows, choice].sum())
        return {"gbps": round(float(nbytes[te].sum()) / t / 1e6, 1),
                "regret": round(t / float(Tt.min(axis=1).sum()) - 1.0, 4)}

    table = {"autotuner_best": by_labels(np.argmin(Tt, axis=1)),
             "fixed_best": by_labels(np.full(n_test, fixed)),
             "default": by_labels(np.full(n_test, default)),
             "tuned_table": by_labels(nn_cls),
             "learned": by_labels(pred)}
    # measured end to end through the submission path (median of 3 per batch)
    def measured(sched):
        tot = 0.0
        for i in range(n_test):
            d = batch_descs(n_train + i)
            ms = []
            for _ in range(3):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                rc, _ = H.hicr_memcpy_batch(ctx, d, sched)
                e1.record(stream)
                assert rc == H.OK
                assert H.hicr_fence(ctx) == H.OK
                e1.synchronize()  # recorded after the launch the fence waited for
                ms.append(e0.elapsed_time(e1))
            tot += float(np.median(ms))
        return {"gbps": round(float(nbytes[te].sum()) / tot / 1e6, 1), "total_ms": round(tot, 2)}

    meas = {"fixed_best": measured(H.hicr_sched_class(fixed)[1]),
            "default": measured(H.hicr_sched_class(default)[1]),
            "tuned_table": measured(H.make_sched(65536, 1, 2, H.SCHED_TUNED)),
            "learned": measured(H.make_sched(65536, 1, 2, H.SCHED_LEARNED))}
    out = {"workload": "learned schedule: family batches (8..4096 requests, tiny-like or "
                       "batched-like sizes), 12 classes, median of %d" % reps,
           "n_train": n_train, "n_test": n_test, "fixed_best_class": fixed,
           "label_hist": np.bincount(y, minlength=12).tolist(),
           "accuracy": round(float((pred == y[te]).mean()), 4),
           "tuned_accuracy": round(float((nn_cls == y[te]).mean()), 4),
           "train_seconds": round(train_s, 2), "by_autotune_times": table,
           "measured": meas, "wall_seconds": round(time.time() - t_start, 1)}
    if save:
        rc, params = H.hicr_mlp_get_params(ctx)
        np.savez(save, X=X, T=T, nbytes=nbytes, params=params)
    H.hicr_ctx_destroy(ctx)
    del pool
    torch.cuda.empty_cache()
    return out


def bench_serving(torch, H, duration_s=60.0, rate=2000.0, budget=200_000_000_000, streams=4,
                  max_batch=64, batch=0):
    """The serving configuration: Poisson arrivals (2,000 requests/s), each a
    memcpy batch (8..512 requests, 64 B..16 MiB) or a burst (1..256 messages,
    16 B..256 KiB) through one of 1,024 SPSC channels; admission by an HBM
    arena budget; continuous batching over `streams` launches in flight."""
    from workloads import device as wd
    from workloads import serving as ws
    src_bytes, P, E, nch = 16 << 30, 1 << 20, 64, 1024
    t_gen = time.time()
    tr = ws.trace(duration_s=duration_s, rate=rate, src_bytes=src_bytes, n_channels=nch,
                  batch=batch)
    t_gen = time.time() - t_gen
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK
    src = torch.empty(src_bytes, dtype=torch.uint8, device="cuda")
    wd.fill(src.data_ptr(), src_bytes, 77, 0, stream.cuda_stream)
    arena = torch.empty(budget, dtype=torch.uint8, device="cuda")
    payload = torch.empty(nch * P, dtype=torch.uint8, device="cuda")
    entries = torch.zeros(nch * E, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    _, ss = H.hicr_slot_register(ctx, src.data_ptr(), src_bytes)
    _, aslot = H.hicr_slot_register(ctx, arena.data_ptr(), budget)
    chans = []
    for c in range(nch):
        _, ps = H.hicr_slot_register(ctx, payload.data_ptr() + c * P, P)
        _, es = H.hicr_slot_register(ctx, entries.data_ptr() + c * E * 8, E * 8)
        rc, ch = H.hicr_channel_create(ctx, H.make_channel_cfg(H.CH_VAR, H.CH_SPSC, 1, H.CH_DEVICE,
                                                               ps, es, capacity=P, entries=E))
        assert rc == H.OK
        chans.append(ch)
    n = len(tr.reqs)
    admit = np.zeros(n, np.uint64)
    fin = np.zeros(n, np.uint64)
    rc, st = H.hicr_serve(ctx, tr.reqs, aslot, ss, tr.descs, tr.msg_src_off, tr.msg_size, chans,
                          streams=streams, max_batch_reqs=max_batch, admit_ns=admit, done_ns=fin)
    assert rc == H.OK, H.hicr_last_error(ctx)
    arr = tr.reqs["arrival_ns"].astype(np.int64)
    lat_ms = (fin.astype(np.int64) - arr) / 1e6
    wait_ms = (admit.astype(np.int64) - arr) / 1e6
    kinds = tr.reqs["kind"]
    out = {"requests": n, "duration_s": duration_s, "rate": rate, "budget_bytes": budget,
           "value": round(tr.algorithmic_bytes() / (st.wall_ns / 1e9) / 1e9, 1), "unit": "GB/s",
           "latency_p50_ms": round(float(np.percentile(lat_ms, 50)), 3),
           "latency_p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
           "copy_latency_p99_ms": round(float(np.percentile(lat_ms[kinds == 0], 99)), 3),
           "burst_latency_p99_ms": round(float(np.percentile(lat_ms[kinds == 1], 99)), 3),
           "queue_wait_p50_ms": round(float(np.percentile(wait_ms, 50)), 3),
           "queue_wait_p99_ms": round(float(np.percentile(wait_ms, 99)), 3),
           "peak_arena_bytes": int(st.peak_arena_bytes), "copy_launches": int(st.copy_launches),
           "pump_launches": int(st.pump_launches),
           "max_inflight_requests": int(st.max_inflight_requests),
           "wall_s": round(st.wall_ns / 1e9, 3), "trace_gen_s": round(t_gen, 1)}
    for ch in chans:
        H.hicr_channel_destroy(ch)
    H.hicr_ctx_destroy(ctx)
    del arena, src, payload, entries
    torch.cuda.empty_cache()
    return out


def bench_pingpong(torch, H, max_log2=31, reps=10):
    """Ping-pong goodput G(s) = s / one-way time (half the round trip) for
    s = 1 B .. 2^max_log2 B, `reps` round trips each (mean and std)."""
    smax = 1 << max_log2
    rc, ctx = H.hicr_ctx_create(0, 0)
    assert rc == H.OK
    bufs = [torch.empty(smax, dtype=torch.uint8, device="cuda") for _ in range(5)]
    torch.cuda.synchronize()
    slots = [H.hicr_slot_register(ctx, b.data_ptr(), smax)[1] for b in bufs]
    sizes = [1 << k for k in range(max_log2 + 1)]
    rc, rtt = H.hicr_pingpong(ctx, *slots, sizes, reps + 1, 0)
    assert rc == H.OK, H.hicr_last_error(ctx)
    rows = []
    for s, r in zip(sizes, rtt):
        oneway_s = r[1:].astype(np.float64) / 2 / 1e8   # first round trip is warm-up
        g = s / oneway_s
        rows.append({"bytes": s, "goodput_GBps": round(float(g.mean()) / 1e9, 4),
                     "std_GBps": round(float(g.std()) / 1e9, 4),
                     "one_way_us": round(float(oneway_s.mean()) * 1e6, 3)})
    H.hicr_ctx_destroy(ctx)
    del bufs
    torch.cuda.empty_cache()
    return rows


# The batched line's schedule: a fixed schedule, not one of the 12 classes
# (whose chunks are 4 KiB, 64 KiB and 1 MiB): 32 KiB pieces, at least one per
# request, unroll 4.  In-process sweeps of the chunk size on this workload
# (one pool allocation, two workgroups per CU, batches 0-3): 8 KiB 5,135,
# 16 KiB 5,157, 24 KiB 5,070, 32 KiB 5,740, 40 KiB 5,050, 48 KiB 5,185,
# 64 KiB (class 5) 5,420, 128 KiB 5,085, 1 MiB 4,680 GB/s; 32 KiB at one
# workgroup per CU (the library's default for that chunk) 5,823-5,857.
BATCHED_SCHED = "32768,1,4"


def parse_sched(H, text):
    """A schedule class number, "tuned", "learned", or "chunk,wgs,unroll"
    (a fixed schedule)."""
    if text in ("tuned", "learned"):
        return H.make_sched(64 << 10, 1, 2, H.SCHED_TUNED if text == "tuned" else H.SCHED_LEARNED)
    if "," in text:
        chunk, wgs, unroll = (int(x) for x in text.split(","))
        return H.make_sched(chunk, wgs, unroll)
    rc, s = H.hicr_sched_class(int(text))
    assert rc == H.OK
    return s


def bench_memspace(torch, H, size=1 << 30, reps=5):
    """Memory spaces: slot copies between HBM and pinned host memory (the
    host link) with the fused copy kernel -- one request of `size` bytes, and
    the same bytes as 4,096 requests -- in both directions, beside the DMA
    engine's copy of the same bytes (torch copy_) as the link's reference.
    GB/s counts the bytes moved over the link once."""
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK
    dev = torch.empty(size, dtype=torch.uint8, device="cuda")
    host = torch.empty(size, dtype=torch.uint8).pin_memory()
    dev.fill_(7)
    host.fill_(9)
    torch.cuda.synchronize()
    rc, sd = H.hicr_slot_register(ctx, dev.data_ptr(), size, H.MEM_HBM)
    rc2, sh = H.hicr_slot_register(ctx, host.data_ptr(), size, H.MEM_HOST)
    assert rc == rc2 == H.OK, H.hicr_last_error(ctx)
    sched = H.hicr_sched_class(5)[1]

    def batch(dst, src, n):
        d = np.zeros(n, dtype=H.DESC_DTYPE)
        per = size // n
        d["dst_slot"], d["src_slot"] = dst, src
        d["dst_off"] = np.arange(n, dtype=np.uint64) * np.uint64(per)
        d["src_off"] = d["dst_off"]
        d["size"] = per
        return d

    def timed(fn):
        fn()
        stream.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return round(size / (float(np.median(ts)) * 1e-3) / 1e9, 1)

    def hicr_copy(d):
        def fn():
            assert H.hicr_memcpy_batch(ctx, d, sched)[0] == H.OK
            assert H.hicr_fence(ctx) == H.OK
        return fn

    out = {"workload": f"{size >> 20} MiB between an HBM slot and a pinned host slot", "bytes": size}
    for name, dst, src in (("host_to_hbm", sd, sh), ("hbm_to_host", sh, sd)):
        out[name] = {"memcpy_1_request_gbps": timed(hicr_copy(batch(dst, src, 1))),
                     "memcpy_4096_requests_gbps": timed(hicr_copy(batch(dst, src, 4096)))}
    with torch.cuda.stream(stream):
        out["host_to_hbm"]["dma_copy_gbps"] = timed(lambda: dev.copy_(host, non_blocking=True))
        out["hbm_to_host"]["dma_copy_gbps"] = timed(lambda: host.copy_(dev, non_blocking=True))
    # data objects: a published object fetched by get + fence -- small ones
    # for latency, a large one for bandwidth (HBM to HBM, then host to HBM)
    half = size // 2
    objs = {}
    for name, slot, off, n in (("obj_4KiB_hbm", sd, 0, 4096), ("obj_half_hbm", sd, 0, half),
                               ("obj_4KiB_host", sh, 0, 4096)):
        rc, oid = H.hicr_dobj_publish(ctx, slot, off, n)
        assert rc == H.OK, H.hicr_last_error(ctx)
        rc, hd = H.hicr_dobj_get_handle(ctx, oid)
        assert rc == H.OK
        objs[name] = (oid, hd, n)

    def get_fence(hd):
        assert H.hicr_dobj_get(ctx, hd, sd, half) == H.OK
        assert H.hicr_fence(ctx) == H.OK

    dobj = {}
    for name in ("obj_4KiB_hbm", "obj_4KiB_host"):
        oid, hd, n = objs[name]
        lat = []
        for k in range(550):
            t0 = time.perf_counter()
            get_fence(hd)
            if k >= 50:
                lat.append((time.perf_counter() - t0) * 1e6)
        dobj[name] = {"get_fence_p50_us": round(float(np.percentile(lat, 50)), 2),
                      "get_fence_p99_us": round(float(np.percentile(lat, 99)), 2)}
    oid, hd, n = objs["obj_half_hbm"]
    get_fence(hd)
    t0 = time.perf_counter()
    for _ in range(reps):
        get_fence(hd)
    dobj["obj_half_hbm"] = {"bytes": n, "gbps_rw": round(2 * n * reps / (time.perf_counter() - t0) / 1e9, 1)}
    for oid, _, _ in objs.values():
        assert H.hicr_dobj_unpublish(ctx, oid) == H.OK
    out["data_objects"] = dobj
    H.hicr_ctx_destroy(ctx)
    del dev, host
    torch.cuda.empty_cache()
    return out


def bench_tiny(torch, H, reps=1000, warmup=50):
    """Submit-to-fence latency of the tiny batch (64 packed slots, 256
    requests of 1..8 KiB): one hicr_memcpy_batch + hicr_fence per rep, and
    one replay of a persistent plan of the same batch + hicr_fence per rep."""
    from workloads import device as wd
    from workloads import memcpy as wm
    bases, sizes, pool_len, descs, _ = wm.tiny(0)
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), pool_len, 11, 0, stream.cuda_stream)
    torch.cuda.synchronize()
    slots = np.array([H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(z))[1]
                      for b, z in zip(bases, sizes)], dtype=np.uint32)
    d = descs.copy()
    d["dst_slot"], d["src_slot"] = slots[descs["dst_slot"]], slots[descs["src_slot"]]
    moved = 2 * int(descs["size"].sum())
    sched = H.hicr_sched_class(0)[1]

    def lat(fn):
        us = []
        for k in range(warmup + reps):
            t0 = time.perf_counter()
            fn()
            assert H.hicr_fence(ctx) == H.OK
            if k >= warmup:
                us.append((time.perf_counter() - t0) * 1e6)
        us = np.array(us)
        return {"p50_us": round(float(np.percentile(us, 50)), 2),
                "p99_us": round(float(np.percentile(us, 99)), 2),
                "mean_us": round(float(us.mean()), 2),
                "gbps": round(moved / (us.mean() * 1e-6) / 1e9, 2)}

    def submit():
        assert H.hicr_memcpy_batch(ctx, d, sched)[0] == H.OK

    out = {"workload": "tiny: 64 packed slots (1..64 KiB), 256 requests of 1..8 KiB, "
                       "submit + fence per rep", "bytes_rw": moved, "reps": reps,
           "memcpy_batch": lat(submit)}
    for name, flags in (("plan_replay", 0), ("plan_graph_replay", H.PLAN_GRAPH)):
        rc, plan, _ = H.hicr_plan_create(ctx, d, sched, flags)
        assert rc == H.OK, H.hicr_last_error(ctx)
        out[name] = lat(lambda: H.hicr_plan_launch(plan))
        assert H.hicr_plan_destroy(plan) == H.OK
    H.hicr_ctx_destroy(ctx)
    return out


def bench_halo(torch, H, N=704, Py=2, Pz=22, h=2, iters=200, reps=3):
    """The Jacobi test case's halo exchange: a 704^3 grid of 8-byte cells over
    1 x 2 x 22 subgrids (the paper's best thread grid), ghost layers two
    cells deep (13-point stencil), each subgrid in its own block (3.2 GB in
    all): 61,952 row copies of 5,632 B = 349 MB per exchange.  The 12 classes
    are autotuned on the exchange; then `iters` exchanges run back to back
    (one fence at the end) as one hicr_memcpy_batch per exchange, and as a
    replay of a persistent plan (direct and graph), and one exchange + fence
    is timed alone for latency."""
    from workloads import halo
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK
    sb = halo.sub_bytes(N, Py, Pz, h)
    pool = torch.empty(Py * Pz * sb, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    slots = np.array([H.hicr_slot_register(ctx, pool.data_ptr() + k * sb, sb)[1]
                      for k in range(Py * Pz)], dtype=np.uint32)
    d = halo.exchange(N, Py, Pz, h)
    d["dst_slot"], d["src_slot"] = slots[d["dst_slot"]], slots[d["src_slot"]]
    moved = 2 * int(d["size"].sum())
    rc, times, best = H.hicr_autotune(ctx, d, reps)
    assert rc == H.OK, H.hicr_last_error(ctx)
    sched = H.hicr_sched_class(int(best))[1]

    def run(step):
        step()
        assert H.hicr_fence(ctx) == H.OK
        t0 = time.perf_counter()
        for _ in range(iters):
            step()
        assert H.hicr_fence(ctx) == H.OK
        per = (time.perf_counter() - t0) / iters
        lat = []
        for _ in range(50):
            t1 = time.perf_counter()
            step()
            assert H.hicr_fence(ctx) == H.OK
            lat.append((time.perf_counter() - t1) * 1e6)
        return {"us_per_exchange": round(per * 1e6, 2), "gbps": round(moved / per / 1e9, 1),
                "latency_p50_us": round(float(np.percentile(lat, 50)), 2),
                "latency_p99_us": round(float(np.percentile(lat, 99)), 2)}

    out = {"workload": f"Jacobi halo exchange: {N}^3 8-byte cells over 1x{Py}x{Pz} subgrids, "
                       f"ghost depth {h}, {len(d)} row copies of {N * 8} B per exchange",
           "requests": len(d), "bytes_rw": moved,
           "autotune_ms": [round(float(t), 4) for t in times], "best_class": int(best),
           "memcpy_batch": run(lambda: H.hicr_memcpy_batch(ctx, d, sched))}
    for name, flags in (("plan_replay", 0), ("plan_graph_replay", H.PLAN_GRAPH)):
        rc, plan, _ = H.hicr_plan_create(ctx, d, sched, flags)
        assert rc == H.OK, H.hicr_last_error(ctx)
        out[name] = run(lambda: H.hicr_plan_launch(plan))
        assert H.hicr_plan_destroy(plan) == H.OK
    # the same rows by a plain reference kernel (workloads/csrc/fill.hip: one
    # wave per row, the whole row loaded before it is stored, no piece
    # table), timed with events over `iters` launches, at a few grids
    from workloads import device as wd
    d0 = halo.exchange(N, Py, Pz, h)
    row = int(d0["size"][0])
    assert (d0["size"] == row).all() and row % 16 == 0
    base = np.uint64(pool.data_ptr())
    rows_dst = torch.from_numpy((base + d0["dst_slot"].astype(np.uint64) * np.uint64(sb)
                                 + d0["dst_off"]).view(np.int64)).to("cuda")
    rows_src = torch.from_numpy((base + d0["src_slot"].astype(np.uint64) * np.uint64(sb)
                                 + d0["src_off"]).view(np.int64)).to("cuda")
    torch.cuda.synchronize()
    ref = {}
    for blocks in (768, 2048, 4096):
        def launch():
            wd.ref_rows(rows_dst.data_ptr(), rows_src.data_ptr(), len(d0), row, blocks,
                        stream.cuda_stream)
        for _ in range(3):
            launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(iters):
            launch()
        e1.record(stream)
        e1.synchronize()
        per = e0.elapsed_time(e1) * 1e-3 / iters
        ref[str(blocks)] = {"us_per_exchange": round(per * 1e6, 2), "gbps": round(moved / per / 1e9, 1)}
    out["reference_rows"] = ref
    H.hicr_ctx_destroy(ctx)
    del pool, rows_dst, rows_src
    torch.cuda.empty_cache()
    return out


def bench_placement(torch, H, allocations=8, batches=2, reps=3, shifts=(0, 4096, (256 << 20) + 4096)):
    """The batched workload's rate against the pool's physical placement:
    the pool is allocated, filled and freed `allocations` times in one
    process (the caching allocator hands back the same virtual range; the
    driver places the physical pages anew), and each allocation runs the
    batched workload (class 5, library default grid) with the slot layout at
    a few shifts inside it.  The headline line uses one ordinary allocation;
    this mode only reports how much the placement moves the same kernel."""
    from workloads import device as wd
    from workloads import memcpy as wm
    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK, H.hicr_strerror(rc)
    sched = parse_sched(H, "5")
    descs = [wm.batched(b) for b in range(batches)]
    span = max(shifts)
    out = []
    for a in range(allocations):
        pool = torch.empty(wm.B_POOL + span, dtype=torch.uint8, device="cuda")
        wd.fill(pool.data_ptr(), wm.B_POOL + span, 7, 0, stream.cuda_stream)
        torch.cuda.synchronize()
        by_shift = {}
        for sh in shifts:
            bases, sizes = wm.batched_slots()
            slots = np.empty(len(bases), dtype=np.uint32)
            for k, (b, z) in enumerate(zip(bases, sizes)):
                rc, slots[k] = H.hicr_slot_register(ctx, pool.data_ptr() + sh + int(b), int(z),
                                                    H.MEM_HBM)
                assert rc == H.OK
            rates = []
            for d0 in descs:
                d = d0.copy()
                d["dst_slot"] = slots[d["dst_slot"]]
                d["src_slot"] = slots[d["src_slot"]]
                rc, _ = H.hicr_memcpy_batch(ctx, d, sched)
                assert rc == H.OK and H.hicr_fence(ctx) == H.OK, H.hicr_last_error(ctx)
                ms = []
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    rc, _ = H.hicr_memcpy_batch(ctx, d, sched)
                    e1.record(stream)
                    assert rc == H.OK and H.hicr_fence(ctx) == H.OK
                    e1.synchronize()
                    ms.append(e0.elapsed_time(e1))
                rates.append(round(2 * int(d["size"].sum()) / (np.median(ms) * 1e-3) / 1e9, 1))
            for k in slots:
                assert H.hicr_slot_deregister(ctx, int(k)) == H.OK
            by_shift[str(sh)] = rates
        out.append({"allocation": a, "virtual_base": hex(pool.data_ptr()), "GBps_by_layout_shift": by_shift})
        print(json.dumps(out[-1]), file=sys.stderr, flush=True)
        del pool
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    H.hicr_ctx_destroy(ctx)
    return {"workload": "batched slot memcpy, class 5, one pool allocated and freed per row",
            "allocations": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sched", default=BATCHED_SCHED,
                    help="class number, tuned, learned, or chunk,wgs,unroll")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-channels", action="store_true")
    ap.add_argument("--copy-grid", type=int, default=0,
                    help="copy workgroups per CU (0: the library's per-class default)")
    ap.add_argument("--workload", default="batched",
                    choices=["batched", "channels", "learned", "serving", "pingpong", "tiny",
                             "halo", "memspace", "placement"])
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-budget", type=float, default=200e9)
    ap.add_argument("--learned-train", type=int, default=20000)
    ap.add_argument("--learned-test", type=int, default=1000)
    ap.add_argument("--learned-save", default=None)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-tiny", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--line-learned-train", type=int, default=2000,
                    help="training batches of the learned-schedule part of the default line")
    ap.add_argument("--line-learned-test", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(every run uses exactly one MI355X); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch
    from paper_2509_01425_amd import hicr as H
    from workloads import device as wd
    from workloads import memcpy as wm

    if args.workload == "learned":
        res = bench_learned(torch, H, n_train=args.learned_train, n_test=args.learned_test,
                            save=args.learned_save)
        print(json.dumps({"learned": res}), flush=True)
        return
    if args.workload == "halo":
        print(json.dumps({"halo": bench_halo(torch, H)}), flush=True)
        return
    if args.workload == "placement":
        print(json.dumps({"placement": bench_placement(torch, H)}), flush=True)
        return
    if args.workload == "tiny":
        print(json.dumps({"tiny": bench_tiny(torch, H)}), flush=True)
        return
    if args.workload == "memspace":
        print(json.dumps({"memspace": bench_memspace(torch, H)}), flush=True)
        return
    if args.workload == "pingpong":
        print(json.dumps({"pingpong": bench_pingpong(torch, H)}), flush=True)
        return
    if args.workload == "serving":
        res = bench_serving(torch, H, duration_s=args.serve_seconds, budget=int(args.serve_budget))
        print(json.dumps({"serving": res}), flush=True)
        return
    if args.workload == "channels":
        res = [bench_channels(torch, H, m, steps=args.steps, warmup=args.warmup)
               for m in (H.CH_MPSC_LOCK, H.CH_MPSC_NOLOCK)]
        print(json.dumps({"channels": res}), flush=True)
        return

    stream = torch.cuda.Stream()
    rc, ctx = H.hicr_ctx_create(0, stream.cuda_stream)
    assert rc == H.OK, H.hicr_strerror(rc)
    assert H.hicr_ctx_set_copy_grid(ctx, args.copy_grid) == H.OK
    pool = torch.empty(wm.B_POOL, dtype=torch.uint8, device="cuda")
    wd.fill(pool.data_ptr(), wm.B_POOL, 7, 0, stream.cuda_stream)
    bases, sizes = wm.batched_slots()
    slots = np.empty(len(bases), dtype=np.uint32)
    for k, (b, s) in enumerate(zip(bases, sizes)):
        rc, slots[k] = H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(s), H.MEM_HBM)
        assert rc == H.OK
    sched = parse_sched(H, args.sched)
    batches = []
    for b in range(args.warmup + args.steps):
        d = wm.batched(b)
        d["dst_slot"] = slots[d["dst_slot"]]
        d["src_slot"] = slots[d["src_slot"]]
        batches.append(d)
    moved = [2 * int(d["size"].sum()) for d in batches]
    torch.cuda.synchronize()

    for b in range(args.warmup):
        rc, _ = H.hicr_memcpy_batch(ctx, batches[b], sched)
        assert rc == H.OK, H.hicr_last_error(ctx)
        assert H.hicr_fence(ctx) == H.OK

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    step_s = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        ev[k][0].record(stream)
        rc, _ = H.hicr_memcpy_batch(ctx, batches[args.warmup + k], sched)
        ev[k][1].record(stream)
        assert rc == H.OK, H.hicr_last_error(ctx)
        assert H.hicr_fence(ctx) == H.OK
        step_s.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0

    timed_bytes = sum(moved[args.warmup:])
    kern_ms = np.array([a.elapsed_time(b) for a, b in ev])
    per_launch = np.array(moved[args.warmup:], dtype=np.float64)
    achieved = float(np.mean(per_launch / (kern_ms * 1e-3)) / 1e9)
    traffic = traffic_per_launch()
    ceiling = copy_ceiling(torch, wd, pool, stream)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic["hbm_bytes_per_launch"] if traffic else None,
            "kernel": "hicr::copy_kernel", "avg_launch_ms": round(float(kern_ms.mean()), 4),
            "algorithmic_bytes_per_launch": int(per_launch.mean()),
            "copy_ceiling": ceiling,
            "frac_of_best_copy": round(achieved / ceiling["best_copy_GBps"], 4)}
    out = {
        "metric": METRIC, "value": round(timed_bytes / total / 1e9, 1), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "batched slot memcpy: 4096 requests/batch, sizes log-uniform "
                               "256 B..64 MiB, unaligned offsets, disjoint destinations, 8192 "
                               "slot windows (72 MiB at 8 MiB stride) over a 64 GiB + 64 MiB "
                               "pool, one fused launch + fence per batch",
                   "requests_per_batch": 4096, "slots": 8192, "pool_bytes": wm.B_POOL,
                   "schedule": (args.sched if "," not in args.sched else
                                "fixed: {} B chunks, at least {} piece(s) per request, unroll {}"
                                .format(*args.sched.split(","))),
                   "copy_wgs_per_cu": args.copy_grid or (
                       "library default for the schedule: 4 for chunks of 4 KiB or less, 1 "
                       "above 16 KiB up to 32 KiB, otherwise 2"),
                   "gb_per_batch_rw": round(float(np.mean(moved)) / 1e9, 3)},
        "p50_ms": round(float(np.percentile(step_s, 50)) * 1e3, 4),
        "p99_ms": round(float(np.percentile(step_s, 99)) * 1e3, 4),
        "roofline": roof,
    }
    H.hicr_ctx_destroy(ctx)
    del pool
    torch.cuda.empty_cache()
    def progress(what):
        print(f"bench: {what} ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)

    progress("batched copy measured")
    if not args.no_channels:
        out["channels"] = [bench_channels(torch, H, m) for m in (H.CH_MPSC_LOCK, H.CH_MPSC_NOLOCK)]
        progress("channels measured")
    if not args.no_tiny:
        out["tiny"] = bench_tiny(torch, H)
        progress("tiny batch latency measured")
    if not args.no_serving:
        sv = bench_serving(torch, H, duration_s=args.serve_seconds, budget=int(args.serve_budget))
        out["serving"] = {k: sv[k] for k in (
            "value", "unit", "requests", "duration_s", "rate", "budget_bytes", "latency_p50_ms",
            "latency_p99_ms", "copy_latency_p99_ms", "burst_latency_p99_ms", "queue_wait_p99_ms",
            "peak_arena_bytes", "wall_s")}
        progress("serving measured")
    if not args.no_learned:
        ln = bench_learned(torch, H, n_train=args.line_learned_train, n_test=args.line_learned_test)
        out["learned"] = {k: ln[k] for k in (
            "n_train", "n_test", "fixed_best_class", "accuracy", "train_seconds",
            "by_autotune_times", "measured", "wall_seconds")}
        progress("learned schedule measured")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wm.batched(0))
        out["cpu_baseline"]["channels"] = cpu_channel_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
