"""Seeded input generators: reproducible, and shaped like the configurations
they stand for (rates, size laws, ranges, disjointness)."""
import numpy as np

from workloads import memcpy as wm
from workloads import serving as ws


def test_serving_trace_shape():
    tr = ws.trace(duration_s=2.0, rate=2000, src_bytes=16 << 30, n_channels=1024, batch=1)
    n = len(tr.reqs)
    assert 3600 < n < 4400                                     # Poisson(4000)
    arr = tr.reqs["arrival_ns"].astype(np.int64)
    assert (np.diff(arr) >= 0).all() and arr[-1] <= 2e9
    gaps = np.diff(arr) / 1e9
    assert abs(gaps.mean() - 1 / 2000) < 0.1 / 2000           # exponential gaps, mean 0.5 ms
    kinds = tr.reqs["kind"]
    assert 0.45 < kinds.mean() < 0.55
    for r in tr.reqs:
        f, c = int(r["first"]), int(r["count"])
        if r["kind"] == 0:
            assert 8 <= c <= 512
            d = tr.descs[f:f + c]
            assert (d["size"] >= 64).all() and (d["size"] <= 16 << 20).all()
            ends = d["dst_off"] + d["size"]
            assert (d["dst_off"][1:] >= ends[:-1]).all()      # disjoint, in order
            assert int(ends.max()) == int(r["hbm_bytes"])
            assert (d["src_off"] + d["size"] <= 16 << 30).all()
        else:
            assert 1 <= c <= 256 and r["channel"] < 1024
            sz = tr.msg_size[f:f + c]
            assert (sz >= 16).all() and (sz <= 256 << 10).all()
            assert int(sz.sum()) == int(r["hbm_bytes"])
    a = ws.trace(duration_s=0.05, batch=3)
    b = ws.trace(duration_s=0.05, batch=3)
    assert a.reqs.tobytes() == b.reqs.tobytes() and a.descs.tobytes() == b.descs.tobytes()


def test_family_law():
    fams, ns = [], []
    for b in range(400):
        d, f = wm.family(b)
        fams.append(f)
        ns.append(len(d))
        s = d["size"].astype(np.int64)
        if f == 0:
            assert s.min() >= 1 and s.max() <= 8192
        else:
            assert s.min() >= 256 and s.max() <= 64 << 20
        assert 2 * s.sum() <= 0.9 * wm.B_POOL
    assert 0.4 < np.mean(fams) < 0.6
    assert min(ns) >= 1 and max(ns) <= 4096
    # log-uniform counts: about half of the batches have fewer than sqrt(8*4096) requests
    assert 0.35 < np.mean(np.array(ns) < 181) < 0.65


def test_log_uniform_law():
    g = wm.rng(99)
    x = wm.log_uniform(g, 16, 256 << 10, 200_000).astype(np.float64)
    assert x.min() >= 16 and x.max() <= 256 << 10
    mean = ((256 << 10) - 16) / np.log((256 << 10) / 16)      # (b - a) / ln(b / a)
    assert abs(x.mean() / mean - 1) < 0.02
    assert abs(np.median(x) / np.sqrt(16 * (256 << 10)) - 1) < 0.03


def test_halo_exchange_matches_array_slicing():
    """The halo requests, applied by the oracle, fill every ghost face (h
    planes deep) with the neighbour's boundary planes -- checked against
    numpy slicing of the same grids -- and touch nothing else."""
    import oracle
    from workloads import halo
    for N, Py, Pz, h in [(12, 2, 3, 2), (10, 1, 5, 1), (8, 2, 2, 3)]:
        nx, ny, nz = halo.dims(N, Py, Pz)
        d = halo.exchange(N, Py, Pz, h)
        assert len(d) == halo.n_requests(N, Py, Pz, h)
        assert (d["size"] == nx * 8).all()
        g = np.random.default_rng(N + h)
        shape = (nz + 2 * h, ny + 2 * h, nx + 2 * h)             # [z][y][x]
        grids = [g.integers(0, 2**62, size=shape, dtype=np.int64) for _ in range(Py * Pz)]
        before = [a.copy() for a in grids]
        oc = oracle.Ctx()
        ids = [oc.register(a.view(np.uint8).reshape(-1))[1] for a in grids]
        od = d.copy()
        od["dst_slot"] = np.array(ids)[d["dst_slot"]]
        od["src_slot"] = np.array(ids)[d["src_slot"]]
        assert oc.hazard_check(od)[0] == oracle.OK
        assert oc.memcpy_batch(od)[0] == oracle.OK
        want = [a.copy() for a in before]
        X = slice(h, nx + h)
        Y = slice(h, ny + h)
        Z = slice(h, nz + h)
        for k in range(Pz):
            for j in range(Py):
                s = j + Py * k
                if j + 1 < Py:
                    want[s][Z, ny + h:ny + 2 * h, X] = before[s + 1][Z, h:2 * h, X]
                if j > 0:
                    want[s][Z, 0:h, X] = before[s - 1][Z, ny:ny + h, X]
                if k + 1 < Pz:
                    want[s][nz + h:nz + 2 * h, Y, X] = before[s + Py][h:2 * h, Y, X]
                if k > 0:
                    want[s][0:h, Y, X] = before[s - Py][nz:nz + h, Y, X]
        for s in range(Py * Pz):
            assert np.array_equal(grids[s], want[s]), (N, Py, Pz, h, s)
        sb = halo.sub_bytes(N, Py, Pz, h)
        assert (d["dst_off"] + d["size"] <= sb).all() and (d["src_off"] + d["size"] <= sb).all()
    # the paper's best decomposition: 704^3 over 1 x 2 x 22, 13-point stencil (h = 2)
    assert halo.n_requests(704, 2, 22, 2) == 61_952
