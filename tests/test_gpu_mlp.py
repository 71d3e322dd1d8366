"""GPU parity of the schedule network against the fp64 oracle.

The GPU kernels compute in fp32, the oracle in fp64; tolerances: logits and
loss 1e-4 relative, gradients max-abs error <= 1e-4 * max|g| per tensor,
parameters after Adam steps 2e-5 absolute.  The argmax class must match
except where the oracle's top two logits are within 1e-5 (relative).
"""
import numpy as np
import pytest

from oracle import mlp
from workloads import memcpy as wm
from workloads.mlp_init import he_uniform

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2509_01425_amd import hicr as H
    # The library runs on torch's current stream here, so that the tensors
    # torch makes (gathers, fills) are ordered before the library's kernels,
    # and blocks torch frees are reused only after those kernels ran.
    prev = torch.cuda.current_stream()
    s = torch.cuda.Stream()
    torch.cuda.set_stream(s)
    rc, ctx = H.hicr_ctx_create(0, s.cuda_stream)
    assert rc == H.OK
    yield torch, H, ctx
    assert H.hicr_ctx_destroy(ctx) == H.OK
    torch.cuda.synchronize()
    torch.cuda.set_stream(prev)


def _data(seed, B):
    g = np.random.default_rng(seed)
    x = np.log2(1 + g.integers(0, 400, size=(B, 32)) * (g.random((B, 32)) < 0.4)).astype(np.float32)
    y = g.integers(0, 12, size=B).astype(np.int32)
    return x, y


def _tensors(torch, x, y):
    return (torch.from_numpy(x).cuda().contiguous(), torch.from_numpy(y).cuda().contiguous())


@pytest.mark.parametrize("B", [1, 7, 64, 256, 300, 4096])
def test_forward_and_grad_vs_oracle(env, B):
    torch, H, ctx = env
    theta = he_uniform(B)
    assert H.hicr_mlp_set_params(ctx, theta) == H.OK
    x, y = _data(B, B)
    xd, yd = _tensors(torch, x, y)
    logits = torch.zeros(B, 12, dtype=torch.float32, device="cuda")
    grad = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    assert H.hicr_mlp_forward(ctx, xd.data_ptr(), B, logits.data_ptr()) == H.OK
    assert H.hicr_mlp_grad(ctx, xd.data_ptr(), yd.data_ptr(), B, grad.data_ptr(),
                           loss.data_ptr()) == H.OK
    th64 = theta.astype(np.float64)
    z_ref, _ = mlp.forward(th64, x.astype(np.float64))
    z = logits.cpu().numpy()
    assert np.allclose(z, z_ref, rtol=1e-4, atol=1e-4 * np.abs(z_ref).max())
    srt = np.sort(z_ref, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-5 * np.maximum(np.abs(srt[:, -1]), 1e-30)
    assert (np.argmax(z, 1)[clear] == np.argmax(z_ref, 1)[clear]).all()
    g_ref = mlp.grad(th64, x.astype(np.float64), y)
    L_ref = mlp.loss(th64, x.astype(np.float64), y)
    assert abs(loss.item() - L_ref) <= 1e-4 * max(1.0, abs(L_ref))
    g = grad.cpu().numpy().astype(np.float64)
    gp, rp = mlp.unpack(g), mlp.unpack(g_ref)
    for name, _ in mlp.SHAPES:
        scale = np.abs(rp[name]).max()
        assert np.abs(gp[name] - rp[name]).max() <= 1e-4 * max(scale, 1e-12), name


def test_adam_steps_track_oracle(env):
    torch, H, ctx = env
    theta = he_uniform(9)
    assert H.hicr_mlp_set_params(ctx, theta) == H.OK
    opt = mlp.Adam(mlp.N_PARAMS)
    th = theta.astype(np.float64)
    for step in range(20):
        x, y = _data(100 + step, 64)
        xd, yd = _tensors(torch, x, y)
        assert H.hicr_mlp_train_step(ctx, xd.data_ptr(), yd.data_ptr(), 64, 1e-3) == H.OK
        th = opt.step(th, mlp.grad(th, x.astype(np.float64), y))
    assert H.hicr_fence(ctx) == H.OK
    rc, got = H.hicr_mlp_get_params(ctx)
    assert rc == H.OK
    # Adam normalises each step to about lr per coordinate; fp32 rounding of
    # tiny gradients can flip a step's size, so allow a few ulp-scale drifts
    err = np.abs(got.astype(np.float64) - th)
    assert np.percentile(err, 99) < 2e-5 and err.max() < 2e-3


def test_training_reduces_loss(env):
    torch, H, ctx = env
    g = np.random.default_rng(3)
    # a learnable rule: the class is the index of the largest of the first 12 features
    x = (g.random((2048, 32)) * 4).astype(np.float32)
    y = np.argmax(x[:, :12], axis=1).astype(np.int32)
    xd, yd = _tensors(torch, x, y)
    assert H.hicr_mlp_set_params(ctx, he_uniform(11)) == H.OK
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    assert H.hicr_mlp_grad(ctx, xd.data_ptr(), yd.data_ptr(), 2048, grad.data_ptr(),
                           loss.data_ptr()) == H.OK
    l0 = loss.item()
    for ep in range(15):
        perm = torch.from_numpy(g.permutation(2048)).cuda()
        for i in range(0, 2048, 256):
            idx = perm[i:i + 256]
            xb, yb = xd[idx].contiguous(), yd[idx].contiguous()
            assert H.hicr_mlp_train_step(ctx, xb.data_ptr(), yb.data_ptr(), 256, 3e-3) == H.OK
    assert H.hicr_fence(ctx) == H.OK
    assert H.hicr_mlp_grad(ctx, xd.data_ptr(), yd.data_ptr(), 2048, grad.data_ptr(),
                           loss.data_ptr()) == H.OK
    assert loss.item() < 0.5 * l0


def test_out_of_range_labels_give_nan_loss_and_no_gradient(env):
    """Labels outside [0, 12) are never used as indices: the mean loss is NaN
    and the gradient is the valid samples' share of the batch mean."""
    torch, H, ctx = env
    B = 40
    theta = he_uniform(21)
    assert H.hicr_mlp_set_params(ctx, theta) == H.OK
    x, y = _data(21, B)
    bad = np.array([0, 7, 39])
    y[bad] = [12, -1, 1 << 30]
    xd, yd = _tensors(torch, x, y)
    grad = torch.zeros(mlp.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    assert H.hicr_mlp_grad(ctx, xd.data_ptr(), yd.data_ptr(), B, grad.data_ptr(),
                           loss.data_ptr()) == H.OK
    assert np.isnan(loss.item())
    ok = np.setdiff1d(np.arange(B), bad)
    th64 = theta.astype(np.float64)
    g_ref = mlp.grad(th64, x[ok].astype(np.float64), y[ok]) * (len(ok) / B)
    g = grad.cpu().numpy().astype(np.float64)
    gp, rp = mlp.unpack(g), mlp.unpack(g_ref)
    for name, _ in mlp.SHAPES:
        assert np.abs(gp[name] - rp[name]).max() <= 1e-4 * max(np.abs(rp[name]).max(), 1e-12), name


def test_learned_submission_picks_oracle_class_and_moves_bytes(env):
    """HICR_SCHED_LEARNED: the class the library's network picks for the
    batch equals the oracle network's argmax on the oracle's feature, and the
    bytes are exact."""
    torch, H, ctx = env
    import oracle
    from workloads import device as wd
    from workloads.content import content
    bases, sizes, pool_len, descs, _ = wm.tiny(3)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    seed = 66
    wd.fill(pool.data_ptr(), pool_len, seed)
    torch.cuda.synchronize()
    slots = np.array([H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(s))[1]
                      for b, s in zip(bases, sizes)], dtype=np.uint32)
    d = descs.copy()
    d["dst_slot"], d["src_slot"] = slots[descs["dst_slot"]], slots[descs["src_slot"]]
    for k in range(6):
        theta = he_uniform(200 + k)
        # bias the last layer so that several different classes win
        p = mlp.unpack(theta.astype(np.float64))
        p["b3"][:] = 0
        p["b3"][(3 * k) % 12] = 5.0
        theta = mlp.pack(p).astype(np.float32)
        assert H.hicr_mlp_set_params(ctx, theta) == H.OK
        wd.fill(pool.data_ptr(), pool_len, seed)
        torch.cuda.synchronize()
        rc, _ = H.hicr_memcpy_batch(ctx, d, H.make_sched(65536, 1, 2, H.SCHED_LEARNED))
        assert rc == H.OK, H.hicr_last_error(ctx)
        assert H.hicr_fence(ctx) == H.OK
        rc, cls = H.hicr_last_choice(ctx)
        f = mlp.features(descs["size"])
        assert rc == H.OK and cls == int(mlp.predict(theta.astype(np.float64), f)[0])
        host = content(seed, 0, pool_len)
        oc = oracle.Ctx()
        for b, s in zip(bases, sizes):
            oc.register(host, offset=int(b), size=int(s))
        assert oc.memcpy_batch(descs)[0] == oracle.OK
        assert np.array_equal(pool.cpu().numpy(), host)
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK




def test_device_forward_argmax_equals_host_choice(env):
    """The learned submission infers on the host; the device forward kernel
    sums every layer in the same order with fused multiply-adds, so for any
    parameters the argmax of the device logits is the host's class.  Checked
    with unbiased random parameters on 40 random subsets of a hazard-free
    batch (random request counts give varied features)."""
    torch, H, ctx = env
    bases, sizes, pool_len, descs, _ = wm.tiny(5)
    pool = torch.empty(pool_len, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    slots = np.array([H.hicr_slot_register(ctx, pool.data_ptr() + int(b), int(s))[1]
                      for b, s in zip(bases, sizes)], dtype=np.uint32)
    d_all = descs.copy()
    d_all["dst_slot"], d_all["src_slot"] = slots[descs["dst_slot"]], slots[descs["src_slot"]]
    theta = he_uniform(300).astype(np.float32)
    assert H.hicr_mlp_set_params(ctx, theta) == H.OK
    g = np.random.default_rng(17)
    x = torch.empty(1, 32, dtype=torch.float32, device="cuda")
    z = torch.empty(1, 12, dtype=torch.float32, device="cuda")
    for _ in range(40):
        k = int(g.integers(1, len(d_all) + 1))
        d = d_all[np.sort(g.choice(len(d_all), size=k, replace=False))]
        rc, _ = H.hicr_memcpy_batch(ctx, d, H.make_sched(65536, 1, 2, H.SCHED_LEARNED))
        assert rc == H.OK, H.hicr_last_error(ctx)
        assert H.hicr_fence(ctx) == H.OK
        rc, cls = H.hicr_last_choice(ctx)
        assert rc == H.OK
        rc, f = H.hicr_sched_features(d)
        assert rc == H.OK
        x.copy_(torch.from_numpy(f).reshape(1, 32))
        torch.cuda.synchronize()
        assert H.hicr_mlp_forward(ctx, x.data_ptr(), 1, z.data_ptr()) == H.OK
        assert int(torch.argmax(z.cpu()[0])) == cls, (k, cls, z.cpu()[0])
    for s in slots:
        assert H.hicr_slot_deregister(ctx, int(s)) == H.OK


def test_tuned_table_lookup_is_the_nearest_feature(env):
    """The tuned table's choice equals a brute-force nearest neighbour over
    the oracle's features (first minimum on ties); an empty table is an
    error."""
    torch, H, ctx = env
    assert H.hicr_tune_clear(ctx) == H.OK
    assert H.hicr_tune_lookup(ctx, wm.family(0)[0])[0] == H.EINVAL
    table = [wm.family(b)[0] for b in range(300)]
    g = np.random.default_rng(4)
    labels = g.integers(0, 12, size=len(table))
    for d, c in zip(table, labels):
        assert H.hicr_tune_add(ctx, d, int(c)) == H.OK
    feats = np.array([mlp.features(d["size"]) for d in table])
    for b in range(300, 420):
        d = wm.family(b)[0]
        dist = ((feats - mlp.features(d["size"])[None, :]) ** 2).sum(1)
        # the library sums in fp32: any entry within rounding of the minimum
        # may win; otherwise the choice is unique
        near = dist <= dist.min() + 1e-4 * max(1.0, dist.min())
        rc, got = H.hicr_tune_lookup(ctx, d)
        assert rc == H.OK and got in set(int(x) for x in labels[near]), b
        if near.sum() == 1:
            assert got == int(labels[int(np.argmin(dist))])
    assert H.hicr_tune_clear(ctx) == H.OK
