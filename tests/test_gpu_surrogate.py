"""GPU surrogate kernels against the FP64 reference network (bfloat16
rounding emulated at the points where the kernels round): forward, loss,
gradients, Adam, routing.  All calls go through the C-ABI.

Tolerances: with the same bfloat16 rounding points on both sides the kernels
differ from the reference only by FP32 accumulation (about 1e-7 relative).
That flips a rounding decision of a hidden activation in roughly one element
in 10^4-10^5, each flip moving that activation by one bfloat16 step (2^-8), so
the output moves by a few 1e-5 relative on the 922k-parameter net: the
forward bound is 5e-4, the gradient bound (one more product chain) 5e-3."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M

pytestmark = pytest.mark.gpu

FULL = [5, 512, 512, 512, 512, 256]
SMALL = [5, 128, 64, 192]


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _setup(widths, nets=1, rows=1024, seed=0, n=256):
    from paper_2207_06908_amd import sur
    e = sur.Ensemble(widths, n_nets=nets, max_rows=rows)
    rng = np.random.default_rng(seed)
    ps = [M.init_params(widths, seed + 10 + q) for q in range(nets)]
    for q in range(nets):
        e.set_params(q, M.flat(ps[q]))
    X = rng.uniform(-1, 1, (n, widths[0])).astype(np.float32)
    T = (0.5 * rng.standard_normal((n, widths[-1]))).astype(np.float32)
    return e, ps, X, T


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("widths,n", [(SMALL, 100), (SMALL, 256), (FULL, 1024)])
def test_forward_matches_emulated_reference(widths, n):
    e, ps, X, T = _setup(widths, n=n)
    # parameters survive the round trip through the device exactly
    assert np.array_equal(e.get_params(0), M.flat(ps[0]).astype(np.float32))
    y = e.forward(0, _dev(X)).cpu().numpy()
    p32 = M.unflat(M.flat(ps[0]).astype(np.float32).astype(np.float64), widths)
    ref, _ = M.forward(p32, X.astype(np.float64), bf=True)
    err = _rel(y, ref)
    print(f"forward {widths} n={n} rel L2 {err:.2e}")
    assert err < 5e-4


@pytest.mark.parametrize("widths,batch", [(SMALL, 64), (SMALL, 100), (FULL, 1024)])
def test_loss_and_gradients_match_reference(widths, batch):
    e, ps, X, T = _setup(widths, n=max(batch, 256))
    rng = np.random.default_rng(3)
    rows = rng.permutation(X.shape[0])[:batch].astype(np.int32)
    loss = e.train_step(0, _dev(X), _dev(T), rows=_dev(rows), lr=0.0, update=False)
    g = e.get_grads(0)
    p32 = M.unflat(M.flat(ps[0]).astype(np.float32).astype(np.float64), widths)
    Xb, Tb = X[rows].astype(np.float64), T[rows].astype(np.float64)
    y, cache = M.forward(p32, Xb, bf=True)
    L, dY = M.mse(y, Tb)
    assert abs(float(loss.item()) - L) <= 2e-3 * L
    ref = M.backward(p32, cache, dY, bf=True)
    got = M.unflat(g.astype(np.float64), widths)
    for l, ((gW, gb), (rW, rb)) in enumerate(zip(got, ref)):
        eW, eb = _rel(gW, rW), _rel(gb, rb)
        cos = float(np.dot(gW.ravel(), rW.ravel()) / (np.linalg.norm(gW) * np.linalg.norm(rW)))
        print(f"layer {l}: dW rel L2 {eW:.2e} cos {cos:.6f}  db rel L2 {eb:.2e}")
        assert eW < 5e-3 and eb < 5e-3 and cos > 0.9999
    # against the exact FP64 gradient (no bfloat16 rounding anywhere)
    y2, c2 = M.forward(p32, Xb)
    exact = M.flat(M.backward(p32, c2, M.mse(y2, Tb)[1]))
    assert _rel(g, exact) < 5e-2


def test_gradients_are_deterministic():
    e, ps, X, T = _setup(SMALL, n=256)
    e.train_step(0, _dev(X), _dev(T), batch=256, lr=0.0, update=False)
    g1 = e.get_grads(0)
    e.train_step(0, _dev(X), _dev(T), batch=256, lr=0.0, update=False)
    assert np.array_equal(g1, e.get_grads(0))


def test_adam_step_matches_reference_on_the_same_gradient():
    e, ps, X, T = _setup(SMALL, n=256)
    p0 = e.get_params(0).astype(np.float64)
    opt = M.Adam(M.unflat(p0, SMALL), lr=1e-3)
    cur = M.unflat(p0, SMALL)
    for step in range(3):
        e.train_step(0, _dev(X), _dev(T), batch=256, lr=1e-3, update=True)
        g = e.get_grads(0).astype(np.float64)
        cur = opt.step(cur, M.unflat(g, SMALL))
        got = e.get_params(0).astype(np.float64)
        d = np.abs(got - M.flat(cur))
        print(f"adam step {step}: max |diff| {d.max():.2e}")
        assert d.max() < 2e-6


def test_training_reduces_the_loss():
    from paper_2207_06908_amd import sur
    rng = np.random.default_rng(9)
    e = sur.Ensemble(SMALL, n_nets=1, max_rows=256)
    e.init_params(0, 123)
    X = rng.uniform(-1, 1, (2048, 5)).astype(np.float32)
    tt = np.linspace(0, 1, SMALL[-1])
    T = (np.sin(2.0 * X[:, :1] + 3.0 * tt[None, :] * (1.5 + X[:, 1:2])) * (1 + 0.3 * X[:, 2:3])).astype(np.float32)
    xd, td = _dev(X), _dev(T)
    first = None
    for it in range(300):
        rows = _dev(rng.integers(0, 2048, 256).astype(np.int32))
        loss = e.train_step(0, xd, td, rows=rows, lr=2e-3)
        if first is None:
            first = float(loss.item())
    y = e.forward(0, xd).cpu().numpy()
    final = float(np.mean((y - T) ** 2))
    print("first batch loss", first, "final loss", final)
    assert final < 0.1 * first


def test_infer_route_matches_reference():
    nets = 3
    e, ps, X, T = _setup(SMALL, nets=nets, rows=128, n=300)
    Xd = _dev(X)
    ym, spread, ids, cnt = e.infer_route(Xd, 0.05)
    torch.cuda.synchronize()
    ys = [M.forward(M.unflat(M.flat(p).astype(np.float32).astype(np.float64), SMALL), X.astype(np.float64),
                    bf=True)[0] for p in ps]
    assert _rel(ym.cpu().numpy(), np.mean(ys, axis=0)) < 2e-3
    pk = np.stack([y.max(axis=1) for y in ys])
    sp = (pk.max(0) - pk.min(0)) / np.abs(pk.mean(0))
    got = spread.cpu().numpy()
    assert np.allclose(got, sp, rtol=2e-2, atol=1e-4)
    # the routing decision is taken on the kernel's own spread values
    want = np.nonzero(~(got <= 0.05))[0]
    n = int(cnt.item())
    assert n == want.size and np.array_equal(ids[:n].cpu().numpy(), want)
    # each net alone through sur_forward gives the same outputs as the ensemble path
    y0 = e.forward(0, Xd).cpu().numpy()
    assert _rel(y0, ys[0]) < 2e-3


def test_four_net_route_and_fallback_list_exact():
    """Four nets take the vectorized routing kernel: its means and spreads
    equal an FP32 emulation from the nets' own outputs (sums over the nets in
    order from 0, exact peaks, the spread formed in the same order) bit for
    bit, and the fallback list is exactly the rows whose spread is above the
    threshold or not finite, in order (5,003 rows: chunks of several rows per
    thread and a ragged tail)."""
    e, ps, X, T = _setup(SMALL, nets=4, rows=8192, n=5003, seed=4)
    Xd = _dev(X)
    ym, spread, ids, cnt = e.infer_route(Xd, 0.05)
    torch.cuda.synchronize()
    ys = [e.forward(q, Xd).cpu().numpy().astype(np.float32) for q in range(4)]
    acc = np.zeros_like(ys[0])
    for y in ys:
        acc = (acc + y).astype(np.float32)
    assert np.array_equal(ym.cpu().numpy(), (acc / np.float32(4)).astype(np.float32))
    pk = [y.max(axis=1) for y in ys]
    pmax = np.full(pk[0].shape, -np.inf, np.float32)
    pmin = np.full(pk[0].shape, np.inf, np.float32)
    psum = np.zeros(pk[0].shape, np.float32)
    for p in pk:
        pmax, pmin, psum = np.maximum(pmax, p), np.minimum(pmin, p), (psum + p).astype(np.float32)
    sp = ((pmax - pmin) / np.abs(psum / np.float32(4))).astype(np.float32)
    got = spread.cpu().numpy()
    assert np.array_equal(got, sp)
    for thr in (0.05, float(np.median(got)), 0.0, float("inf")):
        ym, spread, ids, cnt = e.infer_route(Xd, thr)
        want = np.nonzero(~(spread.cpu().numpy() <= thr))[0]
        n = int(cnt.item())
        assert n == want.size and np.array_equal(ids[:n].cpu().numpy(), want), thr
    # 70,001 rows: two 64-row segments per thread of the compaction, and a tail
    Xb = _dev(np.random.default_rng(9).uniform(-1, 1, (70001, SMALL[0])).astype(np.float32))
    ym, spread, ids, cnt = e.infer_route(Xb, 0.05)
    want = np.nonzero(~(spread.cpu().numpy() <= 0.05))[0]
    n = int(cnt.item())
    assert 0 < n < 70001 and n == want.size and np.array_equal(ids[:n].cpu().numpy(), want)


def test_infer_route_empty_and_chunked():
    e, ps, X, T = _setup(SMALL, nets=2, rows=64, n=200)
    ym, spread, ids, cnt = e.infer_route(_dev(X[:0]), 0.02)
    assert int(cnt.item()) == 0
    ym, spread, ids, cnt = e.infer_route(_dev(X), 0.02)   # 200 rows in chunks of 64
    ym2 = []
    for c0 in range(0, 200, 64):
        a, _s, _i, _c = e.infer_route(_dev(X[c0:c0 + 64]), 0.02)
        ym2.append(a.cpu().numpy())
    assert np.array_equal(ym.cpu().numpy(), np.concatenate(ym2))


def test_large_and_small_product_tiles_give_the_same_bits():
    """Products with at least 1024 blocks of 128 x 128 use 4 x 4 fragments per
    wave, smaller ones 2 x 2; every output still accumulates its K steps in
    the same order, so a 65,536-row inference (128 x 128 tiles) must equal
    the same rows run in 8,192-row chunks (64 x 64 tiles) bit for bit."""
    from paper_2207_06908_amd import sur
    big, ps, X, _T = _setup(FULL, nets=2, rows=65536, n=65536, seed=3)
    big.set_kernel(0)        # per-layer products (the fused kernel is checked below)
    small = sur.Ensemble(FULL, n_nets=2, max_rows=8192)
    small.set_kernel(0)
    for q in range(2):
        small.set_params(q, M.flat(ps[q]))
    xd = _dev(X)
    ym_big, sp_big, _i, _c = big.infer_route(xd, 0.02)
    ym_small, sp_small, _i2, _c2 = small.infer_route(xd, 0.02)
    assert np.array_equal(ym_big.cpu().numpy(), ym_small.cpu().numpy())
    assert np.array_equal(sp_big.cpu().numpy(), sp_small.cpu().numpy())
    y0 = big.forward(0, xd[:4096]).cpu().numpy()
    y1 = small.forward(0, xd[:4096]).cpu().numpy()
    assert np.array_equal(y0, y1)


def test_fused_inference_equals_the_layer_products():
    """The fused inference kernel (every layer of every net in one launch,
    activations on chip) gives the same bits as one product launch per layer
    and net: same routing means and spreads over 65,536 rows and a ragged
    chunk, and the same single-net outputs."""
    from paper_2207_06908_amd import sur
    ens, ps, X, _T = _setup(FULL, nets=4, rows=65536, n=65536, seed=8)
    xd = _dev(X)
    out = {}
    for fused in (1, 0):
        ens.set_kernel(fused)
        ym, sp, ids, cnt = ens.infer_route(xd, 0.02)
        yr, spr, _i, _c = ens.infer_route(xd[:1000], 0.02)    # 1000 rows: a block of 128 with 64 pad rows
        out[fused] = (ym.cpu().numpy(), sp.cpu().numpy(), ids[:int(cnt.item())].cpu().numpy(),
                      yr.cpu().numpy(), spr.cpu().numpy(), ens.forward(1, xd[:777]).cpu().numpy())
    for a, b in zip(out[1], out[0]):
        assert np.array_equal(a, b)
    assert np.abs(out[1][0]).max() > 0
