"""The learned direction proposal on the GPU against the CPU references.

Exact: histograms, the top-8 choice on the GPU's own scores, the extra
extreme slots, labels, survivors and hulls.  Within tolerance (bf16 products,
fp32 accumulation vs binary64): network scores and gradients.  Monotonicity:
learned survivors are a subset of the plain ones and the hull never changes.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1405_3454_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1405_3454_amd.api import Hull
    h = Hull(0)
    yield h
    torch.cuda.synchronize()
    h.close()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def u32(t):
    from paper_1405_3454_amd.api import as_u32
    return as_u32(t)


def mixed_batch(sizes, seed):
    return inputs.batch(sizes, seed, kinds=("mixture", "ellipse", "disk", "square"))


def bf16_bits(a):
    r = np.asarray(mlp.bf16(np.asarray(a, np.float64)), np.float32)
    return (r.view(np.uint32) >> 16).astype(np.uint16)


def test_histogram_parity(H):
    sizes = [1, 2, 5, 100, 16384, 16385, 40000, 70001]
    x, y, off, _ = mixed_batch(sizes, 3)
    hb, hf = H.histogram_batched(dev(x), dev(y), dev(off))
    hf = hf.cpu().numpy()
    hb = hb.cpu().numpy().view(np.uint16)
    for s in range(len(sizes)):
        want = oracle.histogram(x[off[s]:off[s + 1]], y[off[s]:off[s + 1]])
        assert np.array_equal(hf[s], want), s
        assert np.array_equal(hb[s], bf16_bits(want)), s


def _hist_batch(H, B, seed):
    sizes = list(np.random.default_rng(seed).integers(2000, 30000, size=B))
    x, y, off, _ = mixed_batch(sizes, seed)
    hb, hf = H.histogram_batched(dev(x), dev(y), dev(off))
    return hb, hf.cpu().numpy()


def elementwise_excess(got, ref):
    """Largest |got - ref| / (1e-2 |ref| + 2^-8 max|ref|) over the elements:
    at most 1 when every element is within 1 % of its reference value, or
    within one bf16 rounding step (2^-8) of the block's largest magnitude.
    The second term covers elements whose reference value is a sum that
    nearly cancels: there a single bf16 activation rounded the other way
    (fp32 accumulation order on the GPU vs binary64 in the reference) moves
    the element by about 2^-8 of one of its terms."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    tol = 1e-2 * np.abs(ref) + 2.0 ** -8 * np.abs(ref).max()
    return float((np.abs(got - ref) / np.maximum(tol, 1e-300)).max())


def test_forward_backward_against_binary64(H):
    import torch
    p = mlp.he_init(11)
    p[mlp.N_PARAMS - 64:] = np.linspace(-0.1, 0.1, 64, dtype=np.float32)   # non-zero b3
    H.mlp_set_params(p)
    hb, hf = _hist_batch(H, 100, 5)
    scores = H.mlp_forward(hb).cpu().numpy()
    want, cache = mlp.forward(p, hf, emulate=True)
    ex = elementwise_excess(scores, want)
    print("scores: worst element at %.3f of the tolerance" % ex)
    assert ex <= 1.0, ex
    dS = np.random.default_rng(6).standard_normal((100, 64)).astype(np.float32)
    g = H.mlp_backward(hb, torch.from_numpy(dS).to("cuda:0")).cpu().numpy().astype(np.float64)
    gw = mlp.backward(cache, dS, emulate=True)
    for part, (a, b) in zip(("W1", "b1", "W2", "b2", "W3", "b3"), zip(mlp.split(g), mlp.split(gw))):
        ex = elementwise_excess(a, b)
        print("%s: worst element at %.3f of the tolerance" % (part, ex))
        assert ex <= 1.0, (part, ex)


@pytest.mark.parametrize("gap", [0, 1, 2, 3])
def test_top_directions_exact(H, gap):
    import torch
    r = np.random.default_rng(9)
    sc = r.standard_normal((37, 64)).astype(np.float32)
    sc[3, :] = 0.0                     # all ties
    sc[4, [1, 2, 60]] = 5.0            # partial ties
    sc[5, 10] = np.nan
    sc[6, :] = -0.0
    sc[7, :] = -np.abs(np.arange(64) - 10)
    H.set_direction_gap(gap)
    try:
        got = H.top_directions(torch.from_numpy(sc).to("cuda:0")).cpu().numpy()
    finally:
        H.set_direction_gap(H.DEFAULT_DIRECTION_GAP)
    assert np.array_equal(got, mlp.top_directions(sc, gap=gap))


def test_learned_extremes_survivors_and_hull(H):
    p = mlp.he_init(21)
    H.mlp_set_params(p)
    sizes = [3000, 1, 70000, 12345, 500]
    x, y, off, _ = mixed_batch(sizes, 8)
    xt, yt, ot = dev(x), dev(y), dev(off)
    hb, _ = H.histogram_batched(xt, yt, ot)
    dirs = H.top_directions(H.mlp_forward(hb)).cpu().numpy()
    cd, sd = oracle.direction_table()
    slots = u32(H.extremes_batched(xt, yt, ot, learned=True))
    plain = u32(H.extremes_batched(xt, yt, ot))
    assert np.array_equal(slots[:, :16], plain)
    for s in range(len(sizes)):
        a, b = off[s], off[s + 1]
        es, _ = oracle.extremes_dirs(x[a:b], y[a:b], cd[dirs[s]], sd[dirs[s]])
        assert np.array_equal(slots[s, 16:].astype(np.int64), es.astype(np.int64) + a), s
    sv_l, so_l = H.discard_batched(xt, yt, ot, dev(slots.view(np.int32)))
    sv_p, so_p = H.discard_batched(xt, yt, ot, dev(plain.view(np.int32)))
    so_l, so_p = so_l.cpu().numpy(), so_p.cpu().numpy()
    sv_l, sv_p = u32(sv_l), u32(sv_p)
    hl, hlo = H.compute_batched(xt, yt, ot, learned=True)
    hp, hpo = H.compute_batched(xt, yt, ot)
    hl, hp, hlo, hpo = u32(hl), u32(hp), hlo.cpu().numpy(), hpo.cpu().numpy()
    for s in range(len(sizes)):
        a, b = off[s], off[s + 1]
        L = sv_l[so_l[s]:so_l[s + 1]]
        Pn = sv_p[so_p[s]:so_p[s + 1]]
        assert set(L) <= set(Pn)
        verts = oracle.polygon(x[a:b], y[a:b], slots[s] - a)
        want = oracle.discard(x[a:b], y[a:b], verts).astype(np.int64) + a
        assert np.array_equal(L.astype(np.int64), want), s
        hw = oracle.hull_subset(x[a:b], y[a:b]).astype(np.int64) + a
        assert np.array_equal(hl[hlo[s]:hlo[s + 1]].astype(np.int64), hw)
        assert np.array_equal(hp[hpo[s]:hpo[s + 1]].astype(np.int64), hw)


def test_labels_parity(H):
    sizes = [2000, 7000, 1, 4, 30000]
    x, y, off, _ = mixed_batch(sizes, 12)
    g = H.labels_batched(dev(x), dev(y), dev(off)).cpu().numpy()
    for s in range(len(sizes)):
        a, b = off[s], off[s + 1]
        want = oracle.labels(x[a:b], y[a:b]).astype(np.float32)
        assert np.array_equal(g[s], want), (s, g[s][:8], want[:8])


def test_label_targets_parity(H):
    """Greedy joint targets and orders: bit-exact against the oracle."""
    sizes = [2000, 7000, 1, 4, 30000, 0, 12345]
    x, y, off, _ = mixed_batch(sizes, 13)
    t, o = H.label_targets_batched(dev(x), dev(y), dev(off), rounds=8)
    t, o = t.cpu().numpy(), o.cpu().numpy()
    for s in range(len(sizes)):
        a, b = off[s], off[s + 1]
        wt, wo = oracle.label_targets(x[a:b], y[a:b], rounds=8)
        assert np.array_equal(o[s], wo), (s, o[s], wo)
        assert np.array_equal(t[s], wt), s


def test_train_step_matches_binary64_adam(H):
    """One training step on the GPU against the binary64 loss gradient and
    Adam step.  The loss matches within the bf16 tolerance.  Adam's first
    step is lr * g / (|g| + eps') per element, i.e. +-lr wherever the
    gradient is clearly non-zero: every parameter whose reference gradient
    exceeds the elementwise gradient tolerance must move by the reference
    step (same sign, magnitude within 1e-3 lr plus float32 rounding of the
    parameter), and no parameter may move by more than lr (1 + 1e-3)."""
    import torch
    p = mlp.he_init(31)
    H.mlp_set_params(p)
    hb, hf = _hist_batch(H, 64, 14)
    gain = np.abs(np.random.default_rng(2).standard_normal((64, 64))).astype(np.float32) * 0.01
    lr = 1e-3
    loss = H.mlp_train_step(hb, torch.from_numpy(gain).to("cuda:0"), lr).item()
    S, cache = mlp.forward(p, hf, emulate=True)
    L, dS = mlp.loss_and_grad(S, gain)
    assert loss == pytest.approx(L, rel=2e-2)
    g = mlp.backward(cache, dS, emulate=True)
    p2, _, _ = mlp.adam(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    got = H.mlp_get_params().astype(np.float64)
    step_got, step_ref = got - p, p2 - p
    ulp = np.spacing(np.abs(p).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(step_got) <= lr * (1 + 1e-3) + ulp)
    checked = 0
    for a, b, pg, pu in zip(mlp.split(step_got), mlp.split(step_ref), mlp.split(g), mlp.split(ulp)):
        sure = np.abs(pg) > 1e-2 * np.abs(pg) + 2.0 ** -8 * np.abs(pg).max()
        # eps (1e-8) shortens a step by lr eps / |g|; the GPU's gradient may
        # differ from the reference's by up to the tolerance, hence the
        # second term
        bound = lr * (1e-3 + 4e-8 / np.abs(pg[sure])) + pu[sure]
        assert np.all(np.sign(a[sure]) == np.sign(b[sure]))
        assert np.all(np.abs(a[sure] - b[sure]) <= bound)
        checked += int(sure.sum())
    assert checked > 0.05 * len(p)


def test_checkpoint_resume(H):
    """Training state saved after one step and restored gives the same next
    steps bit for bit (parameters, both Adam moments, step count); setting
    only the parameters starts a new run (zero moments, step 0)."""
    import torch
    p = mlp.he_init(77)
    hb, _ = _hist_batch(H, 64, 21)
    gains = [torch.from_numpy(np.abs(np.random.default_rng(10 + i).standard_normal((64, 64)))
                              .astype(np.float32) * 0.01).to("cuda:0") for i in range(3)]
    H.mlp_set_params(p)
    H.mlp_train_step(hb, gains[0], 1e-3)
    ckpt, step = H.mlp_get_state()
    assert step == 1
    n = H.mlp_param_count()
    assert np.any(ckpt[n:2 * n] != 0) and np.any(ckpt[2 * n:] != 0)
    for g in gains[1:]:
        H.mlp_train_step(hb, g, 1e-3)
    run_a, step_a = H.mlp_get_state()
    H.mlp_set_params(mlp.he_init(78))                  # something else in between
    H.mlp_train_step(hb, gains[0], 1e-3)
    H.mlp_set_state(ckpt, step)
    again, step_again = H.mlp_get_state()
    assert step_again == 1 and np.array_equal(again, ckpt)
    for g in gains[1:]:
        H.mlp_train_step(hb, g, 1e-3)
    run_b, step_b = H.mlp_get_state()
    assert step_a == step_b == 3
    assert np.array_equal(run_a, run_b)
    # set_params: a fresh run, the same as restoring zero moments at step 0
    H.mlp_set_params(p)
    H.mlp_train_step(hb, gains[0], 1e-3)
    fresh, _ = H.mlp_get_state()
    z = np.concatenate([p.astype(np.float32), np.zeros(2 * n, np.float32)])
    H.mlp_set_state(z, 0)
    H.mlp_train_step(hb, gains[0], 1e-3)
    fresh2, _ = H.mlp_get_state()
    assert np.array_equal(fresh, fresh2)
    from paper_1405_3454_amd._lib import HullError
    with pytest.raises(HullError):
        H.mlp_set_state(z[:-1], 0)


def test_training_gains_over_plain(H):
    """A short training run on the GPU: the trained proposal discards more
    than the plain 16-extreme filter and more than the untrained network."""
    from paper_1405_3454_amd import train
    x, y, off = train.batch_tensors(256, 1 << 15, 424242, H.device)
    H.mlp_set_params(train.init_params(5))
    untrained = train.evaluate(H, x, y, off)
    params, losses = train.train(H, sets=256 * 128, batch=128, points=1 << 15, lr=1e-3, seed=5)
    trained = train.evaluate(H, x, y, off)
    print("untrained", untrained, "trained", trained, "loss", losses[0], losses[-1])
    assert trained["plain"] == untrained["plain"]
    assert trained["learned"] >= trained["plain"]
    assert trained["learned"] - trained["plain"] > untrained["learned"] - untrained["plain"]
    assert losses[-1] < losses[0]


def test_learned_graph_replay_matches_eager(H):
    """hipGraph of the learned batched method (histogram, network, top-8,
    extremes, discard, hull) replayed several times, with eager work in
    between: every replay equals the eager learned result and the oracle."""
    import torch
    H.mlp_set_params(mlp.he_init(41))
    sizes = [5000, 1, 30000, 777, 12000]
    x, y, off, _ = mixed_batch(sizes, 17)
    xt, yt, ot = dev(x), dev(y), dev(off)
    eager, eho = H.compute_batched(xt, yt, ot, learned=True)
    eager = u32(eager)[: int(eho[-1].item())].copy()
    hull = torch.full((len(x),), -7, dtype=torch.int32, device="cuda:0")
    ho = torch.zeros(len(sizes) + 1, dtype=torch.int64, device="cuda:0")
    H.graph_capture(xt, yt, ot, hull, ho, learned=True)
    for rep in range(3):
        hull.fill_(-7)
        ho.zero_()
        torch.cuda.synchronize()
        H.graph_launch()
        torch.cuda.synchronize()
        assert np.array_equal(u32(hull)[: int(ho[-1].item())], eager), rep
        H.extremes_batched(xt, yt, ot, learned=True)       # eager work between replays
    eo = eho.cpu().numpy()
    for s in range(len(sizes)):
        a, b = off[s], off[s + 1]
        want = oracle.hull_subset(x[a:b], y[a:b]).astype(np.int64) + a
        assert np.array_equal(eager[eo[s]:eo[s + 1]].astype(np.int64), want)
