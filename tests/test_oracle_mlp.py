"""Pins for the network reference in oracle/mlp.py (CPU only)."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa -> 1
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-3.0) == -3.0 and mlp.bf16(0.0) == 0.0
    x = np.random.default_rng(0).standard_normal(1000)
    r = mlp.bf16(x)
    # 8 significant bits: r * 2^(8 - e) is an integer
    m, e = np.frexp(r)
    assert np.all(np.rint(m * 256) == m * 256)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_forward_hand_case():
    """All-ones first layer and unit later weights: every score equals the
    sum of ReLU(sum(x)) over the hidden units (computed by hand)."""
    W1 = np.ones((512, 1024))
    W2 = np.eye(512)
    W3 = np.zeros((64, 512))
    W3[:, 0] = 1.0
    p = mlp.join(W1, np.zeros(512), W2, np.zeros(512), W3, np.full(64, 0.5))
    X = np.zeros((2, 1024))
    X[0, :3] = [1.0, 2.0, 3.0]
    X[1, 0] = -5.0
    S, _ = mlp.forward(p, X, emulate=False)
    assert np.allclose(S[0], 6.5) and np.allclose(S[1], 0.5)


def test_backward_matches_finite_differences():
    r = np.random.default_rng(3)
    p = mlp.he_init(7).astype(np.float64) + 0.01 * r.standard_normal(mlp.N_PARAMS)
    X = np.abs(r.standard_normal((5, 1024)))
    dS = r.standard_normal((5, 64))
    S, cache = mlp.forward(p, X, emulate=False)
    g = mlp.backward(cache, dS, emulate=False)
    W1, b1, W2, b2, W3, b3 = mlp.split(np.arange(mlp.N_PARAMS, dtype=np.float64))
    idx = [int(W1[3, 17]), int(b1[9]), int(W2[100, 5]), int(b2[511]), int(W3[63, 200]), int(b3[0]),
           int(W1[511, 1023])]
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fp = (mlp.forward(pp, X, emulate=False)[0] * dS).sum()
        fm = (mlp.forward(pm, X, emulate=False)[0] * dS).sum()
        fd = (fp - fm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-4, abs=1e-7), i


def test_loss_gradient_finite_differences():
    r = np.random.default_rng(4)
    s = r.standard_normal((3, 64))
    gain = np.abs(r.standard_normal((3, 64)))
    gain[1] = 0.0
    L, d = mlp.loss_and_grad(s, gain)
    for (i, j) in [(0, 0), (1, 5), (2, 63)]:
        sp = s.copy(); sp[i, j] += 1e-6
        sm = s.copy(); sm[i, j] -= 1e-6
        fd = (mlp.loss_and_grad(sp, gain)[0] - mlp.loss_and_grad(sm, gain)[0]) / 2e-6
        assert d[i, j] == pytest.approx(fd, rel=1e-5)
    assert np.all(mlp.targets(gain)[1] == 0) and np.isclose(mlp.targets(gain)[0].max(), 1.0)


def test_adam_first_step_is_sign_times_lr():
    p = np.zeros(4)
    g = np.array([3.0, -2.0, 1e-3, 0.0])
    p2, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, 0.1)
    # after one bias-corrected step the update is lr * g / (|g| + eps)
    assert np.allclose(p2[:3], -0.1 * np.sign(g[:3]), rtol=1e-4) and p2[3] == 0.0


def test_top_directions_ties_and_nan():
    s = np.zeros((1, 64))
    s[0, [5, 9, 40]] = 2.0
    s[0, 7] = np.nan
    s[0, 63] = 3.0
    top = mlp.top_directions(s)[0]
    assert list(top[:4]) == [63, 5, 9, 40]
    assert list(top[4:]) == [0, 1, 2, 3]


def test_top_directions_gap_hand_case():
    """Scores peaking at direction 10 (score -|d - 10|): without a gap the
    picks walk outwards from the peak; with gap 2 every pick rules out its
    two neighbours on each side."""
    sc = -np.abs(np.arange(64) - 10).astype(np.float32)[None, :]
    assert list(mlp.top_directions(sc)[0]) == [10, 9, 11, 8, 12, 7, 13, 6]
    assert list(mlp.top_directions(sc, gap=2)[0]) == [10, 7, 13, 4, 16, 1, 19, 22]
    # wrap-around: the peak at 0 rules out 62, 63, 1, 2
    sc = -np.minimum(np.arange(64), 64 - np.arange(64)).astype(np.float32)[None, :]
    assert list(mlp.top_directions(sc, gap=2)[0]) == [0, 3, 61, 6, 58, 9, 55, 12]
