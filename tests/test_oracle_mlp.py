"""Pins of the oracle's learned-selector pieces (no GPU): block features against values the
definition fixes, binary32 scores against an independent float64 evaluation, float64
gradients against finite differences, Adam's first step against its closed form, and the
selection rule against the forced-class path."""
import numpy as np
import pytest

from oracle import mlp

LEARNED = 0x200


def test_piecewise_log_features_exact_values(orc):
    # lg(u) = e + (u - 2^e) 2^-e: exact at powers of two and at their midpoints
    for vmin, want in [(0, 0.0), (1, 1.0), (2, 1.5), (3, 2.0), (5, 2.5), (1023, 10.0), (1535, 10.5),
                       ((1 << 32) - 1, 32.0)]:
        x = orc.block_features([0], vmin, vmin)
        assert x[16] == np.float32(want / 32), (vmin, x[16])
        assert x[17] == x[16]  # max == min here


def test_histogram_features_place_digits_by_octave(orc):
    # B - 1 = 100 -> beta = 7; digit d lands in bin 7 - bitlen(d) (capped at 15)
    d = [0, 1, 2, 3, 4, 64, 100, 63]
    x = orc.block_features(d, 1000, 1100)
    H = np.rint(x[:16] * len(d)).astype(int)
    assert list(H) == [2, 1, 0, 0, 1, 2, 1, 1] + [0] * 8
    assert x[18] == np.float32(len(d) / 4096)
    # the counts sum to the block length
    assert int(H.sum()) == len(d)


def test_histogram_caps_deep_octaves_and_constant_blocks(orc):
    # beta = 32: digits 0 and 1 are 32 and 31 octaves down -> both in bin 15
    x = orc.block_features([0, 1, (1 << 32) - 1], 0, (1 << 32) - 1)
    assert x[15] == np.float32(2 / 3) and x[0] == np.float32(1 / 3)
    # constant block: B = 1, every digit 0 and beta = 0 -> all in bin 0
    x = orc.block_features([0] * 7, 42, 42)
    assert x[0] == 1.0 and not np.any(x[1:16])


def test_array_features_match_block_features(orc):
    rng = np.random.default_rng(3)
    a = (rng.normal(300, 8, 5 * 40 + 7).round()).astype(np.uint16)
    F, W = orc.features(a, 40)
    assert F.shape == (6, 19) and W.shape == (6, 16)
    for b in range(6):
        blk = a[40 * b:40 * (b + 1)].astype(np.int64)
        x = orc.block_features(blk - blk.min(), int(blk.min()), int(blk.max()))
        assert np.array_equal(F[b], x)
        facts = orc.block_facts(blk.astype(np.uint16), 40, 0x100)
        ok = W[b] != np.iinfo(np.uint64).max
        assert W[b][int(facts["cls"][0])] == W[b][ok].min()  # exhaustive picks the smallest


def test_scores_match_float64_evaluation(orc):
    rng = np.random.default_rng(7)
    p = mlp.init_params(11)
    p[mlp.HID * mlp.IN:mlp.HID * mlp.IN + mlp.HID] = rng.normal(0, 0.1, mlp.HID)  # non-zero b1
    X = rng.random((50, 19)).astype(np.float32)
    s32 = orc.mlp_scores(p, X)
    s64, _ = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    scale = np.abs(s64).max()
    assert np.max(np.abs(s32 - s64)) <= 1e-5 * scale
    margin = np.sort(s64, axis=1)
    clear = margin[:, -1] - margin[:, -2] > 1e-4 * scale
    assert np.array_equal(orc.mlp_predict(p, X)[clear], np.argmax(s64, axis=1)[clear])


def test_scores_with_zero_weights_are_the_biases(orc):
    p = np.zeros(mlp.N_PARAMS, np.float32)
    p[-16:] = np.arange(16, dtype=np.float32) % 5  # max 4 first at k = 4
    X = np.random.default_rng(0).random((3, 19)).astype(np.float32)
    assert np.array_equal(orc.mlp_scores(p, X), np.tile(p[-16:], (3, 1)))
    assert list(orc.mlp_predict(p, X)) == [4, 4, 4]


def test_float64_gradients_match_finite_differences():
    rng = np.random.default_rng(5)
    p = mlp.init_params(3).astype(np.float64)
    p[mlp.HID * mlp.IN:mlp.HID * mlp.IN + mlp.HID] = rng.normal(0, 0.5, mlp.HID)
    X = rng.random((20, 19))
    y = rng.integers(0, 16, 20)
    L, g = mlp.loss_grad(p, X, y)
    assert abs(L - mlp.loss(p, X, y)) < 1e-12
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, y) - mlp.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (i, fd, g[i])


def test_adam_first_step_is_lr_times_sign():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    # m_hat = g, v_hat = g^2 -> step = lr g / (|g| + eps)
    assert np.allclose(p[:3], -0.01 * np.sign(g[:3]), rtol=1e-5) and p[3] == 0.0


def test_learned_selection_equals_forced_prediction(orc):
    rng = np.random.default_rng(9)
    x = np.clip(rng.laplace(30000, 40, 37 * 256), 0, 65535).astype(np.uint16)
    x[::97] = rng.integers(0, 65536, x[::97].size)
    nb = (x.size + 255) // 256
    for c in (0, 3, 9, 13):
        p = np.zeros(mlp.N_PARAMS, np.float32)
        p[-16 + c] = 1.0  # every block predicts class c
        orc.set_model(p)
        try:
            got = orc.compress(x, 256, LEARNED)
        finally:
            orc.set_model(None)
        assert got == orc.compress(x, 256, LEARNED, forced=np.full(nb, c, np.uint8))
        facts = orc.block_facts(x, 256, LEARNED, forced=np.full(nb, c, np.uint8))
        base = orc.block_facts(x, 256, 0)
        assert np.all(facts["words"] <= base["words"])  # never larger than class 0
        assert set(np.unique(facts["cls"])) <= {0, c}
        assert np.array_equal(orc.decompress(got), x)


def test_learned_needs_a_model(orc):
    orc.set_model(None)
    with pytest.raises(ValueError):
        orc.compress(np.zeros(10, np.uint16), 4, LEARNED)
