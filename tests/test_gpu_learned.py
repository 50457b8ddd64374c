"""Learned class selector on the GPU: features, scores and streams bit-exact to the oracle;
gradients and Adam against the float64 reference; training lowers the loss; the shipped
network gains over the plain method and never beats exhaustive search."""
import os

import numpy as np
import pytest
import torch

import datagen
from oracle import mlp

pytestmark = pytest.mark.gpu

EXH, LEARNED = 0x100, 0x200


@pytest.fixture(scope="module")
def pc():
    import paper_1805_01844_amd as pc

    pc.init()
    return pc


def _as_np(x: torch.Tensor) -> np.ndarray:
    x = x.cpu().reshape(-1)
    if x.dtype == torch.uint16:
        return x.view(torch.int16).numpy().view(np.uint16)
    if x.dtype == torch.uint32:
        return x.view(torch.int32).numpy().view(np.uint32)
    return x.numpy()


def _cases():
    return [
        ("camera", datagen.camera_events(3, seed=61).reshape(-1), 40),
        ("laplace_u8", datagen.laplace_blocks(40, 1024, torch.uint8, seed=62, const_rate=0.1, full_rate=0.1)
         .reshape(-1)[:40 * 1024 - 3], 1024),
        ("laplace_u16", datagen.laplace_blocks(60, 512, torch.uint16, seed=63).reshape(-1), 512),
        ("laplace_u32", datagen.laplace_blocks(30, 256, torch.uint32, seed=64, outlier_rate=0.02).reshape(-1), 256),
        ("event_u32", datagen.uneven_events(2, seed=65, shapes=[(300, 96)])[1].reshape(-1), 4096),
    ]


def _random_params(seed):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed)
    p[mlp.HID * mlp.IN:mlp.HID * mlp.IN + mlp.HID] = rng.normal(0, 0.2, mlp.HID)
    p[-16:] = rng.normal(0, 0.5, 16)
    return p.astype(np.float32)


def test_features_labels_and_sizes_bit_exact(pc, orc):
    for name, x, L in _cases():
        print("case:", name, "n=%d L=%d" % (x.numel(), L), flush=True)
        fx, words, lab = pc.block_features(x.cuda(), L)
        F, W = orc.features(_as_np(x), L)
        assert np.array_equal(fx.cpu().numpy().view(np.uint32), F.view(np.uint32)), name + ": features"
        Wg = words.cpu().numpy().view(np.uint32).astype(np.uint64)
        Wg[Wg == 0xFFFFFFFF] = np.iinfo(np.uint64).max
        assert np.array_equal(Wg, W), name + ": class sizes"
        cls = orc.block_facts(_as_np(x), L, EXH)["cls"]
        assert np.array_equal(lab.cpu().numpy(), cls), name + ": exhaustive labels"


def test_scores_bit_exact(pc, orc):
    x = datagen.uneven_events(3, seed=66, shapes=[(500, 40), (200, 128)])
    fx = torch.cat([pc.block_features(e.reshape(-1).cuda(), 256)[0] for e in x])
    for seed in (1, 2):
        p = _random_params(seed)
        got = pc.mlp_scores(torch.from_numpy(p).cuda(), fx).cpu().numpy()
        want = orc.mlp_scores(p, fx.cpu().numpy())
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("seed", [3, 4])
def test_learned_streams_match_oracle(pc, orc, seed):
    p = _random_params(seed)
    pc.set_model(p)
    orc.set_model(p)
    try:
        seen = set()
        for name, x, L in _cases():
            print("case:", name, "seed", seed, flush=True)
            s = pc.compress(x.cuda(), L, LEARNED)
            want = orc.compress(_as_np(x), L, LEARNED)
            assert s.cpu().numpy().tobytes() == want, name
            assert np.array_equal(_as_np(pc.decompress(s)), _as_np(x)), name
            seen |= set(np.unique(orc.block_facts(_as_np(x), L, LEARNED)["cls"]).tolist())
        assert len(seen) > 1  # the network did choose classes other than 0
        # the same choice inside a batch
        segs = [x for _, x, _ in _cases()]
        b = pc.Batch([t.cuda() for t in segs], block_len=(1024, 512, 256), variant=LEARNED)
        b.compress()
        for t, st in zip(segs, b.streams()):
            L = (1024, 512, 256)[{1: 0, 2: 1, 4: 2}[t.element_size()]]
            assert st.cpu().numpy().tobytes() == orc.compress(_as_np(t), L, LEARNED)
    finally:
        pc.set_model(None)
        orc.set_model(None)


def test_learned_without_model_is_refused(pc):
    pc.set_model(None)
    with pytest.raises(pc.PcompError):
        pc.compress(torch.zeros(100, dtype=torch.uint16, device="cuda"), 40, LEARNED)


def _training_data(pc, seed, n_events=48):
    ev = datagen.uneven_events(n_events, seed=seed, shapes=[(300, 40), (200, 96), (400, 128)])
    from paper_1805_01844_amd import learn

    return learn.dataset([e.reshape(-1).cuda() for e in ev], lambda k, s: (256, 1024)[k % 2])


def test_gradients_match_float64_reference(pc):
    X, y, _ = _training_data(pc, 70, 6)
    n = min(3000, X.shape[0])
    X, y = X[:n].contiguous(), y[:n].contiguous()
    p = _random_params(5)
    tr = pc.MLPTrainer(torch.from_numpy(p).cuda(), n)
    tr.loss_grad(X, y)
    g = tr.grad.cpu().numpy().astype(np.float64)
    L64, g64 = mlp.loss_grad(p.astype(np.float64), X.cpu().numpy().astype(np.float64), y.cpu().numpy())
    assert abs(float(tr.loss.item()) - L64) <= 1e-5 * max(1.0, abs(L64))
    assert np.max(np.abs(g - g64)) <= 1e-4 * np.max(np.abs(g64))
    # deterministic: the same call gives the same bits
    g1 = tr.grad.clone()
    tr.loss_grad(X, y)
    assert torch.equal(g1.view(torch.int32), tr.grad.view(torch.int32))


def test_adam_step_matches_float64(pc):
    rng = np.random.default_rng(8)
    p = rng.normal(0, 1, pc.MLP_PARAMS).astype(np.float32)
    tr = pc.MLPTrainer(torch.from_numpy(p).cuda(), 256, lr=1e-2)
    m = rng.normal(0, 0.1, pc.MLP_PARAMS).astype(np.float32)
    v = rng.random(pc.MLP_PARAMS).astype(np.float32) * 0.01
    g = rng.normal(0, 0.1, pc.MLP_PARAMS).astype(np.float32)
    tr.m.copy_(torch.from_numpy(m))
    tr.v.copy_(torch.from_numpy(v))
    tr.grad.copy_(torch.from_numpy(g))
    tr.step_no = 4
    rc = pc.lib().pcomp_mlp_adam(pc._vp(tr.params), pc._vp(tr.grad), pc._vp(tr.m), pc._vp(tr.v), 5, 1e-2, 0.9,
                                 0.999, 1e-8, pc._stream_handle())
    assert rc == 0
    want, wm, wv = mlp.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                                 v.astype(np.float64), 5, 1e-2)
    assert np.allclose(tr.params.cpu().numpy(), want, rtol=1e-5, atol=1e-6)
    assert np.allclose(tr.m.cpu().numpy(), wm, rtol=1e-5, atol=1e-7)


def test_training_lowers_loss_and_gains_over_plain(pc):
    from paper_1805_01844_amd import learn

    X, y, W = _training_data(pc, 71)
    params, hist = learn.train(X, y, epochs=25, batch=256, lr=3e-3, seed=1)
    print("losses", hist[0], hist[-1], flush=True)
    assert hist[-1] < 0.7 * hist[0]
    Xt, yt, Wt = _training_data(pc, 72)
    r = learn.payload_words(params, Xt, yt, Wt)
    print(r, flush=True)
    assert r["exhaustive"] <= r["learned"] <= r["plain"]
    assert r["learned"] < r["plain"]


def test_shipped_selector_gains_over_plain(pc, orc):
    from paper_1805_01844_amd import learn

    if not os.path.exists(learn.MODEL_PATH):
        pytest.skip("no trained selector shipped")
    p = learn.use_selector()
    orc.set_model(p.numpy())
    try:
        ev = datagen.uneven_events(6, seed=73, shapes=[(1855, 40), (2048, 96)])
        tot = {0: 0, LEARNED: 0, EXH: 0}
        raw = 0
        for e in ev:
            x = e.reshape(-1)
            raw += x.numel() * x.element_size()
            for v in tot:
                s = pc.compress(x.cuda(), 1024, v)
                tot[v] += s.numel()
                if v == LEARNED:
                    assert s.cpu().numpy().tobytes() == orc.compress(_as_np(x), 1024, LEARNED)
        print({v: raw / t for v, t in tot.items()}, flush=True)
        assert tot[EXH] <= tot[LEARNED] < tot[0]
    finally:
        pc.set_model(None)
        orc.set_model(None)
