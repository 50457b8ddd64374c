"""Batches on the GPU: every segment's stream equals the oracle's stream of that segment
alone; the batch decoder restores every segment; a captured graph replays correctly."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

EXH = 0x100


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


def _mixed_segments(seed: int):
    """Uneven camera events (scaled-down shapes), plus u8 stress blocks, empty and one-value
    segments, in an interleaved order."""
    ev = datagen.uneven_events(7, seed=seed, shapes=[(185, 40), (64, 96), (113, 128)])
    segs = [e.reshape(-1) for e in ev]
    segs.insert(2, torch.zeros(0, dtype=torch.uint16))
    segs.insert(4, datagen.laplace_blocks(9, 300, torch.uint8, seed=seed + 1).reshape(-1)[:2653])
    segs.insert(5, torch.tensor([7], dtype=torch.int32).to(torch.uint32))
    segs.append(datagen.laplace_blocks(5, 1000, torch.uint32, seed=seed + 2, full_rate=0.3).reshape(-1))
    segs.append(torch.zeros(0, dtype=torch.uint8))
    return segs


def _check_batch(pc, orc, segs, block_len, variant, grid, what):
    print("case:", what, "segments=%d L=%s variant=%d grid=%d" % (len(segs), block_len, variant, grid), flush=True)
    dev = [s.cuda() for s in segs]
    b = pc.Batch(dev, block_len=block_len, variant=variant, grid=grid)
    b.compress()
    streams = b.streams()
    Ls = pc._block_lens(block_len)
    wants = []
    for i, (x, s) in enumerate(zip(segs, streams)):
        L = Ls[{1: 0, 2: 1, 4: 2}[x.element_size()]]
        want = orc.compress(_as_np(x), L, variant)
        got = s.cpu().numpy().tobytes()
        assert got == want, "%s: segment %d (n=%d %s) stream differs (%d vs %d bytes)" % (
            what, i, x.numel(), x.dtype, len(got), len(want))
        wants.append(want)
    # the batch is one file: the oracle's streams back to back, in the segments' order
    assert b.file().cpu().numpy().tobytes() == b"".join(wants), "%s: batch file differs" % what
    offs = np.cumsum([0] + [len(w) for w in wants])[:-1].tolist()
    assert b.offsets() == offs, "%s: stream offsets" % what
    outs = [torch.empty_like(d) for d in dev]
    dec = pc.BatchDecoder(b, outs, grid=grid)
    dec()
    dec.check()
    for i, (x, o) in enumerate(zip(segs, outs)):
        assert np.array_equal(_as_np(o), _as_np(x)), "%s: segment %d round trip" % (what, i)
    return b


@pytest.mark.parametrize("variant", [0, 8, 3, 13, EXH])
def test_batch_matches_oracle_per_segment(pc, orc, variant):
    segs = _mixed_segments(11)
    _check_batch(pc, orc, segs, (300, 40, 1000), variant, 0, "batch")


@pytest.mark.parametrize("grid", [1, 7, 256])
def test_batch_persistent_grids(pc, orc, grid):
    segs = _mixed_segments(12)
    _check_batch(pc, orc, segs, (256, 512, 1024), EXH, grid, "persistent")


@pytest.mark.parametrize("L", [256, 512, 1024, 4096])
def test_batch_tuner_block_lengths(pc, orc, L):
    segs = _mixed_segments(13)
    _check_batch(pc, orc, segs, L, EXH, 0, "block length")


def test_batch_only_empty_segments(pc, orc):
    segs = [torch.zeros(0, dtype=torch.uint16), torch.zeros(0, dtype=torch.uint32)]
    _check_batch(pc, orc, segs, 1024, EXH, 0, "empty")


def test_batch_graph_replays(pc, orc):
    """Capture the batch once, then change the inputs in place between replays (with eager
    work and synchronisations in between); every replay must equal the oracle."""
    segs = _mixed_segments(14)
    dev = [s.cuda() for s in segs]
    b = pc.Batch(dev, block_len=(256, 512, 1024), variant=EXH, grid=0)
    g = b.capture()
    gen = torch.Generator(device="cpu")
    gen.manual_seed(5)
    for rep in range(3):
        print("case: graph replay", rep, flush=True)
        b.total.zero_()
        b.seg_offsets.fill_(-1)
        for d in dev:  # new values, same shapes, written eagerly
            if d.numel():
                hi = {1: 255, 2: 4000, 4: 1 << 20}[d.element_size()]
                vals = torch.randint(0, hi, (d.numel(),), generator=gen, dtype=torch.int64)
                d.copy_(vals.to(torch.int32).to(d.dtype) if d.dtype != torch.uint8 else vals.to(torch.uint8))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        streams = b.streams()
        wants = []
        for i, (d, s) in enumerate(zip(dev, streams)):
            L = (256, 512, 1024)[{1: 0, 2: 1, 4: 2}[d.element_size()]]
            want = orc.compress(_as_np(d), L, EXH)
            assert s.cpu().numpy().tobytes() == want, "replay %d segment %d" % (rep, i)
            wants.append(want)
        assert b.file().cpu().numpy().tobytes() == b"".join(wants), "replay %d: batch file" % rep


def test_batch_decoder_reports_corrupt_header(pc, orc):
    segs = _mixed_segments(15)[:4]
    dev = [s.cuda() for s in segs]
    b = pc.Batch(dev, block_len=1024, variant=0)
    b.compress()
    torch.cuda.synchronize()
    buf = b.out.clone()
    off = b.offsets()[1]
    buf[off + 16] ^= 1  # n of the second stream no longer matches the plan
    outs = [torch.empty_like(d) for d in dev]
    dec = pc.BatchDecoder(b, outs)
    dec(buf)
    assert int(dec.status.item()) == pc.ECORRUPT
    # an offset that is not a stream start (unaligned, or past the buffer) is reported too
    # (segment 0 has values, so its stream is read)
    for bad in (b.offsets()[0] + 4, b.out.numel() + 64):
        offs = b.seg_offsets.clone()
        offs[0] = bad
        dec(b.out, offs)
        assert int(dec.status.item()) == pc.ECORRUPT


def test_autotuner_picks_valid_configuration(pc, orc, tmp_path, monkeypatch):
    from paper_1805_01844_amd import tune

    monkeypatch.setenv("PCOMP_TUNE_CACHE", str(tmp_path / "tune.json"))
    segs = [e.reshape(-1).cuda() for e in datagen.uneven_events(12, seed=16, shapes=[(185, 40), (64, 96)])]
    res = tune.autotune(segs, EXH, reps=1, verbose=True)
    assert all(L in tune.CANDIDATE_L for L in res["block_len"]) and res["grid"] in tune.CANDIDATE_GRID
    assert tune.autotune(segs, EXH)["cached"]
    _check_batch(pc, orc, [s.cpu() for s in segs], res["block_len"], EXH, res["grid"], "tuned")
