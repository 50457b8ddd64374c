"""Full-size workloads on the GPU, in the launch configuration bench.py times.

Camera waveforms (10,000 events x 1855 pixels x 40 samples u16, block = one trace): compressed by
the single-call path, round-tripped exactly, and sampled tiles equal the oracle's stream of the
same blocks byte for byte (block arrays and payload).

Uneven events (50,000 events of shapes 1855x40, 2048x96, 11328x128, u16/u32, ~86 GB): one batch
compressed from a captured HIP graph, with exhaustive search and with the shipped learned
selector; sampled segments' streams equal the oracle's, and decompression restores every segment
(a 64-bit weighted sum of each segment's bytes is compared, since a second full copy of the data
would not fit beside the input and the streams; sampled segments are compared exactly)."""
import numpy as np
import pytest
import torch

import datagen
from streamfmt import parse, tile_parts

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


@pytest.mark.parametrize("variant", [EXH, 0])
def test_camera_full_size_sampled_tiles(pc, orc, variant):
    L = 40
    x = datagen.camera_events(10000, seed=1, device="cuda").reshape(-1)  # the benchmark's input
    print("case: camera 10000 events, variant %#x, %.3f GB" % (variant, x.numel() * 2 / 1e9), flush=True)
    c = pc.Compressor(x.numel(), torch.uint16, L, variant)
    c(x)
    st = c.stream()
    out = torch.empty_like(x)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    pc.decompress_into(st, out, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert torch.equal(out.view(torch.int16), x.view(torch.int16))
    del out
    host = st.cpu().numpy()
    meta = parse(host)
    nt = meta["ntiles"]
    rng = np.random.default_rng(17)
    picks = sorted(set([0, nt - 1] + rng.integers(0, nt, 10).tolist()))
    tb = meta["tb"]
    for t in picks:
        v0, v1 = t * tb * L, min(x.numel(), (t + 1) * tb * L)
        want = np.frombuffer(orc.compress(_as_np(x[v0:v1]), L, variant), np.uint8)
        assert tile_parts(host, meta, t) == tile_parts(want, parse(want), 0), "tile %d differs from the oracle" % t
    print("tiles sampled: %d of %d" % (len(picks), nt), flush=True)


def _weighted_sums(segs, weights):
    """Per segment: sum of byte_i * w_i in wrapping 64-bit arithmetic (w: fixed random words)."""
    return torch.stack([(s.view(torch.uint8).to(torch.int64) * weights[:s.numel() * s.element_size()]).sum()
                        for s in segs])


def test_uneven_events_full_size_batch(pc, orc):
    from paper_1805_01844_amd import learn

    segs = [e.reshape(-1) for e in datagen.uneven_events(50000, seed=3, device="cuda")]
    torch.cuda.synchronize()
    raw = sum(s.numel() * s.element_size() for s in segs)
    print("case: uneven events, %d segments, %.3f GB" % (len(segs), raw / 1e9), flush=True)
    longest = max(s.numel() * s.element_size() for s in segs)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    weights = torch.randint(-(1 << 62), 1 << 62, (longest,), generator=g, device="cuda", dtype=torch.int64)
    ref = _weighted_sums(segs, weights)
    rng = np.random.default_rng(23)
    picks = sorted(rng.choice(len(segs), 8, replace=False).tolist())
    keep = {i: segs[i].clone() for i in picks}
    group = {1: 0, 2: 1, 4: 2}
    try:
        for variant, Ls in ((EXH, (1024, 1024, 512)), (LEARNED, (1024, 1024, 1024))):
            if variant == LEARNED:
                orc.set_model(learn.use_selector().numpy())
            b = pc.Batch(segs, block_len=Ls, variant=variant)
            graph = b.capture()
            graph.replay()
            torch.cuda.synchronize()
            assert b.error_flag() == 0
            streams = b.streams()
            print("variant %#x: ratio %.4f" % (variant, raw / b.total_bytes()), flush=True)
            for i in picks:
                L = Ls[group[keep[i].element_size()]]
                want = orc.compress(_as_np(keep[i]), L, variant)
                assert streams[i].cpu().numpy().tobytes() == want, "segment %d differs from the oracle" % i
            del streams
            for s in segs:
                s.view(torch.uint8).fill_(0x5A)  # decoded values must replace every byte
            dec = pc.BatchDecoder(b, segs)
            dec()
            dec.check()
            assert torch.equal(_weighted_sums(segs, weights), ref), "a segment did not round-trip"
            for i in picks:
                assert torch.equal(segs[i].view(torch.uint8), keep[i].view(torch.uint8))
            del graph, b, dec
            torch.cuda.empty_cache()
    finally:
        pc.set_model(None)
        orc.set_model(None)
