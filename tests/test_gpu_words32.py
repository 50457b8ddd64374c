"""Streams of 32-bit words on the GPU (pcomp_compress32 / pcomp_decompress32) against the
oracle's, byte for byte, through the C ABI (MI355X)."""
import numpy as np
import pytest
import torch

import datagen
from streamfmt import parse, tile_parts

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


def _to_torch(x: np.ndarray) -> torch.Tensor:
    if x.dtype == np.uint16:
        return torch.from_numpy(x.view(np.int16).copy()).view(torch.uint16)
    if x.dtype == np.uint32:
        return torch.from_numpy(x.view(np.int32).copy()).view(torch.uint32)
    return torch.from_numpy(x.copy())


def _check(pc, orc, x: np.ndarray, L: int, variant: int, what: str):
    print("case:", what, "n=%d L=%d variant=%d dtype=%s" % (x.size, L, variant, x.dtype), flush=True)
    xd = _to_torch(x).cuda()
    s = pc.compress32(xd, L, variant)
    got = s.cpu().numpy().tobytes()
    want = orc.compress32(x, L, variant)
    if got != want:
        a, b = np.frombuffer(got, np.uint8), np.frombuffer(want, np.uint8)
        m = min(a.size, b.size)
        bad = np.nonzero(a[:m] != b[:m])[0]
        raise AssertionError("%s: stream differs: len %d vs %d, first diff at %s" % (
            what, a.size, b.size, bad[:5] if bad.size else "length"))
    assert np.array_equal(_as_np(pc.decompress32(s)), x), what + ": GPU round trip"
    s2 = torch.from_numpy(np.frombuffer(want, np.uint8).copy()).cuda()
    assert np.array_equal(_as_np(pc.decompress32(s2)), x), what + ": GPU decode of the oracle's stream"


def _sample(rng, dtype, n, spread):
    bits = np.dtype(dtype).itemsize * 8
    x = rng.normal(1 << (bits - 1), spread, n).clip(0, (1 << bits) - 1).astype(dtype)
    if n:
        x[rng.integers(0, n, 5)] = rng.integers(0, 1 << bits, 5, dtype=np.uint64).astype(dtype)
    return x


@pytest.mark.parametrize("variant", [0, 8, EXH])
@pytest.mark.parametrize("dtype,L,n", [(np.uint8, 64, 70001), (np.uint16, 40, 123457), (np.uint16, 7, 9999),
                                       (np.uint16, 1000, 77777), (np.uint16, 8192, 40000), (np.uint8, 1, 3000),
                                       (np.uint8, 16384, 50000)])
def test_words32_parity(pc, orc, variant, dtype, L, n):
    rng = np.random.default_rng(L + variant)
    for spread in (2.0, 60.0, 5000.0):
        _check(pc, orc, _sample(rng, dtype, n, spread), L, variant, "gauss %.0f" % spread)


@pytest.mark.parametrize("variant", [0, 8, EXH])
def test_words32_camera(pc, orc, variant):
    x = _as_np(datagen.camera_events(6, seed=21))
    _check(pc, orc, x, 40, variant, "camera")


def test_words32_u32_basic(pc, orc):
    rng = np.random.default_rng(4)
    for spread in (10.0, 1e5, 1e9):
        _check(pc, orc, _sample(rng, np.uint32, 50003, spread), 256, 0, "u32 %.0g" % spread)
    x = np.zeros(4096, dtype=np.uint32)
    x[::2] = 0xFFFFFFFF  # B = 2^32: one digit per word
    _check(pc, orc, x, 128, 0, "u32 full range")


def test_words32_every_u16_base(pc, orc):
    # one block per base B = 1 .. 65536 (min 0, max B - 1): every table entry of both packings
    L = 64
    rng = np.random.default_rng(6)
    x = rng.integers(0, 1 << 16, (65536, L), dtype=np.uint64)
    B = np.arange(1, 65537, dtype=np.uint64)
    x = (x % B[:, None]).astype(np.uint16)
    x[:, 0] = 0
    x[:, 1] = (B - 1).astype(np.uint16)
    x = x.reshape(-1)
    for v in (0, 8):
        _check(pc, orc, x, L, v, "every u16 base")


def test_words32_constant_blocks_and_empty(pc, orc):
    x = np.full(10000, 777, dtype=np.uint16)
    x[5000:5100] = 0
    for v in (0, 8, EXH):
        _check(pc, orc, x, 100, v, "constant")
    e = torch.zeros(0, dtype=torch.uint8, device="cuda")
    s = pc.compress32(e, 16, 8)
    assert s.cpu().numpy().tobytes() == orc.compress32(np.zeros(0, np.uint8), 16, 8)
    assert pc.decompress32(s).numel() <= 1


def test_words32_errors(pc, orc):
    rng = np.random.default_rng(7)
    x = _sample(rng, np.uint16, 50000, 30.0)  # 1250 blocks, 10 tiles
    xd = _to_torch(x).cuda()
    s32 = pc.compress32(xd, 40, 8)
    s64 = pc.compress(xd, 40, 8)
    out = torch.empty(50000, dtype=torch.uint16, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")

    def status32(stream, L=40, o=out):
        pc.decompress32_into(stream, o, st, L)
        return int(st.item())

    assert status32(s32) == 0
    assert status32(s64) == pc.ECORRUPT  # a stream of 64-bit words
    pc.decompress_into(s32, out, st, dtype_bytes=2, block_len=40)
    assert int(st.item()) == pc.ECORRUPT  # and the other way round
    assert status32(s32, L=41) == pc.ECORRUPT  # another block length
    assert status32(s32[:-4]) == pc.ECORRUPT  # truncated
    assert status32(s32, o=out[:49999]) == pc.ENOSPC
    bad = s32.clone()
    meta = parse(s32.cpu().numpy())
    bad[meta["off"]["index"] + 8] += 1  # tile 1 starts one word late
    assert status32(bad) == pc.ECORRUPT
    with pytest.raises(pc.PcompError):
        pc.compress32(_to_torch(x.astype(np.uint32)).cuda(), 40, 8)  # advanced needs u8 / u16
    with pytest.raises(pc.PcompError):
        pc.compress32(xd, 40, 3)


def test_words32_camera_full_size_sampled_tiles(pc, orc):
    L = 40
    x = datagen.camera_events(10000, seed=1, device="cuda").reshape(-1)
    print("case: camera 10000 events, 32-bit words, exhaustive", flush=True)
    c = pc.Compressor32(x.numel(), torch.uint16, L, EXH)
    c(x)
    s = c.stream()
    out = torch.empty_like(x)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pc.decompress32_into(s, out, st, L)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert torch.equal(out.view(torch.int16), x.view(torch.int16))
    del out
    host = s.cpu().numpy()
    meta = parse(host)
    nt, tb = meta["ntiles"], meta["tb"]
    rng = np.random.default_rng(18)
    picks = sorted(set([0, nt - 1] + rng.integers(0, nt, 10).tolist()))
    for t in picks:
        v0, v1 = t * tb * L, min(x.numel(), (t + 1) * tb * L)
        want = np.frombuffer(orc.compress32(_as_np(x[v0:v1]), L, EXH), np.uint8)
        assert tile_parts(host, meta, t) == tile_parts(want, parse(want), 0), "tile %d differs from the oracle" % t
