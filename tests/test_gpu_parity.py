"""GPU path vs the CPU oracle, byte for byte, through the C ABI (MI355X)."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu

EXH = 0x100
ALL_VARIANTS = list(range(16)) + [EXH]


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


def _check(pc, orc, x: torch.Tensor, L: int, variant: int, what: str):
    print("case:", what, "n=%d L=%d variant=%d dtype=%s" % (x.numel(), L, variant, x.dtype), flush=True)
    xd = x.reshape(-1).cuda()
    s = pc.compress(xd, L, variant)
    got = s.cpu().numpy().tobytes()
    want = orc.compress(_as_np(x), L, variant)
    if got != want:
        a = np.frombuffer(got, np.uint8)
        b = np.frombuffer(want, np.uint8)
        m = min(a.size, b.size)
        bad = np.nonzero(a[:m] != b[:m])[0]
        raise AssertionError("%s: stream differs: len %d vs %d, first diff at %s" % (
            what, a.size, b.size, bad[:5] if bad.size else "length"))
    y = pc.decompress(s)
    assert np.array_equal(_as_np(y), _as_np(x)), what + ": GPU round trip"
    # the GPU decoder also reads the oracle's stream
    s2 = torch.from_numpy(np.frombuffer(want, np.uint8).copy()).cuda()
    assert np.array_equal(_as_np(pc.decompress(s2)), _as_np(x)), what + ": GPU decode of oracle stream"


def test_tiny_gaussian_basic_and_advanced(pc, orc):
    x = datagen.tiny_gaussian()
    for v in (0, 8, EXH):
        _check(pc, orc, x, 1024, v, "tiny_gaussian")


@pytest.mark.parametrize("variant", ALL_VARIANTS)
def test_camera_events_every_variant(pc, orc, variant):
    x = datagen.camera_events(6, seed=21)  # 11130 traces of 40 samples, ragged last tile
    _check(pc, orc, x, 40, variant, "camera")


@pytest.mark.parametrize("dtype", [torch.uint8, torch.uint16, torch.uint32])
@pytest.mark.parametrize("variant", [0, 8, 2, 13, EXH])
def test_laplace_outliers_constant_fullrange(pc, orc, dtype, variant):
    x = datagen.laplace_blocks(300, 1024, dtype, seed=31, const_rate=0.05, full_rate=0.05, outlier_rate=2e-3)
    _check(pc, orc, x, 1024, variant, "laplace")


@pytest.mark.parametrize("L", [1, 2, 7, 13, 255, 256, 1000, 4096])
def test_ragged_block_lengths(pc, orc, L):
    x = datagen.camera_events(1, seed=L).reshape(-1)[: 3 * 4096 + 11]
    for v in (0, 8, 5, 12, EXH):
        _check(pc, orc, x, L, v, "ragged")


def test_max_block_length_per_dtype(pc, orc):
    for dt, L in [(torch.uint8, 16384), (torch.uint16, 8192), (torch.uint32, 4096)]:
        x = datagen.laplace_blocks(3, L, dt, seed=41).reshape(-1)[: 3 * L - 5]
        for v in (0, 8, EXH):
            _check(pc, orc, x, L, v, "maxL")


def test_empty_and_single(pc, orc):
    for v in (0, 8, EXH):
        _check(pc, orc, torch.zeros(1, dtype=torch.uint16), 40, v, "single")
        xd = torch.zeros(0, dtype=torch.uint16, device="cuda")
        s = pc.compress(xd, 40, v)
        assert s.cpu().numpy().tobytes() == orc.compress(np.zeros(0, np.uint16), 40, v)
        assert pc.decompress(s).numel() == 0


def test_base_sweep_u32_every_base_to_2_16(pc, orc):
    x = datagen.base_sweep_u32(L=256, lo=2, hi=1 << 16)
    for v in (0, 8):
        _check(pc, orc, x, 256, v, "base_sweep")


def test_wide_u32_bases_outside_tables(pc, orc):
    g = torch.Generator().manual_seed(5)
    x = torch.randint(0, 1 << 31, (64 * 512,), generator=g, dtype=torch.int64)
    x[::512] = 0
    x = x.to(torch.uint32)
    for v in (0, 8, 9, 15, EXH):
        _check(pc, orc, x, 512, v, "wide_u32")


def _series_span(B: int) -> int:
    """mu + lam of the carried base of the Sec. 3.2 series of base B with 64-bit words (words
    before the period plus its length), walked here in Python integers."""
    k = 1
    while B ** (k + 1) <= 1 << 64:
        k += 1
    Q = [(1 << 64) // B ** p for p in range(k + 1)]
    s, seen = 1, {}
    while s not in seen:
        seen[s] = len(seen)
        p = k if s <= Q[k] else k - 1
        R = Q[p] // s
        s = 1 if R >= B else -(-B // R)
    return len(seen)


@pytest.mark.parametrize("L", [128, 256, 512, 1024, 2048, 4096])
def test_u32_series_periods_outside_tables(pc, orc, L):
    # u32 blocks of bases outside the tables whose series repeat after 1 .. 250 words: lane
    # groups of 8 to 256 lanes hold the period in their registers when it fits, and walk the
    # series lane by lane when it does not; the last block is ragged
    rng = np.random.default_rng(L)
    spans = {}
    while len(spans) < 24:
        B = int(rng.integers((1 << 16) + 2, (1 << 32) + 1))
        m = _series_span(B)
        bucket = min(m.bit_length(), 8)
        if sum(1 for v in spans.values() if v == bucket) < 4:
            spans[B] = bucket
    bases = list(spans)
    nblk = max(24, 40000 // L)
    x = np.empty(nblk * L, np.uint32)
    for b in range(nblk):
        B = bases[b % len(bases)]
        lo = int(rng.integers(0, (1 << 32) - B + 1))
        v = rng.integers(0, B, L, dtype=np.uint64)
        v[rng.integers(0, L)] = 0
        v[rng.integers(0, L)] = B - 1
        x[b * L:(b + 1) * L] = (v + lo).astype(np.uint32)
    x = torch.from_numpy(x[: nblk * L - 7].view(np.int32)).view(torch.uint32)
    for v in (8, 9, 12, EXH):
        _check(pc, orc, x, L, v, "u32_periods")


def test_misaligned_input(pc, orc):
    base = datagen.camera_events(1, seed=9).reshape(-1).cuda()
    for off in (1, 3, 5):
        x = base[off: off + 5000]  # not 16-byte aligned
        s = pc.compress(x, 40, EXH)
        assert s.cpu().numpy().tobytes() == orc.compress(_as_np(x), 40, EXH)


def test_deterministic(pc):
    x = datagen.camera_events(4, seed=2).reshape(-1).cuda()
    a = pc.compress(x, 40, EXH).cpu()
    b = pc.compress(x, 40, EXH).cpu()
    assert torch.equal(a, b)


def test_corrupt_stream_sets_status(pc, orc):
    x = datagen.camera_events(1, seed=3).reshape(-1)
    want = np.frombuffer(orc.compress(_as_np(x), 40, EXH), np.uint8).copy()
    bad = want.copy()
    bad[0] ^= 1
    with pytest.raises(pc.PcompError):
        pc.decompress(torch.from_numpy(bad).cuda())
    n, w, L, tot = pc.stream_info(torch.from_numpy(want))
    out = torch.empty(n, dtype=torch.uint16, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    bad = want.copy()
    nb = -(-n // L)
    nt = -(-nb // 128)
    bad[64 + 8 * nt + 4 * nb] = 77  # class byte of block 0 out of range
    pc.decompress_into(torch.from_numpy(bad).cuda(), out, st)
    assert int(st.item()) == pc.ECORRUPT
    pc.decompress_into(torch.from_numpy(want).cuda(), out[: n // 2], st)
    assert int(st.item()) == pc.ENOSPC


@pytest.mark.parametrize("variant", [6, 7, 14, 15, EXH])
def test_dense_excess_lists(pc, orc, variant):
    """Near-uniform data with high thresholds: most values are excess, so a tile's excess lists
    overflow the compaction buffer and packing reads them straight from the tile."""
    g = torch.Generator().manual_seed(77)
    for dt, hi, L in [(torch.uint16, 1 << 16, 1024), (torch.uint8, 256, 2048), (torch.uint32, 1 << 20, 512)]:
        x = torch.randint(0, hi, (7 * L + 13,), generator=g, dtype=torch.int64)
        x = x.to(torch.int32).to(dt) if dt != torch.uint8 else x.to(dt)
        _check(pc, orc, x, L, variant, "dense_excess")


def test_decompress_into_checks_the_output_dtype(pc):
    """The library counts the output capacity in values of the stream's dtype, so an output of
    another dtype is refused by the binding instead of being written past its end."""
    x = torch.arange(5000, dtype=torch.int32).to(torch.uint16).cuda()
    st = pc.compress(x, 40)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        pc.decompress_into(st, torch.empty(x.numel(), dtype=torch.uint8, device="cuda"), status)
    with pytest.raises(ValueError):
        pc.decompress_into(st, torch.empty(x.numel(), dtype=torch.uint8, device="cuda"), status, dtype_bytes=2)
    out = torch.empty_like(x)
    pc.decompress_into(st, out, status)
    assert int(status.item()) == 0 and torch.equal(out.view(torch.int16), x.view(torch.int16))
    with pytest.raises(ValueError):
        pc.mlp_scores(torch.zeros(pc.MLP_PARAMS, device="cuda"), torch.zeros(4, pc.MLP_IN - 1, device="cuda"))
