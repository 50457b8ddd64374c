"""Stream-level checks of the oracle: layout, round trips on every config shape, bounds, errors."""
import struct

import numpy as np
import pytest
import torch

import datagen

VARIANTS = [0, 8, 1, 4, 9, 12, 0x100]


def _hdr(s):
    magic, ver, w, flags, fixed, sel, _r, L, n, nb, tb, _r2, pw, tot, _r3 = struct.unpack_from(
        "<IHBBBBHIQQIIQQQ", s, 0)
    return dict(magic=magic, ver=ver, w=w, flags=flags, fixed=fixed, sel=sel, L=L, n=n, nb=nb, tb=tb, pw=pw,
                tot=tot)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype,L", [(np.uint8, 1024), (np.uint16, 40), (np.uint16, 1000), (np.uint32, 256)])
def test_round_trip_and_header(orc, variant, dtype, L):
    rng = np.random.default_rng(L + variant)
    bits = np.dtype(dtype).itemsize * 8
    n = 37 * L + 17  # ragged last block
    x = (rng.normal(1 << (bits - 1), 20, n)).clip(0, (1 << bits) - 1).astype(dtype)
    x[rng.integers(0, n, 5)] = rng.integers(0, 1 << bits, 5, dtype=np.uint64).astype(dtype)
    s = orc.compress(x, L, variant)
    h = _hdr(s)
    assert h["magic"] == 0x504D4350 and h["ver"] == 1 and h["w"] == x.itemsize
    assert h["L"] == L and h["n"] == n and h["nb"] == -(-n // L) and h["tot"] == len(s)
    assert h["tb"] == orc.tile_blocks(L, x.itemsize)
    assert len(s) <= orc.bound(n, x.itemsize, L, variant)
    assert len(s) % 8 == 0
    assert np.array_equal(orc.decompress(s), x)
    facts = orc.block_facts(x, L, variant)
    assert h["pw"] == int(facts["words"].sum())
    if variant in (0, 8):
        assert h["flags"] == 0 and h["fixed"] == variant
        assert (facts["cls"] == variant).all()
    else:
        assert h["flags"] & 3 == 3


def test_index_points_at_tile_starts(orc):
    x = datagen.camera_events(2, seed=4).numpy().reshape(-1)
    L = 40
    s = orc.compress(x, L, 0x100)
    h = _hdr(s)
    facts = orc.block_facts(x, L, 0x100)
    offs = np.concatenate([[0], np.cumsum(facts["words"].astype(np.int64))])
    nt = -(-h["nb"] // h["tb"])
    idx = np.frombuffer(s, dtype=np.uint64, count=nt, offset=64)
    assert np.array_equal(idx.astype(np.int64), offs[np.arange(nt) * h["tb"]])


def test_exhaustive_never_larger_than_any_fixed_class(orc):
    x = datagen.camera_events(1, seed=5).numpy().reshape(-1)
    L = 40
    ex = orc.block_facts(x, L, 0x100)["words"]
    for v in range(16):
        f = orc.block_facts(x, L, v)["words"]
        assert (ex <= f).all()
    # and never larger than plain basic t=0, the bound's assumption
    assert (ex <= orc.block_facts(x, L, 0)["words"]).all()


def test_constant_and_full_range_blocks(orc):
    for dt, maxv in [(np.uint8, 255), (np.uint16, 65535), (np.uint32, (1 << 32) - 1)]:
        L = 64
        x = np.zeros(4 * L, dtype=dt)
        x[:L] = 77  # constant block: B = 1, no payload
        x[L:2 * L] = np.arange(L) % 2 * maxv  # full range: no packing gain
        x[2 * L] = maxv
        for v in (0, 8, 0x100):
            f = orc.block_facts(x, L, v)
            assert int(f["B"][0]) == 1 and int(f["words"][0]) == 0
            assert int(f["B"][1]) == maxv + 1
            full = L // (64 // (8 * x.itemsize))
            if v in (0, 8):
                assert int(f["words"][1]) == full  # B = 2^w: no packing gain for t = 0
            else:
                assert int(f["words"][1]) <= full
            assert np.array_equal(orc.decompress(orc.compress(x, L, v)), x)


def test_empty_and_single_value(orc):
    for v in VARIANTS:
        s = orc.compress(np.zeros(0, np.uint16), 40, v)
        assert len(s) == 64 and orc.decompress(s).size == 0
        x = np.array([12345], dtype=np.uint16)
        assert np.array_equal(orc.decompress(orc.compress(x, 40, v)), x)


def test_learned_selector_clamps_and_round_trips(orc):
    x = datagen.camera_events(1, seed=6).numpy().reshape(-1)
    L = 40
    nb = -(-x.size // L)
    rng = np.random.default_rng(0)
    forced = rng.integers(0, 16, nb).astype(np.uint8)
    s = orc.compress(x, L, 0x200, forced=forced)
    assert np.array_equal(orc.decompress(s), x)
    f = orc.block_facts(x, L, 0x200, forced=forced)
    base = orc.block_facts(x, L, 0)["words"]
    ex = orc.block_facts(x, L, 0x100)["words"]
    assert (f["words"] <= base).all() and (f["words"] >= ex).all()
    kept = f["cls"] == forced
    assert ((f["cls"] == 0) | kept).all()


def test_error_paths(orc):
    x = np.arange(1000, dtype=np.uint16)
    s = bytearray(orc.compress(x, 40, 0x100))
    rc, _ = orc.decompress_rc(bytes(s[:40]))
    assert rc == -3  # truncated header
    bad = bytearray(s)
    bad[0] ^= 1
    assert orc.decompress_rc(bytes(bad))[0] == -3  # magic
    bad = bytearray(s)
    bad[4] = 9
    assert orc.decompress_rc(bytes(bad))[0] == -3  # version
    assert orc.decompress_rc(bytes(s[:-8]))[0] == -3  # payload cut
    # class byte out of range
    h = _hdr(bytes(s))
    nt = -(-h["nb"] // h["tb"])
    off_class = 64 + 8 * nt + 2 * 2 * h["nb"]
    bad = bytearray(s)
    bad[off_class] = 99
    assert orc.decompress_rc(bytes(bad))[0] == -3
    assert orc.decompress_rc(bytes(s), out_cap=10)[0] == -2
    assert orc.bound(10, 3, 40, 0) == 0 and orc.bound(10, 2, 0, 0) == 0 and orc.bound(10, 2, 40, 77) == 0


def test_deterministic(orc):
    x = datagen.tiny_gaussian(1 << 16).numpy()
    assert orc.compress(x, 1024, 0x100) == orc.compress(x, 1024, 0x100)


def test_tiny_config_ratio(orc):
    # 2^20 values of round(N(300, 4^2)) in blocks of 1024: B around 22..37, k = 13, ratio about 3.2
    x = datagen.tiny_gaussian().numpy()
    s = orc.compress(x, 1024, 0)
    r = x.nbytes / len(s)
    assert 3.1 < r < 3.3
    f = orc.block_facts(x, 1024, 0)
    assert 20 <= int(f["B"].min()) and int(f["B"].max()) <= 45
