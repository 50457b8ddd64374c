"""The oracle's streams of 32-bit words (the paper's unsigned int words, Sec. 3.1-3.2 with
capacity 2^32), pinned to an independent big-integer encoder and an independent stream writer.

The writer below follows the layout documented in include/pcomp.h (flags bit 3: 32-bit payload
words) and encodes every block with tests/bruteforce.py, which tries every exponent of the
Sec. 3.2 series and builds words as explicit power sums: no code is shared with the oracle."""
import struct

import numpy as np
import pytest

import bruteforce as bf

EXH = 0x100


def _k32(B):
    return bf.k_of(B, 32)


# --- family level: 32-bit words against the big-integer reference ------------------------

@pytest.mark.parametrize("family", [0, 1])
def test_family_words32_equal_bigint_reference(orc, family):
    rng = np.random.default_rng(30 + family)
    bases = list(range(2, 1500)) + [int(b) for b in rng.integers(1500, 65538, 300)] + [65535, 65536, 65537]
    if family == 0:
        bases += [int(b) for b in rng.integers(65538, 1 << 32, 100)] + [(1 << 32) - 1, 1 << 32]
    for B in bases:
        n = int(rng.integers(1, 90))
        d = [int(v) for v in rng.integers(0, B, n, dtype=np.uint64)]
        d[int(rng.integers(0, n))] = B - 1
        ref = bf.family_encode(family, d, B, 32)
        assert all(0 <= w < 2 ** 32 for w in ref)
        ours = orc.family_pack(family, np.array(d, dtype=np.uint64), B, W=32)
        assert [int(x) for x in ours] == ref, B
        assert orc.family_words(family, n, B, 32) == len(ref)
        assert np.array_equal(orc.family_unpack(family, ours, n, B, W=32), np.array(d, dtype=np.uint64)), B


def test_k32_is_eq1_with_exact_capacity():
    # Eq. (1) as printed with 2^32 - 1 differs only where B^p == 2^32 exactly
    import math
    for B in list(range(2, 5000)) + [65535, 65536, 65537, 1 << 20, (1 << 32) - 1]:
        paper = math.floor(math.log(2 ** 32 - 1) / math.log(B))
        k = _k32(B)
        assert k == paper or (k == paper + 1 and B ** k == 2 ** 32)


# --- stream level: an independent writer ------------------------------------------------

def _tile_blocks(L, w):
    P = 256
    while P > 1 and P * L * w > 16384:
        P //= 2
    return P


def _write32(x: np.ndarray, L: int, variant: int) -> bytes:
    """The 32-bit-word stream of x by the documented layout, blocks encoded by the big-integer
    reference; exhaustive takes the smaller of classes 0 and 8, ties to 0."""
    w, n = x.itemsize, x.size
    nb = -(-n // L)
    tb = _tile_blocks(L, w)
    nt = -(-nb // tb)
    flags = 8 | (1 if variant == EXH else 0)
    mins, rngs, cls, payload, index = [], [], [], [], []
    for b in range(nb):
        blk = [int(v) for v in x[b * L:(b + 1) * L]]
        lo, hi = min(blk), max(blk)
        B = hi - lo + 1
        d = [v - lo for v in blk]
        enc = {c: bf.family_encode(c >> 3, d, B, 32) if B > 1 else [] for c in (0, 8)}
        c = (8 if len(enc[8]) < len(enc[0]) else 0) if variant == EXH else variant
        if b % tb == 0:
            index.append(len(payload))
        mins.append(lo)
        rngs.append(B - 1)
        cls.append(c)
        payload += enc[c]
    fmt = {1: "B", 2: "H", 4: "I"}[w]
    arrays = struct.pack("<%dQ" % nt, *index) + struct.pack("<%d%s" % (nb, fmt), *mins) + \
        struct.pack("<%d%s" % (nb, fmt), *rngs)
    if flags & 1:
        arrays += bytes(cls)
    arrays += bytes((-(64 + len(arrays))) % 8)
    body = arrays + struct.pack("<%dI" % len(payload), *payload)
    total = 64 + len(body)
    hdr = struct.pack("<IHBBBBHIQQIIQQQ", 0x504D4350, 1, w, flags, 0 if variant == EXH else variant,
                      1 if variant == EXH else 0, 0, L, n, nb, tb, 0, len(payload), total, 0)
    return hdr + body


def _sample(rng, dtype, n, spread):
    bits = np.dtype(dtype).itemsize * 8
    x = rng.normal(1 << (bits - 1), spread, n).clip(0, (1 << bits) - 1).astype(dtype)
    if n:
        x[rng.integers(0, n, 3)] = rng.integers(0, 1 << bits, 3, dtype=np.uint64).astype(dtype)
    return x


@pytest.mark.parametrize("variant", [0, 8, EXH])
@pytest.mark.parametrize("dtype,L,n", [(np.uint8, 64, 3000), (np.uint16, 40, 2917), (np.uint16, 7, 333),
                                       (np.uint16, 1000, 4321), (np.uint8, 1, 50)])
def test_stream32_equals_independent_writer(orc, variant, dtype, L, n):
    rng = np.random.default_rng(n + variant)
    for spread in (3.0, 40.0, 3000.0):
        x = _sample(rng, dtype, n, spread)
        s = orc.compress32(x, L, variant)
        assert s == _write32(x, L, variant)
        assert len(s) <= orc.bound32(n, x.itemsize, L, variant)
        assert np.array_equal(orc.decompress32(s), x)


def test_stream32_u32_basic(orc):
    rng = np.random.default_rng(5)
    for spread in (10.0, 1e5, 1e9):
        x = _sample(rng, np.uint32, 2000, spread)
        s = orc.compress32(x, 100, 0)
        assert s == _write32(x, 100, 0)
        assert np.array_equal(orc.decompress32(s), x)


def test_stream32_constant_full_range_and_empty(orc):
    x = np.zeros(1000, dtype=np.uint16)
    x[500:600] = 65535
    x[700:] = 1234
    for v in (0, 8, EXH):
        s = orc.compress32(x, 100, v)
        assert s == _write32(x, 100, v)
        assert np.array_equal(orc.decompress32(s), x)
        e = orc.compress32(np.zeros(0, dtype=np.uint8), 16, v)
        assert len(e) == 64 and orc.decompress32(e).size == 0


def test_stream32_errors_and_separation(orc):
    x = np.arange(100, dtype=np.uint32)
    with pytest.raises(ValueError):
        orc.compress32(x, 10, 8)  # advanced needs u8 / u16 data
    with pytest.raises(ValueError):
        orc.compress32(x.astype(np.uint16), 10, 3)  # only classes 0 and 8
    y = np.arange(300, dtype=np.uint16) * 7
    s32 = orc.compress32(y, 30, 8)
    s64 = orc.compress(y, 30, 8)
    assert orc.decompress_rc(s32)[0] == -3 and orc.decompress32_rc(s64)[0] == -3
    bad = bytearray(s32)
    bad[7] |= 2  # excess-count flag: never set in these streams
    assert orc.decompress32_rc(bytes(bad))[0] == -3
    assert orc.decompress32_rc(s32[:-4])[0] == -3
