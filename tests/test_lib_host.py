"""Host-only checks of the HIP library (no GPU needed): exports, bounds, the schedule tables."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pc():
    import paper_1805_01844_amd as pc

    if not os.path.exists(pc.LIB_PATH):
        from paper_1805_01844_amd import build

        build.build()
    pc.lib()
    return pc


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(pcomp_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_function(pc):
    names = _declared_functions()
    assert "pcomp_compress" in names and "pcomp_decompress" in names and "pcomp_bound" in names
    L = ctypes.CDLL(pc.LIB_PATH)
    for name in names:
        assert hasattr(L, name), name


@pytest.mark.parametrize("w,L", [(1, 1), (1, 1024), (2, 40), (2, 1024), (4, 256), (4, 4096), (2, 65535)])
@pytest.mark.parametrize("variant", [0, 8, 3, 0x100, 0x200])
def test_bound_matches_oracle(pc, orc, w, L, variant):
    for n in [0, 1, L - 1, L, 10 * L + 3, 123457]:
        assert pc.bound(n, w, L, variant) == orc.bound(n, w, L, variant)
        assert pc.workspace_size(n, w, L, variant) >= 8


def test_bound_rejects_bad_arguments(pc):
    assert pc.bound(10, 3, 40, 0) == 0
    assert pc.bound(10, 2, 0, 0) == 0
    assert pc.bound(10, 2, 65536, 0) == 0
    assert pc.bound(10, 2, 40, 16) == 0


def test_schedule_tables_match_oracle_series(pc, orc):
    # the cycle form of every tabled base reproduces the oracle's series word by word
    rng = np.random.default_rng(0)
    bases = list(range(2, 300)) + [int(b) for b in rng.integers(300, 65538, 300)] + [65535, 65536, 65537]
    bases += [(1 << j) + 1 for j in range(17, 32)]
    for B in bases:
        n = 4000 if B < 65538 else 300
        p, R, Rp, q = orc.adv_schedule(n, B)
        k, mu, lam, V = pc.atlas_info(B)
        assert k == orc.digits_per_word(B)
        if B > 65537:
            continue
        for i in range(len(p)):
            s_i, p_i, R_i, q_i = pc.atlas_word(B, i)
            assert (s_i, p_i, R_i, q_i) == (int(Rp[i]), int(p[i]), int(R[i]), int(q[i])), (B, i)


def test_schedule_cycles_are_short(pc):
    worst = 0
    for B in range(2, 65538, 7):
        k, mu, lam, V = pc.atlas_info(B)
        worst = max(worst, mu + lam)
        assert lam >= 1 and V > 0
    assert worst < 600


def test_cycle_form_word_counts_match_oracle(pc, orc):
    # the bounded search over the cycle form gives the oracle's word count of the series
    import ctypes
    L = pc.lib()
    L.pcomp_atlas_words.restype = ctypes.c_int
    L.pcomp_atlas_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
    rng = np.random.default_rng(3)
    bases = list(range(2, 200)) + [int(b) for b in rng.integers(200, 65538, 200)] + [65536, 65537]
    bases += [(1 << j) + 1 for j in range(17, 32)]
    out = ctypes.c_uint32()
    for B in bases:
        for n in [1, 2, 5, 13, 14, 40, 41, 154, 1000, 1024, 4096, 65535]:
            assert L.pcomp_atlas_words(B, n, ctypes.byref(out)) == 0
            assert out.value == orc.adv_words(n, B), (B, n)


def test_cycle_form_word_counts_32bit_words_match_oracle(pc, orc):
    # the tables of 32-bit words: word counts of the series with capacity 2^32, for every base
    # in steps and the ends of the range, against the oracle's walk of the series
    import ctypes
    L = pc.lib()
    L.pcomp_atlas32_words.restype = ctypes.c_int
    L.pcomp_atlas32_words.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
    bases = list(range(2, 400)) + list(range(400, 65538, 97)) + [65535, 65536, 65537]
    out = ctypes.c_uint32()
    for B in bases:
        for n in [1, 2, 3, 7, 40, 41, 154, 1000, 4096, 16384]:
            assert L.pcomp_atlas32_words(B, n, ctypes.byref(out)) == 0
            assert out.value == orc.adv_words(n, B, 32), (B, n)
    assert L.pcomp_atlas32_words(65538, 10, ctypes.byref(out)) != 0


@pytest.mark.parametrize("w,L", [(1, 1), (1, 1024), (2, 40), (2, 1024), (4, 256), (4, 4096)])
@pytest.mark.parametrize("variant", [0, 8, 0x100])
def test_bound32_matches_oracle(pc, orc, w, L, variant):
    lib = pc.lib()
    for n in [0, 1, L - 1, L, 10 * L + 3, 123457]:
        want = orc.bound32(n, w, L, variant)
        assert lib.pcomp_bound32(n, w, L, variant) == want
        assert (lib.pcomp_workspace_size32(n, w, L, variant) >= 8) == (want > 0)
    assert lib.pcomp_bound32(10, 2, 40, 3) == 0 and lib.pcomp_bound32(10, 2, 0, 0) == 0


def _segs(pc, spec):
    arr = (pc._Segment * len(spec))()
    for i, (w, n) in enumerate(spec):
        arr[i] = pc._Segment(0x10000 * (i + 1), n, w, 0)  # plans record pointers, never read them
    return arr


def test_batch_plan_capacity_and_tiles(pc, orc):
    """The output capacity of a batch is the sum of its segments' bounds (the streams, packed one
    after another, never take more); tiles are counted per segment with the segment's own tile
    size; the workspace holds one block record per tile slot of each width group."""
    spec = [(2, 74200), (4, 3000), (2, 0), (1, 777), (2, 1), (4, 50000), (1, 0)]
    Ls = (300, 40, 1000)
    for variant in (0, 8, 5, 0x100):
        segs = _segs(pc, spec)
        L3 = (ctypes.c_uint32 * 3)(*Ls)
        nb = pc.lib().pcomp_batch_plan_bytes(segs, len(spec), L3, variant)
        assert nb > 0
        buf = (ctypes.c_uint64 * (nb // 8 + 1))()
        assert pc.lib().pcomp_batch_plan(segs, len(spec), L3, variant, buf, nb) == 0
        assert pc.lib().pcomp_batch_plan(segs, len(spec), L3, variant, buf, nb - 8) == pc.ENOSPC
        ob, wb, nt = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        assert pc.lib().pcomp_batch_info(buf, ctypes.byref(ob), ctypes.byref(wb), ctypes.byref(nt)) == 0
        cap, tiles, slots = 0, 0, 0
        for i, (w, n) in enumerate(spec):
            L = Ls[{1: 0, 2: 1, 4: 2}[w]]
            cap += orc.bound(n, w, L, variant)
            nblk = (n + L - 1) // L
            tb = orc.tile_blocks(L, w)
            tiles += (nblk + tb - 1) // tb
            slots += (nblk + tb - 1) // tb * tb * (2 * w + 4)
        assert ob.value == cap and nt.value == tiles
        assert wb.value >= 8 + 12 * tiles + 8 * len(spec) + slots


def test_batch_plan_rejects_bad_arguments(pc):
    L3 = (ctypes.c_uint32 * 3)(1024, 1024, 1024)
    assert pc.lib().pcomp_batch_plan_bytes(_segs(pc, [(3, 10)]), 1, L3, 0) == 0   # bad dtype
    assert pc.lib().pcomp_batch_plan_bytes(_segs(pc, [(2, 10)]), 1, L3, 16) == 0  # bad variant
    big = (ctypes.c_uint32 * 3)(1024, 8193, 1024)  # u16 blocks over the 16 KiB tile
    assert pc.lib().pcomp_batch_plan_bytes(_segs(pc, [(2, 10)]), 1, big, 0) == 0
    # an unused group's block length is not checked
    assert pc.lib().pcomp_batch_plan_bytes(_segs(pc, [(1, 10)]), 1, big, 0) > 0
    buf = (ctypes.c_uint64 * 8)()
    assert pc.lib().pcomp_batch_info(buf, None, None, None) == pc.EINVAL  # not a plan


def test_binding_rejects_host_tensors_and_bad_shapes(pc):
    """The binding refuses arguments the library cannot take before any call reaches it."""
    import torch

    u8, u16 = torch.zeros(64, dtype=torch.uint8), torch.zeros(8, dtype=torch.uint16)
    i32 = torch.zeros(1, dtype=torch.int32)
    with pytest.raises(ValueError):
        pc.decompress_into(u8, u16, i32)  # host tensors
    with pytest.raises(ValueError):
        pc.block_features(u16, 40)
    with pytest.raises(ValueError):
        pc.mlp_scores(torch.zeros(pc.MLP_PARAMS), torch.zeros(4, pc.MLP_IN))
    with pytest.raises(ValueError):
        pc._block_lens((40, 40))
