"""Time-major blocking (Sec. 4.3.1, the waveform matrix M_ij = i-th time sample of pixel j): the
GPU reads camera events [pixels][samples] column by column, and the stream must equal the
oracle's stream of the transposed array byte for byte; decoding writes the events back in
their own layout."""
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


def _np(x):
    x = x.cpu().contiguous().reshape(-1)
    if x.dtype == torch.uint16:
        return x.view(torch.int16).numpy().view(np.uint16)
    if x.dtype == torch.uint32:
        return x.view(torch.int32).numpy().view(np.uint32)
    return x.numpy()


def _case(pc, orc, x, L, variant, what):
    print("case:", what, tuple(x.shape), x.dtype, "L=%d variant=%d" % (L, variant), flush=True)
    xd = x.cuda()
    s = pc.compress_transposed(xd, L, variant)
    want = orc.compress(_np(x.transpose(1, 2)), L, variant)
    assert s.cpu().numpy().tobytes() == want, "%s: stream differs from the oracle's of the transpose" % what
    out = torch.full_like(xd, 0x5A) if x.dtype == torch.uint8 else torch.zeros_like(xd)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pc.decompress_transposed_into(s, out, st, L)
    assert int(st.item()) == 0
    assert np.array_equal(_np(out), _np(x)), "%s: round trip" % what
    return s


@pytest.mark.parametrize("variant", [0, 8, 3, EXH])
@pytest.mark.parametrize("L", [40, 1855, 256])
def test_camera_time_major_matches_oracle(pc, orc, variant, L):
    x = datagen.camera_events(3, seed=31)
    _case(pc, orc, x, L, variant, "camera")


def test_ragged_and_wide_time_major(pc, orc):
    g = torch.Generator().manual_seed(9)
    x8 = torch.randint(0, 256, (2, 37, 13), generator=g, dtype=torch.int32).to(torch.uint8)
    _case(pc, orc, x8, 100, EXH, "u8 ragged")
    x32 = (torch.randint(0, 1 << 20, (1, 300, 7), generator=g, dtype=torch.int64)).to(torch.uint32)
    _case(pc, orc, x32, 64, EXH, "u32")
    x1 = datagen.camera_events(1, seed=2)[:, :5, :]  # fewer pixels than a wavefront step
    _case(pc, orc, x1.contiguous(), 7, 8, "tiny")


def test_time_major_more_shapes(pc, orc):
    # u8 and u32 matrices, many small matrices in one tile, tiles that start and end inside a
    # column, ragged last blocks
    g = torch.Generator().manual_seed(11)
    x8 = torch.randint(0, 256, (3, 100, 32), generator=g, dtype=torch.int32).to(torch.uint8)
    _case(pc, orc, x8, 37, EXH, "u8 rows of 32")
    x32 = torch.randint(0, 1 << 31, (2, 70, 12), generator=g, dtype=torch.int64).to(torch.uint32)
    _case(pc, orc, x32, 50, 0, "u32 rows of 12")
    xs = torch.randint(0, 4000, (40, 64, 8), generator=g, dtype=torch.int32).to(torch.uint16)
    for L, v in ((5, EXH), (64, 8), (1000, 3)):
        _case(pc, orc, xs, L, v, "u16 small matrices")


def test_time_major_shape_mismatch_is_reported(pc, orc):
    x = datagen.camera_events(2, seed=3).cuda()
    s = pc.compress_transposed(x, 40, EXH)
    out = torch.empty((1, 1855, 40), dtype=torch.uint16, device="cuda")  # one event, the stream holds two
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pc.decompress_transposed_into(s, out, st, 40)
    assert int(st.item()) == pc.ECORRUPT
    # the typed decoder rejects another block length the same way
    flat = torch.empty(x.numel(), dtype=torch.uint16, device="cuda")
    pc.decompress_into(s, flat, st, dtype_bytes=2, block_len=41)
    assert int(st.item()) == pc.ECORRUPT
