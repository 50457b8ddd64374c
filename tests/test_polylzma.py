"""Poly + LZMA (Sec. 4.3.1 Table 1, Sec. 4.3.2 Table 2): LZMA as a second stage over the
polynomial stream. The chunked LZMA container round-trips, the oracle's stream survives it
byte for byte, and the GPU stream does too (LZMA on the host, then the GPU decoder)."""
import numpy as np
import pytest
import torch

import datagen
from paper_1805_01844_amd import polylzma


def _u16(x):
    return x.reshape(-1).view(torch.int16).numpy().view(np.uint16)


@pytest.mark.parametrize("chunk", [1 << 10, 1 << 16, 1 << 25])
def test_chunked_lzma_round_trip(chunk):
    rng = np.random.default_rng(3)
    for n in (0, 1, 1000, 200000):
        data = rng.integers(0, 7, n, dtype=np.uint8).tobytes()
        blob = polylzma.lzma_pack(data, "fast", threads=3, chunk=chunk)
        assert polylzma.lzma_unpack(blob, threads=2) == data


def test_oracle_stream_through_lzma(orc):
    x = _u16(datagen.camera_events(3, seed=5))
    s = orc.compress(x, 40, orc.SELECT_EXHAUSTIVE)
    blob = polylzma.lzma_pack(s, "fast", threads=2, chunk=1 << 16)
    back = polylzma.lzma_unpack(blob)
    assert back == s
    assert np.array_equal(orc.decompress(back), x)
    # the second stage only removes redundancy left in the stream: never much larger than it
    assert len(blob) < len(s) * 1.01 + 256


def test_bad_blob_is_rejected():
    with pytest.raises(ValueError):
        polylzma.lzma_unpack(b"XXXX" + bytes(12))


@pytest.mark.gpu
def test_gpu_stream_through_lzma(orc):
    import paper_1805_01844_amd as pc

    x = datagen.camera_events(4, seed=6).reshape(-1)
    print("case: poly+lzma camera 4 events", flush=True)
    s = pc.compress(x.cuda(), 40, pc.SELECT_EXHAUSTIVE)
    blob = polylzma.compress(s, "fast")
    s2 = polylzma.decompress(blob, device="cuda")
    assert torch.equal(s2, s)
    y = pc.decompress(s2)
    assert torch.equal(y.cpu().view(torch.int16), x.view(torch.int16))
    assert s.cpu().numpy().tobytes() == orc.compress(_u16(x), 40, orc.SELECT_EXHAUSTIVE)
