"""Stress workload on the GPU: 4 GiB of mixed u8/u16/u32 blocks (Laplacian noise with scale
U(1, 50), 0.1% outliers over the full range, constant and full-range blocks) plus one u32
block for every base B in [2, 2^16], as one batch. The streams are packed one after another,
and at a ratio of about 1.37 four GiB of input make 3.3 GB of streams; the test compresses 6 GiB
so that the later streams start past 2^32 bytes.
Every value round-trips on the GPU; sampled tiles equal the oracle's stream of the same
blocks byte for byte (block arrays and payload)."""
import numpy as np
import pytest
import torch

import datagen
from streamfmt import parse as _parse, tile_parts as _tile_parts

pytestmark = pytest.mark.gpu

EXH = 0x100
L = 1024


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


def stress_segments(total_bytes: int = 1 << 32, seed: int = 90):
    """Thirds (by bytes) of u8, u16 and u32 stress blocks, generated on the GPU in chunks, then
    the base sweep."""
    segs = []
    for k, dt in enumerate((torch.uint8, torch.uint16, torch.uint32)):
        w = torch.tensor([], dtype=dt).element_size()
        nblk = total_bytes // 3 // (L * w)
        out = torch.empty(nblk * L, dtype=dt, device="cuda")
        step = (256 << 20) // (L * w)
        for c, b0 in enumerate(range(0, nblk, step)):
            nb = min(step, nblk - b0)
            out[b0 * L:(b0 + nb) * L] = datagen.laplace_blocks(nb, L, dt, seed=seed + 1000 * k + c, device="cuda",
                                                               outlier_rate=1e-3).reshape(-1)
        segs.append(out)
    segs.append(datagen.base_sweep_u32(L=L, device="cuda"))
    return segs


def test_stress_4gib_batch(pc, orc):
    segs = stress_segments(6 << 30)
    raw = sum(s.numel() * s.element_size() for s in segs)
    print("case: stress batch, %d segments, %.3f GB" % (len(segs), raw / 1e9), flush=True)
    assert raw >= 6 << 30
    b = pc.Batch(segs, block_len=L, variant=EXH)
    b.compress()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    offs = b.offsets() + [b.total_bytes()]
    assert offs[-2] > 1 << 32  # the base sweep's stream sits past 2^32 bytes
    sizes = [offs[i + 1] - offs[i] for i in range(len(segs))]
    print("ratio %.4f" % (raw / offs[-1]), flush=True)
    outs = [torch.empty_like(s) for s in segs]
    dec = pc.BatchDecoder(b, outs)
    dec()
    dec.check()
    for i, (s, o) in enumerate(zip(segs, outs)):
        assert torch.equal(s.view(torch.uint8), o.view(torch.uint8)), "segment %d round trip" % i
    del outs
    # sampled tiles against the oracle's stream of the same blocks
    rng = np.random.default_rng(5)
    for i, s in enumerate(segs):
        st = b.out[offs[i]:offs[i] + sizes[i]]
        head = st[:64].cpu().numpy()
        meta0 = _parse(np.concatenate([head, np.zeros(0, np.uint8)]))
        nt = meta0["ntiles"]
        picks = sorted(set([0, nt - 1] + rng.integers(0, nt, 6).tolist()))
        # the tile index, block arrays and the payload pieces of the sampled tiles
        host = st.cpu().numpy() if sizes[i] < (256 << 20) else None
        for t in picks:
            tb = meta0["tb"]
            v0, v1 = t * tb * L, min(s.numel(), (t + 1) * tb * L)
            want = np.frombuffer(orc.compress(_as_np(s[v0:v1]), L, EXH), np.uint8)
            wm = _parse(want)
            if host is None:
                # fetch only what the tile needs: header + index + arrays region + its payload
                o = meta0["off"]
                arrays = st[:o["payload"]].cpu().numpy()
                idx = arrays[o["index"]:o["index"] + 8 * nt].view(np.uint64)
                p0 = int(idx[t])
                p1 = int(idx[t + 1]) if t + 1 < nt else meta0["pw"]
                pay = st[o["payload"] + 8 * p0:o["payload"] + 8 * p1].cpu().numpy()
                buf = np.zeros(o["payload"] + 8 * p1, np.uint8)
                buf[:o["payload"]] = arrays
                buf[o["payload"] + 8 * p0:] = pay
            else:
                buf = host
            got = _tile_parts(buf, _parse(buf), t)
            ref = _tile_parts(want, wm, 0)
            assert got == ref, "segment %d tile %d differs from the oracle" % (i, t)
        print("segment %d: %d tiles sampled" % (i, len(picks)), flush=True)
