"""Integrated-signal workload (Sec. 4.3.2): per-pixel sums of camera waveforms made on the GPU
(checked against a plain sum on the host), then compressed as u32 vectors; streams equal the
oracle's, and decode back."""
import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import paper_1805_01844_amd as pc

    pc.init()
    return pc


def _u32(x):
    return x.cpu().reshape(-1).view(torch.int32).numpy().view(np.uint32)


@pytest.mark.parametrize("shape,dtype", [((5, 1855, 40), torch.uint16), ((3, 2048, 96), torch.uint16),
                                         ((2, 113, 128), torch.uint16), ((4, 77, 300), torch.uint8),
                                         ((2, 9, 1), torch.uint32)])
def test_integrate_matches_host_sum(pc, shape, dtype):
    print("case: integrate", shape, dtype, flush=True)
    g = torch.Generator().manual_seed(sum(shape))
    hi = {torch.uint8: 256, torch.uint16: 65536, torch.uint32: 1 << 32}[dtype]
    x = torch.randint(0, hi, shape, generator=g, dtype=torch.int64)
    want = x.sum(-1).numpy().astype(np.uint32)
    xs = x.to(torch.int32).to(dtype) if dtype != torch.uint32 else x.to(torch.uint32)
    got = pc.integrate(xs.cuda())
    assert got.shape == shape[:-1]
    assert np.array_equal(_u32(got), want.reshape(-1))


@pytest.mark.parametrize("L", [1855, 512])
def test_integrated_events_compress_like_oracle(pc, orc, L):
    ev = datagen.camera_events(6, seed=44)
    sums = pc.integrate(ev.cuda()).reshape(-1)
    ref = ev.to(torch.int64).sum(-1).reshape(-1).numpy().astype(np.uint32)
    assert np.array_equal(_u32(sums), ref)
    for variant in (0, 8, pc.SELECT_EXHAUSTIVE):
        print("case: integrated L=%d variant=%d" % (L, variant), flush=True)
        s = pc.compress(sums, L, variant)
        assert s.cpu().numpy().tobytes() == orc.compress(ref, L, variant)
        assert np.array_equal(_u32(pc.decompress(s)), ref)


def test_integrate_rejects_overflowing_traces(pc):
    for shape, dt in (((3, 2), torch.uint32),       # two u32 samples can sum past 2^32
                      ((1, 8193), torch.uint16)):   # a trace larger than the 16 KiB a workgroup stages
        x = torch.zeros(shape, dtype=dt, device="cuda")
        with pytest.raises(pc.PcompError):
            pc.integrate(x)
