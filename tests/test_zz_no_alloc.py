"""pcomp_compress_noalloc: compression whose workspace is the library's own device buffer.

Its output must equal pcomp_compress's (with a workspace the caller allocates) byte for byte, on
two calls in a row, the second with a smaller input (the buffer keeps the first call's contents),
and equal the oracle's stream."""
import ctypes

import numpy as np
import pytest
import torch

import datagen

pytestmark = pytest.mark.gpu


def _as_np(x):
    x = x.cpu().reshape(-1)
    return x.view(torch.int16).numpy().view(np.uint16) if x.dtype == torch.uint16 else x.numpy()


def _noalloc(pc, x, L, variant):
    lib = pc.lib()
    w = x.element_size()
    cap = pc.bound(x.numel(), w, L, variant)
    out = torch.full((cap,), 0xEE, dtype=torch.uint8, device=x.device)
    size = torch.zeros(1, dtype=torch.int64, device=x.device)
    rc = lib.pcomp_compress_noalloc(ctypes.c_void_p(x.data_ptr()), x.numel(), w, L, variant,
                                    ctypes.c_void_p(out.data_ptr()), cap, ctypes.c_void_p(size.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, "pcomp_compress_noalloc returned %d" % rc
    return out[:int(size.item())]


def test_noalloc_matches_compress_twice(orc):
    import paper_1805_01844_amd as pc

    pc.init()
    for events, variant in ((6, pc.SELECT_EXHAUSTIVE), (2, pc.SELECT_EXHAUSTIVE), (3, 8)):
        print("case: noalloc camera events=%d variant=%d" % (events, variant), flush=True)
        x = datagen.camera_events(events, seed=40 + events).reshape(-1).cuda()
        got = _noalloc(pc, x, 40, variant).cpu().numpy().tobytes()
        want = pc.compress(x, 40, variant).cpu().numpy().tobytes()
        assert got == want, "noalloc stream differs from pcomp_compress (events=%d)" % events
        assert got == orc.compress(_as_np(x), 40, variant)


def test_noalloc_rejects_oversized_call():
    import paper_1805_01844_amd as pc

    pc.init()
    lib = pc.lib()
    n = 1 << 30  # needs more workspace than the library's buffer holds at L = 40
    assert pc.workspace_size(n, 2, 40, pc.SELECT_EXHAUSTIVE) > 32 << 20
    rc = lib.pcomp_compress_noalloc(ctypes.c_void_p(16), n, 2, 40, pc.SELECT_EXHAUSTIVE, ctypes.c_void_p(16),
                                    pc.bound(n, 2, 40, pc.SELECT_EXHAUSTIVE), ctypes.c_void_p(16), None)
    assert rc == pc.ENOWS
