"""Polynomial reduction followed by LZMA (the paper's "Poly + LZMA", Sec. 4.3.1 Table 1 and
Sec. 4.3.2 Table 2): the GPU stream is handed to the host's liblzma (through Python's ``lzma``
module) as a second stage.

The paper uses the polynomial reduction as a pre-compression in front of LZMA: the reduction
packs small values into large ones and flattens the byte profile, so LZMA then reaches about its
own ratio in a fraction of its time (Sec. 4.3.2). Here the first stage runs on the GPU
(``compress`` / ``Batch``), the second on host cores. LZMA works on independent chunks of the
stream (each chunk its own ``.xz`` member, several compressed at once on host threads; liblzma
releases the interpreter lock), so a file is still readable by parts.

Nothing here touches the polynomial arithmetic: decompression is LZMA on the host, then the
library's GPU decoder.
"""
from __future__ import annotations

import concurrent.futures as cf
import lzma
import os
import struct

import torch

# LZMA2 settings of the paper's runs (7z, Sec. 4.3.1): "-mx=1 -mfb=64 -md=32m" (fast) and
# "-mx=9 -mfb=64 -md=200m" (best). "fast" is the default here.
FILTERS = {
    "fast": [{"id": lzma.FILTER_LZMA2, "preset": 1, "nice_len": 64, "dict_size": 32 << 20}],
    "best": [{"id": lzma.FILTER_LZMA2, "preset": 9, "nice_len": 64, "dict_size": 192 << 20}],
}
CHUNK = 4 << 20  # largest independently compressed LZMA member (bytes)
MIN_CHUNK = 1 << 18

_MAGIC = b"PLZ1"


def _threads(threads):
    return max(1, int(threads if threads else (os.cpu_count() or 1)))


def chunk_for(n: int, threads: int = 0) -> int:
    """Member size for n bytes: enough members for every host thread, each between MIN_CHUNK and
    CHUNK bytes."""
    t = _threads(threads)
    return min(CHUNK, max(MIN_CHUNK, -(-n // t)))


def lzma_pack(data: bytes, mode: str = "fast", threads: int = 0, chunk: int = 0) -> bytes:
    """LZMA of `data` in independent chunks (chunk = 0: ``chunk_for``): magic, chunk count, the
    compressed size of every chunk (u64 each), then the chunks."""
    chunk = chunk if chunk > 0 else chunk_for(len(data), threads)
    parts = [data[i:i + chunk] for i in range(0, len(data), chunk)] or [b""]

    def one(p):
        # a dictionary larger than the chunk finds nothing more and only costs memory
        filt = [dict(f, dict_size=max(4096, min(f["dict_size"], len(p)))) for f in FILTERS[mode]]
        return lzma.compress(p, format=lzma.FORMAT_XZ, check=lzma.CHECK_NONE, filters=filt)

    with cf.ThreadPoolExecutor(_threads(threads)) as pool:
        comp = list(pool.map(one, parts))
    head = _MAGIC + struct.pack("<Q", len(comp)) + b"".join(struct.pack("<Q", len(c)) for c in comp)
    return head + b"".join(comp)


def lzma_unpack(blob: bytes, threads: int = 0) -> bytes:
    """Inverse of ``lzma_pack``."""
    if blob[:4] != _MAGIC:
        raise ValueError("not a chunked LZMA blob")
    (n,) = struct.unpack_from("<Q", blob, 4)
    sizes = struct.unpack_from("<%dQ" % n, blob, 12)
    offs, o = [], 12 + 8 * n
    for s in sizes:
        offs.append((o, o + s))
        o += s
    with cf.ThreadPoolExecutor(_threads(threads)) as pool:
        parts = list(pool.map(lambda ab: lzma.decompress(blob[ab[0]:ab[1]], format=lzma.FORMAT_XZ), offs))
    return b"".join(parts)


def compress(stream: torch.Tensor, mode: str = "fast", threads: int = 0, chunk: int = 0) -> bytes:
    """Second stage: LZMA of a polynomial stream (a u8 tensor on the GPU or the host)."""
    host = stream.detach().to("cpu", non_blocking=False).contiguous()
    return lzma_pack(host.numpy().tobytes(), mode, threads, chunk)


def decompress(blob: bytes, device="cuda", threads: int = 0) -> torch.Tensor:
    """First step back: the polynomial stream as a u8 tensor on `device`, ready for the GPU
    decoder (``paper_1805_01844_amd.decompress``)."""
    raw = lzma_unpack(blob, threads)
    host = torch.frombuffer(bytearray(raw), dtype=torch.uint8)
    if device == "cpu":
        return host
    return host.pin_memory().to(device, non_blocking=False)
