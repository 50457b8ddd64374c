"""Reading v1 streams in tests: header fields, array offsets and one tile's parts (block
arrays and payload bytes), following the layout documented in include/pcomp.h."""
import numpy as np


def parse(buf: np.ndarray):
    """Header fields and array offsets of a v1 stream (the documented layout)."""
    h = buf[:64].view(np.uint64)
    w, flags = int(buf[6]), int(buf[7])
    Lb, n, nblocks, tb, pw = int(buf[12:16].view(np.uint32)[0]), int(h[2]), int(h[3]), int(h[4]), int(h[5])
    ntiles = (nblocks + tb - 1) // tb
    o = 64
    off = {"index": o}
    o += 8 * ntiles
    off["min"] = o
    o += w * nblocks
    off["range"] = o
    o += w * nblocks
    off["class"] = o
    if flags & 1:
        o += nblocks
    off["ne"] = o
    neb = 2 if flags & 4 else 1
    if flags & 2:
        o += neb * nblocks
    off["payload"] = (o + 7) & ~7
    return dict(w=w, flags=flags, L=Lb, n=n, nblocks=nblocks, tb=tb, pw=pw, ntiles=ntiles, neb=neb, off=off)


def tile_parts(buf: np.ndarray, meta: dict, t: int):
    """Block arrays and payload bytes of tile t."""
    tb, w, o = meta["tb"], meta["w"], meta["off"]
    b0, b1 = t * tb, min(meta["nblocks"], (t + 1) * tb)
    idx = buf[o["index"]:o["index"] + 8 * meta["ntiles"]].view(np.uint64)
    p0 = int(idx[t])
    p1 = int(idx[t + 1]) if t + 1 < meta["ntiles"] else meta["pw"]
    wb = 4 if meta["flags"] & 8 else 8  # bytes per payload word (flags bit 3: 32-bit words)
    parts = {
        "min": buf[o["min"] + w * b0:o["min"] + w * b1].tobytes(),
        "range": buf[o["range"] + w * b0:o["range"] + w * b1].tobytes(),
        "payload": buf[o["payload"] + wb * p0:o["payload"] + wb * p1].tobytes(),
    }
    if meta["flags"] & 1:
        parts["class"] = buf[o["class"] + b0:o["class"] + b1].tobytes()
    if meta["flags"] & 2:
        parts["ne"] = buf[o["ne"] + meta["neb"] * b0:o["ne"] + meta["neb"] * b1].tobytes()
    return parts
