"""Autotuner for batches: block length per element width and launch grid.

The block length L changes the stream (every block stores its own minimum and range, Sec. 3;
the paper picks L = 154 for its camera data, Sec. 4.2), so the tuner weighs compression
ratio against speed: per width group it keeps the block lengths whose ratio is within
``ratio_slack`` of the best one, and among those takes the fastest (compress + decompress
time). Then it times the launch grid: 0 = one workgroup per tile, or a persistent grid of
that many workgroups (the tiles each workgroup walks: the work per wave). Timing runs the
real kernels on a sample of the batch through a captured HIP graph.

Results are cached per (device, variant, batch signature) in a JSON file:
``$PCOMP_TUNE_CACHE``, else ``~/.cache/pcomp/tune.json``.
"""
from __future__ import annotations

import json
import os

import torch

import paper_1805_01844_amd as pc

CANDIDATE_L = (256, 512, 1024, 4096)
CANDIDATE_GRID = (0, 1024, 2048, 4096)
_GROUP_OF = {1: 0, 2: 1, 4: 2}


def cache_path() -> str:
    return os.environ.get("PCOMP_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "pcomp",
                                                             "tune.json")


def signature(segments, variant: int) -> str:
    """Device, variant and the batch's mix: per width, segment count and values per segment
    (rounded to powers of two)."""
    mix = {}
    for s in segments:
        key = "w%d:2^%d" % (s.element_size(), max(0, int(s.numel()).bit_length() - 1))
        mix[key] = mix.get(key, 0) + 1
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    parts = ["%s=%d" % (k, mix[k]) for k in sorted(mix)]
    return "%s|v%d|%s" % (dev, variant, ",".join(parts))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def sample_segments(segments, max_segments: int = 64, max_bytes: int = 256 << 20):
    """An evenly spaced subset of the segments, bounded in count and bytes."""
    n = len(segments)
    if n == 0:
        return []
    step = max(1, n // max_segments)
    out, tot = [], 0
    for i in range(0, n, step):
        s = segments[i]
        if out and tot + s.numel() * s.element_size() > max_bytes:
            break
        out.append(s)
        tot += s.numel() * s.element_size()
    return out


def _time_batch(segs, block_len, variant, grid, reps):
    """(compress ms, decompress ms, ratio) of the batch, timed with device events around
    graph replays of the compression and eager decompression calls."""
    b = pc.Batch(segs, block_len=block_len, variant=variant, grid=grid)
    g = b.capture()
    outs = [torch.empty_like(s) for s in segs]
    dec = pc.BatchDecoder(b, outs, grid=grid)
    dec()
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tc = td = 0.0
    for _ in range(reps):
        e[0].record()
        g.replay()
        e[1].record()
        dec()
        e[2].record()
        torch.cuda.synchronize()
        tc += e[0].elapsed_time(e[1])
        td += e[1].elapsed_time(e[2])
    dec.check()
    if b.error_flag():
        raise pc.PcompError(pc.EHIP, "autotune: device error word %d" % b.error_flag())
    nbytes = sum(s.numel() * s.element_size() for s in segs)
    ratio = nbytes / max(1, b.total_bytes())
    del g
    return tc / reps, td / reps, ratio


def choose_block_length(results, ratio_slack: float):
    """results: list of (L, compress ms, decompress ms, ratio). Keeps the candidates with a
    ratio >= (1 - ratio_slack) * best ratio and returns the fastest of them (ties: larger
    ratio, then smaller L)."""
    best = max(r[3] for r in results)
    ok = [r for r in results if r[3] >= (1.0 - ratio_slack) * best]
    return min(ok, key=lambda r: (r[1] + r[2], -r[3], r[0]))[0]


def choose_grid(results):
    """results: list of (grid, compress ms, decompress ms). Fastest; ties to the smaller grid."""
    return min(results, key=lambda r: (r[1] + r[2], r[0]))[0]


def autotune(segments, variant: int = 0, ratio_slack: float = 0.01, reps: int = 3, use_cache: bool = True,
             max_segments: int = 64, verbose: bool = False) -> dict:
    """Returns {"block_len": (L_u8, L_u16, L_u32), "grid": g, "signature": ..., "log": [...]}."""
    sig = signature(segments, variant)
    path = cache_path()
    if use_cache:
        hit = _load_cache(path).get(sig)
        if hit:
            hit = dict(hit)
            hit["block_len"] = tuple(hit["block_len"])
            hit["cached"] = True
            return hit
    sample = sample_segments(segments, max_segments)
    log = []
    chosen = [1024, 1024, 1024]
    for grp in range(3):
        segs = [s for s in sample if _GROUP_OF[s.element_size()] == grp and s.numel() > 0]
        if not segs:
            continue
        res = []
        for L in CANDIDATE_L:
            bl = [1024, 1024, 1024]
            bl[grp] = L
            tc, td, r = _time_batch(segs, tuple(bl), variant, 0, reps)
            res.append((L, tc, td, r))
            log.append({"group": grp, "L": L, "compress_ms": tc, "decompress_ms": td, "ratio": r})
            if verbose:
                print("tune: width %d L=%d compress %.3f ms decompress %.3f ms ratio %.4f" % (
                    (1, 2, 4)[grp], L, tc, td, r), flush=True)
        chosen[grp] = choose_block_length(res, ratio_slack)
    gres = []
    live = [s for s in sample if s.numel() > 0]
    if live:
        for grid in CANDIDATE_GRID:
            tc, td, r = _time_batch(live, tuple(chosen), variant, grid, reps)
            gres.append((grid, tc, td))
            log.append({"grid": grid, "compress_ms": tc, "decompress_ms": td, "ratio": r})
            if verbose:
                print("tune: grid %d compress %.3f ms decompress %.3f ms" % (grid, tc, td), flush=True)
    grid = choose_grid(gres) if gres else 0
    result = {"block_len": tuple(chosen), "grid": grid, "signature": sig, "log": log, "cached": False}
    if use_cache:
        cache = _load_cache(path)
        cache[sig] = {"block_len": list(chosen), "grid": grid, "signature": sig, "log": log}
        _store_cache(path, cache)
    return result
