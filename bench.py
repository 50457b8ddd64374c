"""Benchmark of the polynomial compressor on one MI355X.

One step = the whole hot path over one batch: compress (block min/max, class choice,
placement, packing) and decompress (unpacking) of camera-shaped synthetic waveforms,
10,000 events x 1855 pixels x 40 samples of u16 (1.484 GB), one block per pixel trace
(block_len = 40), per-block exhaustive choice over the 16 classes. Inputs are resident in
HBM before timing starts. After the timed steps the round trip is checked bit for bit.

Prints ONE JSON line. `value` is round-trip throughput: uncompressed bytes per step over
(compress + decompress) time; compress and decompress GB/s are reported separately. Extra legs
in the same line (each can be switched off): the 50,000-event batch with plain, exhaustive and
learned selection, the 4 GiB stress batch, the 2^20-value latency case, time-major blocking,
the integrated-signal workload, Poly + LZMA, the CPU oracle on 1 and all host threads, and
the paper's own CPU figures as context.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E

# The paper's measurements (Sec. 4.3, Tables 1 and 2): context, on a laptop CPU, not targets.
PAPER_REFERENCE = {
    "note": "the paper's CPU figures (Sec. 4.3.1 Table 1 and Sec. 4.3.2 Table 2); MB/s = input bytes / time",
    "table1_waveforms": {
        "data": "CTA Prod3 run 3998 full waveforms, u16, 7.6 GB", "cpu": "Intel core i7 M 560, 19 GB RAM, Fedora",
        "advanced_polynomial": {"ratio": 2.71, "compress_s_ram": 176.0, "decompress_s_ram": 150.0,
                                "compress_MBps_ram": 43.2, "decompress_MBps_ram": 50.7},
        "lzma_mx9": {"ratio": 6.52, "compress_s_ram": 7424.0},
        "lzma_mx1": {"ratio": 5.88, "compress_s_ram": 942.0},
        "poly_lzma": {"ratio": 5.02, "compress_s_ram": 297.0},
    },
    "table2_integrated": {
        "data": "CTA Prod3 run 497 integrated signal, 24/32-bit, 474 MB",
        "cpu": "Intel core i5 M 560, 8 GB RAM, Ubuntu 16.4",
        "advanced_polynomial": {"ratio": 3.74, "compress_s_ram": 0.9, "decompress_s_ram": 0.9,
                                "compress_MBps_ram": 527.0, "decompress_MBps_ram": 527.0},
        "lzma_7z": {"ratio": 4.84, "compress_s_ram": 78.0},
        "poly_lzma": {"ratio": 4.84, "compress_s_elapsed": 24.6},
    },
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--events", type=int, default=10000)
    ap.add_argument("--variant", default="exhaustive", help="exhaustive | learned | class id 0..15")
    ap.add_argument("--block-len", type=int, default=40)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target CPU work of each baseline sample")
    ap.add_argument("--batch-events", type=int, default=50000,
                    help="uneven events in the batched leg (0 skips it)")
    ap.add_argument("--stress-bytes", type=float, default=float(1 << 32),
                    help="bytes of the stress decompression leg (0 skips it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the latency, time-major, 32-bit-word, integrated and Poly+LZMA legs")
    ap.add_argument("--extras", default="latency,time_major,words32,integrated,poly_lzma",
                    help="which of those legs to run (comma list)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device three times (reference for the HBM byte counters)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1805_01844_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch from the committed counter summary, if taken on the current kernels."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["hbm_bytes_per_launch"]  # FETCH x calibration + WRITE x calibration


# A GPU machine gives each GPU a share of 16 host cores, whatever the machine's count is.
HOST_CORE_SHARE = 16


def host_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    return max(1, min(HOST_CORE_SHARE, avail))


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(x_host_events, variant: int, L: int, seconds: float):
    """The CPU oracle as it stands, on a bounded sample of the same workload, one stream per
    event, on 1 host thread and on all host threads (ctypes releases the GIL)."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    oracle.lib()
    model, nproc = host_cpu()
    share = host_threads()
    ev = x_host_events

    def work(a):
        st = oracle.compress(a, L, variant)
        b = oracle.decompress(st)
        assert np.array_equal(a, b)
        return len(st)

    t0 = time.perf_counter()
    work(ev[0].reshape(-1))
    per_event = time.perf_counter() - t0
    res = {"kind": "oracle", "unit": "GB/s", "cpu_model": model, "nproc": nproc,
           "threads_note": "all_threads = the host cores this process may use, at most the 16-core share "
                           "a GPU box gives one GPU"}
    for name, threads in (("one_thread", 1), ("all_threads", share)):
        n_ev = int(max(threads, seconds * threads / max(per_event, 1e-6)))
        chunks = [ev[i % len(ev)].reshape(-1) for i in range(n_ev)]
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as pool:
            sizes = list(pool.map(work, chunks))
        dt = time.perf_counter() - t0
        nbytes = sum(c.nbytes for c in chunks)
        res[name] = {"value": nbytes / dt / 1e9, "cores": threads,
                     "sample": "%d events cycled from the first %d of the workload (%.1f MB), compress+decompress "
                               "round trip, one stream per event" % (n_ev, len(ev), nbytes / 1e6),
                     "ratio": nbytes / sum(sizes)}
    # the contract's fields: the all-threads figure
    res["value"] = res["all_threads"]["value"]
    res["cores"] = share
    res["sample"] = res["all_threads"]["sample"]
    return res


def _events(n):
    import torch

    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def _time_pair(comp_fn, dec_fn, reps):
    """Mean device time (s) of comp_fn and dec_fn over reps, timed with events on the current
    stream (where the library launches) after one untimed call of each."""
    import torch

    comp_fn()
    dec_fn()
    torch.cuda.synchronize()
    ev = _events(3 * reps)
    for r in range(reps):
        ev[3 * r].record()
        comp_fn()
        ev[3 * r + 1].record()
        dec_fn()
        ev[3 * r + 2].record()
    torch.cuda.synchronize()
    tc = sum(ev[3 * r].elapsed_time(ev[3 * r + 1]) for r in range(reps)) / reps / 1e3
    td = sum(ev[3 * r + 1].elapsed_time(ev[3 * r + 2]) for r in range(reps)) / reps / 1e3
    return tc, td


def _roofline(alg_bytes, seconds):
    a = alg_bytes / seconds / 1e9
    return {"bound": "hbm", "achieved": round(a, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(a / PEAK_HBM_GBPS, 4), "algorithmic_bytes": int(alg_bytes)}


def _weighted_sums(segs, weights):
    """Per segment: sum of byte_i * w_i in wrapping 64-bit arithmetic (w: fixed random words)."""
    import torch

    return torch.stack([(s.view(torch.uint8).to(torch.int64) * weights[:s.numel() * s.element_size()]).sum()
                        for s in segs])


def batch_leg(n_events: int, reps: int):
    """Uneven camera events (shapes 1855x40, 2048x96, 11328x128; u16 or u32; noise sigma U(2,20);
    pulse fraction U(0,5%)) as one batch: block lengths and grid from the autotuner, the
    compression captured in one HIP graph, per-block class by the plain method (class 0), by
    exhaustive search, and by the shipped learned selector (on the exhaustive leg's block lengths
    and grid). The streams are written back to back
    (one file, offsets on the device). At 50,000 events the input is ~86 GB, so decompression
    writes back into the input tensors: after the timed runs every segment is overwritten with
    0x5A, decoded once more, and its weighted 64-bit byte sum compared with the one taken before
    the first compression."""
    import torch

    import datagen
    import paper_1805_01844_amd as pc
    from paper_1805_01844_amd import learn, tune

    segs = [e.reshape(-1) for e in datagen.uneven_events(n_events, seed=3, device="cuda")]
    torch.cuda.synchronize()
    nbytes = sum(s.numel() * s.element_size() for s in segs)
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    longest = max(s.numel() * s.element_size() for s in segs)
    weights = torch.randint(-(1 << 62), 1 << 62, (longest,), generator=g, device="cuda", dtype=torch.int64)
    ref = _weighted_sums(segs, weights)
    learn.use_selector()
    res = {"workload": "%d uneven camera events, %.3f GB (u16 and u32 mixed)" % (n_events, nbytes / 1e9)}
    tuned = {}
    for name, v in (("plain", 0), ("exhaustive", pc.SELECT_EXHAUSTIVE), ("learned", pc.SELECT_LEARNED)):
        # the learned selector runs on the exhaustive leg's stream configuration (block lengths and
        # grid), so that its ratio loss is the selector's alone
        t = tuned["exhaustive"] if name == "learned" else tune.autotune(segs, v)
        tuned[name] = t
        b = pc.Batch(segs, block_len=t["block_len"], variant=v, grid=t["grid"])
        gr = b.capture()
        dec = pc.BatchDecoder(b, segs, grid=t["grid"])
        tc, td = _time_pair(gr.replay, dec, reps)
        dec.check()
        total = b.total_bytes()
        for s in segs:
            s.view(torch.uint8).fill_(0x5A)  # the check decode must replace every byte
        dec()
        dec.check()
        ok = bool(torch.equal(_weighted_sums(segs, weights), ref))
        assert ok and b.error_flag() == 0, "batched round trip failed (%s)" % name
        alg = nbytes + total
        res[name] = {"block_len": list(t["block_len"]), "grid": t["grid"], "ratio": round(nbytes / total, 4),
                     "file_bytes": total, "compress_GBps": round(nbytes / tc / 1e9, 1),
                     "decompress_GBps": round(nbytes / td / 1e9, 1), "roundtrip_bit_exact": True,
                     "roofline_compress": _roofline(alg, tc), "roofline_decompress": _roofline(alg, td)}
        del gr, b, dec
        torch.cuda.empty_cache()
    pc.set_model(None)
    ex, le = res["exhaustive"], res["learned"]
    res["learned_ratio_loss_vs_exhaustive"] = round(1 - le["ratio"] / ex["ratio"], 5)
    res["learned_ratio_gain_vs_plain"] = round(le["ratio"] / res["plain"]["ratio"] - 1, 5)
    res["learned_compress_speed_vs_exhaustive"] = round(le["compress_GBps"] / ex["compress_GBps"], 4)
    return res


def stress_leg(total_bytes: int, reps: int):
    """Thirds of u8/u16/u32 stress blocks (Laplacian noise, 0.1% full-range outliers, constant and
    full-range blocks; L = 1024) plus one u32 block for every base 2..2^16, as one batch; the
    decompression is the heavy side. The final check decodes into buffers first filled with
    0x5A."""
    import torch

    import datagen
    import paper_1805_01844_amd as pc

    L = 1024
    segs = []
    for k, dt in enumerate((torch.uint8, torch.uint16, torch.uint32)):
        w = torch.tensor([], dtype=dt).element_size()
        nblk = total_bytes // 3 // (L * w)
        out = torch.empty(nblk * L, dtype=dt, device="cuda")
        step = (256 << 20) // (L * w)
        for c, b0 in enumerate(range(0, nblk, step)):
            nb = min(step, nblk - b0)
            out[b0 * L:(b0 + nb) * L] = datagen.laplace_blocks(nb, L, dt, seed=90 + 1000 * k + c, device="cuda",
                                                               outlier_rate=1e-3).reshape(-1)
        segs.append(out)
    segs.append(datagen.base_sweep_u32(L=L, device="cuda"))
    torch.cuda.synchronize()
    nbytes = sum(s.numel() * s.element_size() for s in segs)
    outs = [torch.empty_like(s) for s in segs]
    res = {"workload": "%.3f GB: u8/u16/u32 stress blocks + base sweep 2..65536, L=1024" % (nbytes / 1e9)}
    for name, v in (("plain", 0), ("exhaustive", pc.SELECT_EXHAUSTIVE)):
        b = pc.Batch(segs, block_len=L, variant=v)
        dec = pc.BatchDecoder(b, outs)
        tc, td = _time_pair(b.compress, dec, reps)
        for o in outs:
            o.view(torch.uint8).fill_(0x5A)
        dec()
        dec.check()
        ok = all(torch.equal(a.view(torch.uint8), c.view(torch.uint8)) for a, c in zip(segs, outs))
        assert ok and b.error_flag() == 0, "stress round trip failed (%s)" % name
        total = b.total_bytes()
        alg = nbytes + total
        res[name] = {"ratio": round(nbytes / total, 4), "compress_GBps": round(nbytes / tc / 1e9, 1),
                     "decompress_GBps": round(nbytes / td / 1e9, 1), "roundtrip_bit_exact": True,
                     "max_stream_offset": max(b.offsets()),
                     "roofline_compress": _roofline(alg, tc), "roofline_decompress": _roofline(alg, td)}
        del b, dec
    return res


def latency_leg(reps: int = 50):
    """The tiny case: 2^20 u16 values round(N(300, 4^2)), blocks of 1024, basic packing (class 0):
    2 MiB sits in the caches, so this measures the latency of one call, not bandwidth."""
    import numpy as np
    import torch

    import datagen
    import paper_1805_01844_amd as pc

    x = datagen.tiny_gaussian(device="cuda")
    comp = pc.Compressor(x.numel(), torch.uint16, 1024, 0, device="cuda")
    comp(x)
    n = int(comp.size.item())
    s = comp.out[:n]
    out = torch.empty_like(x)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    tcs, tds = [], []
    ev = _events(3)
    for _ in range(reps):
        ev[0].record()
        comp(x)
        ev[1].record()
        pc.decompress_into(s, out, st, dtype_bytes=2, block_len=1024)
        ev[2].record()
        torch.cuda.synchronize()
        tcs.append(ev[0].elapsed_time(ev[1]))
        tds.append(ev[1].elapsed_time(ev[2]))
    assert int(st.item()) == 0 and torch.equal(out.view(torch.int16), x.view(torch.int16))
    return {"workload": "2^20 u16 round(N(300, 4^2)), L=1024, class 0", "ratio": round(x.numel() * 2 / n, 4),
            "compress_ms_median": round(float(np.median(tcs)), 4), "decompress_ms_median": round(float(np.median(tds)), 4),
            "roundtrip_bit_exact": True}


def time_major_leg(x, L: int, variant: int, reps: int = 5):
    """The camera workload blocked along time rows (the transpose of every event, read column
    by column on the GPU) beside the pixel-trace blocking of the headline."""
    import torch

    import paper_1805_01844_amd as pc

    nbytes = x.numel() * 2
    comp = pc.CompressorTransposed(x.shape, x.dtype, L, variant, device="cuda")
    comp(x)
    s = comp.stream()
    out = torch.full_like(x, 0x5A5A)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    tc, td = _time_pair(lambda: comp(x), lambda: pc.decompress_transposed_into(s, out, st, L), reps)
    assert comp.error_flag() == 0 and int(comp.size.item()) == s.numel()
    out.fill_(0x5A5A)
    pc.decompress_transposed_into(s, out, st, L)
    assert int(st.item()) == 0 and torch.equal(out.view(torch.int16), x.view(torch.int16))
    alg = nbytes + s.numel()
    return {"workload": "same camera events, blocks of %d along time rows (M_ij = time i of pixel j)" % L,
            "ratio": round(nbytes / s.numel(), 4), "compress_GBps": round(nbytes / tc / 1e9, 1),
            "decompress_GBps": round(nbytes / td / 1e9, 1), "roundtrip_bit_exact": True,
            "roofline_compress": _roofline(alg, tc), "roofline_decompress": _roofline(alg, td)}


def words32_leg(x, L: int, reps: int = 10):
    """Streams of 32-bit words (the paper's unsigned int: Sec. 3.1 and 3.2 with capacity 2^32) of
    the camera workload, basic, advanced and the smaller of the two per block, beside the
    64-bit streams (their ratio for the same variants)."""
    import torch

    import paper_1805_01844_amd as pc

    xf = x.reshape(-1)
    n = xf.numel()
    nbytes = n * 2
    out = torch.empty_like(xf)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = {"workload": "same camera events, blocks of %d, payload of 32-bit words" % L}
    for name, v in (("basic", 0), ("advanced", 8), ("exhaustive", pc.SELECT_EXHAUSTIVE)):
        comp = pc.Compressor32(n, torch.uint16, L, v, device="cuda")
        comp(xf)
        sl = int(comp.size.item())
        s = comp.out[:sl]
        tc, td = _time_pair(lambda: comp(xf), lambda: pc.decompress32_into(s, out, st, L), reps)
        assert comp.error_flag() == 0 and int(comp.size.item()) == sl
        out.fill_(0x5A5A)
        pc.decompress32_into(s, out, st, L)
        assert int(st.item()) == 0 and torch.equal(out.view(torch.int16), xf.view(torch.int16))
        c64 = pc.Compressor(n, torch.uint16, L, v, device="cuda")
        c64(xf)
        r64 = nbytes / int(c64.size.item())
        del c64
        alg = nbytes + sl
        res[name] = {"ratio": round(nbytes / sl, 4), "ratio_64bit_words": round(r64, 4),
                     "compress_GBps": round(nbytes / tc / 1e9, 1), "decompress_GBps": round(nbytes / td / 1e9, 1),
                     "roundtrip_bit_exact": True, "roofline_compress": _roofline(alg, tc),
                     "roofline_decompress": _roofline(alg, td)}
        del comp, s
        torch.cuda.empty_cache()
    return res


def integrated_leg(x, reps: int = 10):
    """Integrated signal (Sec. 4.3.2): per-pixel sums of the camera events made on the GPU (u32),
    then compressed one event per block (L = 1855) with exhaustive choice."""
    import torch

    import paper_1805_01844_amd as pc

    sums = pc.integrate(x).reshape(-1)
    n = sums.numel()
    comp = pc.Compressor(n, torch.uint32, 1855, pc.SELECT_EXHAUSTIVE, device="cuda")
    comp(sums)
    sl = int(comp.size.item())
    s = comp.out[:sl]
    out = torch.empty_like(sums)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    tc, td = _time_pair(lambda: comp(sums), lambda: pc.decompress_into(s, out, st, dtype_bytes=4, block_len=1855),
                        reps)
    assert int(st.item()) == 0 and torch.equal(out.view(torch.int32), sums.view(torch.int32))
    nbytes = n * 4
    return {"workload": "%d per-pixel sums (u32) of the camera events, one event per block (L=1855), exhaustive"
                        % n, "ratio": round(nbytes / sl, 4), "compress_GBps": round(nbytes / tc / 1e9, 1),
            "decompress_GBps": round(nbytes / td / 1e9, 1), "roundtrip_bit_exact": True}


def poly_lzma_leg(x_events, L: int, variant: int, batch_events: int = 64):
    """Poly + LZMA (Sec. 4.3.1 Table 1, Sec. 4.3.2 Table 2): LZMA on the host (liblzma through
    Python's lzma, fast settings of the paper's 7z runs, on all host threads) over the raw
    values, against LZMA over the GPU's polynomial stream (GPU time + host LZMA time), on a
    sample of camera events and of uneven events. Both legs split their input into members the
    same way (enough for every thread, 256 KB to 4 MB each)."""
    import torch

    import datagen
    import paper_1805_01844_amd as pc
    from paper_1805_01844_amd import polylzma

    threads = host_threads()

    def one(name, tensors, block_len):
        raw = b"".join(t.cpu().view(torch.uint8).numpy().tobytes() for t in tensors)
        t0 = time.perf_counter()
        a = polylzma.lzma_pack(raw, "fast", threads)
        t_lzma = time.perf_counter() - t0
        dev = [t.cuda() for t in tensors]
        b = pc.Batch(dev, block_len=block_len, variant=variant)
        b.compress()  # first call: plan upload and tables
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.compress()
        f = b.file()
        torch.cuda.synchronize()
        t_gpu = time.perf_counter() - t0
        t1 = time.perf_counter()
        blob = polylzma.compress(f, "fast", threads)
        t_host = time.perf_counter() - t1
        back = polylzma.decompress(blob, device="cuda")
        outs = [torch.empty_like(d) for d in dev]
        dec = pc.BatchDecoder(b, outs)
        dec(back)
        dec.check()
        assert all(torch.equal(o.view(torch.uint8), d.view(torch.uint8)) for o, d in zip(outs, dev))
        mb = len(raw) / 1e6
        return {"sample": name, "MB": round(mb, 1), "lzma_ratio": round(len(raw) / len(a), 4),
                "lzma_MBps": round(mb / t_lzma, 1), "lzma_chunk_KB": polylzma.chunk_for(len(raw), threads) >> 10,
                "poly_ratio": round(len(raw) / f.numel(), 4),
                "poly_lzma_ratio": round(len(raw) / len(blob), 4),
                "poly_lzma_MBps": round(mb / (t_gpu + t_host), 1), "gpu_stage_ms": round(1e3 * t_gpu, 2),
                "poly_lzma_chunk_KB": polylzma.chunk_for(f.numel(), threads) >> 10,
                "speedup_vs_lzma": round(t_lzma / (t_gpu + t_host), 2), "roundtrip_bit_exact": True}

    cam = [e.reshape(-1) for e in x_events]
    unev = [e.reshape(-1) for e in datagen.uneven_events(batch_events, seed=3)]
    return {"lzma": "liblzma (Python lzma), LZMA2 preset 1, nice_len 64, dict 32 MB or the member size "
                    "(the paper's fast 7z settings), on %d host threads" % threads,
            "camera": one("%d camera events" % len(cam), cam, (L, L, L)),
            "uneven": one("%d uneven events" % batch_events, unev, (1024, 1024, 1024))}


def main():
    args = parse()
    if args.copy_calibration:
        import torch

        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on a single MI355X (--gpus 1).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import datagen
    import paper_1805_01844_amd as pc

    variant = {"exhaustive": pc.SELECT_EXHAUSTIVE, "learned": pc.SELECT_LEARNED}.get(args.variant)
    if variant is None:
        variant = int(args.variant)
    L = args.block_len
    dev = torch.device("cuda:0")
    pc.init()
    x = datagen.camera_events(args.events, seed=1, device=dev)
    torch.cuda.synchronize()
    xf = x.reshape(-1)
    n = xf.numel()
    nbytes = n * 2
    comp = pc.Compressor(n, torch.uint16, L, variant, device=dev)
    out = torch.empty(n, dtype=torch.uint16, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    # one untimed pass to learn the stream size
    comp(xf)
    stream_len = int(comp.size.item())
    stream = comp.out[:stream_len]

    def decode():
        pc.decompress_into(stream, out, status, dtype_bytes=2, block_len=L)

    ev = _events(3 * args.steps)
    for i in range(args.warmup):
        comp(xf)
        decode()
    torch.cuda.synchronize()
    t_c, t_d = [], []
    wall0 = time.perf_counter()
    for i in range(args.steps):
        e0, e1, e2 = ev[3 * i], ev[3 * i + 1], ev[3 * i + 2]
        e0.record()
        comp(xf)
        e1.record()
        decode()
        e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    for i in range(args.steps):
        t_c.append(ev[3 * i].elapsed_time(ev[3 * i + 1]) / 1e3)
        t_d.append(ev[3 * i + 1].elapsed_time(ev[3 * i + 2]) / 1e3)
    tc, td = float(np.mean(t_c)), float(np.mean(t_d))
    # checks after the timed region: bit-exact round trip (into a buffer overwritten first), stable size
    assert int(status.item()) == 0, "decompress status %d" % int(status.item())
    assert int(comp.size.item()) == stream_len and comp.error_flag() == 0
    out.fill_(0x5A5A)
    decode()
    assert int(status.item()) == 0
    assert torch.equal(out.view(torch.int16), xf.view(torch.int16)), "round trip is not bit-exact"

    comp_gbps = nbytes / tc / 1e9
    dec_gbps = nbytes / td / 1e9
    value = nbytes / (tc + td) / 1e9
    ratio = nbytes / stream_len
    # Roofline of the decompression kernel: the pcomp_decompress_typed call is that one kernel
    # (plus a 4-byte status reset), timed live above on the stream it is launched on; its
    # algorithmic bytes are the stream it reads plus the values it writes. Compression is a
    # pipeline of launches (statistics, scan, placement, packing) and is reported as a whole.
    kern = "decompress_kernel<2, false, false>"
    alg = stream_len + nbytes
    roof = _roofline(alg, td)
    roof.update({"kernel": kern, "traffic": traffic_from_profiles(kern), "launch_ms": round(td * 1e3, 4),
                 "algorithmic_bytes_per_launch": alg})
    comp_alg = nbytes + stream_len
    res = {
        "metric": "compress/decompress GB/s on 1 MI355X, bit-exact round-trip; compression ratio",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((tc + td) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": "camera waveforms: %d events x 1855 px x 40 samples u16 (%.3f GB), block = one pixel "
                        "trace (L=%d), %s class choice" % (args.events, nbytes / 1e9, L, args.variant),
            "events": args.events, "block_len": L, "variant": args.variant,
        },
        "compress_GBps": round(comp_gbps, 2),
        "decompress_GBps": round(dec_gbps, 2),
        "ratio": round(ratio, 4),
        "stream_bytes": stream_len,
        "roundtrip_bit_exact": True,
        "wall_s_timed": round(wall, 4),
        "roofline": roof,
        "compress_pipeline": dict(_roofline(comp_alg, tc), ms=round(tc * 1e3, 4),
                                  launches="prep_kernel, stats_kernel, scan_sums_kernel, scan_prefix_kernel, "
                                           "place_kernel, pack_kernel"),
        "paper_reference": PAPER_REFERENCE,
    }
    extras = set() if args.no_extras else set(args.extras.split(","))
    if "latency" in extras:
        res["latency_tiny"] = latency_leg()
    if "time_major" in extras:
        res["time_major"] = time_major_leg(x, L, variant)
    if "words32" in extras:
        res["words32"] = words32_leg(x, L)
    if "integrated" in extras:
        res["integrated"] = integrated_leg(x)
    if "poly_lzma" in extras:
        res["poly_lzma"] = poly_lzma_leg([e for e in x[:400].cpu()], L, variant)
    del comp, out, stream
    torch.cuda.empty_cache()
    xe = x[: min(args.events, 256)].cpu().view(torch.int16).numpy().view(np.uint16)
    del x, xf
    torch.cuda.empty_cache()
    if args.batch_events > 0:
        res["batched"] = batch_leg(args.batch_events, reps=5)
    if args.stress_bytes > 0:
        res["stress"] = stress_leg(int(args.stress_bytes), reps=5)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(xe, variant if variant != pc.SELECT_LEARNED else 0x100, L,
                                           args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
