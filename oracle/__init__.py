"""CPU oracle for the blocked polynomial compressor (arXiv:1805.01844).

TEST INFRASTRUCTURE. Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path
(``paper_1805_01844_amd``) never imports it and shares no code with it.

``pcomp_oracle.c`` holds the arithmetic (exact integers, hardware division);
this module only marshals numpy arrays into it through ctypes. ``mlp.py`` holds
the float64 reference forward/backward of the block-class network.

Parity status: every function here is pinned by the ``-m "not gpu"`` tests
(closed forms, the paper's Eq. (1), the paper's Sec. 4.2 ratios, brute force over
tiny inputs, an independent bit packer, round trips); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcomp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SELECT_EXHAUSTIVE = 0x100
SELECT_LEARNED = 0x200
U64_MAX = (1 << 64) - 1

_lib = None


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc -O2 (plain scalar C, no intrinsics)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        u64, i64, c_int, u32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32
        vp = ctypes.c_void_p
        L.orc_digits_per_word.restype = c_int
        L.orc_digits_per_word.argtypes = [u64, c_int]
        for f in (L.orc_basic_words, L.orc_adv_words):
            f.restype = u64
            f.argtypes = [u64, u64, c_int]
        L.orc_adv_schedule.restype = u64
        L.orc_adv_schedule.argtypes = [u64, u64, c_int, vp, vp, vp, vp, u64]
        L.orc_family_words.restype = u64
        L.orc_family_words.argtypes = [c_int, u64, u64, c_int]
        L.orc_family_pack.restype = u64
        L.orc_family_pack.argtypes = [c_int, vp, u64, u64, c_int, vp]
        L.orc_family_unpack.restype = None
        L.orc_family_unpack.argtypes = [c_int, vp, u64, u64, c_int, vp]
        L.orc_class_valid.restype = c_int
        L.orc_class_valid.argtypes = [c_int, u64]
        L.orc_class_words.restype = u64
        L.orc_class_words.argtypes = [c_int, vp, u64, u64, vp]
        L.orc_class_pack.restype = u64
        L.orc_class_pack.argtypes = [c_int, vp, u64, u64, vp, vp]
        L.orc_class_unpack.restype = None
        L.orc_class_unpack.argtypes = [c_int, vp, u64, u64, u64, vp]
        L.orc_tile_blocks.restype = u32
        L.orc_tile_blocks.argtypes = [u32, c_int]
        L.orc_bound.restype = u64
        L.orc_bound.argtypes = [u64, c_int, u32, c_int]
        L.orc_compress.restype = i64
        L.orc_compress.argtypes = [vp, u64, c_int, u32, c_int, vp, vp, u64]
        L.orc_decompress.restype = i64
        L.orc_decompress.argtypes = [vp, u64, vp, u64]
        L.orc_stream_info.restype = c_int
        L.orc_stream_info.argtypes = [vp, u64, vp, vp, vp, vp]
        L.orc_block_facts.restype = c_int
        L.orc_block_facts.argtypes = [vp, u64, c_int, u32, c_int, vp, vp, vp, vp, vp, vp]
        L.orc_all_class_words.restype = None
        L.orc_all_class_words.argtypes = [vp, u64, u64, vp, vp]
        L.orc_set_model.restype = c_int
        L.orc_set_model.argtypes = [vp, u64]
        L.orc_block_features.restype = None
        L.orc_block_features.argtypes = [vp, u64, u64, u64, vp]
        L.orc_mlp_scores.restype = None
        L.orc_mlp_scores.argtypes = [vp, vp, vp]
        L.orc_mlp_predict.restype = c_int
        L.orc_mlp_predict.argtypes = [vp, vp]
        L.orc_features.restype = c_int
        L.orc_features.argtypes = [vp, u64, c_int, u32, vp, vp]
        L.orc_bound32.restype = u64
        L.orc_bound32.argtypes = [u64, c_int, u32, c_int]
        L.orc_compress32.restype = i64
        L.orc_compress32.argtypes = [vp, u64, c_int, u32, c_int, vp, u64]
        L.orc_decompress32.restype = i64
        L.orc_decompress32.argtypes = [vp, u64, vp, u64]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


_WIDTH = {np.dtype(np.uint8): 1, np.dtype(np.uint16): 2, np.dtype(np.uint32): 4}
_DTYPE = {1: np.uint8, 2: np.uint16, 4: np.uint32}


# ---- building blocks -------------------------------------------------------

def digits_per_word(B: int, W: int = 64) -> int:
    """Sec. 3.1 Eq. (1), exact-integer reading: largest k with B^k <= 2^W."""
    return lib().orc_digits_per_word(B, W)


def basic_words(n: int, B: int, W: int = 64) -> int:
    return lib().orc_basic_words(n, B, W)


def adv_words(n: int, B: int, W: int = 64) -> int:
    """Number of words of the Sec. 3.2 series for n digits of base B."""
    return lib().orc_adv_words(n, B, W)


def adv_schedule(n: int, B: int, W: int = 64):
    """The Sec. 3.2 series: arrays p_i, R_i, R'_{i-1}, q_i for i = 1..m."""
    m = lib().orc_adv_words(n, B, W)
    arrs = [np.zeros(max(m, 1), dtype=np.uint64) for _ in range(4)]
    lib().orc_adv_schedule(n, B, W, *[_ptr(a) for a in arrs], m)
    return tuple(a[:m] for a in arrs)


def family_words(family: int, n: int, base: int, W: int = 64) -> int:
    return lib().orc_family_words(family, n, base, W)


def family_pack(family: int, digits, base: int, W: int = 64) -> np.ndarray:
    d = _u64(digits)
    out = np.zeros(max(d.size + 1, 1), dtype=np.uint64)
    nw = lib().orc_family_pack(family, _ptr(d), d.size, base, W, _ptr(out))
    return out[:nw]


def family_unpack(family: int, words, n: int, base: int, W: int = 64) -> np.ndarray:
    w = _u64(words)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_family_unpack(family, _ptr(w), n, base, W, _ptr(out))
    return out[:n]


def class_valid(cls: int, B: int) -> bool:
    return bool(lib().orc_class_valid(cls, B))


def class_words(cls: int, digits, B: int):
    """(words, n_e) of one block of digits in class cls."""
    d = _u64(digits)
    ne = np.zeros(1, dtype=np.uint64)
    nw = lib().orc_class_words(cls, _ptr(d), d.size, B, _ptr(ne))
    return int(nw), int(ne[0])


def class_pack(cls: int, digits, B: int):
    d = _u64(digits)
    out = np.zeros(d.size + 2, dtype=np.uint64)
    ne = np.zeros(1, dtype=np.uint64)
    nw = lib().orc_class_pack(cls, _ptr(d), d.size, B, _ptr(out), _ptr(ne))
    return out[:nw].copy(), int(ne[0])


def class_unpack(cls: int, words, n: int, B: int, ne: int) -> np.ndarray:
    w = _u64(words)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    lib().orc_class_unpack(cls, _ptr(w) if w.size else None, n, B, ne, _ptr(out))
    return out[:n]


def all_class_words(digits, B: int):
    d = _u64(digits)
    w = np.zeros(16, dtype=np.uint64)
    ne = np.zeros(16, dtype=np.uint64)
    lib().orc_all_class_words(_ptr(d), d.size, B, _ptr(w), _ptr(ne))
    return w, ne


def tile_blocks(L: int, w: int) -> int:
    return lib().orc_tile_blocks(L, w)


# ---- streams -------------------------------------------------------------------

def bound(n: int, w: int, L: int, variant: int) -> int:
    return lib().orc_bound(n, w, L, variant)


def compress(x: np.ndarray, L: int, variant: int, forced: np.ndarray | None = None) -> bytes:
    """Whole-stream compression of a 1-D u8/u16/u32 array."""
    x = np.ascontiguousarray(x)
    w = _WIDTH[x.dtype]
    cap = bound(x.size, w, L, variant)
    if cap == 0:
        raise ValueError("invalid arguments")
    out = np.zeros(cap, dtype=np.uint8)
    f = None
    if forced is not None:
        f = np.ascontiguousarray(np.asarray(forced, dtype=np.uint8))
    rc = lib().orc_compress(_ptr(x), x.size, w, L, variant, _ptr(f) if f is not None else None, _ptr(out), cap)
    if rc < 0:
        raise ValueError("oracle compress failed: %d" % rc)
    return out[:rc].tobytes()


def stream_info(stream: bytes):
    buf = np.frombuffer(stream, dtype=np.uint8)
    n = ctypes.c_uint64()
    w = ctypes.c_int()
    L = ctypes.c_uint32()
    tot = ctypes.c_uint64()
    rc = lib().orc_stream_info(_ptr(buf), buf.size, ctypes.byref(n), ctypes.byref(w), ctypes.byref(L),
                               ctypes.byref(tot))
    if rc:
        raise ValueError("bad stream: %d" % rc)
    return n.value, w.value, L.value, tot.value


def decompress_rc(stream: bytes, out_cap: int | None = None):
    """Returns (rc, values) without raising; rc < 0 is an error code."""
    buf = np.frombuffer(stream, dtype=np.uint8)
    try:
        n, w, L, tot = stream_info(stream)
    except ValueError:
        return -3, None
    cap = n if out_cap is None else out_cap
    out = np.zeros(max(cap, 1), dtype=_DTYPE[w])
    rc = lib().orc_decompress(_ptr(buf), buf.size, _ptr(out), cap)
    return rc, (out[:n] if rc >= 0 else None)


def decompress(stream: bytes) -> np.ndarray:
    rc, out = decompress_rc(stream)
    if rc < 0:
        raise ValueError("oracle decompress failed: %d" % rc)
    return out


# ---- streams of 32-bit words ---------------------------------------------------------

def bound32(n: int, w: int, L: int, variant: int) -> int:
    return lib().orc_bound32(n, w, L, variant)


def compress32(x: np.ndarray, L: int, variant: int) -> bytes:
    """Stream of 32-bit words (variant 0, 8 or SELECT_EXHAUSTIVE) of a 1-D u8/u16/u32 array."""
    x = np.ascontiguousarray(x)
    w = _WIDTH[x.dtype]
    cap = bound32(x.size, w, L, variant)
    if cap == 0:
        raise ValueError("invalid arguments")
    out = np.zeros(cap, dtype=np.uint8)
    rc = lib().orc_compress32(_ptr(x), x.size, w, L, variant, _ptr(out), cap)
    if rc < 0:
        raise ValueError("oracle compress32 failed: %d" % rc)
    return out[:rc].tobytes()


def decompress32_rc(stream: bytes, out_cap: int | None = None):
    """Returns (rc, values) without raising; rc < 0 is an error code."""
    buf = np.frombuffer(stream, dtype=np.uint8)
    try:
        n, w, L, tot = stream_info(stream)
    except ValueError:
        return -3, None
    cap = n if out_cap is None else out_cap
    out = np.zeros(max(cap, 1), dtype=_DTYPE[w])
    rc = lib().orc_decompress32(_ptr(buf), buf.size, _ptr(out), cap)
    return rc, (out[:n] if rc >= 0 else None)


def decompress32(stream: bytes) -> np.ndarray:
    rc, out = decompress32_rc(stream)
    if rc < 0:
        raise ValueError("oracle decompress32 failed: %d" % rc)
    return out


def block_facts(x: np.ndarray, L: int, variant: int, forced=None):
    """Per-block min, B, class, n_e and word count as chosen by the oracle."""
    x = np.ascontiguousarray(x)
    w = _WIDTH[x.dtype]
    nb = (x.size + L - 1) // L
    arrs = dict(mins=np.zeros(max(nb, 1), np.uint64), B=np.zeros(max(nb, 1), np.uint64),
                cls=np.zeros(max(nb, 1), np.uint8), ne=np.zeros(max(nb, 1), np.uint64),
                words=np.zeros(max(nb, 1), np.uint64))
    f = None if forced is None else np.ascontiguousarray(np.asarray(forced, dtype=np.uint8))
    rc = lib().orc_block_facts(_ptr(x), x.size, w, L, variant, _ptr(f) if f is not None else None,
                               _ptr(arrs["mins"]), _ptr(arrs["B"]), _ptr(arrs["cls"]), _ptr(arrs["ne"]),
                               _ptr(arrs["words"]))
    if rc:
        raise ValueError("block_facts failed: %d" % rc)
    return {k: v[:nb] for k, v in arrs.items()}


# ---- learned selector (binary32, bit-exact definition) ---------------------------

MLP_IN, MLP_HID, MLP_OUT = 19, 64, 16
MLP_PARAMS = MLP_HID * MLP_IN + MLP_HID + MLP_OUT * MLP_HID + MLP_OUT


def set_model(params) -> None:
    """Loads the selector's 2320 parameters (None unloads)."""
    if params is None:
        lib().orc_set_model(None, 0)
        return
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    if lib().orc_set_model(_ptr(p), p.size) != 0:
        raise ValueError("model needs %d floats" % MLP_PARAMS)


def block_features(digits, vmin: int, vmax: int) -> np.ndarray:
    d = _u64(digits)
    x = np.zeros(MLP_IN, dtype=np.float32)
    lib().orc_block_features(_ptr(d), d.size, vmin, vmax, _ptr(x))
    return x


def features(x: np.ndarray, L: int, with_words: bool = True):
    """(features [n_blocks, 19] float32, class sizes [n_blocks, 16] uint64 or None) of an array."""
    x = np.ascontiguousarray(x)
    w = _WIDTH[x.dtype]
    nb = (x.size + L - 1) // L
    f = np.zeros((max(nb, 1), MLP_IN), dtype=np.float32)
    words = np.zeros((max(nb, 1), 16), dtype=np.uint64) if with_words else None
    rc = lib().orc_features(_ptr(x), x.size, w, L, _ptr(f), _ptr(words) if with_words else None)
    if rc:
        raise ValueError("features failed: %d" % rc)
    return f[:nb], (words[:nb] if with_words else None)


def mlp_scores(params, x) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    xs = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).reshape(-1, MLP_IN)
    out = np.zeros((xs.shape[0], MLP_OUT), dtype=np.float32)
    for i in range(xs.shape[0]):
        lib().orc_mlp_scores(_ptr(p), ctypes.c_void_p(xs.ctypes.data + 4 * MLP_IN * i),
                             ctypes.c_void_p(out.ctypes.data + 4 * MLP_OUT * i))
    return out


def mlp_predict(params, x) -> np.ndarray:
    s = mlp_scores(params, x)
    return np.argmax(s, axis=1).astype(np.uint8)  # first index of the maximum
