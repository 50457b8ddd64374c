"""Independent pure-Python big-integer reference for tiny blocks.

Written separately from the C oracle (no shared code, different style): every
quantity is an exact Python integer, the search for p_i tries every exponent,
and word values are explicit power sums rather than Horner loops. Only used on
tiny inputs (a few digits).
"""
from __future__ import annotations


def k_of(B: int, W: int = 64) -> int:
    """Largest k with B**k <= 2**W (Sec. 3.1 Eq. (1), exact-integer reading)."""
    k = 0
    while B ** (k + 1) <= 2 ** W:
        k += 1
    return k


def basic_encode(d, B: int, W: int = 64):
    if B <= 1 or not d:
        return []
    k = k_of(B, W)
    out = []
    for j in range(0, len(d), k):
        chunk = list(d[j:j + k]) + [0] * (k - len(d[j:j + k]))
        out.append(sum(v * B ** (k - 1 - i) for i, v in enumerate(chunk)))
    return out


def adv_plan(n: int, B: int, W: int = 64):
    """List of (q, p, R, Rprev) for the Sec. 3.2 series, stopping rule q_m + p_m >= n."""
    if B <= 1 or n == 0:
        return []
    plan = []
    Rprev, q = 1, 0
    while True:
        p = max(pp for pp in range(0, 65) if Rprev * B ** pp <= 2 ** W)
        R = 2 ** W // (Rprev * B ** p)
        plan.append((q, p, R, Rprev))
        if q + p >= n:
            return plan
        Rprev = -(-B // R)
        q = q + p + 1


def adv_encode(d, B: int, W: int = 64):
    n = len(d)
    get = lambda i: d[i] if i < n else 0  # noqa: E731
    words, rprime = [], 0
    for (q, p, R, _Rprev) in adv_plan(n, B, W):
        x = get(q + p)
        r = x % R
        body = sum(get(q + k) * B ** (p - 1 - k) for k in range(p)) + rprime * B ** p
        words.append(r + R * body)
        rprime = x // R
    return words


def family_encode(family: int, d, B: int, W: int = 64):
    return adv_encode(d, B, W) if family else basic_encode(d, B, W)


def class_encode(cls: int, d, B: int):
    """(words, n_e) of the threshold/excess class cls = 8*family + t."""
    family, t = cls >> 3, cls & 7
    if t == 0:
        return family_encode(family, d, B), 0
    beta = (B - 1).bit_length()
    assert t <= beta
    T = 2 ** (beta - t)
    main = [min(v, T) for v in d]
    exc = [v - T for v in d if v >= T]
    return family_encode(family, main, T + 1) + family_encode(family, exc, B - T), len(exc)


def enumerate_decode_basic(words, n: int, B: int):
    """Decode by expanding each word in base B via divmod on Python ints."""
    if B <= 1:
        return [0] * n
    k = k_of(B)
    out = []
    for s in words:
        digs = []
        for _ in range(k):
            s, r = divmod(s, B)
            digs.append(r)
        out.extend(reversed(digs))
    return out[:n]
