// device_math.h -- integer building blocks of the HIP kernels (device code).
//
// Everything here is exact integer arithmetic. Division by a block constant uses
// Granlund-Montgomery multiply-high magic numbers (PLDI 1994, Fig. 4.1); divisions by
// data-dependent values (the schedule of a base outside the precomputed tables) are binary64
// quotients of exact integers with a one-unit correction from the exact remainder, and small
// ones (word counts, cycle positions) a binary32 reciprocal product; there is no integer
// divide on the device.
#pragma once
#include "pcomp_internal.h"

namespace pcomp {

__device__ __forceinline__ uint64_t div_magic(uint64_t x, const Magic &mg) {
    uint64_t t = __umul64hi(mg.m, x);
    return (t + ((x - t) >> mg.sh1)) >> mg.sh2;
}

// floor(a / b) for a < 2^53 and 1 <= b < 2^53: the double-precision quotient of the exact
// operands is within one unit of a / b after truncation, and one integer step corrects it.
__device__ __forceinline__ uint64_t udiv53(uint64_t a, uint64_t b) {
    uint64_t q = (uint64_t)((double)a / (double)b);
    const int64_t r = (int64_t)(a - q * b);
    if (r < 0)
        q--;
    else if ((uint64_t)r >= b)
        q++;
    return q;
}

// floor(X / R) and X mod R for any 64-bit X and 1 <= R < 2^48. The first double quotient
// is within 2^12 / R + 1 of X / R, so the remainder it leaves is below 2^50 in magnitude
// and a second quotient plus one unit correction finish exactly.
__device__ __forceinline__ uint64_t udiv64_48(uint64_t X, uint64_t R, uint64_t &rem) {
    if (R == 1) {
        rem = 0;
        return X;
    }
    uint64_t q = (uint64_t)((double)X / (double)R);
    int64_t r = (int64_t)(X - q * R);
    const int64_t q1 = (int64_t)floor((double)r / (double)R);
    r -= q1 * (int64_t)R;
    q += (uint64_t)q1;
    if (r < 0) {
        r += (int64_t)R;
        q--;
    } else if ((uint64_t)r >= R) {
        r -= (int64_t)R;
        q++;
    }
    rem = (uint64_t)r;
    return q;
}

// 1/d for 1 <= d < 2^53 to within a relative 2^-50: two Newton-Raphson steps
// (r <- r + r (1 - d r), each squaring the relative error) from the hardware estimate.
__device__ __forceinline__ double recip_f64(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double e = __builtin_fma(-d, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-d, r, 1.0);
    return __builtin_fma(r, e, r);
}

// floor(a / d) for integers 0 <= a < 2^53 and 1 <= d < 2^50 held exactly in binary64, with
// a / d < 2^48 and r = recip_f64(d). The product a r is within 1/4 of a / d, so its truncation
// is floor(a / d) or one unit off, and the remainder a - q d (an integer of magnitude below 2d,
// exact from one FMA) tells which way.
__device__ __forceinline__ double floor_div_f64(double a, double d, double r) {
    const double q = __builtin_trunc(a * r);
    const double rem = __builtin_fma(-q, d, a);
    return rem < 0.0 ? q - 1.0 : (rem >= d ? q + 1.0 : q);
}

// floor(X / R) and X mod R for any 64-bit X and 2 <= R < 2^48, with rR = recip_f64(R): the first
// quotient, from X rounded to binary64 times rR, is within 2^14 of X / R, so the remainder it
// leaves is below 2^62 in magnitude; a second product gives the rest to within one unit.
__device__ __forceinline__ uint64_t udiv64_rcp(uint64_t X, uint64_t R, double rR, uint64_t &rem) {
    uint64_t q = (uint64_t)((double)X * rR);
    int64_t r = (int64_t)(X - q * R);
    const int64_t q1 = (int64_t)__builtin_floor((double)r * rR);
    r -= q1 * (int64_t)R;
    q += (uint64_t)q1;
    if (r < 0) {
        r += (int64_t)R;
        q--;
    } else if ((uint64_t)r >= R) {
        r -= (int64_t)R;
        q++;
    }
    rem = (uint64_t)r;
    return q;
}

// Magic numbers for a divisor d in [1, 2^32], computed on the device: m - 1 =
// floor((2^l - d) 2^64 / d) by two 64-bit long-division steps on 32-bit limbs
// (2^l - d < d <= 2^32, so every partial dividend fits 64 bits).
__device__ __forceinline__ Magic magic_dev(uint64_t d) {
    Magic mg;
    if (d <= 1) {
        mg.m = 1;
        mg.sh1 = 0;
        mg.sh2 = 0;
        return mg;
    }
    uint32_t l = 64 - __clzll(d - 1);
    uint64_t h = (1ull << l) - d;
    uint64_t r1, r0;
    const uint64_t q1 = udiv64_48(h << 32, d, r1);
    const uint64_t q0 = udiv64_48(r1 << 32, d, r0);
    mg.m = ((q1 << 32) | q0) + 1;
    mg.sh1 = 1;
    mg.sh2 = l - 1;
    return mg;
}

__device__ __forceinline__ Magic magic_dev_outline(uint64_t d) { return magic_dev(d); }

__device__ __forceinline__ uint32_t bitlen64(uint64_t x) { return x ? 64 - __clzll(x) : 0; }
__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32 - __clz(x) : 0; }

// floor(N / d) for N < 2^20 and 1 <= d < 2^24. On the device without an integer divide:
// (N + 1/2) / d lies at least 1 / (2d) from any integer, and its single-precision product
// with a reciprocal of at most 1 ulp error is within a relative 2^-22 of it, i.e. within
// 1 / (4d), so the truncated product is exact.
__host__ __device__ __forceinline__ uint32_t udiv_small(uint32_t N, uint32_t d) {
#if defined(__HIP_DEVICE_COMPILE__)
    return (uint32_t)(((float)N + 0.5f) * __builtin_amdgcn_rcpf((float)d));
#else
    return N / d;
#endif
}

// Index of base B in the precomputed tables, or -1.
__device__ __forceinline__ int atlas_index(uint64_t B) {
    if (B <= kAtlasDirect) return (int)B;
    uint64_t t = B - 1;
    if ((t & (t - 1)) == 0) {
        int j = 63 - __clzll(t);
        if (j >= 17 && j <= 31) return (int)(kAtlasDirect + 1 + (j - 17));
    }
    return -1;
}

// Digits per word k(B) = max{k : B^k <= 2^64} (Sec. 3.1, Eq. (1), exact reading). B >= 2.
__device__ __forceinline__ uint32_t k_of(const DevTables &T, uint64_t B) {
    int ai = atlas_index(B);
    if (ai >= 0) return T.desc[ai].k;
    uint32_t lo = 1, hi = 64;
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) >> 1;
        if (B <= T.kmax[mid])
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Constants of the series for a base outside the tables (2^16 + 1 < B <= 2^32), also as
// binary64 (every one below 2^48, so held exactly).
struct SlowBase {
    uint64_t B, Qk, Qk1;
    double Bd, Bm1d, Qkd, Qk1d;
    uint32_t k;
};

// floor(2^64 / B^p) for p = 1 .. k by a chain of quotients (floor(floor(x / a) / b) =
// floor(x / (a b))); floor(2^64 / B) < 2^48 for these bases.
__device__ __forceinline__ SlowBase slow_base(const DevTables &T, uint64_t B) {
    SlowBase sb;
    sb.B = B;
    sb.k = k_of(T, B);  // 2 or 3
    uint64_t r;
    uint64_t Q = udiv64_48(UINT64_MAX, B, r);
    if (r == B - 1) Q++;  // B divides 2^64
    uint64_t Qprev = Q;
    for (uint32_t p = 2; p <= sb.k; p++) {
        Qprev = Q;
        Q = udiv53(Q, B);
    }
    sb.Qk = Q;
    sb.Qk1 = Qprev;
    sb.Bd = (double)B;
    sb.Bm1d = (double)(B - 1);
    sb.Qkd = (double)Q;
    sb.Qk1d = (double)Qprev;
    return sb;
}

// One word of the series for a base outside the tables, in binary64: every floor(2^64 / B^p)
// is below 2^48 here (B > 2^16 + 1) and the carried base s is at most B <= 2^32, so
// R = floor(Q_p / s) is a floor_div_f64 of exact integers.
__device__ __forceinline__ void slow_word_f64(const SlowBase &sb, double s, uint32_t &p, double &R) {
    const bool full = s <= sb.Qkd;
    p = full ? sb.k : sb.k - 1;
    R = floor_div_f64(full ? sb.Qkd : sb.Qk1d, s, recip_f64(s));
}

// The carried base of the next word, ceil(B / R) = floor((B - 1) / R) + 1 (1 for R >= B).
__device__ __forceinline__ double slow_next_f64(const SlowBase &sb, double R) {
    return R >= sb.Bd ? 1.0 : floor_div_f64(sb.Bm1d, R, recip_f64(R)) + 1.0;
}

__device__ __forceinline__ void slow_word_fast(const SlowBase &sb, uint64_t s, uint32_t &p, uint64_t &R) {
    double Rd;
    slow_word_f64(sb, (double)s, p, Rd);
    R = (uint64_t)Rd;
}

__device__ __forceinline__ uint64_t slow_next(const SlowBase &sb, uint64_t R) {
    return (uint64_t)slow_next_f64(sb, (double)R);
}

// Brent's cycle search over the carried base of the series (Sec. 3.2): s_t, the state of word
// t, fixes every word after it, so once s_t = s_{t - lam} the series repeats with period lam,
// V values per period, from word t - lam on. step() takes the state and q of each next word.
struct SeriesCycle {
    uint64_t s_mark;
    uint32_t q_mark, power, lam, V;
    bool found;
    __device__ __forceinline__ SeriesCycle() : s_mark(1), q_mark(0), power(1), lam(0), V(0), found(false) {}
    __device__ __forceinline__ void step(uint64_t s, uint32_t q) {
        if (found) return;
        lam++;
        if (s == s_mark) {
            found = true;
            V = q - q_mark;
        } else if (lam == power) {
            s_mark = s;
            q_mark = q;
            power <<= 1;
            lam = 0;
        }
    }
};

// The first of a lane's words i0, i0 + G, ... (G a power of two) at or after word wi.
__device__ __forceinline__ uint32_t next_own_word(uint32_t wi, uint32_t i0, uint32_t G) {
    return wi <= i0 ? i0 : i0 + ((wi - i0 + G - 1) & ~(G - 1));
}

// The schedule of the series of a base outside the tables (Sec. 3.2), held in the registers of
// a group of lanes that walk it in step. Every lane computes the same words; word t is held by
// lane t mod width of the window (the group's first `width` lanes within the wavefront), in its
// register t / width, as R_t | (p_t - 1) << 48 | q_t << 50. The state (p_t, R_t) fixes every later
// word, so the first word whose state equals that of a held one, found by comparing it with
// every held entry at once, closes the period: words from cs on repeat every lam words, V values
// further on. The walk stops there, at the part's last word, or with the window full (ok false:
// the caller then walks the series lane by lane). Every lane of the window calls it with the same
// arguments.
constexpr uint32_t kWinRegs = 4;  // entries per lane: periods up to 4 x width words are held

struct SlowWindow {
    uint64_t e[kWinRegs];  // words gl, gl + width, ... of this lane gl (all ones: none)
    uint32_t seg, shift;   // first lane of the window in the wavefront; log2(width)
    uint32_t last;         // last word held
    uint32_t cs, lam, V;   // the period (lam = 0: none, every word of the part is held)
    bool ok;
};

constexpr uint64_t kWinR = (1ull << 48) - 1;      // R of an entry
constexpr uint64_t kWinState = (1ull << 50) - 1;  // R and p of an entry

// 64 bits of lane `src` of the wavefront (an active lane).
__device__ __forceinline__ uint64_t lane_read64(uint64_t v, uint32_t src) {
    const int a = (int)(src << 2);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(a, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ SlowWindow slow_window(const SlowBase &sb, uint32_t n, uint32_t nwords, uint32_t width) {
    SlowWindow w;
    const uint32_t lane = __lane_id();
    w.seg = lane & ~(width - 1);
    w.shift = 31 - __clz(width);
    const uint32_t gl = lane - w.seg;
    const uint64_t wmask = (width >= 64 ? ~0ull : (1ull << width) - 1) << w.seg;
#pragma unroll
    for (uint32_t r = 0; r < kWinRegs; r++) w.e[r] = ~0ull;  // p - 1 = 3 is no entry's, so it matches nothing
    w.last = 0;
    w.cs = w.lam = w.V = 0;
    w.ok = false;
    double s = 1.0;
    uint32_t q = 0;
    for (uint32_t t = 0;; t++) {
        uint32_t p;
        double R;
        slow_word_f64(sb, s, p, R);
        const uint64_t E = (uint64_t)R | ((uint64_t)(p - 1) << 48) | ((uint64_t)q << 50);
        // the held word of the same state, if any (at most one: the walk stops at the first)
        uint32_t hit = 0;  // 1 + its word index and its q
#pragma unroll
        for (uint32_t r = 0; r < kWinRegs; r++)
            if (((w.e[r] ^ E) & kWinState) == 0) hit = 1u | ((gl + (r << w.shift)) << 1) | ((uint32_t)(w.e[r] >> 50) << 16);
        const uint64_t m = __ballot(hit != 0) & wmask;
        if (m) {
            const uint32_t h = (uint32_t)__shfl((int)hit, (int)(w.seg + __builtin_ctzll(m >> w.seg)), 64);
            w.cs = (h >> 1) & 0x7FFF;
            w.lam = t - w.cs;
            w.V = q - (h >> 16);
        }
        // word t goes to lane t mod width, register t / width
        const uint32_t slot = t >> w.shift;
        if (gl == (t & (width - 1))) {
#pragma unroll
            for (uint32_t r = 0; r < kWinRegs; r++) w.e[r] = r == slot ? E : w.e[r];
        }
        w.last = t;
        if (m || q + p >= n || t + 1 >= nwords) {
            w.ok = true;
            break;
        }
        if (t + 1 >= (kWinRegs << w.shift)) break;
        s = slow_next_f64(sb, R);
        q += p + 1;
    }
    return w;
}

// Entry of word i from a window: its index among the held words and the periods before it.
__device__ __forceinline__ void window_index(const SlowWindow &w, uint32_t i, uint32_t &j, uint32_t &c) {
    j = i;
    c = 0;
    if (w.lam && i > w.cs) {
        c = udiv_small(i - w.cs, w.lam);
        j = i - c * w.lam;
    }
}

// Entry of held word j (every lane of the window calls it; each may ask for another word).
__device__ __forceinline__ uint64_t window_entry(const SlowWindow &w, uint32_t j) {
    j = j <= w.last ? j : w.last;
    const uint32_t src = w.seg + (j & ((1u << w.shift) - 1)), slot = j >> w.shift;
    uint64_t v = 0;
#pragma unroll
    for (uint32_t r = 0; r < kWinRegs; r++) {
        if ((r << w.shift) > w.last) break;  // the same on every lane of the window
        const uint64_t x = lane_read64(w.e[r], src);
        v = r == slot ? x : v;
    }
    return v;
}

__device__ __forceinline__ void window_next(const SlowWindow &w, uint32_t &j, uint32_t &c) {
    j++;
    if (w.lam && j == w.cs + w.lam) {
        j = w.cs;
        c++;
    }
}

// Word count of the series for n digits (1 + the first word t with q_t + p_t >= n) from a
// window walked with no word limit: every held word of the period proposes the first of its
// repeats that reaches n, and the window takes the least. Every lane of the window calls it.
__device__ __forceinline__ uint32_t window_words(const SlowWindow &w, uint32_t n) {
    const uint32_t gl = __lane_id() - w.seg;
    uint32_t best = 0xFFFFFFFFu;
#pragma unroll
    for (uint32_t r = 0; r < kWinRegs; r++) {
        const uint32_t j = gl + (r << w.shift);
        if (j > w.last) continue;
        const uint32_t reach = (uint32_t)(w.e[r] >> 50) + (uint32_t)((w.e[r] >> 48) & 3) + 1;  // q_j + p_j
        uint32_t cand = 0xFFFFFFFFu;
        if (reach >= n)
            cand = j;
        else if (w.lam && j >= w.cs)
            cand = j + udiv_small(n - reach + w.V - 1, w.V) * w.lam;
        best = cand < best ? cand : best;
    }
    for (uint32_t o = 1; o < (1u << w.shift); o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_xor((int)best, (int)o, 64);
        best = y < best ? y : best;
    }
    return best + 1;
}

// Word count of the series (Sec. 3.2) for n digits: walk it word by word. The carried base
// s_t determines everything after word t, so once Brent's cycle search finds s_t = s_{t-lam}
// the series repeats with period lam from there, consuming V = q_t - q_{t-lam} values per
// period; whole periods are then skipped while they end at or before value n.
__device__ __forceinline__ uint32_t adv_words_slow(const SlowBase sb, uint32_t n) {
    uint64_t s = 1, s_mark = 1;
    uint32_t q = 0, t = 0, q_mark = 0;
    uint32_t power = 1, lam = 0;
    bool skipped = false;
    for (;;) {
        uint32_t p;
        uint64_t R;
        slow_word_fast(sb, s, p, R);
        if (q + p >= n) return t + 1;
        s = slow_next(sb, R);
        q += p + 1;
        t++;
        lam++;
        if (skipped) continue;
        if (s == s_mark) {
            const uint32_t V = q - q_mark;
            const uint32_t c = udiv_small(n - q, V);  // q + c V <= n: no word before is the last
            q += c * V;
            t += c * lam;
            skipped = true;
        } else if (lam == power) {
            s_mark = s;
            q_mark = q;
            power <<= 1;
            lam = 0;
        }
    }
}

// c_t = q_t + p_t (values reached by word t, 0-based) from the cycle form: entries
// 0 .. mu+lam-1 are stored, and c_{t + lam} = c_t + V for t >= mu.
// (Entries and descriptors of either word size.)
template <typename Entry, typename Desc>
__host__ __device__ __forceinline__ uint32_t adv_reach(const Entry *E, const Desc &D, uint32_t t) {
    const uint32_t tot = D.mu + D.lam;
    if (t < tot) return E[t].q + E[t].p;
    const uint32_t c = udiv_small(t - D.mu, D.lam);
    const uint32_t r = t - c * D.lam;
    return E[r].q + E[r].p + c * D.V;
}

// Word count of the series for n digits: 1 + the first t with c_t >= n. Every word takes
// k or k + 1 values (p_t is k - 1 or k, plus the split value) and the first takes k,
// so (t+1) k <= c_t <= (t+1)(k+1) - 1: the answer lies in
// [ceil((n+1)/(k+1)) - 1, ceil(n/k) - 1], a range of about n / k^2 words.
template <typename Entry, typename Desc>
__host__ __device__ inline uint32_t adv_words_cycle(const Entry *E, const Desc &D, uint32_t n) {
    const uint32_t k = D.k;
    if (n <= k) return 1;
    uint32_t lo = udiv_small(n + 1 + k, k + 1) - 1;  // ceil((n+1)/(k+1)) - 1
    uint32_t hi = udiv_small(n + k - 1, k) - 1;      // ceil(n/k) - 1
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (adv_reach(E, D, mid) >= n)
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo + 1;
}

__device__ __forceinline__ uint32_t adv_words_atlas(const DevTables &T, const BaseDesc &D, uint32_t n) {
    return adv_words_cycle(T.ent + D.off, D, n);
}

// Entry and q_i of word i from the cycle form.
__device__ __forceinline__ const AtlasEntry *adv_entry(const DevTables &T, const BaseDesc &D, uint32_t i,
                                                       uint32_t &q) {
    const AtlasEntry *E = T.ent + D.off;
    uint32_t tot = D.mu + D.lam;
    if (i < tot) {
        q = E[i].q;
        return E + i;
    }
    uint32_t c = udiv_small(i - D.mu, D.lam);
    uint32_t r = i - c * D.lam;
    q = E[r].q + c * D.V;
    return E + r;
}

// Words of one family (0 basic Sec. 3.1, 1 advanced Sec. 3.2) for n digits of `base`.
__device__ __forceinline__ uint32_t family_words(const DevTables &T, int fam, uint32_t n, uint64_t base) {
    if (n == 0 || base <= 1) return 0;
    if (!fam) {
        uint32_t k = k_of(T, base);
        return udiv_small(n + k - 1, k);
    }
    int ai = atlas_index(base);
    if (ai >= 0) return adv_words_atlas(T, T.desc[ai], n);
    return adv_words_slow(slow_base(T, base), n);
}

}  // namespace pcomp
