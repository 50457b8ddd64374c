// device_math.h -- integer building blocks of the HIP kernels (device code).
//
// Everything here is exact integer arithmetic. Division by a block constant uses
// Granlund-Montgomery multiply-high magic numbers (PLDI 1994, Fig. 4.1); the few
// divisions by data-dependent values (word counts, the schedule of a base outside the
// precomputed table) go through the compiler's integer division.
#pragma once
#include "pcomp_internal.h"

namespace pcomp {

__device__ __forceinline__ uint64_t div_magic(uint64_t x, const Magic &mg) {
    uint64_t t = __umul64hi(mg.m, x);
    return (t + ((x - t) >> mg.sh1)) >> mg.sh2;
}

// Magic numbers for a divisor d in [1, 2^32], computed on the device: m - 1 =
// floor((2^l - d) 2^64 / d) by two 64-bit long-division steps on 32-bit limbs
// (2^l - d < d <= 2^32, so every partial dividend fits 64 bits).
__device__ inline Magic magic_dev(uint64_t d) {
    Magic mg;
    if (d <= 1) {
        mg.m = 1;
        mg.sh1 = 0;
        mg.sh2 = 0;
        return mg;
    }
    uint32_t l = 64 - __clzll(d - 1);
    uint64_t h = (1ull << l) - d;
    uint64_t n1 = h << 32;
    uint64_t q1 = n1 / d, r1 = n1 - q1 * d;
    uint64_t n0 = r1 << 32;
    uint64_t q0 = n0 / d;
    mg.m = ((q1 << 32) | q0) + 1;
    mg.sh1 = 1;
    mg.sh2 = l - 1;
    return mg;
}

__device__ __forceinline__ Magic magic_dev_outline(uint64_t d) { return magic_dev(d); }

__device__ __forceinline__ uint32_t bitlen64(uint64_t x) { return x ? 64 - __clzll(x) : 0; }
__device__ __forceinline__ uint32_t bitlen32(uint32_t x) { return x ? 32 - __clz(x) : 0; }

// floor(2^64 / x) for x >= 2.
__device__ __forceinline__ uint64_t floor_2p64_div(uint64_t x) {
    uint64_t q = UINT64_MAX / x, r = UINT64_MAX - q * x;
    return q + (r == x - 1 ? 1 : 0);
}

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
__device__ inline uint32_t k_of(const DevTables &T, uint64_t B) {
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

// Constants of the series for a base outside the tables (2^16 + 1 < B <= 2^32).
struct SlowBase {
    uint64_t B, Qk, Qk1;
    uint32_t k;
};

__device__ inline SlowBase slow_base(const DevTables &T, uint64_t B) {
    SlowBase sb;
    sb.B = B;
    sb.k = k_of(T, B);
    if (B == (1ull << 32)) {  // B^2 = 2^64 exactly
        sb.Qk = 1;
        sb.Qk1 = 1ull << 32;
        return sb;
    }
    uint64_t bk1 = 1;
    for (uint32_t i = 0; i + 1 < sb.k; i++) bk1 *= B;  // B^(k-1) < 2^64
    sb.Qk1 = floor_2p64_div(bk1);
    sb.Qk = floor_2p64_div(bk1 * B);  // B^k < 2^64 here
    return sb;
}

// One word of the series for a base outside the tables: from the carried base s = R'_{i-1},
// p_i and R_i (p_i is k when s B^k <= 2^64, else k - 1; R_i = floor(floor(2^64 / B^p) / s)).
__device__ __forceinline__ void slow_word(const SlowBase &sb, uint64_t s, uint32_t &p, uint64_t &R) {
    p = (s <= sb.Qk) ? sb.k : sb.k - 1;
    R = ((p == sb.k) ? sb.Qk : sb.Qk1) / s;
}

// Word count of the series (Sec. 3.2) for n digits: walk it word by word.
__device__ __forceinline__ uint32_t adv_words_slow(const SlowBase sb, uint32_t n) {
    uint64_t s = 1;
    uint32_t q = 0, m = 0;
    for (;;) {
        uint32_t p;
        uint64_t R;
        slow_word(sb, s, p, R);
        m++;
        if (q + p >= n) return m;
        s = (sb.B + R - 1) / R;
        q += p + 1;
    }
}

// c_t = q_t + p_t (values reached by word t, 0-based) from the cycle form: entries
// 0 .. mu+lam-1 are stored, and c_{t + lam} = c_t + V for t >= mu.
__host__ __device__ __forceinline__ uint32_t adv_reach(const AtlasEntry *E, const BaseDesc &D, uint32_t t) {
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
__host__ __device__ inline uint32_t adv_words_cycle(const AtlasEntry *E, const BaseDesc &D, uint32_t n) {
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
__device__ inline uint32_t family_words(const DevTables &T, int fam, uint32_t n, uint64_t base) {
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
