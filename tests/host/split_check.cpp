// Host check of the binary64 digit arithmetic of the HIP decoder (split_word, digit_off in
// kernels_common.h), against exact integer division, and of k(B) from the octave tables. Built with hipcc as host code and run on
// the CPU by tests/test_host_split.py; prints "ok <cases>" or the first mismatch.
#include <stdint.h>
#include <stdio.h>

#include "kernels_common.h"

typedef unsigned __int128 u128;

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next64() {  // splitmix64
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint32_t k_of(uint64_t B) {
    u128 acc = 1;
    uint32_t k = 0;
    while (acc * B <= ((u128)1 << 64)) {
        acc *= B;
        k++;
    }
    return k;
}

static long cases = 0;

// split at P = B^h2 and peel k digits of a word X < B^k; compare with integer arithmetic
static int check(uint64_t B, uint64_t X, int full) {
    const uint32_t k = k_of(B);
    const uint32_t h2 = k / 2 > 1 ? k / 2 : 1;
    uint64_t P = 1;
    for (uint32_t i = 0; i < h2; i++) P *= B;
    const double Pd = pcomp::pow_exact((double)B, h2), rP = 1.0 / Pd;
    cases++;
    if (Pd != (double)P) {
        printf("power mismatch B=%llu h2=%u\n", (unsigned long long)B, h2);
        return 1;
    }
    double hi, lo;
    pcomp::split_word(X, Pd, rP, hi, lo);
    cases++;
    if ((uint64_t)hi != X / P || (uint64_t)lo != X % P) {
        printf("split mismatch B=%llu X=%llu P=%llu hi=%.17g lo=%.17g\n", (unsigned long long)B,
               (unsigned long long)X, (unsigned long long)P, hi, lo);
        return 1;
    }
    if (!full) return 0;
    // digits of the low part and of the high part, lowest first, as the decoder peels them
    const double rB = 1.0 / (double)B, hB = 0.5 * rB, Bf = (double)B;
    uint64_t x = X;
    for (uint32_t m = 0; m < k; m++) {
        uint32_t d;
        double &part = m < h2 ? lo : hi;
        part = pcomp::digit_off(part, rB, hB, Bf, d);
        if (d != x % B) {
            printf("digit mismatch B=%llu X=%llu digit %u: %u vs %llu\n", (unsigned long long)B,
                   (unsigned long long)X, m, d, (unsigned long long)(x % B));
            return 1;
        }
        x /= B;
    }
    return 0;
}

// k(B) from the decoder's and packer's octave tables (k_octave, built as fill_size_ctx builds
// them, from k(B) for small bases and the bounds kmax[k]) against the exact definition
static int check_k_tables() {
    static uint8_t ktab[65538];
    for (uint64_t B = 0; B <= 65537; B++) ktab[B] = B < 2 ? 0 : (uint8_t)k_of(B);
    uint64_t kmax[65];
    kmax[0] = 0;
    kmax[1] = UINT64_MAX;
    for (uint32_t k = 2; k <= 64; k++) {  // largest B with B^k <= 2^64, by bisection
        uint64_t lo = 1, hi = 1ull << 32;
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo + 1) / 2;
            if (k_of(mid) >= k) lo = mid; else hi = mid - 1;
        }
        kmax[k] = lo;
    }
    uint8_t k8[260], ktop[36];
    uint32_t km1[8];
    for (uint32_t t = 0; t <= 256; t++) k8[t] = ktab[t];
    for (uint32_t e = 0; e < 33; e++) ktop[e] = (uint8_t)pcomp::ktop_entry(ktab, kmax, e);
    for (uint32_t k = 0; k < 8; k++) km1[k] = pcomp::km1_entry(kmax, k);
    auto one = [&](uint64_t B) {
        cases++;
        if (pcomp::k_octave(k8, ktop, km1, B) != k_of(B)) {
            printf("k mismatch B=%llu\n", (unsigned long long)B);
            return 1;
        }
        return 0;
    };
    for (uint64_t B = 2; B <= (1u << 20); B++)
        if (one(B)) return 1;
    for (uint32_t k = 2; k < 8; k++)
        for (int d = -2; d <= 2; d++)
            if (kmax[k] + d >= 2 && kmax[k] + d <= (1ull << 32) && one(kmax[k] + d)) return 1;
    for (uint32_t e = 9; e <= 32; e++)
        for (int d = -2; d <= 2; d++)
            if ((1ull << e) + d <= (1ull << 32) && one((1ull << e) + d)) return 1;
    for (int r = 0; r < 2000000; r++)
        if (one(2 + next64() % ((1ull << 32) - 1))) return 1;
    return 0;
}

int main() {
    int bad = check_k_tables();
    for (uint64_t B = 2; B <= 65537 && !bad; B++) {
        u128 Bk = 1;
        for (uint32_t i = 0; i < k_of(B); i++) Bk *= B;
        const uint64_t top = Bk > (u128)UINT64_MAX ? UINT64_MAX : (uint64_t)(Bk - 1);
        bad |= check(B, 0, 1) | check(B, top, 1) | check(B, UINT64_MAX, 0);
        for (int r = 0; r < 24 && !bad; r++) {
            const uint64_t X = top == UINT64_MAX ? next64() : next64() % (top + 1);
            bad |= check(B, X, 1);
            bad |= check(B, next64(), 0);
        }
    }
    // bases of u32 data above the tables, and the powers of two around the limits
    const uint64_t edge[] = {65538, 65539, (1ull << 24) - 1, 1ull << 24, (1ull << 24) + 1, (1ull << 31) + 1,
                             0xFFFFFFFFull, 1ull << 32};
    for (int e = 0; e < 8 && !bad; e++)
        for (int r = 0; r < 20000 && !bad; r++) {
            const uint64_t B = edge[e];
            bad |= check(B, next64(), 0);
            u128 Bk = 1;
            for (uint32_t i = 0; i < k_of(B); i++) Bk *= B;
            const uint64_t top = Bk > (u128)UINT64_MAX ? UINT64_MAX : (uint64_t)(Bk - 1);
            bad |= check(B, top == UINT64_MAX ? next64() : next64() % (top + 1), 1);
        }
    for (int r = 0; r < 2000000 && !bad; r++) {
        const uint64_t B = 65538 + next64() % (0xFFFFFFFFull - 65537);
        bad |= check(B, next64(), r & 1);
    }
    if (bad) return 1;
    printf("ok %ld\n", cases);
    return 0;
}
