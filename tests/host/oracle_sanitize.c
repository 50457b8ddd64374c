/* Memory and undefined-behaviour check of the CPU oracle: built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py and run on the CPU. Every buffer
 * is allocated at its exact size, so a read or write past any of them stops the run. Round trips
 * over every element width, block lengths from 1 to 1024 and every kind of variant (64-bit and
 * 32-bit words, the learned selector with random parameters), then decoding of damaged streams
 * (single bytes changed, streams cut short): any return code is fine, a memory error is not.
 * Prints "ok <cases>". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t orc_compress(const void *in, uint64_t n, int w, uint32_t L, int variant, const uint8_t *forced, uint8_t *out,
                     uint64_t cap);
int64_t orc_decompress(const uint8_t *in, uint64_t in_size, void *out, uint64_t out_cap_values);
uint64_t orc_bound(uint64_t n, int w, uint32_t L, int variant);
int64_t orc_compress32(const void *in, uint64_t n, int w, uint32_t L, int variant, uint8_t *out, uint64_t cap);
int64_t orc_decompress32(const uint8_t *in, uint64_t in_size, void *out, uint64_t out_cap_values);
uint64_t orc_bound32(uint64_t n, int w, uint32_t L, int variant);
int orc_set_model(const float *w, uint64_t n);

static uint64_t st = 0x2545F4914F6CDD1Dull;
static uint64_t next64(void)
{
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static long cases = 0;

/* values of width w: a level plus small noise, a few outliers, a constant stretch */
static void *make_input(uint64_t n, int w)
{
    void *x = malloc(n * w + 1);
    uint64_t top = w == 4 ? 0xFFFFFFFFull : (1ull << (8 * w)) - 1;
    uint64_t level = next64() % (top + 1), spread = 1 + next64() % 300;
    for (uint64_t i = 0; i < n; i++) {
        uint64_t v = level + next64() % spread;
        if (next64() % 97 == 0) v = next64();
        if (i > n / 2 && i < n / 2 + 50) v = level;
        v &= top;
        if (w == 1) ((uint8_t *)x)[i] = (uint8_t)v;
        else if (w == 2) ((uint16_t *)x)[i] = (uint16_t)v;
        else ((uint32_t *)x)[i] = (uint32_t)v;
    }
    return x;
}

static int damaged(const uint8_t *s, uint64_t len, uint64_t n, int w, int words32)
{
    for (int k = 0; k < 40; k++) {
        uint64_t cut = len ? next64() % (len + 1) : 0;
        int flip = k % 2;
        uint64_t m = flip ? len : cut;
        uint8_t *b = (uint8_t *)malloc(m ? m : 1);
        memcpy(b, s, m);
        if (flip && m) b[next64() % m] ^= (uint8_t)(1 + next64() % 255);
        void *o = malloc(n * w + 1);
        int64_t rc = words32 ? orc_decompress32(b, m, o, n) : orc_decompress(b, m, o, n);
        (void)rc;
        free(o);
        free(b);
        cases++;
    }
    return 0;
}

static int round_trip(uint64_t n, int w, uint32_t L, int variant, int words32)
{
    uint64_t cap = words32 ? orc_bound32(n, w, L, variant) : orc_bound(n, w, L, variant);
    if (!cap) return 0; /* combination not offered */
    void *x = make_input(n, w);
    uint8_t *s = (uint8_t *)malloc(cap);
    int64_t len = words32 ? orc_compress32(x, n, w, L, variant, s, cap) : orc_compress(x, n, w, L, variant, NULL, s, cap);
    if (len < 0) {
        printf("compress failed n=%llu w=%d L=%u v=%d w32=%d: %lld\n", (unsigned long long)n, w, L, variant, words32,
               (long long)len);
        return 1;
    }
    void *y = malloc(n * w ? n * w : 1);
    int64_t got = words32 ? orc_decompress32(s, (uint64_t)len, y, n) : orc_decompress(s, (uint64_t)len, y, n);
    if (got != (int64_t)n || memcmp(x, y, n * w)) {
        printf("round trip failed n=%llu w=%d L=%u v=%d w32=%d\n", (unsigned long long)n, w, L, variant, words32);
        return 1;
    }
    cases++;
    damaged(s, (uint64_t)len, n, w, words32);
    free(y);
    free(s);
    free(x);
    return 0;
}

int main(void)
{
    static float model[2320];
    for (int i = 0; i < 2320; i++) model[i] = (float)((int64_t)(next64() % 2001) - 1000) / 1000.0f;
    orc_set_model(model, 2320);
    const int widths[3] = {1, 2, 4};
    const uint32_t lens[5] = {1, 7, 40, 255, 1024};
    const int variants[7] = {0, 8, 3, 12, 0x100, 0x200, 15};
    for (int wi = 0; wi < 3; wi++)
        for (int li = 0; li < 5; li++) {
            uint32_t L = lens[li];
            uint64_t sizes[4] = {0, 1, (uint64_t)L + 3, 3000};
            for (int si = 0; si < 4; si++) {
                for (int vi = 0; vi < 7; vi++)
                    if (round_trip(sizes[si], widths[wi], L, variants[vi], 0)) return 1;
                for (int vi = 0; vi < 2; vi++)
                    if (round_trip(sizes[si], widths[wi], L, variants[vi], 1)) return 1;
                if (round_trip(sizes[si], widths[wi], L, 0x100, 1)) return 1;
            }
        }
    printf("ok %ld\n", cases);
    return 0;
}
