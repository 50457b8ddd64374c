/*
 * pcomp_oracle.c -- plain, slow, obviously-correct CPU oracle for the blocked
 * polynomial compressor of Aubert et al., "Polynomial data compression for
 * large-scale physics experiments" (arXiv:1805.01844).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke entry point and the CPU
 * baseline leg of the benchmark may load or call this library. It shares no
 * code, header, table or helper with the GPU library; the only thing the two
 * have in common is the stream format that both write independently.
 *
 * Arithmetic is exact integer arithmetic throughout (unsigned __int128 where a
 * product can exceed 64 bits, hardware '/' and '%' for every division). The
 * word size W is a parameter (64 for streams; 32 only to compare block sizes
 * with the paper's own 32-bit figures).
 *
 * Sections of the paper followed here:
 *   Sec. 3   -- base B = v_max - v_min + 1 of the ring the data live in.
 *   Sec. 3.1 -- Eq. (1): digits per word; Eq. (2): basic packing; decompression
 *               by polynomial division.
 *   Sec. 3.2 -- Eqs. (3)-(11) and the series that closes the section: the
 *               advanced (split-base) packing with R_i, R'_i, p_i, q_i, r_i,
 *               r'_i, s_i.
 *   Sec. 3.3 -- blocked compression: one (min, B) per block.
 * Readings where the paper is silent or inconsistent (capacity 2^W rather than
 * 2^W - 1, first value at the highest power, R'_i = ceil(B / R_i), the stopping
 * rule of the series, the threshold/excess classes, the stream layout) are the
 * ones listed in the design notes; each is restated next to the code it shapes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* Error codes (same numeric values as the public C interface). */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOSPC (-2)
#define ORC_ECORRUPT (-3)
#define ORC_ENOMODEL (-4)

#define ORC_SELECT_EXHAUSTIVE 0x100
#define ORC_SELECT_LEARNED 0x200

#define ORC_MAGIC 0x504D4350u /* "PCMP" little-endian */
#define ORC_VERSION 1u
#define ORC_HDR_BYTES 64u

/* flags byte of the stream header */
#define ORC_F_CLASS 1u /* per-block class array present */
#define ORC_F_NE 2u    /* per-block excess-count array present */
#define ORC_F_NE16 4u  /* excess counts stored as u16 (else u8) */
#define ORC_F_W32 8u   /* payload of 32-bit words (orc_compress32) */

/* ---------------------------------------------------------------------- */
/* Sec. 3.1, Eq. (1): number of base-B digits that fit in one W-bit word.   */
/* Read with exact integers: the largest k >= 0 with B^k <= 2^W (a word     */
/* holds every digit combination iff the product of the bases is at most    */
/* 2^W). Undefined (returned as 0) for B <= 1.                              */
/* ---------------------------------------------------------------------- */
int orc_digits_per_word(uint64_t B, int W)
{
    if (B <= 1) return 0;
    u128 cap = ((u128)1) << W;
    u128 acc = 1;
    int k = 0;
    while (acc * B <= cap) {
        acc *= B;
        k++;
    }
    return k;
}

/* bit length of x: number of bits needed to write x (bitlen(0) = 0) */
static int bitlen64(uint64_t x)
{
    int b = 0;
    while (x) {
        b++;
        x >>= 1;
    }
    return b;
}

/* ---------------------------------------------------------------------- */
/* Sec. 3.1, Eq. (2): basic packing. Word j holds the k digits             */
/* d[jk .. jk+k-1]; the first digit sits at the highest power of B (the    */
/* accumulation order stated in Sec. 3.2), absent tail digits are 0.       */
/* ---------------------------------------------------------------------- */
uint64_t orc_basic_words(uint64_t n, uint64_t B, int W)
{
    if (n == 0 || B <= 1) return 0;
    uint64_t k = (uint64_t)orc_digits_per_word(B, W);
    return (n + k - 1) / k;
}

static uint64_t basic_pack(const uint64_t *d, uint64_t n, uint64_t B, int W, uint64_t *words)
{
    uint64_t nw = orc_basic_words(n, B, W);
    uint64_t k = (uint64_t)orc_digits_per_word(B, W);
    for (uint64_t j = 0; j < nw; j++) {
        u128 s = 0;
        for (uint64_t i = 0; i < k; i++) {
            uint64_t idx = j * k + i;
            uint64_t v = idx < n ? d[idx] : 0;
            s = s * B + v;
        }
        words[j] = (uint64_t)s;
    }
    return nw;
}

/* Decompression "by polynomial division": peel digits from the lowest power. */
static void basic_unpack(const uint64_t *words, uint64_t n, uint64_t B, int W, uint64_t *d)
{
    if (B <= 1) {
        for (uint64_t i = 0; i < n; i++) d[i] = 0;
        return;
    }
    uint64_t nw = orc_basic_words(n, B, W);
    uint64_t k = (uint64_t)orc_digits_per_word(B, W);
    for (uint64_t j = 0; j < nw; j++) {
        uint64_t s = words[j];
        for (uint64_t i = k; i-- > 0;) {
            uint64_t idx = j * k + i;
            uint64_t digit = s % B;
            s /= B;
            if (idx < n) d[idx] = digit;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Sec. 3.2, the series: split-base (advanced) packing.                     */
/*   R'_0 = 1, r'_0 = 0, q_1 = 0, and for every packed word i >= 1:       */
/*   p_i  = max{ p : R'_{i-1} B^p <= 2^W }                                 */
/*   R_i  = floor( 2^W / (R'_{i-1} B^{p_i}) )                              */
/*   R'_i = ceil( B / R_i )                                                */
/*   the value after the p_i full digits, x = d[q_i + p_i], is split into  */
/*   r_i = x mod R_i (bottom of word i) and r'_i = x div R_i (top of word  */
/*   i+1); s_i = ((r'_{i-1} B^{p_i} + sum_k d[q_i+k] B^{p_i-1-k}) R_i + r_i */
/*   q_{i+1} = q_i + p_i + 1                                               */
/*   the series stops at the first word m with q_m + p_m >= n.              */
/* (0-based digit indices; digits past the end of the block are 0.)        */
/* ---------------------------------------------------------------------- */
typedef struct {
    uint64_t p;       /* p_i */
    uint64_t R;       /* R_i */
    uint64_t Rp_prev; /* R'_{i-1} */
    uint64_t q;       /* q_i */
} orc_adv_word;

/* Walks the series; fills sched[0..m-1] when sched != NULL; returns m. */
static uint64_t adv_series(uint64_t n, uint64_t B, int W, orc_adv_word *sched)
{
    if (n == 0 || B <= 1) return 0;
    u128 cap = ((u128)1) << W;
    uint64_t Rp_prev = 1; /* R'_0 */
    uint64_t q = 0;       /* q_1 */
    uint64_t m = 0;
    for (;;) {
        uint64_t p = 0;
        u128 prod = Rp_prev; /* R'_{i-1} B^p */
        while (prod * B <= cap) {
            prod *= B;
            p++;
        }
        uint64_t R = (uint64_t)(cap / prod);
        if (sched) {
            sched[m].p = p;
            sched[m].R = R;
            sched[m].Rp_prev = Rp_prev;
            sched[m].q = q;
        }
        m++;
        if (q + p >= n) break;
        uint64_t Rp = (B + R - 1) / R; /* ceil(B / R_i) */
        q += p + 1;
        Rp_prev = Rp;
    }
    return m;
}

uint64_t orc_adv_words(uint64_t n, uint64_t B, int W) { return adv_series(n, B, W, NULL); }

/* Exposes the series for tests: fills up to max_words entries of p, R, R'_{i-1}, q. */
uint64_t orc_adv_schedule(uint64_t n, uint64_t B, int W, uint64_t *p, uint64_t *R, uint64_t *Rp_prev,
                          uint64_t *q, uint64_t max_words)
{
    uint64_t m = adv_series(n, B, W, NULL);
    if (m == 0 || m > max_words) return m;
    orc_adv_word *s = (orc_adv_word *)malloc(sizeof(orc_adv_word) * m);
    adv_series(n, B, W, s);
    for (uint64_t i = 0; i < m; i++) {
        p[i] = s[i].p;
        R[i] = s[i].R;
        Rp_prev[i] = s[i].Rp_prev;
        q[i] = s[i].q;
    }
    free(s);
    return m;
}

static uint64_t adv_pack(const uint64_t *d, uint64_t n, uint64_t B, int W, uint64_t *words)
{
    uint64_t m = adv_series(n, B, W, NULL);
    if (m == 0) return 0;
    orc_adv_word *sc = (orc_adv_word *)malloc(sizeof(orc_adv_word) * m);
    adv_series(n, B, W, sc);
    uint64_t rp_prev = 0; /* r'_0 */
    for (uint64_t i = 0; i < m; i++) {
        uint64_t q = sc[i].q, p = sc[i].p, R = sc[i].R;
        u128 s = rp_prev;
        for (uint64_t k = 0; k < p; k++) {
            uint64_t idx = q + k;
            s = s * B + (idx < n ? d[idx] : 0);
        }
        uint64_t x = (q + p) < n ? d[q + p] : 0;
        uint64_t r = x % R;
        uint64_t rp = x / R;
        s = s * R + r;
        words[i] = (uint64_t)s;
        rp_prev = rp;
    }
    free(sc);
    return m;
}

static void adv_unpack(const uint64_t *words, uint64_t n, uint64_t B, int W, uint64_t *d)
{
    if (B <= 1) {
        for (uint64_t i = 0; i < n; i++) d[i] = 0;
        return;
    }
    uint64_t m = adv_series(n, B, W, NULL);
    orc_adv_word *sc = (orc_adv_word *)malloc(sizeof(orc_adv_word) * m);
    adv_series(n, B, W, sc);
    uint64_t r_prev = 0;
    for (uint64_t i = 0; i < m; i++) {
        uint64_t q = sc[i].q, p = sc[i].p, R = sc[i].R;
        uint64_t s = words[i];
        uint64_t r = s % R;
        s /= R;
        for (uint64_t k = p; k-- > 0;) {
            uint64_t idx = q + k;
            uint64_t digit = s % B;
            s /= B;
            if (idx < n) d[idx] = digit;
        }
        /* what is left is r'_{i-1}: the top part of the value split at the end of word i-1 */
        if (i > 0) {
            uint64_t idx = sc[i - 1].q + sc[i - 1].p;
            uint64_t v = s * sc[i - 1].R + r_prev;
            if (idx < n) d[idx] = v;
        }
        r_prev = r;
    }
    free(sc);
}

/* ---------------------------------------------------------------------- */
/* Family dispatch: 0 = basic (Sec. 3.1), 1 = advanced (Sec. 3.2).          */
/* A base of 1 carries no information: zero words.                          */
/* ---------------------------------------------------------------------- */
uint64_t orc_family_words(int family, uint64_t n, uint64_t base, int W)
{
    if (base <= 1 || n == 0) return 0;
    return family ? orc_adv_words(n, base, W) : orc_basic_words(n, base, W);
}

uint64_t orc_family_pack(int family, const uint64_t *d, uint64_t n, uint64_t base, int W, uint64_t *words)
{
    if (base <= 1 || n == 0) return 0;
    return family ? adv_pack(d, n, base, W, words) : basic_pack(d, n, base, W, words);
}

void orc_family_unpack(int family, const uint64_t *words, uint64_t n, uint64_t base, int W, uint64_t *d)
{
    if (n == 0) return;
    if (family)
        adv_unpack(words, n, base, W, d);
    else
        basic_unpack(words, n, base, W, d);
}

/* ---------------------------------------------------------------------- */
/* Threshold / excess classes (a value split layered over the two families, */
/* in the spirit of the r / r' split of Sec. 3.2).                           */
/*   class id c = 8 * family + t, t in 0..7; t = 0 is the plain family.     */
/*   beta = bitlen(B - 1); class valid iff t <= beta; T = 2^(beta - t).      */
/*   main digits c_j = min(d_j, T) packed in base T + 1 by the family rule; */
/*   excess list [d_j - T for d_j >= T] (in order, n_e entries) packed in   */
/*   base B - T by the same rule and placed after the main words.           */
/* ---------------------------------------------------------------------- */
int orc_class_valid(int cls, uint64_t B)
{
    if (cls < 0 || cls > 15) return 0;
    int t = cls & 7;
    if (t == 0) return 1;
    if (B < 1) return 0;
    return t <= bitlen64(B - 1);
}

static uint64_t class_threshold(int cls, uint64_t B)
{
    int t = cls & 7;
    int beta = bitlen64(B - 1);
    return ((uint64_t)1) << (beta - t);
}

/* Number of payload words of a block of n digits (all < B) in class cls;
 * *ne_out receives the excess count (0 for t = 0). Class must be valid. */
uint64_t orc_class_words(int cls, const uint64_t *d, uint64_t n, uint64_t B, uint64_t *ne_out)
{
    int family = cls >> 3, t = cls & 7;
    if (t == 0) {
        if (ne_out) *ne_out = 0;
        return orc_family_words(family, n, B, 64);
    }
    uint64_t T = class_threshold(cls, B);
    uint64_t ne = 0;
    for (uint64_t j = 0; j < n; j++)
        if (d[j] >= T) ne++;
    if (ne_out) *ne_out = ne;
    return orc_family_words(family, n, T + 1, 64) + orc_family_words(family, ne, B - T, 64);
}

/* Packs one block of digits in class cls (must be valid); returns words written. */
uint64_t orc_class_pack(int cls, const uint64_t *d, uint64_t n, uint64_t B, uint64_t *words, uint64_t *ne_out)
{
    int family = cls >> 3, t = cls & 7;
    if (t == 0) {
        if (ne_out) *ne_out = 0;
        return orc_family_pack(family, d, n, B, 64, words);
    }
    uint64_t T = class_threshold(cls, B);
    uint64_t *c = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t *e = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t ne = 0;
    for (uint64_t j = 0; j < n; j++) {
        if (d[j] >= T) {
            c[j] = T;
            e[ne++] = d[j] - T;
        } else {
            c[j] = d[j];
        }
    }
    uint64_t nw = orc_family_pack(family, c, n, T + 1, 64, words);
    nw += orc_family_pack(family, e, ne, B - T, 64, words + nw);
    if (ne_out) *ne_out = ne;
    free(c);
    free(e);
    return nw;
}

/* Inverse of orc_class_pack. */
void orc_class_unpack(int cls, const uint64_t *words, uint64_t n, uint64_t B, uint64_t ne, uint64_t *d)
{
    int family = cls >> 3, t = cls & 7;
    if (t == 0) {
        orc_family_unpack(family, words, n, B, 64, d);
        return;
    }
    uint64_t T = class_threshold(cls, B);
    uint64_t nw_main = orc_family_words(family, n, T + 1, 64);
    uint64_t *e = (uint64_t *)malloc(sizeof(uint64_t) * (ne ? ne : 1));
    orc_family_unpack(family, words, n, T + 1, 64, d);
    if (ne) {
        if (B - T <= 1) {
            for (uint64_t j = 0; j < ne; j++) e[j] = 0;
        } else {
            orc_family_unpack(family, words + nw_main, ne, B - T, 64, e);
        }
    }
    uint64_t k = 0;
    for (uint64_t j = 0; j < n; j++)
        if (d[j] == T) d[j] = T + (k < ne ? e[k++] : 0);
    free(e);
}

/* ---------------------------------------------------------------------- */
/* Per-block class choice.                                                   */
/*   fixed t = 0 class: every block uses it (single-class stream).           */
/*   otherwise a candidate c (the fixed class, the argmin over all valid     */
/*   classes with ties to the lowest id, or a class given from outside) is   */
/*   kept only if it is valid and strictly smaller than basic t = 0;         */
/*   else the block falls back to class 0 (basic, t = 0).                    */
/* ---------------------------------------------------------------------- */
/* ---------------------------------------------------------------------- */
/* Learned class selector (an addition to the method: the paper chooses the */
/* variant by hand for a whole file, Sec. 4). A small network reads 19     */
/* features of a block and scores the 16 classes; the best-scoring class is */
/* then kept under the same rule as a fixed class.                          */
/*                                                                          */
/* Features, all in binary32 with correctly rounded operations only, so    */
/* that any IEEE implementation obtains the same bits:                      */
/*   x[b], b = 0..15: H[b] / L_b, H[b] = #{j : min(beta - bitlen(d_j), 15)  */
/*          = b}, beta = bitlen(B - 1) (digits by octave below the top);    */
/*   x[16]: lg(min + 1) / 32, x[17]: lg(max + 1) / 32, lg the piecewise-    */
/*          linear base-2 logarithm: for 2^e <= u < 2^(e+1),                */
/*          lg(u) = e + (u - 2^e) 2^-e, with (u - 2^e) rounded to binary32; */
/*   x[18]: L_b / 4096.                                                     */
/* Network: h_j = relu(b1_j + sum_i W1[j][i] x_i), j < 64;                 */
/* s_k = b2_k + sum_j W2[k][j] h_j, k < 16; each sum taken in index order   */
/* as a chain of fused multiply-adds starting from the bias. Parameters, in */
/* this order: W1 (64 x 19, row-major), b1 (64), W2 (16 x 64), b2 (16):     */
/* 2320 floats. The predicted class is the first index of the largest s_k. */
/* ---------------------------------------------------------------------- */
#define ORC_MLP_IN 19
#define ORC_MLP_HID 64
#define ORC_MLP_OUT 16
#define ORC_MLP_PARAMS (ORC_MLP_HID * ORC_MLP_IN + ORC_MLP_HID + ORC_MLP_OUT * ORC_MLP_HID + ORC_MLP_OUT)

static float g_model[ORC_MLP_PARAMS];
static int g_have_model = 0;

int orc_set_model(const float *w, uint64_t n)
{
    if (!w) {
        g_have_model = 0;
        return ORC_OK;
    }
    if (n != ORC_MLP_PARAMS) return ORC_EINVAL;
    memcpy(g_model, w, sizeof(g_model));
    g_have_model = 1;
    return ORC_OK;
}

static float lg_f32(uint64_t u) /* u >= 1 */
{
    int e = bitlen64(u) - 1;
    float frac = ldexpf((float)(uint32_t)(u - ((uint64_t)1 << e)), -e);
    return (float)e + frac;
}


void orc_block_features(const uint64_t *d, uint64_t n, uint64_t vmin, uint64_t vmax, float *x)
{
    uint64_t H[16] = {0};
    int beta = bitlen64(vmax - vmin);
    for (uint64_t j = 0; j < n; j++) {
        int b = beta - bitlen64(d[j]);
        H[b < 15 ? b : 15]++;
    }
    for (int b = 0; b < 16; b++) x[b] = (float)H[b] / (float)n;
    x[16] = lg_f32(vmin + 1) * 0.03125f;
    x[17] = lg_f32(vmax + 1) * 0.03125f;
    x[18] = (float)n * (1.0f / 4096.0f);
}

void orc_mlp_scores(const float *model, const float *x, float *s)
{
    const float *W1 = model, *b1 = W1 + ORC_MLP_HID * ORC_MLP_IN, *W2 = b1 + ORC_MLP_HID, *b2 = W2 + ORC_MLP_OUT * ORC_MLP_HID;
    float h[ORC_MLP_HID];
    for (int j = 0; j < ORC_MLP_HID; j++) {
        float a = b1[j];
        for (int i = 0; i < ORC_MLP_IN; i++) a = fmaf(W1[j * ORC_MLP_IN + i], x[i], a);
        h[j] = a > 0.0f ? a : 0.0f;
    }
    for (int k = 0; k < ORC_MLP_OUT; k++) {
        float a = b2[k];
        for (int j = 0; j < ORC_MLP_HID; j++) a = fmaf(W2[k * ORC_MLP_HID + j], h[j], a);
        s[k] = a;
    }
}

int orc_mlp_predict(const float *model, const float *x)
{
    float s[ORC_MLP_OUT];
    orc_mlp_scores(model, x, s);
    int best = 0;
    for (int k = 1; k < ORC_MLP_OUT; k++)
        if (s[k] > s[best]) best = k;
    return best;
}

/* Class of one block. Fixed t = 0 classes are taken as given; exhaustive is the
 * smallest valid class (ties to the lowest id); a fixed t > 0 class or the
 * learned prediction is kept only if valid and strictly smaller than class 0.
 * forced >= 0 replaces the learned prediction. */
static int choose_class(int variant, int forced, const uint64_t *d, uint64_t n, uint64_t B, uint64_t vmin)
{
    if (variant == 0 || variant == 8) return variant;
    uint64_t w0 = orc_class_words(0, d, n, B, NULL);
    int cand;
    if (variant == ORC_SELECT_EXHAUSTIVE) {
        cand = 0;
        uint64_t best = w0;
        for (int c = 1; c < 16; c++) {
            if (!orc_class_valid(c, B)) continue;
            uint64_t w = orc_class_words(c, d, n, B, NULL);
            if (w < best) {
                best = w;
                cand = c;
            }
        }
        return cand;
    }
    if (variant == ORC_SELECT_LEARNED) {
        if (forced >= 0) {
            cand = forced;
        } else {
            float x[ORC_MLP_IN];
            orc_block_features(d, n, vmin, vmin + B - 1, x);
            cand = orc_mlp_predict(g_model, x);
        }
    } else {
        cand = variant;
    }
    if (!orc_class_valid(cand, B)) return 0;
    if (orc_class_words(cand, d, n, B, NULL) < w0) return cand;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Stream layout (version 1), all fields little-endian:                      */
/*   [0,64)  header: u32 magic, u16 version, u8 dtype bytes w, u8 flags,    */
/*           u8 fixed class, u8 selector, u16 0, u32 L, u64 n, u64 blocks,  */
/*           u32 tile_blocks, u32 0, u64 payload words, u64 total bytes,    */
/*           u64 0                                                          */
/*   index[n_tiles] u64: payload word offset of block t * tile_blocks       */
/*   min[blocks]   (w bytes each)                                           */
/*   range[blocks] (w bytes each): B - 1                                    */
/*   class[blocks] u8            (flag ORC_F_CLASS)                         */
/*   ne[blocks]    u8 or u16     (flag ORC_F_NE; u16 iff L > 255)           */
/*   zero padding to a multiple of 8 bytes                                  */
/*   payload: u64 words, block after block                                  */
/* tile_blocks = the largest power of two P <= 256 with P * L * w <= 16384, */
/* at least 1.                                                              */
/* ---------------------------------------------------------------------- */
uint32_t orc_tile_blocks(uint32_t L, int w)
{
    uint64_t per = (uint64_t)L * (uint64_t)w;
    uint32_t P = 256;
    while (P > 1 && (uint64_t)P * per > 16384u) P >>= 1;
    return P;
}

static int variant_ok(int variant)
{
    return (variant >= 0 && variant < 16) || variant == ORC_SELECT_EXHAUSTIVE || variant == ORC_SELECT_LEARNED;
}

static unsigned stream_flags(int variant, uint32_t L)
{
    if (variant == 0 || variant == 8) return 0;
    return ORC_F_CLASS | ORC_F_NE | (L > 255 ? ORC_F_NE16 : 0);
}

typedef struct {
    uint64_t n_blocks, n_tiles, tile_blocks;
    uint64_t off_index, off_min, off_range, off_class, off_ne, off_payload;
    unsigned flags;
} orc_layout;

static void layout_of(uint64_t n, int w, uint32_t L, unsigned flags, orc_layout *lo)
{
    lo->n_blocks = (n + L - 1) / L;
    lo->tile_blocks = orc_tile_blocks(L, w);
    lo->n_tiles = (lo->n_blocks + lo->tile_blocks - 1) / lo->tile_blocks;
    lo->flags = flags;
    uint64_t o = ORC_HDR_BYTES;
    lo->off_index = o;
    o += 8 * lo->n_tiles;
    lo->off_min = o;
    o += (uint64_t)w * lo->n_blocks;
    lo->off_range = o;
    o += (uint64_t)w * lo->n_blocks;
    lo->off_class = o;
    if (flags & ORC_F_CLASS) o += lo->n_blocks;
    lo->off_ne = o;
    if (flags & ORC_F_NE) o += lo->n_blocks * ((flags & ORC_F_NE16) ? 2 : 1);
    lo->off_payload = (o + 7) & ~(uint64_t)7;
}

static uint64_t load_val(const void *in, int w, uint64_t i)
{
    if (w == 1) return ((const uint8_t *)in)[i];
    if (w == 2) return ((const uint16_t *)in)[i];
    return ((const uint32_t *)in)[i];
}

static void store_val(void *out, int w, uint64_t i, uint64_t v)
{
    if (w == 1)
        ((uint8_t *)out)[i] = (uint8_t)v;
    else if (w == 2)
        ((uint16_t *)out)[i] = (uint16_t)v;
    else
        ((uint32_t *)out)[i] = (uint32_t)v;
}

static void put_le(uint8_t *p, uint64_t v, int bytes)
{
    for (int i = 0; i < bytes; i++) p[i] = (uint8_t)(v >> (8 * i));
}

static uint64_t get_le(const uint8_t *p, int bytes)
{
    uint64_t v = 0;
    for (int i = 0; i < bytes; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

/* Worst-case stream size: every block at most basic t = 0 size, which is at
 * most ceil(L_b / (64 / w)) words because B <= 2^w. */
uint64_t orc_bound(uint64_t n, int w, uint32_t L, int variant)
{
    if (!(w == 1 || w == 2 || w == 4) || L == 0 || L > 65535 || !variant_ok(variant)) return 0;
    orc_layout lo;
    layout_of(n, w, L, stream_flags(variant, L), &lo);
    uint64_t per = 64 / (8 * (uint64_t)w);
    uint64_t words = 0;
    if (lo.n_blocks) {
        uint64_t last = n - (lo.n_blocks - 1) * L;
        words = (lo.n_blocks - 1) * ((L + per - 1) / per) + (last + per - 1) / per;
    }
    return lo.off_payload + 8 * words;
}

/* Compresses n values of w bytes in blocks of L. forced (length n_blocks) is
 * the externally chosen class vector used by the learned selector. Returns the
 * stream size in bytes, or a negative error. */
int64_t orc_compress(const void *in, uint64_t n, int w, uint32_t L, int variant, const uint8_t *forced,
                     uint8_t *out, uint64_t cap)
{
    if (!(w == 1 || w == 2 || w == 4) || L == 0 || L > 65535 || !variant_ok(variant)) return ORC_EINVAL;
    if (n && !in) return ORC_EINVAL;
    if (variant == ORC_SELECT_LEARNED && n && !forced && !g_have_model) return ORC_ENOMODEL;
    orc_layout lo;
    unsigned flags = stream_flags(variant, L);
    layout_of(n, w, L, flags, &lo);
    uint64_t nb = lo.n_blocks;

    uint64_t *mins = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    uint64_t *Bs = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    int *cls = (int *)calloc(nb + 1, sizeof(int));
    uint64_t *nes = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    uint64_t *nws = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * L);

    /* Pass 1: per block (Sec. 3.3) min, B, class, word count. */
    uint64_t total_words = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        uint64_t vmin = UINT64_MAX, vmax = 0;
        for (uint64_t j = 0; j < Lb; j++) {
            uint64_t v = load_val(in, w, first + j);
            if (v < vmin) vmin = v;
            if (v > vmax) vmax = v;
        }
        uint64_t B = vmax - vmin + 1; /* Sec. 3.1: B = v_max - v_min + 1 */
        for (uint64_t j = 0; j < Lb; j++) d[j] = load_val(in, w, first + j) - vmin;
        int c = choose_class(variant, forced ? forced[b] : -1, d, Lb, B, vmin);
        uint64_t ne = 0;
        uint64_t nw = orc_class_words(c, d, Lb, B, &ne);
        mins[b] = vmin;
        Bs[b] = B;
        cls[b] = c;
        nes[b] = ne;
        nws[b] = nw;
        total_words += nw;
    }
    uint64_t total = lo.off_payload + 8 * total_words;
    if (total > cap || !out) {
        free(mins); free(Bs); free(cls); free(nes); free(nws); free(d);
        return ORC_ENOSPC;
    }
    memset(out, 0, lo.off_payload);

    /* Header. */
    put_le(out + 0, ORC_MAGIC, 4);
    put_le(out + 4, ORC_VERSION, 2);
    out[6] = (uint8_t)w;
    out[7] = (uint8_t)flags;
    out[8] = (uint8_t)((flags & ORC_F_CLASS) ? 0 : variant);
    out[9] = (uint8_t)(variant == ORC_SELECT_EXHAUSTIVE ? 1 : variant == ORC_SELECT_LEARNED ? 2 : 0);
    put_le(out + 12, L, 4);
    put_le(out + 16, n, 8);
    put_le(out + 24, nb, 8);
    put_le(out + 32, lo.tile_blocks, 4);
    put_le(out + 40, total_words, 8);
    put_le(out + 48, total, 8);

    /* Pass 2: block arrays and payload. */
    uint64_t off = 0;
    uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * (L + 1));
    for (uint64_t b = 0; b < nb; b++) {
        if (b % lo.tile_blocks == 0) put_le(out + lo.off_index + 8 * (b / lo.tile_blocks), off, 8);
        put_le(out + lo.off_min + (uint64_t)w * b, mins[b], w);
        put_le(out + lo.off_range + (uint64_t)w * b, Bs[b] - 1, w);
        if (flags & ORC_F_CLASS) out[lo.off_class + b] = (uint8_t)cls[b];
        if (flags & ORC_F_NE) {
            int nb_ne = (flags & ORC_F_NE16) ? 2 : 1;
            put_le(out + lo.off_ne + (uint64_t)nb_ne * b, nes[b], nb_ne);
        }
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        for (uint64_t j = 0; j < Lb; j++) d[j] = load_val(in, w, first + j) - mins[b];
        uint64_t ne = 0;
        uint64_t nw = orc_class_pack(cls[b], d, Lb, Bs[b], words, &ne);
        for (uint64_t i = 0; i < nw; i++) put_le(out + lo.off_payload + 8 * (off + i), words[i], 8);
        off += nw;
    }
    free(words);
    free(mins); free(Bs); free(cls); free(nes); free(nws); free(d);
    return (int64_t)total;
}

/* Reads the header: returns 0 and fills n, w, L when the fixed fields are sane. */
int orc_stream_info(const uint8_t *in, uint64_t in_size, uint64_t *n, int *w, uint32_t *L, uint64_t *total)
{
    if (!in || in_size < ORC_HDR_BYTES) return ORC_ECORRUPT;
    if (get_le(in, 4) != ORC_MAGIC || get_le(in + 4, 2) != ORC_VERSION) return ORC_ECORRUPT;
    int ww = in[6];
    if (!(ww == 1 || ww == 2 || ww == 4)) return ORC_ECORRUPT;
    uint32_t LL = (uint32_t)get_le(in + 12, 4);
    if (LL == 0 || LL > 65535) return ORC_ECORRUPT;
    if (n) *n = get_le(in + 16, 8);
    if (w) *w = ww;
    if (L) *L = LL;
    if (total) *total = get_le(in + 48, 8);
    return 0;
}

/* Decompresses a whole stream into out (capacity in values). Returns the
 * number of values, or a negative error. */
int64_t orc_decompress(const uint8_t *in, uint64_t in_size, void *out, uint64_t out_cap_values)
{
    uint64_t n, total;
    int w;
    uint32_t L;
    int rc = orc_stream_info(in, in_size, &n, &w, &L, &total);
    if (rc) return rc;
    unsigned flags = in[7];
    if (flags & ~7u) return ORC_ECORRUPT;
    int fixed = in[8];
    orc_layout lo;
    layout_of(n, w, L, flags, &lo);
    if (get_le(in + 24, 8) != lo.n_blocks || get_le(in + 32, 4) != lo.tile_blocks) return ORC_ECORRUPT;
    uint64_t pw = get_le(in + 40, 8);
    if (total != lo.off_payload + 8 * pw || total > in_size) return ORC_ECORRUPT;
    if (!(flags & ORC_F_CLASS) && !(fixed == 0 || fixed == 8)) return ORC_ECORRUPT;
    if (n > out_cap_values) return ORC_ENOSPC;
    if (n && !out) return ORC_EINVAL;

    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * L);
    uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * (L + 1));
    uint64_t off = 0;
    int64_t result = (int64_t)n;
    for (uint64_t b = 0; b < lo.n_blocks; b++) {
        if (b % lo.tile_blocks == 0 && get_le(in + lo.off_index + 8 * (b / lo.tile_blocks), 8) != off) {
            result = ORC_ECORRUPT;
            break;
        }
        uint64_t vmin = get_le(in + lo.off_min + (uint64_t)w * b, w);
        uint64_t B = get_le(in + lo.off_range + (uint64_t)w * b, w) + 1;
        int c = (flags & ORC_F_CLASS) ? in[lo.off_class + b] : fixed;
        uint64_t ne = 0;
        if (flags & ORC_F_NE) {
            int nb_ne = (flags & ORC_F_NE16) ? 2 : 1;
            ne = get_le(in + lo.off_ne + (uint64_t)nb_ne * b, nb_ne);
        }
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        if (vmin + B - 1 > (w == 4 ? 0xFFFFFFFFull : (1ull << (8 * w)) - 1) || !orc_class_valid(c, B) ||
            ne > Lb || ((c & 7) == 0 && ne != 0)) {
            result = ORC_ECORRUPT;
            break;
        }
        int family = c >> 3;
        uint64_t nw;
        if ((c & 7) == 0) {
            nw = orc_family_words(family, Lb, B, 64);
        } else {
            uint64_t T = class_threshold(c, B);
            nw = orc_family_words(family, Lb, T + 1, 64) + orc_family_words(family, ne, B - T, 64);
        }
        if (off + nw > pw) {
            result = ORC_ECORRUPT;
            break;
        }
        for (uint64_t i = 0; i < nw; i++) words[i] = get_le(in + lo.off_payload + 8 * (off + i), 8);
        orc_class_unpack(c, words, Lb, B, ne, d);
        for (uint64_t j = 0; j < Lb; j++) store_val(out, w, first + j, d[j] + vmin);
        off += nw;
    }
    if (result >= 0 && off != pw) result = ORC_ECORRUPT;
    free(d);
    free(words);
    return result;
}

/* Per-block facts for tests: min, B, class, n_e, word count for every block of a stream's input. */
int orc_block_facts(const void *in, uint64_t n, int w, uint32_t L, int variant, const uint8_t *forced,
                    uint64_t *mins, uint64_t *Bs, uint8_t *cls, uint64_t *nes, uint64_t *nws)
{
    if (!(w == 1 || w == 2 || w == 4) || L == 0 || !variant_ok(variant)) return ORC_EINVAL;
    if (variant == ORC_SELECT_LEARNED && n && !forced && !g_have_model) return ORC_ENOMODEL;
    uint64_t nb = (n + L - 1) / L;
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * L);
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        uint64_t vmin = UINT64_MAX, vmax = 0;
        for (uint64_t j = 0; j < Lb; j++) {
            uint64_t v = load_val(in, w, first + j);
            if (v < vmin) vmin = v;
            if (v > vmax) vmax = v;
        }
        uint64_t B = vmax - vmin + 1;
        for (uint64_t j = 0; j < Lb; j++) d[j] = load_val(in, w, first + j) - vmin;
        int c = choose_class(variant, forced ? forced[b] : -1, d, Lb, B, vmin);
        uint64_t ne = 0;
        uint64_t nw = orc_class_words(c, d, Lb, B, &ne);
        if (mins) mins[b] = vmin;
        if (Bs) Bs[b] = B;
        if (cls) cls[b] = (uint8_t)c;
        if (nes) nes[b] = ne;
        if (nws) nws[b] = nw;
    }
    free(d);
    return 0;
}

/* Sizes of all 16 classes of one block of digits (UINT64_MAX for invalid classes). */
void orc_all_class_words(const uint64_t *d, uint64_t n, uint64_t B, uint64_t *words16, uint64_t *ne16)
{
    for (int c = 0; c < 16; c++) {
        if (!orc_class_valid(c, B)) {
            words16[c] = UINT64_MAX;
            ne16[c] = 0;
            continue;
        }
        words16[c] = orc_class_words(c, d, n, B, &ne16[c]);
    }
}

/* Features (19 floats per block, as the learned selector reads them) and the
 * sizes of all 16 classes (UINT64_MAX when invalid) of every block of an array. */
int orc_features(const void *in, uint64_t n, int w, uint32_t L, float *x, uint64_t *words16)
{
    if (!(w == 1 || w == 2 || w == 4) || L == 0) return ORC_EINVAL;
    uint64_t nb = (n + L - 1) / L;
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * L);
    uint64_t ne16[16];
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        uint64_t vmin = UINT64_MAX, vmax = 0;
        for (uint64_t j = 0; j < Lb; j++) {
            uint64_t v = load_val(in, w, first + j);
            if (v < vmin) vmin = v;
            if (v > vmax) vmax = v;
        }
        for (uint64_t j = 0; j < Lb; j++) d[j] = load_val(in, w, first + j) - vmin;
        if (x) orc_block_features(d, Lb, vmin, vmax, x + ORC_MLP_IN * b);
        if (words16) orc_all_class_words(d, Lb, vmax - vmin + 1, words16 + 16 * b, ne16);
    }
    free(d);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Streams of 32-bit words: the paper's own word, the unsigned int of       */
/* Sec. 3.1 (Eq. (1) with capacity 2^32) and of the Sec. 3.2 series. Only   */
/* the paper's two packings, t = 0: class 0 (basic) and class 8 (advanced). */
/* Variants: 0, 8 (every block in that class) and ORC_SELECT_EXHAUSTIVE     */
/* (per block the smaller of the two, ties to basic). Advanced packing is   */
/* offered for u8 and u16 data only (every base then lies in [1, 2^16 + 1]);*/
/* u32 data take variant 0.                                                 */
/* Layout: that of orc_compress with flags ORC_F_W32 (plus ORC_F_CLASS for  */
/* the exhaustive variant, no excess counts); the header's payload-word     */
/* count, the tile index and the payload count 32-bit words, and the       */
/* payload holds u32 words; total bytes = payload offset + 4 x words.       */
/* ---------------------------------------------------------------------- */
static int variant32_ok(int variant, int w)
{
    if (variant == 0) return 1;
    return (variant == 8 || variant == ORC_SELECT_EXHAUSTIVE) && w < 4;
}

static unsigned stream_flags32(int variant)
{
    return ORC_F_W32 | (variant == ORC_SELECT_EXHAUSTIVE ? ORC_F_CLASS : 0);
}

/* Worst case: every block in at most ceil(L_b / (4 / w)) words (B <= 2^(8w)
 * gives at least 32 / (8w) digits per word, and the advanced series never
 * takes more words than the basic packing: each of its words closes p_i + 1
 * >= k values). */
uint64_t orc_bound32(uint64_t n, int w, uint32_t L, int variant)
{
    if (!(w == 1 || w == 2 || w == 4) || L == 0 || L > 65535 || !variant32_ok(variant, w)) return 0;
    orc_layout lo;
    layout_of(n, w, L, stream_flags32(variant), &lo);
    uint64_t per = 4 / (uint64_t)w;
    uint64_t words = 0;
    if (lo.n_blocks) {
        uint64_t last = n - (lo.n_blocks - 1) * L;
        words = (lo.n_blocks - 1) * ((L + per - 1) / per) + (last + per - 1) / per;
    }
    return lo.off_payload + 4 * words;
}

int64_t orc_compress32(const void *in, uint64_t n, int w, uint32_t L, int variant, uint8_t *out, uint64_t cap)
{
    if (!(w == 1 || w == 2 || w == 4) || L == 0 || L > 65535 || !variant32_ok(variant, w)) return ORC_EINVAL;
    if (n && !in) return ORC_EINVAL;
    orc_layout lo;
    unsigned flags = stream_flags32(variant);
    layout_of(n, w, L, flags, &lo);
    uint64_t nb = lo.n_blocks;
    uint64_t *mins = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    uint64_t *Bs = (uint64_t *)calloc(nb + 1, sizeof(uint64_t));
    int *cls = (int *)calloc(nb + 1, sizeof(int));
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * L);

    /* Pass 1: per block min, B (Sec. 3.1) and the class. */
    uint64_t total_words = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        uint64_t vmin = UINT64_MAX, vmax = 0;
        for (uint64_t j = 0; j < Lb; j++) {
            uint64_t v = load_val(in, w, first + j);
            if (v < vmin) vmin = v;
            if (v > vmax) vmax = v;
        }
        uint64_t B = vmax - vmin + 1;
        uint64_t w0 = orc_family_words(0, Lb, B, 32);
        int c = variant == ORC_SELECT_EXHAUSTIVE ? (orc_family_words(1, Lb, B, 32) < w0 ? 8 : 0) : variant;
        mins[b] = vmin;
        Bs[b] = B;
        cls[b] = c;
        total_words += orc_family_words(c >> 3, Lb, B, 32);
    }
    uint64_t total = lo.off_payload + 4 * total_words;
    if (total > cap || !out) {
        free(mins); free(Bs); free(cls); free(d);
        return ORC_ENOSPC;
    }
    memset(out, 0, lo.off_payload);
    put_le(out + 0, ORC_MAGIC, 4);
    put_le(out + 4, ORC_VERSION, 2);
    out[6] = (uint8_t)w;
    out[7] = (uint8_t)flags;
    out[8] = (uint8_t)(variant == ORC_SELECT_EXHAUSTIVE ? 0 : variant);
    out[9] = (uint8_t)(variant == ORC_SELECT_EXHAUSTIVE ? 1 : 0);
    put_le(out + 12, L, 4);
    put_le(out + 16, n, 8);
    put_le(out + 24, nb, 8);
    put_le(out + 32, lo.tile_blocks, 4);
    put_le(out + 40, total_words, 8);
    put_le(out + 48, total, 8);

    /* Pass 2: block arrays and payload (each word stored as 4 bytes). */
    uint64_t off = 0;
    uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * (L + 1));
    for (uint64_t b = 0; b < nb; b++) {
        if (b % lo.tile_blocks == 0) put_le(out + lo.off_index + 8 * (b / lo.tile_blocks), off, 8);
        put_le(out + lo.off_min + (uint64_t)w * b, mins[b], w);
        put_le(out + lo.off_range + (uint64_t)w * b, Bs[b] - 1, w);
        if (flags & ORC_F_CLASS) out[lo.off_class + b] = (uint8_t)cls[b];
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        for (uint64_t j = 0; j < Lb; j++) d[j] = load_val(in, w, first + j) - mins[b];
        uint64_t nw = orc_family_pack(cls[b] >> 3, d, Lb, Bs[b], 32, words);
        for (uint64_t i = 0; i < nw; i++) put_le(out + lo.off_payload + 4 * (off + i), words[i], 4);
        off += nw;
    }
    free(words);
    free(mins); free(Bs); free(cls); free(d);
    return (int64_t)total;
}

int64_t orc_decompress32(const uint8_t *in, uint64_t in_size, void *out, uint64_t out_cap_values)
{
    uint64_t n, total;
    int w;
    uint32_t L;
    int rc = orc_stream_info(in, in_size, &n, &w, &L, &total);
    if (rc) return rc;
    unsigned flags = in[7];
    if ((flags & ~(ORC_F_W32 | ORC_F_CLASS)) || !(flags & ORC_F_W32)) return ORC_ECORRUPT;
    int fixed = in[8];
    orc_layout lo;
    layout_of(n, w, L, flags, &lo);
    if (get_le(in + 24, 8) != lo.n_blocks || get_le(in + 32, 4) != lo.tile_blocks) return ORC_ECORRUPT;
    uint64_t pw = get_le(in + 40, 8);
    if (total != lo.off_payload + 4 * pw || total > in_size) return ORC_ECORRUPT;
    if (!(flags & ORC_F_CLASS) && !(fixed == 0 || fixed == 8)) return ORC_ECORRUPT;
    if (n > out_cap_values) return ORC_ENOSPC;
    if (n && !out) return ORC_EINVAL;
    uint64_t *d = (uint64_t *)malloc(sizeof(uint64_t) * L);
    uint64_t *words = (uint64_t *)malloc(sizeof(uint64_t) * (L + 1));
    uint64_t off = 0;
    int64_t result = (int64_t)n;
    for (uint64_t b = 0; b < lo.n_blocks; b++) {
        if (b % lo.tile_blocks == 0 && get_le(in + lo.off_index + 8 * (b / lo.tile_blocks), 8) != off) {
            result = ORC_ECORRUPT;
            break;
        }
        uint64_t vmin = get_le(in + lo.off_min + (uint64_t)w * b, w);
        uint64_t B = get_le(in + lo.off_range + (uint64_t)w * b, w) + 1;
        int c = (flags & ORC_F_CLASS) ? in[lo.off_class + b] : fixed;
        uint64_t first = b * L;
        uint64_t Lb = (n - first < L) ? (n - first) : L;
        /* classes 0 and 8 only; advanced blocks need B <= 2^16 + 1 */
        if (vmin + B - 1 > (w == 4 ? 0xFFFFFFFFull : (1ull << (8 * w)) - 1) || (c != 0 && c != 8) ||
            (c == 8 && B > 65537)) {
            result = ORC_ECORRUPT;
            break;
        }
        uint64_t nw = orc_family_words(c >> 3, Lb, B, 32);
        if (off + nw > pw) {
            result = ORC_ECORRUPT;
            break;
        }
        for (uint64_t i = 0; i < nw; i++) words[i] = get_le(in + lo.off_payload + 4 * (off + i), 4);
        if (B <= 1)
            for (uint64_t j = 0; j < Lb; j++) d[j] = 0;
        else
            orc_family_unpack(c >> 3, words, Lb, B, 32, d);
        for (uint64_t j = 0; j < Lb; j++) store_val(out, w, first + j, d[j] + vmin);
        off += nw;
    }
    if (result >= 0 && off != pw) result = ORC_ECORRUPT;
    free(d);
    free(words);
    return result;
}
