// kernels_common.h -- pieces shared by the compress and decompress kernels (device code).
#pragma once
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "pcomp_internal.h"

namespace pcomp {

template <int W>
struct Elem;
template <>
struct Elem<1> {
    typedef uint8_t T;
    typedef uint32_t Base;  // holds B = max - min + 1
};
template <>
struct Elem<2> {
    typedef uint16_t T;
    typedef uint32_t Base;
};
template <>
struct Elem<4> {
    typedef uint32_t T;
    typedef uint64_t Base;
};

// Lanes per block from which advanced words are decoded in runs of consecutive words per lane
// (fewer lanes take every G-th word; packing always uses runs).
constexpr uint32_t kRunLanes = 8;

// ---------------------------------------------------------------------------------------
// Group collectives: G lanes (a power of two, aligned) cooperate on one block. Within a
// wavefront they use cross-lane shuffles; groups wider than a wavefront combine per-wave
// partials through LDS. Every thread of the workgroup must call these (they may hold
// barriers when G > 64).
// ---------------------------------------------------------------------------------------
template <typename T, typename Op>
__device__ __forceinline__ T group_reduce(T x, uint32_t G, Op op, T *scratch) {
    const uint32_t width = G < 64 ? G : 64;
    for (uint32_t o = 1; o < width; o <<= 1) x = op(x, __shfl_xor(x, o, 64));
    if (G > 64) {
        const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        __syncthreads();
        if (lane == 0) scratch[wave] = x;
        __syncthreads();
        const uint32_t wpg = G >> 6, w0 = (wave / wpg) * wpg;
        T r = scratch[w0];
        for (uint32_t i = 1; i < wpg; i++) r = op(r, scratch[w0 + i]);
        x = r;
        __syncthreads();
    }
    return x;
}

// Exclusive prefix sum over the G lanes of a group, in lane order.
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t x, uint32_t G, uint32_t *scratch) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t width = G < 64 ? G : 64;
    const uint32_t gl = lane & (width - 1);
    uint32_t inc = x;
    for (uint32_t o = 1; o < width; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, width);
        if (gl >= o) inc += y;
    }
    uint32_t excl = inc - x;
    if (G > 64) {
        const uint32_t wave = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 63) scratch[wave] = inc;
        __syncthreads();
        const uint32_t wpg = G >> 6, w0 = (wave / wpg) * wpg;
        for (uint32_t i = w0; i < wave; i++) excl += scratch[i];
        __syncthreads();
    }
    return excl;
}

// Exclusive prefix sum of x over the workgroup (thread order); *total gets the sum.
__device__ __forceinline__ uint32_t wg_excl_scan(uint32_t x, uint32_t *scratch, uint32_t *total) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) scratch[wave] = inc;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (uint32_t w = 0; w < kThreads / 64; w++) {
        const uint32_t v = scratch[w];
        add += w < wave ? v : 0;
        tot += v;
    }
    __syncthreads();
    *total = tot;
    return inc - x + add;
}

// Exclusive prefix sum of 64-bit x over the workgroup; *total gets the sum. It ends without
// a barrier after reading scratch: the caller writes scratch again only after a later one.
__device__ __forceinline__ uint64_t wg_excl_scan64(uint64_t x, uint64_t *scratch, uint64_t *total) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t inc = x;
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) scratch[wave] = inc;
    __syncthreads();
    uint64_t add = 0, tot = 0;
    for (uint32_t w = 0; w < kThreads / 64; w++) {
        const uint64_t v = scratch[w];
        add += w < wave ? v : 0;
        tot += v;
    }
    *total = tot;
    return inc - x + add;
}

// Scalar-register copies of values that every lane of the wavefront holds equally (segment
// descriptors read from memory): keeps them out of vector registers.
__device__ __forceinline__ uint32_t uni32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return ((uint64_t)uni32((uint32_t)(x >> 32)) << 32) | uni32((uint32_t)x);
}
__device__ __forceinline__ SegDesc uniform_seg(const SegDesc &s) {
    SegDesc u;
    u.data = (const uint8_t *)uni64((uint64_t)(uintptr_t)s.data);
    u.lo.n = uni64(s.lo.n);
    u.lo.n_blocks = uni64(s.lo.n_blocks);
    u.lo.n_tiles = uni64(s.lo.n_tiles);
    u.lo.L = uni32(s.lo.L);
    u.lo.w = uni32(s.lo.w);
    u.lo.tile_blocks = uni32(s.lo.tile_blocks);
    u.lo.flags = uni32(s.lo.flags);
    u.lo.off_index = uni64(s.lo.off_index);
    u.lo.off_min = uni64(s.lo.off_min);
    u.lo.off_range = uni64(s.lo.off_range);
    u.lo.off_class = uni64(s.lo.off_class);
    u.lo.off_ne = uni64(s.lo.off_ne);
    u.lo.off_payload = uni64(s.lo.off_payload);
    u.tile0 = uni64(s.tile0);
    u.user = uni32(s.user);
    u.group = uni32(s.group);
    u.rows = uni32(s.rows);
    u.cols = uni32(s.cols);
    return u;
}

// Time-major blocking: where value t of the stream sits in the caller's matrices [rows][cols]
// (t = (e cols + c) rows + r, element (e, r, c)), and the same walk in steps of kThreads.
struct TmCursor {
    uint64_t e;
    uint32_t r, c, rows, cols, dr, dc;
    __device__ TmCursor(uint64_t t, uint32_t rows_, uint32_t cols_) : rows(rows_), cols(cols_) {
        const uint64_t mat = (uint64_t)rows * cols;
        e = t / mat;
        const uint64_t rem = t - e * mat;
        c = (uint32_t)(rem / rows);
        r = (uint32_t)(rem - (uint64_t)c * rows);
        dc = kThreads / rows;
        dr = kThreads - dc * rows;
    }
    __device__ __forceinline__ uint64_t index() const { return (e * rows + r) * cols + c; }
    __device__ __forceinline__ void step() {
        r += dr;
        c += dc;
        if (r >= rows) {
            r -= rows;
            c++;
        }
        while (c >= cols) {
            c -= cols;
            e++;
        }
    }
};

// Stages the input of one tile in LDS (16-byte chunks; the partial chunks at the ends by
// element) and returns the LDS address of its first value.
template <int W>
__device__ __forceinline__ const typename Elem<W>::T *stage_tile(const uint8_t *in, uint64_t v0, uint32_t nvt,
                                                                  uint4 *s_raw) {
    typedef typename Elem<W>::T V;
    uint8_t *s_bytes = (uint8_t *)s_raw;
    const uintptr_t addr = (uintptr_t)(in + v0 * W);
    const uint32_t head = (uint32_t)(addr & 15);
    const uint8_t *gbase = (const uint8_t *)(addr - head);
    const uint32_t span = head + nvt * W;
    const uint32_t nchunks = (span + 15) >> 4;
    for (uint32_t c = threadIdx.x; c < nchunks; c += kThreads) {
        const uint32_t cb = c << 4;
        if (cb >= head && cb + 16 <= span) {
            s_raw[c] = *(const uint4 *)(gbase + cb);
        } else {
            const uint32_t e0 = cb > head ? cb : head, e1 = cb + 16 < span ? cb + 16 : span;
            for (uint32_t b = e0; b < e1; b += W) *(V *)(s_bytes + b) = *(const V *)(gbase + b);
        }
    }
    return (const V *)(s_bytes + head);
}

// Workgroups are dispatched to the 8 XCDs (each with its own L2) in turn: workgroup b runs on
// XCD b mod 8. xcd_order(b, n) renumbers the n workgroups of a launch so that each XCD takes one
// contiguous run of the numbers, and tiles next to each other share an L2 (a bijection of
// [0, n)).
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t n) {
    const uint32_t x = b & 7, q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// A pointer into LDS, as the compiler sees it: a staged tile chosen among several buffers can
// lose that address space, and its reads would then take flat addressing.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(3))) T *lds_ptr(const T *p) {
    return (const __attribute__((address_space(3))) T *)p;
}

struct MinOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a < b ? a : b; }
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a < b ? a : b; }
};
struct MaxOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a > b ? a : b; }
};
struct AddOp {
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; }
};

// ---------------------------------------------------------------------------------------
// Word counts with per-workgroup caches in LDS: k(B) by octave, and, for the main part of
// threshold classes (base 2^j + 1), k and the word counts of a full block.
// ---------------------------------------------------------------------------------------

// k(B) = max{k : B^k <= 2^64} (Sec. 3.1 Eq. (1), exact reading) for 2 <= B <= 2^32, from small
// tables: k8[B] for B <= 256; above, B lies in the octave e = bitlen(B - 1) >= 9, where k takes
// one of two values, ktop[e] = k(2^(e-1) + 1) or one less (64 / (e - 1) - 64 / e < 1 for
// e >= 9), the larger iff B - 1 <= km1[ktop[e]] = kmax(ktop[e]) - 1 (kmax(k), the largest base
// with k digits per word, is at most 2^32 for k >= 2).
__host__ __device__ __forceinline__ uint32_t k_octave(const uint8_t *k8, const uint8_t *ktop, const uint32_t *km1,
                                                      uint64_t B) {
    if (B <= 256) return k8[B];
    const uint32_t bm1 = (uint32_t)(B - 1);
    const uint32_t e = 32 - (uint32_t)__builtin_clz(bm1);
    const uint32_t kc = ktop[e];
    return kc - (bm1 > km1[kc] ? 1u : 0u);
}

// Entries of those tables, from k(B) for B <= 2^16 + 1 (ktab) and the bounds kmax[k].
__host__ __device__ __forceinline__ uint32_t ktop_entry(const uint8_t *ktab, const uint64_t *kmax, uint32_t e) {
    if (e < 9) return 0;  // not used: B <= 256 reads k8
    const uint64_t B = (1ull << (e - 1)) + 1;
    if (B <= kAtlasDirect) return ktab[B];
    uint32_t k = 64 / (e - 1);  // at least k(B); at most two steps down
    while (B > kmax[k]) k--;
    return k;
}
__host__ __device__ __forceinline__ uint32_t km1_entry(const uint64_t *kmax, uint32_t k) {
    return k >= 2 ? (uint32_t)((kmax[k] < (1ull << 32) ? kmax[k] : (1ull << 32)) - 1) : 0xFFFFFFFFu;
}

struct SizeCtx {
    uint8_t k8[260];  // k(B) for B <= 256 (0 for B < 2)
    uint8_t ktop[36];
    uint32_t km1[8];  // k <= 7 above B = 256
    uint32_t p1_k[32];
    uint32_t p1_adv[32];
    uint32_t p1_basic[32];  // basic words of a full block of base 2^j + 1
    // per base B <= 2^16 + 1: words of a full block, basic (bits 0-15) and advanced (16-31), or nullptr
    const uint32_t *fullW;
};

__device__ __forceinline__ void fill_size_ctx(const DevTables &T, uint32_t L, SizeCtx &C, const uint32_t *fullW = nullptr) {
    const uint32_t t = threadIdx.x;
    if (t == 200) C.fullW = fullW;
    if (t < 256) C.k8[t] = T.ktab[t];
    if (t == 0) C.k8[256] = T.ktab[256];
    if (t >= 160 && t < 160 + 33) C.ktop[t - 160] = (uint8_t)ktop_entry(T.ktab, T.kmax, t - 160);
    if (t >= 224 && t < 232) C.km1[t - 224] = km1_entry(T.kmax, t - 224);
    if (t >= 96 && t < 128) {
        const uint32_t j = t - 96;
        const BaseDesc &D = T.desc[atlas_index((1ull << j) + 1)];
        C.p1_k[j] = D.k;
        C.p1_adv[j] = adv_words_atlas(T, D, L);
        C.p1_basic[j] = udiv_small(L + D.k - 1, D.k);
    }
}

__device__ __forceinline__ uint32_t k_fast(const SizeCtx &C, uint64_t B) { return k_octave(C.k8, C.ktop, C.km1, B); }

// Words of family fam (0 basic Sec. 3.1, 1 advanced Sec. 3.2) for n digits of `base`;
// `full` is the block length L (a block of n == L values can use the cache). Wide: the data
// are u32, so a base can lie outside the tables (u8 and u16 bases never do).
template <bool Wide>
__device__ __forceinline__ uint32_t fam_words(const DevTables &T, const SizeCtx &C, int fam, uint32_t n, uint64_t base,
                                     uint32_t full) {
    if (n == 0 || base <= 1) return 0;
    const uint32_t k = k_fast(C, base);
    if (!fam) return udiv_small(n + k - 1, k);
    if (n <= k) return 1;
    if (n == full && C.fullW && base <= kAtlasDirect)
        return ((const __attribute__((address_space(1))) uint32_t *)C.fullW)[base] >> 16;  // global, not flat
    const uint64_t bm1 = base - 1;
    if ((bm1 & (bm1 - 1)) == 0 && n == full) return C.p1_adv[bitlen64(bm1) - 1];  // base 2^j + 1
    const int ai = atlas_index(base);
    if (ai >= 0) return adv_words_atlas(T, T.desc[ai], n);
    if (!Wide) return 0;  // unreachable: every u8 / u16 base is in the tables
    return adv_words_slow(slow_base(T, base), n);
}

// Words of the main part (digits min(d, T) in base T + 1, T = 2^(beta - t)) of a threshold
// class, t >= 1: a lower bound of the class's words.
template <bool Wide>
__device__ __forceinline__ uint32_t main_words(const DevTables &T, const SizeCtx &C, uint32_t L, int fam, int t,
                                               uint32_t Lb, uint32_t beta) {
    const uint32_t j = beta - t;
    if (!fam) return Lb == L ? C.p1_basic[j] : udiv_small(Lb + C.p1_k[j] - 1, C.p1_k[j]);
    return (Lb == L) ? C.p1_adv[j] : fam_words<Wide>(T, C, 1, Lb, (1ull << j) + 1, L);
}

// Advanced words of n digits of `base` once its k is known: one word for n <= k, else the
// series' bounds ceil((n+1)/(k+1)) <= words <= ceil(n/k) (every word after the first takes k
// or k + 1 values), and the series itself only where they differ.
template <bool Wide>
__device__ __forceinline__ uint32_t adv_words_k(const DevTables &T, const SizeCtx &C, uint32_t n, uint64_t base,
                                                uint32_t k, uint32_t full) {
    if (n <= k) return 1;
    const uint32_t lo = udiv_small(n + 1 + k, k + 1), hi = udiv_small(n + k - 1, k);
    if (lo == hi) return lo;
    return fam_words<Wide>(T, C, 1, n, base, full);
}

// Words of class c = 8 family + t for a block of Lb digits of base B (beta = bitlen(B-1));
// ne_t = digits >= T = 2^(beta - t). nw_main receives the main-part words.
template <bool Wide>
__device__ __forceinline__ uint32_t class_words(const DevTables &T, const SizeCtx &C, uint32_t L, int c, uint32_t Lb,
                                       uint64_t B, uint32_t beta, uint32_t ne_t, uint32_t &nw_main) {
    const int fam = c >> 3, t = c & 7;
    if (t == 0) {
        nw_main = fam_words<Wide>(T, C, fam, Lb, B, L);
        return nw_main;
    }
    const uint32_t j = beta - t;
    const uint64_t Th = 1ull << j;
    if (!fam)
        nw_main = udiv_small(Lb + C.p1_k[j] - 1, C.p1_k[j]);
    else
        nw_main = (Lb == L) ? C.p1_adv[j] : fam_words<Wide>(T, C, 1, Lb, Th + 1, L);
    return nw_main + fam_words<Wide>(T, C, fam, ne_t, B - Th, L);
}

// ---------------------------------------------------------------------------------------
// Learned class selector: 19 features of a block -> 64 ReLU units -> 16 class scores.
// Features use correctly rounded binary32 operations only (so every IEEE implementation
// gets the same bits): x[b] = H[b] / L_b for the 16-bin octave histogram
// H[b] = #{j : min(beta - bitlen(d_j), 15) = b}; x[16], x[17] = lg(min + 1) / 32,
// lg(max + 1) / 32 with the piecewise-linear base-2 logarithm lg(u) = e + (u - 2^e) 2^-e
// for 2^e <= u < 2^(e+1); x[18] = L_b / 4096. Every sum of the network is a chain of fused
// multiply-adds in index order starting from the bias. Parameters: W1 (64 x 19,
// row-major), b1 (64), W2 (16 x 64), b2 (16).
// ---------------------------------------------------------------------------------------
constexpr int kMlpIn = 19, kMlpHid = 64, kMlpOut = 16;
constexpr int kMlpW1 = 0, kMlpB1 = kMlpHid * kMlpIn, kMlpW2 = kMlpB1 + kMlpHid, kMlpB2 = kMlpW2 + kMlpOut * kMlpHid;
constexpr int kMlpParams = kMlpB2 + kMlpOut;  // 2320

__device__ __forceinline__ float lg_f32(uint64_t u) {  // u >= 1
    const int e = 63 - __clzll(u);
    const float frac = ldexpf((float)(uint32_t)(u - (1ull << e)), -e);
    return (float)e + frac;
}

// x[0..18] from the histogram (16 counts), L_b and the block's min and max.
__device__ __forceinline__ void block_features(const uint32_t *H, uint32_t Lb, uint64_t vmin, uint64_t vmax,
                                               float *x) {
    const float fl = (float)Lb;
#pragma unroll
    for (int b = 0; b < 16; b++) x[b] = (float)H[b] / fl;
    x[16] = lg_f32(vmin + 1) * 0.03125f;
    x[17] = lg_f32(vmax + 1) * 0.03125f;
    x[18] = fl * (1.0f / 4096.0f);
}

// Feature f alone, the same value as block_features' x[f]; the counts come packed four to a word
// (bin b in bits 16 (b mod 4) of word b / 4), selected without a dynamic register index.
__device__ __forceinline__ float block_feature(uint32_t f, const uint64_t *hw, uint32_t Lb, uint64_t vmin,
                                               uint64_t vmax) {
    const float fl = (float)Lb;
    if (f < 16) {
        const uint32_t q = f >> 2;
        const uint64_t w = q == 0 ? hw[0] : q == 1 ? hw[1] : q == 2 ? hw[2] : hw[3];
        return (float)((uint32_t)(w >> (16 * (f & 3))) & 0xFFFFu) / fl;
    }
    if (f < 18) return lg_f32((f == 16 ? vmin : vmax) + 1) * 0.03125f;
    return fl * (1.0f / 4096.0f);
}

// The 16 scores; P(i) returns parameter i.
template <typename P>
__device__ __forceinline__ void mlp_scores(P prm, const float *x, float *s) {
#pragma unroll
    for (int k = 0; k < kMlpOut; k++) s[k] = prm(kMlpB2 + k);
    for (int j = 0; j < kMlpHid; j++) {
        float a = prm(kMlpB1 + j);
#pragma unroll
        for (int i = 0; i < kMlpIn; i++) a = __builtin_fmaf(prm(kMlpW1 + j * kMlpIn + i), x[i], a);
        a = a > 0.0f ? a : 0.0f;
#pragma unroll
        for (int k = 0; k < kMlpOut; k++) s[k] = __builtin_fmaf(prm(kMlpW2 + k * kMlpHid + j), a, s[k]);
    }
}

// First index of the largest score.
__device__ __forceinline__ int argmax16(const float *s) {
    int best = 0;
    float bv = s[0];
#pragma unroll
    for (int k = 1; k < kMlpOut; k++) {
        const bool gt = s[k] > bv;
        best = gt ? k : best;
        bv = gt ? s[k] : bv;
    }
    return best;
}

// Per-lane octave histogram of digits: bins 0..7 and 8..15 (capped) as eight 8-bit counters
// each (at most 64 digits per lane), widened to four words of four 16-bit counters.
struct Hist16 {
    uint64_t w[4];
};

__device__ __forceinline__ void hist_widen(uint64_t lo8, uint64_t hi8, Hist16 &h) {
    h.w[0] = h.w[1] = h.w[2] = h.w[3] = 0;
#pragma unroll
    for (int t = 0; t < 4; t++) {
        h.w[0] |= ((lo8 >> (8 * t)) & 0xFF) << (16 * t);
        h.w[1] |= ((lo8 >> (8 * (t + 4))) & 0xFF) << (16 * t);
        h.w[2] |= ((hi8 >> (8 * t)) & 0xFF) << (16 * t);
        h.w[3] |= ((hi8 >> (8 * (t + 4))) & 0xFF) << (16 * t);
    }
}

// The same from 8-bit counters of the even bins (ev8, byte i = bin 2i) and the odd bins (od8).
__device__ __forceinline__ void hist_widen_eo(uint64_t ev8, uint64_t od8, Hist16 &h) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const uint64_t e = (ev8 >> (16 * q)) & 0xFFFF, o = (od8 >> (16 * q)) & 0xFFFF;  // bins 4q .. 4q + 3
        h.w[q] = (e & 0xFF) | ((o & 0xFF) << 16) | ((e >> 8) << 32) | ((o >> 8) << 48);
    }
}

__device__ __forceinline__ uint32_t hist_bin(const Hist16 &h, int b) {
    return (uint32_t)(h.w[b >> 2] >> (16 * (b & 3))) & 0xFFFF;
}

// ---------------------------------------------------------------------------------------
// Digit arithmetic in 32-bit chunks (see Chunk).
// ---------------------------------------------------------------------------------------
// One base-B digit off x < 2^51 (held exactly in binary64): returns floor(x / B) and sets
// d = x mod B. The quotient is trunc(fma(x, rB, rB/2)) with rB = 1/B rounded to nearest:
// (x + 1/2) / B lies at least 1/(2B) from every integer (2x + 1 is odd), and the computed value
// is within a relative 2^-52 of it, an error below (x + 1/2) 2^-52 / B < 1/(2B) for x < 2^51;
// so the truncation is floor(x / B) exactly, and fma(-q, B, x) is the exact remainder.
__host__ __device__ __forceinline__ double digit_off(double x, double rB, double hB, double Bf, uint32_t &d) {
    const double q = __builtin_trunc(__builtin_fma(x, rB, hB));
    d = (uint32_t)__builtin_fma(-q, Bf, x);
    return q;
}

// Splits X < 2^64 at P (2^13 <= P <= 2^32, exact in binary64; rP = 1/P rounded to nearest):
// hi = floor(X / P) < 2^51 and lo = X mod P, both exact binary64 integers.
// With X = xh 2^32 + xl: q1 = floor(xh / P) and r1 = xh mod P as in digit_off (xh < 2^32);
// the rest Y = r1 2^32 + xl < P 2^32 then has Y / P < 2^32, and its binary64 estimate (Y rounded,
// times rP, plus 2^-18) errs by less than 2^-19.4 before the added 2^-18, so its truncation is
// floor(Y / P) or one more. lo = Y - q2 P is computed exactly (an integer below 2^34 in
// magnitude); a negative lo means q2 was one too many.
__host__ __device__ __forceinline__ void split_word(uint64_t X, double P, double rP, double &hi, double &lo) {
    const double dh = (double)(uint32_t)(X >> 32), dl = (double)(uint32_t)X;
    const double q1 = __builtin_trunc(__builtin_fma(dh, rP, 0.5 * rP));
    const double r1s = __builtin_ldexp(__builtin_fma(-q1, P, dh), 32);  // (xh mod P) 2^32, exact
    double q2 = __builtin_trunc(__builtin_fma(r1s + dl, rP, 0x1p-18));
    double r = __builtin_fma(-q2, P, r1s) + dl;
    const bool over = r < 0.0;
    r = over ? r + P : r;
    q2 = over ? q2 - 1.0 : q2;
    hi = __builtin_ldexp(q1, 32) + q2;  // exact: below 2^51
    lo = r;
}

// Resolved constants of one base for packing / unpacking a part of a block.
struct PartBase {
    uint64_t base;
    uint32_t k;           // digits per basic word
    Chunk ch;             // chunking (packing h = 0: digit by digit in 64 bits)
    const BaseDesc *D;    // schedule of the advanced series, nullptr outside the tables
};

// B^e by squaring, for B^e <= 2^53: every factor used (B^(2^i) with 2^i <= e) and every partial
// product is at most B^e, so each multiplication is exact.
__host__ __device__ __forceinline__ double pow_exact(double B, uint32_t e) {
    double P = 1.0, sq = B;
    for (;;) {
        if (e & 1) P *= sq;
        e >>= 1;
        if (!e) break;
        sq *= sq;
    }
    return P;
}

// The decoder's constants of a basic-family part, from the base alone (no table load): k(B)
// from the octave tables in LDS, h2, B^h2 by squaring (every power used is at most 2^32, exact in
// binary64), and the correctly rounded reciprocals of IEEE division.
__device__ __forceinline__ PartBase basic_base(const SizeCtx &C, uint64_t base) {
    PartBase pb;
    pb.base = base;
    pb.k = k_fast(C, base);
    pb.ch.h = 0;
    pb.ch.P = 0;
    pb.ch.h2 = pb.k / 2 > 1 ? pb.k / 2 : 1;
    const double Bf = (double)base;
    pb.ch.rB = 1.0 / Bf;
    pb.ch.P2 = pow_exact(Bf, pb.ch.h2);
    pb.ch.rP2 = 1.0 / pb.ch.P2;
    pb.D = nullptr;
    return pb;
}

template <bool Wide>
__device__ __forceinline__ PartBase resolve_base(const DevTables &T, const SizeCtx &C, uint64_t base) {
    PartBase pb;
    pb.base = base;
    const int ai = Wide ? atlas_index(base) : (int)base;  // u8 / u16 bases are all in the tables
    if (!Wide || ai >= 0) {
        const BaseDesc &D = T.desc[ai >= 0 ? ai : 2];
        pb.k = D.k;
        pb.ch = D.ch;
        pb.D = &D;
    } else {
        // 2^16 + 1 < base <= 2^32: k is 2 or 3, and a word splits after its lowest digit
        pb.k = k_fast(C, base);
        pb.ch.h = 0;
        pb.ch.P = 0;
        pb.ch.rB = 1.0 / (double)base;
        pb.ch.h2 = 1;
        pb.ch.P2 = (double)base;
        pb.ch.rP2 = pb.ch.rB;
        pb.D = nullptr;
    }
    return pb;
}

// Horner over a digit sequence, first digit at the highest power: `lead` then
// get(j0) .. get(j0 + cnt - 1). Chunks of h digits use 24-bit multiply-adds; the chunks
// are joined by one 64-bit multiply-add each (the first chunk holds total mod h digits).
template <bool Wide, typename Get>
__device__ __forceinline__ uint64_t horner_digits(const PartBase &pb, uint32_t lead, uint32_t j0, uint32_t cnt,
                                                  Get get) {
    if (Wide && pb.ch.h == 0) {  // base >= 2^24 (u32 data only)
        uint64_t acc = lead;
        for (uint32_t j = 0; j < cnt; j++) acc = acc * pb.base + get(j0 + j);
        return acc;
    }
    const uint32_t B = (uint32_t)pb.base, h = pb.ch.h;
    const uint32_t total = cnt + 1;
    uint32_t first = total - h * udiv_small(total, h);
    if (first == 0) first = h;
    uint32_t j = j0;
    // m digits into the 24-bit chunk s, four reads in flight at a time (in increasing order)
    auto chunk = [&](uint32_t s, uint32_t m) -> uint32_t {
        for (; m >= 4; m -= 4) {
            const uint32_t d0 = (uint32_t)get(j), d1 = (uint32_t)get(j + 1), d2 = (uint32_t)get(j + 2),
                           d3 = (uint32_t)get(j + 3);
            j += 4;
            s = __umul24(__umul24(__umul24(__umul24(s, B) + d0, B) + d1, B) + d2, B) + d3;
        }
        for (; m > 0; m--) s = __umul24(s, B) + (uint32_t)get(j++);
        return s;
    };
    uint64_t acc = chunk(lead, first - 1);
    for (uint32_t c = first; c < total; c += h) acc = acc * pb.ch.P + chunk(0, h);
    return acc;
}

// A word of cnt digits starting at j0, of which only those below n exist (the last word of a
// part ends with absent digits, which are 0): Horner over the existing ones, then times
// B^(absent) by squaring (every power used is at most B^(cnt-1) < 2^64). get is asked only for
// existing digits.
template <bool Wide, typename Get>
__device__ __forceinline__ uint64_t horner_word(const PartBase &pb, uint32_t lead, uint32_t j0, uint32_t cnt,
                                                uint32_t n, Get get) {
    const uint32_t real = j0 < n ? (cnt < n - j0 ? cnt : n - j0) : 0;
    uint64_t acc = horner_digits<Wide>(pb, lead, j0, real, get);
    uint32_t pad = cnt - real;
    if (pad) {
        uint64_t p = 1, b = pb.base;
        for (;;) {
            if (pad & 1) p *= b;
            pad >>= 1;
            if (!pad) break;
            b *= b;
        }
        acc *= p;
    }
    return acc;
}

// Peels the lowest cnt base-B digits off X: put(j0 + cnt - 1, lowest digit), ...,
// put(j0, highest of them); returns what remains above them. cnt >= h2 (every word holds at
// least k - 1 digits). The word splits once at B^h2 and the two parts give their digits side by
// side: the lowest h2 from below the split, the other cnt - h2 (and the rest) from above it.
template <bool Wide, typename Put>
__device__ __forceinline__ uint64_t peel_digits(const PartBase &pb, uint64_t X, uint32_t j0, uint32_t cnt, Put put) {
    const double rB = pb.ch.rB, hB = 0.5 * rB, Bf = (double)pb.base;
    double hi, lo;
    split_word(X, pb.ch.P2, pb.ch.rP2, hi, lo);
    const uint32_t nl = pb.ch.h2, nh = cnt - nl;  // nh is nl - 1, nl or nl + 1
    uint32_t jl = j0 + cnt, jh = j0 + nh;
    const uint32_t both = nl < nh ? nl : nh;
    uint32_t m = 0;
    for (; m + 2 <= both; m += 2) {  // two digits of each part per round
        uint32_t d0, d1, d2, d3;
        lo = digit_off(lo, rB, hB, Bf, d0);
        hi = digit_off(hi, rB, hB, Bf, d1);
        lo = digit_off(lo, rB, hB, Bf, d2);
        hi = digit_off(hi, rB, hB, Bf, d3);
        put(jl - 1, d0);
        put(jh - 1, d1);
        put(jl - 2, d2);
        put(jh - 2, d3);
        jl -= 2;
        jh -= 2;
    }
    if (m < both) {
        uint32_t d0, d1;
        lo = digit_off(lo, rB, hB, Bf, d0);
        hi = digit_off(hi, rB, hB, Bf, d1);
        put(--jl, d0);
        put(--jh, d1);
    }
    if (nl > both) {
        uint32_t d;
        lo = digit_off(lo, rB, hB, Bf, d);
        put(--jl, d);
    }
    if (nh > both) {
        uint32_t d;
        hi = digit_off(hi, rB, hB, Bf, d);
        put(--jh, d);
    }
    return (uint32_t)hi;  // what remains is below B <= 2^32
}

__device__ __forceinline__ void put_le(uint8_t *p, uint64_t v, int bytes) {
    if (bytes == 1) {
        *p = (uint8_t)v;
    } else if (bytes == 2 && !((uintptr_t)p & 1)) {
        *(uint16_t *)p = (uint16_t)v;
    } else if (bytes == 4 && !((uintptr_t)p & 3)) {
        *(uint32_t *)p = (uint32_t)v;
    } else if (bytes == 8 && !((uintptr_t)p & 7)) {
        *(uint64_t *)p = v;
    } else {
        for (int i = 0; i < bytes; i++) p[i] = (uint8_t)(v >> (8 * i));
    }
}

__device__ __forceinline__ uint64_t get_le(const uint8_t *p, int bytes) {
    if (bytes == 1) return *p;
    if (bytes == 2 && !((uintptr_t)p & 1)) return *(const uint16_t *)p;
    if (bytes == 4 && !((uintptr_t)p & 3)) return *(const uint32_t *)p;
    uint64_t v = 0;
    for (int i = 0; i < bytes; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

}  // namespace pcomp
