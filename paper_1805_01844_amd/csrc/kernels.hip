// kernels.hip -- gfx950 kernels of the blocked polynomial compressor.
//
// Compression is one fused, single-pass kernel: each workgroup takes one tile of
// tile_blocks blocks (at most 16 KiB of input), stages it in LDS with 128-bit loads,
// reduces every block to (min, B) with wavefront shuffles (Sec. 3, Sec. 3.3), sizes and
// chooses the block's class, places the tile in the output with a decoupled look-back
// prefix sum over the tiles, and packs the words by 64-bit Horner multiply-add
// (Sec. 3.1 Eq. (2); Sec. 3.2 series), one output word per lane, coalesced stores.
// Decompression is a grid-stride kernel over tiles: the stream's tile index places every
// tile, so each lane decodes one word independently by multiply-high magic-number
// division (Sec. 3.1), the split values of the advanced method are rebuilt from the
// neighbouring word, excess values are merged back by an in-block prefix count, and the
// tile leaves LDS through coalesced stores.
#include <hip/hip_runtime.h>

#include "device_math.h"
#include "pcomp_internal.h"

namespace pcomp {

template <int W>
struct Elem;
template <>
struct Elem<1> {
    typedef uint8_t T;
};
template <>
struct Elem<2> {
    typedef uint16_t T;
};
template <>
struct Elem<4> {
    typedef uint32_t T;
};

// ---------------------------------------------------------------------------------------
// Group reductions: G lanes (a power of two) cooperate on one block. Within a wavefront
// they use cross-lane shuffles; groups wider than a wavefront combine per-wave partials
// through LDS. Every thread of the workgroup must call these (they may hold barriers).
// ---------------------------------------------------------------------------------------
template <typename T, typename Op>
__device__ __forceinline__ T group_reduce(T x, uint32_t G, Op op, T *scratch) {
    uint32_t width = G < 64 ? G : 64;
    for (uint32_t o = 1; o < width; o <<= 1) x = op(x, __shfl_xor(x, o, 64));
    if (G > 64) {
        uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        __syncthreads();
        if (lane == 0) scratch[wave] = x;
        __syncthreads();
        uint32_t wpg = G >> 6, w0 = (wave / wpg) * wpg;
        T r = scratch[w0];
        for (uint32_t i = 1; i < wpg; i++) r = op(r, scratch[w0 + i]);
        x = r;
        __syncthreads();
    }
    return x;
}

// Exclusive prefix sum over the G lanes of a group (lane order).
__device__ __forceinline__ uint32_t group_excl_scan(uint32_t x, uint32_t G, uint32_t *scratch) {
    uint32_t lane = threadIdx.x & 63;
    uint32_t width = G < 64 ? G : 64;
    uint32_t gl = lane & (width - 1);
    uint32_t inc = x;
    for (uint32_t o = 1; o < width; o <<= 1) {
        uint32_t y = __shfl_up(inc, o, width);
        if (gl >= o) inc += y;
    }
    uint32_t excl = inc - x;
    if (G > 64) {
        uint32_t wave = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 63) scratch[wave] = inc;
        __syncthreads();
        uint32_t wpg = G >> 6, w0 = (wave / wpg) * wpg;
        for (uint32_t i = w0; i < wave; i++) excl += scratch[i];
        __syncthreads();
    }
    return excl;
}

struct MinOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a < b ? a : b; }
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a < b ? a : b; }
};
struct MaxOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};
struct AddOp {
    __device__ uint64_t operator()(uint64_t a, uint64_t b) const { return a + b; }
};

// Words of class c for a block of Lb digits of base B; ne_t = digits >= T for t = c & 7.
__device__ inline uint32_t class_words(const DevTables &T, int c, uint32_t Lb, uint64_t B, uint32_t beta,
                                       uint32_t ne_t, uint32_t &nw_main) {
    int fam = c >> 3, t = c & 7;
    if (t == 0) {
        nw_main = family_words(T, fam, Lb, B);
        return nw_main;
    }
    uint64_t Th = 1ull << (beta - t);
    nw_main = family_words(T, fam, Lb, Th + 1);
    return nw_main + family_words(T, fam, ne_t, B - Th);
}

// Per-workgroup cache for the main part of threshold classes: base 2^j + 1 (j = beta - t),
// digits per word and advanced word count of a full block of L digits.
struct P1Cache {
    uint32_t k[32];
    uint32_t adv_full[32];
};

__device__ inline void fill_p1_cache(const DevTables &T, uint32_t L, P1Cache &C) {
    const uint32_t j = threadIdx.x;
    if (j < 32) {
        const uint64_t base = (1ull << j) + 1;
        const int ai = atlas_index(base);
        C.k[j] = T.desc[ai].k;
        C.adv_full[j] = adv_words_atlas(T, T.desc[ai], L);
    }
}

__device__ __forceinline__ uint32_t words_p1(const DevTables &T, const P1Cache &C, int fam, uint32_t j, uint32_t n,
                                             uint32_t L) {
    if (!fam) return (n + C.k[j] - 1) / C.k[j];
    if (n == L) return C.adv_full[j];
    return adv_words_atlas(T, T.desc[atlas_index((1ull << j) + 1)], n);
}

// class_words with the main part of threshold classes served from the cache.
__device__ inline uint32_t class_words_c(const DevTables &T, const P1Cache &C, uint32_t L, int c, uint32_t Lb,
                                         uint64_t B, uint32_t beta, uint32_t ne_t, uint32_t &nw_main) {
    int fam = c >> 3, t = c & 7;
    if (t == 0) {
        nw_main = family_words(T, fam, Lb, B);
        return nw_main;
    }
    const uint32_t j = beta - t;
    const uint64_t Th = 1ull << j;
    nw_main = words_p1(T, C, fam, j, Lb, L);
    return nw_main + family_words(T, fam, ne_t, B - Th);
}

// Resolved description of one packed part of a block (main digits or excess list).
struct Part {
    uint64_t base;
    uint32_t n;     // digits in the part
    uint32_t fam;   // 0 basic, 1 advanced
    int ai;         // table index of the base, -1 if outside the tables
};

__device__ __forceinline__ Part make_part(uint64_t base, uint32_t n, uint32_t fam) {
    Part P;
    P.base = base;
    P.n = n;
    P.fam = fam;
    P.ai = atlas_index(base);
    return P;
}

// ---------------------------------------------------------------------------------------
// Compression
// ---------------------------------------------------------------------------------------
struct CompressArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t *out_size;
    uint64_t *tile_status;  // [n_tiles]: bit 63 = inclusive prefix, bit 62 = aggregate
    uint32_t *ticket;
    uint32_t *err;
    Layout lo;
    int variant;
    DevTables T;
};

constexpr uint64_t kStAgg = 1ull << 62, kStInc = 1ull << 63, kStMask = (1ull << 62) - 1;

__device__ __forceinline__ void put_le(uint8_t *p, uint64_t v, int bytes) {
    for (int i = 0; i < bytes; i++) p[i] = (uint8_t)(v >> (8 * i));
}

__device__ void write_header(const CompressArgs &a, uint64_t payload_words, int variant) {
    const Layout &lo = a.lo;
    uint64_t total = lo.off_payload + 8 * payload_words;
    uint64_t h[8];
    uint32_t sel = variant == PCOMP_SELECT_EXHAUSTIVE ? 1 : variant == PCOMP_SELECT_LEARNED ? 2 : 0;
    uint32_t fixed = (lo.flags & kFlagClass) ? 0 : (uint32_t)variant;
    h[0] = (uint64_t)kMagic | ((uint64_t)kVersion << 32) | ((uint64_t)lo.w << 48) | ((uint64_t)lo.flags << 56);
    h[1] = (uint64_t)fixed | ((uint64_t)sel << 8) | ((uint64_t)lo.L << 32);
    h[2] = lo.n;
    h[3] = lo.n_blocks;
    h[4] = (uint64_t)lo.tile_blocks;
    h[5] = payload_words;
    h[6] = total;
    h[7] = 0;
    uint64_t *o = (uint64_t *)a.out;
    for (int i = 0; i < 8; i++) o[i] = h[i];
    // zero padding between the block arrays and the payload
    uint64_t end_arrays = lo.off_ne + ((lo.flags & kFlagNe) ? lo.n_blocks * ((lo.flags & kFlagNe16) ? 2 : 1) : 0);
    for (uint64_t b = end_arrays; b < lo.off_payload; b++) a.out[b] = 0;
    *a.out_size = total;
}

template <int W>
__global__ __launch_bounds__(kThreads) void compress_kernel(CompressArgs a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    __shared__ uint4 s_exc_raw[kTileBytes / 16];
    __shared__ uint32_t s_min[kMaxTileBlocks], s_rng[kMaxTileBlocks], s_ne[kMaxTileBlocks];
    __shared__ uint32_t s_nwm[kMaxTileBlocks], s_off[kMaxTileBlocks + 1];
    __shared__ uint8_t s_cls[kMaxTileBlocks];
    __shared__ uint64_t s_red64[kThreads / 64];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint32_t s_tile;
    __shared__ uint64_t s_excl;
    __shared__ P1Cache s_p1;

    const Layout &lo = a.lo;
    const DevTables &T = a.T;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_tile = atomicAdd(a.ticket, 1u);
    if (a.variant != 0 && a.variant != 8) fill_p1_cache(T, lo.L, s_p1);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (lo.n_tiles == 0) {
        if (tile == 0 && tid == 0) write_header(a, 0, a.variant);
        return;
    }
    if (tile >= lo.n_tiles) return;

    const uint32_t L = lo.L;
    const uint32_t tb = lo.tile_blocks;
    const uint64_t b0 = (uint64_t)tile * tb;
    const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
    const uint64_t v0 = b0 * L;
    const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);

    // ---- 1. stage the tile's input in LDS (16-byte chunks; partial chunks by element)
    uint8_t *s_bytes = (uint8_t *)s_raw;
    const uintptr_t addr = (uintptr_t)(a.in + v0 * W);
    const uint32_t head = (uint32_t)(addr & 15);
    const uint8_t *gbase = (const uint8_t *)(addr - head);
    const uint32_t span = head + nvt * W;
    const uint32_t nchunks = (span + 15) >> 4;
    for (uint32_t c = tid; c < nchunks; c += kThreads) {
        uint32_t cb = c << 4;
        if (cb >= head && cb + 16 <= span) {
            s_raw[c] = *(const uint4 *)(gbase + cb);
        } else {
            uint32_t e0 = cb > head ? cb : head, e1 = cb + 16 < span ? cb + 16 : span;
            for (uint32_t b = e0; b < e1; b += W) *(V *)(s_bytes + b) = *(const V *)(gbase + b);
        }
    }
    __syncthreads();
    const V *s_val = (const V *)(s_bytes + head);
    V *s_exc = (V *)s_exc_raw;

    // ---- 2. per-block min / max (Sec. 3: B = v_max - v_min + 1) and log-histogram
    const uint32_t G = kThreads / tb;
    const uint32_t blk = tid / G, g = tid % G;
    const bool live = blk < nbt;
    const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
    const V *bv = s_val + (size_t)blk * L;
    uint32_t vmin = 0xFFFFFFFFu, vmax = 0;
    for (uint32_t j = g; j < Lb; j += G) {
        uint32_t v = bv[j];
        vmin = v < vmin ? v : vmin;
        vmax = v > vmax ? v : vmax;
    }
    vmin = group_reduce(vmin, G, MinOp(), s_red32);
    vmax = group_reduce(vmax, G, MaxOp(), s_red32);
    const uint64_t B = live ? (uint64_t)vmax - vmin + 1 : 1;
    const uint32_t beta = bitlen64(B - 1);
    const int variant = a.variant;
    const bool fixed0 = (variant == 0 || variant == 8);
    // H[b] = #{j : min(beta - bitlen(d_j), 15) = b}, four 16-bit counters per u64
    uint64_t h0 = 0, h1 = 0;
    if (!fixed0) {
        for (uint32_t j = g; j < Lb; j += G) {
            uint32_t d = (uint32_t)bv[j] - vmin;
            uint32_t b = beta - bitlen32(d);
            uint64_t inc = 1ull << ((b & 3) * 16);
            h0 += b < 4 ? inc : 0;
            h1 += (b >= 4 && b < 8) ? inc : 0;
        }
        h0 = group_reduce(h0, G, AddOp(), s_red64);
        h1 = group_reduce(h1, G, AddOp(), s_red64);
    }
    // n_e(t) = sum of the first t bins
    uint32_t ne_t[8];
    ne_t[0] = 0;
#pragma unroll
    for (int t = 1; t < 8; t++) {
        uint32_t hb = (uint32_t)(((t - 1) < 4 ? (h0 >> (16 * (t - 1))) : (h1 >> (16 * (t - 5)))) & 0xFFFF);
        ne_t[t] = ne_t[t - 1] + hb;
    }

    // ---- 3. class choice: lanes of the group split the 16 classes; argmin, ties to the lowest id
    uint64_t key = ~0ull;
    if (live) {
        for (int c = (int)g; c < 16; c += (int)G) {
            bool cand = fixed0 ? (c == variant)
                               : (c == 0 || variant == PCOMP_SELECT_EXHAUSTIVE || c == variant);
            if (!cand) continue;
            int t = c & 7;
            if (t > (int)beta) continue;
            uint32_t nwm;
            uint32_t nw = class_words_c(T, s_p1, L, c, Lb, B, beta, ne_t[t], nwm);
            uint64_t k2 = ((uint64_t)nw << 8) | (uint64_t)c;
            key = k2 < key ? k2 : key;
        }
    }
    key = group_reduce(key, G, MinOp(), s_red64);
    const int cls = (int)(key & 0xFF);
    uint32_t nw = (uint32_t)(key >> 8);
    {
        // every chosen class is at most the basic t = 0 size, which the bound assumes; a larger
        // count means an internal error: flag it and keep every write inside the bound
        const uint32_t per = 8 / W, cap = (Lb + per - 1) / per;
        if (live && nw > cap) {
            if (g == 0) atomicOr(a.err, 2u);
            nw = cap;
        }
    }
    const int tcls = cls & 7;
    const uint64_t Th = tcls ? (1ull << (beta - tcls)) : 0;
    if (live && g == 0) {
        uint32_t nwm;
        if (fixed0)
            nwm = nw;
        else
            class_words_c(T, s_p1, L, cls, Lb, B, beta, ne_t[tcls], nwm);
        s_min[blk] = vmin;
        s_rng[blk] = (uint32_t)(B - 1);
        s_cls[blk] = (uint8_t)cls;
        s_ne[blk] = ne_t[tcls];
        s_nwm[blk] = nwm;
        s_off[blk] = nw;
        const uint64_t gb = b0 + blk;
        put_le(a.out + lo.off_min + gb * W, vmin, W);
        put_le(a.out + lo.off_range + gb * W, B - 1, W);
        if (lo.flags & kFlagClass) a.out[lo.off_class + gb] = (uint8_t)cls;
        if (lo.flags & kFlagNe) {
            if (lo.flags & kFlagNe16)
                put_le(a.out + lo.off_ne + gb * 2, ne_t[tcls], 2);
            else
                a.out[lo.off_ne + gb] = (uint8_t)ne_t[tcls];
        }
    }

    // ---- 4. excess lists of threshold blocks, in data order (chunked per lane)
    if (!fixed0) {
        const uint32_t ch = (Lb + G - 1) / G;
        const uint32_t j0 = g * ch < Lb ? g * ch : Lb, j1 = (g + 1) * ch < Lb ? (g + 1) * ch : Lb;
        uint32_t cnt = 0;
        if (tcls)
            for (uint32_t j = j0; j < j1; j++) cnt += ((uint32_t)bv[j] - vmin) >= Th;
        uint32_t pos = group_excl_scan(cnt, G, s_red32);
        if (tcls) {
            V *ex = s_exc + (size_t)blk * L;
            for (uint32_t j = j0; j < j1; j++) {
                uint32_t d = (uint32_t)bv[j] - vmin;
                if (d >= Th) ex[pos++] = (V)(d - Th);
            }
        }
    }
    __syncthreads();

    // ---- 5. exclusive scan of the word counts over the tile's blocks
    {
        uint32_t x = tid < nbt ? s_off[tid] : 0;
        uint32_t lane = tid & 63, wave = tid >> 6;
        uint32_t inc = x;
        for (uint32_t o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) s_red32[wave] = inc;
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t w = 0; w < wave; w++) add += s_red32[w];
        uint32_t excl = inc - x + add;
        __syncthreads();
        if (tid < nbt) s_off[tid] = excl;
        if (tid == nbt - 1) s_off[nbt] = excl + x;
        __syncthreads();
    }
    const uint32_t tile_words = s_off[nbt];

    // ---- 6. decoupled look-back: exclusive prefix of the payload words of earlier tiles.
    // The first wavefront reads 64 predecessors' descriptors at once; lanes up to the
    // nearest inclusive prefix must all be published, their values are summed, and the
    // window moves back by 64 tiles while no inclusive prefix is in sight.
    if (tid < 64) {
        const uint32_t lane = tid;
        if (tile == 0) {
            if (lane == 0)
                __hip_atomic_store(&a.tile_status[0], kStInc | tile_words, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        } else if (lane == 0) {
            __hip_atomic_store(&a.tile_status[tile], kStAgg | tile_words, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        uint64_t excl = 0;
        if (tile > 0) {
            int64_t top = (int64_t)tile - 1;
            uint32_t spins = 0;
            for (;;) {
                const int64_t j = top - (int64_t)lane;
                uint64_t st = kStInc;  // before tile 0: an inclusive prefix of 0
                if (j >= 0) st = __hip_atomic_load(&a.tile_status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t inc_mask = __ballot((st & kStInc) != 0);
                const uint64_t nr_mask = __ballot((st & (kStInc | kStAgg)) == 0);
                const uint32_t first = inc_mask ? (uint32_t)(__ffsll((unsigned long long)inc_mask) - 1) : 64u;
                const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
                if (nr_mask & need) {
                    if (++spins > (1u << 24)) {  // a predecessor never published: flag it and stop
                        if (lane == 0) atomicOr(a.err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint64_t v = lane <= first ? (st & kStMask) : 0;
                for (uint32_t o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
                excl += v;
                if (first < 64 || top < 64) break;  // top < 64: the window reached tile 0
                top -= 64;
            }
            if (lane == 0)
                __hip_atomic_store(&a.tile_status[tile], kStInc | (excl + tile_words), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_excl = excl;
            put_le(a.out + lo.off_index + 8 * (uint64_t)tile, excl, 8);
            if (tile == lo.n_tiles - 1) write_header(a, excl + tile_words, variant);
        }
    }
    __syncthreads();
    const uint64_t excl = s_excl;
    uint64_t *payload = (uint64_t *)(a.out + lo.off_payload) + excl;

    // ---- 7. pack: one output word per lane, in output order
    for (uint32_t w = tid; w < tile_words; w += kThreads) {
        // block of word w: last b with s_off[b] <= w
        uint32_t lo_b = 0, hi_b = nbt - 1;
        while (lo_b < hi_b) {
            uint32_t mid = (lo_b + hi_b + 1) >> 1;
            if (s_off[mid] <= w)
                lo_b = mid;
            else
                hi_b = mid - 1;
        }
        const uint32_t b = lo_b;
        uint32_t i = w - s_off[b];
        const uint32_t nwb = s_off[b + 1] - s_off[b];
        const int c = s_cls[b];
        const int t = c & 7, fam = c >> 3;
        const uint32_t bmin = s_min[b];
        const uint64_t Bb = (uint64_t)s_rng[b] + 1;
        const uint32_t Lbb = (uint32_t)min((uint64_t)L, lo.n - (b0 + b) * L);
        const V *vals = s_val + (size_t)b * L;
        const V *exc = s_exc + (size_t)b * L;
        uint64_t Tb = 0;
        bool excess = false;
        uint32_t part_words;
        Part P;
        if (t == 0) {
            P = make_part(Bb, Lbb, fam);
            part_words = nwb;
        } else {
            Tb = 1ull << (bitlen64(Bb - 1) - t);
            if (i < s_nwm[b]) {
                P = make_part(Tb + 1, Lbb, fam);
                part_words = s_nwm[b];
            } else {
                i -= s_nwm[b];
                excess = true;
                P = make_part(Bb - Tb, s_ne[b], fam);
                part_words = nwb - s_nwm[b];
            }
        }
        // digit j of the part (0 past its end)
        auto digit = [&](uint32_t j) -> uint64_t {
            if (j >= P.n) return 0;
            if (excess) return (uint64_t)exc[j];
            uint64_t d = (uint64_t)vals[j] - bmin;
            if (t) d = d < Tb ? d : Tb;
            return d;
        };
        uint64_t word = 0;
        if (!fam) {
            // Sec. 3.1 Eq. (2): word i holds digits i*k .. i*k+k-1, first digit at the highest power
            const uint32_t k = k_of(T, P.base);
            const uint32_t j0 = i * k;
            for (uint32_t j = 0; j < k; j++) word = word * P.base + digit(j0 + j);
            payload[w] = word;
        } else if (P.ai >= 0) {
            // Sec. 3.2 series from the cycle form of the base's schedule
            const BaseDesc &D = T.desc[P.ai];
            uint32_t q;
            const AtlasEntry *e = adv_entry(T, D, i, q);
            uint64_t rp = 0;  // r'_{i-1}: top part of the value split at the end of word i-1
            if (i > 0) {
                uint32_t qp;
                const AtlasEntry *ep = adv_entry(T, D, i - 1, qp);
                rp = div_magic(digit(q - 1), ep->mR);
            }
            word = rp;
            for (uint32_t j = 0; j < e->p; j++) word = word * P.base + digit(q + j);
            const uint64_t x = digit(q + e->p);
            const uint64_t r = x - div_magic(x, e->mR) * e->R;
            word = word * e->R + r;
            payload[w] = word;
        } else if (i == 0) {
            // base outside the tables: one lane walks the series and writes every word of the part
            const SlowBase sb = slow_base(T, P.base);
            uint64_t s = 1, rp = 0;
            uint32_t q = 0;
            for (uint32_t wi = 0; wi < part_words; wi++) {
                uint32_t p;
                uint64_t R;
                slow_word(sb, s, p, R);
                uint64_t acc = rp;
                for (uint32_t j = 0; j < p; j++) acc = acc * P.base + digit(q + j);
                const uint64_t x = digit(q + p);
                const uint64_t r = x % R;
                rp = x / R;
                payload[w + wi] = acc * R + r;
                if (q + p >= P.n) break;
                s = (P.base + R - 1) / R;
                q += p + 1;
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Decompression
// ---------------------------------------------------------------------------------------
struct DecompressArgs {
    const uint8_t *in;
    uint64_t in_size;
    uint8_t *out;
    uint64_t out_cap;
    int32_t *status;
    DevTables T;
};

__device__ __forceinline__ uint64_t get_le(const uint8_t *p, int bytes) {
    uint64_t v = 0;
    for (int i = 0; i < bytes; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

__device__ __forceinline__ void set_status(int32_t *st, int32_t code) { atomicMin(st, code); }

// Reads and checks the stream header; returns false (and sets the status) if unusable.
__device__ bool read_layout(const DecompressArgs &a, Layout &lo, uint64_t &pw, int &fixed) {
    const uint64_t *h = (const uint64_t *)a.in;
    if (a.in_size < kHdrBytes) return false;
    uint64_t h0 = h[0], h1 = h[1];
    if ((uint32_t)h0 != kMagic || ((h0 >> 32) & 0xFFFF) != kVersion) return false;
    uint32_t w = (uint32_t)((h0 >> 48) & 0xFF), flags = (uint32_t)(h0 >> 56);
    if (!(w == 1 || w == 2 || w == 4) || (flags & ~7u)) return false;
    fixed = (int)(h1 & 0xFF);
    uint32_t L = (uint32_t)(h1 >> 32);
    if (L == 0 || L > 65535) return false;
    if (!(flags & kFlagClass) && !(fixed == 0 || fixed == 8)) return false;
    if ((flags & kFlagNe) && (((flags & kFlagNe16) != 0) != (L > 255))) return false;
    make_layout(h[2], w, L, flags, lo);
    if (h[3] != lo.n_blocks || (uint32_t)h[4] != lo.tile_blocks) return false;
    pw = h[5];
    if (h[6] != lo.off_payload + 8 * pw || h[6] > a.in_size || pw > (a.in_size >> 3)) return false;
    return true;
}

struct DecShared {
    uint4 raw[kTileBytes / 16];
    uint4 exc[kTileBytes / 16];
    uint32_t min[kMaxTileBlocks], rng[kMaxTileBlocks], ne[kMaxTileBlocks];
    uint32_t nwm[kMaxTileBlocks], off[kMaxTileBlocks + 1];
    uint8_t cls[kMaxTileBlocks];
    uint32_t red32[kThreads / 64];
    int bad;
};

template <int W>
__device__ void decompress_tiles(const DecompressArgs &a, const Layout &lo, uint64_t pw, int fixed, DecShared &S) {
    typedef typename Elem<W>::T V;
    uint4 *s_raw = S.raw, *s_exc_raw = S.exc;
    uint32_t *s_min = S.min, *s_rng = S.rng, *s_ne = S.ne, *s_nwm = S.nwm, *s_off = S.off, *s_red32 = S.red32;
    uint8_t *s_cls = S.cls;
    int &s_bad = S.bad;
    const DevTables &T = a.T;
    const uint32_t tid = threadIdx.x;
    const uint32_t L = lo.L, tb = lo.tile_blocks;
    const uint64_t *idx = (const uint64_t *)(a.in + lo.off_index);
    const uint64_t *payload_all = (const uint64_t *)(a.in + lo.off_payload);
    const uint32_t vmaxw = (uint32_t)((1ull << (8 * W)) - 1);
    V *s_val = (V *)s_raw;
    V *s_exc = (V *)s_exc_raw;

    for (uint64_t tile = blockIdx.x; tile < lo.n_tiles; tile += gridDim.x) {
        const uint64_t b0 = tile * tb;
        const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
        const uint64_t v0 = b0 * L;
        const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
        if (tid == 0) s_bad = 0;
        __syncthreads();
        // ---- 1. block arrays of the tile, word counts
        if (tid < nbt) {
            const uint64_t gb = b0 + tid;
            const uint32_t bmin = (uint32_t)get_le(a.in + lo.off_min + gb * W, W);
            const uint32_t rng = (uint32_t)get_le(a.in + lo.off_range + gb * W, W);
            const int c = (lo.flags & kFlagClass) ? a.in[lo.off_class + gb] : fixed;
            uint32_t ne = 0;
            if (lo.flags & kFlagNe)
                ne = (uint32_t)get_le(a.in + lo.off_ne + gb * ((lo.flags & kFlagNe16) ? 2 : 1),
                                      (lo.flags & kFlagNe16) ? 2 : 1);
            const uint32_t Lb = (uint32_t)min((uint64_t)L, lo.n - gb * L);
            const uint64_t B = (uint64_t)rng + 1;
            const uint32_t beta = bitlen64(B - 1);
            const int t = c & 7;
            bool ok = c < 16 && t <= (int)beta && ne <= Lb && (t != 0 || ne == 0) && (uint64_t)bmin + rng <= vmaxw;
            uint32_t nwm = 0, nw = 0;
            if (ok) nw = class_words(T, c, Lb, B, beta, ne, nwm);
            if (!ok) s_bad = 1;
            s_min[tid] = bmin;
            s_rng[tid] = rng;
            s_cls[tid] = (uint8_t)(ok ? c : 0);
            s_ne[tid] = ne;
            s_nwm[tid] = nwm;
            s_off[tid] = nw;
        }
        __syncthreads();
        {
            uint32_t x = tid < nbt ? s_off[tid] : 0;
            uint32_t lane = tid & 63, wave = tid >> 6;
            uint32_t inc = x;
            for (uint32_t o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(inc, o, 64);
                if (lane >= o) inc += y;
            }
            if (lane == 63) s_red32[wave] = inc;
            __syncthreads();
            uint32_t add = 0;
            for (uint32_t w = 0; w < wave; w++) add += s_red32[w];
            uint32_t excl = inc - x + add;
            __syncthreads();
            if (tid < nbt) s_off[tid] = excl;
            if (tid == nbt - 1) s_off[nbt] = excl + x;
            __syncthreads();
        }
        const uint32_t tile_words = s_off[nbt];
        const uint64_t base_off = idx[tile];
        const uint64_t next_off = (tile + 1 < lo.n_tiles) ? idx[tile + 1] : pw;
        if (s_bad || base_off > pw || next_off > pw || next_off != base_off + tile_words) {
            if (tid == 0) set_status(a.status, PCOMP_ECORRUPT);
            __syncthreads();
            continue;
        }
        const uint64_t *payload = payload_all + base_off;

        // ---- 2. decode: one word per lane (digits peeled from the lowest power, Sec. 3.1)
        for (uint32_t w = tid; w < tile_words; w += kThreads) {
            uint32_t lo_b = 0, hi_b = nbt - 1;
            while (lo_b < hi_b) {
                uint32_t mid = (lo_b + hi_b + 1) >> 1;
                if (s_off[mid] <= w)
                    lo_b = mid;
                else
                    hi_b = mid - 1;
            }
            const uint32_t b = lo_b;
            uint32_t i = w - s_off[b];
            const uint32_t nwb = s_off[b + 1] - s_off[b];
            const int c = s_cls[b];
            const int t = c & 7, fam = c >> 3;
            const uint64_t Bb = (uint64_t)s_rng[b] + 1;
            const uint32_t Lbb = (uint32_t)min((uint64_t)L, lo.n - (b0 + b) * L);
            const uint32_t bmin = s_min[b];
            Part P;
            V *dst;
            uint32_t part_words;
            uint32_t add = 0;  // min is added here for plain blocks, after the merge otherwise
            if (t == 0) {
                P = make_part(Bb, Lbb, fam);
                dst = s_val + (size_t)b * L;
                add = bmin;
                part_words = nwb;
            } else {
                const uint64_t Tb = 1ull << (bitlen64(Bb - 1) - t);
                if (i < s_nwm[b]) {
                    P = make_part(Tb + 1, Lbb, fam);
                    dst = s_val + (size_t)b * L;
                    part_words = s_nwm[b];
                } else {
                    i -= s_nwm[b];
                    P = make_part(Bb - Tb, s_ne[b], fam);
                    dst = s_exc + (size_t)b * L;
                    part_words = nwb - s_nwm[b];
                }
            }
            uint64_t X = payload[w];
            if (!fam) {
                uint32_t k;
                Magic mB;
                if (P.ai >= 0) {
                    k = T.desc[P.ai].k;
                    mB = T.desc[P.ai].mB;
                } else {
                    k = k_of(T, P.base);
                    mB = magic_dev(P.base);
                }
                const uint32_t j0 = i * k;
                for (int j = (int)k - 1; j >= 0; j--) {
                    const uint64_t qq = div_magic(X, mB);
                    const uint32_t d = (uint32_t)(X - qq * P.base);
                    X = qq;
                    if (j0 + j < P.n) dst[j0 + j] = (V)(d + add);
                }
            } else if (P.ai >= 0) {
                const BaseDesc &D = T.desc[P.ai];
                uint32_t q;
                const AtlasEntry *e = adv_entry(T, D, i, q);
                uint64_t qR = div_magic(X, e->mR);
                const uint64_t r = X - qR * e->R;
                X = qR;
                for (int j = (int)e->p - 1; j >= 0; j--) {
                    const uint64_t qq = div_magic(X, D.mB);
                    const uint32_t d = (uint32_t)(X - qq * P.base);
                    X = qq;
                    if (q + j < P.n) dst[q + j] = (V)(d + add);
                }
                // the value split between this word (r_i) and the next (r'_i on top)
                if (q + e->p < P.n && i + 1 < part_words) {
                    uint32_t q1;
                    const AtlasEntry *e1 = adv_entry(T, D, i + 1, q1);
                    const uint64_t Y = div_magic(payload[w + 1], e1->mR);
                    const uint64_t rp = div_magic(Y, D.mBp[e1->p == D.k ? 1 : 0]);
                    dst[q + e->p] = (V)(rp * e->R + r + add);
                }
            } else if (i == 0) {
                // base outside the tables: one lane walks the series over the whole part
                const SlowBase sb = slow_base(T, P.base);
                const Magic mB = magic_dev(P.base);
                uint64_t s = 1, r_prev = 0, R_prev = 1;
                uint32_t q = 0, q_prev = 0, p_prev = 0;
                for (uint32_t wi = 0; wi < part_words; wi++) {
                    uint32_t p;
                    uint64_t R;
                    slow_word(sb, s, p, R);
                    uint64_t Xw = payload[w + wi];
                    const uint64_t qR = Xw / R;
                    const uint64_t r = Xw - qR * R;
                    Xw = qR;
                    for (int j = (int)p - 1; j >= 0; j--) {
                        const uint64_t qq = div_magic(Xw, mB);
                        const uint32_t d = (uint32_t)(Xw - qq * P.base);
                        Xw = qq;
                        if (q + j < P.n) dst[q + j] = (V)(d + add);
                    }
                    if (wi > 0 && q_prev + p_prev < P.n) dst[q_prev + p_prev] = (V)(Xw * R_prev + r_prev + add);
                    if (q + p >= P.n) break;
                    r_prev = r;
                    R_prev = R;
                    q_prev = q;
                    p_prev = p;
                    s = (P.base + R - 1) / R;
                    q += p + 1;
                }
            }
        }
        __syncthreads();

        // ---- 3. threshold blocks: main digit T marks an excess value (in order); add min
        {
            const uint32_t G = kThreads / tb;
            const uint32_t blk = tid / G, g = tid % G;
            const bool live = blk < nbt;
            const int c = live ? s_cls[blk] : 0;
            const int t = c & 7;
            const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
            const uint32_t ch = (Lb + G - 1) / G;
            const uint32_t j0 = g * ch < Lb ? g * ch : Lb, j1 = (g + 1) * ch < Lb ? (g + 1) * ch : Lb;
            uint32_t Tb = 0, bmin = 0;
            V *vals = s_val + (size_t)blk * L;
            const V *ex = s_exc + (size_t)blk * L;
            uint32_t cnt = 0;
            if (t) {
                Tb = 1u << (bitlen64((uint64_t)s_rng[blk]) - t);
                bmin = s_min[blk];
                for (uint32_t j = j0; j < j1; j++) cnt += (uint32_t)vals[j] == Tb;
            }
            uint32_t pos = group_excl_scan(cnt, G, s_red32);
            if (live && !t && s_rng[blk] == 0) {  // B = 1: no words, every value is the minimum
                const V m = (V)s_min[blk];
                for (uint32_t j = j0; j < j1; j++) vals[j] = m;
            }
            if (t) {
                const uint32_t ne = s_ne[blk];
                // a base-1 excess list (B - T = 1) has no words: every excess is 0
                const bool exc_words = (uint64_t)s_rng[blk] + 1 - Tb > 1;
                for (uint32_t j = j0; j < j1; j++) {
                    uint32_t d = vals[j];
                    if (d == Tb) {
                        d = Tb + ((exc_words && pos < ne) ? (uint32_t)ex[pos] : 0u);
                        pos++;
                    }
                    vals[j] = (V)(d + bmin);
                }
            }
        }
        __syncthreads();

        // ---- 4. coalesced store of the tile
        {
            const uint8_t *sb = (const uint8_t *)s_raw;
            const uintptr_t addr = (uintptr_t)(a.out + v0 * W);
            const uint32_t head = (uint32_t)((16 - (addr & 15)) & 15);  // bytes before the first aligned chunk
            const uint32_t nbytes = nvt * W;
            const uint32_t hb = head < nbytes ? head : nbytes;
            for (uint32_t b = tid * W; b < hb; b += kThreads * W)
                *(V *)(a.out + v0 * W + b) = *(const V *)(sb + b);
            const uint32_t body = (nbytes - hb) >> 4;
            for (uint32_t c = tid; c < body; c += kThreads) {
                const uint32_t sbo = hb + (c << 4);
                uint4 v;
                const uint32_t *s32 = (const uint32_t *)(sb + sbo);
                if ((sbo & 3) == 0) {
                    v = make_uint4(s32[0], s32[1], s32[2], s32[3]);
                } else {
                    uint8_t tmp[16];
                    for (int q = 0; q < 16; q++) tmp[q] = sb[sbo + q];
                    v = *(const uint4 *)tmp;
                }
                *(uint4 *)(a.out + v0 * W + sbo) = v;
            }
            for (uint32_t b = hb + (body << 4) + tid * W; b < nbytes; b += kThreads * W)
                *(V *)(a.out + v0 * W + b) = *(const V *)(sb + b);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kThreads) void decompress_kernel(DecompressArgs a) {
    __shared__ DecShared S;
    Layout lo;
    uint64_t pw;
    int fixed;
    if (!read_layout(a, lo, pw, fixed)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, PCOMP_ECORRUPT);
        return;
    }
    if ((uint64_t)lo.L * lo.w > kTileBytes) {
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, PCOMP_EINVAL);
        return;
    }
    if (lo.n > a.out_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, PCOMP_ENOSPC);
        return;
    }
    if (lo.w == 1)
        decompress_tiles<1>(a, lo, pw, fixed, S);
    else if (lo.w == 2)
        decompress_tiles<2>(a, lo, pw, fixed, S);
    else
        decompress_tiles<4>(a, lo, pw, fixed, S);
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void set_i32_kernel(int32_t *p, int32_t v) { *p = v; }

}  // namespace pcomp

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------
using namespace pcomp;

namespace {

bool dtype_ok(int w) { return w == 1 || w == 2 || w == 4; }
bool variant_ok(int v) { return (v >= 0 && v < 16) || v == PCOMP_SELECT_EXHAUSTIVE || v == PCOMP_SELECT_LEARNED; }

// Workspace: [ticket u32, err u32] then tile status u64 x n_tiles.
size_t ws_bytes_for(const Layout &lo) { return 8 + 8 * (size_t)(lo.n_tiles ? lo.n_tiles : 1); }

}  // namespace

extern "C" int pcomp_init(void) {
    DevTables t;
    return tables_for_current_device(&t);
}

extern "C" size_t pcomp_bound(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || !variant_ok(variant)) return 0;
    Layout lo;
    make_layout(n, w, block_len, flags_of(variant, block_len), lo);
    const uint64_t per = 8 / w;  // digits per word for a full-range block, 64 / (8 w)
    uint64_t words = 0;
    if (lo.n_blocks) {
        const uint64_t last = n - (lo.n_blocks - 1) * block_len;
        words = (lo.n_blocks - 1) * ((block_len + per - 1) / per) + (last + per - 1) / per;
    }
    return (size_t)(lo.off_payload + 8 * words);
}

extern "C" size_t pcomp_workspace_size(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || !variant_ok(variant)) return 0;
    Layout lo;
    make_layout(n, w, block_len, flags_of(variant, block_len), lo);
    return ws_bytes_for(lo);
}

extern "C" int pcomp_compress(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant,
                              void *d_out, size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes,
                              void *stream) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || !variant_ok(variant)) return PCOMP_EINVAL;
    if ((uint64_t)block_len * w > kTileBytes) return PCOMP_EINVAL;  // GPU tiles hold whole blocks
    if (variant == PCOMP_SELECT_LEARNED) return PCOMP_ENOMODEL;
    if ((n && !d_in) || !d_out || !d_out_size || !d_ws) return PCOMP_EINVAL;
    if (((uintptr_t)d_out & 7) || ((uintptr_t)d_ws & 7) || ((uintptr_t)d_in % w)) return PCOMP_EINVAL;
    Layout lo;
    make_layout(n, w, block_len, flags_of(variant, block_len), lo);
    if (out_capacity < pcomp_bound(n, dtype, block_len, variant)) return PCOMP_ENOSPC;
    if (ws_bytes < ws_bytes_for(lo)) return PCOMP_ENOWS;
    CompressArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    hipStream_t st = (hipStream_t)stream;
    uint64_t *ws = (uint64_t *)d_ws;
    const uint64_t ws_words = ws_bytes_for(lo) / 8;
    const uint64_t fill_blocks = (ws_words + 255) / 256;
    fill_u64_kernel<<<(uint32_t)(fill_blocks < 1024 ? fill_blocks : 1024), 256, 0, st>>>(ws, ws_words, 0);
    a.in = (const uint8_t *)d_in;
    a.out = (uint8_t *)d_out;
    a.out_size = d_out_size;
    a.ticket = (uint32_t *)ws;
    a.err = (uint32_t *)ws + 1;
    a.tile_status = ws + 1;
    a.lo = lo;
    a.variant = variant;
    const uint32_t grid = (uint32_t)(lo.n_tiles ? lo.n_tiles : 1);
    if (w == 1)
        compress_kernel<1><<<grid, kThreads, 0, st>>>(a);
    else if (w == 2)
        compress_kernel<2><<<grid, kThreads, 0, st>>>(a);
    else
        compress_kernel<4><<<grid, kThreads, 0, st>>>(a);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

extern "C" int pcomp_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity,
                                int32_t *d_status, void *stream) {
    if (!d_in || !d_status || (out_capacity && !d_out)) return PCOMP_EINVAL;
    if (((uintptr_t)d_in & 7)) return PCOMP_EINVAL;
    DecompressArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    hipStream_t st = (hipStream_t)stream;
    set_i32_kernel<<<1, 1, 0, st>>>(d_status, PCOMP_OK);
    a.in = (const uint8_t *)d_in;
    a.in_size = in_size;
    a.out = (uint8_t *)d_out;
    a.out_cap = out_capacity;
    a.status = d_status;
    // persistent grid: enough workgroups to fill every CU several times over
    const uint64_t max_tiles = in_size > kHdrBytes ? (in_size - kHdrBytes) / 8 : 1;
    const uint32_t grid = (uint32_t)(max_tiles < 1 ? 1 : (max_tiles < 4096 ? max_tiles : 4096));
    decompress_kernel<<<grid, kThreads, 0, st>>>(a);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

extern "C" int pcomp_stream_info(const void *h_header, uint64_t *n, int *dtype_bytes, uint32_t *block_len,
                                 uint64_t *total_bytes) {
    if (!h_header) return PCOMP_EINVAL;
    const uint64_t *h = (const uint64_t *)h_header;
    if ((uint32_t)h[0] != kMagic || ((h[0] >> 32) & 0xFFFF) != kVersion) return PCOMP_ECORRUPT;
    const int w = (int)((h[0] >> 48) & 0xFF);
    if (!dtype_ok(w)) return PCOMP_ECORRUPT;
    if (n) *n = h[2];
    if (dtype_bytes) *dtype_bytes = w;
    if (block_len) *block_len = (uint32_t)(h[1] >> 32);
    if (total_bytes) *total_bytes = h[6];
    return PCOMP_OK;
}
