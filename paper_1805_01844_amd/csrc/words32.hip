// words32.hip -- streams of 32-bit words: the paper's own word, the unsigned int of Sec. 3.1
// (Eq. (1) with capacity 2^32) and of the series that closes Sec. 3.2. Only the paper's two
// packings (t = 0): class 0 basic and class 8 advanced; a stream holds one of them, or per block
// the smaller of the two (ties to basic). Advanced blocks need B <= 2^16 + 1, which u8 and u16
// data always meet; u32 data take class 0.
//
// Compression: w32_stats_kernel<W> (one workgroup per tile: min and max of every block, its
// class and words, the tile's total), the two scan launches of the 64-bit streams (tile
// offsets), w32_pack_kernel<W> (the tile's block arrays, index entry and words) and
// w32_header_kernel. Decompression: w32_decompress_kernel<W>, persistent over the tiles.
// Every word is below 2^32, so packing is 32-bit multiply-add and every division of decoding is
// a binary64 one by a stored reciprocal, exact for dividends below 2^51 (digit_off).
#include "kernels_common.h"

namespace pcomp {

void launch_tile_scan(uint32_t *tile_words, uint64_t *prefix, uint64_t *sums, uint64_t n_tiles, hipStream_t st);
uint64_t tile_scan_runs(uint64_t n_tiles);

struct W32Args {
    const uint8_t *in;     // values to compress
    uint8_t *out;          // the stream
    uint64_t out_cap;      // bytes at out
    Layout lo;
    int variant;           // 0, 8 or PCOMP_SELECT_EXHAUSTIVE
    DevTables T;
    uint32_t *err;         // error word: bit 2 = a tile's payload would pass the capacity (not written)
    uint32_t *meta;        // [n_blocks]: class | words << 4 (stats -> pack)
    uint32_t *tile_words;  // [n_tiles]
    uint64_t *prefix;      // [n_tiles + 1]
    uint64_t *out_size;    // device u64: the stream's bytes
};

struct W32DecArgs {
    const uint8_t *in;
    uint64_t in_size;
    uint8_t *out;
    uint64_t out_cap;  // values
    int32_t *status;
    uint32_t want_L;
    DevTables T;
};

// Digits per 32-bit word, k = max{k : B^k <= 2^32} (Eq. (1), exact reading), for B >= 2: from
// the tables up to 2^16 + 1, and 1 above (B^2 > 2^32).
__device__ __forceinline__ uint32_t k32_of(const DevTables &T, uint64_t B) {
    return B <= kAtlasDirect ? T.desc32[B].k : 1u;
}

// Words of class c (0 basic, 8 advanced) for Lb digits of base B (B <= 2^16 + 1 for class 8).
__device__ __forceinline__ uint32_t words32(const DevTables &T, int c, uint32_t Lb, uint64_t B) {
    if (Lb == 0 || B <= 1) return 0;
    if (c == 0) {
        const uint32_t k = k32_of(T, B);
        return udiv_small(Lb + k - 1, k);
    }
    const BaseDesc32 &D = T.desc32[B];
    return adv_words_cycle(T.ent32 + D.off, D, Lb);
}

// Entry of word i of the series and its q_i, from the cycle form (entries 0 .. mu + lam - 1
// stored; word i >= mu repeats entry mu + (i - mu) mod lam, V values further on per period).
__device__ __forceinline__ const AtlasEntry32 *entry32(const DevTables &T, const BaseDesc32 &D, uint32_t i,
                                                       uint32_t &q) {
    const AtlasEntry32 *E = T.ent32 + D.off;
    const uint32_t tot = (uint32_t)D.mu + D.lam;
    if (i < tot) {
        q = E[i].q;
        return E + i;
    }
    const uint32_t c = udiv_small(i - D.mu, D.lam);
    const uint32_t r = i - c * D.lam;
    q = E[r].q + c * D.V;
    return E + r;
}

// Consecutive words of the series from the cycle form: the entry of word i, then of i + 1, ...
// without a division per word (entry mu + lam - 1 is followed by entry mu, V values further on).
struct Cursor32 {
    const AtlasEntry32 *E;
    uint32_t idx, cyc, tot, mu, V;
    __device__ __forceinline__ Cursor32(const DevTables &T, const BaseDesc32 &D, uint32_t i) {
        E = T.ent32 + D.off;
        mu = D.mu;
        V = D.V;
        tot = (uint32_t)D.mu + D.lam;
        if (i < tot) {
            idx = i;
            cyc = 0;
        } else {
            cyc = udiv_small(i - D.mu, D.lam);
            idx = i - cyc * D.lam;
        }
    }
    __device__ __forceinline__ const AtlasEntry32 &entry() const { return E[idx]; }
    __device__ __forceinline__ uint32_t q() const { return E[idx].q + cyc * V; }
    __device__ __forceinline__ void next() {
        if (++idx == tot) {
            idx = mu;
            cyc++;
        }
    }
};

// Stores the values of one tile, staged in LDS at the same offsets within 16-byte chunks as
// they take in global memory (value 0 at byte (out + v0 W) mod 16): whole chunks as 16-byte
// stores, the partial chunks at the ends value by value, so no byte outside the tile is written.
template <int W>
__device__ __forceinline__ void unstage_tile(uint8_t *out, uint64_t v0, uint32_t nvt, const uint4 *s_raw) {
    typedef typename Elem<W>::T V;
    const uint8_t *s_bytes = (const uint8_t *)s_raw;
    const uintptr_t addr = (uintptr_t)(out + v0 * W);
    const uint32_t head = (uint32_t)(addr & 15);
    uint8_t *gbase = (uint8_t *)(addr - head);
    const uint32_t span = head + nvt * W;
    const uint32_t nchunks = (span + 15) >> 4;
    for (uint32_t c = threadIdx.x; c < nchunks; c += kThreads) {
        const uint32_t cb = c << 4;
        if (cb >= head && cb + 16 <= span) {
            *(uint4 *)(gbase + cb) = s_raw[c];
        } else {
            const uint32_t e0 = cb > head ? cb : head, e1 = cb + 16 < span ? cb + 16 : span;
            for (uint32_t b = e0; b < e1; b += W) *(V *)(gbase + b) = *(const V *)(s_bytes + b);
        }
    }
}

// Per block of the tile: min and max over the G lanes of the block's group.
template <typename P>
__device__ __forceinline__ void block_minmax(P bv, uint32_t Lb, uint32_t g, uint32_t G, uint32_t *s_red32,
                                             uint32_t &vmin, uint32_t &vmax) {
    vmin = 0xFFFFFFFFu;
    vmax = 0;
    for (uint32_t j = g; j < Lb; j += G) {
        const uint32_t v = bv[j];
        vmin = v < vmin ? v : vmin;
        vmax = v > vmax ? v : vmax;
    }
    vmin = group_reduce(vmin, G, MinOp(), s_red32);
    vmax = group_reduce(vmax, G, MaxOp(), s_red32);
}

// ---- compression -------------------------------------------------------------------------
__global__ void w32_begin_kernel(uint32_t *err) { *err = 0; }

template <int W>
__global__ __launch_bounds__(kThreads) void w32_stats_kernel(W32Args a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint32_t s_nw[kMaxTileBlocks];
    const Layout &lo = a.lo;
    const uint64_t t = blockIdx.x;
    const uint32_t tid = threadIdx.x, L = lo.L, tb = lo.tile_blocks;
    const uint64_t b0 = t * tb;
    const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
    const uint64_t v0 = b0 * L;
    const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
    const V *s_val = stage_tile<W>(a.in, v0, nvt, s_raw);
    __syncthreads();
    const uint32_t G = kThreads / tb, blk = tid / G, g = tid % G;
    const bool live = blk < nbt;
    const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
    uint32_t vmin, vmax;
    block_minmax(lds_ptr(s_val + (size_t)blk * L), Lb, g, G, s_red32, vmin, vmax);
    if (live && g == 0) {
        const uint64_t B = (uint64_t)vmax - vmin + 1;
        int c = a.variant == 8 ? 8 : 0;
        uint32_t nw = words32(a.T, c, Lb, B);
        if (a.variant == PCOMP_SELECT_EXHAUSTIVE) {
            const uint32_t n8 = words32(a.T, 8, Lb, B);
            if (n8 < nw) {
                c = 8;
                nw = n8;
            }
        }
        a.meta[b0 + blk] = (uint32_t)c | (nw << 4);
        s_nw[blk] = nw;
    }
    __syncthreads();
    uint32_t total;
    wg_excl_scan(tid < nbt ? s_nw[tid] : 0u, s_red32, &total);
    if (tid == 0) a.tile_words[t] = total;
}

template <int W>
__global__ __launch_bounds__(kThreads) void w32_pack_kernel(W32Args a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint32_t s_off[kMaxTileBlocks];
    const Layout &lo = a.lo;
    const uint64_t t = blockIdx.x;
    const uint32_t tid = threadIdx.x, L = lo.L, tb = lo.tile_blocks;
    const uint64_t b0 = t * tb;
    const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
    const uint64_t v0 = b0 * L;
    const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
    const V *s_val = stage_tile<W>(a.in, v0, nvt, s_raw);
    // word offsets of the tile's blocks, and where the tile's words start
    uint32_t total;
    const uint32_t ex = wg_excl_scan(tid < nbt ? a.meta[b0 + tid] >> 4 : 0u, s_red32, &total);
    if (tid < nbt) s_off[tid] = ex;
    const uint64_t base = a.prefix[t];
    __syncthreads();
    if (lo.off_payload + 4 * (base + total) > a.out_cap) {  // only if the sizing were wrong
        if (tid == 0) atomicOr(a.err, 4u);
        return;
    }
    if (tid == 0) *(uint64_t *)(a.out + lo.off_index + 8 * t) = base;
    const uint32_t G = kThreads / tb, blk = tid / G, g = tid % G;
    const bool live = blk < nbt;
    const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
    const auto *bv = lds_ptr(s_val + (size_t)blk * L);
    uint32_t vmin, vmax;
    block_minmax(bv, Lb, g, G, s_red32, vmin, vmax);
    if (!live) return;
    const uint64_t b = b0 + blk;
    const uint64_t B = (uint64_t)vmax - vmin + 1;
    const uint32_t meta = a.meta[b];
    const int c = (int)(meta & 15);
    const uint32_t nw = meta >> 4;
    if (g == 0) {
        *(V *)(a.out + lo.off_min + (uint64_t)W * b) = (V)vmin;
        *(V *)(a.out + lo.off_range + (uint64_t)W * b) = (V)(B - 1);
        if (lo.flags & kFlagClass) a.out[lo.off_class + b] = (uint8_t)c;
    }
    uint32_t *dst = (uint32_t *)(a.out + lo.off_payload) + base + s_off[blk];
    auto get = [&](uint32_t j) -> uint32_t { return j < Lb ? (uint32_t)bv[j] - vmin : 0u; };
    if (c == 0) {
        // Eq. (2): k digits per word, the first at the highest power of B
        const uint32_t k = B > 1 ? k32_of(a.T, B) : 1u;
        const uint32_t Bu = (uint32_t)B;  // k >= 2 implies B <= 2^16
        for (uint32_t i = g; i < nw; i += G) {
            uint32_t x;
            if (k == 1) {
                x = get(i);
            } else {
                x = 0;
                const uint32_t j0 = i * k;
                for (uint32_t jj = 0; jj < k; jj++) x = x * Bu + get(j0 + jj);
            }
            dst[i] = x;
        }
    } else if (nw) {
        // the series: word i = (r'_{i-1} B^{p_i} + its p_i digits) R_i + r_i, where the value
        // after those digits is split as r_i = x mod R_i here and r'_i = x div R_i in word i + 1.
        // Lane g packs a run of consecutive words and carries r'_i from one to the next; only
        // the run's first word divides its predecessor's split value.
        const BaseDesc32 &D = a.T.desc32[B];
        const uint32_t Bu = (uint32_t)B;
        const uint32_t run = udiv_small(nw + G - 1, G);
        const uint32_t w0 = g * run, w1 = w0 + run < nw ? w0 + run : nw;
        if (w0 < w1) {
            Cursor32 cur(a.T, D, w0);
            uint32_t top = 0;  // r'_{i-1}
            if (w0 > 0) {
                uint32_t qp;
                const AtlasEntry32 *ep = entry32(a.T, D, w0 - 1, qp);
                top = get(qp + ep->p) / ep->R;
            }
            for (uint32_t i = w0; i < w1; i++) {
                const AtlasEntry32 &e = cur.entry();
                const uint32_t q = cur.q(), p = e.p, R = e.R;
                uint32_t body = top;
                for (uint32_t kk = 0; kk < p; kk++) body = body * Bu + get(q + kk);
                const uint32_t x = get(q + p);
                top = x / R;
                dst[i] = body * R + (x - top * R);
                cur.next();
            }
        }
    }
}

// Header, the zero padding before the payload, and the stream size (after the scans).
__global__ void w32_header_kernel(W32Args a) {
    const Layout &lo = a.lo;
    const uint64_t words = lo.n_tiles ? a.prefix[lo.n_tiles] : 0;
    const uint64_t total = lo.off_payload + 4 * words;
    for (uint64_t o = lo.off_ne + threadIdx.x; o < lo.off_payload; o += blockDim.x) a.out[o] = 0;
    if (threadIdx.x == 0) {
        const bool exh = a.variant == PCOMP_SELECT_EXHAUSTIVE;
        uint64_t *h = (uint64_t *)a.out;
        h[0] = (uint64_t)kMagic | ((uint64_t)kVersion << 32) | ((uint64_t)lo.w << 48) | ((uint64_t)lo.flags << 56);
        h[1] = (uint64_t)(exh ? 0 : a.variant) | ((uint64_t)(exh ? 1 : 0) << 8) | ((uint64_t)lo.L << 32);
        h[2] = lo.n;
        h[3] = lo.n_blocks;
        h[4] = lo.tile_blocks;
        h[5] = words;
        h[6] = total;
        h[7] = 0;
        *a.out_size = total;
    }
}

// ---- decompression -----------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kThreads) void w32_decompress_kernel(W32DecArgs a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 2];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint32_t s_nw[kMaxTileBlocks];
    __shared__ uint32_t s_off[kMaxTileBlocks];
    __shared__ uint32_t s_bad;
    const uint32_t tid = threadIdx.x;
    const bool reporter = blockIdx.x == 0 && tid == 0;
    if (a.in_size < kHdrBytes) {
        if (reporter) *a.status = PCOMP_ECORRUPT;
        return;
    }
    // the header (every lane reads the same 64 bytes)
    const uint64_t *h = (const uint64_t *)a.in;
    const uint64_t h0 = h[0], h1 = h[1], n = h[2], nb = h[3], h4 = h[4], pw = h[5], total = h[6];
    const uint32_t flags = (uint32_t)(h0 >> 56) & 0xFF, w = (uint32_t)(h0 >> 48) & 0xFF, L = (uint32_t)(h1 >> 32);
    const int fixed = (int)(h1 & 0xFF);
    bool ok = (uint32_t)h0 == kMagic && ((h0 >> 32) & 0xFFFF) == kVersion && w == (uint32_t)W && L == a.want_L &&
              (flags == kFlagW32 || flags == (kFlagW32 | kFlagClass)) &&
              ((flags & kFlagClass) || fixed == 0 || fixed == 8) && pw <= a.in_size / 4;
    if (ok && n > a.out_cap) {
        if (reporter) *a.status = PCOMP_ENOSPC;
        return;
    }
    Layout lo;
    if (ok) {
        make_layout(n, W, L, flags, lo);
        ok = nb == lo.n_blocks && (uint32_t)h4 == lo.tile_blocks && (h4 >> 32) == 0 &&
             total == lo.off_payload + 4 * pw && total <= a.in_size;
    }
    if (!ok) {
        if (reporter) *a.status = PCOMP_ECORRUPT;
        return;
    }
    const uint64_t *index = (const uint64_t *)(a.in + lo.off_index);
    const uint32_t *payload = (const uint32_t *)(a.in + lo.off_payload);
    const uint32_t tb = lo.tile_blocks, G = kThreads / tb, blk = tid / G, g = tid % G;
    const uint64_t vmax_w = W == 4 ? 0xFFFFFFFFull : (1ull << (8 * W)) - 1;
    uint8_t *s_bytes = (uint8_t *)s_raw;
    for (uint64_t t = blockIdx.x; t < lo.n_tiles; t += gridDim.x) {
        const uint64_t b0 = t * tb;
        const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
        const uint64_t v0 = b0 * L;
        const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, n - v0);
        const bool live = blk < nbt;
        const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, n - (b0 + blk) * L) : 0;
        const uint64_t b = b0 + blk;
        uint32_t vmin = 0, nw = 0;
        uint64_t B = 1;
        int c = 0;
        bool bad = false;
        if (live) {
            vmin = *(const V *)(a.in + lo.off_min + (uint64_t)W * b);
            B = (uint64_t)*(const V *)(a.in + lo.off_range + (uint64_t)W * b) + 1;
            c = (flags & kFlagClass) ? a.in[lo.off_class + b] : fixed;
            bad = (c != 0 && c != 8) || (c == 8 && B > kAtlasDirect) || (uint64_t)vmin + B - 1 > vmax_w;
            if (!bad) nw = words32(a.T, c, Lb, B);
        }
        if (tid == 0) s_bad = 0;
        if (live && g == 0) s_nw[blk] = nw;
        __syncthreads();
        if (bad) s_bad = 1;
        uint32_t tot;
        const uint32_t ex = wg_excl_scan(tid < nbt ? s_nw[tid] : 0u, s_red32, &tot);
        if (tid < nbt) s_off[tid] = ex;
        const uint64_t p0 = index[t], p1 = t + 1 < lo.n_tiles ? index[t + 1] : pw;
        if (tid == 0 && (p0 > p1 || p1 > pw || p1 - p0 != tot)) s_bad = 1;
        __syncthreads();
        const bool tile_bad = s_bad != 0;
        __syncthreads();  // every lane has read the flag before the next tile resets it
        if (tile_bad) {
            if (tid == 0) *a.status = PCOMP_ECORRUPT;
            continue;
        }
        // decode into LDS, value j of the tile at byte head + j W (head: alignment of the output)
        const uint32_t head = (uint32_t)((uintptr_t)(a.out + v0 * W) & 15);
        V *s_out = (V *)(s_bytes + head) + (size_t)blk * L;
        if (live) {
            const uint32_t *src = payload + p0 + s_off[blk];
            if (B <= 1) {
                for (uint32_t j = g; j < Lb; j += G) s_out[j] = (V)vmin;
            } else if (c == 0) {
                const uint32_t k = k32_of(a.T, B);
                if (k == 1) {
                    for (uint32_t i = g; i < nw; i += G) s_out[i] = (V)(vmin + src[i]);
                } else {
                    // polynomial division (Sec. 3.1): the last digit of the word comes out first
                    const double rB = a.T.desc32[B].rB, hB = 0.5 * rB, Bf = (double)B;
                    for (uint32_t i = g; i < nw; i += G) {
                        double x = (double)src[i];
                        const uint32_t j0 = i * k;
                        for (uint32_t jj = k; jj-- > 0;) {
                            uint32_t d;
                            x = digit_off(x, rB, hB, Bf, d);
                            if (j0 + jj < Lb) s_out[j0 + jj] = (V)(vmin + d);
                        }
                    }
                }
            } else {
                // lane g decodes a run of consecutive words: the value split between two of them
                // is rebuilt from what the lane holds (r_{i-1} from the bottom of word i - 1,
                // r'_{i-1} left on top of word i); only the run's first word reads its predecessor
                const BaseDesc32 &D = a.T.desc32[B];
                const double rB = D.rB, hB = 0.5 * rB, Bf = (double)B;
                const uint32_t run = udiv_small(nw + G - 1, G);
                const uint32_t w0 = g * run, w1 = w0 + run < nw ? w0 + run : nw;
                if (w0 < w1) {
                    Cursor32 cur(a.T, D, w0);
                    uint32_t r_prev = 0, R_prev = 1;
                    if (w0 > 0) {
                        uint32_t qp;
                        const AtlasEntry32 *ep = entry32(a.T, D, w0 - 1, qp);
                        digit_off((double)src[w0 - 1], ep->rR, 0.5 * ep->rR, (double)ep->R, r_prev);
                        R_prev = ep->R;
                    }
                    for (uint32_t i = w0; i < w1; i++) {
                        const AtlasEntry32 &e = cur.entry();
                        const uint32_t q = cur.q(), p = e.p;
                        uint32_t r;
                        double x = digit_off((double)src[i], e.rR, 0.5 * e.rR, (double)e.R, r);  // r_i
                        for (uint32_t kk = p; kk-- > 0;) {
                            uint32_t d;
                            x = digit_off(x, rB, hB, Bf, d);
                            if (q + kk < Lb) s_out[q + kk] = (V)(vmin + d);
                        }
                        // what is left is r'_{i-1}: with r_{i-1}, the value split before this word
                        if (i > 0 && q - 1 < Lb) s_out[q - 1] = (V)(vmin + (uint32_t)x * R_prev + r_prev);
                        r_prev = r;
                        R_prev = e.R;
                        cur.next();
                    }
                }
            }
        }
        __syncthreads();
        unstage_tile<W>(a.out, v0, nvt, s_raw);
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ---- host side ---------------------------------------------------------------------------
// Workspace: [err u32, 0 u32][meta u32 x n_blocks][tile_words u32 x n_tiles][prefix u64 x
// (n_tiles + 1)][scan sums], each part 8-byte aligned.
struct W32Ws {
    uint64_t meta, tile_words, prefix, sums, bytes;
};
static W32Ws w32_ws_layout(const Layout &lo) {
    W32Ws w;
    w.meta = 8;
    w.tile_words = w.meta + 4 * ((lo.n_blocks + 1) & ~1ull);
    w.prefix = w.tile_words + 4 * ((lo.n_tiles + 1) & ~1ull);
    w.sums = w.prefix + 8 * (lo.n_tiles + 1);
    w.bytes = w.sums + 8 * tile_scan_runs(lo.n_tiles);
    return w;
}
uint64_t w32_ws_bytes(const Layout &lo) { return w32_ws_layout(lo).bytes; }

int launch_compress32(const void *d_in, const Layout &lo, int variant, void *d_out, uint64_t out_cap,
                      uint64_t *d_out_size, void *ws, hipStream_t st) {
    W32Args a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    const W32Ws wl = w32_ws_layout(lo);
    uint8_t *wsb = (uint8_t *)ws;
    a.in = (const uint8_t *)d_in;
    a.out = (uint8_t *)d_out;
    a.out_cap = out_cap;
    a.lo = lo;
    a.variant = variant;
    a.err = (uint32_t *)wsb;
    a.meta = (uint32_t *)(wsb + wl.meta);
    a.tile_words = (uint32_t *)(wsb + wl.tile_words);
    a.prefix = (uint64_t *)(wsb + wl.prefix);
    a.out_size = d_out_size;
    const uint64_t nt = lo.n_tiles;
    if (nt > 0x7FFFFFFFull) return PCOMP_EINVAL;  // one workgroup per tile
    w32_begin_kernel<<<1, 1, 0, st>>>(a.err);
    if (nt) {
        const uint32_t grid = (uint32_t)nt;
        if (lo.w == 1)
            w32_stats_kernel<1><<<grid, kThreads, 0, st>>>(a);
        else if (lo.w == 2)
            w32_stats_kernel<2><<<grid, kThreads, 0, st>>>(a);
        else
            w32_stats_kernel<4><<<grid, kThreads, 0, st>>>(a);
        launch_tile_scan(a.tile_words, a.prefix, (uint64_t *)(wsb + wl.sums), nt, st);
        if (lo.w == 1)
            w32_pack_kernel<1><<<grid, kThreads, 0, st>>>(a);
        else if (lo.w == 2)
            w32_pack_kernel<2><<<grid, kThreads, 0, st>>>(a);
        else
            w32_pack_kernel<4><<<grid, kThreads, 0, st>>>(a);
    }
    w32_header_kernel<<<1, kThreads, 0, st>>>(a);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

__global__ void w32_status_kernel(int32_t *p) { *p = PCOMP_OK; }

int launch_decompress32(const void *d_in, size_t in_size, void *d_out, size_t out_capacity, int32_t *d_status,
                        int w, uint32_t L, hipStream_t st) {
    W32DecArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    a.in = (const uint8_t *)d_in;
    a.in_size = in_size;
    a.out = (uint8_t *)d_out;
    a.out_cap = out_capacity;
    a.status = d_status;
    a.want_L = L;
    w32_status_kernel<<<1, 1, 0, st>>>(d_status);
    // at most one tile per 8 bytes of index; a persistent grid walks them
    const uint64_t max_tiles = in_size > kHdrBytes ? (in_size - kHdrBytes) / 8 : 1;
    const uint32_t grid = (uint32_t)(max_tiles < 1 ? 1 : (max_tiles < 4096 ? max_tiles : 4096));
    if (w == 1)
        w32_decompress_kernel<1><<<grid, kThreads, 0, st>>>(a);
    else if (w == 2)
        w32_decompress_kernel<2><<<grid, kThreads, 0, st>>>(a);
    else
        w32_decompress_kernel<4><<<grid, kThreads, 0, st>>>(a);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

}  // namespace pcomp
