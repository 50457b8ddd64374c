// compress.hip -- compression kernels (gfx950).
//
// Three launches, with no communication between workgroups inside any of them:
//   1. stats_kernel, one workgroup per tile of tile_blocks blocks (at most 16 KiB of input):
//      stage the tile in LDS with 128-bit loads; per block (a group of G = 256 / tile_blocks
//      lanes) min and max by wavefront shuffles, B = max - min + 1 (Sec. 3, Sec. 3.1), and
//      when threshold classes are possible the counts of digits at or above 2^(beta - t);
//      size the candidate classes (basic Sec. 3.1 Eq. (1)-(2), advanced Sec. 3.2 series,
//      threshold/excess split), keep the smallest (ties to the lowest id), write the block
//      arrays of the stream and the tile's word total.
//   2. scan_kernel: exclusive prefix sum of the tile totals -> the stream's tile index,
//      payload size and header.
//   3. pack_kernel, one workgroup per tile: stage the tile again, read its block arrays,
//      compact the excess lists of threshold blocks, and pack: the lanes of a block's group
//      take its words in turn, each word a 64-bit Horner multiply-add over its digits, the
//      first digit at the highest power.
#include "kernels_common.h"

namespace pcomp {

struct CompressArgs {
    const uint8_t *in;
    uint8_t *out;
    uint64_t *out_size;
    uint32_t *tile_words;  // [n_tiles] words of every tile (stats -> scan)
    uint32_t *err;
    const SizeCtx *ctx;    // size tables, filled once per launch
    Layout lo;
    int variant;
    DevTables T;
};

__device__ void write_header(const CompressArgs &a, uint64_t payload_words) {
    const Layout &lo = a.lo;
    const int variant = a.variant;
    const uint64_t total = lo.off_payload + 8 * payload_words;
    const uint32_t sel = variant == PCOMP_SELECT_EXHAUSTIVE ? 1 : variant == PCOMP_SELECT_LEARNED ? 2 : 0;
    const uint32_t fixed = (lo.flags & kFlagClass) ? 0 : (uint32_t)variant;
    uint64_t *o = (uint64_t *)a.out;
    o[0] = (uint64_t)kMagic | ((uint64_t)kVersion << 32) | ((uint64_t)lo.w << 48) | ((uint64_t)lo.flags << 56);
    o[1] = (uint64_t)fixed | ((uint64_t)sel << 8) | ((uint64_t)lo.L << 32);
    o[2] = lo.n;
    o[3] = lo.n_blocks;
    o[4] = (uint64_t)lo.tile_blocks;
    o[5] = payload_words;
    o[6] = total;
    o[7] = 0;
    // zero padding between the block arrays and the payload
    const uint64_t end_arrays =
        lo.off_ne + ((lo.flags & kFlagNe) ? lo.n_blocks * ((lo.flags & kFlagNe16) ? 2 : 1) : 0);
    for (uint64_t b = end_arrays; b < lo.off_payload; b++) a.out[b] = 0;
    *a.out_size = total;
}

// Advanced part whose base is outside the tables: one lane walks the series word by word.
template <typename Get>
__device__ __forceinline__ void pack_adv_slow(const DevTables &T, uint64_t base, uint32_t n, uint32_t nwords,
                                           uint64_t *dst, Get get) {
    const SlowBase sb = slow_base(T, base);
    uint64_t s = 1, rp = 0;
    uint32_t q = 0;
    for (uint32_t wi = 0; wi < nwords; wi++) {
        uint32_t p;
        uint64_t R;
        slow_word(sb, s, p, R);
        uint64_t acc = rp;
        for (uint32_t j = 0; j < p; j++) acc = acc * base + get(q + j);
        const uint64_t x = get(q + p);
        const uint64_t r = x % R;
        rp = x / R;
        dst[wi] = acc * R + r;
        if (q + p >= n) break;
        s = (base + R - 1) / R;
        q += p + 1;
    }
}

// Packs the words of one part of a block (main digits or the excess list); the lanes of
// the block's group call it with their first word index and stride. get(j) returns digit j
// of the part, 0 past its end.
template <typename Get>
__device__ __forceinline__ void pack_part(const DevTables &T, const SizeCtx &C, uint64_t base, uint32_t n, int fam,
                                          uint32_t nwords, uint32_t i0, uint32_t G, uint64_t *dst, Get get) {
    if (nwords == 0 || i0 >= nwords) return;
    const PartBase pb = resolve_base(T, C, base);
    if (!fam) {
        // Sec. 3.1 Eq. (2): word i holds digits i*k .. i*k+k-1, the first at the highest power
        for (uint32_t i = i0; i < nwords; i += G) dst[i] = horner_digits(pb, 0, i * pb.k, pb.k, get);
        return;
    }
    if (pb.D) {
        // Sec. 3.2 series: word i = (r'_{i-1} B^{p_i} + digits) R_i + r_i, state from the cycle form
        const BaseDesc &D = *pb.D;
        for (uint32_t i = i0; i < nwords; i += G) {
            uint32_t q;
            const AtlasEntry *e = adv_entry(T, D, i, q);
            uint32_t rp = 0;  // r'_{i-1}: top part of the value split at the end of word i-1
            if (i > 0) {
                uint32_t qp;
                const AtlasEntry *ep = adv_entry(T, D, i - 1, qp);
                rp = (uint32_t)div_magic(get(q - 1), ep->mR);
            }
            const uint64_t x = get(q + e->p);
            const uint64_t r = x - div_magic(x, e->mR) * e->R;
            dst[i] = horner_digits(pb, rp, q, e->p, get) * e->R + r;
        }
        return;
    }
    // base outside the tables: the group's first lane walks the series over the whole part
    if (i0 == 0) pack_adv_slow(T, base, n, nwords, dst, get);
}

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

__device__ __forceinline__ void copy_size_ctx(const SizeCtx *g, SizeCtx &s) {
    if (threadIdx.x < sizeof(SizeCtx) / 4) ((uint32_t *)&s)[threadIdx.x] = ((const uint32_t *)g)[threadIdx.x];
}

// ---- launch 1: block statistics, class choice, block arrays, tile totals ----------------
template <int W>
__global__ __launch_bounds__(kThreads) void stats_kernel(CompressArgs a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    __shared__ uint32_t s_nw[kMaxTileBlocks];
    __shared__ uint64_t s_red64[kThreads / 64];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ SizeCtx s_C;

    const Layout &lo = a.lo;
    const DevTables &T = a.T;
    const uint32_t tid = threadIdx.x;
    const int variant = a.variant;
    const bool fixed0 = (variant == 0 || variant == 8);
    const uint32_t L = lo.L, tb = lo.tile_blocks;
    const uint32_t tile = blockIdx.x;
    if (tile >= lo.n_tiles) return;
    copy_size_ctx(a.ctx, s_C);
    const uint64_t b0 = (uint64_t)tile * tb;
    const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
    const uint64_t v0 = b0 * L;
    const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
    const V *s_val = stage_tile<W>(a.in, v0, nvt, s_raw);
    __syncthreads();

    // per block: min / max (B = v_max - v_min + 1) and excess counts
    const uint32_t G = kThreads / tb;
    const uint32_t blk = tid / G, g = tid % G;
    const bool live = blk < nbt;
    const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
    const V *bv = s_val + (size_t)blk * L;
    uint32_t vmin = 0xFFFFFFFFu, vmax = 0;
    for (uint32_t j = g; j < Lb; j += G) {
        const uint32_t v = bv[j];
        vmin = v < vmin ? v : vmin;
        vmax = v > vmax ? v : vmax;
    }
    vmin = group_reduce(vmin, G, MinOp(), s_red32);
    vmax = group_reduce(vmax, G, MaxOp(), s_red32);
    const uint64_t B = live ? (uint64_t)vmax - vmin + 1 : 1;
    const uint32_t beta = bitlen64(B - 1);
    // bin b = beta - bitlen(d): digits in octave b below the top; n_e(t) = bins 0 .. t-1
    uint32_t ne_t[8];
    ne_t[0] = 0;
    if (!fixed0) {
        uint64_t h = 0;  // eight 8-bit counters (at most 64 digits per lane)
        for (uint32_t j = g; j < Lb; j += G) {
            const uint32_t b = beta - bitlen32((uint32_t)bv[j] - vmin);
            h += b < 8 ? (1ull << (8 * b)) : 0;
        }
        uint64_t h0 = 0, h1 = 0;  // widened to 16-bit counters before the group sum
#pragma unroll
        for (int t = 0; t < 4; t++) {
            h0 |= ((h >> (8 * t)) & 0xFF) << (16 * t);
            h1 |= ((h >> (8 * (t + 4))) & 0xFF) << (16 * t);
        }
        h0 = group_reduce(h0, G, AddOp(), s_red64);
        h1 = group_reduce(h1, G, AddOp(), s_red64);
#pragma unroll
        for (int t = 1; t < 8; t++)
            ne_t[t] = ne_t[t - 1] +
                      (uint32_t)(((t - 1) < 4 ? (h0 >> (16 * (t - 1))) : (h1 >> (16 * (t - 5)))) & 0xFFFF);
    } else {
#pragma unroll
        for (int t = 1; t < 8; t++) ne_t[t] = 0;
    }

    // class choice: lanes of the group split the candidates; argmin, ties to the lowest id
    uint64_t key = ~0ull;
    if (live) {
        for (int c = (int)g; c < 16; c += (int)G) {
            const bool cand = fixed0 ? (c == variant) : (c == 0 || variant == PCOMP_SELECT_EXHAUSTIVE || c == variant);
            const int t = c & 7;
            if (!cand || t > (int)beta) continue;
            uint32_t nwm, net = 0;
#pragma unroll
            for (int tt = 1; tt < 8; tt++) net = (t == tt) ? ne_t[tt] : net;  // no dynamic register index
            const uint32_t nw = class_words(T, s_C, L, c, Lb, B, beta, net, nwm);
            const uint64_t k2 = ((uint64_t)nw << 8) | (uint64_t)c;
            key = k2 < key ? k2 : key;
        }
    }
    key = group_reduce(key, G, MinOp(), s_red64);
    const int cls = (int)(key & 0xFF);
    const int tcls = cls & 7;
    uint32_t nw = live ? (uint32_t)(key >> 8) : 0;
    // every chosen class is at most the basic t = 0 size, which the bound assumes
    const uint32_t per = 8 / W, cap = (Lb + per - 1) / per;
    if (nw > cap) {
        if (g == 0) atomicOr(a.err, 2u);
        nw = cap;
    }
    uint32_t ne = 0;
#pragma unroll
    for (int tt = 1; tt < 8; tt++) ne = (tcls == tt) ? ne_t[tt] : ne;
    if (live && g == 0) {
        s_nw[blk] = nw;
        const uint64_t gb = b0 + blk;
        put_le(a.out + lo.off_min + gb * W, vmin, W);
        put_le(a.out + lo.off_range + gb * W, B - 1, W);
        if (lo.flags & kFlagClass) a.out[lo.off_class + gb] = (uint8_t)cls;
        if (lo.flags & kFlagNe)
            put_le(a.out + lo.off_ne + gb * ((lo.flags & kFlagNe16) ? 2 : 1), ne, (lo.flags & kFlagNe16) ? 2 : 1);
    }
    __syncthreads();
    uint32_t total;
    wg_excl_scan(tid < nbt ? s_nw[tid] : 0, s_red32, &total);
    if (tid == 0) a.tile_words[tile] = total;
}

// ---- launch 2: tile index (exclusive prefix of the tile totals) and header --------------
// Two small launches: every workgroup sums a run of kScanTiles tile totals; then every
// workgroup adds the sums of the runs before its own and scans its run into the index.
constexpr uint32_t kScanPer = 32;                      // tile totals per thread
constexpr uint32_t kScanTiles = kScanPer * kThreads;  // tile totals per workgroup

__global__ __launch_bounds__(kThreads) void scan_sums_kernel(CompressArgs a, uint64_t *sums) {
    __shared__ uint32_t s_red32[kThreads / 64];
    const uint64_t nt = a.lo.n_tiles;
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanTiles;
    uint32_t sum = 0;
    for (uint32_t m = 0; m < kScanPer; m++) {
        const uint64_t t = t0 + (uint64_t)m * kThreads + threadIdx.x;  // coalesced
        if (t < nt) sum += a.tile_words[t];
    }
    uint32_t total;
    wg_excl_scan(sum, s_red32, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kThreads) void scan_index_kernel(CompressArgs a, const uint64_t *sums) {
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint64_t s_red64[kThreads / 64];
    const Layout &lo = a.lo;
    const uint64_t nt = lo.n_tiles;
    const uint32_t tid = threadIdx.x;
    // sum of the runs before this one
    uint64_t before = 0;
    for (uint32_t r = tid; r < blockIdx.x; r += kThreads) before += sums[r];
    before = group_reduce(before, kThreads, AddOp(), s_red64);
    // this thread's kScanPer consecutive tiles
    const uint64_t t0 = (uint64_t)blockIdx.x * kScanTiles + (uint64_t)tid * kScanPer;
    uint32_t v[kScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t m = 0; m < kScanPer; m++) {
        v[m] = (t0 + m < nt) ? a.tile_words[t0 + m] : 0;
        sum += v[m];
    }
    uint32_t total;
    const uint32_t ex = wg_excl_scan(sum, s_red32, &total);
    uint64_t run = before + ex;
    uint64_t *index = (uint64_t *)(a.out + lo.off_index);
#pragma unroll
    for (uint32_t m = 0; m < kScanPer; m++) {
        if (t0 + m < nt) index[t0 + m] = run;
        run += v[m];
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) write_header(a, before + total);
}

// ---- launch 3: packing ----------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kThreads) void pack_kernel(CompressArgs a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    extern __shared__ uint4 s_dyn[];  // excess lists (kTileBytes) when threshold classes are possible
    __shared__ uint32_t s_min[kMaxTileBlocks], s_rng[kMaxTileBlocks], s_ne[kMaxTileBlocks], s_off[kMaxTileBlocks];
    __shared__ uint8_t s_cls[kMaxTileBlocks];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ SizeCtx s_C;

    const Layout &lo = a.lo;
    const DevTables &T = a.T;
    const uint32_t tid = threadIdx.x;
    const int variant = a.variant;
    const bool fixed0 = (variant == 0 || variant == 8);
    const uint32_t L = lo.L, tb = lo.tile_blocks;
    const uint32_t tile = blockIdx.x;
    if (tile >= lo.n_tiles) return;
    copy_size_ctx(a.ctx, s_C);
    const uint64_t b0 = (uint64_t)tile * tb;
    const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
    const uint64_t v0 = b0 * L;
    const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
    const V *s_val = stage_tile<W>(a.in, v0, nvt, s_raw);
    // the tile's block arrays, as the statistics launch wrote them
    if (tid < nbt) {
        const uint64_t gb = b0 + tid;
        s_min[tid] = (uint32_t)get_le(a.out + lo.off_min + gb * W, W);
        s_rng[tid] = (uint32_t)get_le(a.out + lo.off_range + gb * W, W);
        s_cls[tid] = (lo.flags & kFlagClass) ? a.out[lo.off_class + gb] : (uint8_t)variant;
        s_ne[tid] = (lo.flags & kFlagNe) ? (uint32_t)get_le(a.out + lo.off_ne + gb * ((lo.flags & kFlagNe16) ? 2 : 1),
                                                            (lo.flags & kFlagNe16) ? 2 : 1)
                                         : 0;
    }
    __syncthreads();

    const uint32_t G = kThreads / tb;
    const uint32_t blk = tid / G, g = tid % G;
    const bool live = blk < nbt;
    const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
    const V *bv = s_val + (size_t)blk * L;
    const uint32_t bmin = live ? s_min[blk] : 0;
    const uint64_t B = live ? (uint64_t)s_rng[blk] + 1 : 1;
    const uint32_t beta = bitlen64(B - 1);
    const int cls = live ? s_cls[blk] : 0;
    const int tcls = cls & 7, fam = cls >> 3;
    const uint32_t ne = live ? s_ne[blk] : 0;
    uint32_t nwm = 0, nw = 0;
    if (live) {
        nw = class_words(T, s_C, L, cls, Lb, B, beta, ne, nwm);
        const uint32_t per = 8 / W, cap = (Lb + per - 1) / per;
        nw = nw < cap ? nw : cap;
        nwm = nwm < nw ? nwm : nw;
    }
    if (live && g == 0) s_off[blk] = nw;
    const uint64_t Th = tcls ? (1ull << (beta - tcls)) : 0;
    // excess lists of threshold blocks, in data order (chunked per lane)
    V *s_exc = (V *)s_dyn;
    if (!fixed0) {
        const uint32_t ch = (Lb + G - 1) / G;
        const uint32_t j0 = g * ch < Lb ? g * ch : Lb, j1 = (g + 1) * ch < Lb ? (g + 1) * ch : Lb;
        uint32_t cnt = 0;
        if (tcls)
            for (uint32_t j = j0; j < j1; j++) cnt += ((uint32_t)bv[j] - bmin) >= Th;
        uint32_t pos = group_excl_scan(cnt, G, s_red32);
        if (tcls) {
            V *ex = s_exc + (size_t)blk * L;
            for (uint32_t j = j0; j < j1; j++) {
                const uint32_t d = (uint32_t)bv[j] - bmin;
                if (d >= Th && pos < ne) ex[pos++] = (V)(d - Th);
            }
        }
    }
    __syncthreads();
    uint32_t total;
    const uint32_t my = tid < nbt ? s_off[tid] : 0;
    const uint32_t ex_off = wg_excl_scan(my, s_red32, &total);
    if (tid < nbt) s_off[tid] = ex_off;
    __syncthreads();

    // the tile's place in the payload (written by the scan launch), checked against the bound
    const uint64_t base_off = *(const uint64_t *)(a.out + lo.off_index + 8 * (uint64_t)tile);
    const uint64_t max_off = b0 * ((L + (8 / W) - 1) / (8 / W));
    if (base_off > max_off) {
        if (tid == 0) atomicOr(a.err, 4u);
        return;
    }
    if (live && nw) {
        uint64_t *dst = (uint64_t *)(a.out + lo.off_payload) + base_off + s_off[blk];
        if (tcls == 0) {
            pack_part(T, s_C, B, Lb, fam, nw, g, G, dst,
                      [&](uint32_t j) -> uint64_t { return j < Lb ? (uint64_t)((uint32_t)bv[j] - bmin) : 0; });
        } else {
            pack_part(T, s_C, Th + 1, Lb, fam, nwm, g, G, dst, [&](uint32_t j) -> uint64_t {
                if (j >= Lb) return 0;
                const uint64_t d = (uint32_t)bv[j] - bmin;
                return d < Th ? d : Th;
            });
            const V *ex = s_exc + (size_t)blk * L;
            pack_part(T, s_C, B - Th, ne, fam, nw - nwm, g, G, dst + nwm,
                      [&](uint32_t j) -> uint64_t { return j < ne ? (uint64_t)ex[j] : 0; });
        }
    }
}

// Per-launch preparation: clears the error word and fills the size tables that every
// workgroup copies to LDS.
__global__ void prep_kernel(uint32_t *err, SizeCtx *ctx, DevTables T, uint32_t L) {
    fill_size_ctx(T, L, *ctx);
    if (threadIdx.x == 0) *err = 0;
}

// Workspace: [err u32, 0 u32][SizeCtx padded to kCtxBytes][one u32 word total per tile, padded
// to 8 bytes][one u64 sum per run of kScanTiles tiles].
int launch_compress(const void *d_in, const Layout &lo, int variant, void *d_out, uint64_t *d_out_size,
                    uint64_t *ws, uint64_t ws_words, hipStream_t st) {
    CompressArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    static_assert(sizeof(SizeCtx) <= kCtxBytes, "size tables exceed their workspace slot");
    uint8_t *wsb = (uint8_t *)ws;
    a.err = (uint32_t *)wsb;
    a.ctx = (const SizeCtx *)(wsb + 8);
    a.tile_words = (uint32_t *)(wsb + 8 + kCtxBytes);
    a.in = (const uint8_t *)d_in;
    a.out = (uint8_t *)d_out;
    a.out_size = d_out_size;
    a.lo = lo;
    a.variant = variant;
    prep_kernel<<<1, kThreads, 0, st>>>(a.err, (SizeCtx *)(wsb + 8), a.T, lo.L);
    const uint32_t grid = (uint32_t)(lo.n_tiles ? lo.n_tiles : 1);
    const size_t dyn = (variant == 0 || variant == 8) ? 0 : kTileBytes;
    if (lo.n_tiles) {
        if (lo.w == 1)
            stats_kernel<1><<<grid, kThreads, 0, st>>>(a);
        else if (lo.w == 2)
            stats_kernel<2><<<grid, kThreads, 0, st>>>(a);
        else
            stats_kernel<4><<<grid, kThreads, 0, st>>>(a);
    }
    const uint32_t runs = (uint32_t)((lo.n_tiles + kScanTiles - 1) / kScanTiles);
    uint64_t *sums = (uint64_t *)(wsb + 8 + kCtxBytes + 4 * ((lo.n_tiles + 1) & ~1ull));
    if (runs > 0) scan_sums_kernel<<<runs, kThreads, 0, st>>>(a, sums);
    scan_index_kernel<<<runs > 0 ? runs : 1, kThreads, 0, st>>>(a, sums);
    if (lo.n_tiles) {
        if (lo.w == 1)
            pack_kernel<1><<<grid, kThreads, dyn, st>>>(a);
        else if (lo.w == 2)
            pack_kernel<2><<<grid, kThreads, dyn, st>>>(a);
        else
            pack_kernel<4><<<grid, kThreads, dyn, st>>>(a);
    }
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

}  // namespace pcomp
