// compress.hip -- compression kernels (gfx950).
//
// A call compresses a table of segments (one for a single stream, thousands for a batch),
// each into its own stream, the streams one after another in the caller's order. Tiles are
// numbered across the whole table; segments of one element width form a group whose tiles
// one launch of each width-specialised kernel covers. Five steps, with no communication
// between workgroups inside any launch:
//   1. prep_kernel: clears the error word and fills the size tables of every group.
//   2. stats_kernel<W>, per tile of tile_blocks blocks (at most 16 KiB of input): stage the
//      tile in LDS with 128-bit loads; per block (a group of G = 256 / tile_blocks lanes) min
//      and max by wavefront shuffles, B = max - min + 1 (Sec. 3, Sec. 3.1), and when
//      threshold classes are possible the counts of digits at or above 2^(beta - t); size the
//      candidate classes (basic Sec. 3.1 Eq. (1)-(2), advanced Sec. 3.2 series,
//      threshold/excess split), keep the smallest (ties to the lowest id), write the block's
//      record (min, B - 1, class, words, n_e) to the workspace and the tile's word total.
//   3. scan_sums_kernel + scan_prefix_kernel: exclusive prefix sum of all tile totals.
//   4. place_kernel (one workgroup): every stream's size (its fixed part plus its payload
//      words), their exclusive prefix in the caller's order = where each stream starts, the
//      total, and the headers of streams without values.
//   5. pack_kernel<W>, per tile: the tile's payload offset in its stream is its prefix minus
//      that of the segment's first tile; stage the tile again, read its block records, write
//      its part of the stream's block arrays, compact the excess lists of threshold blocks,
//      and pack: the lanes of a block's group take its words in turn, each word a 64-bit
//      Horner multiply-add over its digits, the first digit at the highest power. The tile
//      writes its index entry; the segment's last tile writes the stream header.
// The stats and pack launches are persistent when the caller gives a grid smaller than the
// tile count: each workgroup then walks the tiles with a stride of the grid.
#include <atomic>

#include "kernels_common.h"

namespace pcomp {

// Parameters of the learned class selector on this device (pcomp_set_model).
__constant__ __align__(16) float c_model[kMlpParams];
static_assert(kMlpW2 % 4 == 0 && kMlpB2 % 4 == 0 && kMlpOut % 4 == 0 && kMlpHid == 4 * kMlpOut,
              "the statistics kernel copies the parameters in quads, W2's quad j of row k to j ^ k");
constexpr uint32_t kFeatWords = 11;  // per block in LDS: 16 16-bit counts, min, max, L_b
constexpr uint32_t kExcBytes = 2048;  // compaction buffer of a tile's excess lists
constexpr uint32_t kAdvTab = kAtlasDirect + 1;  // entries of a full-block word table (bases 0 .. 2^16 + 1)
static_assert(kFeatWords * 4 * kMaxTileBlocks <= kTileBytes, "features must fit in the tile buffer");

struct CompressArgs {
    const SegDesc *segs;        // device table of the batch, or nullptr: the one segment is `one`
    uint32_t xcd_tiles;         // tiles in XCD order (xcd_order): the time-major gathers of nearby
                                // tiles read the same lines of the caller's matrices
    const uint32_t *tile_seg;   // plan index of the segment of every global tile (batch)
    const uint32_t *user_seg;   // plan index of every segment, in the caller's order (batch)
    SegDesc one;
    uint64_t tile_lo, tile_hi;  // global tiles of this launch's width group
    uint8_t *out;               // every segment's stream, one after another in the caller's order
    uint64_t *seg_off;          // [n_segs] byte offset of every segment's stream, plan order (place -> pack)
    uint64_t *seg_offsets;      // the same offsets in the caller's order, for the caller (or nullptr)
    uint64_t *total;            // bytes of all streams (device u64, for the caller)
    uint32_t *tile_words;       // [n_tiles] words of every tile (stats -> scan)
    uint64_t *prefix;           // [n_tiles + 1] exclusive prefix of tile_words, then their sum (scan -> place, pack)
    uint8_t *rec;               // block records of this launch's width group (stats -> pack)
    uint64_t rec_n;             // record slots of the group: its tiles x tile_blocks
    uint64_t n_tiles;
    uint32_t n_segs;
    uint32_t *err;
    const SizeCtx *ctx;         // size tables of this group's block length
    int variant;
    DevTables T;
};

// Segment holding global tile gt (the plan maps every tile to its segment), in scalar
// registers, and its plan index.
__device__ __forceinline__ SegDesc seg_of(const CompressArgs &a, uint64_t gt, uint32_t &j) {
    if (a.segs) {
        j = uni32(a.tile_seg[gt]);
        return uniform_seg(a.segs[j]);
    }
    j = 0;
    return a.one;
}

// Block records in the workspace, structure of arrays per width group: min and B - 1 at the
// element width, then one u32 of class (bits 0-3), words (bits 4-15) and n_e (bits 16-31).
// Block b of global tile gt has slot (gt - tile_lo) * tile_blocks + b.
__host__ __device__ inline uint64_t rec_bytes(uint64_t slots, uint32_t w) {
    return 2 * ((w * slots + 7) & ~7ull) + ((4 * slots + 7) & ~7ull);
}
template <int W>
struct Recs {
    uint8_t *min, *rng;
    uint32_t *meta;
    __device__ Recs(uint8_t *base, uint64_t slots) {
        const uint64_t a = (W * slots + 7) & ~7ull;
        min = base;
        rng = base + a;
        meta = (uint32_t *)(base + 2 * a);
    }
};

__device__ __forceinline__ void write_header(uint8_t *s, const Layout &lo, int variant, uint64_t payload_words) {
    const uint64_t total = lo.off_payload + 8 * payload_words;
    const uint32_t sel = variant == PCOMP_SELECT_EXHAUSTIVE ? 1 : variant == PCOMP_SELECT_LEARNED ? 2 : 0;
    const uint32_t fixed = (lo.flags & kFlagClass) ? 0 : (uint32_t)variant;
    uint64_t *o = (uint64_t *)s;
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
    for (uint64_t b = end_arrays; b < lo.off_payload; b++) s[b] = 0;
}

// Advanced part whose base is outside the tables: the state of word i depends on every
// word before it, so each lane of the group walks the series itself and packs its own
// words i0, i0 + G, ... (G a power of two). Once the walk finds the series' period, whole
// periods before the lane's next word are skipped.
template <typename Get>
__device__ __forceinline__ void pack_adv_slow(const DevTables &T, uint64_t base, uint32_t n, uint32_t nwords,
                                              uint32_t i0, uint32_t G, uint64_t *dst, Get get) {
    const SlowBase sb = slow_base(T, base);
    uint64_t s = 1, rp = 0;  // carried base R'_{i-1} and top part r'_{i-1} of the split value
    uint32_t q = 0, p_prev = 0;
    uint64_t R_prev = 1;
    SeriesCycle cyc;
    for (uint32_t wi = 0; wi < nwords; wi++) {
        if (cyc.found) {
            const uint32_t target = next_own_word(wi, i0, G);
            if (target >= nwords) break;
            if (target - wi >= cyc.lam) {
                const uint32_t c = udiv_small(target - wi, cyc.lam);
                wi += c * cyc.lam;
                q += c * cyc.V;
                // word wi - 1 has the state of the word it replaces: the same p and R
                const uint32_t xq = q - 1;  // q_{wi-1} + p_{wi-1}
                const uint64_t x = xq < n ? get(xq) : 0;
                rp = R_prev <= x ? udiv53(x, R_prev) : 0;
            }
        }
        uint32_t p;
        uint64_t R;
        slow_word_fast(sb, s, p, R);
        const bool mine = ((wi - i0) & (G - 1)) == 0 && wi >= i0;
        uint64_t acc = rp;
        if (mine) {  // digits in increasing order (the absent ones of a last word are 0), then the split value
            const uint32_t real = q < n ? min(p, n - q) : 0;
            for (uint32_t j = 0; j < p; j++) acc = acc * base + (j < real ? get(q + j) : 0);
        }
        const uint64_t x = q + p < n ? get(q + p) : 0;  // the value split between this word and the next
        uint64_t r = x, top = 0;
        if (R <= x) {
            top = udiv53(x, R);
            r = x - top * R;
        }
        if (mine) dst[wi] = acc * R + r;
        rp = top;
        p_prev = p;
        R_prev = R;
        if (q + p >= n) break;
        s = slow_next(sb, R);
        q += p + 1;
        cyc.step(s, q);
    }
}

// Advanced part whose base is outside the tables, packed by a group of at least 8 lanes: the
// group walks the series once into its registers (SlowWindow) and lane i0 packs a run of
// consecutive words with the entries read from the lanes holding them; one division of the
// value split between two words gives r_i (its remainder by R_i) and r'_i (the quotient, on top
// of word i + 1), and the run's first word takes r'_{i-1} from the value before it. Digits are
// read in increasing order. Returns false, with nothing written, when the series has no period
// within the window. Every lane of the group calls it.
template <typename Get>
__device__ __forceinline__ bool pack_adv_window(const DevTables &T, uint64_t base, uint32_t n, uint32_t nwords,
                                                uint32_t i0, uint32_t G, uint64_t *dst, Get get) {
    const SlowBase sb = slow_base(T, base);
    const SlowWindow w = slow_window(sb, n, nwords, G < 64 ? G : 64);
    if (!w.ok) return false;
    const uint32_t run = udiv_small(nwords + G - 1, G);
    const uint32_t w0 = min(i0 * run, nwords), w1 = min(w0 + run, nwords);
    uint32_t j, c;  // entry and periods of word w0 - 1 + k (of word 0 for the first lane)
    window_index(w, w0 ? w0 - 1 : 0, j, c);
    uint64_t rp = 0;  // r'_{i-1}
    for (uint32_t k = 0; k <= run; k++) {  // the same count on every lane (entries are read across lanes)
        const uint64_t E = window_entry(w, j);
        const uint64_t R = E & kWinR;
        const uint32_t p = (uint32_t)((E >> 48) & 3) + 1;
        const uint32_t q = (uint32_t)(E >> 50) + c * w.V;
        const uint32_t i = w0 + k - 1;
        // a value below 2^32 divided by R < 2^48
        auto split = [&](uint64_t x) -> uint64_t {
            const double Rd = (double)R;
            return (uint64_t)floor_div_f64((double)x, Rd, recip_f64(Rd));
        };
        if (k == 0) {
            if (w0 > 0 && w0 < w1) {  // the value split between words w0 - 1 and w0
                const uint64_t x = q + p < n ? get(q + p) : 0;
                rp = R <= x ? split(x) : 0;
            }
        } else if (i < w1) {  // digits in increasing order (the absent ones of a last word are 0)
            uint64_t acc = rp;
            const uint32_t real = q < n ? min(p, n - q) : 0;
            for (uint32_t m = 0; m < p; m++) acc = acc * base + (m < real ? get(q + m) : 0);
            const uint64_t x = q + p < n ? get(q + p) : 0;
            uint64_t r = x, top = 0;
            if (R <= x) {
                top = split(x);
                r = x - top * R;
            }
            dst[i] = acc * R + r;
            rp = top;
        }
        if (k > 0 || w0 > 0) window_next(w, j, c);
    }
    return true;
}

// Digits of a threshold block's excess list (d - T for the values d >= T, in data order)
// read straight from the staged tile, for tiles whose excess lists do not fit the compaction
// buffer. Lane c of the block's group holds in pre[c] the number of excess values before its
// chunk of ch values; the digit of rank m lies in the last chunk c with pre[c] <= m. Ranks
// must be asked in increasing order: consecutive ranks continue the scan inside a chunk, and
// a chunk left behind is replaced by the one holding the rank.
template <typename V>
struct ExcessReader {
    const V *bv;
    const uint16_t *pre;
    uint32_t Lb, ch, G, ne, bmin, Th;
    uint32_t j, jend, r;  // next position, end of its chunk, rank of the next excess value from j
    __device__ __forceinline__ void seek(uint32_t m) {
        uint32_t lo = 0, hi = G - 1;
        while (lo < hi) {
            const uint32_t mid = (lo + hi + 1) >> 1;
            if (pre[mid] <= m)
                lo = mid;
            else
                hi = mid - 1;
        }
        j = lo * ch;
        jend = j + ch < Lb ? j + ch : Lb;
        r = pre[lo];
    }
    __device__ __forceinline__ uint64_t operator()(uint32_t m) {
        if (m >= ne) return 0;
        bool sought = m != r || j >= jend;
        if (sought) seek(m);
        for (;;) {
            for (; j < jend; j++) {
                const uint32_t d = (uint32_t)bv[j] - bmin;
                if (d >= Th && r++ == m) {
                    j++;
                    return d - Th;
                }
            }
            if (sought) return 0;  // not reached: the chunk holding rank m was found from the counts
            seek(m);  // the rest of this chunk held no excess value
            sought = true;
        }
    }
};

// Packs the words of one part of a block (main digits or the excess list); the lanes of
// the block's group call it with their first word index and stride. get(j) returns digit j
// of the part; it is asked only for j < n (the absent digits of a last word are 0).
template <bool Wide, typename Get>
__device__ __forceinline__ void pack_part(const DevTables &T, const SizeCtx &C, uint64_t base, uint32_t n, int fam,
                                          uint32_t nwords, uint32_t i0, uint32_t G, uint64_t *dst, Get get) {
    if (nwords == 0) return;
    const PartBase pb = resolve_base<Wide>(T, C, base);
    // a base outside the tables (u32 data only): the whole group walks its series together
    if (Wide && fam && !pb.D && G >= 8 && pack_adv_window(T, base, n, nwords, i0, G, dst, get)) return;
    if (i0 >= nwords) return;
    if (!fam && (G >= 8 || Wide)) {
        // Sec. 3.1 Eq. (2): word i holds digits i*k .. i*k+k-1, the first at the highest power.
        // Groups of 8 or more lanes take the words in turn (consecutive lanes read nearby digits;
        // such tiles take their blocks kind by kind, so families rarely share a wavefront), and
        // so does u32 data (whose packing keeps its registers).
        for (uint32_t i = i0; i < nwords; i += G) dst[i] = horner_word<Wide>(pb, 0, i * pb.k, pb.k, n, get);
        return;
    }
    if (!Wide && G < 8 && (!fam || pb.D)) {
        // Sec. 3.1 Eq. (2) and the Sec. 3.2 series in one loop, so that groups of both families
        // in a wavefront (tiles of 64 blocks or more) run it together. A basic word i holds
        // digits i k .. i k + k - 1, the first at the highest power (R = 1, no split value); an
        // advanced word i is (r'_{i-1} B^{p_i} + digits) R_i + r_i with its state from the cycle
        // form. Lane i0 packs a run of consecutive words: one division of the value split between
        // two advanced words gives both r_i (its remainder by R_i, at the bottom of word i) and
        // r'_i (the quotient, on top of word i + 1).
        const uint32_t run = udiv_small(nwords + G - 1, G);
        const uint32_t w0 = i0 * run, w1 = w0 + run < nwords ? w0 + run : nwords;
        if (w0 >= w1) return;
        uint32_t q = 0, p = pb.k;
        uint64_t R = 1;
        Magic mR = {0, 0, 0};  // division by 1
        auto word = [&](uint32_t i) {
            if (fam) {
                const AtlasEntry *e = adv_entry(T, *pb.D, i, q);
                p = e->p;
                R = e->R;
                mR = e->mR;
            } else {
                q = i * pb.k;
            }
        };
        uint64_t rp = 0;  // r'_{i-1}
        if (fam && w0 > 0) {  // the value split between words w0 - 1 and w0
            word(w0 - 1);
            rp = div_magic(get(q + p), mR);
        }
        for (uint32_t i = w0; i < w1; i++) {
            word(i);
            // digits are read in increasing order (the excess-list reader relies on it)
            const uint64_t acc = horner_word<Wide>(pb, (uint32_t)rp, q, p, n, get);
            const uint64_t x = fam && q + p < n ? get(q + p) : 0;
            const uint64_t qx = div_magic(x, mR);
            dst[i] = acc * R + (x - qx * R);
            rp = qx;
        }
        return;
    }
    if (pb.D) {
        // groups of 8 or more lanes and u32 data: the Sec. 3.2 series alone (the same runs, with
        // fewer registers held)
        const BaseDesc &D = *pb.D;
        const uint32_t run = udiv_small(nwords + G - 1, G);
        const uint32_t w0 = i0 * run, w1 = w0 + run < nwords ? w0 + run : nwords;
        if (w0 >= w1) return;
        uint32_t q;
        const AtlasEntry *e = adv_entry(T, D, w0, q);
        uint64_t rp = 0;  // r'_{i-1}
        if (w0 > 0) {
            uint32_t qp;
            const AtlasEntry *ep = adv_entry(T, D, w0 - 1, qp);
            rp = div_magic(get(q - 1), ep->mR);
        }
        for (uint32_t i = w0; i < w1; i++) {
            if (i > w0) e = adv_entry(T, D, i, q);
            const uint64_t acc = horner_word<Wide>(pb, (uint32_t)rp, q, e->p, n, get);
            const uint64_t x = q + e->p < n ? get(q + e->p) : 0;
            const uint64_t qx = div_magic(x, e->mR);
            dst[i] = acc * e->R + (x - qx * e->R);
            rp = qx;
        }
        return;
    }
    // base outside the tables (u32 data only)
    if (Wide) pack_adv_slow(T, base, n, nwords, i0, G, dst, get);
}

// Stages a tile of a time-major segment: value v0 + j of the stream is gathered from the
// element of the caller's matrices it stands for (one load per value).
template <int W>
__device__ __forceinline__ const typename Elem<W>::T *stage_tile_tm(const SegDesc &sd, uint64_t v0, uint32_t nvt,
                                                                     uint4 *s_raw) {
    typedef typename Elem<W>::T V;
    V *dst = (V *)s_raw;
    const __attribute__((address_space(1))) V *src = (const __attribute__((address_space(1))) V *)sd.data;
    TmCursor cur(v0 + threadIdx.x, sd.rows, sd.cols);
    for (uint32_t j = threadIdx.x; j < nvt; j += kThreads) {
        dst[j] = src[cur.index()];
        cur.step();
    }
    return dst;
}

// Staging of a tile's input with every load in flight at once: the 16-byte chunks that lie
// inside the segment go through buffer loads into registers (a chunk that is not loaded gets an
// offset past the buffer's range, which reads zeros without touching memory, so the loads are
// unconditional; buffer loads are counted apart from LDS operations), and are then stored to
// LDS; chunks at the segment's edges (and a 1025th chunk of an unaligned full tile) are copied
// element by element.
constexpr uint32_t kStageChunks = kTileBytes / 16 / kThreads;
static_assert(kStageChunks == 4, "four chunks per thread");
struct Staged {
    uint4 c0, c1, c2, c3;  // separate members, not an array: they stay in registers
};
struct TileRef {
    const uint8_t *gbase;  // 16-byte aligned address at or below the tile's first value
    uint32_t head, span;   // the tile's bytes are [head, span) from gbase
    const uint8_t *lo, *hi;  // the segment's bytes
};

template <int W>
__device__ __forceinline__ TileRef tile_ref(const SegDesc &sd, uint64_t v0, uint32_t nvt) {
    TileRef t;
    const uintptr_t addr = (uintptr_t)(sd.data + v0 * W);
    t.head = (uint32_t)(addr & 15);
    t.gbase = (const uint8_t *)(addr - t.head);
    t.span = t.head + nvt * W;
    t.lo = sd.data;
    t.hi = sd.data + sd.lo.n * W;
    return t;
}

__device__ __forceinline__ bool chunk_inside(const TileRef &t, uint32_t c) {
    const uint8_t *p = t.gbase + (c << 4);
    return p >= t.lo && p + 16 <= t.hi;
}

__device__ __forceinline__ void tile_fetch(const TileRef &t, Staged &r) {
    const uint32_t nchunks = (t.span + 15) >> 4;
    const auto rsrc = __builtin_amdgcn_make_buffer_rsrc((void *)t.gbase, (short)0, (int)(nchunks << 4), 0x00020000);
    auto get = [&](uint32_t k) -> uint4 {
        const uint32_t c = threadIdx.x + k * kThreads;
        const bool ok = c < nchunks && chunk_inside(t, c);
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc, ok ? (int)(c << 4) : (int)0x40000000, 0, 0);
        return make_uint4(v[0], v[1], v[2], v[3]);
    };
    r.c0 = get(0);
    r.c1 = get(1);
    r.c2 = get(2);
    r.c3 = get(3);
}

template <int W>
__device__ __forceinline__ const typename Elem<W>::T *tile_commit(const TileRef &t, const Staged &r, uint4 *s_raw) {
    typedef typename Elem<W>::T V;
    uint8_t *s_bytes = (uint8_t *)s_raw;
    const uint32_t nchunks = (t.span + 15) >> 4;
    auto copy_elems = [&](uint32_t c) {
        const uint32_t cb = c << 4;
        const uint32_t e0 = cb > t.head ? cb : t.head, e1 = cb + 16 < t.span ? cb + 16 : t.span;
        for (uint32_t b = e0; b < e1; b += W)
            *(V *)(s_bytes + b) = *(const __attribute__((address_space(1))) V *)(t.gbase + b);
    };
    auto put = [&](uint32_t k, const uint4 &v) {
        const uint32_t c = threadIdx.x + k * kThreads;
        if (c < nchunks) {
            if (chunk_inside(t, c))
                s_raw[c] = v;
            else
                copy_elems(c);
        }
    };
    put(0, r.c0);
    put(1, r.c1);
    put(2, r.c2);
    put(3, r.c3);
    if (threadIdx.x + kStageChunks * kThreads < nchunks) copy_elems(threadIdx.x + kStageChunks * kThreads);
    return (const V *)(s_bytes + t.head);
}

__device__ __forceinline__ void copy_size_ctx(const SizeCtx *g, SizeCtx &s) {
    static_assert(sizeof(SizeCtx) / 4 <= kThreads, "one word per thread");
    if (threadIdx.x < sizeof(SizeCtx) / 4) ((uint32_t *)&s)[threadIdx.x] = ((const uint32_t *)g)[threadIdx.x];
}

// ---- launch 2: block statistics, class choice, block arrays, tile totals ----------------
// kPair (tiles of 128 blocks, not persistent): a workgroup takes two consecutive tiles, staged
// side by side in dynamic LDS, and every lane one block (lanes 0-127 the first tile, 128-255
// the second), so no block's work is split between lanes.
constexpr uint32_t kPairBlocks = kThreads / 2;
// 16-byte chunks that a staged tile of tile_bytes may cover (its first value need not be aligned)
__host__ __device__ inline uint32_t pair_region(uint32_t tile_bytes) { return (tile_bytes + 15) / 16 + 1; }
// kLearn: 0 = no learned selector; 1 = learned, the lanes of a block share its network (tiles of
// at most kMaxTileBlocks / 4 blocks); 2 = learned, one thread scores a block (larger tiles);
// 3 = as 1 for tiles of at most kL3Blocks blocks, with the parameters, features and hidden units
// in the tile's LDS once its values are read, so that the learned instance keeps the LDS and
// the occupancy (8 wavefronts per SIMD) of the others.
constexpr uint32_t kL3Blocks = 16;
constexpr uint32_t kL3H = 0, kL3X = kL3H + kL3Blocks * kMlpHid, kL3W2 = (kL3X + kL3Blocks * kMlpIn + 3) & ~3u,
                   kL3Model = kL3W2 + kMlpOut * kMlpHid;  // offsets in floats
static_assert(4 * (kL3Model + kMlpW2 + kMlpOut) <= kTileBytes, "the selector's LDS fits the tile buffer");
template <int W, bool kPersist, int kLearn, bool kPair = false>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(kLearn == 3 && !kPersist ? (W == 4 ? 6 : 8) : 1))) void stats_kernel(CompressArgs a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_one[kPair ? 1 : kTileBytes / 16 + 1];
    extern __shared__ uint4 s_pair[];  // kPair: two regions of pair_region(tile bytes) chunks
    uint4 *const s_raw = kPair ? s_pair : s_one;
    __shared__ uint32_t s_nw[kMaxTileBlocks];
    __shared__ uint8_t s_pred[kMaxTileBlocks];
    __shared__ uint64_t s_red64[kThreads / 64];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ SizeCtx s_C;
    // the selector's parameters, per workgroup: W1, b1 and b2 (at kMlpW2) in s_model; W2 in s_w2s,
    // row k holding W2[k][j] at column j ^ 4k, so that the 16 lanes that score the 16 classes read
    // their rows' quads j .. j + 3 from 16 different bank groups
    __shared__ __align__(16) float s_model[kLearn == 1 || kLearn == 2 ? kMlpW2 + kMlpOut : 4];
    __shared__ __align__(16) float s_w2s[kLearn == 1 || kLearn == 2 ? kMlpOut * kMlpHid : 4];
    // the features of the tile's blocks (lane-shared scoring)
    __shared__ float s_x[kLearn == 1 ? (kMaxTileBlocks / 4) * kMlpIn : 1];

    const DevTables &T = a.T;
    const uint32_t tid = threadIdx.x;
    const int variant = a.variant;
    const bool fixed0 = (variant == 0 || variant == 8);
    const bool learned = kLearn != 0;  // the variant is PCOMP_SELECT_LEARNED
    copy_size_ctx(a.ctx, s_C);
    // lanes read different weights at once: LDS serves those reads without the constant cache's
    // serialisation. Copied in 16-byte quads (W2 moves quad by quad: quad j of row k to j ^ k);
    // read after the first tile's barrier. One tile per workgroup: copied while that tile's
    // loads are in flight.
    float *const m_model = kLearn == 3 ? (float *)s_raw + kL3Model : s_model;
    float *const m_w2s = kLearn == 3 ? (float *)s_raw + kL3W2 : s_w2s;
    float *const m_x = kLearn == 3 ? (float *)s_raw + kL3X : s_x;
    auto fill_model = [&]() {
        constexpr uint32_t kQ1 = (kMlpW2 + kMlpOut) / 4, kQ2 = kMlpOut * kMlpHid / 4, kRow = kMlpHid / 4;
        static_assert(kQ1 + kQ2 <= 3 * kThreads, "three quads per thread");
        const float4 *src = (const float4 *)c_model;
        // quad i of the LDS copy: W1, b1, then b2 (which follows W2 in the parameters), then W2
        // with the quads of row k rotated by k
        auto quad = [&](uint32_t i) -> float4 {
            if (i < kQ1) return src[i < kMlpW2 / 4 ? i : i + kQ2];
            const uint32_t o = i - kQ1, k = o / kRow, jq = (o % kRow) ^ k;
            return src[kMlpW2 / 4 + k * kRow + jq];
        };
        auto put = [&](uint32_t i, float4 v) {
            if (i < kQ1)
                ((float4 *)m_model)[i] = v;
            else if (i < kQ1 + kQ2)
                ((float4 *)m_w2s)[i - kQ1] = v;
        };
        // all three loads are in flight before the first store
        const uint32_t i0 = tid, i1 = tid + kThreads, i2 = tid + 2 * kThreads;
        const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 v0 = quad(i0), v1 = quad(i1), v2 = i2 < kQ1 + kQ2 ? quad(i2) : z;
        put(i0, v0);
        put(i1, v1);
        put(i2, v2);
    };
    constexpr bool kModelAhead = kLearn == 1 || kLearn == 2;  // parameters in LDS of their own
    if (kModelAhead && kPersist) fill_model();
    const uint32_t span = kPair ? 2 : 1;
    const uint32_t wg = a.xcd_tiles ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    for (uint64_t gt0 = a.tile_lo + span * wg; gt0 < a.tile_hi; gt0 = kPersist ? gt0 + gridDim.x : a.tile_hi) {
        const uint32_t half = kPair ? tid / kPairBlocks : 0;
        const uint64_t gt = gt0 + half;
        const bool valid = gt < a.tile_hi;
        uint32_t sj;
        const SegDesc sd = seg_of(a, valid ? gt : gt0, sj);
        const Layout &lo = sd.lo;
        const uint32_t L = lo.L, tb = lo.tile_blocks;
        const uint64_t b0 = (gt - sd.tile0) * tb;
        const uint32_t nbt = valid ? (uint32_t)min((uint64_t)tb, lo.n_blocks - b0) : 0;
        const uint64_t v0 = b0 * L;
        const uint32_t nvt = valid ? (uint32_t)min((uint64_t)nbt * L, lo.n - v0) : 0;
        // one workgroup per tile (or pair): all of its loads at once (persistent grids keep fewer
        // registers)
        const V *s_val;
        if (kPair) {
            // the whole workgroup stages both tiles (the second may lie in another segment)
            const uint32_t region = pair_region(tb * L * W);
            const V *first[2] = {nullptr, nullptr};
            TileRef tr[2];
            Staged stg[2];
            bool have[2];
#pragma unroll
            for (uint32_t h = 0; h < 2; h++) {
                const uint64_t gh = gt0 + h;
                have[h] = gh < a.tile_hi;
                uint32_t jh;
                const SegDesc sh = seg_of(a, have[h] ? gh : gt0, jh);
                const uint64_t vh = (gh - sh.tile0) * sh.lo.tile_blocks * sh.lo.L;
                const uint32_t nh = have[h] ? (uint32_t)min((uint64_t)sh.lo.tile_blocks * sh.lo.L, sh.lo.n - vh) : 0;
                if (sh.rows) {
                    first[h] = have[h] ? stage_tile_tm<W>(sh, vh, nh, s_raw + h * region) : nullptr;
                    have[h] = false;  // staged already
                } else {
                    tr[h] = tile_ref<W>(sh, vh, nh);
                    if (have[h]) tile_fetch(tr[h], stg[h]);
                }
            }
#pragma unroll
            for (uint32_t h = 0; h < 2; h++)
                if (have[h]) first[h] = tile_commit<W>(tr[h], stg[h], s_raw + h * region);
            s_val = half ? first[1] : first[0];
        } else if (sd.rows) {
            if (kModelAhead && !kPersist) fill_model();
            s_val = stage_tile_tm<W>(sd, v0, nvt, s_raw);
        } else if (kPersist) {
            s_val = stage_tile<W>(sd.data, v0, nvt, s_raw);
        } else {
            const TileRef tr = tile_ref<W>(sd, v0, nvt);
            Staged stg;
            tile_fetch(tr, stg);
            if (kModelAhead) fill_model();
            s_val = tile_commit<W>(tr, stg, s_raw);
        }
        __syncthreads();

        // per block: min / max (B = v_max - v_min + 1) and excess counts
        const uint32_t G = kPair ? 1 : kThreads / tb;
        const uint32_t blk = kPair ? tid % kPairBlocks : tid / G, g = kPair ? 0 : tid % G;
        const bool live = blk < nbt;
        const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
        const auto *bv = lds_ptr(s_val + (size_t)blk * L);
        uint32_t vmin = 0xFFFFFFFFu, vmax = 0;
        {
            uint32_t j = g;
            for (; j + 3 * G < Lb; j += 4 * G) {  // four LDS reads in flight at a time
                const uint32_t v0 = bv[j], v1 = bv[j + G], v2 = bv[j + 2 * G], v3 = bv[j + 3 * G];
                vmin = min(vmin, min(min(v0, v1), min(v2, v3)));
                vmax = max(vmax, max(max(v0, v1), max(v2, v3)));
            }
            for (; j < Lb; j += G) {
                const uint32_t v = bv[j];
                vmin = v < vmin ? v : vmin;
                vmax = v > vmax ? v : vmax;
            }
        }
        vmin = group_reduce(vmin, G, MinOp(), s_red32);
        vmax = group_reduce(vmax, G, MaxOp(), s_red32);
        const uint64_t B = live ? (uint64_t)vmax - vmin + 1 : 1;
        const uint32_t beta = bitlen64(B - 1);
        // exhaustive search of a full block: both family sizes of classes 0 and 8 come from one
        // table entry, loaded here so that the histogram below covers its latency
        const bool full_tab = variant == PCOMP_SELECT_EXHAUSTIVE && live && B > 1 && Lb == L && s_C.fullW &&
                              B <= kAtlasDirect;
        const uint32_t fw = full_tab ? ((const __attribute__((address_space(1))) uint32_t *)s_C.fullW)[B] : 0;
        // bin b = beta - bitlen(d): digits in octave b below the top; n_e(t) = bins 0 .. t-1
        uint32_t ne_t[8];
        ne_t[0] = 0;
        Hist16 hist;
        if (!fixed0) {
            // bin b of digit d = v - v_min: b = beta - bitlen(d) = 4-bit counter min(b, 15) of c4,
            // moved to 8-bit counters of the even and odd bins (ev8, od8) after at most 15
            // values; at most 64 values per lane, so 8 bits suffice. Bins past 7 matter only to
            // the learned selector. Below 2^31, bitlen(d) = 31 - clz(2d + 1), and 2d + 1 =
            // 2v + c1 (mod 2^32) never vanishes; u32 values take clz(d), 32 for d = 0.
            const uint32_t c1 = 1u - 2u * vmin;
            uint32_t kofs = 4u * beta - (W == 4 ? 128u : 124u);  // shift = 4 clz + kofs = 4b
            asm volatile("" : "+v"(kofs));  // kept whole: one multiply-add per value, not two adds
            uint64_t c4 = 0, ev8 = 0, od8 = 0;
            auto count = [&](uint32_t v) {
                const uint32_t z = W == 4 ? (uint32_t)__clz((int)(v - vmin)) : (uint32_t)__builtin_clz(2u * v + c1);
                c4 += 1ull << min(4u * z + kofs, 60u);
            };
            uint32_t j = g;
            while (j < Lb) {
                uint32_t q = 0;
                for (; q < 3 && j + 3 * G < Lb; q++, j += 4 * G) {  // four LDS reads in flight at a time
                    const uint32_t v0 = bv[j], v1 = bv[j + G], v2 = bv[j + 2 * G], v3 = bv[j + 3 * G];
                    count(v0);
                    count(v1);
                    count(v2);
                    count(v3);
                }
                if (q < 3)  // fewer than four values left: at most 11 in this round
                    for (; j < Lb; j += G) count(bv[j]);
                ev8 += c4 & 0x0F0F0F0F0F0F0F0Full;
                od8 += (c4 >> 4) & 0x0F0F0F0F0F0F0F0Full;
                c4 = 0;
            }
            hist_widen_eo(ev8, od8, hist);
            hist.w[0] = group_reduce(hist.w[0], G, AddOp(), s_red64);
            hist.w[1] = group_reduce(hist.w[1], G, AddOp(), s_red64);
            if (learned) {
                hist.w[2] = group_reduce(hist.w[2], G, AddOp(), s_red64);
                hist.w[3] = group_reduce(hist.w[3], G, AddOp(), s_red64);
            }
#pragma unroll
            for (int t = 1; t < 8; t++) ne_t[t] = ne_t[t - 1] + hist_bin(hist, t - 1);
        } else {
#pragma unroll
            for (int t = 1; t < 8; t++) ne_t[t] = 0;
        }

        // learned selector. With at least 4 lanes per block (tile_blocks <= 64) the block's lanes
        // share its features (one division each) and hidden units through LDS, and then every lane
        // of the workgroup scores one class of one block (16 lanes a block, the tile's values no
        // longer needed); otherwise the features go through LDS and one thread per block scores it.
        // Both keep every sum's order, so the scores are the same bits.
        int pred = 0;
        if (kLearn == 1 || kLearn == 3) {
            if (kLearn == 3) {  // the tile's values are read: its LDS takes the selector's data
                __syncthreads();
                fill_model();
            }
            if (live)
                for (uint32_t f = g; f < (uint32_t)kMlpIn; f += G)
                    m_x[blk * kMlpIn + f] = block_feature(f, hist.w, Lb, vmin, vmax);
            __syncthreads();
            // hidden unit j of block b at b * kMlpHid + (j ^ 4 (b mod 4)): the four blocks scored
            // by one wave read their quads from four bank groups
            float *s_h = (float *)s_raw + kL3H;
            if (live) {
                const float *xb = m_x + blk * kMlpIn;
                for (uint32_t j = g; j < (uint32_t)kMlpHid; j += G) {
                    float acc = m_model[kMlpB1 + j];
#pragma unroll
                    for (int i = 0; i < kMlpIn; i++) acc = __builtin_fmaf(m_model[kMlpW1 + j * kMlpIn + i], xb[i], acc);
                    s_h[blk * kMlpHid + (j ^ ((blk & 3) << 2))] = acc > 0.0f ? acc : 0.0f;
                }
            }
            __syncthreads();
            for (uint32_t q = tid; q < nbt * kMlpOut; q += kThreads) {  // 16-lane groups stay whole
                const uint32_t sb = q / kMlpOut, k = q % kMlpOut;
                const float4 *hq = (const float4 *)(s_h + sb * kMlpHid);
                const float4 *wq = (const float4 *)(m_w2s + k * kMlpHid);
                float acc = m_model[kMlpW2 + k];  // b2[k]
#pragma unroll 4
                for (uint32_t jq = 0; jq < (uint32_t)kMlpHid / 4; jq++) {
                    const float4 h = hq[jq ^ (sb & 3)], w = wq[jq ^ k];
                    acc = __builtin_fmaf(w.x, h.x, acc);
                    acc = __builtin_fmaf(w.y, h.y, acc);
                    acc = __builtin_fmaf(w.z, h.z, acc);
                    acc = __builtin_fmaf(w.w, h.w, acc);
                }
                uint32_t u = __float_as_uint(acc == 0.0f ? 0.0f : acc);
                u = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
                // (order-preserving score bits, 15 - class): the largest is the first top score
                uint64_t best = ((uint64_t)u << 32) | (uint64_t)(15 - k);
                best = group_reduce(best, kMlpOut, MaxOp(), s_red64);
                if (k == 0) s_pred[sb] = (uint8_t)(15 - (int)(best & 0xFF));
            }
            __syncthreads();
            pred = live ? s_pred[blk] : 0;
        } else if (kLearn == 2) {
            __syncthreads();
            uint32_t *s_feat = (uint32_t *)s_raw;  // kFeatWords per block
            if (live && g == 0) {
                uint32_t *f = s_feat + blk * kFeatWords;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    f[2 * q] = (uint32_t)hist.w[q];
                    f[2 * q + 1] = (uint32_t)(hist.w[q] >> 32);
                }
                f[8] = vmin;
                f[9] = vmax;
                f[10] = Lb;
            }
            __syncthreads();
            if (tid < nbt) {
                const uint32_t *f = s_feat + tid * kFeatWords;
                uint32_t H[16];
#pragma unroll
                for (int b = 0; b < 16; b++) H[b] = (f[b >> 1] >> (16 * (b & 1))) & 0xFFFF;
                float x[kMlpIn], sc[kMlpOut];
                block_features(H, f[10], f[8], f[9], x);
                mlp_scores(
                    [&](int i) {
                        if (i < kMlpW2) return s_model[i];
                        if (i >= kMlpB2) return s_model[i - kMlpOut * kMlpHid];
                        const int k = (i - kMlpW2) / kMlpHid, j = (i - kMlpW2) % kMlpHid;
                        return s_w2s[k * kMlpHid + (j ^ (k << 2))];
                    },
                    x, sc);
                s_pred[tid] = (uint8_t)argmax16(sc);
            }
            __syncthreads();
            pred = live ? s_pred[blk] : 0;
        }

        // class choice: lanes of the group split the candidates; argmin, ties to the lowest id.
        // Exhaustive search sizes classes 0 and 8 on every lane first; a threshold class is then
        // sized only if its main part (plus one word for a non-empty excess list) could still
        // beat the best (words, id) key seen by the lane, so the classes it skips cannot win.
        uint64_t key = ~0ull;
        if (live && variant == PCOMP_SELECT_EXHAUSTIVE) {
            // classes 0 and 8: one load of the full-block table, else k(B) once for both families
            uint32_t w0 = 0, w8 = 0;
            if (full_tab) {
                w0 = fw & 0xFFFFu;
                w8 = fw >> 16;
            } else if (B > 1) {
                const uint32_t kb = k_fast(s_C, B);
                w0 = udiv_small(Lb + kb - 1, kb);
                if (W == 4 && kLearn == 0 && G >= 8 && Lb > kb && atlas_index(B) < 0) {
                    // a base outside the tables: the group walks its series together
                    const uint32_t width = G < 64 ? G : 64;
                    const SlowWindow sw = slow_window(slow_base(T, B), Lb, 0xFFFFFFFFu, width);
                    if (sw.ok) w8 = window_words(sw, Lb);
                }
                if (!w8) w8 = adv_words_k<(W == 4)>(T, s_C, Lb, B, kb, L);
            }
            // keys (words << 8 | id) in 32 bits: a block of at most 2^16 values has fewer than 2^24 words
            uint32_t k32 = w0 << 8;
            if (beta >= 1) k32 = min(k32, (w8 << 8) | 8u);
            // lanes split the thresholds t (unrolled, so that n_e(t) is read without an index); each
            // sizes both families of its t, which share the excess base B - T and its digits per
            // word. Every t <= beta has a non-empty excess list (the maximum digit B - 1 >= T), so
            // a class whose main part plus one word cannot beat the key is skipped, and so is the
            // advanced one whose main part plus the least possible excess words cannot.
#pragma unroll
            for (int t = 1; t < 8; t++) {
                if ((uint32_t)(t - 1) % G != g || t > (int)beta) continue;
                const uint32_t net = ne_t[t];
                const uint32_t m0 = main_words<(W == 4)>(T, s_C, L, 0, t, Lb, beta);
                const uint32_t m1 = main_words<(W == 4)>(T, s_C, L, 1, t, Lb, beta);
                const bool try0 = (((m0 + 1) << 8) | (uint32_t)t) < k32;
                bool try1 = (((m1 + 1) << 8) | (uint32_t)(8 + t)) < k32;
                if (!try0 && !try1) continue;
                const uint64_t Be = B - (1ull << (beta - t));
                uint32_t e0 = 0, e1 = 0;
                if (Be > 1) {
                    const uint32_t ke = k_fast(s_C, Be);
                    e0 = udiv_small(net + ke - 1, ke);
                    if (try1) {
                        const uint32_t lo1 = net <= ke ? 1 : udiv_small(net + 1 + ke, ke + 1);  // every word takes <= k + 1
                        try1 = (((m1 + lo1) << 8) | (uint32_t)(8 + t)) < k32;
                        if (try1) e1 = adv_words_k<(W == 4)>(T, s_C, net, Be, ke, L);
                    }
                }
                if (try0) k32 = min(k32, ((m0 + e0) << 8) | (uint32_t)t);
                if (try1) k32 = min(k32, ((m1 + e1) << 8) | (uint32_t)(8 + t));
            }
            key = k32;
        } else if (live && fixed0) {  // one class: the first lane of the group sizes it
            if (g == 0) {
                uint32_t nwm;
                key = ((uint64_t)class_words<(W == 4)>(T, s_C, L, variant, Lb, B, beta, 0, nwm) << 8) |
                      (uint64_t)variant;
            }
        } else if (live) {
            for (int c = (int)g; c < 16; c += (int)G) {
                const bool cand = c == 0 || c == variant || (learned && c == pred);
                const int t = c & 7;
                if (!cand || t > (int)beta) continue;
                uint32_t nwm, net = 0;
#pragma unroll
                for (int tt = 1; tt < 8; tt++) net = (t == tt) ? ne_t[tt] : net;  // no dynamic register index
                const uint32_t nw = class_words<(W == 4)>(T, s_C, L, c, Lb, B, beta, net, nwm);
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
            if (!kPair) s_nw[blk] = nw;
            const uint64_t r = (gt - a.tile_lo) * tb + blk;
            const Recs<W> rc(a.rec, a.rec_n);
            ((V *)rc.min)[r] = (V)vmin;
            ((V *)rc.rng)[r] = (V)(B - 1);
            rc.meta[r] = (uint32_t)cls | (nw << 4) | (ne << 16);
        }
        if (kPair) {  // each half's tile total
            const uint32_t total = group_reduce(live ? nw : 0u, kPairBlocks, AddOp(), s_red32);
            if (valid && blk == 0) a.tile_words[gt] = total;
            __syncthreads();  // LDS is reused by the next pair
        } else {
            __syncthreads();
            uint32_t total;
            wg_excl_scan(tid < nbt ? s_nw[tid] : 0, s_red32, &total);
            if (tid == 0) a.tile_words[gt] = total;
        }
    }
}

// ---- launch 3: exclusive prefix of the tile totals ----------------------------------------
// Two small launches: every workgroup sums a run of kScanTiles tile totals; then every
// workgroup adds the sums of the runs before its own and scans its run.
constexpr uint32_t kScanPer = 32;                      // tile totals per thread
constexpr uint32_t kScanTiles = kScanPer * kThreads;  // tile totals per workgroup

__global__ __launch_bounds__(kThreads) void scan_sums_kernel(CompressArgs a, uint64_t *sums) {
    __shared__ uint32_t s_red32[kThreads / 64];
    const uint64_t nt = a.n_tiles;
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

__global__ __launch_bounds__(kThreads) void scan_prefix_kernel(CompressArgs a, const uint64_t *sums) {
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint64_t s_red64[kThreads / 64];
    const uint64_t nt = a.n_tiles;
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
#pragma unroll
    for (uint32_t m = 0; m < kScanPer; m++) {
        if (t0 + m < nt) a.prefix[t0 + m] = run;
        run += v[m];
        if (t0 + m + 1 == nt) a.prefix[nt] = run;  // the sum of every tile
    }
}

// ---- launch 4: placement of the streams --------------------------------------------------
// One workgroup. Stream sizes (fixed part + 8 x payload words, from the tile prefix), their
// exclusive prefix in the caller's order, the total, and the header of every stream without
// values (no tile of it runs in the packing launch).
__global__ __launch_bounds__(kThreads) void place_kernel(CompressArgs a) {
    __shared__ uint64_t s_red64[kThreads / 64];
    const uint32_t n = a.n_segs;
    const uint32_t per = (n + kThreads - 1) / kThreads;
    const uint32_t u0 = min(n, threadIdx.x * per), u1 = min(n, u0 + per);
    auto seg = [&](uint32_t u, uint32_t &j) -> SegDesc {
        j = a.segs ? a.user_seg[u] : 0;
        return a.segs ? a.segs[j] : a.one;
    };
    auto size_of = [&](const SegDesc &sd) -> uint64_t {
        const uint64_t pw = sd.lo.n_tiles ? a.prefix[sd.tile0 + sd.lo.n_tiles] - a.prefix[sd.tile0] : 0;
        return sd.lo.off_payload + 8 * pw;
    };
    uint64_t sum = 0;
    for (uint32_t u = u0; u < u1; u++) {
        uint32_t j;
        sum += size_of(seg(u, j));
    }
    uint64_t tot;
    uint64_t run = wg_excl_scan64(sum, s_red64, &tot);
    for (uint32_t u = u0; u < u1; u++) {
        uint32_t j;
        const SegDesc sd = seg(u, j);
        a.seg_off[j] = run;
        if (a.seg_offsets) a.seg_offsets[u] = run;
        if (sd.lo.n_tiles == 0) write_header(a.out + run, sd.lo, a.variant, 0);
        run += size_of(sd);
    }
    if (threadIdx.x == 0) *a.total = tot;
}

// ---- launch 4: packing ----------------------------------------------------------------
// u32 packing keeps six wavefronts per SIMD (at most 80 vector registers).
template <int W, bool kPersist>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(W == 4 && !kPersist ? 6 : 1))) void pack_kernel(
    CompressArgs a) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    __shared__ uint16_t s_cpre[kThreads];  // threshold blocks: excess values before each lane's chunk
    __shared__ uint4 s_exc[kExcBytes / 16];  // compacted excess lists of the tile, when they fit
    __shared__ uint16_t s_exoff[kMaxTileBlocks];
    __shared__ V s_min[kMaxTileBlocks], s_rng[kMaxTileBlocks];  // at the element width
    __shared__ uint16_t s_ne[kMaxTileBlocks], s_off[kMaxTileBlocks + 1];  // a tile holds at most 2304 words
    __shared__ uint8_t s_cls[kMaxTileBlocks];
    __shared__ uint8_t s_perm[kMaxTileBlocks];  // block packed by lane group p
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ uint64_t s_red64[kThreads / 64];
    __shared__ SizeCtx s_C;

    const DevTables &T = a.T;
    const uint32_t tid = threadIdx.x;
    const int variant = a.variant;
    const bool fixed0 = (variant == 0 || variant == 8);
    copy_size_ctx(a.ctx, s_C);
    __syncthreads();  // the size tables are read before the first barrier of a tile
    const uint32_t wg = a.xcd_tiles ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    for (uint64_t gt = a.tile_lo + wg; gt < a.tile_hi; gt = kPersist ? gt + gridDim.x : a.tile_hi) {
        uint32_t sj;
        const SegDesc sd = seg_of(a, gt, sj);
        const Layout &lo = sd.lo;
        const uint32_t L = lo.L, tb = lo.tile_blocks;
        uint8_t *so = a.out + uni64(a.seg_off[sj]);
        const uint64_t tile = gt - sd.tile0;
        const uint64_t b0 = tile * tb;
        const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
        const uint64_t v0 = b0 * L;
        const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
        // the tile's place in its stream's payload, fetched early
        const uint64_t base_off = a.prefix[gt] - a.prefix[sd.tile0];
        // one workgroup per tile: the tile's input is in flight while the block arrays are read
        // (persistent grids stage it first and keep fewer registers)
        const TileRef tr = tile_ref<W>(sd, v0, nvt);
        Staged stg;
        const V *s_val = nullptr;
        const bool tm = sd.rows != 0;
        if (tm)
            s_val = stage_tile_tm<W>(sd, v0, nvt, s_raw);
        else if (kPersist)
            s_val = stage_tile<W>(sd.data, v0, nvt, s_raw);
        else
            tile_fetch(tr, stg);
        // the tile's block records, as the statistics launch wrote them (class, words and n_e
        // included), go to the stream's block arrays. One scan of packed fields gives each block
        // its word offset, its place among the tile's excess values and its lane group (basic
        // blocks first, then advanced ones, so that wavefronts mostly run one family's code).
        uint64_t key = 0;
        const bool fine = tb <= 32;
        const uint32_t cbits = fine ? 6 : 9;
        uint32_t kcat = 0;
        if (tid < nbt) {
            const uint64_t gb = b0 + tid;
            const uint64_t r = (gt - a.tile_lo) * tb + tid;
            const Recs<W> rc(a.rec, a.rec_n);
            const uint32_t mn = ((const V *)rc.min)[r];
            const uint32_t rg = ((const V *)rc.rng)[r];
            const uint32_t meta = rc.meta[r];
            const int c = (int)(meta & 15);
            const uint32_t nw = (meta >> 4) & 0xFFF, ne = meta >> 16;
            s_min[tid] = (V)mn;
            s_rng[tid] = (V)rg;
            s_cls[tid] = (uint8_t)c;
            s_ne[tid] = (uint16_t)ne;
            put_le(so + lo.off_min + gb * W, mn, W);
            put_le(so + lo.off_range + gb * W, rg, W);
            if (lo.flags & kFlagClass) so[lo.off_class + gb] = (uint8_t)c;
            if (lo.flags & kFlagNe)
                put_le(so + lo.off_ne + gb * ((lo.flags & kFlagNe16) ? 2 : 1), ne, (lo.flags & kFlagNe16) ? 2 : 1);
            // words (16 bits: at most one per value, 2^14 in a tile), excess values (15), then the
            // blocks of each kind: for tiles of at most 32 blocks basic, basic threshold,
            // advanced and advanced threshold (6 bits each), else basic and advanced (9 each)
            const uint32_t cat = fine ? (uint32_t)((c >> 3) * 2 + ((c & 7) ? 1 : 0)) : (uint32_t)(c >> 3);
            key = (uint64_t)nw | ((uint64_t)(!fixed0 && (c & 7) ? ne : 0) << 16) | (1ull << (31 + cbits * cat));
            kcat = cat;
        }
        if (!kPersist && !tm) s_val = tile_commit<W>(tr, stg, s_raw);
        uint64_t tot;
        const uint64_t exs = wg_excl_scan64(key, s_red64, &tot);
        const uint32_t total = (uint32_t)(tot & 0xFFFF), extot = (uint32_t)((tot >> 16) & 0x7FFF);
        if (tid < nbt) {
            // lane groups take the blocks kind by kind, so that a wavefront's groups mostly run
            // the same code
            const uint32_t cmask = (1u << cbits) - 1;
            uint32_t first = 0;
            for (uint32_t k = 0; k < kcat; k++) first += (uint32_t)(tot >> (31 + cbits * k)) & cmask;
            s_off[tid] = (uint16_t)(exs & 0xFFFF);
            s_exoff[tid] = (uint16_t)((exs >> 16) & 0x7FFF);
            s_perm[first + ((uint32_t)(exs >> (31 + cbits * kcat)) & cmask)] = (uint8_t)tid;
        }
        if (tid == 0) s_off[nbt] = (uint16_t)total;
        __syncthreads();

        const uint32_t G = kThreads / tb;
        const uint32_t grp = tid / G, g = tid % G;
        const bool live = grp < nbt;
        const uint32_t blk = live ? s_perm[grp] : grp;
        const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
        const V *bv = s_val + (size_t)blk * L;
        const uint32_t bmin = live ? s_min[blk] : 0;
        const uint64_t B = live ? (uint64_t)s_rng[blk] + 1 : 1;
        const uint32_t beta = bitlen64(B - 1);
        const int cls = live ? s_cls[blk] : 0;
        const int tcls = cls & 7, fam = cls >> 3;
        const uint32_t ne = live ? s_ne[blk] : 0;
        const uint32_t nw = live ? (uint32_t)s_off[blk + 1] - s_off[blk] : 0;
        uint32_t nwm = tcls && live ? main_words<(W == 4)>(T, s_C, L, fam, tcls, Lb, beta) : 0;
        nwm = nwm < nw ? nwm : nw;
        const uint64_t Th = tcls ? (1ull << (beta - tcls)) : 0;
        // threshold blocks: count the excess values (d >= T) of every lane's chunk and, when the
        // tile's lists fit the buffer, compact them there in data order
        const uint32_t ch = (Lb + G - 1) / G;
        const bool compact = !fixed0 && extot * W <= kExcBytes;
        V *s_ex = (V *)s_exc;
        if (!fixed0) {
            const uint32_t j0 = g * ch < Lb ? g * ch : Lb, j1 = (g + 1) * ch < Lb ? (g + 1) * ch : Lb;
            uint32_t cnt = 0;
            if (tcls)
                for (uint32_t j = j0; j < j1; j++) cnt += ((uint32_t)bv[j] - bmin) >= Th;
            uint32_t pos = group_excl_scan(cnt, G, s_red32);
            s_cpre[tid] = (uint16_t)pos;
            if (tcls && compact) {
                V *ex = s_ex + (live ? s_exoff[blk] : 0);
                for (uint32_t j = j0; j < j1; j++) {
                    const uint32_t d = (uint32_t)bv[j] - bmin;
                    if (d >= Th && pos < ne) ex[pos++] = (V)(d - Th);
                }
            }
            __syncthreads();
        }

        // the offset is checked against the bound before anything is written at it
        const uint64_t max_off = b0 * ((L + (8 / W) - 1) / (8 / W));
        if (base_off > max_off) {
            if (tid == 0) atomicOr(a.err, 4u);
            __syncthreads();
            continue;
        }
        if (tid == 0) {
            ((uint64_t *)(so + lo.off_index))[tile] = base_off;
            if (tile + 1 == lo.n_tiles) write_header(so, lo, variant, base_off + total);
        }
        if (live && nw) {
            uint64_t *dst = (uint64_t *)(so + lo.off_payload) + base_off + s_off[blk];
            // digit readers: pack_part asks only for digits of the part (j < its length). The main
            // part: the block's only part, or for threshold classes the digits min(d, T) in base
            // T + 1 (one call for both, so that groups of the two kinds in a wavefront run it
            // together; T <= 2^31, and no digit exceeds the bound of a plain block)
            const uint32_t Th32 = tcls ? (uint32_t)Th : 0xFFFFFFFFu;
            pack_part<(W == 4)>(T, s_C, tcls ? Th + 1 : B, Lb, fam, tcls ? nwm : nw, g, G, dst, [&](uint32_t j) -> uint64_t {
                const uint32_t d = (uint32_t)bv[j] - bmin;
                return (uint64_t)(d < Th32 ? d : Th32);
            });
            if (tcls) {
                if (compact) {
                    const V *ex = s_ex + s_exoff[blk];
                    pack_part<(W == 4)>(T, s_C, B - Th, ne, fam, nw - nwm, g, G, dst + nwm,
                                        [&](uint32_t j) -> uint64_t { return (uint64_t)ex[j]; });
                } else {
                    ExcessReader<V> exr{bv, s_cpre + (tid - g), Lb, ch, G, ne, bmin, (uint32_t)Th, 0, 0, 0};
                    pack_part<(W == 4)>(T, s_C, B - Th, ne, fam, nw - nwm, g, G, dst + nwm,
                                        [&](uint32_t j) -> uint64_t { return exr(j); });
                }
            }
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// ---- launch 1: per-call preparation --------------------------------------------------------
// Clears the error word and fills the size tables of the three width groups (block length L[g]).
__global__ __launch_bounds__(kThreads) void prep_kernel(CompressArgs a, SizeCtx *ctx, uint32_t L0, uint32_t L1,
                                                         uint32_t L2, const uint32_t *adv_tab) {
    const uint32_t Ls[3] = {L0, L1, L2};
    for (int g = 0; g < 3; g++)
        if (Ls[g]) fill_size_ctx(a.T, Ls[g], ctx[g], adv_tab ? adv_tab + (size_t)g * kAdvTab : nullptr);
    if (threadIdx.x == 0) *a.err = 0;
}

// Words of a full block (L digits) for every base B <= 2^16 + 1, basic (bits 0-15) and advanced
// (bits 16-31), per call and width group: the statistics launch reads both family sizes of a
// block with one load instead of sizing them, and the series of no block is searched.
__global__ __launch_bounds__(kThreads) void adv_table_kernel(DevTables T, uint32_t L, uint32_t *tab) {
    const uint32_t B = blockIdx.x * kThreads + threadIdx.x;
    if (B >= kAdvTab) return;
    if (B < 2) {
        tab[B] = 0;
        return;
    }
    const BaseDesc &D = T.desc[B];
    tab[B] = udiv_small(L + D.k - 1, D.k) | ((uint32_t)adv_words_atlas(T, D, L) << 16);
}

// Workspace: [err u32, 0 u32][3 size tables, kCtxBytes each][3 advanced-count tables of
// kAdvTab u32][one u32 word total per tile, padded to 8 bytes][one u64
// prefix per tile, then their sum][one u64 sum per run of kScanTiles tiles][one u64 stream
// offset per segment][the block records of each width group].
constexpr uint64_t kAdvTabBytes = 3 * ((4ull * kAdvTab + 7) & ~7ull);
struct WsLayout {
    uint64_t ctx, adv, tile_words, prefix, sums, seg_off, rec[3], rec_n[3], bytes;
};
WsLayout ws_layout(uint64_t n_tiles, uint32_t n_segs, const uint64_t *tile_lo, const uint64_t *tile_hi,
                   const uint32_t *L) {
    WsLayout w;
    const uint64_t nt = n_tiles;
    w.ctx = 8;
    w.adv = w.ctx + 3 * kCtxBytes;
    w.tile_words = w.adv + kAdvTabBytes;
    w.prefix = w.tile_words + 4 * ((nt + 1) & ~1ull);
    w.sums = w.prefix + 8 * (nt + 1);
    w.seg_off = w.sums + 8 * ((nt + kScanTiles - 1) / kScanTiles);
    uint64_t o = w.seg_off + 8 * (uint64_t)n_segs;
    for (int g = 0; g < 3; g++) {
        const uint32_t wb = 1u << g;
        w.rec_n[g] = L[g] ? (tile_hi[g] - tile_lo[g]) * tile_blocks_of(L[g], wb) : 0;
        w.rec[g] = o;
        o += rec_bytes(w.rec_n[g], wb);
    }
    w.bytes = o;
    return w;
}
uint64_t compress_ws_bytes(uint64_t n_tiles, uint32_t n_segs, const uint64_t *tile_lo, const uint64_t *tile_hi,
                           const uint32_t *L) {
    return ws_layout(n_tiles, n_segs, tile_lo, tile_hi, L).bytes;
}

// One per-tile launch (stats or pack) of width W; a persistent grid walks the tiles with a
// stride, otherwise every workgroup takes one tile (the kernel then holds fewer registers).
template <int W>
void launch_tiles(bool stats, bool persist, uint32_t grid, size_t dyn, const CompressArgs &b, hipStream_t st,
                  uint32_t tile_blocks = 0, uint32_t tile_bytes = 0) {
    const bool learned = b.variant == PCOMP_SELECT_LEARNED;
    if (stats && !learned && !persist && tile_blocks == kPairBlocks) {  // pairs of tiles, one lane per block
        stats_kernel<W, false, 0, true><<<(grid + 1) / 2, kThreads, 2 * 16 * pair_region(tile_bytes), st>>>(b);
    } else if (stats && learned && tile_blocks && tile_blocks <= kL3Blocks) {  // all tiles have tile_blocks
        if (persist)
            stats_kernel<W, true, 3><<<grid, kThreads, 0, st>>>(b);
        else
            stats_kernel<W, false, 3><<<grid, kThreads, 0, st>>>(b);
    } else if (stats && learned && tile_blocks && tile_blocks <= kMaxTileBlocks / 4) {
        if (persist)
            stats_kernel<W, true, 1><<<grid, kThreads, 0, st>>>(b);
        else
            stats_kernel<W, false, 1><<<grid, kThreads, 0, st>>>(b);
    } else if (stats && learned) {
        if (persist)
            stats_kernel<W, true, 2><<<grid, kThreads, 0, st>>>(b);
        else
            stats_kernel<W, false, 2><<<grid, kThreads, 0, st>>>(b);
    } else if (stats) {
        if (persist)
            stats_kernel<W, true, 0><<<grid, kThreads, 0, st>>>(b);
        else
            stats_kernel<W, false, 0><<<grid, kThreads, 0, st>>>(b);
    } else if (persist) {
        pack_kernel<W, true><<<grid, kThreads, dyn, st>>>(b);
    } else {
        pack_kernel<W, false><<<grid, kThreads, dyn, st>>>(b);
    }
}

// Exclusive prefix of n_tiles u32 totals by the two scan launches: prefix[t] for every tile
// and prefix[n_tiles] = their sum (nothing is written for n_tiles = 0). `sums` holds
// tile_scan_runs(n_tiles) u64. Used by the streams of 32-bit words.
uint64_t tile_scan_runs(uint64_t n_tiles) { return (n_tiles + kScanTiles - 1) / kScanTiles; }
void launch_tile_scan(uint32_t *tile_words, uint64_t *prefix, uint64_t *sums, uint64_t n_tiles, hipStream_t st) {
    CompressArgs a{};
    a.tile_words = tile_words;
    a.prefix = prefix;
    a.n_tiles = n_tiles;
    const uint32_t runs = (uint32_t)tile_scan_runs(n_tiles);
    if (runs > 0) {
        scan_sums_kernel<<<runs, kThreads, 0, st>>>(a, sums);
        scan_prefix_kernel<<<runs, kThreads, 0, st>>>(a, sums);
    }
}

// Enqueues the launches for the segments of one table. `one` is used when segs is nullptr (a
// single stream). grid = 0 gives the stats and pack launches one workgroup per tile;
// otherwise they are persistent with that many workgroups. The streams go to d_out one after
// another in the caller's order; their offsets (caller's order) go to d_seg_offsets when it is
// not null, and the bytes of all of them to *d_total.
int launch_compress_table(const SegDesc *segs, const uint32_t *tile_seg, const uint32_t *user_seg, const SegDesc &one,
                          uint32_t n_segs, const uint64_t *tile_lo, const uint64_t *tile_hi, const uint32_t *L,
                          uint64_t n_tiles, int variant, void *d_out, uint64_t *d_seg_offsets, uint64_t *d_total,
                          void *ws, uint32_t grid, hipStream_t st) {
    CompressArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    static_assert(sizeof(SizeCtx) <= kCtxBytes, "size tables exceed their workspace slot");
    const WsLayout wl = ws_layout(n_tiles, n_segs, tile_lo, tile_hi, L);
    uint8_t *wsb = (uint8_t *)ws;
    a.segs = segs;
    a.xcd_tiles = (!segs && one.rows) ? 1u : 0u;
    a.tile_seg = tile_seg;
    a.user_seg = user_seg;
    a.one = one;
    a.out = (uint8_t *)d_out;
    a.seg_offsets = d_seg_offsets;
    a.total = d_total;
    a.err = (uint32_t *)wsb;
    SizeCtx *ctx = (SizeCtx *)(wsb + wl.ctx);
    uint32_t *adv_tab = (uint32_t *)(wsb + wl.adv);
    a.tile_words = (uint32_t *)(wsb + wl.tile_words);
    a.prefix = (uint64_t *)(wsb + wl.prefix);
    uint64_t *sums = (uint64_t *)(wsb + wl.sums);
    a.seg_off = (uint64_t *)(wsb + wl.seg_off);
    a.rec = nullptr;
    a.rec_n = 0;
    a.n_segs = n_segs;
    a.n_tiles = n_tiles;
    a.variant = variant;
    a.tile_lo = 0;
    a.tile_hi = 0;
    a.ctx = ctx;
    // the advanced-count tables serve the advanced classes (8..15) and the two selectors
    const bool adv_tables = variant >= 8;
    for (int g = 0; g < 3; g++)
        if (L[g] && adv_tables)
            adv_table_kernel<<<(kAdvTab + kThreads - 1) / kThreads, kThreads, 0, st>>>(a.T, L[g],
                                                                                      adv_tab + (size_t)g * kAdvTab);
    prep_kernel<<<1, kThreads, 0, st>>>(a, ctx, L[0], L[1], L[2], adv_tables ? adv_tab : nullptr);
    const size_t dyn = 0;
    for (int g = 0; g < 3; g++) {
        const uint64_t ntg = tile_hi[g] - tile_lo[g];
        if (!ntg) continue;
        CompressArgs b = a;
        b.tile_lo = tile_lo[g];
        b.tile_hi = tile_hi[g];
        b.ctx = ctx + g;
        b.rec = wsb + wl.rec[g];
        b.rec_n = wl.rec_n[g];
        const bool persist = grid && grid < ntg;
        const uint32_t gg = (uint32_t)(persist ? grid : ntg);
        const uint32_t w = 1u << g, tbg = tile_blocks_of(L[g], w);
        if (g == 0)
            launch_tiles<1>(true, persist, gg, 0, b, st, tbg, tbg * L[g] * w);
        else if (g == 1)
            launch_tiles<2>(true, persist, gg, 0, b, st, tbg, tbg * L[g] * w);
        else
            launch_tiles<4>(true, persist, gg, 0, b, st, tbg, tbg * L[g] * w);
    }
    const uint32_t runs = (uint32_t)((n_tiles + kScanTiles - 1) / kScanTiles);
    if (runs > 0) {
        scan_sums_kernel<<<runs, kThreads, 0, st>>>(a, sums);
        scan_prefix_kernel<<<runs, kThreads, 0, st>>>(a, sums);
    }
    place_kernel<<<1, kThreads, 0, st>>>(a);
    for (int g = 0; g < 3; g++) {
        const uint64_t ntg = tile_hi[g] - tile_lo[g];
        if (!ntg) continue;
        CompressArgs b = a;
        b.tile_lo = tile_lo[g];
        b.tile_hi = tile_hi[g];
        b.ctx = ctx + g;
        b.rec = wsb + wl.rec[g];
        b.rec_n = wl.rec_n[g];
        const bool persist = grid && grid < ntg;
        const uint32_t gg = (uint32_t)(persist ? grid : ntg);
        if (g == 0)
            launch_tiles<1>(false, persist, gg, dyn, b, st);
        else if (g == 1)
            launch_tiles<2>(false, persist, gg, dyn, b, st);
        else
            launch_tiles<4>(false, persist, gg, dyn, b, st);
    }
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

// ---- training data: features, class sizes and the exhaustive choice of every block ----
// One workgroup per tile of one array: per block the 19 selector features, the words of
// each of the 16 classes (0xFFFFFFFF when invalid) and the class exhaustive search picks
// (the smallest, ties to the lowest id).
template <int W>
__global__ __launch_bounds__(kThreads) void features_kernel(const uint8_t *in, Layout lo, float *fx,
                                                            uint32_t *words, uint8_t *label, const SizeCtx *ctx,
                                                            DevTables T) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kTileBytes / 16 + 1];
    __shared__ uint64_t s_red64[kThreads / 64];
    __shared__ uint32_t s_red32[kThreads / 64];
    __shared__ SizeCtx s_C;
    const uint32_t tid = threadIdx.x;
    const uint64_t tile = blockIdx.x;
    if (tile >= lo.n_tiles) return;
    copy_size_ctx(ctx, s_C);
    const uint32_t L = lo.L, tb = lo.tile_blocks;
    const uint64_t b0 = tile * tb;
    const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
    const uint64_t v0 = b0 * L;
    const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
    const V *s_val = stage_tile<W>(in, v0, nvt, s_raw);
    __syncthreads();
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
    uint64_t lo8 = 0, hi8 = 0;
    for (uint32_t j = g; j < Lb; j += G) {
        const uint32_t b = beta - bitlen32((uint32_t)bv[j] - vmin);
        lo8 += b < 8 ? (1ull << (8 * b)) : 0;
        hi8 += b >= 8 ? (1ull << (8 * (b < 15 ? b - 8 : 7))) : 0;
    }
    Hist16 hist;
    hist_widen(lo8, hi8, hist);
#pragma unroll
    for (int q = 0; q < 4; q++) hist.w[q] = group_reduce(hist.w[q], G, AddOp(), s_red64);
    uint32_t ne_t[8];
    ne_t[0] = 0;
#pragma unroll
    for (int t = 1; t < 8; t++) ne_t[t] = ne_t[t - 1] + hist_bin(hist, t - 1);
    uint64_t key = ~0ull;
    if (live) {
        const uint64_t gb = b0 + blk;
        for (int c = (int)g; c < 16; c += (int)G) {
            const int t = c & 7;
            uint32_t nw = 0xFFFFFFFFu;
            if (t <= (int)beta) {
                uint32_t nwm, net = 0;
#pragma unroll
                for (int tt = 1; tt < 8; tt++) net = (t == tt) ? ne_t[tt] : net;  // no dynamic register index
                nw = class_words<(W == 4)>(T, s_C, L, c, Lb, B, beta, net, nwm);
                const uint64_t k2 = ((uint64_t)nw << 8) | (uint64_t)c;
                key = k2 < key ? k2 : key;
            }
            if (words) words[16 * gb + c] = nw;
        }
        if (g == 0 && fx) {
            uint32_t H[16];
#pragma unroll
            for (int b = 0; b < 16; b++) H[b] = hist_bin(hist, b);
            float x[kMlpIn];
            block_features(H, Lb, vmin, vmax, x);
#pragma unroll
            for (int i = 0; i < kMlpIn; i++) fx[(size_t)kMlpIn * gb + i] = x[i];
        }
    }
    key = group_reduce(key, G, MinOp(), s_red64);
    if (live && g == 0 && label) label[b0 + blk] = (uint8_t)(key & 0xFF);
}

__global__ void size_ctx_kernel(SizeCtx *ctx, DevTables T, uint32_t L) { fill_size_ctx(T, L, *ctx); }

int launch_features(const void *d_in, const Layout &lo, float *d_x, uint32_t *d_words, uint8_t *d_label,
                    void *d_ctx, hipStream_t st) {
    DevTables T;
    if (tables_for_current_device(&T) != PCOMP_OK) return PCOMP_EHIP;
    SizeCtx *ctx = (SizeCtx *)d_ctx;
    size_ctx_kernel<<<1, kThreads, 0, st>>>(ctx, T, lo.L);
    if (lo.n_tiles) {
        const uint32_t grid = (uint32_t)lo.n_tiles;
        const uint8_t *in = (const uint8_t *)d_in;
        if (lo.w == 1)
            features_kernel<1><<<grid, kThreads, 0, st>>>(in, lo, d_x, d_words, d_label, ctx, T);
        else if (lo.w == 2)
            features_kernel<2><<<grid, kThreads, 0, st>>>(in, lo, d_x, d_words, d_label, ctx, T);
        else
            features_kernel<4><<<grid, kThreads, 0, st>>>(in, lo, d_x, d_words, d_label, ctx, T);
    }
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

// ---- the selector's parameters, per device -------------------------------------------
static std::atomic<bool> g_model_loaded[64];

int set_model(const float *h, size_t n) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return PCOMP_EHIP;
    if (!h) {
        g_model_loaded[dev] = false;
        return PCOMP_OK;
    }
    if (n != (size_t)kMlpParams) return PCOMP_EINVAL;
    if (hipMemcpyToSymbol(HIP_SYMBOL(c_model), h, n * sizeof(float), 0, hipMemcpyHostToDevice) != hipSuccess)
        return PCOMP_EHIP;
    g_model_loaded[dev] = true;
    return PCOMP_OK;
}

bool model_loaded() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
    return g_model_loaded[dev];
}

// A single stream: a table of one segment (rows > 0: matrices [rows][cols] read time-major).
int launch_compress(const void *d_in, const Layout &lo, int variant, void *d_out, uint64_t *d_out_size, void *ws,
                    uint32_t rows, uint32_t cols, hipStream_t st) {
    SegDesc one = SegDesc();
    one.data = (const uint8_t *)d_in;
    one.lo = lo;
    one.tile0 = 0;
    one.user = 0;
    one.rows = rows;
    one.cols = cols;
    const int g = lo.w == 1 ? 0 : lo.w == 2 ? 1 : 2;
    one.group = (uint32_t)g;
    uint32_t L[3] = {0, 0, 0};
    uint64_t tile_lo[3] = {0, 0, 0}, tile_hi[3] = {0, 0, 0};
    tile_hi[g] = lo.n_tiles;
    L[g] = lo.L;
    return launch_compress_table(nullptr, nullptr, nullptr, one, 1, tile_lo, tile_hi, L, lo.n_tiles, variant, d_out,
                                 nullptr, d_out_size, ws, 0, st);
}

}  // namespace pcomp
