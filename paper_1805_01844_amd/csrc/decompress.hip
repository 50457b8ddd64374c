// decompress.hip -- grid-stride decompression kernel (gfx950).
//
// The stream's tile index gives every tile its payload offset, so tiles decode
// independently. Per tile: every block's word count is recomputed from its arrays (L_b, B,
// class, n_e); the lanes of a block's group decode its words, peeling digits from the lowest
// power (the inverse polynomial division of Sec. 3.1; see peel_digits); for the advanced method
// the value split between word i (r_i) and word i+1 (r'_i on top) is rebuilt from both words;
// threshold blocks merge their excess list back in data order; the tile leaves LDS through
// coalesced stores. A workgroup walks its tiles with loads ahead of use: while one tile's
// values are merged and stored, the next tile's block arrays come into registers and its first
// payload words straight into LDS (global_load_lds), so decoding waits on no payload load.
#include "kernels_common.h"

namespace pcomp {

struct DecompressArgs {
    const uint8_t *in;
    uint64_t in_size;
    uint8_t *out;
    uint64_t out_cap;
    int32_t *status;
    uint64_t n_tm;          // time-major output: the stream must hold n_tm values ...
    uint32_t rows, cols;    // ... of matrices [rows][cols], written back in their own layout (rows = 0: plain)
    int32_t want_w;         // element width the caller expects (0: any) ...
    uint32_t want_L;        // ... and block length (with want_w)
    int32_t report;         // this launch reports an unusable header (one launch of a call does)
    DevTables T;
};

// A batch: the plan's segment table (values go to each segment's `data`), the map from
// global tile to segment, where each segment's stream starts, and the width group of this
// launch.
struct BatchDecArgs {
    const SegDesc *segs;
    const uint32_t *tile_seg;
    const uint64_t *seg_offsets;  // byte offset of every segment's stream, in the caller's order
    uint64_t tile_lo, tile_hi;
    const uint8_t *in;  // the batch buffer
    uint64_t in_size;
    int32_t *status;
    uint32_t L;         // block length of the group
    DevTables T;
};

__device__ __forceinline__ void set_status(int32_t *st, int32_t code) { atomicMin(st, code); }

// Reads and checks a stream header (in_size bytes are readable); returns false if it is
// unusable.
__device__ __forceinline__ bool read_layout(const uint8_t *in, uint64_t in_size, Layout &lo, uint64_t &pw, int &fixed) {
    if (in_size < kHdrBytes) return false;
    const uint64_t *h = (const uint64_t *)in;
    const uint64_t h0 = h[0], h1 = h[1];
    if ((uint32_t)h0 != kMagic || ((h0 >> 32) & 0xFFFF) != kVersion) return false;
    const uint32_t w = (uint32_t)((h0 >> 48) & 0xFF), flags = (uint32_t)(h0 >> 56);
    if (!(w == 1 || w == 2 || w == 4) || (flags & ~7u)) return false;
    fixed = (int)(h1 & 0xFF);
    const uint32_t L = (uint32_t)(h1 >> 32);
    if (L == 0 || L > 65535) return false;
    if (!(flags & kFlagClass) && !(fixed == 0 || fixed == 8)) return false;
    if ((flags & kFlagNe) && (((flags & kFlagNe16) != 0) != (L > 255))) return false;
    make_layout(h[2], w, L, flags, lo);
    if (h[3] != lo.n_blocks || (uint32_t)h[4] != lo.tile_blocks) return false;
    pw = h[5];
    if (pw > (in_size >> 3) || h[6] != lo.off_payload + 8 * pw || h[6] > in_size) return false;
    return true;
}

constexpr uint32_t kDecExcBytes = 2048;
constexpr uint32_t kDecWords = 512;  // payload words of a tile staged in LDS before its decoding
// Words of a tile that the chosen classes can take: every class is at most the basic t = 0 size,
// ceil(L_b / k(B)) <= L_b w / 8 + 1 words since k(B) >= 8 / w, so a tile of at most 16 KiB of
// values has at most 2048 + tile_blocks words. Larger counts (a stream written with other
// choices) find their block by search instead of through the map.
constexpr uint32_t kMapWords = kTileBytes / 8 + kMaxTileBlocks;

struct DecShared {
    uint4 raw[kTileBytes / 16];  // decoded digits / values of the tile
    uint4 exc[kDecExcBytes / 16];  // decoded excess lists of the tile, when they fit
    uint64_t words[kDecWords];     // the tile's first payload words
    uint16_t exoff[kMaxTileBlocks];  // each threshold block's place among the tile's excess values
    uint32_t min[kMaxTileBlocks], rng[kMaxTileBlocks];
    uint16_t ne[kMaxTileBlocks], nwm[kMaxTileBlocks];
    uint32_t off[kMaxTileBlocks + 1];
    uint8_t cls[kMaxTileBlocks];
    uint8_t perm[kMaxTileBlocks];  // block taken by lane group p: basic blocks first, then advanced
    uint16_t advw[kMaxTileBlocks]; // words of advanced blocks before the block (word-by-word decoding)
    uint8_t map[kMapWords];        // block of every word of the tile (word-by-word decoding)
    uint32_t red32[kThreads / 64];
    uint64_t red64[kThreads / 64];
    SizeCtx C;
};
static_assert(sizeof(DecShared) <= 32768, "five workgroups per CU need at most 32 KiB of LDS each");

// Advanced part whose base is outside the tables: each lane of the group walks the series
// itself (the state of word i depends on every word before it) and decodes its own words
// i0, i0 + G, ... (G a power of two), including the value split at the end of each. Once the
// walk finds the series' period, whole periods before the lane's next word are skipped.
template <typename V, bool kOne = false, typename Src, typename Dst>
__device__ __forceinline__ void unpack_adv_slow(const DevTables &T, uint64_t base, uint32_t n, uint32_t nwords,
                                                uint32_t i0, uint32_t G, Src src, Dst dst, uint32_t add) {
    const SlowBase sb = slow_base(T, base);
    const Magic mB = magic_dev(base);
    uint32_t q = 0, p;
    uint64_t R;
    slow_word_fast(sb, 1, p, R);
    SeriesCycle cyc;
    for (uint32_t wi = 0; wi < nwords; wi++) {
        if (cyc.found) {
            const uint32_t target = next_own_word(wi, i0, G);
            if (target >= nwords) break;
            if (target - wi >= cyc.lam) {
                const uint32_t c = udiv_small(target - wi, cyc.lam);
                wi += c * cyc.lam;
                q += c * cyc.V;
            }
        }
        const bool last = (q + p >= n) || wi + 1 >= nwords;
        uint32_t p1 = 0;
        uint64_t R1 = 1, s1 = 1;
        if (!last) {
            s1 = slow_next(sb, R);
            slow_word_fast(sb, s1, p1, R1);
        }
        if (((wi - i0) & (G - 1)) == 0 && wi >= i0) {
            uint64_t r;
            uint64_t X = udiv64_48(src(wi), R, r);  // word = (r'_{i-1} B^p + digits) R + r
            for (int j = (int)p - 1; j >= 0; j--) {
                const uint64_t qq = div_magic(X, mB);
                if (q + j < n) dst[q + j] = (V)((uint32_t)(X - qq * base) + add);
                X = qq;
            }
            if (!last) {  // r'_i sits on top of the next word, above its p_{i+1} digits
                uint64_t r1;
                uint64_t Y = udiv64_48(src(wi + 1), R1, r1);
                for (uint32_t m = 0; m < p1; m++) Y = div_magic(Y, mB);
                dst[q + p] = (V)((uint32_t)(Y * R + r) + add);
            }
            if (kOne) break;  // kOne: word i0 only
        }
        if (last) break;
        q += p + 1;
        p = p1;
        R = R1;
        cyc.step(s1, q);
    }
}

// Decodes words i0, i0+G, ... of one part (main digits or excess list) into dst[0 .. n);
// `add` is added to every digit (the block minimum for plain blocks); src(i) is word i of the
// part.
// Advanced part whose base is outside the tables, decoded by a group of at least 8 lanes: the
// group walks the series once into its registers (SlowWindow) and lane i0 decodes a run of
// consecutive words with the entries read from the lanes holding them, rebuilding the value
// split between two words from r_{i-1} and the part left on top of word i; the value split after
// the run comes from the next run's first word. Returns false, with nothing written, when the
// series has no period within the window. Every lane of the group calls it.
template <typename V, typename Src, typename Dst>
__device__ __forceinline__ bool unpack_adv_window(const DevTables &T, uint64_t base, uint32_t n, uint32_t nwords,
                                                  uint32_t i0, uint32_t G, Src src, Dst dst, uint32_t add) {
    const SlowBase sb = slow_base(T, base);
    const SlowWindow w = slow_window(sb, n, nwords, G < 64 ? G : 64);
    if (!w.ok) return false;
    const Magic mB = magic_dev(base);
    const uint32_t run = udiv_small(nwords + G - 1, G);
    const uint32_t w0 = min(i0 * run, nwords), w1 = min(w0 + run, nwords);
    uint32_t j, c;  // entry and periods of word w0 + k
    window_index(w, w0, j, c);
    uint64_t r_prev = 0, R_prev = 1;
    uint32_t q_end = 0;  // q + p of the previous word: the place of the value split after it
    for (uint32_t k = 0; k <= run; k++) {  // the same count on every lane (entries are read across lanes)
        const uint32_t i = w0 + k;
        const uint64_t E = window_entry(w, j);
        if (w0 < w1 && i <= w1 && i < nwords) {
            const uint64_t R = E & kWinR;
            const uint32_t p = (uint32_t)((E >> 48) & 3) + 1;
            const uint32_t q = (uint32_t)(E >> 50) + c * w.V;
            uint64_t r, X;  // word = (r'_{i-1} B^p + digits) R + r
            if (R == 1) {
                X = src(i);
                r = 0;
            } else {
                X = udiv64_rcp(src(i), R, recip_f64((double)R), r);
            }
            if (i < w1) {
                for (int m = (int)p - 1; m >= 0; m--) {
                    const uint64_t qq = div_magic(X, mB);
                    if (q + (uint32_t)m < n) dst[q + m] = (V)((uint32_t)(X - qq * base) + add);
                    X = qq;
                }
            } else {
                for (uint32_t m = 0; m < p; m++) X = div_magic(X, mB);
            }
            // X is now r'_{i-1}, the top of the value split between words i - 1 and i
            if (i > w0 && q_end < n) dst[q_end] = (V)((uint32_t)(X * R_prev + r_prev) + add);
            r_prev = r;
            R_prev = R;
            q_end = q + p;
        }
        window_next(w, j, c);
    }
    return true;
}

template <typename V, bool Wide, bool kRuns, typename Src, typename Dst>
__device__ __forceinline__ void unpack_part(const DevTables &T, const PartBase &pb, uint32_t n, int fam,
                                            uint32_t nwords, uint32_t i0, uint32_t G, Src src, Dst dst,
                                            uint32_t add) {
    if (nwords == 0) return;
    // a base outside the tables (u32 data only): the whole group walks its series together
    if (Wide && kRuns && fam && !pb.D && unpack_adv_window<V>(T, pb.base, n, nwords, i0, G, src, dst, add)) return;
    if (i0 >= nwords) return;
    auto put = [&](uint32_t j, uint32_t d) {
        if (j < n) dst[j] = (V)(d + add);
    };
    auto put_all = [&](uint32_t j, uint32_t d) { dst[j] = (V)(d + add); };
    if (!fam) {
        // inverse of Sec. 3.1 Eq. (2): the k digits of word i, peeled from the lowest power.
        // Words before the last hold k values each; only the last can hold fewer (its low
        // digits are then padding), so only it checks positions.
        // The next word's load is in flight while a word is peeled.
        const uint32_t k = pb.k;
        uint32_t i = i0;
        uint64_t w = src(i);
        for (; i + 1 < nwords; i += G) {
            const uint64_t wn = i + G < nwords ? src(i + G) : 0;
            peel_digits<Wide>(pb, w, i * k, k, put_all);
            w = wn;
        }
        if (i < nwords) peel_digits<Wide>(pb, w, i * k, k, put);
        return;
    }
    if (pb.D && !kRuns) {
        // few lanes per block: lane i0 takes words i0, i0 + G, ... and reads the next word for
        // the value split at the end of each
        const BaseDesc &D = *pb.D;
        for (uint32_t i = i0; i < nwords; i += G) {
            uint32_t q;
            const AtlasEntry *e = adv_entry(T, D, i, q);
            const uint64_t X = src(i);
            const uint64_t qR = div_magic(X, e->mR);
            const uint64_t r = X - qR * e->R;  // r_i, the low part of the split value
            const uint32_t p = e->p;
            // what remains on top is r'_{i-1}; every word before the last holds only values
            if (i + 1 < nwords)
                peel_digits<Wide>(pb, qR, q, p, put_all);
            else
                peel_digits<Wide>(pb, qR, q, p, put);
            // the value split between this word (r_i at the bottom) and the next (r'_i on top)
            if (q + p < n && i + 1 < nwords) {
                uint32_t q1;
                const AtlasEntry *e1 = adv_entry(T, D, i + 1, q1);
                const uint64_t Y = div_magic(src(i + 1), e1->mR);
                const uint64_t rp = div_magic(Y, D.mBp[e1->p == D.k ? 1 : 0]);
                put(q + p, (uint32_t)(rp * e->R + r));
            }
        }
        return;
    }
    if (pb.D) {
        // Lane i0 of the group decodes a run of consecutive words, so the value split between
        // two of them is rebuilt from what it already has: r_{i-1} from the bottom of word i-1
        // and r'_{i-1}, the part left on top of word i once its digits are peeled. Only the value
        // split after the run's last word reads the next word.
        const BaseDesc &D = *pb.D;
        const uint32_t run = udiv_small(nwords + G - 1, G);
        const uint32_t w0 = i0 * run, w1 = w0 + run < nwords ? w0 + run : nwords;
        uint32_t r_prev = 0, R_prev = 0;  // r_{i-1} < R_{i-1} <= B
        uint32_t q = 0, p = 0;
        for (uint32_t i = w0; i < w1; i++) {
            const AtlasEntry *e = adv_entry(T, D, i, q);
            const uint64_t X = src(i);
            const uint64_t qR = div_magic(X, e->mR);
            const uint64_t r = X - qR * e->R;  // r_i, the low part of the next split value
            p = e->p;
            // every word before the block's last holds only values
            const uint64_t top = i + 1 < nwords ? peel_digits<Wide>(pb, qR, q, p, put_all)
                                                : peel_digits<Wide>(pb, qR, q, p, put);
            if (i > w0) put_all(q - 1, (uint32_t)(top * R_prev + r_prev));
            r_prev = (uint32_t)r;
            R_prev = e->R;
        }
        // the value split between the run's last word and the next run's first
        if (w0 < w1 && w1 < nwords && q + p < n) {
            uint32_t q1;
            const AtlasEntry *e1 = adv_entry(T, D, w1, q1);
            const uint64_t Y = div_magic(src(w1), e1->mR);
            const uint64_t rp = div_magic(Y, D.mBp[e1->p == D.k ? 1 : 0]);
            put(q + p, (uint32_t)(rp * R_prev + r_prev));
        }
        return;
    }
    // base outside the tables (u32 data only)
    if (Wide) unpack_adv_slow<V>(T, pb.base, n, nwords, i0, G, src, dst, add);
}

// Decodes word i (its value X) of one part (n digits in nwords words, constants pb) into
// dst[0 .. n), adding `add` to every digit; src(q) is word q of the part (an advanced word
// also reads the next one, which holds the rest of the value split between them). One code
// path for every word: positions past n (the padding of a last word) are not stored.
template <typename V, bool Wide, typename Src, typename Dst>
__device__ __forceinline__ void unpack_word(const DevTables &T, const PartBase &pb, uint32_t n, int fam,
                                            uint32_t nwords, uint32_t i, uint64_t X, Src src, Dst dst,
                                            uint32_t add) {
    auto put = [&](uint32_t j, uint32_t d) {
        if (j < n) dst[j] = (V)(d + add);
    };
    if (!fam || pb.D) {
        // the inverse of Sec. 3.1 Eq. (2) (k digits of word i) and of the Sec. 3.2 series
        // (r'_{i-1} on top, p_i digits, r_i at the bottom) share the peeling, so that a
        // wavefront holding words of both families runs it once
        uint32_t q = i * pb.k, p = pb.k;
        uint64_t digits = X, r = 0;
        const AtlasEntry *e = nullptr;
        if (fam) {
            e = adv_entry(T, *pb.D, i, q);
            digits = div_magic(X, e->mR);
            r = X - digits * e->R;
            p = e->p;
        }
        peel_digits<Wide>(pb, digits, q, p, put);
        if (fam && q + p < n && i + 1 < nwords) {  // the value split with the next word
            const BaseDesc &D = *pb.D;
            uint32_t q1;
            const AtlasEntry *e1 = adv_entry(T, D, i + 1, q1);
            const uint64_t Y = div_magic(src(i + 1), e1->mR);
            const uint64_t rp = div_magic(Y, D.mBp[e1->p == D.k ? 1 : 0]);
            put(q + p, (uint32_t)(rp * e->R + r));
        }
        return;
    }
    // base outside the tables (u32 data only): the series is walked up to word i
    if (Wide) unpack_adv_slow<V, true>(T, pb.base, n, nwords, i, 1, src, dst, add);
}

// Block arrays of block b of a tile, held by thread b from their load to their use.
struct BlockRaw {
    uint32_t bmin, rng, cne;  // min, B - 1, class | n_e << 8
};

template <int W>
__device__ __forceinline__ BlockRaw load_raw(const uint8_t *in, const Layout &lo, int fixed, uint64_t tile) {
    BlockRaw r = {0, 0, 0};
    const uint64_t b0 = tile * lo.tile_blocks;
    if (threadIdx.x < min((uint64_t)lo.tile_blocks, lo.n_blocks - b0)) {
        const uint64_t gb = b0 + threadIdx.x;
        const int neb = (lo.flags & kFlagNe16) ? 2 : 1;
        r.bmin = (uint32_t)get_le(in + lo.off_min + gb * W, W);
        r.rng = (uint32_t)get_le(in + lo.off_range + gb * W, W);
        const uint32_t c = (lo.flags & kFlagClass) ? in[lo.off_class + gb] : (uint32_t)fixed;
        const uint32_t ne = (lo.flags & kFlagNe) ? (uint32_t)get_le(in + lo.off_ne + gb * neb, neb) : 0;
        r.cne = (c & 0xFF) | (ne << 8);
    }
    return r;
}

// Where a tile's payload starts and ends (payload words), from the index; an inconsistent pair
// leaves the tile with nothing to stage (it is reported corrupt when decoded).
struct TileSpan {
    uint64_t base, next;
    uint32_t staged;  // words of the tile in S.words
};

__device__ __forceinline__ TileSpan tile_span(const uint8_t *in, const Layout &lo, uint64_t pw, uint64_t tile) {
    // scalar loads (the stream is read-only during the call): the entries stay out of vector
    // registers, and waiting for them does not wait for the vector memory operations
    const __attribute__((address_space(4))) uint64_t *idx =
        (const __attribute__((address_space(4))) uint64_t *)(in + lo.off_index);
    TileSpan t;
    t.base = idx[tile];
    t.next = tile + 1 < lo.n_tiles ? idx[tile + 1] : pw;
    const bool ok = t.base <= t.next && t.next <= pw;
    t.staged = ok ? (uint32_t)min(t.next - t.base, (uint64_t)kDecWords) : 0;
    return t;
}

// Starts copying the tile's first payload words into S.words, straight from global memory to
// LDS (one dword per lane and instruction; the wavefront's lanes fill consecutive dwords). The
// copy is complete once the issuing wavefront's vector-memory counter is zero.
__device__ __forceinline__ void stage_words(const uint8_t *in, const Layout &lo, const TileSpan &t, DecShared &S) {
    const uint32_t ndw = 2 * t.staged;
    const uint32_t *g = (const uint32_t *)(in + lo.off_payload) + 2 * t.base;
    uint32_t *l = (uint32_t *)S.words + (threadIdx.x & ~63u);
    for (uint32_t c = 0; c < ndw; c += kThreads)
        if (c + threadIdx.x < ndw)
            __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)(g + c + threadIdx.x),
                                             (__attribute__((address_space(3))) void *)(l + c), 4, 0, 0);
}

// Barrier for data in LDS only: this wavefront's LDS operations are complete, then the
// workgroup's wavefronts meet. Unlike __syncthreads it does not wait for global memory
// operations in flight (the next tile's copies into LDS, stores of finished values); the asm
// statement also keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// s_waitcnt vmcnt(0): this wavefront's vector-memory operations are complete (direct-to-LDS
// copies included).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// A tile's values, decoded into LDS and not yet stored: they go to out + v0 values (nvt values).
struct PendingStore {
    uint8_t *out;
    uint64_t v0;
    uint32_t nvt;  // 0: nothing pending
};

// Coalesced store of the pending tile (16-byte stores where the output is aligned); a
// time-major stream goes back to the caller's matrices value by value. Every thread calls it;
// it only reads LDS, so the next tile's decoding may start after one barrier.
template <int W, bool kTm>
__device__ __forceinline__ void store_pending(PendingStore &pend, DecShared &S, uint32_t rows, uint32_t cols) {
    typedef typename Elem<W>::T V;
    const uint32_t tid = threadIdx.x;
    const uint32_t nvt = pend.nvt;
    const uint64_t v0 = pend.v0;
    uint8_t *const out = pend.out;
    const V *s_val = (const V *)S.raw;
    if (nvt) {
        if (kTm) {
            __attribute__((address_space(1))) V *gv = (__attribute__((address_space(1))) V *)out;
            TmCursor cur(v0 + tid, rows, cols);
            for (uint32_t j = tid; j < nvt; j += kThreads) {
                gv[cur.index()] = s_val[j];
                cur.step();
            }
        } else {
            const uint8_t *sb = (const uint8_t *)S.raw;
            __attribute__((address_space(1))) uint8_t *gdst = (__attribute__((address_space(1))) uint8_t *)(out + v0 * W);
            const uint32_t head = (uint32_t)((16 - ((uintptr_t)gdst & 15)) & 15);
            const uint32_t nbytes = nvt * W;
            const uint32_t hb = head < nbytes ? head : nbytes;
            for (uint32_t b = tid * W; b < hb; b += kThreads * W) *(__attribute__((address_space(1))) V *)(gdst + b) = *(const V *)(sb + b);
            const uint32_t body = (nbytes - hb) >> 4;
            if ((hb & 3) == 0) {
                for (uint32_t c = tid; c < body; c += kThreads) {
                    const uint32_t *s32 = (const uint32_t *)(sb + hb + (c << 4));
                    typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
                    *(__attribute__((address_space(1))) U32x4 *)(gdst + hb + (c << 4)) = U32x4{s32[0], s32[1], s32[2], s32[3]};
                }
            } else {
                for (uint32_t b = hb + tid * W; b < hb + (body << 4); b += kThreads * W)
                    *(__attribute__((address_space(1))) V *)(gdst + b) = *(const V *)(sb + b);
            }
            for (uint32_t b = hb + (body << 4) + tid * W; b < nbytes; b += kThreads * W)
                *(__attribute__((address_space(1))) V *)(gdst + b) = *(const V *)(sb + b);
        }
    }
    pend.nvt = 0;
}

// Decodes tile `tile` of the stream at `in` (layout lo, pw payload words, fixed class of a
// single-class stream) into out. Every thread of the workgroup calls it, with its block's arrays
// (raw) and the tile's span, whose first words are being copied to S.words. `ahead` runs once the
// tile's words are no longer read (it may start the next tile's loads).
template <int W, bool kRuns, bool kTm = false, typename Ahead>
__device__ __forceinline__ void decode_tile(const DevTables &T, const uint8_t *in, const Layout &lo, uint64_t pw,
                                            uint64_t tile, const BlockRaw &raw, const TileSpan &span, uint8_t *out,
                                            int32_t *status, DecShared &S, PendingStore &pend, Ahead ahead,
                                            uint32_t rows = 0, uint32_t cols = 0) {
    typedef typename Elem<W>::T V;
    const uint32_t tid = threadIdx.x;
    const uint32_t L = lo.L, tb = lo.tile_blocks;
    const uint32_t G = kThreads / tb;
    const uint64_t *payload_all = (const uint64_t *)(in + lo.off_payload);
    const uint64_t vmaxw = (1ull << (8 * W)) - 1;
    V *s_val = (V *)S.raw;
    {
        const uint64_t b0 = tile * tb;
        const uint32_t nbt = (uint32_t)min((uint64_t)tb, lo.n_blocks - b0);
        const uint64_t v0 = b0 * L;
        const uint32_t nvt = (uint32_t)min((uint64_t)nbt * L, lo.n - v0);
        // ---- 1. word counts from the block arrays. One scan of packed fields gives each block
        //         its word offset, its place among the tile's excess values and its lane group
        //         (basic blocks first, then advanced ones, so that wavefronts mostly run one
        //         family's code), and counts blocks with invalid fields.
        const uint64_t base_off = span.base, next_off = span.next;
        uint64_t key = 0;
        bool adv = false;
        uint32_t nw_own = 0, cat = 0;
        constexpr uint32_t kExSh = kRuns ? 16 : 18, kCatSh = 31, kBadSh = kRuns ? 55 : 54;
        constexpr uint64_t kNwMask = kRuns ? 0xFFFF : 0x3FFFF, kExMask = kRuns ? 0x7FFF : 0x3FFFF;
        if (tid < nbt) {
            const uint64_t gb = b0 + tid;
            const uint32_t bmin = raw.bmin, rng = raw.rng;
            const int c = (int)(raw.cne & 0xFF);
            const uint32_t ne = raw.cne >> 8;
            const uint32_t Lb = (uint32_t)min((uint64_t)L, lo.n - gb * L);
            const uint64_t B = (uint64_t)rng + 1;
            const uint32_t beta = bitlen64(B - 1);
            const int t = c & 7;
            bool ok = c < 16 && t <= (int)beta && ne <= Lb && (t != 0 || ne == 0) && (uint64_t)bmin + rng <= vmaxw;
            uint32_t nwm = 0, nw = 0;
            if (ok) nw = class_words<(W == 4)>(T, S.C, L, c, Lb, B, beta, ne, nwm);
            ok = ok && nw <= 2 * Lb;  // each part takes at most one word per value
            if (!ok) nw = nwm = 0;
            S.min[tid] = bmin;
            S.rng[tid] = rng;
            S.cls[tid] = (uint8_t)(ok ? c : 0);
            S.ne[tid] = (uint16_t)ne;
            S.nwm[tid] = (uint16_t)nwm;
            adv = ok && (c >> 3);
            nw_own = nw;
            cat = (adv ? 2u : 0u) + (ok && t ? 1u : 0u);
            // Word-by-word decoding: words (18 bits; at most two per value, 2^15 in a tile),
            // excess values (18), the words of advanced blocks (18), invalid blocks (9).
            // Lane groups (at most 32 blocks a tile): words (16), excess values (15), the blocks
            // of each kind (basic, basic threshold, advanced, advanced threshold: 6 each),
            // invalid blocks (6).
            key = (uint64_t)nw | ((uint64_t)(ok && t ? ne : 0) << kExSh) | ((uint64_t)(ok ? 0 : 1) << kBadSh);
            if (kRuns)
                key |= 1ull << (kCatSh + 6 * cat);
            else
                key |= (uint64_t)(adv ? nw : 0) << 36;
        }
        uint64_t tot;
        const uint64_t ex = wg_excl_scan64(key, S.red64, &tot);
        const uint32_t tile_words = (uint32_t)(tot & kNwMask), extot = (uint32_t)((tot >> kExSh) & kExMask);
        const uint32_t n_bad = (uint32_t)(tot >> kBadSh);
        // word-by-word decoding takes the words of basic blocks first (slots 0 .. w_basic - 1),
        // then those of advanced blocks, each family in block order
        const uint32_t w_basic = tile_words - (uint32_t)((tot >> 36) & 0x3FFFF);
        if (tid < nbt) {
            S.off[tid] = (uint32_t)(ex & kNwMask);
            S.exoff[tid] = (uint16_t)((ex >> kExSh) & kExMask);
            if (kRuns) {
                // lane groups take the blocks kind by kind, so that a wavefront's groups mostly
                // run the same code
                uint32_t first = 0;
                for (uint32_t k = 0; k < cat; k++) first += (uint32_t)(tot >> (kCatSh + 6 * k)) & 0x3F;
                S.perm[first + ((uint32_t)(ex >> (kCatSh + 6 * cat)) & 0x3F)] = (uint8_t)tid;
            } else {  // advanced words before the block, and the block of each of its slots
                const uint32_t o = (uint32_t)(ex & 0x3FFFF), ap = (uint32_t)((ex >> 36) & 0x3FFFF);
                S.advw[tid] = (uint16_t)ap;
                const uint32_t s0 = adv ? w_basic + ap : o - ap;
                const uint32_t e = min(s0 + nw_own, kMapWords);
                for (uint32_t q = s0; q < e; q++) S.map[q] = (uint8_t)tid;
            }
        }
        if (tid == 0) S.off[nbt] = tile_words;
        wait_vmem();  // this wavefront's share of the staged words is in LDS
        store_pending<W, kTm>(pend, S, rows, cols);  // the previous tile leaves LDS
        __syncthreads();
        if (n_bad || base_off > pw || next_off > pw || next_off != base_off + tile_words) {
            if (tid == 0) set_status(status, PCOMP_ECORRUPT);
            ahead();
            __syncthreads();
            return;
        }
        const uint32_t staged = span.staged;
        const __attribute__((address_space(1))) uint64_t *payload =
            (const __attribute__((address_space(1))) uint64_t *)(payload_all + base_off);
        // word wi of the tile: from LDS if staged, else from global memory
        auto word_at = [&](uint32_t wi) -> uint64_t { return wi < staged ? S.words[wi] : payload[wi]; };
        // decoded excess digits go to LDS when they fit, else to the tile's own output range,
        // which nothing reads or writes until the final store of the tile
        // (the two places are kept apart in the code, so that each access uses its own address space)
        const bool exc_lds = extot * W <= kDecExcBytes;
        V *const l_exc = (V *)S.exc;
        __attribute__((address_space(1))) V *const g_exc = (__attribute__((address_space(1))) V *)(out + v0 * W);

        // ---- 2. decode. Small blocks (fewer than kRunLanes lanes per block): the workgroup's
        //         lanes take the tile's words in turn, whatever block each belongs to, so every
        //         lane has the same number of words (one more at most). Larger blocks: the lanes
        //         of a block's group take its words in turn (or runs of them).
        const uint32_t grp = tid / G, g = tid % G;
        const bool live = grp < nbt;
        const uint32_t blk = (kRuns && live) ? S.perm[grp] : grp;  // the merge takes blocks in place
        if (!kRuns) {
            const uint32_t last_Lb = nvt - (nbt - 1) * L;  // values of the tile's last block
            for (uint32_t sl = tid; sl < tile_words; sl += kThreads) {
                const bool advs = sl >= w_basic;
                uint32_t b;
                if (sl < kMapWords) {
                    b = S.map[sl];
                } else {  // the last block of the slot's family whose first slot is at or before it
                    uint32_t l = 0, h = nbt;
                    while (h - l > 1) {
                        const uint32_t m = (l + h) >> 1;
                        const uint32_t st = advs ? w_basic + S.advw[m] : S.off[m] - S.advw[m];
                        if (st <= sl) l = m; else h = m;
                    }
                    b = l;
                }
                typedef typename Elem<W>::Base BT;
                const uint32_t o = S.off[b], ap = S.advw[b];
                const uint32_t wi = advs ? sl - w_basic - ap : sl - (o - ap);
                const uint32_t c = S.cls[b];
                const int t = (int)(c & 7), fam = (int)(c >> 3);
                const BT B = (BT)S.rng[b] + 1;
                // the part of the word: the block's only part, or for threshold classes the main
                // part (base T + 1) or the excess list (base B - T)
                BT base = B;
                uint32_t n = b + 1 < nbt ? L : last_Lb, nwords = S.off[b + 1] - o, i = wi, p0 = o, add = S.min[b];
                bool exw = false;
                if (t) {
                    const uint32_t nwm = S.nwm[b];
                    const BT Th = (BT)1 << (bitlen64((uint64_t)B - 1) - t);
                    exw = wi >= nwm;
                    base = exw ? B - Th : Th + 1;
                    if (exw) {
                        n = S.ne[b];
                        nwords -= nwm;
                        i = wi - nwm;
                        p0 = o + nwm;
                        add = 0;
                    } else {
                        nwords = nwm;
                    }
                }
                auto src = [&](uint32_t q) -> uint64_t { return word_at(p0 + q); };
                const PartBase pb = resolve_base<(W == 4)>(T, S.C, (uint64_t)base);
                const uint64_t X = word_at(o + wi);
                if (!exw || exc_lds) {  // into LDS: the block's values, or the tile's excess lists
                    V *d = exw ? l_exc + S.exoff[b] : s_val + (size_t)b * L;
                    unpack_word<V, (W == 4)>(T, pb, n, fam, nwords, i, X, src, d, add);
                } else {
                    unpack_word<V, (W == 4)>(T, pb, n, fam, nwords, i, X, src, g_exc + S.exoff[b], 0);
                }
            }
        } else if (live) {
            const uint32_t nwb = S.off[blk + 1] - S.off[blk];
            const int c = S.cls[blk];
            const int t = c & 7, fam = c >> 3;
            const uint64_t B = (uint64_t)S.rng[blk] + 1;
            const uint32_t Lb = (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L);
            const uint32_t w0 = S.off[blk];
            auto src = [&](uint32_t i) -> uint64_t { return word_at(w0 + i); };
            // the basic family's constants come from the base alone; the advanced family reads
            // the schedule of its series from the tables
            auto base_of = [&](uint64_t base) -> PartBase {
                return fam ? resolve_base<(W == 4)>(T, S.C, base) : basic_base(S.C, base);
            };
            V *vals = s_val + (size_t)blk * L;
            // the main part: the block's only part, or for threshold classes the digits min(d, T)
            // in base T + 1 (one call for both, so that groups of the two kinds in a wavefront
            // run it together)
            const uint64_t Th = t ? 1ull << (bitlen64(B - 1) - t) : 0;
            const uint32_t nwm = t ? (uint32_t)S.nwm[blk] : nwb;
            unpack_part<V, (W == 4), kRuns>(T, base_of(t ? Th + 1 : B), Lb, fam, nwm, g, G, src, vals, S.min[blk]);
            if (t) {
                const PartBase pe = base_of(B - Th);
                auto esrc = [&](uint32_t i) -> uint64_t { return word_at(w0 + nwm + i); };
                if (exc_lds)
                    unpack_part<V, (W == 4), kRuns>(T, pe, S.ne[blk], fam, nwb - nwm, g, G, esrc, l_exc + S.exoff[blk], 0);
                else
                    unpack_part<V, (W == 4), kRuns>(T, pe, S.ne[blk], fam, nwb - nwm, g, G, esrc, g_exc + S.exoff[blk], 0);
            }
        }
        __syncthreads();
        ahead();  // the staged words are no longer read

        // ---- 3. threshold blocks: a main value equal to min + T (digit T) marks the next excess
        //         value, which is added to it. Blocks with B = 1 have no words: every value is
        //         the minimum.
        if (G <= 64) {
            // A block's group lies in one wavefront and takes its values in rounds; ballots rank
            // the marks of a round. The round count depends only on L, so every lane of the
            // wavefront votes.
            const int c = live ? S.cls[blk] : 0;
            const int t = c & 7;
            const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
            V *vals = s_val + (size_t)blk * L;
            if (live && !t && S.rng[blk] == 0) {
                const V m = (V)S.min[blk];
                for (uint32_t j = g; j < Lb; j += G) vals[j] = m;
            }
            if (__ballot(t != 0)) {
                const uint32_t lane = tid & 63;
                const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1)) << (lane - g);
                const uint64_t below = (1ull << lane) - 1;
                const uint32_t Tb = t ? 1u << (bitlen64((uint64_t)S.rng[blk]) - t) : 0;
                const uint32_t ne = t ? S.ne[blk] : 0;
                const uint32_t mark = t ? S.min[blk] + Tb : 0;
                const bool exc_words = t && (uint64_t)S.rng[blk] + 1 - Tb > 1;  // else every excess is 0
                const uint32_t eo = t ? S.exoff[blk] : 0;
                auto excess = [&](uint32_t pos) -> uint32_t {
                    if (!exc_words || pos >= ne) return 0;
                    return exc_lds ? (uint32_t)l_exc[eo + pos] : (uint32_t)g_exc[eo + pos];
                };
                uint32_t run = 0;  // marks of the block in earlier rounds
                if (((L * W) & 15) == 0) {
                    // blocks start on 16-byte boundaries: a lane takes 16 bytes per round and
                    // counts the marks among them; bit-sliced ballots of the counts give it the
                    // marks of the group's lanes before it
                    constexpr uint32_t per = 16 / W;
                    for (uint32_t j0 = g * per; j0 - g * per < L; j0 += G * per) {
                        const uint4 q4 = *(const uint4 *)(vals + j0);
                        uint32_t hits = 0;  // bit q: value j0 + q is a mark
#pragma unroll
                        for (uint32_t q = 0; q < per; q++) {
                            const uint32_t wv = q * W < 4 ? q4.x : q * W < 8 ? q4.y : q * W < 12 ? q4.z : q4.w;
                            const uint32_t v = W == 4 ? wv : (wv >> (8 * ((q * W) & 3))) & ((1u << (8 * W)) - 1);
                            hits |= (t && j0 + q < Lb && v == mark) ? 1u << q : 0u;
                        }
                        const uint32_t cnt = __popc(hits);
                        uint32_t pre = 0, tot = 0;
#pragma unroll
                        for (int b = 0; b < 5; b++) {  // cnt <= 16
                            const uint64_t m = __ballot((cnt >> b) & 1) & gmask;
                            pre += (uint32_t)__popcll(m & below) << b;
                            tot += (uint32_t)__popcll(m) << b;
                        }
                        uint32_t pos = run + pre;
                        while (hits) {
                            const uint32_t q = __ffs(hits) - 1;
                            hits &= hits - 1;
                            vals[j0 + q] = (V)(mark + excess(pos++));
                        }
                        run += tot;
                    }
                } else {
                    // one value per lane per round (consecutive LDS addresses); a ballot ranks the
                    // marks of the round
                    for (uint32_t j = g; j - g < L; j += G) {
                        const bool hit = t && j < Lb && (uint32_t)vals[j] == mark;
                        const uint64_t m = __ballot(hit) & gmask;
                        if (hit) vals[j] = (V)(mark + excess(run + (uint32_t)__popcll(m & below)));
                        run += (uint32_t)__popcll(m);
                    }
                }
            }
        } else {
            const int c = live ? S.cls[blk] : 0;
            const int t = c & 7;
            const uint32_t Lb = live ? (uint32_t)min((uint64_t)L, lo.n - (b0 + blk) * L) : 0;
            const uint32_t ch = (Lb + G - 1) / G;
            const uint32_t j0 = g * ch < Lb ? g * ch : Lb, j1 = (g + 1) * ch < Lb ? (g + 1) * ch : Lb;
            V *vals = s_val + (size_t)blk * L;
            uint32_t Tb = 0, mark = 0;
            uint32_t cnt = 0;
            if (t) {
                Tb = 1u << (bitlen64((uint64_t)S.rng[blk]) - t);
                mark = S.min[blk] + Tb;
                for (uint32_t j = j0; j < j1; j++) cnt += (uint32_t)vals[j] == mark;
            }
            uint32_t pos = group_excl_scan(cnt, G, S.red32);
            if (live && !t && S.rng[blk] == 0) {
                const V m = (V)S.min[blk];
                for (uint32_t j = j0; j < j1; j++) vals[j] = m;
            }
            if (t) {
                const uint32_t ne = S.ne[blk];
                const bool exc_words = (uint64_t)S.rng[blk] + 1 - Tb > 1;  // else every excess is 0
                const uint32_t eo = S.exoff[blk];
                for (uint32_t j = j0; j < j1; j++) {
                    if ((uint32_t)vals[j] == mark) {
                        uint32_t e = 0;
                        if (exc_words && pos < ne) e = exc_lds ? (uint32_t)l_exc[eo + pos] : (uint32_t)g_exc[eo + pos];
                        vals[j] = (V)(mark + e);
                        pos++;
                    }
                }
            }
        }
        lds_barrier();  // the merged values are in LDS (the next tile's loads may still be in flight)

        // ---- 4. the values wait in LDS; the next tile (or the end of the workgroup's tiles)
        //         stores them, once that tile's staged loads are complete
        pend.out = out;
        pend.v0 = v0;
        pend.nvt = nvt;
    }
}

// One kernel per element width and lane-group size (both are known on the device, from the
// stream's header; a caller that knows them launches only the matching kernel): each returns
// at once unless the header matches it, so only one does the work. Word-by-word decoding of u8 and
// u16 runs five wavefronts per SIMD (at most 96 vector registers), and five workgroups per CU fit
// the LDS (under 32 KiB each); lane-group decoding and u32 run four (128 registers, no spills),
// which measured 2-6% faster for them than five with spills.
template <int W, bool kRuns, bool kTm = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(W == 4 || kRuns ? 4 : 5))) void decompress_kernel(
    DecompressArgs a) {
    __shared__ DecShared S;
    Layout lo;
    uint64_t pw;
    int fixed;
    const bool ok = read_layout(a.in, a.in_size, lo, pw, fixed) &&
                    (a.want_w == 0 || ((int32_t)lo.w == a.want_w && lo.L == a.want_L)) &&
                    (a.rows == 0 || lo.n == a.n_tm);
    if (!ok) {  // reported once, by one launch
        if (a.report && blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, PCOMP_ECORRUPT);
        return;
    }
    if (lo.w != W || (kThreads / lo.tile_blocks >= kRunLanes) != kRuns) return;
    if ((uint64_t)lo.L * lo.w > kTileBytes) {
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, PCOMP_EINVAL);
        return;
    }
    if (lo.n > a.out_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) set_status(a.status, PCOMP_ENOSPC);
        return;
    }
    fill_size_ctx(a.T, lo.L, S.C);
    __syncthreads();
    // Tiles tile, tile + grid, ...: the next tile's arrays and words are started while this one
    // is merged and stored, and the index entries one tile further ahead.
    // time-major: tiles in XCD order, so that the scattered stores of nearby tiles meet in one L2
    uint64_t tile = kTm ? xcd_order(blockIdx.x, gridDim.x) : blockIdx.x;
    if (tile >= lo.n_tiles) return;
    BlockRaw raw = load_raw<W>(a.in, lo, fixed, tile);
    TileSpan span = tile_span(a.in, lo, pw, tile);
    stage_words(a.in, lo, span, S);
    uint64_t nxt = tile + gridDim.x;
    TileSpan nspan = nxt < lo.n_tiles ? tile_span(a.in, lo, pw, nxt) : span;
    PendingStore pend = {nullptr, 0, 0};
    for (;;) {
        const bool more = nxt < lo.n_tiles;
        const uint64_t nxt2 = nxt + gridDim.x;
        BlockRaw nraw = raw;
        TileSpan nnspan = nspan;
        auto ahead = [&]() {
            if (more) {
                stage_words(a.in, lo, nspan, S);
                nraw = load_raw<W>(a.in, lo, fixed, nxt);
                if (nxt2 < lo.n_tiles) nnspan = tile_span(a.in, lo, pw, nxt2);
            }
        };
        decode_tile<W, kRuns, kTm>(a.T, a.in, lo, pw, tile, raw, span, a.out, a.status, S, pend, ahead, a.rows,
                                   a.cols);
        if (!more) break;
        tile = nxt;
        raw = nraw;
        span = nspan;
        nspan = nnspan;
        nxt = nxt2;
    }
    store_pending<W, kTm>(pend, S, a.rows, a.cols);
}

// Batch: the tiles of one width group, each decoded into its segment's destination. A
// segment whose stream header disagrees with the plan is reported corrupt and skipped.
template <int W, bool kRuns>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(W == 4 || kRuns ? 4 : 5))) void decompress_batch_kernel(
    BatchDecArgs a) {
    __shared__ DecShared S;
    fill_size_ctx(a.T, a.L, S.C);
    __syncthreads();
    PendingStore pend = {nullptr, 0, 0};
    for (uint64_t gt = a.tile_lo + blockIdx.x; gt < a.tile_hi; gt += gridDim.x) {
        const SegDesc sd = uniform_seg(a.segs[uni32(a.tile_seg[gt])]);
        const uint64_t off = uni64(a.seg_offsets[sd.user]);
        const uint8_t *s = a.in + off;
        Layout lo;
        uint64_t pw;
        int fixed;
        const bool ok = off < a.in_size && (off & 7) == 0 && read_layout(s, a.in_size - off, lo, pw, fixed) &&
                        lo.w == W && lo.n == sd.lo.n && lo.L == sd.lo.L && lo.flags == sd.lo.flags &&
                        (kThreads / lo.tile_blocks >= kRunLanes) == kRuns;
        if (!ok) {
            if (threadIdx.x == 0) set_status(a.status, PCOMP_ECORRUPT);
            continue;
        }
        const uint64_t tile = gt - sd.tile0;
        const BlockRaw raw = load_raw<W>(s, lo, fixed, tile);
        const TileSpan span = tile_span(s, lo, pw, tile);
        stage_words(s, lo, span, S);
        decode_tile<W, kRuns>(a.T, s, lo, pw, tile, raw, span, (uint8_t *)sd.data, a.status, S, pend, [] {});
    }
    store_pending<W, false>(pend, S, 0, 0);
}

__global__ void set_i32_kernel(int32_t *p, int32_t v) { *p = v; }

// want_w = 0: the element width and block length are read on the device, so all six
// (width, lane-group) kernels are launched and five return at once; otherwise only the kernel
// for (want_w, want_L) runs, and it reports a header of another width as corrupt. rows > 0: a
// time-major stream of n_tm values in matrices [rows][cols], written back in their layout.
int launch_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity, int32_t *d_status,
                      int want_w, uint32_t want_L, uint64_t n_tm, uint32_t rows, uint32_t cols, hipStream_t st) {
    DecompressArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    set_i32_kernel<<<1, 1, 0, st>>>(d_status, PCOMP_OK);
    a.in = (const uint8_t *)d_in;
    a.in_size = in_size;
    a.out = (uint8_t *)d_out;
    a.out_cap = out_capacity;
    a.status = d_status;
    a.n_tm = n_tm;
    a.rows = rows;
    a.cols = cols;
    a.want_w = want_w;
    a.want_L = want_L;
    // persistent grid: enough workgroups to fill every CU several times over
    const uint64_t max_tiles = in_size > kHdrBytes ? (in_size - kHdrBytes) / 8 : 1;
    const uint32_t grid = (uint32_t)(max_tiles < 1 ? 1 : (max_tiles < 4096 ? max_tiles : 4096));
    DecompressArgs first = a, rest = a;
    first.report = 1;
    rest.report = 0;
    if (want_w == 0) {
        decompress_kernel<1, false><<<grid, kThreads, 0, st>>>(first);
        decompress_kernel<1, true><<<grid, kThreads, 0, st>>>(rest);
        decompress_kernel<2, false><<<grid, kThreads, 0, st>>>(rest);
        decompress_kernel<2, true><<<grid, kThreads, 0, st>>>(rest);
        decompress_kernel<4, false><<<grid, kThreads, 0, st>>>(rest);
        decompress_kernel<4, true><<<grid, kThreads, 0, st>>>(rest);
    } else if (rows) {  // time-major: the kernels with the value-by-value store
        const bool runs = kThreads / tile_blocks_of(want_L, (uint32_t)want_w) >= kRunLanes;
        if (want_w == 1 && runs)
            decompress_kernel<1, true, true><<<grid, kThreads, 0, st>>>(first);
        else if (want_w == 1)
            decompress_kernel<1, false, true><<<grid, kThreads, 0, st>>>(first);
        else if (want_w == 2 && runs)
            decompress_kernel<2, true, true><<<grid, kThreads, 0, st>>>(first);
        else if (want_w == 2)
            decompress_kernel<2, false, true><<<grid, kThreads, 0, st>>>(first);
        else if (runs)
            decompress_kernel<4, true, true><<<grid, kThreads, 0, st>>>(first);
        else
            decompress_kernel<4, false, true><<<grid, kThreads, 0, st>>>(first);
    } else {
        const bool runs = kThreads / tile_blocks_of(want_L, (uint32_t)want_w) >= kRunLanes;
        if (want_w == 1 && runs)
            decompress_kernel<1, true><<<grid, kThreads, 0, st>>>(first);
        else if (want_w == 1)
            decompress_kernel<1, false><<<grid, kThreads, 0, st>>>(first);
        else if (want_w == 2 && runs)
            decompress_kernel<2, true><<<grid, kThreads, 0, st>>>(first);
        else if (want_w == 2)
            decompress_kernel<2, false><<<grid, kThreads, 0, st>>>(first);
        else if (runs)
            decompress_kernel<4, true><<<grid, kThreads, 0, st>>>(first);
        else
            decompress_kernel<4, false><<<grid, kThreads, 0, st>>>(first);
    }
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

// Batch decompression: one persistent launch per width group present. grid = 0 picks 4096
// workgroups (or one per tile when there are fewer tiles).
int launch_decompress_batch(const BatchPlanHeader &ph, const SegDesc *d_segs, const uint32_t *d_tile_seg,
                            const void *d_in, size_t in_size, const uint64_t *d_seg_offsets, int32_t *d_status,
                            uint32_t grid, hipStream_t st) {
    BatchDecArgs a;
    if (tables_for_current_device(&a.T) != PCOMP_OK) return PCOMP_EHIP;
    set_i32_kernel<<<1, 1, 0, st>>>(d_status, PCOMP_OK);
    a.segs = d_segs;
    a.tile_seg = d_tile_seg;
    a.seg_offsets = d_seg_offsets;
    a.in = (const uint8_t *)d_in;
    a.in_size = in_size;
    a.status = d_status;
    for (int g = 0; g < 3; g++) {
        const uint64_t ntg = ph.tile_hi[g] - ph.tile_lo[g];
        if (!ntg) continue;
        BatchDecArgs b = a;
        b.tile_lo = ph.tile_lo[g];
        b.tile_hi = ph.tile_hi[g];
        b.L = ph.L[g];
        const uint32_t want = grid ? grid : 4096;
        const uint32_t gg = (uint32_t)(ntg < want ? ntg : want);
        const bool runs = kThreads / tile_blocks_of(b.L, 1u << g) >= kRunLanes;
        if (g == 0 && runs)
            decompress_batch_kernel<1, true><<<gg, kThreads, 0, st>>>(b);
        else if (g == 0)
            decompress_batch_kernel<1, false><<<gg, kThreads, 0, st>>>(b);
        else if (g == 1 && runs)
            decompress_batch_kernel<2, true><<<gg, kThreads, 0, st>>>(b);
        else if (g == 1)
            decompress_batch_kernel<2, false><<<gg, kThreads, 0, st>>>(b);
        else if (runs)
            decompress_batch_kernel<4, true><<<gg, kThreads, 0, st>>>(b);
        else
            decompress_batch_kernel<4, false><<<gg, kThreads, 0, st>>>(b);
    }
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

}  // namespace pcomp
