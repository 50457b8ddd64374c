// pcomp_internal.h -- shared host/device definitions of the HIP library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pcomp.h"

namespace pcomp {

constexpr uint32_t kMagic = 0x504D4350u;  // "PCMP"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHdrBytes = 64;
constexpr uint32_t kTileBytes = 16384;  // format constant: tile_blocks * L * w <= kTileBytes
constexpr uint32_t kMaxTileBlocks = 256;
constexpr uint32_t kThreads = 256;  // threads per workgroup of every kernel
constexpr uint32_t kCtxBytes = 1024;  // workspace slot of the per-launch size tables

constexpr unsigned kFlagClass = 1, kFlagNe = 2, kFlagNe16 = 4;
constexpr unsigned kFlagW32 = 8;  // payload of 32-bit words (streams of pcomp_compress32)

// Bases with a precomputed advanced-method schedule: every B in [2, kAtlasDirect]
// plus 2^j + 1 for j = 17..31 (the main base T + 1 of threshold classes on wide data).
constexpr uint32_t kAtlasDirect = 65537;
constexpr uint32_t kAtlasExtra = 15;
constexpr uint32_t kAtlasBases = kAtlasDirect + 1 + kAtlasExtra;  // indexed by B (0, 1 unused)

// GM magic for unsigned division of a 64-bit dividend by d in [1, 2^32]
// (Granlund & Montgomery, PLDI 1994, Fig. 4.1):
//   t = mulhi(m, x); q = (t + ((x - t) >> sh1)) >> sh2.
struct Magic {
    uint64_t m;
    uint32_t sh1, sh2;
};

// Per-base description of the advanced series (Sec. 3.2). With s_i = R'_{i-1}
// (s_0 = 1) every word i uses p_i = k if s_i <= Qk else k - 1, R_i = floor(Q_{p_i} / s_i),
// and the next state is ceil(B / R_i). The state sequence is eventually periodic:
// s_{i + lam} = s_i for i >= mu, so entries 0 .. mu+lam-1 describe every word.
// Packing: digits handled in 32-bit chunks of h digits with P = B^h < 2^32 and B^(h-1) < 2^24,
// so a chunk is built by 24-bit multiply-adds and joined to the word by one 64-bit multiply-add
// (h = 0 when B >= 2^24: digits then go one by one through 64-bit arithmetic).
// Unpacking: a word splits once, at P2 = B^h2 with h2 = max(1, floor(k / 2)), into two parts
// below 2^51 (2^13 <= P2 <= 2^32); inside a part below 2^51 the digits come out by binary64
// division by B (rB = 1 / B rounded to nearest).
struct Chunk {
    uint32_t h;    // digits per packing chunk
    uint32_t P;    // B^h
    double rB;     // 1 / B rounded to nearest binary64
    double P2;     // B^h2, exact
    double rP2;    // 1 / P2 rounded to nearest binary64
    uint32_t h2;   // digits below the split of a word
    uint32_t pad;
};

struct BaseDesc {
    uint64_t Qk;   // floor(2^64 / B^k)
    uint64_t Qk1;  // floor(2^64 / B^(k-1))
    Magic mBp[2];  // division by B^(k-1) and by B^k (the latter unused when B^k = 2^64)
    Chunk ch;      // chunking of digits (packing and unpacking)
    uint32_t off;  // first AtlasEntry
    uint32_t V;    // values consumed by one cycle: q_{mu+lam} - q_mu
    uint16_t mu, lam;
    uint32_t k;    // digits per word (basic), k(B) = max{k : B^k <= 2^64}
};

struct AtlasEntry {
    Magic mR;     // division by R_i
    uint32_t s;   // s_i = R'_{i-1}
    uint32_t R;   // R_i
    uint32_t q;   // q_i: values consumed before word i
    uint32_t p;   // p_i
};

// The series of Sec. 3.2 with 32-bit words (capacity 2^32), for every B in [2, 2^16 + 1]:
// p_i = k if s_i <= Qk else k - 1 (k = max{k : B^k <= 2^32}), R_i = floor(Q_{p_i} / s_i),
// next state ceil(B / R_i), in the same cycle form. Every word is below 2^32, so its
// divisions are binary64 ones by the stored reciprocals (exact below 2^51, as in digit_off).
struct BaseDesc32 {
    double rB;     // 1 / B rounded to nearest
    uint64_t Qk;   // floor(2^32 / B^k)
    uint64_t Qk1;  // floor(2^32 / B^(k-1))
    uint32_t k;    // digits per 32-bit word
    uint32_t off;  // first AtlasEntry32
    uint32_t V;    // values consumed by one cycle
    uint16_t mu, lam;
};

struct AtlasEntry32 {
    double rR;    // 1 / R_i rounded to nearest
    uint32_t s;   // s_i = R'_{i-1}
    uint32_t R;   // R_i
    uint32_t q;   // q_i
    uint32_t p;   // p_i
};

struct DevTables {
    const BaseDesc *desc;    // [kAtlasBases]
    const AtlasEntry *ent;   // entries of every base
    const BaseDesc32 *desc32;   // [kAtlasDirect + 1]: 32-bit words
    const AtlasEntry32 *ent32;  // their entries
    const uint64_t *kmax;    // [65]: kmax[k] = largest B with B^k <= 2^64 (kmax[1] = UINT64_MAX)
    const uint8_t *ktab;     // [kAtlasDirect + 1]: k(B) for every B <= 2^16 + 1 (0 for B < 2)
};

// Stream layout (mirrors the format described in pcomp.h).
struct Layout {
    uint64_t n, n_blocks, n_tiles;
    uint32_t L, w, tile_blocks, flags;
    uint64_t off_index, off_min, off_range, off_class, off_ne, off_payload;
};

__host__ __device__ inline uint32_t tile_blocks_of(uint32_t L, uint32_t w) {
    uint64_t per = (uint64_t)L * w;
    uint32_t P = kMaxTileBlocks;
    while (P > 1 && (uint64_t)P * per > kTileBytes) P >>= 1;
    return P;
}

__host__ __device__ inline unsigned flags_of(int variant, uint32_t L) {
    if (variant == 0 || variant == 8) return 0;
    return kFlagClass | kFlagNe | (L > 255 ? kFlagNe16 : 0);
}

__host__ __device__ inline void make_layout(uint64_t n, uint32_t w, uint32_t L, unsigned flags, Layout &lo) {
    lo.n = n;
    lo.L = L;
    lo.w = w;
    lo.flags = flags;
    lo.n_blocks = (n + L - 1) / L;
    lo.tile_blocks = tile_blocks_of(L, w);
    lo.n_tiles = (lo.n_blocks + lo.tile_blocks - 1) / lo.tile_blocks;
    uint64_t o = kHdrBytes;
    lo.off_index = o;
    o += 8 * lo.n_tiles;
    lo.off_min = o;
    o += (uint64_t)w * lo.n_blocks;
    lo.off_range = o;
    o += (uint64_t)w * lo.n_blocks;
    lo.off_class = o;
    if (flags & kFlagClass) o += lo.n_blocks;
    lo.off_ne = o;
    if (flags & kFlagNe) o += lo.n_blocks * ((flags & kFlagNe16) ? 2 : 1);
    lo.off_payload = (o + 7) & ~(uint64_t)7;
}

// One stream of a call: its values, its layout and its tiles. A batch is a table of these,
// grouped by element width (one group per launch); a single call is a table of one. For
// decompression `data` is the destination of the values. Where a segment's stream starts in
// the output is only known once every block is sized: compression computes it on the device
// (placement launch), decompression reads it from the caller's offsets.
struct SegDesc {
    const uint8_t *data;  // the segment's values (compress: read; decompress: written)
    Layout lo;
    uint64_t tile0;       // global index of the segment's first tile
    uint32_t user;        // position of the segment in the caller's list
    uint32_t group;       // element-width group: 0 u8, 1 u16, 2 u32
    // Time-major blocking (rows > 0): the values are matrices [rows][cols], row-major, and the
    // stream holds each matrix's transpose: value t = (e cols + c) rows + r of the stream is
    // element (e, r, c). rows = 0: the values are read in their own order.
    uint32_t rows, cols;
};

// Host-built plan of a batch: this header, then n_segs SegDesc in group order (the groups'
// global tiles are consecutive), then the segment of every global tile (u32 each, padded to
// 8 bytes), then the plan index of every segment in the caller's order (u32 each).
struct BatchPlanHeader {
    uint64_t magic;                  // kPlanMagic
    uint32_t n_segs;
    int32_t variant;
    uint64_t n_tiles;                // tiles of the whole batch
    uint64_t out_cap;                // output bytes that always suffice: the sum of the segments' bounds
    uint64_t ws_bytes;               // workspace bytes
    uint64_t plan_bytes;             // bytes of the whole plan
    uint64_t tile_lo[3], tile_hi[3]; // global tiles of each group (0 u8, 1 u16, 2 u32)
    uint32_t L[3];                   // block length of each group (0: group empty)
    uint32_t pad;
};
constexpr uint64_t kPlanMagic = 0x4E414C5042504350ull;  // "PCPBPLAN"

// Host side: tables of the current device (built on first use).
int tables_for_current_device(DevTables *out);
// Host side: whether the current device's tables are built (nothing is allocated).
bool tables_ready_for_current_device();

}  // namespace pcomp
