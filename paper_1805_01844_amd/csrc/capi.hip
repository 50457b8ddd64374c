// capi.hip -- the C ABI declared in include/pcomp.h: argument checks, sizes, launches.
#include "pcomp_internal.h"

namespace pcomp {
int launch_compress(const void *d_in, const Layout &lo, int variant, void *d_out, uint64_t *d_out_size,
                    uint64_t *ws, uint64_t ws_words, hipStream_t st);
int launch_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity, int32_t *d_status,
                      hipStream_t st);
}  // namespace pcomp

using namespace pcomp;

namespace {

bool dtype_ok(int w) { return w == 1 || w == 2 || w == 4; }
bool variant_ok(int v) { return (v >= 0 && v < 16) || v == PCOMP_SELECT_EXHAUSTIVE || v == PCOMP_SELECT_LEARNED; }

// Workspace: [err u32, 0 u32][size tables, kCtxBytes][one u32 word total per tile, padded to
// 8 bytes][one u64 sum per run of 8192 tiles].
size_t ws_bytes_for(const Layout &lo) {
    const size_t nt = lo.n_tiles ? lo.n_tiles : 1;
    return 8 + kCtxBytes + 4 * ((nt + 1) & ~(size_t)1) + 8 * ((nt + 8191) / 8192);
}

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
    const uint64_t per = 8 / w;  // digits per word of a full-range block: 64 / (8 w)
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
    return launch_compress(d_in, lo, variant, d_out, d_out_size, (uint64_t *)d_ws, ws_bytes / 8,
                           (hipStream_t)stream);
}

extern "C" int pcomp_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity,
                                int32_t *d_status, void *stream) {
    if (!d_in || !d_status || (out_capacity && !d_out)) return PCOMP_EINVAL;
    if ((uintptr_t)d_in & 7) return PCOMP_EINVAL;
    return launch_decompress(d_in, in_size, d_out, out_capacity, d_status, (hipStream_t)stream);
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
