// capi.hip -- the C ABI declared in include/pcomp.h: argument checks, sizes, launches.
#include <mutex>

#include "pcomp_internal.h"

namespace pcomp {
uint64_t compress_ws_bytes(uint64_t n_tiles, uint32_t n_segs, const uint64_t *tile_lo, const uint64_t *tile_hi,
                           const uint32_t *L);
int launch_compress(const void *d_in, const Layout &lo, int variant, void *d_out, uint64_t *d_out_size, void *ws,
                    uint32_t rows, uint32_t cols, hipStream_t st);
int launch_compress_table(const SegDesc *segs, const uint32_t *tile_seg, const uint32_t *user_seg, const SegDesc &one,
                          uint32_t n_segs, const uint64_t *tile_lo, const uint64_t *tile_hi, const uint32_t *L,
                          uint64_t n_tiles, int variant, void *d_out, uint64_t *d_seg_offsets, uint64_t *d_total,
                          void *ws, uint32_t grid, hipStream_t st);
int launch_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity, int32_t *d_status,
                      int want_w, uint32_t want_L, uint64_t n_tm, uint32_t rows, uint32_t cols, hipStream_t st);
int launch_features(const void *d_in, const Layout &lo, float *d_x, uint32_t *d_words, uint8_t *d_label,
                    void *d_ctx, hipStream_t st);
int set_model(const float *h, size_t n);
int launch_integrate(const void *d_in, int w, uint64_t n_traces, uint32_t samples, uint32_t *d_out, hipStream_t st);
bool model_loaded();
uint64_t mlp_ws_bytes(uint64_t n);
int launch_mlp_scores(const float *prm, const float *X, uint64_t n, float *S, hipStream_t st);
int launch_mlp_loss_grad(const float *prm, const float *X, const uint8_t *Y, uint64_t n, float *grad, float *loss,
                         void *ws, hipStream_t st);
int launch_mlp_adam(float *prm, const float *grad, float *m, float *v, uint32_t step, float lr, float b1, float b2,
                    float eps, hipStream_t st);
int launch_decompress_batch(const BatchPlanHeader &ph, const SegDesc *d_segs, const uint32_t *d_tile_seg,
                            const void *d_in, size_t in_size, const uint64_t *d_seg_offsets, int32_t *d_status,
                            uint32_t grid, hipStream_t st);
uint64_t w32_ws_bytes(const Layout &lo);
int launch_compress32(const void *d_in, const Layout &lo, int variant, void *d_out, uint64_t out_cap,
                      uint64_t *d_out_size, void *ws, hipStream_t st);
int launch_decompress32(const void *d_in, size_t in_size, void *d_out, size_t out_capacity, int32_t *d_status,
                        int w, uint32_t L, hipStream_t st);
}  // namespace pcomp

using namespace pcomp;

namespace {

bool dtype_ok(int w) { return w == 1 || w == 2 || w == 4; }
bool variant_ok(int v) { return (v >= 0 && v < 16) || v == PCOMP_SELECT_EXHAUSTIVE || v == PCOMP_SELECT_LEARNED; }

int group_of(int w) { return w == 1 ? 0 : w == 2 ? 1 : 2; }

size_t ws_bytes_for(const Layout &lo) {
    uint64_t tile_lo[3] = {0, 0, 0}, tile_hi[3] = {0, 0, 0};
    uint32_t L[3] = {0, 0, 0};
    const int g = group_of((int)lo.w);
    tile_hi[g] = lo.n_tiles;
    L[g] = lo.L;
    return (size_t)compress_ws_bytes(lo.n_tiles, 1, tile_lo, tile_hi, L);
}

// Bound of one stream: every block at most its basic t = 0 size (see pcomp_bound).
uint64_t bound_of(const Layout &lo) {
    const uint64_t per = 8 / lo.w;  // digits per word of a full-range block: 64 / (8 w)
    uint64_t words = 0;
    if (lo.n_blocks) {
        const uint64_t last = lo.n - (lo.n_blocks - 1) * lo.L;
        words = (lo.n_blocks - 1) * ((lo.L + per - 1) / per) + (last + per - 1) / per;
    }
    return lo.off_payload + 8 * words;
}

// Checks a batch and returns its tile count and plan size.
int batch_shape(const pcomp_segment *h_segs, uint32_t n_segs, const uint32_t *block_len, int variant,
                uint64_t *n_tiles, uint64_t *plan_bytes) {
    if ((n_segs && !h_segs) || !block_len || !variant_ok(variant)) return PCOMP_EINVAL;
    uint64_t nt = 0;
    for (uint32_t i = 0; i < n_segs; i++) {
        const int w = (int)h_segs[i].dtype;
        if (!dtype_ok(w) || (h_segs[i].n && !h_segs[i].ptr) || ((uintptr_t)h_segs[i].ptr % w)) return PCOMP_EINVAL;
        const uint32_t L = block_len[group_of(w)];
        if (L == 0 || L > 65535 || (uint64_t)L * w > kTileBytes) return PCOMP_EINVAL;
        Layout lo;
        make_layout(h_segs[i].n, w, L, flags_of(variant, L), lo);
        nt += lo.n_tiles;
    }
    if (nt > 0xFFFFFFFFull) return PCOMP_EINVAL;
    *n_tiles = nt;
    *plan_bytes = sizeof(BatchPlanHeader) + (uint64_t)n_segs * sizeof(SegDesc) + 4 * ((nt + 1) & ~1ull) +
                  4 * (((uint64_t)n_segs + 1) & ~1ull);
    return PCOMP_OK;
}

// Checks a host plan; returns its header or nullptr.
const BatchPlanHeader *plan_header(const void *h_plan) {
    if (!h_plan || ((uintptr_t)h_plan & 7)) return nullptr;
    const BatchPlanHeader *ph = (const BatchPlanHeader *)h_plan;
    return ph->magic == kPlanMagic ? ph : nullptr;
}

}  // namespace

// Workspace of pcomp_compress_noalloc: one buffer in every device's global memory, held until
// the process ends. In host code `scratch` is only a host-side stand-in for the symbol: the
// device address comes from hipGetSymbolAddress, once per device, in pcomp_init.
static __device__ __align__(256) uint8_t scratch[PCOMP_SCRATCH_BYTES];
static void *g_scratch_ptr[64];
static std::mutex g_scratch_mu;

extern "C" int pcomp_init(void) {
    DevTables t;
    const int rc = tables_for_current_device(&t);
    if (rc != PCOMP_OK) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return PCOMP_EHIP;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return PCOMP_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    return PCOMP_OK;
}

extern "C" size_t pcomp_bound(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || !variant_ok(variant)) return 0;
    Layout lo;
    make_layout(n, w, block_len, flags_of(variant, block_len), lo);
    return (size_t)bound_of(lo);
}

extern "C" size_t pcomp_workspace_size(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || !variant_ok(variant)) return 0;
    Layout lo;
    make_layout(n, w, block_len, flags_of(variant, block_len), lo);
    return ws_bytes_for(lo);
}

namespace {
// pcomp_compress and pcomp_compress_transposed (rows > 0: n values in matrices [rows][cols]).
int compress_checked(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant, void *d_out,
                     size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes, uint32_t rows,
                     uint32_t cols, void *stream) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || !variant_ok(variant)) return PCOMP_EINVAL;
    if ((uint64_t)block_len * w > kTileBytes) return PCOMP_EINVAL;  // GPU tiles hold whole blocks
    if (variant == PCOMP_SELECT_LEARNED && !model_loaded()) return PCOMP_ENOMODEL;
    if ((n && !d_in) || !d_out || !d_out_size || !d_ws) return PCOMP_EINVAL;
    if (((uintptr_t)d_out & 7) || ((uintptr_t)d_ws & 7) || ((uintptr_t)d_in % w)) return PCOMP_EINVAL;
    Layout lo;
    make_layout(n, w, block_len, flags_of(variant, block_len), lo);
    if (out_capacity < pcomp_bound(n, dtype, block_len, variant)) return PCOMP_ENOSPC;
    if (ws_bytes < ws_bytes_for(lo)) return PCOMP_ENOWS;
    return launch_compress(d_in, lo, variant, d_out, d_out_size, d_ws, rows, cols, (hipStream_t)stream);
}
}  // namespace

extern "C" int pcomp_compress(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant,
                              void *d_out, size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes,
                              void *stream) {
    return compress_checked(d_in, n, dtype, block_len, variant, d_out, out_capacity, d_out_size, d_ws, ws_bytes, 0, 0,
                            stream);
}

extern "C" int pcomp_compress_transposed(const void *d_in, uint64_t n_mat, uint32_t rows, uint32_t cols,
                                         pcomp_dtype dtype, uint32_t block_len, int variant, void *d_out,
                                         size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes,
                                         void *stream) {
    if (rows == 0 || cols == 0) return PCOMP_EINVAL;
    const uint64_t per = (uint64_t)rows * cols;
    if (n_mat > UINT64_MAX / per) return PCOMP_EINVAL;
    return compress_checked(d_in, n_mat * per, dtype, block_len, variant, d_out, out_capacity, d_out_size, d_ws,
                            ws_bytes, rows, cols, stream);
}

extern "C" int pcomp_compress_noalloc(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len,
                                      int variant, void *d_out, size_t out_capacity, uint64_t *d_out_size,
                                      void *stream) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return PCOMP_EHIP;
    void *ptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        ptr = g_scratch_ptr[dev];
    }
    // pcomp_init has not run on this device: its tables and the buffer's address are missing,
    // and setting them up here would allocate
    if (!ptr || !tables_ready_for_current_device()) return PCOMP_ENOINIT;
    const size_t need = pcomp_workspace_size(n, dtype, block_len, variant);
    if (need > PCOMP_SCRATCH_BYTES) return PCOMP_ENOWS;
    return pcomp_compress(d_in, n, dtype, block_len, variant, d_out, out_capacity, d_out_size, ptr,
                          PCOMP_SCRATCH_BYTES, stream);
}

extern "C" int pcomp_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity,
                                int32_t *d_status, void *stream) {
    if (!d_in || !d_status || (out_capacity && !d_out)) return PCOMP_EINVAL;
    if ((uintptr_t)d_in & 7) return PCOMP_EINVAL;
    return launch_decompress(d_in, in_size, d_out, out_capacity, d_status, 0, 0, 0, 0, 0, (hipStream_t)stream);
}

extern "C" int pcomp_decompress_typed(const void *d_in, size_t in_size, pcomp_dtype dtype, uint32_t block_len,
                                      void *d_out, size_t out_capacity, int32_t *d_status, void *stream) {
    const int w = (int)dtype;
    if (!d_in || !d_status || (out_capacity && !d_out) || !dtype_ok(w)) return PCOMP_EINVAL;
    if (block_len == 0 || (uint64_t)block_len * w > kTileBytes || ((uintptr_t)d_in & 7)) return PCOMP_EINVAL;
    return launch_decompress(d_in, in_size, d_out, out_capacity, d_status, w, block_len, 0, 0, 0,
                             (hipStream_t)stream);
}

extern "C" int pcomp_decompress_transposed(const void *d_in, size_t in_size, pcomp_dtype dtype, uint32_t block_len,
                                           uint64_t n_mat, uint32_t rows, uint32_t cols, void *d_out,
                                           size_t out_capacity, int32_t *d_status, void *stream) {
    const int w = (int)dtype;
    if (!d_in || !d_status || (out_capacity && !d_out) || !dtype_ok(w) || rows == 0 || cols == 0)
        return PCOMP_EINVAL;
    if (block_len == 0 || (uint64_t)block_len * w > kTileBytes || ((uintptr_t)d_in & 7)) return PCOMP_EINVAL;
    const uint64_t per = (uint64_t)rows * cols;
    if (n_mat > UINT64_MAX / per) return PCOMP_EINVAL;
    return launch_decompress(d_in, in_size, d_out, out_capacity, d_status, w, block_len, n_mat * per, rows, cols,
                             (hipStream_t)stream);
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

extern "C" size_t pcomp_batch_plan_bytes(const pcomp_segment *h_segs, uint32_t n_segs, const uint32_t *block_len,
                                         int variant) {
    uint64_t nt, pb;
    if (batch_shape(h_segs, n_segs, block_len, variant, &nt, &pb) != PCOMP_OK) return 0;
    return (size_t)pb;
}

extern "C" int pcomp_batch_plan(const pcomp_segment *h_segs, uint32_t n_segs, const uint32_t *block_len,
                                int variant, void *h_plan, size_t plan_bytes) {
    uint64_t nt, pb;
    const int rc = batch_shape(h_segs, n_segs, block_len, variant, &nt, &pb);
    if (rc != PCOMP_OK) return rc;
    if (!h_plan || ((uintptr_t)h_plan & 7)) return PCOMP_EINVAL;
    if (plan_bytes < pb) return PCOMP_ENOSPC;
    BatchPlanHeader *ph = (BatchPlanHeader *)h_plan;
    SegDesc *sd = (SegDesc *)(ph + 1);
    uint32_t *tile_seg = (uint32_t *)(sd + n_segs);
    uint32_t *user_seg = tile_seg + ((nt + 1) & ~1ull);
    *ph = BatchPlanHeader();
    ph->magic = kPlanMagic;
    ph->n_segs = n_segs;
    ph->variant = variant;
    ph->n_tiles = nt;
    ph->plan_bytes = pb;
    // the streams follow one another; together they never exceed the sum of their bounds
    uint64_t cap = 0;
    for (uint32_t i = 0; i < n_segs; i++) {
        const int w = (int)h_segs[i].dtype;
        const uint32_t L = block_len[group_of(w)];
        Layout lo;
        make_layout(h_segs[i].n, w, L, flags_of(variant, L), lo);
        cap += bound_of(lo);
    }
    ph->out_cap = cap;
    // segments and tiles in group order (stable inside a group)
    uint32_t j = 0;
    uint64_t t = 0;
    for (int g = 0; g < 3; g++) {
        ph->tile_lo[g] = t;
        const int wg = g == 0 ? 1 : g == 1 ? 2 : 4;
        for (uint32_t i = 0; i < n_segs; i++) {
            if ((int)h_segs[i].dtype != wg) continue;
            const uint32_t L = block_len[g];
            ph->L[g] = L;
            SegDesc &d = sd[j];
            d = SegDesc();
            d.data = (const uint8_t *)h_segs[i].ptr;
            make_layout(h_segs[i].n, wg, L, flags_of(variant, L), d.lo);
            d.tile0 = t;
            d.user = i;
            d.group = (uint32_t)g;
            user_seg[i] = j;
            for (uint64_t k = 0; k < d.lo.n_tiles; k++) tile_seg[t + k] = j;
            t += d.lo.n_tiles;
            j++;
        }
        ph->tile_hi[g] = t;
    }
    if (nt & 1) tile_seg[nt] = 0;
    if (n_segs & 1) user_seg[n_segs] = 0;
    ph->ws_bytes = compress_ws_bytes(nt, n_segs, ph->tile_lo, ph->tile_hi, ph->L);
    return PCOMP_OK;
}

extern "C" int pcomp_batch_info(const void *h_plan, uint64_t *out_capacity, uint64_t *ws_bytes, uint64_t *n_tiles) {
    const BatchPlanHeader *ph = plan_header(h_plan);
    if (!ph) return PCOMP_EINVAL;
    if (out_capacity) *out_capacity = ph->out_cap;
    if (ws_bytes) *ws_bytes = ph->ws_bytes;
    if (n_tiles) *n_tiles = ph->n_tiles;
    return PCOMP_OK;
}

extern "C" int pcomp_compress_batch(const void *h_plan, const void *d_plan, void *d_out, size_t out_capacity,
                                    uint64_t *d_seg_offsets, uint64_t *d_total, void *d_ws, size_t ws_bytes,
                                    uint32_t grid, void *stream) {
    const BatchPlanHeader *ph = plan_header(h_plan);
    if (!ph || !d_plan || ((uintptr_t)d_plan & 7) || !d_total) return PCOMP_EINVAL;
    if ((ph->n_segs && (!d_out || !d_seg_offsets)) || !d_ws || ((uintptr_t)d_out & 7) || ((uintptr_t)d_ws & 7))
        return PCOMP_EINVAL;
    if (ph->variant == PCOMP_SELECT_LEARNED && !model_loaded()) return PCOMP_ENOMODEL;
    if (out_capacity < ph->out_cap) return PCOMP_ENOSPC;
    if (ws_bytes < ph->ws_bytes) return PCOMP_ENOWS;
    const SegDesc *segs = (const SegDesc *)((const BatchPlanHeader *)d_plan + 1);
    const uint32_t *tile_seg = (const uint32_t *)(segs + ph->n_segs);
    const uint32_t *user_seg = tile_seg + ((ph->n_tiles + 1) & ~1ull);
    SegDesc unused = SegDesc();
    return launch_compress_table(segs, tile_seg, user_seg, unused, ph->n_segs, ph->tile_lo, ph->tile_hi, ph->L,
                                 ph->n_tiles, ph->variant, d_out, d_seg_offsets, d_total, d_ws, grid,
                                 (hipStream_t)stream);
}

extern "C" int pcomp_decompress_batch(const void *h_plan, const void *d_plan, const void *d_in, size_t in_size,
                                      const uint64_t *d_seg_offsets, int32_t *d_status, uint32_t grid, void *stream) {
    const BatchPlanHeader *ph = plan_header(h_plan);
    if (!ph || !d_plan || ((uintptr_t)d_plan & 7) || !d_status) return PCOMP_EINVAL;
    if ((ph->n_segs && (!d_in || !d_seg_offsets)) || ((uintptr_t)d_in & 7)) return PCOMP_EINVAL;
    const SegDesc *segs = (const SegDesc *)((const BatchPlanHeader *)d_plan + 1);
    const uint32_t *tile_seg = (const uint32_t *)(segs + ph->n_segs);
    return launch_decompress_batch(*ph, segs, tile_seg, d_in, in_size, d_seg_offsets, d_status, grid,
                                   (hipStream_t)stream);
}

extern "C" int pcomp_set_model(const float *h_params, size_t n_floats) { return set_model(h_params, n_floats); }

extern "C" int pcomp_block_features(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len,
                                    float *d_x, uint32_t *d_words, uint8_t *d_label, void *d_ws, size_t ws_bytes,
                                    void *stream) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || block_len == 0 || block_len > 65535 || (uint64_t)block_len * w > kTileBytes)
        return PCOMP_EINVAL;
    if ((n && !d_in) || !d_ws || ((uintptr_t)d_ws & 7) || ((uintptr_t)d_in % w)) return PCOMP_EINVAL;
    if (ws_bytes < kCtxBytes) return PCOMP_ENOWS;
    Layout lo;
    make_layout(n, w, block_len, 0, lo);
    return launch_features(d_in, lo, d_x, d_words, d_label, d_ws, (hipStream_t)stream);
}

extern "C" int pcomp_mlp_scores(const float *d_params, const float *d_x, uint64_t n, float *d_scores, void *stream) {
    if (n && (!d_params || !d_x || !d_scores)) return PCOMP_EINVAL;
    return launch_mlp_scores(d_params, d_x, n, d_scores, (hipStream_t)stream);
}

extern "C" size_t pcomp_mlp_workspace_size(uint64_t n) { return (size_t)mlp_ws_bytes(n); }

extern "C" int pcomp_mlp_loss_grad(const float *d_params, const float *d_x, const uint8_t *d_labels, uint64_t n,
                                   float *d_grad, float *d_loss, void *d_ws, size_t ws_bytes, void *stream) {
    if (n == 0 || !d_params || !d_x || !d_labels || !d_grad || !d_ws) return PCOMP_EINVAL;
    if (n > 0xFFFFFFFFull * 256) return PCOMP_EINVAL;
    if (ws_bytes < mlp_ws_bytes(n)) return PCOMP_ENOWS;
    return launch_mlp_loss_grad(d_params, d_x, d_labels, n, d_grad, d_loss, d_ws, (hipStream_t)stream);
}

extern "C" int pcomp_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, uint32_t step, float lr,
                              float beta1, float beta2, float eps, void *stream) {
    if (!d_params || !d_grad || !d_m || !d_v || step == 0) return PCOMP_EINVAL;
    return launch_mlp_adam(d_params, d_grad, d_m, d_v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}

extern "C" int pcomp_integrate(const void *d_in, pcomp_dtype dtype, uint64_t n_traces, uint32_t samples,
                               uint32_t *d_out, void *stream) {
    const int w = (int)dtype;
    if (!dtype_ok(w) || samples == 0 || (n_traces && (!d_in || !d_out)) || ((uintptr_t)d_in % w)) return PCOMP_EINVAL;
    // every sum fits 32 bits, and a workgroup stages at least one whole trace (16 KiB)
    const uint64_t vmax = w == 4 ? 0xFFFFFFFFull : (1ull << (8 * w)) - 1;
    if ((uint64_t)samples * vmax > 0xFFFFFFFFull || (uint64_t)samples * w > 16384) return PCOMP_EINVAL;
    return launch_integrate(d_in, w, n_traces, samples, d_out, (hipStream_t)stream);
}

// ---- streams of 32-bit words --------------------------------------------------------------
namespace {
bool variant32_ok(int v, int w) { return v == 0 || ((v == 8 || v == PCOMP_SELECT_EXHAUSTIVE) && w < 4); }
unsigned flags32_of(int v) { return kFlagW32 | (v == PCOMP_SELECT_EXHAUSTIVE ? kFlagClass : 0u); }
bool args32_ok(int w, uint32_t L, int v) {
    return dtype_ok(w) && L != 0 && L <= 65535 && (uint64_t)L * w <= kTileBytes && variant32_ok(v, w);
}

// Every block at most ceil(L_b / (4 / w)) words: B <= 2^(8w) gives at least 32 / (8w) digits per
// 32-bit word, and the advanced series never takes more words than the basic packing.
uint64_t bound32_of(const Layout &lo) {
    const uint64_t per = 4 / lo.w;
    uint64_t words = 0;
    if (lo.n_blocks) {
        const uint64_t last = lo.n - (lo.n_blocks - 1) * lo.L;
        words = (lo.n_blocks - 1) * ((lo.L + per - 1) / per) + (last + per - 1) / per;
    }
    return lo.off_payload + 4 * words;
}
}  // namespace

extern "C" size_t pcomp_bound32(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant) {
    const int w = (int)dtype;
    if (!args32_ok(w, block_len, variant)) return 0;
    Layout lo;
    make_layout(n, w, block_len, flags32_of(variant), lo);
    return (size_t)bound32_of(lo);
}

extern "C" size_t pcomp_workspace_size32(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant) {
    const int w = (int)dtype;
    if (!args32_ok(w, block_len, variant)) return 0;
    Layout lo;
    make_layout(n, w, block_len, flags32_of(variant), lo);
    return (size_t)w32_ws_bytes(lo);
}

extern "C" int pcomp_compress32(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant,
                                void *d_out, size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes,
                                void *stream) {
    const int w = (int)dtype;
    if (!args32_ok(w, block_len, variant)) return PCOMP_EINVAL;
    if ((n && !d_in) || !d_out || !d_out_size || !d_ws) return PCOMP_EINVAL;
    if (((uintptr_t)d_out & 7) || ((uintptr_t)d_ws & 7) || ((uintptr_t)d_in % w)) return PCOMP_EINVAL;
    Layout lo;
    make_layout(n, w, block_len, flags32_of(variant), lo);
    if (out_capacity < bound32_of(lo)) return PCOMP_ENOSPC;
    if (ws_bytes < w32_ws_bytes(lo)) return PCOMP_ENOWS;
    return launch_compress32(d_in, lo, variant, d_out, out_capacity, d_out_size, d_ws, (hipStream_t)stream);
}

extern "C" int pcomp_decompress32(const void *d_in, size_t in_size, pcomp_dtype dtype, uint32_t block_len,
                                  void *d_out, size_t out_capacity, int32_t *d_status, void *stream) {
    const int w = (int)dtype;
    if (!args32_ok(w, block_len, 0)) return PCOMP_EINVAL;
    if (!d_in || !d_status || (out_capacity && !d_out)) return PCOMP_EINVAL;
    if (((uintptr_t)d_in & 7) || ((uintptr_t)d_out % w)) return PCOMP_EINVAL;
    return launch_decompress32(d_in, in_size, d_out, out_capacity, d_status, w, block_len, (hipStream_t)stream);
}
