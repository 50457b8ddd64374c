/*
 * pcomp.h -- C ABI of the MI355X (gfx950) polynomial compressor.
 *
 * Lossless compression of unsigned integer arrays by the blocked polynomial
 * method of Aubert et al., "Polynomial data compression for large-scale
 * physics experiments" (arXiv:1805.01844):
 *   - the array is cut into blocks of block_len values (Sec. 3.3);
 *   - each block is reduced to its minimum and base B = max - min + 1 (Sec. 3,
 *     Sec. 3.1);
 *   - the digits v - min are packed into 64-bit words by mixed-radix (Horner)
 *     multiply-add, either the basic way, k = max{k : B^k <= 2^64} digits per
 *     word (Sec. 3.1, Eqs. (1)-(2)), or the advanced way that splits the last
 *     base of every word into R_i and R'_i (Sec. 3.2, Eqs. (3)-(11) and the
 *     series that closes the section);
 *   - optionally, values at or above a threshold T = 2^(bitlen(B-1) - t) are
 *     clipped to T in the main digits and their excess is packed separately
 *     (threshold/excess classes t = 1..7, a value split in the spirit of the
 *     r / r' split of Sec. 3.2);
 *   - decompression is the inverse polynomial division (Sec. 3.1): digits come
 *     out as exact binary64 quotients of a word's two halves, and the advanced
 *     series' divisions by R_i use multiply-high magic numbers.
 *
 * Conventions for every entry point:
 *   - d_* pointers are DEVICE pointers (HBM of the current HIP device), h_*
 *     pointers are host pointers. The caller allocates and owns every buffer;
 *     the compress/decompress calls allocate nothing and do not synchronise,
 *     so they may be captured in a HIP graph.
 *   - Work is enqueued on `stream` (NULL = the null stream) and completes
 *     asynchronously; sizes and statuses are written to device memory.
 *   - Return value: PCOMP_OK, or a negative code for errors found on the host
 *     before anything is enqueued. Errors found while reading a stream on the
 *     device are written to *d_status.
 *   - The library keeps per-device constant tables (digits per word, the
 *     advanced-method schedule of every base up to 2^16 + 1, magic numbers).
 *     They are built once per device by pcomp_init() or, failing that, on the
 *     first call on that device; that one-time set-up is the only allocation
 *     the library makes.
 *
 * Stream format (version 1, little-endian, 8-byte aligned):
 *   [0,64)    header: u32 magic "PCMP", u16 version, u8 dtype bytes w, u8 flags,
 *             u8 fixed class, u8 selector, u16 0, u32 block_len L, u64 n,
 *             u64 n_blocks, u32 tile_blocks, u32 0, u64 payload words,
 *             u64 total bytes, u64 0
 *   index     u64 x ceil(n_blocks / tile_blocks): payload word offset of the
 *             first block of every tile (tiles can be decoded independently)
 *   min[]     w bytes per block
 *   range[]   w bytes per block, B - 1
 *   class[]   u8 per block            (flags bit 0)
 *   ne[]      u8 per block, u16 if L > 255 (flags bit 1; bit 2 = u16)
 *   padding to 8 bytes, then the payload: u64 words, block after block
 *   (flags bit 3: 32-bit words instead, see pcomp_compress32).
 *   tile_blocks = the largest power of two P <= 256 with P * L * w <= 16384.
 */
#ifndef PCOMP_H
#define PCOMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types: the value is the element size in bytes. */
typedef enum { PCOMP_U8 = 1, PCOMP_U16 = 2, PCOMP_U32 = 4 } pcomp_dtype;

/* Variant argument.
 *   0..15: one fixed class c = 8 * family + t (family 0 basic, 1 advanced;
 *          t = 0 plain, t = 1..7 threshold/excess). With t = 0 every block
 *          uses that class (single-class stream). With t > 0 a block whose
 *          class is invalid (t > bitlen(B-1)) or not smaller than basic t = 0
 *          falls back to class 0.
 *   PCOMP_SELECT_EXHAUSTIVE: per block, the smallest of the 16 classes (ties to
 *          the lowest id).
 *   PCOMP_SELECT_LEARNED: per block, the class predicted by the network loaded
 *          with pcomp_set_model(), kept only if valid and strictly smaller than
 *          class 0 (PCOMP_ENOMODEL when no network is loaded on the device). */
#define PCOMP_CLASS(family, t) ((family) * 8 + (t))
#define PCOMP_SELECT_EXHAUSTIVE 0x100
#define PCOMP_SELECT_LEARNED 0x200

/* Error codes. */
#define PCOMP_OK 0
#define PCOMP_EINVAL (-1)   /* null pointer, bad dtype, block_len 0 or > 65535, bad variant */
#define PCOMP_ENOSPC (-2)   /* output capacity below pcomp_bound / below n values */
#define PCOMP_ECORRUPT (-3) /* (device status) stream header or block arrays inconsistent */
#define PCOMP_ENOMODEL (-4) /* learned selector requested with no model loaded */
#define PCOMP_EHIP (-5)     /* a HIP runtime call or launch failed */
#define PCOMP_ENOWS (-6)    /* workspace smaller than pcomp_workspace_size */
#define PCOMP_ENOINIT (-7)  /* pcomp_compress_noalloc before pcomp_init on this device */

/* One-time set-up on the current device: the constant tables and the address
 * of the device buffer pcomp_compress_noalloc uses. Optional for every other
 * call; thread-safe; returns PCOMP_OK or PCOMP_EHIP. */
int pcomp_init(void);

/* Host-only, pure. Largest stream the compressor can write for these arguments:
 * every block is at most its basic t = 0 size, ceil(L_b / (64 / (8 w))) words
 * (Sec. 3.1, Eq. (1) with B <= 2^(8w)), plus header, index and block arrays.
 * Returns 0 for invalid arguments. */
size_t pcomp_bound(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant);

/* Host-only, pure. Device workspace bytes that pcomp_compress needs (an error
 * word, size tables, three tables of advanced word counts for full blocks
 * (256 KiB each), per-tile word totals and their prefix sums, and one record
 * of 2 w + 4 bytes per block: min, B - 1, class, words and n_e, passed from
 * the sizing launch to the packing launch). Returns 0 for invalid args. */
size_t pcomp_workspace_size(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant);

/* Compresses n values of `dtype` at d_in (any alignment of the element type)
 * in blocks of block_len (the last block holds the remainder) into one v1
 * stream at d_out (8-byte aligned, out_capacity >= pcomp_bound). The stream
 * size in bytes is written to *d_out_size (device u64). d_ws must hold
 * pcomp_workspace_size bytes and be 8-byte aligned; its contents are
 * overwritten. Calls sharing a workspace must be ordered on one stream.
 * Error word: after the call, the first u32 of d_ws is 0, or has bit 1 set
 * when a block's chosen size exceeded its bound (then clamped, and the stream
 * is not valid) or bit 2 set when a tile's payload offset exceeded the bound
 * (that tile was not written). Neither happens unless the library itself is
 * wrong; a caller that wants the check reads the word after the stream. */
int pcomp_compress(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant,
                   void *d_out, size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes,
                   void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pcomp_compress with
 * its workspace taken from a buffer of PCOMP_SCRATCH_BYTES that the library
 * holds in the global memory of every device it runs on, until the process
 * ends. The call itself allocates nothing. Call pcomp_init() once on the
 * device first (PCOMP_ENOINIT otherwise). Calls whose pcomp_workspace_size
 * exceeds PCOMP_SCRATCH_BYTES return PCOMP_ENOWS (for u16 data in blocks of
 * 40 values that is above about 160 million values; longer blocks allow
 * more). Every call on one device shares that one buffer and leaves its last
 * contents there (each call rewrites all it reads): calls that may overlap on
 * one device (different streams or host threads) race, so the caller must
 * order them. The first u32 of the buffer is the error word described under
 * pcomp_compress. Other arguments, results and errors are those of
 * pcomp_compress. */
#define PCOMP_SCRATCH_BYTES (32u << 20)
int pcomp_compress_noalloc(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant,
                           void *d_out, size_t out_capacity, uint64_t *d_out_size, void *stream);

/* Decompresses the v1 stream at d_in (in_size bytes, 8-byte aligned) into
 * d_out (capacity out_capacity values of the stream's dtype). *d_status
 * (device i32) receives PCOMP_OK or PCOMP_ECORRUPT / PCOMP_ENOSPC; on error
 * the output is unspecified. No workspace is needed. */
int pcomp_decompress(const void *d_in, size_t in_size, void *d_out, size_t out_capacity, int32_t *d_status,
                     void *stream);

/* pcomp_decompress for a caller that knows the stream's element type and block
 * length (those of its compression): only the kernel for them is launched, and
 * a stream of another type or block length is reported PCOMP_ECORRUPT in
 * *d_status. Otherwise as pcomp_decompress. */
int pcomp_decompress_typed(const void *d_in, size_t in_size, pcomp_dtype dtype, uint32_t block_len, void *d_out,
                           size_t out_capacity, int32_t *d_status, void *stream);

/* ---- Time-major blocking (Sec. 4.3.1) --------------------------------------
 * The paper lays camera data out as the matrix M whose element M_ij is the
 * i-th time sample of pixel j, so that a block runs along one time sample
 * across pixels instead of along one pixel's trace. An event stored pixel by
 * pixel ([pixels][samples], row-major) is the transpose of M; these calls read
 * (and write) such matrices column by column without a transposed copy.
 * pcomp_compress_transposed compresses n_mat row-major matrices [rows][cols]
 * at d_in as the stream of their transposes: value t of the stream is element
 * (e, r, c) with t = (e cols + c) rows + r, and the stream is byte for byte
 * pcomp_compress of the transposed array. Other arguments as pcomp_compress;
 * rows = 0 or cols = 0 is PCOMP_EINVAL. */
int pcomp_compress_transposed(const void *d_in, uint64_t n_mat, uint32_t rows, uint32_t cols, pcomp_dtype dtype,
                              uint32_t block_len, int variant, void *d_out, size_t out_capacity,
                              uint64_t *d_out_size, void *d_ws, size_t ws_bytes, void *stream);

/* Decompresses such a stream (element type and block length as compressed) back
 * into n_mat matrices [rows][cols] at d_out (out_capacity values). A stream of
 * another length, type or block length gives PCOMP_ECORRUPT in *d_status. */
int pcomp_decompress_transposed(const void *d_in, size_t in_size, pcomp_dtype dtype, uint32_t block_len,
                                uint64_t n_mat, uint32_t rows, uint32_t cols, void *d_out, size_t out_capacity,
                                int32_t *d_status, void *stream);

/* ---- Integrated signal (Sec. 4.3.2) ----------------------------------------
 * The paper's second data set holds, per pixel and event, the integral of the
 * pixel's waveform (24/32-bit values) rather than its samples. This call makes
 * such vectors on the GPU: d_out[i] (device u32) = the sum of trace i of
 * d_in, n_traces traces of `samples` values each, one after another (a camera
 * event [pixels][samples] gives one sum per pixel). Requires samples *
 * (largest value of dtype) < 2^32 and samples * dtype bytes <= 16384
 * (PCOMP_EINVAL otherwise). The sums can then be compressed as u32 data. */
int pcomp_integrate(const void *d_in, pcomp_dtype dtype, uint64_t n_traces, uint32_t samples, uint32_t *d_out,
                    void *stream);

/* ---- 32-bit words (Sec. 3.1-3.2 with the paper's unsigned int) -------------
 * The paper packs into 32-bit unsigned ints: Eq. (1) and the series of Sec. 3.2
 * with capacity 2^32 (read exactly: k = max{k : B^k <= 2^32}, as above for
 * 2^64). These calls write and read v1 streams of 32-bit words: header flags
 * bit 3 set, the header's payload-word count, the tile index and the payload
 * in 32-bit words (u32, little-endian), total bytes = payload offset + 4 x
 * words, no excess counts. Only the paper's two packings: variant 0 (basic,
 * class 0), 8 (advanced, class 8) or PCOMP_SELECT_EXHAUSTIVE (per block the
 * smaller of the two, ties to basic; flags bit 0 and the class array). The
 * advanced tables cover B <= 2^16 + 1, so variants 8 and exhaustive take u8
 * and u16 data only; u32 data take variant 0. block_len * dtype bytes <=
 * 16384. Other rules, arguments and errors as pcomp_bound,
 * pcomp_workspace_size, pcomp_compress (the error word is the first u32 of
 * d_ws: bit 2 = a tile's payload would have passed the capacity) and
 * pcomp_decompress_typed; PCOMP_EINVAL for an unsupported dtype / variant
 * pair. The two stream kinds are not interchangeable: each decoder reports
 * the other's streams PCOMP_ECORRUPT. */
size_t pcomp_bound32(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant);
size_t pcomp_workspace_size32(uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant);
int pcomp_compress32(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, int variant, void *d_out,
                     size_t out_capacity, uint64_t *d_out_size, void *d_ws, size_t ws_bytes, void *stream);
int pcomp_decompress32(const void *d_in, size_t in_size, pcomp_dtype dtype, uint32_t block_len, void *d_out,
                       size_t out_capacity, int32_t *d_status, void *stream);

/* Host-only: reads n, dtype bytes and total stream size from a header that is
 * already in host memory (first 64 bytes of a stream). Returns PCOMP_OK or
 * PCOMP_ECORRUPT. */
int pcomp_stream_info(const void *h_header, uint64_t *n, int *dtype_bytes, uint32_t *block_len,
                      uint64_t *total_bytes);

/* ---- Batches ----------------------------------------------------------------
 * Many independent arrays ("segments": camera events of any shape and dtype)
 * compressed by one fixed sequence of launches, so a HIP graph can capture a
 * whole batch. Blocks never cross segments (the method blocks each array on its
 * own, Sec. 3.3); every segment becomes its own v1 stream, exactly the stream
 * pcomp_compress would write for it alone with the same block length and
 * variant. The streams are written one after another, in the caller's order,
 * with no gap: the batch buffer's first *d_total bytes are a file that can be
 * read back by parts (one stream per segment, each with its tile index,
 * Sec. 3.3 and Sec. 4.3). Where each stream starts is found on the device once
 * every block is sized, and written to d_seg_offsets.
 *
 * A plan is built on the host from the segment list and must then be copied,
 * byte for byte, to device memory by the caller (8-byte aligned); calls take
 * both copies (sizes and launch shapes come from the host copy, the kernels
 * read the device copy). A plan records the segment pointers: for compression
 * they are the inputs; for decompression build a plan of the same segments
 * (same order, sizes, dtypes, block lengths, variant) whose pointers are the
 * destinations. */
typedef struct {
    const void *ptr; /* device pointer to the segment's values (aligned to its dtype) */
    uint64_t n;      /* values */
    uint32_t dtype;  /* pcomp_dtype */
    uint32_t reserved;
} pcomp_segment;

/* Host-only. Plan bytes for this batch; block_len[3] gives the block length of
 * the u8, u16 and u32 segments (each with block_len * dtype bytes <= 16384
 * where such segments exist). Returns 0 for invalid arguments. */
size_t pcomp_batch_plan_bytes(const pcomp_segment *h_segs, uint32_t n_segs, const uint32_t *block_len,
                              int variant);

/* Host-only. Writes the plan (8-byte aligned host buffer of plan_bytes).
 * Returns PCOMP_OK, PCOMP_EINVAL, PCOMP_ENOSPC (buffer too small) or
 * PCOMP_ENOMODEL. */
int pcomp_batch_plan(const pcomp_segment *h_segs, uint32_t n_segs, const uint32_t *block_len, int variant,
                     void *h_plan, size_t plan_bytes);

/* Host-only. From a host plan: the output capacity a compression needs (the
 * sum of the segments' pcomp_bound: the streams never take more), the
 * workspace bytes and the tile count. Any pointer may be NULL. */
int pcomp_batch_info(const void *h_plan, uint64_t *out_capacity, uint64_t *ws_bytes, uint64_t *n_tiles);

/* Compresses every segment of the plan into d_out (8-byte aligned,
 * out_capacity >= the plan's output capacity). Segment i's stream starts at
 * byte d_seg_offsets[i] (device u64 array of n_segs, caller's order; every
 * offset is a multiple of 8) and ends where the next one starts; *d_total
 * (device u64) receives the bytes of all streams together. grid = 0 runs the
 * per-tile launches with one workgroup per tile; grid > 0 makes them
 * persistent with that many workgroups per width group. The workspace rules of
 * pcomp_compress apply, including its error word. */
int pcomp_compress_batch(const void *h_plan, const void *d_plan, void *d_out, size_t out_capacity,
                         uint64_t *d_seg_offsets, uint64_t *d_total, void *d_ws, size_t ws_bytes, uint32_t grid,
                         void *stream);

/* Decompresses the streams of a batch buffer (in_size bytes at d_in, segment
 * i's stream at byte d_seg_offsets[i], device array in the caller's order, as
 * pcomp_compress_batch wrote it) into the plan's segment pointers. *d_status
 * gets PCOMP_OK or PCOMP_ECORRUPT (an offset is unaligned or out of range, a
 * header disagrees with the plan, or a stream is inconsistent). grid = 0 picks
 * min(tiles, 4096) workgroups per width group. No workspace is needed. */
int pcomp_decompress_batch(const void *h_plan, const void *d_plan, const void *d_in, size_t in_size,
                           const uint64_t *d_seg_offsets, int32_t *d_status, uint32_t grid, void *stream);

/* ---- Learned class selector ----------------------------------------------------
 * The method leaves the choice of packing to the user (basic or advanced, Sec. 3.1-3.2;
 * the paper compares them per file, Sec. 4). PCOMP_SELECT_LEARNED picks a class per
 * block with a small network instead of sizing all 16: 19 features of the block -> 64
 * ReLU units -> 16 class scores, the first largest score wins, and the class is kept
 * only if valid and strictly smaller than class 0 (so output stays lossless and never
 * larger than the plain basic method).
 *
 * Features, computed with correctly rounded binary32 operations only (every IEEE
 * implementation gets the same bits): for b = 0..15, H[b] / L_b with H[b] the number
 * of digits d = v - min with min(bitlen(B - 1) - bitlen(d), 15) = b; lg(min + 1) / 32;
 * lg(max + 1) / 32, where lg(u) = e + (u - 2^e) 2^-e for 2^e <= u < 2^(e+1) (the
 * difference rounded to binary32); and L_b / 4096. Every sum of the network is a chain
 * of fused multiply-adds in index order starting from the bias. Parameters (2320
 * floats, in this order): W1 (64 x 19, row-major), b1 (64), W2 (16 x 64), b2 (16). */
#define PCOMP_MLP_PARAMS 2320

/* Loads the selector's parameters (host array of PCOMP_MLP_PARAMS floats; NULL
 * unloads) on the current device. Synchronous; must not overlap a learned
 * compression on that device. Returns PCOMP_OK, PCOMP_EINVAL or PCOMP_EHIP. */
int pcomp_set_model(const float *h_params, size_t n_floats);

/* Training data: for every block of an array (blocks of block_len as in
 * pcomp_compress), its 19 features (d_x, float [n_blocks][19]), the words of each
 * of the 16 classes (d_words, u32 [n_blocks][16], 0xFFFFFFFF when the class is
 * invalid) and the class exhaustive search picks (d_label, u8 [n_blocks]). Any of
 * the three outputs may be NULL. d_ws: 1024 bytes of device workspace. */
int pcomp_block_features(const void *d_in, uint64_t n, pcomp_dtype dtype, uint32_t block_len, float *d_x,
                         uint32_t *d_words, uint8_t *d_label, void *d_ws, size_t ws_bytes, void *stream);

/* Scores (d_scores, float [n][16]) of n feature vectors (d_x, float [n][19]) under
 * the parameters at d_params, with the selector's exact order of operations. */
int pcomp_mlp_scores(const float *d_params, const float *d_x, uint64_t n, float *d_scores, void *stream);

/* Host-only. Workspace bytes of pcomp_mlp_loss_grad for n samples. */
size_t pcomp_mlp_workspace_size(uint64_t n);

/* Mean cross-entropy of softmax(scores) against the labels (u8 class ids) over n
 * samples, written to *d_loss (device float, may be NULL), and its gradient with
 * respect to the parameters (d_grad, PCOMP_MLP_PARAMS floats). Deterministic: the
 * same inputs give the same bits. */
int pcomp_mlp_loss_grad(const float *d_params, const float *d_x, const uint8_t *d_labels, uint64_t n, float *d_grad,
                        float *d_loss, void *d_ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba, 2015, with bias correction; step counts from 1) on
 * the parameters, with moment buffers d_m and d_v (PCOMP_MLP_PARAMS floats each,
 * zero before the first step). */
int pcomp_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, uint32_t step, float lr,
                   float beta1, float beta2, float eps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PCOMP_H */
