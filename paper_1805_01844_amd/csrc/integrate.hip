// integrate.hip -- integrated-signal workload (Sec. 4.3.2): per-pixel sums of waveform traces.
//
// The paper's second data set stores, per pixel and event, the integral of the pixel's
// waveform (24/32-bit values) instead of the samples; it compresses those vectors. This kernel
// produces them on the GPU from traces [n_traces][samples] (u8/u16/u32): out[i] = sum of trace
// i, as a u32 (the caller's sample count keeps the sum below 2^32). A workgroup stages a run
// of whole traces in LDS with coalesced 16-byte loads and each thread sums one trace there.
#include "kernels_common.h"

namespace pcomp {

constexpr uint32_t kIntBytes = 16384;  // input bytes staged per workgroup and round

template <int W>
__global__ __launch_bounds__(kThreads) void integrate_kernel(const uint8_t *in, uint64_t n_traces, uint32_t samples,
                                                             uint32_t *out) {
    typedef typename Elem<W>::T V;
    __shared__ uint4 s_raw[kIntBytes / 16 + 1];
    const uint32_t per_round = kIntBytes / (samples * W) < kThreads ? kIntBytes / (samples * W) : kThreads;
    for (uint64_t t0 = (uint64_t)blockIdx.x * per_round; t0 < n_traces; t0 += (uint64_t)gridDim.x * per_round) {
        const uint32_t nt = (uint32_t)min((uint64_t)per_round, n_traces - t0);
        const uint8_t *src = in + t0 * samples * W;
        const uint32_t nbytes = nt * samples * W;
        // staged byte b of the run sits at LDS byte head + b (16-byte loads from an aligned base)
        const uint32_t head = (uint32_t)((uintptr_t)src & 15);
        const uint8_t *base = src - head;
        const uint32_t nchunks = (head + nbytes + 15) >> 4;
        uint8_t *sb = (uint8_t *)s_raw;
        for (uint32_t c = threadIdx.x; c < nchunks; c += kThreads) {
            const uint32_t cb = c << 4;
            if (cb >= head && cb + 16 <= head + nbytes) {
                s_raw[c] = *(const uint4 *)(base + cb);
            } else {
                const uint32_t e0 = cb > head ? cb : head, e1 = cb + 16 < head + nbytes ? cb + 16 : head + nbytes;
                for (uint32_t b = e0; b < e1; b += W) *(V *)(sb + b) = *(const V *)(base + b);
            }
        }
        __syncthreads();
        if (threadIdx.x < nt) {
            const V *tr = (const V *)(sb + head) + (size_t)threadIdx.x * samples;
            uint32_t sum = 0;
            for (uint32_t s = 0; s < samples; s++) sum += tr[s];
            out[t0 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

int launch_integrate(const void *d_in, int w, uint64_t n_traces, uint32_t samples, uint32_t *d_out,
                     hipStream_t st) {
    if (n_traces == 0) return PCOMP_OK;
    const uint64_t per_round = kIntBytes / ((uint64_t)samples * w) < kThreads ? kIntBytes / ((uint64_t)samples * w)
                                                                             : kThreads;
    const uint64_t rounds = (n_traces + per_round - 1) / per_round;
    const uint32_t grid = (uint32_t)(rounds < 8192 ? rounds : 8192);
    const uint8_t *in = (const uint8_t *)d_in;
    if (w == 1)
        integrate_kernel<1><<<grid, kThreads, 0, st>>>(in, n_traces, samples, d_out);
    else if (w == 2)
        integrate_kernel<2><<<grid, kThreads, 0, st>>>(in, n_traces, samples, d_out);
    else
        integrate_kernel<4><<<grid, kThreads, 0, st>>>(in, n_traces, samples, d_out);
    return hipGetLastError() == hipSuccess ? PCOMP_OK : PCOMP_EHIP;
}

}  // namespace pcomp
