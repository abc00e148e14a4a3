// Correlator for small arrays: at most 16 stations of complex-float32
// samples.
//
// With few stations a channel holds few baselines (136 at 16 stations, 36 at
// 8), so the block-pair kernels leave most of a workgroup idle and walk the
// integration chunk by chunk, each chunk a round trip to memory; on 8 stations
// x 16 channels x 256 samples they spend 21-25 us per launch, nearly all of it
// waiting for loads.  Here one workgroup takes a whole channel (channels are
// independent, Section 2):
//  * the samples of TC = 128 time steps of all stations (32 KiB at 16
//    stations) are loaded at once, four 16-byte loads per thread all in flight
//    together, and staged in LDS; the next chunk's loads are issued before the
//    current chunk is correlated;
//  * thread (b, g) owns baseline b = (i, j), i <= j, with its four
//    polarisation products (Section 2's four FMAs per complex multiply-add
//    each), over time steps g, g + G, g + 2G, ... of every chunk, where
//    G = min(32, 512 / baselines) time groups share the channel;
//  * the G partial sums of a baseline are added in LDS in the order
//    g = 0, 1, ..., G - 1 (deterministic), and autocorrelations are written
//    Hermitian (XX, YY real, YX = conj(XY)), as the other kernels write them.
// Time-blocked (ring) and station-major input use the addressing of the other
// kernels, and an integration split over workgroups gives every piece a
// workgroup of its own.
#include "common.h"

namespace xc {
namespace small {

constexpr int SMAX = 16;                       // stations
constexpr int THREADS = 512;
constexpr int TC = 128;                        // time steps per chunk
constexpr int LOADS = TC * SMAX / THREADS;     // 16-byte samples per thread and chunk
constexpr int GMAX = 32;                       // time groups at most
static_assert(LOADS * THREADS == TC * SMAX, "every thread loads the same number of samples");
static_assert(THREADS * 8 * sizeof(float) <= 2 * TC * SMAX * sizeof(float4),
              "the partial sums (8 floats per thread at most) fit the staging buffers");

__device__ __forceinline__ void cmac(float &re, float &im, float ar, float ai, float br, float bi) {
    re = fmaf(ar, br, re);
    re = fmaf(ai, bi, re);
    im = fmaf(ai, br, im);
    im = fmaf(-ar, bi, im);
}

// All baselines of channel c of job; stage: 2 TC SMAX float4 of LDS.
__device__ __forceinline__ void correlate_channel(const Job &job, int c, float4 *stage) {
    const int S = job.S, T = job.T;
    const int tid = threadIdx.x;
    const int B = S * (S + 1) / 2;
    const int G = min(GMAX, THREADS / B);
    const int b = tid % B, g = tid / B;
    const bool task = g < G;
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= b) ++j;
    const int i = b - j * (j + 1) / 2;
    const float4 *__restrict__ x = static_cast<const float4 *>(job.x);
    const int nrow = TC * S;                    // samples of one chunk

    float4 reg[LOADS];
    auto load = [&](int ch) {
#pragma unroll
        for (int k = 0; k < LOADS; ++k) {
            const int e = tid + k * THREADS;
            const int t = ch * TC + e / S, s = e % S;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (e < nrow && t < T)
                v = job.sstride ? x[(size_t)c * job.cstride + (size_t)s * job.sstride + t] : x[row_offset(job, c, t) + s];
            reg[k] = v;
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int k = 0; k < LOADS; ++k) {
            const int e = tid + k * THREADS;
            if (e < nrow) stage[buf * TC * SMAX + e] = reg[k];
        }
    };

    float xxr = 0.f, xxi = 0.f, xyr = 0.f, xyi = 0.f, yxr = 0.f, yxi = 0.f, yyr = 0.f, yyi = 0.f;
    const int nch = (T + TC - 1) / TC;
    if (nch > 0) {
        load(0);
        put(0);
    }
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
        if (ch + 1 < nch) load(ch + 1);
        if (task) {
            const float4 *sb = stage + (ch & 1) * TC * SMAX;
            const int tn = min(TC, T - ch * TC);
            for (int t = g; t < tn; t += G) {
                const float4 a = sb[t * S + i], q = sb[t * S + j];
                // (re, im) of pol X then Y; V[p][q] = sum x_ip conj(x_jq)
                cmac(xxr, xxi, a.x, a.y, q.x, q.y);
                cmac(xyr, xyi, a.x, a.y, q.z, q.w);
                cmac(yxr, yxi, a.z, a.w, q.x, q.y);
                cmac(yyr, yyi, a.z, a.w, q.z, q.w);
            }
        }
        // every thread is past chunk ch - 1, whose buffer takes chunk ch + 1
        if (ch + 1 < nch) put((ch + 1) & 1);
        __syncthreads();
    }

    // the time groups' partial sums, added in group order
    float *red = reinterpret_cast<float *>(stage);
    if (task) {
        float *r = red + (size_t)(g * B + b) * 8;
        r[0] = xxr; r[1] = xxi; r[2] = xyr; r[3] = xyi;
        r[4] = yxr; r[5] = yxi; r[6] = yyr; r[7] = yyi;
    }
    __syncthreads();
    if (tid < B) {              // then b = tid, g = 0
        float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int gg = 0; gg < G; ++gg) {
            const float *r = red + (size_t)(gg * B + tid) * 8;
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] += r[k];
        }
        if (i == j) {           // autocorrelations: XX, YY real, YX = conj(XY)
            v[1] = 0.f;
            v[7] = 0.f;
            v[4] = v[2];
            v[5] = -v[3];
        }
        float4 *V = reinterpret_cast<float4 *>(static_cast<float2 *>(job.vis) + ((size_t)c * B + tid) * 4);
        float4 lo = make_float4(v[0], v[1], v[2], v[3]), hi = make_float4(v[4], v[5], v[6], v[7]);
        if (job.accumulate) {
            const float4 olo = V[0], ohi = V[1];
            lo = make_float4(lo.x + olo.x, lo.y + olo.y, lo.z + olo.z, lo.w + olo.w);
            hi = make_float4(hi.x + ohi.x, hi.y + ohi.y, hi.z + ohi.z, hi.w + ohi.w);
        }
        V[0] = lo;
        V[1] = hi;
    }
}

__global__ __launch_bounds__(THREADS) void kernel(Job job, int nwork) {
    __shared__ float4 stage[2 * TC * SMAX];
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    int c, bi, bj;
    unit_decode(job, w, c, bi, bj);     // one block pair (0, 0) per channel
    correlate_channel(job, c, stage);
}

__global__ __launch_bounds__(THREADS) void kernel_batch(const Job *__restrict__ jobs, const Unit *__restrict__ units,
                                                        const int *__restrict__ bounds) {
    __shared__ float4 stage[2 * TC * SMAX];
    const int u = batch_unit(bounds, blockIdx.x);
    if (u < 0) return;
    const Unit un = units[u];
    const Job job = jobs[un.item];
    correlate_channel(job, un.channel, stage);
}

}  // namespace small

hipError_t launch_small(const Job &job, hipStream_t stream) {
    if (job.S < 1 || job.S > small::SMAX || job.npairs != 1) return hipErrorInvalidValue;
    const int nwork = job_units(job);
    hipLaunchKernelGGL(small::kernel, dim3(xcd_grid(nwork)), dim3(small::THREADS), 0, stream, job, nwork);
    return hipGetLastError();
}

hipError_t launch_small_batch(const Job *jobs, const Unit *units, const int *bounds, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(small::kernel_batch, dim3(grid), dim3(small::THREADS), 0, stream, jobs, units, bounds);
    return hipGetLastError();
}

}  // namespace xc
