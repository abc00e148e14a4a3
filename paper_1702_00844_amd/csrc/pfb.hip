// F-engine: a critically sampled polyphase filter bank that turns each
// station's sample stream into the frequency channels the correlator takes
// (Section 2: station data are filtered into channels and delay-compensated
// before correlation, Figure 1's processing chain).  The paper fixes no filter
// design; the filter bank computed here, for N channels and M taps, is
//
//     u[t][n] = sum_m h[m N + n] z[(t + m) N + n]
//     y[t][k] = sum_n u[t][n] exp(-2 pi i k n / N)
//     x[k][t][s][p] = w[s][p][k] y_{s,p}[t][k]         (w optional)
//
// and its output x is the correlator's channel-major, time-major input: the
// FX correlator's corner turn (Section 7) is the last step.
//
// Two HBM-bound kernels:
//  * filter_fft: one workgroup per (station-polarisation stream, block of
//    frames); thread n owns polyphase branch n (and n + 256): its M taps and
//    a sliding window of its last M input samples stay in registers, so each
//    input sample is read once, coalesced (a frame is N consecutive samples);
//    the branch outputs of the block's frames go to LDS and are transformed
//    there by a radix-2 Stockham FFT (two ping-pong buffers, twiddles from a
//    table computed on the host in double precision), then weighted and
//    written as rows of N channels per frame: y[stream][t][k].
//  * the corner turn y[stream][t][k] -> x[k][t][stream] through LDS tiles
//    (transpose.h): coalesced on both sides.
#include <cmath>
#include <vector>

#include "common.h"
#include "transpose.h"

namespace xc {
namespace pfb {

constexpr int MAX_TAPS = 16;
constexpr int THREADS = 256;
constexpr int FFT_LDS = 65536;                 // two buffers of frames x N complex

template <int N>
struct Geo {
    static_assert(N == 256 || N == 512, "256 or 512 channels");
    static constexpr int BR = N / THREADS;                  // branches per thread
    static constexpr int FB = FFT_LDS / 2 / (N * 8);        // frames per workgroup: 16 or 8
    static constexpr int LOG2N = N == 256 ? 8 : 9;
};

template <int N>
__global__ __launch_bounds__(THREADS) void filter_fft(const float2 *__restrict__ z, const float *__restrict__ taps,
                                                      const float2 *__restrict__ weights,
                                                      const float2 *__restrict__ twiddle, float2 *__restrict__ y,
                                                      int M, int n_in, int T) {
    typedef Geo<N> G;
    __shared__ __attribute__((aligned(16))) float2 buf[2][G::FB * N];
    __shared__ float2 tw[N / 2];
    const int tid = threadIdx.x;
    const int stream = blockIdx.y;
    const int f0 = blockIdx.x * G::FB;
    const int nf = T - f0 < G::FB ? T - f0 : G::FB;          // frames of this block
    for (int i = tid; i < N / 2; i += THREADS) tw[i] = twiddle[i];

    const float2 *zs = z + (size_t)stream * n_in;
    float h[MAX_TAPS][G::BR];
    float2 win[MAX_TAPS][G::BR];
#pragma unroll
    for (int m = 0; m < MAX_TAPS; ++m)
#pragma unroll
        for (int b = 0; b < G::BR; ++b) {
            h[m][b] = m < M ? taps[m * N + tid + b * THREADS] : 0.f;
            // the window of the block's first frame, but for its last sample
            win[m][b] = (m < M - 1) ? zs[(size_t)(f0 + m) * N + tid + b * THREADS] : make_float2(0.f, 0.f);
        }
    // filter: frame f needs samples of frames f .. f + M - 1 of the stream
    for (int f = 0; f < nf; ++f) {
#pragma unroll
        for (int b = 0; b < G::BR; ++b) {
            const int n = tid + b * THREADS;
            // newest sample of the window: frame f0 + f + M - 1 (always < T + M - 1)
            float2 v = zs[(size_t)(f0 + f + M - 1) * N + n];
#pragma unroll
            for (int m = 0; m < MAX_TAPS; ++m)
                if (m == M - 1) win[m][b] = v;
            float ur = 0.f, ui = 0.f;
#pragma unroll
            for (int m = 0; m < MAX_TAPS; ++m) {
                if (m < M) {
                    ur += h[m][b] * win[m][b].x;
                    ui += h[m][b] * win[m][b].y;
                }
            }
            buf[0][f * N + n] = make_float2(ur, ui);
            // slide the window by one frame
#pragma unroll
            for (int m = 0; m + 1 < MAX_TAPS; ++m) win[m][b] = win[m + 1][b];
        }
    }
    __syncthreads();

    // Stockham radix-2 FFT of the nf frames: sub-transform size ns doubles each
    // stage; butterfly j of a frame combines elements j and j + N/2 into
    // positions 2 (j - k) + k and 2 (j - k) + k + ns, k = j mod ns, with
    // twiddle exp(-2 pi i k / (2 ns)) = tw[k N / (2 ns)].
    int src = 0;
    for (int s = 0; s < G::LOG2N; ++s) {
        const int ns = 1 << s;
        const float2 *in = buf[src];
        float2 *out = buf[src ^ 1];
        for (int q = tid; q < nf * (N / 2); q += THREADS) {
            const int f = q / (N / 2), j = q - f * (N / 2);
            const int k = j & (ns - 1);
            const float2 a = in[f * N + j];
            const float2 bb = in[f * N + j + N / 2];
            const float2 w = tw[k * (N / (2 * ns))];
            const float2 v = make_float2(bb.x * w.x - bb.y * w.y, bb.x * w.y + bb.y * w.x);
            const int d = f * N + 2 * (j - k) + k;
            out[d] = make_float2(a.x + v.x, a.y + v.y);
            out[d + ns] = make_float2(a.x - v.x, a.y - v.y);
        }
        __syncthreads();
        src ^= 1;
    }

    // weights and the channel rows of the block's frames
    const float2 *ws = weights ? weights + (size_t)stream * N : nullptr;
    float2 *ys = y + ((size_t)stream * T + f0) * N;
    for (int q = tid; q < nf * N; q += THREADS) {
        float2 v = buf[src][q];
        if (ws) {
            const float2 w = ws[q & (N - 1)];
            v = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
        }
        ys[q] = v;
    }
}

template <int N>
hipError_t launch_filter_fft(const void *z, const float *taps, const void *weights, const float2 *twiddle, void *y,
                             int streams, int M, int n_in, int T, hipStream_t stream) {
    const dim3 grid((T + Geo<N>::FB - 1) / Geo<N>::FB, streams);
    hipLaunchKernelGGL(filter_fft<N>, grid, dim3(THREADS), 0, stream, static_cast<const float2 *>(z), taps,
                       static_cast<const float2 *>(weights), twiddle, static_cast<float2 *>(y), M, n_in, T);
    return hipGetLastError();
}

}  // namespace pfb
}  // namespace xc

using namespace xc;

struct xc_pfb {
    int32_t S, P, N, M, n_in, T;
    void *inter = nullptr;       // y[stream][t][k]
    float2 *twiddle = nullptr;   // exp(-2 pi i j / N), j < N / 2
};

static void pfb_free(xc_pfb *p) {
    if (p->inter) (void)hipFree(p->inter);
    if (p->twiddle) (void)hipFree(p->twiddle);
    delete p;
}

extern "C" {

xc_status xc_pfb_create(int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_taps, int64_t n_in,
                        xc_pfb **out) {
    if (!out) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    if (n_pol != 2) return set_error(XC_ERR_UNSUPPORTED, "n_pol = %d: only dual-polarised stations (2) are supported",
                                     n_pol);
    if (n_stations < 1 || n_stations > 16384)       // streams index the grid's y dimension
        return set_error(XC_ERR_INVALID_ARG, "n_stations = %d outside 1 .. 16384", n_stations);
    if (n_channels != 256 && n_channels != 512)
        return set_error(XC_ERR_UNSUPPORTED, "n_channels = %d: the filter bank takes 256 or 512 channels", n_channels);
    if (n_taps < 1 || n_taps > pfb::MAX_TAPS)
        return set_error(XC_ERR_INVALID_ARG, "n_taps = %d outside 1 .. %d", n_taps, pfb::MAX_TAPS);
    if (n_in < (int64_t)n_taps * n_channels || n_in > ((int64_t)1 << 31) - 1)
        return set_error(XC_ERR_INVALID_ARG, "n_in = %lld: need n_taps * n_channels .. 2^31 - 1 samples",
                         (long long)n_in);
    xc_pfb *p = new xc_pfb;
    p->S = n_stations;
    p->P = n_pol;
    p->N = n_channels;
    p->M = n_taps;
    p->n_in = (int32_t)n_in;
    p->T = (int32_t)(n_in / n_channels) - n_taps + 1;
    const size_t inter = (size_t)n_stations * n_pol * p->T * n_channels * sizeof(float2);
    std::vector<float2> tw(n_channels / 2);
    for (int j = 0; j < n_channels / 2; ++j) {
        const double a = -2.0 * M_PI * j / n_channels;
        tw[j] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    hipError_t e = hipMalloc(&p->inter, inter);
    if (e == hipSuccess) e = hipMalloc(&p->twiddle, tw.size() * sizeof(float2));
    if (e == hipSuccess) e = hipMemcpy(p->twiddle, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        pfb_free(p);
        return e == hipErrorOutOfMemory ? set_error(XC_ERR_OUT_OF_MEMORY, "filter-bank buffer of %zu bytes", inter)
                                        : hip_error(e, "filter-bank setup");
    }
    *out = p;
    return XC_OK;
}

xc_status xc_pfb_info(const xc_pfb *p, int32_t *n_frames, int64_t *device_bytes) {
    if (!p) return set_error(XC_ERR_INVALID_ARG, "null filter bank");
    if (n_frames) *n_frames = p->T;
    if (device_bytes)
        *device_bytes = (int64_t)p->S * p->P * p->T * p->N * (int64_t)sizeof(float2) +
                        (int64_t)(p->N / 2) * (int64_t)sizeof(float2);
    return XC_OK;
}

xc_status xc_pfb_run(xc_pfb *p, const void *z, const float *taps, const void *weights, void *x, void *stream) {
    if (!p) return set_error(XC_ERR_INVALID_ARG, "null filter bank");
    if (!z || !taps || !x) return set_error(XC_ERR_INVALID_ARG, "null samples, taps or output pointer");
    if (((uintptr_t)z & 7u) || ((uintptr_t)x & 7u) || ((uintptr_t)weights & 7u) || ((uintptr_t)taps & 3u))
        return set_error(XC_ERR_INVALID_ARG, "misaligned pointer (complex64: 8 bytes, taps: 4 bytes)");
    if (x == z) return set_error(XC_ERR_INVALID_ARG, "the filter bank is out of place (x == z)");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int streams = p->S * p->P;
    hipError_t e = p->N == 256 ? pfb::launch_filter_fft<256>(z, taps, weights, p->twiddle, p->inter, streams, p->M,
                                                             p->n_in, p->T, s)
                               : pfb::launch_filter_fft<512>(z, taps, weights, p->twiddle, p->inter, streams, p->M,
                                                             p->n_in, p->T, s);
    if (e != hipSuccess) return hip_error(e, "filter-bank launch");
    // corner turn: for each frame t, y[stream][t][k] -> x[k][t][stream]
    e = launch_transpose_tiles(p->inter, x, 8, streams, p->N, (int64_t)p->T * p->N, (int64_t)p->T * streams,
                               p->N, streams, p->T, s);
    if (e != hipSuccess) return hip_error(e, "corner-turn launch");
    return XC_OK;
}

void xc_pfb_destroy(xc_pfb *p) {
    if (p) pfb_free(p);
}

}  // extern "C"
