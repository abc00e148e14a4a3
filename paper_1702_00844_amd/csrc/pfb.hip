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
// FX correlator's corner turn (Section 7) is the last step.  The station-major
// form x[k][s][t][p] (the correlator's other input layout) is written by one
// kernel per channel count (filter_fft256_sm, filter_fft_sm): a workgroup
// takes both polarisations of a station, and the spectra are turned in LDS
// into per-channel runs of the block's frames, so there is no intermediate.
//
// Time-major output, two HBM-bound kernels:
//  * filter_fft: one workgroup per (station-polarisation stream, block of
//    frames); thread n owns polyphase branch n (and n + 256): its M taps and
//    the samples of the block's frames (plus the M - 1 frames after them)
//    are loaded into registers at once, coalesced (a frame is N consecutive
//    samples), so that the block waits for memory once;
//    the branch outputs of the block's frames go to LDS and are transformed
//    there: for N = 256 by a four-step 16 x 16 FFT (16-point DFTs in
//    registers, the W_256 twiddle between the passes, LDS rows padded against
//    bank conflicts), for N = 512 by a radix-2 Stockham FFT in two ping-pong
//    LDS buffers; twiddles come from a table computed on the host in double
//    precision.  The channels are then weighted and written as rows of N
//    channels per frame: y[stream][t][k].
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

// Filter and transform frames f0 .. f0 + nf - 1 of one stream zs: thread tid
// (of THREADS) owns branches tid + b THREADS.  The spectra end in
// buf[return value]; every call of a workgroup passes the same number of
// barriers (the two halves of the station-major kernel call it side by side).
template <int N>
__device__ __forceinline__ int filter_transform(const float2 *__restrict__ zs, const float *__restrict__ taps, int M,
                                                int T, int f0, int nf, const float2 *tw,
                                                float2 (*buf)[Geo<N>::FB * N], int tid) {
    typedef Geo<N> G;
    // every input sample of the block's frames (frames f0 .. f0 + nf + M - 2 of
    // the stream) is loaded at once, so that the block waits for memory once;
    // the loads are unconditional (frame indices clamped to the last frame of
    // the input, taps past M zeroed) so that the compiler issues them together
    constexpr int NZ = G::FB + MAX_TAPS - 1;
    const int last = T + M - 2;
    float h[MAX_TAPS][G::BR];
    float2 zin[NZ][G::BR];
#pragma unroll
    for (int m = 0; m < MAX_TAPS; ++m)
#pragma unroll
        for (int b = 0; b < G::BR; ++b) {
            const float v = taps[(m < M ? m : M - 1) * N + tid + b * THREADS];
            h[m][b] = m < M ? v : 0.f;
        }
#pragma unroll
    for (int i = 0; i < NZ; ++i)
#pragma unroll
        for (int b = 0; b < G::BR; ++b) {
            const int fi = f0 + i < last ? f0 + i : last;
            zin[i][b] = zs[(size_t)fi * N + tid + b * THREADS];
        }
    // filter: frame f0 + f sums taps m over the samples of frames f0 + f + m
#pragma unroll
    for (int f = 0; f < G::FB; ++f)
#pragma unroll
        for (int b = 0; b < G::BR; ++b) {
            float ur = 0.f, ui = 0.f;
#pragma unroll
            for (int m = 0; m < MAX_TAPS; ++m) {
                ur += h[m][b] * zin[f + m][b].x;
                ui += h[m][b] * zin[f + m][b].y;
            }
            if (f < nf) buf[0][f * N + tid + b * THREADS] = make_float2(ur, ui);
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
    return src;
}

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
    const int src = filter_transform<N>(z + (size_t)stream * n_in, taps, M, T, f0, nf, tw, buf, tid);

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

// Station-major output for the Stockham kernel's channel counts (512): one
// workgroup of 2 THREADS per (station, block of FB frames), its two halves
// filtering and transforming the station's two polarisation streams side by
// side; the spectra are then turned in LDS into rows of channel k (the
// block's frames x both polarisations) and leave as runs of x[k][s][t][p],
// as in filter_fft256_sm.
template <int N>
__global__ __launch_bounds__(2 * THREADS) void filter_fft_sm(const float2 *__restrict__ z,
                                                             const float *__restrict__ taps,
                                                             const float2 *__restrict__ weights,
                                                             const float2 *__restrict__ twiddle,
                                                             float2 *__restrict__ x, int S, int M, int n_in, int T,
                                                             int nfb, int nwork) {
    typedef Geo<N> G;
    constexpr int OROW = 2 * G::FB + 1;    // one channel: FB frames x 2 pols, padded by one against bank conflicts
    constexpr int NV = G::FB * N / THREADS;   // spectrum values per thread
    static_assert(N * OROW <= 2 * 2 * G::FB * N, "the channel rows fit the filter buffers");
    __shared__ __attribute__((aligned(16))) float2 buf[2][2][G::FB * N];
    __shared__ float2 tw[N / 2];
    const int tid = threadIdx.x;
    const int p = tid / THREADS;           // polarisation of this half
    const int t = tid - p * THREADS;
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    const int s = w / nfb;
    const int f0 = (w - s * nfb) * G::FB;
    const int nf = T - f0 < G::FB ? T - f0 : G::FB;
    const int stream = 2 * s + p;
    for (int i = tid; i < N / 2; i += 2 * THREADS) tw[i] = twiddle[i];
    __syncthreads();
    const int src = filter_transform<N>(z + (size_t)stream * n_in, taps, M, T, f0, nf, tw, buf[p], t);
    // this half's spectra (weighted) into registers, then the channel rows in their place
    const float2 *ws = weights ? weights + (size_t)stream * N : nullptr;
    float2 v[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int q = t + i * THREADS;      // frame q / N, channel q % N
        float2 a = make_float2(0.f, 0.f);
        if (q < nf * N) {
            a = buf[p][src][q];
            if (ws) {
                const float2 c = ws[q & (N - 1)];
                a = make_float2(a.x * c.x - a.y * c.y, a.x * c.y + a.y * c.x);
            }
        }
        v[i] = a;
    }
    __syncthreads();
    float2 *img = &buf[0][0][0];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const int q = t + i * THREADS;
        if (q < nf * N) img[(q & (N - 1)) * OROW + 2 * (q / N) + p] = v[i];
    }
    __syncthreads();
    // channel k, frame r: both polarisations, 16 bytes
    float2 *xs = x + ((size_t)s * T + f0) * 2;
    const size_t kstride = (size_t)S * T * 2;
    for (int e = tid; e < N * G::FB; e += 2 * THREADS) {
        const int k = e / G::FB, r = e - k * G::FB;
        if (r < nf) {
            const float2 v0 = img[k * OROW + 2 * r], v1 = img[k * OROW + 2 * r + 1];
            *reinterpret_cast<float4 *>(xs + k * kstride + 2 * r) = make_float4(v0.x, v0.y, v1.x, v1.y);
        }
    }
}

// ---- 256 channels: the FFT as 16 x 16 (four-step), 16-point DFTs in registers
//
// With n = 16 n1 + n2 and k = k1 + 16 k2:
//   X[k1 + 16 k2] = sum_n2 W16^(n2 k2) W256^(n2 k1) sum_n1 W16^(n1 k1) u[16 n1 + n2].
// Pass 1: thread (frame, n2) takes the 16-point DFT over n1, multiplies by
// W256^(n2 k1) and writes the results back over its own inputs; pass 2:
// thread (frame, k1) takes the 16-point DFT over n2 and writes its channels
// k1 + 16 k2 (16 consecutive channels per 16 lanes).  LDS rows of 16
// elements are padded by one element so that both passes are free of bank
// conflicts.  Two barriers instead of eight LDS passes.

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// exp(-2 pi i m / 16)
__constant__ float2 W16[16] = {
    {1.000000000f, -0.000000000f},
    {0.923879533f, -0.382683432f},
    {0.707106781f, -0.707106781f},
    {0.382683432f, -0.923879533f},
    {0.000000000f, -1.000000000f},
    {-0.382683432f, -0.923879533f},
    {-0.707106781f, -0.707106781f},
    {-0.923879533f, -0.382683432f},
    {-1.000000000f, -0.000000000f},
    {-0.923879533f, 0.382683432f},
    {-0.707106781f, 0.707106781f},
    {-0.382683432f, 0.923879533f},
    {-0.000000000f, 1.000000000f},
    {0.382683432f, 0.923879533f},
    {0.707106781f, 0.707106781f},
    {0.923879533f, 0.382683432f}
};

// In-place forward 4-point DFT: (a, b, c, d) -> (X0, X1, X2, X3).
__device__ __forceinline__ void dft4(float2 &a, float2 &b, float2 &c, float2 &d) {
    const float2 s0 = make_float2(a.x + c.x, a.y + c.y), s1 = make_float2(a.x - c.x, a.y - c.y);
    const float2 s2 = make_float2(b.x + d.x, b.y + d.y), s3 = make_float2(b.x - d.x, b.y - d.y);
    a = make_float2(s0.x + s2.x, s0.y + s2.y);
    c = make_float2(s0.x - s2.x, s0.y - s2.y);
    b = make_float2(s1.x + s3.y, s1.y - s3.x);    // s1 - i s3
    d = make_float2(s1.x - s3.y, s1.y + s3.x);    // s1 + i s3
}

// In-place forward 16-point DFT, natural order in and out (4 x 4 steps).
__device__ __forceinline__ void dft16(float2 (&x)[16]) {
    float2 t[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        float2 a = x[n2], b = x[4 + n2], c = x[8 + n2], d = x[12 + n2];
        dft4(a, b, c, d);
        t[4 * n2 + 0] = a;
        t[4 * n2 + 1] = cmul(b, W16[n2]);
        t[4 * n2 + 2] = cmul(c, W16[2 * n2]);
        t[4 * n2 + 3] = cmul(d, W16[3 * n2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 a = t[k1], b = t[4 + k1], c = t[8 + k1], d = t[12 + k1];
        dft4(a, b, c, d);
        x[k1] = a;
        x[k1 + 4] = b;
        x[k1 + 8] = c;
        x[k1 + 12] = d;
    }
}

__global__ __launch_bounds__(THREADS) void filter_fft256(const float2 *__restrict__ z, const float *__restrict__ taps,
                                                         const float2 *__restrict__ weights,
                                                         const float2 *__restrict__ twiddle, float2 *__restrict__ y,
                                                         int M, int n_in, int T, int nfb, int nwork) {
    constexpr int N = 256, FB = 16, PAD = 17, FROW = 16 * PAD;
    __shared__ __attribute__((aligned(16))) float2 buf[FB * FROW];
    __shared__ float2 tw[N / 2];
    const int tid = threadIdx.x;
    // consecutive frame blocks of a stream on one XCD: the M - 1 frames a block
    // shares with the next one are then read from that XCD's L2
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    const int stream = w / nfb;
    const int f0 = (w - stream * nfb) * FB;
    const int nf = T - f0 < FB ? T - f0 : FB;
    for (int i = tid; i < N / 2; i += THREADS) tw[i] = twiddle[i];

    // filter, as in the general kernel: all inputs of the block loaded at once
    const float2 *zs = z + (size_t)stream * n_in;
    constexpr int NZ = FB + MAX_TAPS - 1;
    const int last = T + M - 2;
    float h[MAX_TAPS];
    float2 zin[NZ];
#pragma unroll
    for (int m = 0; m < MAX_TAPS; ++m) {
        const float v = taps[(m < M ? m : M - 1) * N + tid];
        h[m] = m < M ? v : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NZ; ++i) zin[i] = zs[(size_t)(f0 + i < last ? f0 + i : last) * N + tid];
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        float ur = 0.f, ui = 0.f;
#pragma unroll
        for (int m = 0; m < MAX_TAPS; ++m) {
            ur += h[m] * zin[f + m].x;
            ui += h[m] * zin[f + m].y;
        }
        if (f < nf) buf[f * FROW + tid + (tid >> 4)] = make_float2(ur, ui);
    }
    __syncthreads();

    const int f = tid >> 4, q = tid & 15;
    float2 a[16];
    if (f < nf) {
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = buf[f * FROW + PAD * i + q];       // u[16 i + q]
        dft16(a);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            const int j = q * k1;                                              // W256^j, j <= 225
            const float2 w = j < N / 2 ? tw[j] : make_float2(-tw[j - N / 2].x, -tw[j - N / 2].y);
            buf[f * FROW + PAD * k1 + q] = cmul(a[k1], w);
        }
    }
    __syncthreads();
    if (f < nf) {
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = buf[f * FROW + PAD * q + i];       // pass-1 output n2 = i, k1 = q
        dft16(a);
        float2 *yr = y + ((size_t)stream * T + f0 + f) * N;
        const float2 *ws = weights ? weights + (size_t)stream * N : nullptr;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            const int k = q + 16 * k2;
            yr[k] = ws ? cmul(a[k2], ws[k]) : a[k2];
        }
    }
}

// Station-major output for 256 channels: one workgroup per (station, block of
// 16 frames).  Its two halves filter and transform the station's two
// polarisation streams exactly as filter_fft256 does; the spectra are then
// turned in LDS into rows of channel k holding the block's frames and both
// polarisations, so that each channel leaves as one 256-byte run of
// x[k][s][t][p], the layout the correlator takes as station-major input:
// no intermediate, no corner turn.
__global__ __launch_bounds__(2 * THREADS) void filter_fft256_sm(const float2 *__restrict__ z,
                                                              const float *__restrict__ taps,
                                                              const float2 *__restrict__ weights,
                                                              const float2 *__restrict__ twiddle,
                                                              float2 *__restrict__ x, int S, int M, int n_in, int T,
                                                              int nfb, int nwork) {
    constexpr int N = 256, FB = 16, PAD = 17, FROW = 16 * PAD;
    constexpr int OROW = 2 * FB + 1;    // one channel: FB frames x 2 pols, padded by one against bank conflicts
    static_assert(N * OROW <= 2 * FB * FROW, "the channel rows fit the two filter buffers");
    __shared__ __attribute__((aligned(16))) float2 buf[2 * FB * FROW];
    __shared__ float2 tw[N / 2];
    const int tid = threadIdx.x;
    const int p = tid >> 8;             // polarisation of this half
    const int n = tid & (N - 1);        // branch
    // consecutive frame blocks of a station on one XCD (their inputs overlap by M - 1 frames)
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    const int s = w / nfb;
    const int f0 = (w - s * nfb) * FB;
    const int nf = T - f0 < FB ? T - f0 : FB;
    const int stream = 2 * s + p;
    for (int i = tid; i < N / 2; i += 2 * THREADS) tw[i] = twiddle[i];
    float2 *pb = buf + p * (FB * FROW);

    const float2 *zs = z + (size_t)stream * n_in;
    constexpr int NZ = FB + MAX_TAPS - 1;
    const int last = T + M - 2;
    float h[MAX_TAPS];
    float2 zin[NZ];
#pragma unroll
    for (int m = 0; m < MAX_TAPS; ++m) {
        const float v = taps[(m < M ? m : M - 1) * N + n];
        h[m] = m < M ? v : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NZ; ++i) zin[i] = zs[(size_t)(f0 + i < last ? f0 + i : last) * N + n];
#pragma unroll
    for (int f = 0; f < FB; ++f) {
        float ur = 0.f, ui = 0.f;
#pragma unroll
        for (int m = 0; m < MAX_TAPS; ++m) {
            ur += h[m] * zin[f + m].x;
            ui += h[m] * zin[f + m].y;
        }
        if (f < nf) pb[f * FROW + n + (n >> 4)] = make_float2(ur, ui);
    }
    __syncthreads();

    const int f = n >> 4, q = n & 15;
    float2 a[16];
    if (f < nf) {
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = pb[f * FROW + PAD * i + q];        // u[16 i + q]
        dft16(a);
#pragma unroll
        for (int k1 = 0; k1 < 16; ++k1) {
            const int j = q * k1;                                              // W256^j, j <= 225
            const float2 t = j < N / 2 ? tw[j] : make_float2(-tw[j - N / 2].x, -tw[j - N / 2].y);
            pb[f * FROW + PAD * k1 + q] = cmul(a[k1], t);
        }
    }
    __syncthreads();
    if (f < nf) {
#pragma unroll
        for (int i = 0; i < 16; ++i) a[i] = pb[f * FROW + PAD * q + i];        // pass-1 output n2 = i, k1 = q
        dft16(a);
    }
    __syncthreads();    // both halves are done with their buffers: the channel rows take their place
    if (f < nf) {
        const float2 *ws = weights ? weights + (size_t)stream * N : nullptr;
#pragma unroll
        for (int k2 = 0; k2 < 16; ++k2) {
            const int k = q + 16 * k2;
            buf[k * OROW + 2 * f + p] = ws ? cmul(a[k2], ws[k]) : a[k2];
        }
    }
    __syncthreads();
    // channel k, frame r: both polarisations, 16 bytes; a wave writes four channels' runs
    float2 *xs = x + ((size_t)s * T + f0) * 2;
    const size_t kstride = (size_t)S * T * 2;
    for (int e = tid; e < N * FB; e += 2 * THREADS) {
        const int k = e >> 4, r = e & 15;
        if (r < nf) {
            const float2 v0 = buf[k * OROW + 2 * r], v1 = buf[k * OROW + 2 * r + 1];
            *reinterpret_cast<float4 *>(xs + k * kstride + 2 * r) = make_float4(v0.x, v0.y, v1.x, v1.y);
        }
    }
}

template <int N>
hipError_t launch_filter_fft_sm(const void *z, const float *taps, const void *weights, const float2 *twiddle, void *x,
                                int S, int M, int n_in, int T, hipStream_t stream) {
    const int nfb = (T + Geo<N>::FB - 1) / Geo<N>::FB;
    const int64_t nwork = (int64_t)nfb * S;
    if (nwork > ((int64_t)1 << 31) - kNumXcd) return hipErrorInvalidValue;
    hipLaunchKernelGGL(filter_fft_sm<N>, dim3(xcd_grid((int)nwork)), dim3(2 * THREADS), 0, stream,
                       static_cast<const float2 *>(z), taps, static_cast<const float2 *>(weights), twiddle,
                       static_cast<float2 *>(x), S, M, n_in, T, nfb, (int)nwork);
    return hipGetLastError();
}

hipError_t launch_filter_fft256_sm(const void *z, const float *taps, const void *weights, const float2 *twiddle,
                                   void *x, int S, int M, int n_in, int T, hipStream_t stream) {
    const int nfb = (T + 15) / 16;
    const int64_t nwork = (int64_t)nfb * S;
    if (nwork > ((int64_t)1 << 31) - kNumXcd) return hipErrorInvalidValue;
    hipLaunchKernelGGL(filter_fft256_sm, dim3(xcd_grid((int)nwork)), dim3(2 * THREADS), 0, stream,
                       static_cast<const float2 *>(z), taps, static_cast<const float2 *>(weights), twiddle,
                       static_cast<float2 *>(x), S, M, n_in, T, nfb, (int)nwork);
    return hipGetLastError();
}

template <int N>
hipError_t launch_filter_fft(const void *z, const float *taps, const void *weights, const float2 *twiddle, void *y,
                             int streams, int M, int n_in, int T, hipStream_t stream) {
    if constexpr (N == 256) {
        const int nfb = (T + 15) / 16;
        const int64_t nwork = (int64_t)nfb * streams;
        if (nwork > ((int64_t)1 << 31) - kNumXcd) return hipErrorInvalidValue;
        hipLaunchKernelGGL(filter_fft256, dim3(xcd_grid((int)nwork)), dim3(THREADS), 0, stream,
                           static_cast<const float2 *>(z), taps, static_cast<const float2 *>(weights), twiddle,
                           static_cast<float2 *>(y), M, n_in, T, nfb, (int)nwork);
    } else {
        const dim3 grid((T + Geo<N>::FB - 1) / Geo<N>::FB, streams);
        hipLaunchKernelGGL(filter_fft<N>, grid, dim3(THREADS), 0, stream, static_cast<const float2 *>(z), taps,
                           static_cast<const float2 *>(weights), twiddle, static_cast<float2 *>(y), M, n_in, T);
    }
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
    {
        const int64_t T = n_in / n_channels - n_taps + 1;
        if ((T + 15) / 16 * 2 * (int64_t)n_stations > ((int64_t)1 << 31) - 1024)
            return set_error(XC_ERR_UNSUPPORTED, "too many (stream, frame block) work units");
    }
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

xc_status xc_pfb_run_station_major(xc_pfb *p, const void *z, const float *taps, const void *weights, void *x,
                                   void *stream) {
    if (!p) return set_error(XC_ERR_INVALID_ARG, "null filter bank");
    if (!z || !taps || !x) return set_error(XC_ERR_INVALID_ARG, "null samples, taps or output pointer");
    if (((uintptr_t)z & 7u) || ((uintptr_t)x & 15u) || ((uintptr_t)weights & 7u) || ((uintptr_t)taps & 3u))
        return set_error(XC_ERR_INVALID_ARG,
                         "misaligned pointer (samples and weights: 8 bytes, output: 16 bytes, taps: 4 bytes)");
    if (x == z) return set_error(XC_ERR_INVALID_ARG, "the filter bank is out of place (x == z)");
    hipError_t e = p->N == 256 ? pfb::launch_filter_fft256_sm(z, taps, weights, p->twiddle, x, p->S, p->M, p->n_in,
                                                              p->T, static_cast<hipStream_t>(stream))
                               : pfb::launch_filter_fft_sm<512>(z, taps, weights, p->twiddle, x, p->S, p->M,
                                                                p->n_in, p->T, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_error(e, "filter-bank launch");
    return XC_OK;
}

void xc_pfb_destroy(xc_pfb *p) {
    if (p) pfb_free(p);
}

}  // extern "C"
