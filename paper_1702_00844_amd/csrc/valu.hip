// FP32 vector-ALU correlator kernel (complex-float samples, complex-float output).
//
// Structure, following Section 2 of the paper (register tiles of the
// correlation triangle, reuse between tiles through a shared on-chip store):
//
//  * The triangle of station pairs is split into square blocks of SB = 32
//    stations (Section 4.5 blocks large triangles the same way).  One
//    workgroup owns one (channel, block pair bi <= bj).
//  * Each lane of a wave owns a 4 x 4 tile of station pairs (Table 1: 512
//    flops per 128 bytes of samples, 148 registers minimum) and keeps its 64
//    complex accumulators (4 x 4 stations x 2 x 2 polarisations) in registers.
//    The 64 lanes cover the 8 x 8 tiles of a 32 x 32 block pair.
//  * Samples of both blocks are staged through LDS per chunk of TC time steps,
//    loaded with coalesced 16-byte reads of the time-major layout (all stations
//    of one time step together, Section 4.4) and double-buffered through
//    registers: the next chunk's global loads are in flight while the current
//    chunk is correlated.
//  * TS waves share the block pair; wave w integrates time steps
//    [w TC/TS, (w+1) TC/TS) of every chunk.  Their partial sums are added in
//    LDS after the last chunk, in a fixed order (deterministic), and wave 0
//    stores each visibility once.
//  * One complex multiply-accumulate is four FMAs (Section 2):
//    re += a_r b_r + a_i b_i ; im += a_i b_r - a_r b_i.
//  * Autocorrelations (i == j) are written Hermitian by construction: XX and
//    YY get imaginary part 0 and YX is stored as conj(XY).
#include "common.h"

namespace xc {
namespace valu {

constexpr int SB = 32;            // stations per block
constexpr int TW = 4;             // tile: stations of block I per lane
constexpr int TH = 4;             // tile: stations of block J per lane
constexpr int ROW = 2 * SB + 4;   // float4 slots per staged time step (+1 pad per 16 stations)
constexpr int NACC = TW * TH * 8; // floats of accumulators per lane

// Slot of staged station s in [0, 2 SB): one pad slot after every 16 stations
// so that the 8 distinct tile rows read by a quarter-wave hit distinct banks.
__device__ __forceinline__ int slot(int s) { return s + (s >> 4); }

template <int TC>
struct Stage {
    float4 v[2][TC][ROW];
};

__device__ __forceinline__ void cmac(float &re, float &im, float ar, float ai, float br, float bi) {
    re = fmaf(ar, br, re);
    re = fmaf(ai, bi, re);
    im = fmaf(ai, br, im);
    im = fmaf(-ar, bi, im);
}

template <int TS, int TC>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, Stage<TC> &st) {
    static_assert(TC % TS == 0, "time chunk must split evenly over waves");
    static_assert(sizeof(Stage<TC>) >= 64 * NACC * sizeof(float), "reduction area too small");
    constexpr int NT = 64 * TS;
    constexpr int NELEM = TC * 2 * SB;
    constexpr int NLOAD = (NELEM + NT - 1) / NT;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform across the wave
    const int ti = lane & 7;
    const int tj = lane >> 3;
    const int S = job.S;
    const int T = job.T;
    const bool diag = (bi == bj);
    const int I0 = bi * SB;
    const int J0 = bj * SB;
    const bool active = !(diag && ti > tj);
    const int jbase = diag ? 0 : SB;
    const float4 *__restrict__ x = static_cast<const float4 *>(job.x);

    float acc[NACC];
#pragma unroll
    for (int f = 0; f < NACC; ++f) acc[f] = 0.f;

    float4 pre[NLOAD];
    auto gload = [&](int t0) {
#pragma unroll
        for (int k = 0; k < NLOAD; ++k) {
            const int e = tid + k * NT;
            const int t = e / (2 * SB);
            const int s = e % (2 * SB);
            const int station = s < SB ? I0 + s : J0 + s - SB;
            const bool ok = (e < NELEM) && (t0 + t < T) && station < S && !(diag && s >= SB);
            // time-major: all stations of a time step together; station-major
            // (sstride != 0): each station's series together
            const size_t e_x = job.sstride ? (size_t)c * job.cstride + (size_t)station * job.sstride + (t0 + t)
                                           : row_offset(job, c, t0 + t) + station;
            pre[k] = ok ? x[e_x] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int k = 0; k < NLOAD; ++k) {
            const int e = tid + k * NT;
            const int t = e / (2 * SB);
            const int s = e % (2 * SB);
            if (e < NELEM && !(diag && s >= SB)) st.v[buf][t][slot(s)] = pre[k];
        }
    };

    const int nchunk = (T + TC - 1) / TC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) gload((ch + 1) * TC);
        if (active) {
            const int tbeg = wave * (TC / TS);
            for (int tt = tbeg; tt < tbeg + TC / TS; ++tt) {
                float4 a[TW], b[TH];
#pragma unroll
                for (int i = 0; i < TW; ++i) a[i] = st.v[buf][tt][slot(ti * TW + i)];
#pragma unroll
                for (int j = 0; j < TH; ++j) b[j] = st.v[buf][tt][slot(jbase + tj * TH + j)];
#pragma unroll
                for (int i = 0; i < TW; ++i) {
#pragma unroll
                    for (int j = 0; j < TH; ++j) {
                        float *r = &acc[(i * TH + j) * 8];
                        // pol p of station i: (x, y) = X, (z, w) = Y; same for q of station j
                        cmac(r[0], r[1], a[i].x, a[i].y, b[j].x, b[j].y);  // XX
                        cmac(r[2], r[3], a[i].x, a[i].y, b[j].z, b[j].w);  // XY
                        cmac(r[4], r[5], a[i].z, a[i].w, b[j].x, b[j].y);  // YX
                        cmac(r[6], r[7], a[i].z, a[i].w, b[j].z, b[j].w);  // YY
                    }
                }
            }
        }
        if (ch + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }

    // Add the partial sums of waves 1..TS-1 into wave 0, one wave per round.
    if constexpr (TS > 1) {
        float *red = reinterpret_cast<float *>(&st.v[0][0][0]);
#pragma unroll 1
        for (int w = 1; w < TS; ++w) {
            if (wave == w) {
#pragma unroll
                for (int f = 0; f < NACC; ++f) red[f * 64 + lane] = acc[f];
            }
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int f = 0; f < NACC; ++f) acc[f] += red[f * 64 + lane];
            }
            __syncthreads();
        }
    }

    if (wave != 0 || !active) return;
    float4 *__restrict__ V = static_cast<float4 *>(job.vis) + (size_t)c * ((size_t)S * (S + 1) / 2) * 2;
#pragma unroll
    for (int j = 0; j < TH; ++j) {
        const int jj = J0 + tj * TH + j;
        if (jj >= S) continue;
#pragma unroll
        for (int i = 0; i < TW; ++i) {
            const int ii = I0 + ti * TW + i;
            if (ii > jj) continue;
            const float *r = &acc[(i * TH + j) * 8];
            float4 v0 = make_float4(r[0], r[1], r[2], r[3]);
            float4 v1 = make_float4(r[4], r[5], r[6], r[7]);
            if (ii == jj) {  // Hermitian autocorrelation block
                v0.y = 0.f;
                v1.w = 0.f;
                v1.x = v0.z;
                v1.y = -v0.w;
            }
            const size_t bl = (size_t)jj * (jj + 1) / 2 + ii;
            if (job.accumulate) {
                const float4 o0 = V[2 * bl], o1 = V[2 * bl + 1];
                v0.x += o0.x; v0.y += o0.y; v0.z += o0.z; v0.w += o0.w;
                v1.x += o1.x; v1.y += o1.y; v1.z += o1.z; v1.w += o1.w;
            }
            V[2 * bl] = v0;
            V[2 * bl + 1] = v1;
        }
    }
}

template <int TS, int TC>
__global__ __launch_bounds__(64 * TS) void kernel(Job job, int nwork) {
    __shared__ Stage<TC> st;
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    int c, bi, bj;
    unit_decode(job, w, c, bi, bj);
    unit<TS, TC>(job, c, bi, bj, st);
}

// Batch form: one workgroup per unit of a batch's unit list.
template <int TS, int TC>
__global__ __launch_bounds__(64 * TS) void kernel_batch(const Job *__restrict__ jobs,
                                                         const Unit *__restrict__ units, const int *__restrict__ bounds) {
    __shared__ Stage<TC> st;
    const int u = batch_unit(bounds, blockIdx.x);
    if (u < 0) return;
    const Unit un = units[u];
    const Job job = jobs[un.item];
    unit<TS, TC>(job, un.channel, un.bi, un.bj, st);
}

template <int TS, int TC>
hipError_t launch_t(const Job &job, hipStream_t stream) {
    const int nwork = job_units(job);
    hipLaunchKernelGGL((kernel<TS, TC>), dim3(xcd_grid(nwork)), dim3(64 * TS), 0, stream, job, nwork);
    return hipGetLastError();
}

template <int TS, int TC>
hipError_t launch_batch_t(const Job *jobs, const Unit *units, const int *bounds, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((kernel_batch<TS, TC>), dim3(grid), dim3(64 * TS), 0, stream, jobs, units, bounds);
    return hipGetLastError();
}

}  // namespace valu

hipError_t launch_valu(const Plan &plan, const Job &job, hipStream_t stream) {
    const int ts = plan.time_split, tc = plan.time_chunk;
    if (ts == 1 && tc == 16) return valu::launch_t<1, 16>(job, stream);
    if (ts == 2 && tc == 16) return valu::launch_t<2, 16>(job, stream);
    if (ts == 4 && tc == 16) return valu::launch_t<4, 16>(job, stream);
    if (ts == 2 && tc == 32) return valu::launch_t<2, 32>(job, stream);
    if (ts == 4 && tc == 32) return valu::launch_t<4, 32>(job, stream);
    if (ts == 8 && tc == 32) return valu::launch_t<8, 32>(job, stream);
    return hipErrorInvalidValue;
}

hipError_t launch_valu_batch(const Plan &plan, const Job *jobs, const Unit *units, const int *bounds, int grid,
                             hipStream_t stream) {
    const int ts = plan.time_split, tc = plan.time_chunk;
    if (ts == 1 && tc == 16) return valu::launch_batch_t<1, 16>(jobs, units, bounds, grid, stream);
    if (ts == 2 && tc == 16) return valu::launch_batch_t<2, 16>(jobs, units, bounds, grid, stream);
    if (ts == 4 && tc == 16) return valu::launch_batch_t<4, 16>(jobs, units, bounds, grid, stream);
    if (ts == 2 && tc == 32) return valu::launch_batch_t<2, 32>(jobs, units, bounds, grid, stream);
    if (ts == 4 && tc == 32) return valu::launch_batch_t<4, 32>(jobs, units, bounds, grid, stream);
    if (ts == 8 && tc == 32) return valu::launch_batch_t<8, 32>(jobs, units, bounds, grid, stream);
    return hipErrorInvalidValue;
}

}  // namespace xc
