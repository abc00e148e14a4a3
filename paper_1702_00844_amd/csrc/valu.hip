// FP32 vector-ALU correlator kernel (complex-float samples, complex-float output).
//
// Structure, following Section 2 of the paper (register tiles of the
// correlation triangle, reuse between tiles through a shared on-chip store):
//
//  * The triangle of station pairs is split into square blocks of SB = 32
//    stations (Section 4.5 blocks large triangles the same way).  One
//    workgroup owns one (channel, block pair bi <= bj).
//  * Each lane owns a TW x TH tile of station pairs (TW stations of block I,
//    TH of block J; Table 1: 32 TW TH flops per 16 (TW + TH) bytes of samples,
//    4 (1 + min(TW, TH)) + 8 TW TH registers minimum) and keeps its 4 TW TH
//    complex accumulators (stations x 2 x 2 polarisations) in registers.  The
//    (32 / TW) (32 / TH) lanes of a time group cover the tiles of a 32 x 32
//    block pair (one wave for 4 x 4 and 8 x 2 tiles, two for 4 x 2, four for
//    2 x 2).  The auto-tuner chooses the tile per shape among those whose
//    Table 1 register count fits the register file.
//  * Samples of both blocks are staged through LDS per chunk of TC time steps,
//    loaded with coalesced 16-byte reads of the time-major layout (all stations
//    of one time step together, Section 4.4) and double-buffered through
//    registers: the next chunk's global loads are in flight while the current
//    chunk is correlated.
//  * TS time groups share the block pair; group g integrates time steps
//    [g TC/TS, (g+1) TC/TS) of every chunk.  Their partial sums are added in
//    LDS after the last chunk, in a fixed order (deterministic), and group 0
//    stores each visibility once.
//  * One complex multiply-accumulate is four FMAs (Section 2):
//    re += a_r b_r + a_i b_i ; im += a_i b_r - a_r b_i.
//  * Autocorrelations (i == j) are written Hermitian by construction: XX and
//    YY get imaginary part 0 and YX is stored as conj(XY).
//  * A diagonal block pair (I = J) has outputs in only NA of its tiles (those
//    holding some pair i <= j: 72 of 128 for 4 x 2 tiles).  Rather than
//    leaving the other lanes masked inside their waves, the workgroup's
//    threads are packed as (active tile, time group) tasks: G = threads / NA
//    time groups (7 for 4 x 2 tiles and 512 threads), each taking TCD / G time
//    steps of chunks of TCD steps of the one staged block (a row of one block
//    is half a pair's row, so the stage holds up to 2 TC of them).  The
//    groups' sums are added in a fixed order as for the off-diagonal pairs.
#include "common.h"

namespace xc {
namespace valu {

constexpr int SB = 32;            // stations per block
constexpr int ROW = 2 * SB + 4;   // float4 slots per staged time step (+1 pad per 16 stations)

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

// Lanes of one time group: one per tile of the block pair.
template <int TW, int TH>
constexpr int lanes() { return (SB / TW) * (SB / TH); }

// Tiles of a diagonal block pair that hold some output pair i <= j: in
// column tj, tile rows ti with ti TW <= tj TH + TH - 1; and in all.
template <int TW, int TH>
__host__ __device__ constexpr int diag_col_tiles(int tj) {
    const int n = (tj * TH + TH - 1) / TW + 1;
    return n < SB / TW ? n : SB / TW;
}
template <int TW, int TH>
constexpr int diag_tiles() {
    int n = 0;
    for (int tj = 0; tj < SB / TH; ++tj) n += diag_col_tiles<TW, TH>(tj);
    return n;
}

template <int TW, int TH>
__device__ __forceinline__ void cmac_tile(float *acc, const float4 (&a)[TW], const float4 (&b)[TH]) {
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

// Store (or add, in accumulate mode) one lane's TW x TH tile of block pair
// (I0, J0); pairs past the last station or below the diagonal are skipped.
template <int TW, int TH>
__device__ __forceinline__ void store_lane_tile(const Job &job, int c, const float *acc, int I0, int J0, int ti,
                                                int tj) {
    const int S = job.S;
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

// Diagonal block pair b: (active tile, time group) tasks packed over the
// workgroup's threads.
template <int TW, int TH, int TS, int TC>
__device__ __forceinline__ void unit_diag(const Job &job, int c, int b, Stage<TC> &st) {
    constexpr int NACC = TW * TH * 8;
    constexpr int NT = lanes<TW, TH>() * TS;
    constexpr int NA = diag_tiles<TW, TH>();
    constexpr int G = NT / NA;                     // time groups
    constexpr int TCD = G * ((2 * TC) / G);        // time steps per chunk
    constexpr int STEPS = TCD / G;                 // time steps per group and chunk
    constexpr int DROW = SB + SB / 16;             // float4 slots per staged time step of one block
    constexpr int NELEM = TCD * SB;
    constexpr int NLOAD = (NELEM + NT - 1) / NT;
    static_assert(G >= 1 && STEPS >= 1, "at least one time group and step");
    static_assert(TCD * DROW <= TC * ROW, "a chunk must fit one staging buffer");
    static_assert(NA * NACC * sizeof(float) <= sizeof(Stage<TC>), "reduction area too small");
    static_assert(NACC % 4 == 0, "accumulators move as float4");

    const int tid = threadIdx.x;
    const int g = tid / NA;                        // time group; G: no task
    const int k = tid - g * NA;
    const bool has = g < G;
    int tj = 0, ti = k;
    while (tj < SB / TH - 1 && ti >= diag_col_tiles<TW, TH>(tj)) {
        ti -= diag_col_tiles<TW, TH>(tj);
        ++tj;
    }
    const int S = job.S;
    const int T = job.T;
    const int I0 = b * SB;
    const float4 *__restrict__ x = static_cast<const float4 *>(job.x);
    float4 *buf0 = &st.v[0][0][0];
    float4 *buf1 = &st.v[1][0][0];

    float acc[NACC];
#pragma unroll
    for (int f = 0; f < NACC; ++f) acc[f] = 0.f;

    float4 pre[NLOAD];
    auto gload = [&](int t0) {
#pragma unroll
        for (int q = 0; q < NLOAD; ++q) {
            const int e = tid + q * NT;
            const int t = e / SB;
            const int station = I0 + e % SB;
            const bool ok = (e < NELEM) && (t0 + t < T) && station < S;
            const size_t e_x = job.sstride ? (size_t)c * job.cstride + (size_t)station * job.sstride + (t0 + t)
                                           : row_offset(job, c, t0 + t) + station;
            pre[q] = ok ? x[e_x] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto lstore = [&](float4 *dst) {
#pragma unroll
        for (int q = 0; q < NLOAD; ++q) {
            const int e = tid + q * NT;
            if (e < NELEM) dst[(e / SB) * DROW + slot(e % SB)] = pre[q];
        }
    };

    const int nchunk = (T + TCD - 1) / TCD;
    gload(0);
    lstore(buf0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const float4 *cur = (ch & 1) ? buf1 : buf0;
        if (ch + 1 < nchunk) gload((ch + 1) * TCD);
        if (has) {
            const float4 *row = cur + g * STEPS * DROW;
#pragma unroll 1
            for (int tt = 0; tt < STEPS; ++tt, row += DROW) {
                float4 a[TW], bb[TH];
#pragma unroll
                for (int i = 0; i < TW; ++i) a[i] = row[slot(ti * TW + i)];
#pragma unroll
                for (int j = 0; j < TH; ++j) bb[j] = row[slot(tj * TH + j)];
                cmac_tile<TW, TH>(acc, a, bb);
            }
        }
        if (ch + 1 < nchunk) lstore((ch & 1) ? buf0 : buf1);
        __syncthreads();
    }

    // Add the sums of groups 1 .. G - 1 into group 0, one group per round.
    if constexpr (G > 1) {
        float4 *red = buf0;
#pragma unroll 1
        for (int w = 1; w < G; ++w) {
            if (g == w) {
#pragma unroll
                for (int f = 0; f < NACC / 4; ++f)
                    red[f * NA + k] = make_float4(acc[4 * f], acc[4 * f + 1], acc[4 * f + 2], acc[4 * f + 3]);
            }
            __syncthreads();
            if (g == 0) {
#pragma unroll
                for (int f = 0; f < NACC / 4; ++f) {
                    const float4 o = red[f * NA + k];
                    acc[4 * f] += o.x;
                    acc[4 * f + 1] += o.y;
                    acc[4 * f + 2] += o.z;
                    acc[4 * f + 3] += o.w;
                }
            }
            __syncthreads();
        }
    }
    if (g != 0) return;
    store_lane_tile<TW, TH>(job, c, acc, I0, I0, ti, tj);
}

template <int TW, int TH, int TS, int TC>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, Stage<TC> &st) {
    if (bi == bj) {
        unit_diag<TW, TH, TS, TC>(job, c, bi, st);
        return;
    }
    constexpr int NACC = TW * TH * 8;          // floats of accumulators per lane
    constexpr int NL = lanes<TW, TH>();
    static_assert(NL % 64 == 0, "a time group must be whole waves");
    static_assert(TC % TS == 0, "time chunk must split evenly over time groups");
    static_assert(sizeof(Stage<TC>) >= NL * NACC * sizeof(float), "reduction area too small");
    constexpr int NT = NL * TS;
    constexpr int NELEM = TC * 2 * SB;
    constexpr int NLOAD = (NELEM + NT - 1) / NT;

    const int tid = threadIdx.x;
    const int lane = tid % NL;                                       // tile of this lane
    const int wave = __builtin_amdgcn_readfirstlane(tid / NL);       // time group, uniform across the wave
    const int ti = lane % (SB / TW);
    const int tj = lane / (SB / TW);
    const int S = job.S;
    const int T = job.T;
    const int I0 = bi * SB;
    const int J0 = bj * SB;
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
            const bool ok = (e < NELEM) && (t0 + t < T) && station < S;
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
            if (e < NELEM) st.v[buf][t][slot(s)] = pre[k];
        }
    };

    const int nchunk = (T + TC - 1) / TC;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        if (ch + 1 < nchunk) gload((ch + 1) * TC);
        const int tbeg = wave * (TC / TS);
#pragma unroll 1
        for (int tt = tbeg; tt < tbeg + TC / TS; ++tt) {
            float4 a[TW], b[TH];
#pragma unroll
            for (int i = 0; i < TW; ++i) a[i] = st.v[buf][tt][slot(ti * TW + i)];
#pragma unroll
            for (int j = 0; j < TH; ++j) b[j] = st.v[buf][tt][slot(SB + tj * TH + j)];
            cmac_tile<TW, TH>(acc, a, b);
        }
        if (ch + 1 < nchunk) lstore(buf ^ 1);
        __syncthreads();
    }

    // Add the partial sums of time groups 1..TS-1 into group 0, one group per round.
    if constexpr (TS > 1) {
        float *red = reinterpret_cast<float *>(&st.v[0][0][0]);
#pragma unroll 1
        for (int w = 1; w < TS; ++w) {
            if (wave == w) {
#pragma unroll
                for (int f = 0; f < NACC; ++f) red[f * NL + lane] = acc[f];
            }
            __syncthreads();
            if (wave == 0) {
#pragma unroll
                for (int f = 0; f < NACC; ++f) acc[f] += red[f * NL + lane];
            }
            __syncthreads();
        }
    }

    if (wave != 0) return;
    store_lane_tile<TW, TH>(job, c, acc, I0, J0, ti, tj);
}

// Flat launch, longest units first: each XCD takes a contiguous range of
// cper channels, and its workgroups (dispatched to it in id order) run the
// off-diagonal block pairs of those channels first and the diagonal pairs
// (shorter, their threads being packed over fewer tiles) after them, so that
// the short units fill the end of the launch instead of extending it.  The
// grid is kNumXcd cper npairs; ids past the last channel return false.
__device__ inline bool longest_first(const Job &job, int phys, int cper, int &c, int &bi, int &bj) {
    const int r = phys / kNumXcd;
    const int c0 = (phys % kNumXcd) * cper;
    const int nc = job.C - c0 < cper ? job.C - c0 : cper;
    const int nb = job.nb;
    const int noff = job.npairs - nb;
    if (nc <= 0) return false;
    if (r < nc * noff) {
        int j;
        c = c0 + r / noff;
        pair_decode(r % noff, bi, j);     // off-diagonal pair m = j (j + 1) / 2 + bi: bi <= j < nb - 1
        bj = j + 1;
        return true;
    }
    const int q = r - nc * noff;
    if (q >= nc * nb) return false;
    c = c0 + q / nb;
    bi = bj = q % nb;
    return true;
}

// Channels per XCD for the longest-first order, or 0 for the plain order:
// split integrations, a single block, too few channels to give every XCD a
// whole share, or more than four blocks (diagonal pairs are then a small
// share of the work, and running a channel's pairs together keeps its
// samples in L2: on 256 stations the longest-first order read 2.2 times the
// algorithmic bytes against 1.5 for the plain order, at the same speed).
inline int longest_first_channels(const Job &job) {
    if (job.tsplit > 1 || job.nb < 2 || job.nb > 4 || job.C < 8 * kNumXcd) return 0;
    return (job.C + kNumXcd - 1) / kNumXcd;
}

template <int TW, int TH, int TS, int TC>
__global__ __launch_bounds__((lanes<TW, TH>() * TS)) void kernel(Job job, int nwork, int cper) {
    __shared__ Stage<TC> st;
    int c, bi, bj;
    if (cper > 0) {
        if (!longest_first(job, blockIdx.x, cper, c, bi, bj)) return;
    } else {
        const int w = xcd_remap(blockIdx.x, nwork);
        if (w < 0) return;
        unit_decode(job, w, c, bi, bj);
    }
    unit<TW, TH, TS, TC>(job, c, bi, bj, st);
}

// Batch form: one workgroup per unit of a batch's unit list.
template <int TW, int TH, int TS, int TC>
__global__ __launch_bounds__((lanes<TW, TH>() * TS)) void kernel_batch(const Job *__restrict__ jobs,
                                                                     const Unit *__restrict__ units,
                                                                     const int *__restrict__ bounds) {
    __shared__ Stage<TC> st;
    const int u = batch_unit(bounds, blockIdx.x);
    if (u < 0) return;
    const Unit un = units[u];
    const Job job = jobs[un.item];
    unit<TW, TH, TS, TC>(job, un.channel, un.bi, un.bj, st);
}

template <int TW, int TH, int TS, int TC>
hipError_t launch_t(const Job &job, hipStream_t stream) {
    const int nwork = job_units(job);
    const int cper = longest_first_channels(job);
    const int grid = cper > 0 ? kNumXcd * cper * job.npairs : xcd_grid(nwork);
    hipLaunchKernelGGL((kernel<TW, TH, TS, TC>), dim3(grid), dim3(lanes<TW, TH>() * TS), 0, stream, job, nwork,
                       cper);
    return hipGetLastError();
}

template <int TW, int TH, int TS, int TC>
hipError_t launch_batch_t(const Job *jobs, const Unit *units, const int *bounds, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((kernel_batch<TW, TH, TS, TC>), dim3(grid), dim3(lanes<TW, TH>() * TS), 0, stream, jobs, units,
                       bounds);
    return hipGetLastError();
}

// Every (tile, time chunk, time groups) the library builds: tiles 4 x 4,
// 8 x 2, 4 x 2 and 2 x 2 (those of Table 1's shapes that divide a 32-station
// block, whose register count leaves room for staging, and whose time groups
// are whole waves), each with the (chunk, groups) pairs below, at most 1024
// threads per workgroup.
template <int TW, int TH, typename F>
hipError_t dispatch_tc_ts(int tc, int ts, F &&f) {
    constexpr int NL = lanes<TW, TH>();
    if (tc == 16 && ts == 1) return f.template operator()<TW, TH, 1, 16>();
    if (tc == 16 && ts == 2) return f.template operator()<TW, TH, 2, 16>();
    if (tc == 16 && ts == 4) return f.template operator()<TW, TH, 4, 16>();
    if (tc == 32 && ts == 2) return f.template operator()<TW, TH, 2, 32>();
    if (tc == 32 && ts == 4) return f.template operator()<TW, TH, 4, 32>();
    if constexpr (NL * 8 <= 1024)
        if (tc == 32 && ts == 8) return f.template operator()<TW, TH, 8, 32>();
    return hipErrorInvalidValue;
}

template <typename F>
hipError_t dispatch(const Plan &plan, F &&f) {
    const int w = plan.tile_w, h = plan.tile_h, tc = plan.time_chunk, ts = plan.time_split;
    if (w == 4 && h == 4) return dispatch_tc_ts<4, 4>(tc, ts, f);
    if (w == 8 && h == 2) return dispatch_tc_ts<8, 2>(tc, ts, f);
    if (w == 4 && h == 2) return dispatch_tc_ts<4, 2>(tc, ts, f);
    if (w == 2 && h == 2) return dispatch_tc_ts<2, 2>(tc, ts, f);
    return hipErrorInvalidValue;
}

}  // namespace valu

bool valu_available(int tile_w, int tile_h, int time_chunk, int time_split) {
    const bool tile = (tile_w == 4 && tile_h == 4) || (tile_w == 8 && tile_h == 2) || (tile_w == 4 && tile_h == 2) ||
                      (tile_w == 2 && tile_h == 2);
    const int nl = (32 / tile_w) * (32 / tile_h);
    const bool tcts = (time_chunk == 16 && (time_split == 1 || time_split == 2 || time_split == 4)) ||
                      (time_chunk == 32 && (time_split == 2 || time_split == 4 || (time_split == 8 && nl * 8 <= 1024)));
    return tile && tcts;
}

namespace {
struct FlatLaunch {
    const Job &job;
    hipStream_t stream;
    template <int TW, int TH, int TS, int TC>
    hipError_t operator()() const { return valu::launch_t<TW, TH, TS, TC>(job, stream); }
};
struct BatchLaunch {
    const Job *jobs;
    const Unit *units;
    const int *bounds;
    int grid;
    hipStream_t stream;
    template <int TW, int TH, int TS, int TC>
    hipError_t operator()() const { return valu::launch_batch_t<TW, TH, TS, TC>(jobs, units, bounds, grid, stream); }
};
}  // namespace

hipError_t launch_valu(const Plan &plan, const Job &job, hipStream_t stream) {
    if (plan.block == 16) return launch_small(job, stream);
    return valu::dispatch(plan, FlatLaunch{job, stream});
}

hipError_t launch_valu_batch(const Plan &plan, const Job *jobs, const Unit *units, const int *bounds, int grid,
                             hipStream_t stream) {
    if (plan.block == 16) return launch_small_batch(jobs, units, bounds, grid, stream);
    return valu::dispatch(plan, BatchLaunch{jobs, units, bounds, grid, stream});
}

}  // namespace xc
