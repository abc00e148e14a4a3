// FP32 matrix-core correlator kernel on 16 x 16 x 4 MFMA tiles (gfx950).
//
// Same product as the other MFMA kernels (per channel V = X X^H, computed as
// Re V = Xr Xr^T + Xi Xi^T and Im V = Xi Xr^T - Xr Xi^T on real matrix cores,
// with f32 products and accumulation), but on 16 x 16 output tiles so that the
// triangle of station pairs is covered with little waste:
//
//  * A workgroup owns one (channel, block pair bi <= bj) of SB = 64 stations,
//    i.e. a 128 x 128 square of (station, pol) rows split into 8 x 8 tiles.
//  * Off the diagonal every wave takes a 4 x 4 group of tiles (64 x 64 rows).
//  * On the diagonal only the 36 tiles on or above the diagonal are needed;
//    wave w takes tile rows w and 7 - w (8 - w + w + 1 = 9 tiles), so the four
//    waves carry equal work.  For 64 stations this computes 9216 complex
//    products per time step for 8320 wanted (90 %).
//  * TS = 2 splits every staged chunk of time steps between two groups of four
//    waves (two waves per SIMD); the second group's partial sums are added
//    into the first's through LDS before the single store.
//  * Samples are staged per chunk of 16 (or 32) time steps through LDS in their
//    time-major layout, double-buffered through registers.  A fragment is one
//    (re, im) sample per lane: lane l holds row l % 16 at time step l / 16 of
//    the k-step, for both the A (block I) and B (block J) operands.
#include "common.h"

namespace xc {
namespace mfma16 {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int SB = 64;              // stations per block
constexpr int RB = 2 * SB;          // rows per block
constexpr int PITCH = 2 * RB * 8;   // bytes per staged time step (I then J rows)
// time steps per staged chunk: 16, or 32 when two wave groups share the
// workgroup (one workgroup per CU then, so the larger buffers fit)
template <int TS>
constexpr int kt() { return TS == 2 ? 32 : 16; }
template <int TS>
constexpr int stage() { return kt<TS>() * PITCH; }

// Tile coordinates (tile row, tile column) of wave w's slot s.
template <bool DIAG, int W>
struct Sched;
template <int W>
struct Sched<false, W> {
    static constexpr int NT = 16;
    static constexpr int NA = 4, NB = 4;
    __device__ static constexpr int a_of(int s) { return s / 4; }       // index into the wave's A rows
    __device__ static constexpr int b_of(int s) { return s % 4; }       // index into the wave's B cols
    __device__ static constexpr int arow(int a) { return (W >> 1) * 4 + a; }  // tile row of A fragment a
    __device__ static constexpr int bcol(int b) { return (W & 1) * 4 + b; }   // tile col of B fragment b
};
template <int W>
struct Sched<true, W> {
    // rows W (columns W..7) and 7 - W (columns 7 - W..7)
    static constexpr int NT = 9;
    static constexpr int LO = W < 7 - W ? W : 7 - W;   // first column needed
    static constexpr int NA = 2, NB = 8 - LO;
    __device__ static constexpr int a_of(int s) { return s < 8 - W ? 0 : 1; }
    __device__ static constexpr int col(int s) { return s < 8 - W ? W + s : s - 1; }
    __device__ static constexpr int b_of(int s) { return col(s) - LO; }
    __device__ static constexpr int arow(int a) { return a == 0 ? W : 7 - W; }
    __device__ static constexpr int bcol(int b) { return LO + b; }
};

// Staging: the chunk's time steps x 2 SB station samples (float4 = both pols) are
// spread over all 256 TS threads of the workgroup.
template <int TS>
struct Pre {
    static constexpr int N = kt<TS>() * 2 * SB / (256 * TS);
    float4 v[N];
};

template <int TS>
__device__ __forceinline__ void gload(Pre<TS> &p, const Job &job, int c, int I0, int J0, bool diag, int t0,
                                      int tid) {
    const float4 *xs = static_cast<const float4 *>(job.x);
#pragma unroll
    for (int k = 0; k < Pre<TS>::N; ++k) {
        const int task = tid + 256 * TS * k;
        const int t = task / (2 * SB);
        const int s2 = task % (2 * SB);
        const int blk = s2 / SB;
        const int st = (blk ? J0 : I0) + s2 % SB;
        // out-of-range samples read a clamped, valid address and become zeros
        const bool ok = !(blk && diag) && (t0 + t < job.T) && st < job.S;
        const int tc = t0 + t < job.T ? t0 + t : job.T - 1;
        const int sc = st < job.S ? st : 0;
        const float4 v = xs[row_offset(job, c, tc) + sc];
        p.v[k] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// Loads of a full chunk whose time steps are consecutive rows in memory: one
// uniform base address per chunk plus a per-thread byte offset fixed for the
// whole unit, so a load needs no address arithmetic.  A thread's k-th sample
// is 2 TS rows after its (k-1)-th.  Stations past the last one read the last
// station's sample instead of zeros: they only feed output rows and columns
// that are never stored.  skip (uniform per wave): the thread's samples are
// block J's of a diagonal pair, which are block I's.
template <int TS>
__device__ __forceinline__ void gload_full(Pre<TS> &p, const uint8_t *base, uint32_t voff, uint32_t kstride,
                                           bool skip) {
    if (skip) return;
#pragma unroll
    for (int k = 0; k < Pre<TS>::N; ++k)
        p.v[k] = *reinterpret_cast<const float4 *>(base + (size_t)k * kstride + voff);
}

template <int TS>
__device__ __forceinline__ void lstore(const Pre<TS> &p, uint8_t *lds, bool diag, int tid) {
#pragma unroll
    for (int k = 0; k < Pre<TS>::N; ++k) {
        const int task = tid + 256 * TS * k;
        const int t = task / (2 * SB);
        const int s2 = task % (2 * SB);
        if (s2 >= SB && diag) continue;
        *reinterpret_cast<float4 *>(lds + t * PITCH + s2 * 16) = p.v[k];
    }
}

template <typename OUT>
struct Out;
template <>
struct Out<float2> {
    __device__ static float2 make(float re, float im) { return make_float2(re, im); }
    __device__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
};

// Output of a 16 x 16 tile: element (lane, r) is row 4 (lane / 16) + r, column lane % 16.
__device__ __forceinline__ void store_tile(const Job &job, int c, const v4f &re, const v4f &im, int row0, int col0,
                                           int lane) {
    const int S = job.S;
    const int col = col0 + (lane & 15);
    const int j = col >> 1;
    const int q = col & 1;
    if (j >= S) return;
    float2 *__restrict__ V = static_cast<float2 *>(job.vis) + (size_t)c * ((size_t)S * (S + 1) / 2) * 4;
    const size_t jbase = (size_t)j * (j + 1) / 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = row0 + 4 * (lane >> 4) + r;
        const int i = row >> 1;
        const int p = row & 1;
        if (i > j) continue;
        float vr = re[r];
        float vi = im[r];
        if (i == j) {
            if (p == 1 && q == 0) continue;     // written as conj(XY) by the q = 1 lane
            if (p == q) vi = 0.f;
        }
        float2 v = make_float2(vr, vi);
        const size_t e = (jbase + i) * 4 + p * 2 + q;
        if (job.accumulate) v = Out<float2>::add(v, V[e]);
        V[e] = v;
        if (i == j && p == 0 && q == 1) {
            float2 w = make_float2(vr, -vi);
            const size_t e2 = (jbase + i) * 4 + 2;
            if (job.accumulate) w = Out<float2>::add(w, V[e2]);
            V[e2] = w;
        }
    }
}

// One wave's share of a block pair.  G = time group (0 .. TS-1).
template <bool DIAG, int W, int TS>
__device__ __forceinline__ void wave_unit(const Job &job, int c, int bi, int bj, uint8_t *lds, int tid) {
    typedef Sched<DIAG, W> SC;
    constexpr int NT = SC::NT;
    const int lane = tid & 63;
    const int grp = __builtin_amdgcn_readfirstlane((tid >> 6) / 4);   // time group (uniform per wave)
    const int r16 = lane & 15;
    const int kq = lane >> 4;              // time step within a k-step
    const int I0 = bi * SB, J0 = bj * SB;
    const int S = job.S;
    const int brow_base = DIAG ? 0 : RB;

    // Tiles past the last station are not stored.  A wave with any tile to
    // store computes all of its tiles (on zero samples for the others): the
    // MFMA stream then has no branches, and such waves only occur in the
    // blocks at the end of the station range.
    bool any = false;
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        const int tr = SC::arow(SC::a_of(s)), tc = SC::bcol(SC::b_of(s));
        any |= (I0 * 2 + tr * 16 < 2 * S) && (J0 * 2 + tc * 16 < 2 * S);
    }

    v4f are[NT], aim[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        are[s] = v4f{0.f, 0.f, 0.f, 0.f};
        aim[s] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    constexpr int KT = kt<TS>();
    constexpr int STAGE = stage<TS>();
    // this thread's sample in every chunk: row tid / 2 SB, station s2 of the pair
    const int s2 = tid % (2 * SB);
    const int st = (s2 < SB ? I0 : J0) + s2 % SB;
    const uint32_t voff = (uint32_t)(((tid / (2 * SB)) * S + (st < S ? st : S - 1)) * 16);
    const uint32_t kstride = (uint32_t)(2 * TS * S * 16);
    const bool skip = DIAG && __builtin_amdgcn_readfirstlane(s2 >= SB);
    const uint8_t *x8 = static_cast<const uint8_t *>(job.x);
    auto load_chunk = [&](Pre<TS> &p, int t0) {
        if (t0 + KT <= job.T && rows_contiguous(job, t0, KT))
            gload_full<TS>(p, x8 + row_offset(job, c, t0) * 16, voff, kstride, skip);
        else
            gload<TS>(p, job, c, I0, J0, DIAG, t0, tid);
    };
    Pre<TS> pre;
    const int nchunk = (job.T + KT - 1) / KT;
    load_chunk(pre, 0);
    lstore<TS>(pre, lds, DIAG, tid);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const uint8_t *buf = lds + (ch & 1) * STAGE;
        const bool more = ch + 1 < nchunk;
        uint8_t *next = lds + ((ch & 1) ^ 1) * STAGE;
        if (more) load_chunk(pre, (ch + 1) * KT);
        // This group's k-steps of the chunk: ks = grp, grp + TS, ...  The next
        // k-step's fragments are read from LDS before the current k-step's
        // MFMAs are issued, and the MFMAs are ordered by product kind so that
        // two updates of one accumulator are NT instructions apart.
        constexpr int NK = KT / 4 / TS;
        float2 fa[2][SC::NA], fb[2][SC::NB];
        auto frag = [&](int ks, float2 (&a)[SC::NA], float2 (&b)[SC::NB]) {
            const int t = ks * 4 + kq;
#pragma unroll
            for (int k = 0; k < SC::NA; ++k)
                a[k] = *reinterpret_cast<const float2 *>(buf + t * PITCH + (SC::arow(k) * 16 + r16) * 8);
#pragma unroll
            for (int k = 0; k < SC::NB; ++k)
                b[k] = *reinterpret_cast<const float2 *>(buf + t * PITCH + (brow_base + SC::bcol(k) * 16 + r16) * 8);
        };
        if (any) {
            frag(grp, fa[0], fb[0]);
#pragma unroll
            for (int i = 0; i < NK; ++i) {
                const int cur = i & 1;
                if (i + 1 < NK) frag(grp + (i + 1) * TS, fa[cur ^ 1], fb[cur ^ 1]);
                const float2(&a)[SC::NA] = fa[cur];
                const float2(&b)[SC::NB] = fb[cur];
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    are[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SC::a_of(s)].x, b[SC::b_of(s)].x, are[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    aim[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SC::a_of(s)].y, b[SC::b_of(s)].x, aim[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    are[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SC::a_of(s)].y, b[SC::b_of(s)].y, are[s], 0, 0, 0);
                float nby[SC::NB];
#pragma unroll
                for (int k = 0; k < SC::NB; ++k) nby[k] = -b[k].y;
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    aim[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SC::a_of(s)].x, nby[SC::b_of(s)], aim[s], 0, 0, 0);
                // the next chunk goes to the other buffer (free since the last
                // barrier) behind this wave's last queued MFMAs
                if (i == NK - 1 && more) lstore<TS>(pre, next, DIAG, tid);
            }
        } else if (more) {
            lstore<TS>(pre, next, DIAG, tid);
        }
        __syncthreads();
    }

    if constexpr (TS > 1) {
        // group 1 hands its partial sums to group 0 through LDS (staging is free now)
        float *red = reinterpret_cast<float *>(lds);
        constexpr int NF = NT * 8;
        // two rounds of two waves each keep the area within the staging buffers
#pragma unroll 1
        for (int round = 0; round < 2; ++round) {
            const int wloc = W;                       // wave within its group
            const bool mine = (wloc >> 1) == round;   // waves {0,1} then {2,3}
            const int slot = (wloc & 1) * NF * 64;
            if (grp == 1 && mine) {
#pragma unroll
                for (int s = 0; s < NT; ++s)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        red[slot + ((s * 8 + r) * 64) + lane] = are[s][r];
                        red[slot + ((s * 8 + 4 + r) * 64) + lane] = aim[s][r];
                    }
            }
            __syncthreads();
            if (grp == 0 && mine) {
#pragma unroll
                for (int s = 0; s < NT; ++s)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        are[s][r] += red[slot + ((s * 8 + r) * 64) + lane];
                        aim[s][r] += red[slot + ((s * 8 + 4 + r) * 64) + lane];
                    }
            }
            __syncthreads();
        }
    }
    if (grp != 0) return;
#pragma unroll
    for (int s = 0; s < NT; ++s)
        if (I0 * 2 + SC::arow(SC::a_of(s)) * 16 < 2 * S && J0 * 2 + SC::bcol(SC::b_of(s)) * 16 < 2 * S)
            store_tile(job, c, are[s], aim[s], I0 * 2 + SC::arow(SC::a_of(s)) * 16,
                       J0 * 2 + SC::bcol(SC::b_of(s)) * 16, lane);
}

template <int TS>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, uint8_t *lds) {
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((tid >> 6) & 3);
    if (bi == bj) {
        switch (w) {
        case 0: wave_unit<true, 0, TS>(job, c, bi, bj, lds, tid); break;
        case 1: wave_unit<true, 1, TS>(job, c, bi, bj, lds, tid); break;
        case 2: wave_unit<true, 2, TS>(job, c, bi, bj, lds, tid); break;
        default: wave_unit<true, 3, TS>(job, c, bi, bj, lds, tid); break;
        }
    } else {
        switch (w) {
        case 0: wave_unit<false, 0, TS>(job, c, bi, bj, lds, tid); break;
        case 1: wave_unit<false, 1, TS>(job, c, bi, bj, lds, tid); break;
        case 2: wave_unit<false, 2, TS>(job, c, bi, bj, lds, tid); break;
        default: wave_unit<false, 3, TS>(job, c, bi, bj, lds, tid); break;
        }
    }
}

// LDS: two staging buffers (64 or 128 KiB), reused for the time-group reduction.
template <int TS>
__global__ __launch_bounds__(256 * TS, 2 / TS) void kernel(Job job, int nwork) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * stage<TS>()];
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    const int c = w / job.npairs;
    int bi, bj;
    pair_decode(w - c * job.npairs, bi, bj);
    unit<TS>(job, c, bi, bj, lds);
}

template <int TS>
__global__ __launch_bounds__(256 * TS, 2 / TS) void kernel_batch(const Job *__restrict__ jobs,
                                                                 const Unit *__restrict__ units, Queues q) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * stage<TS>()];
    __shared__ int next;
    drain_queues(units, q, &next, [&](const Unit &un) {
        const Job job = jobs[un.item];
        unit<TS>(job, un.channel, un.bi, un.bj, lds);
    });
}

}  // namespace mfma16

hipError_t launch_mfma16(const Plan &plan, const Job &job, hipStream_t stream) {
    const int nwork = job.C * job.npairs;
    if (plan.time_split == 2) {
        hipLaunchKernelGGL(mfma16::kernel<2>, dim3(xcd_grid(nwork)), dim3(512), 0, stream, job, nwork);
    } else {
        hipLaunchKernelGGL(mfma16::kernel<1>, dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    }
    return hipGetLastError();
}

hipError_t launch_mfma16_batch(const Plan &plan, const Job *jobs, const Unit *units, Queues q, int grid,
                               hipStream_t stream) {
    if (plan.time_split == 2) {
        hipLaunchKernelGGL(mfma16::kernel_batch<2>, dim3(grid), dim3(512), 0, stream, jobs, units, q);
    } else {
        hipLaunchKernelGGL(mfma16::kernel_batch<1>, dim3(grid), dim3(256), 0, stream, jobs, units, q);
    }
    return hipGetLastError();
}

int occupancy_mfma16_batch(const Plan &plan) {
    int n = 0;
    hipError_t e = plan.time_split == 2
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mfma16::kernel_batch<2>, 512, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mfma16::kernel_batch<1>, 256, 0);
    return (e != hipSuccess || n < 1) ? 1 : n;
}

}  // namespace xc
