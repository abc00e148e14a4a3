// FP32 matrix-core correlator kernel on 16 x 16 x 4 MFMA tiles (gfx950).
//
// Same product as the other MFMA kernels (per channel V = X X^H, computed as
// Re V = Xr Xr^T + Xi Xi^T and Im V = Xi Xr^T - Xr Xi^T on real matrix cores,
// with f32 products and accumulation), but on 16 x 16 output tiles so that the
// triangle of station pairs is covered with little waste.  Either four real
// products per tile and time step, or three (Gauss's form for complex
// multiplication): P1 = Xr Xr^T, P2 = Xi Xi^T and P3 = (Xr + Xi)(Xr - Xi)^T,
// with Re V = P1 + P2 and Im V = P3 - P1 + P2 formed once at the end.  The
// sums Xr + Xi and Xr - Xi are two vector adds per fragment; the three-product
// form issues a quarter fewer MFMAs for 50 % more accumulator registers.
//
//  * A workgroup owns one (channel, block pair bi <= bj) of SB = 64 stations,
//    i.e. a 128 x 128 square of (station, pol) rows split into 8 x 8 tiles.
//  * Off the diagonal every wave takes a 4 x 4 group of tiles (64 x 64 rows).
//  * On the diagonal only the 36 tiles on or above the diagonal are needed;
//    wave w takes tile rows w and 7 - w (8 - w + w + 1 = 9 tiles), so the four
//    waves carry equal work.  For 64 stations this computes 9216 complex
//    products per time step for 8320 wanted (90 %).
//  * TS = 2 splits every staged chunk of time steps between two groups of four
//    waves (two waves per SIMD); off the diagonal the second group's partial
//    sums are added into the first's through LDS before the single store, on
//    it each group writes a triangle image of its own and the copy-out adds
//    the two.
//  * Samples go from HBM straight into LDS (global_load_lds, see lds_dma.h),
//    in their time-major layout: one 1 KiB row per block and time step (block
//    I only on the diagonal, I then J elsewhere).  Two stages of 64 KiB (two
//    time groups) or 32 KiB (one) alternate: the next chunk is copied while
//    the current one is computed, with one barrier per chunk.  A diagonal
//    unit stages half the bytes per time step, so its chunks are twice as
//    long (64 or 32 time steps against 32 or 16).
//  * A fragment is one (re, im) sample per lane: lane l holds row l % 16 at
//    time step l / 16 of the k-step, for both the A (block I) and B (block J)
//    operands.
#include "common.h"
#include "lds_dma.h"

namespace xc {
namespace mfma16 {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int SB = 64;              // stations per block
constexpr int RB = 2 * SB;          // rows per block
constexpr int BROW = RB * 8;        // bytes of one block's time step (1 KiB)
// bytes per stage: 64 KiB with two time groups (one workgroup per CU), 32 KiB
// with one (two workgroups per CU)
template <int TS>
constexpr int stage() { return TS == 2 ? 65536 : 32768; }
// a diagonal unit's triangle of baselines as an image of the output: at most
// 2080 baselines x 4 polarisation products
constexpr int IMG = 2080 * 4;
// LDS of a workgroup: the two stages, and with two time groups also one
// triangle image per group (2 KiB more than the stages)
template <int TS>
constexpr int lds_bytes() {
    return TS == 2 && 2 * IMG * 8 > 2 * stage<TS>() ? 2 * IMG * 8 : 2 * stage<TS>();
}
// bytes per staged time step: block I only on the diagonal, I then J elsewhere
template <bool DIAG>
constexpr int pitch() { return DIAG ? BROW : 2 * BROW; }
template <bool DIAG, int TS>
constexpr int kt() { return stage<TS>() / pitch<DIAG>(); }

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
    // accumulate mode: every old value this lane adds to is loaded before the
    // first store, so that the loads are in flight together (a store to V
    // would otherwise keep each later load behind it)
    // (old2[r / 2]: the YX element that rows r = 0, 2 write for an autocorrelation)
    float2 old[4], old2[2];
    if (job.accumulate) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = row0 + 4 * (lane >> 4) + r;
            const int i = (row >> 1) <= j ? (row >> 1) : j;    // clamped: the value is not used
            old[r] = V[(jbase + i) * 4 + (row & 1) * 2 + q];
            if ((r & 1) == 0) old2[r >> 1] = V[(jbase + i) * 4 + 2];
        }
    }
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
        if (job.accumulate) v = Out<float2>::add(v, old[r]);
        V[e] = v;
        if (i == j && p == 0 && q == 1) {
            float2 w = make_float2(vr, -vi);
            const size_t e2 = (jbase + i) * 4 + 2;
            if (job.accumulate) w = Out<float2>::add(w, old2[r >> 1]);
            V[e2] = w;
        }
    }
}

// Diagonal block pair, two time groups: the unit's triangle of baselines
// (local j < nj, i <= j, at local index j (j + 1) / 2 + i, 32 bytes each,
// at most 2080 x 32 = 66 560 bytes) is assembled in LDS as an image of the
// output, one image per time group, written by both groups at once; the
// workgroup then copies out their sum (each element group 0's sum plus
// group 1's, as in the register reduction) in 16-byte granules, a wave
// writing 1 KiB runs of consecutive baselines.  Autocorrelations are written
// as the other stores do: XX, YY real, YX = conj(XY).
__device__ __forceinline__ void image_tile(float2 *__restrict__ img, const v4f &re, const v4f &im, int trow, int tcol,
                                           int nj, int lane) {
    const int col = tcol * 16 + (lane & 15);
    const int jl = col >> 1;
    const int q = col & 1;
    if (jl >= nj) return;
    const int jb = jl * (jl + 1) / 2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = trow * 16 + 4 * (lane >> 4) + r;
        const int il = row >> 1;
        const int p = row & 1;
        if (il > jl) continue;
        float vr = re[r];
        float vi = im[r];
        if (il == jl) {
            if (p == 1 && q == 0) continue;     // written as conj(XY) by the q = 1 lane
            if (p == q) vi = 0.f;
        }
        img[(jb + il) * 4 + p * 2 + q] = make_float2(vr, vi);
        if (il == jl && p == 0 && q == 1) img[(jb + il) * 4 + 2] = make_float2(vr, -vi);
    }
}

// One wave's share of a block pair.  G3 selects the three-product form.
template <bool DIAG, int W, int TS, bool G3>
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

    // Four-product form: are = Re V, aim = Im V.  Three-product form: are =
    // P1 = sum ar br, aim = P2 = sum ai bi, a3 = P3 = sum (ar + ai)(br - bi);
    // then Re V = P1 + P2 and Im V = P3 - P1 + P2.
    v4f are[NT], aim[NT], a3[G3 ? NT : 1];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        are[s] = v4f{0.f, 0.f, 0.f, 0.f};
        aim[s] = v4f{0.f, 0.f, 0.f, 0.f};
        if constexpr (G3) a3[s] = v4f{0.f, 0.f, 0.f, 0.f};
    }

    constexpr int PITCH = pitch<DIAG>();
    constexpr int KT = kt<DIAG, TS>();
    constexpr int STAGE = stage<TS>();
    // Copies: a stage holds KT rows of one block (diagonal) or 2 KT rows
    // alternating I and J; each of the 4 TS waves copies 8 of them per chunk,
    // one 1 KiB row (64 stations x 16 bytes, lane = station) per instruction.
    // Stations past the last one copy the last station: they only feed output
    // rows and columns that are never stored.
    constexpr int NW = 4 * TS;
    constexpr int NCOPY = (DIAG ? KT : 2 * KT) / NW;
    static_assert(NCOPY == 8, "eight copies per wave and chunk");
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int blk = DIAG ? 0 : (wave & 1);                  // NW is even: row parity = wave parity
    const int trow0 = DIAG ? wave : (wave >> 1);            // time row of copy 0
    constexpr int TSTEP = DIAG ? NW : NW / 2;               // time rows between copies
    const int st = (blk ? J0 : I0) + lane;
    const int stc = st < S ? st : S - 1;
    const uint32_t off = (uint32_t)((trow0 * S + stc) * 16);
    const uint32_t step = (uint32_t)(TSTEP * S * 16);
    const uint32_t dst0 = lds_addr(lds) + trow0 * PITCH + blk * BROW;
    const uint8_t *x8 = static_cast<const uint8_t *>(job.x);
    const int T = job.T;
    // station-major input: this lane's station series of channel c
    const uint8_t *srow = x8 + ((size_t)c * job.cstride + (size_t)stc * job.sstride) * 16;
    auto issue = [&](int ch) {
        const int t0 = ch * KT;
        const uint32_t dst = dst0 + (ch & 1) * STAGE;
        if (job.sstride) {
            // the corner turn happens here: lane l copies station l's sample
            // of the time row, so the LDS image is the same as for time-major
            // input (a 128-byte line of a station's series is shared by the
            // copies of 8 consecutive time rows)
#pragma unroll
            for (int k = 0; k < NCOPY; ++k) {
                const int t = t0 + trow0 + k * TSTEP;
                dma16(t < T ? static_cast<const void *>(srow + (size_t)t * 16) : static_cast<const void *>(g_zero16),
                      dst + k * TSTEP * PITCH);
            }
        } else if (t0 + KT <= T && rows_contiguous(job, t0, KT)) {
            const uint8_t *src = x8 + row_offset(job, c, t0) * 16 + off;
#pragma unroll
            for (int k = 0; k < NCOPY; ++k) dma16(src + k * step, dst + k * TSTEP * PITCH);
        } else {
#pragma unroll
            for (int k = 0; k < NCOPY; ++k) {
                const int t = t0 + trow0 + k * TSTEP;
                const void *src = t < T ? static_cast<const void *>(x8 + (row_offset(job, c, t) + stc) * 16)
                                        : static_cast<const void *>(g_zero16);
                dma16(src, dst + k * TSTEP * PITCH);
            }
        }
    };

    const int nchunk = (T + KT - 1) / KT;
    issue(0);
    for (int ch = 0; ch < nchunk; ++ch) {
        // this wave's copies of chunk ch are the only ones pending; once every
        // wave is past the barrier they are visible, and the other stage (chunk
        // ch - 1) is free for chunk ch + 1
        wait_vm<0>();
        barrier_lds();
        if (ch + 1 < nchunk) issue(ch + 1);
        if (!any) continue;
        const uint8_t *buf = lds + (ch & 1) * STAGE;
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
        frag(grp, fa[0], fb[0]);
#pragma unroll
        for (int i = 0; i < NK; ++i) {
            const int cur = i & 1;
            if (i + 1 < NK) frag(grp + (i + 1) * TS, fa[cur ^ 1], fb[cur ^ 1]);
            const float2(&a)[SC::NA] = fa[cur];
            const float2(&b)[SC::NB] = fb[cur];
            if constexpr (G3) {
                float sa[SC::NA], db[SC::NB];
#pragma unroll
                for (int k = 0; k < SC::NA; ++k) sa[k] = a[k].x + a[k].y;
#pragma unroll
                for (int k = 0; k < SC::NB; ++k) db[k] = b[k].x - b[k].y;
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    are[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SC::a_of(s)].x, b[SC::b_of(s)].x, are[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    aim[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[SC::a_of(s)].y, b[SC::b_of(s)].y, aim[s], 0, 0, 0);
#pragma unroll
                for (int s = 0; s < NT; ++s)
                    a3[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(sa[SC::a_of(s)], db[SC::b_of(s)], a3[s], 0, 0, 0);
                continue;
            }
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
        }
    }
    if constexpr (G3) {
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            const v4f re = are[s] + aim[s];
            aim[s] = (a3[s] - are[s]) + aim[s];
            are[s] = re;
        }
    }
    // every wave is done with the stages before they are reused below
    __syncthreads();

    if constexpr (DIAG && TS == 2) {
        static_assert(2 * IMG * 8 <= lds_bytes<TS>(), "the two triangle images fit the workgroup's LDS");
        float2 *img = reinterpret_cast<float2 *>(lds) + grp * IMG;
        const int nj = S - J0 < SB ? S - J0 : SB;
        if (any) {
#pragma unroll
            for (int s = 0; s < NT; ++s)
                image_tile(img, are[s], aim[s], SC::arow(SC::a_of(s)), SC::bcol(SC::b_of(s)), nj, lane);
        }
        __syncthreads();
        const float4 *img4 = reinterpret_cast<const float4 *>(lds);
        const float4 *img4b = img4 + IMG / 2;      // group 1's image
        float4 *__restrict__ V4 = reinterpret_cast<float4 *>(static_cast<float2 *>(job.vis) +
                                                             (size_t)c * ((size_t)S * (S + 1) / 2) * 4);
        const int ng = nj * (nj + 1);     // 16-byte granules: two per baseline
        // granules in groups of NB per thread: in accumulate mode the group's
        // old values are all loaded before its stores
        constexpr int NB = 4;
        for (int g0 = tid; g0 < ng; g0 += NB * 256 * TS) {
            float4 *dst[NB];
            float4 o[NB];
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int g = g0 + n * 256 * TS < ng ? g0 + n * 256 * TS : g0;
                const int bl = g >> 1;
                int jl = (int)((sqrtf(8.f * (float)bl + 1.f) - 1.f) * 0.5f);
                while ((jl + 1) * (jl + 2) / 2 <= bl) ++jl;
                while (jl * (jl + 1) / 2 > bl) --jl;
                const int il = bl - jl * (jl + 1) / 2;
                const int j = J0 + jl;
                dst[n] = V4 + (((size_t)j * (j + 1) / 2 + I0 + il) * 2 + (g & 1));
                if (job.accumulate) o[n] = *dst[n];
            }
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                const int g = g0 + n * 256 * TS;
                if (g >= ng) break;
                float4 v = img4[g];
                const float4 u = img4b[g];
                v = make_float4(v.x + u.x, v.y + u.y, v.z + u.z, v.w + u.w);
                if (job.accumulate) v = make_float4(v.x + o[n].x, v.y + o[n].y, v.z + o[n].z, v.w + o[n].w);
                *dst[n] = v;
            }
        }
        return;
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

template <int TS, bool G3>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, uint8_t *lds) {
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((tid >> 6) & 3);
    if (bi == bj) {
        switch (w) {
        case 0: wave_unit<true, 0, TS, G3>(job, c, bi, bj, lds, tid); break;
        case 1: wave_unit<true, 1, TS, G3>(job, c, bi, bj, lds, tid); break;
        case 2: wave_unit<true, 2, TS, G3>(job, c, bi, bj, lds, tid); break;
        default: wave_unit<true, 3, TS, G3>(job, c, bi, bj, lds, tid); break;
        }
    } else {
        switch (w) {
        case 0: wave_unit<false, 0, TS, G3>(job, c, bi, bj, lds, tid); break;
        case 1: wave_unit<false, 1, TS, G3>(job, c, bi, bj, lds, tid); break;
        case 2: wave_unit<false, 2, TS, G3>(job, c, bi, bj, lds, tid); break;
        default: wave_unit<false, 3, TS, G3>(job, c, bi, bj, lds, tid); break;
        }
    }
}

// LDS: two staging buffers (64 or 128 KiB), reused for the time-group
// reduction (two time groups: 130 KiB, for the groups' two triangle images).
template <int TS, bool G3>
__global__ __launch_bounds__(256 * TS, 2 / TS) void kernel(Job job, int nwork) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[lds_bytes<TS>()];
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    int c, bi, bj;
    unit_decode(job, w, c, bi, bj);
    unit<TS, G3>(job, c, bi, bj, lds);
}

template <int TS, bool G3>
__global__ __launch_bounds__(256 * TS, 2 / TS) void kernel_batch(const Job *__restrict__ jobs,
                                                                 const Unit *__restrict__ units,
                                                                 const int *__restrict__ bounds) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[lds_bytes<TS>()];
    const int u = batch_unit(bounds, blockIdx.x);
    if (u < 0) return;
    const Unit un = units[u];
    const Job job = jobs[un.item];
    unit<TS, G3>(job, un.channel, un.bi, un.bj, lds);
}

}  // namespace mfma16

namespace mfma16 {
template <int TS, bool G3>
hipError_t launch_t(const Job &job, hipStream_t stream) {
    const int nwork = job_units(job);
    hipLaunchKernelGGL((kernel<TS, G3>), dim3(xcd_grid(nwork)), dim3(256 * TS), 0, stream, job, nwork);
    return hipGetLastError();
}
template <int TS, bool G3>
hipError_t launch_batch_t(const Job *jobs, const Unit *units, const int *bounds, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((kernel_batch<TS, G3>), dim3(grid), dim3(256 * TS), 0, stream, jobs, units, bounds);
    return hipGetLastError();
}
}  // namespace mfma16

hipError_t launch_mfma16(const Plan &plan, const Job &job, hipStream_t stream) {
    using namespace mfma16;
    const bool g3 = plan.product == XC_PRODUCT_THREE;
    if (plan.time_split == 2) return g3 ? launch_t<2, true>(job, stream) : launch_t<2, false>(job, stream);
    return g3 ? launch_t<1, true>(job, stream) : launch_t<1, false>(job, stream);
}

hipError_t launch_mfma16_batch(const Plan &plan, const Job *jobs, const Unit *units, const int *bounds, int grid,
                               hipStream_t stream) {
    using namespace mfma16;
    const bool g3 = plan.product == XC_PRODUCT_THREE;
    if (plan.time_split == 2)
        return g3 ? launch_batch_t<2, true>(jobs, units, bounds, grid, stream)
                  : launch_batch_t<2, false>(jobs, units, bounds, grid, stream);
    return g3 ? launch_batch_t<1, true>(jobs, units, bounds, grid, stream)
              : launch_batch_t<1, false>(jobs, units, bounds, grid, stream);
}

}  // namespace xc
