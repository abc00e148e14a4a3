// Matrix-core (MFMA) correlator kernels for gfx950.
//
// Per channel the correlation of Section 2 is the Hermitian product
// V = X X^H of the (station, polarisation) x time sample matrix X.  With
// X = Xr + i Xi it is computed on real matrix cores as two real products
// with a doubled reduction dimension (time, re/im):
//
//     Re V = [Xr Xi] [Xr Xi]^T            (a_r b_r + a_i b_i)
//     Im V = [Xr Xi] [-Xi Xr]^T           (a_i b_r - a_r b_i)
//
// so every lane's B fragment for the imaginary part is its real-part
// fragment with each (re, im) pair replaced by (-im, re).  Negation is exact
// for float types and for int8 in [-127, 127].
//
// Inputs and instructions:
//   complex int8    -> v_mfma_i32_32x32x32_i8   (int32 accumulation, exact)
//   complex f16     -> v_mfma_f32_32x32x16_f16  (f32 accumulation)
//   complex bf16    -> v_mfma_f32_32x32x16_bf16 (f32 accumulation)
//   complex f32     -> v_mfma_f32_32x32x2_f32   (f32 products and accumulation;
//                      the four real products are issued separately; this
//                      variant serves 32-station blocks, while 64-station
//                      blocks of complex f32 use the 16 x 16 tile kernel)
//
// Tiling: the station triangle is split into blocks of SB stations (SB = 32
// or 64, i.e. 2 SB rows of (station, pol)); a workgroup of four waves owns one
// (channel, block pair bi <= bj) and each wave one SB x SB quadrant of its
// 2SB x 2SB rows (SB/32 x SB/32 MFMA tiles of 32 x 32, real and imaginary
// accumulators).  On a diagonal block pair the quadrant and the 32 x 32 tiles
// that lie entirely below the diagonal are skipped, and only i <= j is stored.
//
// Staging: each chunk of time steps of both blocks goes through LDS,
// double-buffered through registers (the next chunk's global loads are in
// flight during the current chunk's MFMAs).  The int8 and 16-bit paths turn
// the time-major samples into rows of consecutive time steps while writing
// LDS (a corner turn in registers with byte permutes), so that each lane's
// MFMA fragment is a single 16-byte LDS read; rows are padded by 16 bytes to
// spread a quarter-wave's reads over all banks.  The f32 path needs no corner
// turn: its fragments hold one time step per lane.
#include "common.h"

#include "mfma_parts.h"

namespace xc {
namespace mfma {

template <int KIND, int SB, typename OUT>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, uint8_t *lds) {
    typedef Geo<KIND, SB> G;
    typedef typename Acc<KIND>::type acc_t;
    constexpr int NS = G::NS;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    // the wave index is uniform across a wave: keep it (and everything derived
    // from it, such as which tiles run) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 1;
    const int wc = wave & 1;

    Blocks bk;
    bk.I0 = bi * SB;
    bk.J0 = bj * SB;
    bk.diag = (bi == bj);

    // rows of this wave's quadrant inside the staged blocks
    const int arow0 = wr * SB;
    const int brow0 = (bk.diag ? 0 : G::RB) + wc * SB;
    const int S = job.S;
    // tiles to run: skip tiles fully below the diagonal and tiles past the last station
    bool run[NS][NS];
    bool any = false;
#pragma unroll
    for (int rs = 0; rs < NS; ++rs) {
#pragma unroll
        for (int cs = 0; cs < NS; ++cs) {
            const int r0 = bk.I0 * 2 + wr * SB + rs * 32;    // first global row
            const int c0 = bk.J0 * 2 + wc * SB + cs * 32;    // first global column
            const bool below = (r0 >> 1) > ((c0 + 31) >> 1);
            run[rs][cs] = !below && (r0 < 2 * S) && (c0 < 2 * S);
            any |= run[rs][cs];
        }
    }

    acc_t are[NS][NS], aim[NS][NS];
#pragma unroll
    for (int rs = 0; rs < NS; ++rs)
#pragma unroll
        for (int cs = 0; cs < NS; ++cs) {
            are[rs][cs] = acc_t{};
            aim[rs][cs] = acc_t{};
        }

    const uint8_t *x = static_cast<const uint8_t *>(job.x);
    const LoadPlan<KIND, SB> lp = make_load_plan<KIND, SB>(job, bk, tid);
    const bool fast = fast_loads_ok<KIND, SB>(job);
    constexpr int SAMPLE = KIND == K_I8 ? 4 : (KIND == K_F32 ? 16 : 8);   // bytes per station sample
    auto load_chunk = [&](Pre<KIND, SB> &p, int t0) {
        if (fast && t0 + G::KT <= job.T && rows_contiguous(job, t0, G::KT))
            gload_full<KIND, SB>(p, x + row_offset(job, c, t0) * SAMPLE, lp);
        else
            gload<KIND, SB>(p, job, x, c, bk, t0, tid);
    };
    Pre<KIND, SB> pre;
    const int nchunk = (job.T + G::KT - 1) / G::KT;
    load_chunk(pre, 0);
    lstore<KIND, SB>(pre, lds, bk, tid);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nchunk;
        uint8_t *next = lds + (buf ^ 1) * G::STAGE_BYTES;
        if (more) load_chunk(pre, (ch + 1) * G::KT);
        // A wave with any tile to do computes all of its tiles: the skipped ones
        // (below the diagonal or past the last station) only occur in waves
        // that are not the slowest of their workgroup, so this costs no time
        // and keeps the MFMA stream free of branches.  The next chunk goes to
        // the other buffer (free since the last barrier) half-way through.
        if (any)
            compute_chunk<KIND, SB, true>(lds + buf * G::STAGE_BYTES, are, aim, arow0, brow0, run, lane, [&] {
                if (more) lstore<KIND, SB>(pre, next, bk, tid);
            });
        else if (more)
            lstore<KIND, SB>(pre, next, bk, tid);
        __syncthreads();
    }

    if (!any) return;
    if constexpr (KIND == K_I8) {
        // the int8 imaginary accumulators hold minus the imaginary part
#pragma unroll
        for (int rs = 0; rs < NS; ++rs)
#pragma unroll
            for (int cs = 0; cs < NS; ++cs) aim[rs][cs] = -aim[rs][cs];
    }
    if constexpr (SB == 64) {
        // the staging buffers are free after the last barrier: one image region per wave
        static_assert(4 * IMG_BYTES <= 2 * G::STAGE_BYTES, "tile images must fit the staging area");
        uint8_t *img = lds + wave * IMG_BYTES;
        store_tiles_lds<acc_t, OUT>(job, c, are, aim, run, bk.I0 * 2 + wr * SB, bk.J0 * 2 + wc * SB, lane, img);
    } else {
#pragma unroll
        for (int rs = 0; rs < NS; ++rs)
#pragma unroll
            for (int cs = 0; cs < NS; ++cs)
                if (run[rs][cs])
                    store_tile<acc_t, OUT>(job, c, are[rs][cs], aim[rs][cs], bk.I0 * 2 + wr * SB + rs * 32,
                                           bk.J0 * 2 + wc * SB + cs * 32, lane);
    }
}

// Two workgroups of four waves per CU: both the staging LDS (<= 72 KiB each)
// and the registers (<= 256 per lane) are sized for it.
template <int KIND, int SB, typename OUT>
__global__ __launch_bounds__(256, 2) void kernel(Job job, int nwork) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * Geo<KIND, SB>::STAGE_BYTES];
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    int c, bi, bj;
    unit_decode(job, w, c, bi, bj);
    unit<KIND, SB, OUT>(job, c, bi, bj, lds);
}

template <int KIND, int SB, typename OUT>
__global__ __launch_bounds__(256, 2) void kernel_batch(const Job *__restrict__ jobs, const Unit *__restrict__ units,
                                                       const int *__restrict__ bounds) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[2 * Geo<KIND, SB>::STAGE_BYTES];
    const int u = batch_unit(bounds, blockIdx.x);
    if (u < 0) return;
    const Unit un = units[u];
    const Job job = jobs[un.item];
    unit<KIND, SB, OUT>(job, un.channel, un.bi, un.bj, lds);
}

template <int KIND, int SB, typename OUT>
hipError_t launch_t(const Job &job, hipStream_t stream) {
    const int nwork = job_units(job);
    hipLaunchKernelGGL((kernel<KIND, SB, OUT>), dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    return hipGetLastError();
}
template <int KIND, int SB, typename OUT>
hipError_t launch_batch_t(const Job *jobs, const Unit *units, const int *bounds, int grid, hipStream_t stream) {
    hipLaunchKernelGGL((kernel_batch<KIND, SB, OUT>), dim3(grid), dim3(256), 0, stream, jobs, units, bounds);
    return hipGetLastError();
}
// Dispatch over (input type, output type, block size).
#define XC_MFMA_DISPATCH(FN, ...)                                                                     \
    switch (in_type) {                                                                                \
    case XC_IN_CI8:                                                                                   \
        if (out_type == XC_OUT_CI32)                                                                  \
            return sb == 32 ? FN<K_I8, 32, int2>(__VA_ARGS__) : FN<K_I8, 64, int2>(__VA_ARGS__);      \
        return sb == 32 ? FN<K_I8, 32, float2>(__VA_ARGS__) : FN<K_I8, 64, float2>(__VA_ARGS__);      \
    case XC_IN_CF16:                                                                                  \
        return sb == 32 ? FN<K_F16, 32, float2>(__VA_ARGS__) : FN<K_F16, 64, float2>(__VA_ARGS__);    \
    case XC_IN_CBF16:                                                                                 \
        return sb == 32 ? FN<K_BF16, 32, float2>(__VA_ARGS__) : FN<K_BF16, 64, float2>(__VA_ARGS__);  \
    case XC_IN_CF32:                                                                                  \
        return FN<K_F32, 32, float2>(__VA_ARGS__);                                                    \
    }

}  // namespace mfma

hipError_t launch_mfma(const Plan &plan, xc_in_type in_type, xc_out_type out_type, const Job &job,
                       hipStream_t stream) {
    using namespace mfma;
    const int sb = plan.block;
    XC_MFMA_DISPATCH(launch_t, job, stream)
    return hipErrorInvalidValue;
}

hipError_t launch_mfma_batch(const Plan &plan, xc_in_type in_type, xc_out_type out_type, const Job *jobs,
                             const Unit *units, const int *bounds, int grid, hipStream_t stream) {
    using namespace mfma;
    const int sb = plan.block;
    XC_MFMA_DISPATCH(launch_batch_t, jobs, units, bounds, grid, stream)
    return hipErrorInvalidValue;
}

}  // namespace xc
