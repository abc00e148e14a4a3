// int8 matrix-core correlator kernel with direct global-to-LDS staging (gfx950).
//
// The product and the tiling are those of the register-staged kernel: a
// workgroup owns one (channel, block pair bi <= bj) of 64-station blocks, a
// 128 x 128 square of (station, pol) rows; each of its four waves holds a
// 64 x 64 quadrant as 2 x 2 tiles of 32 x 32, and V is accumulated over time
// as Re V = [Xr Xi][Xr Xi]^T and (minus) Im V = [Xr Xi][Xi -Xr]^T on i8 MFMAs
// with 32-bit integer sums.  What differs is how samples reach the matrix
// cores:
//
//  * global_load_lds copies 16-byte granules (4 stations, both pols, one time
//    step) from HBM straight into LDS, without passing through registers.  A
//    ring of four stages of 32 time steps keeps three chunks in flight while a
//    fourth is computed; one barrier per chunk both publishes a stage and
//    frees the one that is refilled next.
//  * LDS keeps the time-major layout of the input: one 256-byte row per block
//    and time step.  The corner turn to the MFMA operand layout (a (station,
//    pol) row per lane, time along K) is done by ds_read_b64_tr_b16, which
//    hands every lane four consecutive time steps of one 16-bit (re, im)
//    element; two such reads make a lane's 16-byte fragment.
//  * Granule g of time row t is stored at granule g ^ 4 (t mod 4), so that the
//    four time rows read by one transpose group fall on different banks.
//
// The copies are issued as in lds_dma.h: every wait for them is explicit.
//
// Requires n_stations % 4 == 0 (whole granules); other station counts use the
// register-staged kernel.
#include "common.h"

#include "lds_dma.h"
#include "mfma_parts.h"

namespace xc {
namespace dma {

using mfma::Acc;
using mfma::K_I8;
using mfma::v16i;
using mfma::v4i;

constexpr int SB = 64;              // stations per block
constexpr int ROWB = SB * 4;        // bytes of one block's time step
constexpr int KT = 32;              // time steps per stage
constexpr int BLK = KT * ROWB;      // one block's share of a stage (8 KiB)
constexpr int STAGE = 2 * BLK;      // 16 KiB
constexpr int NSTAGE = 4;
constexpr int LDS_BYTES = NSTAGE * STAGE;
static_assert(4 * mfma::IMG_BYTES <= LDS_BYTES, "tile images must fit the staging ring");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) v4s lds_v4s;

// Wait until at most n of this wave's vector-memory operations are pending
// (n in {0, 2, 4, 8}).
__device__ __forceinline__ void wait_vm_n(int n) {
    switch (n) {
    case 0: wait_vm<0>(); break;
    case 2: wait_vm<2>(); break;
    case 4: wait_vm<4>(); break;
    default: wait_vm<8>(); break;
    }
}

__device__ __forceinline__ v4i tr_frag(const lds_u8 *p) {
    const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)p);
    const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(p + 4 * ROWB));
    const int2 l = __builtin_bit_cast(int2, lo), h = __builtin_bit_cast(int2, hi);
    return v4i{l.x, l.y, h.x, h.y};
}

// Byte offset, within a block's image, of the transpose read of lane `lane`
// for the 32 rows starting at n0 at the first time step of a k-step: lane
// group g = lane / 16 takes rows n0 + 16 (g % 2) on and K half g / 2 (time
// steps 8 (g / 2) on); lane j of a group reads time step j / 4 and the four
// elements from row 4 (j % 4).
__device__ __forceinline__ uint32_t tr_offset(int n0, int lane) {
    const int t = 8 * (lane >> 5) + ((lane & 15) >> 2);
    const int n = n0 + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
    return t * ROWB + (((n >> 3) ^ (4 * (t & 3))) << 4) + (n & 7) * 2;
}

template <typename OUT>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, uint8_t *lds_generic) {
    typedef typename Acc<K_I8>::type acc_t;
    const lds_u8 *lds = (const lds_u8 *)lds_generic;
    const uint32_t lds_base = lds_addr(lds_generic);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 1, wc = wave & 1;
    const int S = job.S, T = job.T;
    const int I0 = bi * SB, J0 = bj * SB;
    const bool diag = bi == bj;
    const uint8_t *x = static_cast<const uint8_t *>(job.x);

    // -- copies: wave w fills 8 (diagonal) or 16 time rows of one block per chunk,
    // four rows (1 KiB) per instruction
    const int blk = diag ? 0 : (wave >> 1);
    const int rbase = diag ? wave * 8 : (wave & 1) * 16;
    const int nload = diag ? 2 : 4;
    const int lrow = lane >> 4;                         // = t mod 4 of the lane's rows
    const int gran = (lane & 15) ^ (4 * lrow);          // source granule of LDS granule lane % 16
    const int st = (blk ? J0 : I0) + 4 * gran;
    const int stc = st < S ? st : S - 4;                // past the last station: a valid granule
    const uint32_t off = (uint32_t)(((rbase + lrow) * S + stc) * 4);
    const uint32_t step = (uint32_t)(4 * S * 4);        // four time rows
    const uint32_t dst0 = lds_base + blk * BLK + rbase * ROWB;

    auto issue = [&](int ch) {
        const int t0 = ch * KT;
        const uint32_t dst = dst0 + (ch % NSTAGE) * STAGE;
        if (t0 + KT <= T && rows_contiguous(job, t0, KT)) {
            const uint8_t *src = x + row_offset(job, c, t0) * 4 + off;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < nload) dma16(src + i * step, dst + i * 4 * ROWB);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i >= nload) break;
                const int t = t0 + rbase + 4 * i + lrow;
                const void *src =
                    t < T ? static_cast<const void *>(x + (row_offset(job, c, t) + stc) * 4) : g_zero16;
                dma16(src, dst + i * 4 * ROWB);
            }
        }
    };

    // -- tiles of this wave (as in the register-staged kernel)
    bool run[2][2];
    bool any = false;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int cs = 0; cs < 2; ++cs) {
            const int r0 = I0 * 2 + wr * SB + rs * 32;
            const int c0 = J0 * 2 + wc * SB + cs * 32;
            const bool below = (r0 >> 1) > ((c0 + 31) >> 1);
            run[rs][cs] = !below && r0 < 2 * S && c0 < 2 * S;
            any |= run[rs][cs];
        }
    acc_t are[2][2], aim[2][2];
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int cs = 0; cs < 2; ++cs) {
            are[rs][cs] = acc_t{};
            aim[rs][cs] = acc_t{};
        }
    uint32_t aoff[2], boff[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        aoff[k] = tr_offset(wr * SB + 32 * k, lane);
        boff[k] = (diag ? 0 : BLK) + tr_offset(wc * SB + 32 * k, lane);
    }

    const int nchunk = (T + KT - 1) / KT;
#pragma unroll
    for (int k = 0; k < NSTAGE - 1; ++k)
        if (k < nchunk) issue(k);
    for (int ch = 0; ch < nchunk; ++ch) {
        // this wave's copies of chunk ch are done once only those of the
        // (at most two) chunks issued after it may be pending
        const int later = min(nchunk - 1 - ch, NSTAGE - 2);
        wait_vm_n(later * nload);
        barrier_lds();
        // every wave is past chunk ch - 1: its stage takes chunk ch + 3
        if (ch + NSTAGE - 1 < nchunk) issue(ch + NSTAGE - 1);
        if (!any) continue;
        const lds_u8 *sb = lds + (ch % NSTAGE) * STAGE;
#pragma unroll
        for (int ks = 0; ks < KT / 16; ++ks) {
            v4i a[2], b[2], bn[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                a[k] = tr_frag(sb + aoff[k] + ks * 16 * ROWB);
                b[k] = tr_frag(sb + boff[k] + ks * 16 * ROWB);
            }
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int e = 0; e < 4; ++e) bn[k][e] = (int)mfma::conj_neg_i8((uint32_t)b[k][e]);
#pragma unroll
            for (int rs = 0; rs < 2; ++rs)
#pragma unroll
                for (int cs = 0; cs < 2; ++cs)
                    are[rs][cs] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[rs], b[cs], are[rs][cs], 0, 0, 0);
#pragma unroll
            for (int rs = 0; rs < 2; ++rs)
#pragma unroll
                for (int cs = 0; cs < 2; ++cs)
                    aim[rs][cs] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[rs], bn[cs], aim[rs][cs], 0, 0, 0);
        }
    }
    // all copies are complete (the last chunk waited for none pending); the
    // ring becomes the tile-image area once every wave is done reading it
    __syncthreads();
    if (!any) return;
    uint8_t *img = lds_generic + wave * mfma::IMG_BYTES;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int cs = 0; cs < 2; ++cs)
            if (run[rs][cs]) {
                acc_t im = -aim[rs][cs];   // the accumulators hold minus the imaginary part
                mfma::store_tile_lds<acc_t, OUT>(job, c, are[rs][cs], im, I0 * 2 + wr * SB + rs * 32,
                                                 J0 * 2 + wc * SB + cs * 32, lane, img);
            }
}

template <typename OUT>
__global__ __launch_bounds__(256, 2) void kernel(Job job, int nwork) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    const int c = w / job.npairs;
    int bi, bj;
    pair_decode(w - c * job.npairs, bi, bj);
    unit<OUT>(job, c, bi, bj, lds);
}

template <typename OUT>
__global__ __launch_bounds__(256, 2) void kernel_batch(const Job *__restrict__ jobs, const Unit *__restrict__ units,
                                                       Queues q) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    __shared__ int next;
    drain_queues(units, q, &next, [&](const Unit &un) {
        const Job job = jobs[un.item];
        unit<OUT>(job, un.channel, un.bi, un.bj, lds);
    });
}

}  // namespace dma

hipError_t launch_mfma_dma(xc_out_type out_type, const Job &job, hipStream_t stream) {
    const int nwork = job.C * job.npairs;
    if (out_type == XC_OUT_CI32)
        hipLaunchKernelGGL(dma::kernel<int2>, dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    else
        hipLaunchKernelGGL(dma::kernel<float2>, dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    return hipGetLastError();
}

hipError_t launch_mfma_dma_batch(xc_out_type out_type, const Job *jobs, const Unit *units, Queues q, int grid,
                                 hipStream_t stream) {
    if (out_type == XC_OUT_CI32)
        hipLaunchKernelGGL(dma::kernel_batch<int2>, dim3(grid), dim3(256), 0, stream, jobs, units, q);
    else
        hipLaunchKernelGGL(dma::kernel_batch<float2>, dim3(grid), dim3(256), 0, stream, jobs, units, q);
    return hipGetLastError();
}

int occupancy_mfma_dma_batch(xc_out_type out_type) {
    int n = 0;
    hipError_t e = out_type == XC_OUT_CI32
                       ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dma::kernel_batch<int2>, 256, 0)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, dma::kernel_batch<float2>, 256, 0);
    return (e != hipSuccess || n < 1) ? 1 : n;
}

}  // namespace xc
