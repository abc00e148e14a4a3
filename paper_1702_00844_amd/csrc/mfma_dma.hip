// Matrix-core correlator kernels for int8 and 16-bit samples with direct
// global-to-LDS staging (gfx950).
//
// The product and the tiling are those of the register-staged kernels: a
// workgroup owns one (channel, block pair bi <= bj) of 64-station blocks, a
// 128 x 128 square of (station, pol) rows; each of its four waves holds a
// 64 x 64 quadrant as 2 x 2 tiles of 32 x 32, and V is accumulated over time
// as Re V = [Xr Xi][Xr Xi]^T and Im V = [Xr Xi][-Xi Xr]^T (int8: minus
// [Xr Xi][Xi -Xr]^T, negated at the store) on 32x32 MFMAs.  What differs is
// how samples reach the matrix cores:
//
//  * global_load_lds copies 16-byte granules (4 int8 or 2 16-bit stations,
//    both pols, one time step) from HBM straight into LDS, without passing
//    through registers (see lds_dma.h).  Two 32 KiB stages (64 int8 or 32
//    16-bit time steps each) alternate: the next chunk is copied while the
//    current one is computed, and one barrier per chunk both publishes a stage
//    and frees the other.  (Measured on the 256-station workload, two long
//    stages beat four short ones, whose extra barriers cost more than the
//    deeper prefetch gains, and a 64 KiB pair, which leaves one workgroup per
//    CU.)
//  * LDS keeps the time-major layout of the input: one row per block and time
//    step (256 bytes int8, 512 bytes 16-bit).  The corner turn to the MFMA
//    operand layout (a (station, pol) row per lane, time along K) happens on
//    the way out of LDS: for int8, ds_read_b64_tr_b16 hands every lane four
//    consecutive time steps of one 16-bit (re, im) element, and two such reads
//    make a lane's 16-byte fragment; for 16-bit samples, whose (re, im) pairs
//    are 32 bits, a lane reads its row at four consecutive time steps with
//    four 4-byte reads.
//  * Granules are XOR-swizzled by time row so that the rows read together fall
//    on different banks: int8 granule g of row t is stored at g ^ 4 (t mod 4)
//    (the four rows of a transpose group), 16-bit granule g at
//    g ^ 8 ((t / 4) mod 2) (the two row sets of a wave's 4-byte reads).
//  * The MFMAs take block J's fragment as their first operand, so that the
//    accumulators hold V with one block-I (station, pol) row per lane: a lane
//    then owns 16 contiguous bytes of the output, and tiles are stored
//    straight from the registers (store_tile_direct), without an LDS image.
//  * On a diagonal block pair the wave of the quadrant below the diagonal
//    computes one tile of quadrant (0, 1), and the diagonal quadrants skip
//    their tile below the diagonal, so that no wave has more than three.
//
// Station counts that are not whole 16-byte granules (n_stations % 4 != 0 for
// int8, odd for 16-bit) are copied in 4-byte granules (G4 below).
#include <type_traits>

#include "common.h"

#include "lds_dma.h"
#include "mfma_parts.h"

namespace xc {
namespace dma {

using mfma::Acc;
using mfma::Out;
using mfma::Vec;
using mfma::K_BF16;
using mfma::K_F16;
using mfma::K_I8;
using mfma::v4i;
using mfma::v8bf;
using mfma::v8h;

constexpr int SB = 64;              // stations per block
constexpr int STAGE = 32768;        // bytes per stage (both blocks)
constexpr int NSTAGE = 2;
// Measured on 256 stations x 1024 channels x 1024 samples: two stages of
// 32 KiB beat three of 24 KiB (0.72 against 0.80 ms for int8), two of 40 KiB
// (0.72) and four of 16 KiB; the kernel is not bound by copy latency.
static_assert(NSTAGE >= 2 && NSTAGE <= 4, "copies in flight are counted for up to two later chunks");
static_assert((NSTAGE - 2) * (STAGE / 2 / 2 / 1024) < 32, "pending copies fit the vmcnt wait");
constexpr int LDS_BYTES = NSTAGE * STAGE;

template <int KIND>
struct Geo {
    static constexpr bool I8 = KIND == K_I8;
    static constexpr int SAMPLE = I8 ? 4 : 8;          // bytes per station (2 pols x (re, im))
    static constexpr int ROWB = SB * SAMPLE;           // bytes of one block's time step
    static constexpr int BLK = STAGE / 2;              // one block's share of a stage
    static constexpr int KT = BLK / ROWB;              // time steps per stage: 64 or 32
    static constexpr int GS = 16 / SAMPLE;             // stations per granule
    static constexpr int LPR = ROWB / 16;              // lanes (granules) per time row: 16 or 32
    static constexpr int RPC = 64 / LPR;               // time rows per copy instruction: 4 or 2
    static constexpr int STEP_T = I8 ? 16 : 8;         // time steps per MFMA k-step
    // LDS granule of logical granule g in time row t (an involution)
    __device__ static int swz(int g, int t) { return I8 ? g ^ (4 * (t & 3)) : g ^ (8 * ((t >> 2) & 1)); }
};

typedef short v4s __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) uint8_t lds_u8;
typedef __attribute__((address_space(3))) v4s lds_v4s;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Wait until at most n (0 <= n < 32) of this wave's vector-memory operations
// are pending.
template <int N = 0>
__device__ __forceinline__ void wait_vm_n(int n) {
    if constexpr (N < 31) {
        if (n == N) wait_vm<N>();
        else wait_vm_n<N + 1>(n);
    } else {
        wait_vm<31>();
    }
}

// Byte offset, within a block's image, of this lane's first read of the 32
// rows from n0 on at the first time step of a k-step.
//  int8: lane group g = lane / 16 takes rows n0 + 16 (g % 2) on and K half
//  g / 2 (time steps 8 (g / 2) on); lane j of a group addresses time step j / 4
//  and the four elements from row 4 (j % 4) (the transpose read then gives
//  lane j row j at four time steps).
//  16-bit: lane l reads row n0 + l % 32 at time step 4 (l / 32) (then + 1, 2, 3).
template <int KIND>
__device__ __forceinline__ uint32_t frag_offset(int n0, int lane) {
    typedef Geo<KIND> G;
    if constexpr (G::I8) {
        const int t = 8 * (lane >> 5) + ((lane & 15) >> 2);
        const int n = n0 + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
        return t * G::ROWB + (G::swz(n >> 3, t) << 4) + (n & 7) * 2;
    } else {
        const int t = 4 * (lane >> 5);
        const int n = n0 + (lane & 31);
        return t * G::ROWB + (G::swz(n >> 2, t) << 4) + (n & 3) * 4;
    }
}

// A lane's 16-byte fragment (K = 8 or 4 time steps of (re, im)) at p.
template <int KIND>
__device__ __forceinline__ v4i frag(const lds_u8 *p) {
    typedef Geo<KIND> G;
    if constexpr (G::I8) {
        const v4s lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)p);
        const v4s hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s *)(p + 4 * G::ROWB));
        const int2 l = __builtin_bit_cast(int2, lo), h = __builtin_bit_cast(int2, hi);
        return v4i{l.x, l.y, h.x, h.y};
    } else {
        return v4i{(int)*(const lds_u32 *)p, (int)*(const lds_u32 *)(p + G::ROWB),
                   (int)*(const lds_u32 *)(p + 2 * G::ROWB), (int)*(const lds_u32 *)(p + 3 * G::ROWB)};
    }
}

template <int KIND, typename ACC>
__device__ __forceinline__ ACC mma(const v4i &a, const v4i &b, const ACC &c) {
    if constexpr (KIND == K_I8)
        return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
    else if constexpr (KIND == K_F16)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), c, 0, 0,
                                                      0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                       0, 0);
}

// Element offset, within one channel's visibilities, of the 16 bytes of
// baseline (i, j) and pol p (both q).  Baselines past the last station or
// below the diagonal are clamped to a valid one, so that accumulate mode can
// fetch a tile's old values without branches (the clamped values are not
// stored).
__device__ __forceinline__ uint32_t piece(int S, int i, int j, int p) {
    const int jc = j < S ? j : S - 1;
    const int ic = i <= jc ? i : jc;
    return (uint32_t)(((size_t)jc * (jc + 1) / 2 + ic) * 4 + p * 2);
}

// Lane L's k-th piece of the tile at (row0, col0) (the order of
// store_tile_direct), for accumulate mode: f(k, element offset).
template <typename F>
__device__ __forceinline__ void tile_pieces(int S, int row0, int col0, int lane, F f) {
    const int m = lane & 31;
    const int i = (row0 >> 1) + (m >> 1);
    const int p = m & 1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int r = (k >> 1) * 4 + (k & 1) * 2;
        const int n = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        f(k, piece(S, i, (col0 >> 1) + (n >> 1), p));
    }
}

// Store (or add, in accumulate mode) one 32 x 32 tile straight from the
// accumulators, whose column (one per lane) is the (station, pol) row
// row0 + lane % 32 of block I and whose register r holds row
// 8 (r / 4) + 4 (lane / 32) + r % 4 of block J's tile from col0.  Registers r
// and r + 1 (r % 4 in {0, 2}) are the two polarisations q of one station j, so
// a lane holds 16 consecutive bytes of V (pol p of station i against both q
// of station j), and the 32 lanes of a half-wave write one baseline row's
// 16 baselines, 512 contiguous bytes: eight 16-byte stores per lane and tile,
// no LDS.  Autocorrelations (i = j) are made Hermitian on the way: XX and YY
// get imaginary part 0 and the p = 1 lane writes YX = conj(XY), XY coming
// from its p = 0 neighbour.  off(k, i, j, p) gives the element offset of the
// lane's k-th 16 bytes (baseline (i, j), pol p); in accumulate mode old(k)
// gives their old value, loaded beforehand at the offsets tile_pieces lists
// (and kept for the stores), so that a tile's eight loads are in flight
// together.
template <typename ACC, typename OUT, bool ACCUMULATE, typename OLD, typename OFF>
__device__ __forceinline__ void store_tile_direct(OUT *__restrict__ V, int S, const ACC &re, const ACC &im, int row0,
                                                  int col0, int lane, OLD old, OFF off) {
    const int m = lane & 31;
    const int i = (row0 >> 1) + (m >> 1);
    const int p = m & 1;
    const bool on_diag = row0 == col0;       // the tile holds autocorrelations (wave-uniform)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int r = (k >> 1) * 4 + (k & 1) * 2;
        const int n = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int jj = (col0 >> 1) + (n >> 1);
        OUT v0 = Out<OUT>::make(re[r], im[r]);            // q = 0
        OUT v1 = Out<OUT>::make(re[r + 1], im[r + 1]);    // q = 1
        if (on_diag) {
            // the p = 0 neighbour's XY (its q = 1 value), for YX = conj(XY)
            const uint32_t xr = (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v1.x), 0xb1, 0xf, 0xf, false);
            const uint32_t xi = (uint32_t)__builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v1.y), 0xb1, 0xf, 0xf, false);
            if (i == jj) {
                if (p == 0) {
                    v0.y = 0;                                  // Im XX
                } else {
                    v0.x = __builtin_bit_cast(decltype(v0.x), xr);
                    v0.y = __builtin_bit_cast(decltype(v0.y), Vec<OUT>::neg(xi));
                    v1.y = 0;                                  // Im YY
                }
            }
        }
        uint4 w = make_uint4(__builtin_bit_cast(uint32_t, v0.x), __builtin_bit_cast(uint32_t, v0.y),
                             __builtin_bit_cast(uint32_t, v1.x), __builtin_bit_cast(uint32_t, v1.y));
        if constexpr (ACCUMULATE) w = Vec<OUT>::add(w, old(k));
        if (jj < S && i <= jj) *reinterpret_cast<uint4 *>(V + off(k, i, jj, p)) = w;
    }
}

// G4: 4-byte granules.  With n_stations a multiple of the 16-byte granule
// (4 int8 or 2 16-bit stations) a copy moves 16 bytes per lane; otherwise a
// time row does not start on a 16-byte boundary, and each lane copies one
// 4-byte word (global_load_lds_dword) instead: a copy then fills 256 bytes of
// one time row (a whole int8 row, half a 16-bit one), four times as many
// copies for the same LDS image.  The swizzle is applied on the source side:
// the word landing at byte 4 L of the row is the one the 16-byte-granule copy
// would have put there.
//
// SM: station-major input x[C][S][T][2] (each station's series contiguous,
// job.sstride = T): the 4-byte copies take each lane's word from its
// station's own series, so the LDS image, and hence the result, is that of
// the time-major input.
template <int KIND, typename OUT, bool G4, bool SM = false>
__device__ __forceinline__ void unit(const Job &job, int c, int bi, int bj, uint8_t *lds_generic) {
    static_assert(G4 || !SM, "station-major input is copied in 4-byte granules");
    typedef Geo<KIND> G;
    typedef typename Acc<KIND>::type acc_t;
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

    // -- copies: per chunk, wave w fills a quarter (diagonal: block I only) or
    // half (elsewhere) of one block's time rows, RPC rows (1 KiB) per copy
    constexpr int NC = G::KT / 2 / G::RPC;              // copies per wave and chunk (half on the diagonal)
    const int blk = diag ? 0 : (wave >> 1);
    const int rbase = diag ? wave * (G::KT / 4) : (wave & 1) * (G::KT / 2);
    const int nload = diag ? NC / 2 : NC;
    const int lrow = lane / G::LPR;
    uint32_t off[NC];     // byte offset of this lane's granule in copy i, from the chunk base
    int stc[NC];          // its first station (past the last station: a valid granule)
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int row = rbase + G::RPC * i + lrow;
        const int st = (blk ? J0 : I0) + G::GS * G::swz(lane % G::LPR, row);
        stc[i] = st < S ? st : S - G::GS;
        off[i] = (uint32_t)((row * S + stc[i]) * G::SAMPLE);
    }
    const uint32_t dst0 = lds_base + blk * G::BLK + rbase * G::ROWB;

    // 4-byte granules: copy i fills bytes 256 h .. 256 h + 255 of time row
    // rbase + i / IPR (h = i % IPR); the word of lane L there belongs to the
    // station and word picked by the row's swizzle phase and h, one of four
    // combinations per lane (rbase is a multiple of 8, so the phase of copy i
    // is i % 4 for int8 and (i / 8) % 2 for 16-bit samples).
    constexpr int IPR = G::ROWB / 256;                  // copies per time row: 1 or 2
    constexpr int NC4 = G::KT / 2 * IPR;                // copies per wave and chunk (half on the diagonal)
    const int nload4 = diag ? NC4 / 2 : NC4;
    uint32_t woff[4];     // byte offset of the lane's word within a time row, per combination
    size_t soff[SM ? 4 : 1];   // station-major: byte offset of the lane's word at time 0 of its station
    if constexpr (G4) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = G::I8 ? v : 4 * (v >> 1);     // a time row of that swizzle phase
            const int h = G::I8 ? 0 : (v & 1);
            const int gl = G::swz(16 * h + lane / 4, t);   // logical granule at the lane's bytes
            const int st = (blk ? J0 : I0) + G::GS * gl + (G::I8 ? lane % 4 : (lane % 4) / 2);
            const int stw = st < S ? st : S - 1;
            woff[v] = (uint32_t)(stw * G::SAMPLE + (G::I8 ? 0 : 4 * (lane & 1)));
            if constexpr (SM)
                soff[v] = ((size_t)c * job.cstride + (size_t)stw * job.sstride) * G::SAMPLE + (G::I8 ? 0 : 4 * (lane & 1));
        }
    }
    auto combo = [&](int i) { return G::I8 ? (i & 3) : (((i >> 3) & 1) * 2 + (i & 1)); };

    auto issue = [&](int ch) {
        const int t0 = ch * G::KT;
        const uint32_t dst = dst0 + (ch % NSTAGE) * STAGE;
        if constexpr (SM) {
#pragma unroll
            for (int i = 0; i < NC4; ++i) {
                if (i >= nload4) break;
                const int t = t0 + rbase + i / IPR;
                const void *src = t < T ? static_cast<const void *>(x + soff[combo(i)] + (size_t)t * G::SAMPLE)
                                        : static_cast<const void *>(g_zero16);
                dma4(src, dst + (i / IPR) * G::ROWB + (i % IPR) * 256);
            }
        } else if constexpr (G4) {
            if (t0 + G::KT <= T && rows_contiguous(job, t0, G::KT)) {
                const uint8_t *src = x + (row_offset(job, c, t0) + (size_t)rbase * S) * G::SAMPLE;
#pragma unroll
                for (int i = 0; i < NC4; ++i)
                    if (i < nload4)
                        dma4(src + (size_t)(i / IPR) * S * G::SAMPLE + woff[combo(i)],
                             dst + (i / IPR) * G::ROWB + (i % IPR) * 256);
            } else {
#pragma unroll
                for (int i = 0; i < NC4; ++i) {
                    if (i >= nload4) break;
                    const int t = t0 + rbase + i / IPR;
                    const void *src = t < T ? static_cast<const void *>(x + row_offset(job, c, t) * G::SAMPLE +
                                                                        woff[combo(i)])
                                            : static_cast<const void *>(g_zero16);
                    dma4(src, dst + (i / IPR) * G::ROWB + (i % IPR) * 256);
                }
            }
        } else if (t0 + G::KT <= T && rows_contiguous(job, t0, G::KT)) {
            const uint8_t *src = x + row_offset(job, c, t0) * G::SAMPLE;
#pragma unroll
            for (int i = 0; i < NC; ++i)
                if (i < nload) dma16(src + off[i], dst + i * G::RPC * G::ROWB);
        } else {
#pragma unroll
            for (int i = 0; i < NC; ++i) {
                if (i >= nload) break;
                const int t = t0 + rbase + G::RPC * i + lrow;
                const void *src = t < T ? static_cast<const void *>(x + (row_offset(job, c, t) + stc[i]) * G::SAMPLE)
                                        : static_cast<const void *>(g_zero16);
                dma16(src, dst + i * G::RPC * G::ROWB);
            }
        }
    };
    const int npend = G4 ? nload4 : nload;    // copies per wave and chunk

    // -- tiles of this wave.  Wave (wr, wc) takes the 2 x 2 tiles of quadrant
    // (wr, wc) of the block pair's 128 x 128 (station, pol) rows.  On a
    // diagonal pair the quadrant below the diagonal has no outputs: its wave
    // takes the last tile of quadrant (0, 1) instead, and the quadrants on
    // the diagonal skip their tile below it, so no wave computes more than
    // three tiles (a diagonal unit then takes three quarters of the time).
    int rrow[2], ccol[2];   // first (station, pol) row of the wave's tile rows (block I) and columns (block J)
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        rrow[k] = wr * SB + 32 * k;
        ccol[k] = wc * SB + 32 * k;
    }
    const bool lend = diag && wr == 0 && wc == 1;
    const bool borrow = diag && wr == 1 && wc == 0;
    if (borrow) {
        rrow[0] = rrow[1] = 32;
        ccol[0] = ccol[1] = SB + 32;
    }
    bool run[2][2];
    bool any = false;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int cs = 0; cs < 2; ++cs) {
            const int r0 = I0 * 2 + rrow[rs];
            const int c0 = J0 * 2 + ccol[cs];
            const bool below = (r0 >> 1) > ((c0 + 31) >> 1);
            run[rs][cs] = !below && r0 < 2 * S && c0 < 2 * S;
        }
    if (lend) run[1][1] = false;
    if (borrow) run[0][0] = run[0][1] = run[1][0] = false;
#pragma unroll
    for (int rs = 0; rs < 2; ++rs)
#pragma unroll
        for (int cs = 0; cs < 2; ++cs) any |= run[rs][cs];
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
        aoff[k] = frag_offset<KIND>(rrow[k], lane);
        boff[k] = (diag ? 0 : G::BLK) + frag_offset<KIND>(ccol[k], lane);
    }

    const int nchunk = (T + G::KT - 1) / G::KT;
#pragma unroll
    for (int k = 0; k < NSTAGE - 1; ++k)
        if (k < nchunk) issue(k);
    // The chunk loop, compiled once per set of tiles a wave computes (bit
    // 2 rs + cs for tile (rs, cs)): every tile (15), a diagonal quadrant
    // without its tile below the diagonal (11), quadrant (0, 1) of a diagonal
    // pair without the tile it hands over (7), the handed-over tile alone (8),
    // none (0: the wave only copies).  Tiles past the last station are
    // computed on clamped samples and not stored.
    auto chunks = [&](auto mask_c) {
        constexpr int MASK = decltype(mask_c)::value;
        constexpr bool NA0 = MASK & 3, NA1 = MASK & 12, NB0 = MASK & 5, NB1 = MASK & 10;
        for (int ch = 0; ch < nchunk; ++ch) {
            // this wave's copies of chunk ch are done once only those of the
            // (at most NSTAGE - 2) chunks issued after it may be pending
            const int later = min(nchunk - 1 - ch, NSTAGE - 2);
            wait_vm_n(later * npend);
            barrier_lds();
            // every wave is past chunk ch - 1: its stage takes chunk ch + NSTAGE - 1
            if (ch + NSTAGE - 1 < nchunk) issue(ch + NSTAGE - 1);
            if constexpr (MASK == 0) continue;
            const lds_u8 *sb = lds + (ch % NSTAGE) * STAGE;
            // (The compiler reads two k-steps' fragments, then issues their
            // MFMAs.  Reading k-step ks + 1 before the MFMAs of ks, held in
            // place by scheduling fences, measured no faster: the other wave
            // of the SIMD covers the LDS latency.)
#pragma unroll
            for (int ks = 0; ks < G::KT / G::STEP_T; ++ks) {
                v4i a[2] = {}, b[2] = {}, bn[2] = {};
                const int dt = ks * G::STEP_T * G::ROWB;
                if constexpr (NA0) a[0] = frag<KIND>(sb + aoff[0] + dt);
                if constexpr (NA1) a[1] = frag<KIND>(sb + aoff[1] + dt);
                if constexpr (NB0) b[0] = frag<KIND>(sb + boff[0] + dt);
                if constexpr (NB1) b[1] = frag<KIND>(sb + boff[1] + dt);
#pragma unroll
                for (int k = 0; k < 2; ++k)
                    if ((k == 0 && NB0) || (k == 1 && NB1))
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            bn[k][e] = (int)(G::I8 ? mfma::conj_neg_i8((uint32_t)b[k][e])
                                                   : mfma::conj_swap_h((uint32_t)b[k][e]));
                // B first: the accumulator's columns (one per lane) are then
                // the (station, pol) rows of block I, its rows (registers)
                // those of block J, which is the order of the output in memory
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (MASK & (1 << t)) are[t >> 1][t & 1] = mma<KIND>(b[t & 1], a[t >> 1], are[t >> 1][t & 1]);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (MASK & (1 << t)) aim[t >> 1][t & 1] = mma<KIND>(bn[t & 1], a[t >> 1], aim[t >> 1][t & 1]);
            }
        }
    };
    // wave-uniform choice of the loop
    const int mask = !any ? 0 : borrow ? 8 : lend ? 7 : (diag && wr == wc) ? 11 : 15;
    switch (mask) {
    case 15: chunks(std::integral_constant<int, 15>{}); break;
    case 11: chunks(std::integral_constant<int, 11>{}); break;
    case 7: chunks(std::integral_constant<int, 7>{}); break;
    case 8: chunks(std::integral_constant<int, 8>{}); break;
    default: chunks(std::integral_constant<int, 0>{}); break;
    }
    if (!any) return;
    if constexpr (G::I8) {
        // the int8 accumulators hold minus the imaginary part
#pragma unroll
        for (int rs = 0; rs < 2; ++rs)
#pragma unroll
            for (int cs = 0; cs < 2; ++cs) aim[rs][cs] = -aim[rs][cs];
    }
    OUT *__restrict__ V = static_cast<OUT *>(job.vis) + (size_t)c * ((size_t)S * (S + 1) / 2) * 4;
    if (!job.accumulate) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int rs = t >> 1, cs = t & 1;
            if (run[rs][cs])
                store_tile_direct<acc_t, OUT, false>(
                    V, S, are[rs][cs], aim[rs][cs], I0 * 2 + rrow[rs], J0 * 2 + ccol[cs], lane,
                    [](int) { return uint4{}; }, [&](int, int i, int j, int p) { return piece(S, i, j, p); });
        }
        return;
    }
    // Accumulate mode, one tile at a time: the tile's old values are loaded
    // together, then added and stored.  (Fetching all tiles' old values at
    // once, two of them into the free stages, measured no faster.)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int rs = t >> 1, cs = t & 1;
        if (!run[rs][cs]) continue;
        const int row0 = I0 * 2 + rrow[rs], col0 = J0 * 2 + ccol[cs];
        uint4 old[8];
        uint32_t e[8];
        tile_pieces(S, row0, col0, lane, [&](int k, uint32_t ek) {
            e[k] = ek;
            old[k] = *reinterpret_cast<const uint4 *>(V + ek);
        });
        store_tile_direct<acc_t, OUT, true>(V, S, are[rs][cs], aim[rs][cs], row0, col0, lane,
                                            [&](int k) { return old[k]; }, [&](int k, int, int, int) { return e[k]; });
    }
}

template <int KIND, typename OUT, bool G4, bool SM = false>
__global__ __launch_bounds__(256, 2) void kernel(Job job, int nwork) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const int w = xcd_remap(blockIdx.x, nwork);
    if (w < 0) return;
    int c, bi, bj;
    unit_decode(job, w, c, bi, bj);
    unit<KIND, OUT, G4, SM>(job, c, bi, bj, lds);
}

template <int KIND, typename OUT, bool G4>
__global__ __launch_bounds__(256, 2) void kernel_batch(const Job *__restrict__ jobs, const Unit *__restrict__ units,
                                                       const int *__restrict__ bounds) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[LDS_BYTES];
    const int u = batch_unit(bounds, blockIdx.x);
    if (u < 0) return;
    const Unit un = units[u];
    const Job job = jobs[un.item];
    unit<KIND, OUT, G4>(job, un.channel, un.bi, un.bj, lds);
}

template <int KIND, typename OUT>
hipError_t launch_t(const Job &job, hipStream_t stream) {
    const int nwork = job_units(job);
    if (job.S % Geo<KIND>::GS)
        hipLaunchKernelGGL((kernel<KIND, OUT, true>), dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    else
        hipLaunchKernelGGL((kernel<KIND, OUT, false>), dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    return hipGetLastError();
}
template <int KIND, typename OUT>
hipError_t launch_sm_t(const Job &job, hipStream_t stream) {
    const int nwork = job_units(job);
    hipLaunchKernelGGL((kernel<KIND, OUT, true, true>), dim3(xcd_grid(nwork)), dim3(256), 0, stream, job, nwork);
    return hipGetLastError();
}
template <int KIND, typename OUT>
hipError_t launch_batch_t(const Job *jobs, const Unit *units, const int *bounds, int grid, bool g4,
                          hipStream_t stream) {
    if (g4)
        hipLaunchKernelGGL((kernel_batch<KIND, OUT, true>), dim3(grid), dim3(256), 0, stream, jobs, units, bounds);
    else
        hipLaunchKernelGGL((kernel_batch<KIND, OUT, false>), dim3(grid), dim3(256), 0, stream, jobs, units, bounds);
    return hipGetLastError();
}
#define XC_DMA_DISPATCH(FN, ...)                                                                      \
    switch (in_type) {                                                                                \
    case XC_IN_CI8:                                                                                   \
        return out_type == XC_OUT_CI32 ? FN<K_I8, int2>(__VA_ARGS__) : FN<K_I8, float2>(__VA_ARGS__); \
    case XC_IN_CF16: return FN<K_F16, float2>(__VA_ARGS__);                                           \
    case XC_IN_CBF16: return FN<K_BF16, float2>(__VA_ARGS__);                                         \
    default: break;                                                                                   \
    }

}  // namespace dma

hipError_t launch_mfma_dma(xc_in_type in_type, xc_out_type out_type, const Job &job, hipStream_t stream) {
    using namespace dma;
    XC_DMA_DISPATCH(launch_t, job, stream)
    return hipErrorInvalidValue;
}

hipError_t launch_mfma_dma_station_major(xc_in_type in_type, xc_out_type out_type, const Job &job,
                                         hipStream_t stream) {
    using namespace dma;
    XC_DMA_DISPATCH(launch_sm_t, job, stream)
    return hipErrorInvalidValue;
}

hipError_t launch_mfma_dma_batch(xc_in_type in_type, xc_out_type out_type, const Job *jobs, const Unit *units,
                                 const int *bounds, int grid, bool g4, hipStream_t stream) {
    using namespace dma;
    XC_DMA_DISPATCH(launch_batch_t, jobs, units, bounds, grid, g4, stream)
    return hipErrorInvalidValue;
}

}  // namespace xc
