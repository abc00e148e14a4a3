// Building blocks shared by the matrix-core correlator kernels (gfx950):
// geometry of a (sample type, block size) variant, staging of time chunks
// (global -> registers -> LDS, with the corner turn for 8- and 16-bit
// samples), one chunk of MFMAs for a wave's quadrant, and the tile stores.
// The kernels themselves are in mfma.hip (register staging, four waves per
// workgroup) and mfma_dma.hip (copies straight into LDS; it stores its tiles
// straight from the accumulators and takes the sample kinds, accumulator and
// output types and conjugation helpers from here).
#pragma once
#include "common.h"

namespace xc {
namespace mfma {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

enum Kind { K_I8 = 0, K_F16 = 1, K_BF16 = 2, K_F32 = 3 };

// Compile-time geometry of one (kind, block size) variant.
template <int KIND, int SB>
struct Geo {
    static constexpr int RB = 2 * SB;                 // rows (station, pol) per block
    static constexpr int NS = SB / 32;                // 32x32 tiles per wave side
    static constexpr bool TRANSPOSED = KIND != K_F32;
    // time steps per staged chunk
    static constexpr int KT = KIND == K_I8 ? 64 : (KIND == K_F32 ? 16 : 32);
    // bytes of one sample (re, im)
    static constexpr int EB = KIND == K_I8 ? 2 : (KIND == K_F32 ? 8 : 4);
    // transposed: one row per (station, pol) of KT samples, +16 bytes pad;
    // f32: one row per time step of both blocks' stations
    static constexpr int PITCH = TRANSPOSED ? KT * EB + 16 : 2 * RB * 8;
    static constexpr int STAGE_BYTES = TRANSPOSED ? 2 * RB * PITCH : KT * PITCH;
    // staging tasks per chunk (both blocks): int8 = 4 stations x 8 steps,
    // 16-bit = 2 stations x 4 steps, f32 = one station x one step
    static constexpr int NTASK = KIND == K_I8 ? 2 * (SB / 4) * (KT / 8)
                               : (KIND == K_F32 ? 2 * SB * KT : 2 * (SB / 2) * (KT / 4));
    static constexpr int NPT = (NTASK + 255) / 256;   // tasks per thread
    static constexpr int WORDS = KIND == K_I8 ? 32 : (KIND == K_F32 ? 4 : 16);  // dwords per task
    static constexpr int STEP_T = KIND == K_I8 ? 16 : (KIND == K_F32 ? 2 : 8);   // time steps per MFMA
};

template <int KIND>
struct Acc {
    typedef v16f type;
};
template <>
struct Acc<K_I8> {
    typedef v16i type;
};

// (re, im) pairs -> (-im, re) pairs.
__device__ __forceinline__ uint32_t conj_swap_i8(uint32_t w) {
    // byte-wise two's-complement negation without carries between bytes
    const uint32_t nw = ~w;
    const uint32_t neg = ((nw & 0x7f7f7f7fu) + 0x01010101u) ^ (nw & 0x80808080u);
    // bytes: [re0 im0 re1 im1] -> [-im0 re0 -im1 re1]
    return __builtin_amdgcn_perm(neg, w, 0x02070005u);
}
// (re, im) pairs -> (im, -re) pairs, i.e. -i times the conjugate swap above:
// products with it accumulate minus the imaginary part.  Each 16-bit half
// h = re + 256 im times 0xff00 is 256 (-re) modulo 2^16; adding im (moved to
// the low byte by a permute) completes the pair.  Two instructions per word.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t conj_neg_i8(uint32_t w) {
    const uint32_t im = __builtin_amdgcn_perm(0u, w, 0x0c030c01u);   // [im0 0 im1 0]
    const u16x2 h = __builtin_bit_cast(u16x2, w);
    const u16x2 r = h * (u16x2){0xff00, 0xff00} + __builtin_bit_cast(u16x2, im);
    return __builtin_bit_cast(uint32_t, r);
}
__device__ __forceinline__ uint32_t conj_swap_h(uint32_t w) {
    // halves: [re im] -> [-im re]   (sign-bit flip is exact negation)
    const uint32_t sw = __builtin_amdgcn_perm(w, w, 0x01000302u);
    return sw ^ 0x00008000u;
}

struct Blocks {
    int I0, J0;     // first station of block I / J
    bool diag;      // bi == bj: J rows are I rows, only I is staged
};

// ---------------------------------------------------------------------------
// Global -> registers -> LDS staging.  Thread tid handles tasks tid, tid + 256...
// Within a block, the time group is the fastest task index so that the eight
// lanes of a group write one 128-byte row segment of LDS.

template <int KIND, int SB>
struct Pre {
    uint32_t w[Geo<KIND, SB>::NPT][Geo<KIND, SB>::WORDS];
};

// Station counts that are multiples of the staging group (4 stations for
// int8, 2 for 16-bit) put every group wholly inside or outside the array, so
// staging loads need no per-station checks: out-of-range groups and time
// steps read a clamped, valid address and are replaced by zeros.
template <int KIND, int SB>
__device__ __forceinline__ void gload(Pre<KIND, SB> &p, const Job &job, const uint8_t *__restrict__ x, int c,
                                      const Blocks &bk, int t0, int tid) {
    typedef Geo<KIND, SB> G;
    const int S = job.S;
    const int T = job.T;
#pragma unroll
    for (int h = 0; h < G::NPT; ++h) {
        const int task = tid + 256 * h;
        if (G::NTASK % 256 != 0 && task >= G::NTASK) break;
        if constexpr (KIND == K_I8) {
            constexpr int NB = G::NTASK / 2;
            const int blk = task / NB;
            const int r = task % NB;
            const int sg = r / (G::KT / 8);
            const int tg = r % (G::KT / 8);
            const int s = (blk ? bk.J0 : bk.I0) + sg * 4;
            if (blk && bk.diag) continue;                 // wave-uniform: J rows are I rows
            const uint32_t *xw = reinterpret_cast<const uint32_t *>(x);
            if ((S & 3) == 0) {
                const bool sok = s < S;
                const int sc = sok ? s : 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int t = t0 + tg * 8 + k;
                    const bool ok = sok && t < T;
                    const int tc = t < T ? t : T - 1;
                    const uint4 v = *reinterpret_cast<const uint4 *>(xw + row_offset(job, c, tc) + sc);
                    p.w[h][4 * k + 0] = ok ? v.x : 0u; p.w[h][4 * k + 1] = ok ? v.y : 0u;
                    p.w[h][4 * k + 2] = ok ? v.z : 0u; p.w[h][4 * k + 3] = ok ? v.w : 0u;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int t = t0 + tg * 8 + k;
                    const bool tok = t < T;
                    const uint32_t *row = xw + (tok ? row_offset(job, c, t) : 0);
#pragma unroll
                    for (int d = 0; d < 4; ++d) p.w[h][4 * k + d] = (tok && s + d < S) ? row[s + d] : 0u;
                }
            }
        } else if constexpr (KIND == K_F32) {
            const int t = task / (2 * SB);
            const int s2 = task % (2 * SB);
            const int blk = s2 / SB;
            const int st = (blk ? bk.J0 : bk.I0) + s2 % SB;
            const bool ok = !(blk && bk.diag) && (t0 + t < T) && st < S;
            const int tc = t0 + t < T ? t0 + t : T - 1;
            const int sc = st < S ? st : 0;
            const float4 *xs = reinterpret_cast<const float4 *>(x);
            const float4 v = xs[row_offset(job, c, tc) + sc];
            p.w[h][0] = ok ? __float_as_uint(v.x) : 0u; p.w[h][1] = ok ? __float_as_uint(v.y) : 0u;
            p.w[h][2] = ok ? __float_as_uint(v.z) : 0u; p.w[h][3] = ok ? __float_as_uint(v.w) : 0u;
        } else {
            constexpr int NB = G::NTASK / 2;
            const int blk = task / NB;
            const int r = task % NB;
            const int sg = r / (G::KT / 4);
            const int tg = r % (G::KT / 4);
            const int s = (blk ? bk.J0 : bk.I0) + sg * 2;
            if (blk && bk.diag) continue;                 // wave-uniform
            const uint32_t *xw = reinterpret_cast<const uint32_t *>(x);
            if ((S & 1) == 0) {
                const bool sok = s < S;
                const int sc = sok ? s : 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int t = t0 + tg * 4 + k;
                    const bool ok = sok && t < T;
                    const int tc = t < T ? t : T - 1;
                    const uint4 v = *reinterpret_cast<const uint4 *>(xw + 2 * row_offset(job, c, tc) + 2 * sc);
                    p.w[h][4 * k + 0] = ok ? v.x : 0u; p.w[h][4 * k + 1] = ok ? v.y : 0u;
                    p.w[h][4 * k + 2] = ok ? v.z : 0u; p.w[h][4 * k + 3] = ok ? v.w : 0u;
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int t = t0 + tg * 4 + k;
                    const bool tok = t < T;
                    const uint32_t *row = xw + (tok ? 2 * row_offset(job, c, t) : 0);
#pragma unroll
                    for (int d = 0; d < 4; ++d)
                        p.w[h][4 * k + d] = (tok && s + (d >> 1) < S) ? row[2 * s + d] : 0u;
                }
            }
        }
    }
}

// Loads of a full chunk whose time steps are consecutive rows in memory, for
// station counts that are multiples of the staging group: a uniform base
// address per chunk plus per-thread byte offsets fixed for the whole unit, so
// that a load needs no address arithmetic.  Groups past the last station read
// the last group instead of zeros: they only feed output rows and columns
// that are never stored.
template <int KIND, int SB>
struct LoadPlan {
    uint32_t voff[Geo<KIND, SB>::NPT];   // byte offset of the task's first sample from the chunk base
    bool skip[Geo<KIND, SB>::NPT];       // uniform per wave: block J of a diagonal pair (or no task)
    uint32_t kstride;                    // bytes between the task's consecutive loads
};

template <int KIND, int SB>
__device__ __forceinline__ bool fast_loads_ok(const Job &job) {
    return KIND == K_I8 ? (job.S & 3) == 0 : (KIND == K_F32 ? true : (job.S & 1) == 0);
}

template <int KIND, int SB>
__device__ __forceinline__ LoadPlan<KIND, SB> make_load_plan(const Job &job, const Blocks &bk, int tid) {
    typedef Geo<KIND, SB> G;
    LoadPlan<KIND, SB> lp;
    const int S = job.S;
#pragma unroll
    for (int h = 0; h < G::NPT; ++h) {
        const int task = tid + 256 * h;
        if constexpr (KIND == K_I8 || KIND == K_F16 || KIND == K_BF16) {
            constexpr int GS = KIND == K_I8 ? 4 : 2;        // stations per task
            constexpr int TG = KIND == K_I8 ? 8 : 4;        // time steps per task
            constexpr int SBYTES = KIND == K_I8 ? 4 : 8;    // bytes per station sample
            constexpr int NB = G::NTASK / 2;
            const int blk = task / NB;
            const int r = task % NB;
            const int sg = r / (G::KT / TG);
            const int tg = r % (G::KT / TG);
            const int st = (blk ? bk.J0 : bk.I0) + sg * GS;
            lp.voff[h] = (uint32_t)((tg * TG * S + (st < S ? st : S - GS)) * SBYTES);
            const bool none = (G::NTASK % 256 != 0 && task >= G::NTASK) || (blk && bk.diag);
            lp.skip[h] = __builtin_amdgcn_readfirstlane((int)none) != 0;
            lp.kstride = (uint32_t)(S * SBYTES);
        } else {
            const int t = task / (2 * SB);
            const int s2 = task % (2 * SB);
            const int st = (s2 < SB ? bk.I0 : bk.J0) + s2 % SB;
            lp.voff[h] = (uint32_t)((t * S + (st < S ? st : S - 1)) * 16);
            lp.skip[h] = false;          // block J of a diagonal pair is loaded and not stored
            lp.kstride = 0;
        }
    }
    return lp;
}

template <int KIND, int SB>
__device__ __forceinline__ void gload_full(Pre<KIND, SB> &p, const uint8_t *base, const LoadPlan<KIND, SB> &lp) {
    typedef Geo<KIND, SB> G;
#pragma unroll
    for (int h = 0; h < G::NPT; ++h) {
        if (lp.skip[h]) continue;
        constexpr int NL = KIND == K_I8 ? 8 : (KIND == K_F32 ? 1 : 4);   // 16-byte loads per task
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const uint4 v = *reinterpret_cast<const uint4 *>(base + (size_t)k * lp.kstride + lp.voff[h]);
            p.w[h][4 * k + 0] = v.x; p.w[h][4 * k + 1] = v.y; p.w[h][4 * k + 2] = v.z; p.w[h][4 * k + 3] = v.w;
        }
    }
}

template <int KIND, int SB>
__device__ __forceinline__ void lstore(const Pre<KIND, SB> &p, uint8_t *lds, const Blocks &bk, int tid) {
    typedef Geo<KIND, SB> G;
#pragma unroll
    for (int h = 0; h < G::NPT; ++h) {
        const int task = tid + 256 * h;
        if (G::NTASK % 256 != 0 && task >= G::NTASK) break;
        if constexpr (KIND == K_I8) {
            constexpr int NB = G::NTASK / 2;
            const int blk = task / NB;
            if (blk && bk.diag) continue;
            const int r = task % NB;
            const int sg = r / (G::KT / 8);
            const int tg = r % (G::KT / 8);
#pragma unroll
            for (int d = 0; d < 4; ++d) {
#pragma unroll
                for (int pol = 0; pol < 2; ++pol) {
                    // bytes of (station d, pol) at 8 consecutive steps
                    const uint32_t sel = pol ? 0x07060302u : 0x05040100u;
                    uint4 o;
                    o.x = __builtin_amdgcn_perm(p.w[h][4 * 1 + d], p.w[h][4 * 0 + d], sel);
                    o.y = __builtin_amdgcn_perm(p.w[h][4 * 3 + d], p.w[h][4 * 2 + d], sel);
                    o.z = __builtin_amdgcn_perm(p.w[h][4 * 5 + d], p.w[h][4 * 4 + d], sel);
                    o.w = __builtin_amdgcn_perm(p.w[h][4 * 7 + d], p.w[h][4 * 6 + d], sel);
                    const int row = blk * G::RB + (sg * 4 + d) * 2 + pol;
                    *reinterpret_cast<uint4 *>(lds + row * G::PITCH + tg * 16) = o;
                }
            }
        } else if constexpr (KIND == K_F32) {
            const int t = task / (2 * SB);
            const int s2 = task % (2 * SB);
            if (s2 >= SB && bk.diag) continue;
            uint4 o;
            o.x = p.w[h][0]; o.y = p.w[h][1]; o.z = p.w[h][2]; o.w = p.w[h][3];
            *reinterpret_cast<uint4 *>(lds + t * G::PITCH + s2 * 16) = o;
        } else {
            constexpr int NB = G::NTASK / 2;
            const int blk = task / NB;
            if (blk && bk.diag) continue;
            const int r = task % NB;
            const int sg = r / (G::KT / 4);
            const int tg = r % (G::KT / 4);
#pragma unroll
            for (int d = 0; d < 4; ++d) {   // d = 2 * station_in_pair + pol == row offset
                uint4 o;
                o.x = p.w[h][0 + d]; o.y = p.w[h][4 + d]; o.z = p.w[h][8 + d]; o.w = p.w[h][12 + d];
                const int row = blk * G::RB + sg * 4 + d;
                *reinterpret_cast<uint4 *>(lds + row * G::PITCH + tg * 16) = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One chunk of MFMAs for one wave's quadrant.  ALL: every tile of the quadrant
// is computed (no per-tile checks in the instruction stream); otherwise tiles
// with run[] false are skipped.  The fragments of the next k-step are read
// from LDS before the current k-step's MFMAs are issued.  mid() is called
// half-way through the k-steps, behind the MFMAs queued so far.
template <int KIND, int SB, bool ALL, typename MID>
__device__ __forceinline__ void compute_chunk(const uint8_t *lds, typename Acc<KIND>::type (&are)[SB / 32][SB / 32],
                                              typename Acc<KIND>::type (&aim)[SB / 32][SB / 32], int arow0,
                                              int brow0, const bool (&run)[SB / 32][SB / 32], int lane, MID &&mid) {
    typedef Geo<KIND, SB> G;
    constexpr int NS = G::NS;
    const int r32 = lane & 31;
    const int half = lane >> 5;
    if constexpr (KIND == K_F32) {
#pragma unroll 2
        for (int ks = 0; ks < G::KT / 2; ++ks) {
            const int t = ks * 2 + half;
            float2 a[NS], b[NS];
#pragma unroll
            for (int rs = 0; rs < NS; ++rs)
                a[rs] = *reinterpret_cast<const float2 *>(lds + t * G::PITCH + (arow0 + rs * 32 + r32) * 8);
#pragma unroll
            for (int cs = 0; cs < NS; ++cs)
                b[cs] = *reinterpret_cast<const float2 *>(lds + t * G::PITCH + (brow0 + cs * 32 + r32) * 8);
#pragma unroll
            for (int rs = 0; rs < NS; ++rs) {
#pragma unroll
                for (int cs = 0; cs < NS; ++cs) {
                    if (!ALL && !run[rs][cs]) continue;
                    are[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rs].x, b[cs].x, are[rs][cs], 0, 0, 0);
                    aim[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rs].y, b[cs].x, aim[rs][cs], 0, 0, 0);
                    are[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rs].y, b[cs].y, are[rs][cs], 0, 0, 0);
                    aim[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[rs].x, -b[cs].y, aim[rs][cs], 0, 0, 0);
                }
            }
            if (ks == G::KT / 4 - 1) mid();
        }
    } else {
        constexpr int NSTEP = G::KT / G::STEP_T;  // 4
        v4i fa[2][NS], fb[2][NS];
        auto frag = [&](int ks, v4i (&a)[NS], v4i (&b)[NS]) {
            const int koff = ks * 32 + half * 16;
#pragma unroll
            for (int rs = 0; rs < NS; ++rs)
                a[rs] = *reinterpret_cast<const v4i *>(lds + (arow0 + rs * 32 + r32) * G::PITCH + koff);
#pragma unroll
            for (int cs = 0; cs < NS; ++cs)
                b[cs] = *reinterpret_cast<const v4i *>(lds + (brow0 + cs * 32 + r32) * G::PITCH + koff);
        };
        frag(0, fa[0], fb[0]);
#pragma unroll
        for (int ks = 0; ks < NSTEP; ++ks) {
            const int cur = ks & 1;
            if (ks + 1 < NSTEP) frag(ks + 1, fa[cur ^ 1], fb[cur ^ 1]);
            const v4i(&a)[NS] = fa[cur];
            const v4i(&b)[NS] = fb[cur];
            v4i bi[NS];
#pragma unroll
            for (int cs = 0; cs < NS; ++cs)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t w = (uint32_t)b[cs][e];
                    bi[cs][e] = (int)(KIND == K_I8 ? conj_neg_i8(w) : conj_swap_h(w));
                }
            // real parts of every tile first, then imaginary parts
#pragma unroll
            for (int rs = 0; rs < NS; ++rs) {
#pragma unroll
                for (int cs = 0; cs < NS; ++cs) {
                    if (!ALL && !run[rs][cs]) continue;
                    if constexpr (KIND == K_I8)
                        are[rs][cs] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[rs], b[cs], are[rs][cs], 0, 0, 0);
                    else if constexpr (KIND == K_F16)
                        are[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(v8h, a[rs]), __builtin_bit_cast(v8h, b[cs]), are[rs][cs], 0, 0, 0);
                    else
                        are[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(v8bf, a[rs]), __builtin_bit_cast(v8bf, b[cs]), are[rs][cs], 0, 0, 0);
                }
            }
#pragma unroll
            for (int rs = 0; rs < NS; ++rs) {
#pragma unroll
                for (int cs = 0; cs < NS; ++cs) {
                    if (!ALL && !run[rs][cs]) continue;
                    if constexpr (KIND == K_I8)
                        aim[rs][cs] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[rs], bi[cs], aim[rs][cs], 0, 0, 0);
                    else if constexpr (KIND == K_F16)
                        aim[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(v8h, a[rs]), __builtin_bit_cast(v8h, bi[cs]), aim[rs][cs], 0, 0, 0);
                    else
                        aim[rs][cs] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(v8bf, a[rs]), __builtin_bit_cast(v8bf, bi[cs]), aim[rs][cs], 0, 0, 0);
                }
            }
            if (ks == NSTEP / 2 - 1) mid();
        }
    }
}

// ---------------------------------------------------------------------------
// Output: accumulator element (lane, r) of a 32 x 32 tile is row
// 8 (r / 4) + 4 (lane / 32) + r % 4, column lane % 32.
template <typename OUT>
struct Out;
template <>
struct Out<float2> {
    __device__ static float2 make(float re, float im) { return make_float2(re, im); }
    __device__ static float2 add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
};
template <>
struct Out<int2> {
    __device__ static int2 make(int re, int im) { return make_int2(re, im); }
    __device__ static int2 add(int2 a, int2 b) { return make_int2(a.x + b.x, a.y + b.y); }
};

template <typename ACC, typename OUT>
__device__ __forceinline__ void store_tile(const Job &job, int c, const ACC &re, const ACC &im, int row0, int col0,
                                           int lane) {
    // row0/col0: global (station, pol) row of the tile's first row/column
    const int S = job.S;
    const int col = col0 + (lane & 31);
    const int j = col >> 1;
    const int q = col & 1;
    if (j >= S) return;
    OUT *__restrict__ V = static_cast<OUT *>(job.vis) + (size_t)c * ((size_t)S * (S + 1) / 2) * 4;
    const size_t jbase = (size_t)j * (j + 1) / 2;
    // two halves of 8 rows; in accumulate mode a half's old values (and the
    // YX elements its even rows write for autocorrelations) are all loaded
    // before its first store, so that the loads are in flight together
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        OUT old[8], old2[4];
        if (job.accumulate) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int r = 8 * h + k;
                const int row = row0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int i = (row >> 1) <= j ? (row >> 1) : j;     // clamped: the value is not used
                old[k] = V[(jbase + i) * 4 + (row & 1) * 2 + q];
                if ((k & 1) == 0) old2[k >> 1] = V[(jbase + i) * 4 + 2];
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = 8 * h + k;
            const int row = row0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int i = row >> 1;
            const int p = row & 1;
            if (i > j) continue;
            auto vr = re[r];
            auto vi = im[r];
            if (i == j) {
                if (p == 1 && q == 0) continue;      // written as conj(XY) by the q = 1 lane
                if (p == q) vi = 0;
            }
            OUT v = Out<OUT>::make(vr, vi);
            const size_t e = (jbase + i) * 4 + p * 2 + q;
            if (job.accumulate) v = Out<OUT>::add(v, old[k]);
            V[e] = v;
            if (i == j && p == 0 && q == 1) {       // YX = conj(XY) for autocorrelations
                OUT w = Out<OUT>::make(vr, -vi);
                const size_t e2 = (jbase + i) * 4 + 2;
                if (job.accumulate) w = Out<OUT>::add(w, old2[k >> 1]);
                V[e2] = w;
            }
        }
    }
}

// Coalesced store of a 32 x 32 tile (16 x 16 station pairs) through this
// wave's private LDS region: the accumulators are written as an image of the
// output (for each station j, the 16 baselines (i, j) of 32 bytes each, rows
// padded by 16 bytes), then every lane stores whole baselines, so that 16
// consecutive lanes write one 512-byte run of V.  Autocorrelations are made
// Hermitian (XX, YY real; YX = conj XY) on the way out.
constexpr int IMG_ROW = 16 * 32 + 16;   // bytes per station j in a tile image
constexpr int IMG_BYTES = 16 * IMG_ROW;
// Byte offset of baseline (i, j) of a tile image: the second half of a row
// is moved up 16 bytes so that the 16 baselines a quarter-wave reads at once
// fall on different banks (the row padding makes room for it).
__device__ __forceinline__ int img_offset(int jl, int il) { return jl * IMG_ROW + il * 32 + (il >> 3) * 16; }

template <typename OUT>
struct Vec;
template <>
struct Vec<float2> {
    __device__ static uint4 add(uint4 a, uint4 b) {
        return make_uint4(__float_as_uint(__uint_as_float(a.x) + __uint_as_float(b.x)),
                          __float_as_uint(__uint_as_float(a.y) + __uint_as_float(b.y)),
                          __float_as_uint(__uint_as_float(a.z) + __uint_as_float(b.z)),
                          __float_as_uint(__uint_as_float(a.w) + __uint_as_float(b.w)));
    }
    __device__ static uint32_t neg(uint32_t v) { return v ^ 0x80000000u; }
};
template <>
struct Vec<int2> {
    __device__ static uint4 add(uint4 a, uint4 b) { return make_uint4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
    __device__ static uint32_t neg(uint32_t v) { return 0u - v; }
};

// Old values of the whole baselines this lane stores for one tile (accumulate
// mode), in the order the store visits them.  Every lane loads: addresses of
// baselines past the last station or below the diagonal are clamped to a
// valid one (its value is discarded), so the loads need no branches and can
// be issued well before they are used.
template <typename OUT>
__device__ __forceinline__ void tile_old(const Job &job, int c, int row0, int col0, int lane, uint4 (&old)[4][2]) {
    const int S = job.S;
    const OUT *__restrict__ V = static_cast<const OUT *>(job.vis) + (size_t)c * ((size_t)S * (S + 1) / 2) * 4;
    const int i0 = row0 >> 1, j0 = col0 >> 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int bl = lane + 64 * k;
        int j = j0 + (bl >> 4);
        j = j < S ? j : S - 1;
        int i = i0 + (bl & 15);
        i = i <= j ? i : j;
        const uint4 *src = reinterpret_cast<const uint4 *>(V + ((size_t)j * (j + 1) / 2 + i) * 4);
        old[k][0] = src[0];
        old[k][1] = src[1];
    }
}

// Coalesced store of one 32 x 32 tile through this wave's LDS region; with
// ACCUM the tile is added to the old values `old` (from tile_old).
template <bool ACCUM, typename ACC, typename OUT>
__device__ __forceinline__ void store_tile_img(const Job &job, int c, const ACC &re, const ACC &im, int row0,
                                               int col0, int lane, uint8_t *img, const uint4 (&old)[4][2]) {
    const int S = job.S;
    // 1. image: element (lane, r) is row 8 (r/4) + 4 (lane/32) + r%4, column lane % 32
    {
        const int col = lane & 31;
        const int jl = col >> 1, q = col & 1;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const OUT v = Out<OUT>::make(re[r], im[r]);
            *reinterpret_cast<OUT *>(img + img_offset(jl, row >> 1) + (row & 1) * 16 + q * 8) = v;
        }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the image is written before any lane reads it
    __builtin_amdgcn_wave_barrier();
    // 2. whole baselines: lane handles baselines lane, lane + 64, ... of the tile
    OUT *__restrict__ V = static_cast<OUT *>(job.vis) + (size_t)c * ((size_t)S * (S + 1) / 2) * 4;
    const int i0 = row0 >> 1, j0 = col0 >> 1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int bl = lane + 64 * k;
        const int jl = bl >> 4, il = bl & 15;
        const int i = i0 + il, j = j0 + jl;
        uint4 lo = *reinterpret_cast<const uint4 *>(img + img_offset(jl, il));        // XX, XY
        uint4 hi = *reinterpret_cast<const uint4 *>(img + img_offset(jl, il) + 16);   // YX, YY
        if (j >= S || i > j) continue;
        if (i == j) {
            lo.y = 0u;                      // Im XX
            hi.w = 0u;                      // Im YY
            hi.x = lo.z;                    // YX = conj(XY)
            hi.y = Vec<OUT>::neg(lo.w);
        }
        uint4 *dst = reinterpret_cast<uint4 *>(V + ((size_t)j * (j + 1) / 2 + i) * 4);
        if constexpr (ACCUM) {
            lo = Vec<OUT>::add(lo, old[k][0]);
            hi = Vec<OUT>::add(hi, old[k][1]);
        }
        dst[0] = lo;
        dst[1] = hi;
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // reads done before the region is reused
    __builtin_amdgcn_wave_barrier();
}

// Stores of a wave's 2 x 2 tiles (row0 + 32 rs, col0 + 32 cs) where run[rs][cs].
// In accumulate mode each tile's old values are loaded before its image is
// assembled, so a wave waits for memory once per tile instead of once per
// group of baselines.
template <typename ACC, typename OUT>
__device__ __forceinline__ void store_tiles_lds(const Job &job, int c, const ACC (&re)[2][2], const ACC (&im)[2][2],
                                                const bool (&run)[2][2], int row0, int col0, int lane,
                                                uint8_t *img) {
    if (job.accumulate) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int rs = t >> 1, cs = t & 1;
            if (!run[rs][cs]) continue;
            uint4 old[4][2];
            __builtin_amdgcn_sched_barrier(0);
            tile_old<OUT>(job, c, row0 + 32 * rs, col0 + 32 * cs, lane, old);
            __builtin_amdgcn_sched_barrier(0);
            store_tile_img<true, ACC, OUT>(job, c, re[rs][cs], im[rs][cs], row0 + 32 * rs, col0 + 32 * cs, lane, img,
                                           old);
        }
    } else {
        const uint4 none[4][2] = {};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int rs = t >> 1, cs = t & 1;
            if (run[rs][cs])
                store_tile_img<false, ACC, OUT>(job, c, re[rs][cs], im[rs][cs], row0 + 32 * rs, col0 + 32 * cs, lane,
                                                img, none);
        }
    }
}

}  // namespace mfma
}  // namespace xc
