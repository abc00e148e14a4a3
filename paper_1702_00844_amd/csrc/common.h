// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xengine.h"

namespace xc {

// Number of XCDs on MI355X.  Workgroups are dispatched to XCDs round-robin by
// workgroup id, so kernels remap ids so that each XCD walks a contiguous range
// of work units (all block pairs of one channel share that XCD's L2).
constexpr int kNumXcd = 8;

// One sub-array to correlate, as the device sees it.
struct Job {
    const void *x;     // samples x[C][T][S][2], or time-blocked (see tblk)
    void *vis;         // visibilities V[C][B][2][2]
    int32_t S, C, T;
    int32_t nb;        // station blocks per side: ceil(S / block)
    int32_t npairs;    // nb (nb + 1) / 2
    int32_t accumulate;
    // Time-blocked input (a run of ring slots of a stream): time t lives in
    // block t / tblk, each block being x[C][tblk][S][2], bstride
    // station-samples apart; block b is slot slot0 + b of a ring of nring
    // slots, wrapping to slot 0 past the last.  Unblocked input has tblk = T
    // and bstride = 0.
    int32_t tblk;
    int64_t bstride;
    int32_t slot0;
    int32_t nring;
    // Unblocked input: station-samples from one channel to the next (T S for
    // a whole block; larger when the job views a sub-range of time).
    int64_t cstride;
    // Integration split over workgroups: unit w of the launch is piece
    // w % tsplit of unit w / tsplit; piece k integrates time steps
    // k tpiece .. k tpiece + tpiece - 1 into its own partial sums, xpiece
    // bytes further into the samples and vpiece bytes further into vis.
    int32_t tsplit;
    int32_t tpiece;
    int64_t xpiece;
    int64_t vpiece;
    // Station-major input (x[C][S][T][2]: each station's time series
    // contiguous): station-samples from one station's series to the next;
    // 0 for the time-major layout.  Read by the 16 x 16 complex-float32
    // matrix-core kernel and the int8 / 16-bit direct-to-LDS kernel (their
    // copies into LDS do the corner turn) and the vector-ALU kernel (its
    // loads into registers do).
    int64_t sstride;
};

// Index (in station-samples, i.e. units of one station's dual-pol sample) of
// the first station of time step t of channel c.
__host__ __device__ inline size_t row_offset(const Job &job, int c, int t) {
    if (job.bstride == 0) return (size_t)c * job.cstride + (size_t)t * job.S;
    const int blk = t / job.tblk;
    int slot = job.slot0 + blk;
    if (slot >= job.nring) slot -= job.nring;
    return (size_t)slot * job.bstride + ((size_t)c * job.tblk + (t - blk * job.tblk)) * job.S;
}

// True when time steps t0 .. t0 + n - 1 of a channel are consecutive rows in
// memory (S station-samples apart): always for unblocked input, and for
// time-blocked input when the steps lie in one block.
__host__ __device__ inline bool rows_contiguous(const Job &job, int t0, int n) {
    return job.bstride == 0 || t0 / job.tblk == (t0 + n - 1) / job.tblk;
}

// A work unit of a batch: item, channel, block pair.
struct Unit {
    int32_t item, channel, bi, bj;
};

// A batch launch runs one workgroup per unit of a flat unit list that is cut
// into one contiguous range per XCD (bounds[x] .. bounds[x+1], balanced by
// work): workgroup g runs on XCD g % kNumXcd (workgroups are dispatched to
// XCDs round-robin) and takes unit bounds[x] + g / kNumXcd of that range, or
// none if the range is shorter.  Returns the unit index or -1.
__device__ inline int batch_unit(const int *__restrict__ bounds, int phys) {
    const int x = phys % kNumXcd;
    const int u = bounds[x] + phys / kNumXcd;
    return u < bounds[x + 1] ? u : -1;
}

// Pair index k (column-major over the upper triangle of the block grid,
// k = bj (bj + 1) / 2 + bi with bi <= bj) -> (bi, bj).
__host__ __device__ inline void pair_decode(int k, int &bi, int &bj) {
    int j = (int)((__builtin_sqrtf(8.0f * (float)k + 1.0f) - 1.0f) * 0.5f);
    // fix rounding at either side
    while ((j + 1) * (j + 2) / 2 <= k) ++j;
    while (j * (j + 1) / 2 > k) --j;
    bj = j;
    bi = k - j * (j + 1) / 2;
}

// XCD-aware remap of a physical workgroup id to a logical work index.
// The grid has kNumXcd * per workgroups; returns -1 for the padding ids.
__device__ inline int xcd_remap(int phys, int nwork) {
    const int per = (nwork + kNumXcd - 1) / kNumXcd;
    const int logical = (phys % kNumXcd) * per + phys / kNumXcd;
    return logical < nwork ? logical : -1;
}

// Work unit w of a flat launch -> channel and block pair; when the
// integration is split over workgroups, the job is narrowed to the unit's
// piece of time (its samples, its length and its partial sums).
__device__ inline void unit_decode(Job &job, int w, int &c, int &bi, int &bj) {
    if (job.tsplit > 1) {
        const int piece = w % job.tsplit;
        w /= job.tsplit;
        job.x = static_cast<const uint8_t *>(job.x) + piece * job.xpiece;
        job.vis = static_cast<uint8_t *>(job.vis) + piece * job.vpiece;
        const int rest = job.T - piece * job.tpiece;
        job.T = rest < job.tpiece ? rest : job.tpiece;
    }
    c = w / job.npairs;
    pair_decode(w - c * job.npairs, bi, bj);
}

// Work units of a flat launch of a job.
inline int job_units(const Job &job) { return job.C * job.npairs * job.tsplit; }

inline int xcd_grid(int nwork) {
    const int per = (nwork + kNumXcd - 1) / kNumXcd;
    return per * kNumXcd;
}

// Resolved configuration of one launch.
struct Plan {
    int kernel;      // XC_KERNEL_VALU or XC_KERNEL_MFMA
    int block;       // stations per block (vector ALU: 32, or 16 for the one-channel small-array kernel)
    int time_chunk;  // time steps per LDS stage
    int time_split;  // waves sharing one output block over time
    int staging;     // XC_STAGING_REGISTERS or XC_STAGING_LDS
    int product;     // XC_PRODUCT_FOUR or XC_PRODUCT_THREE
    int tile_w;      // vector-ALU register tile: stations of block I per lane (0 elsewhere)
    int tile_h;      // vector-ALU register tile: stations of block J per lane (0 elsewhere)
};
// Product form that AUTO picks for complex-float32 on 64-station matrix-core blocks.
constexpr int kDefaultProductF32 = XC_PRODUCT_THREE;

// True when the vector-ALU kernel is built for this register tile, time
// chunk and number of time groups.
bool valu_available(int tile_w, int tile_h, int time_chunk, int time_split);

// Launchers (return hipSuccess or the launch error).
hipError_t launch_valu(const Plan &plan, const Job &job, hipStream_t stream);
// Arrays of at most 16 stations (complex float32): one workgroup per channel.
hipError_t launch_small(const Job &job, hipStream_t stream);
hipError_t launch_small_batch(const Job *jobs, const Unit *units, const int *bounds, int grid, hipStream_t stream);
hipError_t launch_mfma(const Plan &plan, xc_in_type in_type, xc_out_type out_type,
                       const Job &job, hipStream_t stream);

// int8 and 16-bit samples on 64-station blocks staged straight from HBM to
// LDS (16-byte granules when n_stations is a multiple of 4 for int8 or of 2
// for 16-bit samples, 4-byte granules otherwise).
hipError_t launch_mfma_dma(xc_in_type in_type, xc_out_type out_type, const Job &job, hipStream_t stream);
// The same from station-major samples x[C][S][T][2] (job.sstride = T): 4-byte
// copies gather each station's word from its own series (same LDS image).
hipError_t launch_mfma_dma_station_major(xc_in_type in_type, xc_out_type out_type, const Job &job,
                                         hipStream_t stream);
// g4: the items' station counts are not multiples of dma_granule (4-byte copies).
hipError_t launch_mfma_dma_batch(xc_in_type in_type, xc_out_type out_type, const Job *jobs, const Unit *units,
                                 const int *bounds, int grid, bool g4, hipStream_t stream);
// Stations per 16-byte granule of the direct-to-LDS int8/16-bit kernel; other
// station counts are copied in 4-byte granules.
inline int dma_granule(xc_in_type in_type) { return in_type == XC_IN_CI8 ? 4 : 2; }
// True when the plan runs the direct-to-LDS int8/16-bit kernel.
inline bool plan_is_dma(const Plan &p, xc_in_type in_type) {
    return p.kernel == XC_KERNEL_MFMA && p.block == 64 && in_type != XC_IN_CF32 && p.staging == XC_STAGING_LDS;
}

// FP32 samples on 16x16x4 matrix-core tiles (64-station blocks).
hipError_t launch_mfma16(const Plan &plan, const Job &job, hipStream_t stream);
hipError_t launch_mfma16_batch(const Plan &plan, const Job *jobs, const Unit *units, const int *bounds, int grid,
                               hipStream_t stream);

// Batch launchers: one workgroup per unit (see batch_unit).
hipError_t launch_valu_batch(const Plan &plan, const Job *jobs, const Unit *units, const int *bounds, int grid,
                             hipStream_t stream);
hipError_t launch_mfma_batch(const Plan &plan, xc_in_type in_type, xc_out_type out_type, const Job *jobs,
                             const Unit *units, const int *bounds, int grid, hipStream_t stream);

// Process-wide tuning cache: shape bucket -> configuration chosen by
// xc_autotune.  A bucket groups shapes that the same configuration serves:
// the number of 32-station blocks, whether the station count fills whole copy
// granules of the direct-to-LDS kernel, the integration length class
// ceil(log2 T) and the work-unit class ceil(log2(C x 64-station block pairs))
// (how well the shape fills the device), capped at 2^12 units.
struct TuneKey {
    int in, out, sb, gran, tb, ub;
    bool operator==(const TuneKey &o) const {
        return in == o.in && out == o.out && sb == o.sb && gran == o.gran && tb == o.tb && ub == o.ub;
    }
};
TuneKey tune_bucket(int in_type, int out_type, int S, int C, int T);
void tune_put(const TuneKey &k, const xc_config &cfg);
bool tune_get(const TuneKey &k, xc_config *cfg);

// Device capacity helpers.
int device_cu_count();

// Status plumbing.
xc_status set_error(xc_status st, const char *fmt, ...);
xc_status hip_error(hipError_t err, const char *what);

// Validation and plan resolution shared by the entry points.
xc_status resolve(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type, int32_t S,
                  int32_t P, int32_t C, int32_t T, Plan *plan);

}  // namespace xc
