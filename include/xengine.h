/*
 * xengine.h -- C ABI of the MI355X (gfx950) correlator X-engine.
 *
 * The library computes, for every frequency channel c, the visibilities
 *
 *   V[c][b(i,j)][p][q] = sum_{t=0}^{T-1} x[c][t][i][p] * conj(x[c][t][j][q])
 *
 * for all station pairs 0 <= i <= j < S (autocorrelations included) and all
 * four polarisation pairs p, q in {X=0, Y=1}: the correlation equation and
 * pseudo-code (Figure 2) of Section 2 of van Nieuwpoort & Romein, "Correlating
 * Radio Astronomy Signals with Many-Core Hardware".  Each station pair is
 * computed once (V(j,i) = conj V(i,j), Section 2); the conjugated factor is
 * the higher-numbered station j.
 *
 * Layouts (row-major, innermost last):
 *   samples  x[C][T][S][P] complex, time-major (all stations of one time step
 *            together, the layout of Section 4.4).  A complex sample is
 *              XC_IN_CF32 : {float re, im}            8 bytes
 *              XC_IN_CF16 : {_Float16 re, im}         4 bytes
 *              XC_IN_CBF16: {bfloat16 re, im}         4 bytes
 *              XC_IN_CI8  : {int8 re, im}             2 bytes, values in [-127, 127]
 *   vis      V[C][B][P][P] complex, B = S(S+1)/2, b(i,j) = j(j+1)/2 + i
 *            (Figure 2 writes correlation[b][c][p][q]; this is the same data
 *            with the first two axes swapped, so that a channel is contiguous).
 *              XC_OUT_CF32: {float re, im}   (any input type)
 *              XC_OUT_CI32: {int32 re, im}   (XC_IN_CI8 only; exact)
 *
 * Conventions for every call:
 *   - Data pointers are DEVICE pointers owned by the caller; the library never
 *     frees them.  Pointers must be 16-byte aligned.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     enqueue work and return before it completes.
 *   - Argument errors are reported before anything is enqueued; HIP errors
 *     return XC_ERR_HIP.  xc_last_error() gives a thread-local message for the
 *     last failing call.  The library never aborts, and prints nothing
 *     unless XC_LOG is set (below).
 *   - Only n_pol == 2 is supported (dual-polarised stations, Section 2).
 *
 * Environment variables, read by the library:
 *   XC_CHECK=1       scan XC_IN_CI8 input for -128 before correlating
 *                    (xc_correlate and the calls built on it; see below).
 *   XC_TUNE_CACHE    tuning-cache path used by xc_batch_plan_create when it
 *                    gets neither a configuration nor a cache path.
 *   XC_LOG           log of events that happen once per plan, stream or tuning
 *                    run (tuned configurations, cache loads, batch plans,
 *                    stream admission, opening and closing), one line each:
 *                    unset or "0" none, "1" or "stderr" standard error, any
 *                    other value a file appended to.  Read once per process.
 */
#ifndef XENGINE_H
#define XENGINE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum xc_status {
    XC_OK = 0,
    XC_ERR_INVALID_ARG = 1,    /* bad pointer, size, enum or configuration        */
    XC_ERR_UNSUPPORTED = 2,    /* valid but not implemented (e.g. n_pol != 2)     */
    XC_ERR_OUT_OF_MEMORY = 3,  /* a library-owned allocation failed               */
    XC_ERR_OVERFLOW_RISK = 4,  /* int32 output could overflow for this n_times    */
    XC_ERR_ADMISSION = 5,      /* stream does not fit the server's memory budget  */
    XC_ERR_BACKPRESSURE = 6,   /* stream ring full: block not accepted            */
    XC_ERR_HIP = 7,            /* a HIP runtime call failed                       */
    XC_ERR_STATE = 8           /* call not valid in the object's current state    */
} xc_status;

typedef enum xc_in_type {
    XC_IN_CF32 = 0,
    XC_IN_CI8 = 1,
    XC_IN_CF16 = 2,
    XC_IN_CBF16 = 3
} xc_in_type;

typedef enum xc_out_type {
    XC_OUT_CF32 = 0,
    XC_OUT_CI32 = 1
} xc_out_type;

/* Kernel families.  AUTO lets the library choose (tuned choice if a tuning
 * cache entry exists, else a built-in default). */
typedef enum xc_kernel {
    XC_KERNEL_AUTO = 0,
    XC_KERNEL_VALU = 1,   /* FP32 vector FMA, register-tiled (XC_IN_CF32 only)      */
    XC_KERNEL_MFMA = 2    /* matrix cores: f32, f16, bf16 or i8 by input type        */
} xc_kernel;

/* How samples travel from HBM to LDS (matrix-core kernels). */
typedef enum xc_staging {
    XC_STAGING_AUTO = 0,
    XC_STAGING_REGISTERS = 1, /* loaded into registers, corner-turned and stored to LDS */
    XC_STAGING_LDS = 2        /* copied straight into LDS (global_load_lds): 16-byte
                                 granules when n_stations % 4 == 0 for int8 or
                                 % 2 == 0 for 16-bit samples, 4-byte granules
                                 (four times as many copies) otherwise                */
} xc_staging;

/* How a complex multiply-accumulate is formed from real products.  With the
 * conjugate on station j (Section 2), Re V = sum ar br + ai bi and
 * Im V = sum ai br - ar bi: four real products.  The three-product (Gauss)
 * form accumulates P1 = sum ar br, P2 = sum ai bi and
 * P3 = sum (ar + ai)(br - bi) and returns Re V = P1 + P2,
 * Im V = P3 - P1 + P2: a quarter fewer matrix-core instructions, at a
 * rounding error bounded by the magnitudes of P1, P2 and P3 rather than of
 * V (still within single-precision accumulation error in practice; the
 * tests hold it to the same tolerance).  Throughput is still counted at 8
 * flops per complex multiply-accumulate. */
typedef enum xc_product {
    XC_PRODUCT_AUTO = 0,
    XC_PRODUCT_FOUR = 1,   /* four real products (every kernel)                       */
    XC_PRODUCT_THREE = 2   /* three real products: complex-float32 on 64-station
                              matrix-core blocks only                                  */
} xc_product;

/* Largest integration for which XC_OUT_CI32 is exact for every input:
 * |re|,|im| <= 2 * 127^2 * T <= 2^31 - 1  <=>  T <= 66572. */
#define XC_CI32_MAX_TIMES 66572

/* ------------------------------------------------------------------------ */
/* Index helpers (host only, no device access).                              */

/* S(S+1)/2: station pairs including autocorrelations (Section 2). -1 if S < 0. */
int64_t xc_n_baselines(int32_t n_stations);

/* b(i,j) = j(j+1)/2 + i, the dense baseline number of Figure 2's
 * computeBaseline.  -1 unless 0 <= i <= j. */
int64_t xc_baseline_index(int32_t i, int32_t j);

/* Complex elements of one visibility array: C * B * P * P.  -1 on bad args. */
int64_t xc_vis_elems(int32_t n_stations, int32_t n_pol, int32_t n_channels);

/* Bytes of a sample block / visibility array of the given type.  -1 on bad args. */
int64_t xc_sample_bytes(xc_in_type in_type, int32_t n_stations, int32_t n_pol,
                        int32_t n_channels, int32_t n_times);
int64_t xc_vis_bytes(xc_out_type out_type, int32_t n_stations, int32_t n_pol,
                     int32_t n_channels);

/* ------------------------------------------------------------------------ */
/* Correlation (Section 2, correlation equation; Figure 2).                  */

/*
 * vis  = correlation of samples          (accumulate == 0), or
 * vis += correlation of samples          (accumulate == 1; long integrations
 *                                         split into sub-intervals, Section 4.5)
 *
 * samples: device, x[C][T][S][P] of in_type.  vis: device, V[C][B][P][P] of
 * out_type, fully overwritten when accumulate == 0.  Errors:
 *   XC_ERR_INVALID_ARG  null/unaligned pointer, S, C or T < 1, bad enum,
 *                       XC_OUT_CI32 with a non-int8 input;
 *   XC_ERR_UNSUPPORTED  n_pol != 2;
 *   XC_ERR_OVERFLOW_RISK XC_OUT_CI32 and n_times > XC_CI32_MAX_TIMES;
 *   XC_ERR_HIP          launch failure.
 * If the environment variable XC_CHECK=1 is set, XC_IN_CI8 input is scanned
 * for the value -128 first and rejected with XC_ERR_INVALID_ARG; that debug
 * scan synchronises the stream and allocates (and frees) a 4-byte device
 * flag.  Otherwise the call allocates nothing and returns without waiting.
 */
xc_status xc_correlate(const void *samples, xc_in_type in_type, int32_t n_stations,
                       int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis,
                       xc_out_type out_type, int32_t accumulate, void *stream);

/*
 * The same correlation with the integration split over workgroups, for
 * workloads with few (channel, block pair) units, such as few channels and
 * stations (Section 4.5 splits long integrations the same way): the T time
 * steps are cut into pieces of ceil(T / n_split) steps (K pieces, K <= n_split,
 * none empty), each piece's partial sums are written to `work` (device,
 * caller-owned, at least xc_correlate_split_bytes bytes, 16-byte aligned),
 * then vis (+)= the sum over pieces 0 .. K-1 in that order: the reduction
 * order is fixed, so results are reproducible for a given n_split (int32:
 * exact; float: may differ from the unsplit kernel by rounding).  Allocates
 * nothing.  n_split = 1 (or T = 1) is xc_correlate_config.  Errors as
 * xc_correlate_config, and XC_ERR_INVALID_ARG for n_split < 1, a null or
 * misaligned work pointer or too small a work_bytes.
 */
int64_t xc_correlate_split_bytes(int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_times,
                                 int32_t n_split);

/*
 * Kernel configuration.  Zero fields mean "default for this shape".
 *   kernel        xc_kernel.  AUTO: for complex float32 on at most 16 stations
 *                 (and no other field set) VALU with block 16, otherwise MFMA.
 *   block         stations per block of the triangle's block grid (Section 4.5
 *                 splits large triangles into blocks).  VALU: 32 (default), or
 *                 16 for arrays of at most 16 stations: one workgroup per
 *                 channel correlates all its baselines (the chunk of 128 time
 *                 steps and up to 32 time groups are fixed; time_chunk 0 or
 *                 128, time_split 0 or 1, no register tiles).  MFMA: 32 or 64
 *                 (AUTO: 32 for complex-float32 on at most 48 stations, else 64).
 *   time_chunk    time steps staged in LDS per pipeline stage (fixed by the
 *                 other fields except for VALU: 16 or 32, default 32;
 *                 reported for off-diagonal block pairs: diagonal pairs stage
 *                 one block, with up to twice as many steps).
 *   time_split    waves of a workgroup that share one output block, each
 *                 integrating a different part of every time chunk; their
 *                 partial sums are added in LDS before the single store.
 *                 VALU: 1, 2, 4 (default) or 8, for off-diagonal block pairs
 *                 (a diagonal pair packs its threads over its tiles with
 *                 outputs, in as many time groups as fit).  MFMA: 1, or 2 for
 *                 complex-float32 on 64-station blocks.
 *   staging       xc_staging.  Complex-float32 on 64-station blocks always
 *                 copies straight into LDS; VALU and 32-station blocks always
 *                 stage through registers; int8 and 16-bit samples on
 *                 64-station blocks take either (AUTO: LDS).
 *   product       xc_product.  AUTO: three products for complex-float32 on
 *                 64-station matrix-core blocks, four everywhere else.
 *   tile_w,       VALU only: the register tile of one lane, tile_w stations of
 *   tile_h        block I by tile_h stations of block J (Table 1): 4 x 2
 *                 (default), 4 x 4, 8 x 2 or 2 x 2.  VALU time_split 8 needs
 *                 time_chunk 32 and at most 128 lanes per time group (not
 *                 2 x 2).
 *                 Matrix-core kernels: 0.
 */
typedef struct xc_config {
    int32_t kernel;
    int32_t block;
    int32_t time_chunk;
    int32_t time_split;
    int32_t staging;
    int32_t product;
    int32_t tile_w;
    int32_t tile_h;
} xc_config;

/* Checks a configuration against a shape without touching the device.
 * On success, writes the resolved configuration (defaults filled in) to
 * *resolved if it is not NULL.  Same errors as xc_correlate. */
xc_status xc_resolve_config(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type,
                            int32_t n_stations, int32_t n_pol, int32_t n_channels,
                            int32_t n_times, xc_config *resolved);

/* xc_correlate with an explicit configuration (cfg may be NULL = AUTO). */
xc_status xc_correlate_config(const xc_config *cfg, const void *samples, xc_in_type in_type,
                              int32_t n_stations, int32_t n_pol, int32_t n_channels,
                              int32_t n_times, void *vis, xc_out_type out_type,
                              int32_t accumulate, void *stream);

/* See xc_correlate_split_bytes above. */
xc_status xc_correlate_split(const xc_config *cfg, const void *samples, xc_in_type in_type, int32_t n_stations,
                             int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis, xc_out_type out_type,
                             int32_t accumulate, int32_t n_split, void *work, int64_t work_bytes, void *stream);

/*
 * xc_correlate_split without a workspace argument and without any allocation,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the pieces'
 * partial sums go to a fixed scratch array of XC_SPLIT_STATIC_SCRATCH_BYTES
 * in device memory, one per device, that the library holds until the process
 * ends (its device address is looked up on the first call on each device).
 * The call makes no hipMalloc, hipFree or other allocating call, and it does
 * not run the XC_CHECK scan (which allocates).  Every call on a device shares
 * that device's scratch: calls that overlap on one device (different streams,
 * or threads) race and may return wrong sums; serialise them.  The scratch
 * keeps the last call's partial sums, which the next call overwrites
 * completely (nothing needs clearing).  Errors as xc_correlate_split, and
 * XC_ERR_UNSUPPORTED when K x C x B x 4 complex values (8 bytes each) exceed
 * the scratch.  n_split = 1 (or T = 1) runs the unsplit kernel, with no
 * scratch.
 */
#define XC_SPLIT_STATIC_SCRATCH_BYTES (64ll << 20)
xc_status xc_correlate_split_static(const xc_config *cfg, const void *samples, xc_in_type in_type,
                                    int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis,
                                    xc_out_type out_type, int32_t accumulate, int32_t n_split, void *stream);

/*
 * The same correlation from station-major samples, samples[C][S][T][P]
 * (device; each station's time series contiguous, the layout a station's
 * receiver produces; Section 4.4 discusses both layouts).  The corner turn to
 * time-major order happens in the copies into LDS (or the vector-ALU
 * kernel's loads), so there is no transposed copy in device memory: the
 * kernel's LDS image, and hence the result bit for bit, are those of
 * xc_correlate_config on the time-major block.  Kernels: complex float32 on
 * the 64-station matrix-core kernel (kernel AUTO or XC_KERNEL_MFMA, block 0
 * or 64; cfg may set its time split and product form) or on the vector-ALU
 * kernels (XC_KERNEL_VALU; AUTO on at most 16 stations takes the one-channel
 * kernel, block 16, as xc_correlate does); int8 and 16-bit samples on the 64-station
 * direct-to-LDS matrix-core kernel, in 4-byte copies (one station's word per
 * lane, gathered from 64 station series per copy).  Errors as for
 * xc_correlate_config, and XC_ERR_UNSUPPORTED for the 32-station or
 * register-staged matrix-core kernels.  Allocates nothing.
 */
xc_status xc_correlate_station_major(const xc_config *cfg, const void *samples, xc_in_type in_type,
                                     int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_times,
                                     void *vis, xc_out_type out_type, int32_t accumulate, void *stream);

/* ------------------------------------------------------------------------ */
/* Cost model (Section 2, Table 1; Section 3.6 bound-and-bottleneck).        */

/* For a w x h tile of station pairs: flops = 32wh, bytes = 16(w+h) (complex
 * float dual-pol samples), minimum registers = 4(1 + min(w,h)) + 8wh floats.
 * XC_ERR_INVALID_ARG if w or h < 1 or an output pointer is NULL. */
xc_status xc_tile_cost(int32_t w, int32_t h, int64_t *flops, int64_t *bytes,
                       int64_t *min_registers);

/* perf_max = min(perf_peak, AI * bandwidth) (Section 3.6). */
double xc_perf_max(double perf_peak, double arithmetic_intensity, double bandwidth);

/* Global arithmetic intensity of correlating S dual-pol complex-float
 * stations: 32 flops per baseline over 16 bytes per station = S + 1. */
double xc_ai_global(int32_t n_stations);

/* Algorithmic flops of one correlation: 8 per complex multiply-accumulate,
 * 32 per baseline per time step = 32 * C * T * S(S+1)/2. */
double xc_flops(int32_t n_stations, int32_t n_channels, int32_t n_times);

/* ------------------------------------------------------------------------ */
/* Batches of sub-arrays in one launch per kernel configuration.            */
/* Channels (and sub-arrays) are independent (Section 2), so uneven         */
/* workloads combine into one list of work units.                           */

typedef struct xc_subarray {
    const void *samples;   /* device, x[C][T][S][2] of the batch's in_type  */
    void *vis;             /* device, V[C][B][2][2] of the batch's out_type */
    int32_t n_stations;
    int32_t n_channels;
    int32_t n_times;
} xc_subarray;

typedef struct xc_batch_plan xc_batch_plan;

/*
 * Builds a plan for correlating every item of `items` (many sub-arrays and
 * subbands of uneven size; channels are independent, Section 2, so the
 * batch is one flat list of work units).  Items whose resolved
 * configurations are equal share one launch.  Configuration: `cfg` for every
 * item if not NULL; else, with `tune_cache` (a JSON-lines file path, as
 * xc_autotune writes), each item takes the configuration tuned for its shape
 * bucket (the tile size must be tuned per platform and shape, Section 2):
 * the file is loaded first, and every bucket still missing is tuned here on
 * the first item that falls in it (xc_autotune: timing that overwrites that
 * item's vis and synchronises `stream`) and appended to the file -- unless
 * accumulate == 1, in which case missing buckets take the default; with
 * neither, every item runs the default with one time group per workgroup.
 * A launch runs one workgroup per (item, channel, block pair) unit of a
 * device work list cut into one range per XCD: whole channels are dealt to
 * the XCD with the least work so far (items by decreasing integration
 * length), so a channel's block pairs share an L2 and the longest units
 * start first.  If use_graph != 0 the launches are captured into a hipGraph
 * and replayed by xc_batch_plan_run.  The plan owns its device work lists;
 * xc_batch_plan_destroy frees them.  tune_cache NULL (and cfg NULL) takes
 * the path in XC_TUNE_CACHE, if set.  Pointers in `items` are baked into the
 * plan: they must stay valid while the plan is used.
 * Errors: as xc_correlate for each item; XC_ERR_OUT_OF_MEMORY.
 */
xc_status xc_batch_plan_create(const xc_subarray *items, int32_t n_items, int32_t n_pol,
                               xc_in_type in_type, xc_out_type out_type, int32_t accumulate,
                               const xc_config *cfg, const char *tune_cache, int32_t use_graph, void *stream,
                               xc_batch_plan **out);
xc_status xc_batch_plan_run(xc_batch_plan *plan, void *stream);
void xc_batch_plan_destroy(xc_batch_plan *plan);
/* Number of work units (item, channel, block pair) in the plan. */
int64_t xc_batch_plan_units(const xc_batch_plan *plan);

/*
 * Host-only work-list construction, exposed for tests: fills units[k] =
 * {item, channel, block_i, block_j} (4 int32 each) for every work unit of a
 * launch over all the items on blocks of `block` stations, in the plan's
 * order, and, if bounds is not NULL, bounds[0..8] = the start of each XCD's
 * range and the end of the last.  Returns the unit count (or -1 on bad args);
 * writes at most `capacity` units.
 */
int64_t xc_batch_worklist(const int32_t *n_stations, const int32_t *n_channels,
                          const int32_t *n_times, int32_t n_items, int32_t block,
                          int32_t *units, int64_t capacity, int32_t *bounds);

/* ------------------------------------------------------------------------ */
/* Auto-tuning (the tile size must be tuned per platform, Section 2; Table 1 */
/* gives each register tile's flops, bytes and minimum registers).          */

/*
 * Times every candidate configuration for the shape on `stream`
 * (synchronising), using the caller's samples/vis buffers (vis is
 * overwritten), and writes the fastest to *best and its kernel time to
 * *best_ms.  The candidates (xc_tune_candidates) are the matrix-core block
 * sizes, stagings, time groups and product forms, and the vector-ALU register
 * tiles w x h with w, h in {2, 4, 8} (a tile and its mirror image cost the
 * same; one is built) whose Table 1 register count plus the kernel's staging
 * and address registers fits 256, each with every time chunk and time-group
 * count.  The winner is kept for the shape's bucket (xc_tune_bucket), which
 * xc_correlate (AUTO) and batch plans then use for every shape of that
 * bucket in this process; if cache_path is not NULL it is also appended to
 * that JSON-lines file.
 */
xc_status xc_autotune(const void *samples, xc_in_type in_type, int32_t n_stations,
                      int32_t n_pol, int32_t n_channels, int32_t n_times, void *vis,
                      xc_out_type out_type, const char *cache_path, void *stream,
                      xc_config *best, double *best_ms);

/* The candidate configurations of xc_autotune for a sample type, after the
 * Table 1 pruning (host only).  Writes at most `capacity` of them to out (if
 * not NULL); returns their number, or -1 for a bad type. */
int64_t xc_tune_candidates(xc_in_type in_type, xc_config *out, int64_t capacity);

/* The tuning bucket of a shape (host only): key = {in_type, out_type,
 * ceil(S / 32) (0 for at most 16 stations, the one-channel kernel's
 * range), 1 if S fills whole copy granules of the direct-to-LDS kernel
 * (4 int8 or 2 16-bit stations), ceil(log2 T), min(ceil(log2(C x
 * 64-station block pairs)), 12)}.  Shapes with equal keys share a tuned
 * configuration. */
xc_status xc_tune_bucket(xc_in_type in_type, xc_out_type out_type, int32_t n_stations, int32_t n_channels,
                         int32_t n_times, int32_t key[6]);

/* Loads a tuning cache written by xc_autotune into the process's bucket
 * table (entries already there for other buckets are kept; an entry that no
 * longer resolves is skipped).  Returns the number of entries loaded, or -1
 * if the file is unreadable. */
int64_t xc_tune_cache_load(const char *cache_path);

/* ------------------------------------------------------------------------ */
/* Streaming: blocks arrive, partial integrations stay resident on device.   */
/* The correlator is a real-time application whose input arrives as a       */
/* stream (Section 1); an integration spans about one second of samples      */
/* (Section 2) and is built from sub-intervals whose partial results are      */
/* accumulated in memory (Section 4.5); copies and computation overlap        */
/* (Section 4.4).                                                            */

typedef struct xc_stream_desc {
    int32_t n_stations;
    int32_t n_pol;                  /* must be 2 */
    int32_t n_channels;
    int32_t block_times;            /* samples per arriving block                  */
    int32_t blocks_per_integration; /* blocks folded into one published integration
                                       (a multiple of blocks_per_fold)             */
    int32_t blocks_per_fold;        /* k: every channel is folded every k blocks    */
    int32_t ring_blocks;            /* device ring slots (>= 2 * blocks_per_fold)   */
    int32_t in_type;                /* xc_in_type                                    */
    int32_t acc_type;               /* xc_out_type of the resident accumulator       */
    int32_t staggered;              /* 0: every k blocks, one fold of all channels;
                                       1: the channels in k groups, one group folded
                                       per committed block (its outstanding blocks),
                                       every group at the end of an integration;
                                       2: as 1, but at the end of an integration each
                                       group keeps its outstanding blocks until its
                                       next turn (at most k - 1 blocks later) and folds
                                       them then, into that integration's accumulator,
                                       so that every block period gets one group's
                                       fold; an integration is published once every
                                       group has folded past its end, or by
                                       xc_stream_flush                               */
    double block_period_s;          /* arrival period P; block deadline = k * P      */
} xc_stream_desc;

/* Latency accounting.  A block's latency runs from its arrival to the
 * completion of the last fold that integrates it; the real-time deadline is
 * per block: D = blocks_per_fold * block_period.  A fold's latency runs from
 * the arrival of the block whose commit enqueued it to its completion, against
 * the interval between fold launches (block_period when staggered, D
 * otherwise). */
typedef struct xc_latency_stats {
    double p50_ms, p99_ms, max_ms;  /* per block: arrival -> last fold completed    */
    double deadline_ms;             /* per block: blocks_per_fold * block_period     */
    double tflops;                  /* algorithmic TFLOP/s over the measured span   */
    int64_t blocks;                 /* blocks whose latency was measured            */
    int64_t misses;                 /* blocks whose latency exceeded deadline_ms    */
    int64_t pending;                /* committed blocks not yet completely folded   */
    double fold_p50_ms, fold_p99_ms, fold_max_ms;  /* per fold: trigger -> completed */
    double fold_deadline_ms;        /* interval between fold launches               */
    int64_t folds;                  /* folds whose latency was measured             */
    int64_t fold_misses;            /* folds whose latency exceeded fold_deadline_ms */
    int64_t integrations;           /* integrations published                       */
} xc_latency_stats;

typedef struct xc_server xc_server;

/* Creates a server with a device-memory budget (0 = 90% of the free memory
 * of the current device). */
xc_status xc_server_create(size_t hbm_budget_bytes, xc_server **out);
/* Waits for every stream's work and frees everything. */
void xc_server_destroy(xc_server *srv);

/* Fold order across the server's streams (Section 1: the correlator must keep
 * up with every stream it takes).  0 (the default): each stream's folds run on
 * its own HIP stream, concurrently with the other streams'.  1: every fold
 * enqueued from now on waits for the one the server enqueued before it
 * (whatever its stream), so folds run one at a time in enqueue order: streams
 * whose blocks arrive together then do not split the device for the length of
 * each fold.  A stream's hold (xc_stream_hold) or a consumer's late release
 * then delays the folds of the other streams enqueued after it as well.
 * Errors: XC_ERR_INVALID_ARG (null server, value not 0 or 1). */
xc_status xc_server_set_fold_order(xc_server *srv, int32_t one_at_a_time);

/* Device bytes one stream needs: two resident accumulators (one integrating,
 * one published) plus the ring of sample blocks.  0 on bad args. */
size_t xc_stream_footprint(const xc_stream_desc *desc);

/* Admits a stream if its footprint fits the remaining budget
 * (XC_ERR_ADMISSION otherwise), allocates its buffers, a HIP stream, events
 * and a 4-byte host-coherent flag.  Errors: XC_ERR_INVALID_ARG (sizes,
 * blocks_per_integration not a multiple of blocks_per_fold, ring_blocks <
 * 2 * blocks_per_fold), XC_ERR_OVERFLOW_RISK (XC_OUT_CI32 accumulator over
 * more than XC_CI32_MAX_TIMES samples), XC_ERR_OUT_OF_MEMORY, XC_ERR_HIP. */
xc_status xc_stream_open(xc_server *srv, const xc_stream_desc *desc, int32_t *stream_id);

/* Returns the device pointer of the next free ring slot (x[C][block_times][S][2]).
 * XC_ERR_BACKPRESSURE if that slot holds a block whose folds have not all
 * completed; XC_ERR_STATE if the previous slot was not committed. */
xc_status xc_stream_acquire(xc_server *srv, int32_t stream_id, void **block_dev_ptr);

/* Marks the acquired slot as filled (its contents must be in place: written
 * by the host or by device work that has completed); arrival_ns is the
 * block's arrival time on the host clock (CLOCK_MONOTONIC ns).  Enqueues the
 * folds this block triggers (see staggered) on the stream's HIP stream and
 * returns without waiting.  After the last block of an integration the
 * integration is published. */
xc_status xc_stream_commit(xc_server *srv, int32_t stream_id, uint64_t arrival_ns);

/* The same, for a slot filled by work enqueued on producer_stream (a
 * hipStream_t): the folds that read it wait for that work (an event recorded
 * on producer_stream now), and the host need not synchronise. */
xc_status xc_stream_commit_after(xc_server *srv, int32_t stream_id, uint64_t arrival_ns, void *producer_stream);

/* Integration k (0, 1, ... in arrival order) of the stream: *vis = its device
 * buffer V[C][B][2][2] of acc_type, *ready = a hipEvent_t recorded after its
 * last fold (wait on it, e.g. hipStreamWaitEvent, before reading; the event
 * and buffer are the library's).  Returns without blocking.  The buffer is
 * reused by integration k + 2 from that integration's first block on:
 * XC_ERR_STATE if integration k is not yet published or already being
 * overwritten.  Unless the consumer calls xc_stream_release, its reads must
 * be done before then. */
xc_status xc_stream_integration(xc_server *srv, int32_t stream_id, int64_t k, const void **vis, void **ready);

/* Makes work enqueued on `stream` after this call wait for `event` (a
 * hipEvent_t such as xc_stream_integration's ready event): the host does
 * not wait. */
xc_status xc_wait_event(void *event, void *stream);

/* The consumer's reads of integration k are the work enqueued on
 * consumer_stream (a hipStream_t) before this call: the first fold that
 * overwrites the buffer (integration k + 2) waits for that work.  Errors as
 * for xc_stream_integration. */
xc_status xc_stream_release(xc_server *srv, int32_t stream_id, int64_t k, void *consumer_stream);

/* Device pointer to the latest published integration and its sequence
 * number (-1 and NULL if none yet): xc_stream_integration of that number,
 * without the event. */
xc_status xc_stream_latest(xc_server *srv, int32_t stream_id, const void **vis,
                           int64_t *sequence);

/* Holds the stream's folds: work enqueued on the stream after this call
 * starts only once xc_stream_resume is called or max_wait_s (0 .. 60) has
 * passed, whichever comes first (a one-lane kernel polls a host-coherent
 * flag; the time limit bounds the hold whatever the host does).  For starting
 * streams together and for exercising back-pressure deterministically. */
xc_status xc_stream_hold(xc_server *srv, int32_t stream_id, double max_wait_s);
xc_status xc_stream_resume(xc_server *srv, int32_t stream_id);

/* Waits for all folds enqueued on the stream so far, then fills *stats.  The
 * wait does not hold the server's lock, so the server's other streams go on;
 * calls on this stream must not overlap its xc_stream_close.  Every committed
 * block leaves a latency record (its arrival time, and one completion record
 * per fold) that is kept until xc_stream_reset_stats or xc_stream_close: a
 * stream that runs for long should read and reset its statistics
 * periodically. */
xc_status xc_stream_stats(xc_server *srv, int32_t stream_id, xc_latency_stats *stats);

/* Waits for all enqueued folds of the stream, then forgets their latency
 * records (the next xc_stream_stats covers only blocks committed after this
 * call).  Integration state is unchanged. */
xc_status xc_stream_reset_stats(xc_server *srv, int32_t stream_id);

/* Staggered = 2: folds now what the channel groups have left of every
 * integration whose blocks have all been committed, and publishes them (for a
 * stream that stops, or pauses, at the end of an integration).  The blocks of
 * the integration in progress are left to their groups' turns.  No effect for
 * the other schedules, which fold everything at an integration's last block.
 * Errors: XC_ERR_INVALID_ARG (no such stream), XC_ERR_HIP. */
xc_status xc_stream_flush(xc_server *srv, int32_t stream_id);

/* Waits for the stream's work (ending any hold) and frees its buffers. */
xc_status xc_stream_close(xc_server *srv, int32_t stream_id);

/* Host-only helpers, exposed for tests. */
/* q-quantile (0..1) of n values by the nearest-rank method; NaN if n == 0. */
double xc_quantile(const double *values, int64_t n, double q);

/* The fold schedule of a stream (the real-time stream of Section 1,
 * integrated in sub-intervals whose partial sums are added, as Section 4.5
 * does), computed on the host without touching a device: the folds the server
 * enqueues when blocks 0 .. n_blocks - 1 are committed and, with flush = 1,
 * xc_stream_flush is called after them.  Row r of folds (6 int64 per row; the
 * first max_folds rows are written, caller-owned) is {trigger block (whose
 * commit enqueues the fold; n_blocks - 1 for the flush), channel group, first
 * channel, end channel (exclusive; equal to the first when the group has no
 * channels), first block, last block}, in enqueue order, and every fold lies
 * within one integration.  published_after[j] (max_integrations entries,
 * caller-owned) is the block whose commit publishes integration j, n_blocks
 * if the flush does, -1 if neither.  *n_folds is the number of folds, also
 * beyond max_folds.  Errors: the descriptor checks of xc_stream_open,
 * XC_ERR_INVALID_ARG (null output pointers, negative counts, flush not 0 or
 * 1). */
xc_status xc_stream_schedule(const xc_stream_desc *desc, int64_t n_blocks, int32_t flush, int64_t *folds,
                             int64_t max_folds, int64_t *n_folds, int64_t *published_after,
                             int64_t max_integrations);

/* ------------------------------------------------------------------------ */
/* Host ingest: samples in host memory (Section 3.6's host-to-device bound,    */
/* Section 4.4's asynchronous copies and memory-layout transpose).            */

typedef enum xc_layout {
    XC_LAYOUT_TIME_MAJOR = 0,     /* x[C][T][S][P]: all stations of a time step together */
    XC_LAYOUT_STATION_MAJOR = 1   /* x[C][S][T][P]: each station's time series together,
                                     the natural order of the preceding pipeline stages */
} xc_layout;

/*
 * Out-of-place transpose of device samples from the station-major to the
 * time-major layout, per channel (Section 4.4's memory-layout transpose):
 * dst[c][t][s][p] = src[c][s][t][p].  Both buffers device, caller-owned,
 * C * S * T * 2 complex samples of in_type, aligned to one station's
 * dual-polarised sample (4, 8 or 16 bytes), not overlapping.  Enqueued on
 * `stream`; argument errors (null or aligned-wrong pointer, src == dst, bad
 * type or sizes, n_pol != 2) are returned before anything is enqueued.
 */
xc_status xc_transpose_to_time_major(const void *src, void *dst, xc_in_type in_type, int32_t n_stations,
                                     int32_t n_pol, int32_t n_channels, int32_t n_times, void *stream);

/*
 * A plan that correlates C channels of samples held in host memory.  The
 * channels are processed in groups of `channels_per_group` (0: about 128 MiB
 * of samples per group); two device staging slots of one group each (four
 * with station-major input: the copy and its transpose) are allocated here
 * and freed by xc_ingest_destroy, together with a copy stream and events.
 * Errors: XC_ERR_INVALID_ARG (bad type, sizes, layout or group size),
 * XC_ERR_UNSUPPORTED (n_pol != 2), XC_ERR_OUT_OF_MEMORY, XC_ERR_HIP.  A plan
 * keeps the state of its staging slots: use it from one thread at a time.
 */
typedef struct xc_ingest xc_ingest;
xc_status xc_ingest_create(xc_in_type in_type, int32_t n_stations, int32_t n_pol, int32_t n_channels,
                           int32_t n_times, int32_t layout, int32_t channels_per_group, xc_ingest **out);

/* Group size in channels and device bytes held, of a plan (either output may
 * be NULL). */
xc_status xc_ingest_info(const xc_ingest *ingest, int32_t *channels_per_group, int64_t *device_bytes);

/*
 * Enqueues the correlation of host_samples (C channels in the plan's layout,
 * host memory; pinned memory, e.g. hipHostMalloc, makes the copies
 * asynchronous DMA) into vis (device, V[C][B][P][P] of out_type, as for
 * xc_correlate) on `stream`, one group after another: copy to a staging slot,
 * transpose (station-major input), correlate into the group's channels of V.
 * Station-major complex float32 on the 64-station matrix-core kernel or the
 * vector-ALU kernel skips the transpose: those kernels read the staged group
 * as it is (as xc_correlate_station_major does).
 * overlap = 1: copies run on the plan's copy stream, each group's copy
 * overlapping the previous group's correlation; overlap = 0: copies run on
 * `stream`, in order with the computation (synchronous I/O).  The results are
 * those of xc_correlate_config(cfg, ...) on the time-major block.  host_samples
 * must stay valid and unchanged until `stream` has completed the call's work;
 * calls on one plan may follow each other without waiting (slots are reused
 * only after their previous correlation).  Argument and configuration errors
 * are returned before anything is enqueued.  The copies are staged, not
 * asynchronous, if host_samples is pageable memory.
 */
xc_status xc_ingest_run(xc_ingest *ingest, const xc_config *cfg, const void *host_samples, void *vis,
                        xc_out_type out_type, int32_t accumulate, int32_t overlap, void *stream);

/* Waits for the plan's outstanding work and frees it. */
void xc_ingest_destroy(xc_ingest *ingest);

/* ------------------------------------------------------------------------ */
/* F-engine: polyphase filter bank into the correlator's input (Section 2:    */
/* station data are filtered into frequency channels before correlation).    */

/*
 * The filter bank, for N channels and M taps per channel (the paper fixes no
 * filter design; this is the reading taken):
 *     u[t][n] = sum_{m<M} h[m N + n] z[(t + m) N + n]
 *     y[t][k] = sum_{n<N} u[t][n] exp(-2 pi i k n / N)
 *     x[k][t][s][p] = w[s][p][k] y_{s,p}[t][k]     (w optional)
 * for the T = floor(n_in / N) - M + 1 frames whose window lies in the input.
 * x is the correlator's input layout ([C][T][S][P] with C = N), so it can be
 * passed to xc_correlate as it is.
 *
 * xc_pfb_create: N = 256 or 512, 1 <= M <= 16, 1 <= S <= 16384, n_pol = 2,
 * M N <= n_in < 2^31.  Allocates an intermediate of S P T N complex64 and a
 * twiddle table (freed by xc_pfb_destroy).  Errors: XC_ERR_INVALID_ARG,
 * XC_ERR_UNSUPPORTED (other N or n_pol), XC_ERR_OUT_OF_MEMORY, XC_ERR_HIP.
 */
typedef struct xc_pfb xc_pfb;
xc_status xc_pfb_create(int32_t n_stations, int32_t n_pol, int32_t n_channels, int32_t n_taps, int64_t n_in,
                        xc_pfb **out);

/* Frames T and device bytes held, of a filter bank (either output may be NULL). */
xc_status xc_pfb_info(const xc_pfb *pfb, int32_t *n_frames, int64_t *device_bytes);

/*
 * Enqueues the filter bank on `stream`.  All pointers device memory, owned by
 * the caller: z complex64 [S][P][n_in] (each station's and polarisation's
 * sample stream, 8-byte aligned), taps float32 [M N] (the prototype filter
 * h), weights complex64 [S][P][N] or NULL (all ones), x complex64 [N][T][S][P]
 * (written completely, not overlapping z).  Argument errors are returned
 * before anything is enqueued.  Calls on one filter bank share its
 * intermediate buffer: calls on different streams must not overlap.
 */
xc_status xc_pfb_run(xc_pfb *pfb, const void *z, const float *taps, const void *weights, void *x, void *stream);

/*
 * The same filter bank writing x complex64 [N][S][T][P] (channel, station,
 * frame, polarisation: each station's frames contiguous per channel), the
 * layout xc_correlate_station_major takes, in one kernel: no intermediate
 * and no corner turn (the FX correlator's corner turn, Section 7, then
 * happens in the correlator's copies into LDS).  x must be 16-byte aligned.
 * Otherwise as xc_pfb_run, and bit-identical to its output up to the
 * layout.
 */
xc_status xc_pfb_run_station_major(xc_pfb *pfb, const void *z, const float *taps, const void *weights, void *x,
                                   void *stream);

/* Frees a filter bank (its enqueued work must be complete). */
void xc_pfb_destroy(xc_pfb *pfb);

/* ------------------------------------------------------------------------ */
/* Achievable device peaks (for roofline reports).                           */

typedef enum xc_peak {
    XC_PEAK_F32_MFMA16 = 0,   /* v_mfma_f32_16x16x4_f32, TFLOP/s  */
    XC_PEAK_F32_MFMA32 = 1,   /* v_mfma_f32_32x32x2_f32, TFLOP/s  */
    XC_PEAK_I8_MFMA = 2,      /* v_mfma_i32_32x32x32_i8, TOP/s    */
    XC_PEAK_F16_MFMA = 3,     /* v_mfma_f32_32x32x16_f16, TFLOP/s */
    XC_PEAK_BF16_MFMA = 4,    /* v_mfma_f32_32x32x16_bf16, TFLOP/s */
    XC_PEAK_F32_FMA = 5,      /* v_fma_f32 (vector ALU), TFLOP/s  */
    XC_PEAK_HBM_COPY = 6      /* 1 GiB device copy, GB/s (read + write) */
} xc_peak;

/* Times register-only loops of the instruction (8 waves per SIMD, no memory
 * traffic) or a 1 GiB device copy on the current device, synchronously, and
 * writes the achieved rate.  Allocates and frees its own scratch buffers. */
xc_status xc_measure_peak(int32_t which, double *value);

/* ------------------------------------------------------------------------ */
const char *xc_status_string(xc_status status);
const char *xc_last_error(void);
/* Library version string. */
const char *xc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XENGINE_H */
