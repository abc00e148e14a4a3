// Streaming correlator server.
//
// The correlator is a streaming, real-time application (Section 1): sample
// blocks arrive at a fixed period P and must be integrated (Section 2: about
// one second of samples per integration) without falling behind.  Each
// stream owns
//   - a device ring of `ring_blocks` sample blocks x[C][block_times][S][2],
//   - two resident accumulators V[C][B][2][2]: integration n lives in
//     accumulator n % 2, so one is being integrated while the other holds the
//     last published integration,
//   - a HIP stream on which its folds run in order, and events that mark an
//     integration's completion and a consumer's release of it.
// A fold is one accumulate-mode correlation of some channels over a run of
// consecutive blocks of the ring (the integration is split into
// sub-intervals whose partial sums are added into the resident result, as
// Section 4.5 does with the Cell's local store); the first fold of a channel
// in an integration overwrites instead of adding, so nothing is cleared.
//
// Fold schedules, with k = blocks_per_fold:
//   - all channels (staggered = 0): every k committed blocks, one fold of
//     every channel over those k blocks;
//   - staggered (staggered = 1): the channels are cut into k groups, and at
//     every committed block n the group g = n mod k folds the blocks it has
//     not yet folded (k of them in the steady state).  Each channel is still
//     folded every k blocks, but the device gets 1/k of the work every block
//     period instead of all of it every k periods, so a block's last fold
//     ends within (k - 1) P + (one fold of C/k channels) of its arrival.  At
//     the end of an integration every group folds what it has left (oldest
//     pending block first), so that the integration is complete when it is
//     published;
//   - staggered, ends spread (staggered = 2): the same, except that at the
//     end of an integration each group keeps what it has left until its next
//     turn, k - 1 blocks at most, and then folds it (into the old
//     integration's accumulator) together with its first blocks of the new
//     one.  The device then gets one group's fold per block period throughout
//     instead of up to k of them at the last block; each block still meets
//     its deadline, and an integration is published once every group has
//     folded past its end (k - 2 blocks into the next one), or on
//     xc_stream_flush.
// The schedules are host logic of their own (plan_commit, plan_flush,
// plan_published): the server enqueues the folds they plan, and
// xc_stream_schedule returns the same plan without a device.
// Folds of different streams run concurrently on their own HIP streams, or,
// with xc_server_set_fold_order, one at a time in the order they are
// enqueued (each waits for the server's previous fold): streams whose blocks
// arrive together then no longer share the device through each fold, so each
// fold takes its own time instead of both taking twice as long.
// A block's latency runs from its arrival to the completion of the last fold
// that covers it; its deadline is D = k P.  A fold's latency runs from the
// arrival of the block that triggered it to its completion, against the
// interval between fold launches (P staggered, k P otherwise).  Completion
// times come from host functions enqueued after each fold.  Streams are
// admitted only if their device footprint fits the budget.
#include <time.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <mutex>
#include <vector>

#include "common.h"
#include "log.h"

namespace xc {
xc_status resolve(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type, int32_t S, int32_t P, int32_t C,
                  int32_t T, Plan *plan);
Job make_job(const void *samples, void *vis, int S, int C, int T, int block, int accumulate);
xc_status launch_plan(const Plan &plan, xc_in_type in_type, xc_out_type out_type, const Job &job,
                      hipStream_t stream);
}  // namespace xc

using namespace xc;

namespace {

uint64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

int in_elem_bytes(int t) {
    switch (t) {
    case XC_IN_CF32: return 8;
    case XC_IN_CI8: return 2;
    default: return 4;
    }
}

// Completion record of one fold, written by a host function on the stream.
struct FoldDone {
    uint64_t done_ns = 0;
    volatile int done = 0;
};

void on_fold_done(void *arg) {
    FoldDone *f = static_cast<FoldDone *>(arg);
    f->done_ns = now_ns();
    __atomic_store_n(&f->done, 1, __ATOMIC_RELEASE);
}

bool is_done(const FoldDone *f) { return f && __atomic_load_n(&f->done, __ATOMIC_ACQUIRE); }

// Holds a stream until a host flag is set or a time limit has passed (the
// limit bounds the wait whatever the host does).  One lane polls the flag,
// sleeping between reads; s_memrealtime counts at a constant 100 MHz.
__global__ void hold_kernel(const int *flag, uint64_t max_ticks) {
    if (threadIdx.x != 0) return;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) == 0) {
        if (__builtin_amdgcn_s_memrealtime() - t0 >= max_ticks) break;
        __builtin_amdgcn_s_sleep(64);
    }
}

struct Fold {
    FoldDone *rec;
    int64_t trigger;   // block whose commit enqueued the fold
    double flops;      // algorithmic flops of the fold
};

struct Stream {
    bool open = false;
    xc_stream_desc d{};
    Plan plan{};
    int groups = 1;           // channel groups folded in turn (k when staggered)
    size_t footprint = 0;
    size_t block_bytes = 0;   // one ring slot
    size_t acc_bytes = 0;
    size_t chan_sample_bytes = 0;  // one channel of one slot
    size_t chan_vis_bytes = 0;     // one channel of an accumulator
    int64_t block_elems = 0;  // station-samples per slot (C * block_times * S)
    int64_t B = 0;
    void *ring = nullptr;
    void *acc[2] = {nullptr, nullptr};
    hipStream_t hs = nullptr;
    hipEvent_t ready_ev[2] = {nullptr, nullptr};    // recorded after an integration's last fold
    hipEvent_t release_ev[2] = {nullptr, nullptr};  // recorded on a consumer's stream by xc_stream_release
    hipEvent_t fill_ev = nullptr;                   // recorded on a producer's stream by xc_stream_commit_after
    hipEvent_t fold_ev = nullptr;                   // recorded after each fold (fold order across streams)
    int32_t *hold_flag = nullptr;                   // host-coherent flag that ends a hold (xc_stream_hold)
    bool release_pending[2] = {false, false};
    int64_t published_seq = -1;
    int64_t committed = 0;    // blocks committed so far
    bool acquired = false;    // a slot has been handed out and not yet committed
    std::vector<int64_t> group_next;   // per channel group: first block it has not folded
    // per ring slot: the last fold that reads it (nullptr = free)
    std::vector<FoldDone *> slot_busy;
    // latency records of blocks rec_base .. committed - 1: arrival and the
    // last fold covering the block (nullptr while it is not yet folded)
    int64_t rec_base = 0;
    std::deque<uint64_t> arrivals;
    std::deque<FoldDone *> block_fold;
    std::vector<Fold> folds;          // folds enqueued since the last reset
};

}  // namespace

struct xc_server {
    std::mutex mu;
    size_t budget = 0;
    size_t used = 0;
    std::vector<Stream> streams;
    bool ordered = false;   // folds of all streams one at a time, in enqueue order
    int last_fold = -1;     // stream that enqueued the latest fold (ordered)
};

static xc_status validate_desc(const xc_stream_desc *d) {
    if (!d) return set_error(XC_ERR_INVALID_ARG, "null stream descriptor");
    if (d->n_pol != 2) return set_error(XC_ERR_UNSUPPORTED, "n_pol must be 2");
    if (d->n_stations < 1 || d->n_channels < 1 || d->block_times < 1 || d->blocks_per_integration < 1 ||
        d->blocks_per_fold < 1 || d->ring_blocks < 1)
        return set_error(XC_ERR_INVALID_ARG, "stream sizes must be >= 1");
    if (d->blocks_per_integration % d->blocks_per_fold)
        return set_error(XC_ERR_INVALID_ARG, "blocks_per_integration must be a multiple of blocks_per_fold");
    if (d->ring_blocks < 2 * d->blocks_per_fold)
        return set_error(XC_ERR_INVALID_ARG, "ring_blocks must be >= 2 * blocks_per_fold");
    if (d->staggered < 0 || d->staggered > 2) return set_error(XC_ERR_INVALID_ARG, "staggered must be 0, 1 or 2");
    if (!(d->block_period_s >= 0.0)) return set_error(XC_ERR_INVALID_ARG, "block_period_s must be >= 0");
    const int64_t T_int = (int64_t)d->block_times * d->blocks_per_integration;
    if (d->acc_type == XC_OUT_CI32 && T_int > XC_CI32_MAX_TIMES)
        return set_error(XC_ERR_OVERFLOW_RISK, "an integration of %lld samples could overflow int32",
                         (long long)T_int);
    if ((int64_t)d->block_times * d->blocks_per_fold > (1 << 30))
        return set_error(XC_ERR_UNSUPPORTED, "a fold of %d blocks of %d samples is too long", d->blocks_per_fold,
                         d->block_times);
    Plan p;
    return resolve(nullptr, (xc_in_type)d->in_type, (xc_out_type)d->acc_type, d->n_stations, d->n_pol,
                   d->n_channels, d->block_times * d->blocks_per_fold, &p);
}

static void stream_free(Stream &s) {
    if (s.hold_flag) __atomic_store_n(s.hold_flag, 1, __ATOMIC_RELEASE);
    if (s.hs) (void)hipStreamSynchronize(s.hs);
    for (auto &f : s.folds) delete f.rec;
    s.folds.clear();
    if (s.ring) (void)hipFree(s.ring);
    for (auto &a : s.acc)
        if (a) (void)hipFree(a);
    for (int k = 0; k < 2; ++k) {
        if (s.ready_ev[k]) (void)hipEventDestroy(s.ready_ev[k]);
        if (s.release_ev[k]) (void)hipEventDestroy(s.release_ev[k]);
    }
    if (s.fill_ev) (void)hipEventDestroy(s.fill_ev);
    if (s.fold_ev) (void)hipEventDestroy(s.fold_ev);
    if (s.hold_flag) (void)hipHostFree(s.hold_flag);
    if (s.hs) (void)hipStreamDestroy(s.hs);
    s = Stream{};
}

// Channels [c0, c1) of channel group g of groups, over C channels.
static void group_range(int C, int groups, int g, int &c0, int &c1) {
    c0 = (int)((int64_t)C * g / groups);
    c1 = (int)((int64_t)C * (g + 1) / groups);
}

static void group_channels(const Stream &s, int g, int &c0, int &c1) {
    group_range(s.d.n_channels, s.groups, g, c0, c1);
}

// ---- The fold schedule (host logic only, no device calls) ----

struct PlannedFold {
    int g;                 // channel group
    int64_t first, last;   // blocks, all in one integration
};

// Appends the folds of group g over blocks first .. last, one per integration
// they fall in.
static void plan_range(int g, int64_t first, int64_t last, int64_t bpi, std::vector<PlannedFold> &out) {
    while (first <= last) {
        const int64_t end = std::min(last, (first / bpi + 1) * bpi - 1);
        out.push_back(PlannedFold{g, first, end});
        first = end + 1;
    }
}

// Appends, in enqueue order, the folds that the commit of block n starts;
// next[g] (each group's first block not yet folded) is advanced.
static void plan_commit(const xc_stream_desc &d, int groups, int64_t n, std::vector<int64_t> &next,
                        std::vector<PlannedFold> &out) {
    const int64_t bpi = d.blocks_per_integration, m = n % bpi;
    const int k = d.blocks_per_fold;
    const bool spread = d.staggered == 2;
    if (m == 0 && !spread)
        for (auto &g : next) g = n;
    auto take = [&](int g) {
        plan_range(g, next[g], n, bpi, out);
        next[g] = n + 1;
    };
    if (groups == 1) {
        if ((m + 1) % k == 0) take(0);
    } else if (spread) {
        // group m mod k folds its outstanding blocks, the rest of the last
        // integration first
        const int g = (int)(m % k);
        if (next[g] <= n) take(g);
    } else {
        // group m mod k folds its outstanding blocks.  At the end of the
        // integration every group does, in the order of their oldest pending
        // block (the regular group's k blocks first, then the others' shorter
        // remainders), so that each block's last fold comes as early as it can.
        const bool last = m == bpi - 1;
        std::vector<int> order;
        for (int g = 0; g < groups; ++g)
            if ((last || g == (int)(m % k)) && next[g] <= n) order.push_back(g);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return next[a] < next[b]; });
        for (int g : order) take(g);
    }
}

// Spread ends: the folds that complete every integration whose blocks have
// all been committed, oldest pending block first.
static void plan_flush(const xc_stream_desc &d, int groups, int64_t committed, std::vector<int64_t> &next,
                       std::vector<PlannedFold> &out) {
    if (d.staggered != 2) return;     // nothing is left over past an integration's end
    const int64_t bpi = d.blocks_per_integration;
    const int64_t end = committed / bpi * bpi;
    std::vector<int> order;
    for (int g = 0; g < groups; ++g)
        if (next[g] < end) order.push_back(g);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return next[a] < next[b]; });
    for (int g : order) {
        plan_range(g, next[g], end - 1, bpi, out);
        next[g] = end;
    }
}

// Last integration published once `committed` blocks are in and the groups
// have folded up to next: with spread ends, every integration that all groups
// have folded past; otherwise each integration at its last block.
static int64_t plan_published(const xc_stream_desc &d, int64_t committed, const std::vector<int64_t> &next) {
    const int64_t bpi = d.blocks_per_integration;
    int64_t folded = committed;
    if (d.staggered == 2)
        for (int64_t g : next) folded = std::min(folded, g);
    return folded / bpi - 1;
}

// Enqueues the fold of channel group g over blocks first .. last (absolute
// numbers, all in one integration) after prev's latest fold (if not null),
// and records it.
static xc_status enqueue_fold(Stream &s, const Stream *prev, int g, int64_t first, int64_t last, int64_t trigger) {
    int c0, c1;
    group_channels(s, g, c0, c1);
    if (c1 <= c0) return XC_OK;
    const int64_t bpi = s.d.blocks_per_integration;
    const int64_t integ = first / bpi;
    const int nblk = (int)(last - first + 1);
    const int slot0 = (int)(first % s.d.ring_blocks);
    const bool overwrite = first == integ * bpi;
    Job job = make_job(static_cast<uint8_t *>(s.ring) + (size_t)c0 * s.chan_sample_bytes,
                       static_cast<uint8_t *>(s.acc[integ % 2]) + (size_t)c0 * s.chan_vis_bytes, s.d.n_stations,
                       c1 - c0, s.d.block_times * nblk, s.plan.block, overwrite ? 0 : 1);
    job.tblk = s.d.block_times;
    job.bstride = s.block_elems;
    job.slot0 = slot0;
    job.nring = s.d.ring_blocks;
    if (prev) {
        hipError_t e = hipStreamWaitEvent(s.hs, prev->fold_ev, 0);
        if (e != hipSuccess) return hip_error(e, "fold order");
    }
    xc_status st = launch_plan(s.plan, (xc_in_type)s.d.in_type, (xc_out_type)s.d.acc_type, job, s.hs);
    if (st != XC_OK) return st;
    {
        hipError_t e = hipEventRecord(s.fold_ev, s.hs);
        if (e != hipSuccess) return hip_error(e, "fold event");
    }
    FoldDone *rec = new FoldDone;
    hipError_t e = hipLaunchHostFunc(s.hs, on_fold_done, rec);
    if (e != hipSuccess) {
        delete rec;
        return hip_error(e, "hipLaunchHostFunc");
    }
    for (int64_t b = first; b <= last; ++b) {
        s.slot_busy[(size_t)(b % s.d.ring_blocks)] = rec;
        if (b >= s.rec_base) s.block_fold[(size_t)(b - s.rec_base)] = rec;
    }
    s.folds.push_back(Fold{rec, trigger, 32.0 * (c1 - c0) * (double)s.d.block_times * nblk * (double)s.B});
    return XC_OK;
}

extern "C" {

size_t xc_stream_footprint(const xc_stream_desc *d) {
    if (!d || d->n_stations < 1 || d->n_channels < 1 || d->block_times < 1 || d->ring_blocks < 1) return 0;
    const size_t B = (size_t)d->n_stations * (d->n_stations + 1) / 2;
    const size_t acc = (size_t)d->n_channels * B * 4 * 8;
    const size_t block = (size_t)d->n_channels * d->block_times * d->n_stations * 2 * in_elem_bytes(d->in_type);
    return 2 * acc + (size_t)d->ring_blocks * block;
}

xc_status xc_stream_schedule(const xc_stream_desc *desc, int64_t n_blocks, int32_t flush, int64_t *folds,
                             int64_t max_folds, int64_t *n_folds, int64_t *published_after,
                             int64_t max_integrations) {
    if (!n_folds || (max_folds > 0 && !folds) || (max_integrations > 0 && !published_after))
        return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (n_blocks < 0 || max_folds < 0 || max_integrations < 0)
        return set_error(XC_ERR_INVALID_ARG, "negative count");
    if (flush != 0 && flush != 1) return set_error(XC_ERR_INVALID_ARG, "flush must be 0 or 1");
    xc_status st = validate_desc(desc);
    if (st != XC_OK) return st;
    const xc_stream_desc &d = *desc;
    const int groups = d.staggered ? d.blocks_per_fold : 1;
    std::vector<int64_t> next((size_t)groups, 0);
    std::vector<PlannedFold> plan;
    for (int64_t j = 0; j < max_integrations; ++j) published_after[j] = -1;
    int64_t count = 0, published = -1;
    auto emit = [&](int64_t trigger) {
        for (const auto &f : plan) {
            if (count < max_folds) {
                int c0, c1;
                group_range(d.n_channels, groups, f.g, c0, c1);
                int64_t *r = folds + 6 * count;
                r[0] = trigger;
                r[1] = f.g;
                r[2] = c0;
                r[3] = c1;
                r[4] = f.first;
                r[5] = f.last;
            }
            ++count;
        }
        plan.clear();
    };
    auto publish = [&](int64_t committed, int64_t when) {
        const int64_t last = plan_published(d, committed, next);
        for (int64_t j = published + 1; j <= last && j < max_integrations; ++j) published_after[j] = when;
        published = std::max(published, last);
    };
    for (int64_t n = 0; n < n_blocks; ++n) {
        plan_commit(d, groups, n, next, plan);
        emit(n);
        publish(n + 1, n);
    }
    if (flush) {
        plan_flush(d, groups, n_blocks, next, plan);
        emit(n_blocks - 1);
        publish(n_blocks, n_blocks);
    }
    *n_folds = count;
    return XC_OK;
}

double xc_quantile(const double *values, int64_t n, double q) {
    if (!values || n <= 0) return NAN;
    std::vector<double> v(values, values + n);
    std::sort(v.begin(), v.end());
    // nearest rank: the smallest value with at least q n values <= it
    int64_t rank = (int64_t)std::ceil(q * (double)n);
    if (rank < 1) rank = 1;
    if (rank > n) rank = n;
    return v[(size_t)rank - 1];
}

xc_status xc_server_create(size_t hbm_budget_bytes, xc_server **out) {
    if (!out) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    size_t budget = hbm_budget_bytes;
    if (budget == 0) {
        size_t free_b = 0, total = 0;
        hipError_t e = hipMemGetInfo(&free_b, &total);
        if (e != hipSuccess) return hip_error(e, "hipMemGetInfo");
        budget = (size_t)(0.9 * (double)free_b);
    }
    xc_server *s = new xc_server;
    s->budget = budget;
    *out = s;
    log_line("server: device-memory budget %.3f GB", budget / 1e9);
    return XC_OK;
}

void xc_server_destroy(xc_server *srv) {
    if (!srv) return;
    for (auto &s : srv->streams)
        if (s.open) stream_free(s);
    delete srv;
}

xc_status xc_stream_open(xc_server *srv, const xc_stream_desc *desc, int32_t *stream_id) {
    if (!srv || !stream_id) return set_error(XC_ERR_INVALID_ARG, "null server or id pointer");
    xc_status st = validate_desc(desc);
    if (st != XC_OK) return st;
    std::lock_guard<std::mutex> lk(srv->mu);
    const size_t fp = xc_stream_footprint(desc);
    if (srv->used + fp > srv->budget) {
        log_line("stream refused: %d stations x %d channels, k %d, needs %.3f GB, %.3f of %.3f GB left",
                 desc->n_stations, desc->n_channels, desc->blocks_per_fold, fp / 1e9, (srv->budget - srv->used) / 1e9,
                 srv->budget / 1e9);
        return set_error(XC_ERR_ADMISSION, "stream needs %zu bytes, %zu of %zu left", fp, srv->budget - srv->used,
                         srv->budget);
    }
    Stream s;
    s.d = *desc;
    resolve(nullptr, (xc_in_type)desc->in_type, (xc_out_type)desc->acc_type, desc->n_stations, 2, desc->n_channels,
            desc->block_times * desc->blocks_per_fold, &s.plan);
    s.groups = desc->staggered ? desc->blocks_per_fold : 1;
    s.footprint = fp;
    s.B = (int64_t)desc->n_stations * (desc->n_stations + 1) / 2;
    s.acc_bytes = (size_t)desc->n_channels * s.B * 4 * 8;
    s.chan_vis_bytes = (size_t)s.B * 4 * 8;
    s.block_elems = (int64_t)desc->n_channels * desc->block_times * desc->n_stations;
    s.block_bytes = (size_t)s.block_elems * 2 * in_elem_bytes(desc->in_type);
    s.chan_sample_bytes = (size_t)desc->block_times * desc->n_stations * 2 * in_elem_bytes(desc->in_type);
    hipError_t e = hipMalloc(&s.ring, s.block_bytes * desc->ring_blocks);
    if (e == hipSuccess) e = hipMalloc(&s.acc[0], s.acc_bytes);
    if (e == hipSuccess) e = hipMalloc(&s.acc[1], s.acc_bytes);
    if (e != hipSuccess) {
        stream_free(s);
        return set_error(XC_ERR_OUT_OF_MEMORY, "stream allocation failed: %s", hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&s.hs, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&s.ready_ev[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.release_ev[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.fill_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.fold_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.hold_flag, sizeof(int32_t), hipHostMallocCoherent);
    if (e == hipSuccess) __atomic_store_n(s.hold_flag, 1, __ATOMIC_RELEASE);
    if (e != hipSuccess) {
        stream_free(s);
        return hip_error(e, "stream or event creation");
    }
    s.slot_busy.assign(desc->ring_blocks, nullptr);
    s.group_next.assign(s.groups, 0);
    s.open = true;
    srv->used += fp;
    int id = -1;
    for (size_t k = 0; k < srv->streams.size(); ++k)
        if (!srv->streams[k].open) {
            id = (int)k;
            break;
        }
    if (id < 0) {
        srv->streams.emplace_back();
        id = (int)srv->streams.size() - 1;
    }
    srv->streams[id] = std::move(s);
    *stream_id = id;
    log_line("stream %d opened: %d stations x %d channels, blocks of %d samples, k %d (%s), ring %d blocks, "
             "%.3f GB", id, desc->n_stations, desc->n_channels, desc->block_times, desc->blocks_per_fold,
             desc->staggered == 2 ? "staggered, ends spread" : desc->staggered ? "staggered" : "all channels",
             desc->ring_blocks, fp / 1e9);
    return XC_OK;
}

static Stream *get_stream(xc_server *srv, int32_t id) {
    if (!srv || id < 0 || (size_t)id >= srv->streams.size() || !srv->streams[id].open) return nullptr;
    return &srv->streams[id];
}

xc_status xc_stream_acquire(xc_server *srv, int32_t id, void **block_dev_ptr) {
    if (!block_dev_ptr) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    if (s->acquired) return set_error(XC_ERR_STATE, "stream %d: previous slot not committed", id);
    const int slot = (int)(s->committed % s->d.ring_blocks);
    FoldDone *busy = s->slot_busy[slot];
    if (busy) {
        if (!is_done(busy))
            return set_error(XC_ERR_BACKPRESSURE, "stream %d: ring full (slot %d still being folded)", id, slot);
        s->slot_busy[slot] = nullptr;
    }
    s->acquired = true;
    *block_dev_ptr = static_cast<uint8_t *>(s->ring) + (size_t)slot * s->block_bytes;
    return XC_OK;
}

// Enqueues a planned fold of stream id, after the server's previous fold when
// folds run in order.
static xc_status enqueue_planned(xc_server *srv, Stream &s, int32_t id, const PlannedFold &f, int64_t trigger) {
    const Stream *prev = nullptr;
    if (srv->ordered && srv->last_fold >= 0 && srv->last_fold != id && srv->streams[srv->last_fold].open)
        prev = &srv->streams[srv->last_fold];
    xc_status st = enqueue_fold(s, prev, f.g, f.first, f.last, trigger);
    if (st == XC_OK) srv->last_fold = id;
    return st;
}

// Enqueues the planned folds in order; each group's progress is kept as far
// as its folds were enqueued, the planned progress once all were.
static xc_status enqueue_plan(xc_server *srv, Stream &s, int32_t id, const std::vector<PlannedFold> &plan,
                              const std::vector<int64_t> &next, int64_t trigger) {
    for (const auto &f : plan) {
        xc_status st = enqueue_planned(srv, s, id, f, trigger);
        if (st != XC_OK) return st;
        s.group_next[f.g] = f.last + 1;
    }
    s.group_next = next;
    return XC_OK;
}

// Records the ready event of every integration up to `last` not yet published.
static xc_status publish_up_to(Stream &s, int64_t last) {
    while (s.published_seq < last) {
        const int64_t j = s.published_seq + 1;
        hipError_t e = hipEventRecord(s.ready_ev[j % 2], s.hs);
        if (e != hipSuccess) return hip_error(e, "integration event");
        s.published_seq = j;
    }
    return XC_OK;
}

static xc_status commit_locked(xc_server *srv, Stream *s, int32_t id, uint64_t arrival_ns, hipStream_t producer) {
    if (!s->acquired) return set_error(XC_ERR_STATE, "stream %d: commit without acquire", id);
    if (producer) {
        // the folds that read this slot run after the producer's work so far
        hipError_t e = hipEventRecord(s->fill_ev, producer);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->hs, s->fill_ev, 0);
        if (e != hipSuccess) return hip_error(e, "producer event");
    }
    s->acquired = false;
    const int64_t n = s->committed++;
    s->arrivals.push_back(arrival_ns);
    s->block_fold.push_back(nullptr);
    const int64_t bpi = s->d.blocks_per_integration;
    const int64_t integ = n / bpi, m = n % bpi;
    if (m == 0 && s->release_pending[integ % 2]) {
        // a new integration starts: its accumulator held integration integ - 2,
        // which a consumer may still be reading
        hipError_t e = hipStreamWaitEvent(s->hs, s->release_ev[integ % 2], 0);
        if (e != hipSuccess) return hip_error(e, "release event");
        s->release_pending[integ % 2] = false;
    }
    std::vector<int64_t> next = s->group_next;
    std::vector<PlannedFold> plan;
    plan_commit(s->d, s->groups, n, next, plan);
    xc_status st = enqueue_plan(srv, *s, id, plan, next, n);
    if (st != XC_OK) return st;
    return publish_up_to(*s, plan_published(s->d, s->committed, s->group_next));
}

xc_status xc_stream_commit(xc_server *srv, int32_t id, uint64_t arrival_ns) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    return commit_locked(srv, s, id, arrival_ns, nullptr);
}

xc_status xc_stream_commit_after(xc_server *srv, int32_t id, uint64_t arrival_ns, void *producer_stream) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    return commit_locked(srv, s, id, arrival_ns, static_cast<hipStream_t>(producer_stream));
}

xc_status xc_stream_integration(xc_server *srv, int32_t id, int64_t k, const void **vis, void **ready) {
    if (!vis || !ready) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    // integration k + 2 reuses the buffer from its first block on
    const int64_t started = s->committed ? (s->committed - 1) / s->d.blocks_per_integration : -1;
    if (k < 0 || k > s->published_seq || started >= k + 2)
        return set_error(XC_ERR_STATE, "stream %d: integration %lld is not available (published: %lld, started: %lld)",
                         id, (long long)k, (long long)s->published_seq, (long long)started);
    *vis = s->acc[k % 2];
    *ready = s->ready_ev[k % 2];
    return XC_OK;
}

xc_status xc_wait_event(void *event, void *stream) {
    if (!event) return set_error(XC_ERR_INVALID_ARG, "null event");
    hipError_t e = hipStreamWaitEvent(static_cast<hipStream_t>(stream), static_cast<hipEvent_t>(event), 0);
    if (e != hipSuccess) return hip_error(e, "hipStreamWaitEvent");
    return XC_OK;
}

xc_status xc_stream_release(xc_server *srv, int32_t id, int64_t k, void *consumer_stream) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    const int64_t started = s->committed ? (s->committed - 1) / s->d.blocks_per_integration : -1;
    if (k < 0 || k > s->published_seq || started >= k + 2)
        return set_error(XC_ERR_STATE, "stream %d: integration %lld is not available", id, (long long)k);
    hipError_t e = hipEventRecord(s->release_ev[k % 2], static_cast<hipStream_t>(consumer_stream));
    if (e != hipSuccess) return hip_error(e, "release event");
    s->release_pending[k % 2] = true;
    return XC_OK;
}

xc_status xc_stream_latest(xc_server *srv, int32_t id, const void **vis, int64_t *sequence) {
    if (!vis || !sequence) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    *vis = s->published_seq >= 0 ? s->acc[s->published_seq % 2] : nullptr;
    *sequence = s->published_seq;
    return XC_OK;
}

xc_status xc_stream_hold(xc_server *srv, int32_t id, double max_wait_s) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    if (!(max_wait_s >= 0.0 && max_wait_s <= 60.0)) return set_error(XC_ERR_INVALID_ARG, "max_wait_s must be in [0, 60]");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    __atomic_store_n(s->hold_flag, 0, __ATOMIC_RELEASE);
    const uint64_t ticks = (uint64_t)(max_wait_s * 1e8);   // s_memrealtime: 100 MHz
    hipLaunchKernelGGL(hold_kernel, dim3(1), dim3(64), 0, s->hs, (const int *)s->hold_flag, ticks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        __atomic_store_n(s->hold_flag, 1, __ATOMIC_RELEASE);
        return hip_error(e, "hold launch");
    }
    return XC_OK;
}

xc_status xc_stream_resume(xc_server *srv, int32_t id) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    __atomic_store_n(s->hold_flag, 1, __ATOMIC_RELEASE);
    return XC_OK;
}

xc_status xc_stream_stats(xc_server *srv, int32_t id, xc_latency_stats *stats) {
    if (!stats) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    hipStream_t hs;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        Stream *s = get_stream(srv, id);
        if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
        hs = s->hs;
    }
    // wait without the lock: the server's other streams go on
    hipError_t e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s || s->hs != hs) return set_error(XC_ERR_STATE, "stream %d was closed during the call", id);
    const double P_ms = 1e3 * s->d.block_period_s;
    const double deadline = P_ms * s->d.blocks_per_fold;
    const double fold_deadline = s->groups > 1 ? P_ms : deadline;
    std::vector<double> lat, flat;
    uint64_t t_first = UINT64_MAX, t_last = 0;
    int64_t pending = 0;
    for (size_t b = 0; b < s->arrivals.size(); ++b) {
        const FoldDone *f = s->block_fold[b];
        if (!is_done(f)) {       // not folded yet (or folded by work enqueued after the wait)
            pending++;
            continue;
        }
        const uint64_t a = s->arrivals[b];
        lat.push_back(f->done_ns > a ? (double)(f->done_ns - a) * 1e-6 : 0.0);
        t_first = std::min(t_first, a);
    }
    double flops = 0;
    for (auto &f : s->folds) {
        if (!is_done(f.rec)) continue;
        const int64_t b = f.trigger - s->rec_base;
        if (b >= 0 && (size_t)b < s->arrivals.size()) {
            const uint64_t a = s->arrivals[(size_t)b];
            flat.push_back(f.rec->done_ns > a ? (double)(f.rec->done_ns - a) * 1e-6 : 0.0);
        }
        flops += f.flops;
        t_last = std::max(t_last, f.rec->done_ns);
    }
    xc_latency_stats r{};
    r.blocks = (int64_t)lat.size();
    r.pending = pending;
    r.folds = (int64_t)flat.size();
    r.deadline_ms = deadline;
    r.fold_deadline_ms = fold_deadline;
    r.p50_ms = xc_quantile(lat.data(), (int64_t)lat.size(), 0.50);
    r.p99_ms = xc_quantile(lat.data(), (int64_t)lat.size(), 0.99);
    r.max_ms = lat.empty() ? NAN : *std::max_element(lat.begin(), lat.end());
    r.fold_p50_ms = xc_quantile(flat.data(), (int64_t)flat.size(), 0.50);
    r.fold_p99_ms = xc_quantile(flat.data(), (int64_t)flat.size(), 0.99);
    r.fold_max_ms = flat.empty() ? NAN : *std::max_element(flat.begin(), flat.end());
    for (double v : lat)
        if (deadline > 0 && v > deadline) r.misses++;
    for (double v : flat)
        if (fold_deadline > 0 && v > fold_deadline) r.fold_misses++;
    const double span = (t_last > t_first && t_first != UINT64_MAX) ? (double)(t_last - t_first) * 1e-9 : 0.0;
    r.tflops = span > 0 ? flops / span * 1e-12 : 0.0;
    r.integrations = s->published_seq + 1;
    *stats = r;
    return XC_OK;
}

xc_status xc_stream_reset_stats(xc_server *srv, int32_t id) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    hipStream_t hs;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        Stream *s = get_stream(srv, id);
        if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
        hs = s->hs;
    }
    hipError_t e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s || s->hs != hs) return set_error(XC_ERR_STATE, "stream %d was closed during the call", id);
    // folds enqueued by another thread after the wait may still run: wait for them too
    e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    for (auto &b : s->slot_busy) b = nullptr;
    for (auto &f : s->folds) delete f.rec;
    s->folds.clear();
    s->arrivals.clear();
    s->block_fold.clear();
    s->rec_base = s->committed;
    return XC_OK;
}

xc_status xc_stream_flush(xc_server *srv, int32_t id) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    std::vector<int64_t> next = s->group_next;
    std::vector<PlannedFold> plan;
    plan_flush(s->d, s->groups, s->committed, next, plan);
    xc_status st = enqueue_plan(srv, *s, id, plan, next, s->committed - 1);
    if (st != XC_OK) return st;
    return publish_up_to(*s, plan_published(s->d, s->committed, s->group_next));
}

xc_status xc_server_set_fold_order(xc_server *srv, int32_t one_at_a_time) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    if (one_at_a_time != 0 && one_at_a_time != 1) return set_error(XC_ERR_INVALID_ARG, "one_at_a_time must be 0 or 1");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->ordered = one_at_a_time != 0;
    srv->last_fold = -1;
    return XC_OK;
}

xc_status xc_stream_close(xc_server *srv, int32_t id) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    if (srv->last_fold == id) srv->last_fold = -1;
    srv->used -= s->footprint;
    log_line("stream %d closed after %lld blocks", id, (long long)s->committed);
    stream_free(*s);
    return XC_OK;
}

}  // extern "C"
