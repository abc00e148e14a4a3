// Streaming correlator server.
//
// The correlator is a streaming, real-time application (Section 1): sample
// blocks arrive at a fixed period and must be integrated (Section 2: about one
// second of samples per integration) without falling behind.  Each stream owns
//   - a device ring of `ring_blocks` sample blocks x[C][block_times][S][2],
//   - two resident accumulators V[C][B][2][2]: one integrating, one holding
//     the last published integration,
//   - a HIP stream on which its folds run in order.
// Every `blocks_per_fold` committed blocks, one accumulate-mode correlation
// over those consecutive ring slots is enqueued (the integration is split into
// sub-intervals whose partial sums are added into the resident result, as
// Section 4.5 does with the Cell's local store).  The first fold of an
// integration overwrites instead of adding, so no clearing pass is needed.
// A host function enqueued after each fold records its completion time on
// the host clock; per-block latency = completion - arrival, per-fold latency
// = completion - arrival of the fold's last block (the deadline applies to
// folds: finish before the next fold's blocks are all in).
// Streams are admitted only if their device footprint fits the budget.
#include <time.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "common.h"

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

struct Stream {
    bool open = false;
    xc_stream_desc d{};
    Plan plan{};
    size_t footprint = 0;
    size_t block_bytes = 0;   // one ring slot
    size_t acc_bytes = 0;
    int64_t block_elems = 0;  // station-samples per slot (C * block_times * S)
    void *ring = nullptr;
    void *acc[2] = {nullptr, nullptr};
    hipStream_t hs = nullptr;
    int active = 0;           // accumulator being integrated
    int64_t published_seq = -1;
    int published = -1;       // accumulator index of the last published integration
    int64_t committed = 0;    // blocks committed so far
    bool acquired = false;    // a slot has been handed out and not yet committed
    // per ring slot: fold record that must complete before reuse (nullptr = free)
    std::vector<FoldDone *> slot_busy;
    std::vector<uint64_t> pending_arrivals;  // arrivals of the blocks of the open fold
    // per fold: completion record and the arrivals of its blocks
    struct Fold {
        FoldDone *rec;
        std::vector<uint64_t> arrivals;
    };
    std::vector<Fold> folds;
    double flops_per_fold = 0;
};

}  // namespace

struct xc_server {
    std::mutex mu;
    size_t budget = 0;
    size_t used = 0;
    std::vector<Stream> streams;
};

static xc_status validate_desc(const xc_stream_desc *d) {
    if (!d) return set_error(XC_ERR_INVALID_ARG, "null stream descriptor");
    if (d->n_pol != 2) return set_error(XC_ERR_UNSUPPORTED, "n_pol must be 2");
    if (d->n_stations < 1 || d->n_channels < 1 || d->block_times < 1 || d->blocks_per_integration < 1 ||
        d->blocks_per_fold < 1 || d->ring_blocks < 1)
        return set_error(XC_ERR_INVALID_ARG, "stream sizes must be >= 1");
    if (d->blocks_per_integration % d->blocks_per_fold)
        return set_error(XC_ERR_INVALID_ARG, "blocks_per_integration must be a multiple of blocks_per_fold");
    if (d->ring_blocks % d->blocks_per_fold || d->ring_blocks < 2 * d->blocks_per_fold)
        return set_error(XC_ERR_INVALID_ARG, "ring_blocks must be a multiple of blocks_per_fold and >= 2 folds");
    if (!(d->block_period_s >= 0.0)) return set_error(XC_ERR_INVALID_ARG, "block_period_s must be >= 0");
    const int64_t T_int = (int64_t)d->block_times * d->blocks_per_integration;
    if (d->acc_type == XC_OUT_CI32 && T_int > XC_CI32_MAX_TIMES)
        return set_error(XC_ERR_OVERFLOW_RISK, "an integration of %lld samples could overflow int32",
                         (long long)T_int);
    Plan p;
    return resolve(nullptr, (xc_in_type)d->in_type, (xc_out_type)d->acc_type, d->n_stations, d->n_pol,
                   d->n_channels, d->block_times * d->blocks_per_fold, &p);
}

static void stream_free(Stream &s) {
    if (s.hs) (void)hipStreamSynchronize(s.hs);
    for (auto &f : s.folds) delete f.rec;
    s.folds.clear();
    if (s.ring) (void)hipFree(s.ring);
    for (auto &a : s.acc)
        if (a) (void)hipFree(a);
    if (s.hs) (void)hipStreamDestroy(s.hs);
    s = Stream{};
}

extern "C" {

size_t xc_stream_footprint(const xc_stream_desc *d) {
    if (!d || d->n_stations < 1 || d->n_channels < 1 || d->block_times < 1 || d->ring_blocks < 1) return 0;
    const size_t B = (size_t)d->n_stations * (d->n_stations + 1) / 2;
    const size_t acc = (size_t)d->n_channels * B * 4 * 8;
    const size_t block = (size_t)d->n_channels * d->block_times * d->n_stations * 2 * in_elem_bytes(d->in_type);
    return 2 * acc + (size_t)d->ring_blocks * block;
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
    if (srv->used + fp > srv->budget)
        return set_error(XC_ERR_ADMISSION, "stream needs %zu bytes, %zu of %zu left", fp, srv->budget - srv->used,
                         srv->budget);
    Stream s;
    s.d = *desc;
    resolve(nullptr, (xc_in_type)desc->in_type, (xc_out_type)desc->acc_type, desc->n_stations, 2, desc->n_channels,
            desc->block_times * desc->blocks_per_fold, &s.plan);
    s.footprint = fp;
    const size_t B = (size_t)desc->n_stations * (desc->n_stations + 1) / 2;
    s.acc_bytes = (size_t)desc->n_channels * B * 4 * 8;
    s.block_elems = (int64_t)desc->n_channels * desc->block_times * desc->n_stations;
    s.block_bytes = (size_t)s.block_elems * 2 * in_elem_bytes(desc->in_type);
    hipError_t e = hipMalloc(&s.ring, s.block_bytes * desc->ring_blocks);
    if (e == hipSuccess) e = hipMalloc(&s.acc[0], s.acc_bytes);
    if (e == hipSuccess) e = hipMalloc(&s.acc[1], s.acc_bytes);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.hs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        stream_free(s);
        return set_error(XC_ERR_OUT_OF_MEMORY, "stream allocation failed: %s", hipGetErrorString(e));
    }
    s.slot_busy.assign(desc->ring_blocks, nullptr);
    s.flops_per_fold = 32.0 * desc->n_channels * (double)desc->block_times * desc->blocks_per_fold * (double)B;
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
        if (!__atomic_load_n(&busy->done, __ATOMIC_ACQUIRE))
            return set_error(XC_ERR_BACKPRESSURE, "stream %d: ring full (slot %d still being folded)", id, slot);
        s->slot_busy[slot] = nullptr;
    }
    s->acquired = true;
    *block_dev_ptr = static_cast<uint8_t *>(s->ring) + (size_t)slot * s->block_bytes;
    return XC_OK;
}

xc_status xc_stream_commit(xc_server *srv, int32_t id, uint64_t arrival_ns) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    if (!s->acquired) return set_error(XC_ERR_STATE, "stream %d: commit without acquire", id);
    s->acquired = false;
    s->pending_arrivals.push_back(arrival_ns);
    s->committed++;
    const int k = s->d.blocks_per_fold;
    if (s->committed % k) return XC_OK;
    // enqueue the fold over the last k slots
    const int64_t first_block = s->committed - k;
    const int slot0 = (int)(first_block % s->d.ring_blocks);
    const int64_t in_integration = first_block % s->d.blocks_per_integration;
    Job job = make_job(static_cast<uint8_t *>(s->ring) + (size_t)slot0 * s->block_bytes, s->acc[s->active],
                       s->d.n_stations, s->d.n_channels, s->d.block_times * k, s->plan.block,
                       in_integration == 0 ? 0 : 1);
    job.tblk = s->d.block_times;
    job.bstride = s->block_elems;
    xc_status st = launch_plan(s->plan, (xc_in_type)s->d.in_type, (xc_out_type)s->d.acc_type, job, s->hs);
    if (st != XC_OK) return st;
    FoldDone *rec = new FoldDone;
    hipError_t e = hipLaunchHostFunc(s->hs, on_fold_done, rec);
    if (e != hipSuccess) {
        delete rec;
        return hip_error(e, "hipLaunchHostFunc");
    }
    for (int b = 0; b < k; ++b) s->slot_busy[(slot0 + b) % s->d.ring_blocks] = rec;
    s->folds.push_back(Stream::Fold{rec, std::move(s->pending_arrivals)});
    s->pending_arrivals.clear();
    if ((s->committed % s->d.blocks_per_integration) == 0) {
        s->published = s->active;
        s->published_seq = s->committed / s->d.blocks_per_integration - 1;
        s->active ^= 1;
    }
    return XC_OK;
}

xc_status xc_stream_latest(xc_server *srv, int32_t id, const void **vis, int64_t *sequence) {
    if (!vis || !sequence) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    *vis = s->published >= 0 ? s->acc[s->published] : nullptr;
    *sequence = s->published_seq;
    return XC_OK;
}

xc_status xc_stream_stats(xc_server *srv, int32_t id, xc_latency_stats *stats) {
    if (!stats) return set_error(XC_ERR_INVALID_ARG, "null output pointer");
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    hipError_t e = hipStreamSynchronize(s->hs);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    std::vector<double> lat, flat;
    uint64_t t_first = UINT64_MAX, t_last = 0;
    for (auto &f : s->folds) {
        while (!__atomic_load_n(&f.rec->done, __ATOMIC_ACQUIRE)) {
        }
        uint64_t last_arrival = 0;
        for (uint64_t a : f.arrivals) {
            lat.push_back(f.rec->done_ns > a ? (double)(f.rec->done_ns - a) * 1e-6 : 0.0);
            t_first = std::min(t_first, a);
            last_arrival = std::max(last_arrival, a);
        }
        if (!f.arrivals.empty())
            flat.push_back(f.rec->done_ns > last_arrival ? (double)(f.rec->done_ns - last_arrival) * 1e-6 : 0.0);
        t_last = std::max(t_last, f.rec->done_ns);
    }
    const double deadline = 1e3 * s->d.block_period_s * s->d.blocks_per_fold;
    xc_latency_stats r{};
    r.blocks = (int64_t)lat.size();
    r.folds = (int64_t)flat.size();
    r.deadline_ms = deadline;
    r.p50_ms = xc_quantile(lat.data(), (int64_t)lat.size(), 0.50);
    r.p99_ms = xc_quantile(lat.data(), (int64_t)lat.size(), 0.99);
    r.max_ms = lat.empty() ? NAN : *std::max_element(lat.begin(), lat.end());
    r.fold_p50_ms = xc_quantile(flat.data(), (int64_t)flat.size(), 0.50);
    r.fold_p99_ms = xc_quantile(flat.data(), (int64_t)flat.size(), 0.99);
    r.fold_max_ms = flat.empty() ? NAN : *std::max_element(flat.begin(), flat.end());
    for (double v : flat)
        if (deadline > 0 && v > deadline) r.misses++;
    for (double v : lat)
        if (deadline > 0 && v > deadline) r.block_misses++;
    const double span = (t_last > t_first && t_first != UINT64_MAX) ? (double)(t_last - t_first) * 1e-9 : 0.0;
    r.tflops = span > 0 ? s->flops_per_fold * (double)s->folds.size() / span * 1e-12 : 0.0;
    r.integrations = s->published_seq + 1;
    *stats = r;
    return XC_OK;
}

xc_status xc_stream_reset_stats(xc_server *srv, int32_t id) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    hipError_t e = hipStreamSynchronize(s->hs);
    if (e != hipSuccess) return hip_error(e, "hipStreamSynchronize");
    for (auto &f : s->folds) {
        while (!__atomic_load_n(&f.rec->done, __ATOMIC_ACQUIRE)) {
        }
    }
    // ring slots still point at completed records: release them first
    for (auto &b : s->slot_busy) b = nullptr;
    for (auto &f : s->folds) delete f.rec;
    s->folds.clear();
    return XC_OK;
}

xc_status xc_stream_close(xc_server *srv, int32_t id) {
    if (!srv) return set_error(XC_ERR_INVALID_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    Stream *s = get_stream(srv, id);
    if (!s) return set_error(XC_ERR_INVALID_ARG, "no open stream %d", id);
    srv->used -= s->footprint;
    stream_free(*s);
    return XC_OK;
}

}  // extern "C"
