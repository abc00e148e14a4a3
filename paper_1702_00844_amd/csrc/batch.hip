// Batches of uneven sub-arrays in one launch per kernel configuration,
// optionally replayed from a hipGraph.  Channels are independent (Section 2),
// so a batch is a flat list of (sub-array, channel, block pair) work units,
// one workgroup each.  The list is cut into one range per XCD, balanced by
// work, with whole channels on one XCD (a channel's block pairs then share its
// L2); within a range the longest units come first.  (An earlier design ran a
// persistent grid that took units from per-XCD counters; a unit's first wait
// for its copied samples then also waited for the previous unit's stores to
// drain, which cost about a fifth of the time.  With one workgroup per unit the
// next workgroup starts while the previous one's stores drain.)
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "common.h"
#include "log.h"

namespace xc {
xc_status resolve(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type, int32_t S, int32_t P, int32_t C,
                  int32_t T, Plan *plan);
Job make_job(const void *samples, void *vis, int S, int C, int T, int block, int accumulate);

// Units of the given items (indices into S, C, T) on blocks of `block`
// stations: whole channels are dealt to the XCD with the least work so far,
// items taken by decreasing integration length; the XCDs' ranges are then
// concatenated (bounds[x] .. bounds[x+1] is XCD x's).  Returns the unit count;
// fills *out and bounds if given.
static int64_t build_units(const std::vector<int> &items, const int32_t *S, const int32_t *C, const int32_t *T,
                           int block, std::vector<Unit> *out, int *bounds) {
    std::vector<int> order(items);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return T[a] > T[b]; });
    int64_t n = 0;
    for (int it : order) {
        const int64_t nb = (S[it] + block - 1) / block;
        n += (int64_t)C[it] * (nb * (nb + 1) / 2);
    }
    if (!out) return n;
    std::vector<Unit> per[kNumXcd];
    double work[kNumXcd] = {};
    for (int it : order) {
        const int nb = (S[it] + block - 1) / block;
        const double cost = (double)T[it] * (nb * (nb + 1) / 2);
        for (int c = 0; c < C[it]; ++c) {
            int x = 0;
            for (int k = 1; k < kNumXcd; ++k)
                if (work[k] < work[x]) x = k;
            work[x] += cost;
            for (int bj = 0; bj < nb; ++bj)
                for (int bi = 0; bi <= bj; ++bi) per[x].push_back(Unit{it, c, bi, bj});
        }
    }
    out->clear();
    out->reserve((size_t)n);
    for (int x = 0; x < kNumXcd; ++x) {
        if (bounds) bounds[x] = (int)out->size();
        out->insert(out->end(), per[x].begin(), per[x].end());
    }
    if (bounds) bounds[kNumXcd] = (int)out->size();
    return n;
}

}  // namespace xc

using namespace xc;

// One launch: the items that resolved to the same configuration.
struct Segment {
    Plan plan;
    bool g4;             // direct-to-LDS kernel with 4-byte granules (station count not a granule multiple)
    int64_t n_units;
    int grid;            // kNumXcd x the longest XCD range
    Unit *d_units;
    int *d_bounds;       // kNumXcd + 1
};

struct xc_batch_plan {
    xc_in_type in_type;
    xc_out_type out_type;
    int n_items;
    int64_t n_units;
    Job *d_jobs;
    std::vector<Segment> segs;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t capture_stream;
};

static void plan_free(xc_batch_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (p->d_jobs) (void)hipFree(p->d_jobs);
    for (Segment &g : p->segs) {
        if (g.d_units) (void)hipFree(g.d_units);
        if (g.d_bounds) (void)hipFree(g.d_bounds);
    }
    delete p;
}

static hipError_t plan_enqueue(xc_batch_plan *p, hipStream_t s) {
    for (const Segment &g : p->segs) {
        hipError_t e;
        if (g.plan.kernel == XC_KERNEL_VALU)
            e = launch_valu_batch(g.plan, p->d_jobs, g.d_units, g.d_bounds, g.grid, s);
        else if (p->in_type == XC_IN_CF32 && g.plan.block == 64)
            e = launch_mfma16_batch(g.plan, p->d_jobs, g.d_units, g.d_bounds, g.grid, s);
        else if (plan_is_dma(g.plan, p->in_type))
            e = launch_mfma_dma_batch(p->in_type, p->out_type, p->d_jobs, g.d_units, g.d_bounds, g.grid, g.g4, s);
        else
            e = launch_mfma_batch(g.plan, p->in_type, p->out_type, p->d_jobs, g.d_units, g.d_bounds, g.grid, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

static bool same_plan(const Plan &a, const Plan &b) {
    return a.kernel == b.kernel && a.block == b.block && a.time_chunk == b.time_chunk &&
           a.time_split == b.time_split && a.staging == b.staging &&
           a.product == b.product && a.tile_w == b.tile_w && a.tile_h == b.tile_h;
}

extern "C" {

int64_t xc_batch_worklist(const int32_t *n_stations, const int32_t *n_channels, const int32_t *n_times,
                          int32_t n_items, int32_t block, int32_t *units, int64_t capacity, int32_t *bounds) {
    if (!n_stations || !n_channels || !n_times || n_items < 0 || block < 1) return -1;
    for (int i = 0; i < n_items; ++i)
        if (n_stations[i] < 1 || n_channels[i] < 1 || n_times[i] < 1) return -1;
    std::vector<int> all(n_items);
    for (int i = 0; i < n_items; ++i) all[i] = i;
    std::vector<Unit> v;
    int b[kNumXcd + 1];
    const int64_t n = build_units(all, n_stations, n_channels, n_times, block, (units || bounds) ? &v : nullptr, b);
    if (bounds)
        for (int x = 0; x <= kNumXcd; ++x) bounds[x] = b[x];
    if (units) {
        const int64_t m = std::min<int64_t>(n, capacity);
        for (int64_t k = 0; k < m; ++k) {
            units[4 * k + 0] = v[k].item;
            units[4 * k + 1] = v[k].channel;
            units[4 * k + 2] = v[k].bi;
            units[4 * k + 3] = v[k].bj;
        }
    }
    return n;
}

xc_status xc_batch_plan_create(const xc_subarray *items, int32_t n_items, int32_t n_pol, xc_in_type in_type,
                               xc_out_type out_type, int32_t accumulate, const xc_config *cfg,
                               const char *tune_cache, int32_t use_graph, void *stream, xc_batch_plan **out) {
    if (!out) return set_error(XC_ERR_INVALID_ARG, "null output plan pointer");
    *out = nullptr;
    if (!items || n_items < 1) return set_error(XC_ERR_INVALID_ARG, "a batch needs at least one item");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    // Without an explicit configuration: with a tuning cache, each item takes
    // the configuration tuned for its shape bucket (buckets the cache lacks are
    // tuned now on their first item, unless the batch accumulates); without
    // one, every item runs one time group per workgroup.  Items whose
    // configurations differ (also the staging of int8 samples, which depends on
    // the station count) get one launch each.
    const xc_config one_group = {XC_KERNEL_AUTO, 0, 0, 1, XC_STAGING_AUTO, XC_PRODUCT_AUTO, 0, 0};
    if (!cfg && !tune_cache) {
        const char *env = getenv("XC_TUNE_CACHE");
        if (env && *env) tune_cache = env;
    }
    if (!cfg && tune_cache) {
        (void)xc_tune_cache_load(tune_cache);      // a missing file is an empty cache
        for (int i = 0; i < n_items; ++i) {
            const xc_subarray &it = items[i];
            if (it.n_stations < 1 || it.n_channels < 1 || it.n_times < 1 || !it.samples || !it.vis) break;
            xc_config tuned;
            if (tune_get(tune_bucket(in_type, out_type, it.n_stations, it.n_channels, it.n_times), &tuned)) continue;
            if (accumulate) continue;              // tuning would overwrite the results being accumulated into
            double ms;
            xc_status st = xc_autotune(it.samples, in_type, it.n_stations, n_pol, it.n_channels, it.n_times, it.vis,
                                       out_type, tune_cache, stream, &tuned, &ms);
            if (st != XC_OK) return st;
        }
    } else if (!cfg) {
        cfg = &one_group;
    }
    std::vector<int32_t> S(n_items), C(n_items), T(n_items);
    std::vector<Plan> plans;                 // distinct configurations, in order of first use
    std::vector<std::vector<int>> members;   // their items
    std::vector<bool> plan_g4;               // their copy granule (direct-to-LDS kernel)
    std::vector<int> item_seg(n_items);
    for (int i = 0; i < n_items; ++i) {
        Plan pi;
        xc_status st = resolve(cfg, in_type, out_type, items[i].n_stations, n_pol, items[i].n_channels,
                               items[i].n_times, &pi);
        if (st != XC_OK) return st;
        if (!items[i].samples || !items[i].vis) return set_error(XC_ERR_INVALID_ARG, "item %d: null pointer", i);
        if (((uintptr_t)items[i].samples & 15u) || ((uintptr_t)items[i].vis & 15u))
            return set_error(XC_ERR_INVALID_ARG, "item %d: pointers must be 16-byte aligned", i);
        // the direct-to-LDS kernel copies 16- or 4-byte granules by station count: one launch each
        const bool g4 = plan_is_dma(pi, in_type) && items[i].n_stations % dma_granule(in_type) != 0;
        size_t g = 0;
        while (g < plans.size() && !(same_plan(plans[g], pi) && plan_g4[g] == g4)) ++g;
        if (g == plans.size()) {
            plans.push_back(pi);
            plan_g4.push_back(g4);
            members.emplace_back();
        }
        members[g].push_back(i);
        item_seg[i] = (int)g;
        S[i] = items[i].n_stations;
        C[i] = items[i].n_channels;
        T[i] = items[i].n_times;
    }
    std::vector<Job> jobs(n_items);
    for (int i = 0; i < n_items; ++i)
        jobs[i] = make_job(items[i].samples, items[i].vis, S[i], C[i], T[i], plans[item_seg[i]].block, accumulate);

    xc_batch_plan *p = new xc_batch_plan{};
    p->in_type = in_type;
    p->out_type = out_type;
    p->n_items = n_items;
    p->n_units = 0;
    hipError_t e = hipMalloc(&p->d_jobs, sizeof(Job) * n_items);
    if (e == hipSuccess) e = hipMemcpy(p->d_jobs, jobs.data(), sizeof(Job) * n_items, hipMemcpyHostToDevice);
    for (size_t g = 0; g < plans.size() && e == hipSuccess; ++g) {
        Segment seg{};
        seg.plan = plans[g];
        seg.g4 = plan_g4[g];
        std::vector<Unit> units;
        int bounds[kNumXcd + 1];
        seg.n_units = build_units(members[g], S.data(), C.data(), T.data(), seg.plan.block, &units, bounds);
        if (seg.n_units > (int64_t)1 << 30) {
            plan_free(p);
            return set_error(XC_ERR_UNSUPPORTED, "too many work units");
        }
        int longest = 1;
        for (int x = 0; x < kNumXcd; ++x) longest = std::max(longest, bounds[x + 1] - bounds[x]);
        seg.grid = kNumXcd * longest;
        p->n_units += seg.n_units;
        e = hipMalloc(&seg.d_units, sizeof(Unit) * (size_t)std::max<int64_t>(seg.n_units, 1));
        if (e == hipSuccess) e = hipMalloc(&seg.d_bounds, sizeof(bounds));
        p->segs.push_back(seg);
        if (e == hipSuccess && seg.n_units > 0)
            e = hipMemcpy(seg.d_units, units.data(), sizeof(Unit) * (size_t)seg.n_units, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(seg.d_bounds, bounds, sizeof(bounds), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        plan_free(p);
        return set_error(XC_ERR_OUT_OF_MEMORY, "batch plan setup failed: %s", hipGetErrorString(e));
    }
    if (use_graph) {
        e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = plan_enqueue(p, p->capture_stream);
            e = hipStreamEndCapture(p->capture_stream, &p->graph);
            if (le != hipSuccess) e = le;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            plan_free(p);
            return hip_error(e, "batch graph capture");
        }
    }
    (void)stream;
    *out = p;
    log_line("batch plan: %d items, %lld work units, %zu launch%s (%s)%s%s", n_items, (long long)p->n_units,
             p->segs.size(), p->segs.size() == 1 ? "" : "es", use_graph ? "graph" : "direct",
             tune_cache && !cfg ? ", tune cache " : "", tune_cache && !cfg ? tune_cache : "");
    return XC_OK;
}

xc_status xc_batch_plan_run(xc_batch_plan *plan, void *stream) {
    if (!plan) return set_error(XC_ERR_INVALID_ARG, "null plan");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = plan->exec ? hipGraphLaunch(plan->exec, s) : plan_enqueue(plan, s);
    if (e != hipSuccess) return hip_error(e, "batch launch");
    return XC_OK;
}

void xc_batch_plan_destroy(xc_batch_plan *plan) { plan_free(plan); }

int64_t xc_batch_plan_units(const xc_batch_plan *plan) { return plan ? plan->n_units : -1; }

}  // extern "C"
