// Batches of uneven sub-arrays in one persistent launch, optionally replayed
// from a hipGraph.  Channels are independent (Section 2), so a batch is a flat
// list of (sub-array, channel, block pair) work units that a fixed grid of
// workgroups drains through an atomic counter.
#include <algorithm>
#include <vector>

#include "common.h"

namespace xc {
xc_status resolve(const xc_config *cfg, xc_in_type in_type, xc_out_type out_type, int32_t S, int32_t P, int32_t C,
                  int32_t T, Plan *plan);
Job make_job(const void *samples, void *vis, int S, int C, int T, int block, int accumulate);

__global__ void reset_counters_kernel(int *counters) {
    if (threadIdx.x < kNumXcd) counters[threadIdx.x] = 0;
}

hipError_t launch_reset_counters(int *counters, hipStream_t stream) {
    hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, stream, counters);
    return hipGetLastError();
}

// Work-list order: sub-arrays by decreasing integration length (longest
// units first), then channel, then block pair, so that the block pairs of one
// channel are taken by workgroups at about the same time and share its
// samples in the caches.
static int64_t build_units(const int32_t *S, const int32_t *C, const int32_t *T, int n_items, int block,
                           std::vector<Unit> *out) {
    std::vector<int> order(n_items);
    for (int i = 0; i < n_items; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return T[a] > T[b]; });
    int64_t n = 0;
    for (int it : order) {
        const int64_t nb = (S[it] + block - 1) / block;
        n += (int64_t)C[it] * (nb * (nb + 1) / 2);
    }
    if (out) {
        out->clear();
        out->reserve((size_t)n);
        for (int it : order) {
            const int nb = (S[it] + block - 1) / block;
            for (int c = 0; c < C[it]; ++c)
                for (int bj = 0; bj < nb; ++bj)
                    for (int bi = 0; bi <= bj; ++bi) out->push_back(Unit{it, c, bi, bj});
        }
    }
    return n;
}

}  // namespace xc

using namespace xc;

struct xc_batch_plan {
    Plan plan;
    xc_in_type in_type;
    xc_out_type out_type;
    int n_items;
    int64_t n_units;
    int grid;
    Job *d_jobs;
    Unit *d_units;
    int *d_queue;        // kNumXcd + 1 segment bounds, then kNumXcd counters
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
    if (p->d_units) (void)hipFree(p->d_units);
    if (p->d_queue) (void)hipFree(p->d_queue);
    delete p;
}

static hipError_t plan_enqueue(xc_batch_plan *p, hipStream_t s) {
    Queues q{p->d_queue, p->d_queue + kNumXcd + 1};
    hipError_t e = launch_reset_counters(q.counters, s);
    if (e != hipSuccess) return e;
    if (p->plan.kernel == XC_KERNEL_VALU) return launch_valu_batch(p->plan, p->d_jobs, p->d_units, q, p->grid, s);
    if (p->in_type == XC_IN_CF32 && p->plan.block == 64)
        return launch_mfma16_batch(p->plan, p->d_jobs, p->d_units, q, p->grid, s);
    if (plan_is_dma(p->plan, p->in_type))
        return launch_mfma_dma_batch(p->in_type, p->out_type, p->d_jobs, p->d_units, q, p->grid, s);
    return launch_mfma_batch(p->plan, p->in_type, p->out_type, p->d_jobs, p->d_units, q, p->grid, s);
}

extern "C" {

int64_t xc_batch_worklist(const int32_t *n_stations, const int32_t *n_channels, const int32_t *n_times,
                          int32_t n_items, int32_t block, int32_t *units, int64_t capacity) {
    if (!n_stations || !n_channels || !n_times || n_items < 0 || block < 1) return -1;
    for (int i = 0; i < n_items; ++i)
        if (n_stations[i] < 1 || n_channels[i] < 1 || n_times[i] < 1) return -1;
    std::vector<Unit> v;
    const int64_t n = build_units(n_stations, n_channels, n_times, n_items, block, units ? &v : nullptr);
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
                               xc_out_type out_type, int32_t accumulate, const xc_config *cfg, int32_t use_graph,
                               void *stream, xc_batch_plan **out) {
    if (!out) return set_error(XC_ERR_INVALID_ARG, "null output plan pointer");
    *out = nullptr;
    if (!items || n_items < 1) return set_error(XC_ERR_INVALID_ARG, "a batch needs at least one item");
    if (accumulate != 0 && accumulate != 1) return set_error(XC_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    Plan plan{};
    // Without an explicit configuration every item runs one time group per
    // workgroup, so that all items share one persistent kernel.
    const xc_config one_group = {XC_KERNEL_AUTO, 0, 0, 1, XC_STAGING_AUTO};
    if (!cfg) cfg = &one_group;
    std::vector<int32_t> S(n_items), C(n_items), T(n_items);
    for (int i = 0; i < n_items; ++i) {
        Plan pi;
        xc_status st = resolve(cfg, in_type, out_type, items[i].n_stations, n_pol, items[i].n_channels,
                               items[i].n_times, &pi);
        if (st != XC_OK) return st;
        if (!items[i].samples || !items[i].vis) return set_error(XC_ERR_INVALID_ARG, "item %d: null pointer", i);
        if (((uintptr_t)items[i].samples & 15u) || ((uintptr_t)items[i].vis & 15u))
            return set_error(XC_ERR_INVALID_ARG, "item %d: pointers must be 16-byte aligned", i);
        if (i == 0) plan = pi;
        // one persistent kernel serves every item: without an explicit
        // time_chunk, an item that the direct-to-LDS kernel cannot take moves
        // the whole batch to the register-staged one
        if (pi.staging != plan.staging && plan_is_dma(plan, in_type) && cfg->staging == XC_STAGING_AUTO)
            plan.staging = pi.staging;
        S[i] = items[i].n_stations;
        C[i] = items[i].n_channels;
        T[i] = items[i].n_times;
    }
    std::vector<Unit> units;
    const int64_t n_units = build_units(S.data(), C.data(), T.data(), n_items, plan.block, &units);
    if (n_units > (int64_t)1 << 30) return set_error(XC_ERR_UNSUPPORTED, "too many work units");
    std::vector<Job> jobs(n_items);
    for (int i = 0; i < n_items; ++i)
        jobs[i] = make_job(items[i].samples, items[i].vis, S[i], C[i], T[i], plan.block, accumulate);

    xc_batch_plan *p = new xc_batch_plan{};
    p->plan = plan;
    p->in_type = in_type;
    p->out_type = out_type;
    p->n_items = n_items;
    p->n_units = n_units;
    hipError_t e = hipMalloc(&p->d_jobs, sizeof(Job) * n_items);
    if (e == hipSuccess) e = hipMalloc(&p->d_units, sizeof(Unit) * (size_t)n_units);
    if (e == hipSuccess) e = hipMalloc(&p->d_queue, sizeof(int) * (2 * kNumXcd + 1));
    if (e != hipSuccess) {
        plan_free(p);
        return set_error(XC_ERR_OUT_OF_MEMORY, "batch plan allocation failed: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->d_jobs, jobs.data(), sizeof(Job) * n_items, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_units, units.data(), sizeof(Unit) * (size_t)n_units, hipMemcpyHostToDevice);
    // one contiguous segment of the list per XCD, cut at channel boundaries
    // where possible so that a channel's block pairs stay on one XCD
    int bounds[kNumXcd + 1];
    bounds[0] = 0;
    for (int x = 1; x < kNumXcd; ++x) {
        int64_t b = n_units * x / kNumXcd;
        while (b > bounds[x - 1] && b < n_units &&
               (units[b].item == units[b - 1].item && units[b].channel == units[b - 1].channel))
            --b;
        bounds[x] = (int)b;
    }
    bounds[kNumXcd] = (int)n_units;
    if (e == hipSuccess) e = hipMemcpy(p->d_queue, bounds, sizeof(bounds), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        plan_free(p);
        return hip_error(e, "batch plan upload");
    }
    // persistent grid: every CU filled to the kernel's occupancy
    const int cus = device_cu_count();
    const int per_cu = plan.kernel == XC_KERNEL_VALU                    ? occupancy_valu_batch(plan)
                       : (in_type == XC_IN_CF32 && plan.block == 64) ? occupancy_mfma16_batch(plan)
                       : plan_is_dma(plan, in_type)                  ? occupancy_mfma_dma_batch(in_type, out_type)
                                                                     : occupancy_mfma_batch(plan, in_type, out_type);
    p->grid = (int)std::min<int64_t>((int64_t)cus * per_cu, n_units);
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
