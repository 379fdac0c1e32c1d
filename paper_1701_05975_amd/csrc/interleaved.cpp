// interleaved.cpp -- host driver of the source-interleaved form: sources in
// groups of 64 (one wave lane each), as many groups per sweep as the device
// memory budget allows, every pass a sequence of queue rounds whose lengths
// the host reads between launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "bc_internal.h"

namespace {

// Bytes per (group, vertex) entry: rows of distances (4), counts (8),
// dependencies (8) and pending counts (4) for 64 lanes, the lane masks and
// stamp, the two queues and two far lists, the taken mask and a work item.
constexpr size_t IL_ENTRY_BYTES = 64 * (4 + 8 + 8 + 4) + 8 + 8 + 4 + 4 * 4 + 8 + 8;

// Work items of one round beyond one per entry: a queue holds each entry at
// most once, and a vertex of degree D gives ceil(D / IL_CHUNK) items.
static size_t extra_items_per_group(int64_t nnz) { return (size_t)nnz / IL_CHUNK + 1; }
constexpr size_t IL_BUDGET_CAP = 160ull << 30;

template <class T> T *carve(char *&p, size_t count)
{
    T *r = reinterpret_cast<T *>(p);
    p += (count * sizeof(T) + 255) & ~(size_t)255;
    return r;
}

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EventPair()
    {
        hip_check(hipEventCreate(&e0), "event");
        hip_check(hipEventCreate(&e1), "event");
    }
    ~EventPair()
    {
        if (e0)
            (void)hipEventDestroy(e0);
        if (e1)
            (void)hipEventDestroy(e1);
    }
};

struct Staging {
    IlCtl *host = nullptr; // pinned: [0] read back, [1] written to the device
    Staging() { hip_check(hipHostMalloc((void **)&host, 2 * sizeof(IlCtl)), "hipHostMalloc"); }
    ~Staging() { (void)hipHostFree(host); }
};

} // namespace

int interleaved_groups_per_sweep(int32_t n, int64_t nnz, int64_t k, size_t free_bytes)
{
    const int64_t total = (k + 63) / 64;
    const size_t budget = std::min(free_bytes / 10 * 6, IL_BUDGET_CAP);
    const size_t per_group = (size_t)n * IL_ENTRY_BYTES + extra_items_per_group(nnz) * 8;
    int64_t gs = (int64_t)(budget / per_group);
    gs = std::min<int64_t>(gs, total);
    gs = std::min<int64_t>(gs, (int64_t)(INT32_MAX / 2) / std::max<int32_t>(n, 1));
    // one round's work items are counted in 32 bits
    gs = std::min<int64_t>(gs, (int64_t)INT32_MAX /
                                   ((int64_t)n + (int64_t)extra_items_per_group(nnz)));
    return (int)std::max<int64_t>(gs, 0);
}

void run_interleaved(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev, int64_t k,
                     double *bc_dev, DevCounters &cnt, float &ms)
{
    hipStream_t st = r.stream;
    const int32_t n = g->n;
    reset_device_counters(g, st);
    hip_check(launch_fill_u64((unsigned long long *)bc_dev, (size_t)n, 0ull, st), "zero");
    EventPair ev;
    hip_check(hipEventRecord(ev.e0, st), "event");
    uint64_t rounds = 0, bands = 0, reached = 0;
    if (k > 0) {
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        int gs = interleaved_groups_per_sweep(n, g->nnz, k, free_b);
        if (r.il_groups > 0 && gs > 0)
            gs = std::min(gs, r.il_groups);
        if (gs < 1)
            throw bc_error(BC_E_NOMEM, "one group of 64 sources needs %zu bytes, %zu free",
                           (size_t)n * IL_ENTRY_BYTES, free_b);
        const size_t entries = (size_t)gs * (size_t)n;
        const size_t cells = entries * 64;
        const size_t items = entries + (size_t)gs * extra_items_per_group(g->nnz);
        const size_t need = cells * (4 + 8 + 8 + 4) + entries * (8 + 8 + 4 + 16 + 8) +
                            items * 8 + (size_t)gs * 64 * 4 + 20 * 256 + sizeof(IlCtl);
        DevBuf buf;
        buf.alloc(need);
        char *p = (char *)buf.p;
        IlArgs a;
        a.g = g->view();
        a.n = n;
        a.d = carve<uint32_t>(p, cells);
        a.sigma = carve<unsigned long long>(p, cells);
        a.delta = carve<double>(p, cells);
        a.cnt = carve<int32_t>(p, cells);
        a.act = carve<unsigned long long>(p, entries);
        a.far = carve<unsigned long long>(p, entries);
        a.stamp = carve<uint32_t>(p, entries);
        uint32_t *qa = carve<uint32_t>(p, entries), *qb = carve<uint32_t>(p, entries);
        uint32_t *fa = carve<uint32_t>(p, entries), *fb = carve<uint32_t>(p, entries);
        a.lane_src = carve<int32_t>(p, (size_t)gs * 64);
        a.qm = carve<unsigned long long>(p, entries);
        a.items = carve<unsigned long long>(p, items);
        a.ctl = carve<IlCtl>(p, 1);
        DevCounters *dc = (DevCounters *)g->ctl.p;
        a.err = dc->err;
        Staging stg;
        IlCtl *rd = &stg.host[0], *wr = &stg.host[1];
        const uint32_t delta = (uint32_t)std::max(r.delta, 1);
        // every band settles at least one (vertex, source) pair or jumps to one
        // that it then settles, and a relax round without progress ends the band
        const uint64_t bound = 16ull * (uint64_t)cells + 1024;
        auto set_ctl = [&](uint32_t flen, uint32_t minkept) {
            memset(wr, 0, sizeof(IlCtl));
            wr->flen = flen;
            wr->minkept = minkept;
            hip_check(hipMemcpyAsync(a.ctl, wr, sizeof(IlCtl), hipMemcpyHostToDevice, st),
                      "ctl");
        };
        auto get_ctl = [&]() {
            hip_check(hipMemcpyAsync(rd, a.ctl, sizeof(IlCtl), hipMemcpyDeviceToHost, st),
                      "ctl");
            hip_check(hipStreamSynchronize(st), "synchronize");
        };
        const int64_t total_groups = (k + 63) / 64;
        for (int64_t g0 = 0; g0 < total_groups; g0 += gs) {
            a.groups = (int)std::min<int64_t>(gs, total_groups - g0);
            a.src_base = g0 * 64;
            const int64_t ks = std::min<int64_t>((int64_t)a.groups * 64, k - g0 * 64);
            uint32_t round = 1;
            set_ctl(0, BC_INF);
            hip_check(launch_il_init(a, src_dev + g0 * 64, ks, g->iperm_dev(), qa, round, st),
                      "interleaved init");
            get_ctl();
            uint32_t *q = qa, *qn = qb, *f = fa, *fn = fb;
            uint32_t qlen = rd->qlen, flen = 0;
            uint64_t thr = delta, steps = 0;
            // forward: near-far bands shared by the group's sources
            for (;;) {
                while (qlen > 0) {
                    if (++steps > bound)
                        throw bc_error(BC_E_INTERNAL, "interleaved forward pass did not end");
                    set_ctl(flen, BC_INF);
                    hip_check(launch_il_relax(a, g->packed, q, qlen, qn, f, (uint32_t)thr,
                                              ++round, st),
                              "interleaved relax");
                    get_ctl();
                    qlen = rd->qlen;
                    flen = rd->flen;
                    std::swap(q, qn);
                }
                if (flen == 0)
                    break;
                uint64_t thr_old = thr, thr_new = std::min<uint64_t>(thr + delta, BC_INF);
                for (;;) {
                    if (++steps > bound)
                        throw bc_error(BC_E_INTERNAL, "interleaved far pile did not drain");
                    set_ctl(0, BC_INF);
                    hip_check(launch_il_far(a, f, flen, q, fn, (uint32_t)thr_old,
                                            (uint32_t)thr_new, ++round, st),
                              "interleaved far pass");
                    get_ctl();
                    qlen = rd->qlen;
                    flen = rd->flen;
                    std::swap(f, fn);
                    thr = thr_new;
                    ++bands;
                    if (qlen > 0 || flen == 0)
                        break;
                    // nothing moved: go straight to the band of the least kept distance
                    thr_old = thr_new;
                    thr_new = std::min<uint64_t>(((uint64_t)rd->minkept / delta + 1) * delta,
                                                 BC_INF);
                }
            }
            // counts, then dependencies, each in Kahn's order over the DAGs
            for (int phase = 0; phase < 2; ++phase) {
                set_ctl(0, BC_INF);
                hip_check(launch_il_count(a, g->packed, phase == 0, q, ++round, st),
                          "interleaved count");
                get_ctl();
                if (phase == 0)
                    reached += rd->reached;
                qlen = rd->qlen;
                uint64_t guard = 0;
                while (qlen > 0) {
                    if (++guard > (uint64_t)n + 2)
                        throw bc_error(BC_E_INTERNAL, "interleaved DAG rounds did not end");
                    set_ctl(0, BC_INF);
                    hip_check(launch_il_round(a, g->packed, phase == 1, q, qlen, qn, ++round, st),
                              "interleaved round");
                    get_ctl();
                    qlen = rd->qlen;
                    std::swap(q, qn);
                    ++steps;
                }
            }
            hip_check(launch_il_bc(a, bc_dev, g->perm_dev(), st), "interleaved accumulation");
            rounds += steps;
        }
    }
    hip_check(hipEventRecord(ev.e1, st), "event");
    read_device_counters(g, st, cnt);
    hip_check(hipEventElapsedTime(&ms, ev.e0, ev.e1), "event time");
    cnt.stats.reached = reached;
    cnt.stats.iterations = rounds;
    cnt.stats.bands = bands;
}
