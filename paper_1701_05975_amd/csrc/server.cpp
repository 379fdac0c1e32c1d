// server.cpp -- the serving form: a request loop with continuous batching.
//
// Graphs stay resident (they are bc_graph handles owned by the caller).  A
// scheduler thread owns all device work: per graph it keeps a few sweep
// contexts (state slabs, counters, item buffers, a stream); a sweep is one
// bounded launch of the batched kernel over (source, request) items taken
// from the admitted requests of that graph, oldest first, each source adding
// its dependencies into its own request's result with FP64 atomics.  Requests
// are admitted first-come first-served when the free device memory and the
// server's budget allow their result buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bc.h"
#include "bc_internal.h"
#include "kernels.h"
#include "server_core.h"

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SweepCtx {
    int gidx = 0;
    Workspace ws;
    DevBuf counters;
    DevBuf d_src, d_out, d_err;
    unsigned int *h_err = nullptr;
    int32_t *h_src = nullptr;
    double **h_out = nullptr;
    DevCounters *h_cnt = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    int cap = 0;
    int slots = 0;
    int lds_vertices = 0;
    int lds_bits = 32;
    std::vector<bcserve::SweepItem> items;
    ~SweepCtx()
    {
        if (stream) {
            (void)hipStreamSynchronize(stream);
            (void)hipStreamDestroy(stream);
        }
        if (done)
            (void)hipEventDestroy(done);
        if (h_src)
            (void)hipHostFree(h_src);
        if (h_out)
            (void)hipHostFree(h_out);
        if (h_cnt)
            (void)hipHostFree(h_cnt);
        if (h_err)
            (void)hipHostFree(h_err);
    }
};

struct GraphEntry {
    bc_graph *g = nullptr;
    int64_t m = 0; // edges for throughput accounting
    double share = 0.0; // share of the GPU's resident workgroups one sweep holds
    std::vector<std::unique_ptr<SweepCtx>> ctx;
    int fail_status = 0; // its sweep contexts could not be created: fail the sweep
    std::string fail_msg;
};

class HipExec {
  public:
    HipExec(const bc_server_opts &o, size_t reserve) : opts_(o), reserve_(reserve) {}

    int graph_index(bc_graph *g)
    {
        auto it = index_.find(g);
        if (it != index_.end())
            return it->second;
        GraphEntry e;
        e.g = g;
        e.m = g->directed ? g->nnz : g->nnz / 2;
        graphs_.push_back(std::move(e));
        g->server_refs.fetch_add(1); // bc_destroy_graph refuses it until the server ends
        index_[g] = (int)graphs_.size() - 1;
        return (int)graphs_.size() - 1;
    }

    const GraphEntry &entry(int gidx) const { return graphs_[(size_t)gidx]; }

    int free_contexts(int gidx)
    {
        GraphEntry &e = graphs_[(size_t)gidx];
        if (e.ctx.empty())
            try_create_contexts(e, gidx);
        if (e.fail_status)
            return 1; // one sweep that fails its items (see launch)
        int f = 0;
        for (auto &c : e.ctx)
            f += !c->busy;
        return f;
    }

    bool alloc_result(bcserve::Request &r)
    {
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        if (free_b < r.bytes + reserve_)
            return false; // wait until memory frees up
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(r.bytes, 8)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        hip_check(launch_fill_u64((unsigned long long *)p, r.bytes / 8, 0ull, admin_stream()),
                  "zero result");
        hip_check(hipStreamSynchronize(admin_stream()), "zero result");
        r.out = p;
        return true;
    }

    void free_result(bcserve::Request &r)
    {
        if (r.out)
            (void)hipFree(r.out);
        r.out = nullptr;
    }

    void set_outputs(std::map<uint64_t, double *> *m) { outs_ = m; }

    void launch(int gidx, const std::vector<bcserve::SweepItem> &items)
    {
        GraphEntry &e = graphs_[(size_t)gidx];
        if (e.fail_status) {
            // no context for this graph: its items fail, other graphs go on;
            // the next request of the graph tries to create the contexts again
            bcserve::Finished f;
            f.graph = gidx;
            f.items = items;
            f.err_status = e.fail_status;
            failed_.push_back(std::move(f));
            e.fail_status = 0;
            return;
        }
        SweepCtx *c = nullptr;
        for (auto &x : e.ctx)
            if (!x->busy) {
                c = x.get();
                break;
            }
        if (!c)
            throw bc_error(BC_E_INTERNAL, "no free sweep context");
        const int k = (int)items.size();
        if (k > c->cap)
            throw bc_error(BC_E_INTERNAL, "sweep larger than its buffers");
        for (int i = 0; i < k; ++i) {
            c->h_src[i] = items[(size_t)i].source;
            c->h_out[i] = (*outs_)[items[(size_t)i].ticket];
        }
        hipStream_t st = c->stream;
        hip_check(hipMemcpyAsync(c->d_src.p, c->h_src, (size_t)k * 4, hipMemcpyHostToDevice, st),
                  "items");
        hip_check(hipMemcpyAsync(c->d_out.p, c->h_out, (size_t)k * sizeof(double *),
                                 hipMemcpyHostToDevice, st),
                  "items");
        DevCounters *dc = (DevCounters *)c->counters.p;
        hip_check(launch_fill_u64((unsigned long long *)dc, sizeof(DevCounters) / 8, 0ull, st),
                  "counters");
        hip_check(launch_fill_u64(&dc->err[1], 1, (unsigned long long)INT64_MAX, st), "counters");
        hip_check(launch_fill_u32((uint32_t *)c->d_err.p, (size_t)k, 0u, st), "item flags");
        bc_graph *g = e.g;
        BatchArgs a;
        a.g = g->view();
        a.slab_base = (char *)c->ws.base.p;
        a.L = c->ws.L;
        a.sources = (const int32_t *)c->d_src.p;
        a.k = k;
        a.next_src = &dc->next_src;
        a.bc_out = nullptr;
        a.item_out = (double *const *)c->d_out.p;
        a.item_err = (unsigned int *)c->d_err.p;
        a.iperm = g->iperm_dev();
        a.perm = g->perm_dev();
        a.H = c->lds_vertices;
        a.lds_bits = c->lds_bits;
        set_tier_args(g, tier_for(g, 0), tier_for(g, 1), tier_for(g, 2), a);
        a.kahn = dep_mode_for(g) == 1 ? 1 : 0;
        a.ebc = nullptr;
        a.emap = nullptr;
        a.vw = opts_.compute.virtual_warp;
        a.node_parallel = 0;
        a.delta = (uint32_t)delta_for(g);
        a.lane_max = lane_max_for(g);
        a.stats = &dc->stats;
        a.err = dc->err;
        {
            // far values: the bucket ring or the two-tier pile, as in bc_compute
            ResolvedOptions ro;
            ro.delta = (int)a.delta;
            ro.far_buckets = opts_.compute.far_buckets;
            bucket_plan(g, ro, a.buckets, a.nbk);
            a.bcap = (int32_t)std::min<size_t>(
                (a.L.bx + 8 * (size_t)g->n - a.L.fa) / 4 / (size_t)a.nbk, (size_t)INT32_MAX);
        }
        const int nslabs = std::min(c->slots, k);
        hip_check(launch_batched(a, g->packed, wg_for(g), true, nslabs, st), "sweep");
        hip_check(hipMemcpyAsync(c->h_cnt, dc, sizeof(DevCounters), hipMemcpyDeviceToHost, st),
                  "counters");
        hip_check(hipMemcpyAsync(c->h_err, c->d_err.p, (size_t)k * 4, hipMemcpyDeviceToHost, st),
                  "item flags");
        hip_check(hipEventRecord(c->done, st), "event");
        c->items = items;
        c->busy = true;
        ++sweeps_;
    }

    void poll(std::vector<bcserve::Finished> &fin)
    {
        for (auto &f : failed_)
            fin.push_back(std::move(f));
        failed_.clear();
        for (size_t gi = 0; gi < graphs_.size(); ++gi)
            for (auto &c : graphs_[gi].ctx) {
                if (!c->busy)
                    continue;
                hipError_t q = hipEventQuery(c->done);
                if (q == hipErrorNotReady)
                    continue;
                hip_check(q, "sweep");
                bcserve::Finished f;
                f.graph = (int)gi;
                f.items = std::move(c->items);
                const DevCounters &cnt = *c->h_cnt;
                if (cnt.err[0] & BC_ERRBIT_INTERNAL)
                    f.err_status = BC_E_INTERNAL;
                f.item_status = BC_E_SIGMA_OVERFLOW;
                f.item_fail.assign(f.items.size(), 0);
                if (cnt.err[0] & BC_ERRBIT_SIGMA)
                    for (size_t i = 0; i < f.items.size(); ++i)
                        f.item_fail[i] = c->h_err[i] != 0;
                c->busy = false;
                c->items.clear();
                fin.push_back(std::move(f));
            }
    }

    int64_t sweeps() const { return sweeps_; }

    double sweep_share(int gidx)
    {
        GraphEntry &e = graphs_[(size_t)gidx];
        if (e.ctx.empty())
            try_create_contexts(e, gidx);
        return e.share;
    }

    double source_cost(int gidx)
    {
        const bc_graph *g = graphs_[(size_t)gidx].g;
        return (double)g->n + (double)g->nnz;
    }

    int max_items(int gidx)
    {
        GraphEntry &e = graphs_[(size_t)gidx];
        if (e.ctx.empty())
            try_create_contexts(e, gidx);
        if (e.fail_status)
            return 1 << 30; // every pending item of the graph goes into the failing sweep
        return e.ctx.front()->cap;
    }

    void drain()
    {
        for (auto &e : graphs_)
            for (auto &c : e.ctx)
                if (c->stream)
                    (void)hipStreamSynchronize(c->stream);
    }

    ~HipExec()
    {
        drain();
        for (auto &e : graphs_)
            e.g->server_refs.fetch_sub(1);
        graphs_.clear();
        if (admin_)
            (void)hipStreamDestroy(admin_);
    }

  private:
    hipStream_t admin_stream()
    {
        if (!admin_)
            hip_check(hipStreamCreateWithFlags(&admin_, hipStreamNonBlocking), "stream");
        return admin_;
    }

    int delta_for(bc_graph *g) const
    {
        if (opts_.compute.delta)
            return opts_.compute.delta;
        return g->tuned.valid ? g->tuned.delta : default_delta(g);
    }
    int lane_max_for(bc_graph *g) const
    {
        if (opts_.compute.lane_max_deg)
            return opts_.compute.lane_max_deg;
        return g->tuned.valid ? g->tuned.lane_max : 32;
    }
    // expansion degree tiers: 0 lane, 1 group of lanes, 2 workgroup
    int tier_for(bc_graph *g, int which) const
    {
        const bc_options &o = opts_.compute;
        const int given[3] = {o.expand_lane_deg, o.wave_max_deg, o.wg_min_deg};
        const int tuned[3] = {g->tuned.lane_deg, g->tuned.wave_deg, g->tuned.wg_deg};
        const int def[3] = {BC_DEF_LANE_DEG, BC_DEF_WAVE_DEG, BC_HUB_DEG};
        int t[3];
        for (int i = 0; i < 3; ++i)
            t[i] = given[i] > 0 ? given[i] : (g->tuned.valid && tuned[i] > 0 ? tuned[i] : def[i]);
        t[1] = std::max(t[1], t[0]);
        t[2] = std::max(t[2], t[1]);
        return t[which];
    }
    int dep_mode_for(bc_graph *g) const
    {
        if (opts_.compute.dep_mode)
            return opts_.compute.dep_mode;
        return g->tuned.valid && g->tuned.dep_mode ? g->tuned.dep_mode : 1;
    }
    int wg_for(bc_graph *g) const
    {
        if (opts_.compute.wg_threads)
            return opts_.compute.wg_threads;
        return g->tuned.valid ? g->tuned.wg_threads : 256;
    }

    // Creates the graph's sweep contexts; on failure (not enough device
    // memory, a failed allocation) leaves none and records the status, so
    // that only this graph's requests fail.
    void try_create_contexts(GraphEntry &e, int gidx)
    {
        e.fail_status = 0;
        try {
            create_contexts(e, gidx);
        } catch (const bc_error &err) {
            e.ctx.clear();
            (void)hipGetLastError();
            e.fail_status = err.status;
            e.fail_msg = err.msg;
        }
    }

    void create_contexts(GraphEntry &e, int gidx)
    {
        bc_graph *g = e.g;
        const int nt = wg_for(g);
        int H = 0, per_cu = 1;
        const int bits = lds_bits_for(g, opts_.compute.lds_bits);
        batched_lds_plan(g, nt, true, opts_.compute.lds_vertices, bits, H, per_cu);
        const int fill = g->num_cus * per_cu;
        const SlabLayout L = slab_layout(g->n, g->nnz);
        // A sweep takes a quarter of the GPU by default, so sweeps of other
        // graphs (and of later requests) run beside it instead of behind it.
        int slots = opts_.slots_per_sweep ? opts_.slots_per_sweep : std::max(32, fill / 4);
        const int64_t by_mem = (int64_t)(opts_.slab_bytes_per_sweep / std::max<size_t>(L.stride, 1));
        slots = (int)std::max<int64_t>(1, std::min<int64_t>(slots, by_mem));
        const int nctx = opts_.sweeps_per_graph ? opts_.sweeps_per_graph : 4;
        // at most half of the memory free now goes to this graph's contexts,
        // beyond the reserve, so that other graphs and results still fit
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        const size_t avail = free_b > reserve_ ? (free_b - reserve_) / 2 : 0;
        const int64_t fit = (int64_t)(avail / ((size_t)nctx * std::max<size_t>(L.stride, 1)));
        if (fit < 1)
            throw bc_error(BC_E_NOMEM,
                           "sweep contexts of a graph with n = %d need %zu bytes per source; "
                           "%zu bytes are free",
                           g->n, L.stride, free_b);
        slots = (int)std::min<int64_t>(slots, fit);
        const int cap = opts_.items_per_sweep ? opts_.items_per_sweep : slots;
        e.share = (double)slots / (double)std::max(fill, 1);
        for (int i = 0; i < nctx; ++i) {
            auto c = std::make_unique<SweepCtx>();
            c->gidx = gidx;
            c->slots = slots;
            c->cap = cap;
            c->lds_vertices = H;
            c->lds_bits = bits;
            hip_check(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking), "stream");
            hip_check(hipEventCreateWithFlags(&c->done, hipEventDisableTiming), "event");
            c->ws.L = L;
            c->ws.base.alloc(L.stride * (size_t)slots);
            c->ws.nslabs = slots;
            hip_check(launch_slab_reset((char *)c->ws.base.p, L, slots, g->n, c->stream),
                      "slab reset");
            c->counters.alloc(sizeof(DevCounters));
            c->d_src.alloc((size_t)cap * 4);
            c->d_out.alloc((size_t)cap * sizeof(double *));
            c->d_err.alloc((size_t)cap * 4);
            hip_check(hipHostMalloc((void **)&c->h_err, (size_t)cap * 4), "pinned");
            hip_check(hipHostMalloc((void **)&c->h_src, (size_t)cap * 4), "pinned");
            hip_check(hipHostMalloc((void **)&c->h_out, (size_t)cap * sizeof(double *)), "pinned");
            hip_check(hipHostMalloc((void **)&c->h_cnt, sizeof(DevCounters)), "pinned");
            hip_check(hipStreamSynchronize(c->stream), "context");
            e.ctx.push_back(std::move(c));
        }
    }

    bc_server_opts opts_;
    size_t reserve_ = 0; // device memory always left free
    std::vector<GraphEntry> graphs_;
    std::map<bc_graph *, int> index_;
    std::map<uint64_t, double *> *outs_ = nullptr;
    std::vector<bcserve::Finished> failed_; // sweeps failed without a launch
    hipStream_t admin_ = nullptr;
    int64_t sweeps_ = 0;
};

// Result buffers by ticket, shared between the scheduler (which allocates
// them through the executor) and the sweeps (which need the pointers).
struct OutputTable {
    std::map<uint64_t, double *> map;
};

struct ExecAdapter {
    HipExec *ex;
    OutputTable *outs;
    int free_contexts(int g) { return ex->free_contexts(g); }
    int max_items(int g) { return ex->max_items(g); }
    double sweep_share(int g) { return ex->sweep_share(g); }
    double source_cost(int g) { return ex->source_cost(g); }
    bool alloc_result(bcserve::Request &r)
    {
        if (!ex->alloc_result(r))
            return false;
        outs->map[r.ticket] = (double *)r.out;
        return true;
    }
    void free_result(bcserve::Request &r)
    {
        outs->map.erase(r.ticket);
        ex->free_result(r);
    }
    void launch(int g, const std::vector<bcserve::SweepItem> &items) { ex->launch(g, items); }
    void poll(std::vector<bcserve::Finished> &f) { ex->poll(f); }
};

} // namespace

struct bc_server {
    bc_server_opts opts{};
    int device = 0;
    std::unique_ptr<HipExec> exec;
    OutputTable outs;
    ExecAdapter adapter{};
    std::unique_ptr<bcserve::Scheduler<ExecAdapter>> sched;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    std::atomic<bool> stop{false};
    std::string thread_error;
    int thread_status = 0;
    double t_first_arrival = -1, t_last_done = -1;
    std::map<uint64_t, int64_t> work_of; // ticket -> k * m
    double total_work = 0;

    void loop()
    {
        if (hipSetDevice(device) != hipSuccess) {
            thread_status = BC_E_DEVICE;
            thread_error = "hipSetDevice failed in the server thread";
            return;
        }
        while (!stop.load()) {
            bool changed = false;
            {
                std::unique_lock<std::mutex> lk(mu);
                try {
                    changed = sched->step(now_s());
                } catch (const bc_error &e) {
                    thread_status = e.status;
                    thread_error = e.msg;
                    cv_done.notify_all();
                    return;
                }
                if (changed)
                    cv_done.notify_all();
                if (!changed && sched->idle())
                    cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
            if (!changed)
                std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
};

static bc_status server_fail(bc_status s, const std::string &m);

extern "C" {

bc_status bc_server_create(const bc_server_opts *o, bc_server **out)
{
    try {
        if (!out)
            throw bc_error(BC_E_INVAL, "out is NULL");
        if (o && (o->order < 0 || o->order > 1))
            throw bc_error(BC_E_INVAL, "order must be 0 (oldest first) or 1 (fewest left first)");
        if (o && (o->graph_order < 0 || o->graph_order > 1))
            throw bc_error(BC_E_INVAL,
                           "graph_order must be 0 (oldest request) or 1 (least work left)");
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
            (void)hipGetLastError();
            throw bc_error(BC_E_DEVICE, "no HIP device available");
        }
        std::unique_ptr<bc_server> sv(new bc_server());
        if (o)
            sv->opts = *o;
        hip_check(hipGetDevice(&sv->device), "hipGetDevice");
        size_t free_b = 0, total_b = 0;
        hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        if (sv->opts.result_budget_bytes <= 0)
            sv->opts.result_budget_bytes = (int64_t)(free_b / 4);
        if (sv->opts.slab_bytes_per_sweep <= 0)
            sv->opts.slab_bytes_per_sweep = (int64_t)(free_b / 16);
        if (sv->opts.max_active <= 0)
            sv->opts.max_active = 64;
        sv->exec.reset(new HipExec(sv->opts, (size_t)256 << 20));
        sv->adapter.ex = sv->exec.get();
        sv->adapter.outs = &sv->outs;
        sv->exec->set_outputs(&sv->outs.map);
        bcserve::Policy pol;
        pol.budget_bytes = (size_t)sv->opts.result_budget_bytes;
        pol.max_active = sv->opts.max_active;
        pol.max_items_per_sweep = 1 << 30; // bounded per context by its buffers below
        pol.shortest_first = sv->opts.order == 1;
        pol.least_work_first = sv->opts.graph_order == 1;
        if (sv->opts.starve_after_s < 0)
            throw bc_error(BC_E_INVAL, "starve_after_s must be >= 0");
        pol.starve_after = sv->opts.starve_after_s;
        pol.gpu_share = sv->opts.gpu_share == 0.0 ? 1.0 : sv->opts.gpu_share < 0 ? 0.0
                                                                                 : sv->opts.gpu_share;
        sv->sched.reset(new bcserve::Scheduler<ExecAdapter>(sv->adapter, pol));
        bc_server *raw = sv.get();
        sv->worker = std::thread([raw] { raw->loop(); });
        *out = sv.release();
        return BC_OK;
    } catch (const bc_error &e) {
        return server_fail(e.status, e.msg);
    } catch (...) {
        return server_fail(BC_E_INTERNAL, "server creation failed");
    }
}

bc_status bc_server_submit(bc_server *sv, bc_graph *g, const int32_t *sources, int64_t k,
                           uint64_t *ticket)
{
    try {
        if (!sv || !g || !ticket || k < 0 || (k > 0 && !sources))
            throw bc_error(BC_E_INVAL, "bad argument");
        for (int64_t i = 0; i < k; ++i)
            if (sources[i] < 0 || sources[i] >= g->n)
                throw bc_error(BC_E_INVAL, "sources[%lld] = %d out of range", (long long)i,
                               sources[i]);
        const size_t bytes = (size_t)g->n * sizeof(double);
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->thread_status)
            throw bc_error((bc_status)sv->thread_status, "%s", sv->thread_error.c_str());
        if ((int64_t)bytes > sv->opts.result_budget_bytes)
            throw bc_error(BC_E_BUSY, "a result of %zu bytes exceeds the server budget", bytes);
        const int gidx = sv->exec->graph_index(g);
        // cap sweep size by the context buffers: split the request's items
        const double t = now_s();
        const uint64_t tk = sv->sched->submit(gidx, sources, k, bytes, t);
        if (sv->t_first_arrival < 0)
            sv->t_first_arrival = t;
        sv->work_of[tk] = k * sv->exec->entry(gidx).m;
        *ticket = tk;
        sv->cv_work.notify_all();
        return BC_OK;
    } catch (const bc_error &e) {
        return server_fail(e.status, e.msg);
    }
}

bc_status bc_server_wait(bc_server *sv, uint64_t ticket, int64_t timeout_us, bc_result **out)
{
    try {
        if (!sv || !out)
            throw bc_error(BC_E_INVAL, "bad argument");
        std::unique_lock<std::mutex> lk(sv->mu);
        auto pred = [&] {
            if (sv->thread_status)
                return true;
            auto r = sv->sched->find(ticket);
            return !r || r->phase == bcserve::ReqPhase::Done ||
                   r->phase == bcserve::ReqPhase::Failed;
        };
        if (timeout_us < 0)
            sv->cv_done.wait(lk, pred);
        else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
            throw bc_error(BC_E_TIMEOUT, "request %llu not finished", (unsigned long long)ticket);
        if (sv->thread_status)
            throw bc_error((bc_status)sv->thread_status, "%s", sv->thread_error.c_str());
        auto r = sv->sched->find(ticket);
        if (!r)
            throw bc_error(BC_E_INVAL, "unknown or already retrieved ticket %llu",
                           (unsigned long long)ticket);
        sv->t_last_done = std::max(sv->t_last_done, r->t_done);
        sv->total_work += (double)sv->work_of[ticket];
        sv->work_of.erase(ticket);
        if (r->phase == bcserve::ReqPhase::Failed) {
            const int st = r->status;
            const long long bad = (long long)r->first_bad;
            sv->adapter.free_result(*r);
            sv->sched->release(ticket);
            if (st == BC_E_SIGMA_OVERFLOW)
                throw bc_error(BC_E_SIGMA_OVERFLOW,
                               "shortest-path count exceeded 2^64-1 (first source-list index %lld)",
                               bad);
            throw bc_error((bc_status)st, "request failed");
        }
        std::unique_ptr<bc_result> res(new bc_result());
        res->n = (int32_t)(r->bytes / sizeof(double));
        res->bc.p = r->out;
        res->bc.bytes = r->bytes;
        res->stats.sources = (int64_t)r->sources.size();
        res->stats.ms = (r->t_done - r->t_arrival) * 1e3;
        res->stats.first_bad_source = -1;
        res->stats.mode = BC_MODE_BATCHED;
        sv->outs.map.erase(ticket);
        r->out = nullptr;
        sv->sched->release(ticket);
        *out = res.release();
        return BC_OK;
    } catch (const bc_error &e) {
        return server_fail(e.status, e.msg);
    }
}

bc_status bc_server_get_stats(bc_server *sv, bc_server_stats *st)
{
    try {
        if (!sv || !st)
            throw bc_error(BC_E_INVAL, "bad argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        bc_server_stats s;
        memset(&s, 0, sizeof s);
        std::vector<double> lat;
        for (const auto &r : sv->sched->finished_log()) {
            if (r.phase == bcserve::ReqPhase::Done) {
                lat.push_back((r.t_done - r.t_arrival) * 1e3);
                ++s.completed;
            } else {
                ++s.failed;
            }
            s.queue_ms_sum += (r.t_admit - r.t_arrival) * 1e3;
        }
        s.submitted = sv->sched->submitted();
        s.waiting = (int64_t)sv->sched->waiting();
        s.active = sv->sched->active();
        s.p50_ms = bcserve::percentile(lat, 50);
        s.p99_ms = bcserve::percentile(lat, 99);
        s.max_ms = lat.empty() ? 0 : *std::max_element(lat.begin(), lat.end());
        double sum = 0;
        for (double x : lat)
            sum += x;
        s.mean_ms = lat.empty() ? 0 : sum / (double)lat.size();
        const double span = sv->t_last_done - sv->t_first_arrival;
        s.gteps = span > 0 ? sv->total_work / span / 1e9 : 0.0;
        s.sweeps = sv->exec->sweeps();
        s.device_bytes_in_use = (int64_t)sv->sched->in_use();
        *st = s;
        return BC_OK;
    } catch (const bc_error &e) {
        return server_fail(e.status, e.msg);
    }
}

bc_status bc_server_destroy(bc_server *sv)
{
    if (!sv)
        return BC_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop.store(true);
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable())
        sv->worker.join();
    sv->exec->drain();
    // free results nobody retrieved
    for (auto &kv : sv->outs.map)
        (void)hipFree(kv.second);
    sv->outs.map.clear();
    delete sv;
    return BC_OK;
}

} // extern "C"

static bc_status server_fail(bc_status s, const std::string &m)
{
    bc_set_last_error(m);
    return s;
}
