// server_core.h -- admission and scheduling policy of the serving form.
//
// Header-only and free of HIP so that the policy can be exercised on the CPU
// with a fake executor and a fake clock.  The executor runs "sweeps": one
// bounded launch of the batched kernel over a list of (source, request)
// items of one graph.  Continuous batching: a request that arrives while
// others run is admitted as soon as memory and request slots allow, and its
// sources join the next sweep of its graph alongside the sources of earlier
// requests; sweeps of different graphs (and several sweeps of one graph)
// run concurrently.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <vector>

namespace bcserve {

enum class ReqPhase { Waiting, Active, Done, Failed };

struct Request {
    uint64_t ticket = 0;
    int graph = 0;                 // executor-side graph index
    std::vector<int32_t> sources;
    int64_t next_item = 0;         // next source to hand to a sweep
    int64_t done_items = 0;        // sources whose sweeps have finished
    int64_t inflight_items = 0;
    size_t bytes = 0;              // device bytes held while admitted (result buffer)
    double t_arrival = 0, t_admit = 0, t_done = 0;
    ReqPhase phase = ReqPhase::Waiting;
    int status = 0;                // 0 ok, else a bc_status of the failure
    int64_t first_bad = -1;        // index (in this request's source list) of an overflow
    void *out = nullptr;           // executor-owned result buffer
    bool retrieved = false;
};

struct SweepItem {
    int32_t source;
    uint64_t ticket;
    int64_t index_in_request;
};

struct Policy {
    size_t budget_bytes = 0;       // device bytes the requests may hold at once
    int max_active = 64;           // admitted, unfinished requests
    int max_items_per_sweep = 1024;
    bool shortest_first = false;   // within a graph, fewest sources left first (else oldest)
    // Share of the GPU that sweeps in flight may hold together (the executor
    // reports each sweep's share); 0 = no bound.  With a bound, a launched
    // sweep finds free compute units and starts at once instead of queueing
    // behind long-running workgroups of other sweeps.
    double gpu_share = 0.0;
    // Across graphs, serve first the graph whose best request has the least
    // work left (sources left x the executor's per-source cost); else the
    // graph of the oldest request.
    bool least_work_first = false;
    // A request waiting (since arrival) at least this many seconds is served
    // before all younger ones, oldest first, in both orders above; 0 = never.
    // It bounds how long least-work-first can hold a large request back.
    double starve_after = 0.0;
};

// Executor interface:
//   int  free_contexts(int graph)                 sweeps that could start now
//   int  max_items(int graph)                     sources one sweep of the graph can take
//   double sweep_share(int graph)                 share of the GPU one sweep holds
//   double source_cost(int graph)                 relative cost of one source
//   bool alloc_result(Request&)                   device buffer for the result (zeroed)
//   void free_result(Request&)
//   void launch(int graph, const std::vector<SweepItem>&)
//   void poll(std::vector<Finished>&)             sweeps finished since last poll
struct Finished {
    int graph;
    std::vector<SweepItem> items;
    int err_status = 0;              // bc_status of a sweep-wide device error, 0 if none
    std::vector<uint8_t> item_fail;  // per item: 1 if its path counts overflowed
    int item_status = 0;             // bc_status reported for a failed item
};

template <class Exec> class Scheduler {
  public:
    Scheduler(Exec &ex, Policy p) : ex_(ex), pol_(p) {}

    uint64_t submit(int graph, const int32_t *src, int64_t k, size_t result_bytes, double now)
    {
        auto r = std::make_shared<Request>();
        r->ticket = ++last_ticket_;
        r->graph = graph;
        r->sources.assign(src, src + k);
        r->bytes = result_bytes;
        r->t_arrival = now;
        reqs_[r->ticket] = r;
        waiting_.push_back(r->ticket);
        ++submitted_;
        return r->ticket;
    }

    // One scheduling step: collect finished sweeps, admit, dispatch.
    // Returns true if anything changed.
    bool step(double now)
    {
        bool changed = collect(now);
        changed |= admit(now);
        changed |= dispatch(now);
        return changed;
    }

    std::shared_ptr<Request> find(uint64_t t) const
    {
        auto it = reqs_.find(t);
        return it == reqs_.end() ? nullptr : it->second;
    }

    // The caller took ownership of the result (or dropped it): the memory
    // it held is no longer charged to the budget.
    void release(uint64_t t)
    {
        auto r = find(t);
        if (!r)
            return;
        if (r->phase == ReqPhase::Done || r->phase == ReqPhase::Failed) {
            if (!r->retrieved) {
                r->retrieved = true;
                in_use_ -= std::min(in_use_, r->bytes);
            }
            finished_.push_back(*r);
            reqs_.erase(t);
        }
    }

    size_t in_use() const { return in_use_; }
    int active() const { return active_; }
    size_t waiting() const { return waiting_.size(); }
    int64_t submitted() const { return submitted_; }
    const std::vector<Request> &finished_log() const { return finished_; }
    bool idle() const { return waiting_.empty() && active_ == 0 && inflight_sweeps_ == 0; }

    template <class F> void for_each_request(F f) const
    {
        for (auto &kv : reqs_)
            f(*kv.second);
    }

  private:
    bool collect(double now)
    {
        std::vector<Finished> fin;
        ex_.poll(fin);
        for (auto &f : fin) {
            --inflight_sweeps_;
            inflight_share_ -= ex_.sweep_share(f.graph);
            if (inflight_sweeps_ == 0 || inflight_share_ < 0)
                inflight_share_ = 0;
            for (size_t i = 0; i < f.items.size(); ++i) {
                auto r = find(f.items[i].ticket);
                if (!r)
                    continue;
                r->inflight_items -= 1;
                r->done_items += 1;
                const bool failed = i < f.item_fail.size() && f.item_fail[i];
                if (failed && (r->first_bad < 0 ||
                               f.items[i].index_in_request < r->first_bad)) {
                    r->status = f.item_status;
                    r->first_bad = f.items[i].index_in_request;
                }
                if (f.err_status && r->status == 0)
                    r->status = f.err_status;
            }
            for (auto &it : f.items) {
                auto r = find(it.ticket);
                if (r && r->phase == ReqPhase::Active &&
                    r->done_items == (int64_t)r->sources.size())
                    finish(*r, now);
            }
        }
        return !fin.empty();
    }

    void finish(Request &r, double now)
    {
        r.phase = r.status ? ReqPhase::Failed : ReqPhase::Done;
        r.t_done = now;
        --active_;
    }

    bool admit(double now)
    {
        bool changed = false;
        while (!waiting_.empty()) {
            auto r = find(waiting_.front());
            if (!r) {
                waiting_.pop_front();
                continue;
            }
            if (active_ >= pol_.max_active)
                break;
            if (in_use_ + r->bytes > pol_.budget_bytes)
                break; // FIFO: the head waits for memory, later requests wait behind it
            if (!ex_.alloc_result(*r))
                break;
            waiting_.pop_front();
            in_use_ += r->bytes;
            r->phase = ReqPhase::Active;
            r->t_admit = now;
            ++active_;
            order_.push_back(r->ticket);
            changed = true;
            if (r->sources.empty())
                finish(*r, now);
        }
        return changed;
    }

    // true if request r has waited past the starvation bound
    bool overdue(const Request &r, double now) const
    {
        return pol_.starve_after > 0 && now - r.t_arrival >= pol_.starve_after;
    }

    bool dispatch(double now)
    {
        bool changed = false;
        // graphs with pending items, oldest request first
        std::vector<int> graphs;
        for (auto it = order_.begin(); it != order_.end();) {
            auto r = find(*it);
            if (!r || r->phase != ReqPhase::Active ||
                r->next_item == (int64_t)r->sources.size()) {
                it = order_.erase(it);
                continue;
            }
            if (std::find(graphs.begin(), graphs.end(), r->graph) == graphs.end())
                graphs.push_back(r->graph);
            ++it;
        }
        if (pol_.least_work_first) {
            // each graph ranked by its best request's remaining work
            std::map<int, double> least;
            for (uint64_t t : order_) {
                auto r = find(t);
                if (!r)
                    continue;
                const double w = (double)((int64_t)r->sources.size() - r->next_item) *
                                 ex_.source_cost(r->graph);
                auto it2 = least.find(r->graph);
                if (it2 == least.end() || w < it2->second)
                    least[r->graph] = w;
            }
            std::stable_sort(graphs.begin(), graphs.end(),
                             [&](int x, int y) { return least[x] < least[y]; });
        }
        if (pol_.starve_after > 0) {
            // graphs holding an overdue request first, the one overdue longest first
            // (order_ is in admission order, so the first overdue request of a
            // graph is its oldest)
            std::map<int, double> first_arrival;
            for (uint64_t t : order_) {
                auto r = find(t);
                if (r && overdue(*r, now) && !first_arrival.count(r->graph))
                    first_arrival[r->graph] = r->t_arrival;
            }
            std::stable_sort(graphs.begin(), graphs.end(), [&](int x, int y) {
                const bool ox = first_arrival.count(x) > 0, oy = first_arrival.count(y) > 0;
                if (ox != oy)
                    return ox;
                return ox && first_arrival[x] < first_arrival[y];
            });
        }
        for (int gidx : graphs) {
            const int cap = std::min(pol_.max_items_per_sweep, ex_.max_items(gidx));
            // the graph's requests in service order
            std::vector<uint64_t> serve;
            for (uint64_t t : order_) {
                auto r = find(t);
                if (r && r->graph == gidx)
                    serve.push_back(t);
            }
            if (pol_.shortest_first)
                std::stable_sort(serve.begin(), serve.end(), [&](uint64_t x, uint64_t y) {
                    auto rx = find(x), ry = find(y);
                    return (int64_t)rx->sources.size() - rx->next_item <
                           (int64_t)ry->sources.size() - ry->next_item;
                });
            if (pol_.starve_after > 0)
                std::stable_sort(serve.begin(), serve.end(), [&](uint64_t x, uint64_t y) {
                    auto rx = find(x), ry = find(y);
                    const bool ox = overdue(*rx, now), oy = overdue(*ry, now);
                    if (ox != oy)
                        return ox;
                    return ox && rx->t_arrival < ry->t_arrival;
                });
            const double share = ex_.sweep_share(gidx);
            while (ex_.free_contexts(gidx) > 0) {
                if (pol_.gpu_share > 0 && inflight_sweeps_ > 0 &&
                    inflight_share_ + share > pol_.gpu_share + 1e-9)
                    break; // the GPU is full: the graph waits for a sweep to end
                std::vector<SweepItem> items;
                for (uint64_t t : serve) {
                    auto r = find(t);
                    if (!r)
                        continue;
                    while (r->next_item < (int64_t)r->sources.size() &&
                           (int)items.size() < cap) {
                        items.push_back({r->sources[(size_t)r->next_item], r->ticket,
                                         r->next_item});
                        r->next_item += 1;
                        r->inflight_items += 1;
                    }
                    if ((int)items.size() >= cap)
                        break;
                }
                if (items.empty())
                    break;
                ex_.launch(gidx, items);
                ++inflight_sweeps_;
                inflight_share_ += share;
                changed = true;
            }
        }
        return changed;
    }

    Exec &ex_;
    Policy pol_;
    std::map<uint64_t, std::shared_ptr<Request>> reqs_;
    std::deque<uint64_t> waiting_;
    std::deque<uint64_t> order_;
    std::vector<Request> finished_;
    uint64_t last_ticket_ = 0;
    size_t in_use_ = 0;
    int active_ = 0;
    int inflight_sweeps_ = 0;
    double inflight_share_ = 0.0;
    int64_t submitted_ = 0;
};

// Percentile of a sample (nearest rank), 0 for an empty sample.
inline double percentile(std::vector<double> v, double p)
{
    if (v.empty())
        return 0.0;
    std::sort(v.begin(), v.end());
    size_t rank = (size_t)std::max(1.0, std::ceil(p / 100.0 * (double)v.size()));
    return v[std::min(rank, v.size()) - 1];
}

} // namespace bcserve
