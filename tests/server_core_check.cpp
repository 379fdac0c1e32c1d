// CPU check of the serving scheduler policy (no HIP): a fake executor whose
// sweeps finish when the test says so, and a fake clock.
#include <cassert>
#include <cstdio>
#include <cstring>
#include <map>
#include <vector>

#include "../paper_1701_05975_amd/csrc/server_core.h"

using namespace bcserve;

struct FakeExec {
    std::map<int, int> ctx_per_graph;     // contexts per graph
    std::map<int, int> busy;              // busy contexts per graph
    int cap = 8;                          // items per sweep
    std::vector<std::pair<int, std::vector<SweepItem>>> running;
    std::vector<Finished> ready;          // sweeps the test has finished
    int allocs = 0, alloc_fail_after = 1 << 30;
    std::map<int, double> share, cost;   // per graph: GPU share of a sweep, cost of a source
    int free_contexts(int g) { return ctx_per_graph.count(g) ? ctx_per_graph[g] - busy[g] : 2 - busy[g]; }
    int max_items(int) { return cap; }
    double sweep_share(int g) { return share.count(g) ? share[g] : 0.0; }
    double source_cost(int g) { return cost.count(g) ? cost[g] : 1.0; }
    bool alloc_result(Request &r) {
        if (allocs >= alloc_fail_after) return false;
        ++allocs;
        r.out = (void *)0x1;
        return true;
    }
    void free_result(Request &r) { r.out = nullptr; }
    void launch(int g, const std::vector<SweepItem> &items) {
        busy[g] += 1;
        running.push_back({g, items});
    }
    void poll(std::vector<Finished> &out) { for (auto &f : ready) out.push_back(f); ready.clear(); }
    // finish the oldest running sweep; optionally mark one item (index) failed
    void finish_oldest(int fail_index = -1, int err_status = 0) {
        auto s = running.front();
        running.erase(running.begin());
        busy[s.first] -= 1;
        Finished f;
        f.graph = s.first;
        f.items = s.second;
        f.err_status = err_status;
        f.item_status = 5;
        f.item_fail.assign(f.items.size(), 0);
        if (fail_index >= 0) f.item_fail[(size_t)fail_index] = 1;
        ready.push_back(f);
    }
};

static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); ++fails; } } while (0)

int main() {
    std::vector<int32_t> s10(10), s3 = {1, 2, 3};
    for (int i = 0; i < 10; ++i) s10[(size_t)i] = i;
    // 1. FIFO admission under a memory budget of two results
    {
        FakeExec ex;
        Policy p; p.budget_bytes = 200; p.max_active = 10; p.max_items_per_sweep = 1 << 20;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t a = sc.submit(0, s3.data(), 3, 100, 0.0);
        uint64_t b = sc.submit(0, s3.data(), 3, 100, 0.1);
        uint64_t c = sc.submit(1, s3.data(), 3, 100, 0.2);
        sc.step(1.0);
        CHECK(sc.active() == 2 && sc.waiting() == 1);
        CHECK(sc.find(c)->phase == ReqPhase::Waiting);
        // continuous batching: a and b share the first sweep of graph 0
        CHECK(ex.running.size() == 1 && ex.running[0].second.size() == 6);
        ex.finish_oldest();
        sc.step(2.0);
        CHECK(sc.find(a)->phase == ReqPhase::Done && sc.find(b)->phase == ReqPhase::Done);
        CHECK(sc.find(a)->t_done == 2.0 && sc.find(a)->t_arrival == 0.0);
        // memory stays charged until the results are retrieved
        CHECK(sc.find(c)->phase == ReqPhase::Waiting);
        sc.release(a);
        sc.step(3.0);
        CHECK(sc.find(c)->phase == ReqPhase::Active);
        CHECK(sc.find(c)->t_admit == 3.0);
    }
    // 1b. shortest first: a later, shorter request of the same graph is served first
    {
        FakeExec ex; ex.cap = 4; ex.ctx_per_graph[0] = 1;
        Policy p; p.budget_bytes = 1 << 20; p.max_active = 10; p.shortest_first = true;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t a = sc.submit(0, s10.data(), 10, 8, 0.0);
        uint64_t b = sc.submit(0, s3.data(), 3, 8, 0.0);
        sc.step(0.5);
        CHECK(ex.running.size() == 1);
        auto &first = ex.running[0].second;
        CHECK(first.size() == 4 && first[0].ticket == b && first[2].ticket == b &&
              first[3].ticket == a);                    // b's 3 sources, then a's first
        while (!ex.running.empty()) { ex.finish_oldest(); sc.step(1.0); }
        CHECK(sc.find(b)->phase == ReqPhase::Done && sc.find(a)->phase == ReqPhase::Done);
        CHECK(sc.find(b)->t_done <= sc.find(a)->t_done);
    }
    // 2. a request larger than one sweep is split; sweeps per graph bounded; order kept
    {
        FakeExec ex; ex.cap = 4; ex.ctx_per_graph[0] = 2;
        Policy p; p.budget_bytes = 1 << 20; p.max_active = 10;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t a = sc.submit(0, s10.data(), 10, 8, 0.0);
        uint64_t b = sc.submit(0, s3.data(), 3, 8, 0.0);
        sc.step(0.5);
        CHECK(ex.running.size() == 2);                 // two contexts, both busy
        CHECK(ex.running[0].second[0].ticket == a);    // oldest request first
        CHECK(ex.running[1].second.size() == 4);
        ex.finish_oldest();
        sc.step(1.0);
        CHECK(ex.running.size() == 2);
        // third sweep: a's last 2 items then b's 2 first items
        auto &third = ex.running.back().second;
        CHECK(third.size() == 4 && third[0].ticket == a && third[2].ticket == b);
        while (!ex.running.empty()) { ex.finish_oldest(); sc.step(2.0); }
        sc.step(2.5);
        CHECK(sc.find(a)->phase == ReqPhase::Done && sc.find(b)->phase == ReqPhase::Done);
        CHECK(sc.idle());
    }
    // 3. failure isolation: one failing source fails only its own request
    {
        FakeExec ex;
        Policy p; p.budget_bytes = 1 << 20;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t a = sc.submit(0, s3.data(), 3, 8, 0.0);
        uint64_t b = sc.submit(0, s3.data(), 3, 8, 0.0);
        sc.step(0.1);
        ex.finish_oldest(4);                            // item 4 = b's second source
        sc.step(0.2);
        CHECK(sc.find(a)->phase == ReqPhase::Done);
        CHECK(sc.find(b)->phase == ReqPhase::Failed && sc.find(b)->first_bad == 1);
        CHECK(sc.find(b)->status == 5);
    }
    // 4. empty request completes at admission; max_active respected
    {
        FakeExec ex;
        Policy p; p.budget_bytes = 1 << 20; p.max_active = 1;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t e = sc.submit(0, nullptr, 0, 8, 0.0);
        uint64_t a = sc.submit(0, s3.data(), 3, 8, 0.0);
        uint64_t b = sc.submit(0, s3.data(), 3, 8, 0.0);
        sc.step(1.0);
        CHECK(sc.find(e)->phase == ReqPhase::Done && sc.find(e)->t_done == 1.0);
        CHECK(sc.find(a)->phase == ReqPhase::Active && sc.find(b)->phase == ReqPhase::Waiting);
        ex.finish_oldest();
        sc.step(2.0);
        CHECK(sc.find(a)->phase == ReqPhase::Done && sc.find(b)->phase == ReqPhase::Active);
    }
    // 5. admission waits while the device has no memory for the result
    {
        FakeExec ex; ex.alloc_fail_after = 1;
        Policy p; p.budget_bytes = 1 << 20;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t a = sc.submit(0, s3.data(), 3, 8, 0.0);
        uint64_t b = sc.submit(0, s3.data(), 3, 8, 0.0);
        sc.step(1.0);
        CHECK(sc.find(a)->phase == ReqPhase::Active && sc.find(b)->phase == ReqPhase::Waiting);
        ex.alloc_fail_after = 2;
        sc.step(2.0);
        CHECK(sc.find(b)->phase == ReqPhase::Active);
    }
    // 6. a sweep that fails as a whole (the executor found no memory for the
    //    graph's state): the requests of that graph fail with its status, the
    //    other graph's request completes
    {
        FakeExec ex; ex.cap = 8;
        Policy p; p.budget_bytes = 1 << 20;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t a = sc.submit(0, s3.data(), 3, 8, 0.0);
        uint64_t b = sc.submit(1, s10.data(), 10, 8, 0.0);
        sc.step(0.1);
        CHECK(ex.running.size() == 3); // graph 0: one sweep; graph 1: 8 + 2 items
        while (!ex.running.empty()) {
            const int g = ex.running.front().first;
            ex.finish_oldest(-1, g == 1 ? 6 : 0);
            sc.step(0.2);
        }
        CHECK(sc.find(a)->phase == ReqPhase::Done && sc.find(a)->status == 0);
        CHECK(sc.find(b)->phase == ReqPhase::Failed && sc.find(b)->status == 6);
        CHECK(sc.idle());
    }
    // 6b. GPU share bound and least work first across graphs: graph 0 is big
    //     (costly sources, an old long request), graph 1 small; sweeps hold half
    //     the GPU each
    {
        FakeExec ex; ex.cap = 4;
        ex.ctx_per_graph[0] = 4; ex.ctx_per_graph[1] = 4;
        ex.share[0] = 0.5; ex.share[1] = 0.5;
        ex.cost[0] = 100.0; ex.cost[1] = 1.0;
        Policy p; p.budget_bytes = 1 << 20; p.gpu_share = 1.0; p.least_work_first = true;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t big = sc.submit(0, s10.data(), 10, 8, 0.0);
        sc.step(0.1);
        CHECK(ex.running.size() == 2);          // the GPU holds two half sweeps
        uint64_t small = sc.submit(1, s3.data(), 3, 8, 0.2);
        sc.step(0.3);
        CHECK(ex.running.size() == 2);          // full: the small request waits
        ex.finish_oldest();
        sc.step(0.4);
        CHECK(ex.running.size() == 2 && ex.running.back().first == 1);  // small one goes next
        CHECK(ex.running.back().second.size() == 3 && ex.running.back().second[0].ticket == small);
        while (!ex.running.empty()) { ex.finish_oldest(); sc.step(1.0); }
        CHECK(sc.find(small)->t_done <= sc.find(big)->t_done);
        CHECK(sc.find(big)->phase == ReqPhase::Done && sc.idle());
    }
    // 6c. starvation bound: with least work first, a big request that has
    //     waited past starve_after goes before a newer small one
    {
        FakeExec ex; ex.cap = 4;
        ex.ctx_per_graph[0] = 4; ex.ctx_per_graph[1] = 4;
        ex.share[0] = 1.0; ex.share[1] = 1.0;   // one sweep fills the GPU
        ex.cost[0] = 100.0; ex.cost[1] = 1.0;
        Policy p; p.budget_bytes = 1 << 20; p.gpu_share = 1.0; p.least_work_first = true;
        p.starve_after = 5.0;
        Scheduler<FakeExec> sc(ex, p);
        uint64_t s1 = sc.submit(1, s3.data(), 3, 8, 0.0);
        sc.step(0.0);                            // small request takes the GPU
        uint64_t big = sc.submit(0, s10.data(), 10, 8, 0.5);
        uint64_t s2 = sc.submit(1, s3.data(), 3, 8, 1.0);
        ex.finish_oldest();
        sc.step(2.0);                            // not overdue yet: the small one goes first
        CHECK(ex.running.size() == 1 && ex.running.back().first == 1);
        CHECK(ex.running.back().second[0].ticket == s2);
        uint64_t s3t = sc.submit(1, s3.data(), 3, 8, 6.0);
        ex.finish_oldest();
        sc.step(6.0);                            // big has waited 5.5 s: it goes before s3t
        CHECK(ex.running.size() == 1 && ex.running.back().first == 0);
        CHECK(ex.running.back().second[0].ticket == big);
        while (!ex.running.empty()) { ex.finish_oldest(); sc.step(7.0); }
        CHECK(sc.find(s1)->phase == ReqPhase::Done && sc.find(s3t)->phase == ReqPhase::Done);
        CHECK(sc.find(big)->phase == ReqPhase::Done && sc.idle());
    }
    // 7. percentile (nearest rank)
    {
        std::vector<double> v = {5, 1, 4, 2, 3};
        CHECK(percentile(v, 50) == 3 && percentile(v, 99) == 5 && percentile({}, 50) == 0);
    }
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "OK", fails);
    return fails ? 1 : 0;
}
