// The serving scheduler driven the way the server drives it, under the thread
// sanitizer: one scheduler thread steps the policy under the server mutex and
// signals completions on a condition variable, several client threads submit
// requests and wait for them under the same mutex, and a fake executor
// finishes each sweep a little later.  No HIP; csrc/server_core.h is used as
// the library uses it.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>

#include "../../paper_1701_05975_amd/csrc/server_core.h"

using namespace bcserve;
using clk = std::chrono::steady_clock;

static double now_s()
{
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct FakeExec {
    struct Sweep {
        int graph;
        std::vector<SweepItem> items;
        double t_done;
    };
    std::vector<Sweep> running;
    std::vector<int> busy = std::vector<int>(4, 0);
    int free_contexts(int g) { return 2 - busy[(size_t)g]; }
    int max_items(int) { return 16; }
    double sweep_share(int) { return 0.25; }
    double source_cost(int g) { return 1.0 + g; }
    bool alloc_result(Request &r)
    {
        r.out = new double[4]();
        return true;
    }
    void free_result(Request &r)
    {
        delete[] static_cast<double *>(r.out);
        r.out = nullptr;
    }
    void launch(int g, const std::vector<SweepItem> &items)
    {
        busy[(size_t)g] += 1;
        running.push_back({g, items, now_s() + 1e-4 * (double)(1 + items.size() % 3)});
    }
    void poll(std::vector<Finished> &out)
    {
        const double t = now_s();
        for (size_t i = 0; i < running.size();) {
            if (running[i].t_done <= t) {
                Finished f;
                f.graph = running[i].graph;
                f.items = running[i].items;
                f.item_fail.assign(f.items.size(), 0);
                // every 97th source overflows: its request fails, the others not
                for (size_t j = 0; j < f.items.size(); ++j)
                    f.item_fail[j] = f.items[j].source % 97 == 96;
                f.item_status = 5;
                busy[(size_t)f.graph] -= 1;
                out.push_back(std::move(f));
                running.erase(running.begin() + (long)i);
            } else {
                ++i;
            }
        }
    }
};

int main()
{
    FakeExec ex;
    Policy pol;
    pol.budget_bytes = 64 * 8;
    pol.max_active = 16;
    pol.gpu_share = 1.0;           // four sweeps of a quarter each at once
    pol.least_work_first = true;
    pol.starve_after = 0.002;      // overdue requests reorder the queues too
    Scheduler<FakeExec> sched(ex, pol);
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::atomic<bool> stop{false};
    std::thread worker([&] {
        while (!stop.load()) {
            bool changed;
            {
                std::unique_lock<std::mutex> lk(mu);
                changed = sched.step(now_s());
                if (changed)
                    cv_done.notify_all();
                if (!changed && sched.idle())
                    cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
            if (!changed)
                std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    });
    std::atomic<int> done{0}, failed{0}, bad{0};
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c)
        clients.emplace_back([&, c] {
            for (int i = 0; i < 50; ++i) {
                std::vector<int32_t> src((size_t)(1 + (c * 7 + i) % 40));
                for (size_t j = 0; j < src.size(); ++j)
                    src[j] = (int32_t)((c * 1000 + i * 31 + (int)j) % 200);
                uint64_t t;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    t = sched.submit(c % 4, src.data(), (int64_t)src.size(), 8, now_s());
                    cv_work.notify_all();
                }
                std::unique_lock<std::mutex> lk(mu);
                cv_done.wait(lk, [&] {
                    auto r = sched.find(t);
                    return r && (r->phase == ReqPhase::Done || r->phase == ReqPhase::Failed);
                });
                auto r = sched.find(t);
                bool expect_fail = false;
                for (int32_t s : src)
                    expect_fail |= s % 97 == 96;
                if ((r->phase == ReqPhase::Failed) != expect_fail)
                    bad.fetch_add(1);
                (r->phase == ReqPhase::Done ? done : failed).fetch_add(1);
                ex.free_result(*r);
                sched.release(t);
            }
        });
    for (auto &t : clients)
        t.join();
    {
        std::lock_guard<std::mutex> lk(mu);
        stop.store(true);
        cv_work.notify_all();
    }
    worker.join();
    const bool ok = bad.load() == 0 && done.load() + failed.load() == 200 && sched.idle();
    std::printf("%s: %d done, %d failed, %d wrong outcomes\n", ok ? "OK" : "FAILED", done.load(),
                failed.load(), bad.load());
    return ok ? 0 : 1;
}
