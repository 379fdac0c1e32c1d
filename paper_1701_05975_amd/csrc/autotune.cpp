// autotune.cpp -- per-graph search over the batched form's settings.
//
// Coordinate descent over the near-far band width, the workgroup size, the
// lane/wave degree threshold and the number of sources in flight, each
// candidate timed on a prefix of the caller's source list.  The winner is
// cached on the graph handle and reused by later calls.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bc_internal.h"

static double time_candidate(bc_graph *g, const ResolvedOptions &r, const int32_t *src_dev,
                             int64_t k, double *scratch)
{
    DevCounters cnt;
    float ms = 0.f;
    run_batched(g, r, src_dev, k, scratch, cnt, ms, nullptr);
    if (cnt.err[0])
        return 1e30; // a setting that trips a bound is never chosen
    return (double)ms;
}

void autotune(bc_graph *g, ResolvedOptions &r, const bc_options *opt, const int32_t *src_dev,
              int64_t k)
{
    bc_options o;
    memset(&o, 0, sizeof o);
    if (opt)
        o = *opt;
    if (!g->tuned.valid) {
        const int fill = r.batch;
        // one full occupancy of sources, so that each trial runs the GPU in the
        // regime of the real call; on large graphs at most ~2e10 arc-sources
        int64_t sample = std::min<int64_t>(k, std::max<int64_t>((int64_t)fill, 64));
        while (sample > 64 && (double)sample * (double)std::max<int64_t>(g->nnz, 1) > 2e10)
            sample /= 2;
        DevBuf scratch;
        scratch.alloc((size_t)g->n * sizeof(double));
        ResolvedOptions c = r;
        c.batch = (int)std::min<int64_t>(fill, sample);
        // warm-up: allocates the slabs and faults in the graph
        time_candidate(g, c, src_dev, sample, (double *)scratch.p);
        double best = time_candidate(g, c, src_dev, sample, (double *)scratch.p);

        if (!o.delta) {
            // coarse factors of the default band width, then a finer step around the winner
            const int d0 = c.delta;
            for (double f : {0.125, 0.25, 0.5, 2.0, 4.0, 8.0}) {
                ResolvedOptions t = c;
                t.delta = std::max(1, (int)(d0 * f));
                const double ms = time_candidate(g, t, src_dev, sample, (double *)scratch.p);
                if (ms < best) {
                    best = ms;
                    c = t;
                }
            }
            const int d1 = c.delta;
            for (double f : {0.7, 1.4}) {
                ResolvedOptions t = c;
                t.delta = std::max(1, (int)(d1 * f));
                if (t.delta == d1)
                    continue;
                const double ms = time_candidate(g, t, src_dev, sample, (double *)scratch.p);
                if (ms < best) {
                    best = ms;
                    c = t;
                }
            }
        }
        if (!o.wg_threads) {
            for (int nt : {256, 512, 1024}) {
                if (nt == c.wg_threads)
                    continue;
                ResolvedOptions t = c;
                t.wg_threads = nt;
                int H = 0, per_cu = 1;
                batched_lds_plan(g, nt, t.accumulate == 2, o.lds_vertices, t.lds_bits, H, per_cu);
                t.lds_vertices = H;
                // a batch the caller fixed stays fixed; else a full occupancy
                const int64_t want = o.batch ? (int64_t)o.batch : (int64_t)g->num_cus * per_cu;
                t.batch = std::max(1, (int)std::min<int64_t>(want, sample));
                const double ms = time_candidate(g, t, src_dev, sample, (double *)scratch.p);
                if (ms < best) {
                    best = ms;
                    c = t;
                }
            }
        }
        if (!o.dep_mode) {
            ResolvedOptions t = c;
            t.dep_mode = c.dep_mode == 1 ? 2 : 1;
            const double ms = time_candidate(g, t, src_dev, sample, (double *)scratch.p);
            if (ms < best) {
                best = ms;
                c = t;
            }
        }
        if (!o.lane_max_deg) {
            for (int lm : {4, 8, 16, 64, 128}) {
                ResolvedOptions t = c;
                t.lane_max = lm;
                const double ms = time_candidate(g, t, src_dev, sample, (double *)scratch.p);
                if (ms < best) {
                    best = ms;
                    c = t;
                }
            }
        }
        g->tuned.valid = true;
        g->tuned.delta = c.delta;
        g->tuned.lane_max = c.lane_max;
        g->tuned.wg_threads = c.wg_threads;
        g->tuned.dep_mode = c.dep_mode;
        g->tuned.best_ms_per_source = best / (double)sample;
    }
    if (!o.delta)
        r.delta = g->tuned.delta;
    if (!o.lane_max_deg)
        r.lane_max = g->tuned.lane_max;
    if (!o.dep_mode)
        r.dep_mode = g->tuned.dep_mode;
    if (!o.wg_threads && r.wg_threads != g->tuned.wg_threads) {
        r.wg_threads = g->tuned.wg_threads;
        int H = 0, per_cu = 1;
        batched_lds_plan(g, r.wg_threads, r.accumulate == 2, o.lds_vertices, r.lds_bits, H,
                         per_cu);
        r.lds_vertices = H;
        if (!o.batch)
            r.batch = std::max(1, (int)std::min<int64_t>((int64_t)g->num_cus * per_cu, k));
    }
}
