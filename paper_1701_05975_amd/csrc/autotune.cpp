// autotune.cpp -- per-graph search over the batched form's settings.
//
// Coordinate descent, each candidate timed on a prefix of the caller's
// source list: the near-far band width, the workgroup size, the dependency
// method, the width of the LDS distance entries, the count pass's lane
// threshold, the three degree thresholds of the frontier expansion (the
// degree-aware thread mapping of Sec. 3.4, whose virtual warp width the paper
// tunes per graph, Fig. 5) and the number of sources in flight.  The winner is cached on the graph handle and reused by
// later calls; fields the caller sets are never searched.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bc_internal.h"

namespace {

struct Search {
    bc_graph *g;
    const int32_t *src_dev;
    int64_t sample;
    double *scratch;
    ResolvedOptions best;
    double best_ms;

    double time(const ResolvedOptions &r)
    {
        DevCounters cnt;
        float ms = 0.f;
        g->tune_trials += 1;
        run_batched(g, r, src_dev, sample, scratch, cnt, ms, nullptr);
        if (cnt.err[0])
            return 1e30; // a setting that trips a bound is never chosen
        return (double)ms;
    }

    void consider(const ResolvedOptions &t)
    {
        const double ms = time(t);
        if (ms < best_ms) {
            best_ms = ms;
            best = t;
        }
    }
};

// Keeps the tier thresholds in order (lane <= group <= workgroup).
void order_tiers(ResolvedOptions &t)
{
    t.wave_deg = std::max(t.wave_deg, t.lane_deg);
    t.wg_deg = std::max(t.wg_deg, t.wave_deg);
}

} // namespace

void autotune(bc_graph *g, ResolvedOptions &r, const bc_options *opt, const int32_t *src_dev,
              int64_t k)
{
    bc_options o;
    memset(&o, 0, sizeof o);
    if (opt)
        o = *opt;
    const int64_t cap = batch_cap(g);
    auto fill_for = [&](int nt, int bits, int &H) {
        int per_cu = 1;
        batched_lds_plan(g, nt, r.accumulate == 2, o.lds_vertices, bits, H, per_cu, o.batch);
        return (int64_t)g->num_cus * per_cu;
    };
    if (!g->tuned.valid) {
        int H0 = 0;
        const int64_t fill = fill_for(r.wg_threads, r.lds_bits, H0);
        // one full occupancy of sources, so that each trial runs the GPU in the
        // regime of the real call; on large graphs at most ~2e10 arc-sources
        int64_t sample = std::min<int64_t>(k, std::max<int64_t>(fill, 64));
        while (sample > 64 && (double)sample * (double)std::max<int64_t>(g->nnz, 1) > 2e10)
            sample /= 2;
        DevBuf scratch;
        scratch.alloc((size_t)g->n * sizeof(double));
        Search S{g, src_dev, sample, (double *)scratch.p, r, 0.0};
        S.best.batch = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)r.batch, sample, cap}));
        S.time(S.best); // warm-up: allocates the slabs and faults in the graph
        S.best_ms = S.time(S.best);

        if (!o.delta) {
            // coarse factors of the default band width, then a finer step around the winner
            const int d0 = S.best.delta;
            for (double f : {0.125, 0.25, 0.5, 2.0, 4.0, 8.0}) {
                ResolvedOptions t = S.best;
                t.delta = std::max(1, (int)(d0 * f));
                if (t.delta != d0)
                    S.consider(t);
            }
            const int d1 = S.best.delta;
            for (double f : {0.7, 1.4}) {
                ResolvedOptions t = S.best;
                t.delta = std::max(1, (int)(d1 * f));
                if (t.delta != d1)
                    S.consider(t);
            }
        }
        if (!o.wg_threads) {
            const int nt0 = S.best.wg_threads;
            for (int nt : {256, 512, 1024}) {
                if (nt == nt0)
                    continue;
                ResolvedOptions t = S.best;
                t.wg_threads = nt;
                int H = 0;
                const int64_t f = fill_for(nt, t.lds_bits, H);
                t.lds_vertices = H;
                // a batch the caller fixed stays fixed; else a full occupancy
                const int64_t want = o.batch ? (int64_t)o.batch : f;
                t.batch = (int)std::max<int64_t>(1, std::min<int64_t>({want, sample, cap}));
                S.consider(t);
            }
        }
        if (!o.lds_bits) {
            // entry width of the LDS distance cache (8-bit entries for packed arcs only)
            const int b0 = S.best.lds_bits;
            for (int bits : {8, 16, 32}) {
                if (bits == b0 || (bits == 8 && !g->packed))
                    continue;
                ResolvedOptions t = S.best;
                t.lds_bits = bits;
                int H = 0;
                (void)fill_for(t.wg_threads, bits, H);
                t.lds_vertices = H;
                S.consider(t);
            }
        }
        if (!o.dep_mode) {
            ResolvedOptions t = S.best;
            t.dep_mode = S.best.dep_mode == 1 ? 2 : 1;
            S.consider(t);
        }
        if (!o.lane_max_deg) {
            const int l0 = S.best.lane_max;
            for (int lm : {4, 8, 16, 32, 64, 128}) {
                if (lm == l0)
                    continue;
                ResolvedOptions t = S.best;
                t.lane_max = lm;
                S.consider(t);
            }
        }
        if (!o.expand_lane_deg) {
            const int l0 = S.best.lane_deg;
            for (int ld : {4, 16, 32}) {
                if (ld == l0)
                    continue;
                ResolvedOptions t = S.best;
                t.lane_deg = ld;
                order_tiers(t);
                S.consider(t);
            }
        }
        if (!o.wave_max_deg) {
            const int w0 = S.best.wave_deg;
            for (int wd : {32, 128, 256}) {
                if (wd == w0 || wd < S.best.lane_deg)
                    continue;
                ResolvedOptions t = S.best;
                t.wave_deg = wd;
                order_tiers(t);
                S.consider(t);
            }
        }
        if (!o.wg_min_deg && g->maxdeg > 256 && !S.best.vw) {
            // only graphs with vertices above the candidates have a workgroup tier
            const int h0 = S.best.wg_deg;
            for (int hd : {256, 1024, 4096}) {
                if (hd == h0 || hd < S.best.wave_deg || hd >= g->maxdeg)
                    continue;
                ResolvedOptions t = S.best;
                t.wg_deg = hd;
                S.consider(t);
            }
        }
        if (!o.batch) {
            // sources in flight: the full occupancy against a half and a quarter of it
            // (fewer state slabs, a smaller working set per sweep)
            const int b0 = S.best.batch;
            for (int div : {2, 4}) {
                ResolvedOptions t = S.best;
                t.batch = std::max(1, b0 / div);
                if (t.batch < 32 || t.batch == b0)
                    continue;
                S.consider(t);
            }
        }
        const ResolvedOptions &c = S.best;
        g->tuned.valid = true;
        g->tuned.delta = c.delta;
        g->tuned.lane_max = c.lane_max;
        g->tuned.wg_threads = c.wg_threads;
        g->tuned.dep_mode = c.dep_mode;
        g->tuned.lane_deg = c.lane_deg;
        g->tuned.wave_deg = c.wave_deg;
        g->tuned.wg_deg = c.wg_deg;
        g->tuned.lds_bits = c.lds_bits;
        // sources in flight as a fraction of the full occupancy of the chosen
        // workgroup size (so that it carries over to calls with other k)
        int Hc = 0;
        const int64_t fc = fill_for(c.wg_threads, c.lds_bits, Hc);
        g->tuned.batch = c.batch >= std::min<int64_t>(fc, sample) ? 0 : c.batch;
        g->tuned.best_ms_per_source = S.best_ms / (double)sample;
    }
    // apply the cached choice to the fields the caller left open
    if (!o.delta)
        r.delta = g->tuned.delta;
    if (!o.lane_max_deg)
        r.lane_max = g->tuned.lane_max;
    if (!o.dep_mode)
        r.dep_mode = g->tuned.dep_mode;
    if (!o.expand_lane_deg)
        r.lane_deg = g->tuned.lane_deg;
    if (!o.wave_max_deg)
        r.wave_deg = g->tuned.wave_deg;
    if (!o.wg_min_deg)
        r.wg_deg = g->tuned.wg_deg;
    order_tiers(r);
    if (!o.lds_bits && g->tuned.lds_bits && r.lds_bits != g->tuned.lds_bits) {
        r.lds_bits = g->tuned.lds_bits;
        int H = 0;
        (void)fill_for(r.wg_threads, r.lds_bits, H);
        r.lds_vertices = H;
    }
    if (!o.wg_threads && r.wg_threads != g->tuned.wg_threads) {
        r.wg_threads = g->tuned.wg_threads;
        int H = 0;
        const int64_t f = fill_for(r.wg_threads, r.lds_bits, H);
        r.lds_vertices = H;
        if (!o.batch)
            r.batch = (int)std::max<int64_t>(1, std::min<int64_t>({f, k, cap}));
    }
    if (!o.batch && g->tuned.batch > 0)
        r.batch = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)g->tuned.batch, k, cap}));
}
