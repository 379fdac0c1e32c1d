// noalloc.hip -- bc_compute_device_noalloc: the batched form with its state
// slabs in a fixed device array, for callers that cannot allocate device
// memory during a call.
//
// The slabs (the per-source state of the batched kernel) normally live in a
// per-graph workspace that the library grows with hipMalloc.  Here they live
// in `scratch`, one file-scope device array per GPU, held from the moment the
// library's code object is loaded on that GPU until the process ends.  Host
// code never passes the array's name to a kernel (on the host that name is a
// stand-in, not a device address): the device address is looked up once per
// device with hipGetSymbolAddress and kept in `g_scratch_ptr`.
//
// Every call on one GPU shares that GPU's array and leaves its contents
// behind, so each call resets the slabs it uses (a kernel, no memset node) before
// the batched launch.  Calls that overlap on one GPU, on any streams or host
// threads, race on the array; callers serialise them.
#include <mutex>

#include "bc_internal.h"

static __device__ __align__(256) char scratch[BC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up on the first call for
// that device with the device current (each GPU holds its own copy).
char *scratch_on(int device)
{
    if (device < 0 || device >= kMaxDevices)
        throw bc_error(BC_E_DEVICE, "device %d out of the supported range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device])
        return g_scratch_ptr[device];
    int prev = 0;
    hip_check(hipGetDevice(&prev), "hipGetDevice");
    if (prev != device)
        hip_check(hipSetDevice(device), "hipSetDevice");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device)
        (void)hipSetDevice(prev);
    hip_check(e, "hipGetSymbolAddress(scratch)");
    if (!p)
        throw bc_error(BC_E_DEVICE, "scratch array has no device address");
    g_scratch_ptr[device] = (char *)p;
    return (char *)p;
}

void compute_noalloc(bc_graph *g, const int32_t *src_dev, int64_t k, const bc_options *opt,
                     double *bc_dev, bc_stats *stats)
{
    if (opt && opt->mode != BC_MODE_AUTO && opt->mode != BC_MODE_BATCHED)
        throw bc_error(BC_E_INVAL, "the allocation-free entry point runs the batched form only");
    if (opt && opt->autotune)
        throw bc_error(BC_E_INVAL, "the allocation-free entry point does not autotune");
    ResolvedOptions r = resolve_options(g, opt, k);
    const SlabLayout L = slab_layout(g->n, g->nnz);
    const int64_t fit = (int64_t)(BC_NOALLOC_SCRATCH_BYTES / std::max<size_t>(L.stride, 1));
    if (fit < 1)
        throw bc_error(BC_E_NOMEM,
                       "one state slab of this graph needs %zu bytes; the allocation-free "
                       "scratch holds %zu",
                       L.stride, (size_t)BC_NOALLOC_SCRATCH_BYTES);
    r.batch = (int)std::min<int64_t>(r.batch, fit);
    char *base = scratch_on(g->device);
    hipStream_t st = r.stream;
    DevCounters cnt;
    float kms = 0.f;
    reset_device_counters(g, st);
    if (r.accumulate == 2 || k == 0)
        hip_check(launch_fill_u64((unsigned long long *)bc_dev, (size_t)g->n, 0ull, st), "zero");
    if (k > 0) {
        const int nslabs = (int)std::min<int64_t>(r.batch, k);
        hip_check(launch_slab_reset(base, L, nslabs, g->n, st), "slab reset");
        launch_batched_pass(g, r, src_dev, k, bc_dev, base, L, nslabs, nullptr, st);
    }
    read_device_counters(g, st, cnt);
    if (k > 0)
        hip_check(hipEventElapsedTime(&kms, g->ev_k0, g->ev_k1), "event time");
    check_device_errors(cnt);
    fill_stats(g, r, cnt, k, (double)kms, (double)kms, k > 0 ? 1 : 0, stats);
    g->last_stats_valid = true;
    fill_stats(g, r, cnt, k, (double)kms, (double)kms, k > 0 ? 1 : 0, &g->last_stats);
}

} // namespace

extern "C" bc_status bc_compute_device_noalloc(bc_graph *g, const int32_t *sources_dev,
                                               int64_t k, const bc_options *opt, double *bc_dev,
                                               bc_stats *stats)
{
    return bc_guarded([&] {
        if (!g || !bc_dev || (k > 0 && !sources_dev))
            throw bc_error(BC_E_INVAL, "null argument");
        if (k < 0)
            throw bc_error(BC_E_INVAL, "k must be >= 0");
        compute_noalloc(g, sources_dev, k, opt, bc_dev, stats);
    });
}
