"""Launch settings of the batched form for the benchmark workloads.

The library's autotuner picked these on MI355X (``python bench.py --autotune``
prints its choice); they are pinned so that the benchmark, its rocprofv3
profiles and the full-size parity tests launch identical kernels.  The grid
workload is configured with 256 sources in flight per launch.  R-MAT's entry
width and tiers were then measured on full runs: the tuner, whose trials run
on a sample of the sources, picks 16-bit entries and tiers 8/64/1024 (1497 ms
per launch) where 8-bit entries with tiers 16/64/4096 take 1480 ms.
"""

LAUNCH = {
    "ba100k": dict(delta=100, wg_threads=1024, lane_max_deg=16),
    "er1000": dict(delta=400, wg_threads=256, lane_max_deg=16),
    "grid1000": dict(delta=182, wg_threads=1024, lane_max_deg=128, batch=256),
    "rmat22": dict(delta=2, wg_threads=1024, lane_max_deg=8, expand_lane_deg=16,
                   wave_max_deg=64, wg_min_deg=4096, lds_bits=8),
}

# Serving run over the eight resident graphs: the Poisson arrival rate is
# fixed (measured once with `python bench.py --config serving --calibrate` at
# 0.7 of the closed-loop capacity of the stream's first 64 requests), and the
# first `warmup` requests of the `requests` are left out of the percentiles.
SERVING = dict(rate=1.4331, requests=512, warmup=32, starve_after_s=5.0)
