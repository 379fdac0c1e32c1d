"""Launch settings of the batched form for the benchmark workloads.

The library's autotuner picked these on MI355X (``python bench.py --autotune``
prints its choice); they are pinned so that the benchmark, its rocprofv3
profiles and the full-size parity tests launch identical kernels.  The grid
workload is configured with 256 sources in flight per launch.
"""

LAUNCH = {
    "ba100k": dict(delta=100, wg_threads=1024, lane_max_deg=16),
    "er1000": dict(delta=400, wg_threads=256, lane_max_deg=16),
    "grid1000": dict(delta=182, wg_threads=1024, lane_max_deg=128, batch=256),
    "rmat22": dict(delta=3, wg_threads=1024, lane_max_deg=32),
}
