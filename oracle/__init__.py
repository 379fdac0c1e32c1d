"""CPU oracle for weighted betweenness centrality -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never uses it.
"""
from .oracle import (  # noqa: F401
    OracleError,
    SigmaOverflow,
    build,
    host_threads,
    oracle_bc,
    oracle_bc_edges,
    oracle_changed_sources,
    oracle_source_changed,
    oracle_source_state,
    lib_path,
)
