"""The oracle's pins must catch plausible mistakes (CPU only).

Each mutant is a copy of oracle.c with one plausible slip planted in it (a
non-strict comparison, a dropped term, a transposed ratio, a wrong index...),
compiled into a temporary library.  The pin battery below -- literal path
enumeration, closed forms and invariants -- must reject every one of them,
while accepting the unmodified oracle.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import oracle
from brute import enumerate_bc
from paper_1701_05975_amd import graphgen as gg

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "relax_non_strict": ("if (nd < d[u]) {", "if (nd <= d[u]) {"),
    "count_reset_to_one": ("sigma[u] = sigma[v];\n                heap_push", "sigma[u] = 1;\n                heap_push"),
    "drop_one_plus": ("* (1.0 + delta[u]);", "* (delta[u]);"),
    "transposed_ratio": ("((double)sigma[v] / (double)sigma[u])", "((double)sigma[u] / (double)sigma[v])"),
    "weight_ignored_forward": ("int64_t nd = d[v] + (int64_t)w[e];", "int64_t nd = d[v] + 1;"),
    "tight_test_wrong": ("d[u] == d[v] + (int64_t)w[e])", "d[u] > d[v])"),
    "source_not_excluded": ("if (v != s)\n                job->bc[v]", "if (1)\n                job->bc[v]"),
    "backward_skips_first": ("for (int32_t i = n_order - 1; i >= 0; --i)", "for (int32_t i = n_order - 1; i > 0; --i)"),
    "forward_order_reversed": ("for (int32_t i = n_order - 1; i >= 0; --i) {\n        int32_t v = ws->order[i];",
                               "for (int32_t i = 0; i < n_order; ++i) {\n        int32_t v = ws->order[i];"),
    "equal_adds_own_count": ("uint64_t sum = sigma[u] + sigma[v];", "uint64_t sum = sigma[u] + sigma[u];"),
}


def battery(lib):
    """Returns the list of failed pin names for the library at `lib`."""
    failed = []

    def chk(name, ok):
        if not ok:
            failed.append(name)

    for seed in range(3):
        g = gg.random_graph(7, 0.5, 1, 2, seed=seed)
        exact, dist, sig = enumerate_bc(g)
        try:
            bc = oracle.oracle_bc(g, np.arange(g.n), lib=lib)
            chk("enumeration_bc", all(abs(bc[v] - float(exact[v])) <= 1e-12 * max(1, float(exact[v]))
                                      for v in range(g.n)))
            for s in range(g.n):
                d, sigma, delta, _ = oracle.oracle_source_state(g, s, lib=lib)
                for t in range(g.n):
                    if (s, t) in dist:
                        chk("enumeration_sigma", int(sigma[t]) == sig[(s, t)])
                reached = int(np.sum(d != oracle.oracle.INF64))
                chk("delta_source", abs(delta[s] - (reached - 1)) < 1e-9)
        except oracle.OracleError:
            failed.append("raised")
    n = 9
    bc = oracle.oracle_bc(gg.path_graph(n, np.arange(1, n)), np.arange(n), lib=lib)
    chk("path", all(bc[i] == 2 * i * (n - 1 - i) for i in range(n)))
    bc = oracle.oracle_bc(gg.star_graph(n, np.arange(2, n + 1)), np.arange(n), lib=lib)
    chk("star", bc[0] == (n - 1) * (n - 2))
    return failed


def test_unmodified_oracle_passes_battery():
    assert battery(None) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_every_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for {name} not unique"
    src = tmp_path / "oracle_mut.c"
    src.write_text(text.replace(old, new))
    lib = oracle.build(src=str(src), out=str(tmp_path / "liboracle_mut.so"))
    assert battery(lib) != [], f"mutant {name} passed every pin"
