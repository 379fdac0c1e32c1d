"""Exact brute-force betweenness for tiny graphs (test helper, pure Python).

Two independent routes, both exact (``fractions.Fraction``):

* :func:`enumerate_bc` lists every simple path between every ordered pair,
  keeps the shortest ones, and counts how many pass through each vertex --
  the definition of Eq. 1 (Sec. 2.1) taken literally.  Feasible for n <= ~9.
* :func:`pairwise_bc` uses all-pairs distances (Floyd-Warshall) and all-pairs
  path counts, then sums sigma_sv * sigma_vt / sigma_st over pairs with
  d(s,v) + d(v,t) = d(s,t) (the pair-dependency definition in Sec. 2.1).
  Feasible for n <= ~64.

Neither shares code with the oracle.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

INF = float("inf")


def arcs_of(g):
    out = [[] for _ in range(g.n)]
    for v in range(g.n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            out[v].append((int(g.col[e]), int(g.w[e])))
    return out


def enumerate_paths(g, sources=None):
    """For each ordered pair (s, t): (shortest length, list of shortest paths).
    Parallel arcs count as distinct paths (paths are arc sequences)."""
    adj = arcs_of(g)
    res = {}
    srcs = range(g.n) if sources is None else sources
    for s in srcs:
        best = {}
        stack = [(s, 0, (s,), frozenset([s]))]
        while stack:
            v, L, path, seen = stack.pop()
            if v != s:
                cur = best.get(v)
                if cur is None or L < cur[0]:
                    best[v] = (L, [path])
                elif L == cur[0]:
                    cur[1].append(path)
            for (u, w) in adj[v]:
                if u not in seen:
                    stack.append((u, L + w, path + (u,), seen | {u}))
        for t, (L, paths) in best.items():
            res[(s, t)] = (L, paths)
    return res


def enumerate_bc(g, sources=None):
    """(bc list of Fraction, dist dict, sigma dict) by literal path enumeration."""
    res = enumerate_paths(g, sources)
    bc = [Fraction(0)] * g.n
    for (s, t), (L, paths) in res.items():
        tot = len(paths)
        through = [0] * g.n
        for p in paths:
            for v in p[1:-1]:
                through[v] += 1
        for v in range(g.n):
            if through[v]:
                bc[v] += Fraction(through[v], tot)
    dist = {k: v[0] for k, v in res.items()}
    sig = {k: len(v[1]) for k, v in res.items()}
    return bc, dist, sig


def all_pairs(g):
    """Floyd-Warshall distances (float inf for no path) and path counts (int)."""
    n = g.n
    D = [[INF] * n for _ in range(n)]
    for v in range(n):
        D[v][v] = 0
    adj = arcs_of(g)
    for v in range(n):
        for (u, w) in adj[v]:
            if w < D[v][u]:
                D[v][u] = w
    for k in range(n):
        Dk = D[k]
        for i in range(n):
            dik = D[i][k]
            if dik == INF:
                continue
            Di = D[i]
            for j in range(n):
                nd = dik + Dk[j]
                if nd < Di[j]:
                    Di[j] = nd
    # path counts: sigma[s][t] = sum over arcs (u,t,w) with D[s][u] + w == D[s][t]
    S = [[0] * n for _ in range(n)]
    rev = [[] for _ in range(n)]
    for v in range(n):
        for (u, w) in adj[v]:
            rev[u].append((v, w))
    for s in range(n):
        S[s][s] = 1
        order = sorted((t for t in range(n) if D[s][t] != INF), key=lambda t: D[s][t])
        for t in order:
            if t == s:
                continue
            tot = 0
            for (u, w) in rev[t]:
                if D[s][u] != INF and D[s][u] + w == D[s][t]:
                    tot += S[s][u]
            S[s][t] = tot
    return D, S


def pairwise_bc(g, sources=None):
    """Exact BC via sum_{s,t} sigma_sv sigma_vt / sigma_st over v on s-t shortest paths."""
    D, S = all_pairs(g)
    n = g.n
    srcs = range(n) if sources is None else sources
    bc = [Fraction(0)] * n
    for s in srcs:
        for t in range(n):
            if t == s or D[s][t] == INF:
                continue
            for v in range(n):
                if v == s or v == t:
                    continue
                if D[s][v] != INF and D[v][t] != INF and D[s][v] + D[v][t] == D[s][t]:
                    bc[v] += Fraction(S[s][v] * S[v][t], S[s][t])
    return bc, D, S


def hop_invariant(g, sources):
    """sum over s in sources, t reached, t != s, of (mean hop count of the s-t
    shortest paths - 1), computed with an independent forward recurrence:
    H[t] = total hops over all shortest s-t paths = sum over tight in-arcs of
    (H[u] + sigma[u])."""
    D, S = all_pairs(g)
    n = g.n
    adj = arcs_of(g)
    rev = [[] for _ in range(n)]
    for v in range(n):
        for (u, w) in adj[v]:
            rev[u].append((v, w))
    total = Fraction(0)
    for s in sources:
        H = [0] * n
        order = sorted((t for t in range(n) if D[s][t] != INF), key=lambda t: D[s][t])
        for t in order:
            if t == s:
                continue
            h = 0
            for (u, w) in rev[t]:
                if D[s][u] != INF and D[s][u] + w == D[s][t]:
                    h += H[u] + S[s][u]
            H[t] = h
            total += Fraction(h, S[s][t]) - 1
    return total


def enumerate_ebc(g, sources=None):
    """Edge betweenness by literal enumeration of shortest paths as arc
    sequences (parallel arcs are distinct): for every ordered pair (s, t) and
    every arc e, the fraction of shortest s-t paths that use e."""
    out = [[] for _ in range(g.n)]
    for v in range(g.n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            out[v].append((int(g.col[e]), int(g.w[e]), e))
    ebc = [Fraction(0)] * g.nnz
    srcs = range(g.n) if sources is None else sources
    for s in srcs:
        best = {}
        stack = [(s, 0, (), frozenset([s]))]
        while stack:
            v, L, arcs, seen = stack.pop()
            if v != s:
                cur = best.get(v)
                if cur is None or L < cur[0]:
                    best[v] = (L, [arcs])
                elif L == cur[0]:
                    cur[1].append(arcs)
            for (u, w, e) in out[v]:
                if u not in seen:
                    stack.append((u, L + w, arcs + (e,), seen | {u}))
        for t, (L, paths) in best.items():
            for p in paths:
                for e in p:
                    ebc[e] += Fraction(1, len(paths))
    return ebc
