"""CPU model of the count pass's predecessor recording (batched form).

The expansion keeps, per vertex, the least (distance, tail) over the
improvements it received (the key) and up to TIE_MAX (distance, tail) pairs of
relaxations that matched its distance at the time (ties), written into the
vertex's own slice of the DAG-list array.  The count pass takes a vertex's
shortest-path count from the key's tail and the tails of the pairs at the
key's distance, unless a tie was not kept or a tail repeats (a tail expanded
twice at its final distance, or parallel tight arcs), in which case it scans
the in-arcs, in that round and every later one.

This model replays the scheme on small random multigraphs under arbitrary
relaxation orders (label-correcting, with forced repeated expansions), bands
and count rounds in which a vertex waits for predecessors of its own band and
a waiting scan has already written over the pairs, and checks the counts
against a direct count over the tight arcs.  Without the repeated-tail rule,
or with the scan decision not kept across rounds, seeds fail (checked below).
"""
from __future__ import annotations

import collections
import random

TIE_MAX = 7


def run(seed: int, dedupe: bool = True, sticky: bool = True) -> bool:
    rng = random.Random(seed)
    n = rng.randint(2, 40)
    arcs = [(rng.randrange(n), rng.randrange(n), rng.randint(1, rng.choice([1, 2, 3])))
            for _ in range(rng.randint(1, 6 * n))]
    if rng.random() < 0.3:  # parallel arcs, equal weights
        arcs += [arcs[rng.randrange(len(arcs))] for _ in range(len(arcs) // 3)]
    out = collections.defaultdict(list)
    inn = collections.defaultdict(list)
    for a, b, w in arcs:
        out[a].append((b, w))
        inn[b].append((a, w))
    s = rng.randrange(n)
    INF = 1 << 40
    d = [INF] * n
    d[s] = 0
    key = [None] * n
    cnt = [0] * n
    slice_ = {v: [None] * len(inn[v]) for v in range(n)}
    q, inq = [s], {s}
    while q:  # label-correcting in random order: non-final ties and repeats
        v = q.pop(rng.randrange(len(q)))
        inq.discard(v)
        reps = 2 if rng.random() < 0.3 else 1
        for u, w in out[v] * reps:
            nd = d[v] + w
            if nd < d[u]:
                d[u] = nd
                key[u] = (nd, v) if key[u] is None else min(key[u], (nd, v))
                if u not in inq:
                    q.append(u)
                    inq.add(u)
            elif nd == d[u]:
                t = cnt[u]
                cnt[u] += 1
                if t < TIE_MAX and 2 * (t + 1) <= len(inn[u]):
                    slice_[u][2 * t] = nd
                    slice_[u][2 * t + 1] = v
    sig = [0] * n
    sig[s] = 1
    scan_flag = [False] * n

    def keyed(v):
        nt, P = cnt[v], slice_[v]
        if nt > TIE_MAX or 2 * nt > len(P) or scan_flag[v]:
            return None
        dk, u0 = key[v]
        tails = [u0] + [P[2 * i + 1] for i in range(nt) if P[2 * i] == dk]
        if dedupe and len(set(tails)) != len(tails):
            if sticky:
                scan_flag[v] = True
            return None
        if any(not isinstance(t, int) or not 0 <= t < n for t in tails):
            return "bad"
        if any(sig[t] == 0 for t in tails):
            return "wait"
        sig[v] = sum(sig[t] for t in tails)
        return "done"

    def scan(v):
        tight, P = 0, slice_[v]
        for pos, (a, w) in enumerate(inn[v]):
            if d[a] + w == d[v]:
                if sig[a] == 0:
                    return "wait"
                P[tight] = pos  # the DAG list over the pairs
                tight += 1
        sig[v] = sum(sig[a] for a, w in inn[v] if d[a] + w == d[v])
        return "done"

    delta = rng.choice([1, 2, 3, 100])
    reached = [v for v in range(n) if d[v] < INF]
    bands = collections.defaultdict(list)
    for v in reached:
        bands[d[v] // delta].append(v)
    for b in sorted(bands):
        items = [v for v in bands[b] if v != s]
        for _ in range(len(bands[b]) + 2):
            if not items:
                break
            rng.shuffle(items)
            nxt = []
            for v in items:
                r = keyed(v)
                if r is None:
                    r = scan(v)
                if r == "bad":
                    return False
                if r == "wait":
                    nxt.append(v)
            items = nxt
        if items:
            return False
    ref = [0] * n
    ref[s] = 1
    for v in sorted(reached, key=lambda x: d[x]):
        if v != s:
            ref[v] = sum(ref[a] for a, w in inn[v] if d[a] + w == d[v])
    return sig == ref


def test_counts_from_keys_and_ties_match_tight_arcs():
    assert all(run(seed) for seed in range(1500))


def test_each_rule_is_needed():
    # the model is sharp enough to see either rule removed
    assert not all(run(seed, dedupe=False) for seed in range(1500))
    assert not all(run(seed, sticky=False) for seed in range(1500))
