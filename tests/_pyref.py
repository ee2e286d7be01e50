"""Independent pure-Python/numpy reference pieces used to pin the oracle.

Nothing here imports the oracle or the HIP library. Each function restates a
plain definition:
  * SplitMix64's output function (pinned by the published vectors in
    golden/splitmix64_kat.txt),
  * the greedy matching (paper, Section 3: sort edges by decreasing weight,
    scan, take an edge iff both endpoints are free), under the same strict key,
  * brute-force maximum weight matching for tiny graphs,
  * validity and maximality of a matching (paper, Section 1).
"""
from __future__ import annotations

import os

import numpy as np

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def mix64(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix_outputs(seed: int, count: int):
    s = seed & M64
    out = []
    for _ in range(count):
        s = (s + GAMMA) & M64
        out.append(mix64(s))
    return out


def load_kat():
    rows = []
    with open(os.path.join(GOLDEN, "splitmix64_kat.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            s, i, v = line.split()
            rows.append((int(s, 0), int(i, 0), int(v, 0)))
    return rows


def load_edge_hash_kat():
    rows = []
    with open(os.path.join(GOLDEN, "edge_hash_kat.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            s, lo, hi, v = line.split()
            rows.append((int(s, 0), int(lo, 0), int(hi, 0), int(v, 0)))
    return rows


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def seed_mix(seed: int) -> int:
    """Per-run seed mix of the tie-break key: mix(seed XOR gamma)."""
    return mix64((seed & M64) ^ GAMMA)


def edge_hash(seed: int, lo: int, hi: int) -> int:
    """H(seed, lo, hi) in Python big integers."""
    return mix64((((lo & 0xFFFFFFFF) << 32) | (hi & 0xFFFFFFFF)) ^ seed_mix(seed))


def edge_hash_np(seed: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    S = np.uint64(seed_mix(seed))
    pair = (lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64)
    return mix64_np(pair ^ S)


def undirected_edges(g):
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    sel = rows < g.col
    return rows[sel], g.col[sel].astype(np.int64), g.w[sel]


def greedy(g, seed: int):
    """Greedy matching under the key (w numerically, then H unsigned)."""
    lo, hi, w = undirected_edges(g)
    w = (w.astype(np.float32) + np.float32(0.0)).astype(np.float64)  # -0 -> +0
    H = edge_hash_np(seed, lo, hi)
    order = np.lexsort((H, w))[::-1]
    mate = np.full(g.n, -1, dtype=np.int32)
    for j in order:
        a, b = lo[j], hi[j]
        if mate[a] == -1 and mate[b] == -1:
            mate[a] = b
            mate[b] = a
    return mate


def edge_ranks(lo, hi, w, seed: int, hash_fn=None) -> np.ndarray:
    """Rank of every undirected edge in the strict key order (w numerically,
    -0 == +0, then H unsigned); 0 is the smallest key."""
    wf = (w.astype(np.float32) + np.float32(0.0)).astype(np.float64)
    H = edge_hash_np(seed, lo, hi) if hash_fn is None else hash_fn(lo, hi)
    order = np.lexsort((H, wf))
    r = np.empty(len(lo), dtype=np.int64)
    r[order] = np.arange(len(lo), dtype=np.int64)
    return r


def local_max_log(g, seed: int, key_of_phase=None):
    """Local max by its definition (paper, Section 1), edge by edge: in every
    phase an edge joins M iff its key beats the key of every other live edge
    sharing an endpoint; then every edge touching a matched vertex dies.
    Returns (mate, log) with log rows (|E_t|, V_t, matched_t): live edges and
    vertices with a live edge at the start of phase t, edges matched in it.
    key_of_phase(t, lo, hi, w) may give per-phase ranks (renewed keys)."""
    lo, hi, w = undirected_edges(g)
    live = np.arange(len(lo))
    fixed = edge_ranks(lo, hi, w, seed) if key_of_phase is None else None
    mate = np.full(g.n, -1, dtype=np.int32)
    log = []
    t = 0
    while len(live):
        t += 1
        a, b = lo[live], hi[live]
        r = fixed[live] if fixed is not None else key_of_phase(t, a, b, w[live])
        best = np.full(g.n, -1, dtype=np.int64)
        np.maximum.at(best, a, r)
        np.maximum.at(best, b, r)
        lm = (best[a] == r) & (best[b] == r)
        vt = len(np.unique(np.concatenate([a, b])))
        mate[a[lm]] = b[lm]
        mate[b[lm]] = a[lm]
        log.append((len(live), vt, int(lm.sum())))
        live = live[(mate[a] == -1) & (mate[b] == -1)]
    return mate, np.array(log, dtype=np.int64).reshape(-1, 3)


def is_valid_maximal(g, mate) -> bool:
    mate = np.asarray(mate)
    n = g.n
    for v in range(n):
        p = mate[v]
        if p == -1:
            continue
        if not (0 <= p < n) or mate[p] != v:
            return False
        row = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        if p not in row:
            return False
    lo, hi, _ = undirected_edges(g)
    free_free = (mate[lo] == -1) & (mate[hi] == -1)
    return not bool(free_free.any())


def matching_weight(g, mate) -> float:
    lo, hi, w = undirected_edges(g)
    sel = mate[lo] == hi
    return float(np.sum(w[sel].astype(np.float64)))


def matching_weight_exact(g, mate):
    """(w(M) correctly rounded, sum of |w| over M, |M|) with math.fsum."""
    import math
    lo, hi, w = undirected_edges(g)
    sel = mate[lo] == hi
    ws = w[sel].astype(np.float64)
    return math.fsum(ws.tolist()), math.fsum(np.abs(ws).tolist()), int(sel.sum())


def brute_mwm(g) -> float:
    """Maximum weight matching by DP over vertex subsets (n <= 16)."""
    n = g.n
    adj = [dict() for _ in range(n)]
    for v in range(n):
        for k in range(g.row_ptr[v], g.row_ptr[v + 1]):
            adj[v][int(g.col[k])] = float(g.w[k])
    memo = {0: 0.0}

    def f(mask):
        if mask in memo:
            return memo[mask]
        i = (mask & -mask).bit_length() - 1
        rest = mask & ~(1 << i)
        best = f(rest)
        for j, wij in adj[i].items():
            if rest >> j & 1:
                best = max(best, wij + f(rest & ~(1 << j)))
        memo[mask] = best
        return best

    return f((1 << n) - 1)
