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


def mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def edge_hash_np(seed: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    S = np.uint64(splitmix_outputs(seed, 1)[0])
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
