"""Pins of the oracle's contraction by a matching (the coarsening step of
multilevel partitioning, Section 1; contraction instances, Section 3.1).

The coarse graph as a weighted set is fixed by linear algebra: with P the
n x nc membership matrix (P[v, cmap[v]] = 1), the coarse adjacency is P^T A P
with its diagonal removed, and the coarse vertex weights are P^T vw. The
layout readings (coarse ids in representative order, rows in first-occurrence
order, fp32 sums in fine-edge order) are pinned by their own properties,
closed forms on ladders and cycles, and a hand-worked fp32 example
(tests/golden/contract_fp32_sums.txt). Planted mistakes must fail a pin.
"""
import ctypes
import multiprocessing as mp
import os
import subprocess

import numpy as np
import pytest

import lmgen
import oracle
from tests import _pyref as ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lm_oracle.c")
GOLDEN = os.path.join(ROOT, "tests", "golden", "contract_fp32_sums.txt")


def _dense(n, rp, col, w):
    a = np.zeros((n, n), np.float64)
    for v in range(n):
        for k in range(rp[v], rp[v + 1]):
            a[v, col[k]] += 1.0 if w is None else float(w[k])
    return a


def _membership(mate):
    """P from the definition: representatives in increasing order, a pair
    shares its representative's column."""
    n = len(mate)
    rep = np.array([v if mate[v] < 0 or v < mate[v] else mate[v] for v in range(n)], np.int64)
    reps = np.flatnonzero(rep == np.arange(n))
    cid = np.searchsorted(reps, rep)
    p = np.zeros((n, len(reps)), np.float64)
    p[np.arange(n), cid] = 1.0
    return p, cid


def _random_pairing(rng, g, kind):
    n = g.n
    mate = np.full(n, -1, np.int32)
    if kind == "matching":  # a maximal matching of the graph (greedy over a random edge order)
        lo, hi, _ = ref.undirected_edges(g)
        for e in rng.permutation(len(lo)):
            a, b = lo[e], hi[e]
            if mate[a] < 0 and mate[b] < 0:
                mate[a], mate[b] = b, a
    else:  # an arbitrary pairing, not necessarily along edges
        perm = rng.permutation(n)
        k = int(rng.integers(0, n // 2 + 1))
        for i in range(k):
            a, b = perm[2 * i], perm[2 * i + 1]
            mate[a], mate[b] = b, a
    return mate


def _check_structure(g, mate, out, w_int):
    cmap, crp, ccol, cw, cvw = out
    n = g.n
    p, cid = _membership(mate)
    nc = p.shape[1]
    assert len(crp) == nc + 1 and np.array_equal(cmap, cid)
    assert nc == n - int((mate >= 0).sum()) // 2
    c = _dense(nc, crp, ccol, cw)
    want = p.T @ _dense(n, g.row_ptr, g.col, g.w) @ p
    np.fill_diagonal(want, 0.0)
    if w_int:  # small integers: every fp32 sum is exact
        assert np.array_equal(c, want)
    else:
        absw = p.T @ np.abs(_dense(n, g.row_ptr, g.col, g.w)) @ p
        np.fill_diagonal(absw, 0.0)
        assert np.all(np.abs(c - want) <= 4 * np.finfo(np.float32).eps * absw + 1e-30)
    for v in range(nc):  # simple: no self-loops, no duplicates
        row = ccol[crp[v]:crp[v + 1]]
        assert v not in row and len(np.unique(row)) == len(row)
    # symmetric with bitwise-equal weights both ways
    assert np.array_equal(c, c.T)
    # rows list a neighbour once, in order of its first fine entry (a's row, then b's)
    reps = np.flatnonzero(np.array([m < 0 or v < m for v, m in enumerate(mate)]))
    for ci, a in enumerate(reps):
        seq = []
        for s in ([a] if mate[a] < 0 else [a, mate[a]]):
            for k in range(g.row_ptr[s], g.row_ptr[s + 1]):
                d = cid[g.col[k]]
                if d != ci and d not in seq:
                    seq.append(d)
        assert list(ccol[crp[ci]:crp[ci + 1]]) == seq
    vw = np.arange(1, n + 1, dtype=np.int64)
    assert np.array_equal(oracle.contract_graph(g, mate, vw)[4], (p.T @ vw).astype(np.int64))
    assert np.array_equal(cvw, (p.T @ np.ones(n)).astype(np.int64))


@pytest.mark.parametrize("kind", ["matching", "pairing"])
@pytest.mark.parametrize("wkind", ["int", "float", "signed"])
def test_coarse_graph_is_PtAP(kind, wkind):
    rng = np.random.default_rng({"int": 1, "float": 2, "signed": 3}[wkind] * 10 + (kind == "pairing"))
    for _ in range(40):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, n * (n - 1) // 2 + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**62))) if m > 0 else lmgen.from_edges(n, np.zeros((0, 2)), [])
        lo, hi, _ = ref.undirected_edges(g)
        if wkind == "int":
            w = rng.integers(1, 9, len(lo)).astype(np.float32)
        elif wkind == "float":
            w = rng.random(len(lo)).astype(np.float32)
        else:
            w = (rng.standard_normal(len(lo)) * 10.0 ** rng.integers(-3, 9, len(lo))).astype(np.float32)
        g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
        mate = _random_pairing(rng, g, kind)
        _check_structure(g, mate, oracle.contract_graph(g, mate), wkind == "int")


def test_unweighted_counts_fine_edges():
    g = lmgen.er(200, 1500, seed=4)
    mate, _ = oracle.local_max_graph(g, 1)
    cmap, crp, ccol, cw, _ = oracle.contract_graph(g, mate, unweighted=True)
    p, _ = _membership(mate)
    want = p.T @ (_dense(g.n, g.row_ptr, g.col, None)) @ p
    np.fill_diagonal(want, 0)
    assert np.array_equal(_dense(len(crp) - 1, crp, ccol, cw), want)


def test_identity_when_nothing_matched():
    g = lmgen.rgg(3000, 10.0, seed=3)
    out = oracle.contract_graph(g, np.full(g.n, -1, np.int32), vw=np.arange(g.n) * 3)
    cmap, crp, ccol, cw, cvw = out
    assert np.array_equal(cmap, np.arange(g.n)) and np.array_equal(crp, g.row_ptr)
    assert np.array_equal(ccol, g.col) and np.array_equal(cw, g.w) and np.array_equal(cvw, np.arange(g.n) * 3)


def test_ladder_contracts_to_path():
    """Ladder: rails u_i (weights p_i) and v_i (weights q_i), rungs u_i - v_i.
    Matched on the rungs it becomes the path of the rung pairs with weights
    p_i + q_i (two fine edges per coarse edge), vertex weights 2."""
    k = 50
    rng = np.random.default_rng(5)
    p = rng.integers(1, 100, k - 1)
    q = rng.integers(1, 100, k - 1)
    edges, w = [], []
    for i in range(k):
        edges.append([2 * i, 2 * i + 1])  # rung
        w.append(1000)
    for i in range(k - 1):
        edges += [[2 * i, 2 * i + 2], [2 * i + 1, 2 * i + 3]]
        w += [p[i], q[i]]
    g = lmgen.from_edges(2 * k, edges, w)
    mate = np.array([v ^ 1 for v in range(2 * k)], np.int32)
    cmap, crp, ccol, cw, cvw = oracle.contract_graph(g, mate)
    assert np.array_equal(cmap, np.arange(2 * k) // 2) and np.all(cvw == 2)
    path = lmgen.from_edges(k, [[i, i + 1] for i in range(k - 1)], (p + q).astype(np.float32))
    assert np.array_equal(crp, path.row_ptr) and np.array_equal(ccol, path.col) and np.array_equal(cw, path.w)


@pytest.mark.parametrize("k", [2, 3, 7])
def test_cycle_halves(k):
    """C_2k matched on alternate edges {2i, 2i+1} becomes C_k on the other
    edges; for k = 2 the two remaining edges are parallel and merge."""
    n = 2 * k
    edges = [[i, (i + 1) % n] for i in range(n)]
    w = np.arange(1, n + 1, dtype=np.float32)
    g = lmgen.from_edges(n, edges, w)
    mate = np.array([v ^ 1 for v in range(n)], np.int32)
    _, crp, ccol, cw, _ = oracle.contract_graph(g, mate)
    if k == 2:
        assert list(crp) == [0, 1, 2] and list(ccol) == [1, 0] and list(cw) == [w[1] + w[3]] * 2
    else:
        want = {}
        for i in range(k):  # fine edge {2i+1, 2i+2 mod n} joins coarse i and i+1 mod k
            a, b = i, (i + 1) % k
            want[(min(a, b), max(a, b))] = w[2 * i + 1]
        got = {(v, int(ccol[j])): float(cw[j]) for v in range(k) for j in range(crp[v], crp[v + 1])}
        assert len(got) == 2 * k
        for (a, b), x in want.items():
            assert got[(a, b)] == x and got[(b, a)] == x


def _golden():
    edges, w, mate, rows, vw, n = [], [], None, [], None, None
    for line in open(GOLDEN):
        t = line.split()
        if not t or t[0].startswith("#"):
            continue
        if t[0] == "edge":
            edges.append([int(t[1]), int(t[2])])
            w.append(float(t[3]))
        elif t[0] == "mate":
            mate = np.array([int(x) for x in t[1:]], np.int32)
        elif t[0] == "expect_n":
            n = int(t[1])
        elif t[0] == "expect_row":
            rows.append((int(t[1]), int(t[2]), float(t[3])))
        elif t[0] == "expect_vw":
            vw = [int(x) for x in t[1:]]
    return edges, np.array(w, np.float32), mate, n, rows, vw


def test_fp32_sum_order_hand_worked():
    edges, w, mate, nc, rows, vw = _golden()
    base = lmgen.from_edges(len(mate), edges, w)
    rng = np.random.default_rng(9)
    for trial in range(6):  # any entry order within the fine rows gives the same coarse graph
        col, ww = base.col.copy(), base.w.copy()
        if trial:
            for v in range(base.n):
                a, b = base.row_ptr[v], base.row_ptr[v + 1]
                pm = rng.permutation(b - a)
                col[a:b], ww[a:b] = col[a:b][pm], ww[a:b][pm]
        cmap, crp, ccol, cw, cvw = oracle.contract(base.n, base.row_ptr, col, ww, mate)
        assert len(crp) - 1 == nc and list(cvw) == vw
        for v, d, x in rows:
            j = crp[v] + list(ccol[crp[v]:crp[v + 1]]).index(d)
            assert cw[j] == np.float32(x)


def test_bad_pairings_rejected():
    g = lmgen.er(10, 20, seed=1)
    for bad in ([1, 0, 3, 2, 5, 4, 7, 6, 9, 9], [1, 0, 3, 2, 5, 4, 7, 6, 9, 10], [1, 2, 0, -1, -1, -1, -1, -1, -1, -1],
                [-2] + [-1] * 9):
        with pytest.raises(ValueError):
            oracle.contract_graph(g, np.array(bad, np.int32))


# ---- planted mistakes

CONTRACT_MUTANTS = {
    "matched_edge_kept": ("        if (d == c) continue;\n        if (pos[d] < 0) {",
                          "        if (pos[d] < 0) {"),
    "rep_is_larger_end": ("    if (mate[v] == LMO_NONE || v < mate[v]) cmap[v] = (int32_t)nc++;",
                          "    if (mate[v] == LMO_NONE || v > mate[v]) cmap[v] = (int32_t)nc++;"),
    "sum_in_scan_order": ("    qsort(cb, (size_t)ncb, sizeof(lmo_contrib), contrib_less);", ""),
    "partner_weight_dropped": ("(b == LMO_NONE ? 0 : (vw ? vw[b] : 1))", "0"),
    "parallel_edges_not_summed": ("        cw[cb[i].slot] += cb[i].w;", "        cw[cb[i].slot] = cb[i].w;"),
    "second_row_skipped": ("    for (int side = 0; side < 2; ++side) {", "    for (int side = 0; side < 1; ++side) {"),
}

_P64 = ctypes.POINTER(ctypes.c_int64)
_P32 = ctypes.POINTER(ctypes.c_int32)
_PF = ctypes.POINTER(ctypes.c_float)


def _run_pins_with(so_path):
    """Runs the pins above against a rebuilt oracle library; True if one fails."""
    lib = ctypes.CDLL(so_path)
    lib.lmo_contract.argtypes = [ctypes.c_int64, _P64, _P32, _PF, _P32, _P64, _P32, _P64, _P32, _PF, _P64, _P64]
    lib.lmo_contract.restype = ctypes.c_int64
    oracle._lib = lib  # this child process only
    try:
        test_ladder_contracts_to_path()
        for k in (2, 3, 7):
            test_cycle_halves(k)
        test_fp32_sum_order_hand_worked()
        for kind in ("matching", "pairing"):
            for wk in ("int", "signed"):
                test_coarse_graph_is_PtAP(kind, wk)
    except (AssertionError, ValueError, IndexError):
        return True
    return False


def _child(so, q):
    q.put(_run_pins_with(so))


@pytest.mark.parametrize("name", ["identity"] + sorted(CONTRACT_MUTANTS))
def test_contract_mutants_are_caught(tmp_path, name):
    src = open(SRC).read()
    if name != "identity":
        old, new = CONTRACT_MUTANTS[name]
        assert old in src, f"mutation anchor for {name} not found"
        src = src.replace(old, new, 1)
    path = tmp_path / f"{name}.c"
    path.write_text(src)
    so = str(tmp_path / f"{name}.so")
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", so, str(path)])
    ctx = mp.get_context("spawn")
    q = ctx.Queue()
    p = ctx.Process(target=_child, args=(so, q))
    p.start()
    p.join(120)
    caught = True
    if p.is_alive():
        p.kill()
        p.join()
    elif not q.empty():
        caught = bool(q.get())
    if name == "identity":
        assert not caught, "the unmodified oracle must pass the contraction pins"
    else:
        assert caught, f"pins did not catch mutant {name}"
