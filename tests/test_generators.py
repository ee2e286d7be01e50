"""The input generators keep the graph contract both sides rely on.

Oracle and HIP path consume the same generated arrays, and the method is
stated on a simple undirected graph (paper, Section 1): symmetric entries with
equal weights both ways, no self-loops, no duplicate edges. These checks run on
every family at small and medium sizes, plus determinism (a graph is a pure
function of its parameters and seed) and the weight domains of the recipes.
"""
import numpy as np
import pytest

import lmgen


def _check_contract(g, sorted_rows=True):
    n, rp, col, w = g.n, g.row_ptr, g.col, g.w
    assert rp.dtype == np.int64 and col.dtype == np.int32 and w.dtype == np.float32
    assert rp.shape == (n + 1,) and rp[0] == 0 and rp[-1] == len(col) == len(w)
    assert (np.diff(rp) >= 0).all()
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    assert ((col >= 0) & (col < n)).all(), "ids out of range"
    assert (rows != col).all(), "self-loop"
    if sorted_rows:
        same = rows[1:] == rows[:-1]
        assert (col[1:][same] > col[:-1][same]).all(), "rows not strictly increasing"
    key = rows * n + col
    assert len(np.unique(key)) == len(key), "duplicate entry"
    # symmetry with equal weights: the entry (u, v) exists for every (v, u) and
    # carries the same weight bits
    tkey = col.astype(np.int64) * n + rows
    o1, o2 = np.argsort(key), np.argsort(tkey)
    assert np.array_equal(key[o1], tkey[o2]), "asymmetric"
    assert np.array_equal(w[o1].view(np.uint32), w[o2].view(np.uint32)), "unequal weights"
    assert np.isfinite(w).all()


CASES = [
    ("er small", lambda: lmgen.er(300, 900, seed=3)),
    ("er config", lambda: lmgen.er(4096, 32768, seed=1)),
    ("er empty", lambda: lmgen.er(50, 0, seed=1)),
    ("er dense", lambda: lmgen.er(40, 780, seed=2)),
    ("rgg 2^12", lambda: lmgen.rgg(1 << 12, 10.0, 1)),
    ("rgg 2^18", lambda: lmgen.rgg(1 << 18, 10.0, 1)),
    ("rmat 10", lambda: lmgen.rmat(10, 16, seed=1)),
    ("rmat 16", lambda: lmgen.rmat(16, 16, seed=1)),
    ("rmat 14 uniform", lambda: lmgen.rmat(14, 16, seed=2, weights="uniform")),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_generator_contract(name, make):
    g = make()
    _check_contract(g)
    h = make()
    assert np.array_equal(g.row_ptr, h.row_ptr) and np.array_equal(g.col, h.col)
    assert np.array_equal(g.w.view(np.uint32), h.w.view(np.uint32)), "not deterministic"


def test_weight_domains():
    g = lmgen.er(2000, 8000, seed=5)
    # k * 2^-24, k in [1, 2^24]: (0, 1], exact multiples of 2^-24
    assert (g.w > 0).all() and (g.w <= 1).all()
    k = g.w.astype(np.float64) * 2.0**24
    assert np.array_equal(k, np.round(k))
    u = lmgen.er(2000, 8000, seed=5, weights="unit")
    assert (u.w == 1.0).all()
    assert (lmgen.rmat(12, 16, seed=1).w == 1.0).all()
    r = lmgen.rgg(1 << 14, 10.0, 3)
    rad = lmgen.rgg_radius(1 << 14, 10.0)
    # w = fp32(1 - d) with d < r
    assert (r.w >= np.float32(1.0 - rad) - 1e-7).all() and (r.w <= 1.0).all()


def test_rgg_average_degree():
    g = lmgen.rgg(1 << 18, 10.0, 1)
    assert 9.5 < g.nnz / g.n < 10.5


def test_rmat_edge_factor_and_hubs():
    g = lmgen.rmat(16, 16, seed=1)
    # at most edge_factor * 2^scale samples, so m <= 16 n; duplicates and
    # self-loops removed; low ids are hubs (no permutation)
    assert g.m <= 16 * g.n
    deg = np.diff(g.row_ptr)
    assert deg[0] == deg.max()
    assert (deg == 0).sum() > 0


def test_batch_contract():
    b = lmgen.er_batch(40, seed=3, lg_lo=4.0, lg_hi=10.0)
    assert b.vtx_off[0] == 0 and (np.diff(b.vtx_off) > 0).all()
    assert b.row_ptr[0] == 0 and b.row_ptr[-1] == len(b.col)
    for k in range(b.graphs):
        g = b.graph(k)
        _check_contract(g)
        d = g.nnz / g.n
        assert 3.0 <= d <= 33.0  # average degree drawn from U[4, 32] (rounded edge counts)
    c = lmgen.er_batch(40, seed=3, lg_lo=4.0, lg_hi=10.0)
    assert np.array_equal(b.col, c.col) and np.array_equal(b.vtx_off, c.vtx_off)


def test_shuffled_rows_keep_the_contract_unsorted():
    g = lmgen.er(500, 3000, seed=9)
    rng = np.random.default_rng(0)
    col, w = g.col.copy(), g.w.copy()
    for v in range(g.n):
        a, b = g.row_ptr[v], g.row_ptr[v + 1]
        p = rng.permutation(b - a) + a
        col[a:b], w[a:b] = col[p], w[p]
    _check_contract(lmgen.Graph(g.n, g.row_ptr, col, w), sorted_rows=False)
