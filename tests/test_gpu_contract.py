"""Contraction by a matching on the GPU (lm_contract) against the oracle,
element by element: cmap, coarse row_ptr, col, weights (bit for bit) and
vertex weights.

Short coarse rows (deg(a) + deg(b) <= 512) are merged in LDS tiles, longer
ones through device-memory hash tables; the cases below cover both, rows cut
into several tiles, pairings that are not matchings, host and device
buffers, and a multilevel loop (match, contract, match the coarse graph...).
"""
import numpy as np
import pytest

import lmgen
import oracle
from tests import _pyref as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def ctx(torch_dev):
    import paper_1302_4587_amd as lm
    c = lm.Context(0)
    yield c
    c.close()


def _gpu_contract(ctx, torch_dev, g, mate, vw=None, unweighted=False, host=False):
    import torch
    w = None if unweighted else g.w
    if host:
        out = ctx.contract(g.row_ptr, g.col, w, mate, vw)
        return out[:5], out[5]
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(torch_dev)
    out = ctx.contract(t(g.row_ptr, np.int64), t(g.col, np.int32), None if w is None else t(w, np.float32),
                       t(mate, np.int32), None if vw is None else t(vw, np.int64))
    torch.cuda.synchronize()
    return tuple(x.cpu().numpy() for x in out[:5]), out[5]


def _compare(got, want, what):
    names = ("cmap", "row_ptr", "col", "w", "vwgt")
    for nm, a, b in zip(names, got, want):
        if nm == "w":
            a, b = a.view(np.uint32), np.asarray(b, np.float32).view(np.uint32)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b) if a.shape == b.shape else None
            raise AssertionError(f"{what}: {nm} differs (shapes {a.shape} vs {b.shape}, first at "
                                 f"{None if bad is None else bad[:5]})")


def _case(ctx, torch_dev, g, mate, what, vw=None, unweighted=False, host=False):
    print(f"case: contract {what} n={g.n} nnz={g.nnz} host={host}", flush=True)
    want = oracle.contract(g.n, g.row_ptr, g.col, None if unweighted else g.w, mate, vw)
    got, st = _gpu_contract(ctx, torch_dev, g, mate, vw, unweighted, host)
    _compare(got, want, what)
    return st


def _symmetric(g):
    """Every entry (v, u, w) has its mirror (u, v, w), weights bit for bit."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    a = np.lexsort((g.col, rows))
    b = np.lexsort((rows, g.col))
    return (np.array_equal(rows[a], g.col[b]) and np.array_equal(g.col[a], rows[b])
            and np.array_equal(g.w[a].view(np.uint32), g.w[b].view(np.uint32)))


def _star(leaves, w=None):
    e = np.array([[0, i] for i in range(1, leaves + 1)])
    return lmgen.from_edges(leaves + 1, e, np.linspace(0.1, 1.0, leaves) if w is None else w)


def test_contract_matchings_equal_oracle(ctx, torch_dev):
    cases = [
        ("er 4096 uniform", lmgen.er(4096, 32768, seed=1), False),
        ("rgg 40000", lmgen.rgg(40000, 10.0, seed=2), False),
        ("rmat 14 unweighted", lmgen.rmat(14, 16, seed=8), True),
        ("rmat 13 uniform", lmgen.rmat(13, 16, seed=4, weights="uniform"), False),
        ("er 20000 unit", lmgen.er(20000, 160000, seed=7, weights="unit"), False),
        ("star 5000 (one long row)", _star(5000), False),
        ("increasing path 301", lmgen.from_edges(302, [[i, i + 1] for i in range(301)], np.arange(1, 302)), False),
        ("single edge", lmgen.from_edges(2, [[0, 1]], [0.5]), False),
        ("isolated vertices only", lmgen.from_edges(7, np.zeros((0, 2), np.int64), np.zeros(0)), False),
    ]
    long_seen = 0
    for name, g, unw in cases:
        gg = g if not unw else lmgen.from_edges(g.n, np.stack(ref.undirected_edges(g)[:2], 1),
                                                np.ones(g.nnz // 2, np.float32))
        mate, _ = oracle.local_max_graph(gg, 3)
        st = _case(ctx, torch_dev, g, mate, name, unweighted=unw)
        long_seen += st.long_rows
        if name.startswith("star"):
            assert st.long_rows == 1
    assert long_seen >= 2


@pytest.mark.parametrize("wkind", ["uniform", "tied", "signed"])
def test_contract_random_pairings(ctx, torch_dev, wkind):
    """Pairings that are not matchings of the graph (any involution)."""
    rng = np.random.default_rng({"uniform": 71, "tied": 72, "signed": 73}[wkind])
    for it in range(6):
        n = int(rng.integers(2, 6000))
        m = int(rng.integers(1, min(n * (n - 1) // 2, 40 * n) + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
        if wkind != "uniform":
            lo, hi, _ = ref.undirected_edges(g)
            w = (rng.integers(1, 4, len(lo)).astype(np.float32) if wkind == "tied" else
                 (rng.standard_normal(len(lo)) * 10.0 ** rng.integers(-3, 9, len(lo))).astype(np.float32))
            g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
        mate = np.full(n, -1, np.int32)
        perm = rng.permutation(n)
        k = int(rng.integers(0, n // 2 + 1))
        mate[perm[0:2 * k:2]] = perm[1:2 * k:2]
        mate[perm[1:2 * k:2]] = perm[0:2 * k:2]
        vw = rng.integers(1, 1000, n).astype(np.int64)
        _case(ctx, torch_dev, g, mate, f"{wkind} pairing it={it}", vw=vw)


def test_contract_long_and_tiled_rows(ctx, torch_dev):
    """Hubs matched to each other (one coarse row of both hub rows), hubs
    joined to many pairs (four fine edges per coarse edge), rows just below
    and above the LDS bound, and a chunk whose rows fill several tiles."""
    rng = np.random.default_rng(5)
    edges = []
    L = 3000
    # hubs 0 and 1, leaves 2..2L+1 matched in pairs (2i, 2i+1); both hubs see both leaves of a pair
    edges.append([0, 1])
    for v in range(2, 2 * L + 2):
        edges += [[0, v], [1, v]]
    for i in range(2, 2 * L + 2, 2):
        edges.append([i, i + 1])
    # rows of degree 255..258 around the bound 512 = deg(a) + deg(b)
    base = 2 * L + 2
    for d in (250, 255, 256, 257, 262):
        a, b = base, base + 1
        edges.append([a, b])
        for j in range(d - 1):
            edges += [[a, base + 2 + j], [b, base + 2 + d + j]]
        base += 2 + 2 * d
    n = base
    w = rng.random(len(edges)).astype(np.float32)
    g = lmgen.from_edges(n, np.array(edges), w)
    mate = np.full(n, -1, np.int32)
    mate[0], mate[1] = 1, 0
    for i in range(2, 2 * L + 2, 2):
        mate[i], mate[i + 1] = i + 1, i
    st = _case(ctx, torch_dev, g, mate, "hubs and bounds")
    assert st.long_rows >= 1
    # the same with the greedy-free matching of the library's own solve
    import torch
    mate2, _ = ctx.match(torch.from_numpy(g.row_ptr).to(torch_dev), torch.from_numpy(g.col).to(torch_dev),
                         torch.from_numpy(g.w).to(torch_dev), seed=2)
    _case(ctx, torch_dev, g, mate2.cpu().numpy(), "hubs and bounds, solved")


def test_contract_bucket_overflow_falls_back(ctx, torch_dev):
    """A long row whose coarse neighbours all hash into one bucket (more
    entries than a bucket holds in LDS): the long rows take the per-row
    table path, with the same result."""
    nb = 3
    want = 1100
    leaves = []
    v = 2
    while len(leaves) < want:
        d = v - 1  # the coarse id of leaf v once vertices 0 and 1 are one pair
        if (((d * 0x9E3779B1) & 0xFFFFFFFF) * nb) >> 32 == 0:
            leaves.append(v)
        v += 1
    n = v
    edges = [[0, 1]] + [[0, x] for x in leaves]
    w = np.random.default_rng(3).random(len(edges)).astype(np.float32)
    g = lmgen.from_edges(n, np.array(edges), w)
    mate = np.full(n, -1, np.int32)
    mate[0], mate[1] = 1, 0
    assert (g.row_ptr[1] - g.row_ptr[0]) + (g.row_ptr[2] - g.row_ptr[1]) == want + 2  # bound 1102: 3 buckets
    st = _case(ctx, torch_dev, g, mate, "bucket overflow")
    assert st.long_rows == 1 and st.table_rows == 1


def test_contract_host_buffers(ctx, torch_dev):
    g = lmgen.rmat(12, 16, seed=3, weights="uniform")
    mate, _ = oracle.local_max_graph(g, 1)
    _case(ctx, torch_dev, g, mate, "rmat 12 host", vw=np.arange(g.n, dtype=np.int64) + 5, host=True)
    _case(ctx, torch_dev, g, np.full(g.n, -1, np.int32), "nothing matched, host", host=True)


def test_multilevel_coarsening(ctx, torch_dev):
    """Match, contract, match the coarse graph... (the multilevel use): every
    level equals the oracle's, and the coarse graphs stay simple and
    symmetric with equal weights both ways."""
    import torch
    for name, g in (("rgg 60000", lmgen.rgg(60000, 10.0, seed=4)), ("er 30000", lmgen.er(30000, 200000, seed=6))):
        vw = np.ones(g.n, np.int64)
        cur_g, cur_vw = g, vw
        for level in range(6):
            if cur_g.nnz == 0:
                break
            rp, col, w = (torch.from_numpy(x).to(torch_dev) for x in (cur_g.row_ptr, cur_g.col, cur_g.w))
            mate_t, _ = ctx.match(rp, col, w, seed=level + 1)
            mate = mate_t.cpu().numpy()
            ref_mate, _ = oracle.local_max_graph(cur_g, level + 1)
            assert np.array_equal(mate, ref_mate), f"{name} level {level}: matching"
            want = oracle.contract(cur_g.n, cur_g.row_ptr, cur_g.col, cur_g.w, mate, cur_vw)
            print(f"case: multilevel {name} level={level} n={cur_g.n} nnz={cur_g.nnz}", flush=True)
            out = ctx.contract(rp, col, w, mate_t, torch.from_numpy(cur_vw).to(torch_dev))
            torch.cuda.synchronize()
            got = tuple(x.cpu().numpy() for x in out[:5])
            _compare(got, want, f"{name} level {level}")
            _, crp, ccol, cw, cvw = got
            cg = lmgen.Graph(len(crp) - 1, crp, ccol, cw)
            assert _symmetric(cg), f"{name} level {level}: coarse graph not symmetric"
            assert int(cvw.sum()) == g.n
            cur_g, cur_vw = cg, cvw


def test_contract_errors(ctx, torch_dev):
    import paper_1302_4587_amd as lm
    g = lmgen.er(100, 300, seed=1)
    mate, _ = oracle.local_max_graph(g, 1)
    bad = mate.copy()
    i = int(np.flatnonzero(bad >= 0)[0])
    bad[i] = -1  # no longer an involution
    with pytest.raises(lm.LMError) as e:
        _gpu_contract(ctx, torch_dev, g, bad)
    assert e.value.status == lm._lib.LM_EINVAL
    col = g.col.copy()
    col[5] = g.n + 3  # neighbour id out of range
    g2 = lmgen.Graph(g.n, g.row_ptr, col, g.w)
    with pytest.raises(lm.LMError) as e:
        _gpu_contract(ctx, torch_dev, g2, mate)
    assert e.value.status == lm._lib.LM_EGRAPH
    rp = g.row_ptr.copy()
    rp[-1] -= 1  # last offset is not nnz
    g3 = lmgen.Graph(g.n, rp, g.col, g.w)
    with pytest.raises(lm.LMError) as e:
        _gpu_contract(ctx, torch_dev, g3, mate)
    assert e.value.status == lm._lib.LM_EGRAPH
    # five fine edges between two pairs: duplicate entries
    dup = lmgen.Graph(4, np.array([0, 6, 7, 8, 9], np.int64), np.array([2, 2, 2, 3, 3, 1, 0, 0, 0], np.int32),
                      np.ones(9, np.float32))
    with pytest.raises(lm.LMError) as e:
        _gpu_contract(ctx, torch_dev, dup, np.array([1, 0, 3, 2], np.int32))
    assert e.value.status == lm._lib.LM_EGRAPH
    # the context still works afterwards
    _case(ctx, torch_dev, g, mate, "after errors")
