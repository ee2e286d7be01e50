"""LM_CHECK_GRAPH on device inputs and the error code of every entry point's
failure modes (the simple undirected graph of Section 1 is the input
contract).

The device check covers offsets, ids, self-loops, finite weights, symmetry
with equal weights both ways (a fingerprint of the entries against one of
their mirrors) and duplicate entries within a row (the contraction's
grouping kernels with every vertex free); each violation is planted in an
otherwise valid graph, on short rows and on rows long enough for the
device-memory grouping path, and valid graphs still solve to the oracle's
matching with the check on.
"""
import numpy as np
import pytest

import lmgen
import oracle

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


def _t(torch_dev, x, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(torch_dev)


def _solve_checked(ctx, torch_dev, rp, col, w, **kw):
    return ctx.match(_t(torch_dev, rp, np.int64), _t(torch_dev, col, np.int32),
                     None if w is None else _t(torch_dev, w, np.float32), seed=1, check_graph=True, **kw)


def _status(ctx, torch_dev, rp, col, w):
    import paper_1302_4587_amd as lm
    try:
        _solve_checked(ctx, torch_dev, rp, col, w)
    except lm.LMError as e:
        return e.status
    return 0


def _hub(deg, seed=3):
    """A hub joined to deg leaves, the leaves in a path: the hub's row is long."""
    rng = np.random.default_rng(seed)
    e = [[0, i] for i in range(1, deg + 1)] + [[i, i + 1] for i in range(1, deg)]
    return lmgen.from_edges(deg + 1, np.array(e), rng.random(len(e)).astype(np.float32))


def _graphs():
    return [("er 2000", lmgen.er(2000, 8000, seed=2)), ("hub 3000", _hub(3000)),
            ("rmat 13", lmgen.rmat(13, 16, seed=4, weights="uniform"))]


def test_valid_graphs_pass_and_match_oracle(ctx, torch_dev):
    for name, g in _graphs():
        print(f"case: checked solve {name}", flush=True)
        mate, st = _solve_checked(ctx, torch_dev, g.row_ptr, g.col, g.w)
        ref, _ = oracle.local_max_graph(g, 1)
        assert np.array_equal(mate.cpu().numpy(), ref), name
    g = lmgen.rmat(13, 16, seed=5)
    mate, _ = _solve_checked(ctx, torch_dev, g.row_ptr, g.col, None)  # unweighted
    gu = lmgen.Graph(g.n, g.row_ptr, g.col, np.ones(g.nnz, np.float32))
    assert np.array_equal(mate.cpu().numpy(), oracle.local_max_graph(gu, 1)[0])


def _entry_of(g, v, u):
    k = np.flatnonzero(g.col[g.row_ptr[v]:g.row_ptr[v + 1]] == u)
    return int(g.row_ptr[v] + k[0])


def test_asymmetric_weights_rejected(ctx, torch_dev):
    from paper_1302_4587_amd import _lib as L
    for name, g in _graphs():
        v = 0
        u = int(g.col[g.row_ptr[v]])
        w = g.w.copy()
        w[_entry_of(g, v, u)] += 0.25  # (v, u) and (u, v) now differ
        print(f"case: asymmetric weight {name}", flush=True)
        assert _status(ctx, torch_dev, g.row_ptr, g.col, w) == L.LM_EGRAPH, name
        w = g.w.copy()
        w[_entry_of(g, v, u)] = -0.0  # -0 against +0 is no violation
        w[_entry_of(g, u, v)] = 0.0
        assert _status(ctx, torch_dev, g.row_ptr, g.col, w) == 0


def test_missing_mirror_rejected(ctx, torch_dev):
    from paper_1302_4587_amd import _lib as L
    for name, g in _graphs():
        # move one entry of row 0 to another neighbour: (0, u') has no mirror and (u, 0) has none
        col = g.col.copy()
        v = int(np.flatnonzero(np.diff(g.row_ptr) > 0)[-1])  # the last vertex with an entry
        row = set(col[g.row_ptr[v]:g.row_ptr[v + 1]].tolist())
        cand = next(x for x in range(g.n) if x not in row and x != v)
        col[g.row_ptr[v]] = cand
        print(f"case: missing mirror {name}", flush=True)
        assert _status(ctx, torch_dev, g.row_ptr, col, g.w) == L.LM_EGRAPH, name


def test_duplicate_entries_rejected(ctx, torch_dev):
    """A symmetric duplicate (both mirrors twice) passes the fingerprint;
    the row grouping finds it, in a short row and in a long one."""
    from paper_1302_4587_amd import _lib as L
    two_hubs = lmgen.from_edges(2002, np.array([[0, 1]] + [[h, i] for h in (0, 1) for i in range(2, 2002)]),
                                np.random.default_rng(1).random(4001).astype(np.float32))
    for name, g, v in (("er 2000", lmgen.er(2000, 8000, seed=2), 5), ("hub 3000", _hub(3000), 0),
                       ("two hubs, duplicate between them", two_hubs, 0)):
        lo = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        keep = lo < g.col
        e = np.stack([lo[keep], g.col[keep]], 1)
        ww = g.w[keep]
        j = int(np.flatnonzero(e[:, 0] == v)[0])  # an edge of v, listed twice (two hubs: the edge 0-1)
        e2 = np.concatenate([e, e[j:j + 1]])
        w2 = np.concatenate([ww, ww[j:j + 1]])
        src = np.concatenate([e2[:, 0], e2[:, 1]])
        dst = np.concatenate([e2[:, 1], e2[:, 0]])
        wa = np.concatenate([w2, w2]).astype(np.float32)
        order = np.lexsort((dst, src))
        rp = np.zeros(g.n + 1, np.int64)
        np.cumsum(np.bincount(src, minlength=g.n), out=rp[1:])
        print(f"case: duplicate {name}", flush=True)
        assert _status(ctx, torch_dev, rp, dst[order], wa[order]) == L.LM_EGRAPH, name


def test_other_violations(ctx, torch_dev):
    from paper_1302_4587_amd import _lib as L
    g = lmgen.er(500, 2000, seed=9)
    col = g.col.copy()
    col[0] = g.n  # id out of range
    assert _status(ctx, torch_dev, g.row_ptr, col, g.w) == L.LM_EGRAPH
    col = g.col.copy()
    col[g.row_ptr[7]] = 7  # self-loop
    assert _status(ctx, torch_dev, g.row_ptr, col, g.w) == L.LM_EGRAPH
    for bad in (np.nan, np.inf, -np.inf):
        w = g.w.copy()
        w[3] = bad
        assert _status(ctx, torch_dev, g.row_ptr, g.col, w) == L.LM_EWEIGHT
    rp = g.row_ptr.copy()
    rp[10], rp[11] = rp[11], rp[10]  # offsets out of order
    assert _status(ctx, torch_dev, rp, g.col, g.w) == L.LM_EGRAPH


def test_batch_check(ctx, torch_dev):
    from paper_1302_4587_amd import _lib as L
    import paper_1302_4587_amd as lm
    b = lmgen.er_batch(16, seed=3, lg_lo=5.0, lg_hi=9.0)
    mate, _, _ = ctx.match_batch(b.vtx_off, _t(torch_dev, b.row_ptr, np.int64), _t(torch_dev, b.col, np.int32),
                                 _t(torch_dev, b.w, np.float32), seed0=2, check_graph=True)
    ref, _ = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=2)
    assert np.array_equal(mate.cpu().numpy(), ref)
    # the same local ids in two graphs must not pair up across graphs: graph 3's
    # entry weight changed breaks its own symmetry
    w = b.w.copy()
    k = int(b.row_ptr[b.vtx_off[3]])
    w[k] += 1.0
    with pytest.raises(lm.LMError) as e:
        ctx.match_batch(b.vtx_off, _t(torch_dev, b.row_ptr, np.int64), _t(torch_dev, b.col, np.int32),
                        _t(torch_dev, w, np.float32), seed0=2, check_graph=True)
    assert e.value.status == L.LM_EGRAPH


def test_flag_errors(ctx, torch_dev):
    from paper_1302_4587_amd import _lib as L
    import ctypes
    g = lmgen.er(100, 300, seed=1)
    rp, col, w = _t(torch_dev, g.row_ptr, np.int64), _t(torch_dev, g.col, np.int32), _t(torch_dev, g.w, np.float32)
    mate = _t(torch_dev, np.zeros(g.n), np.int32)
    csr = L.Csr(g.n, g.nnz, rp.data_ptr(), col.data_ptr(), w.data_ptr())
    dev = L.LM_IN_DEVICE | L.LM_OUT_DEVICE
    lib = L.load()
    h = ctx.handle
    assert lib.lm_match(h, ctypes.byref(csr), 1, mate.data_ptr(), dev | 0x10000, None, None) == L.LM_EINVAL
    assert lib.lm_match(h, ctypes.byref(csr), 1, mate.data_ptr(), dev | L.LM_ASYNC | L.LM_CHECK_GRAPH, None,
                        None) == L.LM_EINVAL
    assert lib.lm_match(h, ctypes.byref(csr), 1, None, dev, None, None) == L.LM_EINVAL
    bad = L.Csr(g.n, -1, rp.data_ptr(), col.data_ptr(), w.data_ptr())
    assert lib.lm_match(h, ctypes.byref(bad), 1, mate.data_ptr(), dev, None, None) == L.LM_EINVAL
    big = L.Csr(1 << 31, g.nnz, rp.data_ptr(), col.data_ptr(), w.data_ptr())
    assert lib.lm_match(h, ctypes.byref(big), 1, mate.data_ptr(), dev, None, None) == L.LM_EINVAL
    # still usable
    m, _ = ctx.match(rp, col, w, seed=1)
    assert np.array_equal(m.cpu().numpy(), oracle.local_max_graph(g, 1)[0])
