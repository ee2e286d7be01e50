"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

mate[] must be identical element by element (integer work: tolerance 0), and
the per-phase log (live entries, live rows, matched edges) must equal the
oracle's iteration log, because both run synchronous phases of the same
method (paper, Section 2, sequential model; Lemma 1 counts).
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


def _dev(torch_dev, g):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(torch_dev),
            torch.from_numpy(np.ascontiguousarray(g.col)).to(torch_dev),
            torch.from_numpy(np.ascontiguousarray(g.w)).to(torch_dev))


def _solve(ctx, torch_dev, g, seed, host=False, **kw):
    if host:
        mate, st = ctx.match(g.row_ptr, g.col, g.w, seed=seed, **kw)
        return np.asarray(mate), st
    rp, col, w = _dev(torch_dev, g)
    mate, st = ctx.match(rp, col, w, seed=seed, **kw)
    return mate.cpu().numpy(), st


def _assert_parity(g, seed, mate, st, what=""):
    ref_mate, ref_log = oracle.local_max_graph(g, seed)
    if not np.array_equal(mate, ref_mate):
        bad = np.flatnonzero(mate != ref_mate)
        raise AssertionError(f"{what}: mate differs at {len(bad)} vertices, first {bad[:5]}")
    assert st.phases == len(ref_log), f"{what}: phases {st.phases} vs oracle {len(ref_log)}"
    assert st.matched_edges == int((ref_mate >= 0).sum()) // 2
    L = min(len(st.log), len(ref_log))
    assert np.array_equal(st.log[:L, 0], 2 * ref_log[:L, 0]), f"{what}: live entries differ"
    assert np.array_equal(st.log[:L, 1], ref_log[:L, 1]), f"{what}: live rows differ"
    assert np.array_equal(st.log[:L, 2], ref_log[:L, 2]), f"{what}: matched per phase differ"


def test_config1_er_4096(ctx, torch_dev):
    print("case: ER n=4096 m=32768 seed=1", flush=True)
    g = lmgen.er(4096, 32768, seed=1)
    mate, st = _solve(ctx, torch_dev, g, 1)
    _assert_parity(g, 1, mate, st, "config1")
    assert np.array_equal(mate, ref.greedy(g, 1))


DENORMALS = np.array([-2.0**-140, -2.0**-149, -0.0, 0.0, 2.0**-149, 2.0**-148, 2.0**-130, 2.0**-127,
                      2.0**-126, 1e-30], dtype=np.float32)


@pytest.mark.parametrize("wkind", ["uniform", "tied", "unit", "signed", "denormal"])
def test_random_small_graphs(ctx, torch_dev, wkind):
    rng = np.random.default_rng({"uniform": 11, "tied": 12, "unit": 13, "signed": 14, "denormal": 15}[wkind])
    for it in range(40):
        n = int(rng.integers(1, 3000))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 12 * n) + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
        if wkind != "uniform":
            lo, hi, _ = ref.undirected_edges(g)
            if wkind == "tied":
                w = rng.integers(1, 4, len(lo)).astype(np.float32)
            elif wkind == "unit":
                w = np.ones(len(lo), np.float32)
            elif wkind == "denormal":  # subnormal weights: ordered by value, never flushed to zero
                w = rng.choice(DENORMALS, len(lo))
            else:
                w = rng.choice(np.array([-2.5, -0.0, 0.0, 1e-30, 3.0], np.float32), len(lo))
            g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        print(f"case: {wkind} it={it} n={n} m={m} seed={seed}", flush=True)
        mate, st = _solve(ctx, torch_dev, g, seed)
        _assert_parity(g, seed, mate, st, f"{wkind} it={it}")


def _star(k, center=0, n=None, unit=False, rng=None):
    n = n or k + 1
    leaves = [i for i in range(n) if i != center][:k]
    e = np.array([[center, x] for x in leaves])
    w = np.ones(k) if unit else (rng.random(k) if rng is not None else np.linspace(0.1, 1, k))
    return lmgen.from_edges(n, e, w)


def test_hubs_and_long_rows(ctx, torch_dev):
    rng = np.random.default_rng(5)
    cases = [
        ("star 5000", _star(5000, rng=rng)),
        ("star 5000 unit", _star(5000, unit=True)),
        ("star 2048", _star(2048, rng=rng)),
        ("star 2049", _star(2049, rng=rng)),
        ("rmat 14", lmgen.rmat(14, 16, seed=3)),
        ("rmat 15 uniform", lmgen.rmat(15, 16, seed=4, weights="uniform")),
    ]
    for name, g in cases:
        for seed in (1, 99):
            print(f"case: {name} seed={seed}", flush=True)
            mate, st = _solve(ctx, torch_dev, g, seed)
            _assert_parity(g, seed, mate, st, name)


def _unit(g):
    return lmgen.Graph(g.n, g.row_ptr, g.col, np.ones(g.nnz, np.float32))


def test_unweighted_equals_unit_weights(ctx, torch_dev):
    """w=None (an unweighted graph: every edge weighs 1, Section 1) takes the
    kernels that neither load nor store weights; the result must equal the
    oracle on the same graph with unit weights, and the weighted path fed an
    all-ones array."""
    import torch
    rng = np.random.default_rng(21)
    cases = [("rmat 14", lmgen.rmat(14, 16, seed=3)), ("rmat 13 seed 8", lmgen.rmat(13, 16, seed=8)),
             ("star 5000", _unit(_star(5000, unit=True))), ("star 2049", _unit(_star(2049, unit=True))),
             ("rgg 30000", _unit(lmgen.rgg(30000, 10.0, seed=9))),
             ("er 20000", lmgen.er(20000, 160000, seed=7, weights="unit"))]
    for it in range(24):
        n = int(rng.integers(1, 3000))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 12 * n) + 1))
        cases.append((f"er it={it} n={n} m={m}", lmgen.er(n, m, int(rng.integers(1, 2**62)), weights="unit")))
    for name, g in cases:
        for seed in (1, 12345):
            print(f"case: unweighted {name} seed={seed}", flush=True)
            rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(torch_dev)
            col = torch.from_numpy(np.ascontiguousarray(g.col)).to(torch_dev)
            mate, st = ctx.match(rp, col, None, seed=seed)
            _assert_parity(g, seed, mate.cpu().numpy(), st, f"unweighted {name}")
    # host inputs, validation and the captured-graph mode without a weight array
    g = lmgen.rmat(12, 16, seed=5)
    print("case: unweighted host inputs, checks, hip graph", flush=True)
    mate, st = ctx.match(g.row_ptr, g.col, None, seed=7, check_graph=True)
    _assert_parity(g, 7, np.asarray(mate), st, "unweighted host")
    rp = torch.from_numpy(g.row_ptr).to(torch_dev)
    col = torch.from_numpy(g.col).to(torch_dev)
    mate, st = ctx.match(rp, col, None, seed=7, hip_graph=True)
    _assert_parity(g, 7, mate.cpu().numpy(), st, "unweighted hip graph")
    # an entry array that is not 16-byte aligned (a view one entry in) takes
    # the one-graph kernel's entry-by-entry loads
    big = lmgen.rmat(13, 16, seed=6)
    colx = torch.zeros(big.nnz + 1, dtype=torch.int32, device=torch_dev)
    colx[1:] = torch.from_numpy(big.col).to(torch_dev)
    print("case: unweighted unaligned col", flush=True)
    mate, st = ctx.match(torch.from_numpy(big.row_ptr).to(torch_dev), colx[1:], None, seed=3)
    _assert_parity(big, 3, mate.cpu().numpy(), st, "unweighted unaligned col")
    # tuning shapes cut rows at other workgroup boundaries
    base = ctx.tuning()
    try:
        for be in (4096, 65536):
            ctx.set_tuning(block_entries=be, grid_per_cu=1)
            print(f"case: unweighted tuning be={be}", flush=True)
            mate, st = ctx.match(rp, col, None, seed=7)
            _assert_parity(g, 7, mate.cpu().numpy(), st, f"unweighted tuning {be}")
    finally:
        ctx.set_tuning(**base)
    # a batch without a weight array
    b = lmgen.er_batch(64, seed=5, lg_lo=5.0, lg_hi=11.0, weights="unit")
    print("case: unweighted batch of 64", flush=True)
    mate, st, gph = ctx.match_batch(b.vtx_off, b.row_ptr, b.col, None, seed0=3)
    ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=3)
    assert np.array_equal(np.asarray(mate), ref_mate)
    assert np.array_equal(gph, ref_ph)


@pytest.mark.parametrize("block_entries", [2048, 4096, 65536])
def test_tuning_invariance(ctx, torch_dev, block_entries):
    """Range sizes and launch shapes change where rows are cut between
    workgroups, never the result."""
    gs = [lmgen.er(20000, 160000, seed=7), lmgen.rmat(13, 16, seed=8), lmgen.rgg(30000, 10.0, seed=9),
          _star(30000, unit=True)]
    base = ctx.tuning()
    try:
        for gp in sorted({1, base["grid_per_cu"]}):
            for pps in (1, 8):
                ctx.set_tuning(block_entries=block_entries, grid_per_cu=gp, phases_per_sync=pps)
                for i, g in enumerate(gs):
                    print(f"case: tuning be={block_entries} gp={gp} pps={pps} graph={i}", flush=True)
                    mate, st = _solve(ctx, torch_dev, g, 3)
                    _assert_parity(g, 3, mate, st, f"tuning {block_entries}/{gp}/{pps} graph {i}")
    finally:
        ctx.set_tuning(**base)


@pytest.mark.parametrize("kind", ["rmat22", "rgg22"])
def test_large_graph_matched_bits(ctx, torch_dev, kind):
    """At 2^22 vertices and more the compactions of one graph read the matched
    state from bits when k_init's sample finds the neighbour ids scattered
    (R-MAT) and from the byte array when they are local (RGG): both equal the
    oracle, in the host-polled and the captured solve."""
    import torch
    g = lmgen.rmat(22, 16, seed=3) if kind == "rmat22" else lmgen.rgg(1 << 22, 10.0, seed=3)
    unw = kind == "rmat22"
    gg = lmgen.Graph(g.n, g.row_ptr, g.col, np.ones(g.nnz, np.float32)) if unw else g
    ref_mate, ref_log = oracle.local_max_graph(gg, 2)
    rp, col = (torch.from_numpy(x).to(torch_dev) for x in (g.row_ptr, g.col))
    w = None if unw else torch.from_numpy(g.w).to(torch_dev)
    for kw in ({}, {"hip_graph": True}):
        print(f"case: {kind} {kw}", flush=True)
        mate, st = ctx.match(rp, col, w, seed=2, **kw)
        assert np.array_equal(mate.cpu().numpy(), ref_mate), f"{kind} {kw}"
        assert st.phases == len(ref_log)


def test_edge_cases(ctx, torch_dev):
    cases = [
        ("isolated", lmgen.from_edges(7, np.zeros((0, 2)), np.zeros(0))),
        ("single edge", lmgen.from_edges(2, [[0, 1]], [0.5])),
        ("single edge + isolated", lmgen.from_edges(5, [[3, 1]], [2.0])),
        ("triangle", lmgen.from_edges(3, [[0, 1], [1, 2], [0, 2]], [0.5, 0.9, 0.7])),
        ("disjoint", lmgen.from_edges(200, [[2 * i, 2 * i + 1] for i in range(100)], np.linspace(1, 2, 100))),
        ("increasing path 301", lmgen.from_edges(302, [[i, i + 1] for i in range(301)], np.arange(1, 302))),
        ("all ties clique 40", lmgen.from_edges(40, [[i, j] for i in range(40) for j in range(i + 1, 40)],
                                               np.ones(780))),
    ]
    for name, g in cases:
        print(f"case: {name}", flush=True)
        mate, st = _solve(ctx, torch_dev, g, 5)
        _assert_parity(g, 5, mate, st, name)
    g = cases[5][1]
    mate, st = _solve(ctx, torch_dev, g, 5)
    assert st.phases == 151  # ceil(301 / 2): one edge per phase


def test_empty_graph(ctx, torch_dev):
    import torch
    rp = torch.zeros(1, dtype=torch.int64, device=torch_dev)
    col = torch.zeros(0, dtype=torch.int32, device=torch_dev)
    w = torch.zeros(0, dtype=torch.float32, device=torch_dev)
    mate, st = ctx.match(rp, col, w, seed=1)
    assert mate.numel() == 0 and st.phases == 0


def test_entry_order_and_host_inputs(ctx, torch_dev):
    g = lmgen.er(5000, 40000, seed=21)
    rng = np.random.default_rng(0)
    col, w = g.col.copy(), g.w.copy()
    for v in range(g.n):
        a, b = g.row_ptr[v], g.row_ptr[v + 1]
        p = rng.permutation(b - a)
        col[a:b] = col[a:b][p]
        w[a:b] = w[a:b][p]
    shuffled = lmgen.Graph(g.n, g.row_ptr, col, w)
    print("case: shuffled rows, device", flush=True)
    m1, _ = _solve(ctx, torch_dev, g, 2)
    m2, _ = _solve(ctx, torch_dev, shuffled, 2)
    print("case: host inputs", flush=True)
    m3, st3 = _solve(ctx, torch_dev, g, 2, host=True)
    assert np.array_equal(m1, m2) and np.array_equal(m1, m3)
    _assert_parity(g, 2, m3, st3, "host")


def test_repeatable(ctx, torch_dev):
    g = lmgen.rmat(14, 16, seed=31)
    outs = []
    for i in range(10):
        print(f"case: repeat {i}", flush=True)
        outs.append(_solve(ctx, torch_dev, g, 4)[0])
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def test_checks_and_errors(ctx, torch_dev):
    import paper_1302_4587_amd as lm
    from paper_1302_4587_amd import _lib as L
    g = lmgen.er(100, 300, seed=2)
    bad = g.col.copy()
    bad[0] = 0  # row 0 gets a self-loop
    with pytest.raises(lm.LMError) as e:
        ctx.match(*_dev(torch_dev, lmgen.Graph(g.n, g.row_ptr, bad, g.w)), seed=1, check_graph=True)
    assert e.value.status == L.LM_EGRAPH
    badw = g.w.copy()
    badw[3] = np.nan
    with pytest.raises(lm.LMError) as e:
        ctx.match(*_dev(torch_dev, lmgen.Graph(g.n, g.row_ptr, g.col, badw)), seed=1, check_graph=True)
    assert e.value.status == L.LM_EWEIGHT
    # host checks: asymmetric weight
    w2 = g.w.copy()
    w2[5] += 1.0
    with pytest.raises(lm.LMError) as e:
        ctx.match(g.row_ptr, g.col, w2, seed=1, check_graph=True)
    assert e.value.status == L.LM_EGRAPH
    # bad offsets on the device: the init kernel flags them
    rp = g.row_ptr.copy()
    rp[-1] += 1
    import torch
    with pytest.raises(lm.LMError) as e:
        ctx.match(torch.from_numpy(rp).to(torch_dev), *(_dev(torch_dev, g)[1:]), seed=1)
    assert e.value.status == L.LM_EGRAPH
    # the context still works after errors
    mate, st = _solve(ctx, torch_dev, g, 1)
    _assert_parity(g, 1, mate, st, "after errors")


def test_budget_too_small(torch_dev):
    import paper_1302_4587_amd as lm
    from paper_1302_4587_amd import _lib as L
    g = lmgen.er(4096, 32768, seed=1)
    with lm.Context(0, hbm_budget_bytes=1 << 16) as small:
        with pytest.raises(lm.LMError) as e:
            small.match(*_dev(torch_dev, g), seed=1)
        assert e.value.status == L.LM_ETOOBIG


def test_profile_stats(ctx, torch_dev):
    g = lmgen.rgg(100000, 10.0, seed=3)
    saved = ctx.tuning()
    try:
        # every phase through the phase kernels (no hand-over to the tail kernel)
        ctx.set_tuning(tail_entries=0)
        mate, st = _solve(ctx, torch_dev, g, 1, profile=True)
        _assert_parity(g, 1, mate, st, "profile")
        assert st.kernel_launches["init"] == 1 and st.kernel_launches["argmax"] == 1
        assert st.kernel_launches["mutual"] >= st.phases and st.kernel_launches["compact"] >= st.phases
        assert st.kernel_launches["tail"] == 0
        assert all(st.kernel_ms[k] > 0 for k in ("init", "argmax", "mutual", "compact"))
        assert st.bytes_alg > 8 * g.nnz
        # the graph is below the hand-over size: one tail launch runs every phase
        ctx.set_tuning(tail_entries=1 << 20)
        mate, st = _solve(ctx, torch_dev, g, 1, profile=True)
        _assert_parity(g, 1, mate, st, "profile with tail")
        assert st.kernel_launches["tail"] == 1 and st.kernel_ms["tail"] > 0
        assert st.kernel_launches["mutual"] == 0 and st.kernel_launches["compact"] == 0
        assert st.kernel_bytes["tail"] > 8 * g.nnz
    finally:
        ctx.set_tuning(**saved)


def test_hip_graph_mode_matches_eager(ctx, torch_dev):
    """LM_GRAPH captures the whole solve into one HIP graph per call: set-up,
    guarded phases and the tail kernel, which runs whatever the guarded phases
    leave. Several graph solves in a row, with eager solves and host syncs in
    between, must each equal the eager result and the oracle."""
    import torch
    cases = [
        ("er 4096", lmgen.er(4096, 32768, seed=1)),
        ("rmat 13", lmgen.rmat(13, 16, seed=8)),
        ("increasing path 301", lmgen.from_edges(302, [[i, i + 1] for i in range(301)], np.arange(1, 302))),
        ("single edge", lmgen.from_edges(2, [[0, 1]], [0.5])),
    ]
    for rep in range(3):
        for name, g in cases:
            print(f"case: hip graph rep={rep} {name}", flush=True)
            eager, st_e = _solve(ctx, torch_dev, g, 7)
            torch.cuda.synchronize()
            graphed, st_g = _solve(ctx, torch_dev, g, 7, hip_graph=True)
            assert np.array_equal(eager, graphed), f"{name}: graph result differs from eager"
            assert st_g.phases == st_e.phases and np.array_equal(st_g.log, st_e.log)
            _assert_parity(g, 7, graphed, st_g, f"graph {name}")


def test_empty_rows_in_first_live_set(ctx, torch_dev):
    """A single graph's first live set is read from the CSR, empty rows
    included; workgroup ranges split entries plus a fixed weight per row.
    Isolated vertices appended at the end change neither keys nor matching
    (mate[] on the original vertices is identical, phase log too); isolated
    vertices interleaved (v -> 2v) relabel the edges, so with distinct weights
    the matching maps through the relabelling. Every solve equals the oracle."""
    for seed, (n, m) in ((1, (6000, 60000)), (2, (20000, 200000)), (3, (1500, 15000))):
        g = lmgen.er(n, m, seed=seed)
        lo, hi, w = ref.undirected_edges(g)
        print(f"case: empty rows n={n} m={m} seed={seed}", flush=True)
        mate, st = _solve(ctx, torch_dev, g, 9)
        _assert_parity(g, 9, mate, st, "plain")
        gd = lmgen.from_edges(2 * n, np.stack([lo, hi], 1), w)  # n isolated vertices appended
        mated, std = _solve(ctx, torch_dev, gd, 9)
        _assert_parity(gd, 9, mated, std, "appended")
        assert np.array_equal(mated[:n], mate) and np.all(mated[n:] == -1)
        assert np.array_equal(std.log, st.log)
        gi = lmgen.from_edges(2 * n, np.stack([2 * lo, 2 * hi], 1), w)  # one isolated vertex after each
        matei, sti = _solve(ctx, torch_dev, gi, 9)
        _assert_parity(gi, 9, matei, sti, "interleaved")
        assert np.all(matei[1::2] == -1)
        if len(np.unique(w)) == len(w):  # weights decide every comparison: the hash never does
            assert np.array_equal(matei[0::2], np.where(mate >= 0, 2 * mate, -1))
    # a long stretch of empty rows between two dense blocks, cut at many range sizes
    dense = lmgen.er(3000, 40000, seed=4)
    lo, hi, w = ref.undirected_edges(dense)
    lo2 = np.concatenate([lo, lo + 200000]).astype(np.int64)
    hi2 = np.concatenate([hi, hi + 200000]).astype(np.int64)
    gg = lmgen.from_edges(203000, np.stack([lo2, hi2], 1), np.concatenate([w, w]))
    base = ctx.tuning()
    try:
        for be in (2048, 65536):
            ctx.set_tuning(block_entries=be, grid_per_cu=1)
            print(f"case: empty stretch block_entries={be}", flush=True)
            mate, st = _solve(ctx, torch_dev, gg, 5)
            _assert_parity(gg, 5, mate, st, f"empty stretch {be}")
    finally:
        ctx.set_tuning(**base)


def test_unweighted_empty_rows(ctx, torch_dev):
    """The one-graph unweighted first argmax walks R_1 with a window of 64
    row ends: runs of empty rows shorter and longer than the window (ids
    spread by 2, 64 and 100, and a stretch of 197000 empty rows between two
    dense blocks) and many range sizes. Every solve equals the oracle on the
    same graph with unit weights."""
    import torch
    dense = lmgen.er(3000, 40000, seed=4, weights="unit")
    lo, hi, _ = ref.undirected_edges(dense)
    cases = []
    for k in (2, 64, 100):
        cases.append((f"ids x{k}", lmgen.from_edges(3000 * k, np.stack([k * lo, k * hi], 1), np.ones(len(lo)))))
    lo2 = np.concatenate([lo, lo + 200000]).astype(np.int64)
    hi2 = np.concatenate([hi, hi + 200000]).astype(np.int64)
    cases.append(("empty stretch", lmgen.from_edges(203000, np.stack([lo2, hi2], 1), np.ones(len(lo2)))))
    base = ctx.tuning()
    try:
        for name, g in cases:
            rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(torch_dev)
            col = torch.from_numpy(np.ascontiguousarray(g.col)).to(torch_dev)
            for be in (2048, 65536, None):
                if be is None:
                    ctx.set_tuning(**base)
                else:
                    ctx.set_tuning(block_entries=be, grid_per_cu=1)
                print(f"case: unweighted {name} block_entries={be}", flush=True)
                mate, st = ctx.match(rp, col, None, seed=5)
                _assert_parity(_unit(g), 5, mate.cpu().numpy(), st, f"unweighted {name} {be}")
    finally:
        ctx.set_tuning(**base)


def test_unweighted_first_compaction(ctx, torch_dev):
    """With no hand-over to the tail kernel, the compaction of phase 1 of one
    unweighted graph runs over R_1 read from the CSR (empty rows as pieces of
    length 0, matched rows skipped unloaded) even for small graphs:
    power-law, star, geometric and uniform graphs, runs of empty rows, an
    entry array that is not 16-byte aligned, and range sizes that cut rows at
    many places. Every solve, phase log included, equals the oracle on the
    same graph with unit weights."""
    import torch
    dense = lmgen.er(3000, 40000, seed=4, weights="unit")
    lo, hi, _ = ref.undirected_edges(dense)
    cases = [("rmat 14", lmgen.rmat(14, 16, seed=3)), ("rmat 13 seed 8", lmgen.rmat(13, 16, seed=8)),
             ("star 5000", _unit(_star(5000, unit=True))), ("rgg 30000", _unit(lmgen.rgg(30000, 10.0, seed=9))),
             ("er 20000", lmgen.er(20000, 160000, seed=7, weights="unit"))]
    for k in (2, 100):
        cases.append((f"ids x{k}", lmgen.from_edges(3000 * k, np.stack([k * lo, k * hi], 1), np.ones(len(lo)))))
    lo2 = np.concatenate([lo, lo + 200000]).astype(np.int64)
    hi2 = np.concatenate([hi, hi + 200000]).astype(np.int64)
    cases.append(("empty stretch", lmgen.from_edges(203000, np.stack([lo2, hi2], 1), np.ones(len(lo2)))))
    rng = np.random.default_rng(33)
    for it in range(6):
        n = int(rng.integers(2, 3000))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 12 * n) + 1))
        cases.append((f"er it={it} n={n} m={m}", lmgen.er(n, m, int(rng.integers(1, 2**62)), weights="unit")))
    base = ctx.tuning()
    try:
        for name, g in cases:
            rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(torch_dev)
            col = torch.from_numpy(np.ascontiguousarray(g.col)).to(torch_dev)
            for be in (None, 2048, 65536):
                if be is None:
                    ctx.set_tuning(**{**base, "tail_entries": 0})
                else:
                    ctx.set_tuning(**{**base, "tail_entries": 0, "block_entries": be, "grid_per_cu": 1})
                print(f"case: unweighted first compaction {name} block_entries={be}", flush=True)
                mate, st = ctx.match(rp, col, None, seed=5)
                _assert_parity(_unit(g), 5, mate.cpu().numpy(), st, f"first compaction {name} {be}")
        big = lmgen.rmat(13, 16, seed=6)
        colx = torch.zeros(big.nnz + 1, dtype=torch.int32, device=torch_dev)
        colx[1:] = torch.from_numpy(big.col).to(torch_dev)
        ctx.set_tuning(**{**base, "tail_entries": 0})
        print("case: unweighted first compaction, unaligned col", flush=True)
        mate, st = ctx.match(torch.from_numpy(big.row_ptr).to(torch_dev), colx[1:], None, seed=3)
        _assert_parity(_unit(big), 3, mate.cpu().numpy(), st, "first compaction unaligned col")
    finally:
        ctx.set_tuning(**base)


def _weight_tol(abs_sum, edges, exact):
    # Any order of 2|M| double additions (each matched edge from both ends,
    # then halved exactly) is within (2|M| - 1) 2^-53 sum|w| of the exact sum;
    # the exact sum itself is rounded once (half an ulp).
    return 2 * edges * 2.0**-53 * abs_sum + 2.0**-52 * abs(exact)


def test_matched_weight(ctx, torch_dev):
    """LM_WEIGHT_SUM: w(M) against math.fsum over the oracle's matching, within
    the rounding bound of double summation; exact for unit weights; identical
    on a repeated call."""
    import torch
    rng = np.random.default_rng(31)
    cases = [("er uniform", lmgen.er(20000, 160000, seed=3)),
             ("rmat 15 uniform", lmgen.rmat(15, 16, seed=4, weights="uniform")),
             ("star 5000", _star(5000, rng=rng)), ("rgg 30000", lmgen.rgg(30000, 10.0, seed=9))]
    lo, hi, _ = ref.undirected_edges(cases[0][1])
    wsg = rng.choice(np.array([-2.5, -0.0, 0.0, 1e-30, 3.0], np.float32), len(lo))
    cases.append(("er signed", lmgen.from_edges(cases[0][1].n, np.stack([lo, hi], 1), wsg)))
    for name, g in cases:
        print(f"case: matched weight {name}", flush=True)
        ref_mate, _ = oracle.local_max_graph(g, 5)
        exact, abs_sum, edges = ref.matching_weight_exact(g, ref_mate)
        mate, st = _solve(ctx, torch_dev, g, 5, weight_sum=True)
        assert np.array_equal(mate, ref_mate), name
        assert abs(st.matched_weight - exact) <= _weight_tol(abs_sum, edges, exact), (name, st.matched_weight, exact)
        _, st2 = _solve(ctx, torch_dev, g, 5, weight_sum=True)
        assert st2.matched_weight == st.matched_weight, name
        _, st3 = _solve(ctx, torch_dev, g, 5)
        assert st3.matched_weight is None
    # host inputs
    g = cases[0][1]
    mate, st = ctx.match(g.row_ptr, g.col, g.w, seed=5, weight_sum=True)
    exact, abs_sum, edges = ref.matching_weight_exact(g, np.asarray(mate))
    assert abs(st.matched_weight - exact) <= _weight_tol(abs_sum, edges, exact)
    # unit weights: w(M) = |M| exactly, with the weight array and without one
    g = lmgen.rmat(14, 16, seed=3)
    rp = torch.from_numpy(g.row_ptr).to(torch_dev)
    col = torch.from_numpy(g.col).to(torch_dev)
    for w in (torch.from_numpy(g.w).to(torch_dev), None):
        print(f"case: matched weight rmat 14 unit, weight array {w is not None}", flush=True)
        mate, st = ctx.match(rp, col, w, seed=1, weight_sum=True)
        assert st.matched_weight == float(st.matched_edges)
        assert st.matched_edges == int((mate.cpu().numpy() >= 0).sum()) // 2
    # a batch: the sum over all graphs (local ids in col and mate)
    b = lmgen.er_batch(64, seed=5, lg_lo=5.0, lg_hi=11.0)
    print("case: matched weight batch of 64", flush=True)
    mate, st, _ = ctx.match_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=3, weight_sum=True)
    mate = np.asarray(mate)
    ref_mate, _ = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=3)
    assert np.array_equal(mate, ref_mate)
    tot, tabs, tm = [], [], 0
    for k in range(b.graphs):
        gk = b.graph(k)
        e, a_, m_ = ref.matching_weight_exact(gk, mate[b.vtx_off[k]:b.vtx_off[k + 1]])
        tot.append(e)
        tabs.append(a_)
        tm += m_
    import math
    exact = math.fsum(tot)
    assert abs(st.matched_weight - exact) <= _weight_tol(math.fsum(tabs), tm, exact)


def test_batch_hip_graph_matches_eager(ctx, torch_dev):
    import torch
    b = lmgen.er_batch(128, seed=4, lg_lo=4.0, lg_hi=12.0)
    rp, col, w = (torch.from_numpy(np.ascontiguousarray(x)).to(torch_dev) for x in (b.row_ptr, b.col, b.w))
    ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=3)
    for rep in range(3):
        print(f"case: batch hip graph rep={rep}", flush=True)
        m_e, _, ph_e = ctx.match_batch(b.vtx_off, rp, col, w, seed0=3, hip_graph=False)
        m_g, _, ph_g = ctx.match_batch(b.vtx_off, rp, col, w, seed0=3, hip_graph=True)
        assert np.array_equal(m_e.cpu().numpy(), ref_mate) and np.array_equal(m_g.cpu().numpy(), ref_mate)
        assert np.array_equal(ph_e, ref_ph) and np.array_equal(ph_g, ref_ph)


def test_autotune_batch_and_cache(ctx, torch_dev, tmp_path):
    import torch
    b = lmgen.er_batch(48, seed=9, lg_lo=6.0, lg_hi=11.0)
    rp, col, w = (torch.from_numpy(np.ascontiguousarray(x)).to(torch_dev) for x in (b.row_ptr, b.col, b.w))
    base = ctx.tuning()
    cache = str(tmp_path / "tune.jsonl")
    try:
        print("case: autotune batch of 48", flush=True)
        t1 = ctx.autotune_batch(b.vtx_off, rp, col, w, cache_path=cache)
        assert 2048 <= t1["block_entries"] <= 4194304 and t1["grid_per_cu"] >= 1 and t1["phases_per_sync"] >= 1
        assert t1["tail_entries"] >= 0
        assert ctx.tuning() == t1
        lines = open(cache).read().strip().splitlines()
        assert len(lines) == 1 and '"block_entries"' in lines[0] and '"tail_entries"' in lines[0]
        ctx.set_tuning(**base)
        t2 = ctx.autotune_batch(b.vtx_off, rp, col, w, cache_path=cache)  # answered from the cache
        assert t2 == t1 and len(open(cache).read().strip().splitlines()) == 1
        mate, _, gph = ctx.match_batch(b.vtx_off, rp, col, w, seed0=1)
        ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=1)
        assert np.array_equal(mate.cpu().numpy(), ref_mate) and np.array_equal(gph, ref_ph)
    finally:
        ctx.set_tuning(**base)
