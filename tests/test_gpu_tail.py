"""The device-side tail of the phase loop against the oracle.

Once the live set is small, one persistent launch (k_tail) runs every
remaining phase (Section 2: a phase is linear in the live edges, so the
launch and host round trip of the phase kernels dominate a small one). The
result and the per-phase log must not depend on where the hand-over happens:
each case is solved with the phase kernels only, with the tail from the
first phase, with a hand-over in mid-solve (rows cut at workgroup
boundaries reach the tail as several pieces), as one captured HIP graph
(guarded phases, then the tail), and stream-ordered (LM_ASYNC), and every
solve is compared with the oracle element by element (tolerance 0).
"""
import numpy as np
import pytest

import lmgen
import oracle
from tests import _pyref as ref

pytestmark = pytest.mark.gpu

# (name, tuning, solve keywords)
MODES = [
    ("phase kernels only", dict(tail_entries=0), {}),
    ("tail from the start", dict(tail_entries=1 << 30), {}),
    ("hand-over mid-solve", dict(tail_entries=2048, block_entries=2048), {}),
    ("captured graph, hand-over mid-solve", dict(tail_entries=2048, block_entries=2048), {"hip_graph": True}),
    ("captured graph, tail from the start", dict(tail_entries=1 << 30), {"hip_graph": True}),
    ("stream-ordered", dict(tail_entries=2048, block_entries=2048), {"asynchronous": True}),
]


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


def _dev(torch_dev, g, unweighted=False):
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(torch_dev)
    col = torch.from_numpy(np.ascontiguousarray(g.col)).to(torch_dev)
    w = None if unweighted else torch.from_numpy(np.ascontiguousarray(g.w)).to(torch_dev)
    return rp, col, w


def _check(g, seed, mate, st, what):
    ref_mate, ref_log = oracle.local_max_graph(g, seed)
    if not np.array_equal(mate, ref_mate):
        bad = np.flatnonzero(mate != ref_mate)
        raise AssertionError(f"{what}: mate differs at {len(bad)} vertices, first {bad[:5]}")
    if st is None:  # stream-ordered: no statistics
        return
    assert st.phases == len(ref_log), f"{what}: phases {st.phases} vs oracle {len(ref_log)}"
    assert st.matched_edges == int((ref_mate >= 0).sum()) // 2, what
    assert np.array_equal(st.log[:, 0], 2 * ref_log[:, 0]), f"{what}: live entries differ"
    assert np.array_equal(st.log[:, 1], ref_log[:, 1]), f"{what}: live rows differ"
    assert np.array_equal(st.log[:, 2], ref_log[:, 2]), f"{what}: matched per phase differ"


def _solve_modes(ctx, torch_dev, g, seed, name, unweighted=False):
    import torch
    saved = ctx.tuning()
    gg = g
    if unweighted:  # the oracle sees the same graph with unit weights
        gg = lmgen.from_edges(g.n, np.stack(ref.undirected_edges(g)[:2], 1), np.ones(g.nnz // 2, np.float32))
    try:
        for mode, tun, kw in MODES:
            ctx.set_tuning(**{**saved, **tun})
            rp, col, w = _dev(torch_dev, g, unweighted)
            print(f"case: {name} seed={seed} mode={mode}", flush=True)
            mate, st = ctx.match(rp, col, w, seed=seed, **kw)
            torch.cuda.synchronize()
            _check(gg, seed, mate.cpu().numpy(), st, f"{name} [{mode}]")
    finally:
        ctx.set_tuning(**saved)


def _star_path(leaves, seed):
    """A hub joined to every leaf by light edges, the leaves joined in a path by
    heavier ones: the hub's row loses a few leaves per phase, so it stays long
    for several phases and is cut at workgroup boundaries."""
    rng = np.random.default_rng(seed)
    hub = [[0, i] for i in range(1, leaves + 1)]
    path = [[i, i + 1] for i in range(1, leaves)]
    w = np.concatenate([0.01 + 0.001 * rng.random(leaves), 0.5 + 0.5 * rng.random(leaves - 1)])
    return lmgen.from_edges(leaves + 1, np.array(hub + path), w.astype(np.float32))


def test_tail_modes_equal_oracle(ctx, torch_dev):
    cases = [
        ("er 4096", lmgen.er(4096, 32768, seed=1), 1, False),
        ("star-path 6000", _star_path(6000, 3), 5, False),
        ("star 5000", lmgen.from_edges(5001, np.array([[0, i] for i in range(1, 5001)]),
                                       np.linspace(0.1, 1.0, 5000).astype(np.float32)), 2, False),
        ("increasing path 301", lmgen.from_edges(302, [[i, i + 1] for i in range(301)], np.arange(1, 302)), 1, False),
        ("rmat 14 unweighted", lmgen.rmat(14, 16, seed=8), 3, True),
        ("rmat 13 uniform", lmgen.rmat(13, 16, seed=4, weights="uniform"), 9, False),
        ("rgg 30000", lmgen.rgg(30000, 10.0, seed=2), 1, False),
        ("er 20000 unit", lmgen.er(20000, 160000, seed=7, weights="unit"), 4, False),
        ("single edge", lmgen.from_edges(2, [[0, 1]], [0.5]), 1, False),
        ("isolated vertices only", lmgen.from_edges(7, np.zeros((0, 2), np.int64), np.zeros(0)), 1, False),
    ]
    for name, g, seed, unw in cases:
        _solve_modes(ctx, torch_dev, g, seed, name, unweighted=unw)


@pytest.mark.parametrize("wkind", ["uniform", "tied", "unit", "signed"])
def test_tail_modes_random_small(ctx, torch_dev, wkind):
    rng = np.random.default_rng({"uniform": 21, "tied": 22, "unit": 23, "signed": 24}[wkind])
    for it in range(6):
        n = int(rng.integers(2, 4000))
        m = int(rng.integers(1, min(n * (n - 1) // 2, 12 * n) + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
        if wkind != "uniform":
            lo, hi, _ = ref.undirected_edges(g)
            if wkind == "tied":
                w = rng.integers(1, 4, len(lo)).astype(np.float32)
            elif wkind == "unit":
                w = np.ones(len(lo), np.float32)
            else:
                w = rng.choice(np.array([-2.5, -0.0, 0.0, 1e-30, 3.0], np.float32), len(lo))
            g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        _solve_modes(ctx, torch_dev, g, seed, f"{wkind} it={it} n={n} m={m}")


def test_tail_batch_modes(ctx, torch_dev):
    """Per-graph results and phase counts of a batch do not depend on the
    hand-over either (the tail keeps every row's graph, local ids and seed)."""
    import torch
    b = lmgen.er_batch(96, seed=6, lg_lo=4.0, lg_hi=12.0)
    ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=3)
    saved = ctx.tuning()
    try:
        for mode, tun, kw in MODES:
            ctx.set_tuning(**{**saved, **tun})
            rp = torch.from_numpy(b.row_ptr).to(torch_dev)
            col = torch.from_numpy(b.col).to(torch_dev)
            w = torch.from_numpy(b.w).to(torch_dev)
            hip_graph = kw.get("hip_graph", False)
            print(f"case: batch of 96 mode={mode}", flush=True)
            mate, st, ph = ctx.match_batch(b.vtx_off, rp, col, w, seed0=3, hip_graph=hip_graph,
                                           asynchronous=kw.get("asynchronous", False))
            torch.cuda.synchronize()
            assert np.array_equal(mate.cpu().numpy(), ref_mate), f"batch [{mode}]: mate differs"
            if ph is not None:
                assert np.array_equal(ph, ref_ph), f"batch [{mode}]: per-graph phases differ"
                assert st.phases == int(ref_ph.max())
    finally:
        ctx.set_tuning(**saved)


def test_tail_rejects_asymmetric_input(ctx, torch_dev):
    """Row 0 names vertex 3, whose row is empty: that entry has no twin, so
    once the edge {1, 2} is matched a phase matches nothing. Both the phase
    kernels and the tail report LM_EGRAPH instead of looping."""
    import torch
    import paper_1302_4587_amd as lm
    from paper_1302_4587_amd import _lib as L
    row_ptr = np.array([0, 1, 2, 3, 3], np.int64)
    col = np.array([3, 2, 1], np.int32)
    w = np.ones(3, np.float32)
    saved = ctx.tuning()
    try:
        for mode, tun, kw in MODES:
            if kw.get("asynchronous"):
                continue  # no status to report
            ctx.set_tuning(**{**saved, **tun})
            print(f"case: asymmetric mode={mode}", flush=True)
            with pytest.raises(lm.LMError) as e:
                ctx.match(torch.from_numpy(row_ptr).to(torch_dev), torch.from_numpy(col).to(torch_dev),
                          torch.from_numpy(w).to(torch_dev), seed=1, **kw)
            assert e.value.status == L.LM_EGRAPH, mode
        ctx.set_tuning(**saved)
        g = lmgen.er(300, 900, seed=4)
        mate, st = ctx.match(*_dev(torch_dev, g), seed=1)
        _check(g, 1, mate.cpu().numpy(), st, "after the errors")
    finally:
        ctx.set_tuning(**saved)


def test_async_validation_and_ordering(ctx, torch_dev):
    """LM_ASYNC takes device buffers only and reports nothing back; solves
    enqueued back to back on one stream each equal the oracle, and a normal
    call after them waits for them."""
    import torch
    import paper_1302_4587_amd as lm
    from paper_1302_4587_amd import _lib as L
    g = lmgen.er(4096, 32768, seed=1)
    rp, col, w = _dev(torch_dev, g)
    with pytest.raises(lm.LMError) as e:
        ctx.match(g.row_ptr, g.col, g.w, seed=1, asynchronous=True)  # host arrays
    assert e.value.status == L.LM_EINVAL
    with pytest.raises(lm.LMError) as e:
        ctx.match(rp, col, w, seed=1, asynchronous=True, check_graph=True)
    assert e.value.status == L.LM_EINVAL
    outs = []
    for seed in (1, 2, 3):
        mate = torch.full((g.n,), -7, dtype=torch.int32, device=torch_dev)
        ctx.match(rp, col, w, seed=seed, mate=mate, asynchronous=True)
        outs.append((seed, mate))
    sync_mate, st = ctx.match(rp, col, w, seed=4)
    torch.cuda.synchronize()
    for seed, mate in outs:
        _check(g, seed, mate.cpu().numpy(), None, f"async seed={seed}")
    _check(g, 4, sync_mate.cpu().numpy(), st, "sync after async")
