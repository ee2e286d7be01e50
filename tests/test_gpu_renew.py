"""Renewed tie-break keys (LM_RENEW_KEYS) on the GPU against the oracle's
renewed mode, element by element (mate[] and the phase log, tolerance 0).

Phase t breaks ties with H_t = mix(pair XOR mix(S + t gamma)) (the fresh
noise per iteration of Lemma 1's footnote and of Section 2.1, step 1): the
first argmax uses t = 1, the compaction of phase t (and the device tail)
computes the candidates of phase t + 1 with t + 1. Every hand-over mode of
the tail, the captured whole-solve graph and batches are covered.
"""
import numpy as np
import pytest

import lmgen
import oracle
from tests import _pyref as ref

pytestmark = pytest.mark.gpu

MODES = [
    ("phase kernels only", dict(tail_entries=0), {}),
    ("tail from the start", dict(tail_entries=1 << 30), {}),
    ("hand-over mid-solve", dict(tail_entries=2048, block_entries=2048), {}),
    ("captured graph", dict(tail_entries=2048, block_entries=2048), {"hip_graph": True}),
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


def _check(ctx, torch_dev, g, seed, name, unweighted=False):
    import torch
    gg = g
    if unweighted:
        gg = lmgen.from_edges(g.n, np.stack(ref.undirected_edges(g)[:2], 1), np.ones(g.nnz // 2, np.float32))
    ref_mate, ref_log = oracle.local_max_graph(gg, seed, renew=True)
    saved = ctx.tuning()
    try:
        for mode, tun, kw in MODES:
            ctx.set_tuning(**{**saved, **tun})
            rp = torch.from_numpy(g.row_ptr).to(torch_dev)
            col = torch.from_numpy(g.col).to(torch_dev)
            w = None if unweighted else torch.from_numpy(g.w).to(torch_dev)
            print(f"case: renewed {name} seed={seed} mode={mode}", flush=True)
            mate, st = ctx.match(rp, col, w, seed=seed, renew_keys=True, **kw)
            torch.cuda.synchronize()
            got = mate.cpu().numpy()
            if not np.array_equal(got, ref_mate):
                bad = np.flatnonzero(got != ref_mate)
                raise AssertionError(f"{name} [{mode}]: mate differs at {len(bad)} vertices, first {bad[:5]}")
            if st is None:  # stream-ordered: no statistics
                continue
            assert st.phases == len(ref_log), f"{name} [{mode}]: phases {st.phases} vs {len(ref_log)}"
            assert np.array_equal(st.log[:, 0], 2 * ref_log[:, 0]), f"{name} [{mode}]: live entries"
            assert np.array_equal(st.log[:, 1], ref_log[:, 1]), f"{name} [{mode}]: live rows"
            assert np.array_equal(st.log[:, 2], ref_log[:, 2]), f"{name} [{mode}]: matched per phase"
    finally:
        ctx.set_tuning(**saved)


def test_renewed_keys_equal_oracle(ctx, torch_dev):
    cases = [
        ("er 4096 uniform", lmgen.er(4096, 32768, seed=1), 1, False),
        ("er 20000 unit", lmgen.er(20000, 160000, seed=7, weights="unit"), 4, False),
        ("rmat 14 unweighted", lmgen.rmat(14, 16, seed=8), 3, True),
        ("rmat 13 uniform", lmgen.rmat(13, 16, seed=4, weights="uniform"), 9, False),
        ("rgg 30000", lmgen.rgg(30000, 10.0, seed=2), 1, False),
        ("star 5000 unit", lmgen.from_edges(5001, np.array([[0, i] for i in range(1, 5001)]), np.ones(5000)), 2,
         False),
        ("increasing path 301", lmgen.from_edges(302, [[i, i + 1] for i in range(301)], np.arange(1, 302)), 1,
         False),
    ]
    for name, g, seed, unw in cases:
        _check(ctx, torch_dev, g, seed, name, unweighted=unw)


@pytest.mark.parametrize("wkind", ["unit", "tied", "signed"])
def test_renewed_keys_random_small(ctx, torch_dev, wkind):
    rng = np.random.default_rng({"unit": 61, "tied": 62, "signed": 63}[wkind])
    for it in range(6):
        n = int(rng.integers(2, 4000))
        m = int(rng.integers(1, min(n * (n - 1) // 2, 12 * n) + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
        lo, hi, _ = ref.undirected_edges(g)
        if wkind == "unit":
            w = np.ones(len(lo), np.float32)
        elif wkind == "tied":
            w = rng.integers(1, 4, len(lo)).astype(np.float32)
        else:
            w = rng.choice(np.array([-2.5, -0.0, 0.0, 1e-30, 3.0], np.float32), len(lo))
        g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
        _check(ctx, torch_dev, g, int(rng.integers(0, 2**64, dtype=np.uint64)), f"{wkind} it={it}")


def test_renewed_keys_batch(ctx, torch_dev):
    """Every graph of a batch with its own seed, renewed keys, equals the
    oracle solving it alone; per-graph phase counts too."""
    import torch
    b = lmgen.er_batch(96, seed=8, lg_lo=4.0, lg_hi=12.0, weights="unit")
    seeds = np.random.default_rng(3).integers(0, 2**63, b.graphs, dtype=np.uint64)
    ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seeds=seeds, renew=True)
    saved = ctx.tuning()
    try:
        for mode, tun, kw in MODES[:4]:
            ctx.set_tuning(**{**saved, **tun})
            rp = torch.from_numpy(b.row_ptr).to(torch_dev)
            col = torch.from_numpy(b.col).to(torch_dev)
            w = torch.from_numpy(b.w).to(torch_dev)
            print(f"case: renewed batch mode={mode}", flush=True)
            mate, st, ph = ctx.match_batch(b.vtx_off, rp, col, w, seeds=seeds, renew_keys=True,
                                           hip_graph=kw.get("hip_graph", False))
            assert np.array_equal(mate.cpu().numpy(), ref_mate), f"batch [{mode}]"
            assert np.array_equal(ph, ref_ph), f"batch [{mode}]: phases"
    finally:
        ctx.set_tuning(**saved)


def test_distinct_weights_renewal_changes_nothing(ctx, torch_dev):
    import torch
    g = lmgen.rgg(50000, 10.0, seed=5)
    lo, hi, _ = ref.undirected_edges(g)
    wd = (np.random.default_rng(5).permutation(len(lo)) + 1).astype(np.float32) * np.float32(2**-24)
    g = lmgen.from_edges(g.n, np.stack([lo, hi], 1), wd)
    rp, col, w = (torch.from_numpy(x).to(torch_dev) for x in (g.row_ptr, g.col, g.w))
    a, sa = ctx.match(rp, col, w, seed=3)
    b, sb = ctx.match(rp, col, w, seed=3, renew_keys=True)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy()) and sa.phases == sb.phases
