"""GPU parity of the batched solve and the request server.

Keys use each graph's local vertex ids and its own seed, so every graph of a
batch and every served request must equal the oracle's solve of that graph
alone: mate[] element by element and the graph's phase count (integer work,
tolerance 0). Phases of a batch are synchronous over the union, so the
union's phase count is the largest per-graph count.
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


def _dev(torch_dev, *arrays):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(torch_dev) for a in arrays)


def _graph_slice(b, k):
    a, e = int(b.vtx_off[k]), int(b.vtx_off[k + 1])
    e0, e1 = int(b.row_ptr[a]), int(b.row_ptr[e])
    return a, e, lmgen.Graph(e - a, b.row_ptr[a:e + 1] - e0, b.col[e0:e1], b.w[e0:e1])


def test_batch_equals_each_graph_alone(ctx, torch_dev):
    print("case: batch of 300 ER graphs, n in [2^3, 2^12]", flush=True)
    b = lmgen.er_batch(300, seed=3, lg_lo=3.0, lg_hi=12.0)
    rp, col, w = _dev(torch_dev, b.row_ptr, b.col, b.w)
    mate, st, gph = ctx.match_batch(b.vtx_off, rp, col, w, seed0=1)
    ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seed0=1)
    got = mate.cpu().numpy()
    if not np.array_equal(got, ref_mate):
        bad = np.flatnonzero(got != ref_mate)
        g = np.searchsorted(b.vtx_off, bad[0], side="right") - 1
        raise AssertionError(f"{len(bad)} vertices differ, first in graph {g}")
    assert np.array_equal(gph, ref_ph)
    assert st.phases == int(ref_ph.max())


def test_batch_of_one_graph(ctx, torch_dev):
    """A batch of one graph reads its first live set straight from the CSR
    (empty rows included); its mate[] and its phase count must equal the
    oracle's, also for a graph with no edge at all (0 phases)."""
    cases = [("er 5000/3000 (isolated vertices)", lmgen.er(5000, 3000, seed=6)),
             ("er 100/0 (no edge)", lmgen.er(100, 0, seed=6)),
             ("rmat 12", lmgen.rmat(12, 16, seed=2))]
    for name, g in cases:
        vo = np.array([0, g.n], dtype=np.int64)
        ref_mate, ref_ph = oracle.local_max_batch(vo, g.row_ptr, g.col, g.w, seed0=4)
        for hip_graph in (False, True):
            print(f"case: batch of one, {name}, hip_graph={hip_graph}", flush=True)
            rp, col, w = _dev(torch_dev, g.row_ptr, g.col, g.w)
            mate, st, gph = ctx.match_batch(vo, rp, col, w, seed0=4, hip_graph=hip_graph)
            assert np.array_equal(mate.cpu().numpy(), ref_mate), name
            assert np.array_equal(gph, ref_ph), (name, gph, ref_ph)
            assert st.phases == int(ref_ph[0])


def test_batch_per_graph_seeds_and_host_inputs(ctx, torch_dev):
    print("case: batch of 64 graphs with per-graph seeds, host inputs", flush=True)
    b = lmgen.er_batch(64, seed=5, lg_lo=5.0, lg_hi=11.0, weights="unit")
    seeds = np.random.default_rng(2).integers(0, 2**63, size=64, dtype=np.uint64)
    mate, st, gph = ctx.match_batch(b.vtx_off, b.row_ptr, b.col, b.w, seeds=seeds)
    ref_mate, ref_ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seeds=seeds)
    assert np.array_equal(np.asarray(mate), ref_mate)
    assert np.array_equal(gph, ref_ph)
    # one graph of the batch solved alone on the GPU gives the same slice
    k = 17
    a, e, g = _graph_slice(b, k)
    alone, _ = ctx.match(g.row_ptr, g.col, g.w, seed=int(seeds[k]))
    assert np.array_equal(np.asarray(alone), ref_mate[a:e])


def _oracle_parallel(jobs, threads=16):
    """Runs oracle.local_max_graph(g, seed) for every (g, seed) on a thread
    pool (the C oracle releases the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda js: oracle.local_max_graph(js[0], js[1]), jobs))


def test_batch_full_size_all_graphs(ctx, torch_dev):
    """The bench's batch (4096 graphs, n log-uniform in [2^8, 2^16], average
    degree U[4, 32]): every graph against the oracle solving it alone, mate[]
    and phase count."""
    print("case: batch of 4096 ER graphs (full size), every graph", flush=True)
    b = lmgen.er_batch(4096, 1)
    rp, col, w = _dev(torch_dev, b.row_ptr, b.col, b.w)
    mate, st, gph = ctx.match_batch(b.vtx_off, rp, col, w, seed0=1)
    got = mate.cpu().numpy()
    del rp, col, w
    slices = [_graph_slice(b, k) for k in range(b.graphs)]
    refs = _oracle_parallel([(g, 1) for _, _, g in slices])
    bad = [k for k, ((a, e, _), (rm, rl)) in enumerate(zip(slices, refs))
           if not np.array_equal(got[a:e], rm) or gph[k] != len(rl)]
    assert not bad, f"{len(bad)} of {b.graphs} graphs differ, first {bad[:5]}"
    assert st.phases == int(gph.max())


def test_server_request_sizes_up_to_2_22(ctx, torch_dev):
    """Requests of the serving workload's full size range, n log-uniform in
    [2^10, 2^22] with the largest size of both kinds included, RGG and R-MAT
    half and half, several resident at once: every result equals the
    oracle."""
    import paper_1302_4587_amd as lm
    rng = np.random.default_rng(23)
    sizes = [("rgg", 1 << 22), ("rmat", 1 << 22)]
    for _ in range(14):
        sizes.append(("rgg" if rng.random() < 0.5 else "rmat", int(round(2.0 ** rng.uniform(10.0, 22.0)))))
    reqs = [(lmgen.serving_graph(kind, n, seed=i + 1), int(rng.integers(0, 2**63))) for i, (kind, n) in
            enumerate(sizes)]
    print(f"case: server, {len(reqs)} requests up to n=2^22, nnz total {sum(g.nnz for g, _ in reqs)}", flush=True)
    with lm.Server(ctx, hbm_budget_bytes=64 << 30, max_resident=8, mode=lm.LM_SERVE_BATCHED) as srv:
        tickets = [srv.submit(g.row_ptr, g.col, g.w, seed=s) for g, s in reqs]
        results = [srv.wait(t, 120000) for t in tickets]
    refs = _oracle_parallel(reqs)
    for i, ((g, s), r, (rm, rl)) in enumerate(zip(reqs, results, refs)):
        assert r is not None, f"request {i} not done"
        mate, info = r
        assert np.array_equal(mate, rm), f"request {i} (n={g.n}) differs from the oracle"
        assert info["phases"] == len(rl)


def _request_mix(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(2.0 ** rng.uniform(6.0, 13.0)))
        kind = "rgg" if rng.random() < 0.5 else "rmat"
        out.append((lmgen.serving_graph(kind, n, seed=int(rng.integers(1, 2**31))), int(rng.integers(0, 2**63))))
    return out


@pytest.mark.parametrize("mode", ["batched", "fifo"])
def test_server_results_equal_alone(ctx, torch_dev, mode):
    import paper_1302_4587_amd as lm
    reqs = _request_mix(40, 11)
    m = lm.LM_SERVE_BATCHED if mode == "batched" else lm.LM_SERVE_FIFO
    print(f"case: server {mode}, 40 mixed requests", flush=True)
    with lm.Server(ctx, hbm_budget_bytes=1 << 30, max_resident=8, mode=m) as srv:
        tickets = [srv.submit(g.row_ptr, g.col, g.w, seed=s) for g, s in reqs]
        results = [srv.wait(t, 60000) for t in tickets]
    for i, ((g, s), r) in enumerate(zip(reqs, results)):
        assert r is not None, f"request {i} not done"
        mate, info = r
        ref_mate, ref_log = oracle.local_max_graph(g, s)
        assert np.array_equal(mate, ref_mate), f"request {i} differs from the oracle"
        assert info["phases"] == len(ref_log)
        alone, _ = ctx.match(g.row_ptr, g.col, g.w, seed=s)
        assert np.array_equal(np.asarray(alone), mate), f"request {i}: served differs from alone"


def test_server_errors(ctx, torch_dev):
    import paper_1302_4587_amd as lm
    from paper_1302_4587_amd import _lib as L
    g = lmgen.er(64, 200, seed=1)
    with lm.Server(ctx, hbm_budget_bytes=1 << 30, queue_cap=2, max_resident=1) as srv:
        with pytest.raises(lm.LMError) as e:
            srv.poll(12345)
        assert e.value.status == L.LM_ENOTFOUND
        t = srv.submit(g.row_ptr, g.col, g.w, seed=1)
        r = srv.wait(t, 60000)
        assert r is not None and np.array_equal(r[0], oracle.local_max_graph(g, 1)[0])
        with pytest.raises(lm.LMError) as e:
            srv.poll(t)  # retired
        assert e.value.status == L.LM_ENOTFOUND
    with lm.Server(ctx, hbm_budget_bytes=1 << 12) as tiny:
        with pytest.raises(lm.LMError) as e:
            tiny.submit(g.row_ptr, g.col, g.w, seed=1)
        assert e.value.status == L.LM_ETOOBIG
