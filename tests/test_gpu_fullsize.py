"""Full-size parity in the launch configurations the benchmark times.

RGG 2^24 (average degree 10, w = 1 - distance): mate[] and the phase log
against the oracle, element by element. R-MAT scale 24 (edge factor 16,
unit weights, so the order is the tie-break hash alone), solved as the bench
solves it (no weight array: the unweighted kernels): mate[] and the phase log
against the oracle on the unit-weight graph, element by element; the same
graph with its all-ones weight array (the weighted kernels) must give the
same mate[], and passes the greedy certificate (every matched edge is the
largest-key edge among those not blocked by a larger matched edge). The
matched weight w(M) of the RGG solve is checked against an exactly rounded
sum over the oracle's matching.
"""
import numpy as np
import pytest

import lmgen
import oracle
from tests import _pyref as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4587_amd as lm
    c = lm.Context(0)
    yield c
    c.close()


def _solve_device(ctx, g, seed, weights=True, **kw):
    import torch
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev) if weights else None
    mate, st = ctx.match(rp, col, w, seed=seed, **kw)
    out = mate.cpu().numpy()
    del rp, col, w, mate
    torch.cuda.empty_cache()
    return out, st


def _log_invariants(st, mate):
    log = st.log
    assert st.phases == len(log) and st.phases >= 1
    assert np.all(np.diff(log[:, 0]) < 0), "live entries must shrink every phase"
    assert int(log[:, 2].sum()) == int((mate >= 0).sum()) // 2 == st.matched_edges


def test_rgg_2p24_equals_oracle(ctx):
    print("case: rgg n=2^24 avg_degree=10 seed=1 (bench workload)", flush=True)
    g = lmgen.rgg(1 << 24, 10.0, 1)
    mate, st = _solve_device(ctx, g, 1)
    ref_mate, ref_log = oracle.local_max_graph(g, 1)
    if not np.array_equal(mate, ref_mate):
        bad = np.flatnonzero(mate != ref_mate)
        raise AssertionError(f"{len(bad)} vertices differ, first {bad[:5]}")
    assert st.phases == len(ref_log)
    assert np.array_equal(st.log[:, 0], 2 * ref_log[:, 0])
    assert np.array_equal(st.log[:, 1], ref_log[:, 1])
    assert np.array_equal(st.log[:, 2], ref_log[:, 2])
    _log_invariants(st, mate)
    # w(M) at full size (LM_WEIGHT_SUM), against math.fsum over the oracle's matching
    print("case: rgg n=2^24 matched weight", flush=True)
    mate2, st2 = _solve_device(ctx, g, 1, weight_sum=True)
    assert np.array_equal(mate2, ref_mate)
    exact, abs_sum, edges = ref.matching_weight_exact(g, ref_mate)
    tol = 2 * edges * 2.0**-53 * abs_sum + 2.0**-52 * abs(exact)
    assert abs(st2.matched_weight - exact) <= tol, (st2.matched_weight, exact)


@pytest.fixture(scope="module")
def rmat24():
    print("case: generating rmat scale=24 edge_factor=16 unit weights seed=1", flush=True)
    return lmgen.rmat(24, 16, seed=1)


def test_rmat_scale24_unweighted_equals_oracle(ctx, rmat24):
    g = rmat24
    print("case: rmat scale=24 unweighted (bench launch configuration) vs oracle", flush=True)
    mate, st = _solve_device(ctx, g, 1, weights=False)
    ref_mate, ref_log = oracle.local_max_graph(g, 1)
    if not np.array_equal(mate, ref_mate):
        bad = np.flatnonzero(mate != ref_mate)
        raise AssertionError(f"{len(bad)} vertices differ, first {bad[:5]}")
    assert st.phases == len(ref_log)
    assert np.array_equal(st.log[:, 0], 2 * ref_log[:, 0])
    assert np.array_equal(st.log[:, 1], ref_log[:, 1])
    assert np.array_equal(st.log[:, 2], ref_log[:, 2])
    _log_invariants(st, mate)


def test_rmat_scale24_weight_array_certificate(ctx, rmat24):
    g = rmat24
    print("case: rmat scale=24 with the all-ones weight array", flush=True)
    mate, st = _solve_device(ctx, g, 1)
    viol = oracle.greedy_certificate(g.n, g.row_ptr, g.col, g.w, 1, mate)
    assert viol == 0, f"{viol} certificate violations"
    _log_invariants(st, mate)
    unw, _ = _solve_device(ctx, g, 1, weights=False)
    assert np.array_equal(mate, unw), "weighted and unweighted kernels differ on unit weights"
