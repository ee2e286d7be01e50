"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every check here is independent of the oracle's own code:
  * SplitMix64 published vectors (golden/splitmix64_kat.txt) pin the hash;
  * the greedy scan (paper, Section 3) must equal local max under a strict key;
  * validity and maximality (paper, Section 1);
  * 1/2-approximation of maximum weight (paper, Section 1, Preis' family)
    against brute force on tiny graphs;
  * closed forms for paths, stars, triangles, disjoint edges;
  * Lemma 1: at least half the edges go in the first iteration, in
    expectation, for unit weights (about three quarters observed, footnote 4);
  * iteration-log consistency.
"""
import math

import numpy as np
import pytest

import lmgen
import oracle
from tests import _pyref as ref


# ---------------------------------------------------------------- hash pins

def test_splitmix_python_matches_published_vectors():
    for seed, idx, val in ref.load_kat():
        assert ref.splitmix_outputs(seed, idx + 1)[idx] == val


def test_oracle_mix_matches_published_vectors():
    for seed, idx, val in ref.load_kat():
        state = (seed + (idx + 1) * ref.GAMMA) & ref.M64
        assert oracle.mix64(state) == val


def _seed_for_state(state: int) -> int:
    """The seed whose mix input (seed XOR gamma) is the given generator state."""
    return (state ^ ref.GAMMA) & ref.M64


def test_oracle_seed_mix_hits_published_vectors():
    # seed_mix(s) = mix(s XOR gamma): with s = state XOR gamma for the state
    # behind a published output, seed_mix must return that output.
    for seed, idx, val in ref.load_kat():
        state = (seed + (idx + 1) * ref.GAMMA) & ref.M64
        assert oracle.seed_mix(_seed_for_state(state)) == val
    # seed 0: 0 XOR gamma = 0 + gamma, the generator's own first output
    assert oracle.seed_mix(0) == [v for s, i, v in ref.load_kat() if s == 0 and i == 0][0]


def test_edge_hash_hits_published_vectors():
    # Choose the hash seed so that S = seed_mix(seed) is a published output,
    # and the pair so that pair XOR S equals the state behind another
    # published output; then H must be exactly that output.
    for gseed in (0, 1234567):
        outs = [v for s, i, v in sorted(ref.load_kat()) if s == gseed]
        seed = _seed_for_state((gseed + ref.GAMMA) & ref.M64)
        S = outs[0]
        assert oracle.seed_mix(seed) == S
        for k in range(1, len(outs)):
            state = (gseed + (k + 1) * ref.GAMMA) & ref.M64
            pair = state ^ S
            lo = pair >> 32
            hi = pair & 0xFFFFFFFF
            lo_s = lo - (1 << 32) if lo >= 1 << 31 else lo
            hi_s = hi - (1 << 32) if hi >= 1 << 31 else hi
            assert oracle.edge_hash(seed, lo_s, hi_s) == outs[k]


def test_edge_hash_contract_values():
    # known answers of the tie-break contract H(seed, lo, hi), stated with the
    # key definition and derived from it with big-integer arithmetic
    for seed, lo, hi, val in ref.load_edge_hash_kat():
        assert ref.edge_hash(seed, lo, hi) == val
        assert oracle.edge_hash(seed, lo, hi) == val


def test_edge_hash_numpy_reference_agrees():
    rng = np.random.default_rng(5)
    lo = rng.integers(0, 1 << 31, 200)
    hi = rng.integers(0, 1 << 31, 200)
    for seed in (0, 1, 2**64 - 1):
        h = ref.edge_hash_np(seed, lo, hi)
        for a, b, x in zip(lo[:20], hi[:20], h[:20]):
            assert oracle.edge_hash(seed, int(a), int(b)) == int(x)


# ---------------------------------------------------------------- graphs

def _random_graph(rng, n, m, wkind):
    g = lmgen.er(n, m, int(rng.integers(1, 2**63)))
    if wkind == "tied":
        lo, hi, _ = ref.undirected_edges(g)
        w = rng.integers(1, 4, len(lo)).astype(np.float32)
        return lmgen.from_edges(n, np.stack([lo, hi], 1), w)
    if wkind == "unit":
        return lmgen.Graph(g.n, g.row_ptr, g.col, np.ones_like(g.w))
    if wkind == "signed":
        lo, hi, _ = ref.undirected_edges(g)
        w = rng.choice(np.array([-1.5, -0.0, 0.0, 0.25, 2.0], dtype=np.float32), len(lo))
        return lmgen.from_edges(n, np.stack([lo, hi], 1), w)
    if wkind == "denormal":
        lo, hi, _ = ref.undirected_edges(g)
        return lmgen.from_edges(n, np.stack([lo, hi], 1), rng.choice(DENORMALS, len(lo)))
    return g


# subnormal fp32 weights (and their neighbours): a compare that flushed them to
# zero would tie them with +-0 and hand the decision to the hash
DENORMALS = np.array([-2.0**-140, -2.0**-149, -0.0, 0.0, 2.0**-149, 2.0**-148, 2.0**-130, 2.0**-127,
                      2.0**-126, 1e-30], dtype=np.float32)


@pytest.mark.parametrize("wkind", ["uniform", "tied", "unit", "signed", "denormal"])
def test_oracle_equals_greedy(wkind):
    rng = np.random.default_rng({"uniform": 1, "tied": 2, "unit": 3, "signed": 4, "denormal": 5}[wkind])
    for _ in range(120):
        n = int(rng.integers(2, 60))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 4 * n) + 1))
        g = _random_graph(rng, n, m, wkind)
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        mate, log = oracle.local_max_graph(g, seed)
        assert np.array_equal(mate, ref.greedy(g, seed)), (n, m, seed)
        assert ref.is_valid_maximal(g, mate)


def test_oracle_equals_greedy_medium():
    g = lmgen.er(4096, 32768, 1)
    mate, log = oracle.local_max_graph(g, 1)
    assert np.array_equal(mate, ref.greedy(g, 1))


def test_oracle_half_approximation_bruteforce():
    rng = np.random.default_rng(11)
    for _ in range(60):
        n = int(rng.integers(2, 13))
        m = int(rng.integers(1, n * (n - 1) // 2 + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**63)))
        mate, _ = oracle.local_max_graph(g, int(rng.integers(1, 2**63)))
        opt = ref.brute_mwm(g)
        got = ref.matching_weight(g, mate)
        assert 2.0 * got >= opt - 1e-9, (got, opt)
        # unit weights: at least half the maximum cardinality
        gu = lmgen.Graph(g.n, g.row_ptr, g.col, np.ones_like(g.w))
        mu, _ = oracle.local_max_graph(gu, 7)
        assert 2 * ((mu >= 0).sum() // 2) >= ref.brute_mwm(gu) - 1e-9


# ---------------------------------------------------------------- closed forms

def test_empty_graph():
    g = lmgen.from_edges(5, np.zeros((0, 2)), np.zeros(0))
    mate, log = oracle.local_max_graph(g, 1)
    assert (mate == -1).all() and len(log) == 0


def test_disjoint_edges_one_phase():
    k = 50
    e = np.array([[2 * i, 2 * i + 1] for i in range(k)])
    g = lmgen.from_edges(2 * k + 3, e, np.linspace(0.1, 1.0, k))
    mate, log = oracle.local_max_graph(g, 3)
    assert len(log) == 1 and log[0, 2] == k
    assert all(mate[2 * i] == 2 * i + 1 for i in range(k))
    assert (mate[2 * k:] == -1).all()


def test_star_center_takes_heaviest_leaf():
    k = 17
    rng = np.random.default_rng(2)
    w = rng.permutation(np.arange(1, k + 1)).astype(np.float32)
    e = np.array([[0, i + 1] for i in range(k)])
    g = lmgen.from_edges(k + 1, e, w)
    mate, log = oracle.local_max_graph(g, 9)
    assert len(log) == 1
    assert mate[0] == int(np.argmax(w)) + 1
    assert (mate >= 0).sum() == 2


def test_star_unit_weights_follow_hash():
    k = 33
    e = np.array([[0, i + 1] for i in range(k)])
    g = lmgen.from_edges(k + 1, e, np.ones(k))
    for seed in (1, 2, 3):
        mate, log = oracle.local_max_graph(g, seed)
        h = [oracle.edge_hash(seed, 0, i + 1) for i in range(k)]
        assert mate[0] == int(np.argmax(np.array(h, dtype=np.uint64))) + 1
        assert len(log) == 1


@pytest.mark.parametrize("k", [1, 2, 3, 7, 10, 31])
def test_increasing_path_phases(k):
    # path 0-1-...-k, edge i = (i, i+1) with weight i+1: the heaviest edge is
    # the only local max each iteration, so ceil(k/2) iterations, matching
    # e_k, e_{k-2}, ...
    e = np.array([[i, i + 1] for i in range(k)])
    g = lmgen.from_edges(k + 1, e, np.arange(1, k + 1))
    mate, log = oracle.local_max_graph(g, 1)
    assert len(log) == math.ceil(k / 2)
    matched = {i for i in range(k) if mate[i] == i + 1}
    assert matched == set(range(k - 1, -1, -2))
    assert all(r[2] == 1 for r in log)


def test_alternating_path_one_phase():
    k = 41
    e = np.array([[i, i + 1] for i in range(k)])
    w = np.where(np.arange(k) % 2 == 0, 2.0, 1.0)
    g = lmgen.from_edges(k + 1, e, w)
    mate, log = oracle.local_max_graph(g, 1)
    assert len(log) == 1
    assert all(mate[i] == i + 1 for i in range(0, k, 2))


def test_triangle_heaviest_edge():
    g = lmgen.from_edges(3, [[0, 1], [1, 2], [0, 2]], [0.5, 0.9, 0.7])
    mate, log = oracle.local_max_graph(g, 1)
    assert list(mate) == [-1, 2, 1] and len(log) == 1


# ---------------------------------------------------------------- Lemma 1, log

def test_lemma1_removal_fraction_unit_weights():
    fr = []
    for s in range(40):
        g = lmgen.er(2000, 16000, 100 + s, weights="unit")
        _, log = oracle.local_max_graph(g, 500 + s)
        e1 = log[0, 0]
        e2 = log[1, 0] if len(log) > 1 else 0
        fr.append(1.0 - e2 / e1)
    mean = float(np.mean(fr))
    assert mean >= 0.5
    assert 0.6 <= mean <= 0.95  # about 3/4 per footnote 4


@pytest.mark.parametrize("wkind", ["uniform", "tied", "unit", "signed", "denormal"])
def test_phase_log_equals_edge_definition(wkind):
    # every column of the oracle's log, phase by phase, against the
    # edge-by-edge local-max definition (ranks, not candidates)
    rng = np.random.default_rng({"uniform": 21, "tied": 22, "unit": 23, "signed": 24, "denormal": 25}[wkind])
    for _ in range(60):
        n = int(rng.integers(2, 200))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 5 * n) + 1))
        g = _random_graph(rng, n, m, wkind)
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        mate, log = oracle.local_max_graph(g, seed)
        rm, rlog = ref.local_max_log(g, seed)
        assert np.array_equal(mate, rm)
        assert np.array_equal(log, rlog), (n, m, seed)


def test_phase_log_first_row_counts_the_input():
    # |E_1| = m and V_1 = vertices of positive degree, on every family
    for g in (lmgen.er(3000, 2000, 4), lmgen.rgg(4000, 10.0, 2), lmgen.rmat(12, 16, seed=3),
              lmgen.er(500, 0, 1)):
        _, log = oracle.local_max_graph(g, 1)
        if g.m == 0:
            assert len(log) == 0
            continue
        assert log[0, 0] == g.m
        assert log[0, 1] == int((np.diff(g.row_ptr) > 0).sum())


def test_phase_log_closed_forms():
    # star of k leaves: one phase, k edges, k + 1 live vertices
    k = 23
    g = lmgen.from_edges(k + 5, [[3, i] for i in range(k + 5) if i != 3][:k], np.arange(1, k + 1))
    _, log = oracle.local_max_graph(g, 1)
    assert log.tolist() == [[k, k + 1, 1]]
    # k disjoint edges: one phase, 2k live vertices, k matched
    e = [[2 * i, 2 * i + 1] for i in range(k)]
    _, log = oracle.local_max_graph(lmgen.from_edges(2 * k + 4, e, np.ones(k)), 5)
    assert log.tolist() == [[k, 2 * k, k]]
    # increasing path of k edges: |E_t| = k - 2(t-1), V_t = k - 2t + 3, one match per phase
    for k in (1, 2, 5, 12, 33):
        g = lmgen.from_edges(k + 1, [[i, i + 1] for i in range(k)], np.arange(1, k + 1))
        _, log = oracle.local_max_graph(g, 1)
        want = [[k - 2 * (t - 1), k - 2 * t + 3, 1] for t in range(1, math.ceil(k / 2) + 1)]
        assert log.tolist() == want, k
    # triangle with a light pendant edge at vertex 0: phase 1 matches the
    # heaviest triangle edge {1,2} and kills {0,1} and {0,2}; the pendant
    # edge {0,3} is alone in phase 2
    g = lmgen.from_edges(4, [[0, 1], [1, 2], [0, 2], [0, 3]], [0.5, 0.9, 0.7, 0.1])
    mate, log = oracle.local_max_graph(g, 1)
    assert log.tolist() == [[4, 4, 1], [1, 2, 1]]
    assert mate.tolist() == [3, 2, 1, 0]


def test_denormal_weights_order_by_value():
    # a star whose leaves carry distinct subnormal weights: the centre takes the
    # largest by value, never a tie broken by the hash
    w = np.array([2.0**-149, 2.0**-140, 2.0**-135, 2.0**-133, 2.0**-128], dtype=np.float32)
    for perm in ([0, 1, 2, 3, 4], [4, 3, 2, 1, 0], [2, 4, 0, 3, 1]):
        g = lmgen.from_edges(6, [[0, i + 1] for i in range(5)], w[perm])
        for seed in (1, 2, 3):
            mate, _ = oracle.local_max_graph(g, seed)
            assert mate[0] == 1 + perm.index(4)


def test_log_consistency():
    for g in (lmgen.er(3000, 20000, 4), lmgen.rgg(4000, 10.0, 2), lmgen.rmat(12, 16, seed=3)):
        mate, log = oracle.local_max_graph(g, 1)
        assert log[0, 0] == g.m
        assert (np.diff(log[:, 0]) < 0).all()
        assert int(log[:, 2].sum()) == int((mate >= 0).sum()) // 2
        assert (log[:, 2] >= 1).all()  # the globally heaviest live edge is always local max
        assert (log[:, 1] <= g.n).all()


def test_batch_equals_alone():
    b = lmgen.er_batch(12, 3, lg_lo=4, lg_hi=9)
    seeds = np.arange(12, dtype=np.uint64) * 7 + 1
    mate, ph = oracle.local_max_batch(b.vtx_off, b.row_ptr, b.col, b.w, seeds=seeds)
    for g in range(b.graphs):
        gg = b.graph(g)
        m1, l1 = oracle.local_max_graph(gg, int(seeds[g]))
        assert np.array_equal(mate[b.vtx_off[g]:b.vtx_off[g + 1]], m1)
        assert ph[g] == len(l1)


# ---------------------------------------------------------------- certificate

def test_certificate_accepts_oracle_and_rejects_others():
    g = lmgen.er(500, 3000, 8)
    mate, _ = oracle.local_max_graph(g, 5)
    assert oracle.greedy_certificate(g.n, g.row_ptr, g.col, g.w, 5, mate) == 0
    # distinct weights: the hash never decides, any seed certifies the same
    assert oracle.greedy_certificate(g.n, g.row_ptr, g.col, g.w, 6, mate) == 0
    # greedy under a different seed on a unit graph is maximal but not ours
    gu = lmgen.Graph(g.n, g.row_ptr, g.col, np.ones_like(g.w))
    other = ref.greedy(gu, 99)
    assert ref.is_valid_maximal(gu, other)
    assert oracle.greedy_certificate(gu.n, gu.row_ptr, gu.col, gu.w, 5, other) > 0
    # drop one matched edge: maximality fails
    bad = mate.copy()
    v = int(np.flatnonzero(bad >= 0)[0])
    bad[bad[v]] = -1
    bad[v] = -1
    assert oracle.greedy_certificate(g.n, g.row_ptr, g.col, g.w, 5, bad) > 0


def test_oracle_rejects_bad_input():
    g = lmgen.from_edges(3, [[0, 1]], [1.0])
    col = g.col.copy()
    col[0] = 0  # self-loop
    with pytest.raises(ValueError):
        oracle.local_max(g.n, g.row_ptr, col, g.w, 1)
    col[0] = 7  # out of range
    with pytest.raises(ValueError):
        oracle.local_max(g.n, g.row_ptr, col, g.w, 1)
