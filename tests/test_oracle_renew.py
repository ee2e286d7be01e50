"""Pins of the oracle's renewed-key mode (fresh tie-break keys every phase).

The paper's Lemma 1 assumes random noise drawn anew in every iteration (its
footnote; Section 2.1, step 1 of the CREW algorithm), and Section 4 asks
whether renewing it matters. In renewed mode iteration t breaks ties with
H_t(lo, hi) = mix(((lo << 32) | hi) XOR S_t), S_t = mix(S + t * GAMMA),
S = mix(seed XOR GAMMA). The greedy pin of the fixed-key mode no longer
applies, so these pins carry parity instead:

* the pure-Python definition (tests/_pyref.py, Section 1's local max edge by
  edge) with its own big-integer SplitMix64 gives the same mate[] and phase
  log on random graphs with unit, tied, integer and signed weights;
* known answers of H_t from an independent big-integer evaluation;
* with distinct weights the hash never decides: renewed = fixed = greedy;
* validity, maximality, and the 1/2 bound against a brute-force maximum
  weight matching on tiny graphs (Section 1, Preis' family);
* Lemma 1 in every phase: with fresh keys the mean fraction of live edges a
  phase removes is at least 1/2 on unit-weight graphs;
* entry order within rows does not matter;
* planted mistakes in the renewed path (stale or frozen phase seed, a seed
  stream with the wrong increment) are caught by these pins.
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


def _h_phase_np(seed, t, lo, hi):
    S = ref.seed_mix(seed)
    st = ref.mix64((S + t * ref.GAMMA) & ref.M64)
    pair = (lo.astype(np.uint64) << np.uint64(32)) | hi.astype(np.uint64)
    return ref.mix64_np(pair ^ np.uint64(st))


def _pyref_renewed(g, seed):
    def key_of_phase(t, lo, hi, w):
        return ref.edge_ranks(lo, hi, w, seed, hash_fn=lambda a, b: _h_phase_np(seed, t, a, b))
    return ref.local_max_log(g, seed, key_of_phase=key_of_phase)


def _random_graph(rng, kind):
    n = int(rng.integers(2, 60))
    m = int(rng.integers(1, min(n * (n - 1) // 2, 4 * n) + 1))
    g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
    if kind == "uniform":
        return g
    lo, hi, _ = ref.undirected_edges(g)
    if kind == "unit":
        w = np.ones(len(lo), np.float32)
    elif kind == "tied":
        w = rng.integers(1, 4, len(lo)).astype(np.float32)
    else:
        w = rng.choice(np.array([-2.5, -0.0, 0.0, 1e-30, 3.0], np.float32), len(lo))
    return lmgen.from_edges(n, np.stack([lo, hi], 1), w)


@pytest.mark.parametrize("kind", ["unit", "tied", "signed", "uniform"])
def test_renewed_equals_definition(kind):
    rng = np.random.default_rng({"unit": 31, "tied": 32, "signed": 33, "uniform": 34}[kind])
    for _ in range(40):
        g = _random_graph(rng, kind)
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        mate, log = oracle.local_max_graph(g, seed, renew=True)
        pm, plog = _pyref_renewed(g, seed)
        assert np.array_equal(mate, pm)
        assert np.array_equal(log, plog)
        assert ref.is_valid_maximal(g, mate)


def test_phase_hash_known_answers():
    for seed, t, lo, hi in [(1, 1, 0, 1), (1, 2, 0, 1), (1, 7, 3, 4095), (0, 1, 0, 1), (2**64 - 1, 3, 5, 9)]:
        S = ref.seed_mix(seed)
        st = ref.mix64((S + t * ref.GAMMA) & ref.M64)
        want = ref.mix64((((lo << 32) | hi) ^ st) & ref.M64)
        assert oracle.edge_hash_phase(seed, t, lo, hi) == want


def test_distinct_weights_renewed_equals_fixed_equals_greedy():
    for seed in (1, 5, 2**40 + 3):
        for g in (lmgen.er(3000, 12000, seed=seed), lmgen.rgg(5000, 10.0, seed=seed)):
            lo, hi, w = ref.undirected_edges(g)
            if len(np.unique(w)) != len(w):  # the rgg's weights repeat: keep the distinct case pure
                wd = np.arange(1, len(lo) + 1, dtype=np.float32) * np.float32(2**-24)
                g = lmgen.from_edges(g.n, np.stack([lo, hi], 1), wd)
            a, _ = oracle.local_max_graph(g, seed, renew=True)
            b, _ = oracle.local_max_graph(g, seed, renew=False)
            assert np.array_equal(a, b)
            assert np.array_equal(a, ref.greedy(g, seed))


def test_half_bound_against_brute_force():
    rng = np.random.default_rng(41)
    for _ in range(60):
        n = int(rng.integers(2, 11))
        m = int(rng.integers(1, n * (n - 1) // 2 + 1))
        g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
        lo, hi, _ = ref.undirected_edges(g)
        w = rng.integers(1, 4, len(lo)).astype(np.float32)  # ties: the renewed keys decide
        g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
        mate, _ = oracle.local_max_graph(g, int(rng.integers(1, 2**62)), renew=True)
        assert ref.is_valid_maximal(g, mate)
        assert 2.0 * ref.matching_weight(g, mate) >= ref.brute_mwm(g) - 1e-9


def test_lemma1_every_phase_removes_half():
    """Unit weights: the keys are the only order. Lemma 1 (fresh random keys in
    every phase): a phase removes at least half of the live edges in
    expectation. Averaged over seeds, every phase with enough edges does."""
    fr = {}
    for s in range(24):
        g = lmgen.er(3000, 15000, seed=100 + s, weights="unit")
        _, log = oracle.local_max_graph(g, 7 + s, renew=True)
        E = list(log[:, 0]) + [0]
        for t in range(len(log)):
            if E[t] >= 400:
                fr.setdefault(t, []).append(1.0 - E[t + 1] / E[t])
    assert len(fr) >= 2
    for t, xs in fr.items():
        assert np.mean(xs) >= 0.5, f"phase {t + 1}: mean removed fraction {np.mean(xs):.3f}"


def test_row_order_does_not_matter():
    rng = np.random.default_rng(43)
    g = lmgen.er(2000, 9000, seed=9, weights="unit")
    col = g.col.copy()
    for v in range(g.n):
        a, b = g.row_ptr[v], g.row_ptr[v + 1]
        col[a:b] = rng.permutation(col[a:b])
    mate0, log0 = oracle.local_max(g.n, g.row_ptr, g.col, g.w, 3, renew=True)
    mate1, log1 = oracle.local_max(g.n, g.row_ptr, col, g.w, 3, renew=True)
    assert np.array_equal(mate0, mate1) and np.array_equal(log0, log1)


# ---- planted mistakes in the renewed path

RENEW_MUTANTS = {
    "phase_seed_stale": ("E[j].h = lmo_edge_hash_phase(seed, t, E[j].lo, E[j].hi);",
                         "E[j].h = lmo_edge_hash_phase(seed, t - 1, E[j].lo, E[j].hi);"),
    "phase_seed_frozen": ("E[j].h = lmo_edge_hash_phase(seed, t, E[j].lo, E[j].hi);",
                          "E[j].h = lmo_edge_hash_phase(seed, 1, E[j].lo, E[j].hi);"),
    "stream_increment_wrong": ("lmo_seed_mix(seed) + (uint64_t)t * LMO_GAMMA",
                               "lmo_seed_mix(seed) + (uint64_t)t"),
    "renewal_skipped": ("    if (renew) /* the keys of this iteration */", "    if (0) /* the keys of this iteration */"),
}

_P64 = ctypes.POINTER(ctypes.c_int64)
_P32 = ctypes.POINTER(ctypes.c_int32)
_PF = ctypes.POINTER(ctypes.c_float)


def _mutant_fails_pins(so_path):
    lib = ctypes.CDLL(so_path)
    lib.lmo_local_max_ex.argtypes = [ctypes.c_int64, _P64, _P32, _PF, ctypes.c_uint64, ctypes.c_int, _P32, _P64,
                                     ctypes.c_int64]
    lib.lmo_local_max_ex.restype = ctypes.c_int64
    rng = np.random.default_rng(51)
    for kind in ("unit", "tied"):
        for _ in range(20):
            g = _random_graph(rng, kind)
            seed = int(rng.integers(1, 2**62))
            mate = np.empty(g.n, np.int32)
            log = np.zeros((4096, 3), np.int64)
            t = lib.lmo_local_max_ex(g.n, np.ascontiguousarray(g.row_ptr).ctypes.data_as(_P64),
                                     np.ascontiguousarray(g.col).ctypes.data_as(_P32),
                                     np.ascontiguousarray(g.w).ctypes.data_as(_PF), seed, 1,
                                     mate.ctypes.data_as(_P32), log.ctypes.data_as(_P64), 4096)
            pm, plog = _pyref_renewed(g, seed)
            if t < 0 or not np.array_equal(mate, pm) or not np.array_equal(log[:t], plog):
                return True
    return False


def _child(so, q):
    q.put(_mutant_fails_pins(so))


@pytest.mark.parametrize("name", ["identity"] + sorted(RENEW_MUTANTS))
def test_renew_mutants_are_caught(tmp_path, name):
    src = open(SRC).read()
    if name != "identity":
        old, new = RENEW_MUTANTS[name]
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
    p.join(60)
    caught = True
    if p.is_alive():
        p.kill()
        p.join()
    elif not q.empty():
        caught = bool(q.get())
    if name == "identity":
        assert not caught, "the unmodified oracle must pass the renewed-key pins"
    else:
        assert caught, f"pins did not catch mutant {name}"
