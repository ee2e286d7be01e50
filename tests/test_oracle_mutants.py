"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/lm_oracle.c`` into a temporary directory, applies
one plausible slip (a flipped compare, a swapped index, a dropped term or
step), compiles it on the CPU and runs the pins of ``test_oracle_pins``
against it. A pin set that lets a mutant through is too weak.
"""
import ctypes
import multiprocessing as mp
import os
import subprocess

import numpy as np
import pytest

import lmgen
from tests import _pyref as ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lm_oracle.c")

MUTANTS = {
    "hash_compare_reversed": ("return a->h > b->h;", "return a->h < b->h;"),
    "weight_compare_dropped": ("  if (a->w > b->w) return 1;\n  if (a->w < b->w) return 0;\n", ""),
    "weight_compare_reversed": ("if (a->w > b->w) return 1;\n  if (a->w < b->w) return 0;",
                                "if (a->w < b->w) return 1;\n  if (a->w > b->w) return 0;"),
    "pair_halves_swapped": ("((uint64_t)(uint32_t)lo << 32) | (uint64_t)(uint32_t)hi",
                            "((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo"),
    "seed_premix_dropped": ("lmo_mix64(pair ^ lmo_seed_mix(seed))", "lmo_mix64(pair ^ seed)"),
    "seed_premix_added": ("lmo_mix64(seed ^ LMO_GAMMA)", "lmo_mix64(seed + LMO_GAMMA)"),
    "mix_constant_typo": ("0xBF58476D1CE4E5B9ULL", "0xBF58476D1CE4E5B8ULL"),
    "mix_shift_typo": ("z ^ (z >> 27)", "z ^ (z >> 26)"),
    "candidate_reset_dropped": ("      C[e.lo] = LMO_NONE;\n      C[e.hi] = LMO_NONE;\n", ""),
    "pass1_hi_endpoint_dropped": (
        "      if (C[e->hi] == LMO_NONE || key_greater(e, &E[C[e->hi]])) C[e->hi] = j;\n", ""),
    "mutual_check_one_sided": ("C[e->lo] == j && C[e->hi] == j", "C[e->lo] == j || C[e->hi] == j"),
    "removal_needs_both_ends": ("if (mate[e.lo] != -1 || mate[e.hi] != -1) continue;",
                                "if (mate[e.lo] != -1 && mate[e.hi] != -1) continue;"),
    "candidate_picks_lightest_at_lo": ("key_greater(e, &E[C[e->lo]])", "key_greater(&E[C[e->lo]], e)"),
    "live_vertices_one_endpoint": ("      if (seen[E[j].hi] != t) {\n        seen[E[j].hi] = t;\n        ++vt;\n      }\n", ""),
    "live_vertices_counted_once_ever": ("if (seen[E[j].lo] != t) {", "if (seen[E[j].lo] == 0) {"),
    "log_counts_survivors": ("log[3 * (t - 1) + 0] = m;", "log[3 * (t - 1) + 0] = keep;"),
}

_P64 = ctypes.POINTER(ctypes.c_int64)
_P32 = ctypes.POINTER(ctypes.c_int32)
_PF = ctypes.POINTER(ctypes.c_float)


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new, 1))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(path)])
    lib = ctypes.CDLL(str(so))
    lib.lmo_mix64.argtypes = [ctypes.c_uint64]
    lib.lmo_mix64.restype = ctypes.c_uint64
    lib.lmo_edge_hash.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
    lib.lmo_edge_hash.restype = ctypes.c_uint64
    lib.lmo_local_max.argtypes = [ctypes.c_int64, _P64, _P32, _PF, ctypes.c_uint64, _P32, _P64, ctypes.c_int64]
    lib.lmo_local_max.restype = ctypes.c_int64
    return lib


def _solve(lib, g, seed):
    rp = np.ascontiguousarray(g.row_ptr, np.int64)
    cc = np.ascontiguousarray(g.col, np.int32)
    ww = np.ascontiguousarray(g.w, np.float32)
    mate = np.empty(g.n, np.int32)
    log = np.zeros((4096, 3), np.int64)
    t = lib.lmo_local_max(g.n, rp.ctypes.data_as(_P64), cc.ctypes.data_as(_P32), ww.ctypes.data_as(_PF), seed,
                          mate.ctypes.data_as(_P32), log.ctypes.data_as(_P64), 4096)
    return mate, log[:max(t, 0)], t


def _pins_fail(lib) -> bool:
    for seed, idx, val in ref.load_kat():
        if lib.lmo_mix64((seed + (idx + 1) * ref.GAMMA) & ref.M64) != val:
            return True
    rng = np.random.default_rng(77)
    for kind in ("uniform", "tied", "unit"):
        for _ in range(25):
            n = int(rng.integers(3, 40))
            m = int(rng.integers(1, min(n * (n - 1) // 2, 3 * n) + 1))
            g = lmgen.er(n, m, int(rng.integers(1, 2**62)))
            if kind != "uniform":
                lo, hi, _ = ref.undirected_edges(g)
                w = np.ones(len(lo), np.float32) if kind == "unit" else rng.integers(1, 4, len(lo)).astype(np.float32)
                g = lmgen.from_edges(n, np.stack([lo, hi], 1), w)
            seed = int(rng.integers(1, 2**62))
            mate, log, t = _solve(lib, g, seed)
            if t < 0 or not np.array_equal(mate, ref.greedy(g, seed)) or not ref.is_valid_maximal(g, mate):
                return True
            if not np.array_equal(log, ref.local_max_log(g, seed)[1]):
                return True
    k = 9  # increasing path: ceil(k/2) iterations
    g = lmgen.from_edges(k + 1, [[i, i + 1] for i in range(k)], np.arange(1, k + 1))
    mate, log, t = _solve(lib, g, 1)
    if t != 5:
        return True
    return False


def _child(so_dir, name, old, new, q):
    import pathlib
    q.put(_pins_fail(_build(pathlib.Path(so_dir), name, old, new)))


def _run_pins(tmp_path, name, old, new, limit_s=90.0):
    """Runs the pins on a mutant in a child process. A mutant whose loop never
    ends (no edge is ever removed) counts as caught: the iteration count is
    bounded by the edge count for the real method."""
    ctx = mp.get_context("spawn")  # a forked child could inherit a busy OpenMP pool (generators)
    q = ctx.Queue()
    p = ctx.Process(target=_child, args=(str(tmp_path), name, old, new, q))
    p.start()
    p.join(limit_s)
    if p.is_alive():
        p.kill()
        p.join()
        return True
    return bool(q.get()) if not q.empty() else True


def test_unmodified_oracle_passes_the_pins(tmp_path):
    assert not _run_pins(tmp_path, "identity", "lmo_", "lmo_")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    assert _run_pins(tmp_path, name, old, new, limit_s=20.0), f"pins did not catch mutant {name}"
