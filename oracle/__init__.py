"""CPU oracle for local-max matching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding) never imports it, and the two share no code.

The oracle is plain single-threaded C (``lm_oracle.c``) following the
paper's sequential model (Section 2): a candidate per vertex, three passes per
iteration, candidates initialised once. Ties are broken by the fixed key
(weight, H(seed, lo, hi)) with H built from the SplitMix64 output function.
See the header of ``lm_oracle.c`` for the exact definition and the pins that
check it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblm_oracle.so")

EINVAL = -1
ENOMEM = -2


def build(force: bool = False) -> str:
    """Compile lm_oracle.c with gcc -O2 (no fast-math) into liblm_oracle.so."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None
_P64 = ctypes.POINTER(ctypes.c_int64)
_P32 = ctypes.POINTER(ctypes.c_int32)
_PF = ctypes.POINTER(ctypes.c_float)
_PU64 = ctypes.POINTER(ctypes.c_uint64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.lmo_mix64.argtypes = [ctypes.c_uint64]
        lib.lmo_mix64.restype = ctypes.c_uint64
        lib.lmo_seed_mix.argtypes = [ctypes.c_uint64]
        lib.lmo_seed_mix.restype = ctypes.c_uint64
        lib.lmo_edge_hash.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32]
        lib.lmo_edge_hash.restype = ctypes.c_uint64
        lib.lmo_local_max.argtypes = [ctypes.c_int64, _P64, _P32, _PF, ctypes.c_uint64, _P32, _P64, ctypes.c_int64]
        lib.lmo_local_max.restype = ctypes.c_int64
        lib.lmo_local_max_batch.argtypes = [ctypes.c_int64, _P64, _P64, _P32, _PF, _PU64, ctypes.c_uint64,
                                            _P32, _P64]
        lib.lmo_local_max_batch.restype = ctypes.c_int64
        lib.lmo_local_max_ex.argtypes = [ctypes.c_int64, _P64, _P32, _PF, ctypes.c_uint64, ctypes.c_int, _P32,
                                         _P64, ctypes.c_int64]
        lib.lmo_local_max_ex.restype = ctypes.c_int64
        lib.lmo_local_max_batch_ex.argtypes = [ctypes.c_int64, _P64, _P64, _P32, _PF, _PU64, ctypes.c_uint64,
                                               ctypes.c_int, _P32, _P64]
        lib.lmo_local_max_batch_ex.restype = ctypes.c_int64
        lib.lmo_edge_hash_phase.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
        lib.lmo_edge_hash_phase.restype = ctypes.c_uint64
        lib.lmo_greedy_certificate.argtypes = [ctypes.c_int64, _P64, _P32, _PF, ctypes.c_uint64, _P32]
        lib.lmo_greedy_certificate.restype = ctypes.c_int64
        lib.lmo_contract.argtypes = [ctypes.c_int64, _P64, _P32, _PF, _P32, _P64, _P32, _P64, _P32, _PF, _P64, _P64]
        lib.lmo_contract.restype = ctypes.c_int64
        lib.lmo_hem.argtypes = [ctypes.c_int64, _P64, _P32, _PF, _P32, _P32]
        lib.lmo_hem.restype = ctypes.c_int64
        lib.lmo_gpa.argtypes = [ctypes.c_int64, _P64, _P32, _PF, _P32]
        lib.lmo_gpa.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def mix64(z: int) -> int:
    return int(_load().lmo_mix64(z & (2**64 - 1)))


def seed_mix(seed: int) -> int:
    return int(_load().lmo_seed_mix(seed & (2**64 - 1)))


def edge_hash(seed: int, lo: int, hi: int) -> int:
    return int(_load().lmo_edge_hash(seed & (2**64 - 1), lo, hi))


def edge_hash_phase(seed: int, t: int, lo: int, hi: int) -> int:
    """Renewed tie-break value of {lo, hi} in iteration t."""
    return int(_load().lmo_edge_hash_phase(seed & (2**64 - 1), t, lo, hi))


def local_max(n, row_ptr, col, w, seed: int = 1, log_cap: int = 1 << 16, renew: bool = False):
    """Returns (mate int32[n], log int64[phases, 3]) where log rows hold
    (|E_t|, V_t, edges matched in iteration t). renew=True draws the
    tie-break keys anew in every iteration (see lm_oracle.c)."""
    rp = _c(row_ptr, np.int64)
    cc = _c(col, np.int32)
    ww = _c(w, np.float32)
    mate = np.empty(max(n, 1), dtype=np.int32)[:n]
    log = np.zeros((log_cap, 3), dtype=np.int64)
    t = _load().lmo_local_max_ex(n, rp.ctypes.data_as(_P64), cc.ctypes.data_as(_P32), ww.ctypes.data_as(_PF),
                                 seed & (2**64 - 1), 1 if renew else 0, mate.ctypes.data_as(_P32),
                                 log.ctypes.data_as(_P64), log_cap)
    if t < 0:
        raise ValueError(f"oracle rejected the graph (code {t})")
    return mate, log[: min(int(t), log_cap)].copy()


def local_max_graph(g, seed: int = 1, renew: bool = False):
    return local_max(g.n, g.row_ptr, g.col, g.w, seed, renew=renew)


def local_max_batch(vtx_off, row_ptr, col, w, seeds=None, seed0: int = 1, renew: bool = False):
    """Solves every graph of a batch alone. Returns (mate local ids, phases[G])."""
    vo = _c(vtx_off, np.int64)
    rp = _c(row_ptr, np.int64)
    cc = _c(col, np.int32)
    ww = _c(w, np.float32)
    G = len(vo) - 1
    N = int(vo[-1])
    mate = np.empty(max(N, 1), dtype=np.int32)[:N]
    ph = np.zeros(max(G, 1), dtype=np.int64)[:G]
    sp = None
    if seeds is not None:
        sa = _c(np.asarray(seeds, dtype=np.uint64), np.uint64)
        sp = sa.ctypes.data_as(_PU64)
    t = _load().lmo_local_max_batch_ex(G, vo.ctypes.data_as(_P64), rp.ctypes.data_as(_P64),
                                       cc.ctypes.data_as(_P32), ww.ctypes.data_as(_PF), sp, seed0 & (2**64 - 1),
                                       1 if renew else 0, mate.ctypes.data_as(_P32), ph.ctypes.data_as(_P64))
    if t < 0:
        raise ValueError(f"oracle rejected the batch (code {t})")
    return mate, ph


def greedy_certificate(n, row_ptr, col, w, seed, mate) -> int:
    """Number of violations of the greedy characterisation (0 iff mate is
    exactly the greedy matching under the oracle's key)."""
    rp = _c(row_ptr, np.int64)
    cc = _c(col, np.int32)
    ww = _c(w, np.float32)
    mm = _c(mate, np.int32)
    r = _load().lmo_greedy_certificate(n, rp.ctypes.data_as(_P64), cc.ctypes.data_as(_P32),
                                       ww.ctypes.data_as(_PF), seed & (2**64 - 1), mm.ctypes.data_as(_P32))
    if r < 0:
        raise ValueError(f"certificate check rejected the input (code {r})")
    return int(r)


def contract(n, row_ptr, col, w, mate, vw=None):
    """Contraction by a pairing (see lm_oracle.c). w=None: every fine edge
    weighs 1; vw=None: every vertex weighs 1. Returns (cmap int32[n],
    coarse row_ptr int64[nc + 1], col int32[nnz_c], w float32[nnz_c],
    vertex weights int64[nc])."""
    rp = _c(row_ptr, np.int64)
    cc = _c(col, np.int32)
    nnz = int(rp[-1]) if n > 0 else 0
    ww = None if w is None else _c(w, np.float32)
    mm = _c(mate, np.int32)
    vv = None if vw is None else _c(vw, np.int64)
    cmap = np.empty(max(n, 1), dtype=np.int32)
    crp = np.zeros(n + 1, dtype=np.int64)
    ccol = np.empty(max(nnz, 1), dtype=np.int32)
    cw = np.empty(max(nnz, 1), dtype=np.float32)
    cvw = np.empty(max(n, 1), dtype=np.int64)
    nc = ctypes.c_int64(0)
    r = _load().lmo_contract(n, rp.ctypes.data_as(_P64), cc.ctypes.data_as(_P32),
                             ww.ctypes.data_as(_PF) if ww is not None else None, mm.ctypes.data_as(_P32),
                             vv.ctypes.data_as(_P64) if vv is not None else None, cmap.ctypes.data_as(_P32),
                             crp.ctypes.data_as(_P64), ccol.ctypes.data_as(_P32), cw.ctypes.data_as(_PF),
                             cvw.ctypes.data_as(_P64), ctypes.byref(nc))
    if r < 0:
        raise ValueError(f"oracle rejected the pairing (code {r})")
    k = int(nc.value)
    return cmap[:n].copy(), crp[: k + 1].copy(), ccol[:r].copy(), cw[:r].copy(), cvw[:k].copy()


def contract_graph(g, mate, vw=None, unweighted=False):
    return contract(g.n, g.row_ptr, g.col, None if unweighted else g.w, mate, vw)


def hem(g, order, unweighted=False):
    """Heavy edge matching visiting the vertices in `order` (Section 3's
    comparison baseline; reporting only). Returns mate."""
    rp = _c(g.row_ptr, np.int64)
    cc = _c(g.col, np.int32)
    ww = None if unweighted else _c(g.w, np.float32)
    od = _c(order, np.int32)
    mate = np.empty(max(g.n, 1), dtype=np.int32)
    r = _load().lmo_hem(g.n, rp.ctypes.data_as(_P64), cc.ctypes.data_as(_P32),
                        ww.ctypes.data_as(_PF) if ww is not None else None, od.ctypes.data_as(_P32),
                        mate.ctypes.data_as(_P32))
    if r < 0:
        raise ValueError(f"hem rejected the input (code {r})")
    return mate[:g.n].copy()


def gpa(g, unweighted=False):
    """Global path algorithm (Section 3's quality reference; reporting only).
    Returns mate."""
    rp = _c(g.row_ptr, np.int64)
    cc = _c(g.col, np.int32)
    ww = None if unweighted else _c(g.w, np.float32)
    mate = np.empty(max(g.n, 1), dtype=np.int32)
    r = _load().lmo_gpa(g.n, rp.ctypes.data_as(_P64), cc.ctypes.data_as(_P32),
                        ww.ctypes.data_as(_PF) if ww is not None else None, mate.ctypes.data_as(_P32))
    if r < 0:
        raise ValueError(f"gpa rejected the input (code {r})")
    return mate[:g.n].copy()
