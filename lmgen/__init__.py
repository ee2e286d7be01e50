"""Seeded synthetic inputs for local-max matching (generators only).

The workloads follow the input families of the paper's experiments
(Section 3): Erdos-Renyi random graphs with uniform weights, 2-D random
geometric graphs with weight 1 - distance, and R-MAT graphs with unit weights
(the unweighted case, Section 1). Batches of random graphs and a Poisson
request trace complete the set. Generation runs in C (``gen.c``) with a
counter-based SplitMix64 stream, so every graph is a pure function of its
parameters and seed.

Nothing here computes any part of the matching method; both the CPU oracle
and the GPU path consume these arrays.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "liblmgen.so")

W_UNIFORM = 0
W_UNIT = 1


class _Csr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("w", ctypes.POINTER(ctypes.c_float)),
    ]


class _Batch(ctypes.Structure):
    _fields_ = [
        ("graphs", ctypes.c_int64),
        ("n_total", ctypes.c_int64),
        ("nnz_total", ctypes.c_int64),
        ("vtx_off", ctypes.POINTER(ctypes.c_int64)),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("w", ctypes.POINTER(ctypes.c_float)),
    ]


def build(force: bool = False) -> str:
    """Compile gen.c into liblmgen.so next to it (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.lmg_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_Csr)]
        lib.lmg_rgg.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_Csr)]
        lib.lmg_rmat.argtypes = [
            ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(_Csr),
        ]
        lib.lmg_er_batch.argtypes = [
            ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Batch),
        ]
        lib.lmg_free.argtypes = [ctypes.POINTER(_Csr)]
        lib.lmg_batch_free.argtypes = [ctypes.POINTER(_Batch)]
        lib.lmg_stream_u01.argtypes = [
            ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
        ]
        for f in (lib.lmg_er, lib.lmg_rgg, lib.lmg_rmat, lib.lmg_er_batch):
            f.restype = ctypes.c_int
        lib.lmg_free.restype = None
        lib.lmg_batch_free.restype = None
        lib.lmg_stream_u01.restype = None
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR: row_ptr int64[n+1], col int32[nnz], w float32[nnz]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2


@dataclass
class Batch:
    """Disjoint union of graphs: vtx_off int64[G+1], row_ptr int64[N+1]
    (global offsets), col int32 (LOCAL ids), w float32."""

    vtx_off: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray

    @property
    def graphs(self) -> int:
        return len(self.vtx_off) - 1

    @property
    def n_total(self) -> int:
        return int(self.vtx_off[-1])

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def graph(self, g: int) -> Graph:
        a, b = int(self.vtx_off[g]), int(self.vtx_off[g + 1])
        e0, e1 = int(self.row_ptr[a]), int(self.row_ptr[b])
        return Graph(b - a, self.row_ptr[a : b + 1] - e0, self.col[e0:e1], self.w[e0:e1])


def _take_csr(c: _Csr) -> Graph:
    lib = _load()
    n, nnz = int(c.n), int(c.nnz)
    rp = np.ctypeslib.as_array(c.row_ptr, shape=(n + 1,)).copy()
    col = np.ctypeslib.as_array(c.col, shape=(max(nnz, 1),))[:nnz].copy()
    w = np.ctypeslib.as_array(c.w, shape=(max(nnz, 1),))[:nnz].copy()
    lib.lmg_free(ctypes.byref(c))
    return Graph(n, rp, col, w)


def er(n: int, m: int, seed: int = 1, weights: str = "uniform") -> Graph:
    """G(n, m): m distinct non-loop pairs, uniform by rejection; weights
    k*2^-24 with k uniform in [1, 2^24] ("uniform") or 1.0 ("unit")."""
    c = _Csr()
    mode = W_UNIT if weights == "unit" else W_UNIFORM
    if _load().lmg_er(n, m, seed & (2**64 - 1), mode, ctypes.byref(c)) != 0:
        raise ValueError(f"lmg_er failed for n={n} m={m}")
    return _take_csr(c)


def rgg_radius(n: int, avg_degree: float = 10.0) -> float:
    """Radius giving the requested expected degree, pi r^2 n = avg_degree."""
    return math.sqrt(avg_degree / (math.pi * n))


def rgg(n: int, avg_degree: float = 10.0, seed: int = 1, radius: float | None = None) -> Graph:
    """2-D random geometric graph; ids in grid-cell order; w = fp32(1 - d)."""
    r = rgg_radius(n, avg_degree) if radius is None else radius
    c = _Csr()
    if _load().lmg_rgg(n, r, seed & (2**64 - 1), ctypes.byref(c)) != 0:
        raise ValueError(f"lmg_rgg failed for n={n}")
    return _take_csr(c)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, weights: str = "unit") -> Graph:
    """R-MAT with edge_factor * 2^scale samples, deduplicated, symmetrised."""
    cs = _Csr()
    mode = W_UNIT if weights == "unit" else W_UNIFORM
    if _load().lmg_rmat(scale, edge_factor, a, b, c, seed & (2**64 - 1), mode, ctypes.byref(cs)) != 0:
        raise ValueError(f"lmg_rmat failed for scale={scale}")
    return _take_csr(cs)


def er_batch(graphs: int, seed: int = 1, lg_lo: float = 8.0, lg_hi: float = 16.0,
             d_lo: float = 4.0, d_hi: float = 32.0, weights: str = "uniform") -> Batch:
    """Batch of G(n, m) graphs with n log-uniform in [2^lg_lo, 2^lg_hi] and
    average degree uniform in [d_lo, d_hi]."""
    bb = _Batch()
    lib = _load()
    mode = W_UNIT if weights == "unit" else W_UNIFORM
    if lib.lmg_er_batch(graphs, seed & (2**64 - 1), lg_lo, lg_hi, d_lo, d_hi, mode, ctypes.byref(bb)) != 0:
        raise ValueError("lmg_er_batch failed")
    G, N, E = int(bb.graphs), int(bb.n_total), int(bb.nnz_total)
    vo = np.ctypeslib.as_array(bb.vtx_off, shape=(G + 1,)).copy()
    rp = np.ctypeslib.as_array(bb.row_ptr, shape=(N + 1,)).copy()
    col = np.ctypeslib.as_array(bb.col, shape=(max(E, 1),))[:E].copy()
    w = np.ctypeslib.as_array(bb.w, shape=(max(E, 1),))[:E].copy()
    lib.lmg_batch_free(ctypes.byref(bb))
    return Batch(vo, rp, col, w)


def stream_u01(seed: int, tag: int, count: int, first: int = 0) -> np.ndarray:
    """count uniforms in [0,1) from the generator's tagged sub-stream."""
    out = np.empty(count, dtype=np.float64)
    _load().lmg_stream_u01(seed & (2**64 - 1), tag, first, count,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def from_edges(n: int, edges, weights) -> Graph:
    """Symmetric CSR (rows sorted by neighbour) from undirected (u, v) pairs.
    Caller guarantees no self-loops or duplicates; used for hand-built cases."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    wt = np.asarray(weights, dtype=np.float32).reshape(-1)
    if len(e) != len(wt):
        raise ValueError("edges and weights differ in length")
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    ww = np.concatenate([wt, wt])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    counts = np.bincount(src, minlength=n) if len(src) else np.zeros(n, dtype=np.int64)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    return Graph(n, rp, dst.astype(np.int32), ww.astype(np.float32))


# ---------------------------------------------------------------- workloads

TAG_TRACE = 101


def serving_trace(requests: int, rate_per_s: float, seed: int = 1, lg_lo: float = 10.0,
                  lg_hi: float = 22.0):
    """Poisson request trace: list of (arrival_s, kind, n) with exponential
    inter-arrival times at rate_per_s, kind 'rgg' or 'rmat' with equal
    probability and n log-uniform in [2^lg_lo, 2^lg_hi]."""
    u = stream_u01(seed, TAG_TRACE, 3 * requests)
    t = 0.0
    out = []
    for i in range(requests):
        t += -math.log(1.0 - u[3 * i]) / rate_per_s
        kind = "rgg" if u[3 * i + 1] < 0.5 else "rmat"
        n = int(round(2.0 ** (lg_lo + (lg_hi - lg_lo) * u[3 * i + 2])))
        out.append((t, kind, n))
    return out


def serving_graph(kind: str, n: int, seed: int = 1) -> Graph:
    """The graph of one serving request: RGG with average degree 10, or R-MAT
    with edge factor 16 at scale round(log2 n) and uniform weights."""
    if kind == "rgg":
        return rgg(n, 10.0, seed)
    return rmat(max(1, int(round(math.log2(n)))), 16, seed=seed, weights="uniform")
