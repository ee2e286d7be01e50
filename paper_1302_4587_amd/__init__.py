"""Local-max matching on AMD MI355X (gfx950): Python binding of include/lm.h.

The matching itself (paper: Birn, Osipov, Sanders, Schulz, Sitchinava,
"Efficient Parallel and External Matching", Section 1 "local max" and
Section 2) runs entirely in the HIP library ``liblm.so``; this module only
marshals arguments. Inputs may be torch tensors on the GPU (device pointers,
torch's current stream) or host numpy arrays (the library stages them).

    ctx = Context()
    mate, st = ctx.match(row_ptr, col, w, seed=1)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _lib
from ._lib import (KERNEL_KINDS, LM_ASYNC, LM_CHECK_GRAPH, LM_GRAPH, LM_IN_DEVICE, LM_OUT_DEVICE, LM_PROFILE,
                   LM_RENEW_KEYS, LM_SERVE_BATCHED, LM_SERVE_FIFO, LM_WEIGHT_SUM, LMError, check)

__all__ = ["Context", "Server", "MatchStats", "ContractStats", "LMError", "library_path", "LM_SERVE_BATCHED", "LM_SERVE_FIFO"]


def library_path() -> str:
    return _lib.LIB_PATH


def _is_torch(x) -> bool:
    return hasattr(x, "data_ptr") and hasattr(x, "is_cuda")


_TORCH_DTYPES = {}


def _torch_dtype(dtype):
    if not _TORCH_DTYPES:
        import torch
        _TORCH_DTYPES.update({np.int64: torch.int64, np.int32: torch.int32, np.float32: torch.float32})
    return _TORCH_DTYPES[dtype]


def _ptr(x, dtype, on_device=False):
    """(pointer, on_device, keepalive) for a torch tensor or numpy array; None
    (an absent weight array: unweighted graph) takes the residence given."""
    if x is None:
        return None, on_device, None
    if _is_torch(x):
        want = _torch_dtype(dtype)
        if x.dtype != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr(), bool(x.is_cuda), x
    a = np.asarray(x)
    if a.dtype != dtype:
        a = a.astype(dtype)
    a = np.ascontiguousarray(a)
    return a.ctypes.data, False, a


@dataclass
class MatchStats:
    phases: int
    matched_edges: int
    device_ms: float
    bytes_alg: float
    log: np.ndarray  # (phases, 4): live_entries, live_rows, matched_edges, matched_entries
    kernel_launches: dict = field(default_factory=dict)
    kernel_ms: dict = field(default_factory=dict)
    kernel_bytes: dict = field(default_factory=dict)
    matched_weight: float | None = None  # w(M), when asked for (weight_sum=True)


@dataclass
class ContractStats:
    device_ms: float
    bytes_alg: float
    long_rows: int      # coarse rows with deg(a) + deg(b) > 512 (bucketed, merged in LDS)
    long_entries: int   # their fine entries
    table_rows: int = 0  # long rows merged through device-memory hash tables instead


def _stats_out(st: _lib.Stats, logbuf, weight_sum=False) -> MatchStats:
    n = int(st.log_len)
    # lm_phase_rec is four int64: copy the first n records out of the reused buffer
    log = np.frombuffer(logbuf, dtype=np.int64, count=4 * n).reshape(n, 4).copy()
    return MatchStats(int(st.phases), int(st.matched_edges), float(st.device_ms), float(st.bytes_alg), log,
                      {k: int(st.k_launches[i]) for i, k in enumerate(KERNEL_KINDS)},
                      {k: float(st.k_ms[i]) for i, k in enumerate(KERNEL_KINDS)},
                      {k: float(st.k_bytes[i]) for i, k in enumerate(KERNEL_KINDS)},
                      float(st.matched_weight) if weight_sum else None)


class Context:
    """A device context (lm_ctx): device memory pool, stream, tuning."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self._lib = _lib.load()
        h = ctypes.c_void_p()
        check(self._lib.lm_create(device, hbm_budget_bytes, ctypes.byref(h)), "lm_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.lm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def _logbuf(self, log_cap: int):
        """Phase-log buffer of log_cap records, kept across solves (the stats
        copy what they return)."""
        cap = max(int(log_cap), 1)
        buf = getattr(self, "_logbufs", {}).get(cap)
        if buf is None:
            buf = (_lib.PhaseRec * cap)()
            self._logbufs = {cap: buf}
        return buf

    # -------------------------------------------------------------- tuning
    def tuning(self) -> dict:
        t = _lib.Tuning()
        check(self._lib.lm_get_tuning(self._h, ctypes.byref(t)), "lm_get_tuning")
        return {"block_entries": t.block_entries, "grid_per_cu": t.grid_per_cu,
                "phases_per_sync": t.phases_per_sync, "tail_entries": t.tail_entries}

    def set_tuning(self, block_entries=None, grid_per_cu=None, phases_per_sync=None, tail_entries=None):
        cur = self.tuning()
        t = _lib.Tuning(block_entries or cur["block_entries"], grid_per_cu or cur["grid_per_cu"],
                        phases_per_sync or cur["phases_per_sync"],
                        cur["tail_entries"] if tail_entries is None else tail_entries)
        check(self._lib.lm_set_tuning(self._h, ctypes.byref(t)), "lm_set_tuning")

    # -------------------------------------------------------------- solves
    def _flags_stream(self, dev_in, dev_out, check_graph, profile, stream, hip_graph=False, weight_sum=False,
                      asynchronous=False, renew_keys=False):
        flags = (LM_IN_DEVICE if dev_in else 0) | (LM_OUT_DEVICE if dev_out else 0)
        flags |= (LM_CHECK_GRAPH if check_graph else 0) | (LM_PROFILE if profile else 0)
        flags |= (LM_GRAPH if hip_graph else 0) | (LM_WEIGHT_SUM if weight_sum else 0)
        flags |= (LM_ASYNC if asynchronous else 0) | (LM_RENEW_KEYS if renew_keys else 0)
        s = None
        if stream is not None:
            s = stream if isinstance(stream, int) else getattr(stream, "cuda_stream", None)
        elif dev_in or dev_out:
            import torch
            s = torch.cuda.current_stream().cuda_stream
        return flags, s

    def match(self, row_ptr, col, w, seed: int = 1, mate=None, *, check_graph=False, profile=False, stream=None,
              log_cap: int = 4096, hip_graph=False, profile_kinds=None, weight_sum=False, asynchronous=False,
              renew_keys=False):
        """Solves one graph. Returns (mate, MatchStats). hip_graph=True runs the
        whole solve as one captured HIP graph (LM_GRAPH); weight_sum=True also
        returns w(M) in MatchStats.matched_weight (LM_WEIGHT_SUM);
        asynchronous=True (LM_ASYNC, device tensors only) enqueues the solve on
        the stream and returns (mate, None) at once; renew_keys=True breaks ties
        with keys drawn anew in every phase (LM_RENEW_KEYS)."""
        n = int(row_ptr.shape[0]) - 1
        nnz = int(col.shape[0])
        rp, d0, k0 = _ptr(row_ptr, np.int64)
        cp, d1, k1 = _ptr(col, np.int32)
        wp, d2, k2 = _ptr(w, np.float32, d0)  # w=None: unweighted (every edge weighs 1)
        if not (d0 == d1 == d2):
            raise ValueError("row_ptr, col, w must all be on the device or all on the host")
        if mate is None:
            if d0:
                import torch
                mate = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
            else:
                mate = np.empty(max(n, 0), dtype=np.int32)
        mp, dm, km = _ptr(mate, np.int32)
        flags, s = self._flags_stream(d0, dm, check_graph, profile, stream, hip_graph, weight_sum, asynchronous,
                                      renew_keys)
        g = _lib.Csr(n, nnz, rp, cp, wp)
        if asynchronous:
            check(self._lib.lm_match(self._h, ctypes.byref(g), seed & (2**64 - 1), mp, flags, s, None), "lm_match")
            return mate, None
        logbuf = self._logbuf(log_cap)
        st = _lib.Stats()
        st.log = logbuf
        st.log_cap = log_cap
        if profile_kinds:  # names from KERNEL_KINDS: time only these kinds
            st.profile_kinds = sum(1 << KERNEL_KINDS.index(k) for k in set(profile_kinds))
        check(self._lib.lm_match(self._h, ctypes.byref(g), seed & (2**64 - 1), mp, flags, s, ctypes.byref(st)),
              "lm_match")
        return mate, _stats_out(st, logbuf, weight_sum)

    def contract(self, row_ptr, col, w, mate, vwgt=None, *, want_vwgt=True, stream=None):
        """lm_contract: contracts the graph by the pairing mate (coarsening).
        Device tensors in give device tensors out; numpy arrays in give numpy
        arrays out. w=None: every fine edge weighs 1; vwgt=None: every vertex
        weighs 1. Returns (cmap, coarse row_ptr, col, w, vertex weights or
        None, ContractStats), the coarse arrays trimmed to their sizes."""
        n = int(row_ptr.shape[0]) - 1
        nnz = int(col.shape[0])
        rp, d0, k0 = _ptr(row_ptr, np.int64)
        cp, d1, k1 = _ptr(col, np.int32)
        wp, d2, k2 = _ptr(w, np.float32, d0)
        mp, d3, k3 = _ptr(mate, np.int32)
        vp_, d4, k4 = _ptr(vwgt, np.int64, d0)
        if not (d0 == d1 == d2 == d3 == d4):
            raise ValueError("all inputs must be on the device or all on the host")
        if d0:
            import torch
            dev = row_ptr.device
            mk = lambda k, dt: torch.empty(max(k, 1), dtype=dt, device=dev)
            cmap, crp, ccol, cw = (mk(n, torch.int32), mk(n + 1, torch.int64), mk(nnz, torch.int32),
                                   mk(nnz, torch.float32))
            cvw = mk(n, torch.int64) if want_vwgt else None
        else:
            cmap, crp = np.empty(max(n, 1), np.int32), np.empty(n + 1, np.int64)
            ccol, cw = np.empty(max(nnz, 1), np.int32), np.empty(max(nnz, 1), np.float32)
            cvw = np.empty(max(n, 1), np.int64) if want_vwgt else None
        ptr = (lambda x: x.data_ptr()) if d0 else (lambda x: x.ctypes.data)
        out = _lib.Coarse(0, 0, ptr(crp), ptr(ccol), ptr(cw), ptr(cvw) if cvw is not None else None)
        flags, s = self._flags_stream(d0, d0, False, False, stream)
        g = _lib.Csr(n, nnz, rp, cp, wp)
        st = _lib.ContractStats()
        check(self._lib.lm_contract(self._h, ctypes.byref(g), mp, vp_, ptr(cmap), ctypes.byref(out), flags, s,
                                    ctypes.byref(st)), "lm_contract")
        nc, mc = int(out.n), int(out.nnz)
        return (cmap[:n], crp[:nc + 1], ccol[:mc], cw[:mc], cvw[:nc] if cvw is not None else None,
                ContractStats(float(st.device_ms), float(st.bytes_alg), int(st.long_rows), int(st.long_entries),
                              int(st.table_rows)))

    def match_noalloc(self, row_ptr, col, w, seed: int = 1, mate=None, *, check_graph=False, stream=None,
                      log_cap: int = 4096):
        """lm_match_noalloc: the allocation-free solve of one graph whose tensors
        are on the device (working buffers from the library's fixed per-GPU
        scratch array). Returns (mate, MatchStats)."""
        n = int(row_ptr.shape[0]) - 1
        nnz = int(col.shape[0])
        rp, d0, k0 = _ptr(row_ptr, np.int64)
        cp, d1, k1 = _ptr(col, np.int32)
        wp, d2, k2 = _ptr(w, np.float32, d0)
        if not (d0 and d1 and d2):
            raise ValueError("match_noalloc takes device tensors only")
        if mate is None:
            import torch
            mate = torch.empty(max(n, 0), dtype=torch.int32, device=row_ptr.device)
        mp, dm, km = _ptr(mate, np.int32)
        if not dm:
            raise ValueError("match_noalloc writes a device tensor")
        flags, s = self._flags_stream(True, True, check_graph, False, stream)
        g = _lib.Csr(n, nnz, rp, cp, wp)
        logbuf = self._logbuf(log_cap)
        st = _lib.Stats()
        st.log = logbuf
        st.log_cap = log_cap
        check(self._lib.lm_match_noalloc(self._h, ctypes.byref(g), seed & (2**64 - 1), mp, flags, s,
                                         ctypes.byref(st)), "lm_match_noalloc")
        return mate, _stats_out(st, logbuf)

    def match_batch(self, vtx_off, row_ptr, col, w, seeds=None, seed0: int = 1, mate=None, *, check_graph=False,
                    profile=False, stream=None, log_cap: int = 4096, want_graph_phases=True, hip_graph=True,
                    weight_sum=False, asynchronous=False, renew_keys=False):
        """Solves a batch (disjoint union, local ids) in one captured HIP graph
        launch unless hip_graph=False or profile=True. Returns (mate, MatchStats,
        graph_phases); with asynchronous=True (LM_ASYNC) (mate, None, None) at
        once."""
        vo = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
        G = len(vo) - 1
        N = int(vo[-1])
        nnz = int(col.shape[0])
        rp, d0, k0 = _ptr(row_ptr, np.int64)
        cp, d1, k1 = _ptr(col, np.int32)
        wp, d2, k2 = _ptr(w, np.float32, d0)  # w=None: unweighted (every edge weighs 1)
        if not (d0 == d1 == d2):
            raise ValueError("row_ptr, col, w must all be on the device or all on the host")
        if mate is None:
            if d0:
                import torch
                mate = torch.empty(N, dtype=torch.int32, device=row_ptr.device)
            else:
                mate = np.empty(N, dtype=np.int32)
        mp, dm, km = _ptr(mate, np.int32)
        sp = None
        sk = None
        if seeds is not None:
            sk = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
            sp = sk.ctypes.data
        flags, s = self._flags_stream(d0, dm, check_graph, profile, stream, hip_graph, weight_sum, asynchronous,
                                      renew_keys)
        if asynchronous:
            check(self._lib.lm_match_batch(self._h, G, vo.ctypes.data, nnz, rp, cp, wp, sp, seed0 & (2**64 - 1), mp,
                                           flags, s, None, None), "lm_match_batch")
            return mate, None, None
        gph = np.zeros(G, dtype=np.int32) if want_graph_phases else None
        logbuf = self._logbuf(log_cap)
        st = _lib.Stats()
        st.log = logbuf
        st.log_cap = log_cap
        check(self._lib.lm_match_batch(self._h, G, vo.ctypes.data, nnz, rp, cp, wp, sp, seed0 & (2**64 - 1), mp,
                                       flags, s, ctypes.byref(st),
                                       gph.ctypes.data if gph is not None else None), "lm_match_batch")
        return mate, _stats_out(st, logbuf, weight_sum), gph

    def autotune_batch(self, vtx_off, row_ptr, col, w, cache_path=None, hip_graph=True) -> dict:
        """lm_autotune_batch: keeps the fastest tuning for this batch in the
        context (timed as captured launches unless hip_graph=False)."""
        vo = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
        rp, d0, k0 = _ptr(row_ptr, np.int64)
        cp, d1, k1 = _ptr(col, np.int32)
        wp, d2, k2 = _ptr(w, np.float32, d0)
        t = _lib.Tuning()
        flags = (LM_IN_DEVICE if d0 else 0) | (LM_GRAPH if hip_graph else 0)
        check(self._lib.lm_autotune_batch(self._h, len(vo) - 1, vo.ctypes.data, int(col.shape[0]), rp, cp, wp, flags,
                                          cache_path.encode() if cache_path else None, ctypes.byref(t)),
              "lm_autotune_batch")
        return {"block_entries": t.block_entries, "grid_per_cu": t.grid_per_cu,
                "phases_per_sync": t.phases_per_sync, "tail_entries": t.tail_entries}


class Server:
    """Request server (lm_server_*): submit host graphs, poll/wait results."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 64 << 30, max_resident: int = 256,
                 queue_cap: int = 1 << 16, phases_per_step: int = 2, mode: int = LM_SERVE_BATCHED):
        self._lib = _lib.load()
        self._ctx = ctx
        o = _lib.ServerOpts(hbm_budget_bytes, max_resident, queue_cap, phases_per_step, mode)
        h = ctypes.c_void_p()
        check(self._lib.lm_server_create(ctx.handle, ctypes.byref(o), ctypes.byref(h)), "lm_server_create")
        self._h = h
        self._n = {}

    def submit(self, row_ptr, col, w, seed: int = 1) -> int:
        rp, _, k0 = _ptr(row_ptr, np.int64)
        cp, _, k1 = _ptr(col, np.int32)
        wp, _, k2 = _ptr(w, np.float32)
        n = len(row_ptr) - 1
        g = _lib.Csr(n, len(col), rp, cp, wp)
        t = ctypes.c_uint64()
        check(self._lib.lm_server_submit(self._h, ctypes.byref(g), seed & (2**64 - 1), ctypes.byref(t)),
              "lm_server_submit")
        self._n[t.value] = n
        return t.value

    def _result(self, fn, ticket, *extra):
        n = self._n.get(ticket, 0)
        mate = np.empty(max(n, 1), dtype=np.int32)
        st = _lib.RequestStats()
        r = fn(self._h, ticket, mate.ctypes.data, ctypes.byref(st), *extra)
        if r == _lib.LM_PENDING:
            return None
        check(r, "lm_server result")
        self._n.pop(ticket, None)
        return mate[:n], {"phases": st.phases, "matched_edges": st.matched_edges,
                          "queue_ms": st.submit_to_admit_ms, "latency_ms": st.submit_to_done_ms,
                          "device_ms": st.admit_to_solved_ms, "copy_back_ms": st.solved_to_done_ms}

    def poll(self, ticket: int):
        return self._result(self._lib.lm_server_poll, ticket)

    def wait(self, ticket: int, timeout_ms: int = -1):
        return self._result(self._lib.lm_server_wait, ticket, timeout_ms)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            check(self._lib.lm_server_destroy(self._h), "lm_server_destroy")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
