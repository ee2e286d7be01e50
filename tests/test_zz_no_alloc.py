"""lm_match_noalloc (the allocation-free single-graph solve) against lm_match,
through the C ABI: identical mate[], phase count and phase log on two calls
in a row, the second on a smaller graph (the shared scratch array keeps the
first call's contents), for a weighted and an unweighted graph; sizes past the
scratch array and host buffers are refused before any device work."""
import ctypes

import numpy as np
import pytest

import lmgen

pytestmark = pytest.mark.gpu


def _dev(g, torch, weighted=True):
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev) if weighted else None
    return rp, col, w


def _same(ctx, g, torch, seed, weighted=True):
    rp, col, w = _dev(g, torch, weighted)
    ref, st_ref = ctx.match(rp, col, w, seed=seed)
    torch.cuda.synchronize()
    # the noalloc call writes into a buffer holding stale values
    out = torch.full((g.n,), 12345, dtype=torch.int32, device=rp.device)
    got, st = ctx.match_noalloc(rp, col, w, seed=seed, mate=out)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
    assert st.phases == st_ref.phases and st.matched_edges == st_ref.matched_edges
    assert np.array_equal(st.log, st_ref.log)
    return st


def test_noalloc_equals_match_twice_smaller_second():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4587_amd as lm

    with lm.Context(0) as ctx:
        big = lmgen.er(4096, 32768, seed=1)  # ER 4096 / 32768, uniform weights
        small = lmgen.er(700, 2100, seed=5)
        for weighted in (True, False):
            s1 = _same(ctx, big, torch, seed=1, weighted=weighted)
            s2 = _same(ctx, small, torch, seed=3, weighted=weighted)
            assert s1.phases >= 1 and s2.phases >= 1
        # a larger graph that still fits: RGG with 2^17 vertices
        rg = lmgen.rgg(1 << 17, 10.0, seed=2)
        _same(ctx, rg, torch, seed=1)
        _same(ctx, small, torch, seed=1)


def test_noalloc_limits_and_flags():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_4587_amd as lm
    from paper_1302_4587_amd import _lib as L

    lib = L.load()
    with lm.Context(0) as ctx:
        g = lmgen.er(500, 1500, seed=2)
        rp, col, w = _dev(g, torch)
        mate = torch.empty(g.n, dtype=torch.int32, device=rp.device)
        csr = L.Csr(g.n, g.nnz, rp.data_ptr(), col.data_ptr(), w.data_ptr())
        dev = L.LM_IN_DEVICE | L.LM_OUT_DEVICE
        # host buffers (no device flags) and flags that need allocation are refused
        for flags in (0, L.LM_IN_DEVICE, L.LM_OUT_DEVICE, dev | L.LM_PROFILE, dev | L.LM_GRAPH,
                      dev | L.LM_WEIGHT_SUM):
            assert lib.lm_match_noalloc(ctx.handle, ctypes.byref(csr), 1, mate.data_ptr(), flags, None,
                                        None) == L.LM_EINVAL
        # a graph whose working set exceeds the scratch array: refused before any device work
        # (the sizes alone decide; the pointers are never read)
        huge = L.Csr(1 << 20, 1 << 23, rp.data_ptr(), col.data_ptr(), w.data_ptr())
        assert lib.lm_match_noalloc(ctx.handle, ctypes.byref(huge), 1, mate.data_ptr(), dev, None,
                                    None) == L.LM_ETOOBIG
        # the checked path works without allocating too
        assert lib.lm_match_noalloc(ctx.handle, ctypes.byref(csr), 1, mate.data_ptr(), dev | L.LM_CHECK_GRAPH,
                                    None, None) == L.LM_OK
        torch.cuda.synchronize()
        ref, _ = ctx.match(rp, col, w, seed=1)
        assert np.array_equal(mate.cpu().numpy(), ref.cpu().numpy())
        # an empty graph
        e = L.Csr(0, 0, rp.data_ptr(), None, None)
        assert lib.lm_match_noalloc(ctx.handle, ctypes.byref(e), 1, mate.data_ptr(), dev, None, None) == L.LM_OK
