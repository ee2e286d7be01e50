"""CPU-side checks of the C-ABI library: it loads, exports every entry point
declared in include/lm.h, and its host-side logic behaves. No kernel runs."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = _declared()
    for must in ("lm_create", "lm_destroy", "lm_match", "lm_match_batch", "lm_server_create", "lm_server_submit",
                 "lm_server_poll", "lm_server_wait", "lm_server_destroy", "lm_strerror", "lm_autotune_batch"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1302_4587_amd._lib as L
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), f"{name} declared in lm.h but not exported"
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (lm_[a-z_]+)\b", out))
    assert set(_declared()) <= exported
    assert set(L.EXPORTED) <= exported


def test_strerror_messages():
    import paper_1302_4587_amd._lib as L
    lib = L.load()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8):
        s = lib.lm_strerror(code).decode()
        assert s and s != "unknown status"
    assert lib.lm_strerror(-99).decode() == "unknown status"


def test_header_compiles_as_c():
    src = '#include "lm.h"\nint main(void){ lm_csr g; (void)g; return lm_strerror(0) != 0 ? 0 : 1; }\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", f"-I{ROOT}/include", "-x", "c", "-"],
                       input=src, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_struct_layouts_match_header():
    """ctypes mirrors agree with the C compiler's layout of lm.h."""
    import paper_1302_4587_amd._lib as L
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "lm.h"\nint main(void){'
           'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(lm_csr), sizeof(lm_stats), sizeof(lm_phase_rec),'
           'sizeof(lm_tuning), sizeof(lm_server_opts), sizeof(lm_request_stats), offsetof(lm_stats, k_bytes),'
           'offsetof(lm_stats, log_cap), offsetof(lm_stats, matched_weight));'
           'printf("%zu %zu %zu\\n", sizeof(lm_coarse), sizeof(lm_contract_stats), offsetof(lm_coarse, vwgt));'
           'return 0; }\n')
    exe = os.path.join(ROOT, "_build", "layout_probe")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    r = subprocess.run(["gcc", "-std=c99", f"-I{ROOT}/include", "-x", "c", "-", "-o", exe], input=src,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    vals = [int(x) for x in subprocess.run([exe], capture_output=True, text=True).stdout.split()]
    mine = [ctypes.sizeof(L.Csr), ctypes.sizeof(L.Stats), ctypes.sizeof(L.PhaseRec), ctypes.sizeof(L.Tuning),
            ctypes.sizeof(L.ServerOpts), ctypes.sizeof(L.RequestStats), L.Stats.k_bytes.offset, L.Stats.log_cap.offset,
            L.Stats.matched_weight.offset, ctypes.sizeof(L.Coarse), ctypes.sizeof(L.ContractStats),
            L.Coarse.vwgt.offset]
    assert vals == mine


def test_create_without_gpu_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; this checks the no-device path")
    import paper_1302_4587_amd._lib as L
    lib = L.load()
    h = ctypes.c_void_p()
    assert lib.lm_create(0, 0, ctypes.byref(h)) == L.LM_EDEVICE
    assert not h.value


def test_null_arguments_rejected_without_device():
    import paper_1302_4587_amd._lib as L
    lib = L.load()
    assert lib.lm_create(0, 0, None) == L.LM_EINVAL
    assert lib.lm_match(None, None, 1, None, 0, None, None) == L.LM_EINVAL
    assert lib.lm_match_batch(None, 1, None, 0, None, None, None, None, 1, None, 0, None, None, None) == L.LM_EINVAL
    assert lib.lm_server_create(None, None, None) == L.LM_EINVAL
    assert lib.lm_server_submit(None, None, 1, None) == L.LM_EINVAL
    assert lib.lm_server_poll(None, 1, None, None) == L.LM_EINVAL
    assert lib.lm_server_destroy(None) == L.LM_EINVAL
    assert lib.lm_set_tuning(None, None) == L.LM_EINVAL
    assert lib.lm_contract(None, None, None, None, None, None, 0, None, None) == L.LM_EINVAL


def test_package_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1302_4587_amd._lib as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        L.load()


def test_constants_match_header():
    """Flags, status codes, kernel kinds and server modes of the binding are
    the values include/lm.h defines."""
    import paper_1302_4587_amd._lib as L
    text = open(HEADER).read()
    defs = {}
    for name, val in re.findall(r"#define\s+(LM_[A-Z0-9_]+)\s+\(?(-?(?:0x)?[0-9a-fA-F]+)u?\)?", text):
        defs[name] = int(val, 0)
    names = [n for n in dir(L) if n.startswith("LM_") and isinstance(getattr(L, n), int)]
    assert {"LM_WEIGHT_SUM", "LM_GRAPH", "LM_IN_DEVICE", "LM_EDEVICE", "LM_SERVE_FIFO"} <= set(names)
    for n in names:
        assert n in defs, f"{n} is not defined in lm.h"
        assert getattr(L, n) == defs[n], f"{n}: binding {getattr(L, n)} vs header {defs[n]}"
    assert len(L.KERNEL_KINDS) == defs["LM_K_KINDS"]


def test_bench_refuses_more_than_one_gpu():
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
