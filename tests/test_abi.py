"""The C-ABI library loads and exports every function declared in include/ttortho.h.

No compute call is made here (no GPU on this host); the GPU parity tests call
the same symbols through the binding.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttortho.h")
LIB = os.path.join(ROOT, "paper_2211_08770_amd", "libttortho.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(tt_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tt_round", "tt_round_batched", "tt_norm", "tt_engine_step", "tt_axpy", "tt_dot", "tt_dot_batched",
                     "tt_orthogonalize", "tt_loo", "tt_ctx_create", "tt_ctx_destroy", "tt_laplacian",
                     "tt_krylov_laplacian", "tt_round_randomized"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_host_only_queries():
    lib = ctypes.CDLL(LIB)
    lib.tt_status_str.restype = ctypes.c_char_p
    assert lib.tt_status_str(0) == b"ok"
    assert b"positive definite" in lib.tt_status_str(-4)
    lib.tt_round_out_capacity.restype = ctypes.c_int64
    assert lib.tt_round_out_capacity(None) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2211_08770_amd import tt
    monkeypatch.setattr(tt, "_HERE", str(tmp_path))
    monkeypatch.setattr(tt, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        tt._load()


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
