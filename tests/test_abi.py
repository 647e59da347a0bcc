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


def _declarations():
    """(return type, name, [argument declarations]) of every function in the header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = []
    for ret, name, args in re.findall(r"^(tt_status|int32_t|int64_t|size_t|double|void|const char\*)\s+(tt_\w+)\(([^;]*)\);",
                                      text, flags=re.M):
        out.append((ret, name, [a.strip() for a in " ".join(args.split()).split(",") if a.strip()]))
    return out


def _typed_zero_call(lib, ret, name, args, first=None):
    f = getattr(lib, name)
    types, vals = [], []
    for a in args:
        if "*" in a:
            types.append(ctypes.c_void_p)
            vals.append(None)
        elif a.startswith("double"):
            types.append(ctypes.c_double)
            vals.append(0.0)
        elif a.startswith(("int64_t", "size_t")):
            types.append(ctypes.c_int64)
            vals.append(0)
        else:
            types.append(ctypes.c_int32)
            vals.append(0)
    f.argtypes = types
    f.restype = None if ret == "void" else {"int64_t": ctypes.c_int64, "size_t": ctypes.c_int64,
                                            "double": ctypes.c_double,
                                            "const char*": ctypes.c_char_p}.get(ret, ctypes.c_int)
    return f(*vals)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_context_and_null_arguments_are_rejected_before_any_device_work():
    """Every call that takes a context or an engine returns TT_EINVAL (-1) for a null one, and the
    host-only queries reject null inputs, without touching the device (this host has none: a call
    that reached the HIP runtime would fail differently or crash)."""
    lib = ctypes.CDLL(LIB)   # a fresh handle: argument types are set here only
    decl = _declarations()
    assert len(decl) >= 30
    seen = 0
    for ret, name, args in decl:
        if not args or name.endswith("_create"):
            continue
        takes_handle = args[0].startswith(("tt_ctx*", "const tt_ctx*", "tt_engine*", "const tt_engine*"))
        host_query = name in ("tt_round_out_capacity", "tt_round_workspace_bytes", "tt_round_effective_delta",
                              "tt_request_out_capacity", "tt_request_scratch_bytes", "tt_orthogonalize_capacity",
                              "tt_dot_noalloc")
        if not (takes_handle or host_query):
            continue
        r = _typed_zero_call(lib, ret, name, args)
        seen += 1
        if ret == "void":
            continue                                   # destroy(NULL) is a no-op
        if ret == "const char*":
            assert isinstance(r, bytes), name          # a message, never a null pointer
            continue
        if name in ("tt_ctx_required_bytes", "tt_engine_pending"):
            assert r == 0, name
        else:
            assert r == -1, (name, r)
    assert seen >= 30
