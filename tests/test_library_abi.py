"""The C-ABI library loads and exports every entry point include/zeuler.h declares.

CPU only: no call here reaches the GPU (ze_create with an invalid N fails before any HIP
call; ze_strerror is a table lookup).
"""

import ctypes
import os
import re

import pytest

import paper_2206_05466_amd as pkg
from paper_2206_05466_amd import zeuler

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zeuler.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ze_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ze_create", "ze_destroy", "ze_stream_solve", "ze_isomp_step",
                     "ze_casimirs", "ze_basis_assemble"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = pkg.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    assert sorted(zeuler.SIGNATURES) == declared_functions()


def test_strerror_and_invalid_create_without_gpu():
    lib = pkg.load_library()
    assert lib.ze_strerror(zeuler.ZE_ENOTCONV).decode().startswith("fixed-point")
    out = ctypes.c_void_p(123)
    assert lib.ze_create(0, None, ctypes.byref(out)) == zeuler.ZE_EINVAL
    assert out.value is None
    assert lib.ze_create(16385, None, ctypes.byref(out)) == zeuler.ZE_EINVAL
    assert lib.ze_create(16, None, None) == zeuler.ZE_EINVAL
    assert lib.ze_size(None) == 0
    assert lib.ze_destroy(None) == zeuler.ZE_OK
    assert lib.ze_stream_solve(None, None, None) == zeuler.ZE_EINVAL
    assert lib.ze_isomp_step(None, None, 0.1, 1e-12, 5, 0, None, None) == zeuler.ZE_EINVAL
    # setters with no context
    assert lib.ze_set_steady_cap(None, 2, 4) == zeuler.ZE_EINVAL
    assert lib.ze_set_initial_guess(None, 3) == zeuler.ZE_EINVAL
    assert lib.ze_set_stopping(None, 1) == zeuler.ZE_EINVAL
    assert lib.ze_set_continuation(None, 1) == zeuler.ZE_EINVAL
    assert lib.ze_ensemble_set_continuation(None, 1) == zeuler.ZE_EINVAL


def test_noalloc_product_refuses_sizes_without_gpu():
    """ze_zgemm_noalloc checks N (1..16384) and its pointers before any HIP call."""
    lib = pkg.load_library()
    p = ctypes.c_void_p(4096)
    for N in (0, -1, 16385):
        assert lib.ze_zgemm_noalloc(N, p, ctypes.c_void_p(8192), ctypes.c_void_p(12288), None) == zeuler.ZE_EINVAL
        assert b"outside 1..16384" in lib.ze_last_error()
    assert lib.ze_zgemm_noalloc(64, p, ctypes.c_void_p(8192), p, None) == zeuler.ZE_EINVAL
    assert lib.ze_zgemm_noalloc(64, None, p, ctypes.c_void_p(8192), None) == zeuler.ZE_EINVAL


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(zeuler, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(zeuler, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        zeuler.load_library()


def declared_prototypes():
    """{name: (return type, [parameter types])} from the comment-stripped header."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    protos = {}
    for ret, name, params in re.findall(r"([A-Za-z_][\w\s\*]*?)\b(ze_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
        types = []
        for p in params.split(","):
            p = " ".join(p.split())
            if not p or p == "void":
                continue
            # drop the parameter name: the last identifier, unless the declaration is only a type
            m = re.match(r"^(.*?[\s\*])([A-Za-z_]\w*)$", p)
            types.append((m.group(1) if m else p).replace(" ", "").strip())
        protos[name] = (" ".join(ret.split()), types)
    return protos


def ctypes_kind(t):
    if t in (ctypes.c_int,):
        return "int"
    if t is ctypes.c_double:
        return "double"
    if t is ctypes.c_char_p:
        return "string"
    if t is ctypes.c_void_p:
        return "pointer"
    if isinstance(t, type) and issubclass(t, ctypes._Pointer):
        inner = t._type_
        return {ctypes.c_int: "int*", ctypes.c_double: "double*", ctypes.c_longlong: "longlong*",
                ctypes.c_void_p: "pointer*"}[inner]
    raise AssertionError(f"unexpected ctypes type {t}")


def c_kind(t):
    t = t.replace("const", "")
    if t in ("int", "ze_status"):
        return "int"
    if t == "double":
        return "double"
    if t == "char*":
        return "string"
    if t == "int*":
        return "int*"
    if t == "double*":
        return "double*"
    if t == "longlong*":
        return "longlong*"
    if t in ("ze_ctx**", "ze_ens**", "void**"):
        return "pointer*"
    if t in ("void*", "ze_ctx*", "ze_ens*"):
        return "pointer"
    raise AssertionError(f"unexpected C type {t!r}")


def test_binding_signatures_match_the_header():
    """Every ctypes argtypes/restype of the binding has the arity and kind of the header's
    prototype (an int passed where a double is declared would be marshalled wrongly)."""
    protos = declared_prototypes()
    assert sorted(protos) == declared_functions()
    for name, (res, args) in zeuler.SIGNATURES.items():
        ret, params = protos[name]
        ckinds = [c_kind(p) for p in params]
        pykinds = [ctypes_kind(a) for a in args]
        assert ckinds == pykinds, (name, params, pykinds)
        want_ret = "string" if "char" in ret else ("int" if ret in ("ze_status", "int") else ret)
        assert ctypes_kind(res) == want_ret, (name, ret, res)
