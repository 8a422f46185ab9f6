"""The C ABI: libtfi.so loads on a CPU host and exports every function that
include/tfi.h declares; the binding's option struct matches the header's
field order. No compute calls (no GPU here)."""
import ctypes as C
import os
import re

from paper_2609_34025_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header():
    return open(os.path.join(ROOT, "include", "tfi.h")).read()


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", header(), flags=re.S)
    return sorted(set(re.findall(r"\b(tfi_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(_lib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(_lib.EXPORTED)


def test_build_opts_layout_matches_header():
    text = header()
    body = text[text.index("typedef struct {"):text.index("} tfi_build_opts;")]
    fields = re.findall(r"^\s*(?:int32_t|uint64_t|float)\s+(\w+)", body, flags=re.M)
    assert [f for f in fields] == [f[0] for f in _lib.BuildOpts._fields_]
    assert C.sizeof(_lib.BuildOpts) == 56


def test_fft_params_layout_matches_header():
    text = header()
    body = text[text.index("typedef struct tfi_fft_params {"):text.index("} tfi_fft_params;")]
    fields = re.findall(r"^\s*int32_t\s+(\w+)", body, flags=re.M)
    assert fields == [f[0] for f in _lib.FftParams._fields_]
    assert C.sizeof(_lib.FftParams) == 28
    assert _lib.load().tfi_get_fft_params(None, None) == -1


def test_last_error_and_null_handle_paths():
    lib = _lib.load()
    assert lib.tfi_kernel_length(None) == -1
    assert lib.tfi_num_vertices(None) == -1
    rc = lib.tfi_integrate(None, None, None, 1, 0, None, None)
    assert rc == -1 and b"null handle" in lib.tfi_last_error()
    assert lib.tfi_plan_stats(None, None, 0) == -1
    lib.tfi_destroy(None)
