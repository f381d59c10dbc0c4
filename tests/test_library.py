"""CPU checks of the C-ABI library: it loads and exports every declared symbol,
and host-side argument validation rejects bad calls (no device work)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "velo.h")
LIB = os.path.join(ROOT, "paper_2412_05041_amd",
                   "libvelo_san.so" if os.environ.get("VELO_SANITIZE") == "1" else "libvelo.so")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(velo_[a-z0-9_]+)\s*\(", src)) - {"VELO_STATUS_WORDS"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2412_05041_amd import build
        build.build(sanitize=os.environ.get("VELO_SANITIZE") == "1")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings_and_errors(lib):
    lib.velo_status_string.restype = C.c_char_p
    lib.velo_last_error.restype = C.c_char_p
    assert lib.velo_status_string(0) == b"ok"
    assert lib.velo_status_string(-2).startswith(b"workspace")
    # null arguments are rejected before any device call
    assert lib.velo_create(None, None, 0, None) == -1
    assert b"null" in lib.velo_last_error()
    assert lib.velo_cluster(None, 1, None, None, None, None, None, None, None, C.c_int64(0), None, None) == -1
    assert lib.velo_fit(None, C.c_int64(5), None, None, None, None, None, None, None, None) == -1


def header_arg_counts():
    src = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b(velo_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src):
        args = m.group(2).strip()
        out[m.group(1)] = 0 if args in ("", "void") else args.count(",") + 1
    return out


def test_binding_signatures_match_header():
    from paper_2412_05041_amd import velo
    counts = header_arg_counts()
    for name, args in velo._SIGS.items():
        assert name in counts, name
        assert len(args) == counts[name], (name, len(args), counts[name])
    # every declared entry point has a binding
    assert set(counts) == set(velo._SIGS), set(counts) ^ set(velo._SIGS)
