"""The C-ABI library loads and exports every symbol include/bluebild.h declares (no compute calls)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "bluebild.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bb_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ("bb_context_create", "bb_synth_create", "bb_synth_collect", "bb_synth_collect_eig",
              "bb_synth_collect_eig_batched", "bb_synth_eig_backward", "bb_synth_destroy"):
        assert n in names


def test_binding_covers_header():
    from paper_2310_09200_amd import _lib
    assert sorted(_lib.PROTOS) == declared_symbols()


def test_library_loads_and_exports_all_symbols():
    from paper_2310_09200_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2310_09200_amd.build import build
        build()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in declared_symbols():
        assert hasattr(lib, n), n
    lib = _lib.load()
    assert lib.bb_status_string(3) == b"BB_ERR_NOT_POSDEF"


def test_missing_library_fails_loudly(tmp_path):
    from paper_2310_09200_amd import _lib
    with pytest.raises(RuntimeError):
        _lib.load(str(tmp_path / "nope.so"))
