"""Autotune cache (BB_TUNE_CACHE) read on the host: bb_tune_cache_lookup touches
no device, so the file format, keying and precedence are checked on the CPU."""

import ctypes

import pytest

from paper_2310_09200_amd import _lib

LINES = [
    '{"arch": "gfx950", "precision": 2, "k_class": 1, "pix_log2": 18, "tile": 9, "ms": 177.0}',
    '{"arch": "gfx950", "precision": 2, "k_class": 2, "pix_log2": 18, "tile": 6, "ms": 577.6}',
    'not an entry at all',
    '{"arch": "gfx942", "precision": 2, "k_class": 0, "pix_log2": 18, "tile": 8, "ms": 1.0}',
    '{"arch": "gfx950", "precision": 3, "k_class": 0, "pix_log2": 18, "tile": 3, "ms": 1.0}',
    '{"arch": "gfx950", "precision": 2, "k_class": 3, "pix_log2": 20, "tile": 4, "ms": 99.0}',
    # a tile class 0 may not use (256 eigenpairs per pass): ignored
    '{"arch": "gfx950", "precision": 2, "k_class": 0, "pix_log2": 18, "tile": 0, "ms": 1.0}',
    # a later line for the same key wins
    '{"arch": "gfx950", "precision": 2, "k_class": 2, "pix_log2": 18, "tile": 11, "ms": 565.8}',
]


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def lookup(lib, arch, precision, n_pix):
    out = (ctypes.c_int32 * _lib.BB_K_CLASSES)()
    st = lib.bb_tune_cache_lookup(arch.encode(), precision, n_pix, out)
    return st, list(out)


def test_lookup_keys_and_precedence(lib, tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    path.write_text("\n".join(LINES) + "\n")
    monkeypatch.setenv("BB_TUNE_CACHE", str(path))
    assert lookup(lib, "gfx950", 2, 512 * 512) == (_lib.BB_OK, [-1, 9, 11, -1])
    # the key is floor(log2(n_pix)): 2^18 .. 2^19 - 1 share it
    assert lookup(lib, "gfx950", 2, 2 ** 19 - 1)[1] == [-1, 9, 11, -1]
    assert lookup(lib, "gfx950", 2, 2 ** 18 - 1)[1] == [-1, -1, -1, -1]
    assert lookup(lib, "gfx950", 2, 1024 * 1024)[1] == [-1, -1, -1, 4]
    assert lookup(lib, "gfx942", 2, 512 * 512)[1] == [8, -1, -1, -1]
    assert lookup(lib, "gfx950", 3, 512 * 512)[1] == [3, -1, -1, -1]
    assert lookup(lib, "gfx950", 0, 512 * 512)[1] == [-1, -1, -1, -1]


def test_lookup_without_cache(lib, tmp_path, monkeypatch):
    monkeypatch.delenv("BB_TUNE_CACHE", raising=False)
    assert lookup(lib, "gfx950", 2, 512 * 512) == (_lib.BB_OK, [-1, -1, -1, -1])
    monkeypatch.setenv("BB_TUNE_CACHE", str(tmp_path / "missing.jsonl"))
    assert lookup(lib, "gfx950", 2, 512 * 512) == (_lib.BB_OK, [-1, -1, -1, -1])


def test_lookup_rejects_bad_arguments(lib):
    out = (ctypes.c_int32 * _lib.BB_K_CLASSES)()
    assert lib.bb_tune_cache_lookup(None, 2, 100, out) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_tune_cache_lookup(b"gfx950", 2, 0, out) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_tune_cache_lookup(b"gfx950", 7, 100, out) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_tune_cache_lookup(b"gfx950", 2, 100, None) == _lib.BB_ERR_INVALID_ARG
