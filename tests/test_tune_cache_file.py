"""The tune cache file (MANYCLAW_TUNE_CACHE) read and written by the
library's host code, without a GPU: entries in the library's own layout and
in any JSON layout (one line, several per line, indented) are found, and a
store keeps the other entries."""
import ctypes
import json
import os

import pytest


def _lib():
    from paper_1308_1464_amd import manyclaw as mc
    L = mc.lib()
    L.mc__tune_cache_lookup.restype = ctypes.c_int
    L.mc__tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
    L.mc__tune_cache_store.restype = None
    L.mc__tune_cache_store.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int]
    return L


def _lookup(L, key):
    v = (ctypes.c_int32 * 8)()
    n = L.mc__tune_cache_lookup(key.encode(), v, 8)
    return list(v[:n])


@pytest.mark.parametrize("layout", ["one_line", "indented", "own"])
def test_cache_layouts(tmp_path, monkeypatch, layout):
    L = _lib()
    path = tmp_path / "tune.json"
    monkeypatch.setenv("MANYCLAW_TUNE_CACHE", str(path))
    entries = {"abc-1": [8, 16, 32, 64], "rows-4-0-4-1-96x96-gfx950-256": [0], "x": [24]}
    if layout == "one_line":
        path.write_text(json.dumps(entries))
    elif layout == "indented":
        path.write_text(json.dumps(entries, indent=4))
    else:
        path.write_text("{\n" + ",\n".join(f'"{k}": [{", ".join(map(str, v))}]' for k, v in entries.items())
                        + "\n}\n")
    for k, v in entries.items():
        assert _lookup(L, k) == v, (layout, k)
    assert _lookup(L, "missing") == []
    # a store adds its entry and keeps the others; the result is valid JSON
    v = (ctypes.c_int32 * 1)(40)
    L.mc__tune_cache_store(b"new-key", v, 1)
    back = json.loads(path.read_text())
    assert back == dict(entries, **{"new-key": [40]})
    assert not [p for p in os.listdir(tmp_path) if p != "tune.json"]


def test_no_cache_without_the_variable(tmp_path, monkeypatch):
    L = _lib()
    monkeypatch.delenv("MANYCLAW_TUNE_CACHE", raising=False)
    v = (ctypes.c_int32 * 1)(40)
    L.mc__tune_cache_store(b"k", v, 1)
    assert _lookup(L, "k") == []
