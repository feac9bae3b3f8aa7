"""The C ABI library loads and exports every entry point bfs.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2103_13577_amd as pkg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bfs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfs_[a-z_]+)\s*\(", src)) - {"bfs_exchange_fn"})


def test_library_exports_every_declared_symbol():
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libbfs.so not built")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    names = _declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pkg.EXPORTED)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(pkg, "_lib", None)
    with pytest.raises(ImportError):
        pkg.lib()


def test_create_error_without_device():
    """Argument errors are reported through status codes, not exceptions."""
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("libbfs.so not built")
    L = pkg.lib()
    h = ctypes.c_void_p(0)
    g = pkg.bfs_graph(0, 0, 0, 0, 0, 0)
    st = L.bfs_plan_create(ctypes.byref(g), 1, None, 256, 1 << 20, ctypes.byref(h))
    assert st == 1 and not h.value
    assert b"bad sizes" in L.bfs_last_error(None)
    sz = ctypes.c_size_t(0)
    assert L.bfs_workspace_size(None, 0, None, ctypes.byref(sz)) == 1


def test_stats_wrapper_mirrors_c_struct():
    """The Python Stats record carries every field of bfs_stats."""
    import paper_2103_13577_amd as pkg
    assert [f for f, _ in pkg.bfs_stats._fields_] == list(pkg.Stats.__dataclass_fields__)


def _header():
    src = open(os.path.join(ROOT, "include", "bfs.h")).read()
    return re.sub(r"/\*.*?\*/", "", src, flags=re.S)


def _struct_fields(src, name):
    body = re.search(r"typedef struct\s*\{([^{}]*)\}\s*" + name + r"\s*;", src).group(1)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            out.append(re.findall(r"[A-Za-z_][A-Za-z_0-9]*", decl)[-1])
    return out


@pytest.mark.parametrize("name", ["bfs_options", "bfs_tuning", "bfs_stats", "bfs_graph", "bfs_query",
                                  "bfs_batch_result", "bfs_batch_counters"])
def test_binding_structs_follow_the_header(name):
    """Every ctypes mirror lists the C struct's members in the header's order
    (a missing or reordered field would shift every field after it)."""
    fields = _struct_fields(_header(), name)
    assert [f for f, _ in getattr(pkg, name)._fields_] == fields


def test_binding_constants_follow_the_header():
    src = _header()
    defs = dict(re.findall(r"#define\s+(BFS_(?:LOOP|DIR)_[A-Z_]+)\s+(\d+)", src))
    for c, v in defs.items():
        py = c[len("BFS_"):]
        assert getattr(pkg, py) == int(v), c
    assert "BFS_LOOP_ENQUEUE" in defs and "BFS_DIR_OPTIMIZING" in defs
