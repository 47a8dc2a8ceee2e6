"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/pargeo_hip.h declares, and rejects bad arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pargeo_hip.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2207_01834_amd import _binding
    if not os.path.exists(_binding.SO):
        pytest.fail("libpargeo_hip.so is not built (run __graft_entry__.build())")
    return _binding.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pg_kdtree_build", "pg_knn", "pg_knn_all", "pg_tree_free", "pg_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2207_01834_amd import _binding
    assert set(declared_functions()) <= set(_binding.SIGNATURES)


def _err(L):
    return L.pg_last_error().decode()


def test_build_argument_errors(L):
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cases = [
        (fake, 10, 0, 16, 0, "d must be"),
        (fake, 10, 9, 16, 0, "d must be"),
        (fake, 10, 3, 0, 0, "leaf must be"),
        (fake, 10, 3, 65, 0, "leaf must be"),
        (fake, -1, 3, 16, 0, "n must be"),
        (fake, 1 << 31, 3, 16, 0, "n must be"),
        (fake, 10, 3, 16, 7, "bad dtype"),
        (None, 10, 3, 16, 0, "points is NULL"),
    ]
    for pts, n, d, leaf, dt, msg in cases:
        st = L.pg_kdtree_build(pts, n, d, leaf, dt, None, ctypes.byref(out))
        assert st == 1, (n, d, leaf, dt)
        assert msg in _err(L)
    assert L.pg_kdtree_build(fake, 10, 3, 16, 0, None, None) == 1


def test_knn_argument_errors(L):
    assert L.pg_knn(None, None, 1, 1, None, None, None) == 1
    assert "tree is NULL" in _err(L)
    assert L.pg_knn_all(None, 3, None, None, None) == 1
    assert L.pg_tree_info(None, None, None, None, None, None) == 1
    assert L.pg_tree_export(None, None, None, None) == 1
    L.pg_tree_free(None)  # no-op


def test_range_graph_spatial_argument_errors(L):
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p()
    assert L.pg_range_count(None, fake, 1, fake, None, None, None) == 1
    assert "tree is NULL" in _err(L)
    assert L.pg_range_report(None, fake, 1, fake, fake, 1, None) == 1
    assert L.pg_range_search(None, fake, 1, None, fake, fake, 1, None, None) == 1
    assert L.pg_knn_graph(None, 3, fake, fake, None) == 1
    assert L.pg_tree_offsets(None, fake, None) == 1
    st = L.pg_kdtree_build_spatial(fake, 10, 0, 16, 0, 0, None, ctypes.byref(out))
    assert st == 1 and "d must be" in _err(L)
    st = L.pg_kdtree_build_spatial(None, 10, 3, 16, 0, 0, None, ctypes.byref(out))
    assert st == 1 and "points is NULL" in _err(L)
    st = L.pg_kdtree_build_spatial(fake, 10, 3, 16, 0, 4, None, ctypes.byref(out))
    assert st == 1 and "dim_rule" in _err(L)
    assert L.pg_tree_split_dims(None, fake, None) == 1


def test_baseline_argument_errors(L):
    fake = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p()
    assert L.pg_b1_create(0, 0, 16, ctypes.byref(out)) == 1 and "d must be" in _err(L)
    assert L.pg_b1_create(3, 7, 16, ctypes.byref(out)) == 1 and "bad dtype" in _err(L)
    assert L.pg_b1_insert(None, fake, 1, None, None) == 1 and "handle is NULL" in _err(L)
    assert L.pg_b1_erase(None, fake, 1, None, None) == 1
    assert L.pg_b1_knn(None, fake, 1, 3, fake, fake, None) == 1
    assert L.pg_b1_size(None) == -1
    L.pg_b1_free(None)
    assert L.pg_b2_create(fake, 10, 3, 0, 0, None, ctypes.byref(out)) == 1 and "leaf must be" in _err(L)
    assert L.pg_b2_create(fake, -5, 3, 16, 0, None, ctypes.byref(out)) == 1 and "n must be" in _err(L)
    assert L.pg_b2_insert(None, fake, 1, None, None) == 1
    assert L.pg_b2_erase(None, fake, 1, None, None) == 1
    assert L.pg_b2_knn(None, fake, 1, 65, fake, fake, None) == 1
    assert L.pg_b2_stats(None, None, None) == 1
    assert L.pg_b2_size(None) == -1
    L.pg_b2_free(None)
    # a host-only B1 handle: argument checks on it need no device
    h = ctypes.c_void_p()
    assert L.pg_b1_create(3, 0, 16, ctypes.byref(h)) == 0
    assert L.pg_b1_insert(h, None, 5, None, None) == 1 and "points is NULL" in _err(L)
    assert L.pg_b1_knn(h, fake, 1, 0, fake, fake, None) == 1 and "k must be" in _err(L)
    assert L.pg_b1_size(h) == 0
    L.pg_b1_free(h)
    # spatial-median forms: the same checks, host-only handles
    assert L.pg_b1_create_spatial(9, 0, 16, ctypes.byref(out)) == 1 and "d must be" in _err(L)
    assert L.pg_bdl_create_spatial(3, 0, 16, 0, ctypes.byref(out)) == 1 and "buffer_X" in _err(L)
    st = L.pg_b2_create_spatial(fake, 10, 3, 65, 0, None, ctypes.byref(out))
    assert st == 1 and "leaf must be" in _err(L)
    for make, free in ((lambda o: L.pg_b1_create_spatial(2, 1, 8, o), L.pg_b1_free),
                       (lambda o: L.pg_bdl_create_spatial(2, 1, 8, 64, o), L.pg_bdl_free)):
        h = ctypes.c_void_p()
        assert make(ctypes.byref(h)) == 0 and h.value
        free(h)


def test_set_allocator_arguments(L):
    from paper_2207_01834_amd import _binding
    assert L.pg_set_allocator(None) == 0
    half = _binding.Allocator()
    half.alloc = _binding.Allocator._fields_[0][1](lambda n, s, c: None)
    assert L.pg_set_allocator(ctypes.byref(half)) == 1 and "both" in _err(L)
    assert L.pg_set_allocator(None) == 0


def test_header_is_plain_c(tmp_path):
    """The boundary header compiles as pedantic C99 (no C++ in the
    signatures) and as C++17."""
    import shutil
    import subprocess
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    src = tmp_path / "h.c"
    src.write_text('#include "pargeo_hip.h"\nint main(void) { return 0; }\n')
    for cc, args in (("gcc", ["-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror"]),
                     ("g++", ["-std=c++17", "-Wall", "-Werror", "-x", "c++"])):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        r = subprocess.run([cc, *args, "-I", inc, "-fsyntax-only", str(src)],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
