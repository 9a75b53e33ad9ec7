"""The C-ABI library loads and exports every symbol include/bumbar.h declares.

No compute call is made (these run without a GPU).
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bumbar.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bumbar_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2609_03541_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("libbumbar.so is not built (run __graft_entry__.build())")
    return _capi.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2609_03541_amd import _capi
    assert set(declared_functions()) == set(_capi.SIGNATURES)


def test_default_options_are_the_papers_settings(lib):
    from paper_2609_03541_amd import _capi
    o = _capi.Options()
    lib.bumbar_default_options(C.byref(o))
    # n0 = 100, eps = 1e-3, inc = 10, N_intermediate = 20 (Section 2, after Algorithm 1)
    assert (o.n0, o.eps, o.inc, o.n_intermediate) == (100, 1e-3, 10, 20)
    assert o.tol > 0 and o.finisher == _capi.FINISH_NEWTON


def test_library_was_built_from_this_tree(lib):
    # bumbar_version ends with the hash of the sources, header and flags
    from paper_2609_03541_amd.build import source_hash
    v = lib.bumbar_version().decode()
    assert v.endswith("src:" + source_hash()), (v, source_hash())


def test_version_and_null_context(lib):
    from paper_2609_03541_amd import _capi
    assert lib.bumbar_version().decode().startswith("bumbar")
    assert lib.bumbar_last_error(None) == b""
    assert lib.bumbar_create(None, 0, None) == -1
    nb = C.c_size_t()
    assert lib.bumbar_query_workspace(None, 4, 10, 0, None, C.byref(nb)) == -1
    assert lib.bumbar_model_energies(None, 4, 10, 1, 2, None, None, 0, None) == -1
    srv = C.c_void_p()
    assert lib.bumbar_server_create(None, C.byref(srv)) == -1
    bad = _capi.ServerOptions(0, 1 << 20, 0, 1)  # max_active < 1 is rejected before any HIP call
    assert lib.bumbar_server_create(C.byref(bad), C.byref(srv)) == -1
    t = C.c_uint64()
    assert lib.bumbar_server_submit(None, None, C.byref(t)) == -1
    assert lib.bumbar_server_poll(None, 1, None) == -1
    assert lib.bumbar_server_wait(None, 1) == -1
    n = C.c_int(7)
    assert lib.bumbar_server_progress(None, C.byref(n)) == -1 and n.value == 0
    assert lib.bumbar_server_counters(None, None, None, None, None) == -1
    lib.bumbar_server_destroy(None)


def test_struct_layouts_match_header():
    # field order of the ctypes mirrors follows the header text
    from paper_2609_03541_amd import _capi
    text = open(os.path.join(ROOT, "include", "bumbar.h")).read()
    for struct, cls in [("bumbar_options", _capi.Options), ("bumbar_stats", _capi.Stats),
                        ("bumbar_check", _capi.Check),
                        ("bumbar_server_options", _capi.ServerOptions),
                        ("bumbar_request", _capi.Request)]:
        m = re.search(r"typedef struct \{((?:(?!typedef).)*?)\}\s*" + struct + ";", text,
                      flags=re.S)
        body = re.sub(r"/\*.*?\*/", "", m.group(1), flags=re.S)
        fields = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*;", body)
        assert fields == [f for f, _ in cls._fields_], struct


def test_fused_server_needs_caller_driven(lib):
    # fuse = 1 is refused for a threaded server and for values other than
    # 0/1, before any device call
    from paper_2609_03541_amd import _capi
    h = C.c_void_p()
    for caller_driven, fuse in ((0, 1), (1, 2), (1, -1)):
        o = _capi.ServerOptions(0, 1 << 20, 2, caller_driven, fuse)
        assert lib.bumbar_server_create(C.byref(o), C.byref(h)) == -1
        assert not h.value
