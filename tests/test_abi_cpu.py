"""Host-side checks that need no GPU: the library builds, loads, and exports every
entry point include/pasta.h declares (no compute calls)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "pasta.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pasta_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("pasta_coo_create", "pasta_mttkrp", "pasta_cp_grad", "pasta_cp_sample", "pasta_adam_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1902_03317_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == declared()


def test_status_strings_and_host_argument_checks():
    from paper_1902_03317_amd._lib import lib
    assert lib.pasta_status_str(0) == b"ok"
    assert lib.pasta_status_str(2) == b"coordinate out of range"
    n = ctypes.c_size_t()
    dims = (ctypes.c_uint64 * 3)(100, 80, 60)
    assert lib.pasta_coo_workspace_bytes(3, dims, 20000, ctypes.byref(n)) == 0
    # 3 modes x (3 index copies + values + perm); every mode sorts in one 8-bit pass
    assert 3 * 5 * 20000 * 4 <= n.value < 3 * 5 * 20000 * 4 + 300_000
    big = (ctypes.c_uint64 * 3)(1000, 80, 60)
    assert lib.pasta_coo_workspace_bytes(3, big, 20000, ctypes.byref(n)) == 0
    # two ping-pong sets of (key, permutation, 2 indices, values) for multi-pass sorts
    assert n.value >= 3 * 5 * 20000 * 4 + 2 * 5 * 20000 * 4
    assert lib.pasta_coo_workspace_bytes(1, dims, 10, ctypes.byref(n)) == 3  # order 1 unsupported
    assert lib.pasta_coo_workspace_bytes(9, dims, 10, ctypes.byref(n)) == 3
    assert lib.pasta_coo_workspace_bytes(3, None, 10, ctypes.byref(n)) == 1
    zero = (ctypes.c_uint64 * 3)(100, 0, 60)
    assert lib.pasta_coo_workspace_bytes(3, zero, 10, ctypes.byref(n)) == 1
    # the largest sizes taken: nnz < 2^32 (32-bit positions), order 8
    assert lib.pasta_coo_workspace_bytes(3, dims, (1 << 32) - 1, ctypes.byref(n)) == 0
    assert lib.pasta_coo_workspace_bytes(3, dims, 1 << 32, ctypes.byref(n)) == 3
    dims8 = (ctypes.c_uint64 * 8)(*([4] * 8))
    assert lib.pasta_coo_workspace_bytes(8, dims8, 1000, ctypes.byref(n)) == 0
    # the static-scratch entry point and the check refuse a null handle before touching the device
    assert lib.pasta_mttkrp_static(None, 0, None, 0, 8, 8, None, 1.0, None, 8, None) == 1
    assert lib.pasta_coo_check(None, None) == 1
    assert lib.pasta_status_str(6) == b"a kernel found the preprocessed tensor inconsistent"
    h = ctypes.c_void_p()
    # a workspace that is too small is refused before anything touches the device
    assert lib.pasta_coo_create(3, dims, 0, None, None, None, 0, None, ctypes.byref(h)) == 4
    assert lib.pasta_mttkrp(None, 0, None, 0, 8, 8, None, 1.0, None, 8, None, 0, None) == 1
