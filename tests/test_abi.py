"""The C-ABI library loads without a GPU and exports every function include/qlra.h declares;
argument checks that need no device run on the CPU."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header="qlra.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|double|size_t|const char\*)\s+(qlra\w*)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for required in ("qlra", "qlra_workspace_size", "qlra_status", "qlra_strerror", "qlra_omega", "qlra_qgemm",
                     "qlra_cholqr", "qlra_qsvd"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2507_13731_amd import qlra as Q
    lib = ctypes.CDLL(Q.LIB_PATH)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared()) == set(Q.EXPORTS)


def test_library_exports_the_no_alloc_entry_points():
    from paper_2507_13731_amd import qlra as Q
    names = declared("qlra_noalloc.h")
    assert names == ["qlra_noalloc", "qlra_noalloc_max_bytes", "qlra_noalloc_status"]
    lib = ctypes.CDLL(Q.LIB_PATH)
    assert all(hasattr(lib, n) for n in names)
    lib.qlra_noalloc_max_bytes.restype = ctypes.c_size_t
    assert lib.qlra_noalloc_max_bytes() == 128 << 20


def test_workspace_size_and_argument_errors_without_gpu():
    from paper_2507_13731_amd import qlra as Q
    assert Q.qlra_workspace_size(2048, 2048, 50, 10, 6, "subspace") > 0
    assert Q.qlra_workspace_size(16384, 16384, 128, 32, 8, "block_krylov") > 0
    for args in [(10, 8, 0, 2, 2, 0), (10, 8, 3, -1, 2, 0), (10, 8, 3, 2, 1, 0), (10, 8, 7, 2, 2, 0),
                 (10, 8, 3, 2, 2, 5)]:
        try:
            Q.qlra_workspace_size(*args)
        except Q.QlraError as e:
            assert e.code == Q.QLRA_E_ARG
        else:
            raise AssertionError(args)
    assert Q.strerror(Q.QLRA_E_NUMERIC).startswith("numerical")


def test_completion_workspace_and_argument_errors_without_gpu():
    from paper_2507_13731_amd import qlra as Q
    small = Q.qlra_complete_workspace_size(256, 256, 30, 10, 2, "subspace", 0.6)
    assert small > 4 * 256 * 256 * 4
    assert Q.qlra_complete_workspace_size(256, 256, 30, 10, 2, "subspace", 0.0) > 0
    assert Q.qlra_complete_workspace_size(300, 200, 20, 5, 4, "krylov", 8.0 / 3.0, transpose=True) > 0
    for sigma in (2.7, float("nan")):          # radius ceil(3 sigma) > 8, or no number
        try:
            Q.qlra_complete_workspace_size(64, 64, 4, 2, 2, "subspace", sigma)
        except Q.QlraError as e:
            assert e.code == Q.QLRA_E_UNSUPPORTED
        else:
            raise AssertionError(sigma)
    try:
        Q.qlra_complete_workspace_size(10, 8, 7, 2, 2, "subspace", 0.6)
    except Q.QlraError as e:
        assert e.code == Q.QLRA_E_ARG
    else:
        raise AssertionError("rank + p > min(m, n)")
