"""C-ABI checks that need no GPU: the library loads and exports every symbol
that include/mala.h declares, and the pure host functions behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mala.h")
LIB = os.path.join(ROOT, "paper_2411_19617_amd", "libmala.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mala_[a-z_]+)\s*\(", src)))


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for n in ("mala_descriptors", "mala_ldos_infer", "mala_integrate", "mala_predict", "mala_create",
              "mala_weights_load", "mala_last_error"):
        assert n in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libmala.so not built")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_n_descriptors_matches_paper_formula(lib):
    lib.mala_n_descriptors.restype = ctypes.c_int32
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "snap_dim.txt"))
            if l.strip() and not l.startswith("#")]
    for tj, n in rows:
        assert lib.mala_n_descriptors(int(tj)) == int(n)
    assert lib.mala_n_descriptors(-1) == -1


def test_null_arguments_are_rejected_without_a_device(lib):
    lib.mala_last_error.restype = ctypes.c_char_p
    lib.mala_create.restype = ctypes.c_int32
    assert lib.mala_create(0, None, None) == -1
    assert b"NULL" in lib.mala_last_error()
    for name in ("mala_descriptors", "mala_ldos_infer", "mala_integrate", "mala_predict", "mala_synchronize"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int32
    assert lib.mala_synchronize(None) == -1
    assert lib.mala_destroy(None) == 0
    assert lib.mala_weights_free(None) == 0


def test_version_string(lib):
    lib.mala_version.restype = ctypes.c_char_p
    assert lib.mala_version().startswith(b"mala-gfx950")


def test_result_record_layout():
    # mala_result as the Python binding decodes it: 4 doubles, 4 int32, 2 doubles
    import paper_2411_19617_amd as mala
    assert mala.RESULT_BYTES == 64
    assert ctypes.sizeof(mala.Result) == 64
    assert mala.Result.entropy.offset == 48 and mala.Result.e_entropy.offset == 56


@pytest.mark.parametrize("nmax4,lmax4", [(1, 1), (1, 2), (2, 2), (3, 2), (2, 3), (3, 3)])
def test_ace4_set_matches_oracle(lib, nmax4, lmax4):
    """The library chooses its non-redundant rank-4 set by Gram-Schmidt on
    the symmetrised coupling coefficients of its own Clebsch-Gordan table;
    the oracle by the rank of the same coefficients from the Racah formula.
    Both must give the same (p1, p2, p3, p4, L) list in the same order."""
    import oracle
    n = lib.mala_ace4_count(nmax4, lmax4)
    buf = (ctypes.c_int32 * (5 * n))()
    assert lib.mala_ace4_list(nmax4, lmax4, buf, n) == n
    got = [tuple(buf[5 * k:5 * k + 5]) for k in range(n)]
    assert got == [tuple(int(x) for x in d) for d in oracle.ace4_set(nmax4, lmax4)]


def test_ace4_unsupported_sizes(lib):
    assert lib.mala_ace4_count(4, 2) < 0 and lib.mala_ace4_count(2, 4) < 0 and lib.mala_ace4_count(0, 1) < 0
