"""The C-ABI library loads and exports every entry point that include/fk.h declares
(no compute calls: this runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fk.h")
LIB = os.path.join(ROOT, "paper_2509_02649_amd", "libfastkernel.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:fk_status|const char\*|size_t)\s+(fk_[a-z0-9_]+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfastkernel.so is not built; run python -m paper_2509_02649_amd.build")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ["fk_create", "fk_destroy", "fk_gram", "fk_solve", "fk_fit", "fk_predict", "fk_heldout_mse",
                 "fk_fit_backward", "fk_additive_gram", "fk_additive_fit", "fk_status_string"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_table_matches_header():
    from paper_2509_02649_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


def test_status_strings(lib):
    f = lib.fk_status_string
    f.restype = C.c_char_p
    f.argtypes = [C.c_int]
    assert f(0) == b"ok"
    assert b"outside" in f(2)
    assert f(99) == b"unknown status"


def test_workspace_queries_and_host_validation(lib):
    from paper_2509_02649_amd import _lib
    L = _lib.load(LIB)
    nb = C.c_size_t()
    assert L.fk_gram_workspace_size(None, 2, 10_000_000, 1, 32, C.byref(nb)) == 0
    # 2-D: FP64 grid 2 x 512^2, records 3 words per point, bin tables
    assert nb.value >= 10_000_000 * 12 + 2 * 512 * 512 * 8
    assert L.fk_gram_workspace_size(None, 3, 100, 1, 8, C.byref(nb)) == 0          # 3-D: FP64 grid 2 x 128^3
    assert nb.value >= 2 * 128 ** 3 * 8
    assert L.fk_gram_workspace_size(None, 3, 100, 1, 32, C.byref(nb)) == 1         # 3-D m > 31 rejected
    assert L.fk_gram_workspace_size(None, 4, 100, 1, 4, C.byref(nb)) == 1          # d = 4 rejected
    assert L.fk_fit_workspace_size(None, 3, 100, 1, 8, 1, C.byref(nb)) == 1        # dense fit is 1-D / 2-D
    assert L.fk_gram_workspace_size(None, 1, 0, 1, 8, C.byref(nb)) == 1            # n = 0 rejected
    assert L.fk_gram_workspace_size(None, 1, 100, 1, 65, C.byref(nb)) == 1         # m > 64 rejected
    assert L.fk_solve_workspace_size(None, 2, 32, 16, 64, C.byref(nb)) == 0
    Np = 4288
    assert nb.value >= 64 * Np * Np * 4 + 2 * Np * Np * 8
    # the fit's two parts: the solve's layout (as fk_solve's) and the type-1 scratch, summing to fk_fit's
    solve_b = nb.value
    sb, tb, fb = C.c_size_t(), C.c_size_t(), C.c_size_t()
    assert L.fk_fit_kept_workspace_size(None, 2, 10_000_000, 16, 32, 64, C.byref(sb), C.byref(tb)) == 0
    assert L.fk_fit_workspace_size(None, 2, 10_000_000, 16, 32, 64, C.byref(fb)) == 0
    assert sb.value == solve_b and sb.value + tb.value == fb.value
    assert L.fk_fit_kept_workspace_size(None, 3, 100, 1, 8, 1, C.byref(sb), C.byref(tb)) == 1   # 1-D / 2-D only
    assert L.fk_predict_workspace_size(None, 2, 32, 1, C.byref(nb)) == 0
    assert L.fk_additive_fit_workspace_size(None, 10, 1000, 1, 32, 1, C.byref(nb)) == 0
    assert L.fk_additive_gram_workspace_size(None, 1, 1000, 1, 32, C.byref(nb)) == 1   # d = 1 rejected
    # iterative solve: spectrum Lf^d, two intermediates Lf^(d-1) (2m+1) and three vectors per system
    assert L.fk_solve_cg_workspace_size(None, 2, 32, 16, 64, C.byref(nb)) == 0
    assert nb.value >= 256 * 256 * 16 + 2 * 1024 * 256 * 65 * 16 + 3 * 1024 * 65 * 65 * 16
    assert L.fk_solve_cg_workspace_size(None, 3, 16, 1, 1, C.byref(nb)) == 0
    assert L.fk_solve_cg_workspace_size(None, 3, 64, 1, 1, C.byref(nb)) == 1        # 3-D m > 63 rejected
    assert L.fk_solve_cg_workspace_size(None, 2, 256, 1, 1, C.byref(nb)) == 1       # Lf > 1024 rejected
    assert L.fk_solve_cg_workspace_size(None, 4, 4, 1, 1, C.byref(nb)) == 1         # d = 4 rejected
    assert L.fk_solve_cg_workspace_size(None, 2, 8, 1024, 128, C.byref(nb)) == 1    # > 65536 systems
    plain = nb.value
    assert L.fk_solve_cg_collocation_workspace_size(None, 2, 8, 1024, 128, C.byref(nb)) == 1
    assert L.fk_solve_cg_collocation_workspace_size(None, 3, 16, 1, 1, C.byref(nb)) == 0
    assert nb.value > plain                                                        # + spectrum, D x, Sigma_r D x
    assert L.fk_toeplitz_apply_workspace_size(None, 1, 255, 3, C.byref(nb)) == 0
    assert L.fk_toeplitz_apply_workspace_size(None, 1, 8, 0, C.byref(nb)) == 1      # no vectors
    # entry points reject a null context before touching the device
    assert L.fk_gram(None, 1, 10, 0, C.c_void_p(1), 0, None, 4, C.c_void_p(1), None, C.c_void_p(1), 1 << 20,
                     None) == 1


def test_autotune_table_file_roundtrip(tmp_path):
    # host-only: the table file format of the launch-shape autotuner (no device is touched)
    from paper_2509_02649_amd import _lib
    L = _lib.load(LIB)
    path = tmp_path / "tune.txt"
    path.write_text(
        "# measured on gfx950\n"
        "gfx950 t1 d=2 nf=512 w=7 nw=16 n=2^30 = mb=2 spread_pts=16384 sort_blk=512 sort_slice=65536 ms=75.3\n"
        "gfx950 dense Np=4288 nlam=64 ntgt=16 = pair=1 trsm_wg=256   # trailing comment\n"
        "gfx950 broken = mb=two\n"
        "no separator here\n"
        "gfx950 empty = \n")
    assert L.fk_autotune_clear() == 0
    assert L.fk_autotune_load(str(path).encode()) == 0
    n = C.c_size_t()
    assert L.fk_autotune_table(None, 0, C.byref(n)) == 0
    buf = C.create_string_buffer(n.value + 1)
    assert L.fk_autotune_table(buf, 2, C.byref(n)) == 1                     # too small
    assert L.fk_autotune_table(buf, n.value + 1, C.byref(n)) == 0
    lines = buf.value.decode().splitlines()
    assert lines == ["gfx950 dense Np=4288 nlam=64 ntgt=16 = pair=1 trsm_wg=256",
                     "gfx950 t1 d=2 nf=512 w=7 nw=16 n=2^30 = mb=2 spread_pts=16384 sort_blk=512 sort_slice=65536 "
                     "ms=75.3"]
    assert L.fk_autotune_load(str(tmp_path / "missing.txt").encode()) == 1
    assert L.fk_autotune_clear() == 0
    assert L.fk_autotune_table(None, 0, C.byref(n)) == 0 and n.value == 0
