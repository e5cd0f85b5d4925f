"""The C-ABI library: it loads, exports what include/afmm.h declares, and rejects bad
arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "afmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(afmm_[A-Za-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def afmm():
    if not os.path.exists(os.path.join(ROOT, "paper_1308_2400_amd", "libafmm.so")):
        from paper_1308_2400_amd import _build
        _build.build_library()
    import paper_1308_2400_amd
    return paper_1308_2400_amd


def test_header_declares_the_boundary():
    names = _header_functions()
    for must in ("afmm_multiply_caseA", "afmm_multiply_caseB", "afmm_multiply_batched",
                 "afmm_count_adds", "afmm_validate", "afmm_batched_plan_create", "afmm_batched_plan_launch",
                 "afmm_batched_plan_destroy", "afmm_workspace_size", "afmm_status_string"):
        assert must in names


def test_every_declared_symbol_is_exported(afmm):
    lib = ctypes.CDLL(afmm.LIB_PATH)
    for name in _header_functions():
        assert hasattr(lib, name), name
        assert hasattr(afmm, name), f"binding lacks {name}"


def test_status_strings_and_version(afmm):
    for code in range(10):
        s = afmm.afmm_status_string(code)
        assert s and s != b"unknown status"
    assert afmm.afmm_version().decode().count(".") == 2


def test_workspace_sizes(afmm):
    for case in (0, 1):
        for n in (1, 63, 64, 65, 4096):
            s = afmm.afmm_workspace_size(case, n, 0)
            assert s >= ((n + 63) // 64 * 64) ** 2
            assert afmm.afmm_workspace_size(case, n, 1) >= 4 * 2 * n * n
    assert afmm.afmm_workspace_size(0, 0, 0) == 0
    assert afmm.afmm_workspace_size(2, 8, 0) == 0


def test_argument_errors_on_host(afmm):
    f = afmm.afmm_multiply_caseB
    # n < 1, null pointers, bad mode: rejected before any device call
    assert f(0, 16, 4096, 8192, 0, None, 0, None) == 1
    assert f(8, None, 4096, 8192, 0, None, 0, None) == 1
    assert f(8, 16, 4096, 8192, 7, None, 0, None) == 1
    assert f(1 << 20, 16, 4096, 8192, 0, None, 0, None) == 1
    # Z overlapping X or Y
    assert f(8, 4096, 8192, 4096 + 64, 0, None, 0, None) == 2
    assert afmm.afmm_multiply_caseA(8, 4096, 8192, 8192 + 4, 0, None, 0, None) == 2
    # misaligned pointers
    assert f(8, 4098, 16384, 32768, 0, None, 0, None) == 1
    # count: bad case / null output
    assert afmm.afmm_count_adds(3, 8, 16, 4096, 8192, None, None, None, 0, None) == 1
    assert afmm.afmm_count_adds(0, 8, 16, 4096, None, None, None, None, 0, None) == 1


def test_rectangular_argument_errors_on_host(afmm):
    fA, fB = afmm.afmm_multiply_caseA_ex, afmm.afmm_multiply_caseB_ex
    X, Y, Z = 4096, 1 << 20, 1 << 24
    # extents below 1, leading dimensions below the row length, null pointers
    assert fB(0, 4, 4, X, 4, Y, 4, Z, 4, 0, None, 0, None) == 1
    assert fB(4, 4, 0, X, 4, Y, 4, Z, 4, 0, None, 0, None) == 1
    assert fB(4, 8, 4, X, 7, Y, 4, Z, 4, 0, None, 0, None) == 1
    assert fB(4, 8, 6, X, 8, Y, 5, Z, 6, 0, None, 0, None) == 1
    assert fA(4, 8, 6, X, 8, Y, 6, Z, 5, 0, None, 0, None) == 1
    assert fA(4, 8, 6, None, 8, Y, 6, Z, 6, 0, None, 0, None) == 1
    assert fA(70000, 8, 6, X, 8, Y, 6, Z, 6, 0, None, 0, None) == 1
    # Z's range (m-1)*ldz + n elements overlaps X's (m-1)*ldx + k
    assert fA(3, 5, 2, X, 100, Y, 2, X + 4 * 150, 2, 0, None, 0, None) == 2
    # adjacent ranges are no alias: the call gets past that check and stops at the
    # invalid mode after it (every call here must fail on the host: the addresses
    # are placeholders, and a valid call would launch kernels on them on a machine
    # with a GPU)
    assert fA(3, 5, 2, X, 5, Y, 2, X + 4 * 15, 2, 7, None, 0, None) == 1
    # counting: bad leading dimension
    assert afmm.afmm_count_adds_ex(1, 4, 8, 6, X, 7, Y, 6, Z, None, None, None, 0, None) == 1


def test_rectangular_workspace_sizes(afmm):
    for case in (0, 1):
        for (m, k, n) in [(1, 1, 1), (5, 700, 3), (300, 2, 900)]:
            s = afmm.afmm_workspace_size_ex(case, m, k, n, 0)
            rows = n if case == 0 else m
            assert s >= ((rows + 63) // 64 * 64) * ((k + 63) // 64 * 64)
            assert s >= 8 * (m + k)
            assert afmm.afmm_workspace_size_ex(case, m, k, n, 1) >= 2 * 4 * (m + n) * k
        assert afmm.afmm_workspace_size_ex(case, 64, 64, 64, 0) == afmm.afmm_workspace_size(case, 64, 0)
    assert afmm.afmm_workspace_size_ex(0, 0, 4, 4, 0) == 0


def test_config_table(afmm):
    assert afmm.config_supported("B", (0, 8, 8, 8))
    assert afmm.config_supported("A", (0, 4, 4, 4))
    assert not afmm.config_supported("B", (0, 3, 3, 3))
    assert not afmm.config_supported("B", (1, 8, 8, 8))  # mapping 1 is not compiled
    for n in (1, 100, 256, 2048, 4096, 16384):
        assert afmm.config_supported("B", afmm.default_config("B", n))
    assert afmm.config_supported("B", (0, 8, 8, 8, 2))
    assert not afmm.config_supported("B", (2, 8, 8, 4, 2))  # unroll 2 only in the LDS kernels
    assert afmm.config_supported("A", (3, 2, 16, 16, 1, 8))  # sparse-k variant
    assert afmm.config_supported("B", (3, 4, 8, 16, 2, 16))
    assert not afmm.config_supported("B", (3, 2, 16, 16, 1, 16))  # 128 KB of LDS: not built
    assert afmm.config_supported("A", (4, 4, 16, 8, 1, 16))  # compacted-base variant
    assert not afmm.config_supported("A", (4, 4, 16, 8, 1, 8))  # not instantiated
    assert afmm.config_supported("B", (7, 1, 16, 16, 1, 16))  # row lists of both factors
    assert not afmm.config_supported("B", (7, 2, 16, 16, 1, 16))  # one row per wave only
    afmm.set_tuning([])
    builtin = afmm.default_config("B", 4096)
    afmm.set_tuning([("B", 1000, 5000, (0, 4, 4, 4))])
    assert afmm.default_config("B", 4096) == (0, 4, 4, 4, 1, 16)
    assert afmm.default_config("B", 999) != (0, 4, 4, 4, 1) or builtin == (0, 4, 4, 4, 1, 16)
    assert afmm.default_config("A", 4096) == afmm.default_config("A", 4096)
    with pytest.raises(afmm.AfmmError):
        afmm.set_tuning([("B", 1, 2, (0, 3, 3, 3))])
    assert afmm.default_config("B", 4096) == (0, 4, 4, 4, 1, 16)  # rejected table left it unchanged
    afmm.set_tuning([])
    assert afmm.default_config("B", 4096) == builtin
    afmm.load_tuning()


def test_binding_fails_loudly_without_library(tmp_path):
    """The product path has no CPU fallback: a missing library is an import error."""
    import subprocess
    import sys
    code = ("import os, shutil, sys; sys.path.insert(0, %r); "
            "import importlib.util as u; "
            "spec = u.spec_from_file_location('p', %r); m = u.module_from_spec(spec); "
            "spec.loader.exec_module(m)") % (str(tmp_path), str(tmp_path / "pkg" / "__init__.py"))
    (tmp_path / "pkg").mkdir()
    src = open(os.path.join(ROOT, "paper_1308_2400_amd", "__init__.py")).read()
    (tmp_path / "pkg" / "__init__.py").write_text(src)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert r.returncode != 0 and "is not built" in r.stderr


def test_workspace_per_config(afmm):
    """The compacted-base form needs room for its lists: 8 bytes per lane column
    (rounded up to the band) per k (rounded up to 16), plus the lengths."""
    n = 1000
    base = afmm.workspace_size("A", n, config=(0, 4, 16, 16, 1, 16))
    acc = afmm.workspace_size("A", n, config=(4, 4, 16, 8, 1, 16))
    lists = 8 * 1024 * 1008
    assert base > 0 and acc >= base + lists
    assert afmm.workspace_size("A", n, config=(4, 4, 4, 8, 1, 16)) >= base + 8 * 1024 * 1008
    assert afmm.workspace_size("A", n, config=(0, 3, 3, 3)) == 0  # not compiled
    afmm.set_tuning([])
    try:
        afmm.set_tuning([("A", 1, 1 << 30, (4, 4, 16, 8, 1, 16))])
        assert afmm.workspace_size("A", n) == acc  # the picked configuration's needs
    finally:
        afmm.set_tuning([])
        afmm.load_tuning()


def test_workspace_of_the_list_forms(afmm):
    """The row-list form (mapping 7) needs only its lists: 8 bytes per element of X
    (rows padded to 64 entries) and of Y (rows padded to the 64*C band), plus one
    length per list; none of the count-byte or transpose space."""
    n = 1000
    for C in (16, 32):
        ws = afmm.workspace_size("B", n, config=(7, 1, C, 16, 1, 16))
        band = 64 * C
        lists = 8 * n * 1024 + 8 * n * ((n + band - 1) // band) * band
        assert lists <= ws <= lists + 4 * n * 2 + 4 * 256
    # unsupported shapes of the form are not compiled
    assert afmm.workspace_size("B", n, config=(7, 1, 24, 16, 1, 16)) == 0


def test_plain_strict_workspace_covers_every_form(afmm):
    """From n = 1024 to 16384 the plain strict call may take the compacted-base or
    the row-list form, so its workspace covers their lists too; outside that
    range it is the size-keyed form's alone."""
    for case in ("A", "B"):
        c = afmm._case_id(case)
        for n in (1023, 1024, 4096, 16384, 16385):
            plain = afmm.afmm_workspace_size(c, n, 0)
            keyed = afmm.workspace_size(case, n, config=afmm.default_config(case, n))
            if 1024 <= n <= 16384:
                assert plain >= keyed + 16 * n * n  # row lists of both factors: 8 B each
                assert plain >= afmm.workspace_size(case, n, config=(4, 2, 16, 8, 1, 16))
            else:
                assert plain == keyed


def test_new_entry_points_reject_bad_arguments_on_host(afmm):
    assert afmm.afmm_set_batch_shapes(64, 128) == 1   # n_mid above n_wide
    assert afmm.afmm_set_batch_shapes(64, 0) == 1
    assert afmm.afmm_set_batch_shapes(512, 128) == 0  # the built-in pair
    afmm.load_tuning()  # back to the tuned pair
    out = 1 << 20
    assert afmm.afmm_plain_form(0, 0, 4096, 8192, out, None, 0, None) == 1
    assert afmm.afmm_plain_form(2, 64, 4096, 8192, out, None, 0, None) == 1
    assert afmm.afmm_plain_form(1, 64, None, 8192, out, None, 0, None) == 1
    assert afmm.afmm_plain_form(1, 64, 4096, 8192, None, None, 0, None) == 1
    # the compacted-base list read-back: k, n_c, ldq and C checked before any device work
    q, ent, lens = 4096, 8192, 1 << 16
    assert afmm.afmm_base_lists(q, 0, 64, 64, 1, ent, lens, None) == 1      # k < 1
    assert afmm.afmm_base_lists(q, 4, 0, 64, 1, ent, lens, None) == 1      # n_c < 1
    assert afmm.afmm_base_lists(q, 4, 64, 63, 1, ent, lens, None) == 1     # ldq < n_c
    assert afmm.afmm_base_lists(q, 4, 64, 64, 0, ent, lens, None) == 1     # C < 1
    assert afmm.afmm_base_lists(q, 4, 64, 64, 65, ent, lens, None) == 1    # C > 64
    assert afmm.afmm_base_lists(None, 4, 64, 64, 1, ent, lens, None) == 1  # null pointers
    assert afmm.afmm_base_lists(q, 4, 64, 64, 1, None, lens, None) == 1
    assert afmm.afmm_base_lists(q, 4, 64, 64, 1, ent, None, None) == 1
    assert afmm.afmm_base_lists(q, 65537, 64, 64, 1, ent, lens, None) == 1  # above AFMM_MAX_N
    # the row-list read-back
    m_ = 4096
    assert afmm.afmm_row_lists(2, m_, 4, 64, 64, 64, ent, lens, None) == 1     # is_int not 0/1
    assert afmm.afmm_row_lists(1, m_, 0, 64, 64, 64, ent, lens, None) == 1     # rows < 1
    assert afmm.afmm_row_lists(1, m_, 4, 0, 64, 64, ent, lens, None) == 1      # cols < 1
    assert afmm.afmm_row_lists(1, m_, 4, 64, 63, 64, ent, lens, None) == 1     # ld < cols
    assert afmm.afmm_row_lists(1, m_, 4, 64, 64, 0, ent, lens, None) == 1      # band < 1
    assert afmm.afmm_row_lists(1, None, 4, 64, 64, 64, ent, lens, None) == 1   # null pointers
    assert afmm.afmm_row_lists(1, m_, 65536, 65536, 65536, 1, ent, lens, None) == 1  # > 2^31 lists
