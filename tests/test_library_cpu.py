"""Host-side checks of libfastfact that need no GPU: the C ABI loads, exports every
symbol include/fastfact.h declares, and rejects invalid arguments before any
device work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastfact.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1812_02056_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_1812_02056_amd import build
        build.build()
    return binding.load()


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("chol_factor", "lu_nopiv_factor", "chol_solve"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1812_02056_amd import binding
    names = _declared_functions()
    assert sorted(names) == sorted(binding.EXPORTED)
    for n in names:
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value


def test_version_and_status_strings(lib):
    from paper_1812_02056_amd import binding
    assert "gfx950" in binding.version()
    assert binding.status_string(0) == "success"
    assert "workspace" in binding.status_string(-101)
    assert "invalid argument" in binding.status_string(-4)


def test_invalid_arguments_are_rejected_on_the_host(lib):
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    assert lib.chol_factor(-1, 4, fake, 1, 0, 0, null, 0, fake, null) == -1
    assert lib.chol_factor(8, 0, fake, 8, 0, 0, null, 0, fake, null) == -2
    assert lib.chol_factor(8, 4, null, 8, 0, 0, null, 0, fake, null) == -3
    assert lib.chol_factor(8, 4, fake, 7, 0, 0, null, 0, fake, null) == -4
    assert lib.chol_factor(8, 4, fake, 8, 7, 0, null, 0, fake, null) == -5
    assert lib.chol_factor(8, 4, fake, 8, 0, 1 << 9, null, 0, fake, null) == -6
    assert lib.chol_factor(8, 4, fake, 8, 0, 0, null, 0, null, null) == -9
    # binary32 storage needs a binary64 workspace for the diagonal blocks
    assert lib.chol_factor(8, 4, fake, 8, 1, 0, null, 0, fake, null) == -101
    assert lib.lu_nopiv_factor(8, 4, fake, 8, 1, 0, null, 0, fake, null) == -102
    assert lib.ff_update_syrk(8, 4, fake, 7, fake, 8, 0, 0, null) == -4
    assert lib.ff_update_gemm(8, 4, fake, 8, fake, 8, fake, 3, 0, 0, null) == -8


def test_workspace_sizes(lib):
    assert lib.ff_chol_workspace_size(100, 27, 0, 0) == 0
    assert lib.ff_chol_workspace_size(100, 27, 1, 0) >= 27 * 27 * 8
    assert lib.ff_chol_workspace_size(10, 27, 2, 0) >= 10 * 10 * 8
    assert lib.ff_trisolve_workspace_size(130, 0) >= 3 * 64 * 64 * 8
    assert lib.ff_solve_workspace_size(1000, 64, 4, 1, 0) > lib.ff_solve_workspace_size(1000, 64, 1, 1, 0)
    assert lib.ff_solve_workspace_size(0, 64, 4, 1, 0) == 0
    # escalation to binary64 needs an n x n binary64 factor in the workspace
    assert (lib.ff_solve_workspace_size(1000, 64, 1, 2, 8) - lib.ff_solve_workspace_size(1000, 64, 1, 2, 0)
            >= 1000 * 1000 * 8)
    assert lib.ff_solve_workspace_size(1000, 64, 1, 0, 8) == lib.ff_solve_workspace_size(1000, 64, 1, 0, 0)


def _header_without_comments():
    return re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)


def test_flag_constants_match_the_header():
    # the binding's flag values are the header's FF_FLAG_* enumerators
    from paper_1812_02056_amd import binding
    text = _header_without_comments()
    flags = dict(re.findall(r"\b(FF_FLAG_[A-Z0-9_]+)\s*=\s*1u\s*<<\s*(\d+)", text))
    assert set(flags) == {"FF_FLAG_STRASSEN1", "FF_FLAG_NO_LOOKAHEAD", "FF_FLAG_FIXED_STEP", "FF_FLAG_ESCALATE",
                          "FF_FLAG_GMRES_IR", "FF_FLAG_STRASSEN2"}
    for name, shift in flags.items():
        assert getattr(binding, name[3:]) == 1 << int(shift), name


def test_kernel_profile_layout_matches_the_header():
    # ff_kernel_profile: the ctypes mirror has the header's fields, in order
    from paper_1812_02056_amd import binding
    text = _header_without_comments()
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*ff_kernel_profile;", text).group(1)
    fields = re.findall(r"(int64_t|double)\s+(\w+);", body)
    ctype = {"int64_t": ctypes.c_int64, "double": ctypes.c_double}
    assert [(n, ctype[t]) for t, n in fields] == list(binding.KernelProfile._fields_)


def test_noalloc_rejects_sizes_beyond_its_scratch(lib):
    # the size check runs on the host before any device work: the pointers are
    # never dereferenced
    fake = ctypes.c_void_p(0x1000)
    null = ctypes.c_void_p(0)
    assert lib.ff_trisolve_workspace_size(9344, 0) <= 32 << 20 < lib.ff_trisolve_workspace_size(9345, 0)
    assert lib.ff_trisolve_workspace_size(18688, 1) <= 32 << 20 < lib.ff_trisolve_workspace_size(18689, 1)
    assert lib.chol_trisolve_noalloc(9345, 1, fake, 9345, 0, fake, 9345, null, null) == -103
    assert lib.chol_trisolve_noalloc(18689, 1, fake, 18689, 1, fake, 18689, null, null) == -103
    assert lib.chol_trisolve_noalloc(-1, 1, fake, 1, 0, fake, 1, null, null) == -1
    assert lib.chol_trisolve_noalloc(8, 1, fake, 7, 0, fake, 8, null, null) == -4
    from paper_1812_02056_amd import binding
    assert "static scratch" in binding.status_string(-103)


def test_solve_info_layout_matches_the_header():
    from paper_1812_02056_amd import binding
    text = _header_without_comments()
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*ff_solve_info;", text).group(1)
    fields = re.findall(r"(int32_t|double)\s+(\w+);", body)
    ctype = {"int32_t": ctypes.c_int32, "double": ctypes.c_double}
    assert [(n, ctype[t]) for t, n in fields] == list(binding.SolveInfo._fields_)


def test_qr_argument_checks_and_workspace(lib):
    # rejected before any device work: these run without a GPU
    info = ctypes.c_int32(0)
    p = ctypes.c_void_p(16)
    assert lib.qr_factor(10, 20, 4, p, 10, p, 10, p, 20, 0, 0, p, 1 << 20, ctypes.byref(info), None) == -1
    assert lib.qr_factor(20, 10, 0, p, 20, p, 20, p, 10, 0, 0, p, 1 << 20, ctypes.byref(info), None) == -3
    assert lib.qr_factor(20, 10, 4, p, 19, p, 20, p, 10, 0, 0, p, 1 << 20, ctypes.byref(info), None) == -5
    assert lib.qr_factor(20, 10, 4, p, 20, p, 20, p, 9, 0, 0, p, 1 << 20, ctypes.byref(info), None) == -9
    assert lib.qr_factor(20, 10, 4, p, 20, p, 20, p, 10, 0, 1, p, 1 << 20, ctypes.byref(info), None) == -11
    assert lib.qr_factor(20, 10, 4, p, 20, p, 20, p, 10, 0, 0, p, 1 << 20, None, None) == -14
    assert lib.ff_qr_workspace_size(20, 10, 4, 0, 0) > 0
    assert lib.ff_qr_workspace_size(10, 20, 4, 0, 0) == 0
    assert lib.ff_qr_step(1000, 1000, 100) == 100
    assert lib.ff_qr_step(1000, 50, 100) == 50
    assert 1 <= lib.ff_qr_step(16384, 16384, 10 ** 6) <= 256


def test_strassen2_flag_checks_and_workspace(lib):
    p = ctypes.c_void_p(16)
    info = ctypes.c_int32(0)
    # two levels need a workspace for LU (binary64 only), and are not taken by Cholesky
    assert lib.ff_lu_workspace_size(4096, 512, 0, 32) >= (2048 * 2048 + 2 * 2048 * 256) * 8
    assert lib.ff_lu_workspace_size(4096, 512, 0, 0) == 0
    assert lib.lu_nopiv_factor(4096, 512, p, 4096, 0, 32, None, 0, ctypes.byref(info), None) == -101
    assert lib.lu_nopiv_factor(4096, 512, p, 4096, 0, 1 | 32, p, 1 << 40, ctypes.byref(info), None) == -6
    assert lib.chol_factor(4096, 512, p, 4096, 0, 32, p, 1 << 40, ctypes.byref(info), None) == -102
