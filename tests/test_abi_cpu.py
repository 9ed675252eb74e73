"""The C-ABI library loads and exports exactly what include/fvpcg.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvpcg.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"FVPCG_API\s+(?:const\s+)?\w+\*?\s+\**(fvpcg_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_1505_07630_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1505_07630_amd import build

        build.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = declared()
    for n in ["fvpcg_mesh_create", "fvpcg_matrix_create", "fvpcg_solve", "fvpcg_solve_mixed",
              "fvpcg_solve_mixed_reliable", "fvpcg_solve_batched",
              "fvpcg_solve_backward", "fvpcg_spmv", "fvpcg_stream_calibrate", "fvpcg_last_error",
              "fvpcg_solve_bicgstab", "fvpcg_solve_bicgstab_multi"]:
        assert n in names
    assert len(names) == 35


def test_library_exports_every_declared_symbol(lib_path):
    import torch  # noqa: F401  (the binding loads torch's HIP runtime first)

    L = ctypes.CDLL(lib_path)
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True, check=True).stdout
    exported = sorted(set(re.findall(r" T (fvpcg_\w+)$", out, re.M)))
    assert exported == declared()


def test_binding_signatures_cover_header(lib_path):
    from paper_1505_07630_amd import _lib

    assert sorted(_lib.SIGNATURES) == declared()
    L = _lib.load()
    assert L.fvpcg_version() == 10000
    assert isinstance(L.fvpcg_last_error(), bytes)


def test_stats_struct_layout():
    """Python Stats mirrors fvpcg_stats: 4 int32 + 6 doubles = 64 bytes."""
    from paper_1505_07630_amd._lib import Stats

    assert ctypes.sizeof(Stats) == 64
    src = open(HEADER).read()
    body = src[src.index("typedef struct fvpcg_stats"):src.index("} fvpcg_stats;")]
    fields = re.findall(r"(int32_t|double)\s+(\w+);", body)
    assert [f for _, f in fields] == [f for f, _ in Stats._fields_]


def test_missing_extension_fails_loudly(tmp_path):
    code = ("import paper_1505_07630_amd._lib as L; L.LIB_PATH = '/nonexistent/libfvpcg.so'\n"
            "try:\n    L.load()\nexcept L.ExtensionMissing as e:\n    print('missing', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "missing" in r.stdout


def test_kernel_sources_build_for_gfx950_only():
    from paper_1505_07630_amd import build

    assert "--offload-arch=gfx950" in build.FLAGS
    assert "-packed-fp32-ops" in build.FLAGS
    for src in build.SOURCES:
        text = open(os.path.join(build.CSRC, src)).read()
        assert "__CUDA" not in text and "__HIP_PLATFORM" not in text


def test_binding_has_every_declared_name():
    """The Python binding exposes each C-ABI entry point under the same name."""
    import paper_1505_07630_amd as fv

    for n in declared():
        assert callable(getattr(fv, n, None)), n
