"""The C-ABI library loads on a machine without a GPU and exports every entry
point include/sivf.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sivf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sivf_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sivf_build_centroid_ivf", "sivf_assign", "sivf_update", "sivf_run_lloyd",
                 "sivf_soft_assign_fwd", "sivf_soft_assign_bwd"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2103_16141_amd import _native, build
    if not os.path.exists(_native.LIB_PATH):
        build.build()
    lib = ctypes.CDLL(_native.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for each of them
    bound = _native.load()
    for n in declared_functions():
        assert getattr(bound, n).argtypes is not None, n


def test_default_options_without_gpu():
    from paper_2103_16141_amd import _native as N
    lib = N.load()
    opt = N.sivf_options()
    assert lib.sivf_default_options(ctypes.byref(opt)) == 0
    assert opt.posting_dtype == N.SIVF_F32 and opt.certify == 1 and opt.filter_mode == N.SIVF_MODE_SIVF
    assert opt.k_tile == 0 and opt.workspace_cap_bytes == 0 and opt.head_density == -1.0
    assert opt.tiles_per_launch == 0
    assert lib.sivf_default_options(None) == -1


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2103_16141_amd import _native as N
    saved = N._lib
    N._lib = None
    try:
        with pytest.raises(ImportError):
            N.load(str(tmp_path / "missing.so"))
    finally:
        N._lib = saved
