"""MI355X-native structured inverted-file spherical k-means (SIVF).

The compute path is libsivf.so (HIP kernels for gfx950 behind the C ABI in
include/sivf.h).  This package is its Python binding; importing it does not
load the library, the first call does, and fails loudly if it is not built.
"""
from ._native import LIB_PATH, SivfError, load  # noqa: F401


def __getattr__(name):
    if name in ("Context", "DeviceCsr", "Ivf", "Lloyd", "run_lloyd"):
        from . import api
        return getattr(api, name)
    if name == "SoftAssignLoss":
        from .soft_assign import SoftAssignLoss
        return SoftAssignLoss
    raise AttributeError(name)
