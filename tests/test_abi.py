"""The C-ABI library loads and exports every function include/far.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "far.h")
LIB = os.path.join(ROOT, "paper_2606_26010_amd", "libfar.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(far_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ["far_map_create", "far_map_destroy", "far_map_insert", "far_map_knn",
                 "far_scan_covariances", "far_gicp_linearize", "far_gicp_align",
                 "far_gicp_align_batch", "far_map_stats", "far_map_export",
                 "far_status_str", "far_last_error"]:
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfar.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.far_status_str.restype = ctypes.c_char_p
    assert lib.far_status_str(2) == b"capacity exceeded"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfar.so not built")
def test_binding_names_match_header():
    from paper_2606_26010_amd import far
    names = declared_functions()
    for n in names:
        assert n in far._SIGS, n
        assert hasattr(far, n) or n in ("far_status_str", "far_last_error"), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfar.so not built")
def test_invalid_arguments_rejected_without_gpu():
    # argument checks happen before any HIP call
    from paper_2606_26010_amd import far
    L = far.lib()
    p = far.far_map_params_t(0.0, 20, -1.0, 1000, 0, 5)       # voxel_size 0
    h = ctypes.c_void_p()
    assert L.far_map_create(ctypes.byref(p), None, ctypes.byref(h)) == far.FAR_E_INVALID
    assert b"parameter" in L.far_last_error()
    p = far.far_map_params_t(1.0, 65, -1.0, 1000, 0, 5)       # N_max > 64
    assert L.far_map_create(ctypes.byref(p), None, ctypes.byref(h)) == far.FAR_E_INVALID
    assert L.far_map_insert(None, None, 0, None, None, None) == far.FAR_E_INVALID
    assert L.far_map_knn(None, None, 0, 5, 1.0, None, None, None, None) == far.FAR_E_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfar.so not built")
def test_threshold_is_host_only_and_matches_oracle(orc):
    # far_threshold_* is plain host arithmetic: checked here without a GPU
    import numpy as np
    from scipy.spatial.transform import Rotation
    from paper_2606_26010_amd import far, synth
    g = np.random.default_rng(4)
    a, b = far.Threshold(1.0 / 3.0, 120.0, 0.1), orc.Threshold(1.0 / 3.0, 120.0, 0.1)
    assert a.get() == b.get()
    for i in range(40):
        P = synth.pose(Rotation.from_rotvec(g.normal(size=3)).as_matrix(), g.normal(size=3) * 50)
        D = synth.pose(Rotation.from_rotvec(g.normal(size=3) * 10 ** g.uniform(-6, -2)).as_matrix(),
                       g.normal(size=3) * 10 ** g.uniform(-3, 0))
        da, db = a.update(P, P @ D), b.update(P, P @ D)
        assert abs(da - db) <= 1e-9 * max(1.0, db), (i, da, db)
        assert a.get() == pytest.approx(b.get(), rel=1e-9)
    with pytest.raises(far.FarError):
        far.Threshold(0.0, 120.0)
