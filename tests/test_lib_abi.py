"""The C-ABI library loads and exports every function declared in include/flusi.h
(no compute calls: runs without a GPU)."""
import ctypes
import os

import pytest

import paper_1506_06513_amd as F


def test_library_exports_every_header_function():
    if not os.path.exists(F.LIB_PATH):
        pytest.fail(f"{F.LIB_PATH} not built; run python -m paper_1506_06513_amd.build")
    lib = ctypes.CDLL(F.LIB_PATH)
    names = F.header_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(F._SIGS)


def test_struct_layouts_match_header():
    # flusi_insect: 4 ints + 47 doubles, then 4 ints, the angle series, the Fourier wing and the
    # head/eye spheres, the rectangle and the wing inertia; flusi_step_params: 2 ints, 5 doubles, 1 pointer
    assert ctypes.sizeof(F.flusi_insect) == 16 + 8 * 47 + 16 + 8 * (3 * 2 * 25 + 2 + 2 * 33 + 8 + 4 + 6)
    assert ctypes.sizeof(F.flusi_step_params) == 8 + 5 * 8 + 8


def test_error_paths_without_gpu():
    lib = F.lib()
    h = ctypes.c_void_p()
    assert lib.flusi_plan_create(64, 64, 32, 1.0, 0.1, 1e-3, F.FLUSI_F64, ctypes.byref(h)) == F.FLUSI_EUNSUPPORTED
    assert b"ny = nz" in lib.flusi_last_error()
    assert lib.flusi_plan_create(40, 32, 32, 1.0, 0.1, 1e-3, F.FLUSI_F64, ctypes.byref(h)) == F.FLUSI_EUNSUPPORTED
    assert b"40 x 32 x 32 not supported" in lib.flusi_last_error()
    assert lib.flusi_plan_create(100, 100, 100, 1.0, 0.1, 1e-3, F.FLUSI_F64, ctypes.byref(h)) == F.FLUSI_EUNSUPPORTED
    assert lib.flusi_plan_create(64, 64, 64, -1.0, 0.1, 1e-3, F.FLUSI_F64, ctypes.byref(h)) == F.FLUSI_EINVAL
    assert lib.flusi_plan_create(64, 64, 64, 1.0, 0.1, 1e-3, 7, ctypes.byref(h)) == F.FLUSI_EINVAL
    assert lib.flusi_plan_create(64, 64, 64, 1.0, 0.1, 1e-3, F.FLUSI_F64, None) == F.FLUSI_EINVAL
    assert lib.flusi_step(None, None, None, None) == F.FLUSI_EINVAL
    assert lib.flusi_state_bytes(None) == 0


def test_insect_struct_from_dict():
    import workloads as W
    s = F.make_insect(W.model_insect(256, 4.0))
    assert s.body == F.FLUSI_BODY_ELLIPSOID and s.wings == 1 and s.smooth == F.FLUSI_SMOOTH_COS
    assert abs(s.wing_t - 4 * 4.0 / 256) < 1e-15
    assert list(s.pivot_r) == [0.0, -0.15, 0.0]
    assert list(s.wing_J) == [0.0] * 6
    s = F.make_insect(dict(W.model_insect(64, 4.0), wing_J=(1, 2, 3, 4, 5, 6)))
    assert list(s.wing_J) == [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]


def test_size_queries_need_no_device():
    # footprints are computed on the host from the grid size alone
    for n in F.SUPPORTED_N:
        ws, sb = F.flusi_sizes(n, F.FLUSI_F32)
        ws64, sb64 = F.flusi_sizes(n, F.FLUSI_F64)
        assert 0 < sb < ws and ws64 > ws and sb64 > sb
        assert F.flusi_request_bytes(n, F.FLUSI_F32) > ws + sb
    with pytest.raises(F.FlusiError) as e:
        F.flusi_sizes(100, F.FLUSI_F32)
    assert e.value.code == F.FLUSI_EUNSUPPORTED
    assert F.flusi_request_bytes(100, F.FLUSI_F32) == 0
