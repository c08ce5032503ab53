"""Host paths of the library under AddressSanitizer and UndefinedBehavior-
Sanitizer (run as a subprocess by test_host_sanitizers.py, with the ASan
runtime preloaded and the sanitized build of the library, on a host without
a GPU): the argument checks and error paths of the ABI that return before
(or because of) a failing device call, including the clean-up of a plan,
ensemble or server whose device calls fail."""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import paper_1506_06513_amd as F  # noqa: E402
from paper_1506_06513_amd.build import SAN_LIB  # noqa: E402

F.LIB_PATH = SAN_LIB
L = F.lib()
OK, EINVAL, EUNSUP = F.FLUSI_OK, F.FLUSI_EINVAL, F.FLUSI_EUNSUPPORTED


def rc_of(fn, *args):
    try:
        fn(*args)
        return OK
    except F.FlusiError as e:
        return e.code


def host_only():
    assert L.flusi_last_error() is not None
    ws, sb = ctypes.c_size_t(), ctypes.c_size_t()
    for n in (16, 32):
        for dt in (F.FLUSI_F32, F.FLUSI_F64):
            assert L.flusi_sizes(n, dt, ctypes.byref(ws), ctypes.byref(sb)) == OK and ws.value > 0 and sb.value > 0
            assert L.flusi_request_bytes(n, dt) > 0
    assert L.flusi_sizes(40, F.FLUSI_F32, ctypes.byref(ws), ctypes.byref(sb)) == EUNSUP
    assert L.flusi_sizes(16, 7, ctypes.byref(ws), ctypes.byref(sb)) == EINVAL
    assert L.flusi_request_bytes(40, F.FLUSI_F32) == 0
    p = ctypes.c_void_p()
    assert L.flusi_plan_create(16, 16, 8, 1.0, 0.1, 1.0, F.FLUSI_F32, ctypes.byref(p)) == EUNSUP
    assert L.flusi_plan_create(16, 16, 16, -1.0, 0.1, 1.0, F.FLUSI_F32, ctypes.byref(p)) == EINVAL
    assert L.flusi_plan_create(16, 16, 16, 1.0, 0.1, 1.0, 9, ctypes.byref(p)) == EINVAL
    assert L.flusi_plan_create(17, 17, 17, 1.0, 0.1, 1.0, F.FLUSI_F32, ctypes.byref(p)) == EUNSUP
    assert L.flusi_plan_create(16, 16, 16, 1.0, 0.1, 1.0, F.FLUSI_F32, None) == EINVAL
    # a valid plan: without a GPU its device allocations fail and the partly
    # built plan is released; with one it is created and destroyed
    rc = L.flusi_plan_create(16, 16, 16, 1.0, 0.1, 1.0, F.FLUSI_F64, ctypes.byref(p))
    assert rc in (OK, F.FLUSI_ENOMEM, F.FLUSI_EDEVICE), rc
    if rc == OK:
        assert L.flusi_plan_destroy(p) == OK
    assert L.flusi_plan_destroy(None) == OK
    for name in ("flusi_fft_r2c", "flusi_fft_c2r", "flusi_fft_c2r_noalloc"):
        assert getattr(L, name)(None, None, None, 1) == EINVAL
    assert L.flusi_step(None, None, None, None) == EINVAL
    assert L.flusi_plan_set_integrator(None, 0) == EINVAL
    assert L.flusi_ensemble_create(5, ctypes.byref(p)) == EINVAL
    assert L.flusi_ensemble_step(None, 1, 0) == EINVAL
    assert L.flusi_ensemble_destroy(None) == OK
    assert L.flusi_server_create(5, 1 << 20, 1, ctypes.byref(p)) == EINVAL
    assert L.flusi_server_create(F.FLUSI_F32, 0, 1, ctypes.byref(p)) == EINVAL
    assert L.flusi_server_destroy(None) == OK
    # valid ensemble and server: without a GPU their stream creation fails and
    # the partly built objects are released
    for create, destroy, args in ((L.flusi_ensemble_create, L.flusi_ensemble_destroy, (F.FLUSI_F32,)),
                                  (L.flusi_server_create, L.flusi_server_destroy, (F.FLUSI_F32, 1 << 30, 4))):
        rc = create(*args, ctypes.byref(p))
        assert rc in (OK, F.FLUSI_EDEVICE, F.FLUSI_ENOMEM), rc
        if rc == OK:
            assert destroy(p) == OK
    st = F.flusi_server_stats()
    assert L.flusi_server_stats_get(None, ctypes.byref(st)) == EINVAL
    print("host paths: ok", flush=True)


if __name__ == "__main__":
    host_only()
