"""Python binding of libflusi (the MI355X pseudo-spectral penalized Navier-Stokes path).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libflusi.so.  PyTorch supplies device memory and the stream.  The
flusi_* functions mirror the C ABI of include/flusi.h one to one; `Plan` is a
small convenience wrapper around them that allocates torch tensors.

There is no fallback: if libflusi.so is missing or no GPU is present, the calls
raise.
"""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np
import torch  # loads the HIP runtime that libflusi shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libflusi.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "flusi.h")

FLUSI_OK = 0
FLUSI_EINVAL = -1
FLUSI_EUNSUPPORTED = -2
FLUSI_ENOMEM = -3
FLUSI_EDEVICE = -4
FLUSI_ENONFINITE = -5
FLUSI_F32, FLUSI_F64 = 0, 1
FLUSI_BODY_NONE, FLUSI_BODY_SPHERE, FLUSI_BODY_ELLIPSOID = 0, 1, 2
FLUSI_SMOOTH_COS, FLUSI_SMOOTH_TANH = 0, 1
FLUSI_MEAN_FIXED, FLUSI_MEAN_FREE = 0, 1
FLUSI_NDIAG = 41
FLUSI_NPASS = 6
PASS_NAMES = ("z_inverse", "y_inverse", "x_pass", "kinematics", "y_forward", "z_pass")
SUPPORTED_N = (16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512)


class FlusiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"flusi error {code}: {msg}")
        self.code = code


FLUSI_INT_AB2, FLUSI_INT_RK4 = 0, 1
FLUSI_KIN_SINE, FLUSI_KIN_FOURIER, FLUSI_KIN_HERMITE = 0, 1, 2
FLUSI_KIN_MAX = 24
FLUSI_WING_ELLIPSE, FLUSI_WING_FOURIER, FLUSI_WING_RECT = 0, 1, 2
FLUSI_WING_MAX = 32
FLUSI_RTABLE = 25000
_KIN = {"sine": FLUSI_KIN_SINE, "fourier": FLUSI_KIN_FOURIER, "hermite": FLUSI_KIN_HERMITE}
_WING = {"ellipse": FLUSI_WING_ELLIPSE, "fourier": FLUSI_WING_FOURIER, "rectangle": FLUSI_WING_RECT}


class flusi_insect(ctypes.Structure):
    _fields_ = [
        ("body", ctypes.c_int), ("wings", ctypes.c_int), ("smooth", ctypes.c_int), ("free_flight", ctypes.c_int),
        ("c_smth", ctypes.c_double),
        ("x_cntr", ctypes.c_double * 3), ("u_cntr", ctypes.c_double * 3),
        ("psi", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
        ("psi_dot", ctypes.c_double), ("beta_dot", ctypes.c_double), ("gamma_dot", ctypes.c_double),
        ("radius", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
        ("eta_stroke", ctypes.c_double),
        ("pivot_l", ctypes.c_double * 3), ("pivot_r", ctypes.c_double * 3),
        ("wing_A", ctypes.c_double), ("wing_B", ctypes.c_double), ("wing_t", ctypes.c_double),
        ("freq", ctypes.c_double),
        ("phi", ctypes.c_double * 3), ("alpha", ctypes.c_double * 3), ("theta", ctypes.c_double * 3),
        ("mass", ctypes.c_double), ("inertia", ctypes.c_double * 3), ("gravity", ctypes.c_double),
        ("dof", ctypes.c_double * 6),
        ("kin_type", ctypes.c_int), ("kin_n", ctypes.c_int), ("wing_shape", ctypes.c_int), ("wing_n", ctypes.c_int),
        ("kin_coef", ((ctypes.c_double * (FLUSI_KIN_MAX + 1)) * 2) * 3),
        ("wing_c", ctypes.c_double * 2),
        ("wing_coef", (ctypes.c_double * (FLUSI_WING_MAX + 1)) * 2),
        ("head_x", ctypes.c_double * 3), ("head_r", ctypes.c_double),
        ("eye_x", ctypes.c_double * 3), ("eye_r", ctypes.c_double),
        ("wing_rect", ctypes.c_double * 4),
        ("wing_J", ctypes.c_double * 6),
    ]


class flusi_step_params(ctypes.Structure):
    _fields_ = [
        ("nsteps", ctypes.c_int), ("mean_mode", ctypes.c_int),
        ("dt_fixed", ctypes.c_double), ("cfl", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("eta_cap", ctypes.c_double), ("t_end", ctypes.c_double),
        ("history", ctypes.c_void_p),
    ]


class flusi_schedule(ctypes.Structure):
    _fields_ = [("y_inverse", ctypes.c_int), ("x_pass", ctypes.c_int), ("y_forward", ctypes.c_int),
                ("z_pass", ctypes.c_int), ("split_z", ctypes.c_int), ("reserved", ctypes.c_int * 3)]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k in ("y_inverse", "x_pass", "y_forward", "z_pass", "split_z")}


class flusi_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("has_insect", ctypes.c_int),
                ("L", ctypes.c_double), ("nu", ctypes.c_double), ("eta", ctypes.c_double),
                ("ins", flusi_insect), ("p", flusi_step_params), ("u0", ctypes.c_void_p)]


class flusi_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("waiting", ctypes.c_longlong), ("active", ctypes.c_longlong),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("point_steps", ctypes.c_double), ("busy_s", ctypes.c_double),
                ("mpoint_steps_per_s", ctypes.c_double), ("peak_bytes", ctypes.c_size_t),
                ("peak_active", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {k: (getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


_P = ctypes.c_void_p
_SIGS = {
    "flusi_last_error": (ctypes.c_char_p, []),
    "flusi_plan_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.POINTER(_P)]),
    "flusi_plan_destroy": (ctypes.c_int, [_P]),
    "flusi_set_stream": (ctypes.c_int, [_P, _P]),
    "flusi_plan_workspace_bytes": (ctypes.c_size_t, [_P]),
    "flusi_state_bytes": (ctypes.c_size_t, [_P]),
    "flusi_tables": (ctypes.c_int, [_P, _P, _P]),
    "flusi_fft_r2c": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "flusi_fft_c2r": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "flusi_fft_c2r_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_int]),
    "flusi_mask_insect": (ctypes.c_int, [_P, ctypes.POINTER(flusi_insect), ctypes.c_double, _P, _P, _P]),
    "flusi_rhs": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "flusi_state_init": (ctypes.c_int, [_P, _P, _P, ctypes.c_double]),
    "flusi_state_export_uhat": (ctypes.c_int, [_P, _P, _P]),
    "flusi_state_velocity": (ctypes.c_int, [_P, _P, _P]),
    "flusi_state_time": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "flusi_step": (ctypes.c_int, [_P, _P, ctypes.POINTER(flusi_insect), ctypes.POINTER(flusi_step_params)]),
    "flusi_forces": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "flusi_state_solid": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "flusi_plan_set_integrator": (ctypes.c_int, [_P, ctypes.c_int]),
    "flusi_plan_set_walls": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "flusi_state_set_solid": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_double)]),
    "flusi_profile": (ctypes.c_int, [_P, ctypes.c_int]),
    "flusi_pass_times": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
    "flusi_plan_set_sponge": (ctypes.c_int, [_P, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "flusi_plan_get_schedule": (ctypes.c_int, [_P, ctypes.POINTER(flusi_schedule)]),
    "flusi_plan_set_schedule": (ctypes.c_int, [_P, ctypes.POINTER(flusi_schedule)]),
    "flusi_autotune": (ctypes.c_int, [_P, _P, ctypes.POINTER(flusi_insect), ctypes.POINTER(flusi_step_params),
                                      ctypes.c_int, ctypes.POINTER(flusi_schedule)]),
    "flusi_ensemble_autotune": (ctypes.c_int, [_P, ctypes.c_int]),
    "flusi_sizes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t)]),
    "flusi_request_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "flusi_server_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_P)]),
    "flusi_server_destroy": (ctypes.c_int, [_P]),
    "flusi_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(flusi_request), ctypes.POINTER(ctypes.c_longlong)]),
    "flusi_server_wait": (ctypes.c_int, [_P, ctypes.c_longlong, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]),
    "flusi_server_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(flusi_server_stats)]),
    "flusi_ensemble_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_P)]),
    "flusi_ensemble_destroy": (ctypes.c_int, [_P]),
    "flusi_ensemble_set_stream": (ctypes.c_int, [_P, _P]),
    "flusi_ensemble_add": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(flusi_insect), ctypes.POINTER(flusi_step_params),
                                          ctypes.POINTER(ctypes.c_int)]),
    "flusi_ensemble_remove": (ctypes.c_int, [_P, ctypes.c_int]),
    "flusi_ensemble_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "flusi_ensemble_step": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libflusi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1506_06513_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/flusi.h."""
    txt = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*\s]+?\b(flusi_\w+)\s*\(", txt, re.M)))


def _check(rc: int):
    if rc != FLUSI_OK:
        raise FlusiError(rc, lib().flusi_last_error().decode())


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        if not t.is_cuda:
            raise ValueError("flusi needs device tensors")
        if not t.is_contiguous():
            raise ValueError("flusi needs contiguous tensors")
        return t.data_ptr()
    return int(t)


# ----------------------------------------------------------------------------
# C ABI, one to one
# ----------------------------------------------------------------------------

def flusi_plan_create(nx: int, ny: int, nz: int, L: float, nu: float, eta: float, dtype: int):
    h = _P()
    _check(lib().flusi_plan_create(nx, ny, nz, L, nu, eta, dtype, ctypes.byref(h)))
    return h


def flusi_plan_destroy(plan):
    _check(lib().flusi_plan_destroy(plan))


def flusi_set_stream(plan, stream):
    _check(lib().flusi_set_stream(plan, _P(stream)))


def flusi_plan_workspace_bytes(plan) -> int:
    return int(lib().flusi_plan_workspace_bytes(plan))


def flusi_state_bytes(plan) -> int:
    return int(lib().flusi_state_bytes(plan))


def flusi_tables(plan, n: int):
    j = (ctypes.c_int * n)()
    k = (ctypes.c_int * n)()
    _check(lib().flusi_tables(plan, ctypes.cast(j, _P), ctypes.cast(k, _P)))
    return np.array(j[:], dtype=np.int64), np.array(k[:], dtype=np.int64)


def flusi_fft_r2c(plan, inp, out, nf: int):
    _check(lib().flusi_fft_r2c(plan, _ptr(inp), _ptr(out), nf))


def flusi_fft_c2r(plan, inp, out, nf: int):
    _check(lib().flusi_fft_c2r(plan, _ptr(inp), _ptr(out), nf))


def flusi_fft_c2r_noalloc(plan, inp, out, nf: int):
    _check(lib().flusi_fft_c2r_noalloc(plan, _ptr(inp), _ptr(out), nf))


def flusi_mask_insect(plan, ins: flusi_insect, t: float, chi, us, colour):
    _check(lib().flusi_mask_insect(plan, ctypes.byref(ins), t, _ptr(chi), _ptr(us), _ptr(colour)))


def flusi_rhs(plan, uhat, chi, us, rhs_hat, mean_mode: int, want_umax: bool = False):
    um = ctypes.c_double(0.0)
    _check(lib().flusi_rhs(plan, _ptr(uhat), _ptr(chi), _ptr(us), _ptr(rhs_hat), mean_mode,
                           ctypes.byref(um) if want_umax else None))
    return um.value if want_umax else None


def flusi_state_init(plan, state, u0, t0: float):
    _check(lib().flusi_state_init(plan, _ptr(state), _ptr(u0), t0))


def flusi_state_export_uhat(plan, state, uhat):
    _check(lib().flusi_state_export_uhat(plan, _ptr(state), _ptr(uhat)))


def flusi_state_velocity(plan, state, u):
    _check(lib().flusi_state_velocity(plan, _ptr(state), _ptr(u)))


def flusi_state_time(plan, state):
    t = ctypes.c_double()
    n = ctypes.c_longlong()
    _check(lib().flusi_state_time(plan, _ptr(state), ctypes.byref(t), ctypes.byref(n)))
    return t.value, n.value


def flusi_step(plan, state, ins: flusi_insect | None, params: flusi_step_params):
    _check(lib().flusi_step(plan, _ptr(state), ctypes.byref(ins) if ins is not None else None,
                            ctypes.byref(params)))


def flusi_forces(plan, state):
    out = (ctypes.c_double * FLUSI_NDIAG)()
    rc = lib().flusi_forces(plan, _ptr(state), out)
    return rc, np.array(out[:])


def flusi_state_solid(plan, state) -> np.ndarray:
    out = (ctypes.c_double * 13)()
    _check(lib().flusi_state_solid(plan, _ptr(state), out))
    return np.array(out[:])


def flusi_state_set_solid(plan, state, y):
    v = (ctypes.c_double * 13)(*[float(x) for x in y])
    _check(lib().flusi_state_set_solid(plan, _ptr(state), v))


def flusi_profile(plan, enable: bool):
    _check(lib().flusi_profile(plan, 1 if enable else 0))


def flusi_pass_times(plan):
    ms = (ctypes.c_double * FLUSI_NPASS)()
    cnt = (ctypes.c_longlong * FLUSI_NPASS)()
    _check(lib().flusi_pass_times(plan, ms, cnt))
    return np.array(ms[:]), np.array(cnt[:], dtype=np.int64)


def flusi_plan_set_sponge(plan, c_sp: float, thickness=None):
    th = (ctypes.c_double * 3)(*[float(v) for v in thickness]) if thickness is not None else None
    _check(lib().flusi_plan_set_sponge(plan, c_sp, th))


def flusi_plan_get_schedule(plan) -> flusi_schedule:
    s = flusi_schedule()
    _check(lib().flusi_plan_get_schedule(plan, ctypes.byref(s)))
    return s


def flusi_plan_set_schedule(plan, sched: flusi_schedule):
    _check(lib().flusi_plan_set_schedule(plan, ctypes.byref(sched)))


def flusi_autotune(plan, state, ins: flusi_insect | None, params: flusi_step_params, reps: int) -> flusi_schedule:
    s = flusi_schedule()
    _check(lib().flusi_autotune(plan, _ptr(state), ctypes.byref(ins) if ins is not None else None,
                                ctypes.byref(params), reps, ctypes.byref(s)))
    return s


def flusi_ensemble_autotune(ens, reps: int):
    _check(lib().flusi_ensemble_autotune(ens, reps))


def make_schedule(d: dict) -> flusi_schedule:
    s = flusi_schedule()
    for k, v in d.items():
        setattr(s, k, int(v))
    return s


def flusi_sizes(n: int, dtype: int):
    w = ctypes.c_size_t()
    st = ctypes.c_size_t()
    _check(lib().flusi_sizes(n, dtype, ctypes.byref(w), ctypes.byref(st)))
    return w.value, st.value


def flusi_request_bytes(n: int, dtype: int) -> int:
    return int(lib().flusi_request_bytes(n, dtype))


def flusi_server_create(dtype: int, hbm_budget: int, max_chunk: int):
    h = _P()
    _check(lib().flusi_server_create(dtype, hbm_budget, max_chunk, ctypes.byref(h)))
    return h


def flusi_server_destroy(srv):
    _check(lib().flusi_server_destroy(srv))


def flusi_server_submit(srv, req: flusi_request) -> int:
    i = ctypes.c_longlong()
    _check(lib().flusi_server_submit(srv, ctypes.byref(req), ctypes.byref(i)))
    return i.value


def flusi_server_wait(srv, rid: int, timeout_ms: float, u_host, diag: bool = True):
    """Returns (status, diag array, latency ms); status 1 = timed out."""
    d = (ctypes.c_double * FLUSI_NDIAG)()
    lat = ctypes.c_double()
    rc = lib().flusi_server_wait(srv, rid, timeout_ms, u_host, d, ctypes.byref(lat))
    return rc, np.array(d[:]), lat.value


def flusi_server_stats_get(srv) -> dict:
    st = flusi_server_stats()
    _check(lib().flusi_server_stats_get(srv, ctypes.byref(st)))
    return st.as_dict()


def flusi_ensemble_create(dtype: int):
    h = _P()
    _check(lib().flusi_ensemble_create(dtype, ctypes.byref(h)))
    return h


def flusi_ensemble_destroy(ens):
    _check(lib().flusi_ensemble_destroy(ens))


def flusi_ensemble_set_stream(ens, stream):
    _check(lib().flusi_ensemble_set_stream(ens, _P(stream)))


def flusi_ensemble_add(ens, plan, state, ins: flusi_insect | None, params: flusi_step_params) -> int:
    i = ctypes.c_int(-1)
    _check(lib().flusi_ensemble_add(ens, plan, _ptr(state), ctypes.byref(ins) if ins is not None else None,
                                    ctypes.byref(params), ctypes.byref(i)))
    return i.value


def flusi_ensemble_remove(ens, member: int):
    _check(lib().flusi_ensemble_remove(ens, member))


def flusi_ensemble_size(ens):
    m = ctypes.c_int()
    g = ctypes.c_int()
    _check(lib().flusi_ensemble_size(ens, ctypes.byref(m), ctypes.byref(g)))
    return m.value, g.value


def flusi_ensemble_step(ens, nsteps: int, use_graph: bool):
    _check(lib().flusi_ensemble_step(ens, nsteps, 1 if use_graph else 0))


# ----------------------------------------------------------------------------
# Conveniences
# ----------------------------------------------------------------------------

_BODY = {"none": FLUSI_BODY_NONE, "sphere": FLUSI_BODY_SPHERE, "ellipsoid": FLUSI_BODY_ELLIPSOID}
_SMOOTH = {"cos": FLUSI_SMOOTH_COS, "tanh": FLUSI_SMOOTH_TANH}


def make_insect(d: dict | None) -> flusi_insect | None:
    """flusi_insect from a plain parameter dict (the keys of the struct)."""
    if d is None:
        return None
    s = flusi_insect()
    s.body = _BODY[d.get("body", "none")]
    s.wings = 1 if d.get("wings", False) else 0
    s.smooth = _SMOOTH[d.get("smooth", "cos")]
    s.c_smth = float(d.get("c_smth", 1.0))
    s.free_flight = 1 if d.get("free_flight", False) else 0
    s.mass = float(d.get("mass", 1.0))
    s.inertia[:] = [float(v) for v in d.get("inertia", (1.0, 1.0, 1.0))]
    s.gravity = float(d.get("gravity", 0.0))
    s.dof[:] = [float(v) for v in d.get("dof", (1.0,) * 6)]
    kin = d.get("kin", "sine")
    s.kin_type = _KIN[kin]
    if kin != "sine":
        series = [d.get(k, ((), ())) for k in ("kin_phi", "kin_alpha", "kin_theta")]
        lens = {len(c[0]) for c in series} | {len(c[1]) for c in series}
        if len(lens) != 1:
            raise ValueError("wing angle series need equal lengths for all angles and both rows")
        m = lens.pop()
        if m < 1 or m > FLUSI_KIN_MAX + 1:
            raise ValueError(f"wing angle series: 1..{FLUSI_KIN_MAX + 1} entries per row")
        s.kin_n = m - 1 if kin == "fourier" else m
        for a, c in enumerate(series):
            for r in range(2):
                for i, v in enumerate(c[r]):
                    s.kin_coef[a][r][i] = float(v)
    s.wing_shape = _WING[d.get("wing_shape", "ellipse")]
    if s.wing_shape == FLUSI_WING_FOURIER:
        fa, fb = d.get("wing_fa", ()), d.get("wing_fb", ())
        if len(fa) != len(fb) or not 1 <= len(fa) <= FLUSI_WING_MAX + 1:
            raise ValueError(f"Fourier wing: 1..{FLUSI_WING_MAX + 1} coefficients, as many b as a")
        s.wing_n = len(fa) - 1
        for i in range(len(fa)):
            s.wing_coef[0][i] = float(fa[i])
            s.wing_coef[1][i] = float(fb[i])
        s.wing_c[:] = [float(v) for v in d.get("wing_c", (0.0, 0.0))]
    if s.wing_shape == FLUSI_WING_RECT:
        s.wing_rect[:] = [float(d.get(k, dv)) for k, dv in
                          (("rect_a", 0.0), ("rect_tip", 1.0), ("rect_b", 0.0), ("rect_B", 0.0))]
    s.head_x[:] = [float(v) for v in d.get("head_x", (0.0, 0.0, 0.0))]
    s.head_r = float(d.get("head_r", 0.0))
    s.eye_x[:] = [float(v) for v in d.get("eye_x", (0.0, 0.0, 0.0))]
    s.eye_r = float(d.get("eye_r", 0.0))
    s.wing_J[:] = [float(v) for v in d.get("wing_J", (0.0,) * 6)]
    for k in ("x_cntr", "u_cntr", "pivot_l", "pivot_r", "phi", "alpha", "theta"):
        default = {"pivot_l": (0.0, 0.15, 0.0), "pivot_r": (0.0, -0.15, 0.0)}.get(k, (0.0, 0.0, 0.0))
        getattr(s, k)[:] = [float(v) for v in d.get(k, default)]
    for k, dv in (("psi", 0.0), ("beta", 0.0), ("gamma", 0.0), ("psi_dot", 0.0), ("beta_dot", 0.0),
                  ("gamma_dot", 0.0), ("radius", 0.5), ("a", 0.5), ("b", 0.1), ("eta_stroke", 0.0),
                  ("wing_A", 0.175), ("wing_B", 0.5), ("wing_t", 0.0), ("freq", 1.0)):
        setattr(s, k, float(d.get(k, dv)))
    return s


class Plan:
    """A plan plus torch-allocated buffers on the current device and stream."""

    def __init__(self, n: int, L: float, nu: float, eta: float, dtype: str = "f64", nx: int | None = None):
        """n points and side L on y and z; nx points on x (default n), whose side
        is L*nx/n (one grid spacing on every axis)."""
        if not torch.cuda.is_available():
            raise RuntimeError("flusi needs a ROCm GPU")
        self.nx = n if nx is None else nx
        self.n, self.L, self.nu, self.eta = n, L, nu, eta
        self.Lx = L if self.nx == n else L * self.nx / n
        self.dtype = dtype
        self.rdt = torch.float64 if dtype == "f64" else torch.float32
        self.cdt = torch.complex128 if dtype == "f64" else torch.complex64
        self.handle = flusi_plan_create(self.nx, n, n, L, nu, eta, FLUSI_F64 if dtype == "f64" else FLUSI_F32)
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.sync_stream()

    def sync_stream(self):
        flusi_set_stream(self.handle, torch.cuda.current_stream().cuda_stream)

    def close(self):
        if self.handle is not None:
            flusi_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # tensors
    @property
    def shape(self):
        """Physical field shape [z][y][x]."""
        return (self.n, self.n, self.nx)

    def _fields(self, t, nf_shape, what):
        if tuple(t.shape[1:]) != nf_shape or t.dim() != 4:
            raise ValueError(f"{what}: expected [nf]{list(nf_shape)}, got {list(t.shape)}")

    def real(self, nf: int):
        return torch.empty((nf,) + self.shape, dtype=self.rdt, device=self.dev)

    def spec(self, nf: int):
        return torch.empty((nf, self.n, self.n, self.nx // 2 + 1), dtype=self.cdt, device=self.dev)

    def r2c(self, f: torch.Tensor) -> torch.Tensor:
        f = f.to(self.dev, self.rdt).contiguous()
        self._fields(f, self.shape, "r2c")
        nf = f.shape[0]
        out = self.spec(nf)
        flusi_fft_r2c(self.handle, f, out, nf)
        return out

    def c2r(self, fh: torch.Tensor) -> torch.Tensor:
        fh = fh.to(self.dev, self.cdt).contiguous()
        self._fields(fh, (self.n, self.n, self.nx // 2 + 1), "c2r")
        nf = fh.shape[0]
        out = self.real(nf)
        flusi_fft_c2r(self.handle, fh, out, nf)
        return out

    def mask(self, insect: dict, t: float):
        chi = torch.empty(self.shape, dtype=self.rdt, device=self.dev)
        us = self.real(3)
        col = torch.empty(self.shape, dtype=torch.int16, device=self.dev)
        flusi_mask_insect(self.handle, make_insect(insect), t, chi, us, col)
        return chi, us, col

    def rhs(self, uhat, chi=None, us=None, mean_mode: int = FLUSI_MEAN_FIXED, want_umax=False):
        uhat = uhat.to(self.dev, self.cdt).contiguous()
        out = self.spec(3)
        chi = None if chi is None else chi.to(self.dev, self.rdt).contiguous()
        us = None if us is None else us.to(self.dev, self.rdt).contiguous()
        um = flusi_rhs(self.handle, uhat, chi, us, out, mean_mode, want_umax)
        return (out, um) if want_umax else out

    def new_state(self, u0, t0: float = 0.0) -> torch.Tensor:
        st = torch.empty(flusi_state_bytes(self.handle), dtype=torch.uint8, device=self.dev)
        u0 = torch.as_tensor(u0).to(self.dev, self.rdt).contiguous()
        if tuple(u0.shape) != (3,) + self.shape:
            raise ValueError(f"new_state: expected [3]{list(self.shape)}, got {list(u0.shape)}")
        flusi_state_init(self.handle, st, u0, t0)
        return st

    def step(self, state, nsteps: int, insect: dict | None = None, dt_fixed: float = 0.0, cfl: float = 0.1,
             dt_max: float = 0.0, eta_cap: float = 0.5, t_end: float = 0.0, mean_mode: int = FLUSI_MEAN_FIXED,
             history: bool = False):
        hist = torch.zeros((nsteps, FLUSI_NDIAG), dtype=torch.float64, device=self.dev) if history else None
        p = flusi_step_params(nsteps, mean_mode, dt_fixed, cfl, dt_max, eta_cap, t_end,
                              hist.data_ptr() if hist is not None else None)
        flusi_step(self.handle, state, make_insect(insect), p)
        return hist

    def forces(self, state):
        return flusi_forces(self.handle, state)

    def solid(self, state) -> np.ndarray:
        """Free-flight state (x_cntr, u_cntr, eps, Omega_b) of the current time level."""
        return flusi_state_solid(self.handle, state)

    def set_solid(self, state, y):
        flusi_state_set_solid(self.handle, state, y)

    def set_integrator(self, name: str):
        """'ab2' (integrating-factor AB2, default) or 'rk4' (explicit diffusion)."""
        _check(lib().flusi_plan_set_integrator(self.handle, {"ab2": FLUSI_INT_AB2, "rk4": FLUSI_INT_RK4}[name]))

    def set_walls(self, thickness=(0.0, 0.0, 0.0), u_wall=(0.0, 0.0, 0.0)):
        """Dirichlet layers at the top end of the axes with thickness > 0, u = u_wall there."""
        th = (ctypes.c_double * 3)(*[float(v) for v in thickness])
        uw = (ctypes.c_double * 3)(*[float(v) for v in u_wall])
        _check(lib().flusi_plan_set_walls(self.handle, th, uw))

    def set_sponge(self, c_sp: float, thickness=(0.0, 0.0, 0.0)):
        """Vorticity sponge (layers at the top end of the axes with thickness > 0)."""
        flusi_plan_set_sponge(self.handle, c_sp, thickness)

    def schedule(self) -> dict:
        return flusi_plan_get_schedule(self.handle).as_dict()

    def set_schedule(self, sched: dict):
        cur = self.schedule()
        cur.update(sched)
        flusi_plan_set_schedule(self.handle, make_schedule(cur))

    def autotune(self, state, insect: dict | None = None, reps: int = 10, **controls) -> dict:
        return flusi_autotune(self.handle, state, make_insect(insect), step_params(0, **controls), reps).as_dict()

    def velocity(self, state) -> torch.Tensor:
        u = self.real(3)
        flusi_state_velocity(self.handle, state, u)
        return u

    def uhat(self, state) -> torch.Tensor:
        out = self.spec(3)
        flusi_state_export_uhat(self.handle, state, out)
        return out

    def time(self, state):
        return flusi_state_time(self.handle, state)


def step_params(nsteps: int = 0, dt_fixed: float = 0.0, cfl: float = 0.1, dt_max: float = 0.0, eta_cap: float = 0.5,
                t_end: float = 0.0, mean_mode: int = FLUSI_MEAN_FIXED, history=None) -> flusi_step_params:
    return flusi_step_params(nsteps, mean_mode, dt_fixed, cfl, dt_max, eta_cap, t_end,
                             _ptr(history) if history is not None else None)


class Ensemble:
    """Many (plan, state) members advanced together by flusi_ensemble_step.

    Keeps references to the member plans and states so that they outlive the
    ensemble."""

    def __init__(self, dtype: str = "f32"):
        self.dtype = dtype
        self.handle = flusi_ensemble_create(FLUSI_F64 if dtype == "f64" else FLUSI_F32)
        self._keep = {}
        flusi_ensemble_set_stream(self.handle, torch.cuda.current_stream().cuda_stream)

    def add(self, plan: Plan, state: torch.Tensor, insect: dict | None = None, history=None, **controls) -> int:
        p = step_params(0, history=history, **controls)
        i = flusi_ensemble_add(self.handle, plan.handle, state, make_insect(insect), p)
        self._keep[i] = (plan, state, history)
        return i

    def remove(self, member: int):
        flusi_ensemble_remove(self.handle, member)
        self._keep.pop(member, None)

    def size(self):
        return flusi_ensemble_size(self.handle)

    def step(self, nsteps: int, graph: bool = False):
        flusi_ensemble_step(self.handle, nsteps, graph)

    def autotune(self, reps: int = 5):
        flusi_ensemble_autotune(self.handle, reps)

    def close(self):
        if self.handle is not None:
            flusi_ensemble_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop with continuous batching (flusi_server_*).

    submit() copies the request (and its initial field) and returns an id;
    wait() returns (status, u [3][n][n][n] as numpy, diagnostics, latency ms)."""

    def __init__(self, dtype: str = "f32", hbm_budget: int | None = None, max_chunk: int = 20):
        self.dtype = dtype
        self.np_dt = np.float64 if dtype == "f64" else np.float32
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.8)
        self.budget = hbm_budget
        self.handle = flusi_server_create(FLUSI_F64 if dtype == "f64" else FLUSI_F32, hbm_budget, max_chunk)
        self._n = {}

    def submit(self, n: int, L: float, nu: float, eta: float, steps: int, insect: dict | None = None,
               u0: np.ndarray | None = None, **controls) -> int:
        r = flusi_request()
        r.n, r.L, r.nu, r.eta = n, L, nu, eta
        ins = make_insect(insect)
        r.has_insect = 1 if ins is not None else 0
        if ins is not None:
            r.ins = ins
        r.p = step_params(steps, **controls)
        keep = None
        if u0 is not None:
            keep = np.ascontiguousarray(u0, dtype=self.np_dt)
            assert keep.shape == (3, n, n, n)
            r.u0 = keep.ctypes.data
        rid = flusi_server_submit(self.handle, r)
        self._n[rid] = n
        return rid

    def wait(self, rid: int, timeout_ms: float = -1.0, want_u: bool = True):
        n = self._n[rid]
        u = np.empty((3, n, n, n), dtype=self.np_dt) if want_u else None
        rc, diag, lat = flusi_server_wait(self.handle, rid, timeout_ms, u.ctypes.data if want_u else None)
        if rc != 1:
            self._n.pop(rid, None)
        return rc, u, diag, lat

    def stats(self) -> dict:
        return flusi_server_stats_get(self.handle)

    def close(self):
        if self.handle is not None:
            flusi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
