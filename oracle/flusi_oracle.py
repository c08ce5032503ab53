"""FP64 NumPy/SciPy oracle of the FluSI hot path (arXiv:1506.06513).

TEST INFRASTRUCTURE ONLY -- used by tests/, the smoke check and the benchmark's
CPU-baseline leg.  It is written from the paper, step by step, with no blocking,
fusion or pruning, and it shares no code with the HIP library.

What it computes (paper section / equation in brackets):

* the volume-penalized Navier-Stokes equations in rotational form
  [Sec. 2.1, eq. PNST_org_momentum], with the optional vorticity sponge
  [Sec. 2.3],
* Fourier pseudo-spectral discretization: derivatives as multiplication by
  i*k, products in physical space, the 2/3 rule always on [Sec. 2.4],
* the pressure handled by the projection of Algorithm 1 step (d) [Alg. 1],
* Adams-Bashforth 2 with integrating factor for the viscous term [Sec. 2.4,
  Alg. 1 step (e)], or classical RK4 with explicit diffusion [Sec. 2.4],
* the smoothed mask from a signed distance [Sec. 2.2, eq.
  smoothing_mask_as_function_of_delta],
* the insect model: rotation matrices, body/stroke/wing frames, body and wing
  velocity fields [Sec. 3.1-3.3, eqs. M_body_yawpitchroll,
  body_velocity_field, wing_velocity_field], wing angles as sinusoids,
  Fourier or Hermite series [Sec. 3.3], body shape with head and eyes
  [Sec. 3.2] and the wing shapes: polar radius (closed-form ellipse or
  Fourier series through a 25 000-sample table) or rectangle [Sec. 3.4],
* force and torque from the penalization integral with the unsteady
  correction [Sec. 2.1, eqs. force_with_unst_corrections, moment_of_love],
* the time loop of Algorithm 1 (mask -> dt -> sources -> projection -> AB2
  -> free flight),
* free flight: Newton's law and the quaternion form of Euler's equations
  [Sec. 3.6, eq. oh_my_god_look_a_vector] stepped with the same AB2, and the
  aerodynamic power of a wing [Sec. 3.5, eq. insect_power].

Where the paper is silent or garbled the readings below are used (each is
listed in the design notes of the repository):

  FFT sign/normalization: forward unnormalized with exp(-i k.x), inverse
      scaled by 1/(nx ny nz); arrays are [z][y][x] with x fastest and the
      half spectrum along x.
  Wavenumbers: j = i for i < n/2, j = i - n otherwise (Nyquist = -n/2); the
      derivative of a Nyquist mode is zero.
  Box: n points on y and z (side L), nx on x (side Lx), one spacing
      dx = L/n = Lx/nx on every axis (the paper's non-cubic box, 6x4x4 at
      1152x768x768, has one spacing); k_a = (2 pi/L_a) j_a and the 2/3 rule
      on each axis with its own point count.
  2/3 rule: a mode is kept iff 3|j| < n on every axis; applied to the whole
      right-hand side after the forward transform and to the initial field.
  k = 0: the projection is the identity there; mean mode FIXED sets the k=0
      right-hand side to zero (the mean velocity stays at its initial value),
      FREE keeps it.
  Nonlinear term on the right-hand side: u x w (= -w x u).
  Vorticity sponge: -(1/C_sp) curl (chi_sp w)/Laplacian read as the
      Biot-Savart damping of the vorticity, i.e. -(1/C_sp) (i k x W_hat)/|k|^2
      with W = chi_sp w (the printed sign with the Laplacian -|k|^2 would
      amplify); chi_sp = 1 in layers at the top end of chosen axes, sharp.
  AB2-IF with variable step: AB2 on v = exp(nu|k|^2 t) u_hat with the
      variable-step weights b1 = 1 + r/2, b2 = -r/2, r = dt_n/dt_{n-1};
      the first step is integrating-factor Euler.
  Time step: dt = min(CFL dx / max|u|, eta_cap*C_eta (only with a mask),
      dt_max), clamped to land on t_end; or a fixed dt.
  RK4 (the paper's second integrator, diffusion explicit): the classical
      four stages on R = (projected, dealiased source) - nu|k|^2 u_hat with the
      mask at t, t + dt/2, t + dt/2, t + dt; diagnostics from the first stage;
      the adaptive dt is also kept below 2.5/(nu max|k|^2) (explicit diffusion
      stability; the paper gives no rule).  Free flight stays with AB2.
  Mask: cosine layer with h = c_smth*dx, or 0.5*(1 - tanh(delta/(c_smth*dx)));
      delta < 0 inside the solid.
  Ellipsoid thorax: max(sqrt(y^2+z^2) - b sqrt(max(0, 1-(x/a)^2)), |x| - a).
  Elliptic wing: polar-radius form with the ellipse centred at (0, B) in the
      wing plane, span along +y_w, chord along x_w, thickness along z_w.
  Frames: x_w = M_wing M_stroke (x_b - pivot); the wing angular velocity in
      the wing frame is M_wing M_stroke Omega_w^(b), and the wing velocity in
      the global frame is M_body^T M_stroke^T M_wing^T (Omega^(w) x x_w).
  Parts combine by the maximum of chi; u_s and colour come from the argmax
      part, where a later part wins only if its chi exceeds the best so far
      by more than the relative tie tolerance TIE_REL (ties, including
      values equal up to rounding such as both wings on the mirror plane of a
      symmetric insect, go to the lowest colour).  Colours: 0 fluid, 1 body,
      2 left wing, 3 right wing.
  Force on the solid: F = (1/C_eta) sum chi (u - u_s) dV + (I^n - I^{n-1})/dt_{n-1}
      with I = sum chi u_s dV (no unsteady term at the first step); torques
      about the body centre (body) or the wing pivot (wings).
  Energy: E = 1/2 sum |u|^2 dV.
  Dirichlet walls: layers at the top end of chosen axes (sharp, placed like
      the sponge's) where chi = 1 and u_s = u_wall; they take precedence over a
      body and carry colour 0 (outside the body's force integrals).
  Wing angle series: Fourier coefficients use the convention of eq.
      Fourier_radious_wing with the phase f t (in periods) as the variable;
      Hermite coefficients are values and rates at K equidistant times of
      one period, joined by periodic cubic Hermite interpolation.
  Fourier wing: the series variable is the polar angle in turns (angle/2pi,
      counterclockwise from +x_w about x_c^(w)); the table holds 25 000
      samples at j/25 000 and is interpolated linearly and periodically.
  Rectangular wing: the printed distance repeats the sign of its first chord
      term; read as max(x - b, -x - (B - b), y - tip, a - y, |z| - t/2), a
      chord of length B from -(B - b) to b and a span from a to tip (the
      printed tip is 1, the normalized pivot-to-tip distance).  The printed
      example value a = 1.6667 leaves that span empty; 0.16667 gives the
      aspect ratio 2 of its chord 0.4167.
  Body parts: head and eye spheres get radii (not printed) and join the
      thorax as a union, i.e. the minimum of the signed distances (with
      delta < 0 inside, the printed maximum would be the intersection).
  Quaternion matrix: the printed matrix of the quaternion maps body-frame
      vectors to the global frame; M_body (global to body) is its transpose.
      Only then does the printed initial quaternion reproduce eq.
      M_body_yawpitchroll, and only then does eps' = 1/2 S^T Omega^(b)
      describe the rotation with body angular velocity Omega^(b).
  Free flight: F is the sum of the corrected forces of all parts; m is the
      torque about the centre of gravity x_cntr, m = (1/C_eta) sum
      (x - x_cntr) x chi (u - u_s) dV + (J^n - J^{n-1})/dt_{n-1} with
      J = sum (x - x_cntr) x chi u_s dV, turned into the body frame by
      M_body; gravity acts along -z.  The 6-vector of DoF switches multiplies
      the three translational and the three rotational acceleration rows.
      AB2 with the fluid's weights, Euler on the first free-flight step; the
      quaternion is renormalized to unit length after every step.  The first
      free-flight step starts from the prescribed kinematics at its time.
  Aerodynamic power: P = -m . (Omega_w - Omega_b) with m the wing torque
      about its pivot and Omega_w - Omega_b the wing's angular velocity
      relative to the body (the Omega_w^(b) of Sec. 3.3), in the global
      frame.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, os.cpu_count() or 1)

MEAN_FIXED = 0
MEAN_FREE = 1

COLOUR_FLUID, COLOUR_BODY, COLOUR_WING_L, COLOUR_WING_R = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# Grid, wavenumbers and the 2/3 rule  [Sec. 2.4]
# ---------------------------------------------------------------------------

def signed_index(n: int) -> np.ndarray:
    """Integer wavenumber of FFT bin i on an axis of n points (Nyquist -> -n/2)."""
    i = np.arange(n, dtype=np.int64)
    return np.where(i < n // 2, i, i - n)


def half_index(n: int) -> np.ndarray:
    """Integer wavenumbers 0..n/2 of the half (real-to-complex) axis."""
    return np.arange(n // 2 + 1, dtype=np.int64)


def dealias_keep(j: np.ndarray, n: int) -> np.ndarray:
    """2/3 rule on one axis: keep a mode iff 3|j| < n  [Sec. 2.4]."""
    return 3 * np.abs(j) < n


def dealias_kmax(n: int) -> int:
    """Largest kept |j| under the 2/3 rule."""
    j = np.arange(n)
    return int(j[dealias_keep(j, n)].max())


@dataclass
class Grid:
    """Periodic box with n points per axis on y and z (side L) and nx points on
    x (side Lx; nx = 0 means n, a cubic box), x_i = i*dx with one spacing
    dx = L/n = Lx/nx on every axis (the non-cubic box of Sec. 4 and 6,
    6x4x4 at 1152x768x768)."""
    n: int
    L: float
    nx: int = 0
    Lx: float = 0.0

    def __post_init__(self):
        if self.nx == 0:
            self.nx, self.Lx = self.n, self.L
        if abs(self.Lx / self.nx - self.L / self.n) > 1e-12 * (self.L / self.n):
            raise ValueError("the grid spacing must be the same on every axis")

    @property
    def dx(self) -> float:
        return self.L / self.n

    @property
    def dV(self) -> float:
        return self.dx ** 3

    @property
    def shape(self):
        """Physical array shape [z][y][x]."""
        return (self.n, self.n, self.nx)

    @property
    def lengths(self):
        """Box side per axis (x, y, z)."""
        return (self.Lx, self.L, self.L)

    def coords(self):
        """Physical coordinates as three [z][y][x] arrays."""
        x1 = np.arange(self.nx, dtype=np.float64) * self.dx
        y1 = np.arange(self.n, dtype=np.float64) * self.dx
        z, y, x = np.meshgrid(y1, y1, x1, indexing="ij")
        return x, y, z

    def wavenumbers(self):
        """(jx, jy, jz) integer tables broadcastable over [kz][ky][kx]."""
        n = self.n
        jx = half_index(self.nx)[None, None, :]
        jy = signed_index(n)[None, :, None]
        jz = signed_index(n)[:, None, None]
        return jx, jy, jz

    def k_vectors(self, derivative: bool):
        """Wavevector components (2 pi / L_a) j_a.  For derivatives the Nyquist
        wavenumber is zeroed (a Nyquist mode has no defined derivative)."""
        n = self.n
        cx = 2.0 * math.pi / self.Lx
        c = 2.0 * math.pi / self.L
        jx, jy, jz = self.wavenumbers()
        kx, ky, kz = (cx * jx.astype(np.float64), c * jy.astype(np.float64),
                      c * jz.astype(np.float64))
        if derivative:
            kx = np.where(jx == self.nx // 2, 0.0, kx)
            ky = np.where(np.abs(jy) == n // 2, 0.0, ky)
            kz = np.where(np.abs(jz) == n // 2, 0.0, kz)
        return kx, ky, kz

    def k2(self):
        kx, ky, kz = self.k_vectors(derivative=False)
        return kx * kx + ky * ky + kz * kz

    def dealias(self):
        """Boolean mask over the half spectrum: True where the 2/3 rule keeps the mode."""
        n = self.n
        jx, jy, jz = self.wavenumbers()
        return dealias_keep(jx, self.nx) & dealias_keep(jy, n) & dealias_keep(jz, n)


# ---------------------------------------------------------------------------
# 3D real transforms  [Sec. 2.4]
# ---------------------------------------------------------------------------

def r2c(f: np.ndarray) -> np.ndarray:
    """Forward real-to-complex 3D transform of [..., z, y, x] arrays, unnormalized."""
    return sfft.rfftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def c2r(fh: np.ndarray, n) -> np.ndarray:
    """Inverse complex-to-real 3D transform, scaled by 1/(points); n is the
    points per axis of a cubic grid or the physical shape (nz, ny, nx)."""
    s = (n, n, n) if isinstance(n, (int, np.integer)) else tuple(n)
    return sfft.irfftn(fh, s=s, axes=(-3, -2, -1), workers=_WORKERS)


# ---------------------------------------------------------------------------
# Spectral operators  [Sec. 2.4, Alg. 1 step (d)]
# ---------------------------------------------------------------------------

def curl_hat(g: Grid, uh: np.ndarray) -> np.ndarray:
    """Vorticity coefficients w_hat = i k x u_hat."""
    kx, ky, kz = g.k_vectors(derivative=True)
    ux, uy, uz = uh
    return np.stack([1j * (ky * uz - kz * uy),
                     1j * (kz * ux - kx * uz),
                     1j * (kx * uy - ky * ux)])


def divergence_hat(g: Grid, uh: np.ndarray) -> np.ndarray:
    kx, ky, kz = g.k_vectors(derivative=True)
    return 1j * (kx * uh[0] + ky * uh[1] + kz * uh[2])


def project(g: Grid, fh: np.ndarray) -> np.ndarray:
    """Leray projection F - k (k.F)/|k|^2 of Alg. 1 step (d); identity at k = 0.

    Step (d) subtracts the gradient of the solution of a Poisson problem whose
    right-hand side is the divergence of F; in Fourier space that is the
    subtraction of the component of F_hat along k."""
    kx, ky, kz = g.k_vectors(derivative=True)
    k2 = kx * kx + ky * ky + kz * kz
    kdotf = kx * fh[0] + ky * fh[1] + kz * fh[2]
    with np.errstate(invalid="ignore", divide="ignore"):
        s = np.where(k2 > 0.0, kdotf / np.where(k2 > 0.0, k2, 1.0), 0.0)
    return np.stack([fh[0] - kx * s, fh[1] - ky * s, fh[2] - kz * s])


def import_field(g: Grid, u0: np.ndarray) -> np.ndarray:
    """Initial coefficients: 2/3 rule and projection of the sampled field [Eq. PNST_inicond]."""
    uh = r2c(u0) * g.dealias()
    return project(g, uh)


# ---------------------------------------------------------------------------
# Rotation matrices and insect kinematics  [Sec. 3]
# ---------------------------------------------------------------------------

def Rx(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, s], [0.0, -s, c]])


def Ry(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0.0, -s], [0.0, 1.0, 0.0], [s, 0.0, c]])


def Rz(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])


@dataclass
class Insect:
    """Rigid tethered insect (or a single body) with sinusoidal wing angles.

    Angles in radians.  Each wing angle is mean + amp*cos(2 pi freq t + phase).
    body: 'none' | 'sphere' | 'ellipsoid'.  smooth: 'cos' | 'tanh'."""
    body: str = "none"
    x_cntr: tuple = (0.0, 0.0, 0.0)
    u_cntr: tuple = (0.0, 0.0, 0.0)
    psi: float = 0.0
    beta: float = 0.0
    gamma: float = 0.0
    psi_dot: float = 0.0
    beta_dot: float = 0.0
    gamma_dot: float = 0.0
    radius: float = 0.5
    a: float = 0.5
    b: float = 0.1
    smooth: str = "cos"
    c_smth: float = 1.0
    wings: bool = False
    eta_stroke: float = 0.0
    pivot_l: tuple = (0.0, 0.15, 0.0)
    pivot_r: tuple = (0.0, -0.15, 0.0)
    wing_A: float = 0.175
    wing_B: float = 0.5
    wing_t: float = 0.0
    freq: float = 1.0
    phi: tuple = (0.0, 0.0, 0.0)
    alpha: tuple = (0.0, 0.0, 0.0)
    theta: tuple = (0.0, 0.0, 0.0)
    kin: str = "sine"                    # wing angles: 'sine' | 'fourier' | 'hermite'  [Sec. 3.3]
    kin_phi: tuple = ((), ())            # fourier: (a_0..a_n), (b_0..b_n); hermite: (values), (rates)
    kin_alpha: tuple = ((), ())
    kin_theta: tuple = ((), ())
    wing_shape: str = "ellipse"          # 'ellipse' | 'fourier' | 'rectangle'  [Sec. 3.4]
    rect_a: float = 0.0                  # rectangle: span from rect_a ...
    rect_tip: float = 1.0                # ... to rect_tip along y_w
    rect_b: float = 0.0                  # rectangle: leading edge at x_w = rect_b ...
    rect_B: float = 0.0                  # ... chord rect_B (trailing edge at -(B - b))
    wing_c: tuple = (0.0, 0.0)           # fourier wing: centre x_c^(w) in the wing plane
    wing_fa: tuple = ()                  # fourier wing: a_0..a_n
    wing_fb: tuple = ()                  # fourier wing: b_0..b_n (b_0 unused)
    head_x: tuple = (0.0, 0.0, 0.0)      # head sphere centre (body frame); head_r <= 0: none
    head_r: float = 0.0
    eye_x: tuple = (0.0, 0.0, 0.0)       # eye spheres at (x, +y, z) and (x, -y, z); eye_r <= 0: none
    eye_r: float = 0.0
    free_flight: bool = False            # Sec. 3.6: the body moves under F, m and gravity
    mass: float = 1.0                    # M
    inertia: tuple = (1.0, 1.0, 1.0)     # principal moments J_x, J_y, J_z (body frame)
    gravity: float = 0.0                 # g, acting along -z
    dof: tuple = (1.0, 1.0, 1.0, 1.0, 1.0, 1.0)  # translation x,y,z; rotation x,y,z
    wing_J: tuple = (0.0,) * 6           # wing inertia (wing frame, about the pivot): Jxx, Jyy, Jzz, Jxy, Jxz, Jyz

    @staticmethod
    def from_dict(d: dict) -> "Insect":
        return Insect(**d)


def fourier_angle(a, b, freq: float, t: float):
    """Angle a_0/2 + sum_i a_i cos(2 pi i f t) + b_i sin(2 pi i f t) and its
    time derivative: the series of eq. Fourier_radious_wing with the phase
    f t (in periods) as its variable  [Sec. 3.3, 3.4]."""
    v = 0.5 * float(a[0])
    dv = 0.0
    for i in range(1, len(a)):
        w = 2.0 * math.pi * i * freq
        ai, bi = float(a[i]), float(b[i])
        v += ai * math.cos(w * t) + bi * math.sin(w * t)
        dv += w * (-ai * math.sin(w * t) + bi * math.cos(w * t))
    return v, dv


def hermite_angle(vals, rates, freq: float, t: float):
    """Angle and its time derivative from periodic cubic Hermite interpolation
    of K values and rates at the equidistant times j/(K f), j = 0..K-1, of one
    period  [Sec. 3.3]."""
    K = len(vals)
    T = 1.0 / freq
    h = T / K
    s = (t % T) / h
    j = min(int(math.floor(s)), K - 1)
    u = s - j
    j1 = (j + 1) % K
    v0, v1 = float(vals[j]), float(vals[j1])
    m0, m1 = float(rates[j]) * h, float(rates[j1]) * h
    h00, h10, h01, h11 = 2 * u ** 3 - 3 * u ** 2 + 1, u ** 3 - 2 * u ** 2 + u, -2 * u ** 3 + 3 * u ** 2, u ** 3 - u ** 2
    d00, d10, d01, d11 = 6 * u ** 2 - 6 * u, 3 * u ** 2 - 4 * u + 1, -6 * u ** 2 + 6 * u, 3 * u ** 2 - 2 * u
    return h00 * v0 + h10 * m0 + h01 * v1 + h11 * m1, (d00 * v0 + d10 * m0 + d01 * v1 + d11 * m1) / h


def wing_angles(ins: Insect, t: float):
    """(phi, alpha, theta) and their time derivatives at time t."""
    if ins.kin == "fourier":
        out = [fourier_angle(c[0], c[1], ins.freq, t) for c in (ins.kin_phi, ins.kin_alpha, ins.kin_theta)]
    elif ins.kin == "hermite":
        out = [hermite_angle(c[0], c[1], ins.freq, t) for c in (ins.kin_phi, ins.kin_alpha, ins.kin_theta)]
    else:
        w = 2.0 * math.pi * ins.freq
        out = []
        for mean, amp, ph in (ins.phi, ins.alpha, ins.theta):
            out.append((mean + amp * math.cos(w * t + ph), -amp * w * math.sin(w * t + ph)))
    (phi, dphi), (alpha, dalpha), (theta, dtheta) = out
    return phi, alpha, theta, dphi, dalpha, dtheta


def body_angles(ins: Insect, t: float):
    """Body roll/pitch/yaw at t (constant rates from the initial angles)."""
    return (ins.psi + ins.psi_dot * t, ins.beta + ins.beta_dot * t,
            ins.gamma + ins.gamma_dot * t)


def M_body(ins: Insect, t: float) -> np.ndarray:
    """x_b = M_body (x_g - x_cntr), M_body = Rx(psi) Ry(beta) Rz(gamma)  [eq. M_body_yawpitchroll]."""
    psi, beta, gamma = body_angles(ins, t)
    return Rx(psi) @ Ry(beta) @ Rz(gamma)


def omega_body_b(ins: Insect, t: float) -> np.ndarray:
    """Body angular velocity in the body frame  [Sec. 3.1]."""
    psi, beta, gamma = body_angles(ins, t)
    og = Rz(gamma).T @ (np.array([0.0, 0.0, ins.gamma_dot])
                        + Ry(beta).T @ (np.array([0.0, ins.beta_dot, 0.0])
                                        + Rx(psi).T @ np.array([ins.psi_dot, 0.0, 0.0])))
    return M_body(ins, t) @ og


def M_stroke(ins: Insect, side: str) -> np.ndarray:
    """Stroke-plane matrices: left Ry(eta), right Rx(pi) Ry(eta)  [Sec. 3.3]."""
    if side == "l":
        return Ry(ins.eta_stroke)
    return Rx(math.pi) @ Ry(ins.eta_stroke)


def M_wing(ins: Insect, t: float, side: str) -> np.ndarray:
    """Wing matrices: left Ry(a) Rz(-th) Rx(phi); right Ry(-a) Rz(-th) Rx(-phi)  [Sec. 3.3]."""
    phi, alpha, theta, *_ = wing_angles(ins, t)
    if side == "l":
        return Ry(alpha) @ Rz(-theta) @ Rx(phi)
    return Ry(-alpha) @ Rz(-theta) @ Rx(-phi)


def omega_wing_s(ins: Insect, t: float, side: str) -> np.ndarray:
    """Wing angular velocity in the stroke-plane frame  [Sec. 3.3].

    Right wing: the same expression with (alpha, phi) and their rates negated,
    matching its wing matrix."""
    phi, alpha, theta, dphi, dalpha, dtheta = wing_angles(ins, t)
    if side == "r":
        phi, alpha, dphi, dalpha = -phi, -alpha, -dphi, -dalpha
    # Omega^(s) = Rx^T(phi)[ (dphi,0,0) + Rz^T(-theta)[ (0,0,-dtheta) + Ry^T(alpha)(0,dalpha,0) ] ]
    return Rx(phi).T @ (np.array([dphi, 0.0, 0.0])
                        + Rz(-theta).T @ (np.array([0.0, 0.0, -dtheta])
                                          + Ry(alpha).T @ np.array([0.0, dalpha, 0.0])))


def omega_wing_b(ins: Insect, t: float, side: str) -> np.ndarray:
    """Wing angular velocity in the body frame  [Sec. 3.3]."""
    return M_stroke(ins, side).T @ omega_wing_s(ins, t, side)


def omega_wing_w(ins: Insect, t: float, side: str) -> np.ndarray:
    """Wing angular velocity Omega_w^(w) in the wing's own frame: the stroke-frame
    vector mapped by the wing matrix  [Sec. 3.3, 3.5]."""
    return M_wing(ins, t, side) @ omega_wing_s(ins, t, side)


def wing_inertia(ins: Insect) -> np.ndarray:
    """Symmetric wing tensor of inertia J^(w) from (Jxx, Jyy, Jzz, Jxy, Jxz, Jyz)."""
    jxx, jyy, jzz, jxy, jxz, jyz = (float(v) for v in ins.wing_J)
    return np.array([[jxx, jxy, jxz], [jxy, jyy, jyz], [jxz, jyz, jzz]])


def inertial_power(ins: Insect, t: float, side: str) -> float:
    """P_inert = Omega^(w) . (J^(w) dOmega^(w)/dt + Omega^(w) x J^(w) Omega^(w)) of one
    wing  [Sec. 3.5].  The paper does not say how the angular acceleration is
    obtained; here it is the fourth-order central difference of Omega^(w)(t)
    with a step of 1e-4 of a period (truncation below 1e-8 relative for the
    harmonics the angle series allow)."""
    J = wing_inertia(ins)
    if not J.any():
        return 0.0
    h = 1e-4 / ins.freq if ins.freq > 0.0 else 1e-4
    om = omega_wing_w(ins, t, side)
    dom = (omega_wing_w(ins, t - 2 * h, side) - 8.0 * omega_wing_w(ins, t - h, side)
           + 8.0 * omega_wing_w(ins, t + h, side) - omega_wing_w(ins, t + 2 * h, side)) / (12.0 * h)
    return float(np.dot(om, J @ dom + np.cross(om, J @ om)))


# ---------------------------------------------------------------------------
# Mask from signed distances  [Sec. 2.2, 3.2, 3.4]
# ---------------------------------------------------------------------------

def chi_of_delta(delta: np.ndarray, ins: Insect, dx: float) -> np.ndarray:
    h = ins.c_smth * dx
    if ins.smooth == "tanh":
        return 0.5 * (1.0 - np.tanh(delta / h))
    # eq. smoothing_mask_as_function_of_delta
    out = np.where(delta <= -h, 1.0, 0.0)
    mid = (delta > -h) & (delta < h)
    return np.where(mid, 0.5 * (1.0 + np.cos(math.pi * (delta + h) / (2.0 * h))), out)


def delta_ellipsoid(xb, yb, zb, a, b):
    """Thorax ellipsoid, continued for |x| > a so that it is defined everywhere."""
    rad = np.sqrt(yb * yb + zb * zb)
    prof = b * np.sqrt(np.maximum(0.0, 1.0 - (xb / a) ** 2))
    return np.maximum(rad - prof, np.abs(xb) - a)


def delta_elliptic_wing(xw, yw, zw, A, B, t):
    """Polar-radius wing [Sec. 3.4] with the closed-form radius of an ellipse
    with semi-axes A (chord, x_w) and B (span, y_w) centred at (0, B)."""
    ex = xw
    ey = yw - B
    r = np.sqrt(ex * ex + ey * ey)
    rho = np.sqrt((ex / A) ** 2 + (ey / B) ** 2)
    with np.errstate(invalid="ignore", divide="ignore"):
        inplane = np.where(r > 0.0, r - r / np.where(rho > 0.0, rho, 1.0), -A)
    return np.maximum(np.abs(zw) - 0.5 * t, inplane)


# Samples of the wing radius table  [Sec. 3.4]
R_TABLE_SIZE = 25000


def wing_radius_series(fa, fb, v):
    """R(v) = a_0/2 + sum_i a_i cos(2 pi i v) + b_i sin(2 pi i v)  [eq. Fourier_radious_wing];
    v is the polar angle in turns (angle / 2 pi)."""
    v = np.asarray(v, dtype=np.float64)
    r = np.full(v.shape, 0.5 * float(fa[0]))
    for i in range(1, len(fa)):
        r = r + float(fa[i]) * np.cos(2.0 * np.pi * i * v) + float(fb[i]) * np.sin(2.0 * np.pi * i * v)
    return r


def wing_radius_table(fa, fb) -> np.ndarray:
    """R at the R_TABLE_SIZE angles v_j = j / R_TABLE_SIZE (evaluated once)  [Sec. 3.4]."""
    return wing_radius_series(fa, fb, np.arange(R_TABLE_SIZE) / R_TABLE_SIZE)


def wing_radius_lookup(table: np.ndarray, v):
    """Linear interpolation in the periodic radius table  [Sec. 3.4]."""
    n = table.shape[0]
    p = np.mod(np.asarray(v, dtype=np.float64), 1.0) * n
    j = np.minimum(np.floor(p).astype(np.int64), n - 1)
    f = p - j
    return (1.0 - f) * table[j] + f * table[(j + 1) % n]


def delta_fourier_wing(xw, yw, zw, ins: Insect, table: np.ndarray):
    """Polar-radius wing  [Sec. 3.4]: max(|z_w| - t/2, r - R(v)) with r and the
    angle v (in turns, counterclockwise from +x_w) about the centre x_c^(w)."""
    ex = xw - float(ins.wing_c[0])
    ey = yw - float(ins.wing_c[1])
    r = np.sqrt(ex * ex + ey * ey)
    v = np.arctan2(ey, ex) / (2.0 * np.pi)
    return np.maximum(np.abs(zw) - 0.5 * ins.wing_t, r - wing_radius_lookup(table, v))


def delta_rect_wing(xw, yw, zw, ins: Insect):
    """Rectangular wing  [Sec. 3.4, eq. signed_distance_rectangular_wing]:
    the intersection of the half-spaces x_w <= b, x_w >= -(B - b), y_w <= tip,
    y_w >= a and |z_w| <= t/2, i.e. the maximum of their signed distances."""
    return np.maximum.reduce([xw - ins.rect_b, -xw - (ins.rect_B - ins.rect_b), yw - ins.rect_tip,
                              ins.rect_a - yw, np.abs(zw) - 0.5 * ins.wing_t])


def delta_body(ins: Insect, xb):
    """Body signed distance in the body frame  [Sec. 3.2]: the thorax
    ellipsoid joined with the head and eye spheres (union: min of the
    distances; a sphere's distance is |x - x_0| - radius)."""
    d = delta_ellipsoid(xb[0], xb[1], xb[2], ins.a, ins.b)
    sph = []
    if ins.head_r > 0.0:
        sph.append((ins.head_x, ins.head_r))
    if ins.eye_r > 0.0:
        ex, ey, ez = ins.eye_x
        sph += [((ex, ey, ez), ins.eye_r), ((ex, -ey, ez), ins.eye_r)]
    for c, rad in sph:
        ds = np.sqrt((xb[0] - c[0]) ** 2 + (xb[1] - c[1]) ** 2 + (xb[2] - c[2]) ** 2) - rad
        d = np.minimum(d, ds)
    return d


def _cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def _apply(M, v):
    """M @ v for a 3x3 matrix and a [3][...] array of vectors."""
    return np.einsum("ij,j...->i...", M, v)


@dataclass
class Pose:
    """Position, velocity, orientation and angular velocity of the body."""
    xc: np.ndarray    # centre (global frame)
    uc: np.ndarray    # centre velocity (global frame)
    Mb: np.ndarray    # M_body: x_b = Mb (x_g - xc)
    omb: np.ndarray   # body angular velocity, body frame


def prescribed_pose(ins: Insect, t: float) -> Pose:
    """Tethered body: the given centre and velocity, M_body and Omega_b^(b)
    from the body angles at t  [Sec. 3.1]."""
    return Pose(np.asarray(ins.x_cntr, dtype=np.float64), np.asarray(ins.u_cntr, dtype=np.float64),
                M_body(ins, t), omega_body_b(ins, t))


def _pose(ins: Insect, t: float, pose: Pose | None) -> Pose:
    return prescribed_pose(ins, t) if pose is None else pose


def body_velocity(ins: Insect, t: float, xb, pose: Pose | None = None):
    """u_b = u_cntr + M_body^T (Omega_b^(b) x x_b)  [eq. body_velocity_field]."""
    ps = _pose(ins, t, pose)
    om = ps.omb.reshape((3,) + (1,) * (np.ndim(xb) - 1))
    ub = _apply(ps.Mb.T, _cross(np.broadcast_to(om, np.shape(xb)), xb))
    return ub + ps.uc.reshape((3,) + (1,) * (np.ndim(xb) - 1))


def wing_frame(ins: Insect, t: float, side: str, xb):
    """x_w = M_wing M_stroke (x_b - pivot)  [Sec. 3.3]."""
    piv = np.asarray(ins.pivot_l if side == "l" else ins.pivot_r, dtype=np.float64)
    xrel = xb - piv.reshape((3,) + (1,) * (np.ndim(xb) - 1))
    return _apply(M_wing(ins, t, side) @ M_stroke(ins, side), xrel)


def wing_velocity(ins: Insect, t: float, side: str, xb, pose: Pose | None = None):
    """Solid velocity inside a wing, u_w + u_b  [eq. wing_velocity_field]:
    u_w^(w) = Omega_w^(w) x x_w with Omega_w^(w) = M_wing M_stroke Omega_w^(b),
    u_w^(g) = M_body^T M_stroke^T M_wing^T u_w^(w)."""
    Ms = M_stroke(ins, side)
    Mw = M_wing(ins, t, side)
    xw = wing_frame(ins, t, side, xb)
    om_w = (Mw @ Ms @ omega_wing_b(ins, t, side)).reshape((3,) + (1,) * (np.ndim(xb) - 1))
    uw_w = _cross(np.broadcast_to(om_w, np.shape(xw)), xw)
    ps = _pose(ins, t, pose)
    back = ps.Mb.T @ Ms.T @ Mw.T
    return _apply(back, uw_w) + body_velocity(ins, t, xb, ps)


def to_body(ins: Insect, t: float, xg, pose: Pose | None = None):
    """x_b = M_body (x_g - x_cntr)  [eq. M_body_yawpitchroll]."""
    ps = _pose(ins, t, pose)
    return _apply(ps.Mb, xg - ps.xc.reshape((3,) + (1,) * (np.ndim(xg) - 1)))


# Relative tolerance under which two part values count as a tie.
TIE_REL = 1e-9


def part_of_max(stack: np.ndarray) -> np.ndarray:
    """Index of the part that supplies u_s and the colour at each point.

    Parts are taken in colour order; a later part replaces the current one only
    if its chi is larger by more than TIE_REL relative, so ties (up to rounding)
    resolve to the lowest colour."""
    part = np.zeros(stack.shape[1:], dtype=np.int64)
    best = stack[0].copy()
    for p in range(1, stack.shape[0]):
        take = stack[p] > best * (1.0 + TIE_REL)
        part[take] = p
        best = np.where(take, stack[p], best)
    return part


def mask_at(ins: Insect, t: float, dx: float, x, y, z, pose: Pose | None = None):
    """chi, u_s [3] and colour at points with global coordinates x, y, z (arrays
    of one shape), smoothing width set by the grid spacing dx  [Alg. 1 step (a)].
    pose: the body's pose (default: the prescribed kinematics at t)."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    shp = x.shape
    ps = _pose(ins, t, pose)
    xg = np.stack([x, y, z])
    xb = to_body(ins, t, xg, ps)
    ub = body_velocity(ins, t, xb, ps)

    chis, uss = [], []
    if ins.body == "sphere":
        xc = ps.xc
        d = np.sqrt((x - xc[0]) ** 2 + (y - xc[1]) ** 2 + (z - xc[2]) ** 2) - ins.radius
        chis.append(chi_of_delta(d, ins, dx))
        uss.append(ub)
    elif ins.body == "ellipsoid":
        d = delta_body(ins, xb)
        chis.append(chi_of_delta(d, ins, dx))
        uss.append(ub)
    else:
        chis.append(np.zeros(shp))
        uss.append(np.zeros((3,) + shp))

    if ins.wings:
        table = wing_radius_table(ins.wing_fa, ins.wing_fb) if ins.wing_shape == "fourier" else None
        for side in ("l", "r"):
            xw = wing_frame(ins, t, side, xb)
            if table is not None:
                d = delta_fourier_wing(xw[0], xw[1], xw[2], ins, table)
            elif ins.wing_shape == "rectangle":
                d = delta_rect_wing(xw[0], xw[1], xw[2], ins)
            else:
                d = delta_elliptic_wing(xw[0], xw[1], xw[2], ins.wing_A, ins.wing_B, ins.wing_t)
            chis.append(chi_of_delta(d, ins, dx))
            uss.append(wing_velocity(ins, t, side, xb, ps))
    else:
        chis += [np.zeros(shp)] * 2
        uss += [np.zeros((3,) + shp)] * 2

    stack = np.stack(chis)
    part = part_of_max(stack)
    chi = np.max(stack, axis=0)
    us = np.zeros((3,) + shp)
    for p in range(3):
        sel = part == p
        us[:, sel] = uss[p][:, sel]
    colour = np.where(chi > 0.0, part + 1, 0).astype(np.int16)
    us = us * (chi > 0.0)
    return chi, us, colour


def insect_mask(g: Grid, ins: Insect, t: float, pose: Pose | None = None):
    """chi, u_s [3] and colour on every grid point at time t  [Alg. 1 step (a)]."""
    x, y, z = g.coords()
    return mask_at(ins, t, g.dx, x, y, z, pose)


def reference_points(ins: Insect, t: float, pose: Pose | None = None) -> np.ndarray:
    """Torque reference points (global frame) per colour 1..3: body centre, pivots."""
    ps = _pose(ins, t, pose)
    return np.stack([ps.xc, ps.xc + ps.Mb.T @ np.asarray(ins.pivot_l, dtype=np.float64),
                     ps.xc + ps.Mb.T @ np.asarray(ins.pivot_r, dtype=np.float64)])


# ---------------------------------------------------------------------------
# Free flight  [Sec. 3.6, eq. oh_my_god_look_a_vector]
#
# Solid state y (13 values): x_cntr (3), u_cntr (3), quaternion eps (4),
# Omega^(b) (3).
# ---------------------------------------------------------------------------

def quaternion_from_angles(psi: float, beta: float, gamma: float) -> np.ndarray:
    """Quaternion of the orientation with roll psi, pitch beta, yaw gamma  [Sec. 3.6]."""
    cp, sp = math.cos(psi / 2), math.sin(psi / 2)
    cb, sb = math.cos(beta / 2), math.sin(beta / 2)
    cg, sg = math.cos(gamma / 2), math.sin(gamma / 2)
    return np.array([cp * cb * cg + sp * sb * sg,
                     sp * cb * cg - cp * sb * sg,
                     cp * sb * cg + sp * cb * sg,
                     cp * cb * sg - sp * sb * cg])


def quaternion_matrix(eps) -> np.ndarray:
    """The rotation matrix of a unit quaternion as the paper prints it  [Sec. 3.6];
    it maps body-frame vectors to the global frame."""
    e0, e1, e2, e3 = (float(v) for v in eps)
    return np.array([
        [e0 * e0 + e1 * e1 - e2 * e2 - e3 * e3, 2 * (e1 * e2 - e3 * e0), 2 * (e1 * e3 + e2 * e0)],
        [2 * (e1 * e2 + e3 * e0), e0 * e0 - e1 * e1 + e2 * e2 - e3 * e3, 2 * (e2 * e3 - e1 * e0)],
        [2 * (e1 * e3 - e2 * e0), 2 * (e2 * e3 + e1 * e0), e0 * e0 - e1 * e1 - e2 * e2 + e3 * e3]])


def M_body_of_quaternion(eps) -> np.ndarray:
    """M_body (global to body) of the free-flight case: the transpose of the
    printed quaternion matrix (so that it agrees with eq. M_body_yawpitchroll
    for the initial quaternion of the same angles)."""
    return quaternion_matrix(eps).T


def solid_pose(y) -> Pose:
    """Pose of the body from the free-flight state."""
    y = np.asarray(y, dtype=np.float64)
    return Pose(y[0:3].copy(), y[3:6].copy(), M_body_of_quaternion(y[6:10]), y[10:13].copy())


def solid_init(ins: Insect, t: float) -> np.ndarray:
    """Free-flight state equal to the prescribed kinematics at time t."""
    psi, beta, gamma = body_angles(ins, t)
    return np.concatenate([np.asarray(ins.x_cntr, dtype=np.float64), np.asarray(ins.u_cntr, dtype=np.float64),
                           quaternion_from_angles(psi, beta, gamma), omega_body_b(ins, t)])


def pose_record(ins: Insect, t: float, y=None) -> np.ndarray:
    """The 13 state values of the body at t: the free-flight state y, or the
    prescribed kinematics (quaternion from the body angles) when y is None."""
    return np.asarray(y, dtype=np.float64).copy() if y is not None else solid_init(ins, t)


def solid_rhs(ins: Insect, y, F, m_g) -> np.ndarray:
    """Right-hand side of the 13 free-flight equations  [eq. oh_my_god_look_a_vector].

    F: aerodynamic force (global frame); m_g: torque about x_cntr (global
    frame), turned into the body frame with M_body; gravity g along -z; the
    DoF switches multiply the translational and rotational acceleration rows."""
    y = np.asarray(y, dtype=np.float64)
    uc, eps, om = y[3:6], y[6:10], y[10:13]
    e0, e1, e2, e3 = eps
    ox, oy, oz = om
    Jx, Jy, Jz = ins.inertia
    mb = M_body_of_quaternion(eps) @ np.asarray(m_g, dtype=np.float64)
    dof = np.asarray(ins.dof, dtype=np.float64)
    f = np.empty(13)
    f[0:3] = uc
    f[3:6] = np.asarray(F, dtype=np.float64) / ins.mass
    f[5] -= ins.gravity
    f[3:6] *= dof[0:3]
    f[6] = 0.5 * (-e1 * ox - e2 * oy - e3 * oz)
    f[7] = 0.5 * (e0 * ox - e3 * oy + e2 * oz)
    f[8] = 0.5 * (e3 * ox + e0 * oy - e1 * oz)
    f[9] = 0.5 * (-e2 * ox + e1 * oy + e0 * oz)
    f[10] = ((Jy - Jz) * oy * oz + mb[0]) / Jx
    f[11] = ((Jz - Jx) * oz * ox + mb[1]) / Jy
    f[12] = ((Jx - Jy) * ox * oy + mb[2]) / Jz
    f[10:13] *= dof[3:6]
    return f


def solid_step(ins: Insect, y, f_prev, F, m_g, dt: float, dt_prev: float):
    """AB2 step of the free-flight state  [Alg. 1 step (f)]: Euler when f_prev
    is None, else the variable-step weights of the fluid; the quaternion is
    renormalized.  Returns (y_new, f) with f the right-hand side at y."""
    f = solid_rhs(ins, y, F, m_g)
    if f_prev is None:
        yn = np.asarray(y, dtype=np.float64) + dt * f
    else:
        r = dt / dt_prev
        yn = np.asarray(y, dtype=np.float64) + dt * ((1.0 + 0.5 * r) * f - 0.5 * r * np.asarray(f_prev))
    yn[6:10] /= math.sqrt(float(np.sum(yn[6:10] ** 2)))
    return yn, f


def aero_power(m_wing_g, Mb, om_w_b) -> float:
    """P_aero = -m . (Omega_w - Omega_b) of one wing  [Sec. 3.5, eq. insect_power],
    with the wing's angular velocity relative to the body given in the body
    frame and the torque about the pivot in the global frame."""
    return -float(np.dot(np.asarray(m_wing_g), Mb.T @ np.asarray(om_w_b)))


# ---------------------------------------------------------------------------
# Right-hand side, time step and diagnostics  [Alg. 1 steps (b)-(e)]
# ---------------------------------------------------------------------------

@dataclass
class Params:
    n: int
    L: float
    nu: float
    eta: float
    mean_mode: int = MEAN_FIXED
    nx: int = 0                            # points on x (0: n, a cubic box)
    Lx: float = 0.0                        # box side on x (with nx; same spacing as y and z)
    c_sp: float = 0.0                      # vorticity sponge constant C_sp (0: no sponge)
    sponge: tuple = (0.0, 0.0, 0.0)        # sponge layer thickness per axis (0: none on that axis)
    integrator: str = "ab2"                # 'ab2' (integrating-factor AB2) | 'rk4' (explicit diffusion)
    wall: tuple = (0.0, 0.0, 0.0)          # Dirichlet layer thickness per axis (0: none on that axis)
    u_wall: tuple = (0.0, 0.0, 0.0)        # velocity imposed in the layers


def grid_of(p: Params) -> Grid:
    return Grid(p.n, p.L, p.nx, p.Lx)


def sponge_mask(g: Grid, thickness) -> np.ndarray:
    """chi_sp on the grid: 1 where, for an axis a with thickness d_a > 0, the
    coordinate x_a lies in the top layer [L - d_a, L) of the periodic box
    (upstream of the seam), 0 elsewhere  [Sec. 2.3, wake removal]."""
    x, y, z = g.coords()
    chi = np.zeros_like(x)
    for c, d, La in zip((x, y, z), thickness, g.lengths):
        if d > 0.0:
            chi = np.where(c >= La - d, 1.0, chi)
    return chi


def walls_on(p: Params) -> bool:
    return any(d > 0.0 for d in p.wall)


def apply_walls(p: Params, g: Grid, chi, us, colour):
    """Dirichlet layers  [Sec. 2.3]: the velocity u_wall is imposed by the
    volume penalization in layers at the top end of the axes with thickness
    > 0 (placed like the sponge's).  There chi = 1 and u_s = u_wall; the layers
    take precedence over a body, and their points carry colour 0, so they do
    not enter the body's force integrals."""
    if not walls_on(p):
        return chi, us, colour
    wm = sponge_mask(g, p.wall) > 0.0
    shp = wm.shape
    chi = np.zeros(shp) if chi is None else chi
    us = np.zeros((3,) + shp) if us is None else us
    colour = np.zeros(shp, dtype=np.int16) if colour is None else colour
    uw = np.asarray(p.u_wall, dtype=np.float64).reshape(3, 1, 1, 1)
    return (np.where(wm, 1.0, chi), np.where(wm[None], np.broadcast_to(uw, us.shape), us),
            np.where(wm, 0, colour).astype(np.int16))


def sponge_hat(g: Grid, w: np.ndarray, chi_sp: np.ndarray, c_sp: float) -> np.ndarray:
    """Vorticity sponge term in Fourier space  [Sec. 2.1 eq. PNST_org_momentum,
    Sec. 2.3]: -(1/C_sp) (i k x W_hat)/|k|^2 with W = chi_sp * w, zero at k = 0.

    The Biot-Savart form of damping the vorticity by chi_sp/C_sp: with
    chi_sp = 1 it equals -u_hat/C_sp for a divergence-free u, i.e. damping at
    the rate 1/C_sp; it is divergence-free and leaves the mean flow alone."""
    wh = r2c(chi_sp * w)
    kx, ky, kz = g.k_vectors(derivative=True)
    k2 = kx * kx + ky * ky + kz * kz
    with np.errstate(invalid="ignore", divide="ignore"):
        f = np.where(k2 > 0.0, -1.0 / (c_sp * np.where(k2 > 0.0, k2, 1.0)), 0.0)
    return np.stack([1j * (ky * wh[2] - kz * wh[1]) * f,
                     1j * (kz * wh[0] - kx * wh[2]) * f,
                     1j * (kx * wh[1] - ky * wh[0]) * f])


def physical_fields(g: Grid, uh: np.ndarray):
    """u and w = curl u on the grid."""
    return c2r(uh, g.shape), c2r(curl_hat(g, uh), g.shape)


def source_physical(u, w, chi, us, eta):
    """N = u x w - (chi/C_eta)(u - u_s)  [Alg. 1 step (c), sign per -w x u]."""
    cross = np.stack([u[1] * w[2] - u[2] * w[1],
                      u[2] * w[0] - u[0] * w[2],
                      u[0] * w[1] - u[1] * w[0]])
    return cross - (chi / eta) * (u - us)


def rhs_hat(p: Params, g: Grid, uh, chi, us):
    """Dealiased, projected right-hand side N_hat and the physical velocity."""
    u, w = physical_fields(g, uh)
    if chi is None:
        nphys = source_physical(u, w, 0.0, 0.0, p.eta)
    else:
        nphys = source_physical(u, w, chi, us, p.eta)
    nh = r2c(nphys)
    if p.c_sp > 0.0 and any(d > 0.0 for d in p.sponge):
        nh = nh + sponge_hat(g, w, sponge_mask(g, p.sponge), p.c_sp)
    nh = nh * g.dealias()
    nh = project(g, nh)
    if p.mean_mode == MEAN_FIXED:
        nh[:, 0, 0, 0] = 0.0
    return nh, u


def umax_of(u) -> float:
    m = np.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    return float(np.max(m))


@dataclass
class StepControl:
    dt_fixed: float = 0.0
    cfl: float = 0.1
    dt_max: float = math.inf
    t_end: float = math.inf
    eta_cap: float = 0.5


def choose_dt(ctl: StepControl, umax: float, dx: float, eta: float, masked: bool, t: float) -> float:
    if ctl.dt_fixed > 0.0:
        dt = ctl.dt_fixed
    else:
        dt = ctl.cfl * dx / umax if umax > 0.0 else math.inf
        if masked:
            dt = min(dt, ctl.eta_cap * eta)
        dt = min(dt, ctl.dt_max)
    if t + dt > ctl.t_end:
        dt = ctl.t_end - t
    return dt


# RK4 with explicit diffusion: dt * nu * max|k|^2 is kept below this (the
# classical RK4 is stable on the negative real axis up to about 2.785).
RK4_VISC = 2.5


def rk4_visc_cap(p: Params, g: Grid) -> float:
    """Largest dt with dt * nu * max|k|^2 <= RK4_VISC over the kept modes."""
    k2max = float(np.max(g.k2() * g.dealias()))
    return RK4_VISC / (p.nu * k2max) if p.nu > 0.0 and k2max > 0.0 else math.inf


def ab2_if(p: Params, g: Grid, uh, nh, nh_prev, dt, dt_prev):
    """Integrating-factor AB2 (Euler on the first step)  [Alg. 1 step (e)]."""
    k2 = g.k2()
    e_now = np.exp(-p.nu * k2 * dt)
    if nh_prev is None:
        return e_now * (uh + dt * nh)
    r = dt / dt_prev
    b1, b2 = 1.0 + 0.5 * r, -0.5 * r
    e_prev = np.exp(-p.nu * k2 * dt_prev)
    return e_now * (uh + dt * (b1 * nh + b2 * e_prev * nh_prev))


@dataclass
class State:
    uh: np.ndarray
    nh_prev: np.ndarray | None = None
    t: float = 0.0
    dt_prev: float = 0.0
    n: int = 0
    I_prev: np.ndarray | None = None     # [3 colours][6]: sum chi u_s dV and its moment
    J_prev: np.ndarray | None = None     # sum (x - x_cntr) x chi u_s dV of the previous step
    solid: np.ndarray | None = None      # free-flight state (13) at t
    solid_f: np.ndarray | None = None    # its right-hand side of the previous step


def init_state(p: Params, u0: np.ndarray, t0: float = 0.0) -> State:
    g = grid_of(p)
    return State(uh=import_field(g, u0), t=t0)


def force_sums(g: Grid, u, chi, us, colour, xref, eta):
    """Per colour 1..3: penalization force/torque and I = sum chi u_s dV (+ moment)."""
    x, y, z = g.coords()
    pos = np.stack([x, y, z])
    pen = chi * (u - us) / eta * g.dV
    ius = chi * us * g.dV
    F = np.zeros((3, 3)); M = np.zeros((3, 3)); I = np.zeros((3, 6))
    for c in range(3):
        sel = colour == (c + 1)
        r = pos[:, sel] - xref[c][:, None]
        pc = pen[:, sel]
        ic = ius[:, sel]
        F[c] = pc.sum(axis=1)
        M[c] = np.cross(r.T, pc.T).sum(axis=0)
        I[c, :3] = ic.sum(axis=1)
        I[c, 3:] = np.cross(r.T, ic.T).sum(axis=0)
    return F, M, I


def torque_about(g: Grid, u, chi, us, xc, eta, colour):
    """Penalization torque and J = sum (x - xc) x chi u_s dV about the point xc,
    over the whole body: every point of a part (colour > 0); the points of
    wall layers (colour 0) are not the body's  [eq. moment_of_love, Sec. 2.3]."""
    chi = np.where(colour > 0, chi, 0.0)
    x, y, z = g.coords()
    r = np.stack([x - xc[0], y - xc[1], z - xc[2]])
    pen = chi * (u - us) / eta * g.dV
    ius = chi * us * g.dV
    return _cross(r, pen).reshape(3, -1).sum(axis=1), _cross(r, ius).reshape(3, -1).sum(axis=1)


def step(p: Params, st: State, ctl: StepControl, ins: Insect | None, fixed_mask=None):
    """One pass of Algorithm 1; returns the new state and the diagnostics at t^n
    (with an insect also its pose record, the aerodynamic power of the wings
    and, in free flight, the total force and the torque about x_cntr that
    drive step (f)).

    fixed_mask = (chi, u_s, colour, xref) replaces the insect by a
    time-independent mask (used by tests)."""
    g = grid_of(p)
    masked = ins is not None or fixed_mask is not None or walls_on(p)
    if fixed_mask is not None:
        chi, us, colour, xref = fixed_mask
    elif ins is not None:
        ysol = None
        if ins.free_flight:
            ysol = st.solid if st.solid is not None else solid_init(ins, st.t)
            pose = solid_pose(ysol)
        else:
            pose = prescribed_pose(ins, st.t)
        chi, us, colour = insect_mask(g, ins, st.t, pose)              # (a)
        xref = reference_points(ins, st.t, pose)
    else:
        chi = us = colour = xref = None
    if walls_on(p):
        chi, us, colour = apply_walls(p, g, chi, us, colour)
        if xref is None:
            xref = np.zeros((3, 3))
    u, w = physical_fields(g, st.uh)                                   # u^n, w^n
    umax = umax_of(u)
    if not np.isfinite(umax):
        raise FloatingPointError("non-finite velocity")
    dt = choose_dt(ctl, umax, g.dx, p.eta, masked, st.t)               # (b)
    if p.integrator == "rk4" and ctl.dt_fixed <= 0.0:
        dt = min(dt, rk4_visc_cap(p, g))
        if st.t + dt > ctl.t_end:
            dt = ctl.t_end - st.t
    nphys = source_physical(u, w, 0.0 if chi is None else chi,
                            0.0 if us is None else us, p.eta)          # (c)
    nh = r2c(nphys)
    if p.c_sp > 0.0 and any(d > 0.0 for d in p.sponge):
        nh = nh + sponge_hat(g, w, sponge_mask(g, p.sponge), p.c_sp)  # (c), sponge
    nh = project(g, nh * g.dealias())                                  # (d)
    if p.mean_mode == MEAN_FIXED:
        nh[:, 0, 0, 0] = 0.0
    diag = {"t": st.t, "dt": dt, "umax": umax,
            "E": 0.5 * float(np.sum(u * u)) * g.dV}
    if masked:
        F, M, I = force_sums(g, u, chi, us, colour, xref, p.eta)
        if st.I_prev is not None and st.dt_prev > 0.0:
            F = F + (I[:, :3] - st.I_prev[:, :3]) / st.dt_prev
            M = M + (I[:, 3:] - st.I_prev[:, 3:]) / st.dt_prev
        diag["F"] = F
        diag["M"] = M
        I_now = I
    else:
        I_now = None
    J_now = solid_new = f_new = None
    if p.integrator == "rk4" and ins is not None and ins.free_flight:
        raise ValueError("free flight is stepped with AB2 only")
    if ins is not None and fixed_mask is None:
        diag["pose"] = pose_record(ins, st.t, ysol)
        diag["P_aero"] = np.array([aero_power(M[1 + k], pose.Mb, omega_wing_b(ins, st.t, side)) if ins.wings
                                   else 0.0 for k, side in enumerate(("l", "r"))])
        diag["P_inert"] = np.array([inertial_power(ins, st.t, side) if ins.wings else 0.0 for side in ("l", "r")])
        # total power without energy storage in the muscles  [Sec. 3.5]
        diag["P_total"] = np.maximum(diag["P_inert"] + diag["P_aero"], 0.0)
        m_pen, J_now = torque_about(g, u, chi, us, pose.xc, p.eta, colour)
        if ins.free_flight:
            Ft = F.sum(axis=0)
            mt = m_pen
            if st.J_prev is not None and st.dt_prev > 0.0:
                mt = mt + (J_now - st.J_prev) / st.dt_prev
            diag["F_total"], diag["m_cntr"] = Ft, mt
            if dt > 0.0:                                               # (f)
                solid_new, f_new = solid_step(ins, ysol, st.solid_f, Ft, mt, dt, st.dt_prev)
            else:
                solid_new, f_new = ysol, st.solid_f
    if p.integrator == "rk4":
        uh_new = rk4_step(p, g, st.uh, nh, st.t, dt, ins, fixed_mask)   # (e), RK4
        new = State(uh=uh_new, nh_prev=None, t=st.t + dt, dt_prev=dt, n=st.n + 1, I_prev=I_now,
                    J_prev=J_now, solid=solid_new, solid_f=f_new)
        return new, diag
    uh_new = ab2_if(p, g, st.uh, nh, st.nh_prev, dt,
                    st.dt_prev if st.nh_prev is not None else dt)      # (e)
    new = State(uh=uh_new, nh_prev=nh, t=st.t + dt, dt_prev=dt, n=st.n + 1, I_prev=I_now,
                J_prev=J_now, solid=solid_new, solid_f=f_new)
    return new, diag


def rk4_step(p: Params, g: Grid, uh, nh1, t: float, dt: float, ins: Insect | None, fixed_mask=None):
    """Classical fourth-order Runge-Kutta with explicit diffusion  [Sec. 2.4]:
    R(u_hat, t) = (projected, dealiased right-hand side at t) - nu |k|^2 u_hat,
    with the mask and solid velocity of each stage's time.  nh1 is the
    projected right-hand side of the first stage (at u_hat, t)."""
    k2 = g.k2()

    def R(v, ts):
        if fixed_mask is not None:
            chi, us = fixed_mask[0], fixed_mask[1]
        elif ins is not None:
            chi, us, _ = insect_mask(g, ins, ts)
        else:
            chi = us = None
        chi, us, _ = apply_walls(p, g, chi, us, None)
        return rhs_hat(p, g, v, chi, us)[0] - p.nu * k2 * v

    if dt <= 0.0:
        return uh
    k1 = nh1 - p.nu * k2 * uh
    k2s = R(uh + 0.5 * dt * k1, t + 0.5 * dt)
    k3 = R(uh + 0.5 * dt * k2s, t + 0.5 * dt)
    k4 = R(uh + dt * k3, t + dt)
    return uh + dt / 6.0 * (k1 + 2.0 * k2s + 2.0 * k3 + k4)


def run(p: Params, u0: np.ndarray, nsteps: int, ctl: StepControl,
        ins: Insect | None = None, t0: float = 0.0, fixed_mask=None):
    """Run nsteps of Algorithm 1 from the sampled initial field u0."""
    st = init_state(p, u0, t0)
    hist = []
    for _ in range(nsteps):
        st, d = step(p, st, ctl, ins, fixed_mask)
        hist.append(d)
    return st, hist


def velocity(p: Params, st: State) -> np.ndarray:
    return c2r(st.uh, grid_of(p).shape)


def energy_spectral(g: Grid, uh: np.ndarray) -> float:
    """E = 1/2 sum |u|^2 dV through Parseval on the half spectrum."""
    npts = float(g.nx) * g.n * g.n
    w = np.full(uh.shape[-1], 2.0)
    w[0] = 1.0
    if g.nx % 2 == 0:
        w[-1] = 1.0
    return 0.5 * g.Lx * g.L ** 2 / npts ** 2 * float(np.sum(w * np.abs(uh) ** 2))


def penalization_K(nu: float, eta: float, dx: float) -> float:
    """Points per penalization boundary layer, K = sqrt(nu C_eta)/dx  [Sec. 2.1]."""
    return math.sqrt(nu * eta) / dx


__all__ = [n for n in dir() if not n.startswith("_")]
