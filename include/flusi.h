/*
 * flusi.h -- C ABI of the MI355X (gfx950) pseudo-spectral penalized
 * Navier-Stokes hot path.
 *
 * Method: Engels, Kolomenskiy, Schneider, Sesterhenn, "FluSI: A novel parallel
 * simulation tool for flapping insect flight using a Fourier method with
 * volume penalization", arXiv:1506.06513.  Section and equation names below
 * refer to that paper.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns an int status: FLUSI_OK (0) or a negative FLUSI_E*
 *    code.  flusi_last_error() returns a thread-local message for the last
 *    failure.  No C++ exception crosses the ABI.
 *  - Box: n points per axis on y and z (side L) and nx on x (side L*nx/n),
 *    one spacing L/n, grid points x_i = i*L/n.  Cubic grids (nx = n) for n in
 *    16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512 (even and of the form
 *    2^a 3^b); boxes 48x32x32, 64x32x32 and 192x128x128 (see
 *    flusi_plan_create).
 *  - Physical fields: [field][z][y][x] row-major, x fastest, real type of the
 *    plan (float for FLUSI_F32, double for FLUSI_F64).
 *  - Spectral fields, full layout: [field][kz][ky][kx] with kx = 0..nx/2
 *    (fastest), ky and kz in FFT order (bin i holds j = i for i < n/2 and
 *    j = i - n otherwise); complex values are interleaved (re, im) pairs of
 *    the plan's real type.  The forward transform is unnormalized with
 *    exp(-i k.x); the inverse is scaled by 1/(nx n n).
 *  - Every field/state pointer is a DEVICE pointer owned by the caller,
 *    contiguous and 16-byte aligned.  The plan owns twiddle tables, integer
 *    tables and scratch memory.
 *  - Work is enqueued on the stream set with flusi_set_stream (default: the
 *    null stream); calls return without synchronizing unless their
 *    description says otherwise.
 *  - Scalars (times, forces, coefficients) are always double.
 */
#ifndef FLUSI_H
#define FLUSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLUSI_OK 0
#define FLUSI_EINVAL (-1)        /* bad argument (null pointer, wrong size, ...) */
#define FLUSI_EUNSUPPORTED (-2)  /* grid size or combination not supported */
#define FLUSI_ENOMEM (-3)        /* device allocation failed */
#define FLUSI_EDEVICE (-4)       /* a HIP runtime call failed */
#define FLUSI_ENONFINITE (-5)    /* the velocity became NaN or infinite */

#define FLUSI_F32 0
#define FLUSI_F64 1

#define FLUSI_BODY_NONE 0
#define FLUSI_BODY_SPHERE 1
#define FLUSI_BODY_ELLIPSOID 2

#define FLUSI_KIN_SINE 0     /* wing angle = mean + amplitude*cos(2*pi*freq*t + phase) */
#define FLUSI_KIN_FOURIER 1  /* wing angle = a_0/2 + sum_i a_i cos(2*pi*i*freq*t) + b_i sin(...) */
#define FLUSI_KIN_HERMITE 2  /* periodic cubic Hermite through values and rates at kin_n times */
#define FLUSI_KIN_MAX 24     /* harmonics (Fourier) or nodes (Hermite) per angle */

#define FLUSI_WING_ELLIPSE 0 /* elliptic outline: half chord wing_A, half span wing_B, centre (0, B) */
#define FLUSI_WING_FOURIER 1 /* polar-radius outline R(v) as a Fourier series (Sec. 3.4) */
#define FLUSI_WING_RECT 2    /* rectangle: chord [-(B - b), b] along x_w, span [a, tip] along y_w */
#define FLUSI_WING_MAX 32    /* radius harmonics */
#define FLUSI_RTABLE 25000   /* samples of the radius table (Sec. 3.4) */

#define FLUSI_SMOOTH_COS 0   /* cosine layer, Sec. 2.2 eq. smoothing_mask_as_function_of_delta */
#define FLUSI_SMOOTH_TANH 1  /* 0.5*(1 - tanh(delta/h)) */

#define FLUSI_INT_AB2 0      /* integrating-factor AB2 (Alg. 1 step (e)) */
#define FLUSI_INT_RK4 1      /* classical RK4 with explicit diffusion (Sec. 2.4) */

#define FLUSI_MEAN_FIXED 0   /* k = 0 right-hand side set to zero: the mean velocity is held */
#define FLUSI_MEAN_FREE 1    /* k = 0 right-hand side kept */

/* Per-step diagnostics record (doubles), written by flusi_step and returned
 * by flusi_forces:
 *   [0] t^n   [1] dt_n   [2] max|u|   [3] E = 1/2 sum |u|^2 dV
 *   [4 + 6*(c-1) + 0..2]  force  F on colour c (c = 1 body, 2 left wing, 3 right wing)
 *   [4 + 6*(c-1) + 3..5]  torque m on colour c
 *   [22..24] x_cntr  [25..27] u_cntr  [28..31] quaternion eps_0..3
 *   [32..34] Omega_b^(b): the body's state at t^n (Sec. 3.6; for a tethered
 *            body the prescribed kinematics, eps from the body angles)
 *   [35] [36] aerodynamic power P_aero of the left and right wing
 *            (Sec. 3.5, eq. insect_power)
 *   [37] [38] inertial power P_inert of the left and right wing (Sec. 3.5)
 *   [39] [40] P_total = max(P_inert + P_aero, 0) of the left and right wing
 * Force and torque follow eqs. force_with_unst_corrections / moment_of_love
 * (Sec. 2.1): the penalization integral plus the time derivative of the solid
 * momentum, as the force acting on the solid.  Torques are taken about the
 * body centre (body) and the wing pivots (wings).  P_aero = -m . (Omega_w -
 * Omega_b) with m the wing torque about its pivot and Omega_w - Omega_b the
 * wing's angular velocity relative to the body.  P_inert = W . (J W' + W x J W)
 * with W the wing's angular velocity in its own frame, W' its time derivative
 * (exact, from the angle series' second derivatives) and J = wing_J; zero when
 * wing_J is zero.  Without a mask [4..40] are zero. */
#define FLUSI_NDIAG 41

typedef struct flusi_plan_s* flusi_plan;

/* Rigid insect (Sec. 3), or a single body when wings == 0.  Angles in
 * radians.  Each wing angle is mean + amplitude*cos(2*pi*freq*t + phase).
 *
 * Tethered (free_flight == 0): body angles evolve as angle + rate*t; x_cntr is
 * the body centre at the current time (the body is not translated by the
 * library) and u_cntr its velocity.
 *
 * Free flight (free_flight == 1, Sec. 3.6, eq. oh_my_god_look_a_vector): the
 * state keeps the 13 values x_cntr (centre of gravity), u_cntr, the unit
 * quaternion eps and Omega_b^(b), advanced after every step with the fluid's
 * AB2 weights (Euler on the first free-flight step) from the total force F
 * and the torque m about x_cntr:  M u_cntr' = F - M g e_z,
 * J Omega' + Omega x J Omega = M_body m, eps' = 1/2 S^T Omega.  M_body (global
 * to body) is the transpose of the printed quaternion matrix; eps is
 * renormalized after each step.  dof multiplies the acceleration rows
 * (translation x, y, z; rotation about the body axes x, y, z; 1 on, 0 off).
 * The first free-flight step of a state starts from the tethered kinematics
 * at its time (x_cntr, u_cntr, eps of psi/beta/gamma at t, their Omega_b);
 * a tethered step drops the free-flight state.  Requires a body or wings,
 * mass > 0 and inertia > 0.  Wing kinematics stay prescribed relative to the
 * body. */
typedef struct {
    int body;            /* FLUSI_BODY_* */
    int wings;           /* 0: no wings; 1: left and right wing */
    int smooth;          /* FLUSI_SMOOTH_* */
    int free_flight;     /* 0 tethered, 1 free flight */
    double c_smth;       /* smoothing half-width h = c_smth*dx */
    double x_cntr[3];
    double u_cntr[3];
    double psi, beta, gamma;              /* roll, pitch, yaw: M_body = Rx(psi) Ry(beta) Rz(gamma) */
    double psi_dot, beta_dot, gamma_dot;
    double radius;       /* sphere radius */
    double a, b;         /* ellipsoid thorax: semi-axis a along x_b, b across */
    double eta_stroke;   /* anatomical stroke-plane angle */
    double pivot_l[3];   /* wing pivots in the body frame */
    double pivot_r[3];
    double wing_A;       /* elliptic wing: half chord (x_w) */
    double wing_B;       /* half span (y_w); the ellipse is centred at (0, B) */
    double wing_t;       /* wing thickness (z_w) */
    double freq;
    double phi[3];       /* positional angle: mean, amplitude, phase */
    double alpha[3];     /* feathering angle */
    double theta[3];     /* deviation angle */
    double mass;         /* free flight: M */
    double inertia[3];   /* principal moments J_x, J_y, J_z about the body axes */
    double gravity;      /* g, acting along -z of the global frame */
    double dof[6];       /* 1/0: translation x, y, z; rotation about x_b, y_b, z_b */
    /* Wing angle parametrization (Sec. 3.3).  FLUSI_KIN_SINE uses phi/alpha/
     * theta above.  FLUSI_KIN_FOURIER: kin_coef[angle][0][i] = a_i and
     * [angle][1][i] = b_i, i = 0..kin_n (b_0 unused), angle 0 phi, 1 alpha,
     * 2 theta.  FLUSI_KIN_HERMITE: kin_n nodes at t_j = j/(kin_n*freq) of one
     * period; kin_coef[angle][0][j] = value, [angle][1][j] = rate (rad per time
     * unit); joined by periodic cubic Hermite interpolation. */
    int kin_type;        /* FLUSI_KIN_* */
    int kin_n;           /* Fourier: highest harmonic (0..FLUSI_KIN_MAX); Hermite: nodes (2..FLUSI_KIN_MAX) */
    int wing_shape;      /* FLUSI_WING_* */
    int wing_n;          /* Fourier wing: highest harmonic (0..FLUSI_WING_MAX) */
    double kin_coef[3][2][FLUSI_KIN_MAX + 1];
    /* Fourier wing (Sec. 3.4, eq. Fourier_radious_wing): in the wing plane,
     * about the centre wing_c, r - R(v) with v the polar angle in turns
     * (counterclockwise from +x_w) and R(v) = a_0/2 + sum_i a_i cos(2 pi i v) +
     * b_i sin(2 pi i v), wing_coef[0][i] = a_i, wing_coef[1][i] = b_i.  R is
     * sampled at FLUSI_RTABLE angles when the coefficients change (plan-owned
     * table) and interpolated linearly.  Thickness: wing_t. */
    double wing_c[2];
    double wing_coef[2][FLUSI_WING_MAX + 1];
    /* Body parts (Sec. 3.2, ellipsoid bodies): head sphere and a mirrored pair
     * of eye spheres at (x, +y, z) and (x, -y, z), body frame; joined with the
     * thorax as a union (minimum of the signed distances).  Radius 0: none. */
    double head_x[3], head_r;
    double eye_x[3], eye_r;
    /* Rectangular wing (Sec. 3.4, eq. signed_distance_rectangular_wing, read as
     * max(x - b, -x - (B - b), y - tip, a - y, |z| - t/2)): wing_rect = {a, tip,
     * b, B}; thickness wing_t. */
    double wing_rect[4];
    /* Wing tensor of inertia J^(w) about the pivot in the wing's own frame, for
     * the inertial power (Sec. 3.5; the paper gives no values): {J_xx, J_yy,
     * J_zz, J_xy, J_xz, J_yz}, symmetric, the same for both wings in their own
     * frames.  All zero: no inertial power. */
    double wing_J[6];
} flusi_insect;

/* Controls of flusi_step (Algorithm 1 steps (a)-(e)). */
typedef struct {
    int nsteps;          /* number of time steps to take */
    int mean_mode;       /* FLUSI_MEAN_* */
    double dt_fixed;     /* > 0: use this step; otherwise adaptive */
    double cfl;          /* adaptive: dt = cfl*dx/max|u| ... */
    double dt_max;       /* ... capped by dt_max (<= 0: no cap) ... */
    double eta_cap;      /* ... and by eta_cap*C_eta when a mask is present ... */
    double t_end;        /* ... and clamped to land on t_end (<= 0: none) */
    double* history;     /* optional DEVICE pointer [nsteps][FLUSI_NDIAG]; may be NULL */
} flusi_step_params;

/* Message for the last failed call on this thread (never NULL). */
const char* flusi_last_error(void);

/* Create a plan for a periodic box of nx x ny x nz points (Sec. 2.4: Fourier
 * discretization with the 2/3 rule) with ny = nz = n and one grid spacing
 * L/n on every axis: L is the side along y and z, the side along x is
 * L*nx/n (the non-cubic box of Sec. 4 and 6, 6x4x4 at 1152x768x768, has one
 * spacing).  Grids: the cubic n^3 for n in {16, 24, 32, 48, 64, 96, 128, 192,
 * 256, 384, 512} and the boxes 48x32x32, 64x32x32 and 192x128x128.
 * nu: kinematic viscosity; eta: penalization constant C_eta (Sec. 2.1);
 * dtype: FLUSI_F32 or FLUSI_F64.  Builds the integer wavenumber and
 * dealiasing tables (kept iff 3|j| < n_a on axis a), FP64 twiddle tables (and
 * FP32 copies rounded from them) and the scratch buffers of the stepping
 * schedule.  Every physical field is [z][y][x] with x fastest (nx), every
 * full-layout spectrum [z][y][nx/2+1].  Errors: EINVAL, EUNSUPPORTED (ny !=
 * nz or a grid not listed), ENOMEM. */
int flusi_plan_create(int nx, int ny, int nz, double L, double nu, double eta, int dtype,
                      flusi_plan* out);
int flusi_plan_destroy(flusi_plan plan);

/* Device bytes a plan of the cubic n^3 grid and dtype allocates at creation
 * (workspace) and that one state occupies, without allocating anything.
 * Errors: EINVAL, EUNSUPPORTED. */
int flusi_sizes(int n, int dtype, size_t* workspace_bytes, size_t* state_bytes);

/* Time integrator of this plan's later flusi_step calls (Sec. 2.4).
 * FLUSI_INT_AB2 (default): integrating-factor AB2 as in Algorithm 1.
 * FLUSI_INT_RK4: classical fourth-order Runge-Kutta with explicit diffusion,
 * du_hat/dt = P D FFT(u x w - (chi/C_eta)(u - u_s) [+ sponge]) - nu |k|^2 u_hat,
 * with the mask and solid velocity at t, t + dt/2, t + dt/2 and t + dt; the
 * diagnostics record is that of the first stage; the adaptive dt is also kept
 * below 2.5/(nu max|k|^2) over the kept modes (explicit diffusion stability).
 * RK4 allocates three fields of stage velocity (synchronously, once) and uses
 * the state's AB2 history storage for its stage sum, so a later AB2 step
 * starts with Euler.  Free flight is AB2 only (flusi_step and
 * flusi_ensemble_add return EUNSUPPORTED for it under RK4).  Errors: EINVAL,
 * ENOMEM. */
int flusi_plan_set_integrator(flusi_plan plan, int integrator);

/* Dirichlet layers (Sec. 2.3: velocity conditions imposed by the volume
 * penalization, e.g. u = u_infinity at the domain borders or channel walls)
 * for every later step of this plan: chi = 1 and u_s = u_wall where x_a >=
 * L_a - thickness[a] (L_a the box side on axis a) for an axis a with
 * thickness[a] > 0 (sharp layers at the
 * top end of the axes, placed like the sponge's).  The layers take
 * precedence over a body and are not part of its force integrals (their
 * points carry colour 0); a step with layers applies the C_eta step cap.
 * thickness and u_wall are host arrays of 3 doubles (NULL: zeros).  All
 * thicknesses 0 switch the layers off.  Errors: EINVAL (thickness outside
 * [0, L_a], non-finite velocity). */
int flusi_plan_set_walls(flusi_plan plan, const double* thickness, const double* u_wall);

/* Vorticity sponge (Sec. 2.3, wake removal; the sponge term of eq.
 * PNST_org_momentum) for every later step of this plan: the right-hand side
 * gains -(1/C_sp) (i k x W_hat)/|k|^2 with W = chi_sp * w, the Biot-Savart form
 * of damping the vorticity at rate chi_sp/C_sp (divergence-free, zero at
 * k = 0).  chi_sp = 1 where x_a >= L_a - thickness[a] for an axis a with
 * thickness[a] > 0 (a layer at the top end of that axis, just upstream of the
 * periodic seam), 0 elsewhere.  c_sp <= 0 or all thicknesses 0 switch it off.
 * thickness is a host array of 3 doubles (may be NULL: off).  Switching it
 * on enlarges the plan's scratch (6 instead of 3 forward fields; synchronizes
 * the device before the old buffer is freed).  Not used by flusi_rhs.  Errors: EINVAL (thickness < 0
 * or > L_a), ENOMEM. */
int flusi_plan_set_sponge(flusi_plan plan, double c_sp, const double* thickness);

/* All further launches of this plan go to `stream` (a hipStream_t). */
int flusi_set_stream(flusi_plan plan, void* stream);

/* Device bytes held by the plan (tables + scratch) and bytes of one state
 * buffer (header + velocity coefficients + previous right-hand side). */
size_t flusi_plan_workspace_bytes(flusi_plan plan);
size_t flusi_state_bytes(flusi_plan plan);

/* Copies of the integer tables the plan uses: j for the n bins of the signed
 * axes y and z (FFT order), and the dealias flags (1 kept, 0 removed) of
 * those bins.  Host pointers of n ints each; synchronous. */
int flusi_tables(flusi_plan plan, int* j_signed, int* keep_signed);

/* Forward 3D real-to-complex transform of nf fields (Sec. 2.4).
 * in: [nf][n][n][nx] real; out: [nf][n][n][nx/2+1] complex (full layout). */
int flusi_fft_r2c(flusi_plan plan, const void* in, void* out, int nf);

/* Inverse 3D complex-to-real transform with 1/n^3, input preserved.  The
 * imaginary parts of the kx = 0 and kx = n/2 bins are ignored (Hermitian
 * input assumed).  May allocate plan scratch on first use. */
int flusi_fft_c2r(flusi_plan plan, const void* in, void* out, int nf);

/* flusi_fft_c2r for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and results, bit for bit, with the intermediate spectra in
 * a fixed 64 MiB array of the library (one copy per GPU, held until the
 * process ends) instead of plan scratch.  Allocates nothing.  The scratch
 * must hold nf full-layout spectra, nf * n * n * (nx/2+1) complex values of
 * the plan's type: three 128^3 fields in FP64 (51 MB) or two 192^3 fields in
 * FP32 (57 MB) fit, one 256^3 FP32 field (67.6 MB) does not; larger requests
 * return EINVAL with the sizes.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams or host threads) race and must be ordered by the caller.  Nothing
 * in the array needs to start at zero.  Errors: EINVAL (sizes, null
 * pointers), EDEVICE (launch failure, or the array's address unavailable). */
int flusi_fft_c2r_noalloc(flusi_plan plan, const void* in, void* out, int nf);

/* Algorithm 1 step (a): mask chi, solid velocity u_s and colour at time t
 * (Sec. 2.2, Sec. 3.1-3.4).  chi: [n][n][nx] real; us: [3][n][n][nx] real;
 * colour: [n][n][nx] int16 (0 fluid, 1 body, 2 left wing, 3 right wing).  Parts
 * combine by the maximum of chi; u_s and colour come from that part (ties go
 * to the lower colour); u_s = 0 where chi = 0.  Any output pointer may be
 * NULL. */
int flusi_mask_insect(flusi_plan plan, const flusi_insect* ins, double t, void* chi, void* us,
                      int16_t* colour);

/* Unfused right-hand side of Algorithm 1 steps (c)-(d): from full-layout
 * uhat [3] (assumed dealiased), chi and us (physical, may be NULL for no
 * mask) computes rhs_hat = P D r2c(u x w - (chi/C_eta)(u - u_s)) with w the
 * curl, D the 2/3 rule and P the projection (identity at k = 0; the k = 0
 * value is zeroed for FLUSI_MEAN_FIXED).  umax_host (may be NULL) receives
 * max|u| (this call then synchronizes).  Cubic grids only (EUNSUPPORTED
 * otherwise). */
int flusi_rhs(flusi_plan plan, const void* uhat, const void* chi, const void* us, void* rhs_hat,
              int mean_mode, double* umax_host);

/* Initialize a state buffer of flusi_state_bytes() bytes (caller-owned device
 * memory) from the physical velocity u0 [3][n][n][nx] sampled on the grid
 * (eq. PNST_inicond): the coefficients are dealiased and projected; time t0,
 * no step history. */
int flusi_state_init(flusi_plan plan, void* state, const void* u0, double t0);

/* Write the velocity of a state as a full-layout spectrum [3][n][n][nx/2+1]
 * (zeros outside the 2/3 band). */
int flusi_state_export_uhat(flusi_plan plan, const void* state, void* uhat);

/* Physical velocity u [3][n][n][nx] of a state. */
int flusi_state_velocity(flusi_plan plan, const void* state, void* u);

/* Time and step count of a state (synchronous). */
int flusi_state_time(flusi_plan plan, const void* state, double* t, long long* n);

/* Advance a state by p->nsteps steps of Algorithm 1: mask and solid velocity
 * at t^n (ins may be NULL: no mask), dt from the FP64 max|u| reduction, the
 * source u x w - (chi/C_eta)(u - u_s) with the FP64 force, torque and energy
 * integrals, the 2/3 rule and projection, and the integrating-factor AB2
 * update (Euler on the first step of a state).  No host synchronization;
 * graph-capturable once the plan exists.  A non-finite velocity stops the
 * state (later steps do nothing) and is reported by flusi_forces. */
int flusi_step(flusi_plan plan, void* state, const flusi_insect* ins, const flusi_step_params* p);

/* Diagnostics record (FLUSI_NDIAG doubles, see above) of the last step taken
 * on this state, copied to host memory (synchronous).  Returns
 * FLUSI_ENONFINITE if the state was stopped by a non-finite velocity. */
int flusi_forces(flusi_plan plan, const void* state, double* out);

/* Free-flight state of the current time level (Sec. 3.6): out[13] =
 * x_cntr[3], u_cntr[3], eps[4], Omega_b^(b)[3] (host array; synchronous).
 * Errors: EINVAL if the state has no free-flight body (never stepped in free
 * flight, or last stepped tethered); ENONFINITE if it was stopped. */
int flusi_state_solid(flusi_plan plan, const void* state, double* out);

/* Set the free-flight state of the current time level from y[13] (host
 * array, same layout); the next free-flight step starts from it with an
 * Euler step (for restarts and prescribed initial rates).  The quaternion must
 * have unit length (within 1e-12).  Enqueued on the plan's stream.  Errors:
 * EINVAL. */
int flusi_state_set_solid(flusi_plan plan, void* state, const double* y);

/* Instrumentation.  While enabled, flusi_step brackets each pass it launches
 * with HIP events on the plan's stream.  Passes: 0 inverse z of the state at
 * the start of a call, 1 y-inverse, 2 x-pass (inverse x, source, forward x),
 * 3 body kinematics of a time level (and the free-flight advance), 4
 * y-forward (with the first-level reduction), 5 z-pass (forward z,
 * projection, AB2, inverse z).  flusi_profile(plan, 1) clears the records and starts
 * recording, flusi_profile(plan, 0) stops.  flusi_pass_times synchronizes the
 * stream and returns, per pass, the summed event time in milliseconds and the
 * number of launches recorded since the last flusi_profile(plan, 1); ms and
 * launches are host arrays of FLUSI_NPASS entries (either may be NULL). */
#define FLUSI_NPASS 6
int flusi_profile(flusi_plan plan, int enable);
int flusi_pass_times(flusi_plan plan, double* ms, long long* launches);

/* ------------------------------------------------------------------------
 * Schedules and the autotuner.
 *
 * Each stepping pass (y-inverse, x-pass, y-forward, z-pass) exists in three
 * tile variants: 0 (default), 1 and 2 (y passes: a half / a quarter of the
 * columns per workgroup; x-pass: a half / a quarter of the rows, at least two;
 * z-pass: two or three / four or six times the threads per column).  The
 * z-pass runs either as one launch (update, curl and inverse z) or as two
 * (update, then curl + inverse z).  The velocity field does not depend on
 * the schedule (every variant performs the same operations per value); the
 * x-pass variant changes only the summation order of the FP64 diagnostic
 * integrals (energy, force, torque), at round-off level.
 * ------------------------------------------------------------------------ */
typedef struct {
    int y_inverse;   /* tile variant, 0, 1 or 2 */
    int x_pass;
    int y_forward;
    int z_pass;
    int split_z;     /* 1: z-pass as update + inverse launches, 0: one launch */
    int reserved[3]; /* zero */
} flusi_schedule;

/* Schedule used by this plan's flusi_step calls (and by an ensemble size
 * group whose first member is this plan).  Errors: EINVAL (variant out of
 * range, split_z not 0/1). */
int flusi_plan_get_schedule(flusi_plan plan, flusi_schedule* out);
int flusi_plan_set_schedule(flusi_plan plan, const flusi_schedule* s);

/* Times every variant of every pass over reps steps (after 2 warm-up steps)
 * on a scratch copy of `state` with body ins and controls p, keeps the
 * fastest variant per pass, then the faster of the one- and two-launch
 * z-pass, and makes that the plan's schedule (also returned in *out, which
 * may be NULL).  The state itself is not modified.  Synchronous.  Errors:
 * EINVAL, ENOMEM, EDEVICE. */
int flusi_autotune(flusi_plan plan, const void* state, const flusi_insect* ins, const flusi_step_params* p,
                   int reps, flusi_schedule* out);

/* ------------------------------------------------------------------------
 * Ensembles: many independent simulations advanced together.
 *
 * A member is a (plan, state) pair with its body and step controls; plans
 * may differ in grid, L, nu, eta and integrator but share the ensemble's
 * dtype, and a plan belongs to at most one member (its scratch buffers are the
 * member's).  Members of equal grid shape and integrator form a size group
 * (the group is fixed when the ensemble is next stepped after an add or
 * remove).  flusi_ensemble_step launches each
 * pass of Algorithm 1 once per size group over all of its members (one
 * workgroup grid spanning every member), with the size groups on parallel
 * streams forked from the ensemble's stream.  Each member follows exactly the
 * arithmetic of flusi_step on its own plan, so results are bitwise equal to
 * stepping the members one by one with the same schedule.
 *
 * Ownership: the ensemble keeps the plan and state pointers (it owns
 * neither); destroy the ensemble before them.  Adding or removing members
 * invalidates captured graphs (they are rebuilt on the next call).
 * Changing a member plan's options (flusi_plan_set_sponge, _set_walls,
 * _set_integrator, _set_schedule, flusi_autotune) is allowed between calls:
 * the next flusi_ensemble_* call synchronizes the ensemble's streams, rebuilds
 * the launch tables from the plan's current options and buffers and drops the
 * captured graphs, so the member again equals flusi_step on its plan.  Such a
 * change must not overlap a running ensemble call on another host thread.
 * ------------------------------------------------------------------------ */
typedef struct flusi_ensemble_s* flusi_ensemble;

/* Empty ensemble for plans of the given dtype.  Errors: EINVAL, ENOMEM. */
int flusi_ensemble_create(int dtype, flusi_ensemble* out);
/* Synchronizes the ensemble's streams and frees its tables and graphs. */
int flusi_ensemble_destroy(flusi_ensemble e);
/* Stream (hipStream_t) on which flusi_ensemble_step is ordered. */
int flusi_ensemble_set_stream(flusi_ensemble e, void* stream);
/* Adds a member.  ins: body (NULL: no mask), copied; p: step controls as for
 * flusi_step (p->nsteps is ignored; p->history, when set, receives one record
 * per step of each flusi_ensemble_step call, row s for step s of the call).
 * *id receives a member index that stays valid until the member is removed.
 * Errors: EINVAL (dtype mismatch, plan already a member, bad controls),
 * EUNSUPPORTED (free flight on an RK4 plan). */
int flusi_ensemble_add(flusi_ensemble e, flusi_plan plan, void* state, const flusi_insect* ins,
                       const flusi_step_params* p, int* id);
/* Removes member id (its state is left as it is). */
int flusi_ensemble_remove(flusi_ensemble e, int id);
/* Number of members and of size groups. */
int flusi_ensemble_size(flusi_ensemble e, int* members, int* groups);
/* Advances every member by nsteps steps (Algorithm 1, as flusi_step).
 * use_graph != 0: the whole call (all groups, all steps) is captured once per
 * distinct nsteps into a hipGraph and replayed on later calls.  No host
 * synchronization. */
int flusi_ensemble_step(flusi_ensemble e, int nsteps, int use_graph);
/* Autotunes every size group as a whole (all of its members in each timed
 * launch, as flusi_ensemble_step runs them) on scratch copies of the member
 * states, and stores the chosen schedule in the group's first plan.  Member
 * states are not modified.  Synchronous. */
int flusi_ensemble_autotune(flusi_ensemble e, int reps);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * A server owns a worker thread, an ensemble and the device memory of the
 * requests it has admitted.  Submitted requests queue in arrival order; the
 * worker admits the oldest waiting requests while their device footprint
 * (plan workspace + state + velocity-export scratch + output field) fits the
 * HBM budget, advances every admitted request together (all grid sizes in
 * one ensemble step, size groups on parallel streams) in chunks of at most
 * max_chunk steps, never past any request's last step, and retires a request
 * as soon as its steps are done: its final velocity and diagnostics are
 * copied to host memory and its device memory is freed, which admits the
 * next waiting requests.  A request's result is bitwise the same as stepping
 * it alone with flusi_step (same plan parameters, body, controls and steps).
 * Latency = completion time - submit time (host steady clock).
 * ------------------------------------------------------------------------ */
typedef struct flusi_server_s* flusi_server;

typedef struct {
    int n;                 /* grid points per axis */
    int has_insect;        /* 0: no mask; otherwise `ins` is used */
    double L, nu, eta;     /* box side, viscosity, C_eta */
    flusi_insect ins;
    flusi_step_params p;   /* controls; p.nsteps = steps of the request; p.history is ignored */
    const void* u0;        /* HOST pointer to the initial velocity [3][n][n][n] of the server's real
                              type (copied by flusi_server_submit), or NULL: fluid at rest */
} flusi_request;

typedef struct {
    long long submitted, completed, failed, waiting, active;
    double p50_ms, p99_ms, max_ms;  /* latency over completed requests */
    double point_steps;             /* sum of n^3 * steps over completed requests */
    double busy_s;                  /* first submit to last completion */
    double mpoint_steps_per_s;      /* point_steps / busy_s / 1e6 */
    size_t peak_bytes;              /* largest admitted footprint sum */
    int peak_active;                /* most requests on the device at once */
    int reserved;
} flusi_server_stats;

/* Footprint a request of grid n occupies while admitted (bytes). */
size_t flusi_request_bytes(int n, int dtype);
/* Server for requests of one dtype; hbm_budget: device bytes the admitted
 * requests may occupy together; max_chunk >= 1: steps per batch iteration.
 * Starts the worker thread on the current device.  Errors: EINVAL, EDEVICE. */
int flusi_server_create(int dtype, size_t hbm_budget, int max_chunk, flusi_server* out);
/* Stops the worker (after the request in flight of each batch iteration) and
 * frees every request and result. */
int flusi_server_destroy(flusi_server s);
/* Queues a request (thread-safe; copies r and the initial field) and returns
 * its id.  Errors: EINVAL (bad parameters), EUNSUPPORTED (grid size), ENOMEM
 * (footprint larger than the whole budget). */
int flusi_server_submit(flusi_server s, const flusi_request* r, long long* id);
/* Waits up to timeout_ms (< 0: no limit) for request id to finish.  Then
 * copies its final velocity [3][n][n][n] to u_host (may be NULL), its last
 * diagnostics record (FLUSI_NDIAG doubles) to diag (may be NULL) and its
 * latency in ms to latency_ms (may be NULL), forgets the request and returns
 * its status (FLUSI_OK, FLUSI_ENONFINITE, ...).  Returns 1 on time-out (the
 * request stays).  Errors: EINVAL (unknown id). */
int flusi_server_wait(flusi_server s, long long id, double timeout_ms, void* u_host, double* diag,
                      double* latency_ms);
/* Counters and latency percentiles so far. */
int flusi_server_stats_get(flusi_server s, flusi_server_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* FLUSI_H */
