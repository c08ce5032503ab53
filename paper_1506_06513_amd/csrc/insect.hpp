// Insect kinematics and mask evaluation (FP64), Sec. 2.2 and Sec. 3.
//
// The kinematics block is evaluated once per time level by one workgroup and
// read by every mask evaluation; the mask is evaluated pointwise inside the
// physical-space pass (no chi / u_s arrays in HBM).
#pragma once
#include "common.hpp"
#include "../../include/flusi.h"

namespace flusi {

// Per-time-level insect state in the global frame.
struct Kin {
    double Mb[9];      // M_body = Rx(psi) Ry(beta) Rz(gamma): x_b = Mb (x_g - xc)
    double xc[3];      // body centre
    double uc[3];      // body centre velocity
    double omb[3];     // body angular velocity, body frame
    double eps[4];     // orientation quaternion (free-flight state, or of the body angles)
    double Mws[2][9];  // M_wing M_stroke for the left [0] and right [1] wing
    double piv[2][3];  // pivots, body frame
    double omw[2][3];  // wing angular velocities, body frame
    double pinert[2];  // inertial power of the left and right wing (Sec. 3.5)
    double xref[3][3]; // torque reference points (global): body centre, left pivot, right pivot
    double r2all;      // squared radius (about xc) outside which chi == 0 exactly
    double thr;        // delta above which chi == 0 exactly
    double h;          // smoothing half width
    double radius, ea, eb;       // sphere radius; ellipsoid semi-axes
    double wA, wB, wt;           // elliptic wing: half chord, half span, thickness
    double wcen[2];    // wing outline centre in the wing plane: ellipse (0, B); Fourier wing x_c^(w)
    double wrad;       // in-plane radius of the outline about wcen is at most this
    double sph[3][4];  // body spheres (head, left eye, right eye): centre (body frame), radius
    const double* rtab;  // Fourier wing radius table (FLUSI_RTABLE + 1 samples, last = first)
    const float* rtab32; // the same rounded to FP32
    int body, wings, smooth, wshape, nsph, pad;
};

// Radius table of a Fourier wing (Sec. 3.4): the coefficients it is built from.
struct WingCoef {
    int n, pad;
    double a[FLUSI_WING_MAX + 1], b[FLUSI_WING_MAX + 1];
};

// sin and cos of one angle, out of line: one shared copy of the FP64
// expansion keeps the kinematics code (fetched cold every launch) short.
// Returned by value (registers), so callers keep their matrices in registers.
struct SinCos {
    double s, c;
};
__host__ __device__ __attribute__((noinline)) inline SinCos sin_cos(double x) { return SinCos{sin(x), cos(x)}; }

// Where the kinematics take their sines and cosines from: evaluated in place
// (TrigEval), or looked up in a table that the lanes of a workgroup filled in
// parallel beforehand, in the order the kinematics ask for them (TrigTable).
// A table entry is used only when its argument is bitwise the one asked for,
// so the result never depends on the table; a miss evaluates in place.
struct TrigEval {
    __host__ __device__ SinCos operator()(double x) { return sin_cos(x); }
};
struct TrigTable {
    const double* arg;
    const SinCos* val;
    int n, i;  // entries; index of the next request
    __device__ SinCos operator()(double x) {
        const int j = i++;
        if (j < n && __double_as_longlong(arg[j]) == __double_as_longlong(x)) return val[j];
        return sin_cos(x);
    }
};

template <class TR = TrigEval>
__host__ __device__ inline void mat_rx(double a, double* M, TR&& tr = TR{}) {
    const SinCos q = tr(a);
    const double c = q.c, s = q.s;
    M[0] = 1; M[1] = 0; M[2] = 0;
    M[3] = 0; M[4] = c; M[5] = s;
    M[6] = 0; M[7] = -s; M[8] = c;
}
template <class TR = TrigEval>
__host__ __device__ inline void mat_ry(double a, double* M, TR&& tr = TR{}) {
    const SinCos q = tr(a);
    const double c = q.c, s = q.s;
    M[0] = c; M[1] = 0; M[2] = -s;
    M[3] = 0; M[4] = 1; M[5] = 0;
    M[6] = s; M[7] = 0; M[8] = c;
}
template <class TR = TrigEval>
__host__ __device__ inline void mat_rz(double a, double* M, TR&& tr = TR{}) {
    const SinCos q = tr(a);
    const double c = q.c, s = q.s;
    M[0] = c; M[1] = s; M[2] = 0;
    M[3] = -s; M[4] = c; M[5] = 0;
    M[6] = 0; M[7] = 0; M[8] = 1;
}
__host__ __device__ inline void mat_mul(const double* A, const double* B, double* C) {
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
    for (int i = 0; i < 9; ++i) C[i] = t[i];
}
__host__ __device__ inline void mat_vec(const double* A, const double* v, double* o) {
    const double a = A[0] * v[0] + A[1] * v[1] + A[2] * v[2];
    const double b = A[3] * v[0] + A[4] * v[1] + A[5] * v[2];
    const double c = A[6] * v[0] + A[7] * v[1] + A[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}
// A^T v
__host__ __device__ inline void mat_tvec(const double* A, const double* v, double* o) {
    const double a = A[0] * v[0] + A[3] * v[1] + A[6] * v[2];
    const double b = A[1] * v[0] + A[4] * v[1] + A[7] * v[2];
    const double c = A[2] * v[0] + A[5] * v[1] + A[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}
__host__ __device__ inline void cross3(const double* a, const double* b, double* o) {
    const double x = a[1] * b[2] - a[2] * b[1];
    const double y = a[2] * b[0] - a[0] * b[2];
    const double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}

// M_body (global to body) of a unit quaternion: the transpose of the matrix
// the free-flight section prints, which maps body vectors to the global frame
// (Sec. 3.6).
__host__ __device__ inline void quat_mbody(const double* e, double* M) {
    const double e0 = e[0], e1 = e[1], e2 = e[2], e3 = e[3];
    M[0] = e0 * e0 + e1 * e1 - e2 * e2 - e3 * e3;
    M[1] = 2.0 * (e1 * e2 + e3 * e0);
    M[2] = 2.0 * (e1 * e3 - e2 * e0);
    M[3] = 2.0 * (e1 * e2 - e3 * e0);
    M[4] = e0 * e0 - e1 * e1 + e2 * e2 - e3 * e3;
    M[5] = 2.0 * (e2 * e3 + e1 * e0);
    M[6] = 2.0 * (e1 * e3 + e2 * e0);
    M[7] = 2.0 * (e2 * e3 - e1 * e0);
    M[8] = e0 * e0 - e1 * e1 - e2 * e2 + e3 * e3;
}

// Quaternion of roll psi, pitch beta, yaw gamma (Sec. 3.6).
template <class TR = TrigEval>
__host__ __device__ inline void quat_of_angles(double psi, double beta, double gam, double* e, TR&& tr = TR{}) {
    const SinCos qp = tr(0.5 * psi), qb = tr(0.5 * beta), qg = tr(0.5 * gam);
    const double cp = qp.c, sp = qp.s, cb = qb.c, sb = qb.s, cg = qg.c, sg = qg.s;
    e[0] = cp * cb * cg + sp * sb * sg;
    e[1] = sp * cb * cg - cp * sb * sg;
    e[2] = cp * sb * cg + sp * cb * sg;
    e[3] = cp * cb * sg - sp * sb * cg;
}

// Right-hand side of the 13 free-flight equations (Sec. 3.6, eq.
// oh_my_god_look_a_vector).  y: x_cntr, u_cntr, eps, Omega^(b); F: total force
// and m: torque about x_cntr, both in the global frame.
__host__ __device__ inline void solid_rhs(const flusi_insect& in, const double* y, const double* F,
                                          const double* m, double* f) {
    double Mb[9], mb[3];
    quat_mbody(y + 6, Mb);
    mat_vec(Mb, m, mb);
    const double e0 = y[6], e1 = y[7], e2 = y[8], e3 = y[9];
    const double ox = y[10], oy = y[11], oz = y[12];
    const double Jx = in.inertia[0], Jy = in.inertia[1], Jz = in.inertia[2];
    for (int i = 0; i < 3; ++i) f[i] = y[3 + i];
    f[3] = F[0] / in.mass * in.dof[0];
    f[4] = F[1] / in.mass * in.dof[1];
    f[5] = (F[2] / in.mass - in.gravity) * in.dof[2];
    f[6] = 0.5 * (-e1 * ox - e2 * oy - e3 * oz);
    f[7] = 0.5 * (e0 * ox - e3 * oy + e2 * oz);
    f[8] = 0.5 * (e3 * ox + e0 * oy - e1 * oz);
    f[9] = 0.5 * (-e2 * ox + e1 * oy + e0 * oz);
    f[10] = ((Jy - Jz) * oy * oz + mb[0]) / Jx * in.dof[3];
    f[11] = ((Jz - Jx) * oz * ox + mb[1]) / Jy * in.dof[4];
    f[12] = ((Jx - Jy) * ox * oy + mb[2]) / Jz * in.dof[5];
}

// Wing angles phi, alpha, theta and their rates at time t (Sec. 3.3): the
// sinusoid, a Fourier series a_0/2 + sum a_i cos(2 pi i f t) + b_i sin(2 pi i f t),
// or periodic cubic Hermite interpolation of values and rates at kin_n
// equidistant times of a period; with acc, also the second derivatives (the
// Hermite cubic's within its interval).
template <class TR = TrigEval>
__host__ __device__ inline void wing_angle_values(const flusi_insect& in, double t, double* ang, double* rate,
                                                  TR&& tr = TR{}, double* acc = nullptr) {
    if (in.kin_type == FLUSI_KIN_FOURIER) {
        for (int a = 0; a < 3; ++a) {
            double v = 0.5 * in.kin_coef[a][0][0], dv = 0.0, d2v = 0.0;
            for (int i = 1; i <= in.kin_n; ++i) {
                const double w = 2.0 * M_PI * i * in.freq;
                const double ai = in.kin_coef[a][0][i], bi = in.kin_coef[a][1][i];
                const SinCos q = tr(w * t);
                const double c = q.c, sn = q.s;
                v += ai * c + bi * sn;
                dv += w * (-ai * sn + bi * c);
                d2v -= w * w * (ai * c + bi * sn);
            }
            ang[a] = v;
            rate[a] = dv;
            if (acc) acc[a] = d2v;
        }
    } else if (in.kin_type == FLUSI_KIN_HERMITE) {
        const int K = in.kin_n;
        const double T = 1.0 / in.freq, h = T / K;
        const double s = (t - floor(t / T) * T) / h;
        int j = (int)floor(s);
        if (j > K - 1) j = K - 1;
        if (j < 0) j = 0;
        const double u = s - j;
        const int j1 = (j + 1) % K;
        const double u2 = u * u, u3 = u2 * u;
        const double h00 = 2 * u3 - 3 * u2 + 1, h10 = u3 - 2 * u2 + u, h01 = -2 * u3 + 3 * u2, h11 = u3 - u2;
        const double d00 = 6 * u2 - 6 * u, d10 = 3 * u2 - 4 * u + 1, d01 = -6 * u2 + 6 * u, d11 = 3 * u2 - 2 * u;
        const double e00 = 12 * u - 6, e10 = 6 * u - 4, e01 = -12 * u + 6, e11 = 6 * u - 2;
        for (int a = 0; a < 3; ++a) {
            const double v0 = in.kin_coef[a][0][j], v1 = in.kin_coef[a][0][j1];
            const double m0 = in.kin_coef[a][1][j] * h, m1 = in.kin_coef[a][1][j1] * h;
            ang[a] = h00 * v0 + h10 * m0 + h01 * v1 + h11 * m1;
            rate[a] = (d00 * v0 + d10 * m0 + d01 * v1 + d11 * m1) / h;
            if (acc) acc[a] = (e00 * v0 + e10 * m0 + e01 * v1 + e11 * m1) / (h * h);
        }
    } else {
        const double om = 2.0 * M_PI * in.freq;
        const double* P[3] = {in.phi, in.alpha, in.theta};
        for (int a = 0; a < 3; ++a) {
            const double ph = om * t + P[a][2];
            const SinCos q = tr(ph);
            ang[a] = P[a][0] + P[a][1] * q.c;
            rate[a] = -P[a][1] * om * q.s;
            if (acc) acc[a] = -P[a][1] * om * om * q.c;
        }
    }
}

// Inertial power of a wing (Sec. 3.5): W . (J W' + W x J W), with W the
// wing's angular velocity in its own frame and J = {J_xx, J_yy, J_zz, J_xy,
// J_xz, J_yz} its inertia tensor there.  With A = Ry(alpha) and B = Rz(-theta)
// (the wing matrix is A B Rx(phi)), W = phi' A B e_x - theta' A e_z + alpha' e_y,
// so W' = phi'' A B e_x + phi' (alpha' A_a B e_x + theta' A (sin(-theta),
// cos(-theta), 0)) - theta'' A e_z - theta' alpha' A_a e_z + alpha'' e_y, with
// A_a = dRy/dalpha.
__host__ __device__ inline double wing_inertial_power(const double* Jw, const double* A, const double* B,
                                                      double dphi, double dal, double dth, double ddphi,
                                                      double ddal, double ddth) {
    const double bx[3] = {B[0], B[3], B[6]};  // B e_x
    double abx[3], abd[3];
    mat_vec(A, bx, abx);
    const double bd[3] = {B[1], B[0], 0.0};  // d(B e_x)/d(theta)
    mat_vec(A, bd, abd);
    const double az[3] = {A[2], A[5], A[8]};                                              // A e_z
    const double aabx[3] = {-A[6] * bx[0] - A[0] * bx[2], 0.0, A[0] * bx[0] - A[6] * bx[2]};  // A_a B e_x
    const double aaz[3] = {-A[0], 0.0, -A[6]};                                             // A_a e_z
    double W[3], Wd[3];
    for (int i = 0; i < 3; ++i) {
        W[i] = dphi * abx[i] - dth * az[i] + (i == 1 ? dal : 0.0);
        Wd[i] = ddphi * abx[i] + dphi * (dal * aabx[i] + dth * abd[i]) - ddth * az[i] - dth * dal * aaz[i] +
                (i == 1 ? ddal : 0.0);
    }
    const double J[9] = {Jw[0], Jw[3], Jw[4], Jw[3], Jw[1], Jw[5], Jw[4], Jw[5], Jw[2]};
    double JW[3], JWd[3];
    mat_vec(J, W, JW);
    mat_vec(J, Wd, JWd);
    const double g0 = W[1] * JW[2] - W[2] * JW[1], g1 = W[2] * JW[0] - W[0] * JW[2], g2 = W[0] * JW[1] - W[1] * JW[0];
    return W[0] * (JWd[0] + g0) + W[1] * (JWd[1] + g1) + W[2] * (JWd[2] + g2);
}

// Arguments of the sines and cosines that compute_kin evaluates, in its
// order: the body rotations and quaternion half angles (prescribed body
// motion), the angle series, then per wing the stroke plane, the half turn
// (right wing) and the three wing angles.  The wing angles come from the
// series: fill == 0 writes every other entry and flags these in dep; fill ==
// 1 writes only these, from the series values ang.  Returns the count (at
// most KIN_TRIG_MAX).
constexpr int KIN_TRIG_MAX = 6 + 3 * FLUSI_KIN_MAX + 9;
__device__ inline int kin_trig_args(const flusi_insect& in, double t, bool pose, int fill, const double* ang,
                                    double* arg, unsigned char* dep) {
    int n = 0;
    auto put = [&](double x, bool wing_angle) {
        if (n >= KIN_TRIG_MAX) return;  // only for a description the host would reject
        if (wing_angle == (fill == 1)) arg[n] = x;
        if (fill == 0) dep[n] = wing_angle ? 1 : 0;
        ++n;
    };
    if (!pose) {
        const double psi = in.psi + in.psi_dot * t;
        const double beta = in.beta + in.beta_dot * t;
        const double gam = in.gamma + in.gamma_dot * t;
        put(psi, false);
        put(beta, false);
        put(gam, false);
        put(0.5 * psi, false);
        put(0.5 * beta, false);
        put(0.5 * gam, false);
    }
    if (!in.wings) return n;
    if (in.kin_type == FLUSI_KIN_FOURIER) {
        for (int a = 0; a < 3; ++a)
            for (int i = 1; i <= in.kin_n; ++i) {
                const double w = 2.0 * M_PI * i * in.freq;
                put(w * t, false);
            }
    } else if (in.kin_type != FLUSI_KIN_HERMITE) {
        const double om = 2.0 * M_PI * in.freq;
        const double* P[3] = {in.phi, in.alpha, in.theta};
        for (int a = 0; a < 3; ++a) put(om * t + P[a][2], false);
    }
    for (int s = 0; s < 2; ++s) {
        const double sg = s == 0 ? 1.0 : -1.0;
        put(in.eta_stroke, false);
        if (s == 1) put(M_PI, false);
        put(fill ? sg * ang[1] : 0.0, true);
        put(fill ? -ang[2] : 0.0, true);
        put(fill ? sg * ang[0] : 0.0, true);
    }
    return n;
}

// Kinematics at time t (Sec. 3.1 and 3.3).  dx is the grid spacing.  pose
// (13 values: x_cntr, u_cntr, eps, Omega^(b)) replaces the prescribed body
// motion in free flight (Sec. 3.6); null for a tethered body.
// In three parts, which the device runs on different lanes: kin_body (the
// body, the outline and every field but the wing frames; returns the cull
// radius of the body parts about x_cntr), kin_wing (the frames, rates and
// reference point of wing s, from the wing angles; returns the cull radius
// that wing adds), kin_nowings.  The sines and cosines are requested in the
// order kin_trig_args lists them: kin_body's six, the angle series
// (wing_angle_values), then four for the left wing and five for the right.
template <class TR = TrigEval>
__host__ __device__ __forceinline__ double kin_body(const flusi_insect& in, double t, double dx, Kin& k,
                                                    const double* pose = nullptr, TR&& tr = TR{}) {
    if (pose) {
        for (int i = 0; i < 3; ++i) {
            k.xc[i] = pose[i];
            k.uc[i] = pose[3 + i];
            k.omb[i] = pose[10 + i];
        }
        for (int i = 0; i < 4; ++i) k.eps[i] = pose[6 + i];
        quat_mbody(pose + 6, k.Mb);
    } else {
        const double psi = in.psi + in.psi_dot * t;
        const double beta = in.beta + in.beta_dot * t;
        const double gam = in.gamma + in.gamma_dot * t;
        double Rx_[9], Ry_[9], Rz_[9], T1[9];
        mat_rx(psi, Rx_, tr);
        mat_ry(beta, Ry_, tr);
        mat_rz(gam, Rz_, tr);
        mat_mul(Rx_, Ry_, T1);
        mat_mul(T1, Rz_, k.Mb);
        // body angular velocity: Rz^T[(0,0,gd) + Ry^T[(0,bd,0) + Rx^T (pd,0,0)]], then to body frame
        double v[3] = {in.psi_dot, 0.0, 0.0}, w[3];
        mat_tvec(Rx_, v, w);
        w[1] += in.beta_dot;
        mat_tvec(Ry_, w, v);
        v[2] += in.gamma_dot;
        mat_tvec(Rz_, v, w);
        mat_vec(k.Mb, w, k.omb);
        quat_of_angles(psi, beta, gam, k.eps, tr);
        for (int i = 0; i < 3; ++i) {
            k.xc[i] = in.x_cntr[i];
            k.uc[i] = in.u_cntr[i];
        }
    }
    for (int i = 0; i < 3; ++i) k.xref[0][i] = k.xc[i];
    k.body = in.body;
    k.wings = in.wings;
    k.smooth = in.smooth;
    k.radius = in.radius;
    k.ea = in.a;
    k.eb = in.b;
    k.wA = in.wing_A;
    k.wB = in.wing_B;
    k.wt = in.wing_t;
    k.h = in.c_smth * dx;
    // chi is exactly 0 beyond delta = h (cosine) or delta = 20 h (tanh rounds to 1)
    k.thr = in.smooth == FLUSI_SMOOTH_TANH ? 20.0 * k.h : k.h;
    double rall = 0.0;
    if (in.body == FLUSI_BODY_SPHERE) rall = in.radius + k.thr;
    if (in.body == FLUSI_BODY_ELLIPSOID) rall = 2.0 * (in.a + in.b) + k.thr;
    // head and eye spheres of an ellipsoid body (Sec. 3.2): fixed slots head,
    // eye at +y, eye at -y; radius 0 marks an absent sphere
    {
        const bool ell = in.body == FLUSI_BODY_ELLIPSOID;
        const double hr = ell && in.head_r > 0.0 ? in.head_r : 0.0;
        const double er = ell && in.eye_r > 0.0 ? in.eye_r : 0.0;
        k.sph[0][0] = in.head_x[0]; k.sph[0][1] = in.head_x[1]; k.sph[0][2] = in.head_x[2]; k.sph[0][3] = hr;
        k.sph[1][0] = in.eye_x[0]; k.sph[1][1] = in.eye_x[1]; k.sph[1][2] = in.eye_x[2]; k.sph[1][3] = er;
        k.sph[2][0] = in.eye_x[0]; k.sph[2][1] = -in.eye_x[1]; k.sph[2][2] = in.eye_x[2]; k.sph[2][3] = er;
        k.nsph = (hr > 0.0 || er > 0.0) ? 3 : 0;
        for (int q = 0; q < 3; ++q)
            if (k.sph[q][3] > 0.0)
                rall = fmax(rall, sqrt(k.sph[q][0] * k.sph[q][0] + k.sph[q][1] * k.sph[q][1] + k.sph[q][2] * k.sph[q][2]) +
                                      k.sph[q][3] + k.thr);
    }
    // wing outline: centre in the wing plane and an outer radius about it
    k.wshape = in.wing_shape;
    if (in.wing_shape == FLUSI_WING_FOURIER) {
        k.wcen[0] = in.wing_c[0];
        k.wcen[1] = in.wing_c[1];
        double rb = fabs(0.5 * in.wing_coef[0][0]);  // |R| <= |a_0|/2 + sum |(a_i, b_i)|
        for (int i = 1; i <= in.wing_n; ++i) rb += sqrt(in.wing_coef[0][i] * in.wing_coef[0][i] +
                                                         in.wing_coef[1][i] * in.wing_coef[1][i]);
        k.wrad = rb;
    } else if (in.wing_shape == FLUSI_WING_RECT) {
        // rectangle about its centre: half chord and half span in wA, wB
        const double a = in.wing_rect[0], tip = in.wing_rect[1], b = in.wing_rect[2], B = in.wing_rect[3];
        k.wcen[0] = b - 0.5 * B;
        k.wcen[1] = 0.5 * (a + tip);
        k.wA = 0.5 * B;
        k.wB = 0.5 * (tip - a);
        // delta = max(|ex| - wA, |ey| - wB) stays below thr only inside the box
        // widened by thr, whose circumscribed circle has radius wrad + thr
        // (wrad grows with thr, so the FP64 cut-off also covers the FP32 one)
        k.wrad = sqrt((k.wA + k.thr) * (k.wA + k.thr) + (k.wB + k.thr) * (k.wB + k.thr)) - k.thr;
    } else {
        k.wcen[0] = 0.0;
        k.wcen[1] = in.wing_B;
        k.wrad = fmax(in.wing_A, in.wing_B);
    }
    k.rtab = nullptr;
    k.rtab32 = nullptr;
    return rall;
}

__host__ __device__ inline void kin_nowings(Kin& k) {
    // no wings: identity wing frames, zero rates, reference points at the centre
    for (int s = 0; s < 2; ++s) {
        for (int i = 0; i < 9; ++i) k.Mws[s][i] = (i % 4 == 0) ? 1.0 : 0.0;
        for (int i = 0; i < 3; ++i) {
            k.piv[s][i] = 0.0;
            k.omw[s][i] = 0.0;
            k.xref[1 + s][i] = k.xc[i];
        }
        k.pinert[s] = 0.0;
    }
}

// wing s (0 left, 1 right) from the wing angles ang, their rates and second
// derivatives; inert: the wings have a tensor of inertia
template <class TR = TrigEval>
__host__ __device__ __forceinline__ double kin_wing(const flusi_insect& in, Kin& k, int s, const double* ang,
                                                    const double* rate, const double* acc, bool inert,
                                                    TR&& tr = TR{}) {
    const double phi0 = ang[0], dphi0 = rate[0], al0 = ang[1], dal0 = rate[1], th = ang[2], dth = rate[2];
    const double sg = s == 0 ? 1.0 : -1.0;  // right wing: alpha and phi mirrored
    const double phi = sg * phi0, dphi = sg * dphi0, al = sg * al0, dal = sg * dal0;
    double Ms[9], Mw[9], A[9], B[9], C[9];
    mat_ry(in.eta_stroke, Ms, tr);
    if (s == 1) {
        double Rpi[9];
        mat_rx(M_PI, Rpi, tr);
        mat_mul(Rpi, Ms, Ms);
    }
    mat_ry(al, A, tr);
    mat_rz(-th, B, tr);
    mat_rx(phi, C, tr);
    mat_mul(A, B, Mw);
    mat_mul(Mw, C, Mw);
    mat_mul(Mw, Ms, k.Mws[s]);
    // stroke-frame angular velocity: Rx^T(phi)[(dphi,0,0) + Rz^T(-th)[(0,0,-dth) + Ry^T(al)(0,dal,0)]]
    double a1[3] = {0.0, dal, 0.0}, a2[3];
    mat_tvec(A, a1, a2);
    a2[2] -= dth;
    mat_tvec(B, a2, a1);
    a1[0] += dphi;
    mat_tvec(C, a1, a2);
    mat_tvec(Ms, a2, k.omw[s]);
    k.pinert[s] = inert ? wing_inertial_power(in.wing_J, A, B, dphi, dal, dth, sg * acc[0], sg * acc[1], acc[2])
                        : 0.0;
    const double* pv = s == 0 ? in.pivot_l : in.pivot_r;
    for (int i = 0; i < 3; ++i) k.piv[s][i] = pv[i];
    double pg[3];
    mat_tvec(k.Mb, pv, pg);
    for (int i = 0; i < 3; ++i) k.xref[1 + s][i] = k.xc[i] + pg[i];
    const double e1 = k.wrad + k.thr, e2 = 0.5 * in.wing_t + k.thr;
    const double pn = sqrt(pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2]);
    const double cn = sqrt(k.wcen[0] * k.wcen[0] + k.wcen[1] * k.wcen[1]);
    return pn + cn + sqrt(e1 * e1 + e2 * e2);
}

__host__ __device__ inline bool wings_inert(const flusi_insect& in) {
    bool inert = false;
    for (int i = 0; i < 6; ++i) inert = inert || in.wing_J[i] != 0.0;
    return inert;
}

template <class TR = TrigEval>
__host__ __device__ __forceinline__ void compute_kin(const flusi_insect& in, double t, double dx, Kin& k,
                                                     const double* pose = nullptr, TR&& tr = TR{}) {
    double rall = kin_body(in, t, dx, k, pose, tr);
    if (!in.wings) {
        kin_nowings(k);
        k.r2all = rall * rall;
        return;
    }
    double ang[3], rate[3], acc[3];
    wing_angle_values(in, t, ang, rate, tr, acc);
    const bool inert = wings_inert(in);
    for (int s = 0; s < 2; ++s) rall = fmax(rall, kin_wing(in, k, s, ang, rate, acc, inert, tr));
    k.r2all = rall * rall;
}

// Copy of the kinematics in the precision the mask is evaluated in (FP64 for
// the FP64 path; FP32 for the FP32 path, whose fields are FP32 anyway).
template <typename TM>
struct KinT {
    TM Mb[9], xc[3], uc[3], omb[3], Mws[2][9], piv[2][3], omw[2][3], xref[3][3];
    TM r2all, thr, h, radius, ea, eb, wA, wB, wt;
    TM r2b;          // squared radius about xc outside which the body's chi == 0
    TM wc[2][3];     // wing outline centres (global frame)
    TM r2w;          // squared radius about wc outside which a wing's chi == 0
    TM wcx, wcy, wrad;  // outline centre in the wing plane, outer radius about it
    TM sph[3][4];       // body spheres: centre (body frame), radius
    const TM* rtab;     // Fourier wing radius table in this precision
    int body, wings, smooth, wshape, nsph, pad;
};

// FP32 tanh reaches 1 near 9.01 and FP64 tanh near 19.06: beyond these
// multiples of h the tanh mask is exactly zero in that precision.
template <typename TM>
__device__ __forceinline__ TM tanh_cut() { return sizeof(TM) == 4 ? TM(10) : TM(20); }

// The conversion in two parts: the 69 array elements (Mb, xc, uc, omb; Mws,
// piv, omw; xref; sph), which the lanes of a wave share (element e on lane
// e mod nl), and the rest with the cull radii (one lane).
template <typename TM>
__device__ inline void kin_cast_arrays(const Kin& a, KinT<TM>& b, int lane, int nl) {
    // runs of arrays that are contiguous in both layouts
    static_assert(offsetof(Kin, xc) == offsetof(Kin, Mb) + 9 * sizeof(double) &&
                      offsetof(Kin, omb) == offsetof(Kin, Mb) + 15 * sizeof(double) &&
                      offsetof(Kin, omw) == offsetof(Kin, Mws) + 24 * sizeof(double) &&
                      offsetof(KinT<TM>, xc) == offsetof(KinT<TM>, Mb) + 9 * sizeof(TM) &&
                      offsetof(KinT<TM>, omb) == offsetof(KinT<TM>, Mb) + 15 * sizeof(TM) &&
                      offsetof(KinT<TM>, Mws) == offsetof(KinT<TM>, Mb) + 18 * sizeof(TM) &&
                      offsetof(KinT<TM>, omw) == offsetof(KinT<TM>, Mws) + 24 * sizeof(TM),
                  "contiguous kinematics arrays");
    const char* pa = reinterpret_cast<const char*>(&a);
    char* pb = reinterpret_cast<char*>(&b);
    for (int e = lane; e < 69; e += nl) {
        size_t oa, ob;
        int o;
        if (e < 18) { oa = offsetof(Kin, Mb); ob = offsetof(KinT<TM>, Mb); o = e; }
        else if (e < 48) { oa = offsetof(Kin, Mws); ob = offsetof(KinT<TM>, Mws); o = e - 18; }
        else if (e < 57) { oa = offsetof(Kin, xref); ob = offsetof(KinT<TM>, xref); o = e - 48; }
        else { oa = offsetof(Kin, sph); ob = offsetof(KinT<TM>, sph); o = e - 57; }
        reinterpret_cast<TM*>(pb + ob)[o] = TM(reinterpret_cast<const double*>(pa + oa)[o]);
    }
}

template <typename TM>
__device__ inline void kin_cast_rest(const Kin& a, KinT<TM>& b) {
    b.h = TM(a.h);
    b.radius = TM(a.radius); b.ea = TM(a.ea); b.eb = TM(a.eb);
    b.wA = TM(a.wA); b.wB = TM(a.wB); b.wt = TM(a.wt);
    b.body = a.body; b.wings = a.wings; b.smooth = a.smooth; b.pad = 0;
    b.wshape = a.wshape; b.nsph = a.nsph;
    b.wcx = TM(a.wcen[0]); b.wcy = TM(a.wcen[1]); b.wrad = TM(a.wrad);
    if constexpr (sizeof(TM) == 4) b.rtab = reinterpret_cast<const TM*>(a.rtab32);
    else b.rtab = reinterpret_cast<const TM*>(a.rtab);
    // cull radius recomputed for the precision's own tanh cut-off
    const double thr = a.smooth == FLUSI_SMOOTH_TANH ? (sizeof(TM) == 4 ? 10.0 : 20.0) * a.h : a.h;
    b.thr = TM(thr);
    // Culls (chi == 0 exactly beyond them), widened by a relative margin so they
    // stay conservative after rounding:
    //  body: sphere delta = |r| - R; ellipsoid: if |r|^2 > (a+thr)^2 + (b+thr)^2
    //        then |x_b| > a + thr or rho > b + thr, and either way delta > thr
    //  wing: the in-plane outline radius is at most wrad (ellipse: max(A, B)),
    //        so beyond a distance sqrt((wrad+thr)^2 + (t/2+thr)^2) from the
    //        outline centre either r - R > thr or |z_w| - t/2 > thr
    //  body spheres: beyond |c| + r + thr from the body centre
    double rb2 = 0.0;
    if (a.body == FLUSI_BODY_SPHERE) rb2 = (a.radius + thr) * (a.radius + thr);
    if (a.body == FLUSI_BODY_ELLIPSOID) rb2 = (a.ea + thr) * (a.ea + thr) + (a.eb + thr) * (a.eb + thr);
    for (int q = 0; q < 3; ++q) {
        // a sphere's distance exceeds thr beyond |c| + r + thr from the body centre
        if (!(a.sph[q][3] > 0.0)) continue;
        const double e = sqrt(a.sph[q][0] * a.sph[q][0] + a.sph[q][1] * a.sph[q][1] + a.sph[q][2] * a.sph[q][2]) +
                         a.sph[q][3] + thr;
        rb2 = fmax(rb2, e * e);
    }
    b.r2b = TM(rb2 * (1.0 + 1e-5));
    double rall = sqrt(rb2);
    const double e1 = a.wrad + thr, e2 = 0.5 * a.wt + thr;
    const double rw = sqrt(e1 * e1 + e2 * e2);
    b.r2w = TM(rw * rw * (1.0 + 1e-5));
    for (int s = 0; s < 2; ++s) {
        // outline centre (cx, cy, 0) of the wing frame: body frame piv + (M_wing M_stroke)^T (cx, cy, 0)
        double cb[3], cg[3];
        for (int i = 0; i < 3; ++i) cb[i] = a.piv[s][i] + a.Mws[s][i] * a.wcen[0] + a.Mws[s][3 + i] * a.wcen[1];
        mat_tvec(a.Mb, cb, cg);
        for (int i = 0; i < 3; ++i) b.wc[s][i] = TM(a.xc[i] + cg[i]);
        if (a.wings) rall = fmax(rall, sqrt(cg[0] * cg[0] + cg[1] * cg[1] + cg[2] * cg[2]) + rw);
    }
    b.r2all = TM(rall * rall * (1.0 + 1e-5));
}

template <typename TM>
__device__ inline void kin_cast(const Kin& a, KinT<TM>& b) {
    kin_cast_arrays(a, b, 0, 1);
    kin_cast_rest(a, b);
}

template <typename TM>
__device__ __forceinline__ TM chi_of(TM delta, const KinT<TM>& k) {
    if (k.smooth == FLUSI_SMOOTH_TANH) return TM(0.5) * (TM(1) - tanh(delta / k.h));
    if (delta <= -k.h) return TM(1);
    if (delta >= k.h) return TM(0);
    return TM(0.5) * (TM(1) + cos(TM(M_PI) * (delta + k.h) / (TM(2) * k.h)));
}

template <typename TM>
struct MaskPt {
    TM chi;
    TM us[3];
    int colour;
};

template <typename TM>
__device__ __forceinline__ void mvec(const TM* A, const TM* v, TM* o) {
    const TM a = A[0] * v[0] + A[1] * v[1] + A[2] * v[2];
    const TM b = A[3] * v[0] + A[4] * v[1] + A[5] * v[2];
    const TM c = A[6] * v[0] + A[7] * v[1] + A[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}
template <typename TM>
__device__ __forceinline__ void mtvec(const TM* A, const TM* v, TM* o) {
    const TM a = A[0] * v[0] + A[3] * v[1] + A[6] * v[2];
    const TM b = A[1] * v[0] + A[4] * v[1] + A[7] * v[2];
    const TM c = A[2] * v[0] + A[5] * v[1] + A[8] * v[2];
    o[0] = a; o[1] = b; o[2] = c;
}
template <typename TM>
__device__ __forceinline__ void cross(const TM* a, const TM* b, TM* o) {
    const TM x = a[1] * b[2] - a[2] * b[1];
    const TM y = a[2] * b[0] - a[0] * b[2];
    const TM z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}

// Relative tolerance under which two part values count as a tie: a later part
// replaces the current one only if its chi is larger by more than this, so ties
// (including values equal up to rounding, e.g. both wings on the mirror plane
// of a symmetric insect) go to the lowest colour.
constexpr double TIE_REL = 1e-9;

// Polar radius of a Fourier wing at in-plane offset (ex, ey) from its centre
// (Sec. 3.4): angle in turns, linear interpolation in the table.  Out of line:
// only wing points reach it, and inlined atan2 would set the register count of
// the whole physical-space pass.
template <typename TM>
__device__ __attribute__((noinline)) TM table_radius(const TM* tab, TM ex, TM ey) {
    TM v = atan2(ey, ex) / TM(2.0 * M_PI);
    if (v < TM(0)) v += TM(1);
    const TM pos = v * TM(FLUSI_RTABLE);
    int j = (int)floor(pos);
    j = j < 0 ? 0 : (j > FLUSI_RTABLE - 1 ? FLUSI_RTABLE - 1 : j);
    const TM f = pos - TM(j);
    return (TM(1) - f) * tab[j] + f * tab[j + 1];
}

// chi of each part (body, left wing, right wing; 0 where absent or culled) and
// the body-frame coordinates of the point.
template <typename TM>
__device__ __forceinline__ void part_chis(const KinT<TM>& k, TM x, TM y, TM z, TM (&c)[3], TM (&xb)[3]) {
    c[0] = c[1] = c[2] = TM(0);
    const TM rel[3] = {x - k.xc[0], y - k.xc[1], z - k.xc[2]};
    const TM r2 = rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2];
    mvec(k.Mb, rel, xb);
    if (r2 > k.r2b) {
        // outside the body's cull sphere: chi_body == 0
    } else if (k.body == FLUSI_BODY_SPHERE) {
        c[0] = chi_of(sqrt(r2) - k.radius, k);
    } else if (k.body == FLUSI_BODY_ELLIPSOID) {
        const TM q = xb[0] / k.ea;
        const TM rad = sqrt(xb[1] * xb[1] + xb[2] * xb[2]);
        TM d = fmax(rad - k.eb * sqrt(fmax(TM(0), TM(1) - q * q)), fabs(xb[0]) - k.ea);
        // head and eyes: union with the thorax (Sec. 3.2)
        if (k.nsph) {
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                if (!(k.sph[p][3] > TM(0))) continue;
                const TM s0 = xb[0] - k.sph[p][0], s1 = xb[1] - k.sph[p][1], s2 = xb[2] - k.sph[p][2];
                d = fmin(d, sqrt(s0 * s0 + s1 * s1 + s2 * s2) - k.sph[p][3]);
            }
        }
        c[0] = chi_of(d, k);
    }
    if (k.wings) {
        for (int s = 0; s < 2; ++s) {
            const TM g0 = x - k.wc[s][0], g1 = y - k.wc[s][1], g2 = z - k.wc[s][2];
            if (g0 * g0 + g1 * g1 + g2 * g2 > k.r2w) continue;  // outside the wing's cull sphere: chi == 0
            const TM d0[3] = {xb[0] - k.piv[s][0], xb[1] - k.piv[s][1], xb[2] - k.piv[s][2]};
            TM xw[3];
            mvec(k.Mws[s], d0, xw);
            const TM dz = fabs(xw[2]) - TM(0.5) * k.wt;
            const TM ex = xw[0] - k.wcx, ey = xw[1] - k.wcy;
            const TM r = sqrt(ex * ex + ey * ey);
            if (dz >= k.thr || r - k.wrad >= k.thr) continue;  // chi == 0 exactly
            TM inplane;
            if (k.wshape == FLUSI_WING_FOURIER) {
                inplane = r - table_radius<TM>(k.rtab, ex, ey);
            } else if (k.wshape == FLUSI_WING_RECT) {
                inplane = fmax(fabs(ex) - k.wA, fabs(ey) - k.wB);
            } else {
                const TM qa = ex / k.wA, qb = ey / k.wB;
                const TM rho = sqrt(qa * qa + qb * qb);
                inplane = r > TM(0) ? r - r / rho : -k.wA;
            }
            const TM cw = chi_of(fmax(dz, inplane), k);
            if (s == 0) c[1] = cw;
            else c[2] = cw;
        }
    }
}

// Part that supplies u_s and the colour (parts in colour order, ties to the
// lowest).
template <typename TV>
__device__ __forceinline__ int part_of_max(const TV (&c)[3]) {
    int part = 0;
    TV best = c[0];
    if (c[1] > best * TV(1.0 + TIE_REL)) {
        part = 1;
        best = c[1];
    }
    if (c[2] > best * TV(1.0 + TIE_REL)) part = 2;
    return part;
}

// Part choice in FP64 at a point where two parts overlap.  Out of line: the
// FP64 geometry is rare and would otherwise set the register count of the
// FP32 kernels that call eval_mask.
__device__ __attribute__((noinline)) int part_of_max64(const KinT<double>* k64, double x, double y, double z) {
    double c64[3], xb64[3];
    part_chis(*k64, x, y, z, c64, xb64);
    return part_of_max(c64);
}

// chi, u_s and colour at the grid point with global coordinates (x, y, z).
// Reads only the kinematics blocks (kept in LDS by the callers).  With TM =
// float, k64 (the FP64 kinematics) decides the part wherever two parts
// overlap, so the integer part choice is taken in FP64 as in the FP64 path.
//
// defer != nullptr: where two parts overlap, set *defer and return an empty
// point instead of deciding (the caller revisits such points with k64).
template <typename TM>
__device__ __forceinline__ MaskPt<TM> eval_mask(const KinT<TM>& k, double x, double y, double z,
                                                const KinT<double>* k64, bool* defer = nullptr) {
    MaskPt<TM> o;
    o.chi = TM(0);
    o.us[0] = o.us[1] = o.us[2] = TM(0);
    o.colour = 0;
    const TM xt = TM(x), yt = TM(y), zt = TM(z);
    {
        const TM r0 = xt - k.xc[0], r1 = yt - k.xc[1], r2c = zt - k.xc[2];
        if (r0 * r0 + r1 * r1 + r2c * r2c > k.r2all) return o;
    }
    TM c[3], xb[3];
    part_chis(k, xt, yt, zt, c, xb);
    const TM chimax = fmax(c[0], fmax(c[1], c[2]));
    if (chimax <= TM(0)) return o;
    int part;
    const bool overlap = (int(c[0] > TM(0)) + int(c[1] > TM(0)) + int(c[2] > TM(0))) >= 2;
    if (overlap && defer != nullptr) {
        *defer = true;
        return o;
    }
    if (overlap && k64 != nullptr) {
        part = part_of_max64(k64, x, y, z);
    } else {
        part = part_of_max(c);
    }
    o.chi = chimax;
    o.colour = part + 1;
    // u_b = u_cntr + Mb^T (omb x x_b)
    TM cr[3], ub[3];
    cross(k.omb, xb, cr);
    mtvec(k.Mb, cr, ub);
    for (int i = 0; i < 3; ++i) ub[i] += k.uc[i];
    if (part == 0) {
        o.us[0] = ub[0]; o.us[1] = ub[1]; o.us[2] = ub[2];
    } else {
        const int s = part - 1;
        const TM d0[3] = {xb[0] - k.piv[s][0], xb[1] - k.piv[s][1], xb[2] - k.piv[s][2]};
        TM uw[3];
        cross(k.omw[s], d0, cr);
        mtvec(k.Mb, cr, uw);
        o.us[0] = uw[0] + ub[0]; o.us[1] = uw[1] + ub[1]; o.us[2] = uw[2] + ub[2];
    }
    return o;
}

}  // namespace flusi
