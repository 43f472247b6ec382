// gv_field.h -- magnetic field maps and Runge-Kutta integration of charged
// tracks in them (Sec. 3.6: field evaluation at the track's points, the
// Lorentz force, one Runge-Kutta step with an error estimate, and the
// accept / retry / next-step-size decision around it).
//
// Field maps: uniform B, or a finite solenoid along z (coil radius R,
// half-length L, central field B0): on the axis a uniform current sheet gives
// g(z) = B0 f(z)/f(0), f(z) = (z+L)/sqrt(R^2+(z+L)^2) - (z-L)/sqrt(R^2+(z-L)^2);
// off the axis the field is expanded to second order in r,
// B_r = -(r/2) g', B_z = g - (r^2/4) g''.
//
// Equation of motion in path length s for a unit direction u:
//   dx/ds = u,  du/ds = (q kKB / p) u x B(x).
#pragma once
#include "gv_common.h"
#include "gv_geom.h"
#include "gv_physics.h"

namespace gv {

enum : int { kMapUniform = 0, kMapSolenoid = 1 };
enum : int { kFieldHelix = 0, kFieldRk4 = 1, kFieldRk45 = 2 };

// Field at a point, in precision R.  sol_c = B0 / f(0) and sol_R2 = R^2 are
// formed once on the host.
template <class R> __device__ __forceinline__ void field_at(const DevGeom& g, const double x[3], R B[3])
{
#pragma clang fp contract(off)
    if (g.field_map != kMapSolenoid) {
        B[0] = (R)g.B[0];
        B[1] = (R)g.B[1];
        B[2] = (R)g.B[2];
        return;
    }
    const R R2 = (R)g.sol_R2, L = (R)g.sol_L, c = (R)g.sol_c;
    const R z = (R)x[2];
    const R a = z + L, b = z - L;
    const R sa = m_sqrt(R2 + a * a), sb = m_sqrt(R2 + b * b);
    // 1/sqrt(R^2 + a^2) and 1/sqrt(R^2 + b^2) from one division
    const R r = (R)1 / (sa * sb);
    const R ia = sb * r, ib = sa * r;
    const R ia2 = ia * ia, ib2 = ib * ib;
    const R ia3 = ia2 * ia, ib3 = ib2 * ib;
    const R g0 = c * (a * ia - b * ib);
    const R g1 = c * R2 * (ia3 - ib3);
    const R g2 = (R)-3 * c * R2 * (a * (ia3 * ia2) - b * (ib3 * ib2));
    const R px = (R)x[0], py = (R)x[1];
    const R r2 = px * px + py * py;
    B[0] = (R)-0.5 * px * g1;
    B[1] = (R)-0.5 * py * g1;
    B[2] = g0 - (R)0.25 * r2 * g2;
}

template <class R> __device__ __forceinline__ void lorentz(R kq, const R B[3], const R u[3], R out[3])
{
#pragma clang fp contract(off)
    out[0] = kq * (u[1] * B[2] - u[2] * B[1]);
    out[1] = kq * (u[2] * B[0] - u[0] * B[2]);
    out[2] = kq * (u[0] * B[1] - u[1] * B[0]);
}

// Classic RK4 with the field taken at each stage point (non-uniform maps), in
// double whatever the precision policy: the turning angle of a long step is
// the integral of the curvature, so any rounding of q kKB |B| / p to float
// would turn into a phase error proportional to the angle.
__device__ inline void rk4_map_move(const DevGeom& g, int type, double T, double s, int nsub, double pos[3],
                                    double u[3])
{
#pragma clang fp contract(off)
    const double q = type == kElectron ? -1.0 : 1.0;
    const double p = sqrt(T * (T + 2.0 * kMe));
    const double kq = q * kKB / p;
    const double h = s / nsub;
    for (int i = 0; i < nsub; ++i) {
        double B[3], k1[3], k2[3], k3[3], k4[3], u2[3], u3[3], u4[3], xs[3];
        field_at<double>(g, pos, B);
        lorentz<double>(kq, B, u, k1);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u2[a] = u[a] + 0.5 * h * k1[a];
            xs[a] = pos[a] + 0.5 * h * u[a];
        }
        field_at<double>(g, xs, B);
        lorentz<double>(kq, B, u2, k2);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u3[a] = u[a] + 0.5 * h * k2[a];
            xs[a] = pos[a] + 0.5 * h * u2[a];
        }
        field_at<double>(g, xs, B);
        lorentz<double>(kq, B, u3, k3);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            u4[a] = u[a] + h * k3[a];
            xs[a] = pos[a] + h * u3[a];
        }
        field_at<double>(g, xs, B);
        lorentz<double>(kq, B, u4, k4);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            pos[a] += h / 6.0 * (u[a] + 2.0 * u2[a] + 2.0 * u3[a] + u4[a]);
            u[a] += h / 6.0 * (k1[a] + 2.0 * k2[a] + 2.0 * k3[a] + k4[a]);
        }
    }
    normalise(u);
}

// Dormand & Prince (1980) RK5(4)7M.  Row i of the stage matrix (i = 1..6);
// row 6 equals the 5th-order weights, so stage 6 is the derivative at the new
// point and becomes stage 0 of the next substep.  kDpE = 5th- minus embedded
// 4th-order weights.
constexpr double kDpA[7][6] = {
    {0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0, 0.0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0.0, 0.0, 0.0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0.0, 0.0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0.0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
constexpr double kDpE[7] = {35.0 / 384.0 - 5179.0 / 57600.0,
                            0.0,
                            500.0 / 1113.0 - 7571.0 / 16695.0,
                            125.0 / 192.0 - 393.0 / 640.0,
                            -2187.0 / 6784.0 - -92097.0 / 339200.0,
                            11.0 / 84.0 - 187.0 / 2100.0,
                            0.0 - 1.0 / 40.0};

// Per-lane tally of one adaptive integration.
struct RkTally {
    int acc;    // accepted substeps
    int rej;    // rejected attempts
    int iters;  // loop iterations the lane's wavefront ran (lane slots)
};

// Error constant of the pair on circular motion: for a small turning angle
// theta = h |du/ds| the error measure below is about kDpK theta^4.
constexpr double kDpK = 8.1e-4;

// Adaptive Dormand-Prince 5(4) over the path length s, in double whatever the
// precision policy (see rk4_map_move).  Error of a substep of length h: the
// larger of max_a |sum_j e_j kx_j[a]| (position error per unit length) and
// max_a |h sum_j e_j ku_j[a]| (direction error); accepted when <= tol.
// First attempt: h = min(s, theta / |du/ds|), theta = 0.8 (tol / kDpK)^(1/4).
// Next h: halved after a rejected attempt, doubled after an accepted substep
// with error <= tol/16, cut to end exactly at s; powers of two keep every
// substep length an exact function of s and theta.  After max_sub attempts
// the integration stops.  Stage sums run in stage order as fused
// multiply-adds (zero coefficients skipped), as does the stage point
// y + h sum.
//
// The integration is written as a state and one attempt at a time, so that
// a lane can run one track's attempts inside its own loop (rk45_move) or
// take attempts of whichever integration it holds from a shared queue (the
// batched driver's integration kernel): both run the same arithmetic.  The
// first stage derivative of an attempt is the direction itself (dx/ds = u),
// and first-same-as-last carries the Lorentz term ku0 of the accepted end
// point into the next attempt.
struct Rk45State {
    double x[3], u[3], ku0[3];
    double done, h, s, kq;
    int acc, rej;
    bool busy;
};

__device__ inline void rk45_begin(const DevGeom& g, int type, double T, double s, double tol, const double pos[3],
                                  const double u[3], Rk45State& st)
{
#pragma clang fp contract(off)
    st.acc = 0;
    st.rej = 0;
    st.done = 0.0;
    st.s = s;
    st.busy = s > 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st.x[a] = pos[a];
        st.u[a] = u[a];
    }
    if (!st.busy) return;
    const double q = type == kElectron ? -1.0 : 1.0;
    const double p = sqrt(T * (T + 2.0 * kMe));
    st.kq = q * kKB / p;
    {
        double B[3];
        field_at<double>(g, st.x, B);
        lorentz<double>(st.kq, B, st.u, st.ku0);
    }
    st.h = s;
    {
        const double w = sqrt(st.ku0[0] * st.ku0[0] + st.ku0[1] * st.ku0[1] + st.ku0[2] * st.ku0[2]);
        const double theta = 0.8 * sqrt(sqrt(tol / kDpK));
        if (st.h * w > theta) st.h = theta / w;
    }
}

// one attempt of a busy integration; clears busy when it is done
__device__ inline void rk45_attempt(const DevGeom& g, double tol, int max_sub, Rk45State& st)
{
#pragma clang fp contract(off)
    double kx[7][3], ku[7][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        kx[0][a] = st.u[a];
        ku[0][a] = st.ku0[a];
    }
    const double rem = st.s - st.done;
    const bool last = st.h >= rem;
    double h = last ? rem : st.h;
    double xs[3], us[3];
#pragma unroll
    for (int i = 1; i < 7; ++i) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double sx = kDpA[i][0] * kx[0][a];
            double su = kDpA[i][0] * ku[0][a];
#pragma unroll
            for (int j = 1; j < i; ++j) {
                if (kDpA[i][j] != 0.0) {
                    sx = fma(kDpA[i][j], kx[j][a], sx);
                    su = fma(kDpA[i][j], ku[j][a], su);
                }
            }
            xs[a] = fma(h, sx, st.x[a]);
            us[a] = fma(h, su, st.u[a]);
        }
        double B[3];
        field_at<double>(g, xs, B);
#pragma unroll
        for (int a = 0; a < 3; ++a) kx[i][a] = us[a];
        lorentz<double>(st.kq, B, us, ku[i]);
    }
    // xs, us: the 5th-order solution (the last stage point)
    double err = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double ex = kDpE[0] * kx[0][a];
#pragma unroll
        for (int j = 2; j < 7; ++j) ex = fma(kDpE[j], kx[j][a], ex);
        if (fabs(ex) > err) err = fabs(ex);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double eu = kDpE[0] * ku[0][a];
#pragma unroll
        for (int j = 2; j < 7; ++j) eu = fma(kDpE[j], ku[j][a], eu);
        eu = h * eu;
        if (fabs(eu) > err) err = fabs(eu);
    }
    if (err <= tol) {
        st.acc += 1;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st.x[a] = xs[a];
            st.u[a] = us[a];
            st.ku0[a] = ku[6][a];
        }
        if (last) {
            st.done = st.s;
            st.h = h;
            st.busy = false;
        } else {
            st.done += h;
            st.h = h;
            if (err <= tol * (1.0 / 16.0)) st.h *= 2.0;
        }
    } else {
        st.rej += 1;
        st.h = h * 0.5;
    }
    if (st.acc + st.rej >= max_sub) st.busy = false;
}

// One track's whole integration on its own lane.  The loop runs while any
// lane of the wavefront still integrates, each lane working only while it has
// work: every lane then knows how many iterations its wavefront spent, which
// gives the idle-lane statistic.  Returns the length integrated (s unless
// attempts ran out); pos and u (normalised) are updated.
__device__ inline double rk45_move(const DevGeom& g, int type, double T, double s, double tol, int max_sub,
                                   double pos[3], double u[3], RkTally& tally)
{
#pragma clang fp contract(off)
    tally.acc = 0;
    tally.rej = 0;
    tally.iters = 0;
    if (!(s > 0.0)) return 0.0;
    Rk45State st;
    rk45_begin(g, type, T, s, tol, pos, u, st);
    while (__any(st.busy)) {
        tally.iters += 1;
        if (st.busy) rk45_attempt(g, tol, max_sub, st);
    }
    tally.acc = st.acc;
    tally.rej = st.rej;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pos[a] = st.x[a];
        u[a] = st.u[a];
    }
    normalise(u);
    return st.done;
}

}  // namespace gv
