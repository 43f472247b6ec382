/*
 * Oracle kinematics (test infrastructure only): charged-particle motion in a
 * magnetic field (Sec. 3.6: exact helix in the field at the start point,
 * classic 4th-order Runge-Kutta, or adaptive Dormand-Prince 5(4), on
 * du/ds = (q kB / p) u x B(x), dx/ds = u), direction rotation,
 * Highland multiple scattering, and the final-state samplers of Sec. 3.5 by
 * composition-rejection.
 *
 * Rejection iteration j of an interaction draws the block
 * (event, tid, step, FS0 + j) and uses its four words as 32-bit uniforms
 * u0..u3, so a history does not depend on how many other tracks share a
 * basket or how many iterations they needed.
 *
 * Sampler outputs (out[4]):
 *   compton: eps = k'/k, cos(theta_gamma), phi, sin^2(theta_gamma)
 *   pair:    x = E-/k, phi_minus, -, -
 *   brems:   k (photon energy), -, -, -
 *   moller/bhabha: eps = T_delta/T, phi, -, -
 */
#include "or_internal.h"

/* ---------------- field ---------------- */

static double charge_of(int32_t type) { return type == OR_ELECTRON ? -1.0 : 1.0; }

void or_helix_move(int32_t type, double ekin, const double B[3], double s, double pos[3], double dir[3])
{
    double Bm = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    double p = sqrt(ekin * (ekin + 2.0 * OR_ME));
    double b[3] = {B[0] / Bm, B[1] / Bm, B[2] / Bm};
    double upar = dir[0] * b[0] + dir[1] * b[1] + dir[2] * b[2];
    double uperp[3] = {dir[0] - upar * b[0], dir[1] - upar * b[1], dir[2] - upar * b[2]};
    double bxu[3] = {b[1] * uperp[2] - b[2] * uperp[1], b[2] * uperp[0] - b[0] * uperp[2],
                     b[0] * uperp[1] - b[1] * uperp[0]};
    double th = -(charge_of(type) * OR_KB * Bm / p) * s;
    double sn = sin(th), hs = sin(0.5 * th);
    double omc = 2.0 * hs * hs;  /* 1 - cos(theta) */
    double cs = 1.0 - omc;
    double f1, f2;               /* sin(t)/t and (1-cos t)/t */
    if (fabs(th) < 1.0e-4) {
        f1 = 1.0 - th * th / 6.0;
        f2 = 0.5 * th;
    } else {
        f1 = sn / th;
        f2 = omc / th;
    }
    for (int a = 0; a < 3; ++a) {
        pos[a] += s * (upar * b[a] + f1 * uperp[a] + f2 * bxu[a]);
        dir[a] = upar * b[a] + cs * uperp[a] + sn * bxu[a];
    }
    double nn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    dir[0] /= nn;
    dir[1] /= nn;
    dir[2] /= nn;
}

static void lorentz(double kq, const double B[3], const double u[3], double out[3])
{
    out[0] = kq * (u[1] * B[2] - u[2] * B[1]);
    out[1] = kq * (u[2] * B[0] - u[0] * B[2]);
    out[2] = kq * (u[0] * B[1] - u[1] * B[0]);
}

/* Field of a finite solenoid along z (coil radius R, half-length L, central
 * field B0).  On the axis a uniform current sheet gives
 *   g(z) = B0 f(z) / f(0),  f(z) = (z+L)/sqrt(R^2+(z+L)^2) - (z-L)/sqrt(R^2+(z-L)^2);
 * off the axis the axisymmetric field is expanded to second order in r:
 *   B_r = -(r/2) g'(z),  B_z = g(z) - (r^2/4) g''(z),
 * which has zero curl exactly and a divergence of order r^2 g'''. */
static void solenoid_field(double B0, double R, double L, const double x[3], double out[3])
{
    double R2 = R * R;
    double f0 = 2.0 * L / sqrt(R2 + L * L);
    double c = B0 / f0;
    double a = x[2] + L, b = x[2] - L;
    double qa = R2 + a * a, qb = R2 + b * b;
    double sa = sqrt(qa), sb = sqrt(qb);
    double g = c * (a / sa - b / sb);
    double g1 = c * R2 * (1.0 / (qa * sa) - 1.0 / (qb * sb));               /* g'  */
    double g2 = -3.0 * c * R2 * (a / (qa * qa * sa) - b / (qb * qb * sb));  /* g'' */
    double r2 = x[0] * x[0] + x[1] * x[1];
    out[0] = -0.5 * x[0] * g1;
    out[1] = -0.5 * x[1] * g1;
    out[2] = g - 0.25 * r2 * g2;
}

void or_field_eval(const or_field* f, const double x[3], double B[3])
{
    if (f->map == OR_MAP_SOLENOID) {
        solenoid_field(f->B[2], f->sol[0], f->sol[1], x, B);
    } else {
        B[0] = f->B[0];
        B[1] = f->B[1];
        B[2] = f->B[2];
    }
}

void or_rk4_field_move(int32_t type, double ekin, const or_field* f, double s, int32_t nsub,
                       double pos[3], double dir[3])
{
    double p = sqrt(ekin * (ekin + 2.0 * OR_ME));
    double kq = charge_of(type) * OR_KB / p;
    double h = s / nsub;
    for (int i = 0; i < nsub; ++i) {
        double k1u[3], k2u[3], k3u[3], k4u[3], u2[3], u3[3], u4[3], x2[3], x3[3], x4[3];
        double B1[3], B2[3], B3[3], B4[3];
        /* dx/ds = u: the position stages are the u stages */
        or_field_eval(f, pos, B1);
        lorentz(kq, B1, dir, k1u);
        for (int a = 0; a < 3; ++a) {
            u2[a] = dir[a] + 0.5 * h * k1u[a];
            x2[a] = pos[a] + 0.5 * h * dir[a];
        }
        or_field_eval(f, x2, B2);
        lorentz(kq, B2, u2, k2u);
        for (int a = 0; a < 3; ++a) {
            u3[a] = dir[a] + 0.5 * h * k2u[a];
            x3[a] = pos[a] + 0.5 * h * u2[a];
        }
        or_field_eval(f, x3, B3);
        lorentz(kq, B3, u3, k3u);
        for (int a = 0; a < 3; ++a) {
            u4[a] = dir[a] + h * k3u[a];
            x4[a] = pos[a] + h * u3[a];
        }
        or_field_eval(f, x4, B4);
        lorentz(kq, B4, u4, k4u);
        for (int a = 0; a < 3; ++a) {
            pos[a] += h / 6.0 * (dir[a] + 2.0 * u2[a] + 2.0 * u3[a] + u4[a]);
            dir[a] += h / 6.0 * (k1u[a] + 2.0 * k2u[a] + 2.0 * k3u[a] + k4u[a]);
        }
    }
    double nn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    dir[0] /= nn;
    dir[1] /= nn;
    dir[2] /= nn;
}

void or_rk4_move(int32_t type, double ekin, const double B[3], double s, int32_t nsub,
                 double pos[3], double dir[3])
{
    or_field f = {OR_MAP_UNIFORM, 0, {B[0], B[1], B[2]}, {0.0, 0.0}};
    or_rk4_field_move(type, ekin, &f, s, nsub, pos, dir);
}

/* Dormand & Prince (1980), RK5(4)7M: rows of the stage matrix, the 5th-order
 * weights (equal to the last row, so the last stage is the derivative at the
 * new point) and the embedded 4th-order weights. */
static const double DP_A[7][6] = {
    {0.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0, 0.0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0.0, 0.0, 0.0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0.0, 0.0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0.0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
static const double DP_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0,
                               -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double DP_BH[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0,
                                -92097.0 / 339200.0, 187.0 / 2100.0, 1.0 / 40.0};
static const double DP_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};

void or_dp45_tableau(double* a, double* b, double* bh, double* c)
{
    for (int i = 0; i < 7; ++i) {
        for (int j = 0; j < 7; ++j) a[7 * i + j] = j < 6 ? DP_A[i][j] : 0.0;
        b[i] = DP_B[i];
        bh[i] = DP_BH[i];
        c[i] = DP_C[i];
    }
}

/* One stage derivative of y = (x, u): dx/ds = u, du/ds = kq u x B(x). */
static void dp_deriv(const or_field* f, double kq, const double y[6], double k[6])
{
    double B[3];
    or_field_eval(f, y, B);
    k[0] = y[3];
    k[1] = y[4];
    k[2] = y[5];
    lorentz(kq, B, y + 3, k + 3);
}

/* Adaptive Dormand-Prince integration of the equation of motion over the
 * path length s (Sec. 3.6: a Runge-Kutta step with an error estimate, then
 * the accept / retry / next-size decision).
 *   error measure of a substep of length h, with e = b - bh:
 *     err = max( max_a |sum_j e_j kx_j[a]|,  max_a |h sum_j e_j ku_j[a]| )
 *   (position error per unit length, and direction error); accepted when
 *   err <= tol.
 *   first attempt: h = min(s, theta / |du/ds|) with theta =
 *   0.8 (tol / RK45_K)^(1/4), where RK45_K is the constant of this pair's
 *   error measure on circular motion (err ~ RK45_K (h |du/ds|)^4 for small
 *   turning angles);
 *   next h: halved after a rejected attempt, doubled after an accepted
 *   substep with err <= tol/16 (the position part scales as h^4), never past
 *   the end of the interval.  Powers of two keep every substep length an
 *   exact function of s and theta, so any two IEEE implementations take the
 *   same substeps.  Stops after max_sub attempts.  Stage sums are the plain
 *   sums of the tableau rows, in stage order. */
#define RK45_K 8.1e-4
int32_t or_rk45_move(int32_t type, double ekin, const or_field* f, double s, double tol,
                     int32_t max_sub, double pos[3], double dir[3], double* s_done, int32_t* n_rej)
{
    double p = sqrt(ekin * (ekin + 2.0 * OR_ME));
    double kq = charge_of(type) * OR_KB / p;
    double y[6] = {pos[0], pos[1], pos[2], dir[0], dir[1], dir[2]};
    double done = 0.0, h = s;
    int32_t acc = 0, rej = 0;
    *s_done = 0.0;
    *n_rej = 0;
    if (!(s > 0.0)) return 0;
    {
        double k0[6];
        dp_deriv(f, kq, y, k0);
        double w = sqrt(k0[3] * k0[3] + k0[4] * k0[4] + k0[5] * k0[5]);
        double theta = 0.8 * sqrt(sqrt(tol / RK45_K));
        if (h * w > theta) h = theta / w;
    }
    while (acc + rej < max_sub) {
        double rem = s - done;
        int last = h >= rem;
        if (last) h = rem;
        double k[7][6], yi[6];
        dp_deriv(f, kq, y, k[0]);
        for (int i = 1; i < 7; ++i) {
            for (int c = 0; c < 6; ++c) {
                double sum = 0.0;
                for (int j = 0; j < i; ++j) sum += DP_A[i][j] * k[j][c];
                yi[c] = y[c] + h * sum;
            }
            dp_deriv(f, kq, yi, k[i]);
        }
        /* yi now holds the 5th-order solution (the last row equals DP_B) */
        double err = 0.0;
        for (int c = 0; c < 6; ++c) {
            double e = 0.0;
            for (int j = 0; j < 7; ++j) e += (DP_B[j] - DP_BH[j]) * k[j][c];
            if (c >= 3) e = h * e;
            if (fabs(e) > err) err = fabs(e);
        }
        if (err <= tol) {
            ++acc;
            for (int c = 0; c < 6; ++c) y[c] = yi[c];
            if (last) {
                done = s;
                break;
            }
            done += h;
            if (err <= tol * (1.0 / 16.0)) h *= 2.0;
        } else {
            ++rej;
            h *= 0.5;
        }
    }
    double nn = sqrt(y[3] * y[3] + y[4] * y[4] + y[5] * y[5]);
    for (int a = 0; a < 3; ++a) {
        pos[a] = y[a];
        dir[a] = y[3 + a] / nn;
    }
    *s_done = done;
    *n_rej = rej;
    return acc;
}

/* ---------------- rotation and MSC ---------------- */

/* turn dir by polar angle theta (given as cos, sin) and azimuth phi about itself */
void or_rotate(double u[3], double ct, double st, double phi)
{
    double e1[3], e2[3];
    double up = sqrt(u[0] * u[0] + u[1] * u[1]);
    if (up > 0.0) {
        e1[0] = u[0] * u[2] / up;
        e1[1] = u[1] * u[2] / up;
        e1[2] = -up;
        e2[0] = -u[1] / up;
        e2[1] = u[0] / up;
        e2[2] = 0.0;
    } else {
        e1[0] = 1.0; e1[1] = 0.0; e1[2] = 0.0;
        e2[0] = 0.0; e2[1] = (u[2] >= 0.0) ? 1.0 : -1.0; e2[2] = 0.0;
    }
    double cp = cos(phi), sp = sin(phi);
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = ct * u[a] + st * (cp * e1[a] + sp * e2[a]);
    double nn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    u[0] = v[0] / nn;
    u[1] = v[1] / nn;
    u[2] = v[2] / nn;
}

/* Highland width of the projected angle (PDG form with the logarithmic term) */
double or_highland(int32_t m, double ekin, double s)
{
    double E = ekin + OR_ME;
    double p = sqrt(ekin * (ekin + 2.0 * OR_ME));
    double beta = p / E;
    double x = s / G.X0[m];
    double corr = 1.0 + 0.038 * log(x / (beta * beta));
    if (corr < 0.0) corr = 0.0;
    return 13.6 / (beta * p) * sqrt(x) * corr;
}

/* ---------------- final states ---------------- */

static void fs_block(uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, int j, double u[4])
{
    uint32_t w[4];
    or_stream(seed, event, tid, nstep, OR_PURP_FS0 + (uint32_t)j, w);
    for (int i = 0; i < 4; ++i) u[i] = or_u32(w[i]);
}

/* Klein-Nishina by the Butcher-Messel composition: eps from 1/eps on
 * [eps0, exp(-a1)] or from eps on [eps0, 1], accepted with 1 - eps sin^2/(1+eps^2) */
int or_sample_compton(double kMeV, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double k = kMeV / OR_ME;
    double eps0 = 1.0 / (1.0 + 2.0 * k);
    double a1 = -log(eps0);
    double a2 = 0.5 * (1.0 - eps0 * eps0);
    double eps = 1.0, cost = 1.0, phi = 0.0, sin2 = 0.0;
    int j;
    for (j = 0; j < OR_FS_MAX_ITER; ++j) {
        double u[4];
        fs_block(seed, event, tid, nstep, j, u);
        if (u[0] * (a1 + a2) < a1) eps = exp(-a1 * u[1]);
        else eps = sqrt(eps0 * eps0 + (1.0 - eps0 * eps0) * u[1]);
        double t = (1.0 - eps) / (k * eps);
        sin2 = t * (2.0 - t);
        cost = 1.0 - t;
        phi = 2.0 * OR_PI * u[3];
        if (u[2] <= 1.0 - eps * sin2 / (1.0 + eps * eps)) break;
    }
    out[0] = eps;
    out[1] = cost;
    out[2] = phi;
    out[3] = sin2;
    return j < OR_FS_MAX_ITER ? j + 1 : -OR_FS_MAX_ITER;
}

/* pair: x uniform on [a, 1-a] accepted with 1 - 4/3 x(1-x) */
int or_sample_pair(double k, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double a = OR_ME / k, b = 1.0 - a;
    double x = 0.5, phi = 0.0;
    int j;
    for (j = 0; j < OR_FS_MAX_ITER; ++j) {
        double u[4];
        fs_block(seed, event, tid, nstep, j, u);
        x = a + (b - a) * u[0];
        phi = 2.0 * OR_PI * u[2];
        if (u[1] <= 1.0 - (4.0 / 3.0) * x * (1.0 - x)) break;
    }
    out[0] = x;
    out[1] = phi;
    out[2] = out[3] = 0.0;
    return j < OR_FS_MAX_ITER ? j + 1 : -OR_FS_MAX_ITER;
}

/* bremsstrahlung: k from 1/k on [k_cut, T], accepted with 1 - y + 3/4 y^2, y = k/E */
int or_sample_brems(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double kc = G.cfg.k_cut;
    double E = T + OR_ME;
    double k = kc;
    int j;
    for (j = 0; j < OR_FS_MAX_ITER; ++j) {
        double u[4];
        fs_block(seed, event, tid, nstep, j, u);
        k = kc * pow(T / kc, u[0]);
        double y = k / E;
        if (u[1] <= 1.0 - y + 0.75 * y * y) break;
    }
    out[0] = k;
    out[1] = out[2] = out[3] = 0.0;
    return j < OR_FS_MAX_ITER ? j + 1 : -OR_FS_MAX_ITER;
}

/* Moller: eps from 1/eps^2 on [ec, 1/2], accepted with eps^2 [dcs bracket] / (2 + g1/4) */
int or_sample_moller(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double E = T + OR_ME, g = E / OR_ME;
    double g1 = ((g - 1.0) / g) * ((g - 1.0) / g);
    double g2 = (2.0 * g - 1.0) / (g * g);
    double ec = G.cfg.t_cut / T;
    double H = 2.0 + 0.25 * g1;
    double eps = ec, phi = 0.0;
    int j;
    for (j = 0; j < OR_FS_MAX_ITER; ++j) {
        double u[4];
        fs_block(seed, event, tid, nstep, j, u);
        eps = ec / (1.0 - u[0] * (1.0 - ec / 0.5));
        double f = g1 * eps * eps + 1.0 + eps * eps / ((1.0 - eps) * (1.0 - eps)) - g2 * eps / (1.0 - eps);
        phi = 2.0 * OR_PI * u[2];
        if (u[1] * H <= f) break;
    }
    out[0] = eps;
    out[1] = phi;
    out[2] = out[3] = 0.0;
    return j < OR_FS_MAX_ITER ? j + 1 : -OR_FS_MAX_ITER;
}

/* Bhabha: eps from 1/eps^2 on [ec, 1], accepted with eps^2 [dcs bracket] beta^2 */
int or_sample_bhabha(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double E = T + OR_ME, g = E / OR_ME;
    double b2 = 1.0 - 1.0 / (g * g);
    double y = 1.0 / (g + 1.0);
    double B1 = 2.0 - y * y;
    double B2 = (1.0 - 2.0 * y) * (3.0 + y * y);
    double B4 = (1.0 - 2.0 * y) * (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double B3 = B4 + (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double ec = G.cfg.t_cut / T;
    double eps = ec, phi = 0.0;
    int j;
    for (j = 0; j < OR_FS_MAX_ITER; ++j) {
        double u[4];
        fs_block(seed, event, tid, nstep, j, u);
        eps = ec / (1.0 - u[0] * (1.0 - ec));
        double f = 1.0 / b2 - B1 * eps + B2 * eps * eps - B3 * eps * eps * eps + B4 * eps * eps * eps * eps;
        phi = 2.0 * OR_PI * u[2];
        if (u[1] * (1.0 / b2) <= f) break;
    }
    out[0] = eps;
    out[1] = phi;
    out[2] = out[3] = 0.0;
    return j < OR_FS_MAX_ITER ? j + 1 : -OR_FS_MAX_ITER;
}
