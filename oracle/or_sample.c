/*
 * Oracle kinematics (test infrastructure only): charged-particle motion in a
 * uniform magnetic field (Sec. 3.6: exact helix, or classic 4th-order
 * Runge-Kutta on du/ds = (q kB / p) u x B, dx/ds = u), direction rotation,
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

void or_rk4_move(int32_t type, double ekin, const double B[3], double s, int32_t nsub,
                 double pos[3], double dir[3])
{
    double p = sqrt(ekin * (ekin + 2.0 * OR_ME));
    double kq = charge_of(type) * OR_KB / p;
    double h = s / nsub;
    for (int i = 0; i < nsub; ++i) {
        double k1u[3], k2u[3], k3u[3], k4u[3], u2[3], u3[3], u4[3];
        lorentz(kq, B, dir, k1u);
        for (int a = 0; a < 3; ++a) u2[a] = dir[a] + 0.5 * h * k1u[a];
        lorentz(kq, B, u2, k2u);
        for (int a = 0; a < 3; ++a) u3[a] = dir[a] + 0.5 * h * k2u[a];
        lorentz(kq, B, u3, k3u);
        for (int a = 0; a < 3; ++a) u4[a] = dir[a] + h * k3u[a];
        lorentz(kq, B, u4, k4u);
        for (int a = 0; a < 3; ++a) {
            /* dx/ds = u: the position stages are the u stages */
            pos[a] += h / 6.0 * (dir[a] + 2.0 * u2[a] + 2.0 * u3[a] + u4[a]);
            dir[a] += h / 6.0 * (k1u[a] + 2.0 * k2u[a] + 2.0 * k3u[a] + k4u[a]);
        }
    }
    double nn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    dir[0] /= nn;
    dir[1] /= nn;
    dir[2] /= nn;
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
