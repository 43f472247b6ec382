// gv_physics.h -- EM physics on the device (Sec. 3.5 model set, in textbook
// closed forms): table lookup, the cross-section and stopping-power formulas
// the table builder evaluates, composition-rejection final-state samplers,
// Highland multiple scattering, direction rotation and charged-particle
// motion in a uniform field (Sec. 3.6).
#pragma once
#include "gv_common.h"

namespace gv {

struct DevMat {
    double n_el;       // electrons / cm^3
    double X0;         // cm
    double I;          // MeV
    double hwp;        // plasma energy, MeV
};

struct DevPhys {
    int n_nodes;
    int n_mats;
    int field_method;
    int pad;
    double e_min, bpd, log10_emin;
    double t_cut, k_cut, t_track;
    double chord_tol, push, rk_frac;
    long long max_steps;
    DevMat mat[16];
    double r_track[16][2];   // range at the tracking cut, per material, e-/e+
    float r_track_f[16][2];
};

// Table access for one precision: records of kCols values per
// (material, particle type, node), node energies, range-inverse index.
template <class R> struct TabView {
    const R* rec;      // [(m*3 + type) * n_nodes + i] * kCols + col
    const R* E;        // node energies
    int n;
};

template <class R>
__device__ __forceinline__ int find_bin(const TabView<R>& tv, R T, double log10_emin, double bpd)
{
    int i = (int)m_floor((m_log10(T) - (R)log10_emin) * (R)bpd);
    i = i < 0 ? 0 : (i > tv.n - 2 ? tv.n - 2 : i);
    while (i > 0 && T < tv.E[i]) --i;
    while (i < tv.n - 2 && T >= tv.E[i + 1]) ++i;
    return i;
}

// interpolate columns (c0, c1) of one record pair at bin i
template <class R>
__device__ __forceinline__ R lerp_col(const TabView<R>& tv, const R* base, int i, int col, R w)
{
    const R y0 = base[i * kCols + col], y1 = base[(i + 1) * kCols + col];
    return y0 + (y1 - y0) * w;
}

template <class R>
__device__ __forceinline__ const R* tab_base(const TabView<R>& tv, int m, int type)
{
    return tv.rec + (size_t)(m * 3 + type) * tv.n * kCols;
}

// inverse of the linearly interpolated range: the kinetic energy at range r
template <class R>
__device__ inline R range_inverse(const TabView<R>& tv, const R* base, R r)
{
    const int n = tv.n;
    if (r <= base[3]) return tv.E[0] * r / base[3];
    int lo = 0, hi = n - 1;
    if (r >= base[(n - 1) * kCols + 3]) {
        lo = n - 2;
    } else {
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (base[mid * kCols + 3] <= r) lo = mid;
            else hi = mid;
        }
    }
    const R r0 = base[lo * kCols + 3], r1 = base[(lo + 1) * kCols + 3];
    return tv.E[lo] + (tv.E[lo + 1] - tv.E[lo]) * (r - r0) / (r1 - r0);
}

// ---------------------------------------------------------------------------
// FP64 formulas evaluated by the table builder (per material m)
// ---------------------------------------------------------------------------

// Klein-Nishina per electron (cm^2); Taylor series about Thomson below k = 0.01 m
__device__ inline double xs_kn_per_electron(double kMeV)
{
    const double k = kMeV / kMe;
    if (k < 0.01) {
        const double c[9] = {1.0, -2.0, 26.0 / 5.0, -133.0 / 10.0, 1144.0 / 35.0, -544.0 / 7.0,
                             3784.0 / 21.0, -6148.0 / 15.0, 151552.0 / 165.0};
        double acc = c[8];
        for (int n = 7; n >= 0; --n) acc = acc * k + c[n];
        return (8.0 * kPi * kRe * kRe / 3.0) * acc;
    }
    const double l = log(1.0 + 2.0 * k);
    const double q = 1.0 + 2.0 * k;
    return 2.0 * kPi * kRe * kRe *
           (((1.0 + k) / (k * k)) * (2.0 * (1.0 + k) / q - l / k) + l / (2.0 * k) - (1.0 + 3.0 * k) / (q * q));
}

__device__ inline double xs_pair(const DevMat& M, double k)
{
    if (k <= 2.0 * kMe) return 0.0;
    const double a = kMe / k, b = 1.0 - a;
    return ((b - a) - (2.0 / 3.0) * (b * b - a * a) + (4.0 / 9.0) * (b * b * b - a * a * a)) / M.X0;
}

__device__ inline double xs_brems(const DevMat& M, double T, double kc)
{
    if (T <= kc) return 0.0;
    const double E = T + kMe;
    return ((4.0 / 3.0) * log(T / kc) - (4.0 / 3.0) * (T - kc) / E + (T * T - kc * kc) / (2.0 * E * E)) / M.X0;
}

__device__ inline double xs_moller(const DevMat& M, double T, double tc)
{
    if (T <= 2.0 * tc) return 0.0;
    const double g = (T + kMe) / kMe;
    const double b2 = 1.0 - 1.0 / (g * g);
    const double g1 = ((g - 1.0) / g) * ((g - 1.0) / g);
    const double g2 = (2.0 * g - 1.0) / (g * g);
    const double e = tc / T;
    const double br = g1 * (0.5 - e) + 1.0 / e - 1.0 / (1.0 - e) - g2 * log((1.0 - e) / e);
    return M.n_el * 2.0 * kPi * kRe * kRe * kMe / (b2 * T) * br;
}

__device__ inline double xs_bhabha(const DevMat& M, double T, double tc)
{
    if (T <= tc) return 0.0;
    const double g = (T + kMe) / kMe;
    const double b2 = 1.0 - 1.0 / (g * g);
    const double y = 1.0 / (g + 1.0);
    const double x = 1.0 - 2.0 * y;
    const double B1 = 2.0 - y * y, B2 = x * (3.0 + y * y), B4 = x * x * x, B3 = B4 + x * x;
    const double e = tc / T;
    const double br = (1.0 / b2) * (1.0 / e - 1.0) - B1 * log(1.0 / e) + B2 * (1.0 - e) -
                      0.5 * B3 * (1.0 - e * e) + (B4 / 3.0) * (1.0 - e * e * e);
    return M.n_el * 2.0 * kPi * kRe * kRe * kMe / T * br;
}

// restricted collision + sub-threshold radiative stopping power (MeV/cm)
__device__ inline double dedx_total(const DevMat& M, double T, bool positron, double tc, double kc)
{
    const double tau = T / kMe, g = tau + 1.0;
    const double b2 = 1.0 - 1.0 / (g * g);
    const double Im = M.I / kMe;
    double F;
    if (!positron) {
        const double d = fmin(tc, 0.5 * T) / kMe;
        F = -1.0 - b2 + log((tau - d) * d) + tau / (tau - d) +
            (0.5 * d * d + (2.0 * tau + 1.0) * log(1.0 - d / tau)) / (g * g);
    } else {
        const double d = fmin(tc, T) / kMe;
        const double y = 1.0 / (g + 1.0);
        const double d2 = d * d, d3 = d2 * d, d4 = d3 * d;
        F = log(tau * d) - (b2 / tau) * (tau + 2.0 * d - 1.5 * d2 * y - (d - d3 / 3.0) * y * y -
                                         (0.5 * d2 - tau * d3 / 3.0 + 0.25 * d4) * y * y * y);
    }
    const double bg = sqrt(T * (T + 2.0 * kMe)) / kMe;
    double delta = 2.0 * log(bg) + 2.0 * log(M.hwp / M.I) - 1.0;
    delta = delta > 0.0 ? delta : 0.0;
    const double col = 2.0 * kPi * kRe * kRe * kMe * M.n_el / b2 * (log(2.0 * (tau + 2.0) / (Im * Im)) + F - delta);
    const double E = T + kMe;
    const double K = fmin(kc, T);
    const double rad = ((4.0 / 3.0) * K - (2.0 / 3.0) * K * K / E + K * K * K / (3.0 * E * E)) / M.X0;
    return col + rad;
}

// ---------------------------------------------------------------------------
// Direction rotation: turn u by polar angle (cos, sin) and azimuth phi about
// itself, then renormalise.
// ---------------------------------------------------------------------------
template <class R> __device__ inline void rotate(R u[3], R ct, R st, R phi)
{
    const R up = m_sqrt(u[0] * u[0] + u[1] * u[1]);
    R e1[3], e2[3];
    if (up > (R)0) {
        e1[0] = u[0] * u[2] / up;
        e1[1] = u[1] * u[2] / up;
        e1[2] = -up;
        e2[0] = -u[1] / up;
        e2[1] = u[0] / up;
        e2[2] = (R)0;
    } else {
        e1[0] = (R)1; e1[1] = (R)0; e1[2] = (R)0;
        e2[0] = (R)0; e2[1] = u[2] >= (R)0 ? (R)1 : (R)-1; e2[2] = (R)0;
    }
    const R cp = m_cos(phi), sp = m_sin(phi);
    R v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = ct * u[a] + st * (cp * e1[a] + sp * e2[a]);
    const R inv = (R)1 / m_sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = v[a] * inv;
}

template <class R> __device__ __forceinline__ void normalise(R u[3])
{
    const R inv = (R)1 / m_sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    u[0] *= inv;
    u[1] *= inv;
    u[2] *= inv;
}

// Highland width of the projected scattering angle
template <class R> __device__ __forceinline__ R highland(R T, R s, R X0)
{
    const R E = T + (R)kMe;
    const R p = m_sqrt(T * (T + (R)(2.0 * kMe)));
    const R beta = p / E;
    const R x = s / X0;
    R corr = (R)1 + (R)0.038 * m_log(x / (beta * beta));
    corr = corr < (R)0 ? (R)0 : corr;
    return (R)13.6 / (beta * p) * m_sqrt(x) * corr;
}

// ---------------------------------------------------------------------------
// Final-state samplers: iteration j draws block (event, tid, step, FS0 + j);
// its four words are 32-bit uniforms.  After kFsMaxIter iterations the last
// candidate is kept and the exhaustion is counted.
// ---------------------------------------------------------------------------
struct Key {
    uint64_t seed;
    uint64_t tid;
    uint32_t event;
    uint32_t nstep;
};

template <class R> struct FS4 {
    R u[4];
};

template <class R> __device__ __forceinline__ FS4<R> fs_uniforms(const Key& k, uint32_t j)
{
    const U4 b = stream_block(k.seed, k.event, k.tid, k.nstep, kPurpFs0 + j);
    FS4<R> f;
#pragma unroll
    for (int i = 0; i < 4; ++i) f.u[i] = u32<R>(b.w[i]);
    return f;
}

// Klein-Nishina (Butcher-Messel): eps = k'/k, om = 1 - eps (formed without
// cancellation), t = 1 - cos(theta)
template <class R> __device__ inline bool sample_compton(R kMeV, const Key& key, R& eps, R& om, R& t, R& phi)
{
    const R k = kMeV / (R)kMe;
    const R e0 = (R)1 / ((R)1 + (R)2 * k);
    const R a1 = -m_log(e0);
    const R e02 = e0 * e0;
    const R a2 = (R)0.5 * ((R)1 - e02);
    for (uint32_t j = 0; j < kFsMaxIter; ++j) {
        const FS4<R> f = fs_uniforms<R>(key, j);
        if (f.u[0] * (a1 + a2) < a1) {
            eps = m_exp(-a1 * f.u[1]);
            om = -m_expm1(-a1 * f.u[1]);
        } else {
            eps = m_sqrt(e02 + ((R)1 - e02) * f.u[1]);
            om = ((R)1 - e02) * ((R)1 - f.u[1]) / ((R)1 + eps);
        }
        t = om / (k * eps);
        phi = (R)(2.0 * kPi) * f.u[3];
        if (f.u[2] <= (R)1 - eps * (t * ((R)2 - t)) / ((R)1 + eps * eps)) return true;
    }
    return false;
}

// pair: x = E-/k uniform on [m/k, 1 - m/k], accepted with 1 - 4/3 x(1-x)
template <class R> __device__ inline bool sample_pair(R k, const Key& key, R& x, R& phi)
{
    const R a = (R)kMe / k, w = (R)1 - (R)2 * a;
    for (uint32_t j = 0; j < kFsMaxIter; ++j) {
        const FS4<R> f = fs_uniforms<R>(key, j);
        x = a + w * f.u[0];
        phi = (R)(2.0 * kPi) * f.u[2];
        if (f.u[1] <= (R)1 - (R)(4.0 / 3.0) * x * ((R)1 - x)) return true;
    }
    return false;
}

// bremsstrahlung: k on [kc, T] from 1/k, accepted with 1 - y + 3/4 y^2
template <class R> __device__ inline bool sample_brems(R T, R kc, const Key& key, R& k)
{
    const R E = T + (R)kMe;
    const R ratio = T / kc;
    for (uint32_t j = 0; j < kFsMaxIter; ++j) {
        const FS4<R> f = fs_uniforms<R>(key, j);
        k = kc * m_pow(ratio, f.u[0]);
        const R y = k / E;
        if (f.u[1] <= (R)1 - y + (R)0.75 * y * y) return true;
    }
    return false;
}

// Moller: eps on [tc/T, 1/2] from 1/eps^2, bound 2 + g1/4
template <class R> __device__ inline bool sample_moller(R T, R tc, const Key& key, R& eps, R& phi)
{
    const R g = (T + (R)kMe) / (R)kMe;
    const R g1 = ((g - (R)1) / g) * ((g - (R)1) / g);
    const R g2 = ((R)2 * g - (R)1) / (g * g);
    const R ec = tc / T;
    const R H = (R)2 + (R)0.25 * g1;
    const R span = (R)1 - ec / (R)0.5;
    for (uint32_t j = 0; j < kFsMaxIter; ++j) {
        const FS4<R> f = fs_uniforms<R>(key, j);
        eps = ec / ((R)1 - f.u[0] * span);
        const R om = (R)1 - eps;
        const R val = g1 * eps * eps + (R)1 + eps * eps / (om * om) - g2 * eps / om;
        phi = (R)(2.0 * kPi) * f.u[2];
        if (f.u[1] * H <= val) return true;
    }
    return false;
}

// Bhabha: eps on [tc/T, 1] from 1/eps^2, bound 1/beta^2
template <class R> __device__ inline bool sample_bhabha(R T, R tc, const Key& key, R& eps, R& phi)
{
    const R g = (T + (R)kMe) / (R)kMe;
    const R b2 = (R)1 - (R)1 / (g * g);
    const R y = (R)1 / (g + (R)1);
    const R x = (R)1 - (R)2 * y;
    const R B1 = (R)2 - y * y, B2 = x * ((R)3 + y * y), B4 = x * x * x, B3 = B4 + x * x;
    const R ec = tc / T;
    const R ib2 = (R)1 / b2;
    for (uint32_t j = 0; j < kFsMaxIter; ++j) {
        const FS4<R> f = fs_uniforms<R>(key, j);
        eps = ec / ((R)1 - f.u[0] * ((R)1 - ec));
        const R val = ib2 - B1 * eps + B2 * eps * eps - B3 * eps * eps * eps + B4 * eps * eps * eps * eps;
        phi = (R)(2.0 * kPi) * f.u[2];
        if (f.u[1] * ib2 <= val) return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Uniform field.  Helix by arc length s (exact); RK4 on du/ds = (q kB/p) u x B,
// dx/ds = u with n equal substeps.  Position accumulates in double; the
// increment and the direction are computed in the policy's precision.
// ---------------------------------------------------------------------------
template <class R>
__device__ inline void helix_move(int type, R T, const double Bhat[3], double kB, double s, double pos[3], R u[3])
{
#pragma clang fp contract(off)
    // The turning angle is formed and reduced to [-pi, pi] in double so that
    // long steps keep their phase; trigonometry of the reduced angle and the
    // direction update run in the policy's precision.  kB = kKB |B| and
    // Bhat = B / |B| are formed once at set-up (q kKB |B| is the same double
    // either way, q being +-1).
    const double q = type == kElectron ? -1.0 : 1.0;
    const double Td = (double)T;
    const double p = sqrt(Td * (Td + 2.0 * kMe));
    const double th = -(q * kB / p) * s;
    const double thr = sizeof(R) == sizeof(double) ? th : th - 2.0 * kPi * rint(th * (0.5 / kPi));
    const R b[3] = {(R)Bhat[0], (R)Bhat[1], (R)Bhat[2]};
    const R upar = u[0] * b[0] + u[1] * b[1] + u[2] * b[2];
    const R up[3] = {u[0] - upar * b[0], u[1] - upar * b[1], u[2] - upar * b[2]};
    const R bxu[3] = {b[1] * up[2] - b[2] * up[1], b[2] * up[0] - b[0] * up[2], b[0] * up[1] - b[1] * up[0]};
    const R sn = m_sin((R)thr), hs = m_sin((R)(0.5 * thr));
    const R omc = (R)2 * hs * hs;  // 1 - cos
    R f1, f2;                      // sin(th)/th and (1 - cos th)/th
    if (fabs(th) < 1.0e-4) {
        f1 = (R)(1.0 - th * th / 6.0);
        f2 = (R)(0.5 * th);
    } else {
        f1 = sn / (R)th;
        f2 = omc / (R)th;
    }
    const R cs = (R)1 - omc;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pos[a] += s * (double)(upar * b[a] + f1 * up[a] + f2 * bxu[a]);
        u[a] = upar * b[a] + cs * up[a] + sn * bxu[a];
    }
    normalise(u);
}

template <class R>
__device__ inline void rk4_move(int type, R T, const double B[3], double s, int nsub, double pos[3], R u[3])
{
#pragma clang fp contract(off)
    const R q = type == kElectron ? (R)-1 : (R)1;
    const R p = m_sqrt(T * (T + (R)(2.0 * kMe)));
    const R kq = q * (R)kKB / p;
    const R Bx = (R)B[0], By = (R)B[1], Bz = (R)B[2];
    const R h = (R)(s / nsub);
    for (int i = 0; i < nsub; ++i) {
        R k1[3], k2[3], k3[3], k4[3], u2[3], u3[3], u4[3];
        k1[0] = kq * (u[1] * Bz - u[2] * By);
        k1[1] = kq * (u[2] * Bx - u[0] * Bz);
        k1[2] = kq * (u[0] * By - u[1] * Bx);
        for (int a = 0; a < 3; ++a) u2[a] = u[a] + (R)0.5 * h * k1[a];
        k2[0] = kq * (u2[1] * Bz - u2[2] * By);
        k2[1] = kq * (u2[2] * Bx - u2[0] * Bz);
        k2[2] = kq * (u2[0] * By - u2[1] * Bx);
        for (int a = 0; a < 3; ++a) u3[a] = u[a] + (R)0.5 * h * k2[a];
        k3[0] = kq * (u3[1] * Bz - u3[2] * By);
        k3[1] = kq * (u3[2] * Bx - u3[0] * Bz);
        k3[2] = kq * (u3[0] * By - u3[1] * Bx);
        for (int a = 0; a < 3; ++a) u4[a] = u[a] + h * k3[a];
        k4[0] = kq * (u4[1] * Bz - u4[2] * By);
        k4[1] = kq * (u4[2] * Bx - u4[0] * Bz);
        k4[2] = kq * (u4[0] * By - u4[1] * Bx);
        for (int a = 0; a < 3; ++a) {
            pos[a] += (double)(h / (R)6 * (u[a] + (R)2 * u2[a] + (R)2 * u3[a] + u4[a]));
            u[a] += h / (R)6 * (k1[a] + (R)2 * k2[a] + (R)2 * k3[a] + k4[a]);
        }
    }
    normalise(u);
}

}  // namespace gv
