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
    double rk_tol;           // RK45 error tolerance
    int rk_max_sub;          // RK45 attempts per step
    int pad3;
    long long max_steps;
    // final-state tables (alias sampling): model m uses them when bit m of
    // fs_alias is set; records per (model, node) as built by k_build_alias
    int fs_alias;
    int pad2;
    const double* al_rec64;
    const float* al_rec32;
    const double* al_E64;
    const float* al_E32;
    const int* al_alias;
    const int* al_valid;
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
// Final states from tables (the sampling tables of Sec. 3.5): a discrete
// variable picks the lower or upper of the two primary-energy nodes around E
// (probability of the upper = the linear weight in ln E); Walker's alias
// table of that node picks one of kAlNX sub-intervals of a transformed
// variable xi in [0, 1]; inside it xi follows the tabulated linear density
// exactly.  No loop, a fixed four uniforms (block FS0) plus the azimuth
// (block FS0 + 1).  Transformed variables and their densities:
//   Compton  eps = eps0^xi                 p ~ 1 + eps^2 - eps sin^2(theta)
//   pair     x = a + xi (1 - 2a), a = m/k  p ~ 1 - 4/3 x (1 - x)
//   brems    k = kc (T / kc)^xi            p ~ 1 - y + 3/4 y^2, y = k / E
//   Moller   eps = ec (1 / (2 ec))^xi      p ~ eps dsigma/deps
//   Bhabha   eps = ec (1 / ec)^xi          p ~ eps dsigma/deps
// ---------------------------------------------------------------------------
constexpr int kAlNX = 64;          // sub-intervals per node
constexpr int kAlNPD = 20;         // nodes per decade of primary energy
constexpr int kAlNE = 121;         // 0.1 MeV .. 100 GeV
constexpr int kAlNMod = 5;
constexpr int kAlRec = 2 * kAlNX + 1;   // record: density at kAlNX + 1 points, kAlNX alias thresholds
constexpr double kAlE0 = 0.1;
enum { kAlCompton = 0, kAlPair = 1, kAlBrems = 2, kAlMoller = 3, kAlBhabha = 4 };

__host__ __device__ inline bool alias_model_valid(int m, double E, double tc, double kc)
{
    return m == kAlPair ? E > 2.0 * kMe : m == kAlBrems ? E > kc : m == kAlMoller ? E > 2.0 * tc
                                        : m == kAlBhabha ? E > tc : E > 0.0;
}

// the sampled quantity at primary energy E for transformed variable xi
template <class R> __device__ inline R alias_var(int m, R E, R xi, R tc, R kc)
{
    if (m == kAlCompton) return m_exp(xi * m_log((R)1 / ((R)1 + (R)2 * (E / (R)kMe))));
    if (m == kAlPair) {
        const R a = (R)kMe / E;
        return a + xi * ((R)1 - (R)2 * a);
    }
    if (m == kAlBrems) return kc * m_exp(xi * m_log(E / kc));
    const R ec = tc / E;
    if (m == kAlMoller) return ec * m_exp(xi * m_log((R)0.5 / ec));
    return ec * m_exp(xi * m_log((R)1 / ec));
}

// density of xi (unnormalised), for the table builder (double)
__device__ inline double alias_pdf(int m, double E, double xi, double tc, double kc)
{
    const double v = alias_var<double>(m, E, xi, tc, kc);
    if (m == kAlCompton) {
        const double kk = E / kMe;
        const double t = (1.0 - v) / (kk * v);
        const double sin2 = t * (2.0 - t);
        return 1.0 + v * v - v * sin2;
    }
    if (m == kAlPair) return 1.0 - (4.0 / 3.0) * v * (1.0 - v);
    if (m == kAlBrems) {
        const double y = v / (E + kMe);
        return 1.0 - y + 0.75 * y * y;
    }
    const double g = (E + kMe) / kMe;
    if (m == kAlMoller) {
        const double g1 = ((g - 1.0) / g) * ((g - 1.0) / g);
        const double g2 = (2.0 * g - 1.0) / (g * g);
        return (g1 * v * v + 1.0 + v * v / ((1.0 - v) * (1.0 - v)) - g2 * v / (1.0 - v)) / v;
    }
    const double b2 = 1.0 - 1.0 / (g * g);
    const double y = 1.0 / (g + 1.0);
    const double B1 = 2.0 - y * y;
    const double B2 = (1.0 - 2.0 * y) * (3.0 + y * y);
    const double B4 = (1.0 - 2.0 * y) * (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    const double B3 = B4 + (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    return (1.0 / b2 - B1 * v + B2 * v * v - B3 * v * v * v + B4 * v * v * v * v) / v;
}

template <class R> struct AliasView {
    const R* rec;
    const R* E;
    const int* alias;
    const int* valid;
};
template <class R> __device__ __forceinline__ AliasView<R> alias_view(const DevPhys& ph);
template <> __device__ __forceinline__ AliasView<double> alias_view<double>(const DevPhys& ph)
{
    return AliasView<double>{ph.al_rec64, ph.al_E64, ph.al_alias, ph.al_valid};
}
template <> __device__ __forceinline__ AliasView<float> alias_view<float>(const DevPhys& ph)
{
    return AliasView<float>{ph.al_rec32, ph.al_E32, ph.al_alias, ph.al_valid};
}

// one sample of xi for model m at energy E (valid for the model) from u[0..3]
template <class R> __device__ inline R alias_xi(const AliasView<R>& av, int m, R E, const R u[4])
{
    int j = (int)m_floor(m_log10(E / (R)kAlE0) * (R)kAlNPD);
    j = j < 0 ? 0 : (j > kAlNE - 2 ? kAlNE - 2 : j);
    while (j > 0 && E < av.E[j]) --j;
    while (j < kAlNE - 2 && E >= av.E[j + 1]) ++j;
    const R lam = m_log(E / av.E[j]) / m_log(av.E[j + 1] / av.E[j]);
    int jj = u[0] < lam ? j + 1 : j;
    if (!av.valid[m * kAlNE + jj]) jj = j + 1;
    const int node = m * kAlNE + jj;
    const R* rec = av.rec + (size_t)node * kAlRec;
    int k = (int)(u[1] * (R)kAlNX);
    k = k > kAlNX - 1 ? kAlNX - 1 : k;
    if (u[2] > rec[kAlNX + 1 + k]) k = av.alias[node * kAlNX + k];
    const R a = rec[k], b = rec[k + 1];
    R tau = u[3];
    if (a + b > (R)0) tau = u[3] * (a + b) / (a + m_sqrt(a * a + (b * b - a * a) * u[3]));
    tau = tau > (R)1 ? (R)1 : tau;
    return ((R)k + tau) / (R)kAlNX;
}

// the four table uniforms and the azimuth
template <class R> __device__ __forceinline__ R alias_uniforms(const Key& key, R u[4])
{
    const FS4<R> f = fs_uniforms<R>(key, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[i] = f.u[i];
    return (R)(2.0 * kPi) * fs_uniforms<R>(key, 1).u[0];
}

// Compton from the table: eps, om = 1 - eps (from expm1, no cancellation),
// t = 1 - cos(theta), phi
template <class R>
__device__ inline void alias_compton(const AliasView<R>& av, R kMeV, const Key& key, R& eps, R& om, R& t, R& phi)
{
    R u[4];
    phi = alias_uniforms<R>(key, u);
    const R k = kMeV / (R)kMe;
    const R lg = m_log((R)1 / ((R)1 + (R)2 * k));
    const R xi = alias_xi<R>(av, kAlCompton, kMeV, u);
    eps = m_exp(xi * lg);
    om = -m_expm1(xi * lg);
    t = om / (k * eps);
}

// pair, bremsstrahlung, Moller and Bhabha from their tables
template <class R> __device__ inline R alias_sample(const AliasView<R>& av, int m, R E, R tc, R kc, const Key& key, R& phi)
{
    R u[4];
    phi = alias_uniforms<R>(key, u);
    return alias_var<R>(m, E, alias_xi<R>(av, m, E, u), tc, kc);
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
