/*
 * Oracle final-state sampling from tables with the alias method (test
 * infrastructure only): the "sampling tables" technique of Sec. 3.5, in
 * which a discrete random variable first picks one of the two primary-energy
 * nodes around the actual energy (with the linear weight in ln E), and the
 * node's table then yields the sampled variable without any rejection loop.
 *
 * For every model the sampled quantity is mapped to a transformed variable
 * xi in [0, 1] on which the density is smooth and bounded:
 *   Compton  eps = k'/k = eps0^xi,              p ~ 1 + eps^2 - eps sin^2(theta)
 *   pair     x = a + xi (1 - 2a), a = m/k,       p ~ 1 - 4/3 x (1 - x)
 *   brems    k = k_c (T / k_c)^xi,              p ~ 1 - y + 3/4 y^2, y = k / E
 *   Moller   eps = e_c (1 / (2 e_c))^xi,        p ~ eps dsigma/deps
 *   Bhabha   eps = e_c (1 / e_c)^xi,            p ~ eps dsigma/deps
 * (e_c = T_cut / T; eps dsigma/deps is the rejection samplers' acceptance
 * function divided by eps).  A node holds
 * the density at OR_AL_NX + 1 equally spaced xi; the sub-intervals carry the
 * trapezoid weights, indexed by Walker's alias table (Vose's construction);
 * inside the chosen sub-interval xi follows the linear density exactly.
 * Uniforms: block FS0 gives u0 (node), u1 (column), u2 (alias test), u3
 * (inside the sub-interval); block FS0 + 1 gives the azimuth.  The sampled
 * variable is mapped back with the actual energy.
 */
#include <stdlib.h>
#include "or_internal.h"

typedef struct {
    double p[OR_AL_NX + 1];
    double q[OR_AL_NX];
    int32_t a[OR_AL_NX];
    int32_t valid;
} al_node;

static al_node AT[OR_AL_NMOD][OR_AL_NE];
static double AE[OR_AL_NE];

double or_alias_node_energy(int32_t j) { return (j >= 0 && j < OR_AL_NE) ? AE[j] : 0.0; }

static int model_valid(int32_t m, double E)
{
    switch (m) {
    case OR_AL_PAIR: return E > 2.0 * OR_ME;
    case OR_AL_BREMS: return E > G.cfg.k_cut;
    case OR_AL_MOLLER: return E > 2.0 * G.cfg.t_cut;
    case OR_AL_BHABHA: return E > G.cfg.t_cut;
    default: return E > 0.0;
    }
}

/* the sampled quantity for transformed variable xi at primary energy E */
double or_alias_var(int32_t m, double E, double xi)
{
    if (m == OR_AL_COMPTON) {
        const double eps0 = 1.0 / (1.0 + 2.0 * (E / OR_ME));
        return exp(xi * log(eps0));
    }
    if (m == OR_AL_PAIR) {
        const double a = OR_ME / E;
        return a + xi * (1.0 - 2.0 * a);
    }
    if (m == OR_AL_BREMS) {
        const double kc = G.cfg.k_cut;
        return kc * exp(xi * log(E / kc));
    }
    const double ec = G.cfg.t_cut / E;
    if (m == OR_AL_MOLLER) return ec * exp(xi * log(0.5 / ec));
    return ec * exp(xi * log(1.0 / ec));
}

/* density of xi (unnormalised) at primary energy E */
double or_alias_pdf(int32_t m, double E, double xi)
{
    const double v = or_alias_var(m, E, xi);
    if (m == OR_AL_COMPTON) {
        const double kk = E / OR_ME;
        const double t = (1.0 - v) / (kk * v);
        const double sin2 = t * (2.0 - t);
        return 1.0 + v * v - v * sin2;
    }
    if (m == OR_AL_PAIR) return 1.0 - (4.0 / 3.0) * v * (1.0 - v);
    if (m == OR_AL_BREMS) {
        const double y = v / (E + OR_ME);
        return 1.0 - y + 0.75 * y * y;
    }
    const double g = (E + OR_ME) / OR_ME;
    if (m == OR_AL_MOLLER) {
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

/* Walker's alias table for the sub-interval weights of one node (Vose):
 * scaled weights s = N w / sum(w); indices below 1 and at or above 1 go to two
 * stacks in increasing order; repeatedly the top small index keeps s of its
 * own column and hands the rest to the top large one. */
static void walker(const double* p, double* q, int32_t* a)
{
    double s[OR_AL_NX];
    int32_t small[OR_AL_NX], large[OR_AL_NX];
    int ns = 0, nl = 0;
    double sum = 0.0;
    for (int k = 0; k < OR_AL_NX; ++k) {
        s[k] = 0.5 * (p[k] + p[k + 1]);
        sum += s[k];
    }
    for (int k = 0; k < OR_AL_NX; ++k) {
        s[k] = (double)OR_AL_NX * s[k] / sum;
        if (s[k] < 1.0) small[ns++] = k;
        else large[nl++] = k;
    }
    while (ns > 0 && nl > 0) {
        const int32_t lo = small[--ns], hi = large[--nl];
        q[lo] = s[lo];
        a[lo] = hi;
        s[hi] = (s[hi] + s[lo]) - 1.0;
        if (s[hi] < 1.0) small[ns++] = hi;
        else large[nl++] = hi;
    }
    while (nl > 0) {
        const int32_t k = large[--nl];
        q[k] = 1.0;
        a[k] = k;
    }
    while (ns > 0) {
        const int32_t k = small[--ns];
        q[k] = 1.0;
        a[k] = k;
    }
}

void or_build_alias(void)
{
    for (int j = 0; j < OR_AL_NE; ++j) AE[j] = OR_AL_E0 * pow(10.0, (double)j / OR_AL_NPD);
    for (int m = 0; m < OR_AL_NMOD; ++m)
        for (int j = 0; j < OR_AL_NE; ++j) {
            al_node* N = &AT[m][j];
            N->valid = model_valid(m, AE[j]);
            if (!N->valid) continue;
            for (int k = 0; k <= OR_AL_NX; ++k) N->p[k] = or_alias_pdf(m, AE[j], (double)k / OR_AL_NX);
            walker(N->p, N->q, N->a);
        }
}

int32_t or_alias_table(int32_t m, int32_t j, double* p, double* q, int32_t* a)
{
    if (m < 0 || m >= OR_AL_NMOD || j < 0 || j >= OR_AL_NE) return -1;
    const al_node* N = &AT[m][j];
    for (int k = 0; k <= OR_AL_NX; ++k) p[k] = N->p[k];
    for (int k = 0; k < OR_AL_NX; ++k) {
        q[k] = N->q[k];
        a[k] = N->a[k];
    }
    return N->valid;
}

/* one sample of xi at energy E (E valid for the model) from u0..u3 */
double or_alias_xi(int32_t m, double E, const double u[4])
{
    int j = (int)floor(log10(E / OR_AL_E0) * OR_AL_NPD);
    if (j < 0) j = 0;
    if (j > OR_AL_NE - 2) j = OR_AL_NE - 2;
    while (j > 0 && E < AE[j]) --j;
    while (j < OR_AL_NE - 2 && E >= AE[j + 1]) ++j;
    const double lam = log(E / AE[j]) / log(AE[j + 1] / AE[j]);
    int jj = u[0] < lam ? j + 1 : j;
    if (!AT[m][jj].valid) jj = j + 1;
    const al_node* N = &AT[m][jj];
    int k = (int)(u[1] * OR_AL_NX);
    if (k > OR_AL_NX - 1) k = OR_AL_NX - 1;
    if (u[2] > N->q[k]) k = N->a[k];
    const double a = N->p[k], b = N->p[k + 1];
    double tau = u[3];
    if (a + b > 0.0) tau = u[3] * (a + b) / (a + sqrt(a * a + (b * b - a * a) * u[3]));
    if (tau > 1.0) tau = 1.0;
    return ((double)k + tau) / OR_AL_NX;
}

static void blocks(uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double u[4], double* phi)
{
    uint32_t w[4];
    or_stream(seed, event, tid, nstep, OR_PURP_FS0, w);
    for (int i = 0; i < 4; ++i) u[i] = or_u32(w[i]);
    or_stream(seed, event, tid, nstep, OR_PURP_FS0 + 1, w);
    *phi = 2.0 * OR_PI * or_u32(w[0]);
}

int or_sample_compton_alias(double kMeV, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double u[4], phi;
    blocks(seed, event, tid, nstep, u, &phi);
    const double eps = or_alias_var(OR_AL_COMPTON, kMeV, or_alias_xi(OR_AL_COMPTON, kMeV, u));
    const double t = (1.0 - eps) / ((kMeV / OR_ME) * eps);
    out[0] = eps;
    out[1] = 1.0 - t;
    out[2] = phi;
    out[3] = t * (2.0 - t);
    return 1;
}

int or_sample_pair_alias(double k, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double u[4], phi;
    blocks(seed, event, tid, nstep, u, &phi);
    out[0] = or_alias_var(OR_AL_PAIR, k, or_alias_xi(OR_AL_PAIR, k, u));
    out[1] = phi;
    out[2] = out[3] = 0.0;
    return 1;
}

int or_sample_brems_alias(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double u[4], phi;
    blocks(seed, event, tid, nstep, u, &phi);
    out[0] = or_alias_var(OR_AL_BREMS, T, or_alias_xi(OR_AL_BREMS, T, u));
    out[1] = out[2] = out[3] = 0.0;
    return 1;
}

int or_sample_moller_alias(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double u[4], phi;
    blocks(seed, event, tid, nstep, u, &phi);
    out[0] = or_alias_var(OR_AL_MOLLER, T, or_alias_xi(OR_AL_MOLLER, T, u));
    out[1] = phi;
    out[2] = out[3] = 0.0;
    return 1;
}

int or_sample_bhabha_alias(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4])
{
    double u[4], phi;
    blocks(seed, event, tid, nstep, u, &phi);
    out[0] = or_alias_var(OR_AL_BHABHA, T, or_alias_xi(OR_AL_BHABHA, T, u));
    out[1] = phi;
    out[2] = out[3] = 0.0;
    return 1;
}
