/*
 * Oracle physics: material constants, cross sections, stopping powers and the
 * log-grid tables (test infrastructure only).
 *
 * The paper names the model set (Sec. 3.5: the Geant4 EM "standard" list) but
 * prints no formula, so these are the textbook closed forms:
 *   Compton      Klein-Nishina, free electrons at rest
 *   pair         Bethe-Heitler in complete screening, dsigma/dx ~ 1-4/3 x(1-x)
 *   bremsstrahlung  complete screening, k dsigma/dk ~ 4/3-4/3 y+y^2, k >= k_cut
 *   Moller / Bhabha  per-electron DCS above the delta-ray threshold
 *   dE/dx        restricted Bethe-Bloch (Berger-Seltzer form) with the
 *                high-energy density-effect asymptote, plus the sub-threshold
 *                bremsstrahlung loss
 *   X0           Tsai's formula, mixtures by mass fraction
 * Tables: nodes E_i = e_min 10^(i/bins_per_decade); linear interpolation in E;
 * range by 8-point Gauss-Legendre per bin in ln E starting from
 * R(e_min) = e_min / S(e_min); inverse range by bisection + linear inverse.
 */
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

/* ---------------- materials ---------------- */

static double tsai_inv_x0_per_gram(int Z, double A)
{
    double Lrad, Lprime;
    if (Z == 1) {
        Lrad = 5.31;
        Lprime = 6.144;
    } else {
        Lrad = log(184.15 * pow((double)Z, -1.0 / 3.0));
        Lprime = log(1194.0 * pow((double)Z, -2.0 / 3.0));
    }
    double a = OR_ALPHA * Z;
    double a2 = a * a;
    double fc = a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2
                      - 0.002 * a2 * a2 * a2);
    return 4.0 * OR_ALPHA * OR_RE * OR_RE * (OR_NA / A) * ((double)Z * Z * (Lrad - fc) + Z * Lprime);
}

int or_setup_materials(const or_material* mats, int32_t n)
{
    G.n_mats = n;
    for (int m = 0; m < n; ++m) {
        const or_material* M = &mats[m];
        G.mat[m] = *M;
        double zoa = 0.0, inv_x0 = 0.0, lnI_num = 0.0;
        for (int j = 0; j < M->n_elem; ++j) {
            double za = M->w[j] * M->Z[j] / M->A[j];
            zoa += za;
            inv_x0 += M->w[j] * tsai_inv_x0_per_gram(M->Z[j], M->A[j]);
            lnI_num += za * log(M->I_elem_eV[j]);
        }
        G.n_el[m] = M->density * OR_NA * zoa;
        G.X0[m] = (M->X0_cm > 0.0) ? M->X0_cm : 1.0 / (inv_x0 * M->density);
        double I_eV = (M->I_eV > 0.0) ? M->I_eV : exp(lnI_num / zoa);
        G.I[m] = I_eV * 1.0e-6;
        G.hwp[m] = 28.816 * sqrt(M->density * zoa) * 1.0e-6;
    }
    return 0;
}

double or_mat_electron_density(int32_t m) { return G.n_el[m]; }
double or_mat_X0(int32_t m) { return G.X0[m]; }
double or_mat_I(int32_t m) { return G.I[m]; }
double or_mat_plasma_energy(int32_t m) { return G.hwp[m]; }

/* ---------------- cross sections ---------------- */

/* Klein-Nishina total cross section per electron; k in MeV */
double or_xs_compton_per_electron(double kMeV)
{
    double k = kMeV / OR_ME;
    double pre = 2.0 * OR_PI * OR_RE * OR_RE;
    if (k < 0.01) {
        /* Taylor series about the Thomson limit (the closed form cancels
         * catastrophically here): sigma_T sum c_n k^n, n = 0..8 */
        static const double c[9] = {1.0, -2.0, 26.0 / 5.0, -133.0 / 10.0, 1144.0 / 35.0,
                                    -544.0 / 7.0, 3784.0 / 21.0, -6148.0 / 15.0, 151552.0 / 165.0};
        double sT = 8.0 * OR_PI * OR_RE * OR_RE / 3.0;
        double acc = c[8];
        for (int n = 7; n >= 0; --n) acc = acc * k + c[n];
        return sT * acc;
    }
    double l = log(1.0 + 2.0 * k);
    double t1 = ((1.0 + k) / (k * k)) * (2.0 * (1.0 + k) / (1.0 + 2.0 * k) - l / k);
    double t2 = l / (2.0 * k);
    double t3 = (1.0 + 3.0 * k) / ((1.0 + 2.0 * k) * (1.0 + 2.0 * k));
    return pre * (t1 + t2 - t3);
}

double or_xs_compton(int32_t m, double k) { return G.n_el[m] * or_xs_compton_per_electron(k); }

/* complete-screening pair production: x = E-/k in [a, 1-a], a = m/k */
double or_xs_pair(int32_t m, double k)
{
    if (k <= 2.0 * OR_ME) return 0.0;
    double a = OR_ME / k, b = 1.0 - a;
    double v = (b - a) - (2.0 / 3.0) * (b * b - a * a) + (4.0 / 9.0) * (b * b * b - a * a * a);
    return v / G.X0[m];
}

/* complete-screening bremsstrahlung, photons k in [k_cut, T] */
double or_xs_brems(int32_t m, double T)
{
    double kc = G.cfg.k_cut;
    if (T <= kc) return 0.0;
    double E = T + OR_ME;
    double v = (4.0 / 3.0) * log(T / kc) - (4.0 / 3.0) * (T - kc) / E + (T * T - kc * kc) / (2.0 * E * E);
    return v / G.X0[m];
}

/* Moller (e- e-), delta rays eps = T_delta/T in [T_cut/T, 1/2] */
double or_xs_moller(int32_t m, double T)
{
    double tc = G.cfg.t_cut;
    if (T <= 2.0 * tc) return 0.0;
    double E = T + OR_ME, g = E / OR_ME;
    double b2 = 1.0 - 1.0 / (g * g);
    double g1 = ((g - 1.0) / g) * ((g - 1.0) / g);
    double g2 = (2.0 * g - 1.0) / (g * g);
    double ec = tc / T;
    double br = g1 * (0.5 - ec) + 1.0 / ec - 1.0 / (1.0 - ec) - g2 * log((1.0 - ec) / ec);
    return G.n_el[m] * (2.0 * OR_PI * OR_RE * OR_RE * OR_ME / (b2 * T)) * br;
}

/* Bhabha (e+ e-), eps in [T_cut/T, 1] */
double or_xs_bhabha(int32_t m, double T)
{
    double tc = G.cfg.t_cut;
    if (T <= tc) return 0.0;
    double E = T + OR_ME, g = E / OR_ME;
    double b2 = 1.0 - 1.0 / (g * g);
    double y = 1.0 / (g + 1.0);
    double B1 = 2.0 - y * y;
    double B2 = (1.0 - 2.0 * y) * (3.0 + y * y);
    double B4 = (1.0 - 2.0 * y) * (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double B3 = B4 + (1.0 - 2.0 * y) * (1.0 - 2.0 * y);
    double ec = tc / T;
    double br = (1.0 / b2) * (1.0 / ec - 1.0) - B1 * log(1.0 / ec) + B2 * (1.0 - ec)
                - 0.5 * B3 * (1.0 - ec * ec) + (B4 / 3.0) * (1.0 - ec * ec * ec);
    return G.n_el[m] * (2.0 * OR_PI * OR_RE * OR_RE * OR_ME / T) * br;
}

/* ---------------- stopping powers ---------------- */

double or_density_effect(int32_t m, double T)
{
    double bg = sqrt(T * (T + 2.0 * OR_ME)) / OR_ME;
    double d = 2.0 * log(bg) + 2.0 * log(G.hwp[m] / G.I[m]) - 1.0;
    return d > 0.0 ? d : 0.0;
}

/* restricted collision stopping power (MeV/cm); energy transfers below t_cut */
double or_dedx_col(int32_t m, double T, int32_t positron, double t_cut)
{
    double tau = T / OR_ME;
    double g = tau + 1.0;
    double b2 = 1.0 - 1.0 / (g * g);
    double Im = G.I[m] / OR_ME;
    double F;
    if (!positron) {
        double d = fmin(t_cut, 0.5 * T) / OR_ME;
        F = -1.0 - b2 + log((tau - d) * d) + tau / (tau - d)
            + (0.5 * d * d + (2.0 * tau + 1.0) * log(1.0 - d / tau)) / (g * g);
    } else {
        double d = fmin(t_cut, T) / OR_ME;
        double y = 1.0 / (g + 1.0);
        double d2 = d * d, d3 = d2 * d, d4 = d3 * d;
        F = log(tau * d)
            - (b2 / tau) * (tau + 2.0 * d - 1.5 * d2 * y - (d - d3 / 3.0) * y * y
                            - (0.5 * d2 - tau * d3 / 3.0 + 0.25 * d4) * y * y * y);
    }
    double L = log(2.0 * (tau + 2.0) / (Im * Im)) + F - or_density_effect(m, T);
    return 2.0 * OR_PI * OR_RE * OR_RE * OR_ME * G.n_el[m] / b2 * L;
}

/* radiative loss to photons below k_cut */
double or_dedx_rad(int32_t m, double T, double k_cut)
{
    double E = T + OR_ME;
    double K = fmin(k_cut, T);
    return ((4.0 / 3.0) * K - (2.0 / 3.0) * K * K / E + K * K * K / (3.0 * E * E)) / G.X0[m];
}

double or_dedx_total(int32_t m, double T, int32_t positron)
{
    return or_dedx_col(m, T, positron, G.cfg.t_cut) + or_dedx_rad(m, T, G.cfg.k_cut);
}

/* ---------------- tables ---------------- */

/* 8-point Gauss-Legendre abscissae and weights on [-1, 1] */
static const double GL_X[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                               -0.1834346424956498, 0.1834346424956498, 0.5255324099163290,
                               0.7966664774136267, 0.9602898564975363};
static const double GL_W[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                               0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                               0.2223810344533745, 0.1012285362903763};

double or_gl_integrate(double (*f)(double), double a, double b)
{
    double h = 0.5 * (b - a), c = 0.5 * (b + a), s = 0.0;
    for (int j = 0; j < 8; ++j) s += GL_W[j] * f(c + h * GL_X[j]);
    return s * h;
}

void or_free_tables(void)
{
    free(G.node_E);
    G.node_E = NULL;
    for (int m = 0; m < OR_MAX_MATS; ++m)
        for (int t = 0; t < OR_NTAB; ++t) {
            free(G.tab[m][t]);
            G.tab[m][t] = NULL;
        }
}

int32_t or_n_nodes(void) { return G.cfg.n_nodes; }
double or_node_energy(int32_t i) { return G.node_E[i]; }
double or_table_node(int32_t m, int32_t which, int32_t i) { return G.tab[m][which][i]; }

/* bin i with E_i <= T < E_{i+1}, clamped to [0, n-2] */
static int32_t find_bin(double T)
{
    int32_t n = G.cfg.n_nodes;
    int32_t i = (int32_t)floor((log10(T) - log10(G.cfg.e_min)) * G.cfg.bins_per_decade);
    if (i < 0) i = 0;
    if (i > n - 2) i = n - 2;
    while (i > 0 && T < G.node_E[i]) --i;
    while (i < n - 2 && T >= G.node_E[i + 1]) ++i;
    return i;
}

double or_table_value(int32_t m, int32_t which, double T)
{
    const double* y = G.tab[m][which];
    int32_t i = find_bin(T);
    double e0 = G.node_E[i], e1 = G.node_E[i + 1];
    return y[i] + (y[i + 1] - y[i]) * (T - e0) / (e1 - e0);
}

/* kinetic energy whose tabulated range is r (linear inverse on the R table) */
double or_range_inverse(int32_t m, int32_t positron, double r)
{
    const double* R = G.tab[m][positron ? OR_T_R_EP : OR_T_R_EM];
    int32_t n = G.cfg.n_nodes;
    if (r <= R[0]) return G.node_E[0] * r / R[0];
    int32_t lo = 0, hi = n - 1;
    if (r >= R[hi]) lo = n - 2;
    else {
        while (hi - lo > 1) {
            int32_t mid = (lo + hi) / 2;
            if (R[mid] <= r) lo = mid;
            else hi = mid;
        }
    }
    double e0 = G.node_E[lo], e1 = G.node_E[lo + 1];
    return e0 + (e1 - e0) * (r - R[lo]) / (R[lo + 1] - R[lo]);
}

int or_build_tables(void)
{
    int32_t n = G.cfg.n_nodes;
    G.node_E = (double*)malloc(sizeof(double) * n);
    for (int32_t i = 0; i < n; ++i)
        G.node_E[i] = G.cfg.e_min * pow(10.0, (double)i / G.cfg.bins_per_decade);
    for (int32_t m = 0; m < G.n_mats; ++m) {
        for (int t = 0; t < OR_NTAB; ++t) G.tab[m][t] = (double*)malloc(sizeof(double) * n);
        for (int32_t i = 0; i < n; ++i) {
            double E = G.node_E[i];
            G.tab[m][OR_T_COMPTON][i] = or_xs_compton(m, E);
            G.tab[m][OR_T_PAIR][i] = or_xs_pair(m, E);
            G.tab[m][OR_T_MOLLER][i] = or_xs_moller(m, E);
            G.tab[m][OR_T_BREMS_EM][i] = or_xs_brems(m, E);
            G.tab[m][OR_T_S_EM][i] = or_dedx_total(m, E, 0);
            G.tab[m][OR_T_BHABHA][i] = or_xs_bhabha(m, E);
            G.tab[m][OR_T_BREMS_EP][i] = or_xs_brems(m, E);
            G.tab[m][OR_T_S_EP][i] = or_dedx_total(m, E, 1);
            if (!(G.tab[m][OR_T_S_EM][i] > 0.0) || !(G.tab[m][OR_T_S_EP][i] > 0.0)) {
                or_set_error("non-positive stopping power in table");
                return -1;
            }
        }
        /* range: R(E_0) = E_0 / S(E_0), then GL over ln E per bin of E / S(E) */
        for (int pos = 0; pos < 2; ++pos) {
            double* R = G.tab[m][pos ? OR_T_R_EP : OR_T_R_EM];
            R[0] = G.node_E[0] / or_dedx_total(m, G.node_E[0], pos);
            for (int32_t i = 0; i + 1 < n; ++i) {
                double la = log(G.node_E[i]), lb = log(G.node_E[i + 1]);
                double h = 0.5 * (lb - la), c = 0.5 * (lb + la), s = 0.0;
                for (int j = 0; j < 8; ++j) {
                    double E = exp(c + h * GL_X[j]);
                    s += GL_W[j] * E / or_dedx_total(m, E, pos);
                }
                R[i + 1] = R[i] + s * h;
            }
            G.r_track[m][pos] = or_table_value(m, pos ? OR_T_R_EP : OR_T_R_EM, G.cfg.t_track);
        }
    }
    return 0;
}
