"""Pins of the oracle's cross sections, stopping powers and tables.

The paper names the EM model set (Sec. 3.5) but prints no formula; each
closed form the oracle uses is pinned here against something other than
itself: a different textbook form of the same quantity (the Klein-Nishina
angular cross section, the unrestricted Rohrlich-Carlson stopping powers, the
ultra-relativistic Moller/Bhabha limits), numerical integration of the
differential cross sections, PDG radiation lengths, limits (Thomson, 7/9 X0,
radiation-length identity) and exact quadrature properties.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import quad

import gv_inputs

ME = 0.51099895
RE = 2.8179403262e-13
NA = 6.02214076e23


@pytest.fixture
def slab(oracle_mod):
    return oracle_mod.Oracle(gv_inputs.slab_calorimeter(2))


# ---------------------------------------------------------------- X0 (Tsai)

def _golden(name):
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                rows[k] = [float(x) for x in v]
    return rows


def test_radiation_lengths_match_pdg(oracle_mod):
    pdg = {k: v[0] for k, v in _golden("radiation_lengths_pdg.txt").items()}
    for geom in (gv_inputs.slab_calorimeter(2), gv_inputs.barrel()):
        o = oracle_mod.Oracle(geom)
        for m, md in enumerate(geom["materials"]):
            x0 = o.lib.or_mat_X0(m) * md["density"]
            if md["name"] in pdg:
                assert abs(x0 / pdg[md["name"]] - 1) < 2e-3, (md["name"], x0)
            else:  # brass lies between its constituents
                assert pdg["Zn"] < x0 < pdg["Cu"]


def test_electron_density_and_plasma_energy(slab):
    # Pb: n_el = rho N_A Z/A ; plasma energy 28.816 sqrt(rho Z/A) eV = 61.07 eV
    ne = 11.35 * NA * 82 / 207.2
    assert abs(slab.lib.or_mat_electron_density(0) / ne - 1) < 1e-14
    assert abs(slab.lib.or_mat_plasma_energy(0) * 1e6 - 61.07) < 0.01


def test_bragg_mean_excitation_brass(oracle_mod):
    o = oracle_mod.Oracle(gv_inputs.barrel())
    I = o.lib.or_mat_I(2) * 1e6
    assert 322.0 < I < 330.0


# ---------------------------------------------------------------- Klein-Nishina

def _kn_from_angular(k_mev):
    """sigma = int dOmega (re^2/2) P^2 (P + 1/P - sin^2), P = k'/k: the
    angular Klein-Nishina formula, integrated numerically."""
    k = k_mev / ME

    def f(c):
        P = 1.0 / (1.0 + k * (1.0 - c))
        return 0.5 * RE * RE * P * P * (P + 1.0 / P - (1.0 - c * c)) * 2.0 * math.pi
    return quad(f, -1.0, 1.0, epsabs=0, epsrel=1e-13, limit=200)[0]


@pytest.mark.parametrize("k", [0.1, 0.2, ME, 1.0, 10.0, 1e3, 1e5])
def test_klein_nishina_total_vs_angular_integral(slab, k):
    got = slab.lib.or_xs_compton_per_electron(k)
    assert abs(got / _kn_from_angular(k) - 1) < 1e-11


def test_klein_nishina_thomson_limit(slab):
    sT = 8 * math.pi * RE * RE / 3
    lib = slab.lib
    assert abs(lib.or_xs_compton_per_electron(1e-9) / sT - 1) < 1e-8
    # the small-k series and the closed form meet smoothly at k = 0.01 m
    k = 0.01 * ME
    a = lib.or_xs_compton_per_electron(k * (1 - 1e-12))
    b = lib.or_xs_compton_per_electron(k * (1 + 1e-12))
    assert abs(a / b - 1) < 1e-9
    assert abs(a / _kn_from_angular(k) - 1) < 1e-9


# ---------------------------------------------------------------- pair

def test_pair_threshold_and_limit(slab):
    lib = slab.lib
    x0 = lib.or_mat_X0(0)
    assert lib.or_xs_pair(0, 2 * ME) == 0.0
    assert lib.or_xs_pair(0, 1.0) == 0.0
    assert lib.or_xs_pair(0, 2 * ME * 1.0001) > 0.0
    assert abs(lib.or_xs_pair(0, 1e5) * x0 / (7 / 9) - 1) < 1e-4


@pytest.mark.parametrize("k", [1.5, 10.0, 1e3])
def test_pair_total_vs_dcs_integral(slab, k):
    a = ME / k
    x0 = slab.lib.or_mat_X0(0)
    ref = quad(lambda x: 1 - 4 / 3 * x * (1 - x), a, 1 - a, epsrel=1e-13)[0] / x0
    assert abs(slab.lib.or_xs_pair(0, k) / ref - 1) < 1e-12


# ---------------------------------------------------------------- bremsstrahlung

@pytest.mark.parametrize("T", [1.5, 30.0, 1e4])
def test_brems_total_vs_dcs_integral(slab, T):
    E = T + ME
    x0 = slab.lib.or_mat_X0(0)
    ref = quad(lambda k: (4 / 3 - 4 / 3 * k / E + (k / E) ** 2) / k, 1.0, T, epsrel=1e-13)[0] / x0
    assert abs(slab.lib.or_xs_brems(0, T) / ref - 1) < 1e-12
    assert slab.lib.or_xs_brems(0, 1.0) == 0.0


def test_radiation_length_identity(slab):
    """Unrestricted radiative loss (all photon energies up to T) tends to E/X0."""
    lib = slab.lib
    x0 = lib.or_mat_X0(0)
    for T in [1e3, 1e4, 1e5]:
        E = T + ME
        s = lib.or_dedx_rad(0, T, T)
        assert abs(s * x0 / E - 1) < 2 * ME / T


# ---------------------------------------------------------------- Moller / Bhabha

def _moller_dcs(T, e):
    g = (T + ME) / ME
    g1 = ((g - 1) / g) ** 2
    g2 = (2 * g - 1) / g**2
    return g1 + 1 / e**2 + 1 / (1 - e) ** 2 - g2 / (e * (1 - e))


def _bhabha_dcs(T, e):
    g = (T + ME) / ME
    b2 = 1 - 1 / g**2
    y = 1 / (g + 1)
    B1 = 2 - y * y
    B2 = (1 - 2 * y) * (3 + y * y)
    B4 = (1 - 2 * y) ** 3
    B3 = B4 + (1 - 2 * y) ** 2
    return 1 / (b2 * e * e) - B1 / e + B2 - B3 * e + B4 * e * e


@pytest.mark.parametrize("T", [2.5, 20.0, 5e3])
def test_moller_bhabha_total_vs_dcs_integral(slab, T):
    lib = slab.lib
    ne = lib.or_mat_electron_density(0)
    g = (T + ME) / ME
    b2 = 1 - 1 / g**2
    ec = 1.0 / T
    pre = 2 * math.pi * RE * RE * ME / T
    m_ref = ne * pre / b2 * quad(lambda e: _moller_dcs(T, e), ec, 0.5, epsrel=1e-13)[0]
    b_ref = ne * pre * quad(lambda e: _bhabha_dcs(T, e), ec, 1.0, epsrel=1e-13)[0]
    assert abs(lib.or_xs_moller(0, T) / m_ref - 1) < 1e-11
    assert abs(lib.or_xs_bhabha(0, T) / b_ref - 1) < 1e-11
    assert lib.or_xs_moller(0, 2.0) == 0.0 and lib.or_xs_bhabha(0, 1.0) == 0.0


def test_moller_bhabha_ultrarelativistic_forms(slab):
    """At gamma -> infinity the Moller bracket is 1 + 1/e^2 + 1/(1-e)^2 and the
    Bhabha bracket is (1 - e + e^2)^2 / e^2 (textbook limits)."""
    lib = slab.lib
    T = 1e5
    ne = lib.or_mat_electron_density(0)
    pre = 2 * math.pi * RE * RE * ME / T
    ec = 1.0 / T
    m_ur = ne * pre * quad(lambda e: 1 + 1 / e**2 + 1 / (1 - e) ** 2, ec, 0.5, epsrel=1e-12, limit=400)[0]
    b_ur = ne * pre * quad(lambda e: (1 - e + e * e) ** 2 / e**2, ec, 1.0, epsrel=1e-12, limit=400)[0]
    assert abs(lib.or_xs_moller(0, T) / m_ur - 1) < 1e-4
    assert abs(lib.or_xs_bhabha(0, T) / b_ur - 1) < 1e-4


# ---------------------------------------------------------------- stopping power

def _rohrlich_carlson(lib, m, T, positron):
    """Unrestricted collision stopping power, textbook (ICRU 37) form."""
    tau = T / ME
    g = tau + 1
    b2 = 1 - 1 / g**2
    Im = lib.or_mat_I(m) / ME
    if positron:
        F = 2 * math.log(2) - b2 / 12 * (23 + 14 / (tau + 2) + 10 / (tau + 2) ** 2 + 4 / (tau + 2) ** 3)
    else:
        F = 1 - b2 + (tau * tau / 8 - (2 * tau + 1) * math.log(2)) / (tau + 1) ** 2
    L = math.log(tau * tau * (tau + 2) / (2 * Im * Im)) + F - lib.or_density_effect(m, T)
    return 2 * math.pi * RE * RE * ME * lib.or_mat_electron_density(m) / b2 * L


@pytest.mark.parametrize("T", [0.2, 1.0, 7.0, 100.0, 1e4])
def test_restricted_loss_reduces_to_unrestricted(slab, T):
    lib = slab.lib
    for m in (0, 1):
        for pos in (0, 1):
            got = lib.or_dedx_col(m, T, pos, 1e9)  # threshold above the kinematic limit
            ref = _rohrlich_carlson(lib, m, T, pos)
            assert abs(got / ref - 1) < 1e-12, (m, T, pos)


@pytest.mark.parametrize("T", [2.5, 10.0, 300.0, 1e4])
def test_restricted_loss_matches_delta_ray_dcs(slab, T):
    """S(unrestricted) - S(T_cut) = n_el int_{T_cut}^{T_max} T_d dsigma/dT_d:
    ties the restricted formula to the Moller/Bhabha differential cross
    sections used for delta-ray production."""
    lib = slab.lib
    ne = lib.or_mat_electron_density(0)
    g = (T + ME) / ME
    b2 = 1 - 1 / g**2
    ec = 1.0 / T
    pre = 2 * math.pi * RE * RE * ME / T
    diff_e = lib.or_dedx_col(0, T, 0, 1e9) - lib.or_dedx_col(0, T, 0, 1.0)
    ref_e = ne * pre / b2 * T * quad(lambda e: e * _moller_dcs(T, e), ec, 0.5, epsrel=1e-13)[0]
    diff_p = lib.or_dedx_col(0, T, 1, 1e9) - lib.or_dedx_col(0, T, 1, 1.0)
    ref_p = ne * pre * T * quad(lambda e: e * _bhabha_dcs(T, e), ec, 1.0, epsrel=1e-13)[0]
    assert abs(diff_e - ref_e) <= 1e-11 * lib.or_dedx_col(0, T, 0, 1e9)
    assert abs(diff_p - ref_p) <= 1e-11 * lib.or_dedx_col(0, T, 1, 1e9)


def test_lead_minimum_ionisation(slab):
    lib = slab.lib
    Ts = np.geomspace(0.3, 30, 400)
    s = np.array([lib.or_dedx_col(0, T, 0, 1e9) for T in Ts]) / 11.35
    assert 1.0 < s.min() < 1.25   # MeV cm^2/g
    assert 0.6 < Ts[np.argmin(s)] < 3.0


def test_density_effect_limits(slab):
    lib = slab.lib
    assert lib.or_density_effect(0, 0.1) == 0.0
    # high-energy slope 2 ln(beta gamma)
    d1, d2 = lib.or_density_effect(0, 1e4), lib.or_density_effect(0, 1e5)
    bg1 = math.sqrt(1e4 * (1e4 + 2 * ME)) / ME
    bg2 = math.sqrt(1e5 * (1e5 + 2 * ME)) / ME
    assert abs((d2 - d1) - 2 * math.log(bg2 / bg1)) < 1e-12


# ---------------------------------------------------------------- tables / range

def test_gauss_legendre_exact_to_degree_15(oracle_mod, slab):
    import ctypes as C
    lib = slab.lib
    cb = C.CFUNCTYPE(C.c_double, C.c_double)
    lib.or_gl_integrate.argtypes = [cb, C.c_double, C.c_double]
    lib.or_gl_integrate.restype = C.c_double
    for deg in range(16):
        f = cb(lambda x, d=deg: x**d)
        got = lib.or_gl_integrate(f, 0.3, 1.7)
        ref = (1.7 ** (deg + 1) - 0.3 ** (deg + 1)) / (deg + 1)
        assert abs(got - ref) < 1e-14 * max(1.0, abs(ref)), deg
    f = cb(lambda x: x**16)
    assert abs(lib.or_gl_integrate(f, 0.0, 1.0) - 1 / 17) > 1e-12


def test_table_nodes_and_interpolation(slab):
    lib = slab.lib
    E = slab.nodes()
    assert len(E) == 801
    assert abs(E[0] - 1e-3) < 1e-18 and abs(E[-1] / 1e5 - 1) < 1e-14
    assert np.all(np.diff(E) > 0)
    comp = slab.table(0, "compton")
    for i in [200, 333, 799]:
        assert slab.table_value(0, "compton", E[i]) == comp[i]
        mid = 0.5 * (E[i] + E[i + 1])
        assert abs(slab.table_value(0, "compton", mid) - 0.5 * (comp[i] + comp[i + 1])) < 1e-15 * comp[i]
    for i in range(0, 801, 37):
        assert abs(comp[i] / lib.or_xs_compton(0, E[i]) - 1) < 1e-15


def test_range_table(slab):
    lib = slab.lib
    E = slab.nodes()
    for pos, rname in ((0, "R_em"), (1, "R_ep")):
        R = slab.table(0, rname)
        assert np.all(np.diff(R) > 0)
        # per-bin increments against adaptive quadrature of 1/S
        for i in [0, 150, 200, 400, 650, 799]:
            ref = quad(lambda T: 1.0 / lib.or_dedx_total(0, T, pos), E[i], E[i + 1], epsrel=1e-13)[0]
            assert abs((R[i + 1] - R[i]) / ref - 1) < 1e-11, (pos, i)
        # linear inverse is the exact inverse of the interpolated range
        for T in np.geomspace(0.1, 1e5, 200):
            r = slab.table_value(0, rname, T)
            assert abs(lib.or_range_inverse(0, pos, r) / T - 1) < 1e-12
