"""Pins of the oracle's final-state samplers (composition-rejection, Sec. 3.5)
and of per-interaction conservation.

Each sampler is checked by a chi-square test of its output against the
normalised differential cross section integrated per bin (the Klein-Nishina
pdf is taken from the angular formula, not from the sampler's acceptance
function); single steps are checked for energy conservation of every step and
momentum conservation of every Compton scattering.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.integrate import quad

import gv_inputs

ME = 0.51099895
N = 60_000


@pytest.fixture
def orc(oracle_mod):
    return oracle_mod.Oracle(gv_inputs.slab_calorimeter(2))


def _sample(orc, name, E, n=N):
    fn = getattr(orc.lib, "or_sample_" + name)
    out = np.zeros(4)
    res = np.empty((n, 4))
    iters = np.empty(n, dtype=np.int64)
    p = out.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_double))
    for i in range(n):
        iters[i] = fn(E, 0xABC, i % 977, i, 5, p)
        res[i] = out
    return res, iters


def _chi2(samples, pdf, lo, hi, bins=60, log=False):
    edges = np.geomspace(lo, hi, bins + 1) if log else np.linspace(lo, hi, bins + 1)
    counts, _ = np.histogram(samples, bins=edges)
    norm = quad(pdf, lo, hi, limit=400, epsrel=1e-10)[0]
    exp = np.array([quad(pdf, edges[i], edges[i + 1], limit=200)[0] for i in range(bins)]) / norm
    exp *= counts.sum()
    keep = exp > 5
    chi2 = ((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum()
    return stats.chi2.sf(chi2, keep.sum() - 1)


@pytest.mark.parametrize("k", [0.2, 1.0, 10.0, 1e3])
def test_compton_epsilon_distribution(orc, k):
    res, it = _sample(orc, "compton", k)
    kk = k / ME
    eps0 = 1 / (1 + 2 * kk)

    def pdf(e):  # KN angular formula mapped to eps = k'/k: ~ (eps + 1/eps - sin^2)
        c = 1 - (1 - e) / (kk * e)
        return e + 1 / e - (1 - c * c)
    assert _chi2(res[:, 0], pdf, eps0, 1.0, log=kk > 5) > 1e-3
    # the reported polar angle belongs to the sampled eps, and phi is uniform
    c = 1 - (1 - res[:, 0]) / (kk * res[:, 0])
    assert np.allclose(res[:, 1], c, rtol=0, atol=1e-12)
    assert np.allclose(res[:, 3], (1 - c) * (1 + c), rtol=0, atol=1e-12)
    assert stats.kstest(res[:, 2] / (2 * math.pi), "uniform").pvalue > 1e-3
    assert it.min() >= 1


@pytest.mark.parametrize("k", [1.5, 20.0, 5e3])
def test_pair_x_distribution(orc, k):
    res, _ = _sample(orc, "pair", k)
    a = ME / k
    assert res[:, 0].min() >= a and res[:, 0].max() <= 1 - a
    assert _chi2(res[:, 0], lambda x: 1 - 4 / 3 * x * (1 - x), a, 1 - a) > 1e-3


@pytest.mark.parametrize("T", [3.0, 100.0, 5e4])
def test_brems_k_distribution(orc, T):
    res, _ = _sample(orc, "brems", T)
    E = T + ME
    assert res[:, 0].min() >= 1.0 and res[:, 0].max() <= T
    pdf = lambda k: (4 / 3 - 4 / 3 * k / E + (k / E) ** 2) / k
    assert _chi2(res[:, 0], pdf, 1.0, T, log=True) > 1e-3


@pytest.mark.parametrize("T", [2.5, 50.0, 1e4])
def test_moller_bhabha_distributions(orc, T):
    g = (T + ME) / ME
    ec = 1.0 / T
    g1 = ((g - 1) / g) ** 2
    g2 = (2 * g - 1) / g**2
    res, _ = _sample(orc, "moller", T)
    assert res[:, 0].min() >= ec and res[:, 0].max() <= 0.5
    pdf_m = lambda e: g1 + 1 / e**2 + 1 / (1 - e) ** 2 - g2 / (e * (1 - e))
    assert _chi2(res[:, 0], pdf_m, ec, 0.5, log=True) > 1e-3
    b2 = 1 - 1 / g**2
    y = 1 / (g + 1)
    B1, B2, B4 = 2 - y * y, (1 - 2 * y) * (3 + y * y), (1 - 2 * y) ** 3
    B3 = B4 + (1 - 2 * y) ** 2
    res, _ = _sample(orc, "bhabha", T)
    assert res[:, 0].min() >= ec and res[:, 0].max() <= 1.0
    pdf_b = lambda e: 1 / (b2 * e * e) - B1 / e + B2 - B3 * e + B4 * e * e
    assert _chi2(res[:, 0], pdf_b, ec, 1.0, log=True) > 1e-3


def test_rejection_bounds_never_violated():
    """The envelope constants used by the Moller (2 + g1/4) and Bhabha (1/beta^2)
    rejection bound eps^2 * DCS on the whole sampling interval."""
    for T in np.geomspace(0.11, 1e5, 80):
        g = (T + ME) / ME
        b2 = 1 - 1 / g**2
        y = 1 / (g + 1)
        B1, B2, B4 = 2 - y * y, (1 - 2 * y) * (3 + y * y), (1 - 2 * y) ** 3
        B3 = B4 + (1 - 2 * y) ** 2
        e = np.linspace(1e-9, 1, 100001)
        fb = 1 / b2 - B1 * e + B2 * e**2 - B3 * e**3 + B4 * e**4
        assert fb.max() <= (1 / b2) * (1 + 1e-12)
        if T > 2:
            g1 = ((g - 1) / g) ** 2
            g2 = (2 * g - 1) / g**2
            e = np.linspace(1e-9, 0.5, 100001)
            fm = g1 * e * e + 1 + e * e / (1 - e) ** 2 - g2 * e / (1 - e)
            assert fm.max() <= 2 + g1 / 4


def test_single_step_conservation(oracle_mod):
    geom = gv_inputs.slab_calorimeter(10)
    o = oracle_mod.Oracle(geom)
    st = gv_inputs.random_states(40_000, 11, geom)
    out = o.single_step(st, 0x5EED)
    T_in = st["ekin"]
    annih = (out["process"] == -1) & (out["n_children"] == 2)   # e+ annihilation at rest or after stop
    pair = out["process"] == 1
    lhs = T_in + 2 * ME * annih - 2 * ME * pair
    ch = np.where(out["ch_type"] >= 0, out["ch_ekin"], 0.0).sum(1)
    alive_T = np.where(out["status"] == 3, 0.0, out["ekin"])      # killed: none in this test
    rhs = alive_T + out["edep"] + ch
    assert np.all(np.abs(lhs - rhs) <= 1e-12 * lhs)
    assert (out["status"] == 3).sum() == 0
    # Compton: k u = k' u' + p_e u_e
    c = (out["process"] == 0) & (out["n_children"] == 1) & (out["status"] == 0)
    assert c.sum() > 50
    k = T_in[c]
    pin = k[:, None] * st["dir"][c]
    k1 = out["ekin"][c]
    Te = out["ch_ekin"][c, 0]
    pe = np.sqrt(Te * (Te + 2 * ME))
    pout = k1[:, None] * out["dir"][c] + pe[:, None] * out["ch_dir"][c, 0]
    assert np.max(np.abs(pin - pout)) <= 1e-12 * k.max()
    # unit directions everywhere
    assert np.allclose(np.linalg.norm(out["dir"], axis=1), 1, atol=1e-14)
    has = out["ch_type"] >= 0
    assert np.allclose(np.linalg.norm(out["ch_dir"][has], axis=1), 1, atol=1e-14)
    # every step that moved made progress no longer than its limits
    moved = out["limiter"] >= 0
    assert np.all(out["step"][moved] <= np.minimum(out["s_phys"][moved], out["d_bnd"][moved]) * (1 + 1e-15))


def test_msc_projected_angles_are_gaussian(oracle_mod):
    """Single steps of a 50 MeV electron in Pb: the deflection angle squared is
    the sum of two independent N(0, theta0^2) projected angles, so it follows
    theta0^2 times a chi-square with 2 degrees of freedom."""
    geom = gv_inputs.single_slab("Pb", 100.0)
    o = oracle_mod.Oracle(geom)
    n = 20_000
    st = dict(type=np.full(n, 1, np.int32), pos=np.tile([0.0, 0.0, 50.0], (n, 1)),
              dir=np.tile([0.0, 0.0, 1.0], (n, 1)), ekin=np.full(n, 50.0),
              event=np.arange(n, dtype=np.uint32), tid=np.arange(n, dtype=np.uint64),
              nstep=np.zeros(n, np.uint32))
    out = o.single_step(st, 77)
    sel = (out["limiter"] == 1) & (out["process"] == -1)  # pure continuous-loss steps, no delta/brems
    s = out["step"][sel]
    assert np.allclose(s, s[0])
    th0 = o.lib.or_highland(0, 50.0, s[0])
    cos_t = out["dir"][sel, 2]
    theta2 = np.arccos(np.clip(cos_t, -1, 1)) ** 2
    assert stats.kstest(theta2 / th0**2, stats.chi2(2).cdf).pvalue > 1e-3


def test_highland_scaling(oracle_mod):
    """theta0 is inversely proportional to beta*p at fixed beta and step,
    and grows as sqrt(x/X0) (1 + 0.038 ln(x/(X0 beta^2)))."""
    o = oracle_mod.Oracle(gv_inputs.slab_calorimeter(1))
    lib = o.lib
    x0 = lib.or_mat_X0(0)
    # ultra-relativistic: beta ~ 1 so theta0 * p is energy independent
    a, b = lib.or_highland(0, 5e3, 0.1), lib.or_highland(0, 1e4, 0.1)
    pa, pb = math.sqrt(5e3 * (5e3 + 2 * ME)), math.sqrt(1e4 * (1e4 + 2 * ME))
    assert abs(a * pa / (b * pb) - 1) < 1e-7
    # at x = X0 beta^2 the log term vanishes: theta0 = 13.6/(beta p) sqrt(beta^2)
    T = 3.0
    E = T + ME
    p = math.sqrt(T * (T + 2 * ME))
    beta = p / E
    s = x0 * beta * beta
    assert abs(lib.or_highland(0, T, s) / (13.6 / (beta * p) * beta) - 1) < 1e-13
    # the log correction is clamped at zero for very short steps
    assert lib.or_highland(0, 1e4, 1e-30) == 0.0
