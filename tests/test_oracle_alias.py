"""Pins of the oracle's table (alias) final-state samplers, the "sampling
tables" of Sec. 3.5.

* Walker's identity: every column's total probability (its own share plus the
  shares handed to it as an alias) equals its trapezoid weight.
* At a node energy, sampled xi follows the node's piecewise-linear density
  exactly (chi-square on fine bins), and that density is the model's
  analytic one to interpolation accuracy.
* Between nodes, xi follows the ln E-weighted mixture of the two nodes
  (the discrete intermediate variable), within a small total-variation
  distance of the analytic density at that energy.
* The physical variables (eps, x, k) follow the analytic differential cross
  sections (same chi-square as the rejection samplers), and interactions
  still conserve energy; showers still close their energy ledger.
"""
import ctypes as C
import math

import numpy as np
import pytest
from scipy import stats

import gv_inputs

ME = 0.51099895
NX = 64
MODELS = {"compton": 0, "pair": 1, "brems": 2, "moller": 3, "bhabha": 4}


@pytest.fixture(scope="module")
def orc(oracle_mod):
    return oracle_mod.Oracle(gv_inputs.slab_calorimeter(2), run_spec={"fs_alias": 31})


def _table(orc, m, j):
    p, q, a = np.zeros(NX + 1), np.zeros(NX), np.zeros(NX, dtype=np.int32)
    ok = orc.lib.or_alias_table(m, j, p.ctypes.data_as(C.POINTER(C.c_double)),
                                q.ctypes.data_as(C.POINTER(C.c_double)), a.ctypes.data_as(C.POINTER(C.c_int32)))
    return ok, p, q, a


def _xi_samples(orc, m, E, n, seed=1):
    rng = np.random.default_rng(seed)
    u = rng.random((n, 4))
    u[u == 0] = 0.5
    out = np.empty(n)
    buf = np.zeros(4)
    ptr = buf.ctypes.data_as(C.POINTER(C.c_double))
    for i in range(n):
        buf[:] = u[i]
        out[i] = orc.lib.or_alias_xi(m, E, ptr)
    return out


def _pl_cdf(p, x):
    """CDF of the piecewise-linear density through p at xi = k/NX."""
    w = 0.5 * (p[:-1] + p[1:]) / NX
    cum = np.concatenate([[0.0], np.cumsum(w)])
    k = np.minimum((x * NX).astype(int), NX - 1)
    t = x * NX - k
    a, b = p[k], p[k + 1]
    part = (a * t + 0.5 * (b - a) * t * t) / NX
    return (cum[k] + part) / cum[-1]


@pytest.mark.parametrize("model", list(MODELS))
def test_walker_identity(orc, model):
    m = MODELS[model]
    for j in (10, 40, 60, 90, 120):
        ok, p, q, a = _table(orc, m, j)
        if not ok:
            continue
        w = 0.5 * (p[:-1] + p[1:])
        target = w / w.sum()
        got = q.copy()
        for i in range(NX):
            if a[i] != i:
                got[a[i]] += 1.0 - q[i]
        assert np.allclose(got / NX, target, rtol=0, atol=1e-14), (model, j)
        assert (q >= 0).all() and (q <= 1).all() and (a >= 0).all() and (a < NX).all()


@pytest.mark.parametrize("model", list(MODELS))
def test_node_sampling_follows_table_and_model(orc, model):
    m = MODELS[model]
    j = 60                                    # 100 MeV
    E = orc.lib.or_alias_node_energy(j)
    ok, p, q, a = _table(orc, m, j)
    assert ok
    xi = _xi_samples(orc, m, E, 40_000)
    assert stats.kstest(xi, lambda x: _pl_cdf(p, np.asarray(x))).pvalue > 1e-3
    # the node's density is the model's at the node points and interpolates it closely
    xs = np.linspace(0, 1, NX + 1)
    pdf = np.array([orc.lib.or_alias_pdf(m, E, x) for x in xs])
    assert np.allclose(p, pdf, rtol=1e-15, atol=0)
    mid = (xs[:-1] + xs[1:]) / 2
    pm = np.array([orc.lib.or_alias_pdf(m, E, x) for x in mid])
    assert np.max(np.abs(0.5 * (p[:-1] + p[1:]) - pm) / pm.max()) < 3e-3   # linear-interpolation error, 64 intervals


@pytest.mark.parametrize("model", ["compton", "brems", "moller"])
def test_between_nodes_mixture(orc, model):
    m = MODELS[model]
    j = 70
    E0, E1 = orc.lib.or_alias_node_energy(j), orc.lib.or_alias_node_energy(j + 1)
    E = math.sqrt(E0 * E1)                      # lambda = 1/2 in ln E
    _, p0, _, _ = _table(orc, m, j)
    _, p1, _, _ = _table(orc, m, j + 1)
    xi = _xi_samples(orc, m, E, 40_000, seed=2)
    mix = lambda x: 0.5 * _pl_cdf(p0, np.asarray(x)) + 0.5 * _pl_cdf(p1, np.asarray(x))
    assert stats.kstest(xi, mix).pvalue > 1e-3
    # the mixture approximates the model's density at E closely
    xs = np.linspace(0, 1, 4001)
    pdf = np.array([orc.lib.or_alias_pdf(m, E, x) for x in xs])
    cdf = np.concatenate([[0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]))])
    cdf /= cdf[-1]
    assert np.max(np.abs(mix(xs) - cdf)) < 5e-3


def _sample(orc, name, E, n=40_000):
    fn = getattr(orc.lib, "or_sample_" + name + "_alias")
    out = np.zeros(4)
    res = np.empty((n, 4))
    p = out.ctypes.data_as(C.POINTER(C.c_double))
    for i in range(n):
        assert fn(E, 0xA11A5, i % 977, i, 3, p) == 1
        res[i] = out
    return res


def _chi2(samples, cdf, lo, hi, bins=40, log=False):
    edges = np.geomspace(lo, hi, bins + 1) if log else np.linspace(lo, hi, bins + 1)
    counts, _ = np.histogram(samples, bins=edges)
    c = cdf(edges)
    exp = np.diff(c) / (c[-1] - c[0]) * counts.sum()
    keep = exp > 5
    return stats.chi2.sf(((counts[keep] - exp[keep]) ** 2 / exp[keep]).sum(), keep.sum() - 1)


def _num_cdf(pdf, lo, hi, log=False, n=20001):
    x = np.geomspace(lo, hi, n) if log else np.linspace(lo, hi, n)
    f = pdf(x)
    c = np.concatenate([[0], np.cumsum(0.5 * (f[1:] + f[:-1]) * np.diff(x))])
    return lambda e: np.interp(e, x, c)


@pytest.mark.parametrize("k", [0.5, 10.0, 1e3])
def test_compton_alias_physical(orc, k):
    res = _sample(orc, "compton", k)
    kk = k / ME
    eps0 = 1 / (1 + 2 * kk)
    pdf = lambda e: e + 1 / e - (1 - (1 - (1 - e) / (kk * e)) ** 2)
    assert _chi2(res[:, 0], _num_cdf(pdf, eps0, 1.0, log=True), eps0, 1.0, log=kk > 5) > 1e-3
    c = 1 - (1 - res[:, 0]) / (kk * res[:, 0])
    assert np.allclose(res[:, 1], c, atol=1e-12)
    assert stats.kstest(res[:, 2] / (2 * math.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("T", [5.0, 300.0, 3e4])
def test_brems_moller_bhabha_alias_physical(orc, T):
    E = T + ME
    res = _sample(orc, "brems", T)
    assert res[:, 0].min() >= 1.0 and res[:, 0].max() <= T
    pdf = lambda k: (4 / 3 - 4 / 3 * k / E + (k / E) ** 2) / k
    assert _chi2(res[:, 0], _num_cdf(pdf, 1.0, T, log=True), 1.0, T, log=True) > 1e-3
    g = E / ME
    ec = 1.0 / T
    g1, g2 = ((g - 1) / g) ** 2, (2 * g - 1) / g ** 2
    res = _sample(orc, "moller", T)
    pdf_m = lambda e: g1 + 1 / e ** 2 + 1 / (1 - e) ** 2 - g2 / (e * (1 - e))
    assert _chi2(res[:, 0], _num_cdf(pdf_m, ec, 0.5, log=True), ec, 0.5, log=True) > 1e-3
    b2 = 1 - 1 / g ** 2
    y = 1 / (g + 1)
    B1, B2, B4 = 2 - y * y, (1 - 2 * y) * (3 + y * y), (1 - 2 * y) ** 3
    B3 = B4 + (1 - 2 * y) ** 2
    res = _sample(orc, "bhabha", T)
    pdf_b = lambda e: 1 / (b2 * e * e) - B1 / e + B2 - B3 * e + B4 * e * e
    assert _chi2(res[:, 0], _num_cdf(pdf_b, ec, 1.0, log=True), ec, 1.0, log=True) > 1e-3


@pytest.mark.parametrize("k", [1.2, 30.0, 4e3])
def test_pair_alias_physical(orc, k):
    res = _sample(orc, "pair", k)
    a = ME / k
    assert res[:, 0].min() >= a and res[:, 0].max() <= 1 - a
    pdf = lambda x: 1 - 4 / 3 * x * (1 - x)
    assert _chi2(res[:, 0], _num_cdf(pdf, a, 1 - a), a, 1 - a) > 1e-3


def test_alias_showers_close_their_ledger(oracle_mod):
    geom, prim, seed = gv_inputs.workload("c2", 4)
    o = oracle_mod.Oracle(geom, run_spec={"fs_alias": 31})
    r = o.transport(prim, seed)
    L = r["ledger"]
    Ein = np.bincount(prim["event"], weights=prim["ekin"])
    lhs = Ein + 2 * ME * L[:, 3] - 2 * ME * L[:, 2]
    rhs = r["edep"].sum(1) + L[:, 0] + L[:, 1]
    assert np.max(np.abs(lhs - rhs) / lhs) < 1e-10
    assert r["counters"]["rejection_exhausted"] == 0
    # the tables change the histories but not the scale of a contained shower
    ref = oracle_mod.Oracle(geom).transport(prim, seed)
    assert abs(r["edep"].sum() / ref["edep"].sum() - 1) < 0.03
