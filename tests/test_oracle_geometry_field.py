"""Pins of the oracle's layered geometry (GeomQuery, Sec. 3.4) and field
propagation (Sec. 3.6).

Distances are compared with brute-force ray marching plus bisection against
point-containment predicates written here from the layer definitions; safety
must never exceed the distance along any direction; locating the point just
past the boundary must give the reported next volume.  The helix is checked
against its invariants (unit direction, conserved momentum component along B,
return after one turn shifted by the pitch) and RK4 against fourth-order
convergence and the helix.
"""
import math

import numpy as np
import pytest

import gv_inputs

ME = 0.51099895
KB = 2.99792458


def _inside_pred(geom):
    b = geom["bounds"]
    n = len(geom["material"])
    env, w = geom["env"], geom["world"]
    if geom["axis"] == 0:
        def vol_of(p):
            if abs(p[0]) <= env[0] and abs(p[1]) <= env[1] and b[0] <= p[2] <= b[-1]:
                return int(min(max(np.searchsorted(b, p[2], side="right"), 1), n))
            if abs(p[0]) <= w[0] and abs(p[1]) <= w[1] and w[2] <= p[2] <= w[3]:
                return 0
            return -1
    else:
        def vol_of(p):
            r = math.hypot(p[0], p[1])
            if r <= b[-1] and abs(p[2]) <= env[0]:
                return int(min(max(np.searchsorted(b, r, side="right"), 1), n))
            if r <= w[0] and abs(p[2]) <= w[1]:
                return 0
            return -1
    return vol_of


def _march(vol_of, v0, p, d, tmax, h):
    """first t at which the containing volume changes (bisection to 1e-11)"""
    t = 0.0
    while t < tmax:
        t2 = t + h
        if vol_of(p + t2 * d) != v0:
            lo, hi = t, t2
            while hi - lo > 1e-11:
                mid = 0.5 * (lo + hi)
                if vol_of(p + mid * d) != v0:
                    hi = mid
                else:
                    lo = mid
            return hi
        t = t2
    return None


@pytest.mark.parametrize("which", ["slab", "barrel"])
def test_distance_vs_ray_marching(oracle_mod, which):
    geom = gv_inputs.slab_calorimeter(4) if which == "slab" else gv_inputs.barrel()
    o = oracle_mod.Oracle(geom)
    vol_of = _inside_pred(geom)
    rng = np.random.default_rng(5)
    st = gv_inputs.random_states(400, 3, geom)
    checked = 0
    for p, d in zip(st["pos"], st["dir"]):
        v = o.locate(p)
        assert v == vol_of(p)
        t, nxt = o.dist_out(v, p, d)
        h = 0.01 if which == "slab" else 0.05
        ref = _march(vol_of, v, p, d, t + 2 * h, h)
        if ref is None:
            continue
        # a marched step can skip a thin layer only if it is thinner than h
        if abs(ref - t) > 1e-9:
            assert ref > t, (p, d, v, t, ref)
            continue
        assert vol_of(p + (t + 1e-9) * d) == nxt
        checked += 1
        # safety never exceeds the distance along random directions
        s = o.safety(v, p)
        for _ in range(5):
            dd = rng.normal(size=3)
            dd /= np.linalg.norm(dd)
            assert s <= o.dist_out(v, p, dd)[0] + 1e-12
    assert checked > 250


def test_axis_aligned_slab_distances(oracle_mod):
    geom = gv_inputs.slab_calorimeter(3)
    o = oracle_mod.Oracle(geom)
    # from the world in front of the stack along +z
    t, nx = o.dist_out(0, np.array([0.0, 0.0, -1.0]), np.array([0.0, 0.0, 1.0]))
    assert t == 1.0 and nx == 1
    # through Pb_0 (0..0.23) into lAr_0
    t, nx = o.dist_out(1, np.array([1.0, 2.0, 0.1]), np.array([0.0, 0.0, 1.0]))
    assert abs(t - 0.13) < 1e-15 and nx == 2
    # sideways out of the envelope into the world
    t, nx = o.dist_out(2, np.array([19.0, 0.0, 0.5]), np.array([1.0, 0.0, 0.0]))
    assert t == 1.0 and nx == 0
    # leaving the world backwards
    t, nx = o.dist_out(0, np.array([0.0, 0.0, -1.0]), np.array([0.0, 0.0, -1.0]))
    assert t == 9.0 and nx == -1
    # safety inside a slab and in the world
    assert abs(o.safety(1, np.array([0.0, 0.0, 0.1])) - 0.1) < 1e-15
    assert abs(o.safety(0, np.array([0.0, 0.0, -1.0])) - 1.0) < 1e-15
    # world faces at 7, 6, 6, 16.4; envelope box at sqrt(3^2 + 4^2 + 4^2)
    assert abs(o.safety(0, np.array([23.0, 24.0, -4.0])) - min(6.0, math.sqrt(9 + 16 + 16))) < 1e-14


def test_barrel_surface_crossing_is_direction_aware(oracle_mod):
    """A point exactly on the envelope's end cap enters only when moving inward."""
    geom = gv_inputs.barrel()
    o = oracle_mod.Oracle(geom)
    p = np.array([30.0, 40.0, -350.0])
    t, nx = o.dist_out(0, p, np.array([0.0, 0.6, -0.8]))
    assert nx == -1 and t > 0
    t, nx = o.dist_out(0, p, np.array([0.0, 0.6, 0.8]))
    assert t == 0.0 and nx >= 1


def _pitch_test(oracle_mod, fn):
    o = oracle_mod.Oracle(gv_inputs.slab_calorimeter(1, (0.0, 4.0, 0.0)))
    lib = o.lib
    import ctypes as C
    dp = C.POINTER(C.c_double)
    B = np.array([0.0, 4.0, 0.0])
    T = 10.0
    p = math.sqrt(T * (T + 2 * ME))
    d0 = np.array([0.6, 0.28, 0.0])
    d0[2] = math.sqrt(1 - d0[0] ** 2 - d0[1] ** 2)
    x0 = np.array([1.0, 2.0, 3.0])
    s_turn = 2 * math.pi * p / (KB * 4.0)
    pos, dr = x0.copy(), d0.copy()
    fn(lib, pos, dr, B, T, s_turn, dp)
    return x0, d0, pos, dr, s_turn


def test_helix_one_turn_returns_shifted_by_pitch(oracle_mod):
    def fn(lib, pos, dr, B, T, s, dp):
        lib.or_helix_move(1, T, B.ctypes.data_as(dp), s, pos.ctypes.data_as(dp), dr.ctypes.data_as(dp))
    x0, d0, pos, dr, s = _pitch_test(oracle_mod, fn)
    assert np.allclose(dr, d0, atol=1e-13)
    assert np.allclose(pos, x0 + np.array([0, 1, 0]) * d0[1] * s, atol=1e-12)


def test_helix_invariants_and_rk4_convergence(oracle_mod):
    o = oracle_mod.Oracle(gv_inputs.slab_calorimeter(1, (0.0, 4.0, 0.0)))
    lib = o.lib
    import ctypes as C
    dp = C.POINTER(C.c_double)
    B = np.array([0.3, 4.0, -0.5])
    bh = B / np.linalg.norm(B)
    rng = np.random.default_rng(9)
    for _ in range(50):
        T = 10 ** rng.uniform(-1, 3)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        typ = int(rng.integers(1, 3))
        s = rng.uniform(0.01, 5.0)
        pos = np.zeros(3)
        dr = d.copy()
        lib.or_helix_move(typ, T, B.ctypes.data_as(dp), s, pos.ctypes.data_as(dp), dr.ctypes.data_as(dp))
        assert abs(np.linalg.norm(dr) - 1) < 1e-14
        assert abs(dr @ bh - d @ bh) < 1e-13
        # the chord is never longer than the arc
        assert np.linalg.norm(pos) <= s * (1 + 1e-14)
    # RK4: error falls ~16x per halving, and converges to the helix
    T, s = 5.0, 1.0
    d = np.array([0.6, 0.0, 0.8])
    ref_p, ref_d = np.zeros(3), d.copy()
    lib.or_helix_move(2, T, B.ctypes.data_as(dp), s, ref_p.ctypes.data_as(dp), ref_d.ctypes.data_as(dp))
    errs = []
    for n in (8, 16, 32, 64):
        p2, d2 = np.zeros(3), d.copy()
        lib.or_rk4_move(2, T, B.ctypes.data_as(dp), s, n, p2.ctypes.data_as(dp), d2.ctypes.data_as(dp))
        errs.append(np.linalg.norm(p2 - ref_p))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(13 < r < 19 for r in ratios), ratios
    p2, d2 = np.zeros(3), d.copy()
    lib.or_rk4_move(2, T, B.ctypes.data_as(dp), s, 2000, p2.ctypes.data_as(dp), d2.ctypes.data_as(dp))
    assert np.linalg.norm(p2 - ref_p) < 1e-9
