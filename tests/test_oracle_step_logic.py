"""Pins of the oracle's step logic: the decisions one step takes, checked
against values worked out by hand from the geometry, the closed-form cross
sections and the kinematics of a helix, never by re-running the oracle's own
formula.

Each test names the reading it pins (the stage order of Sec. 2.1.2, the field
step rule of Sec. 3.4, the process choice and final states of Sec. 3.5) and
the plausible mistakes in the oracle that it catches:

* continuous-loss limit: a step limited by the energy loss is the whole
  range below 1 mm (the track stops in that step), 1 mm for ranges up to
  5 mm, and 20 % of the range above (the residual range after the step is
  80 % of the initial one);
* linear loss below 1 % of the range, range inversion above;
* straight steps: the boundary distance of a ray, the shorter of physics and
  boundary lengths, the limiter label, exact placement on the crossed face,
  and exponentially distributed physics lengths with mean 1 / Sigma_tot;
* the field rule min(min(phys, bnd), max(field, safety)) with the bending
  estimate sqrt(2 rho eps) (rho the helix's radius of curvature, so that the
  end point leaves the straight line by eps), on both sides of
  max(field, safety), and the push past a boundary;
* relocation after a field move: a change of volume makes the step
  geometry-limited, with no discrete interaction;
* process selection: frequencies Sigma_p / Sigma_tot per particle type at
  three energies (binomial, 4 sigma);
* multiple scattering with the pre-step energy;
* annihilation at rest: two back-to-back 511 keV photons, isotropic.
"""
import math

import numpy as np
import pytest

import gv_inputs

ME = 0.51099895
KB = 2.99792458       # p [MeV] = KB * B [T] * R [cm]
CHORD = 1.0e-3        # bending tolerance of the field rule, cm
PUSH = 1.0e-7         # push past a boundary, cm
GAMMA, ELECTRON, POSITRON = 0, 1, 2
LIM_PHYS, LIM_ELOSS, LIM_GEOM, LIM_FIELD = 0, 1, 2, 3
ALIVE, DEAD = 0, 1
COMPTON, PAIR, MOLLER, BHABHA, BREMS_EM, BREMS_EP = 0, 1, 2, 3, 4, 5
SEED = 0x57E9


def _states(n, typ, T, pos, direction, tid0=0):
    pos = np.broadcast_to(np.asarray(pos, dtype=np.float64), (n, 3)).copy()
    d = np.broadcast_to(np.asarray(direction, dtype=np.float64), (n, 3)).copy()
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return dict(type=np.full(n, typ, dtype=np.int32), pos=pos, dir=d,
                ekin=np.broadcast_to(np.asarray(T, dtype=np.float64), (n,)).copy(),
                event=np.full(n, 7, dtype=np.uint32),
                tid=np.arange(tid0, tid0 + n, dtype=np.uint64), nstep=np.full(n, 3, dtype=np.uint32))


def _isotropic(n, seed):
    rng = np.random.Generator(np.random.Philox(seed))
    c = rng.uniform(-1, 1, n)
    p = rng.uniform(0, 2 * math.pi, n)
    s = np.sqrt(1 - c * c)
    return np.stack([s * np.cos(p), s * np.sin(p), c], axis=1)


def _slab(material, thickness, B=(0.0, 0.0, 0.0)):
    g = gv_inputs.single_slab(material, thickness)
    g["B"] = np.asarray(B, dtype=np.float64)
    return g


def _ks_uniform(x):
    """Kolmogorov-Smirnov distance of x (in [0, 1]) from the uniform law and
    its 1e-3 critical value."""
    x = np.sort(np.asarray(x))
    n = len(x)
    i = np.arange(1, n + 1)
    d = max(np.max(i / n - x), np.max(x - (i - 1) / n))
    return d, 1.95 / math.sqrt(n)


# ---------------------------------------------------------------------------
# continuous-loss step limit (reading: R if R <= 1 mm, else max(0.2 R, 1 mm))
# ---------------------------------------------------------------------------

def test_eloss_limit_below_one_mm_is_the_whole_range(oracle_mod):
    """Below 1 mm of range an energy-loss-limited step is the range itself:
    the track stops in that step and deposits all of its energy.
    Catches: a floor applied below 1 mm (step 1 mm), a fraction applied
    below 1 mm (step 0.2 R, track alive afterwards)."""
    o = oracle_mod.Oracle(_slab("Pb", 20.0))
    for T in (0.2, 0.5, 1.0):
        R = o.table_value(0, "R_em", T)
        assert R < 0.1
        n = 3000
        st = _states(n, ELECTRON, T, (0, 0, 10.0), _isotropic(n, 11))
        r = o.single_step(st, SEED)
        el = r["limiter"] == LIM_ELOSS
        assert el.sum() > n // 2
        assert np.all(np.abs(r["step"][el] - R) <= 1e-12 * R)
        assert np.all(r["status"][el] == DEAD) and np.all(r["ekin"][el] == 0.0)
        assert np.allclose(r["edep"][el], T, rtol=0, atol=1e-15)
        assert np.all(r["step"] <= R * (1 + 1e-12))


def test_eloss_limit_floor_and_fraction(oracle_mod):
    """Ranges of 1-5 mm give 1 mm steps; above 5 mm the step is 20 % of the
    range, so the residual range after an energy-loss-limited step is 80 %
    of the initial one (range table forward and inverse, both pinned by the
    range round trip).  Catches a wrong fraction (0.1, 0.25, ...) or floor."""
    o = oracle_mod.Oracle(_slab("lAr", 400.0))
    Ts = {"floor": None, "fraction": None}
    for T in np.geomspace(0.3, 60.0, 200):
        R = o.table_value(0, "R_em", T)
        if Ts["floor"] is None and 0.15 < R < 0.45:
            Ts["floor"] = T
        if Ts["fraction"] is None and R > 2.0:
            Ts["fraction"] = T
    n = 3000
    for typ, rname in ((ELECTRON, "R_em"), (POSITRON, "R_ep")):
        T = Ts["floor"]
        st = _states(n, typ, T, (0, 0, 200.0), _isotropic(n, 12))
        r = o.single_step(st, SEED)
        el = r["limiter"] == LIM_ELOSS
        assert el.sum() > n // 2
        assert np.all(r["step"][el] == 0.1)
        T = Ts["fraction"]
        R = o.table_value(0, rname, T)
        st = _states(n, typ, T, (0, 0, 200.0), _isotropic(n, 13))
        r = o.single_step(st, SEED)
        el = (r["limiter"] == LIM_ELOSS) & (r["process"] < 0)
        assert el.sum() > n // 2
        assert np.all(np.abs(r["step"][el] - 0.2 * R) <= 1e-12 * R)
        R_after = np.array([o.table_value(0, rname, t) for t in r["ekin"][el]])
        assert np.all(np.abs(R_after - 0.8 * R) <= 1e-9 * R)


def test_linear_loss_below_one_percent_of_the_range(oracle_mod):
    """A step shorter than 1 % of the range loses S(T) s exactly; a longer
    one follows the range: R(T_after) = R(T) - s.  The two differ by more
    than 1e-6 of the loss here (the loss table against the range table's
    secant), so a moved threshold or a swapped branch fails one of the
    checks."""
    o = oracle_mod.Oracle(_slab("lAr", 100.0))
    T = 50.0
    R = o.table_value(0, "R_em", T)
    S = o.table_value(0, "S_em", T)
    n = 400
    for frac, linear in ((0.004, True), (0.008, True), (0.05, False)):
        d = frac * R
        st = _states(n, ELECTRON, T, (0, 0, 100.0 - d), (0, 0, 1))
        r = o.single_step(st, SEED)
        g = (r["limiter"] == LIM_GEOM) & (r["process"] < 0)
        assert g.sum() > n // 2
        s = r["step"][g]
        assert np.all(np.abs(s - d) <= 1e-12)
        assert np.all(r["pos"][g, 2] == 100.0) and np.all(r["vol"][g] == 0)
        dE = r["edep"][g]
        lin_err = np.abs(dE - S * s) / dE
        R_after = np.array([o.table_value(0, "R_em", t) for t in r["ekin"][g]])
        rng_err = np.abs(R_after - (R - s)) / s
        if linear:
            assert lin_err.max() <= 1e-12
            assert rng_err.min() > 1e-7
        else:
            assert rng_err.max() <= 1e-11
            assert lin_err.min() > 1e-6


def test_tracking_cut_during_a_step_deposits_everything(oracle_mod):
    """An electron that would end a step below the tracking cut deposits its
    whole kinetic energy and stops (no sub-cut remainder is carried on)."""
    o = oracle_mod.Oracle(_slab("Pb", 20.0))
    n = 1000
    st = _states(n, ELECTRON, 0.15, (0, 0, 10.0), _isotropic(n, 14))
    r = o.single_step(st, SEED)
    assert np.all((r["status"] == DEAD) | (r["ekin"] >= 0.1))
    dead = r["status"] == DEAD
    assert dead.sum() > n // 2
    assert np.allclose(r["edep"][dead], 0.15, rtol=0, atol=1e-15)
    assert np.all(r["ekin"][dead] == 0.0)


# ---------------------------------------------------------------------------
# straight steps (no field): boundary, physics length, limiter, placement
# ---------------------------------------------------------------------------

def test_straight_photon_steps(oracle_mod):
    """Photon steps in a 1 cm Pb slab: the boundary distance is the ray's
    distance to the slab's face, the step is the shorter of that and the
    physics length, the limiter says which, a boundary-limited step lands
    exactly on the face and enters the next volume, and the physics length
    is exponential with mean 1 / (Sigma_KN + Sigma_pair) from the closed-form
    cross sections.  Catches min/max swaps, a wrong limiter label, a physics
    length drawn from one process only, a missing face snap."""
    o = oracle_mod.Oracle(_slab("Pb", 1.0))
    lib = oracle_mod.load()
    n = 20000
    rng = np.random.Generator(np.random.Philox(15))
    z0 = rng.uniform(0.05, 0.95, n)
    d = _isotropic(n, 16)
    d[:, 2] = np.where(np.abs(d[:, 2]) < 0.05, 0.05, d[:, 2])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pos = np.stack([np.zeros(n), np.zeros(n), z0], axis=1)
    k = 10.0
    st = _states(n, GAMMA, k, pos, d)
    r = o.single_step(st, SEED)
    face = np.where(d[:, 2] > 0, 1.0, 0.0)
    dbnd = (face - z0) / d[:, 2]
    assert np.allclose(r["d_bnd"], dbnd, rtol=1e-12, atol=1e-14)
    assert np.all(r["step"] == np.minimum(r["d_bnd"], r["s_phys"]))
    geo = r["d_bnd"] <= r["s_phys"]
    assert np.all(r["limiter"][geo] == LIM_GEOM) and np.all(r["limiter"][~geo] == LIM_PHYS)
    assert np.all(r["pos"][geo, 2] == face[geo]) and np.all(r["vol"][geo] == 0)
    moved = pos + r["step"][:, None] * d
    assert np.allclose(r["pos"][~geo], moved[~geo], rtol=0, atol=1e-14)
    assert np.all(r["process"][geo] == -1)
    sig = lib.or_xs_compton(0, k) + lib.or_xs_pair(0, k)
    D, crit = _ks_uniform(1.0 - np.exp(-r["s_phys"] * sig))
    assert D < crit, (D, crit)


def test_straight_charged_limiter_labels(oracle_mod):
    """Charged steps without a field: the step is min(physics, energy loss,
    boundary) and the label names the limiting length (boundary first on
    ties, then physics).  The energy-loss length is checked through the
    residual range of energy-loss-limited steps."""
    o = oracle_mod.Oracle(_slab("Pb", 1.0))
    n = 20000
    rng = np.random.Generator(np.random.Philox(17))
    z0 = rng.uniform(0.02, 0.98, n)
    d = _isotropic(n, 18)
    T = 30.0
    st = _states(n, ELECTRON, T, np.stack([np.zeros(n), np.zeros(n), z0], axis=1), d)
    r = o.single_step(st, SEED)
    R = o.table_value(0, "R_em", T)
    s_eloss = max(0.2 * R, 0.1)
    lim = r["limiter"]
    assert {LIM_PHYS, LIM_ELOSS, LIM_GEOM} <= set(np.unique(lim).tolist())
    geo = r["d_bnd"] <= np.minimum(r["s_phys"], s_eloss)
    assert np.all(lim[geo] == LIM_GEOM)
    phys = ~geo & (r["s_phys"] <= s_eloss)
    assert np.all(lim[phys] == LIM_PHYS)
    assert np.all(lim[~geo & ~phys] == LIM_ELOSS)
    assert np.allclose(r["step"], np.minimum(np.minimum(r["d_bnd"], r["s_phys"]), s_eloss), rtol=1e-14, atol=0)


# ---------------------------------------------------------------------------
# the field rule of Sec. 3.4
# ---------------------------------------------------------------------------

def _field_world(B=(0.0, 4.0, 0.0)):
    """A Pb slab z in [0, 0.5] and an lAr slab z in [0.5, 1] (|x|, |y| <=
    20 cm) in a vacuum world |x|, |y| <= 30, z in [-10, 10.8], uniform field."""
    g = gv_inputs.slab_calorimeter(1, B)
    g["bounds"] = np.array([0.0, 0.5, 1.0])
    return g


def _radius(T, B, sin_a=1.0):
    p = math.sqrt(T * (T + 2 * ME))
    return p * sin_a / (KB * B)


def test_field_rule_far_from_boundaries_steps_the_safety(oracle_mod):
    """Deep in the vacuum world the safety exceeds the bending estimate, so
    the step is the safety itself (max(field, safety)), labelled FIELD; the
    safety is the distance to the nearest face worked out by hand.  Catches
    min(field, safety) in place of max."""
    g = _field_world()
    o = oracle_mod.Oracle(g)
    T = 10.0
    delta = math.sqrt(2 * _radius(T, 4.0) * CHORD)
    wx, wy, wz0, wz1 = g["world"]
    ex, ey = g["env"]
    z0, z1 = g["bounds"][0], g["bounds"][-1]
    pts = np.array([[0.0, 0.0, -5.0], [25.0, 0.0, -4.0], [0.0, -22.0, 6.0], [3.0, 4.0, 8.0]])
    dirs = np.array([[1.0, 0, 0], [-1.0, 0, 0], [1.0, 0, 0], [-1.0, 0, 0]])

    def hand_safety(x, y, z):
        walls = min(wx - abs(x), wy - abs(y), z - wz0, wz1 - z)
        qx, qy = max(abs(x) - ex, 0.0), max(abs(y) - ey, 0.0)
        qz = max(z0 - z, z - z1, 0.0)
        return min(walls, math.sqrt(qx * qx + qy * qy + qz * qz))

    hand = np.array([hand_safety(*p) for p in pts])
    assert np.all(hand > delta)
    for typ in (ELECTRON, POSITRON):
        st = _states(len(pts), typ, T, pts, dirs)
        r = o.single_step(st, SEED)
        assert np.allclose(r["safety"], hand, rtol=1e-14, atol=0)
        assert np.all(r["d_bnd"] > hand)
        assert np.all(r["limiter"] == LIM_FIELD)
        assert np.all(r["step"] == r["safety"])


@pytest.mark.parametrize("angle_deg", [90.0, 60.0, 25.0])
def test_field_rule_bending_estimate_and_chord_deviation(oracle_mod, angle_deg):
    """Near a face but moving away from it (safety below the bending estimate,
    the boundary far along the ray), the step is the bending estimate: the
    longest step whose end point on the helix deviates from the straight
    line by the tolerance eps, in the small-angle approximation of Sec. 3.4:
    s^2 / (2 rho) = eps with rho = p / (k_B B sin(alpha)) the radius of
    curvature of the helix.  The end point is checked against the exact
    helix (projected radius a = p sin(alpha) / (k_B B), turning angle
    s k_B B / p), and its distance from the straight-line end point equals
    eps to first order for every pitch angle.  Catches a radius from the
    transverse momentum, a factor other than 2, a wrong tolerance."""
    o = oracle_mod.Oracle(_field_world())
    T = 10.0
    B = 4.0
    a = math.radians(angle_deg)
    p = math.sqrt(T * (T + 2 * ME))
    rho = p / (KB * B * math.sin(a))
    delta = math.sqrt(2 * rho * CHORD)
    # moving away from the back face z = 1, 0.01 cm behind it; the direction
    # makes the angle alpha with B = +y; its transverse part is +z
    u = np.array([0.0, math.cos(a), math.sin(a)])
    start = np.array([0.0, 0.0, 1.01])
    for typ in (ELECTRON, POSITRON):
        st = _states(1, typ, T, start, u)
        r = o.single_step(st, SEED)
        assert r["safety"][0] == pytest.approx(0.01, rel=1e-12)
        assert r["limiter"][0] == LIM_FIELD
        assert r["step"][0] == pytest.approx(delta, rel=1e-12)
        rad = p * math.sin(a) / (KB * B)
        phi = delta * KB * B / p
        disp = r["pos"][0] - start
        assert disp[1] == pytest.approx(delta * math.cos(a), rel=1e-10, abs=1e-15)
        assert disp[2] == pytest.approx(rad * math.sin(phi), rel=1e-10)
        assert abs(disp[0]) == pytest.approx(rad * (1.0 - math.cos(phi)), rel=1e-8)
        # F = q u x B with u x B along -x: the electron bends to +x
        assert np.sign(disp[0]) == (1.0 if typ == ELECTRON else -1.0)
        dev = np.linalg.norm(r["pos"][0] - (start + delta * u))
        assert dev == pytest.approx(CHORD, rel=0.01)


@pytest.mark.parametrize("side", ["below", "above"])
def test_field_rule_boundary_against_bending_estimate(oracle_mod, side):
    """A charged track approaching the stack's front face obliquely at a
    perpendicular distance of half the bending estimate: if the ray meets
    the face before the bending estimate, the step is that distance plus the
    push (GEOM) and the track enters the stack; if after, the step is the
    bending estimate (FIELD) and the track stays in the world."""
    o = oracle_mod.Oracle(_field_world())
    T, B = 10.0, 4.0
    delta = math.sqrt(2 * _radius(T, B) * CHORD)
    h = 0.5 * delta
    dbnd = 0.9 * delta if side == "below" else 1.5 * delta
    c = h / dbnd
    u = np.array([math.sqrt(1 - c * c), 0.0, c])   # in the x-z plane, normal to B = +y
    st = _states(2, ELECTRON, T, (0.0, 0.0, -h), u)
    st["type"][1] = POSITRON
    r = o.single_step(st, SEED)
    assert np.allclose(r["d_bnd"], dbnd, rtol=1e-12)
    assert np.allclose(r["safety"], h, rtol=1e-12)
    if side == "below":
        assert np.all(r["limiter"] == LIM_GEOM)
        assert np.allclose(r["step"], dbnd + PUSH, rtol=1e-14, atol=0)
        # the arc bends by up to eps across the face: the end point is in the
        # stack when it lies beyond the face, and relocation says so
        assert np.all((r["vol"] == 1) == (r["pos"][:, 2] >= 0.0))
        assert np.any(r["vol"] == 1)
    else:
        assert np.all(r["limiter"] == LIM_FIELD)
        assert np.allclose(r["step"], delta, rtol=1e-12, atol=0)
        assert np.all(r["vol"] == 0)


def test_relocation_makes_the_step_geometry_limited(oracle_mod):
    """A positron 5 um in front of the stack, moving parallel to its face and
    bending towards it (F = q u x B points to +z), never meets the face along
    its ray; the field step of sqrt(2 R_c eps) bends it 10 um, so the end
    point lies inside the stack: relocation finds the new volume, the step
    is relabelled GEOM and no interaction is taken.  An electron bending the
    other way stays in the world with a FIELD step."""
    o = oracle_mod.Oracle(_field_world())
    T, B = 10.0, 4.0
    delta = math.sqrt(2 * _radius(T, B) * CHORD)
    h = 0.5 * CHORD
    st = _states(2, POSITRON, T, (0.0, 0.0, -h), (1.0, 0.0, 0.0))
    st["type"][1] = ELECTRON
    r = o.single_step(st, SEED)
    assert r["d_bnd"][0] > 1.0 and r["safety"][0] == pytest.approx(h, rel=1e-12)
    assert r["step"][0] == pytest.approx(delta, rel=1e-12)
    assert r["limiter"][0] == LIM_GEOM and r["vol"][0] == 1 and r["process"][0] == -1
    assert r["pos"][0, 2] > 0.0
    assert r["limiter"][1] == LIM_FIELD and r["vol"][1] == 0 and r["pos"][1, 2] < -h


def test_field_steps_across_boundaries_never_interact(oracle_mod):
    """In material with a field, every step whose end point lies in another
    volume is labelled GEOM and takes no discrete interaction, whatever
    limited it nominally (thin layers make many such steps)."""
    g = gv_inputs.slab_calorimeter(10, (0.0, 4.0, 0.0))
    o = oracle_mod.Oracle(g)
    n = 20000
    rng = np.random.Generator(np.random.Philox(19))
    st = _states(n, ELECTRON, 0.0, np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n),
                                             rng.uniform(0.0, 8.0, n)], axis=1), _isotropic(n, 20))
    st["ekin"] = 10.0 ** rng.uniform(0.0, 3.0, n)
    st["type"] = rng.integers(1, 3, n).astype(np.int32)
    r = o.single_step(st, SEED)
    crossed = r["vol"] != r["vol_pre"]
    assert crossed.sum() > 1000
    assert np.all(r["limiter"][crossed] == LIM_GEOM)
    assert np.all(r["process"][crossed] == -1)
    assert np.all(r["n_children"][crossed & (r["status"] == ALIVE)] == 0)


# ---------------------------------------------------------------------------
# process selection (Sec. 3.5): frequencies against the cross sections
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("typ,energies", [(GAMMA, (3.0, 20.0, 2000.0)),
                                          (ELECTRON, (20.0, 200.0, 2000.0)),
                                          (POSITRON, (20.0, 200.0, 2000.0))])
def test_process_selection_frequencies(oracle_mod, typ, energies):
    """Among physics-limited steps in a thick Pb block, the first process
    (Compton, Moller, Bhabha) is chosen with probability Sigma_1 / Sigma_tot
    of the closed-form cross sections at the pre-step energy (binomial,
    4 sigma, plus 1e-3 for table interpolation).  Catches a swapped or
    inverted choice, and a choice made with post-step cross sections."""
    o = oracle_mod.Oracle(_slab("Pb", 2000.0))
    lib = oracle_mod.load()
    n = 30000
    for T in energies:
        st = _states(n, typ, T, (0, 0, 1000.0), _isotropic(n, 21 + int(T)))
        r = o.single_step(st, SEED)
        ph = r["limiter"] == LIM_PHYS
        if typ == GAMMA:
            s1, s2 = lib.or_xs_compton(0, T), lib.or_xs_pair(0, T)
            first, second = COMPTON, PAIR
        elif typ == ELECTRON:
            s1, s2 = lib.or_xs_moller(0, T), lib.or_xs_brems(0, T)
            first, second = MOLLER, BREMS_EM
        else:
            s1, s2 = lib.or_xs_bhabha(0, T), lib.or_xs_brems(0, T)
            first, second = BHABHA, BREMS_EP
        procs = r["process"][ph]
        m = len(procs)
        assert m > 2000
        assert np.all((procs == first) | (procs == second))
        p = s1 / (s1 + s2)
        f = float(np.mean(procs == first))
        sig = math.sqrt(p * (1 - p) / m)
        assert abs(f - p) <= 4 * sig + 1e-3, (T, f, p, sig)
        assert abs(p - 0.5) > 10 * sig   # the check can tell the two processes apart


# ---------------------------------------------------------------------------
# stage order: scattering with the pre-step energy (Sec. 2.1.2)
# ---------------------------------------------------------------------------

def test_scattering_uses_the_pre_step_energy(oracle_mod):
    """Deflection of energy-loss-limited steps of 2 MeV electrons in lAr
    (20 % of the range, ~25 % of the energy lost): the mean squared polar
    angle is 2 theta0^2 with the Highland width at the pre-step energy
    (written out here; its spot values are pinned elsewhere); the post-step
    energy would give ~1.5 times more."""
    o = oracle_mod.Oracle(_slab("lAr", 400.0))
    lib = oracle_mod.load()
    X0 = lib.or_mat_X0(0)
    T = 2.0
    n = 20000
    st = _states(n, ELECTRON, T, (0, 0, 200.0), (0, 0, 1))
    r = o.single_step(st, SEED)
    ok = (r["limiter"] == LIM_ELOSS) & (r["process"] < 0)
    assert ok.sum() > n // 2
    s = r["step"][ok]
    assert np.all(s == s[0])
    th = np.arccos(np.clip(r["dir"][ok, 2], -1.0, 1.0))

    def theta0(Tk):
        p = math.sqrt(Tk * (Tk + 2 * ME))
        beta = p / (Tk + ME)
        x = s[0] / X0
        return 13.6 / (beta * p) * math.sqrt(x) * (1 + 0.038 * math.log(x / beta ** 2))

    pre = 2 * theta0(T) ** 2
    post = 2 * theta0(float(np.mean(r["ekin"][ok]))) ** 2
    m2 = float(np.mean(th ** 2))
    assert post > 1.3 * pre
    assert abs(m2 / pre - 1) < 5 / math.sqrt(ok.sum()), (m2, pre, post)


# ---------------------------------------------------------------------------
# annihilation at rest and the tracking cut
# ---------------------------------------------------------------------------

def test_annihilation_at_rest(oracle_mod):
    """A positron below the tracking cut deposits its kinetic energy and
    annihilates at rest: two photons of 511 keV, back to back, isotropic
    (cos theta uniform on [-1, 1], azimuth uniform; KS at 1e-3).  An
    electron below the cut only deposits its energy."""
    o = oracle_mod.Oracle(_slab("Pb", 20.0))
    n = 20000
    T = 0.05
    st = _states(n, POSITRON, T, (0, 0, 10.0), (0, 0, 1))
    r = o.single_step(st, SEED)
    assert np.all(r["status"] == DEAD) and np.all(r["n_children"] == 2)
    assert np.all(r["ch_type"] == GAMMA)
    assert np.all(r["ch_ekin"] == ME)
    assert np.allclose(r["edep"], T, rtol=0, atol=1e-15)
    u1, u2 = r["ch_dir"][:, 0], r["ch_dir"][:, 1]
    assert np.all(u1 == -u2)
    assert np.allclose(np.linalg.norm(u1, axis=1), 1.0, rtol=0, atol=1e-14)
    D, crit = _ks_uniform(0.5 * (u1[:, 2] + 1.0))
    assert D < crit, D
    phi = np.arctan2(u1[:, 1], u1[:, 0])
    D, crit = _ks_uniform((phi + math.pi) / (2 * math.pi))
    assert D < crit, D
    assert np.all(np.abs(u1.mean(0)) < 4.0 / math.sqrt(3 * n))
    # positrons stopping inside a step annihilate too
    st = _states(2000, POSITRON, 0.3, (0, 0, 10.0), _isotropic(2000, 22))
    r = o.single_step(st, SEED)
    dead = r["status"] == DEAD
    assert dead.sum() > 1000
    assert np.all(r["n_children"][dead] == 2) and np.all(r["ch_ekin"][dead] == ME)
    assert np.allclose(r["edep"][dead], 0.3, rtol=0, atol=1e-14)
    # electrons below the cut: no secondaries
    st = _states(100, ELECTRON, T, (0, 0, 10.0), (0, 0, 1))
    r = o.single_step(st, SEED)
    assert np.all(r["status"] == DEAD) and np.all(r["n_children"] == 0)
    assert np.allclose(r["edep"], T, rtol=0, atol=1e-15)


def test_tracking_cut_after_a_linear_loss(oracle_mod):
    """The stop rule has two conditions: the energy after the step below the
    tracking cut, or the residual range below the cut's range.  For a short
    (linear-loss) step they differ at second order; a step length between
    (T - T_cut) / S(T) and R(T) - R(T_cut) meets only the first, and the
    track must stop there (the loss S(T) s already takes it below the cut)."""
    o = oracle_mod.Oracle(_slab("Pb", 20.0))
    T = 0.1005
    S = o.table_value(0, "S_em", T)
    R = o.table_value(0, "R_em", T)
    Rc = o.table_value(0, "R_em", 0.1)
    lo, hi = (T - 0.1) / S, R - Rc
    assert hi > lo * (1 + 1e-4) and hi < 0.01 * R
    s = 0.5 * (lo + hi)
    n = 200
    st = _states(n, ELECTRON, T, (0, 0, 20.0 - s), (0, 0, 1))
    r = o.single_step(st, SEED)
    g = r["limiter"] == LIM_GEOM
    assert g.sum() > n // 2
    assert np.all(np.abs(r["step"][g] - s) <= 1e-14)
    assert np.all(r["status"][g] == DEAD) and np.all(r["ekin"][g] == 0.0)
    assert np.allclose(r["edep"][g], T, rtol=0, atol=1e-15)


def test_pair_and_brems_secondary_angles(oracle_mod):
    """Secondary directions of the readings where the paper is silent: the
    pair leptons leave at theta = m / E on opposite azimuths about the
    photon's direction; a bremsstrahlung photon follows its parent."""
    o = oracle_mod.Oracle(_slab("Pb", 2000.0))
    n = 4000
    st = _states(n, GAMMA, 200.0, (0, 0, 1000.0), (0, 0, 1))
    r = o.single_step(st, SEED)
    pair = (r["process"] == PAIR) & (r["n_children"] == 2)
    assert pair.sum() > 1000
    c = r["ch_type"][pair]
    assert np.all(c[:, 0] == ELECTRON) and np.all(c[:, 1] == POSITRON)
    E = r["ch_ekin"][pair] + ME
    u = r["ch_dir"][pair]
    assert np.allclose(u[:, :, 2], np.cos(ME / E), rtol=0, atol=1e-14)
    perp = u[:, :, :2] / np.linalg.norm(u[:, :, :2], axis=2, keepdims=True)
    assert np.allclose(np.sum(perp[:, 0] * perp[:, 1], axis=1), -1.0, rtol=0, atol=1e-9)
    st = _states(n, ELECTRON, 500.0, (0, 0, 1000.0), _isotropic(n, 23))
    r = o.single_step(st, SEED)
    br = r["process"] == BREMS_EM
    assert br.sum() > 1000
    assert np.all(r["ch_type"][br, 0] == GAMMA)
    assert np.all(r["ch_dir"][br, 0] == r["dir"][br])


@pytest.mark.parametrize("which", ["slab0", "slab4T", "barrel"])
def test_stage_prefixes_agree_with_the_whole_step(oracle_mod, which):
    """The step ended after each stage (the per-stage reference of the GPU
    stage tests) is the whole step's state at that point: ComputeIntLen
    leaves the track unmoved and gives the whole step's s_phys, with the
    continuous-loss length of the eloss pins (the whole range below 1 mm,
    else 20 % of it but at least 1 mm, infinite for photons and vacuum);
    GeomQuery adds the whole step's boundary distance and safety;
    Propagation the whole step's length and limiter, and, for a photon or a
    track in vacuum (no deflection or loss follows), its end state;
    scattering the whole step's direction and the loss its energy and
    deposit wherever no discrete interaction follows.  Catches an early exit
    placed in the wrong stage or a stage that writes its output late."""
    geom = {"slab0": gv_inputs.slab_calorimeter(50), "slab4T": gv_inputs.slab_calorimeter(50, (0.0, 4.0, 0.0)),
            "barrel": gv_inputs.barrel()}[which]
    o = oracle_mod.Oracle(geom)
    st = gv_inputs.random_states(4000, 77, geom)
    full = o.single_step(st, SEED)
    alive = full["status"] == 0
    r = o.single_step(st, SEED, oracle_mod.STOP_LIMIT)
    walked = full["limiter"] >= 0
    assert np.array_equal(r["pos"], st["pos"]) and np.array_equal(r["dir"], st["dir"])
    assert np.array_equal(r["ekin"][walked], st["ekin"][walked])
    assert np.array_equal(r["s_phys"], full["s_phys"]) and np.all(r["step"] == 0.0) and np.all(r["limiter"] == -1)
    for i in np.where(walked)[0]:
        typ, T = int(st["type"][i]), float(st["ekin"][i])
        m = int(geom["material"][r["vol_pre"][i] - 1]) if r["vol_pre"][i] >= 1 else -1
        if typ == GAMMA or m < 0:
            assert r["s_eloss"][i] >= 1e299
        else:
            R = o.table_value(m, "R_em" if typ == ELECTRON else "R_ep", T)
            assert r["s_eloss"][i] == (R if R <= 0.1 else max(0.2 * R, 0.1))
    r = o.single_step(st, SEED, oracle_mod.STOP_GEOM)
    assert np.array_equal(r["d_bnd"], full["d_bnd"]) and np.array_equal(r["safety"], full["safety"])
    assert np.array_equal(r["pos"], st["pos"]) and np.all(r["step"] == 0.0)
    r = o.single_step(st, SEED, oracle_mod.STOP_MOVE)
    assert np.array_equal(r["step"], full["step"]) and np.array_equal(r["limiter"], full["limiter"])
    vac = np.array([v < 1 or geom["material"][v - 1] < 0 for v in full["vol_pre"]])
    same = walked & ((st["type"] == GAMMA) | vac) & (full["process"] < 0)
    assert same.sum() > 100
    assert np.array_equal(r["pos"][same], full["pos"][same]) and np.array_equal(r["dir"][same], full["dir"][same])
    assert np.array_equal(r["vol"][walked], full["vol"][walked])
    r = o.single_step(st, SEED, oracle_mod.STOP_MSC)
    quiet = walked & (full["process"] < 0) & alive
    assert np.array_equal(r["dir"][quiet], full["dir"][quiet]) and np.array_equal(r["pos"][quiet], full["pos"][quiet])
    r = o.single_step(st, SEED, oracle_mod.STOP_ELOSS)
    assert quiet.sum() > 1000
    assert np.array_equal(r["ekin"][quiet], full["ekin"][quiet]) and np.array_equal(r["edep"][quiet], full["edep"][quiet])
