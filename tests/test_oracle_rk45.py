"""Pins of the oracle's non-uniform field and adaptive Runge-Kutta
integration (Sec. 3.6).

* The Dormand-Prince coefficients satisfy every order condition up to order
  five (seventeen rooted trees) for the propagating weights, up to order four
  for the embedded weights, the row-sum condition, and first-same-as-last.
* In a uniform field the adaptive integration reproduces the closed-form
  helix within a multiple of the tolerance, its error falls as the tolerance
  is tightened, and a move cut short by the attempt cap lands on the helix
  at the length it did integrate.
* The solenoid map equals the field of a finite current sheet computed here
  independently, by quadrature of exact current-loop fields (complete
  elliptic integrals), to the order of its off-axis expansion; it is curl
  free, has the textbook half-strength field at the coil ends, and becomes
  uniform as the coil grows long.
* In the map, RK45 and fine-step RK4 converge to the same trajectory.
* A transport with RK45 closes the energy ledger and counts its substeps.
"""
import math

import numpy as np
import pytest

import gv_inputs

ME = 0.51099895
KB = 2.99792458


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------- tableau
def test_dp45_order_conditions(oracle_mod):
    A, b, bh, c = oracle_mod.dp45_tableau()
    one = np.ones(7)
    # explicit: strictly lower triangular; row sums are the nodes
    assert np.all(np.triu(A) == 0.0)
    assert np.allclose(A @ one, c, atol=1e-15)
    # first same as last: the last row is the 5th-order weight vector, node 1
    assert np.array_equal(A[6], b)
    assert c[6] == 1.0
    Ac = A @ c
    trees = [  # (elementary weight as a function of the weights w, 1/gamma)
        (lambda w: w @ one, 1.0),
        (lambda w: w @ c, 1 / 2),
        (lambda w: w @ c**2, 1 / 3),
        (lambda w: w @ Ac, 1 / 6),
        (lambda w: w @ c**3, 1 / 4),
        (lambda w: w @ (c * Ac), 1 / 8),
        (lambda w: w @ (A @ c**2), 1 / 12),
        (lambda w: w @ (A @ Ac), 1 / 24),
        (lambda w: w @ c**4, 1 / 5),
        (lambda w: w @ (c**2 * Ac), 1 / 10),
        (lambda w: w @ (Ac**2), 1 / 20),
        (lambda w: w @ (c * (A @ c**2)), 1 / 15),
        (lambda w: w @ (A @ c**3), 1 / 20),
        (lambda w: w @ (c * (A @ Ac)), 1 / 30),
        (lambda w: w @ (A @ (c * Ac)), 1 / 40),
        (lambda w: w @ (A @ (A @ c**2)), 1 / 60),
        (lambda w: w @ (A @ (A @ Ac)), 1 / 120),
    ]
    for k, (phi, g) in enumerate(trees):
        assert abs(phi(b) - g) < 1e-14, ("5th-order weights, tree", k)
    for k, (phi, g) in enumerate(trees[:8]):
        assert abs(phi(bh) - g) < 1e-14, ("embedded weights, tree", k)
    # the embedded pair is genuinely of order 4: it misses some 5th-order tree
    assert max(abs(phi(bh) - g) for phi, g in trees[8:]) > 1e-4


def test_dp45_fixed_step_order_on_a_nonlinear_problem(oracle_mod):
    # a textbook explicit RK driver on y' = 1 + y^2, y(0) = 0 (exact tan t):
    # per halving of the step the global error of the embedded weights falls
    # ~16x (order 4) and that of the propagating weights at least 2^5 = 32x
    # (this pair's 5th-order error constants are small, so order-6 terms
    # still show at these steps)
    A, b, bh, c = oracle_mod.dp45_tableau()

    def run(w, n):
        y, h = 0.0, 1.0 / n
        for _ in range(n):
            k = np.zeros(7)
            for i in range(7):
                k[i] = 1.0 + (y + h * (A[i, :i] @ k[:i])) ** 2
            y = y + h * (w @ k)
        return y

    exact = math.tan(1.0)
    e5 = [abs(run(b, n) - exact) for n in (10, 20, 40)]
    e4 = [abs(run(bh, n) - exact) for n in (10, 20, 40)]
    r5 = [e5[i] / e5[i + 1] for i in range(2)]
    r4 = [e4[i] / e4[i + 1] for i in range(2)]
    assert all(r > 30 for r in r5), r5
    assert all(13 < r < 19 for r in r4), r4


# ---------------------------------------------------------- uniform field
@pytest.mark.parametrize("typ,T,B,d,s", [
    (1, 10.0, (0.0, 0.0, 3.8), (0.8, 0.0, 0.6), 20.0),      # e-, many turns
    (2, 2.0, (0.0, 4.0, 0.0), (0.3, 0.1, 0.95), 3.0),        # e+
    (1, 500.0, (0.3, 4.0, -0.5), (0.0, 0.0, 1.0), 50.0),     # stiff, oblique field
    (2, 0.3, (0.0, 0.0, 3.8), (1.0, 0.0, 0.0), 0.01),        # short step, one substep
])
def test_rk45_matches_helix_in_uniform_field(oracle_mod, typ, T, B, d, s):
    d = _unit(d)
    f = oracle_mod.make_field(oracle_mod.MAP_UNIFORM, B)
    x0 = np.array([1.0, -2.0, 3.0])
    for tol in (1e-5, 1e-7, 1e-9):
        p, u, sd, na, nr = oracle_mod.rk45_move(typ, T, f, s, tol, 100000, x0, d)
        ph, uh = oracle_mod.helix_move(typ, T, B, s, x0, d)
        assert sd == s and na >= 1
        assert abs(np.linalg.norm(u) - 1.0) < 1e-14
        # errors are per unit length (position) and per substep (direction)
        assert np.linalg.norm(p - ph) < 20 * tol * s + 1e-12, (tol, np.linalg.norm(p - ph))
        assert np.linalg.norm(u - uh) < 20 * tol * (na + nr) + 1e-12
        # the momentum component along B is conserved
        bh = _unit(B)
        assert abs(u @ bh - d @ bh) < 20 * tol * (na + nr) + 1e-12


def test_rk45_error_and_work_follow_the_tolerance(oracle_mod):
    f = oracle_mod.make_field(oracle_mod.MAP_UNIFORM, (0.0, 0.0, 3.8))
    d = _unit((0.8, 0.0, 0.6))
    ph, _ = oracle_mod.helix_move(1, 10.0, (0.0, 0.0, 3.8), 20.0, np.zeros(3), d)
    errs, work = [], []
    for tol in (1e-4, 1e-6, 1e-8, 1e-10):
        p, u, sd, na, nr = oracle_mod.rk45_move(1, 10.0, f, 20.0, tol, 100000, np.zeros(3), d)
        errs.append(np.linalg.norm(p - ph))
        work.append(na)
    assert all(errs[i] > 5 * errs[i + 1] for i in range(3)), errs
    assert all(work[i] < work[i + 1] for i in range(3)), work
    # the position error per unit length of a substep goes as h^4, so 100x
    # tighter tolerance needs about 100^(1/4) ~ 3.2x shorter substeps
    assert 2.5 < work[3] / work[2] < 4.2 and 2.5 < work[2] / work[1] < 4.2, work


def test_rk45_error_constant_and_first_attempt(oracle_mod):
    """The first substep is sized from the pair's error on circular motion,
    err ~ K (h |du/ds|)^4 with K = 8.1e-4: K is recomputed here from the
    tableau, and a long step in a uniform field then runs with few rejected
    attempts."""
    A, b, bh, c = oracle_mod.dp45_tableau()
    e = b - bh

    def err(theta, phi):
        h = theta
        y = np.array([0.0, 0.0, 0.0, math.cos(phi), math.sin(phi), 0.0])
        k = np.zeros((7, 6))
        for i in range(7):
            yi = y + h * (A[i, :i] @ k[:i])
            k[i, :3] = yi[3:]
            k[i, 3:] = (yi[4], -yi[3], 0.0)
        ex = e @ k
        return max(np.abs(ex[:3]).max(), h * np.abs(ex[3:]).max())

    K = max(err(0.02, p) / 0.02**4 for p in np.linspace(0.0, math.pi / 2, 64))
    assert abs(K / 8.1e-4 - 1) < 0.01, K
    f = oracle_mod.make_field(oracle_mod.MAP_UNIFORM, (0.0, 0.0, 3.8))
    for tol in (1e-5, 1e-6, 1e-7):
        p, u, sd, na, nr = oracle_mod.rk45_move(1, 10.0, f, 50.0, tol, 100000, np.zeros(3), (1.0, 0.0, 0.0))
        assert sd == 50.0 and nr <= 2, (tol, na, nr)


def test_rk45_attempt_cap_cuts_the_step_on_the_trajectory(oracle_mod):
    f = oracle_mod.make_field(oracle_mod.MAP_UNIFORM, (0.0, 0.0, 3.8))
    d = _unit((0.8, 0.0, 0.6))
    p, u, sd, na, nr = oracle_mod.rk45_move(1, 10.0, f, 20.0, 1e-7, 12, np.zeros(3), d)
    assert na + nr == 12 and 0.0 < sd < 20.0
    ph, uh = oracle_mod.helix_move(1, 10.0, (0.0, 0.0, 3.8), sd, np.zeros(3), d)
    assert np.linalg.norm(p - ph) < 1e-5 and np.linalg.norm(u - uh) < 1e-5
    # no length: nothing moves, no substep
    p, u, sd, na, nr = oracle_mod.rk45_move(1, 10.0, f, 0.0, 1e-7, 10, np.ones(3), d)
    assert (sd, na, nr) == (0.0, 0, 0) and np.array_equal(p, np.ones(3)) and np.allclose(u, d)


# ---------------------------------------------------------- solenoid map
def _loop_field(a, rho, z):
    """Exact field of a circular current loop of radius a in the plane z=0,
    per unit mu0 I: (B_rho, B_z) at cylindrical (rho, z)."""
    from scipy.special import ellipe, ellipk
    q = (a + rho) ** 2 + z * z
    m = 4 * a * rho / q
    K, E = ellipk(m), ellipe(m)
    d = (a - rho) ** 2 + z * z
    bz = 1 / (2 * math.pi * math.sqrt(q)) * (K + (a * a - rho * rho - z * z) / d * E)
    if rho == 0.0:
        return 0.0, bz
    br = z / (2 * math.pi * rho * math.sqrt(q)) * (-K + (a * a + rho * rho + z * z) / d * E)
    return br, bz


def _sheet_field(R, L, rho, z):
    """Finite current sheet = loops spread uniformly over [-L, L] (unit
    current per length), by adaptive quadrature."""
    from scipy.integrate import quad
    kw = dict(epsabs=1e-13, epsrel=1e-12, limit=200)
    br = quad(lambda z0: _loop_field(R, rho, z - z0)[0], -L, L, **kw)[0]
    bz = quad(lambda z0: _loop_field(R, rho, z - z0)[1], -L, L, **kw)[0]
    return br, bz


def test_solenoid_matches_current_sheet_by_biot_savart(oracle_mod):
    R, L, B0 = 1.0, 3.0, 3.8
    f = oracle_mod.make_field(oracle_mod.MAP_SOLENOID, (0.0, 0.0, B0), (R, L))
    norm = B0 / _sheet_field(R, L, 0.0, 0.0)[1]
    phi = 0.7
    for z in (0.0, 1.5, 2.7, 3.0, 3.4, 4.5):
        for rho in (0.0, 0.02, 0.05):
            x = np.array([rho * math.cos(phi), rho * math.sin(phi), z])
            B = oracle_mod.field_eval(f, x)
            br, bz = _sheet_field(R, L, rho, z)
            br, bz = br * norm, bz * norm
            # the second-order expansion leaves O(rho^3) in B_r, O(rho^4) in B_z
            tol = 1e-10 + 2e1 * B0 * rho**3 / R**3
            assert abs(B[2] - bz) < tol, (z, rho, B[2], bz)
            assert abs(math.hypot(B[0], B[1]) - abs(br)) < tol, (z, rho, B, br)
            if rho > 0:
                # radial component points along +-(x, y) with the sheet's sign
                assert (B[0] * x[0] + B[1] * x[1]) * br >= 0.0


def test_solenoid_limits_and_curl(oracle_mod):
    B0 = 3.8
    f = oracle_mod.make_field(oracle_mod.MAP_SOLENOID, (0.0, 0.0, B0), (315.0, 630.0))
    assert np.allclose(oracle_mod.field_eval(f, [0.0, 0.0, 0.0]), [0.0, 0.0, B0], rtol=0, atol=1e-14)
    # long coil: uniform inside, half strength at the ends
    flong = oracle_mod.make_field(oracle_mod.MAP_SOLENOID, (0.0, 0.0, B0), (1.0, 1.0e5))
    for x in ([0.3, -0.2, 0.0], [0.1, 0.4, 50.0]):
        assert np.allclose(oracle_mod.field_eval(flong, x), [0.0, 0.0, B0], atol=1e-8)
    assert abs(oracle_mod.field_eval(flong, [0.0, 0.0, 1.0e5])[2] / B0 - 0.5) < 1e-9
    # symmetric in z, and B_r odd in z
    a = oracle_mod.field_eval(f, [40.0, 30.0, 200.0])
    b = oracle_mod.field_eval(f, [40.0, 30.0, -200.0])
    assert np.allclose([a[0], a[1], a[2]], [-b[0], -b[1], b[2]], atol=1e-14)
    # zero curl (central differences), divergence of order r^2
    h = 1e-3
    for x in ([40.0, 30.0, 200.0], [-100.0, 20.0, 600.0], [5.0, 0.0, 650.0]):
        x = np.array(x)
        J = np.zeros((3, 3))  # J[i, j] = dB_i / dx_j
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            J[:, j] = (oracle_mod.field_eval(f, x + e) - oracle_mod.field_eval(f, x - e)) / (2 * h)
        curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        assert np.abs(curl).max() < 1e-8, curl
        r = math.hypot(x[0], x[1])
        assert abs(np.trace(J)) < 5 * B0 * r**2 / 315.0**3
    # uniform map returns its vector everywhere
    fu = oracle_mod.make_field(oracle_mod.MAP_UNIFORM, (0.1, 0.2, 0.3))
    assert np.array_equal(oracle_mod.field_eval(fu, [9.0, 8.0, 7.0]), [0.1, 0.2, 0.3])


def test_rk45_and_rk4_agree_in_the_solenoid(oracle_mod):
    f = oracle_mod.make_field(oracle_mod.MAP_SOLENOID, (0.0, 0.0, 3.8), (3.0, 5.0))
    x0 = np.array([0.5, 0.0, 3.5])   # near the coil end, where the field bends
    d = _unit((0.2, 0.9, 0.4))
    p5, u5, sd, na, nr = oracle_mod.rk45_move(1, 20.0, f, 30.0, 1e-10, 100000, x0, d)
    p4, u4 = oracle_mod.rk4_field_move(1, 20.0, f, 30.0, 40000, x0, d)
    assert sd == 30.0
    assert np.linalg.norm(p5 - p4) < 1e-7 and np.linalg.norm(u5 - u4) < 1e-7
    # a helix in the start-point field is not the same trajectory here
    ph, _ = oracle_mod.helix_move(1, 20.0, oracle_mod.field_eval(f, x0), 30.0, x0, d)
    assert np.linalg.norm(ph - p5) > 1e-3


# -------------------------------------------------------------- transport
def test_transport_with_rk45_in_the_map(oracle_mod):
    geom, prim, seed = gv_inputs.workload("c5m", 6)
    prim = prim.copy()
    prim["ekin"] = 2000.0
    o = oracle_mod.Oracle(geom, run_spec={"field_method": oracle_mod.FIELD_RK45})
    r = o.transport(prim, seed)
    L = r["ledger"]
    e_in = np.bincount(prim["event"], weights=prim["ekin"], minlength=len(L))
    resid = np.abs(e_in - r["edep"].sum(1) - L[:, 0] - L[:, 1] - 2 * ME * (L[:, 2] - L[:, 3]))
    assert resid.max() < 1e-8 * e_in.max()
    c = r["counters"]
    assert c["rk_substeps"] > 0 and c["rk_substeps"] >= c["steps_electron"] // 4
    # the helix leaves the RK counters at zero
    rh = oracle_mod.Oracle(geom).transport(prim, seed)
    assert rh["counters"]["rk_substeps"] == 0 and rh["counters"]["rk_rejected"] == 0


def test_rk45_uniform_field_single_steps_match_helix(oracle_mod):
    # no attempt cap here: every step is integrated over its full length
    geom = gv_inputs.slab_calorimeter(4, (0.0, 4.0, 0.0))
    st = gv_inputs.random_states(400, 31, geom)
    a = oracle_mod.Oracle(geom).single_step(st, 5)
    b = oracle_mod.Oracle(geom, run_spec={"field_method": oracle_mod.FIELD_RK45,
                                          "rk_tol": 1e-9, "rk_max_sub": 100000}).single_step(st, 5)
    charged = st["type"] != 0
    assert charged.sum() > 100
    # same step lengths and limiters; positions within the tolerance per length
    same = (a["limiter"] == b["limiter"]) & (a["vol"] == b["vol"])
    assert (~same).mean() < 0.01
    assert np.array_equal(a["step"][same], b["step"][same])
    dp = np.linalg.norm(a["pos"] - b["pos"], axis=1)
    assert np.all(dp[same] <= 1e-7 * np.maximum(a["step"][same], 1.0))
