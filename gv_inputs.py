"""Seeded synthetic inputs shared by the oracle and the HIP library.

This module holds only *data*: material compositions, layer stacks, beam
definitions and seeded primary generators.  It contains none of the transport
method's arithmetic (no cross sections, no radiation lengths, no geometry
queries, no Philox); each side derives everything it needs from these plain
numbers on its own.

Workloads (Sec. 4 of the paper describes the TestEm3 sampling calorimeter,
50 x (2.3 mm Pb + 5.7 mm liquid Ar), 10 GeV electrons, 4 T transverse field;
the barrel is a synthetic stand-in for the CMS setup of Sec. 6):

* ``c1``: 10 Pb/lAr layers, 100 e- at 1 GeV along +z, no field.
* ``c2``: 50 layers, 1000 e- at 10 GeV, no field.
* ``c3``: 10 layers, 1000 e- at 10 GeV, uniform 4 T along +y.
* ``c4``: 50 layers, 4 T along +y, 10000 events of one primary each,
  e-/e+/gamma by event mod 3, kinetic energy log-uniform 100 MeV..100 GeV,
  Gaussian angular spread of 1 mrad per projected angle.
* ``c5``: cylindrical barrel (10 Si shells, PbWO4 shell, 20 brass/polystyrene
  pairs) in a 3.8 T solenoidal field along z; 2000 events of 50 GeV e-/gamma
  (event mod 2) with eta uniform in [-1, 1], phi uniform.
* ``c5m``: ``c5`` in the field of a finite solenoid (coil radius 315 cm,
  half-length 630 cm, 3.8 T at the centre) instead of a uniform one.
* ``t5``: 10 MeV e- at normal incidence on 2 mm of lead, no field.

Units: cm, MeV, g/cm^3, tesla.
"""
from __future__ import annotations

import math

import numpy as np

PDG_ELECTRON = 11
PDG_POSITRON = -11
PDG_GAMMA = 22

AXIS_Z_SLABS = 0
AXIS_R_SHELLS = 1

# Primary record: 64 bytes, identical field order on both sides.
PRIMARY_DTYPE = np.dtype([
    ("pdg", "<i4"),
    ("event", "<i4"),
    ("ekin", "<f8"),
    ("pos", "<f8", (3,)),
    ("dir", "<f8", (3,)),
])
assert PRIMARY_DTYPE.itemsize == 64

# ---------------------------------------------------------------------------
# Materials: density, elemental composition by mass fraction (Z, A [g/mol],
# w, elemental mean excitation energy [eV]) and the material's mean excitation
# energy I [eV] (0 => combine the elemental values by Bragg additivity).
# Values are the PDG "Atomic and Nuclear Properties" numbers.
# ---------------------------------------------------------------------------
MATERIALS = {
    "Pb": dict(density=11.35, elements=[(82, 207.2, 1.0, 823.0)], I_eV=823.0),
    "lAr": dict(density=1.396, elements=[(18, 39.948, 1.0, 188.0)], I_eV=188.0),
    "Si": dict(density=2.329, elements=[(14, 28.0855, 1.0, 173.0)], I_eV=173.0),
    "PbWO4": dict(density=8.28,
                  elements=[(82, 207.2, 0.45535, 823.0),
                            (74, 183.84, 0.40401, 727.0),
                            (8, 15.999, 0.14064, 95.0)],
                  I_eV=600.7),
    "brass": dict(density=8.53,
                  elements=[(29, 63.546, 0.70, 322.0), (30, 65.38, 0.30, 330.0)],
                  I_eV=0.0),
    "polystyrene": dict(density=1.06,
                        elements=[(6, 12.011, 0.92257, 78.0), (1, 1.008, 0.07743, 19.2)],
                        I_eV=68.7),
}

# Table grid and thresholds (1 keV..100 GeV, 100 bins per decade; 1 MeV
# delta-ray and bremsstrahlung production thresholds; 100 keV tracking cut).
TABLE_SPEC = dict(e_min=1.0e-3, bins_per_decade=100, n_nodes=801,
                  t_cut=1.0, k_cut=1.0, t_track=0.1)

# Transport constants that are run parameters rather than physics.
RUN_SPEC = dict(chord_tol=1.0e-3, push=1.0e-7, rk_frac=0.05,
                max_steps=1 << 20, field_method=0, fs_alias=0,
                rk_tol=1.0e-5, rk_max_sub=16)


def material_list(names):
    return [dict(name=n, **MATERIALS[n]) for n in names]


def slab_calorimeter(n_layers: int, b_tesla=(0.0, 0.0, 0.0)):
    """Layer k: Pb z in [8k, 8k+2.3] mm, lAr z in [8k+2.3, 8k+8] mm.

    Stack volumes are numbered 1..2N (1+2k = Pb_k, 2+2k = lAr_k); volume 0
    is the vacuum world box |x|,|y| <= 30 cm, z in [-10, 0.8N+10] cm; the
    stack's transverse envelope is |x|,|y| <= 20 cm.  Cell = volume - 1.
    """
    bounds = [0.0]
    mats, cells = [], []
    for k in range(n_layers):
        bounds.append(0.8 * k + 0.23)
        bounds.append(0.8 * k + 0.8)
        mats += [0, 1]
        cells += [2 * k, 2 * k + 1]
    return dict(axis=AXIS_Z_SLABS,
                materials=material_list(["Pb", "lAr"]),
                bounds=np.array(bounds, dtype=np.float64),
                material=np.array(mats, dtype=np.int32),
                cell=np.array(cells, dtype=np.int32),
                env=np.array([20.0, 20.0], dtype=np.float64),
                world=np.array([30.0, 30.0, -10.0, 0.8 * n_layers + 10.0], dtype=np.float64),
                B=np.array(b_tesla, dtype=np.float64),
                n_cells=2 * n_layers)


def single_slab(material: str, thickness_cm: float, half_xy: float = 1.0e4):
    """One slab z in [0, thickness] inside a vacuum world (TestEm5-like)."""
    return dict(axis=AXIS_Z_SLABS,
                materials=material_list([material]),
                bounds=np.array([0.0, thickness_cm], dtype=np.float64),
                material=np.array([0], dtype=np.int32),
                cell=np.array([0], dtype=np.int32),
                env=np.array([half_xy, half_xy], dtype=np.float64),
                world=np.array([2 * half_xy, 2 * half_xy, -10.0, thickness_cm + 10.0],
                               dtype=np.float64),
                B=np.zeros(3),
                n_cells=1)


MAP_UNIFORM = 0
MAP_SOLENOID = 1
# synthetic solenoid map (stand-in for an interpolated detector field map):
# coil radius and half-length in cm, central field from B[2]
SOLENOID = (315.0, 630.0)


def barrel(b_tesla=(0.0, 0.0, 3.8), field_map=MAP_UNIFORM, sol=SOLENOID):
    """Cylindrical barrel; every shell has half-length 350 cm.

    Shells from r = 0: beam vacuum [0, 3); ten 300 um Si shells at
    r_in = 3 + i*107/9 separated by vacuum; vacuum up to 129; PbWO4
    [129, 152]; 20 x {brass 5 cm, polystyrene 3.7 mm} with pitch 5.37 cm.
    Outer world: vacuum cylinder r <= 300, |z| <= 400.  Material shells are
    cells 0..50 (Si 0..9, PbWO4 10, then brass/polystyrene alternating).
    """
    VAC = -1
    bounds = [0.0]
    mats, cells = [], []
    cell = 0

    def add(r_hi, m):
        nonlocal cell
        bounds.append(r_hi)
        mats.append(m)
        if m == VAC:
            cells.append(-1)
        else:
            cells.append(cell)
            cell += 1

    for i in range(10):
        r_in = 3.0 + i * 107.0 / 9.0
        add(r_in, VAC)                   # beam vacuum, then the gaps
        add(r_in + 0.03, 0)              # Si
    add(129.0, VAC)
    add(152.0, 1)                        # PbWO4
    for j in range(20):
        add(157.0 + 5.37 * j, 2)         # brass
        add(157.37 + 5.37 * j, 3)        # polystyrene
    assert len(mats) == 62 and cell == 51
    return dict(axis=AXIS_R_SHELLS,
                materials=material_list(["Si", "PbWO4", "brass", "polystyrene"]),
                bounds=np.array(bounds, dtype=np.float64),
                material=np.array(mats, dtype=np.int32),
                cell=np.array(cells, dtype=np.int32),
                env=np.array([350.0, 0.0], dtype=np.float64),
                world=np.array([300.0, 400.0, 0.0, 0.0], dtype=np.float64),
                B=np.array(b_tesla, dtype=np.float64),
                field_map=field_map,
                sol=np.array(sol if field_map == MAP_SOLENOID else (0.0, 0.0), dtype=np.float64),
                n_cells=cell)


def beam(n_events: int, pdg: int, ekin: float, pos=(0.0, 0.0, -1.0), direction=(0.0, 0.0, 1.0)):
    p = np.zeros(n_events, dtype=PRIMARY_DTYPE)
    p["pdg"] = pdg
    p["event"] = np.arange(n_events, dtype=np.int32)
    p["ekin"] = ekin
    p["pos"] = np.asarray(pos, dtype=np.float64)
    d = np.asarray(direction, dtype=np.float64)
    p["dir"] = d / np.linalg.norm(d)
    return p


def mixed_beam(n_events: int, seed: int, e_lo=100.0, e_hi=1.0e5, sigma_rad=1.0e-3,
               pos=(0.0, 0.0, -1.0)):
    """Type by event mod 3 (e-, e+, gamma); T log-uniform in [e_lo, e_hi];
    projected angles N(0, sigma); direction proportional to (tx, ty, 1)."""
    rng = np.random.Generator(np.random.Philox(seed))
    u = rng.random(n_events)
    tx = rng.normal(0.0, sigma_rad, n_events)
    ty = rng.normal(0.0, sigma_rad, n_events)
    p = np.zeros(n_events, dtype=PRIMARY_DTYPE)
    p["pdg"] = np.array([PDG_ELECTRON, PDG_POSITRON, PDG_GAMMA], dtype=np.int32)[
        np.arange(n_events) % 3]
    p["event"] = np.arange(n_events, dtype=np.int32)
    p["ekin"] = e_lo * (e_hi / e_lo) ** u
    p["pos"] = np.asarray(pos, dtype=np.float64)
    d = np.stack([tx, ty, np.ones(n_events)], axis=1)
    p["dir"] = d / np.linalg.norm(d, axis=1, keepdims=True)
    return p


def barrel_beam(n_events: int, seed: int, ekin=5.0e4):
    """Type by event mod 2 (e-, gamma) from the origin; eta ~ U[-1,1], phi ~ U[0,2pi)."""
    rng = np.random.Generator(np.random.Philox(seed))
    eta = rng.uniform(-1.0, 1.0, n_events)
    phi = rng.uniform(0.0, 2.0 * math.pi, n_events)
    theta = 2.0 * np.arctan(np.exp(-eta))
    p = np.zeros(n_events, dtype=PRIMARY_DTYPE)
    p["pdg"] = np.array([PDG_ELECTRON, PDG_GAMMA], dtype=np.int32)[np.arange(n_events) % 2]
    p["event"] = np.arange(n_events, dtype=np.int32)
    p["ekin"] = ekin
    p["pos"] = 0.0
    d = np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)], axis=1)
    p["dir"] = d / np.linalg.norm(d, axis=1, keepdims=True)
    return p


def workload(name: str, n_events: int | None = None):
    """Return (geometry, primaries, seed) for a named workload."""
    if name == "c1":
        n = 100 if n_events is None else n_events
        return slab_calorimeter(10), beam(n, PDG_ELECTRON, 1000.0), 0xC1
    if name == "c2":
        n = 1000 if n_events is None else n_events
        return slab_calorimeter(50), beam(n, PDG_ELECTRON, 1.0e4), 0xC2
    if name == "c3":
        n = 1000 if n_events is None else n_events
        return slab_calorimeter(10, (0.0, 4.0, 0.0)), beam(n, PDG_ELECTRON, 1.0e4), 0xC3
    if name == "c4":
        n = 10000 if n_events is None else n_events
        return slab_calorimeter(50, (0.0, 4.0, 0.0)), mixed_beam(n, 0xC4), 0xC4
    if name == "c5":
        n = 2000 if n_events is None else n_events
        return barrel(), barrel_beam(n, 0xC5), 0xC5
    if name == "c5m":
        # the barrel in the solenoid map (field integrated by adaptive RK45)
        n = 2000 if n_events is None else n_events
        return barrel(field_map=MAP_SOLENOID), barrel_beam(n, 0xC5), 0xC5
    if name == "t5":
        # single-slab transmission / reflection (TestEm5-like, Sec. 4): 10 MeV
        # e- at normal incidence on 2 mm of lead (0.36 X0), no field
        n = 20000 if n_events is None else n_events
        return single_slab("Pb", 0.2), beam(n, PDG_ELECTRON, 10.0), 0x75
    raise ValueError(f"unknown workload {name!r}")


def random_states(n: int, seed: int, geom, e_lo=0.1, e_hi=1.0e5):
    """Random single-step input states for per-step parity tests: positions
    spread over the stack and the world, isotropic directions, log-uniform
    kinetic energies, types uniform over (e-, e+, gamma).  Volume is NOT
    given: each side locates the point itself."""
    rng = np.random.Generator(np.random.Philox(seed))
    st = {}
    st["type"] = rng.integers(0, 3, n).astype(np.int32)
    cth = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    sth = np.sqrt(1.0 - cth * cth)
    st["dir"] = np.stack([sth * np.cos(ph), sth * np.sin(ph), cth], axis=1)
    st["ekin"] = e_lo * (e_hi / e_lo) ** rng.random(n)
    b = geom["bounds"]
    if geom["axis"] == AXIS_Z_SLABS:
        w = geom["world"]
        x = rng.uniform(-w[0] * 0.99, w[0] * 0.99, n)
        y = rng.uniform(-w[1] * 0.99, w[1] * 0.99, n)
        # three quarters inside the stack's z range
        z = np.where(rng.random(n) < 0.75, rng.uniform(b[0], b[-1], n),
                     rng.uniform(w[2] * 0.99, w[3] * 0.99, n))
        pos = np.stack([x, y, z], axis=1)
    else:
        w = geom["world"]
        r = np.where(rng.random(n) < 0.75, rng.uniform(0.0, b[-1], n), rng.uniform(0.0, w[0] * 0.99, n))
        a = rng.uniform(0.0, 2.0 * math.pi, n)
        z = rng.uniform(-w[1] * 0.99, w[1] * 0.99, n)
        pos = np.stack([r * np.cos(a), r * np.sin(a), z], axis=1)
    st["pos"] = pos
    st["event"] = rng.integers(0, 1 << 20, n).astype(np.uint32)
    st["tid"] = rng.integers(0, 1 << 62, n, dtype=np.uint64)
    st["nstep"] = rng.integers(0, 1000, n).astype(np.uint32)
    return st
