"""Edge cases and error paths of the C ABI on the GPU.

* Invalid run options, primaries and geometries are rejected with the
  documented status code, and the context keeps working afterwards.
* Degenerate primaries (on a boundary, axis-aligned, at the top table node,
  just above and below the tracking cut, parallel to B, outside the world,
  empty events in between) in a ragged batch of 264: the FP64 drivers
  reproduce the oracle's deposits and ledgers.
"""
import numpy as np
import pytest

import gv_inputs

pytestmark = pytest.mark.gpu
INVALID_ARG, GEOMETRY = 1, 2


@pytest.fixture(scope="module")
def gv():
    import paper_2005_00949_amd as gvlib
    return gvlib


def test_invalid_run_options_are_rejected(gv):
    geom, prim, seed = gv_inputs.workload("c1", 4)
    # fixed-point scores: a repeated transport is bit-identical
    eng = gv.Engine(geom, precision=gv.P64, deposit_mode=gv.DEPOSIT_FIXED)
    ref = eng.transport(prim, seed)
    bad = [dict(field_method=3), dict(rk_tol=1.5), dict(rk_tol=-1.0), dict(rk_max_substeps=-1),
           dict(rk_max_substeps=(1 << 20) + 1), dict(basket=100), dict(basket=8192), dict(occupancy=40),
           dict(driver=gv.DRIVER_PLAIN, precision=gv.PMIX), dict(queue_order=2), dict(deposit_mode=3),
           dict(fs_alias=32), dict(graph_steps=3), dict(max_steps_per_track=0), dict(chord_tol_cm=0.0)]
    for kw in bad:
        with pytest.raises(gv.GvError) as ei:
            eng.configure(**kw)
        assert ei.value.code == INVALID_ARG, kw
    # the previous configuration still holds
    assert np.array_equal(eng.transport(prim, seed), ref)


def test_invalid_primaries_are_rejected(gv):
    geom, prim, seed = gv_inputs.workload("c1", 4)
    eng = gv.Engine(geom, precision=gv.P64, deposit_mode=gv.DEPOSIT_FIXED)
    ref = eng.transport(prim, seed)
    mutations = [("pdg", 13), ("event", -1), ("ekin", 0.0), ("ekin", 2.0e5), ("ekin", np.nan),
                 ("pos", (np.nan, 0.0, 0.0)), ("dir", (1.0, 1.0, 0.0))]
    for field, value in mutations:
        p = prim.copy()
        p[field][1] = value
        with pytest.raises(gv.GvError) as ei:
            eng.transport(p, seed)
        assert ei.value.code == INVALID_ARG, field
    with pytest.raises(gv.GvError) as ei:
        eng.stage(prim[:0])
    assert ei.value.code == INVALID_ARG
    assert np.array_equal(eng.transport(prim, seed), ref)


def test_invalid_geometries_are_rejected(gv):
    def expect(geom, code):
        with pytest.raises(gv.GvError) as ei:
            gv.Engine(geom)
        assert ei.value.code == code

    g = gv_inputs.slab_calorimeter(4)
    g["bounds"] = g["bounds"].copy()
    g["bounds"][2] = g["bounds"][1]
    expect(g, GEOMETRY)
    g = gv_inputs.slab_calorimeter(4)
    g["material"] = g["material"].copy()
    g["material"][0] = 7
    expect(g, GEOMETRY)
    g = gv_inputs.slab_calorimeter(4)
    g["cell"] = g["cell"].copy()
    g["cell"][0] = -1
    expect(g, GEOMETRY)
    g = gv_inputs.barrel(field_map=gv_inputs.MAP_SOLENOID)
    g["field_map"] = 5
    expect(g, GEOMETRY)
    g = gv_inputs.barrel(b_tesla=(0.5, 0.0, 3.8), field_map=gv_inputs.MAP_SOLENOID)
    expect(g, GEOMETRY)
    g = gv_inputs.barrel(field_map=gv_inputs.MAP_SOLENOID, sol=(0.0, 630.0))
    expect(g, GEOMETRY)
    # a valid geometry still initialises afterwards
    gv.Engine(gv_inputs.slab_calorimeter(4))


def _edge_primaries(geom):
    b = geom["bounds"]
    rows = [  # pdg, T, pos, dir
        (11, 1000.0, (0.0, 0.0, b[0]), (0.0, 0.0, 1.0)),          # on the front face, inward
        (22, 10.0, (1.0, 2.0, b[3]), (0.0, 0.0, -1.0)),           # on an inner boundary, backward
        (-11, 50.0, (0.0, 0.0, 0.5 * (b[2] + b[3])), (1.0, 0.0, 0.0)),   # along x inside a layer
        (11, 1.0e5, (0.0, 0.0, -1.0), (0.0, 0.0, 1.0)),           # the top table node
        (11, 0.1001, (0.0, 0.0, 0.5 * (b[0] + b[1])), (0.6, 0.0, 0.8)),  # just above the tracking cut
        (-11, 0.0999, (0.0, 0.0, 0.5 * (b[1] + b[2])), (0.0, 0.6, 0.8)), # below it: stops, annihilates
        (22, 0.11, (0.0, 0.0, 0.5 * (b[0] + b[1])), (0.0, 1.0, 0.0)),    # soft photon along y
        (11, 30.0, (0.0, 0.0, -1.0), (0.0, 1.0, 0.0)),            # parallel to B (4 T along y)
        (22, 100.0, (1.0e4, 0.0, 0.0), (0.0, 0.0, 1.0)),          # outside the world: escapes at once
        (11, 2.0, (0.0, 0.0, b[-1] + 1e-9), (0.0, 0.0, -1.0)),    # just behind the back face
    ]
    reps = 26
    n = len(rows) * reps + 4
    p = np.zeros(n, dtype=gv_inputs.PRIMARY_DTYPE)
    k = 0
    for r in range(reps):
        for j, (pdg, T, pos, d) in enumerate(rows):
            p[k]["pdg"], p[k]["ekin"] = pdg, T
            p[k]["event"] = 2 * (r * len(rows) + j)        # odd events stay empty
            p[k]["pos"] = pos
            p[k]["dir"] = np.asarray(d) / np.linalg.norm(d)
            k += 1
    for r in range(4):                                    # four extra in the last event
        p[k] = p[r]
        p[k]["event"] = p[k - 1]["event"]
        k += 1
    return p


@pytest.mark.parametrize("driver", ["plain", "batched"])
def test_edge_primaries_match_oracle(gv, oracle_mod, driver):
    geom = gv_inputs.slab_calorimeter(10, (0.0, 4.0, 0.0))
    prim = _edge_primaries(geom)
    assert len(prim) == 264
    seed = 0xED6E
    ref = oracle_mod.Oracle(geom).transport(prim, seed)
    eng = gv.Engine(geom, precision=gv.P64,
                    driver=gv.DRIVER_PLAIN if driver == "plain" else gv.DRIVER_BATCHED)
    edep = eng.transport(prim, seed)
    L = eng.ledger()
    assert edep.shape == ref["edep"].shape
    scale = max(1.0, float(ref["edep"].max()))
    assert np.allclose(edep, ref["edep"], rtol=1e-8, atol=1e-8 * scale)
    assert np.allclose(L, ref["ledger"], rtol=1e-8, atol=1e-8 * scale)
    assert not edep[1::2].any() and not L[1::2].any()      # empty events score nothing
    st = eng.stats()
    c = ref["counters"]
    assert st["total_steps"] == c["steps_gamma"] + c["steps_electron"] + c["steps_positron"]
    assert st["escaped"] == c["escaped"]
