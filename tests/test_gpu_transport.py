"""GPU transport parity against the oracle, through the C ABI.

* Tiny showers (brute force): every step record (event, track id, step) of the
  FP64 GPU drivers equals the oracle's, with continuous fields within a
  history tolerance (1e-6 normwise: single-step differences of ~1e-16 grow
  along long histories in a field).
* Per-event energy ledger closes for every driver and precision.
* Determinism: identical histories for any basket / occupancy / inner-step /
  queue-order setting (deposits equal up to atomic summation order).
* Queue overflow: the event window is rerun with half the events in flight
  and reproduces the unconstrained result.
* Per-layer deposits of the mixed-precision batched path against the oracle:
  paired test, |mean difference| <= 3 sigma_paired and <= 0.5% for layers
  holding at least 1% of the deposit.
"""
import math

import numpy as np
import pytest

import gv_inputs

pytestmark = pytest.mark.gpu
ME = 0.51099895


@pytest.fixture(scope="module")
def gv():
    import paper_2005_00949_amd as gvlib
    return gvlib


def _trace_map(tr):
    return {(int(r["event"]), int(r["tid"]), int(r["nstep"])): r for r in tr}


def _compare_histories(got, ref, tol):
    g, r = _trace_map(got), _trace_map(ref)
    missing = set(r) - set(g)
    extra = set(g) - set(r)
    worst = 0.0
    bad = 0
    for k in set(r) & set(g):
        a, b = g[k], r[k]
        if (a["limiter"], a["vol_pre"], a["vol_post"], a["process"], a["n_children"], a["type"]) != \
           (b["limiter"], b["vol_pre"], b["vol_post"], b["process"], b["n_children"], b["type"]):
            bad += 1
            continue
        # normwise, as for single steps: energies against the pre-step kinetic
        # energy, lengths against max(|position|, 1 cm), directions as unit vectors
        e_scale = max(abs(float(b["ekin"])) + abs(float(b["edep"])), 1e-3)
        l_scale = max(float(np.max(np.abs(b["pos"]))), abs(float(b["step"])), 1.0)
        for f, sc in (("pos", l_scale), ("dir", 1.0), ("ekin", e_scale), ("edep", e_scale), ("step", l_scale)):
            e = np.max(np.abs(np.asarray(a[f]) - np.asarray(b[f]))) / sc
            worst = max(worst, float(e))
    return len(missing), len(extra), bad, worst


CASES = {
    "slab_e10": (lambda: gv_inputs.slab_calorimeter(10), lambda: gv_inputs.beam(10, 11, 10.0)),
    "slab_g50": (lambda: gv_inputs.slab_calorimeter(10), lambda: gv_inputs.beam(10, 22, 50.0)),
    # 100 MeV: a 10 MeV e- at 4 T (radius 0.87 cm) starting 1 cm before the
    # stack circles in vacuum until the looper cap
    "field_e100": (lambda: gv_inputs.slab_calorimeter(10, (0.0, 4.0, 0.0)), lambda: gv_inputs.beam(10, 11, 100.0)),
    "barrel_g50": (lambda: gv_inputs.barrel(), lambda: gv_inputs.barrel_beam(4, 5, 50.0)),
}
# History tolerance per case, normwise: without a field the GPU and the oracle
# round the same expressions in the same order (measured worst 9e-13); in a
# field, helix phases carry last-bit differences of the trigonometric
# functions and amplify them along hundreds of steps (measured 1e-10 on the
# slab in 4 T, 3.3e-8 in the barrel with table sampling).
HIST_TOL = {"slab_e10": 1e-11, "slab_g50": 1e-11, "field_e100": 1e-8, "barrel_g50": 1e-7}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("driver", ["plain", "batched1", "batched8", "batched4_stable", "plain_tables",
                                    "batched4_tables"])
def test_tiny_shower_histories_fp64(gv, oracle_mod, case, driver):
    geom, prim = CASES[case][0](), CASES[case][1]()
    seed = 0x5EED
    fs = 31 if driver.endswith("tables") else 0
    ref = oracle_mod.Oracle(geom, run_spec={"fs_alias": fs}).transport(prim, seed, trace_cap=2_000_000)
    cfg = dict(precision=gv.P64, trace_cap=2_000_000, fs_alias=fs)
    if driver.startswith("plain"):
        cfg["driver"] = gv.DRIVER_PLAIN
    else:
        cfg.update(driver=gv.DRIVER_BATCHED, inner_steps={"batched1": 1, "batched8": 8}.get(driver, 4), basket=128,
                   queue_order=gv.ORDER_STABLE if driver.endswith("stable") else gv.ORDER_ARRIVAL)
    eng = gv.Engine(geom, **cfg)
    edep = eng.transport(prim, seed)
    got = eng.trace()
    st = eng.stats()
    assert st["trace_records"] < 2_000_000
    missing, extra, bad, worst = _compare_histories(got, ref["trace"], HIST_TOL[case])
    n_ref = len(ref["trace"])
    print(f"\n[{case}/{driver}] oracle steps {n_ref}, gpu {len(got)}, missing {missing}, extra {extra}, "
          f"discrete mismatches {bad}, worst scaled error {worst:.2e}")
    assert missing == 0 and extra == 0 and bad == 0
    # single steps agree to 1e-12; along a history the differences are carried
    # and amplified by later steps (scattering angles, helix phases, distances
    # to nearly tangent boundaries)
    assert worst < HIST_TOL[case]
    assert np.allclose(edep, ref["edep"], rtol=1e-8, atol=1e-8 * max(1.0, ref["edep"].max()))
    counts = ref["counters"]
    assert st["total_steps"] == counts["steps_gamma"] + counts["steps_electron"] + counts["steps_positron"] \
        or missing + extra > 0


def _ledger_ok(prim, edep, L, tol):
    Ein = np.bincount(prim["event"], weights=prim["ekin"])
    lhs = Ein + 2 * ME * L[:, 3] - 2 * ME * L[:, 2]
    rhs = edep.sum(1) + L[:, 0] + L[:, 1]
    return float(np.max(np.abs(lhs - rhs) / lhs))


@pytest.mark.parametrize("name,n", [("c1", 40), ("c3", 10), ("c4", 60), ("c5", 4)])
@pytest.mark.parametrize("mode", ["plain64", "batch64", "batchmix", "batchmix_tables"])
def test_ledger_closure(gv, name, n, mode):
    geom, prim, seed = gv_inputs.workload(name, n)
    cfg = {"plain64": dict(driver=gv.DRIVER_PLAIN, precision=gv.P64),
           "batch64": dict(driver=gv.DRIVER_BATCHED, precision=gv.P64),
           "batchmix": dict(driver=gv.DRIVER_BATCHED, precision=gv.PMIX),
           "batchmix_tables": dict(driver=gv.DRIVER_BATCHED, precision=gv.PMIX, fs_alias=gv.FS_ALL)}[mode]
    eng = gv.Engine(geom, **cfg)
    edep = eng.transport(prim, seed)
    resid = _ledger_ok(prim, edep, eng.ledger(), 0)
    assert resid < (1e-10 if not mode.startswith("batchmix") else 1e-5), resid
    st = eng.stats()
    assert st["killed"] == 0


@pytest.mark.parametrize("driver", ["plain", "batched"])
def test_lane_use_counter(gv, driver):
    """lane_slots counts 64 lanes per step-loop iteration of every wavefront:
    never fewer than the steps taken, and 0 for the plain driver."""
    geom, prim, seed = gv_inputs.workload("c3", 30)
    eng = gv.Engine(geom, precision=gv.P64, driver=gv.DRIVER_PLAIN if driver == "plain" else gv.DRIVER_BATCHED,
                    basket=128, inner_steps=4)
    eng.transport(prim, seed)
    st = eng.stats()
    if driver == "plain":
        assert st["lane_slots"] == 0
    else:
        use = st["total_steps"] / st["lane_slots"]
        print(f"\n[c3 batched] lane use {use:.3f}")
        assert 0.05 < use <= 1.0


def test_determinism_across_knobs(gv):
    geom, prim, seed = gv_inputs.workload("c3", 20)
    ref = None
    for basket, occ, inner, order in [(64, 1, 1, 0), (512, 2, 4, 1), (4096, 4, 16, 0), (256, 8, 2, 1), (128, 2, 4, 0)]:
        eng = gv.Engine(geom, precision=gv.P64, basket=basket, occupancy=occ, inner_steps=inner, queue_order=order)
        e = eng.transport(prim, seed)
        st = eng.stats()
        if ref is None:
            ref, ref_steps = e, st["total_steps"]
        else:
            assert st["total_steps"] == ref_steps
            assert np.allclose(e, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("prec", ["p64", "pmix"])
def test_queue_orders_agree(gv, prec):
    """Arrival-order and stable queues hold the same tracks in different
    slots; keyed random streams make the physics identical: equal step,
    track and interaction counts, deposits equal up to atomic summation order."""
    geom, prim, seed = gv_inputs.workload("c4", 150)
    p = gv.P64 if prec == "p64" else gv.PMIX
    out = {}
    for order in (gv.ORDER_STABLE, gv.ORDER_ARRIVAL):
        eng = gv.Engine(geom, precision=p, queue_order=order)
        e = eng.transport(prim, seed)
        st = eng.stats()
        out[order] = (e, st["steps"], st["tracks"], st["interactions"], eng.ledger())
    a, b = out[gv.ORDER_STABLE], out[gv.ORDER_ARRIVAL]
    assert a[1] == b[1] and a[2] == b[2] and a[3] == b[3]
    assert np.allclose(a[0], b[0], rtol=1e-12, atol=1e-12 * max(1.0, a[0].max()))
    assert np.allclose(a[4], b[4], rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("mode", ["arrival", "stable", "plain"])
def test_capacity_overflow_restarts(gv, mode):
    """Queues far too small for all events at once: the driver discards the
    window on overflow, halves the events in flight and reruns; the result
    equals the run with ample capacity."""
    geom, prim, seed = gv_inputs.workload("c1", 40)
    cfg = dict(precision=gv.P64)
    if mode == "plain":
        cfg["driver"] = gv.DRIVER_PLAIN
    else:
        cfg["queue_order"] = gv.ORDER_ARRIVAL if mode == "arrival" else gv.ORDER_STABLE
    cfg["trace_cap"] = 1_000_000
    eng0 = gv.Engine(geom, **cfg)
    ref = eng0.transport(prim, seed)
    st0, h0 = eng0.stats(), eng0.escape_hist()
    eng0.close()
    eng = gv.Engine(geom, capacity=256, **cfg)
    e = eng.transport(prim, seed)
    st = eng.stats()
    print(f"\n[overflow {mode}] restarts {st['overflow_restarts']}")
    assert st["overflow_restarts"] > 0
    assert np.allclose(e, ref, rtol=1e-12, atol=1e-12 * max(1.0, ref.max()))
    # counters, escape spectra and step records of the discarded windows are
    # taken back: the totals equal those of the run with ample capacity
    for k in ("steps", "tracks", "interactions", "escaped", "killed", "trace_records", "rejection_exhausted"):
        assert st[k] == st0[k], (k, st[k], st0[k])
    assert np.array_equal(eng.escape_hist(), h0)
    assert st["state_bytes"] <= st0["state_bytes"] * 1.5 + 1e6


@pytest.mark.parametrize("fs", ["rejection", "tables", "field_c3"])
def test_paired_layer_deposits_mixed_vs_oracle(gv, oracle_mod, fs):
    """Per-layer mean deposits of the mixed batched path against the oracle on
    the same seeds: every layer within 3 sigma of the paired differences, and
    layers holding >= 1 % of the deposit within 0.5 % wherever the sample
    resolves 0.5 % (3 sigma below it).  Without a field (c1) every big layer is
    resolved; in 4 T (c3) the field decorrelates the mixed and FP64 histories
    and 150 events resolve only the 3-sigma bar (the full c4 batch in bench.py
    resolves 0.5 %)."""
    if fs == "field_c3":
        geom, prim, seed = gv_inputs.workload("c3", 150)     # 10 GeV e- in 4 T
    else:
        geom, prim, seed = gv_inputs.workload("c1", 400)
    fsa = gv.FS_ALL if fs == "tables" else 0
    ref = oracle_mod.Oracle(geom, run_spec={"fs_alias": fsa}).transport(prim, seed)["edep"]
    eng = gv.Engine(geom, precision=gv.PMIX, fs_alias=fsa)
    got = eng.transport(prim, seed)
    N = len(prim)
    d = got - ref
    m = ref.mean(0)
    delta = d.mean(0)
    sig = d.std(0, ddof=1) / np.sqrt(N)
    total = m.sum()
    ok3 = np.abs(delta) <= 3 * sig + 1e-9 * np.abs(m)
    big = m >= 0.01 * total
    resolved = 3 * sig <= 0.005 * np.abs(m)
    ok05 = ~(big & resolved) | (np.abs(delta) <= 0.005 * np.abs(m))
    print("\n[%s PMix vs oracle] worst |delta|/m on big layers: %.2e, layers failing 3 sigma: %d, "
          "big layers resolving 0.5 %%: %d of %d" % (fs, float(np.max(np.abs(delta[big]) / m[big])),
                                                    int((~ok3).sum()), int((big & resolved).sum()), int(big.sum())))
    if fs != "field_c3":
        assert resolved[big].all()
    assert ok05.all()
    assert (~ok3).sum() <= 1   # 20 layers at 3 sigma: allow one excursion


@pytest.mark.parametrize("driver", ["plain", "batched"])
def test_events_in_flight_window(gv, driver):
    """Transporting the batch in windows of 7 events gives the same scores as
    all events in flight (fixed-point: bit for bit)."""
    geom, prim, seed = gv_inputs.workload("c3", 40)
    cfg = dict(precision=gv.P64, deposit_mode=gv.DEPOSIT_FIXED,
               driver=gv.DRIVER_PLAIN if driver == "plain" else gv.DRIVER_BATCHED)
    eng = gv.Engine(geom, **cfg)
    ref = eng.transport(prim, seed)
    ref_l = eng.ledger()
    eng.configure(max_events_in_flight=7)
    got = eng.transport(prim, seed)
    assert np.array_equal(got, ref) and np.array_equal(eng.ledger(), ref_l)


def test_staged_batch_reused_across_drivers(gv, oracle_mod):
    """One staged batch transported by the batched drivers and then by the
    plain driver: each must reproduce the oracle (the queue layouts of the
    drivers differ, so staged primaries must be re-laid-out per driver)."""
    geom, prim, seed = gv_inputs.workload("c4", 90)
    ref = oracle_mod.Oracle(geom).transport(prim, seed)
    eng = gv.Engine(geom)
    eng.stage(prim)
    scale = max(1.0, ref["edep"].max())
    for cfg in [dict(driver=gv.DRIVER_BATCHED, precision=gv.PMIX), dict(driver=gv.DRIVER_BATCHED, precision=gv.P64),
                dict(driver=gv.DRIVER_PLAIN, precision=gv.P64), dict(driver=gv.DRIVER_BATCHED, precision=gv.P64)]:
        eng.configure(**cfg)
        e = eng.transport_staged(seed)
        st = eng.stats()
        n_ref = sum(ref["counters"][k] for k in ("steps_gamma", "steps_electron", "steps_positron"))
        if cfg["precision"] == gv.P64:
            assert st["total_steps"] == n_ref, (cfg, st["total_steps"], n_ref)
            assert np.allclose(e, ref["edep"], rtol=1e-8, atol=1e-8 * scale), cfg
        else:
            assert abs(st["total_steps"] / n_ref - 1) < 0.01, (cfg, st["total_steps"], n_ref)


def test_autotuner_choice_is_cached_and_exact(gv):
    """Knobs left at 0 on a batch of >= 4096 primaries are chosen by trial
    transports of a sample; the choice is cached, and the transport with the
    chosen knobs equals one with the same knobs given explicitly."""
    geom, prim, seed = gv_inputs.workload("c1", 4200)
    eng = gv.Engine(geom, precision=gv.P64)
    e1 = eng.transport(prim, seed)
    st1 = eng.stats()
    assert st1["tuned"] == 1 and st1["autotune_ms"] > 0
    assert st1["basket"] in (64, 128, 256, 512) and st1["occupancy"] in (1, 2, 3, 4, 6, 8)
    assert st1["inner_steps"] in (1, 2, 4, 8)
    e2 = eng.transport(prim, seed)
    st2 = eng.stats()
    assert st2["tuned"] == 1 and st2["autotune_ms"] == 0
    assert (st2["basket"], st2["occupancy"], st2["inner_steps"]) == (st1["basket"], st1["occupancy"],
                                                                      st1["inner_steps"])
    fixed = gv.Engine(geom, precision=gv.P64, basket=st1["basket"], occupancy=st1["occupancy"],
                      inner_steps=st1["inner_steps"])
    e3 = fixed.transport(prim, seed)
    st3 = fixed.stats()
    assert st3["tuned"] == 0 and st3["total_steps"] == st1["total_steps"]
    scale = max(1.0, e3.max())
    assert np.allclose(e1, e3, rtol=1e-12, atol=1e-12 * scale)
    assert np.allclose(e2, e3, rtol=1e-12, atol=1e-12 * scale)


@pytest.mark.parametrize("prec", ["p64", "pmix"])
def test_fixed_point_scores_bit_identical(gv, prec):
    """Fixed-point scoring: deposits and ledgers are bit-identical for any
    basket, occupancy, inner steps and queue order (and, in FP64, for the
    plain driver too), and equal the FP64-atomic sums to rounding."""
    geom, prim, seed = gv_inputs.workload("c4", 150)
    p = gv.P64 if prec == "p64" else gv.PMIX
    runs = []
    for basket, occ, inner, order in [(256, 4, 4, gv.ORDER_ARRIVAL), (64, 1, 1, gv.ORDER_STABLE),
                                      (512, 2, 2, gv.ORDER_ARRIVAL), (128, 8, 8, gv.ORDER_STABLE)]:
        eng = gv.Engine(geom, precision=p, basket=basket, occupancy=occ, inner_steps=inner, queue_order=order,
                        deposit_mode=gv.DEPOSIT_FIXED)
        runs.append((eng.transport(prim, seed), eng.ledger(), eng.stats()["total_steps"]))
    if prec == "p64":
        eng = gv.Engine(geom, driver=gv.DRIVER_PLAIN, precision=gv.P64, deposit_mode=gv.DEPOSIT_FIXED)
        runs.append((eng.transport(prim, seed), eng.ledger(), eng.stats()["total_steps"]))
    for k, (e, led, n) in enumerate(runs[1:], 1):
        print(f"\n[fixed {prec} run {k}] steps {n}, cells differing {int((e != runs[0][0]).sum())}, "
              f"max |diff| {float(np.abs(e - runs[0][0]).max()):.3e}, ledger differing {int((led != runs[0][1]).sum())}")
    for e, led, n in runs[1:]:
        assert n == runs[0][2]
        assert np.array_equal(e, runs[0][0])
        assert np.array_equal(led, runs[0][1])
    ef = gv.Engine(geom, precision=p).transport(prim, seed)
    assert np.allclose(runs[0][0], ef, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("mode", ["plain64", "batch64", "batchmix"])
def test_escape_histogram_vs_oracle(gv, oracle_mod, mode):
    """Single-slab transmission / reflection spectra (10 MeV e- on 2 mm Pb):
    the FP64 drivers count exactly the oracle's escapes, bin for bin; the
    mixed path agrees in the transmitted and reflected fractions of each
    particle type within 3 sigma."""
    geom, prim, seed = gv_inputs.workload("t5", 3000)
    ref = oracle_mod.Oracle(geom).transport(prim, seed)
    cfg = {"plain64": dict(driver=gv.DRIVER_PLAIN, precision=gv.P64),
           "batch64": dict(precision=gv.P64), "batchmix": dict(precision=gv.PMIX)}[mode]
    eng = gv.Engine(geom, **cfg)
    eng.transport(prim, seed)
    h, r = eng.escape_hist(), ref["escape_hist"]
    assert h.sum() == eng.stats()["escaped"]
    if mode != "batchmix":
        assert np.array_equal(h, r)
        return
    n = len(prim)
    for ty in range(3):
        for half in (slice(0, 10), slice(10, 20)):
            a, b = h[ty, :, half].sum() / n, r[ty, :, half].sum() / n
            sig = math.sqrt(max(b * (1 - b), 1.0 / n) / n)
            print(f"\n[t5 type {ty} {'fwd' if half.start else 'back'}] gpu {a:.4f} oracle {b:.4f}")
            assert abs(a - b) <= 3 * math.sqrt(2) * sig + 1e-12
