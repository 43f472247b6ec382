"""Shared helpers of the GPU parity tests (comparison rules only; no physics)."""
import math

import numpy as np

# per-field scale below which an absolute error is used: |a-b| <= tol * max(|b|, scale)
SCALES = dict(pos=1.0, dir=1.0, ekin=1e-3, edep=1e-3, step=1e-4, s_phys=1e-4, d_bnd=1e-4,
              safety=1e-4, ch_ekin=1e-3, ch_dir=1.0)
DISCRETE = ["vol", "vol_pre", "limiter", "process", "status", "n_children"]


def close(a, b, tol, scale):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    both_inf = (b >= 1e299) & (a >= 1e299)
    return both_inf | (np.abs(a - b) <= tol * np.maximum(np.abs(b), scale))


ME = 0.51099895


def _mom(T, typ):
    T = np.asarray(T, dtype=np.float64)
    return np.where(typ == 0, T, np.sqrt(np.maximum(T, 0) * (np.maximum(T, 0) + 2 * ME)))


def compare_steps(gpu, ref, st, tol):
    """Normwise comparison of one-step outputs.  Returns (n_flips, worst):
    a flip is any disagreement of a discrete output or a child id/type;
    `worst` maps each continuous field to its largest scaled error over the
    records without a flip (and `<field>_violations` counts records above tol).

    Scales: energies relative to the step's input kinetic energy; directions
    as momentum vectors relative to the input momentum (|p_out| |du| / |p_in|);
    lengths relative to max(|value|, |input position|, 1 cm); positions
    relative to max(|value|, 1 cm); the physics length relative to itself."""
    n = len(ref["limiter"])
    typ = np.asarray(st["type"])
    T_in = np.asarray(st["ekin"], dtype=np.float64)
    p_in = np.maximum(_mom(T_in, typ), 1e-300)
    pos_in = np.max(np.abs(np.asarray(st["pos"], dtype=np.float64)), axis=1)
    flip = np.zeros(n, dtype=bool)
    for k in DISCRETE:
        flip |= gpu[k] != ref[k]
    flip |= np.any(gpu["ch_type"] != ref["ch_type"], axis=1)
    flip |= np.any(gpu["ch_tid"] != ref["ch_tid"], axis=1)
    ok = ~flip
    errs = {}
    big = lambda a: np.asarray(a, dtype=np.float64)
    # energies
    for k in ("ekin", "edep"):
        errs[k] = np.abs(big(gpu[k]) - big(ref[k])) / np.maximum(T_in, 1e-3)
    has = ref["ch_type"] >= 0
    errs["ch_ekin"] = np.where(has, np.abs(big(gpu["ch_ekin"]) - big(ref["ch_ekin"])), 0).max(1) / \
        np.maximum(T_in, 1e-3)
    # directions as momentum vectors
    p_out = np.where(ref["status"] == 0, _mom(ref["ekin"], typ), p_in)
    du = np.linalg.norm(big(gpu["dir"]) - big(ref["dir"]), axis=1)
    errs["dir"] = du * np.minimum(p_out / p_in, 1.0)
    p_ch = np.where(has, _mom(ref["ch_ekin"], np.where(has, ref["ch_type"], 0)), 0.0)
    dch = np.linalg.norm(big(gpu["ch_dir"]) - big(ref["ch_dir"]), axis=2)
    errs["ch_dir"] = (dch * p_ch).max(1) / p_in
    # lengths and positions
    for k in ("step", "d_bnd", "safety"):
        b = big(ref[k])
        fin = b < 1e299
        e = np.zeros(n)
        e[fin] = np.abs(big(gpu[k])[fin] - b[fin]) / np.maximum(np.maximum(np.abs(b[fin]), pos_in[fin]), 1.0)
        e[~fin] = np.where(big(gpu[k])[~fin] >= 1e299, 0.0, np.inf)
        errs[k] = e
    b = big(ref["s_phys"])
    fin = b < 1e299
    e = np.zeros(n)
    e[fin] = np.abs(big(gpu["s_phys"])[fin] - b[fin]) / np.maximum(np.abs(b[fin]), 1e-300)
    e[~fin] = np.where(big(gpu["s_phys"])[~fin] >= 1e299, 0.0, np.inf)
    errs["s_phys"] = e
    errs["pos"] = (np.abs(big(gpu["pos"]) - big(ref["pos"])) / np.maximum(np.abs(big(ref["pos"])), 1.0)).max(1)
    worst = {}
    for k, e in errs.items():
        ek = e[ok]
        worst[k] = float(ek.max()) if ek.size else 0.0
        nv = int((ek > tol).sum())
        if nv:
            worst[k + "_violations"] = nv
    return int(flip.sum()), worst


def stable_partition_reference(codes):
    """Queue q receives input*4 + slot for every (input, slot) whose code is q,
    in input order then slot order."""
    codes = np.asarray(codes).reshape(-1, 3)
    out = [[], [], []]
    for i, row in enumerate(codes):
        for j, q in enumerate(row):
            if q >= 0:
                out[q].append(i * 4 + j)
    return [np.array(o, dtype=np.int32) for o in out]


KB = 2.99792458
PURP_STEP = 0


def flip_margins(gpu, ref, st, orc, geom, seed, t_track=0.1, chord=1e-3, push=1e-7):
    """For every record whose discrete outputs differ between the GPU and the
    oracle, the oracle-side margin of the decision that can differ, as a
    fraction of its own scale (inf when the difference is of no recognised
    kind).  A flip is admissible only where this margin is small: the two
    sides then sit on either side of a threshold within rounding.
      relocation  distance of either end point from the nearest boundary,
                  over max(step, 1 cm);
      limiter     distance of the chosen step length from the nearest other
                  candidate of the rule (physics, energy loss, boundary,
                  max(field, safety)), over the larger;
      process     |u Sigma_tot - Sigma_1| / Sigma_tot at the pre-step energy,
                  u from the track's STEP block;
      cut         distance of a post-step or secondary kinetic energy from the
                  tracking cut, over the pre-step kinetic energy."""
    import oracle as _o
    n = len(ref["limiter"])
    flip = np.zeros(n, dtype=bool)
    for k in DISCRETE:
        flip |= gpu[k] != ref[k]
    flip |= np.any(gpu["ch_type"] != ref["ch_type"], axis=1)
    flip |= np.any(gpu["ch_tid"] != ref["ch_tid"], axis=1)
    out = {}
    names = {0: ("compton", "pair"), 1: ("moller", "brems_em"), 2: ("bhabha", "brems_ep")}
    Bv = np.asarray(geom["B"], dtype=np.float64)
    Bm = float(np.linalg.norm(Bv))
    for i in np.where(flip)[0]:
        T0 = float(st["ekin"][i])
        typ = int(st["type"][i])
        margin = np.inf
        step = float(ref["step"][i])
        for side in (gpu, ref):
            p = np.asarray(side["pos"][i], dtype=np.float64)
            v = orc.locate(p)
            if v >= 0:
                margin = min(margin, orc.safety(v, p) / max(step, 1.0))
        vol = int(ref["vol_pre"][i])
        m = int(geom["material"][vol - 1]) if vol >= 1 else -1
        cands = [float(ref["s_phys"][i]), float(ref["d_bnd"][i])]
        if typ != 0 and m >= 0:
            R = orc.table_value(m, "R_em" if typ == 1 else "R_ep", T0)
            cands.append(R if R <= 0.1 else max(0.2 * R, 0.1))
        if typ != 0 and Bm > 0.0 and geom.get("field_map", 0) == 0:
            u = np.asarray(st["dir"][i], dtype=np.float64)
            sin_a = float(np.linalg.norm(np.cross(u, Bv / Bm)))
            if sin_a > 0.0:
                rho = math.sqrt(T0 * (T0 + 2 * ME)) / (KB * Bm * sin_a)
                cands.append(max(math.sqrt(2 * rho * chord), float(ref["safety"][i])))
        chosen = step - push if int(ref["limiter"][i]) == 2 else step
        for c in cands:
            if c < 1e299 and chosen > 0.0 and abs(c - chosen) > 0.0:
                margin = min(margin, abs(c - chosen) / max(c, chosen))
        if gpu["process"][i] != ref["process"][i] and m >= 0:
            w = _o.stream(seed, int(st["event"][i]), int(st["tid"][i]), int(st["nstep"][i]), PURP_STEP)
            usel = ((((w[2] << 32) | w[3]) >> 11) + 1) * 2.0 ** -53
            a, b = names[typ]
            s1, s2 = orc.table_value(m, a, T0), orc.table_value(m, b, T0)
            if s1 + s2 > 0:
                margin = min(margin, abs(usel * (s1 + s2) - s1) / (s1 + s2))
        for side in (gpu, ref):
            for e in [float(side["ekin"][i])] + [float(x) for x in side["ch_ekin"][i]]:
                if e > 0.0:
                    margin = min(margin, abs(e - t_track) / max(T0, 1e-3))
        out[int(i)] = margin
    return out


def assert_single_step_parity(flips, worst, margins, tol, fp64):
    """The single-step bar: no continuous output beyond tol on any record
    whose discrete outputs agree; in FP64 no discrete flip at all; in mixed
    precision a flip only where the oracle's decision margin is below
    10 tol."""
    viol = {k: v for k, v in worst.items() if k.endswith("_violations")}
    assert not viol, worst
    if fp64:
        assert flips == 0, worst
    else:
        wide = {i: m for i, m in margins.items() if not m < 10 * tol}
        assert not wide, wide
