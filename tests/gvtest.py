"""Shared helpers of the GPU parity tests (comparison rules only; no physics)."""
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
