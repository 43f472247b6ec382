"""Mutation check of the oracle's CPU pins (not collected by pytest; run as
``python tests/oracle_mutations.py [name filter ...]``).

Each entry plants one plausible mistake in a copy of the oracle's C sources
under a scratch directory, rebuilds that copy and runs the oracle pin tests
against it; a mistake that no test fails would be a gap in the pins.  The
repository's own oracle is never modified.  Takes a few minutes on 8 cores.
"""
import os, shutil, subprocess, sys, json
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
T = "or_transport.c"
S = "or_sample.c"
MUT = [
 ("floor below 1 mm", T, "s_eloss = (R <= R_FLOOR) ? R : fmax(R_FRAC * R, R_FLOOR);", "s_eloss = fmax(R_FRAC * R, R_FLOOR);"),
 ("range fraction 0.25", T, "#define R_FRAC 0.2 ", "#define R_FRAC 0.25 "),
 ("floor 0.05 cm", T, "#define R_FLOOR 0.1 ", "#define R_FLOOR 0.05 "),
 ("linear branch below 0.1 %", T, "#define LIN_FRAC 0.01 ", "#define LIN_FRAC 0.001 "),
 ("linear branch below 10 %", T, "#define LIN_FRAC 0.01 ", "#define LIN_FRAC 0.1 "),
 ("min(field, safety)", T, "double c = fmax(dfield, safety);", "double c = fmin(dfield, safety);"),
 ("max(phys, bnd)", T, "double s0 = fmin(s_lim, d_bnd);", "double s0 = fmax(s_lim, d_bnd);"),
 ("bending estimate sqrt(8 rho eps)", T, "dfield = sqrt(2.0 * rcurv * cf->chord_tol);", "dfield = sqrt(8.0 * rcurv * cf->chord_tol);"),
 ("radius from p_perp", T, "rcurv = p / (OR_KB * Bm * sqrt(sin2));", "rcurv = p * sqrt(sin2) / (OR_KB * Bm);"),
 ("no push past the boundary", T, "if (lim == OR_LIM_GEOM) s += cf->push;", ""),
 ("relocation keeps the nominal limiter", T, "            t->vol = nv;\n            lim = OR_LIM_GEOM;\n", "            t->vol = nv;\n"),
 ("process choice inverted", T, "interact(seed, ev, t, usel * stot < sa, si, L, C);", "interact(seed, ev, t, usel * stot >= sa, si, L, C);"),
 ("physics length from the first process only", T, "or_expo(b0[0], b0[1]) / stot", "or_expo(b0[0], b0[1]) / sa"),
 ("annihilation into a hemisphere", T, "double cost = 2.0 * or_u53(w[0], w[1]) - 1.0;", "double cost = or_u53(w[0], w[1]);"),
 ("annihilation photons not back to back", T, "double v[3] = {-u[0], -u[1], -u[2]};", "double v[3] = {-u[0], -u[1], u[2]};"),
 ("tracking cut ignored within a step", T, "if (T_pre - dE < cf->t_track || R - s <= G.r_track[m][positron]) {", "if (R - s <= G.r_track[m][positron]) {"),
 ("limiter labels PHYS/ELOSS swapped", T, "            lim = (s_phys <= s_eloss) ? OR_LIM_PHYS : OR_LIM_ELOSS;\n        }\n        for", "            lim = (s_phys <= s_eloss) ? OR_LIM_ELOSS : OR_LIM_PHYS;\n        }\n        for"),
 ("no face snap", T, "if (snap_axis >= 0) t->pos[snap_axis] = snap_val;", ""),
 ("MSC with the post-step energy", T, "double th0 = or_highland(m, T_pre, s);", "double th0 = or_highland(m, T_pre - (s < LIN_FRAC * R ? or_table_value(m, positron ? OR_T_S_EP : OR_T_S_EM, T_pre) * s : T_pre - or_range_inverse(m, positron, R - s)), s);"),
 ("Compton electron sign", T, "double de[3] = {k * u0[0] - k1 * t->dir[0]", "double de[3] = {k * u0[0] + k1 * t->dir[0]"),
 ("pair positron same azimuth", T, "or_rotate(dp, cos(th_p), sin(th_p), out[1] + OR_PI);", "or_rotate(dp, cos(th_p), sin(th_p), out[1]);"),
 ("RK45 error weights b only", S, "for (int j = 0; j < 7; ++j) e += (DP_B[j] - DP_BH[j]) * k[j][c];", "for (int j = 0; j < 7; ++j) e += (DP_B[j]) * k[j][c] * 1e-3;"),
 ("solenoid g'' sign", S, "double g2 = -3.0 * c * R2", "double g2 = 3.0 * c * R2"),
]
only = sys.argv[1:]
res = {}
for name, f, old, new in MUT:
    if only and not any(o in name for o in only):
        continue
    d = os.path.join(os.environ.get("TMPDIR", "/tmp"), "oracle_mut", str(abs(hash(name)) % 10**8))
    shutil.rmtree(d, ignore_errors=True)
    os.makedirs(d)
    for item in ("oracle", "tests", "gv_inputs.py", "pytest.ini"):
        src = os.path.join(ROOT, item)
        if os.path.isdir(src):
            shutil.copytree(src, os.path.join(d, item), ignore=shutil.ignore_patterns("_build", "__pycache__"))
        else:
            shutil.copy(src, d)
    p = os.path.join(d, "oracle", f)
    s = open(p).read()
    assert s.count(old) == 1, (name, s.count(old))
    open(p, "w").write(s.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        "tests/test_oracle_step_logic.py", "tests/test_oracle_transport.py", "tests/test_oracle_sampling.py",
                        "tests/test_oracle_rk45.py", "tests/test_oracle_geometry_field.py", "tests/test_oracle_physics.py"],
                       cwd=d, capture_output=True, text=True)
    fails = [l.split("::")[1].split(" ")[0] for l in r.stdout.splitlines() if l.startswith("FAILED")]
    res[name] = fails if fails else ("ALL PASS" if r.returncode == 0 else r.stdout[-300:])
    print(f"{name}: {res[name]}", flush=True)
    shutil.rmtree(d, ignore_errors=True)
json.dump(res, open(os.path.join(os.environ.get("TMPDIR", "/tmp"), "oracle_mutations.json"), "w"), indent=1)
