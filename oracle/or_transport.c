/*
 * Oracle transport (test infrastructure only): plain history-based stepping,
 * one track at a time, depth-first within an event, threads over events.
 *
 * One step follows the stage sequence of Sec. 2.1.2:
 *   PreStep         tracking cut (e+- below t_track stop; e+ annihilates at
 *                   rest), looper cap
 *   ComputeIntLen   cross sections from the tables at the pre-step energy;
 *                   physics length = exponential / Sigma_tot; charged
 *                   particles also get the continuous-loss limit from the
 *                   range (R if R <= 1 mm, else max(0.2 R, 1 mm))
 *   GeomQuery       distance to the next boundary, safety, next volume
 *   Propagation     neutral or field-free: straight to min(physics, boundary);
 *                   charged in a field: the rule of Sec. 3.4, step =
 *                   min(min(physics, boundary), max(field, safety)), moved
 *                   along the helix (or RK4) and always relocated; a change
 *                   of volume makes the step geometry-limited
 *   PostPropagation Highland multiple scattering (pre-step energy)
 *   AlongStepAction restricted continuous loss (linear below 1% of the
 *                   range, otherwise by range inversion), deposited in the
 *                   pre-step volume's cell
 *   PostStepActions discrete interaction if the physics length limited the
 *                   step; process chosen with the pre-step cross sections,
 *                   final state sampled at the post-loss energy
 *   SteppingActions stop (e+ annihilation), escape, scoring
 * Random numbers: counter-based blocks keyed by (event, track id, step,
 * purpose); a child's track id comes from the parent's CHILD block (the
 * collision-resistant daughter seeding of Sec. 5.1).
 */
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

or_ctx G;
static __thread char g_err[256];

void or_set_error(const char* msg)
{
    strncpy(g_err, msg, sizeof(g_err) - 1);
    g_err[sizeof(g_err) - 1] = 0;
}
const char* or_error(void) { return g_err; }

int or_setup_materials(const or_material* mats, int32_t n);
double or_dist_out_face(int32_t vol, const double p[3], const double d[3], int32_t* next,
                        int32_t* snap_axis, double* snap_val);

#define INF_LEN 1.0e300
#define R_FLOOR 0.1     /* cm: continuous-loss step floor */
#define R_FRAC 0.2      /* fraction of the range per step */
#define LIN_FRAC 0.01   /* linear-loss branch below this fraction of the range */

int or_setup(const or_material* mats, int32_t n_mats, const or_geometry* geom, const or_config* cfg)
{
    if (!mats || n_mats <= 0 || n_mats > OR_MAX_MATS || !geom || !cfg) {
        or_set_error("invalid arguments");
        return -1;
    }
    or_free_tables();
    free(G.bounds);
    free(G.vmat);
    free(G.vcell);
    memset(&G, 0, sizeof(G));
    G.cfg = *cfg;
    if (G.cfg.n_nodes < 2) {
        or_set_error("table needs at least two nodes");
        return -1;
    }
    or_setup_materials(mats, n_mats);
    or_build_alias();
    G.axis = geom->axis;
    G.n_vol = geom->n_vol;
    if (G.n_vol <= 0) {
        or_set_error("empty stack");
        return -1;
    }
    G.bounds = (double*)malloc(sizeof(double) * (G.n_vol + 1));
    G.vmat = (int32_t*)malloc(sizeof(int32_t) * G.n_vol);
    G.vcell = (int32_t*)malloc(sizeof(int32_t) * G.n_vol);
    memcpy(G.bounds, geom->bounds, sizeof(double) * (G.n_vol + 1));
    memcpy(G.vmat, geom->material, sizeof(int32_t) * G.n_vol);
    memcpy(G.vcell, geom->cell, sizeof(int32_t) * G.n_vol);
    memcpy(G.env, geom->env, sizeof(G.env));
    memcpy(G.world, geom->world, sizeof(G.world));
    memcpy(G.B, geom->B, sizeof(G.B));
    if (geom->field_map != OR_MAP_UNIFORM && geom->field_map != OR_MAP_SOLENOID) {
        or_set_error("unknown field map");
        return -1;
    }
    if (geom->field_map == OR_MAP_SOLENOID &&
        (G.B[0] != 0.0 || G.B[1] != 0.0 || !(geom->sol[0] > 0.0) || !(geom->sol[1] > 0.0))) {
        or_set_error("solenoid needs B along z and a positive radius and half-length");
        return -1;
    }
    if (G.cfg.field_method < OR_FIELD_HELIX || G.cfg.field_method > OR_FIELD_RK45 ||
        (G.cfg.field_method == OR_FIELD_RK45 && (!(G.cfg.rk_tol > 0.0) || G.cfg.rk_max_sub < 1))) {
        or_set_error("bad field method or RK45 settings");
        return -1;
    }
    G.field.map = geom->field_map;
    G.field.pad = 0;
    memcpy(G.field.B, geom->B, sizeof(G.field.B));
    G.field.sol[0] = geom->sol[0];
    G.field.sol[1] = geom->sol[1];
    G.n_cells = 0;
    for (int32_t v = 0; v < G.n_vol; ++v) {
        if (!(G.bounds[v + 1] > G.bounds[v])) {
            or_set_error("stack boundaries not strictly increasing");
            return -1;
        }
        if (G.vmat[v] < -1 || G.vmat[v] >= n_mats) {
            or_set_error("volume material out of range");
            return -1;
        }
        if (G.vmat[v] >= 0 && G.vcell[v] < 0) {
            or_set_error("material volume without a cell");
            return -1;
        }
        if (G.vcell[v] + 1 > G.n_cells) G.n_cells = G.vcell[v] + 1;
    }
    if (or_build_tables() != 0) return -1;
    G.ready = 1;
    return 0;
}

/* ---------------- one step ---------------- */

typedef struct {
    int32_t type, vol;
    double pos[3], dir[3], T;
    uint64_t tid;
    uint32_t nstep;
} trk_t;

typedef struct {
    int32_t did_step, lim, proc, vol_pre, status, n_child;
    double s, s_phys, s_eloss, d_bnd, safety, edep;
    trk_t child[2];
} step_t;

enum { ST_ALIVE = 0, ST_DEAD = 1, ST_ESCAPED = 2, ST_KILLED = 3 };

static void child_ids(uint64_t seed, uint32_t ev, const trk_t* t, uint64_t ids[2])
{
    uint32_t w[4];
    or_stream(seed, ev, t->tid, t->nstep, OR_PURP_CHILD, w);
    ids[0] = ((uint64_t)w[1] << 32) | w[0];
    ids[1] = ((uint64_t)w[3] << 32) | w[2];
}

static void make_child(step_t* si, int slot, const uint64_t ids[2], int32_t type, double T,
                       const double dir[3], const trk_t* parent)
{
    trk_t* c = &si->child[si->n_child++];
    c->type = type;
    c->vol = parent->vol;
    c->T = T;
    c->tid = ids[slot];
    c->nstep = 0;
    for (int a = 0; a < 3; ++a) {
        c->pos[a] = parent->pos[a];
        c->dir[a] = dir[a];
    }
}

/* e+ at rest: two back-to-back 511 keV photons, isotropic */
static void annihilate(uint64_t seed, uint32_t ev, trk_t* t, step_t* si, double* L, int64_t* C)
{
    uint32_t w[4];
    or_stream(seed, ev, t->tid, t->nstep, OR_PURP_ANNIH, w);
    double cost = 2.0 * or_u53(w[0], w[1]) - 1.0;
    double phi = 2.0 * OR_PI * or_u53(w[2], w[3]);
    double sint = sqrt((1.0 - cost) * (1.0 + cost));
    double u[3] = {sint * cos(phi), sint * sin(phi), cost};
    double v[3] = {-u[0], -u[1], -u[2]};
    uint64_t ids[2];
    child_ids(seed, ev, t, ids);
    make_child(si, 0, ids, OR_GAMMA, OR_ME, u, t);
    make_child(si, 1, ids, OR_GAMMA, OR_ME, v, t);
    L[OR_L_NANNIH] += 1.0;
    C[OR_C_PROC0 + OR_PROC_ANNIH] += 1;
}

static void count_rej(int r, int64_t* C)
{
    if (r < 0) C[OR_C_REJ_EXHAUSTED] += 1;
}

/* discrete interaction at the post-loss energy; the track is alive on entry */
static void interact(uint64_t seed, uint32_t ev, trk_t* t, int first, step_t* si, double* L, int64_t* C)
{
    const or_config* cf = &G.cfg;
    uint64_t ids[2];
    double out[4];
    if (t->type == OR_GAMMA) {
        double k = t->T;
        if (first) {  /* Compton */
            si->proc = OR_PROC_COMPTON;
            count_rej((cf->fs_alias >> OR_AL_COMPTON) & 1 ? or_sample_compton_alias(k, seed, ev, t->tid, t->nstep, out)
                                                         : or_sample_compton(k, seed, ev, t->tid, t->nstep, out), C);
            double k1 = out[0] * k, Te = k - k1;
            double u0[3] = {t->dir[0], t->dir[1], t->dir[2]};
            or_rotate(t->dir, out[1], sqrt(out[3]), out[2]);
            child_ids(seed, ev, t, ids);
            if (Te >= cf->t_track) {
                double de[3] = {k * u0[0] - k1 * t->dir[0], k * u0[1] - k1 * t->dir[1],
                                k * u0[2] - k1 * t->dir[2]};
                double nn = sqrt(de[0] * de[0] + de[1] * de[1] + de[2] * de[2]);
                de[0] /= nn; de[1] /= nn; de[2] /= nn;
                make_child(si, 0, ids, OR_ELECTRON, Te, de, t);
            } else {
                si->edep += Te;
            }
            if (k1 < cf->t_track) {
                si->edep += k1;
                t->T = 0.0;
                si->status = ST_DEAD;
            } else {
                t->T = k1;
            }
        } else {  /* pair */
            if (k <= 2.0 * OR_ME) {
                si->proc = OR_PROC_NULL;
                C[OR_C_PROC0 + OR_PROC_NULL] += 1;
                return;
            }
            si->proc = OR_PROC_PAIR;
            count_rej((cf->fs_alias >> OR_AL_PAIR) & 1 ? or_sample_pair_alias(k, seed, ev, t->tid, t->nstep, out)
                                                      : or_sample_pair(k, seed, ev, t->tid, t->nstep, out), C);
            double Em = out[0] * k, Ep = (1.0 - out[0]) * k;
            double Tm = Em - OR_ME, Tp = Ep - OR_ME;
            double th_m = OR_ME / Em, th_p = OR_ME / Ep;
            double dm[3] = {t->dir[0], t->dir[1], t->dir[2]};
            double dp[3] = {t->dir[0], t->dir[1], t->dir[2]};
            or_rotate(dm, cos(th_m), sin(th_m), out[1]);
            or_rotate(dp, cos(th_p), sin(th_p), out[1] + OR_PI);
            child_ids(seed, ev, t, ids);
            if (Tm >= cf->t_track) make_child(si, 0, ids, OR_ELECTRON, Tm, dm, t);
            else si->edep += Tm;
            make_child(si, 1, ids, OR_POSITRON, Tp, dp, t);
            L[OR_L_NPAIR] += 1.0;
            t->T = 0.0;
            si->status = ST_DEAD;
        }
    } else {
        double T = t->T;
        if (first) {  /* Moller (e-) or Bhabha (e+) */
            int pos = (t->type == OR_POSITRON);
            if ((!pos && T <= 2.0 * cf->t_cut) || (pos && T <= cf->t_cut)) {
                si->proc = OR_PROC_NULL;
                C[OR_C_PROC0 + OR_PROC_NULL] += 1;
                return;
            }
            si->proc = pos ? OR_PROC_BHABHA : OR_PROC_MOLLER;
            if (pos) count_rej((cf->fs_alias >> OR_AL_BHABHA) & 1 ? or_sample_bhabha_alias(T, seed, ev, t->tid, t->nstep, out)
                                                                : or_sample_bhabha(T, seed, ev, t->tid, t->nstep, out), C);
            else count_rej((cf->fs_alias >> OR_AL_MOLLER) & 1 ? or_sample_moller_alias(T, seed, ev, t->tid, t->nstep, out)
                                                            : or_sample_moller(T, seed, ev, t->tid, t->nstep, out), C);
            double Td = out[0] * T;
            double cost = sqrt(Td * (T + 2.0 * OR_ME) / (T * (Td + 2.0 * OR_ME)));
            double sint = sqrt(2.0 * OR_ME * (T - Td) / (T * (Td + 2.0 * OR_ME)));
            double ud[3] = {t->dir[0], t->dir[1], t->dir[2]};
            or_rotate(ud, cost, sint, out[1]);
            double p = sqrt(T * (T + 2.0 * OR_ME)), pd = sqrt(Td * (Td + 2.0 * OR_ME));
            double np[3] = {p * t->dir[0] - pd * ud[0], p * t->dir[1] - pd * ud[1],
                            p * t->dir[2] - pd * ud[2]};
            double nn = sqrt(np[0] * np[0] + np[1] * np[1] + np[2] * np[2]);
            child_ids(seed, ev, t, ids);
            make_child(si, 0, ids, OR_ELECTRON, Td, ud, t);
            if (nn > 0.0) {
                t->dir[0] = np[0] / nn;
                t->dir[1] = np[1] / nn;
                t->dir[2] = np[2] / nn;
            }
            t->T = T - Td;
        } else {  /* bremsstrahlung */
            if (T <= cf->k_cut) {
                si->proc = OR_PROC_NULL;
                C[OR_C_PROC0 + OR_PROC_NULL] += 1;
                return;
            }
            si->proc = (t->type == OR_POSITRON) ? OR_PROC_BREMS_EP : OR_PROC_BREMS_EM;
            count_rej((cf->fs_alias >> OR_AL_BREMS) & 1 ? or_sample_brems_alias(T, seed, ev, t->tid, t->nstep, out)
                                                       : or_sample_brems(T, seed, ev, t->tid, t->nstep, out), C);
            double k = out[0];
            child_ids(seed, ev, t, ids);
            make_child(si, 0, ids, OR_GAMMA, k, t->dir, t);
            t->T = T - k;
        }
    }
    C[OR_C_PROC0 + si->proc] += 1;
}

/* One step of one track in the stage order of Sec. 2.1.2.  stop > 0 ends
 * it after the named stage (OR_STOP_*), with what that stage has produced
 * so far: the per-stage reference of the single-step tests. */
static void one_step_to(uint64_t seed, uint32_t ev, trk_t* t, step_t* si, double* L, int64_t* C, int stop)
{
    const or_config* cf = &G.cfg;
    memset(si, 0, sizeof(*si));
    si->proc = -1;
    si->lim = -1;
    si->vol_pre = t->vol;
    si->status = ST_ALIVE;
    const int charged = (t->type != OR_GAMMA);
    const int positron = (t->type == OR_POSITRON);

    /* ---- PreStep ---- */
    if (t->vol == OR_OUTSIDE) {
        L[OR_L_ESCAPED] += t->T;
        C[OR_C_ESCAPED] += 1;
        si->status = ST_ESCAPED;
        return;
    }
    if (charged && t->T < cf->t_track) {
        si->edep = t->T;
        t->T = 0.0;
        if (positron) annihilate(seed, ev, t, si, L, C);
        si->status = ST_DEAD;
        return;
    }
    if ((int64_t)t->nstep >= cf->max_steps) {
        L[OR_L_KILLED] += t->T;
        C[OR_C_KILLED] += 1;
        si->status = ST_KILLED;
        return;
    }
    const int32_t m = or_vol_material(t->vol);

    /* ---- ComputeIntLen ---- */
    uint32_t b0[4];
    or_stream(seed, ev, t->tid, t->nstep, OR_PURP_STEP, b0);
    double sa = 0.0, sb = 0.0, R = 0.0;
    if (m >= 0) {
        if (t->type == OR_GAMMA) {
            sa = or_table_value(m, OR_T_COMPTON, t->T);
            sb = or_table_value(m, OR_T_PAIR, t->T);
        } else if (!positron) {
            sa = or_table_value(m, OR_T_MOLLER, t->T);
            sb = or_table_value(m, OR_T_BREMS_EM, t->T);
        } else {
            sa = or_table_value(m, OR_T_BHABHA, t->T);
            sb = or_table_value(m, OR_T_BREMS_EP, t->T);
        }
    }
    const double stot = sa + sb;
    const double s_phys = (stot > 0.0) ? or_expo(b0[0], b0[1]) / stot : INF_LEN;
    double s_eloss = INF_LEN;
    if (charged && m >= 0) {
        R = or_table_value(m, positron ? OR_T_R_EP : OR_T_R_EM, t->T);
        s_eloss = (R <= R_FLOOR) ? R : fmax(R_FRAC * R, R_FLOOR);
    }
    const double s_lim = fmin(s_phys, s_eloss);
    si->s_phys = s_phys;
    si->s_eloss = s_eloss;
    if (stop == OR_STOP_LIMIT) return;

    /* ---- GeomQuery ---- */
    int32_t next, snap_axis;
    double snap_val;
    const double d_bnd = or_dist_out_face(t->vol, t->pos, t->dir, &next, &snap_axis, &snap_val);
    const double safety = or_safety(t->vol, t->pos);
    si->d_bnd = d_bnd;
    si->safety = safety;
    if (stop == OR_STOP_GEOM) return;

    /* ---- Propagation ---- */
    const double T_pre = t->T;
    double Bl[3]; /* the field at the pre-step point */
    or_field_eval(&G.field, t->pos, Bl);
    const double Bm = sqrt(Bl[0] * Bl[0] + Bl[1] * Bl[1] + Bl[2] * Bl[2]);
    double s;
    int lim, crossed = 0;
    if (!charged || Bm == 0.0) {
        if (d_bnd <= s_lim) {
            s = d_bnd;
            lim = OR_LIM_GEOM;
        } else {
            s = s_lim;
            lim = (s_phys <= s_eloss) ? OR_LIM_PHYS : OR_LIM_ELOSS;
        }
        for (int a = 0; a < 3; ++a) t->pos[a] += s * t->dir[a];
        if (lim == OR_LIM_GEOM) {
            if (snap_axis >= 0) t->pos[snap_axis] = snap_val;
            t->vol = next;
            crossed = 1;
        }
    } else {
        double p = sqrt(T_pre * (T_pre + 2.0 * OR_ME));
        /* transverse momentum relative to B: p |u x B/|B|| */
        double b[3] = {Bl[0] / Bm, Bl[1] / Bm, Bl[2] / Bm};
        double cx = t->dir[1] * b[2] - t->dir[2] * b[1];
        double cy = t->dir[2] * b[0] - t->dir[0] * b[2];
        double cz = t->dir[0] * b[1] - t->dir[1] * b[0];
        double sin2 = cx * cx + cy * cy + cz * cz;
        double rcurv = INF_LEN, dfield = INF_LEN;
        if (sin2 > 0.0) {
            rcurv = p / (OR_KB * Bm * sqrt(sin2));
            dfield = sqrt(2.0 * rcurv * cf->chord_tol);
        }
        double c = fmax(dfield, safety);
        double s0 = fmin(s_lim, d_bnd);
        if (s0 <= c) {
            s = s0;
            lim = (d_bnd <= s_lim) ? OR_LIM_GEOM : ((s_phys <= s_eloss) ? OR_LIM_PHYS : OR_LIM_ELOSS);
        } else {
            s = c;
            lim = OR_LIM_FIELD;
        }
        if (lim == OR_LIM_GEOM) s += cf->push;
        if (cf->field_method == OR_FIELD_RK4) {
            double nsub = (rcurv < INF_LEN) ? ceil(s / (cf->rk_frac * rcurv)) : 1.0;
            if (nsub < 1.0) nsub = 1.0;
            if (nsub > 100000.0) nsub = 100000.0;
            or_rk4_field_move(t->type, T_pre, &G.field, s, (int32_t)nsub, t->pos, t->dir);
        } else if (cf->field_method == OR_FIELD_RK45) {
            double s_done;
            int32_t n_rej;
            int32_t n_acc = or_rk45_move(t->type, T_pre, &G.field, s, cf->rk_tol, cf->rk_max_sub,
                                         t->pos, t->dir, &s_done, &n_rej);
            C[OR_C_RK_SUB] += n_acc;
            C[OR_C_RK_REJ] += n_rej;
            if (s_done < s) { /* attempts ran out: the step ends where integration stopped */
                s = s_done;
                lim = OR_LIM_FIELD;
            }
        } else {
            or_helix_move(t->type, T_pre, Bl, s, t->pos, t->dir);
        }
        int32_t nv = or_locate(t->pos);
        if (nv != t->vol) {
            t->vol = nv;
            lim = OR_LIM_GEOM;
            crossed = 1;
        }
    }
    si->did_step = 1;
    si->s = s;
    si->lim = lim;
    if (stop == OR_STOP_MOVE) return;

    /* ---- PostPropagation: multiple scattering ---- */
    if (charged && m >= 0 && s > 0.0) {
        double th0 = or_highland(m, T_pre, s);
        uint32_t b1[4];
        or_stream(seed, ev, t->tid, t->nstep, OR_PURP_MSC, b1);
        double g1, g2;
        or_box_muller(or_u53(b1[0], b1[1]), or_u53(b1[2], b1[3]), &g1, &g2);
        double tx = th0 * g1, ty = th0 * g2;
        double th = sqrt(tx * tx + ty * ty);
        double phi = atan2(ty, tx);
        or_rotate(t->dir, cos(th), sin(th), phi);
    }
    if (stop == OR_STOP_MSC) return;

    /* ---- AlongStepAction: continuous loss ---- */
    int stopped = 0;
    if (charged && m >= 0) {
        double dE;
        if (s < LIN_FRAC * R) dE = or_table_value(m, positron ? OR_T_S_EP : OR_T_S_EM, T_pre) * s;
        else dE = T_pre - or_range_inverse(m, positron, R - s);
        if (T_pre - dE < cf->t_track || R - s <= G.r_track[m][positron]) {
            dE = T_pre;
            stopped = 1;
        }
        si->edep += dE;
        t->T = T_pre - dE;
    }
    if (stop == OR_STOP_ELOSS) return;

    /* ---- PostStepActions: discrete interaction ---- */
    if (lim == OR_LIM_PHYS && !crossed && !stopped) {
        double usel = or_u53(b0[2], b0[3]);
        interact(seed, ev, t, usel * stot < sa, si, L, C);
    }

    /* ---- SteppingActions ---- */
    if (stopped) {
        if (positron) annihilate(seed, ev, t, si, L, C);
        si->status = ST_DEAD;
    } else if (si->status == ST_ALIVE && t->vol == OR_OUTSIDE) {
        L[OR_L_ESCAPED] += t->T;
        C[OR_C_ESCAPED] += 1;
        si->status = ST_ESCAPED;
    }
    C[OR_C_STEPS_G + t->type] += 1;
    t->nstep += 1;
}

static void one_step(uint64_t seed, uint32_t ev, trk_t* t, step_t* si, double* L, int64_t* C)
{
    one_step_to(seed, ev, t, si, L, C, 0);
}

/* ---------------- transport ---------------- */

typedef struct {
    const or_primary* prim;
    const int64_t* ev_start;   /* primaries sorted by event: offsets */
    const int64_t* order;      /* primary indices grouped by event, stable */
    int64_t n_events;
    int32_t tidx, nthr;
    uint64_t seed;
    double* edep;
    double* ledger;
    int64_t counters[OR_NCOUNT];
    int64_t hist[OR_EH_SIZE];  /* escaping particles */
    or_trace* trace;
    int64_t trace_cap;
    int64_t* trace_n;
    int rc;
} job_t;

static int32_t type_of_pdg(int32_t pdg)
{
    if (pdg == 22) return OR_GAMMA;
    if (pdg == 11) return OR_ELECTRON;
    if (pdg == -11) return OR_POSITRON;
    return -1;
}

static int64_t g_esc_hist[OR_EH_SIZE];

int or_escape_hist(int64_t* out)
{
    if (!out) return -1;
    memcpy(out, g_esc_hist, sizeof(g_esc_hist));
    return 0;
}

/* one escaping particle into the histogram (H may be NULL) */
static void escape_hist(int64_t* H, const trk_t* t)
{
    if (!H) return;
    int eb = t->T > 0.0 ? (int)floor(log10(t->T / 1.0e-3) * 5.0) : 0;
    eb = eb < 0 ? 0 : (eb > OR_EH_NE - 1 ? OR_EH_NE - 1 : eb);
    int cb = (int)floor((t->dir[2] + 1.0) * 0.5 * OR_EH_NC);
    cb = cb < 0 ? 0 : (cb > OR_EH_NC - 1 ? OR_EH_NC - 1 : cb);
    H[(t->type * OR_EH_NE + eb) * OR_EH_NC + cb] += 1;
}

static void deposit(double* edep_row, double* L, int32_t vol, double e)
{
    if (e == 0.0) return;
    int32_t c = or_vol_cell(vol);
    if (c >= 0) edep_row[c] += e;
    else L[OR_L_KILLED] += e;
}

static void record(job_t* J, uint32_t ev, const trk_t* before, const trk_t* after, const step_t* si)
{
    if (!J->trace) return;
    int64_t k = __atomic_fetch_add(J->trace_n, 1, __ATOMIC_RELAXED);
    if (k >= J->trace_cap) {
        J->counters[OR_C_TRACE_DROPPED] += 1;
        return;
    }
    or_trace* r = &J->trace[k];
    r->tid = before->tid;
    r->event = ev;
    r->nstep = before->nstep;
    r->type = before->type;
    r->limiter = si->lim;
    r->vol_pre = si->vol_pre;
    r->vol_post = after->vol;
    r->process = si->proc;
    r->n_children = si->n_child;
    for (int a = 0; a < 3; ++a) {
        r->pos[a] = after->pos[a];
        r->dir[a] = after->dir[a];
    }
    r->ekin = after->T;
    r->edep = si->edep;
    r->step = si->s;
}

static void* worker(void* arg)
{
    job_t* J = (job_t*)arg;
    size_t cap = 1024, n = 0;
    trk_t* stack = (trk_t*)malloc(sizeof(trk_t) * cap);
    int64_t* C = J->counters;
    for (int64_t ev = J->tidx; ev < J->n_events; ev += J->nthr) {
        double* row = J->edep + ev * (int64_t)G.n_cells;
        double* L = J->ledger + ev * OR_NLEDGER;
        int64_t b = J->ev_start[ev], e = J->ev_start[ev + 1];
        /* push in reverse so the first primary of the event runs first */
        for (int64_t q = e - 1; q >= b; --q) {
            const or_primary* P = &J->prim[J->order[q]];
            trk_t t;
            t.type = type_of_pdg(P->pdg);
            t.T = P->ekin;
            double nn = sqrt(P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1] + P->dir[2] * P->dir[2]);
            for (int a = 0; a < 3; ++a) {
                t.pos[a] = P->pos[a];
                t.dir[a] = P->dir[a] / nn;
            }
            t.tid = (uint64_t)(q - b);
            t.nstep = 0;
            t.vol = or_locate(t.pos);
            if (n == cap) {
                cap *= 2;
                stack = (trk_t*)realloc(stack, sizeof(trk_t) * cap);
            }
            stack[n++] = t;
            C[OR_C_TRACKS_G + t.type] += 1;
        }
        while (n > 0) {
            trk_t t = stack[--n];
            for (;;) {
                step_t si;
                trk_t before = t;
                one_step(J->seed, (uint32_t)ev, &t, &si, L, C);
                if (si.status == ST_ESCAPED) escape_hist(J->hist, &t);
                deposit(row, L, si.vol_pre, si.edep);
                if (si.did_step) record(J, (uint32_t)ev, &before, &t, &si);
                for (int c = 0; c < si.n_child; ++c) {
                    if (n == cap) {
                        cap *= 2;
                        stack = (trk_t*)realloc(stack, sizeof(trk_t) * cap);
                    }
                    stack[n++] = si.child[c];
                    C[OR_C_TRACKS_G + si.child[c].type] += 1;
                }
                if (si.status != ST_ALIVE) break;
            }
        }
    }
    free(stack);
    return NULL;
}

int or_transport(const or_primary* prim, int64_t n, uint64_t seed, int32_t n_threads,
                 double* edep, double* ledger, int64_t* counters,
                 or_trace* trace, int64_t trace_cap, int64_t* trace_n)
{
    if (!G.ready) {
        or_set_error("not set up");
        return -1;
    }
    if (!prim || n <= 0 || !edep || !ledger || !counters) {
        or_set_error("invalid arguments");
        return -1;
    }
    int64_t n_events = 0;
    for (int64_t i = 0; i < n; ++i) {
        const or_primary* P = &prim[i];
        double nn = sqrt(P->dir[0] * P->dir[0] + P->dir[1] * P->dir[1] + P->dir[2] * P->dir[2]);
        if (type_of_pdg(P->pdg) < 0 || P->event < 0 || !(P->ekin > 0.0) || !(P->ekin <= 1.0e5) ||
            !(fabs(nn - 1.0) <= 1.0e-6)) {
            or_set_error("invalid primary");
            return -1;
        }
        if (P->event + 1 > n_events) n_events = P->event + 1;
    }
    int64_t* ev_start = (int64_t*)calloc(n_events + 1, sizeof(int64_t));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * n);
    for (int64_t i = 0; i < n; ++i) ev_start[prim[i].event + 1] += 1;
    for (int64_t e = 0; e < n_events; ++e) ev_start[e + 1] += ev_start[e];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * n_events);
    memcpy(fill, ev_start, sizeof(int64_t) * n_events);
    for (int64_t i = 0; i < n; ++i) order[fill[prim[i].event]++] = i;
    free(fill);

    memset(edep, 0, sizeof(double) * n_events * G.n_cells);
    memset(ledger, 0, sizeof(double) * n_events * OR_NLEDGER);
    memset(counters, 0, sizeof(int64_t) * OR_NCOUNT);
    int64_t tn = 0;
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    job_t* jobs = (job_t*)calloc(n_threads, sizeof(job_t));
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * n_threads);
    for (int32_t t = 0; t < n_threads; ++t) {
        job_t* J = &jobs[t];
        J->prim = prim;
        J->ev_start = ev_start;
        J->order = order;
        J->n_events = n_events;
        J->tidx = t;
        J->nthr = n_threads;
        J->seed = seed;
        J->edep = edep;
        J->ledger = ledger;
        J->trace = trace;
        J->trace_cap = trace_cap;
        J->trace_n = &tn;
        pthread_create(&th[t], NULL, worker, J);
    }
    memset(g_esc_hist, 0, sizeof(g_esc_hist));
    for (int32_t t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        for (int c = 0; c < OR_NCOUNT; ++c) counters[c] += jobs[t].counters[c];
        for (int b = 0; b < OR_EH_SIZE; ++b) g_esc_hist[b] += jobs[t].hist[b];
    }
    if (trace_n) *trace_n = tn < trace_cap ? tn : trace_cap;
    free(jobs);
    free(th);
    free(ev_start);
    free(order);
    return 0;
}

/* ---------------- single step on arbitrary states ---------------- */

int or_single_step(int64_t n, uint64_t seed,
                   const int32_t* type, const double* pos, const double* dir, const double* ekin,
                   const uint32_t* event, const uint64_t* tid, const uint32_t* nstep,
                   double* pos_out, double* dir_out, double* ekin_out, double* edep_out,
                   int32_t* vol_out, int32_t* vol_pre_out, int32_t* lim_out, int32_t* proc_out,
                   int32_t* status_out, int32_t* nchild_out,
                   int32_t* ch_type, double* ch_ekin, double* ch_dir, uint64_t* ch_tid,
                   double* s_out, double* sphys_out, double* dbnd_out, double* safety_out)
{
    return or_stage_step(0, n, seed, type, pos, dir, ekin, event, tid, nstep, pos_out, dir_out, ekin_out,
                         edep_out, vol_out, vol_pre_out, lim_out, proc_out, status_out, nchild_out, ch_type,
                         ch_ekin, ch_dir, ch_tid, s_out, sphys_out, dbnd_out, safety_out, NULL);
}

int or_stage_step(int32_t stop, int64_t n, uint64_t seed,
                  const int32_t* type, const double* pos, const double* dir, const double* ekin,
                  const uint32_t* event, const uint64_t* tid, const uint32_t* nstep,
                  double* pos_out, double* dir_out, double* ekin_out, double* edep_out,
                  int32_t* vol_out, int32_t* vol_pre_out, int32_t* lim_out, int32_t* proc_out,
                  int32_t* status_out, int32_t* nchild_out,
                  int32_t* ch_type, double* ch_ekin, double* ch_dir, uint64_t* ch_tid,
                  double* s_out, double* sphys_out, double* dbnd_out, double* safety_out, double* seloss_out)
{
    if (!G.ready) {
        or_set_error("not set up");
        return -1;
    }
    if (stop < 0 || stop > OR_STOP_ELOSS) {
        or_set_error("unknown stage");
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) {
        trk_t t;
        t.type = type[i];
        t.T = ekin[i];
        for (int a = 0; a < 3; ++a) {
            t.pos[a] = pos[3 * i + a];
            t.dir[a] = dir[3 * i + a];
        }
        t.tid = tid[i];
        t.nstep = nstep[i];
        t.vol = or_locate(t.pos);
        double L[OR_NLEDGER] = {0};
        int64_t C[OR_NCOUNT] = {0};
        step_t si;
        one_step_to(seed, event[i], &t, &si, L, C, stop);
        for (int a = 0; a < 3; ++a) {
            pos_out[3 * i + a] = t.pos[a];
            dir_out[3 * i + a] = t.dir[a];
        }
        ekin_out[i] = t.T;
        edep_out[i] = si.edep;
        vol_out[i] = t.vol;
        vol_pre_out[i] = si.vol_pre;
        lim_out[i] = si.lim;
        proc_out[i] = si.proc;
        status_out[i] = si.status;
        nchild_out[i] = si.n_child;
        for (int c = 0; c < 2; ++c) {
            int64_t k = 2 * i + c;
            if (c < si.n_child) {
                ch_type[k] = si.child[c].type;
                ch_ekin[k] = si.child[c].T;
                ch_tid[k] = si.child[c].tid;
                for (int a = 0; a < 3; ++a) ch_dir[3 * k + a] = si.child[c].dir[a];
            } else {
                ch_type[k] = -1;
                ch_ekin[k] = 0.0;
                ch_tid[k] = 0;
                for (int a = 0; a < 3; ++a) ch_dir[3 * k + a] = 0.0;
            }
        }
        s_out[i] = si.s;
        sphys_out[i] = si.s_phys;
        dbnd_out[i] = si.d_bnd;
        safety_out[i] = si.safety;
        if (seloss_out) seloss_out[i] = si.s_eloss;
    }
    return 0;
}
