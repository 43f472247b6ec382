// gv_step.h -- one transport step of one track, split into the simulation
// stages of Sec. 2.1.2:
//   PreStep         (stage_prestep)   tracking cut / e+ annihilation at rest,
//                                     looper cap, leaving the world
//   ComputeIntLen   (stage_limit)     table cross sections, physics length from
//                                     an exponential draw, continuous-loss limit
//   GeomQuery       (stage_geom)      distance to boundary, next volume, safety
//   Propagation     (stage_move)      straight line, or in a field the rule of
//                                     Sec. 3.4: min(min(phys, boundary),
//                                     max(field, safety)), helix/RK4/RK45
//                                     (Sec. 3.6), relocate
//   PostPropagation (stage_msc)       Highland multiple scattering
//   AlongStepAction (stage_eloss)     restricted continuous loss, deposit
//   PostStepActions + SteppingActions (stage_finish)  discrete interaction at
//                                     the post-loss energy, stop, escape
// The plain driver runs each stage as its own kernel with the intermediates in
// HBM; the batched driver runs the whole chain in registers (step_track).
#pragma once
#include "gv_common.h"
#include "gv_geom.h"
#include "gv_physics.h"
#include "gv_field.h"

namespace gv {

template <class P> struct Track {
    using R = typename P::R;
    double x[3];
    R u[3];
    R T;
    int vol;
    int type;
    uint32_t ev;
    uint32_t nstep;
    uint64_t tid;
};

template <class R> struct Child {
    int type;
    R T;
    R u[3];
    uint64_t tid;
};

// per-step outputs that leave the track itself
template <class R> struct StepOut {
    RkTally rk;         // adaptive integration work of this step (RK45 only)
    int status;         // kAlive / kDead / kEscaped / kKilled
    int did_step;       // a propagation happened (counts as a step)
    int lim;
    int proc;           // -1 none
    int vol_pre;        // volume whose cell receives edep
    int nchild;
    int rej_exhausted;
    int n_pair, n_annih;
    double edep;        // MeV, into cell(vol_pre)
    double e_escaped, e_killed;
    double s, s_phys, d_bnd, safety;
    Child<R> ch[2];
};

template <class R> struct Limits {
    R s_phys;   // physics length (kInf-like if no process)
    R s_eloss;
    R range;
    R stot, sa;
    R usel;
    int m;      // material of the pre-step volume (-1 vacuum)
};

struct Geo {
    double d_bnd;
    double safety;
    int next;
    int snap_axis;
    double snap_val;
};

template <class R> struct Prop {
    double s;
    R T_pre;
    int lim;
    int crossed;
    RkTally rk;
    double rcurv;   // radius of curvature at the pre-step point (charged tracks in a field)
};

template <class P> struct Ctx {
    using R = typename P::R;
    uint64_t seed;
    const DevGeom* g;
    const DevPhys* ph;
    TabView<R> tv;
};

template <class R> __device__ __forceinline__ R big_len() { return (R)1.0e30; }

template <class P, class R = typename P::R>
__device__ __forceinline__ void init_out(const Track<P>& t, StepOut<R>& o)
{
    o.rk.acc = 0;
    o.rk.rej = 0;
    o.rk.iters = 0;
    o.status = kAlive;
    o.did_step = 0;
    o.lim = -1;
    o.proc = -1;
    o.vol_pre = t.vol;
    o.nchild = 0;
    o.rej_exhausted = 0;
    o.n_pair = 0;
    o.n_annih = 0;
    o.edep = 0.0;
    o.e_escaped = 0.0;
    o.e_killed = 0.0;
    o.s = 0.0;
    o.s_phys = 0.0;
    o.d_bnd = 0.0;
    o.safety = 0.0;
}

template <class P, class R = typename P::R>
__device__ __forceinline__ void child_ids(const Ctx<P>& c, const Track<P>& t, uint64_t ids[2])
{
    const U4 b = stream_block(c.seed, t.ev, t.tid, t.nstep, kPurpChild);
    ids[0] = ((uint64_t)b.w[1] << 32) | b.w[0];
    ids[1] = ((uint64_t)b.w[3] << 32) | b.w[2];
}

template <class R> __device__ __forceinline__ void set_child(Child<R>& ch, int type, R T, const R u[3], uint64_t tid)
{
    ch.type = type;
    ch.T = T;
    ch.u[0] = u[0];
    ch.u[1] = u[1];
    ch.u[2] = u[2];
    ch.tid = tid;
}

// append a secondary (constant-index stores keep the record in registers)
template <class R> __device__ __forceinline__ void add_child(StepOut<R>& o, int type, R T, const R u[3], uint64_t tid)
{
    if (o.nchild == 0) set_child(o.ch[0], type, T, u, tid);
    else set_child(o.ch[1], type, T, u, tid);
    o.nchild += 1;
}

// e+ at rest: two back-to-back 511 keV photons, isotropic (ANNIH block)
template <class P, class R = typename P::R>
__device__ inline void annihilate(const Ctx<P>& c, const Track<P>& t, StepOut<R>& o)
{
    const U4 b = stream_block(c.seed, t.ev, t.tid, t.nstep, kPurpAnnih);
    const R ct = (R)2 * u53<R>(b.w[0], b.w[1]) - (R)1;
    const R phi = (R)(2.0 * kPi) * u53<R>(b.w[2], b.w[3]);
    const R st = m_sqrt(((R)1 - ct) * ((R)1 + ct));
    const R a[3] = {st * m_cos(phi), st * m_sin(phi), ct};
    const R bm[3] = {-a[0], -a[1], -a[2]};
    uint64_t ids[2];
    child_ids(c, t, ids);
    add_child(o, kGamma, (R)kMe, a, ids[0]);
    add_child(o, kGamma, (R)kMe, bm, ids[1]);
    o.n_annih += 1;
}

// ---- PreStep: returns true when the track goes on to take a step --------
template <class P, class R = typename P::R>
__device__ inline bool stage_prestep(const Ctx<P>& c, Track<P>& t, StepOut<R>& o)
{
    if (t.vol == kOutside) {
        o.e_escaped += (double)t.T;
        o.status = kEscaped;
        return false;
    }
    if (t.type != kGamma && t.T < (R)c.ph->t_track) {
        o.edep += (double)t.T;
        t.T = (R)0;
        if (t.type == kPositron) annihilate(c, t, o);
        o.status = kDead;
        return false;
    }
    if ((long long)t.nstep >= c.ph->max_steps) {
        o.e_killed += (double)t.T;
        o.status = kKilled;
        return false;
    }
    return true;
}

// ---- ComputeIntLen ------------------------------------------------------
// VAC: the track is known to be in a volume without material
template <class P, bool VAC = false, class R = typename P::R>
__device__ inline void stage_limit(const Ctx<P>& c, const Track<P>& t, Limits<R>& L)
{
    const int m = VAC ? -1 : vol_material(*c.g, t.vol);
    L.m = m;
    L.sa = (R)0;
    L.stot = (R)0;
    L.range = (R)0;
    L.s_eloss = big_len<R>();
    L.usel = (R)0;
    L.s_phys = big_len<R>();
    // vacuum has no process: its STEP block is never needed (the streams are
    // counter-based, so not drawing it changes no other number)
    if (m < 0) return;
    const U4 b0 = stream_block(c.seed, t.ev, t.tid, t.nstep, kPurpStep);
    L.usel = u53<R>(b0.w[2], b0.w[3]);
    {
        const R* base = tab_base(c.tv, m, t.type);
        const int i = find_bin(c.tv, t.T, c.ph->log10_emin, c.ph->bpd);
        const R w = (t.T - c.tv.E[i]) / (c.tv.E[i + 1] - c.tv.E[i]);
        L.sa = lerp_col(c.tv, base, i, 0, w);
        const R sb = lerp_col(c.tv, base, i, 1, w);
        L.stot = L.sa + sb;
        if (t.type != kGamma) {
            L.range = lerp_col(c.tv, base, i, 3, w);
            L.s_eloss = L.range <= (R)0.1 ? L.range : m_max((R)0.2 * L.range, (R)0.1);
        }
    }
    L.s_phys = L.stot > (R)0 ? expo<R>(b0.w[0], b0.w[1]) / L.stot : big_len<R>();
}

// ---- GeomQuery ----------------------------------------------------------
// WORLD: the track is known to be in the world volume
template <class P, bool WORLD = false, class R = typename P::R>
__device__ inline void stage_geom(const Ctx<P>& c, const Track<P>& t, Geo& G)
{
    const int v = WORLD ? 0 : t.vol;
    const double d[3] = {(double)t.u[0], (double)t.u[1], (double)t.u[2]};
    const Hit h = distance_out(*c.g, v, t.x, d);
    G.d_bnd = h.t;
    G.next = h.next;
    G.snap_axis = h.snap_axis;
    G.snap_val = h.snap_val;
    G.safety = safety(*c.g, v, t.x);
}

// ---- Propagation --------------------------------------------------------
// INTEG = false compiles the straight line and the helix only (field_method
// HELIX); INTEG = true adds the RK4 and RK45 integrators, which run in double
// in both precision policies.  VAC (a volume without material in a uniform
// field) leaves out the field-map evaluation.
// PARK (the batched driver's integration queue, field method RK45; no
// integrator is compiled in): a charged move in a field is not made here; the
// function returns true with the step's length, nominal limiter and radius of
// curvature in pr and the track unmoved, and stage_move_resume finishes the
// move from the integrated end point.
template <class P, bool INTEG, bool VAC = false, bool PARK = false, class R = typename P::R>
__device__ inline bool stage_move(const Ctx<P>& c, Track<P>& t, const Limits<R>& L, const Geo& G, Prop<R>& pr)
{
#pragma clang fp contract(off)
    static_assert(!(PARK && INTEG), "a parked move is integrated by the integration queue");
    const DevGeom& g = *c.g;
    const double s_phys = L.s_phys >= big_len<R>() ? kInf : (double)L.s_phys;
    const double s_eloss = L.s_eloss >= big_len<R>() ? kInf : (double)L.s_eloss;
    const double s_lim = fmin(s_phys, s_eloss);
    pr.T_pre = t.T;
    pr.crossed = 0;
    pr.rk.acc = 0;
    pr.rk.rej = 0;
    pr.rk.iters = 0;
    // the field at the pre-step point: its direction and kKB |B|
    double Bm = g.Bmag, kB = g.kB;
    double bh[3] = {g.Bhat[0], g.Bhat[1], g.Bhat[2]};
    if (!VAC && t.type != kGamma && g.field_map == kMapSolenoid) {
        // in double: the helix phase is kB s / p (see rk4_map_move)
        double Bd[3];
        field_at<double>(g, t.x, Bd);
        Bm = sqrt(Bd[0] * Bd[0] + Bd[1] * Bd[1] + Bd[2] * Bd[2]);
        kB = kKB * Bm;
#pragma unroll
        for (int a = 0; a < 3; ++a) bh[a] = Bm > 0.0 ? Bd[a] / Bm : 0.0;
    }
    if (t.type == kGamma || Bm == 0.0) {
        if (G.d_bnd <= s_lim) {
            pr.s = G.d_bnd;
            pr.lim = kLimGeom;
        } else {
            pr.s = s_lim;
            pr.lim = s_phys <= s_eloss ? kLimPhys : kLimEloss;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) t.x[a] += pr.s * (double)t.u[a];
        if (pr.lim == kLimGeom) {
            if (G.snap_axis == 0) t.x[0] = G.snap_val;
            else if (G.snap_axis == 1) t.x[1] = G.snap_val;
            else if (G.snap_axis == 2) t.x[2] = G.snap_val;
            t.vol = G.next;
            pr.crossed = 1;
        }
        return false;
    }
    // charged particle in a field
    const R p = m_sqrt(t.T * (t.T + (R)(2.0 * kMe)));
    // sine of the pitch angle from |u x b| (no cancellation near 0 or pi)
    const R bx = (R)bh[0], by = (R)bh[1], bz = (R)bh[2];
    const R cx = t.u[1] * bz - t.u[2] * by, cy = t.u[2] * bx - t.u[0] * bz, cz = t.u[0] * by - t.u[1] * bx;
    const R sin2 = cx * cx + cy * cy + cz * cz;
    double rcurv = kInf, dfield = kInf;
    if (sin2 > (R)0) {
        const R rc = p / ((R)kB * m_sqrt(sin2));
        rcurv = (double)rc;
        dfield = (double)m_sqrt((R)2 * rc * (R)c.ph->chord_tol);
    }
    const double cap = fmax(dfield, G.safety);
    const double s0 = fmin(s_lim, G.d_bnd);
    if (s0 <= cap) {
        pr.s = s0;
        pr.lim = G.d_bnd <= s_lim ? kLimGeom : (s_phys <= s_eloss ? kLimPhys : kLimEloss);
    } else {
        pr.s = cap;
        pr.lim = kLimField;
    }
    if (pr.lim == kLimGeom) pr.s += c.ph->push;
    if constexpr (PARK) {
        pr.rcurv = rcurv;
        return true;
    }
    if (INTEG && c.ph->field_method != kFieldHelix) {
        double ud[3] = {(double)t.u[0], (double)t.u[1], (double)t.u[2]};
        const double T = (double)t.T;
        if (c.ph->field_method == kFieldRk45) {
            const double s_done = rk45_move(g, t.type, T, pr.s, c.ph->rk_tol, c.ph->rk_max_sub, t.x, ud, pr.rk);
            if (s_done < pr.s) {  // attempts ran out: the step ends where integration stopped
                pr.s = s_done;
                pr.lim = kLimField;
            }
        } else {
            double nsub = rcurv < kInf ? ceil(pr.s / (c.ph->rk_frac * rcurv)) : 1.0;
            nsub = nsub < 1.0 ? 1.0 : (nsub > 100000.0 ? 100000.0 : nsub);
            if (g.field_map == kMapSolenoid) rk4_map_move(g, t.type, T, pr.s, (int)nsub, t.x, ud);
            else rk4_move<double>(t.type, T, g.B, pr.s, (int)nsub, t.x, ud);
        }
        t.u[0] = (R)ud[0];
        t.u[1] = (R)ud[1];
        t.u[2] = (R)ud[2];
    } else {
        helix_move<R>(t.type, t.T, bh, kB, pr.s, t.x, t.u);
    }
    const int nv = locate(g, t.x, t.vol, G.next);
    if (nv != t.vol) {
        t.vol = nv;
        pr.lim = kLimGeom;
        pr.crossed = 1;
    }
    return false;
}

// The end of a parked RK45 move (see stage_move): the integrated end point x,
// unit direction u and length s_done, then relocation, as stage_move does
// after its own integration.  pr holds the parked step's length and limiter.
template <class P, class R = typename P::R>
__device__ inline void stage_move_resume(const Ctx<P>& c, Track<P>& t, const Geo& G, Prop<R>& pr, const double x[3],
                                         const double u[3], double s_done, int acc, int rej)
{
    pr.T_pre = t.T;
    pr.crossed = 0;
    pr.rk.acc = acc;
    pr.rk.rej = rej;
    pr.rk.iters = 0;
    if (s_done < pr.s) {  // attempts ran out: the step ends where integration stopped
        pr.s = s_done;
        pr.lim = kLimField;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        t.x[a] = x[a];
        t.u[a] = (R)u[a];
    }
    const int nv = locate(*c.g, t.x, t.vol, G.next);
    if (nv != t.vol) {
        t.vol = nv;
        pr.lim = kLimGeom;
        pr.crossed = 1;
    }
}

// ---- PostPropagation: multiple scattering -------------------------------
template <class P, class R = typename P::R>
__device__ inline void stage_msc(const Ctx<P>& c, Track<P>& t, const Limits<R>& L, const Prop<R>& pr)
{
    if (t.type == kGamma || L.m < 0 || !(pr.s > 0.0)) return;
    const R th0 = highland<R>(pr.T_pre, (R)pr.s, (R)c.ph->mat[L.m].X0);
    const U4 b = stream_block(c.seed, t.ev, t.tid, t.nstep, kPurpMsc);
    const R ua = u53<R>(b.w[0], b.w[1]), ub = u53<R>(b.w[2], b.w[3]);
    const R r = m_sqrt((R)-2 * m_log(ua));
    const R a = (R)(2.0 * kPi) * ub;
    const R tx = th0 * (r * m_cos(a)), ty = th0 * (r * m_sin(a));
    const R th = m_sqrt(tx * tx + ty * ty);
    const R phi = m_atan2(ty, tx);
    rotate<R>(t.u, m_cos(th), m_sin(th), phi);
}

// ---- AlongStepAction: continuous loss; returns true if the track stopped --
template <class P, class R = typename P::R>
__device__ inline bool stage_eloss(const Ctx<P>& c, Track<P>& t, const Limits<R>& L, const Prop<R>& pr, StepOut<R>& o)
{
    if (t.type == kGamma || L.m < 0) return false;
    const R* base = tab_base(c.tv, L.m, t.type);
    const R Tp = pr.T_pre;
    const R s = (R)pr.s;
    R dE;
    if (s < (R)0.01 * L.range) {
        const int i = find_bin(c.tv, Tp, c.ph->log10_emin, c.ph->bpd);
        const R w = (Tp - c.tv.E[i]) / (c.tv.E[i + 1] - c.tv.E[i]);
        dE = lerp_col(c.tv, base, i, 2, w) * s;
    } else {
        dE = Tp - range_inverse(c.tv, base, L.range - s);
    }
    const R rtrack = P::kMixed ? (R)c.ph->r_track_f[L.m][t.type == kPositron] : (R)c.ph->r_track[L.m][t.type == kPositron];
    bool stopped = false;
    if (Tp - dE < (R)c.ph->t_track || L.range - s <= rtrack) {
        dE = Tp;
        stopped = true;
    }
    o.edep += (double)dE;
    t.T = Tp - dE;
    return stopped;
}

// ---- PostStepActions: discrete interaction ------------------------------
template <class P, class R = typename P::R>
__device__ inline void interact(const Ctx<P>& c, Track<P>& t, bool first, StepOut<R>& o)
{
    const DevPhys& ph = *c.ph;
    const Key key{c.seed, t.tid, t.ev, t.nstep};
    uint64_t ids[2];
    if (t.type == kGamma) {
        const R k = t.T;
        if (first) {
            o.proc = kCompton;
            R eps, om, tt, phi;
            if ((ph.fs_alias >> kAlCompton) & 1)
                alias_compton<R>(alias_view<R>(ph), k, key, eps, om, tt, phi);
            else if (!sample_compton<R>(k, key, eps, om, tt, phi))
                o.rej_exhausted += 1;
            const R k1 = eps * k, Te = om * k;
            const R st = m_sqrt(tt * ((R)2 - tt));
            R de[3] = {t.u[0], t.u[1], t.u[2]};
            rotate<R>(t.u, (R)1 - tt, st, phi);
            child_ids(c, t, ids);
            if (Te >= (R)ph.t_track) {
                // electron momentum k u - k' u' = (Te + k' t) u - k' sin(theta) n:
                // polar angle atan2(k' sin, Te + k' t) on the opposite azimuth
                const R A = Te + k1 * tt, Bv = k1 * st;
                const R N = m_sqrt(A * A + Bv * Bv);
                rotate<R>(de, A / N, Bv / N, phi + (R)kPi);
                add_child(o, kElectron, Te, de, ids[0]);
            } else {
                o.edep += (double)Te;
            }
            if (k1 < (R)ph.t_track) {
                o.edep += (double)k1;
                t.T = (R)0;
                o.status = kDead;
            } else {
                t.T = k1;
            }
        } else {
            if (k <= (R)(2.0 * kMe)) {
                o.proc = kNull;
                return;
            }
            o.proc = kPair;
            R x, phi;
            if ((ph.fs_alias >> kAlPair) & 1)
                x = alias_sample<R>(alias_view<R>(ph), kAlPair, k, (R)ph.t_cut, (R)ph.k_cut, key, phi);
            else if (!sample_pair<R>(k, key, x, phi))
                o.rej_exhausted += 1;
            const R Em = x * k, Ep = ((R)1 - x) * k;
            const R thm = (R)kMe / Em, thp = (R)kMe / Ep;
            R dm[3] = {t.u[0], t.u[1], t.u[2]};
            R dp[3] = {t.u[0], t.u[1], t.u[2]};
            rotate<R>(dm, m_cos(thm), m_sin(thm), phi);
            rotate<R>(dp, m_cos(thp), m_sin(thp), phi + (R)kPi);
            child_ids(c, t, ids);
            const R Tm = Em - (R)kMe, Tq = Ep - (R)kMe;
            if (Tm >= (R)ph.t_track) add_child(o, kElectron, Tm, dm, ids[0]);
            else o.edep += (double)Tm;
            add_child(o, kPositron, Tq, dp, ids[1]);
            o.n_pair += 1;
            t.T = (R)0;
            o.status = kDead;
        }
        return;
    }
    const R T = t.T;
    if (first) {
        const bool pos = t.type == kPositron;
        if (pos ? T <= (R)ph.t_cut : T <= (R)(2.0 * ph.t_cut)) {
            o.proc = kNull;
            return;
        }
        o.proc = pos ? kBhabha : kMoller;
        R eps, phi;
        const int am = pos ? kAlBhabha : kAlMoller;
        if ((ph.fs_alias >> am) & 1) {
            eps = alias_sample<R>(alias_view<R>(ph), am, T, (R)ph.t_cut, (R)ph.k_cut, key, phi);
        } else {
            const bool ok = pos ? sample_bhabha<R>(T, (R)ph.t_cut, key, eps, phi)
                                : sample_moller<R>(T, (R)ph.t_cut, key, eps, phi);
            if (!ok) o.rej_exhausted += 1;
        }
        const R Td = eps * T;
        const R Tp = T - Td;
        const R m2 = (R)(2.0 * kMe);
        // two-body kinematics on an electron at rest (equal masses): each
        // outgoing particle of kinetic energy T_o leaves at
        // cos = sqrt(T_o (T + 2m) / (T (T_o + 2m))); the two azimuths are opposite
        const R ct = m_sqrt(Td * (T + m2) / (T * (Td + m2)));
        const R st = m_sqrt(m2 * Tp / (T * (Td + m2)));
        R ud[3] = {t.u[0], t.u[1], t.u[2]};
        rotate<R>(ud, ct, st, phi);
        child_ids(c, t, ids);
        add_child(o, kElectron, Td, ud, ids[0]);
        if (Tp > (R)0) {
            const R cp = m_sqrt(Tp * (T + m2) / (T * (Tp + m2)));
            const R sp = m_sqrt(m2 * Td / (T * (Tp + m2)));
            rotate<R>(t.u, cp, sp, phi + (R)kPi);
        }
        t.T = Tp;
    } else {
        if (T <= (R)ph.k_cut) {
            o.proc = kNull;
            return;
        }
        o.proc = t.type == kPositron ? kBremsEp : kBremsEm;
        R k;
        if ((ph.fs_alias >> kAlBrems) & 1) {
            R phi_unused;
            k = alias_sample<R>(alias_view<R>(ph), kAlBrems, T, (R)ph.t_cut, (R)ph.k_cut, key, phi_unused);
        } else if (!sample_brems<R>(T, (R)ph.k_cut, key, k)) {
            o.rej_exhausted += 1;
        }
        child_ids(c, t, ids);
        add_child(o, kGamma, k, t.u, ids[0]);
        t.T = T - k;
    }
}

// ---- PostStepActions + SteppingActions ----------------------------------
template <class P, class R = typename P::R>
__device__ inline void stage_finish(const Ctx<P>& c, Track<P>& t, const Limits<R>& L, const Prop<R>& pr, bool stopped,
                                    StepOut<R>& o)
{
    if (pr.lim == kLimPhys && !pr.crossed && !stopped) interact(c, t, L.usel * L.stot < L.sa, o);
    if (stopped) {
        if (t.type == kPositron) annihilate(c, t, o);
        o.status = kDead;
    } else if (o.status == kAlive && t.vol == kOutside) {
        o.e_escaped += (double)t.T;
        o.status = kEscaped;
    }
    t.nstep += 1;
}

// ---- the whole step in registers ----------------------------------------
// VAC: specialisation for a charged track in a volume without material (the
// world or a vacuum layer) in a uniform field with the helix (the caller
// checks this); WORLD: in the world volume.  It runs the same stage code
// with the material branches decided at compile time, so it takes exactly the
// steps of the general form.
// the stages after Propagation
template <class P, class R = typename P::R>
__device__ __forceinline__ void step_after_move(const Ctx<P>& c, Track<P>& t, const Limits<R>& L, const Geo& G,
                                                const Prop<R>& pr, StepOut<R>& o)
{
    o.did_step = 1;
    o.s = pr.s;
    o.lim = pr.lim;
    o.s_phys = L.s_phys >= big_len<R>() ? kInf : (double)L.s_phys;
    o.d_bnd = G.d_bnd;
    o.safety = G.safety;
    o.rk = pr.rk;
    stage_msc(c, t, L, pr);
    const bool stopped = stage_eloss(c, t, L, pr, o);
    stage_finish(c, t, L, pr, stopped, o);
}

template <class P, bool INTEG, bool VAC = false, bool WORLD = false, class R = typename P::R>
__device__ inline void step_track(const Ctx<P>& c, Track<P>& t, StepOut<R>& o)
{
    static_assert(!(VAC && INTEG), "the vacuum form is helix-only");
    init_out(t, o);
    if (!stage_prestep(c, t, o)) return;
    Limits<R> L;
    stage_limit<P, VAC>(c, t, L);
    Geo G;
    stage_geom<P, WORLD>(c, t, G);
    Prop<R> pr;
    stage_move<P, INTEG, VAC>(c, t, L, G, pr);
    step_after_move(c, t, L, G, pr, o);
}

// The same step ended after one of its stages (Sec. 2.1.2), for the
// per-stage test entry: s_phys and the continuous-loss length after
// ComputeIntLen, then the boundary distance and safety, then the step length,
// limiter and the moved track, then the deflection, then the loss.
enum : int { kThruLimit = 1, kThruGeom = 2, kThruMove = 3, kThruMsc = 4, kThruEloss = 5 };

template <class P, class R = typename P::R>
__device__ inline void step_track_through(const Ctx<P>& c, Track<P>& t, StepOut<R>& o, int stop, double& s_eloss)
{
    init_out(t, o);
    s_eloss = 0.0;
    if (!stage_prestep(c, t, o)) return;
    Limits<R> L;
    stage_limit<P>(c, t, L);
    o.s_phys = L.s_phys >= big_len<R>() ? kInf : (double)L.s_phys;
    s_eloss = L.s_eloss >= big_len<R>() ? kInf : (double)L.s_eloss;
    if (stop == kThruLimit) return;
    Geo G;
    stage_geom<P>(c, t, G);
    o.d_bnd = G.d_bnd;
    o.safety = G.safety;
    if (stop == kThruGeom) return;
    Prop<R> pr;
    stage_move<P, true>(c, t, L, G, pr);
    o.did_step = 1;
    o.s = pr.s;
    o.lim = pr.lim;
    o.rk = pr.rk;
    if (stop == kThruMove) return;
    stage_msc(c, t, L, pr);
    if (stop == kThruMsc) return;
    const bool stopped = stage_eloss(c, t, L, pr, o);
    if (stop == kThruEloss) return;
    stage_finish(c, t, L, pr, stopped, o);
}

// The same step, stopped at an RK45 move (returns true: the track is unmoved
// and L, G, pr hold what the rest of the step needs); any other step is taken
// whole (returns false).
template <class P, class R = typename P::R>
__device__ inline bool step_track_park(const Ctx<P>& c, Track<P>& t, StepOut<R>& o, Limits<R>& L, Geo& G, Prop<R>& pr)
{
    init_out(t, o);
    if (!stage_prestep(c, t, o)) return false;
    stage_limit<P>(c, t, L);
    stage_geom<P>(c, t, G);
    if (stage_move<P, false, false, true>(c, t, L, G, pr)) return true;
    step_after_move(c, t, L, G, pr, o);
    return false;
}

// The rest of a parked step from its integration result.
template <class P, class R = typename P::R>
__device__ inline void step_track_resume(const Ctx<P>& c, Track<P>& t, StepOut<R>& o, const Limits<R>& L, const Geo& G,
                                         Prop<R>& pr, const double x[3], const double u[3], double s_done, int acc,
                                         int rej)
{
    init_out(t, o);
    stage_move_resume(c, t, G, pr, x, u, s_done, acc, rej);
    step_after_move(c, t, L, G, pr, o);
}

// ---- charged tracks in the vacuum world: the looper form ------------------
// A charged track in the world volume of a slab stack, in a uniform field
// with the helix, takes exactly the step of step_track<P, false, true, true>
// (the same expressions in the same order, so the same bits), with savings
// that matter for the low-population tail, where such tracks step one after
// another along a dependent chain:
//   * what vacuum does not change is formed once per run of steps (the
//     momentum and the helix phase per unit length from the kinetic energy,
//     which no vacuum step alters; field and cut constants);
//   * work whose outcome is already decided is skipped.  A ray leaves the
//     world box no sooner than the distance to its nearest wall, and enters
//     the envelope box no sooner than the distance to that box, so when
//     either distance certainly exceeds the field step its candidate is not
//     formed; a candidate that is formed is divided out only if it may be
//     the shorter; the square root of the distance to the envelope is taken
//     only if the safety may exceed the bending estimate.  "Certainly" holds
//     with a margin far above the worst rounding of the quantities compared
//     (2^-40 for quotients and roots, 2^-16 for the distance bounds, which
//     also absorb the rounding of a float direction's length).
template <class P> struct WorldRun {
    using R = typename P::R;
    bool lean;        // the looper form applies (slab stack, field on, charged, above the tracking cut)
    double kq;        // -(q kB / p): helix phase per unit length
    R pf;             // momentum in the policy's precision (bending radius)
    R kBf, chord;     // curvature constant and bending tolerance
    R b[3];           // field direction
    double push;
    double zlo, zhi;  // the envelope's extent along the stack
    double zc, zh;    // ... as centre and half length
};

template <class P, class R = typename P::R>
__device__ __forceinline__ WorldRun<P> world_run(const Ctx<P>& c, const Track<P>& t)
{
#pragma clang fp contract(off)
    WorldRun<P> k;
    const DevGeom& g = *c.g;
    // vacuum keeps the kinetic energy and the type: these tests hold for the run
    k.lean = g.axis == 0 && g.Bmag != 0.0 && t.type != kGamma && !(t.T < (R)c.ph->t_track);
    k.zlo = g.bounds[0];
    k.zhi = g.bounds[g.n_vol];
    k.zc = 0.5 * (g.bounds[0] + g.bounds[g.n_vol]);
    k.zh = 0.5 * (g.bounds[g.n_vol] - g.bounds[0]);
    const double q = t.type == kElectron ? -1.0 : 1.0;
    const double Td = (double)t.T;
    const double p = sqrt(Td * (Td + 2.0 * kMe));
    k.kq = -(q * g.kB / p);
    k.pf = m_sqrt(t.T * (t.T + (R)(2.0 * kMe)));
    k.kBf = (R)g.kB;
    k.chord = (R)c.ph->chord_tol;
#pragma unroll
    for (int a = 0; a < 3; ++a) k.b[a] = (R)g.Bhat[a];
    k.push = c.ph->push;
    return k;
}

// true only if fl(num / den) > cap is certain (num, den > 0)
__device__ __forceinline__ bool quotient_beyond(double num, double den, double cap)
{
#pragma clang fp contract(off)
    const double lim = cap * den;
    return lim > 0x1p-1000 && num > lim * (1.0 + 0x1p-40);
}

// true only if fl(sqrt(q)) < d is certain
__device__ __forceinline__ bool root_below(double q, double d)
{
#pragma clang fp contract(off)
    return q <= (d * d) * (1.0 - 0x1p-40);
}

// The candidates of slab_world without their divisions: entry into the
// envelope box at nn / nd (valid if `entry`), exit from the world box at wn / wd.
struct WorldCand {
    double nn, nd, wn, wd;
    int an;
    bool entry;
};

__device__ __forceinline__ void world_entry(const DevGeom& g, const double p[3], const double d[3], WorldCand& w)
{
#pragma clang fp contract(off)
    const double lo[3] = {-g.env[0], -g.env[1], g.bounds[0]};
    const double hi[3] = {g.env[0], g.env[1], g.bounds[g.n_vol]};
    double nn = -1.0, nd = 0.0, fn = 1.0, fd = 0.0;
    int an = -1;
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool moving = d[a] != 0.0;
        const bool up = d[a] > 0.0;
        const double den = fabs(d[a]);
        const double n_near = up ? lo[a] - p[a] : p[a] - hi[a];
        const double n_far = up ? hi[a] - p[a] : p[a] - lo[a];
        miss = miss | (!moving & ((p[a] < lo[a]) | (p[a] > hi[a])));
        const bool tn = moving & (n_near * nd > nn * den);
        const bool tf = moving & (n_far * fd < fn * den);
        nn = tn ? n_near : nn;
        nd = tn ? den : nd;
        an = tn ? a : an;
        fn = tf ? n_far : fn;
        fd = tf ? den : fd;
    }
    w.nn = nn;
    w.nd = nd;
    w.an = an;
    w.entry = nd != 0.0 && !miss && nn * fd <= fn * nd && fn > 0.0;
}

__device__ __forceinline__ void world_exit(const DevGeom& g, const double p[3], const double d[3], WorldCand& w)
{
#pragma clang fp contract(off)
    const double wlo[3] = {-g.world[0], -g.world[1], g.world[2]};
    const double whi[3] = {g.world[0], g.world[1], g.world[3]};
    double wn = 1.0, wd = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool up = d[a] > 0.0;
        const double n = up ? whi[a] - p[a] : p[a] - wlo[a];
        const double den = fabs(d[a]);
        const bool take = (d[a] != 0.0) & (n * wd < wn * den);
        wn = take ? n : wn;
        wd = take ? den : wd;
    }
    w.wn = wn;
    w.wd = wd;
}

template <class P, class R = typename P::R>
__device__ inline void step_world(const Ctx<P>& c, const WorldRun<P>& k, Track<P>& t, StepOut<R>& o)
{
#pragma clang fp contract(off)
    const DevGeom& g = *c.g;
    if (!k.lean || t.vol != 0 || (long long)t.nstep >= c.ph->max_steps) {
        step_track<P, false, true, true>(c, t, o);
        return;
    }
    init_out(t, o);
    const double p[3] = {t.x[0], t.x[1], t.x[2]};
    const double d[3] = {(double)t.u[0], (double)t.u[1], (double)t.u[2]};
    // bending estimate (stage_move)
    const R cx = t.u[1] * k.b[2] - t.u[2] * k.b[1], cy = t.u[2] * k.b[0] - t.u[0] * k.b[2],
            cz = t.u[0] * k.b[1] - t.u[1] * k.b[0];
    const R sin2 = cx * cx + cy * cy + cz * cz;
    double dfield = kInf;
    if (sin2 > (R)0) {
        const R rc = k.pf / (k.kBf * m_sqrt(sin2));
        dfield = (double)m_sqrt((R)2 * rc * k.chord);
    }
    // safety (slab_world_safety): the world's walls, then the envelope box
    double walls = fmin(g.world[0] - fabs(p[0]), g.world[1] - fabs(p[1]));
    walls = fmin(walls, fmin(p[2] - g.world[2], g.world[3] - p[2]));
    const double qx = fmax(fabs(p[0]) - g.env[0], 0.0);
    const double qy = fmax(fabs(p[1]) - g.env[1], 0.0);
    const double qz = fmax(fabs(p[2] - k.zc) - k.zh, 0.0);
    const double qq = qx * qx + qy * qy + qz * qz;
    double cap;
    if (walls <= dfield || root_below(qq, dfield)) {
        cap = dfield;   // the safety does not exceed the bending estimate
    } else {
        double sf = fmin(walls, sqrt(qq));
        sf = sf > 0.0 ? sf : 0.0;
        cap = fmax(dfield, sf);
    }
    // boundary candidates along the ray (slab_world), formed only where they
    // may be shorter than the field step.  A ray that is outside the
    // envelope's extent along some axis and does not move towards it there
    // never enters (slab_world then finds no valid entry either: the far
    // candidate of that axis is negative, or the axis misses).
    // (across the stack, outside the envelope's extent and moving away from it
    // along that axis: |p| > env and p d >= 0, i.e. qx > 0 and p d >= 0)
    const bool away = ((qx > 0.0) & (p[0] * d[0] >= 0.0)) | ((qy > 0.0) & (p[1] * d[1] >= 0.0)) |
                      ((p[2] > k.zhi) & (d[2] >= 0.0)) | ((p[2] < k.zlo) & (d[2] <= 0.0));
    const bool env_far = away || qq > (cap * cap) * (1.0 + 0x1p-14);
    const bool walls_far = walls > cap * (1.0 + 0x1p-16);
    WorldCand w;
    w.entry = false;
    if (!env_far) world_entry(g, p, d, w);
    const bool entry_far = env_far || !w.entry || (w.nn > 0.0 && quotient_beyond(w.nn, w.nd, cap));
    bool exit_far = walls_far;
    if (!exit_far) {
        world_exit(g, p, d, w);
        exit_far = w.wd > 0.0 && quotient_beyond(w.wn, w.wd, cap);
    }
    double s;
    int lim;
    int next = 0;
    if (entry_far && exit_far) {
        s = cap;                  // every boundary lies beyond the field step
        lim = kLimField;
        o.d_bnd = kInf;
    } else {
        // the exact boundary distance, as slab_world.  A candidate known to
        // lie beyond the field step is also beyond the other one here (which
        // may not exceed the field step by more than rounding), so it cannot
        // be the distance and is not formed: with the walls far, the distance
        // is the envelope entry; with the envelope far (or moved away from),
        // the world exit.
        double dt = kInf;
        if (!env_far && w.entry) {
            dt = w.nn > 0.0 ? w.nn / w.nd : 0.0;
            next = (w.nn > 0.0 && w.an == 2) ? (d[2] > 0.0 ? 1 : g.n_vol) : 0;   // a guess for relocation
        }
        if (!walls_far) {
            double tw = w.wd > 0.0 ? w.wn / w.wd : kInf;
            tw = tw > 0.0 ? tw : 0.0;
            if (!(dt <= tw)) {
                dt = tw;
                next = 0;
            }
        }
        o.d_bnd = dt;
        const double s0 = fmin(kInf, dt);
        if (s0 <= cap) {
            s = s0;
            lim = kLimGeom;
        } else {
            s = cap;
            lim = kLimField;
        }
        if (lim == kLimGeom) s += k.push;
    }
    // helix (helix_move) with the run's phase per unit length
    {
        const double th = k.kq * s;
        const double thr = sizeof(R) == sizeof(double) ? th : th - 2.0 * kPi * rint(th * (0.5 / kPi));
        const R upar = t.u[0] * k.b[0] + t.u[1] * k.b[1] + t.u[2] * k.b[2];
        const R up[3] = {t.u[0] - upar * k.b[0], t.u[1] - upar * k.b[1], t.u[2] - upar * k.b[2]};
        const R bxu[3] = {k.b[1] * up[2] - k.b[2] * up[1], k.b[2] * up[0] - k.b[0] * up[2],
                          k.b[0] * up[1] - k.b[1] * up[0]};
        const R sn = m_sin((R)thr), hs = m_sin((R)(0.5 * thr));
        const R omc = (R)2 * hs * hs;
        R f1, f2;
        if (fabs(th) < 1.0e-4) {
            f1 = (R)(1.0 - th * th / 6.0);
            f2 = (R)(0.5 * th);
        } else {
            f1 = sn / (R)th;
            f2 = omc / (R)th;
        }
        const R cs = (R)1 - omc;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            t.x[a] += s * (double)(upar * k.b[a] + f1 * up[a] + f2 * bxu[a]);
            t.u[a] = upar * k.b[a] + cs * up[a] + sn * bxu[a];
        }
        normalise(t.u);
    }
    const int nv = locate(g, t.x, 0, next);
    if (nv != 0) {
        t.vol = nv;
        lim = kLimGeom;
    }
    o.did_step = 1;
    o.s = s;
    o.lim = lim;
    o.s_phys = kInf;
    if (t.vol == kOutside) {
        o.e_escaped += (double)t.T;
        o.status = kEscaped;
    }
    t.nstep += 1;
}

}  // namespace gv
