/*
 * Oracle geometry (test infrastructure only): a 1-D stack of volumes along one
 * axis inside a common envelope inside an outer vacuum world.  This is the
 * layered case of the GeomQuery stage (Sec. 3.4): distance to the next
 * boundary along the direction, isotropic safety, and the next volume.  In a
 * layered detector the navigator reduces to index +-1 across stack faces.
 *
 * Volume ids: 0 = outer world, 1..n = stack volumes, OR_OUTSIDE = -1.
 *   Z slabs : volume v is the box |x|<=env0, |y|<=env1, z in [b_{v-1}, b_v];
 *             world box |x|<=w0, |y|<=w1, z in [w2, w3].
 *   R shells: volume v is r in [b_{v-1}, b_v], |z| <= env0 (b_0 = 0 means a
 *             solid cylinder); world cylinder r <= w0, |z| <= w1.
 * On an exact tie between faces the first face in the order x-, x+, y-, y+,
 * z-, z+ (shells: inner, outer, z-, z+) wins.
 *
 * Every distance also reports the plane face it ends on (axis and value), so
 * that a straight boundary-limited step can place the point exactly on that
 * plane; cylinder surfaces report no face.
 */
#include "or_internal.h"

#define BIG 1.0e300

int32_t or_vol_material(int32_t vol) { return (vol >= 1) ? G.vmat[vol - 1] : -1; }
int32_t or_vol_cell(int32_t vol) { return (vol >= 1) ? G.vcell[vol - 1] : -1; }

/* index v in 1..n with b_{v-1} <= c < b_v (c >= b_n maps to n, c <= b_0 to 1) */
static int32_t stack_index(double c)
{
    if (c <= G.bounds[0]) return 1;
    if (c >= G.bounds[G.n_vol]) return G.n_vol;
    int32_t lo = 0, hi = G.n_vol;
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) / 2;
        if (G.bounds[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo + 1;
}

int32_t or_locate(const double p[3])
{
    if (G.axis == OR_AXIS_Z_SLABS) {
        if (fabs(p[0]) <= G.env[0] && fabs(p[1]) <= G.env[1] && p[2] >= G.bounds[0] &&
            p[2] <= G.bounds[G.n_vol])
            return stack_index(p[2]);
        if (fabs(p[0]) <= G.world[0] && fabs(p[1]) <= G.world[1] && p[2] >= G.world[2] &&
            p[2] <= G.world[3])
            return 0;
        return OR_OUTSIDE;
    }
    double r = sqrt(p[0] * p[0] + p[1] * p[1]);
    if (r <= G.bounds[G.n_vol] && fabs(p[2]) <= G.env[0]) return stack_index(r);
    if (r <= G.world[0] && fabs(p[2]) <= G.world[1]) return 0;
    return OR_OUTSIDE;
}

typedef struct {
    double t;
    int32_t next;
    int32_t snap_axis;   /* -1: no plane face */
    double snap_val;
} hit_t;

/* ---- slabs ---- */

static hit_t slab_dist_out(int32_t v, const double p[3], const double d[3])
{
    double lo[3] = {-G.env[0], -G.env[1], G.bounds[v - 1]};
    double hi[3] = {G.env[0], G.env[1], G.bounds[v]};
    double best = BIG;
    int face = -1;
    for (int a = 0; a < 3; ++a) {
        if (d[a] < 0.0) {
            double t = (lo[a] - p[a]) / d[a];
            if (t < best) { best = t; face = 2 * a; }
        } else if (d[a] > 0.0) {
            double t = (hi[a] - p[a]) / d[a];
            if (t < best) { best = t; face = 2 * a + 1; }
        }
    }
    hit_t h;
    h.t = best > 0.0 ? best : 0.0;
    if (face == 4) h.next = (v == 1) ? 0 : v - 1;
    else if (face == 5) h.next = (v == G.n_vol) ? 0 : v + 1;
    else h.next = 0;
    h.snap_axis = face / 2;
    h.snap_val = (face & 1) ? hi[face / 2] : lo[face / 2];
    return h;
}

static double slab_safety(int32_t v, const double p[3])
{
    double s = p[2] - G.bounds[v - 1];
    s = fmin(s, G.bounds[v] - p[2]);
    s = fmin(s, G.env[0] - fabs(p[0]));
    s = fmin(s, G.env[1] - fabs(p[1]));
    return s > 0.0 ? s : 0.0;
}

/* world box: entry into the envelope box, or exit from the world */
static hit_t slab_world_dist(const double p[3], const double d[3])
{
    double lo[3] = {-G.env[0], -G.env[1], G.bounds[0]};
    double hi[3] = {G.env[0], G.env[1], G.bounds[G.n_vol]};
    double tnear = -BIG, tfar = BIG;
    int axis_near = -1, miss = 0;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (p[a] < lo[a] || p[a] > hi[a]) miss = 1;
            continue;
        }
        double t1 = (lo[a] - p[a]) / d[a], t2 = (hi[a] - p[a]) / d[a];
        double tmin = t1 < t2 ? t1 : t2, tmax = t1 < t2 ? t2 : t1;
        if (tmin > tnear) { tnear = tmin; axis_near = a; }
        if (tmax < tfar) tfar = tmax;
    }
    hit_t h;
    double t_env = BIG;
    int32_t v_env = 0;
    int snap_axis = -1;
    double snap_val = 0.0;
    if (!miss && tnear <= tfar && tfar > 0.0) {
        if (tnear > 0.0) {
            t_env = tnear;
            snap_axis = axis_near;
            snap_val = d[axis_near] > 0.0 ? lo[axis_near] : hi[axis_near];
            if (axis_near == 2) v_env = (d[2] > 0.0) ? 1 : G.n_vol;
            else v_env = stack_index(p[2] + t_env * d[2]);
        } else {  /* on or inside the envelope surface already */
            t_env = 0.0;
            v_env = stack_index(p[2]);
        }
    }
    double wlo[3] = {-G.world[0], -G.world[1], G.world[2]};
    double whi[3] = {G.world[0], G.world[1], G.world[3]};
    double t_w = BIG;
    for (int a = 0; a < 3; ++a) {
        double t = BIG;
        if (d[a] < 0.0) t = (wlo[a] - p[a]) / d[a];
        else if (d[a] > 0.0) t = (whi[a] - p[a]) / d[a];
        if (t < t_w) t_w = t;
    }
    if (t_w < 0.0) t_w = 0.0;
    if (t_env <= t_w) {
        h.t = t_env;
        h.next = v_env;
        h.snap_axis = snap_axis;
        h.snap_val = snap_val;
    } else {
        h.t = t_w;
        h.next = OR_OUTSIDE;
        h.snap_axis = -1;
        h.snap_val = 0.0;
    }
    return h;
}

static double slab_world_safety(const double p[3])
{
    double s = G.world[0] - fabs(p[0]);
    s = fmin(s, G.world[1] - fabs(p[1]));
    s = fmin(s, p[2] - G.world[2]);
    s = fmin(s, G.world[3] - p[2]);
    /* Euclidean distance to the envelope box from outside */
    double cz = 0.5 * (G.bounds[0] + G.bounds[G.n_vol]);
    double hz = 0.5 * (G.bounds[G.n_vol] - G.bounds[0]);
    double qx = fabs(p[0]) - G.env[0], qy = fabs(p[1]) - G.env[1], qz = fabs(p[2] - cz) - hz;
    qx = qx > 0.0 ? qx : 0.0;
    qy = qy > 0.0 ? qy : 0.0;
    qz = qz > 0.0 ? qz : 0.0;
    s = fmin(s, sqrt(qx * qx + qy * qy + qz * qz));
    return s > 0.0 ? s : 0.0;
}

/* ---- shells ---- */

/* exit through the cylinder of radius R from inside: the larger root */
static double cyl_exit(const double p[3], const double d[3], double R)
{
    double a = d[0] * d[0] + d[1] * d[1];
    if (a == 0.0) return BIG;
    double b = p[0] * d[0] + p[1] * d[1];
    double c = p[0] * p[0] + p[1] * p[1] - R * R;
    double disc = b * b - a * c;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    return (b <= 0.0) ? (-b + sq) / a : -c / (b + sq);
}

/* entry into the cylinder of radius R from outside while moving inward: the
 * smaller root, or BIG if the line misses it */
static double cyl_entry(const double p[3], const double d[3], double R)
{
    double a = d[0] * d[0] + d[1] * d[1];
    if (a == 0.0) return BIG;
    double b = p[0] * d[0] + p[1] * d[1];
    if (b >= 0.0) return BIG;
    double c = p[0] * p[0] + p[1] * p[1] - R * R;
    double disc = b * b - a * c;
    if (disc < 0.0) return BIG;
    return c / (-b + sqrt(disc));
}

static hit_t shell_dist_out(int32_t v, const double p[3], const double d[3])
{
    double rin = G.bounds[v - 1], rout = G.bounds[v], H = G.env[0];
    double best = BIG;
    int face = -1;
    if (rin > 0.0) {
        double t = cyl_entry(p, d, rin);
        if (t < best) { best = t; face = 0; }
    }
    {
        double t = cyl_exit(p, d, rout);
        if (t < best) { best = t; face = 1; }
    }
    if (d[2] < 0.0) {
        double t = (-H - p[2]) / d[2];
        if (t < best) { best = t; face = 2; }
    } else if (d[2] > 0.0) {
        double t = (H - p[2]) / d[2];
        if (t < best) { best = t; face = 3; }
    }
    hit_t h;
    h.t = best > 0.0 ? best : 0.0;
    h.snap_axis = -1;
    h.snap_val = 0.0;
    if (face == 0) h.next = v - 1;
    else if (face == 1) h.next = (v == G.n_vol) ? 0 : v + 1;
    else {
        h.next = 0;
        h.snap_axis = 2;
        h.snap_val = (face == 2) ? -H : H;
    }
    return h;
}

static double shell_safety(int32_t v, const double p[3])
{
    double r = sqrt(p[0] * p[0] + p[1] * p[1]);
    double rin = G.bounds[v - 1], rout = G.bounds[v];
    double s = rout - r;
    if (rin > 0.0) s = fmin(s, r - rin);
    s = fmin(s, G.env[0] - fabs(p[2]));
    return s > 0.0 ? s : 0.0;
}

/* world cylinder: entry into the envelope cylinder r <= R, |z| <= H, found as
 * the overlap of the ray's parameter intervals inside the infinite cylinder
 * and inside the z slab (so a point on the surface enters only when moving
 * inward), or exit from the world */
static hit_t shell_world_dist(const double p[3], const double d[3])
{
    double R = G.bounds[G.n_vol], H = G.env[0];
    double t_env = BIG;
    int32_t v_env = 0;
    int snap_axis = -1;
    double snap_val = 0.0;
    /* interval inside the infinite cylinder */
    double a = d[0] * d[0] + d[1] * d[1];
    double b = p[0] * d[0] + p[1] * d[1];
    double c = p[0] * p[0] + p[1] * p[1] - R * R;
    double c0 = -BIG, c1 = BIG;
    int miss = 0;
    if (a == 0.0) {
        if (c > 0.0) miss = 1;
    } else {
        double disc = b * b - a * c;
        if (disc < 0.0) miss = 1;
        else {
            double sq = sqrt(disc);
            double q = (b >= 0.0) ? -(b + sq) : -(b - sq);
            double r1 = q / a, r2 = (q != 0.0) ? c / q : 0.0;
            c0 = r1 < r2 ? r1 : r2;
            c1 = r1 < r2 ? r2 : r1;
        }
    }
    /* interval inside the z slab */
    double z0 = -BIG, z1 = BIG;
    if (d[2] == 0.0) {
        if (fabs(p[2]) > H) miss = 1;
    } else {
        double ta = (-H - p[2]) / d[2], tb = (H - p[2]) / d[2];
        z0 = ta < tb ? ta : tb;
        z1 = ta < tb ? tb : ta;
    }
    if (!miss) {
        double tnear = c0 > z0 ? c0 : z0;
        double tfar = c1 < z1 ? c1 : z1;
        if (tnear <= tfar && tfar > 0.0) {
            if (tnear > 0.0) {
                t_env = tnear;
                if (z0 > c0) {  /* through an end cap */
                    double x = p[0] + t_env * d[0], y = p[1] + t_env * d[1];
                    v_env = stack_index(sqrt(x * x + y * y));
                    snap_axis = 2;
                    snap_val = d[2] > 0.0 ? -H : H;
                } else {
                    v_env = G.n_vol;
                }
            } else {  /* on or inside the envelope surface already */
                t_env = 0.0;
                v_env = stack_index(sqrt(p[0] * p[0] + p[1] * p[1]));
            }
        }
    }
    double t_w = cyl_exit(p, d, G.world[0]);
    if (d[2] < 0.0) t_w = fmin(t_w, (-G.world[1] - p[2]) / d[2]);
    else if (d[2] > 0.0) t_w = fmin(t_w, (G.world[1] - p[2]) / d[2]);
    if (t_w < 0.0) t_w = 0.0;
    hit_t h;
    if (t_env <= t_w) {
        h.t = t_env;
        h.next = v_env;
        h.snap_axis = snap_axis;
        h.snap_val = snap_val;
    } else {
        h.t = t_w;
        h.next = OR_OUTSIDE;
        h.snap_axis = -1;
        h.snap_val = 0.0;
    }
    return h;
}

static double shell_world_safety(const double p[3])
{
    double r = sqrt(p[0] * p[0] + p[1] * p[1]);
    double R = G.bounds[G.n_vol], H = G.env[0];
    double s = fmin(G.world[0] - r, G.world[1] - fabs(p[2]));
    double dr = r - R, dz = fabs(p[2]) - H, de;
    if (dz <= 0.0) de = dr;
    else if (dr <= 0.0) de = dz;
    else de = sqrt(dr * dr + dz * dz);
    s = fmin(s, de);
    return s > 0.0 ? s : 0.0;
}

static hit_t geom_query(int32_t vol, const double p[3], const double d[3])
{
    if (G.axis == OR_AXIS_Z_SLABS) return vol == 0 ? slab_world_dist(p, d) : slab_dist_out(vol, p, d);
    return vol == 0 ? shell_world_dist(p, d) : shell_dist_out(vol, p, d);
}

double or_dist_out(int32_t vol, const double p[3], const double d[3], int32_t* next)
{
    hit_t h = geom_query(vol, p, d);
    *next = h.next;
    return h.t;
}

double or_dist_out_face(int32_t vol, const double p[3], const double d[3], int32_t* next,
                        int32_t* snap_axis, double* snap_val)
{
    hit_t h = geom_query(vol, p, d);
    *next = h.next;
    *snap_axis = h.snap_axis;
    *snap_val = h.snap_val;
    return h.t;
}

double or_safety(int32_t vol, const double p[3])
{
    if (G.axis == OR_AXIS_Z_SLABS) return vol == 0 ? slab_world_safety(p) : slab_safety(vol, p);
    return vol == 0 ? shell_world_safety(p) : shell_safety(vol, p);
}
