// gv_geom.h -- layered-detector geometry on the device (GeomQuery stage of
// Sec. 3.4 for a 1-D stack of volumes).
//
// Volume ids: 0 = vacuum world, 1..n = stack volumes, -1 = outside.  A slab
// stack is a set of boxes sharing |x| <= env0, |y| <= env1 and tiling z; a
// shell stack is a set of coaxial cylindrical shells tiling r within
// |z| <= env0.  Adjacent stack volumes differ by one in their id, so the
// navigator reduces to a ray-plane / ray-cylinder exit, the isotropic safety,
// and "next = v +- 1 or the world".  The world entry into the envelope is the
// overlap of the ray's parameter intervals (direction aware on surfaces).
//
// Every distance also names the plane face it ends on (axis, value) so that a
// straight boundary-limited step places the point exactly on the plane.
// Plane distances are kept as numerator / |direction component| and compared
// by cross-multiplication; only the chosen one is divided out, which gives the
// same quotient as dividing every candidate (FP64 division is a long
// instruction sequence on gfx950, and the world query needs up to nine).
// Ties between faces resolve in the order x-, x+, y-, y+, z-, z+ (shells:
// inner, outer, z-, z+) with strict comparisons.  All arithmetic is double:
// positions and boundaries stay FP64 under every precision policy, and is not
// contracted into fused multiply-adds, so that distances near a surface round
// exactly as written.
#pragma once
#include "gv_common.h"

#ifndef GV_MAX_VOLS
#define GV_MAX_VOLS 1024
#endif

namespace gv {

struct DevGeom {
    int axis;                     // 0 slabs along z, 1 shells along r
    int n_vol;
    int n_cells;
    int n_mats;
    double env[2];
    double world[4];
    double B[3];
    double Bmag;
    double Bhat[3];               // B / |B| (0 when there is no field)
    double kB;                    // kKB * |B|: curvature per unit momentum, 1/(cm MeV)
    int field_map;                // 0 uniform B, 1 finite solenoid along z (central field B[2])
    int pad_map;
    double sol_R2, sol_L, sol_c;  // solenoid: coil radius^2, half-length, B0 / f(0)
    double bounds[GV_MAX_VOLS + 1];
    int vmat[GV_MAX_VOLS];
    int vcell[GV_MAX_VOLS];
};

struct Hit {
    double t;
    int next;
    int snap_axis;                // -1: ends on a cylinder or leaves the world
    double snap_val;
};

__device__ __forceinline__ int vol_material(const DevGeom& g, int v) { return v >= 1 ? g.vmat[v - 1] : -1; }
__device__ __forceinline__ int vol_cell(const DevGeom& g, int v) { return v >= 1 ? g.vcell[v - 1] : -1; }

// stack volume containing coordinate c along the stack axis: bounds[v-1] <= c < bounds[v]
__device__ __forceinline__ int stack_of(const DevGeom& g, double c)
{
#pragma clang fp contract(off)
    if (c <= g.bounds[0]) return 1;
    if (c >= g.bounds[g.n_vol]) return g.n_vol;
    int lo = 0, hi = g.n_vol;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (g.bounds[mid] <= c) lo = mid;
        else hi = mid;
    }
    return lo + 1;
}

// stack_of with a guess: a point that has moved stays in its volume or enters
// a neighbour, so the guessed volumes are tried before the binary search (the
// answer is the same: bounds[v-1] <= c < bounds[v] holds for one v only, and
// the two ends of the stack fall through to stack_of's own rules)
__device__ __forceinline__ int stack_of_near(const DevGeom& g, double c, int v0, int v1)
{
    if (v0 >= 1 && v0 <= g.n_vol && g.bounds[v0 - 1] <= c && c < g.bounds[v0]) return v0;
    if (v1 >= 1 && v1 <= g.n_vol && g.bounds[v1 - 1] <= c && c < g.bounds[v1]) return v1;
    return stack_of(g, c);
}

// volume containing p; v0, v1: likely stack volumes (0 or -1: no guess)
__device__ inline int locate(const DevGeom& g, const double p[3], int v0 = 0, int v1 = 0)
{
#pragma clang fp contract(off)
    if (g.axis == 0) {
        const bool in_env = (fabs(p[0]) <= g.env[0]) & (fabs(p[1]) <= g.env[1]) & (p[2] >= g.bounds[0]) &
                            (p[2] <= g.bounds[g.n_vol]);
        if (in_env) return stack_of_near(g, p[2], v0, v1);
        const bool in_world = (fabs(p[0]) <= g.world[0]) & (fabs(p[1]) <= g.world[1]) & (p[2] >= g.world[2]) &
                              (p[2] <= g.world[3]);
        return in_world ? 0 : kOutside;
    }
    const double r = sqrt(p[0] * p[0] + p[1] * p[1]);
    if ((r <= g.bounds[g.n_vol]) & (fabs(p[2]) <= g.env[0])) return stack_of_near(g, r, v0, v1);
    return ((r <= g.world[0]) & (fabs(p[2]) <= g.world[1])) ? 0 : kOutside;
}

// ---- slabs ----------------------------------------------------------------

__device__ inline Hit slab_exit(const DevGeom& g, int v, const double p[3], const double d[3])
{
#pragma clang fp contract(off)
    const double lo[3] = {-g.env[0], -g.env[1], g.bounds[v - 1]};
    const double hi[3] = {g.env[0], g.env[1], g.bounds[v]};
    // nearest face so far at bn / bd.  The start (1 / 0) loses to any face:
    // n * 0 < 1 * den for den > 0, so the first axis with motion is taken.
    double bn = 1.0, bd = 0.0;
    double plane = hi[2];
    int face = 5;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool up = d[a] > 0.0;
        const double n = up ? hi[a] - p[a] : p[a] - lo[a];
        const double den = fabs(d[a]);
        const bool take = (d[a] != 0.0) & (n * bd < bn * den);
        bn = take ? n : bn;
        bd = take ? den : bd;
        face = take ? 2 * a + (up ? 1 : 0) : face;
        plane = take ? (up ? hi[a] : lo[a]) : plane;
    }
    const double best = bd > 0.0 ? bn / bd : kInf;
    Hit h;
    h.t = best > 0.0 ? best : 0.0;
    h.next = face == 4 ? (v == 1 ? 0 : v - 1) : face == 5 ? (v == g.n_vol ? 0 : v + 1) : 0;
    h.snap_axis = face >> 1;
    h.snap_val = plane;
    return h;
}

__device__ inline double slab_safety(const DevGeom& g, int v, const double p[3])
{
#pragma clang fp contract(off)
    double s = fmin(p[2] - g.bounds[v - 1], g.bounds[v] - p[2]);
    s = fmin(s, g.env[0] - fabs(p[0]));
    s = fmin(s, g.env[1] - fabs(p[1]));
    return s > 0.0 ? s : 0.0;
}

__device__ inline Hit slab_world(const DevGeom& g, const double p[3], const double d[3])
{
#pragma clang fp contract(off)
    const double lo[3] = {-g.env[0], -g.env[1], g.bounds[0]};
    const double hi[3] = {g.env[0], g.env[1], g.bounds[g.n_vol]};
    // entry (max of near-plane distances) and exit (min of far-plane
    // distances) of the ray's parameter interval inside the envelope box
    // The starts (-1 / 0 and 1 / 0) lose to any axis with motion (n * 0 >
    // -den and n * 0 < den), so the first such axis is taken for both.
    double nn = -1.0, nd = 0.0, fn = 1.0, fd = 0.0, plane = 0.0;
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
        plane = tn ? (up ? lo[a] : hi[a]) : plane;
        fn = tf ? n_far : fn;
        fd = tf ? den : fd;
    }
    const bool have = nd != 0.0;
    Hit h;
    h.t = kInf;
    h.next = 0;
    h.snap_axis = -1;
    h.snap_val = 0.0;
    if (have && !miss && nn * fd <= fn * nd && fn > 0.0) {
        if (nn > 0.0) {
            const double tn = nn / nd;
            h.t = tn;
            h.snap_axis = an;
            h.snap_val = plane;
            h.next = an == 2 ? (d[2] > 0.0 ? 1 : g.n_vol) : stack_of(g, p[2] + tn * d[2]);
        } else {
            h.t = 0.0;
            h.next = stack_of(g, p[2]);
        }
    }
    // leaving the world box: the nearest far plane
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
    double tw = wd > 0.0 ? wn / wd : kInf;
    tw = tw > 0.0 ? tw : 0.0;
    if (!(h.t <= tw)) {
        h.t = tw;
        h.next = kOutside;
        h.snap_axis = -1;
        h.snap_val = 0.0;
    }
    return h;
}

__device__ inline double slab_world_safety(const DevGeom& g, const double p[3])
{
#pragma clang fp contract(off)
    double s = fmin(g.world[0] - fabs(p[0]), g.world[1] - fabs(p[1]));
    s = fmin(s, fmin(p[2] - g.world[2], g.world[3] - p[2]));
    const double zc = 0.5 * (g.bounds[0] + g.bounds[g.n_vol]);
    const double zh = 0.5 * (g.bounds[g.n_vol] - g.bounds[0]);
    const double qx = fmax(fabs(p[0]) - g.env[0], 0.0);
    const double qy = fmax(fabs(p[1]) - g.env[1], 0.0);
    const double qz = fmax(fabs(p[2] - zc) - zh, 0.0);
    s = fmin(s, sqrt(qx * qx + qy * qy + qz * qz));
    return s > 0.0 ? s : 0.0;
}

// ---- shells ---------------------------------------------------------------

// leave the cylinder of radius R from inside (far root)
__device__ __forceinline__ double cyl_out(const double p[3], const double d[3], double R)
{
#pragma clang fp contract(off)
    const double a = d[0] * d[0] + d[1] * d[1];
    if (a == 0.0) return kInf;
    const double b = p[0] * d[0] + p[1] * d[1];
    const double c = p[0] * p[0] + p[1] * p[1] - R * R;
    const double q = sqrt(fmax(b * b - a * c, 0.0));
    return b <= 0.0 ? (q - b) / a : -c / (b + q);
}

// reach the cylinder of radius R from outside while moving inward (near root)
__device__ __forceinline__ double cyl_in(const double p[3], const double d[3], double R)
{
#pragma clang fp contract(off)
    const double a = d[0] * d[0] + d[1] * d[1];
    const double b = p[0] * d[0] + p[1] * d[1];
    if (a == 0.0 || b >= 0.0) return kInf;
    const double c = p[0] * p[0] + p[1] * p[1] - R * R;
    const double disc = b * b - a * c;
    if (disc < 0.0) return kInf;
    return c / (sqrt(disc) - b);
}

__device__ inline Hit shell_exit(const DevGeom& g, int v, const double p[3], const double d[3])
{
#pragma clang fp contract(off)
    const double rin = g.bounds[v - 1], rout = g.bounds[v], H = g.env[0];
    double best = kInf;
    int face = -1;
    if (rin > 0.0) {
        const double t = cyl_in(p, d, rin);
        if (t < best) { best = t; face = 0; }
    }
    {
        const double t = cyl_out(p, d, rout);
        if (t < best) { best = t; face = 1; }
    }
    if (d[2] < 0.0) {
        const double t = (-H - p[2]) / d[2];
        if (t < best) { best = t; face = 2; }
    } else if (d[2] > 0.0) {
        const double t = (H - p[2]) / d[2];
        if (t < best) { best = t; face = 3; }
    }
    Hit h;
    h.t = best > 0.0 ? best : 0.0;
    h.snap_axis = -1;
    h.snap_val = 0.0;
    if (face == 0) h.next = v - 1;
    else if (face == 1) h.next = v == g.n_vol ? 0 : v + 1;
    else {
        h.next = 0;
        h.snap_axis = 2;
        h.snap_val = face == 2 ? -H : H;
    }
    return h;
}

__device__ inline double shell_safety(const DevGeom& g, int v, const double p[3])
{
#pragma clang fp contract(off)
    const double r = sqrt(p[0] * p[0] + p[1] * p[1]);
    const double rin = g.bounds[v - 1];
    double s = g.bounds[v] - r;
    if (rin > 0.0) s = fmin(s, r - rin);
    s = fmin(s, g.env[0] - fabs(p[2]));
    return s > 0.0 ? s : 0.0;
}

__device__ inline Hit shell_world(const DevGeom& g, const double p[3], const double d[3])
{
#pragma clang fp contract(off)
    const double R = g.bounds[g.n_vol], H = g.env[0];
    Hit h;
    h.t = kInf;
    h.next = 0;
    h.snap_axis = -1;
    h.snap_val = 0.0;
    // parameter interval inside the infinite cylinder r <= R
    const double a = d[0] * d[0] + d[1] * d[1];
    const double b = p[0] * d[0] + p[1] * d[1];
    const double c = p[0] * p[0] + p[1] * p[1] - R * R;
    double c0 = -kInf, c1 = kInf;
    bool miss = false;
    if (a == 0.0) {
        miss = c > 0.0;
    } else {
        const double disc = b * b - a * c;
        if (disc < 0.0) {
            miss = true;
        } else {
            const double sq = sqrt(disc);
            const double q = b >= 0.0 ? -(b + sq) : sq - b;
            const double r1 = q / a, r2 = q != 0.0 ? c / q : 0.0;
            c0 = fmin(r1, r2);
            c1 = fmax(r1, r2);
        }
    }
    // parameter interval inside the slab |z| <= H
    double z0 = -kInf, z1 = kInf;
    if (d[2] == 0.0) {
        miss = miss || fabs(p[2]) > H;
    } else {
        const double ta = (-H - p[2]) / d[2], tb = (H - p[2]) / d[2];
        z0 = fmin(ta, tb);
        z1 = fmax(ta, tb);
    }
    if (!miss) {
        const double tn = fmax(c0, z0), tf = fmin(c1, z1);
        if (tn <= tf && tf > 0.0) {
            if (tn > 0.0) {
                h.t = tn;
                if (z0 > c0) {
                    const double x = p[0] + tn * d[0], y = p[1] + tn * d[1];
                    h.next = stack_of(g, sqrt(x * x + y * y));
                    h.snap_axis = 2;
                    h.snap_val = d[2] > 0.0 ? -H : H;
                } else {
                    h.next = g.n_vol;
                }
            } else {
                h.t = 0.0;
                h.next = stack_of(g, sqrt(p[0] * p[0] + p[1] * p[1]));
            }
        }
    }
    double tw = cyl_out(p, d, g.world[0]);
    if (d[2] < 0.0) tw = fmin(tw, (-g.world[1] - p[2]) / d[2]);
    else if (d[2] > 0.0) tw = fmin(tw, (g.world[1] - p[2]) / d[2]);
    tw = tw > 0.0 ? tw : 0.0;
    if (!(h.t <= tw)) {
        h.t = tw;
        h.next = kOutside;
        h.snap_axis = -1;
        h.snap_val = 0.0;
    }
    return h;
}

__device__ inline double shell_world_safety(const DevGeom& g, const double p[3])
{
#pragma clang fp contract(off)
    const double r = sqrt(p[0] * p[0] + p[1] * p[1]);
    const double R = g.bounds[g.n_vol], H = g.env[0];
    const double dr = r - R, dz = fabs(p[2]) - H;
    const double de = dz <= 0.0 ? dr : (dr <= 0.0 ? dz : sqrt(dr * dr + dz * dz));
    const double s = fmin(fmin(g.world[0] - r, g.world[1] - fabs(p[2])), de);
    return s > 0.0 ? s : 0.0;
}

// ---- dispatch -------------------------------------------------------------

__device__ inline Hit distance_out(const DevGeom& g, int v, const double p[3], const double d[3])
{
#pragma clang fp contract(off)
    if (g.axis == 0) return v == 0 ? slab_world(g, p, d) : slab_exit(g, v, p, d);
    return v == 0 ? shell_world(g, p, d) : shell_exit(g, v, p, d);
}

__device__ inline double safety(const DevGeom& g, int v, const double p[3])
{
#pragma clang fp contract(off)
    if (g.axis == 0) return v == 0 ? slab_world_safety(g, p) : slab_safety(g, v, p);
    return v == 0 ? shell_world_safety(g, p) : shell_safety(g, v, p);
}

}  // namespace gv
