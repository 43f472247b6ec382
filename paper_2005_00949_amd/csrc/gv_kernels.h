// gv_kernels.h -- HIP kernels of the stepping library (gfx950, wave64).
#pragma once
#include "gv_common.h"
#include "gv_compact.h"
#include "gv_geom.h"
#include "gv_physics.h"
#include "gv_step.h"
#include "../../include/gv.h"

namespace gv {

__constant__ DevGeom c_geom;
__constant__ DevPhys c_phys;

// ---------------------------------------------------------------------------
// Track state in HBM: structure of arrays, one set per particle-type queue
// (batched) or one mixed pool with a type column (plain).
// ---------------------------------------------------------------------------
template <class P> struct Soa {
    using R = typename P::R;
    double* x;
    double* y;
    double* z;
    R* ux;
    R* uy;
    R* uz;
    R* T;
    int* vol;
    uint32_t* ev;
    uint64_t* tid;
    uint32_t* nstep;
    int8_t* type;  // plain pool only
};

template <class P>
__device__ __forceinline__ void load_track(const Soa<P>& q, size_t i, int type, Track<P>& t)
{
    t.x[0] = q.x[i];
    t.x[1] = q.y[i];
    t.x[2] = q.z[i];
    t.u[0] = q.ux[i];
    t.u[1] = q.uy[i];
    t.u[2] = q.uz[i];
    t.T = q.T[i];
    t.vol = q.vol[i];
    t.ev = q.ev[i];
    t.tid = q.tid[i];
    t.nstep = q.nstep[i];
    t.type = type;
}

template <class P> __device__ __forceinline__ void store_track(const Soa<P>& q, size_t i, const Track<P>& t)
{
    q.x[i] = t.x[0];
    q.y[i] = t.x[1];
    q.z[i] = t.x[2];
    q.ux[i] = t.u[0];
    q.uy[i] = t.u[1];
    q.uz[i] = t.u[2];
    q.T[i] = t.T;
    q.vol[i] = t.vol;
    q.ev[i] = t.ev;
    q.tid[i] = t.tid;
    q.nstep[i] = t.nstep;
    if (q.type) q.type[i] = (int8_t)t.type;
}

template <class P, class R = typename P::R>
__device__ __forceinline__ void store_child(const Soa<P>& q, size_t i, const Track<P>& parent, const Child<R>& c)
{
    q.x[i] = parent.x[0];
    q.y[i] = parent.x[1];
    q.z[i] = parent.x[2];
    q.ux[i] = c.u[0];
    q.uy[i] = c.u[1];
    q.uz[i] = c.u[2];
    q.T[i] = c.T;
    q.vol[i] = parent.vol;
    q.ev[i] = parent.ev;
    q.tid[i] = c.tid;
    q.nstep[i] = 0;
    if (q.type) q.type[i] = (int8_t)c.type;
}

// global counters (gv_stats)
enum : int { kCSteps = 0, kCTracks = 3, kCProc = 6, kCEscaped = 14, kCKilled = 15, kCRej = 16, kCLoads = 17,
             kCStores = 18, kCRkSub = 19, kCRkRej = 20, kCRkSlots = 21, kCLaneSlots = 22, kCHelperSteps = 23,
             kCRkParked = 24, kNCount = 25 };

// per-lane sums of the adaptive-integration tallies over one launch
struct RkSum {
    uint32_t acc, rej, slots;
};

struct Sinks {
    double* edep;                 // [event][cell]
    double* ledger;               // [event][4]: escaped, killed, n_pair, n_annih
    unsigned long long* counters; // kNCount
    gv_trace_rec* trace;
    unsigned long long* trace_n;
    long long trace_cap;
    int fixed;                    // deposits and ledger held as unsigned 2^-40 MeV integers
    unsigned long long* esc_hist; // escaping particles [type][energy bin][cos bin]
};

// Escaping particles, binned like the single-slab observables of Sec. 4:
// 5 energy bins per decade from 1 keV (40) x 20 bins of the direction cosine
// with +z, per particle type; integer counts, so any arrival order gives the
// same histogram.
constexpr int kEhNE = 40, kEhNC = 20, kEhSize = 3 * kEhNE * kEhNC;
template <class R>
__device__ __forceinline__ void escape_count(const Sinks& S, int type, R T, R uz)
{
    const double Td = (double)T;
    int eb = Td > 0.0 ? (int)floor(log10(Td / 1.0e-3) * 5.0) : 0;
    eb = eb < 0 ? 0 : (eb > kEhNE - 1 ? kEhNE - 1 : eb);
    int cb = (int)floor(((double)uz + 1.0) * 0.5 * kEhNC);
    cb = cb < 0 ? 0 : (cb > kEhNC - 1 ? kEhNC - 1 : cb);
    atomicAdd(&S.esc_hist[(type * kEhNE + eb) * kEhNC + cb], 1ull);
}

// Fixed-point scoring: every deposit is rounded once to an integer number of
// 2^-40 MeV and summed with integer atomics, so the sums do not depend on the
// order in which the deposits arrive (basket size, occupancy, queue order).
// 100 GeV in one cell is 1.1e17 units, far below 2^64.
constexpr double kFixedScale = 0x1p40;
__device__ __forceinline__ unsigned long long to_fixed(double e)
{
    return e > 0.0 ? __double2ull_rn(e * kFixedScale) : 0ull;
}
__device__ __forceinline__ void sink_add(const Sinks& S, double* p, double e)
{
    if (S.fixed) atomicAdd(reinterpret_cast<unsigned long long*>(p), to_fixed(e));
    else unsafeAtomicAdd(p, e);
}

template <class P, class R = typename P::R>
__device__ inline void trace_step(const Sinks& S, const Track<P>& before_key, int vol_pre, const Track<P>& after,
                                  const StepOut<R>& o, uint32_t nstep_pre)
{
    const unsigned long long k = atomicAdd(S.trace_n, 1ull);
    if ((long long)k >= S.trace_cap) return;
    gv_trace_rec r;
    r.tid = before_key.tid;
    r.event = before_key.ev;
    r.nstep = nstep_pre;
    r.type = before_key.type;
    r.limiter = o.lim;
    r.vol_pre = vol_pre;
    r.vol_post = after.vol;
    r.process = o.proc;
    r.n_children = o.nchild;
    for (int a = 0; a < 3; ++a) {
        r.pos[a] = after.x[a];
        r.dir[a] = (double)after.u[a];
    }
    r.ekin = (double)after.T;
    r.edep = o.edep;
    r.step = o.s;
    S.trace[k] = r;
}

// ledger and rare counters of one step (escape, kill, conversions, annihilation)
template <class R>
__device__ __forceinline__ void account_rare(const Sinks& S, uint32_t ev, const StepOut<R>& o, unsigned* lds_cnt)
{
    if (o.status == kEscaped) {
        sink_add(S, &S.ledger[(size_t)ev * 4 + 0], o.e_escaped);
        atomicAdd(&lds_cnt[kCEscaped], 1u);
    } else if (o.status == kKilled) {
        sink_add(S, &S.ledger[(size_t)ev * 4 + 1], o.e_killed);
        atomicAdd(&lds_cnt[kCKilled], 1u);
    }
    if (o.n_pair) sink_add(S, &S.ledger[(size_t)ev * 4 + 2], 1.0);
    if (o.n_annih) {
        sink_add(S, &S.ledger[(size_t)ev * 4 + 3], 1.0);
        atomicAdd(&lds_cnt[kCProc + kAnnih], 1u);
    }
    if (o.proc >= 0) atomicAdd(&lds_cnt[kCProc + o.proc], 1u);
    if (o.rej_exhausted) atomicAdd(&lds_cnt[kCRej], (unsigned)o.rej_exhausted);
    if (o.nchild > 0) atomicAdd(&lds_cnt[kCTracks + o.ch[0].type], 1u);
    if (o.nchild > 1) atomicAdd(&lds_cnt[kCTracks + o.ch[1].type], 1u);
}

__device__ __forceinline__ void deposit(const Sinks& S, uint32_t ev, int vol, double e)
{
    if (e == 0.0) return;
    const int cell = vol_cell(c_geom, vol);
    if (cell >= 0) sink_add(S, &S.edep[(size_t)ev * c_geom.n_cells + cell], e);
    else sink_add(S, &S.ledger[(size_t)ev * 4 + 1], e);
}

// Per-workgroup deposit cache (batched driver): an open-addressed table in LDS
// keyed by event * n_cells + cell.  Deposits of a chunk's tracks land there
// with LDS atomics and go to HBM once per (event, cell) when the chunk's
// inner loop is done, instead of one HBM atomic per track and volume.  Keys
// that do not fit 32 bits, or that find no free slot within a few probes, go
// straight to HBM.
constexpr int kDepSlots = 512;
constexpr int kDepProbes = 8;
constexpr uint32_t kDepEmpty = 0xFFFFFFFFu;
struct DepCache {
    uint32_t key[kDepSlots];
    double val[kDepSlots];
};

template <int BLOCK> __device__ __forceinline__ void dep_clear(DepCache& dc)
{
    for (int i = threadIdx.x; i < kDepSlots; i += BLOCK) {
        dc.key[i] = kDepEmpty;
        dc.val[i] = 0.0;
    }
}

// A track's deposits over consecutive steps in one volume: a double sum, or
// in fixed mode the sum of each step's rounded integer (so that the grouping
// of steps into launches cannot change a single bit).
struct DepAcc {
    double e;
    unsigned long long x;
};
__device__ __forceinline__ void acc_add(const Sinks& S, DepAcc& a, double e)
{
    if (S.fixed) a.x += to_fixed(e);
    else a.e += e;
}
__device__ __forceinline__ void sink_add_acc(const Sinks& S, double* p, const DepAcc& a)
{
    if (S.fixed) atomicAdd(reinterpret_cast<unsigned long long*>(p), a.x);
    else unsafeAtomicAdd(p, a.e);
}

__device__ __forceinline__ void dep_add(DepCache& dc, const Sinks& S, uint32_t ev, int vol, const DepAcc& a)
{
    if (a.e == 0.0 && a.x == 0ull) return;
    const int cell = vol_cell(c_geom, vol);
    if (cell < 0) {
        sink_add_acc(S, &S.ledger[(size_t)ev * 4 + 1], a);
        return;
    }
    const uint64_t k64 = (uint64_t)ev * (uint64_t)c_geom.n_cells + (uint64_t)cell;
    if (k64 < kDepEmpty) {
        const uint32_t k = (uint32_t)k64;
        uint32_t h = (k * 2654435761u) >> 23;   // 9 bits: kDepSlots = 512
        for (int probe = 0; probe < kDepProbes; ++probe) {
            const uint32_t old = atomicCAS(&dc.key[h], kDepEmpty, k);
            if (old == kDepEmpty || old == k) {
                // explicit LDS address space: the add must be a ds atomic
                if (S.fixed) {
                    typedef __attribute__((address_space(3))) unsigned long long lds_u64;
                    __hip_atomic_fetch_add((lds_u64*)&dc.val[h], a.x, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                } else {
                    typedef __attribute__((address_space(3))) double lds_double;
                    __hip_atomic_fetch_add((lds_double*)&dc.val[h], a.e, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                return;
            }
            h = (h + 1) & (kDepSlots - 1);
        }
    }
    sink_add_acc(S, &S.edep[k64], a);
}

// write the cached sums to HBM and empty the cache (all threads call it)
template <int BLOCK> __device__ __forceinline__ void dep_flush(DepCache& dc, const Sinks& S)
{
    __syncthreads();
    for (int i = threadIdx.x; i < kDepSlots; i += BLOCK) {
        const uint32_t k = dc.key[i];
        if (k != kDepEmpty) {
            if (S.fixed)   // the slot holds an integer sum
                atomicAdd(reinterpret_cast<unsigned long long*>(&S.edep[k]),
                          (unsigned long long)__double_as_longlong(dc.val[i]));
            else
                unsafeAtomicAdd(&S.edep[k], dc.val[i]);
            dc.key[i] = kDepEmpty;
            dc.val[i] = 0.0;
        }
    }
    __syncthreads();
}

// Final-state tables, one thread per (model, node): node energy, the density
// of the transformed variable at kAlNX + 1 points, and Walker's alias table of
// the sub-interval trapezoid weights (Vose's construction: scaled weights
// below 1 and at or above 1 on two stacks filled in increasing index order; the
// top small column keeps its share and hands the rest to the top large one).
__global__ void k_build_alias(double* rec, int* alias, double* E, int* valid, double tc, double kc)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kAlNMod * kAlNE) return;
    const int m = idx / kAlNE, j = idx % kAlNE;
    const double En = kAlE0 * pow(10.0, (double)j / kAlNPD);
    if (m == 0) E[j] = En;
    double* r = rec + (size_t)idx * kAlRec;
    int* a = alias + (size_t)idx * kAlNX;
    const bool ok = alias_model_valid(m, En, tc, kc);
    valid[idx] = ok ? 1 : 0;
    if (!ok) {
        for (int k = 0; k < kAlRec; ++k) r[k] = 0.0;
        for (int k = 0; k < kAlNX; ++k) a[k] = k;
        return;
    }
    for (int k = 0; k <= kAlNX; ++k) r[k] = alias_pdf(m, En, (double)k / kAlNX, tc, kc);
    double sc[kAlNX];
    int small[kAlNX], large[kAlNX];
    int ns = 0, nl = 0;
    double sum = 0.0;
    for (int k = 0; k < kAlNX; ++k) {
        sc[k] = 0.5 * (r[k] + r[k + 1]);
        sum += sc[k];
    }
    for (int k = 0; k < kAlNX; ++k) {
        sc[k] = (double)kAlNX * sc[k] / sum;
        if (sc[k] < 1.0) small[ns++] = k;
        else large[nl++] = k;
    }
    double* q = r + kAlNX + 1;
    while (ns > 0 && nl > 0) {
        const int lo = small[--ns], hi = large[--nl];
        q[lo] = sc[lo];
        a[lo] = hi;
        sc[hi] = (sc[hi] + sc[lo]) - 1.0;
        if (sc[hi] < 1.0) small[ns++] = hi;
        else large[nl++] = hi;
    }
    while (nl > 0) {
        const int k = large[--nl];
        q[k] = 1.0;
        a[k] = k;
    }
    while (ns > 0) {
        const int k = small[--ns];
        q[k] = 1.0;
        a[k] = k;
    }
}

// fixed-point sums (bit patterns in a double array) to MeV, in place
__global__ void k_fixed_to_double(double* a, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const unsigned long long v = (unsigned long long)__double_as_longlong(a[i]);
    a[i] = (double)v * (1.0 / kFixedScale);
}

// ===========================================================================
// Table builder (FP64 on the device)
// ===========================================================================

// node energies and per-node cross sections / stopping powers
__global__ void k_build_xs(double* rec64, double* E64, float* E32)
{
    const int n = c_phys.n_nodes;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * c_phys.n_mats) return;
    const int m = idx / n, i = idx - m * n;
    const double E = c_phys.e_min * pow(10.0, (double)i / c_phys.bpd);
    if (m == 0) {
        E64[i] = E;
        E32[i] = (float)E;
    }
    const DevMat& M = c_phys.mat[m];
    double* g = rec64 + ((size_t)(m * 3 + kGamma) * n + i) * kCols;
    double* e = rec64 + ((size_t)(m * 3 + kElectron) * n + i) * kCols;
    double* p = rec64 + ((size_t)(m * 3 + kPositron) * n + i) * kCols;
    g[0] = M.n_el * xs_kn_per_electron(E);
    g[1] = xs_pair(M, E);
    g[2] = 0.0;
    g[3] = 0.0;
    e[0] = xs_moller(M, E, c_phys.t_cut);
    e[1] = xs_brems(M, E, c_phys.k_cut);
    e[2] = dedx_total(M, E, false, c_phys.t_cut, c_phys.k_cut);
    p[0] = xs_bhabha(M, E, c_phys.t_cut);
    p[1] = xs_brems(M, E, c_phys.k_cut);
    p[2] = dedx_total(M, E, true, c_phys.t_cut, c_phys.k_cut);
}

// 8-point Gauss-Legendre on [-1, 1]
__device__ __constant__ double c_glx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                                           -0.1834346424956498, 0.1834346424956498, 0.5255324099163290,
                                           0.7966664774136267, 0.9602898564975363};
__device__ __constant__ double c_glw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                                           0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                                           0.2223810344533745, 0.1012285362903763};

// range increment of each bin: int E/S(E) dlnE over [ln E_i, ln E_i+1]
__global__ void k_build_range_bins(const double* E64, double* dR)
{
    const int n = c_phys.n_nodes;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = 2 * (n - 1);
    if (idx >= per * c_phys.n_mats) return;
    const int m = idx / per, r = idx - m * per;
    const int pos = r / (n - 1), i = r - pos * (n - 1);
    const double la = log(E64[i]), lb = log(E64[i + 1]);
    const double h = 0.5 * (lb - la), c = 0.5 * (lb + la);
    double s = 0.0;
    for (int j = 0; j < 8; ++j) {
        const double E = exp(c + h * c_glx[j]);
        s += c_glw[j] * E / dedx_total(c_phys.mat[m], E, pos != 0, c_phys.t_cut, c_phys.k_cut);
    }
    dR[idx] = s * h;
}

// running sum from R(E_0) = E_0 / S(E_0), in node order
__global__ void k_build_range_scan(double* rec64, const double* E64, const double* dR)
{
    const int n = c_phys.n_nodes;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * c_phys.n_mats) return;
    const int m = idx / 2, pos = idx & 1;
    double* base = rec64 + (size_t)(m * 3 + (pos ? kPositron : kElectron)) * n * kCols;
    const double* d = dR + (size_t)(m * 2 + pos) * (n - 1);
    double R = E64[0] / dedx_total(c_phys.mat[m], E64[0], pos != 0, c_phys.t_cut, c_phys.k_cut);
    base[3] = R;
    for (int i = 0; i + 1 < n; ++i) {
        R = R + d[i];
        base[(i + 1) * kCols + 3] = R;
    }
}

__global__ void k_to_float(const double* a, float* b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// range at the tracking cut (per material, e-/e+), in both precisions
__global__ void k_range_at_cut(const double* rec64, const double* E64, const float* rec32, const float* E32,
                               double* out64, float* out32)
{
    const int idx = threadIdx.x;
    if (idx >= 2 * c_phys.n_mats) return;
    const int m = idx / 2, pos = idx & 1;
    const int type = pos ? kPositron : kElectron;
    TabView<double> t64{rec64, E64, c_phys.n_nodes};
    TabView<float> t32{rec32, E32, c_phys.n_nodes};
    {
        const double T = c_phys.t_track;
        const int i = find_bin(t64, T, c_phys.log10_emin, c_phys.bpd);
        const double w = (T - E64[i]) / (E64[i + 1] - E64[i]);
        out64[idx] = lerp_col(t64, tab_base(t64, m, type), i, 3, w);
    }
    {
        const float T = (float)c_phys.t_track;
        const int i = find_bin(t32, T, c_phys.log10_emin, c_phys.bpd);
        const float w = (T - E32[i]) / (E32[i + 1] - E32[i]);
        out32[idx] = lerp_col(t32, tab_base(t32, m, type), i, 3, w);
    }
}

// ===========================================================================
// Test kernels
// ===========================================================================

__global__ void k_dbg_philox(const uint32_t* in, uint32_t* out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t* w = in + 6 * i;
    const U4 r = philox(w[0], w[1], w[2], w[3], w[4], w[5]);
    for (int a = 0; a < 4; ++a) out[4 * i + a] = r.w[a];
}

__global__ void k_dbg_geom(const double* pos, const double* dir, const int* vol_in, double* dbnd, int* next,
                           int* vol_loc, double* saf, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    const double d[3] = {dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
    const int v = vol_in[i] == -2 ? locate(c_geom, p) : vol_in[i];
    vol_loc[i] = v;
    if (v == kOutside) {
        dbnd[i] = 0.0;
        next[i] = kOutside;
        saf[i] = 0.0;
        return;
    }
    const Hit h = distance_out(c_geom, v, p, d);
    dbnd[i] = h.t;
    next[i] = h.next;
    saf[i] = safety(c_geom, v, p);
}

struct DbgStepIO {
    int stop;              // 0: the whole step; else the stage it ends after (kThru*)
    double* s_eloss;       // continuous-loss length (stop > 0 only)
    const int* type;
    const double* pos_in;
    const double* dir_in;
    const double* ekin_in;
    const uint32_t* event;
    const uint64_t* tid;
    const uint32_t* nstep;
    double* pos;
    double* dir;
    double* ekin;
    double* edep;
    int* vol;
    int* vol_pre;
    int* lim;
    int* proc;
    int* status;
    int* nchild;
    int* ch_type;
    double* ch_ekin;
    double* ch_dir;
    uint64_t* ch_tid;
    double* step;
    double* s_phys;
    double* d_bnd;
    double* safety;
};

template <class P>
__global__ void k_dbg_step(DbgStepIO io, long long n, uint64_t seed, TabView<typename P::R> tv)
{
    using R = typename P::R;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Ctx<P> c{seed, &c_geom, &c_phys, tv};
    Track<P> t;
    for (int a = 0; a < 3; ++a) {
        t.x[a] = io.pos_in[3 * i + a];
        t.u[a] = (R)io.dir_in[3 * i + a];
    }
    t.T = (R)io.ekin_in[i];
    t.type = io.type[i];
    t.ev = io.event[i];
    t.tid = io.tid[i];
    t.nstep = io.nstep[i];
    t.vol = locate(c_geom, t.x);
    StepOut<R> o;
    if (io.stop == 0) {
        step_track<P, true>(c, t, o);
    } else {
        double s_eloss;
        step_track_through(c, t, o, io.stop, s_eloss);
        io.s_eloss[i] = s_eloss;
    }
    for (int a = 0; a < 3; ++a) {
        io.pos[3 * i + a] = t.x[a];
        io.dir[3 * i + a] = (double)t.u[a];
    }
    io.ekin[i] = (double)t.T;
    io.edep[i] = o.edep;
    io.vol[i] = t.vol;
    io.vol_pre[i] = o.vol_pre;
    io.lim[i] = o.lim;
    io.proc[i] = o.proc;
    io.status[i] = o.status;
    io.nchild[i] = o.nchild;
    for (int k = 0; k < 2; ++k) {
        const long long j = 2 * i + k;
        if (k < o.nchild) {
            io.ch_type[j] = o.ch[k].type;
            io.ch_ekin[j] = (double)o.ch[k].T;
            io.ch_tid[j] = o.ch[k].tid;
            for (int a = 0; a < 3; ++a) io.ch_dir[3 * j + a] = (double)o.ch[k].u[a];
        } else {
            io.ch_type[j] = -1;
            io.ch_ekin[j] = 0.0;
            io.ch_tid[j] = 0;
            for (int a = 0; a < 3; ++a) io.ch_dir[3 * j + a] = 0.0;
        }
    }
    io.step[i] = o.s;
    io.s_phys[i] = o.s_phys;
    io.d_bnd[i] = o.d_bnd;
    io.safety[i] = o.safety;
}

// stable three-way compaction of given output codes (same machinery as the
// batched step kernel): queue q receives input*4 + slot in expanded order
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_dbg_compact(const int8_t* codes, long long n, int* outq, long long stride,
                                                       uint32_t* counts, uint32_t* ticket, uint64_t* status,
                                                       uint32_t epoch)
{
    uint32_t* err = counts + 3;
    __shared__ ScanShared<BLOCK> sh;
    const long long n_chunks = (n + BLOCK - 1) / BLOCK;
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = (int)atomicAdd(ticket, 1u);
        __syncthreads();
        const long long chunk = sh.ticket;
        __syncthreads();
        if (chunk >= n_chunks) break;
        const long long i = chunk * BLOCK + threadIdx.x;
        int code[3] = {-1, -1, -1};
        if (i < n)
            for (int j = 0; j < 3; ++j) {
                const int c = codes[3 * i + j];
                // a code outside [-1, 2] is reported (bit 2) and dropped
                if (c < -1 || c > 2) atomicOr(err, 4u);
                code[j] = (c < -1 || c > 2) ? -1 : c;
            }
        int cnt[3] = {0, 0, 0};
        for (int j = 0; j < 3; ++j)
            if (code[j] >= 0) cnt[code[j]]++;
        int excl[3], tot[3];
        block_scan3<BLOCK>(cnt, excl, tot, sh);
        lookback3<BLOCK>(status, (uint32_t)chunk, epoch, tot, sh, err);
        int local[3] = {0, 0, 0};
        for (int j = 0; j < 3; ++j) {
            const int q = code[j];
            if (q < 0) continue;
            const long long pos = (long long)sh.prefix[q] + excl[q] + local[q]++;
            outq[q * stride + pos] = (int)(i * 4 + j);
        }
        if (chunk == n_chunks - 1 && threadIdx.x < 3) counts[threadIdx.x] = sh.prefix[threadIdx.x] + sh.total[threadIdx.x];
        __syncthreads();
    }
}

// ===========================================================================
// Batched driver: persistent kernel over per-type queues
// ===========================================================================

struct Ctrl {
    uint32_t count[2][4];   // queue sizes by buffer parity and type
    uint32_t ticket;        // next basket to claim
    uint32_t epoch;         // launch counter tagging look-back status words
    uint32_t overflow;      // bit 0: a queue ran out of capacity; bit 1: a look-back wait gave up
    uint32_t done;          // workgroups finished in this launch
    uint32_t halt;          // overflow as seen at the end of the previous launch
    uint32_t pad;
    uint64_t seed;          // run seed (device-resident so captured graphs are reusable)
    // integration queue, on a cache line of its own (every wavefront that
    // parks a move adds to it): moves parked in this launch per charged type,
    // long ones (above kRkFirstTurns, listed first in the integration order)
    // in the low 32 bits, short ones (listed after them) in the high 32 bits,
    // so that one atomic reserves a wavefront's job slots and order entries
    alignas(128) unsigned long long rk_split[2];
    uint32_t rk_grab;       // next parked move for the integration kernel
    uint32_t rk_ticket;     // next chunk of parked moves for the resume kernel
    uint32_t rk_done;       // resume workgroups finished in this launch
    uint32_t pad2;
};

// Work of an RK45 move before it is integrated (Sec. 3.6 sorts field
// propagation work by length over radius of curvature): its turning angle at
// the start, s / rcurv (rcurv = p / (kKB |B x u|), formed by the step's field
// rule), in units of the turning the integrator allows one attempt, i.e. the
// number of attempts it needs at least.  Parked moves of more than
// kRkFirstTurns are integrated before the others (the paper's pre-processed
// baskets), so the queue drains on single-attempt moves instead of waiting
// for a long integration that started last.
constexpr double kRkFirstTurns = 1.0;

__device__ __forceinline__ double rk_turns(double s, double rcurv)
{
    const double theta = 0.8 * sqrt(sqrt(c_phys.rk_tol / kDpK));
    return s / (theta * rcurv);
}

// A step parked at its RK45 move (the integration queue of the batched
// driver): the track before the move, what the rest of the step needs, and
// the integration's result once the integration kernel has run it.
template <class P> struct RkJob {
    using R = typename P::R;
    Track<P> t;
    Limits<R> L;
    Geo G;
    double s;          // length to integrate
    int lim;           // nominal limiter of the step
    int acc, rej;      // accepted and rejected attempts
    double s_done;     // length integrated
    double x[3], u[3]; // end point and unit direction
};

template <class P> struct BatchArgs {
    Soa<P> in[3];            // input queues of this launch, by type
    Soa<P> out[3];           // output queues, by type
    Ctrl* ctrl;
    uint64_t* status;
    uint32_t cap;
    int parity;              // input buffer parity of this launch
    int basket_chunks;       // chunks per claimed basket
    int inner_bulk;          // steps per track per launch while the population is large
    int inner_tail;          // ... and in the tail
    uint32_t tail_threshold; // population below which the tail setting applies
    Sinks S;
    TabView<typename P::R> tv;
    RkJob<P>* jobs[2];       // integration queue per charged type (RK45 with arrival order)
    uint32_t* order[2];      // integration order per type: long moves from the front, short ones from the back
    uint32_t jcap;           // capacity per type of both
    int regime;              // which populations this step kernel launch takes (kRunAlways, ...)
    int min_lanes;           // a wavefront with fewer tracks still stepping ends its inner steps (0: never)
};

// A launch of the integration queue's bulk graph holds two step kernels: the
// one that integrates inside the step takes a population below the tail
// threshold, the park-only one a population at or above it; the other returns
// before it touches anything.  (The first to run empties the input counts, so
// the second then sees no population and returns too.)
enum : int { kRunAlways = 0, kRunBelowTail = 1, kRunFromTail = 2 };

// Primary ingest (the event server of Sec. 2.1): validated, typed primaries
// with their track id (order within the event) are located in the geometry,
// renormalised and written into the queue slots the host assigned.
struct PrimDev {
    double x, y, z, ux, uy, uz, T;
    int vol, type;
    uint32_t ev;
    uint64_t tid;
};

template <class P>
__global__ void k_ingest(const PrimDev* prim, long long n, const uint32_t* slot, Soa<P> q0, Soa<P> q1, Soa<P> q2)
{
    using R = typename P::R;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const PrimDev p = prim[i];
    const Soa<P>& q = p.type == kGamma ? q0 : (p.type == kElectron ? q1 : q2);
    const size_t k = slot[i];
    const double pos[3] = {p.x, p.y, p.z};
    const double nn = sqrt(p.ux * p.ux + p.uy * p.uy + p.uz * p.uz);
    q.x[k] = p.x;
    q.y[k] = p.y;
    q.z[k] = p.z;
    q.ux[k] = (R)(p.ux / nn);
    q.uy[k] = (R)(p.uy / nn);
    q.uz[k] = (R)(p.uz / nn);
    q.T[k] = (R)p.T;
    q.vol[k] = locate(c_geom, pos);
    q.ev[k] = p.ev;
    q.tid[k] = p.tid;
    q.nstep[k] = 0;
    if (q.type) q.type[k] = (int8_t)p.type;
}

// end of a launch, run by the last of the `participants` workgroups to
// finish: the consumed input counts become the next launch's (empty) output,
// the basket ticket restarts and the look-back epoch advances.  Every
// participant has read the control block before it increments `done`, and
// the other workgroups left without touching it, so nothing reads these words
// afterwards.
__device__ __forceinline__ void finish_launch(Ctrl* ctrl, int parity, uint32_t participants)
{
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t d = atomicAdd(&ctrl->done, 1u);
        if (d == participants - 1) {
            __threadfence();
            ctrl->count[parity][0] = 0;
            ctrl->count[parity][1] = 0;
            ctrl->count[parity][2] = 0;
            ctrl->ticket = 0;
            ctrl->done = 0;
            ctrl->halt = ctrl->overflow;
            ctrl->epoch = ctrl->epoch + 1;
            __threadfence();
        }
    }
}

// write a secondary into the output queue of its type
template <class P, class R = typename P::R>
__device__ __forceinline__ void store_child_q(const BatchArgs<P>& A, int q, uint32_t pos, const Track<P>& parent,
                                              const Child<R>& ch)
{
    if (q == kGamma) store_child(A.out[kGamma], pos, parent, ch);
    else if (q == kElectron) store_child(A.out[kElectron], pos, parent, ch);
    else store_child(A.out[kPositron], pos, parent, ch);
}

template <int Q> __device__ __forceinline__ int is_q(int t) { return t == Q ? 1 : 0; }
__device__ __forceinline__ int pick3(int q, const int v[3]) { return q == 0 ? v[0] : (q == 1 ? v[1] : v[2]); }

// One chunk of BLOCK same-type tracks (TY known at compile time, so the
// photon and charged-particle step paths are specialised): step each track up
// to `inner` times in registers, stopping at its first secondary or its end;
// then compact survivor + secondaries into the output queues.
// Park one step at its RK45 move in the integration queue (lanes parking in
// the same iteration reserve their slots with one atomic per wavefront).
template <class P, int TY, class R = typename P::R>
__device__ __forceinline__ void park_job(const BatchArgs<P>& A, const Track<P>& t, const Limits<R>& L, const Geo& G,
                                         const Prop<R>& pr, double turns)
{
    static_assert(TY == kElectron || TY == kPositron, "only charged steps are parked");
    constexpr int q = TY - 1;
    const bool heavy = turns > kRkFirstTurns;
    const uint64_t pm = __ballot(1), hm = __ballot(heavy), lm = pm & ~hm;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)pm) - 1;
    unsigned long long old = 0ull;
    if (lane == leader)
        old = atomicAdd(&A.ctrl->rk_split[q],
                        (unsigned long long)__popcll(hm) | ((unsigned long long)__popcll(lm) << 32));
    const uint32_t hb = (uint32_t)__shfl((int)(uint32_t)old, leader, 64);
    const uint32_t lb = (uint32_t)__shfl((int)(uint32_t)(old >> 32), leader, 64);
    const uint64_t below = (1ull << lane) - 1ull;
    // job slot in arrival order; integration order: the long moves are listed
    // from the front of the order array, the short ones from its back.  Both
    // order indices are at most k, so every store is in bounds; the regions
    // never meet unless the launch overflows (and is then discarded).
    const uint32_t k = hb + lb + (uint32_t)__popcll(pm & below);
    if (k < A.jcap) {
        RkJob<P>& J = A.jobs[q][k];
        J.t = t;
        J.L = L;
        J.G = G;
        J.s = pr.s;
        J.lim = pr.lim;
        if (heavy) A.order[q][hb + (uint32_t)__popcll(hm & below)] = k;
        else A.order[q][A.jcap - 1u - (lb + (uint32_t)__popcll(lm & below))] = k;
    } else {
        atomicOr(&A.ctrl->overflow, 1u);
    }
}

// parked moves of one type and how many of them are long; none if the
// integration queue overflowed in this launch (the launch is then discarded)
struct RkCounts {
    uint32_t n, heavy;
};
__device__ __forceinline__ RkCounts rk_counts(const Ctrl* ctrl, int q, uint32_t jcap, bool halt)
{
    const unsigned long long v = ctrl->rk_split[q];
    const unsigned long long h = v & 0xffffffffull, l = v >> 32;
    if (halt || h + l > jcap) return RkCounts{0u, 0u};
    return RkCounts{(uint32_t)(h + l), (uint32_t)h};
}

// Lanes (of 64) below which a wavefront stops its inner steps in the bulk
// replays.  A lane whose track stops early (a secondary, the end of the track)
// would otherwise idle until the wavefront's last track has taken its inner
// steps; the few tracks still stepping are cheaper to queue and continue in
// the next launch.  The tail replays keep every track for its inner steps:
// there the wavefronts are sparse by nature and each launch is short.
constexpr int kBulkMinLanes = 32;

template <class P, int TY, int BLOCK, bool STABLE, bool INTEG, bool PARK = false, class R = typename P::R>
__device__ __forceinline__ void process_chunk(const BatchArgs<P>& A, const Ctx<P>& c, uint32_t chunk, uint32_t base,
                                              uint32_t n_t, uint32_t epoch, int inner, ScanShared<BLOCK>& sh,
                                              DepCache& dc, unsigned* cnt_lds, uint32_t& steps_here,
                                              uint32_t& loads, uint32_t& stores, uint32_t n_chunks, RkSum& rks,
                                              unsigned long long* lane_slots_lds, bool vac_ok, int min_lanes)
{
    const uint32_t slot = base + threadIdx.x;
    const bool active = slot < n_t;
    Track<P> t;
    StepOut<R> o;
    o.status = kDead;
    o.nchild = 0;
    o.ch[0].type = -1;
    o.ch[1].type = -1;
    int iters = 0;
    if (active) {
        load_track(A.in[TY], slot, TY, t);
        t.type = TY;
        loads += 1;
        DepAcc acc{0.0, 0ull};
        int acc_vol = t.vol;
        for (; iters < inner;) {
            // a wavefront with fewer than min_lanes tracks still stepping
            // leaves the loop: they are queued as they stand and continue
            // in the next launch, and the wavefront takes its next chunk
            if (iters > 0 && __popcll(__ballot(1)) < min_lanes) break;
            uint32_t ns = t.nstep;
            const bool acc_empty = (acc.e == 0.0) & (acc.x == 0ull);
            if (TY != kGamma && !INTEG && !PARK && vac_ok && __all((t.vol == 0) & acc_empty)) {
                // A wavefront whose charged tracks are all in volumes without
                // material (the loopers of a transport's low-population tail)
                // steps them in the vacuum form of the step, here in the world
                // volume and below in vacuum layers.  A step that leaves its
                // track alive in vacuum changes nothing but the track (no
                // deposit, process, secondary, counter or ledger entry; the
                // deposit accumulator stays empty, so its volume does not
                // matter), so such steps repeat with only the step count and
                // the trace; the step that ends otherwise takes the
                // bookkeeping below like any other.
                const WorldRun<P> run = world_run(c, t);
                for (;;) {
                    step_world(c, run, t, o);
                    steps_here += o.did_step;
                    iters += 1;
                    if (o.status != kAlive || t.vol != 0 || iters >= inner) break;
                    if (A.S.trace && o.did_step) trace_step(A.S, t, o.vol_pre, t, o, ns);
                    ns = t.nstep;
                }
            } else if (TY != kGamma && !INTEG && !PARK && vac_ok &&
                       __all((vol_material(c_geom, t.vol) < 0) & acc_empty)) {
                for (;;) {
                    step_track<P, false, true>(c, t, o);
                    steps_here += o.did_step;
                    iters += 1;
                    if (o.status != kAlive || iters >= inner) break;
                    if (t.vol != o.vol_pre && vol_material(c_geom, t.vol) >= 0) break;
                    if (A.S.trace && o.did_step) trace_step(A.S, t, o.vol_pre, t, o, ns);
                    ns = t.nstep;
                }
            } else if (PARK && TY != kGamma) {
                Limits<R> L;
                Geo G;
                Prop<R> pr;
                iters += 1;
                if (step_track_park(c, t, o, L, G, pr)) {
                    if constexpr (TY != kGamma) park_job<P, TY>(A, t, L, G, pr, rk_turns(pr.s, pr.rcurv));
                    atomicAdd(&cnt_lds[kCRkParked], 1u);
                    o.status = kParked;
                    break;
                }
                steps_here += o.did_step;
            } else {
                step_track<P, INTEG>(c, t, o);
                steps_here += o.did_step;
                iters += 1;
            }
            if (TY != kGamma) {
                rks.acc += (uint32_t)o.rk.acc;
                rks.rej += (uint32_t)o.rk.rej;
                rks.slots += (uint32_t)o.rk.iters;
            }
            if (o.vol_pre != acc_vol) {
                dep_add(dc, A.S, t.ev, acc_vol, acc);
                acc.e = 0.0;
                acc.x = 0ull;
                acc_vol = o.vol_pre;
            }
            acc_add(A.S, acc, o.edep);
            if (A.S.trace && o.did_step) trace_step(A.S, t, o.vol_pre, t, o, ns);
            account_rare(A.S, t.ev, o, cnt_lds);
            if (o.status == kEscaped) escape_count(A.S, TY, t.T, t.u[2]);
            if (o.status != kAlive || o.nchild > 0) break;
        }
        dep_add(dc, A.S, t.ev, acc_vol, acc);
    }
    {
        // lane use: the wavefront ran as many loop iterations as its busiest lane
        int m = iters;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
        if ((threadIdx.x & 63) == 0 && m) atomicAdd(lane_slots_lds, 64ull * (unsigned)m);
    }
    dep_flush<BLOCK>(dc, A.S);
    const int alive = (active && o.status == kAlive) ? 1 : 0;
    const int q1 = o.nchild > 0 ? o.ch[0].type : -1;
    const int q2 = o.nchild > 1 ? o.ch[1].type : -1;
    int cnt[3];
    cnt[0] = (TY == 0 ? alive : 0) + is_q<0>(q1) + is_q<0>(q2);
    cnt[1] = (TY == 1 ? alive : 0) + is_q<1>(q1) + is_q<1>(q2);
    cnt[2] = (TY == 2 ? alive : 0) + is_q<2>(q1) + is_q<2>(q2);
    int excl[3], tot[3];
    block_scan3<BLOCK>(cnt, excl, tot, sh);
    if (STABLE) lookback3<BLOCK>(A.status, chunk, epoch, tot, sh, &A.ctrl->overflow);
    else reserve3<BLOCK>(&A.ctrl->count[A.parity ^ 1][0], A.cap, tot, sh, &A.ctrl->overflow);
    // output positions in expanded order: survivor, child 0, child 1
    if (alive) {
        const uint32_t pos = (uint32_t)sh.prefix[TY] + (uint32_t)excl[TY];
        if (pos < A.cap) {
            store_track(A.out[TY], pos, t);
            stores += 1;
        } else {
            atomicOr(&A.ctrl->overflow, 1u);
        }
    }
    if (q1 >= 0) {
        const uint32_t pos = (uint32_t)sh.prefix[q1] + (uint32_t)pick3(q1, excl) + (uint32_t)((q1 == TY) & alive);
        if (pos < A.cap) {
            store_child_q(A, q1, pos, t, o.ch[0]);
            stores += 1;
        } else {
            atomicOr(&A.ctrl->overflow, 1u);
        }
    }
    if (q2 >= 0) {
        const uint32_t pos = (uint32_t)sh.prefix[q2] + (uint32_t)pick3(q2, excl) +
                             (uint32_t)((q2 == TY) & alive) + (uint32_t)(q2 == q1);
        if (pos < A.cap) {
            store_child_q(A, q2, pos, t, o.ch[1]);
            stores += 1;
        } else {
            atomicOr(&A.ctrl->overflow, 1u);
        }
    }
    if (STABLE && chunk == n_chunks - 1 && threadIdx.x < 3) {
        const uint32_t total = (uint32_t)(sh.prefix[threadIdx.x] + sh.total[threadIdx.x]);
        A.ctrl->count[A.parity ^ 1][threadIdx.x] = total < A.cap ? total : A.cap;
    }
    __syncthreads();
}

// INTEG: field integrators compiled in (field_method RK4 / RK45); the helix
// variant leaves them out and keeps its register budget.  PARK (without
// INTEG): the integration queue's step kernel, which parks every charged move
// in a field and so has the helix variant's register budget.  The mixed-precision
// helix variant is held to three wavefronts per SIMD (168 VGPRs): the step
// chain is latency-bound, and a third resident wavefront hides more of it.
template <class P, int BLOCK, bool STABLE, bool INTEG, bool PARK = false>
__global__ void __launch_bounds__(BLOCK, (!INTEG && sizeof(typename P::R) == sizeof(float)) ? 3 : 1)
k_step_batched(BatchArgs<P> A)
{
    __shared__ ScanShared<BLOCK> sh;
    __shared__ unsigned cnt_lds[kNCount];
    __shared__ unsigned long long rk_lds[4];
    __shared__ DepCache dc;

    const int pin = A.parity;
    // after an overflow (reported to the host, which reruns the window) the
    // remaining launches of the replay do nothing; counts never exceed cap.
    // `halt` changes only between launches, so every participant of this
    // launch sees the same counts and the same participant number.
    const bool ovf = A.ctrl->halt != 0;
    const uint32_t n0 = ovf ? 0u : min(A.ctrl->count[pin][0], A.cap);
    const uint32_t n1 = ovf ? 0u : min(A.ctrl->count[pin][1], A.cap);
    const uint32_t n2 = ovf ? 0u : min(A.ctrl->count[pin][2], A.cap);
    const uint32_t epoch = A.ctrl->epoch;
    const uint32_t c0 = (n0 + BLOCK - 1) / BLOCK, c1 = (n1 + BLOCK - 1) / BLOCK, c2 = (n2 + BLOCK - 1) / BLOCK;
    const uint32_t n_chunks = c0 + c1 + c2;
    const uint32_t population = n0 + n1 + n2;
    const int inner = population < A.tail_threshold ? A.inner_tail : A.inner_bulk;
    // the integration queue pays off while the population fills the GPU; in
    // the low-population tail each lane integrates its own track (inner_tail
    // steps per launch instead of one parked step per launch)
    if (A.regime == kRunBelowTail && population >= A.tail_threshold) return;
    if (A.regime == kRunFromTail && population < A.tail_threshold) return;
    // only as many workgroups as there are baskets take part; the rest leave
    // at once, so a small population costs a small launch
    const uint32_t baskets = (n_chunks + (uint32_t)A.basket_chunks - 1) / (uint32_t)A.basket_chunks;
    const uint32_t participants = baskets < gridDim.x ? (baskets > 0 ? baskets : 1u) : gridDim.x;
    if (blockIdx.x >= participants) return;
    for (int i = threadIdx.x; i < kNCount; i += BLOCK) cnt_lds[i] = 0;
    if (threadIdx.x < 4) rk_lds[threadIdx.x] = 0ull;
    dep_clear<BLOCK>(dc);
    Ctx<P> c{A.ctrl->seed, &c_geom, &c_phys, A.tv};
    const bool vac_ok = c_geom.field_map == kMapUniform;
    uint32_t steps_g = 0, steps_e = 0, steps_p = 0;
    uint32_t loads = 0, stores = 0;
    RkSum rks{0u, 0u, 0u};
    __syncthreads();

    for (;;) {
        if (threadIdx.x == 0) sh.ticket = (int)atomicAdd(&A.ctrl->ticket, 1u);
        __syncthreads();
        const uint32_t first = (uint32_t)sh.ticket * (uint32_t)A.basket_chunks;
        __syncthreads();
        if (first >= n_chunks) break;
        const uint32_t last = min(first + (uint32_t)A.basket_chunks, n_chunks);
        for (uint32_t chunk = first; chunk < last; ++chunk) {
            if (chunk < c0)
                process_chunk<P, kGamma, BLOCK, STABLE, INTEG, PARK>(A, c, chunk, chunk * BLOCK, n0, epoch, inner, sh, dc,
                                                                     cnt_lds, steps_g, loads, stores, n_chunks, rks,
                                                                     &rk_lds[3], vac_ok, A.min_lanes);
            else if (chunk < c0 + c1)
                process_chunk<P, kElectron, BLOCK, STABLE, INTEG, PARK>(A, c, chunk, (chunk - c0) * BLOCK, n1, epoch, inner,
                                                                        sh, dc, cnt_lds, steps_e, loads, stores, n_chunks,
                                                                        rks, &rk_lds[3], vac_ok, A.min_lanes);
            else
                process_chunk<P, kPositron, BLOCK, STABLE, INTEG, PARK>(A, c, chunk, (chunk - c0 - c1) * BLOCK, n2, epoch,
                                                                        inner, sh, dc, cnt_lds, steps_p, loads, stores,
                                                                        n_chunks, rks, &rk_lds[3], vac_ok, A.min_lanes);
        }
    }
    atomicAdd(&cnt_lds[kCSteps + kGamma], steps_g);
    atomicAdd(&cnt_lds[kCSteps + kElectron], steps_e);
    atomicAdd(&cnt_lds[kCSteps + kPositron], steps_p);
    atomicAdd(&cnt_lds[kCLoads], loads);
    atomicAdd(&cnt_lds[kCStores], stores);
    if (rks.slots) {
        atomicAdd(&rk_lds[0], (unsigned long long)rks.acc);
        atomicAdd(&rk_lds[1], (unsigned long long)rks.rej);
        atomicAdd(&rk_lds[2], (unsigned long long)rks.slots);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNCount; i += BLOCK)
        if (cnt_lds[i]) atomicAdd(&A.S.counters[i], (unsigned long long)cnt_lds[i]);
    if (threadIdx.x < 4 && rk_lds[threadIdx.x]) atomicAdd(&A.S.counters[kCRkSub + threadIdx.x], rk_lds[threadIdx.x]);
    finish_launch(A.ctrl, pin, participants);
}

// Low-population helper of the tail replays.  When every track left is a
// charged track in a volume without material (the loopers that end a
// transport), the serial chain of their vacuum steps runs here, in a kernel
// of few registers and without the step kernel's per-launch bookkeeping (a
// lone looper in c4: ~0.95 us per step here, ~1.3 us inside the step
// kernel), before the step kernel sees them.  A step is kept only if its track
// stays alive in vacuum, which changes nothing but the track; the first step
// that would end otherwise is left in the queue and taken by the step kernel
// from the same state with the same arithmetic, so histories, deposits and
// counters are the same as without the helper.  Any photon, track in
// material or population above one workgroup makes it return at once.
constexpr int kVacHelperBlock = 256;

// The helper's step forms: the looper forms of the helix in a uniform field
// (the world step and the vacuum step), the general step with the helix in a
// field map, or the general step with the field integrators; each is the
// function the step kernel runs for such a track.
enum : int { kHelperLooper = 0, kHelperHelix = 1, kHelperInteg = 2 };

// tracer: the lane that writes the step records (in the one-wavefront-per-
// looper form every lane steps the same track, and lane 0 records it)
template <class P, bool TRACE, int HM, class R = typename P::R>
__device__ __forceinline__ void helper_steps(const BatchArgs<P>& A, const Ctx<P>& c, const WorldRun<P>& run,
                                             Track<P>& t, int max_steps, int& calls, int& kept, RkSum& rks,
                                             bool tracer)
{
    for (; calls < max_steps;) {
        Track<P> tn = t;
        StepOut<R> o;
        const uint32_t ns = t.nstep;
        if constexpr (HM == kHelperLooper) {
            if (t.vol == 0) step_world(c, run, tn, o);
            else step_track<P, false, true>(c, tn, o);
        } else {
            step_track<P, HM == kHelperInteg>(c, tn, o);
        }
        calls += 1;
        if (o.status != kAlive) break;
        if (tn.vol != t.vol && vol_material(c_geom, tn.vol) >= 0) break;
        if (TRACE && tracer && o.did_step) trace_step(A.S, tn, o.vol_pre, tn, o, ns);
        if constexpr (HM == kHelperInteg) {
            rks.acc += (uint32_t)o.rk.acc;
            rks.rej += (uint32_t)o.rk.rej;
            rks.slots += (uint32_t)o.rk.iters;
        }
        t = tn;
        kept += 1;
    }
}

// integration work of the helper's kept steps (RK4 / RK45), into the run counters
__device__ __forceinline__ void helper_rk_counts(const Sinks& S, const RkSum& rks)
{
    if (rks.acc) atomicAdd(&S.counters[kCRkSub], (unsigned long long)rks.acc);
    if (rks.rej) atomicAdd(&S.counters[kCRkRej], (unsigned long long)rks.rej);
    if (rks.slots) atomicAdd(&S.counters[kCRkSlots], (unsigned long long)rks.slots);
}
template <class P, int HM>
__global__ void __launch_bounds__(kVacHelperBlock) k_vacuum_helper(BatchArgs<P> A, int max_steps)
{
    if (A.ctrl->halt != 0) return;
    const int pin = A.parity;
    const uint32_t n0 = min(A.ctrl->count[pin][kGamma], A.cap);
    const uint32_t n1 = min(A.ctrl->count[pin][kElectron], A.cap);
    const uint32_t n2 = min(A.ctrl->count[pin][kPositron], A.cap);
    if (n0 != 0 || n1 + n2 == 0 || n1 + n2 > (uint32_t)kVacHelperBlock) return;
    const uint32_t i = threadIdx.x;
    const bool active = i < n1 + n2;
    const int ty = i < n1 ? kElectron : kPositron;
    const uint32_t slot = i < n1 ? i : i - n1;
    Track<P> t;
    if (active) {
        load_track(A.in[ty], slot, ty, t);
        t.type = ty;
    }
    const bool vac = !active || (t.vol != kOutside && vol_material(c_geom, t.vol) < 0);
    if (!__syncthreads_and(vac)) return;
    Ctx<P> c{A.ctrl->seed, &c_geom, &c_phys, A.tv};
    int calls = 0, kept = 0;
    if (n1 + n2 <= (uint32_t)(kVacHelperBlock / 64)) {
        // Few loopers (the usual end of a transport): one wavefront per
        // looper, so that loopers step side by side on separate SIMDs
        // instead of taking turns in the divergent branches of one wavefront
        // (the arithmetic is the same).
        const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
        if (w >= n1 + n2) return;
        const int tw = w < n1 ? kElectron : kPositron;
        const uint32_t sw = w < n1 ? w : w - n1;
        Track<P> tu;
        load_track(A.in[tw], sw, tw, tu);
        const WorldRun<P> run = world_run(c, tu);
        RkSum rks{0u, 0u, 0u};
        const bool lane0 = (threadIdx.x & 63) == 0;
        if (A.S.trace) helper_steps<P, true, HM>(A, c, run, tu, max_steps, calls, kept, rks, lane0);
        else helper_steps<P, false, HM>(A, c, run, tu, max_steps, calls, kept, rks, lane0);
        if (lane0) {
            // (one looper per wavefront: its integration counts once, as one lane's)
            helper_rk_counts(A.S, rks);
            if (kept) {
                store_track(A.in[tw], sw, tu);
                atomicAdd(&A.S.counters[kCSteps + tw], (unsigned long long)kept);
                atomicAdd(&A.S.counters[kCHelperSteps], (unsigned long long)kept);
            }
            if (calls) atomicAdd(&A.S.counters[kCLaneSlots], 64ull * (unsigned)calls);
        }
        return;
    }
    if (active) {
        // vacuum keeps the kinetic energy: the run constants hold for every
        // kept step.  Without a trace the loop is its own copy, in which the
        // step records' other fields are dead.
        const WorldRun<P> run = world_run(c, t);
        RkSum rks{0u, 0u, 0u};
        if (A.S.trace) helper_steps<P, true, HM>(A, c, run, t, max_steps, calls, kept, rks, true);
        else helper_steps<P, false, HM>(A, c, run, t, max_steps, calls, kept, rks, true);
        helper_rk_counts(A.S, rks);
        if (kept) {
            store_track(A.in[ty], slot, t);
            atomicAdd(&A.S.counters[kCSteps + ty], (unsigned long long)kept);
            atomicAdd(&A.S.counters[kCHelperSteps], (unsigned long long)kept);
        }
    }
    // lane slots: the wavefront ran as many step calls as its busiest lane
    int m = calls;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&A.S.counters[kCLaneSlots], 64ull * (unsigned)m);
}

// ===========================================================================
// Integration queue of the batched driver (RK45 with arrival-order queues):
// the step kernel parks every charged step at its RK45 move; one kernel runs
// all parked integrations, each lane taking the next parked move as soon as
// its current one is done (lanes are refilled at every attempt, so a
// wavefront never waits for its slowest integration while the queue still
// holds work); a resume kernel finishes the parked steps and queues their
// survivors and secondaries.  Arithmetic is that of the fused step.
// ===========================================================================

constexpr int kRkBlock = 256;

template <class P>
__global__ void __launch_bounds__(kRkBlock) k_rk_integrate(BatchArgs<P> A)
{
    __shared__ unsigned long long slots_lds;
    if (threadIdx.x == 0) slots_lds = 0ull;
    __syncthreads();
    const bool halt = A.ctrl->halt != 0;
    const RkCounts re = rk_counts(A.ctrl, 0, A.jcap, halt), rp = rk_counts(A.ctrl, 1, A.jcap, halt);
    const uint32_t ne = re.n, np = rp.n;
    const uint32_t total = ne + np;
    // integration order: long moves of both types, then short ones
    const uint32_t he = re.heavy, hp = rp.heavy;
    const uint32_t le = ne - he;
    const double tol = c_phys.rk_tol;
    const int max_sub = c_phys.rk_max_sub;
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    Rk45State st;
    st.busy = false;
    RkJob<P>* job = nullptr;
    bool has = false, dry = total == 0;
    uint32_t iters = 0;
    for (;;) {
        // refill: lanes without an integration take the next parked moves
        const uint64_t need = __ballot(!has);
        if (need && !dry) {
            const int leader = __ffsll((unsigned long long)need) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&A.ctrl->rk_grab, (uint32_t)__popcll(need));
            base = (uint32_t)__shfl((int)base, leader, 64);
            if (base + (uint32_t)__popcll(need) >= total) dry = true;
            if (!has) {
                const uint32_t j = base + (uint32_t)__popcll(need & below);
                if (j < total) {
                    uint32_t ty, o;
                    if (j < he) ty = 0, o = j;
                    else if (j < he + hp) ty = 1, o = j - he;
                    else if (j < he + hp + le) ty = 0, o = A.jcap - 1u - (j - he - hp);
                    else ty = 1, o = A.jcap - 1u - (j - he - hp - le);
                    job = &A.jobs[ty][A.order[ty][o]];
                    const Track<P>& t = job->t;
                    const double pos[3] = {t.x[0], t.x[1], t.x[2]};
                    const double ud[3] = {(double)t.u[0], (double)t.u[1], (double)t.u[2]};
                    rk45_begin(c_geom, t.type, (double)t.T, job->s, tol, pos, ud, st);
                    has = true;
                }
            }
        }
        if (!__any(has)) {
            if (dry) break;
            continue;
        }
        iters += 1;   // an attempt round of the wavefront (some lane holds an integration)
        if (has && st.busy) rk45_attempt(c_geom, tol, max_sub, st);
        if (has && !st.busy) {
            // done: the end point and unit direction, as rk45_move leaves them
            if (job->s > 0.0) normalise(st.u);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                job->x[a] = st.x[a];
                job->u[a] = st.u[a];
            }
            job->s_done = st.done;
            job->acc = st.acc;
            job->rej = st.rej;
            has = false;
        }
    }
    // lane slots: 64 per attempt round of the wavefront (iters is uniform)
    if (lane == 0 && iters) atomicAdd(&slots_lds, 64ull * iters);
    __syncthreads();
    if (threadIdx.x == 0 && slots_lds) atomicAdd(&A.S.counters[kCRkSlots], slots_lds);
}

// Finish the parked steps of one chunk (TY known at compile time) and queue
// survivors and secondaries, as process_chunk does after its step.
template <class P, int TY, int BLOCK, class R = typename P::R>
__device__ __forceinline__ void resume_chunk(const BatchArgs<P>& A, const Ctx<P>& c, uint32_t base, uint32_t n_t,
                                             ScanShared<BLOCK>& sh, DepCache& dc, unsigned* cnt_lds,
                                             uint32_t& steps_here, uint32_t& stores, RkSum& rks)
{
    const uint32_t slot = base + threadIdx.x;
    const bool active = slot < n_t;
    Track<P> t;
    StepOut<R> o;
    o.status = kDead;
    o.nchild = 0;
    o.ch[0].type = -1;
    o.ch[1].type = -1;
    if (active) {
        const RkJob<P>& J = A.jobs[TY - 1][slot];
        t = J.t;
        t.type = TY;
        Prop<R> pr;
        pr.s = J.s;
        pr.lim = J.lim;
        const uint32_t ns = t.nstep;
        const Limits<R> L = J.L;
        const Geo G = J.G;
        step_track_resume(c, t, o, L, G, pr, J.x, J.u, J.s_done, J.acc, J.rej);
        steps_here += o.did_step;
        rks.acc += (uint32_t)o.rk.acc;
        rks.rej += (uint32_t)o.rk.rej;
        DepAcc acc{0.0, 0ull};
        acc_add(A.S, acc, o.edep);
        dep_add(dc, A.S, t.ev, o.vol_pre, acc);
        if (A.S.trace && o.did_step) trace_step(A.S, t, o.vol_pre, t, o, ns);
        account_rare(A.S, t.ev, o, cnt_lds);
        if (o.status == kEscaped) escape_count(A.S, TY, t.T, t.u[2]);
    }
    dep_flush<BLOCK>(dc, A.S);
    const int alive = (active && o.status == kAlive) ? 1 : 0;
    const int q1 = o.nchild > 0 ? o.ch[0].type : -1;
    const int q2 = o.nchild > 1 ? o.ch[1].type : -1;
    int cnt[3];
    cnt[0] = (TY == 0 ? alive : 0) + is_q<0>(q1) + is_q<0>(q2);
    cnt[1] = (TY == 1 ? alive : 0) + is_q<1>(q1) + is_q<1>(q2);
    cnt[2] = (TY == 2 ? alive : 0) + is_q<2>(q1) + is_q<2>(q2);
    int excl[3], tot[3];
    block_scan3<BLOCK>(cnt, excl, tot, sh);
    reserve3<BLOCK>(&A.ctrl->count[A.parity ^ 1][0], A.cap, tot, sh, &A.ctrl->overflow);
    if (alive) {
        const uint32_t pos = (uint32_t)sh.prefix[TY] + (uint32_t)excl[TY];
        if (pos < A.cap) {
            store_track(A.out[TY], pos, t);
            stores += 1;
        } else {
            atomicOr(&A.ctrl->overflow, 1u);
        }
    }
    if (q1 >= 0) {
        const uint32_t pos = (uint32_t)sh.prefix[q1] + (uint32_t)pick3(q1, excl) + (uint32_t)((q1 == TY) & alive);
        if (pos < A.cap) {
            store_child_q(A, q1, pos, t, o.ch[0]);
            stores += 1;
        } else {
            atomicOr(&A.ctrl->overflow, 1u);
        }
    }
    if (q2 >= 0) {
        const uint32_t pos = (uint32_t)sh.prefix[q2] + (uint32_t)pick3(q2, excl) +
                             (uint32_t)((q2 == TY) & alive) + (uint32_t)(q2 == q1);
        if (pos < A.cap) {
            store_child_q(A, q2, pos, t, o.ch[1]);
            stores += 1;
        } else {
            atomicOr(&A.ctrl->overflow, 1u);
        }
    }
    __syncthreads();
}

template <class P, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_rk_resume(BatchArgs<P> A)
{
    __shared__ ScanShared<BLOCK> sh;
    __shared__ unsigned cnt_lds[kNCount];
    __shared__ unsigned long long rk_lds[2];
    __shared__ DepCache dc;
    for (int i = threadIdx.x; i < kNCount; i += BLOCK) cnt_lds[i] = 0;
    if (threadIdx.x < 2) rk_lds[threadIdx.x] = 0ull;
    dep_clear<BLOCK>(dc);
    const bool halt = A.ctrl->halt != 0;
    const uint32_t ne = rk_counts(A.ctrl, 0, A.jcap, halt).n;
    const uint32_t np = rk_counts(A.ctrl, 1, A.jcap, halt).n;
    const uint32_t ce = (ne + BLOCK - 1) / BLOCK, cp = (np + BLOCK - 1) / BLOCK;
    const uint32_t n_chunks = ce + cp;
    const uint32_t participants = n_chunks < gridDim.x ? (n_chunks > 0 ? n_chunks : 1u) : gridDim.x;
    if (blockIdx.x >= participants) return;
    Ctx<P> c{A.ctrl->seed, &c_geom, &c_phys, A.tv};
    uint32_t steps_e = 0, steps_p = 0, stores = 0;
    RkSum rks{0u, 0u, 0u};
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = (int)atomicAdd(&A.ctrl->rk_ticket, 1u);
        __syncthreads();
        const uint32_t chunk = (uint32_t)sh.ticket;
        __syncthreads();
        if (chunk >= n_chunks) break;
        if (chunk < ce)
            resume_chunk<P, kElectron, BLOCK>(A, c, chunk * BLOCK, ne, sh, dc, cnt_lds, steps_e, stores, rks);
        else
            resume_chunk<P, kPositron, BLOCK>(A, c, (chunk - ce) * BLOCK, np, sh, dc, cnt_lds, steps_p, stores, rks);
    }
    atomicAdd(&cnt_lds[kCSteps + kElectron], steps_e);
    atomicAdd(&cnt_lds[kCSteps + kPositron], steps_p);
    atomicAdd(&cnt_lds[kCStores], stores);
    if (rks.acc | rks.rej) {
        atomicAdd(&rk_lds[0], (unsigned long long)rks.acc);
        atomicAdd(&rk_lds[1], (unsigned long long)rks.rej);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNCount; i += BLOCK)
        if (cnt_lds[i]) atomicAdd(&A.S.counters[i], (unsigned long long)cnt_lds[i]);
    if (threadIdx.x < 2 && rk_lds[threadIdx.x]) atomicAdd(&A.S.counters[kCRkSub + threadIdx.x], rk_lds[threadIdx.x]);
    // the last participant empties the integration queue for the next launch
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t d = atomicAdd(&A.ctrl->rk_done, 1u);
        if (d == participants - 1) {
            __threadfence();
            A.ctrl->rk_split[0] = 0ull;
            A.ctrl->rk_split[1] = 0ull;
            A.ctrl->rk_grab = 0;
            A.ctrl->rk_ticket = 0;
            A.ctrl->rk_done = 0;
            __threadfence();
        }
    }
}

// ===========================================================================
// Plain FP64 driver: one kernel per stage, intermediates in HBM
// ===========================================================================

struct PlainArgs {
    Soa<P64> pool;
    Limits<double>* L;
    Geo* G;
    Prop<double>* pr;
    StepOut<double>* o;
    uint8_t* active;
    uint8_t* stopped;
    uint32_t* nsteps_pre;
    int* vol_pre;
    long long n;
    uint64_t seed;
    Sinks S;
    TabView<double> tv;
};

__device__ __forceinline__ void plain_load(const PlainArgs& A, long long i, Track<P64>& t)
{
    load_track(A.pool, (size_t)i, (int)A.pool.type[i], t);
}

__global__ void k_plain_prestep_limit(PlainArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    Ctx<P64> c{A.seed, &c_geom, &c_phys, A.tv};
    Track<P64> t;
    plain_load(A, i, t);
    StepOut<double> o;
    init_out(t, o);
    A.nsteps_pre[i] = t.nstep;
    A.vol_pre[i] = t.vol;
    const bool go = stage_prestep(c, t, o);
    A.active[i] = go ? 1 : 0;
    if (go) {
        Limits<double> L;
        stage_limit(c, t, L);
        A.L[i] = L;
    } else {
        store_track(A.pool, (size_t)i, t);
    }
    A.o[i] = o;
}

__global__ void k_plain_geom(PlainArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n || !A.active[i]) return;
    Ctx<P64> c{A.seed, &c_geom, &c_phys, A.tv};
    Track<P64> t;
    plain_load(A, i, t);
    Geo G;
    stage_geom(c, t, G);
    A.G[i] = G;
}

__global__ void k_plain_move(PlainArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n || !A.active[i]) return;
    Ctx<P64> c{A.seed, &c_geom, &c_phys, A.tv};
    Track<P64> t;
    plain_load(A, i, t);
    const Limits<double> L = A.L[i];
    const Geo G = A.G[i];
    Prop<double> pr;
    stage_move<P64, true>(c, t, L, G, pr);
    A.pr[i] = pr;
    if (pr.rk.iters) {
        atomicAdd(&A.S.counters[kCRkSub], (unsigned long long)pr.rk.acc);
        atomicAdd(&A.S.counters[kCRkRej], (unsigned long long)pr.rk.rej);
        atomicAdd(&A.S.counters[kCRkSlots], (unsigned long long)pr.rk.iters);
    }
    store_track(A.pool, (size_t)i, t);
    StepOut<double>& o = A.o[i];
    o.did_step = 1;
    o.s = pr.s;
    o.lim = pr.lim;
    o.s_phys = L.s_phys >= big_len<double>() ? kInf : L.s_phys;
    o.d_bnd = G.d_bnd;
    o.safety = G.safety;
}

__global__ void k_plain_msc(PlainArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n || !A.active[i]) return;
    Ctx<P64> c{A.seed, &c_geom, &c_phys, A.tv};
    Track<P64> t;
    plain_load(A, i, t);
    t.nstep = A.nsteps_pre[i];
    stage_msc(c, t, A.L[i], A.pr[i]);
    store_track(A.pool, (size_t)i, t);
}

__global__ void k_plain_eloss(PlainArgs A)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n || !A.active[i]) return;
    Ctx<P64> c{A.seed, &c_geom, &c_phys, A.tv};
    Track<P64> t;
    plain_load(A, i, t);
    StepOut<double> o = A.o[i];
    A.stopped[i] = stage_eloss(c, t, A.L[i], A.pr[i], o) ? 1 : 0;
    A.o[i] = o;
    store_track(A.pool, (size_t)i, t);
}

__global__ void k_plain_finish(PlainArgs A)
{
    __shared__ unsigned cnt_lds[kNCount];
    for (int k = threadIdx.x; k < kNCount; k += blockDim.x) cnt_lds[k] = 0;
    __syncthreads();
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < A.n) {
        Ctx<P64> c{A.seed, &c_geom, &c_phys, A.tv};
        Track<P64> t;
        plain_load(A, i, t);
        StepOut<double> o = A.o[i];
        if (A.active[i]) {
            stage_finish(c, t, A.L[i], A.pr[i], A.stopped[i] != 0, o);
            store_track(A.pool, (size_t)i, t);
            atomicAdd(&cnt_lds[kCSteps + t.type], 1u);
            if (A.S.trace) {
                Track<P64> key = t;
                trace_step(A.S, key, A.vol_pre[i], t, o, A.nsteps_pre[i]);
            }
        }
        deposit(A.S, t.ev, A.vol_pre[i], o.edep);
        account_rare(A.S, t.ev, o, cnt_lds);
        if (o.status == kEscaped) escape_count(A.S, t.type, t.T, t.u[2]);
        A.o[i] = o;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kNCount; k += blockDim.x)
        if (cnt_lds[k]) atomicAdd(&A.S.counters[k], (unsigned long long)cnt_lds[k]);
}

// survivors and children into the next pool, stable (single queue)
template <int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_plain_compact(PlainArgs A, Soa<P64> next, Ctrl* ctrl, int parity,
                                                         uint64_t* status, uint32_t cap)
{
    __shared__ ScanShared<BLOCK> sh;
    const long long n_chunks = (A.n + BLOCK - 1) / BLOCK;
    const uint32_t participants = n_chunks < (long long)gridDim.x ? (uint32_t)(n_chunks > 0 ? n_chunks : 1)
                                                                  : gridDim.x;
    if (blockIdx.x >= participants) return;
    const uint32_t epoch = ctrl->epoch;
    uint32_t* count_out = &ctrl->count[parity ^ 1][0];
    uint32_t* overflow = &ctrl->overflow;
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) sh.ticket = (int)atomicAdd(&ctrl->ticket, 1u);
        __syncthreads();
        const long long chunk = sh.ticket;
        __syncthreads();
        if (chunk >= n_chunks) break;
        const long long i = chunk * BLOCK + threadIdx.x;
        int cnt[3] = {0, 0, 0};
        Track<P64> t;
        StepOut<double> o;
        o.status = kDead;
        o.nchild = 0;
        if (i < A.n) {
            plain_load(A, i, t);
            o = A.o[i];
            cnt[0] = (o.status == kAlive ? 1 : 0) + o.nchild;
        }
        int excl[3], tot[3];
        block_scan3<BLOCK>(cnt, excl, tot, sh);
        lookback3<BLOCK>(status, (uint32_t)chunk, epoch, tot, sh, overflow);
        uint32_t pos = (uint32_t)sh.prefix[0] + (uint32_t)excl[0];
        if (i < A.n) {
            if (o.status == kAlive) {
                if (pos < cap) store_track(next, pos, t);
                else atomicOr(overflow, 1u);
                ++pos;
            }
            for (int k = 0; k < o.nchild; ++k, ++pos) {
                if (pos < cap) store_child(next, pos, t, o.ch[k]);
                else atomicOr(overflow, 1u);
            }
        }
        if (chunk == n_chunks - 1 && threadIdx.x == 0) {
            const uint32_t total = (uint32_t)(sh.prefix[0] + sh.total[0]);
            *count_out = total < cap ? total : cap;
        }
        __syncthreads();
    }
    finish_launch(ctrl, parity, participants);
}

}  // namespace gv
