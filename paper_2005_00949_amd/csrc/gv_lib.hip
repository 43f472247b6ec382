// gv_lib.hip -- host runtime and C ABI of the gfx950 stepping library.
//
// gv_init derives material constants, uploads geometry and cuts to constant
// memory and builds the physics tables on the device.  gv_transport ingests
// the primaries into per-type queues and runs one of two drivers:
//   PLAIN   : one kernel per simulation stage per step over a single mixed
//             FP64 pool, host loop with a read-back of the population per step;
//   BATCHED : a persistent kernel per step that claims baskets of same-type
//             tracks from the per-type queues, runs every stage in registers
//             (up to `inner_steps` steps per track), and writes survivors and
//             secondaries into the next queues with a one-pass stable
//             compaction; a graph of K such launches is replayed until the
//             queues are empty.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "gv_kernels.h"

using namespace gv;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(GV_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

double now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class T> struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count)
    {
        if (count <= n && p) return hipSuccess;
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// one set of SoA arrays: 3 types x 2 parities, `cap` slots each
template <class P> struct QueueMem {
    using R = typename P::R;
    void* block = nullptr;
    size_t cap = 0;
    bool with_type = false;
    Soa<P> q[2][3];
    hipError_t alloc(size_t c, int n_sets, bool type_col)
    {
        release();
        const size_t per = c * (3 * sizeof(double) + 4 * sizeof(R) + sizeof(int) + 2 * sizeof(uint32_t) +
                                sizeof(uint64_t) + (type_col ? 1 : 0)) + 16 * 256;
        hipError_t e = hipMalloc(&block, per * (size_t)n_sets);
        if (e != hipSuccess) {
            block = nullptr;
            return e;
        }
        cap = c;
        with_type = type_col;
        char* b = (char*)block;
        auto take = [&](size_t bytes) {
            char* r = b;
            b += (bytes + 255) & ~(size_t)255;
            return (void*)r;
        };
        for (int s = 0; s < n_sets; ++s) {
            Soa<P>& Q = q[s / 3][s % 3];
            Q.x = (double*)take(c * sizeof(double));
            Q.y = (double*)take(c * sizeof(double));
            Q.z = (double*)take(c * sizeof(double));
            Q.ux = (R*)take(c * sizeof(R));
            Q.uy = (R*)take(c * sizeof(R));
            Q.uz = (R*)take(c * sizeof(R));
            Q.T = (R*)take(c * sizeof(R));
            Q.vol = (int*)take(c * sizeof(int));
            Q.ev = (uint32_t*)take(c * sizeof(uint32_t));
            Q.tid = (uint64_t*)take(c * sizeof(uint64_t));
            Q.nstep = (uint32_t*)take(c * sizeof(uint32_t));
            Q.type = type_col ? (int8_t*)take(c) : nullptr;
        }
        return hipSuccess;
    }
    void release()
    {
        if (block) (void)hipFree(block);
        block = nullptr;
        cap = 0;
    }
};

struct GraphKey {
    int prec = -1, block = 0, chunks = 0, inner_bulk = 0, inner_tail = 0, K = 0;
    uint32_t tail = 0;
    size_t cap = 0;
    const void* qblock = nullptr;
    const void* edep = nullptr;
    const void* trace = nullptr;
    long long trace_cap = 0;
    int order = -1, fixed = -1, field = -1;
    int grid = 0, tail_grid = 0, tail_K = 0;
    bool operator==(const GraphKey& o) const
    {
        return prec == o.prec && block == o.block && chunks == o.chunks && inner_bulk == o.inner_bulk &&
               inner_tail == o.inner_tail && K == o.K && tail == o.tail && cap == o.cap && qblock == o.qblock &&
               edep == o.edep && trace == o.trace && trace_cap == o.trace_cap && order == o.order && fixed == o.fixed &&
               field == o.field && grid == o.grid && tail_grid == o.tail_grid && tail_K == o.tail_K;
    }
};

struct Lib {
    bool ready = false;
    bool busy = false;
    int device = -1;
    int n_cu = 256;
    hipStream_t own_stream = nullptr;
    gv_config cfg{};
    DevGeom geom{};
    DevPhys phys{};
    int n_cells = 0;
    // tables
    DBuf<double> rec64, E64;
    DBuf<double> al_rec64, al_E64;   // final-state tables (alias sampling)
    DBuf<float> al_rec32, al_E32;
    DBuf<int> al_alias, al_valid;
    DBuf<float> rec32, E32;
    // transport state
    QueueMem<P64> q64;
    QueueMem<PMix> qmix;
    QueueMem<P64> plain_pool;
    DBuf<Limits<double>> pl_L;
    DBuf<Geo> pl_G;
    DBuf<Prop<double>> pl_pr;
    DBuf<StepOut<double>> pl_o;
    DBuf<uint8_t> pl_active, pl_stopped;
    DBuf<uint32_t> pl_nstep;
    DBuf<int> pl_volpre;
    DBuf<Ctrl> ctrl;
    DBuf<uint64_t> status;
    DBuf<unsigned long long> counters;
    DBuf<double> edep, ledger;
    DBuf<gv_trace_rec> trace;
    DBuf<unsigned long long> esc_hist;
    DBuf<unsigned long long> trace_n;
    DBuf<unsigned long long> snap;   // counters, escape histogram, trace count before a window
    DBuf<char> rk_jobs;              // integration queue (two arrays of RkJob, one per charged type)
    uint32_t rk_jcap = 0;            // its capacity per type
    DBuf<PrimDev> prim;
    DBuf<uint32_t> prim_slot;
    Ctrl* h_ctrl = nullptr;  // pinned
    hipGraphExec_t gexec = nullptr;      // bulk: full grid, bulk inner steps
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec_tail = nullptr; // tail: small grid, tail inner steps
    hipGraph_t graph_tail = nullptr;
    GraphKey gkey;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    gv_stats_t stats{};
    std::vector<double> ledger_h;
    int64_t last_events = 0;
    double init_ms = 0.0;
    double plain_loads = 0.0, plain_stores = 0.0;
    int64_t tail_steps0 = 0;   // step counter when the current window entered its tail
    bool progress = std::getenv("GV_PROGRESS") != nullptr;   // print the population per graph replay
    // the staged batch (gv_stage): primaries grouped by event, resident on the device
    std::vector<PrimDev> hp;
    std::vector<size_t> ev_start;
    int64_t n_events = 0;
    int64_t n_prim = 0;
    double e_in = 0.0;
    int64_t tracks0[3] = {0, 0, 0};
    bool staged = false;
    size_t staged_b = 0, staged_e = 0;   // window whose queue slots are on the device
    bool staged_one_queue = false;       // ... laid out for one mixed pool (plain) or per type
    // autotuner choices, per (precision, queue order, log2 of the batch size);
    // cleared by gv_init
    std::map<std::tuple<int, int, int>, std::array<int, 3>> tune_cache;
    double autotune_ms = 0.0;
    bool tuned = false;
};

Lib L;

gv_config default_config()
{
    gv_config c{};
    c.driver = GV_DRIVER_BATCHED;
    c.precision = GV_PMIX;
    c.basket = 0;
    c.occupancy = 0;
    c.inner_steps = 0;
    c.graph_steps = 0;
    c.field_method = GV_FIELD_HELIX;
    c.edep_on_device = 0;
    c.max_steps_per_track = 1 << 20;
    c.capacity = 0;
    c.max_events_in_flight = 0;
    c.chord_tol_cm = 1.0e-3;
    c.push_cm = 1.0e-7;
    c.rk_frac = 0.05;
    c.hip_stream = nullptr;
    c.trace_cap = 0;
    c.queue_order = GV_ORDER_ARRIVAL;
    c.deposit_mode = GV_DEPOSIT_FLOAT;
    c.fs_alias = 0;
    c.reserved2 = 0;
    c.rk_tol = 0.0;
    c.rk_max_substeps = 0;
    c.reserved3 = 0;
    return c;
}

hipStream_t stream() { return L.cfg.hip_stream ? (hipStream_t)L.cfg.hip_stream : L.own_stream; }

void drop_graph()
{
    if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
    if (L.graph) (void)hipGraphDestroy(L.graph);
    if (L.gexec_tail) (void)hipGraphExecDestroy(L.gexec_tail);
    if (L.graph_tail) (void)hipGraphDestroy(L.graph_tail);
    L.gexec = nullptr;
    L.graph = nullptr;
    L.gexec_tail = nullptr;
    L.graph_tail = nullptr;
    L.gkey = GraphKey{};
}

void release_all()
{
    drop_graph();
    L.rec64.release();
    L.E64.release();
    L.rec32.release();
    L.E32.release();
    L.al_rec64.release();
    L.al_rec32.release();
    L.al_E64.release();
    L.al_E32.release();
    L.al_alias.release();
    L.al_valid.release();
    L.q64.release();
    L.qmix.release();
    L.plain_pool.release();
    L.pl_L.release();
    L.pl_G.release();
    L.pl_pr.release();
    L.pl_o.release();
    L.pl_active.release();
    L.pl_stopped.release();
    L.pl_nstep.release();
    L.pl_volpre.release();
    L.ctrl.release();
    L.status.release();
    L.counters.release();
    L.edep.release();
    L.ledger.release();
    L.trace.release();
    L.esc_hist.release();
    L.trace_n.release();
    L.snap.release();
    L.rk_jobs.release();
    L.rk_jcap = 0;
    L.prim.release();
    L.prim_slot.release();
    if (L.h_ctrl) (void)hipHostFree(L.h_ctrl);
    L.h_ctrl = nullptr;
    if (L.ev0) (void)hipEventDestroy(L.ev0);
    if (L.ev1) (void)hipEventDestroy(L.ev1);
    L.ev0 = L.ev1 = nullptr;
    if (L.own_stream) (void)hipStreamDestroy(L.own_stream);
    L.own_stream = nullptr;
    L.staged = false;
    L.hp.clear();
    L.ev_start.clear();
    L.tune_cache.clear();
    L.ready = false;
}

// ---- material constants (radiation length by Tsai, Bragg mean excitation) --
double tsai_inv_x0(int Z, double A)
{
    double lrad, lpr;
    if (Z == 1) {
        lrad = 5.31;
        lpr = 6.144;
    } else {
        const double z3 = std::cbrt((double)Z);
        lrad = std::log(184.15 / z3);
        lpr = std::log(1194.0 / (z3 * z3));
    }
    const double a2 = (kAlpha * Z) * (kAlpha * Z);
    const double fc = a2 * (1.0 / (1.0 + a2) + 0.20206 + a2 * (-0.0369 + a2 * (0.0083 - 0.002 * a2)));
    return 4.0 * kAlpha * kRe * kRe * kNA / A * ((double)Z * Z * (lrad - fc) + Z * lpr);
}

int derive_material(const gv_material& m, DevMat& out)
{
    if (!(m.density > 0.0) || m.n_elem < 1 || m.n_elem > GV_MAX_ELEM)
        return fail(GV_E_INVALID_ARG, "material density or element count invalid");
    double zoa = 0.0, ix0 = 0.0, lnI = 0.0, wsum = 0.0;
    for (int j = 0; j < m.n_elem; ++j) {
        if (m.Z[j] < 1 || !(m.A[j] > 0.0) || !(m.w[j] >= 0.0))
            return fail(GV_E_INVALID_ARG, "material element invalid");
        const double za = m.w[j] * m.Z[j] / m.A[j];
        zoa += za;
        wsum += m.w[j];
        ix0 += m.w[j] * tsai_inv_x0(m.Z[j], m.A[j]);
        if (m.I_eV <= 0.0) {
            if (!(m.I_elem_eV[j] > 0.0)) return fail(GV_E_INVALID_ARG, "elemental mean excitation energy missing");
            lnI += za * std::log(m.I_elem_eV[j]);
        }
    }
    if (std::fabs(wsum - 1.0) > 1e-6) return fail(GV_E_INVALID_ARG, "mass fractions do not sum to 1");
    out.n_el = m.density * kNA * zoa;
    out.X0 = m.X0_cm > 0.0 ? m.X0_cm : 1.0 / (ix0 * m.density);
    out.I = (m.I_eV > 0.0 ? m.I_eV : std::exp(lnI / zoa)) * 1.0e-6;
    out.hwp = 28.816 * std::sqrt(m.density * zoa) * 1.0e-6;
    return GV_OK;
}

int build_tables()
{
    const int n = L.phys.n_nodes, nm = L.phys.n_mats;
    const size_t nrec = (size_t)nm * 3 * n * kCols;
    HIPCHK(L.rec64.ensure(nrec));
    HIPCHK(L.rec32.ensure(nrec));
    HIPCHK(L.E64.ensure(n));
    HIPCHK(L.E32.ensure(n));
    DBuf<double> dR;
    HIPCHK(dR.ensure((size_t)nm * 2 * (n - 1)));
    DBuf<double> rt64;
    DBuf<float> rt32;
    HIPCHK(rt64.ensure(2 * nm));
    HIPCHK(rt32.ensure(2 * nm));
    hipStream_t s = stream();
    HIPCHK(hipMemsetAsync(L.rec64.p, 0, nrec * sizeof(double), s));
    k_build_xs<<<(n * nm + 127) / 128, 128, 0, s>>>(L.rec64.p, L.E64.p, L.E32.p);
    HIPCHK(hipGetLastError());
    k_build_range_bins<<<(2 * (n - 1) * nm + 127) / 128, 128, 0, s>>>(L.E64.p, dR.p);
    HIPCHK(hipGetLastError());
    k_build_range_scan<<<1, 64, 0, s>>>(L.rec64.p, L.E64.p, dR.p);
    HIPCHK(hipGetLastError());
    k_to_float<<<(unsigned)((nrec + 255) / 256), 256, 0, s>>>(L.rec64.p, L.rec32.p, nrec);
    HIPCHK(hipGetLastError());
    k_range_at_cut<<<1, 64, 0, s>>>(L.rec64.p, L.E64.p, L.rec32.p, L.E32.p, rt64.p, rt32.p);
    HIPCHK(hipGetLastError());
    std::vector<double> h(nrec), hr64(2 * nm);
    std::vector<float> hr32(2 * nm);
    HIPCHK(hipMemcpyAsync(h.data(), L.rec64.p, nrec * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hr64.data(), rt64.p, 2 * nm * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hr32.data(), rt32.p, 2 * nm * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    dR.release();
    rt64.release();
    rt32.release();
    for (size_t i = 0; i < nrec; ++i)
        if (!std::isfinite(h[i])) return fail(GV_E_TABLES, "non-finite table value");
    for (int m = 0; m < nm; ++m)
        for (int ty = 1; ty < 3; ++ty)
            for (int i = 0; i < n; ++i) {
                const double S = h[((size_t)(m * 3 + ty) * n + i) * kCols + 2];
                if (!(S > 0.0)) return fail(GV_E_TABLES, "non-positive stopping power in table");
            }
    for (int m = 0; m < nm; ++m)
        for (int p = 0; p < 2; ++p) {
            L.phys.r_track[m][p] = hr64[2 * m + p];
            L.phys.r_track_f[m][p] = hr32[2 * m + p];
        }
    // final-state tables for alias sampling (independent of material)
    const size_t arec = (size_t)kAlNMod * kAlNE * kAlRec;
    HIPCHK(L.al_rec64.ensure(arec));
    HIPCHK(L.al_rec32.ensure(arec));
    HIPCHK(L.al_E64.ensure(kAlNE));
    HIPCHK(L.al_E32.ensure(kAlNE));
    HIPCHK(L.al_alias.ensure((size_t)kAlNMod * kAlNE * kAlNX));
    HIPCHK(L.al_valid.ensure((size_t)kAlNMod * kAlNE));
    k_build_alias<<<(kAlNMod * kAlNE + 63) / 64, 64, 0, s>>>(L.al_rec64.p, L.al_alias.p, L.al_E64.p, L.al_valid.p,
                                                             L.phys.t_cut, L.phys.k_cut);
    HIPCHK(hipGetLastError());
    k_to_float<<<(unsigned)((arec + 255) / 256), 256, 0, s>>>(L.al_rec64.p, L.al_rec32.p, arec);
    k_to_float<<<1, 256, 0, s>>>(L.al_E64.p, L.al_E32.p, (size_t)kAlNE);
    HIPCHK(hipGetLastError());
    {
        std::vector<double> ha(arec);
        HIPCHK(hipMemcpyAsync(ha.data(), L.al_rec64.p, arec * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (double v : ha)
            if (!std::isfinite(v) || v < 0.0) return fail(GV_E_TABLES, "invalid final-state table value");
    }
    L.phys.al_rec64 = L.al_rec64.p;
    L.phys.al_rec32 = L.al_rec32.p;
    L.phys.al_E64 = L.al_E64.p;
    L.phys.al_E32 = L.al_E32.p;
    L.phys.al_alias = L.al_alias.p;
    L.phys.al_valid = L.al_valid.p;
    HIPCHK(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_phys), &L.phys, sizeof(DevPhys), 0, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return GV_OK;
}

template <class R> TabView<R> tab_view();
template <> TabView<double> tab_view<double>() { return TabView<double>{L.rec64.p, L.E64.p, L.phys.n_nodes}; }
template <> TabView<float> tab_view<float>() { return TabView<float>{L.rec32.p, L.E32.p, L.phys.n_nodes}; }

int validate_config(const gv_config& c)
{
    if (c.driver != GV_DRIVER_PLAIN && c.driver != GV_DRIVER_BATCHED) return fail(GV_E_INVALID_ARG, "driver");
    if (c.precision != GV_P64 && c.precision != GV_PMIX) return fail(GV_E_INVALID_ARG, "precision");
    if (c.driver == GV_DRIVER_PLAIN && c.precision != GV_P64)
        return fail(GV_E_INVALID_ARG, "the plain driver runs in FP64 only");
    if (c.basket != 0 && (c.basket < 64 || c.basket > 4096 || (c.basket & (c.basket - 1))))
        return fail(GV_E_INVALID_ARG, "basket must be 0 or a power of two in [64, 4096]");
    if (c.occupancy < 0 || c.occupancy > 32) return fail(GV_E_INVALID_ARG, "occupancy must be in [0, 32]");
    if (c.inner_steps < 0 || c.inner_steps > 1 << 16) return fail(GV_E_INVALID_ARG, "inner_steps");
    if (c.graph_steps < 0 || c.graph_steps > 4096 || (c.graph_steps & 1))
        return fail(GV_E_INVALID_ARG, "graph_steps must be 0 or an even number <= 4096");
    if (c.field_method != GV_FIELD_HELIX && c.field_method != GV_FIELD_RK4 && c.field_method != GV_FIELD_RK45)
        return fail(GV_E_INVALID_ARG, "field_method");
    if (!(c.rk_tol >= 0.0) || !(c.rk_tol < 1.0) || c.rk_max_substeps < 0 || c.rk_max_substeps > (1 << 20))
        return fail(GV_E_INVALID_ARG, "rk_tol must be in [0, 1), rk_max_substeps in [0, 2^20]");
    if (c.max_steps_per_track < 1 || c.max_steps_per_track >= (1 << 24))
        return fail(GV_E_INVALID_ARG, "max_steps_per_track must be in [1, 2^24)");
    if (c.capacity < 0 || c.capacity > (int64_t)1 << 31) return fail(GV_E_INVALID_ARG, "capacity");
    if (c.max_events_in_flight < 0) return fail(GV_E_INVALID_ARG, "max_events_in_flight");
    if (!(c.chord_tol_cm > 0.0) || !(c.push_cm >= 0.0) || !(c.rk_frac > 0.0))
        return fail(GV_E_INVALID_ARG, "field tolerances");
    if (c.trace_cap < 0) return fail(GV_E_INVALID_ARG, "trace_cap");
    if (c.queue_order != GV_ORDER_ARRIVAL && c.queue_order != GV_ORDER_STABLE)
        return fail(GV_E_INVALID_ARG, "queue_order");
    if (c.deposit_mode != GV_DEPOSIT_FLOAT && c.deposit_mode != GV_DEPOSIT_FIXED)
        return fail(GV_E_INVALID_ARG, "deposit_mode");
    if (c.fs_alias < 0 || c.fs_alias >= (1 << kAlNMod)) return fail(GV_E_INVALID_ARG, "fs_alias");
    if (c.reserved2 != 0 || c.reserved3 != 0) return fail(GV_E_INVALID_ARG, "reserved field must be 0");
    return GV_OK;
}

int apply_run_params()
{
    L.phys.field_method = L.cfg.field_method;
    L.phys.chord_tol = L.cfg.chord_tol_cm;
    L.phys.push = L.cfg.push_cm;
    L.phys.rk_frac = L.cfg.rk_frac;
    L.phys.rk_tol = L.cfg.rk_tol > 0.0 ? L.cfg.rk_tol : 1.0e-5;
    L.phys.rk_max_sub = L.cfg.rk_max_substeps > 0 ? L.cfg.rk_max_substeps : 16;
    L.phys.max_steps = L.cfg.max_steps_per_track;
    L.phys.fs_alias = L.cfg.fs_alias;
    HIPCHK(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_phys), &L.phys, sizeof(DevPhys), 0, hipMemcpyHostToDevice, stream()));
    HIPCHK(hipStreamSynchronize(stream()));
    return GV_OK;
}

// ---- transport helpers ----------------------------------------------------

struct Tuning {
    int block, chunks, occupancy, inner_bulk, inner_tail, K;
    uint32_t tail;       // population below which the tail graph runs
    int tail_grid;       // workgroups of a tail launch
    int tail_K;          // launches per tail graph replay
};

// default knob values, used for small batches and as the autotuner's start
constexpr int kDefBasket = 256, kDefOccupancy = 3, kDefInner = 4;
// batches below this many primaries are not autotuned
constexpr int64_t kTuneMinPrimaries = 4096;

// knob values: the caller's where set, else `choice` (basket, occupancy, inner)
Tuning pick_tuning(const std::array<int, 3>& choice)
{
    Tuning t;
    const int basket = L.cfg.basket ? L.cfg.basket : choice[0];
    t.block = basket >= 256 ? 256 : basket;
    t.chunks = basket / t.block;
    t.occupancy = L.cfg.occupancy ? L.cfg.occupancy : choice[1];
    t.inner_bulk = L.cfg.inner_steps ? L.cfg.inner_steps : choice[2];
    t.inner_tail = std::max(t.inner_bulk, 256);
    t.K = L.cfg.graph_steps ? L.cfg.graph_steps : 16;
    t.tail = (uint32_t)std::min<long long>((long long)L.n_cu * t.block * 2, 1u << 30);
    t.tail_grid = t.occupancy * L.n_cu;
    t.tail_K = 4 * t.K;
    return t;
}

int ensure_common(int64_t n_events)
{
    HIPCHK(L.ctrl.ensure(1));
    HIPCHK(L.counters.ensure(kNCount));
    const size_t ne = (size_t)n_events * (size_t)std::max(L.n_cells, 1);
    if (L.edep.n < ne) {
        drop_graph();
        HIPCHK(L.edep.ensure(ne));
    }
    if (L.ledger.n < (size_t)n_events * 4) {
        drop_graph();
        HIPCHK(L.ledger.ensure((size_t)n_events * 4));
    }
    if (L.cfg.trace_cap > 0 && L.trace.n < (size_t)L.cfg.trace_cap) {
        drop_graph();
        HIPCHK(L.trace.ensure((size_t)L.cfg.trace_cap));
    }
    HIPCHK(L.trace_n.ensure(1));
    if (!L.esc_hist.p) {
        drop_graph();
        HIPCHK(L.esc_hist.ensure(kEhSize));
    }
    HIPCHK(L.snap.ensure(kNCount + kEhSize + 1));
    if (!L.h_ctrl) HIPCHK(hipHostMalloc((void**)&L.h_ctrl, sizeof(Ctrl), hipHostMallocDefault));
    if (!L.ev0) HIPCHK(hipEventCreate(&L.ev0));
    if (!L.ev1) HIPCHK(hipEventCreate(&L.ev1));
    return GV_OK;
}

size_t capacity_for_driver(bool plain)
{
    if (L.cfg.capacity) return (size_t)L.cfg.capacity;
    return plain ? ((size_t)1 << 26) : ((size_t)1 << 25);
}

int ensure_status(size_t cap, int block)
{
    const size_t words = 3 * (3 * ((cap + block - 1) / block) + 3);
    if (L.status.n < words) {
        drop_graph();
        HIPCHK(L.status.ensure(words));
        HIPCHK(hipMemset(L.status.p, 0, words * sizeof(uint64_t)));
        // status words carry an epoch; restart the epoch at 1 over zeroed words
        Ctrl c{};
        c.epoch = 1;
        HIPCHK(hipMemcpy(L.ctrl.p, &c, sizeof(Ctrl), hipMemcpyHostToDevice));
    }
    return GV_OK;
}

Sinks make_sinks()
{
    Sinks S;
    S.edep = L.edep.p;
    S.ledger = L.ledger.p;
    S.counters = L.counters.p;
    S.trace = L.cfg.trace_cap > 0 ? L.trace.p : nullptr;
    S.trace_n = L.trace_n.p;
    S.trace_cap = L.cfg.trace_cap;
    S.fixed = L.cfg.deposit_mode == GV_DEPOSIT_FIXED ? 1 : 0;
    S.esc_hist = L.esc_hist.p;
    return S;
}

// Launches one event window may take before the driver reports a stuck loop.
// Every launch moves every live track by at least one step and a track ends
// within max_steps_per_track + 1 launches, but each secondary starts again at
// step 0, so the bound allows a tree of secondaries kMaxGenerations deep (no
// electromagnetic shower of these energies comes near it); it is also capped
// so that the look-back epoch cannot wrap inside a window.
constexpr uint32_t kEpochMask = (1u << 30) - 1u;
constexpr int64_t kMaxWindowLaunches = (int64_t)1 << 26;
constexpr int64_t kMaxGenerations = 256;
int64_t window_launch_bound()
{
    return std::min<int64_t>((L.cfg.max_steps_per_track + 2) * kMaxGenerations, kMaxWindowLaunches);
}

// Device accumulators that a window adds to besides its own deposit and
// ledger rows: kept before each window and put back when the window is
// rerun with fewer events in flight, so a retried window counts once.
int snapshot_sinks()
{
    hipStream_t s = stream();
    HIPCHK(hipMemcpyAsync(L.snap.p, L.counters.p, kNCount * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(L.snap.p + kNCount, L.esc_hist.p, kEhSize * sizeof(unsigned long long),
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(L.snap.p + kNCount + kEhSize, L.trace_n.p, sizeof(unsigned long long),
                          hipMemcpyDeviceToDevice, s));
    return GV_OK;
}

int restore_sinks()
{
    hipStream_t s = stream();
    HIPCHK(hipMemcpyAsync(L.counters.p, L.snap.p, kNCount * sizeof(unsigned long long), hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(L.esc_hist.p, L.snap.p + kNCount, kEhSize * sizeof(unsigned long long),
                          hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(L.trace_n.p, L.snap.p + kNCount + kEhSize, sizeof(unsigned long long),
                          hipMemcpyDeviceToDevice, s));
    return GV_OK;
}

// set the control block for a window: input counts at parity 0
int upload_ctrl(const uint32_t counts[3], uint64_t seed)
{
    hipStream_t s = stream();
    HIPCHK(hipMemcpyAsync(L.h_ctrl, L.ctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    Ctrl c = *L.h_ctrl;
    for (int t = 0; t < 3; ++t) {
        c.count[0][t] = counts[t];
        c.count[1][t] = 0;
    }
    c.count[0][3] = c.count[1][3] = 0;
    c.rk_split[0] = c.rk_split[1] = 0ull;
    c.rk_grab = c.rk_ticket = c.rk_done = 0;
    c.ticket = 0;
    c.overflow = 0;
    c.done = 0;
    c.halt = 0;
    c.seed = seed;
    if (c.epoch == 0 || c.epoch > kEpochMask - kMaxWindowLaunches) {
        // status words hold 30 bits of the epoch: restart it at 1 over zeroed
        // words before a window could carry it past the mask
        HIPCHK(hipMemsetAsync(L.status.p, 0, L.status.n * sizeof(uint64_t), s));
        c.epoch = 1;
    }
    *L.h_ctrl = c;
    HIPCHK(hipMemcpyAsync(L.ctrl.p, L.h_ctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return GV_OK;
}

int read_ctrl()
{
    HIPCHK(hipMemcpyAsync(L.h_ctrl, L.ctrl.p, sizeof(Ctrl), hipMemcpyDeviceToHost, stream()));
    HIPCHK(hipStreamSynchronize(stream()));
    return GV_OK;
}

template <class P> size_t batch_cap();
template <> size_t batch_cap<P64>() { return L.q64.cap; }
template <> size_t batch_cap<PMix>() { return L.qmix.cap; }

// ingest primaries [b, e) of the staged batch into parity-0 queues
template <class P>
int ingest(size_t b, size_t e, Soa<P> q[3], uint32_t counts[3], size_t cap, bool one_queue)
{
    const size_t n = e - b;
    counts[0] = counts[1] = counts[2] = 0;
    for (size_t i = b; i < e; ++i) counts[one_queue ? 0 : L.hp[i].type]++;
    for (int t = 0; t < 3; ++t)
        if (counts[t] > cap) return GV_E_CAPACITY;
    hipStream_t s = stream();
    if (!(L.staged_b == b && L.staged_e == e && L.staged_one_queue == one_queue && L.prim_slot.n >= n && L.staged)) {
        std::vector<uint32_t> slot(n);
        uint32_t c[3] = {0, 0, 0};
        for (size_t i = 0; i < n; ++i) slot[i] = c[one_queue ? 0 : L.hp[b + i].type]++;
        HIPCHK(L.prim_slot.ensure(std::max<size_t>(n, 1)));
        HIPCHK(hipMemcpyAsync(L.prim_slot.p, slot.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        L.staged_b = b;
        L.staged_e = e;
        L.staged_one_queue = one_queue;
    }
    if (one_queue)
        k_ingest<P><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L.prim.p + b, (long long)n, L.prim_slot.p, q[0], q[0], q[0]);
    else
        k_ingest<P><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L.prim.p + b, (long long)n, L.prim_slot.p, q[0], q[1], q[2]);
    HIPCHK(hipGetLastError());
    return GV_OK;
}

template <class P, int BLOCK, bool INTEG> void launch_step(const BatchArgs<P>& A, int grid, bool stable, hipStream_t s)
{
    if (stable) k_step_batched<P, BLOCK, true, INTEG><<<grid, BLOCK, 0, s>>>(A);
    else k_step_batched<P, BLOCK, false, INTEG><<<grid, BLOCK, 0, s>>>(A);
}

template <class P, bool INTEG>
void launch_step_block(int block, const BatchArgs<P>& A, int grid, bool stable, hipStream_t s)
{
    switch (block) {
    case 64: launch_step<P, 64, INTEG>(A, grid, stable, s); break;
    case 128: launch_step<P, 128, INTEG>(A, grid, stable, s); break;
    default: launch_step<P, 256, INTEG>(A, grid, stable, s); break;
    }
}

template <class P> void launch_step_dispatch(int block, const BatchArgs<P>& A, int grid, bool stable, hipStream_t s)
{
    if (L.cfg.field_method != GV_FIELD_HELIX) launch_step_block<P, true>(block, A, grid, stable, s);
    else launch_step_block<P, false>(block, A, grid, stable, s);
}

// RK45 with arrival-order queues runs its integrations through the
// integration queue: the step kernel parks charged steps at their move, the
// integration kernel runs them with lane refill, the resume kernel finishes them.
bool rk_queue_mode()
{
    return L.cfg.driver == GV_DRIVER_BATCHED && L.cfg.field_method == GV_FIELD_RK45 &&
           L.cfg.queue_order == GV_ORDER_ARRIVAL;
}

// One launch of the integration queue's bulk graph: the step kernel that
// integrates inside the step (taking populations below the tail threshold),
// the park-only step kernel (taking the others), the integration kernel and
// the resume kernel.  The tail graph integrates inside the step only.
template <class P, int BLOCK> void launch_rk_queue_block(const BatchArgs<P>& A, int grid, hipStream_t s, bool tail)
{
    if (tail) {
        k_step_batched<P, BLOCK, false, true><<<grid, BLOCK, 0, s>>>(A);
        return;
    }
    BatchArgs<P> a = A;
    a.regime = kRunBelowTail;
    k_step_batched<P, BLOCK, false, true><<<grid, BLOCK, 0, s>>>(a);
    a.regime = kRunFromTail;
    k_step_batched<P, BLOCK, false, false, true><<<grid, BLOCK, 0, s>>>(a);
    k_rk_integrate<P><<<L.n_cu * 4, kRkBlock, 0, s>>>(A);
    k_rk_resume<P, BLOCK><<<grid, BLOCK, 0, s>>>(A);
}

template <class P> void launch_rk_queue_step(int block, const BatchArgs<P>& A, int grid, hipStream_t s, bool tail)
{
    switch (block) {
    case 64: launch_rk_queue_block<P, 64>(A, grid, s, tail); break;
    case 128: launch_rk_queue_block<P, 128>(A, grid, s, tail); break;
    default: launch_rk_queue_block<P, 256>(A, grid, s, tail); break;
    }
}

// per-type capacity of the integration queue: the charged tracks one launch
// can park (a launch that parks more overflows and the window reruns with
// fewer events, as for the track queues)
constexpr size_t kRkMaxJobs = (size_t)1 << 23;
template <class P> int ensure_rk_jobs(size_t cap)
{
    const uint32_t jcap = (uint32_t)std::min(cap, kRkMaxJobs);
    const size_t bytes = 2 * (size_t)jcap * (sizeof(RkJob<P>) + sizeof(uint32_t));
    if (L.rk_jobs.n < bytes || L.rk_jcap != jcap) {
        drop_graph();
        HIPCHK(L.rk_jobs.ensure(bytes));
        L.rk_jcap = jcap;
    }
    return GV_OK;
}

template <class P> QueueMem<P>& batch_queues();
template <> QueueMem<P64>& batch_queues<P64>() { return L.q64; }
template <> QueueMem<PMix>& batch_queues<PMix>() { return L.qmix; }

// capture K launches alternating parity (K even: a replay ends where it began);
// tail: the tail graph, with the vacuum helper before each step launch and,
// for RK45 with arrival order, integration inside the step only
// vacuum steps per track and helper launch in the tail replays
constexpr int kVacHelperSteps = 4096;

template <class P>
int capture(const Tuning& tu, int grid, int K, int inner_bulk, int inner_tail, bool tail, hipGraph_t* g,
            hipGraphExec_t* ge)
{
    QueueMem<P>& Q = batch_queues<P>();
    hipStream_t s = stream();
    BatchArgs<P> A[2];
    for (int par = 0; par < 2; ++par) {
        for (int t = 0; t < 3; ++t) {
            A[par].in[t] = Q.q[par][t];
            A[par].out[t] = Q.q[par ^ 1][t];
        }
        A[par].ctrl = L.ctrl.p;
        A[par].status = L.status.p;
        A[par].cap = (uint32_t)Q.cap;
        A[par].parity = par;
        A[par].basket_chunks = tu.chunks;
        A[par].inner_bulk = inner_bulk;
        A[par].inner_tail = inner_tail;
        A[par].tail_threshold = tu.tail;
        A[par].S = make_sinks();
        A[par].tv = tab_view<typename P::R>();
        RkJob<P>* jobs = (RkJob<P>*)L.rk_jobs.p;
        A[par].jobs[0] = jobs;
        A[par].jobs[1] = jobs ? jobs + L.rk_jcap : nullptr;
        uint32_t* order = jobs ? (uint32_t*)(jobs + 2 * (size_t)L.rk_jcap) : nullptr;
        A[par].order[0] = order;
        A[par].order[1] = order ? order + L.rk_jcap : nullptr;
        A[par].jcap = jobs ? L.rk_jcap : 0u;
        A[par].regime = kRunAlways;
        A[par].min_lanes = tail ? 0 : kBulkMinLanes;
    }
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const bool stable = L.cfg.queue_order == GV_ORDER_STABLE;
    const bool rkq = rk_queue_mode();
    for (int k = 0; k < K; ++k) {
        if (tail) {
            if (L.cfg.field_method != GV_FIELD_HELIX)
                k_vacuum_helper<P, kHelperInteg><<<1, kVacHelperBlock, 0, s>>>(A[k & 1], kVacHelperSteps);
            else if (L.geom.field_map == kMapUniform)
                k_vacuum_helper<P, kHelperLooper><<<1, kVacHelperBlock, 0, s>>>(A[k & 1], kVacHelperSteps);
            else
                k_vacuum_helper<P, kHelperHelix><<<1, kVacHelperBlock, 0, s>>>(A[k & 1], kVacHelperSteps);
        }
        if (rkq) launch_rk_queue_step<P>(tu.block, A[k & 1], grid, s, tail);
        else launch_step_dispatch<P>(tu.block, A[k & 1], grid, stable, s);
    }
    hipError_t ce = hipStreamEndCapture(s, g);
    if (ce != hipSuccess) return fail(GV_E_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
    HIPCHK(hipGraphInstantiate(ge, *g, nullptr, nullptr, 0));
    return GV_OK;
}

template <class P> int build_graph(const Tuning& tu, const GraphKey& key)
{
    drop_graph();
    int rc = capture<P>(tu, tu.occupancy * L.n_cu, tu.K, tu.inner_bulk, tu.inner_tail, false, &L.graph, &L.gexec);
    if (rc) return rc;
    // the vacuum helper steps the last loopers of the tail replays (with the
    // looper forms of the helix in a uniform field, else the general step)
    rc = capture<P>(tu, tu.tail_grid, tu.tail_K, tu.inner_tail, tu.inner_tail, true, &L.graph_tail, &L.gexec_tail);
    if (rc) return rc;
    L.gkey = key;
    return GV_OK;
}

// batched transport of one event window; returns GV_E_CAPACITY on overflow
template <class P> int run_batched_window(size_t b, size_t e, uint64_t seed, const Tuning& tu)
{
    QueueMem<P>& Q = batch_queues<P>();
    L.tail_steps0 = 0;
    uint32_t counts[3];
    int rc = ingest<P>(b, e, Q.q[0], counts, Q.cap, false);
    if (rc) return rc;
    rc = upload_ctrl(counts, seed);
    if (rc) return rc;
    GraphKey key;
    key.prec = P::kMixed ? GV_PMIX : GV_P64;
    key.block = tu.block;
    key.chunks = tu.chunks;
    key.inner_bulk = tu.inner_bulk;
    key.inner_tail = tu.inner_tail;
    key.K = tu.K;
    key.tail = tu.tail;
    key.cap = Q.cap;
    key.qblock = Q.block;
    key.edep = L.edep.p;
    key.trace = L.cfg.trace_cap > 0 ? L.trace.p : nullptr;
    key.trace_cap = L.cfg.trace_cap;
    key.order = L.cfg.queue_order;
    key.fixed = L.cfg.deposit_mode;
    key.field = L.cfg.field_method;
    key.grid = tu.occupancy * L.n_cu;
    key.tail_grid = tu.tail_grid;
    key.tail_K = tu.tail_K;
    if (!L.gexec || !(L.gkey == key)) {
        rc = build_graph<P>(tu, key);
        if (rc) return rc;
    }
    hipStream_t s = stream();
    uint32_t population = counts[0] + counts[1] + counts[2];
    uint32_t peak = population;
    bool grew = true;   // the last replay raised the population (or none has run yet)
    int64_t launches = 0;
    const int64_t bound = window_launch_bound();
    bool in_tail = false;
    for (;;) {
        // replay the tail graph (more launches per replay, the vacuum helper)
        // once the population is below the tail threshold and past its peak:
        // after a peak at or above the threshold, or, in a window whose
        // population never reaches it, as soon as a replay no longer raises it
        const bool tail = population < tu.tail && (peak >= tu.tail || !grew);
        if (tail && !in_tail) {
            // the steps taken so far, so that the tail's own steps can be told apart
            unsigned long long c3[3];
            HIPCHK(hipMemcpyAsync(c3, L.counters.p + kCSteps, sizeof(c3), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            L.tail_steps0 += (int64_t)(c3[0] + c3[1] + c3[2]);
            in_tail = true;
        }
        HIPCHK(hipEventRecord(L.ev0, s));
        HIPCHK(hipGraphLaunch(tail ? L.gexec_tail : L.gexec, s));
        HIPCHK(hipEventRecord(L.ev1, s));
        rc = read_ctrl();
        if (rc) return rc;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, L.ev0, L.ev1));
        const int K = tail ? tu.tail_K : tu.K;
        L.stats.kernel_ms += ms;
        if (tail) L.stats.tail_kernel_ms += ms;
        L.stats.kernel_launches += K;
        L.stats.iterations += K;
        L.stats.graph_replays += 1;
        launches += K;
        if (L.h_ctrl->overflow & 2u) return fail(GV_E_STATE, "compaction look-back wait exceeded its bound");
        if (L.h_ctrl->overflow) return GV_E_CAPACITY;
        const uint32_t* c = L.h_ctrl->count[0];
        if (L.progress)
            std::fprintf(stderr, "[gv] replay %lld %s: %.3f ms, population %u/%u/%u\n",
                         (long long)L.stats.graph_replays, tail ? "tail" : "bulk", ms, c[0], c[1], c[2]);
        const uint32_t before = population;
        population = c[0] + c[1] + c[2];
        grew = population > before;
        peak = std::max(peak, population);
        if (population == 0) {
            if (in_tail) {
                unsigned long long c3[3];
                HIPCHK(hipMemcpyAsync(c3, L.counters.p + kCSteps, sizeof(c3), hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
                L.stats.tail_steps += (int64_t)(c3[0] + c3[1] + c3[2]) - L.tail_steps0;
                L.tail_steps0 = 0;
            }
            break;
        }
        if (launches > bound) return fail(GV_E_STATE, "step loop did not terminate within its launch bound");
    }
    return GV_OK;
}

// plain transport of one event window
int run_plain_window(size_t b, size_t e, uint64_t seed)
{
    QueueMem<P64>& Q = L.plain_pool;
    uint32_t counts[3];
    // all primaries into the single pool of parity 0 (type column set), in order
    {
        int rc0 = ingest<P64>(b, e, Q.q[0], counts, Q.cap, true);
        if (rc0) return rc0;
    }
    int rc = upload_ctrl(counts, seed);
    if (rc) return rc;
    hipStream_t s = stream();
    uint32_t n = counts[0];
    int parity = 0;
    const int TB = 256;
    int64_t launches = 0;
    const int64_t bound = window_launch_bound();
    while (n > 0) {
        PlainArgs A;
        A.pool = Q.q[parity][0];
        A.L = L.pl_L.p;
        A.G = L.pl_G.p;
        A.pr = L.pl_pr.p;
        A.o = L.pl_o.p;
        A.active = L.pl_active.p;
        A.stopped = L.pl_stopped.p;
        A.nsteps_pre = L.pl_nstep.p;
        A.vol_pre = L.pl_volpre.p;
        A.n = n;
        A.seed = seed;
        A.S = make_sinks();
        A.tv = tab_view<double>();
        const unsigned g = (n + TB - 1) / TB;
        HIPCHK(hipEventRecord(L.ev0, s));
        k_plain_prestep_limit<<<g, TB, 0, s>>>(A);
        k_plain_geom<<<g, TB, 0, s>>>(A);
        k_plain_move<<<g, TB, 0, s>>>(A);
        k_plain_msc<<<g, TB, 0, s>>>(A);
        k_plain_eloss<<<g, TB, 0, s>>>(A);
        k_plain_finish<<<g, TB, 0, s>>>(A);
        const unsigned gc = std::min<unsigned>(g, (unsigned)(L.n_cu * 4));
        k_plain_compact<256><<<gc, 256, 0, s>>>(A, Q.q[parity ^ 1][0], L.ctrl.p, parity, L.status.p, (uint32_t)Q.cap);
        HIPCHK(hipGetLastError());
        HIPCHK(hipEventRecord(L.ev1, s));
        rc = read_ctrl();
        if (rc) return rc;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, L.ev0, L.ev1));
        L.stats.kernel_ms += ms;
        L.stats.kernel_launches += 7;
        L.stats.iterations += 1;
        if (L.h_ctrl->overflow & 2u) return fail(GV_E_STATE, "compaction look-back wait exceeded its bound");
        if (L.h_ctrl->overflow) return GV_E_CAPACITY;
        L.plain_loads += n;
        parity ^= 1;
        n = L.h_ctrl->count[parity][0];
        L.plain_stores += n;
        if (++launches > bound) return fail(GV_E_STATE, "step loop did not terminate within its launch bound");
    }
    return GV_OK;
}

int ensure_plain_buffers(size_t cap)
{
    if (L.plain_pool.cap != cap) {
        drop_graph();
        HIPCHK(L.plain_pool.alloc(cap, 2, true));
        // the pool's parity-p queue lives at q[p][0]: remap the set layout
        QueueMem<P64>& Q = L.plain_pool;
        Q.q[1][0] = Q.q[0][1];
    }
    HIPCHK(L.pl_L.ensure(cap));
    HIPCHK(L.pl_G.ensure(cap));
    HIPCHK(L.pl_pr.ensure(cap));
    HIPCHK(L.pl_o.ensure(cap));
    HIPCHK(L.pl_active.ensure(cap));
    HIPCHK(L.pl_stopped.ensure(cap));
    HIPCHK(L.pl_nstep.ensure(cap));
    HIPCHK(L.pl_volpre.ensure(cap));
    return GV_OK;
}

int type_of_pdg(int pdg)
{
    return pdg == 22 ? kGamma : pdg == 11 ? kElectron : pdg == -11 ? kPositron : -1;
}

// zero the per-run device accumulators (deposits, ledger, counters, trace)
int reset_run_buffers(int64_t n_events)
{
    hipStream_t s = stream();
    const size_t nc = (size_t)std::max(L.n_cells, 1);
    HIPCHK(hipMemsetAsync(L.edep.p, 0, (size_t)n_events * nc * sizeof(double), s));
    HIPCHK(hipMemsetAsync(L.ledger.p, 0, (size_t)n_events * 4 * sizeof(double), s));
    HIPCHK(hipMemsetAsync(L.counters.p, 0, kNCount * sizeof(unsigned long long), s));
    HIPCHK(hipMemsetAsync(L.trace_n.p, 0, sizeof(unsigned long long), s));
    HIPCHK(hipMemsetAsync(L.esc_hist.p, 0, kEhSize * sizeof(unsigned long long), s));
    return GV_OK;
}

// Autotuner for the knobs the caller left at 0 (basket, occupancy, inner
// steps).  Trial transports of a sample of the staged batch (its first
// events, at least 1024 primaries, about an eighth of the batch) are timed by
// step-kernel time; coordinate search over inner steps, then basket, then
// occupancy, from the defaults; a candidate replaces the incumbent only if it
// is at least 3 % faster.  The choice is cached per precision, queue order and
// batch-size class; the trials' deposits and counters are discarded.
template <class P> int tuned_choice(int64_t n_events, uint64_t seed, std::array<int, 3>& choice)
{
    L.tuned = false;
    L.autotune_ms = 0.0;
    const bool free_knob = !L.cfg.basket || !L.cfg.occupancy || !L.cfg.inner_steps;
    if (!free_knob || L.n_prim < kTuneMinPrimaries) return GV_OK;
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= L.n_prim) ++lg;
    const auto key = std::make_tuple((int)P::kMixed, (int)L.cfg.queue_order, lg);
    auto it = L.tune_cache.find(key);
    if (it != L.tune_cache.end()) {
        choice = it->second;
        L.tuned = true;
        return GV_OK;
    }
    const double t0 = now_ms();
    int64_t ne = std::max<int64_t>(1, n_events / 8);
    while (ne < n_events && L.ev_start[ne] < 1024) ne = std::min(n_events, 2 * ne);
    const size_t cap = batch_cap<P>();
    const uint64_t tseed = seed ^ 0x6175746f74756e65ull;
    auto trial = [&](const std::array<int, 3>& c, double& rate) -> int {
        const Tuning tu = pick_tuning(c);
        int rc = ensure_status(cap, tu.block);
        if (rc) return rc;
        rc = reset_run_buffers(ne);
        if (rc) return rc;
        L.stats.iterations = 0;
        const double k0 = L.stats.kernel_ms;
        rc = run_batched_window<P>(L.ev_start[0], L.ev_start[ne], tseed, tu);
        if (rc == GV_E_CAPACITY) {
            rate = 0.0;
            return GV_OK;
        }
        if (rc) return rc;
        unsigned long long cnt[kNCount];
        HIPCHK(hipMemcpyAsync(cnt, L.counters.p, sizeof(cnt), hipMemcpyDeviceToHost, stream()));
        HIPCHK(hipStreamSynchronize(stream()));
        const double ms = L.stats.kernel_ms - k0;
        rate = ms > 0.0 ? (double)(cnt[kCSteps] + cnt[kCSteps + 1] + cnt[kCSteps + 2]) / ms : 0.0;
        if (L.progress)
            std::fprintf(stderr, "[gv] autotune basket %d occupancy %d inner %d: %.4g steps/ms\n", c[0], c[1], c[2],
                         rate);
        return GV_OK;
    };
    std::array<int, 3> best = choice;
    double best_rate = 0.0;
    int rc = trial(best, best_rate);
    if (rc) return rc;
    static const int kCand[3][8] = {{64, 128, 256, 512, 1024, 2048, 4096, 0}, {1, 2, 3, 4, 6, 8, 0, 0},
                                    {1, 2, 4, 8, 0, 0, 0, 0}};
    const int fixed[3] = {L.cfg.basket, L.cfg.occupancy, L.cfg.inner_steps};
    for (int knob : {2, 0, 1}) {
        if (fixed[knob]) continue;
        const std::array<int, 3> base = best;
        for (int v : kCand[knob]) {
            if (v == 0 || v == base[knob]) continue;
            std::array<int, 3> c = base;
            c[knob] = v;
            double r = 0.0;
            rc = trial(c, r);
            if (rc) return rc;
            // a candidate must beat the incumbent by 3 % (timing noise)
            if (r > 1.03 * best_rate) {
                best_rate = r;
                best = c;
            }
        }
    }
    choice = best;
    L.tune_cache[key] = best;
    L.tuned = true;
    L.autotune_ms = now_ms() - t0;
    // discard the trials' results; the transport proper starts clean
    rc = reset_run_buffers(n_events);
    if (rc) return rc;
    const double init_ms = L.stats.init_ms;
    const int32_t drv = L.stats.driver, prec = L.stats.precision;
    L.stats = gv_stats_t{};
    L.stats.init_ms = init_ms;
    L.stats.driver = drv;
    L.stats.precision = prec;
    return GV_OK;
}

template <class P> int transport_batched(int64_t n_events, uint64_t seed)
{
    const std::vector<size_t>& ev_start = L.ev_start;
    const size_t cap = capacity_for_driver(false);
    QueueMem<P>& Q = batch_queues<P>();
    if (Q.cap != cap) {
        drop_graph();
        // only one precision's queues are resident at a time
        L.q64.release();
        L.qmix.release();
        HIPCHK(Q.alloc(cap, 6, false));
    }
    if (rk_queue_mode()) {
        const int rc0 = ensure_rk_jobs<P>(cap);
        if (rc0) return rc0;
    }
    std::array<int, 3> choice{kDefBasket, kDefOccupancy, kDefInner};
    int rc = tuned_choice<P>(n_events, seed, choice);
    if (rc) return rc;
    const Tuning tu = pick_tuning(choice);
    rc = ensure_status(cap, tu.block);
    if (rc) return rc;
    L.stats.basket = tu.block * tu.chunks;
    L.stats.occupancy = tu.occupancy;
    L.stats.inner_steps = tu.inner_bulk;
    L.stats.graph_steps = tu.K;
    L.stats.capacity = (int64_t)cap;
    int64_t window = L.cfg.max_events_in_flight > 0 ? L.cfg.max_events_in_flight : n_events;
    int64_t e0 = 0;
    while (e0 < n_events) {
        const int64_t e1 = std::min(n_events, e0 + window);
        rc = snapshot_sinks();
        if (rc) return rc;
        rc = run_batched_window<P>(ev_start[e0], ev_start[e1], seed, tu);
        if (rc == GV_E_CAPACITY) {
            if (e1 - e0 <= 1) return fail(GV_E_CAPACITY, "track queues overflow with one event in flight");
            // undo the window's partial deposits, ledger rows and counters and
            // retry with half the events
            const size_t nc = (size_t)std::max(L.n_cells, 1);
            HIPCHK(hipMemsetAsync(L.edep.p + (size_t)e0 * nc, 0, (size_t)(e1 - e0) * nc * sizeof(double), stream()));
            HIPCHK(hipMemsetAsync(L.ledger.p + (size_t)e0 * 4, 0, (size_t)(e1 - e0) * 4 * sizeof(double), stream()));
            rc = restore_sinks();
            if (rc) return rc;
            window = std::max<int64_t>(1, (e1 - e0) / 2);
            L.stats.overflow_restarts += 1;
            continue;
        }
        if (rc) return rc;
        e0 = e1;
    }
    return GV_OK;
}

int transport_plain(int64_t n_events, uint64_t seed)
{
    const std::vector<size_t>& ev_start = L.ev_start;
    const size_t cap = capacity_for_driver(true);
    int rc = ensure_plain_buffers(cap);
    if (rc) return rc;
    rc = ensure_status(cap, 256);
    if (rc) return rc;
    L.stats.capacity = (int64_t)cap;
    int64_t window = L.cfg.max_events_in_flight > 0 ? L.cfg.max_events_in_flight : n_events;
    int64_t e0 = 0;
    while (e0 < n_events) {
        const int64_t e1 = std::min(n_events, e0 + window);
        rc = snapshot_sinks();
        if (rc) return rc;
        const double loads0 = L.plain_loads, stores0 = L.plain_stores;
        rc = run_plain_window(ev_start[e0], ev_start[e1], seed);
        if (rc == GV_E_CAPACITY) {
            if (e1 - e0 <= 1) return fail(GV_E_CAPACITY, "track pool overflow with one event in flight");
            const size_t nc = (size_t)std::max(L.n_cells, 1);
            HIPCHK(hipMemsetAsync(L.edep.p + (size_t)e0 * nc, 0, (size_t)(e1 - e0) * nc * sizeof(double), stream()));
            HIPCHK(hipMemsetAsync(L.ledger.p + (size_t)e0 * 4, 0, (size_t)(e1 - e0) * 4 * sizeof(double), stream()));
            rc = restore_sinks();
            if (rc) return rc;
            L.plain_loads = loads0;
            L.plain_stores = stores0;
            window = std::max<int64_t>(1, (e1 - e0) / 2);
            L.stats.overflow_restarts += 1;
            continue;
        }
        if (rc) return rc;
        e0 = e1;
    }
    return GV_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Three-way compaction without allocation.  Its working memory (the basket
// ticket and the look-back status words) lives in `scratch`, one copy per
// device holding the library, kept until the process ends; the caller brings
// inputs and outputs.  Host code reaches the array only through the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNaMaxInputs = (int64_t)1 << 24;                        // inputs per call
constexpr size_t kNaHeader = 8;                                           // words before the status words
constexpr size_t kNaStatus = 3 * (size_t)((kNaMaxInputs + 63) / 64);      // at the smallest block
constexpr size_t kNaWords = kNaHeader + kNaStatus;                        // 6 MiB
constexpr int kNaMaxDevices = 64;
}  // namespace

static __device__ __align__(256) uint64_t scratch[kNaWords];

namespace {
struct NaDevice {
    uint64_t* ptr = nullptr;   // device address of this device's `scratch`
    int n_cu = 0;
};
NaDevice g_na[kNaMaxDevices];
std::mutex g_na_mutex;

// zero the ticket, the caller's counts and the status words one call uses
__global__ void k_na_clear(uint64_t* base, size_t status_words, uint32_t* counts)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kNaHeader) base[i] = 0;
    if (i < 4) counts[i] = 0;
    for (size_t k = i; k < status_words; k += (size_t)gridDim.x * blockDim.x) base[kNaHeader + k] = 0;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* gv_last_error(void) { return g_err.c_str(); }

int gv_init(const gv_material* mats, int32_t n_mats, const gv_geometry* geom, const gv_tables* tables)
{
    if (L.busy) return fail(GV_E_STATE, "transport in progress");
    const double t0 = now_ms();
    if (!mats || n_mats < 1 || n_mats > GV_MAX_MATS || !geom || !tables)
        return fail(GV_E_INVALID_ARG, "null pointer or material count out of range");
    // ---- validate geometry ----
    if (geom->axis != GV_AXIS_Z_SLABS && geom->axis != GV_AXIS_R_SHELLS) return fail(GV_E_GEOMETRY, "axis");
    if (geom->n_vol < 1 || geom->n_vol > GV_MAX_VOLS || !geom->bounds || !geom->material || !geom->cell)
        return fail(GV_E_GEOMETRY, "volume count or arrays invalid");
    DevGeom g{};
    g.axis = geom->axis;
    g.n_vol = geom->n_vol;
    g.n_mats = n_mats;
    int n_cells = 0;
    for (int v = 0; v <= geom->n_vol; ++v) {
        g.bounds[v] = geom->bounds[v];
        if (!std::isfinite(g.bounds[v])) return fail(GV_E_GEOMETRY, "non-finite boundary");
        if (v > 0 && !(g.bounds[v] > g.bounds[v - 1])) return fail(GV_E_GEOMETRY, "boundaries not strictly increasing");
    }
    if (g.axis == GV_AXIS_R_SHELLS && g.bounds[0] < 0.0) return fail(GV_E_GEOMETRY, "negative radius");
    for (int v = 0; v < geom->n_vol; ++v) {
        g.vmat[v] = geom->material[v];
        g.vcell[v] = geom->cell[v];
        if (g.vmat[v] < -1 || g.vmat[v] >= n_mats) return fail(GV_E_GEOMETRY, "volume material out of range");
        if (g.vmat[v] >= 0 && g.vcell[v] < 0) return fail(GV_E_GEOMETRY, "material volume without a cell");
        if (g.vcell[v] < -1) return fail(GV_E_GEOMETRY, "cell out of range");
        n_cells = std::max(n_cells, g.vcell[v] + 1);
    }
    for (int i = 0; i < 2; ++i) g.env[i] = geom->env[i];
    for (int i = 0; i < 4; ++i) g.world[i] = geom->world[i];
    for (int i = 0; i < 3; ++i) g.B[i] = geom->B[i];
    g.Bmag = std::sqrt(g.B[0] * g.B[0] + g.B[1] * g.B[1] + g.B[2] * g.B[2]);
    for (int i = 0; i < 3; ++i) g.Bhat[i] = g.Bmag > 0.0 ? g.B[i] / g.Bmag : 0.0;
    g.kB = kKB * g.Bmag;
    if (geom->reserved != 0) return fail(GV_E_GEOMETRY, "reserved field must be 0");
    if (geom->field_map != GV_MAP_UNIFORM && geom->field_map != GV_MAP_SOLENOID) return fail(GV_E_GEOMETRY, "field_map");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(g.B[i])) return fail(GV_E_GEOMETRY, "non-finite field");
    g.field_map = geom->field_map;
    if (g.field_map == GV_MAP_SOLENOID) {
        const double R = geom->sol_cm[0], Lh = geom->sol_cm[1];
        if (g.B[0] != 0.0 || g.B[1] != 0.0 || !(R > 0.0) || !(Lh > 0.0) || !std::isfinite(R) || !std::isfinite(Lh))
            return fail(GV_E_GEOMETRY, "solenoid needs B along z and a positive finite radius and half-length");
        // B0 / f(0) with f(0) = 2L / sqrt(R^2 + L^2)
        g.sol_R2 = R * R;
        g.sol_L = Lh;
        const double f0 = 2.0 * Lh / std::sqrt(g.sol_R2 + Lh * Lh);
        g.sol_c = g.B[2] / f0;
    }
    if (g.axis == GV_AXIS_Z_SLABS) {
        if (!(g.env[0] > 0 && g.env[1] > 0 && g.world[0] >= g.env[0] && g.world[1] >= g.env[1] &&
              g.world[2] <= g.bounds[0] && g.world[3] >= g.bounds[g.n_vol]))
            return fail(GV_E_GEOMETRY, "envelope not inside the world box");
    } else {
        if (!(g.env[0] > 0 && g.world[0] >= g.bounds[g.n_vol] && g.world[1] >= g.env[0]))
            return fail(GV_E_GEOMETRY, "envelope not inside the world cylinder");
    }
    g.n_cells = n_cells;
    // ---- validate tables spec ----
    const gv_tables& T = *tables;
    if (!(T.e_min_MeV > 0.0) || !(T.bins_per_decade > 0.0) || T.n_nodes < 2 || T.n_nodes > 8192 ||
        !(T.t_cut_MeV > 0.0) || !(T.k_cut_MeV > 0.0) || !(T.t_track_MeV > 0.0))
        return fail(GV_E_TABLES, "table grid or cuts invalid");
    const double e_max = T.e_min_MeV * std::pow(10.0, (T.n_nodes - 1) / T.bins_per_decade);
    if (!(T.t_track_MeV > T.e_min_MeV) || !(e_max > T.t_track_MeV)) return fail(GV_E_TABLES, "tracking cut off the grid");
    DevPhys ph{};
    ph.n_nodes = T.n_nodes;
    ph.n_mats = n_mats;
    ph.e_min = T.e_min_MeV;
    ph.bpd = T.bins_per_decade;
    ph.log10_emin = std::log10(T.e_min_MeV);
    ph.t_cut = T.t_cut_MeV;
    ph.k_cut = T.k_cut_MeV;
    ph.t_track = T.t_track_MeV;
    for (int m = 0; m < n_mats; ++m) {
        int rc = derive_material(mats[m], ph.mat[m]);
        if (rc) return rc;
    }
    // ---- device ----
    release_all();
    L.cfg = default_config();
    HIPCHK(hipGetDevice(&L.device));
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, L.device));
    L.n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    HIPCHK(hipStreamCreateWithFlags(&L.own_stream, hipStreamNonBlocking));
    L.geom = g;
    L.phys = ph;
    L.n_cells = n_cells;
    ph.field_method = L.cfg.field_method;
    L.phys.field_method = L.cfg.field_method;
    L.phys.chord_tol = L.cfg.chord_tol_cm;
    L.phys.push = L.cfg.push_cm;
    L.phys.rk_frac = L.cfg.rk_frac;
    L.phys.rk_tol = 1.0e-5;
    L.phys.rk_max_sub = 16;
    L.phys.max_steps = L.cfg.max_steps_per_track;
    L.phys.fs_alias = L.cfg.fs_alias;
    HIPCHK(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_geom), &L.geom, sizeof(DevGeom), 0, hipMemcpyHostToDevice, stream()));
    HIPCHK(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_phys), &L.phys, sizeof(DevPhys), 0, hipMemcpyHostToDevice, stream()));
    int rc = build_tables();
    if (rc) {
        release_all();
        return rc;
    }
    L.ready = true;
    L.init_ms = now_ms() - t0;
    L.stats = gv_stats_t{};
    L.stats.init_ms = L.init_ms;
    return GV_OK;
}

int gv_configure(const gv_config* cfg)
{
    if (!cfg) return fail(GV_E_INVALID_ARG, "null config");
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (L.busy) return fail(GV_E_STATE, "transport in progress");
    int rc = validate_config(*cfg);
    if (rc) return rc;
    const bool stream_changed = cfg->hip_stream != L.cfg.hip_stream;
    L.cfg = *cfg;
    if (stream_changed) drop_graph();
    return apply_run_params();
}

int gv_stage(const gv_primary* primaries, int64_t n)
{
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (L.busy) return fail(GV_E_STATE, "transport in progress");
    if (!primaries || n <= 0) return fail(GV_E_INVALID_ARG, "null primaries or n <= 0");
    if (n > ((int64_t)1 << 31)) return fail(GV_E_INVALID_ARG, "too many primaries");
    L.staged = false;
    // ---- validate, type, count events (bookkeeping only) ----
    const double e_max = L.phys.e_min * std::pow(10.0, (L.phys.n_nodes - 1) / L.phys.bpd);
    int64_t n_events = 0;
    for (int64_t i = 0; i < n; ++i) {
        const gv_primary& p = primaries[i];
        const double nn = std::sqrt(p.dir[0] * p.dir[0] + p.dir[1] * p.dir[1] + p.dir[2] * p.dir[2]);
        if (type_of_pdg(p.pdg) < 0) return fail(GV_E_INVALID_ARG, "unknown pdg code");
        if (p.event < 0) return fail(GV_E_INVALID_ARG, "negative event id");
        if (!(p.ekin_MeV > 0.0) || !(p.ekin_MeV <= e_max * (1 + 1e-12)))
            return fail(GV_E_INVALID_ARG, "kinetic energy outside (0, last table node]");
        if (!std::isfinite(p.pos_cm[0]) || !std::isfinite(p.pos_cm[1]) || !std::isfinite(p.pos_cm[2]))
            return fail(GV_E_INVALID_ARG, "non-finite position");
        if (!(std::fabs(nn - 1.0) <= 1.0e-6)) return fail(GV_E_INVALID_ARG, "direction not normalised");
        n_events = std::max<int64_t>(n_events, (int64_t)p.event + 1);
    }
    // primaries grouped by event (stable); track id = order within the event
    L.ev_start.assign((size_t)n_events + 1, 0);
    for (int64_t i = 0; i < n; ++i) L.ev_start[(size_t)primaries[i].event + 1]++;
    for (int64_t e = 0; e < n_events; ++e) L.ev_start[e + 1] += L.ev_start[e];
    std::vector<size_t> fill(L.ev_start.begin(), L.ev_start.end() - 1);
    L.hp.resize((size_t)n);
    L.e_in = 0.0;
    L.tracks0[0] = L.tracks0[1] = L.tracks0[2] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const gv_primary& p = primaries[i];
        const size_t k = fill[p.event]++;
        PrimDev d;
        d.x = p.pos_cm[0];
        d.y = p.pos_cm[1];
        d.z = p.pos_cm[2];
        d.ux = p.dir[0];
        d.uy = p.dir[1];
        d.uz = p.dir[2];
        d.T = p.ekin_MeV;
        d.type = type_of_pdg(p.pdg);
        d.vol = 0;
        d.ev = (uint32_t)p.event;
        d.tid = (uint64_t)(k - L.ev_start[p.event]);
        L.hp[k] = d;
        L.e_in += p.ekin_MeV;
        L.tracks0[d.type]++;
    }
    L.n_events = n_events;
    L.n_prim = n;
    HIPCHK(L.prim.ensure((size_t)n));
    HIPCHK(hipMemcpyAsync(L.prim.p, L.hp.data(), (size_t)n * sizeof(PrimDev), hipMemcpyHostToDevice, stream()));
    HIPCHK(hipStreamSynchronize(stream()));
    L.staged_b = L.staged_e = (size_t)-1;
    L.staged = true;
    return GV_OK;
}

int gv_transport_staged(uint64_t seed, double* edep_out)
{
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (L.busy) return fail(GV_E_STATE, "transport in progress");
    if (!L.staged) return fail(GV_E_STATE, "no staged primaries (gv_stage)");
    if (!edep_out) return fail(GV_E_INVALID_ARG, "null edep_out");
    const double t0 = now_ms();
    const int64_t n_events = L.n_events;
    L.busy = true;
    struct Guard {
        ~Guard() { L.busy = false; }
    } guard;
    int rc = ensure_common(n_events);
    if (rc) return rc;
    hipStream_t s = stream();
    rc = reset_run_buffers(n_events);
    if (rc) return rc;
    L.stats = gv_stats_t{};
    L.autotune_ms = 0.0;
    L.tuned = false;
    L.plain_loads = L.plain_stores = 0.0;
    L.stats.init_ms = L.init_ms;
    L.stats.driver = L.cfg.driver;
    L.stats.precision = L.cfg.precision;
    if (L.cfg.driver == GV_DRIVER_PLAIN) rc = transport_plain(n_events, seed);
    else if (L.cfg.precision == GV_P64) rc = transport_batched<P64>(n_events, seed);
    else rc = transport_batched<PMix>(n_events, seed);
    if (rc) return rc;
    // ---- results ----
    const size_t ne = (size_t)n_events * (size_t)L.n_cells;
    if (L.cfg.deposit_mode == GV_DEPOSIT_FIXED) {
        if (ne > 0) k_fixed_to_double<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(L.edep.p, (long long)ne);
        k_fixed_to_double<<<(unsigned)((n_events * 4 + 255) / 256), 256, 0, s>>>(L.ledger.p, (long long)n_events * 4);
        HIPCHK(hipGetLastError());
    }
    if (L.n_cells > 0) {
        if (L.cfg.edep_on_device)
            HIPCHK(hipMemcpyAsync(edep_out, L.edep.p, ne * sizeof(double), hipMemcpyDeviceToDevice, s));
        else
            HIPCHK(hipMemcpyAsync(edep_out, L.edep.p, ne * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    L.ledger_h.resize((size_t)n_events * 4);
    HIPCHK(hipMemcpyAsync(L.ledger_h.data(), L.ledger.p, L.ledger_h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    unsigned long long cnt[kNCount];
    HIPCHK(hipMemcpyAsync(cnt, L.counters.p, sizeof(cnt), hipMemcpyDeviceToHost, s));
    unsigned long long tn = 0;
    HIPCHK(hipMemcpyAsync(&tn, L.trace_n.p, sizeof(tn), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    L.last_events = n_events;
    for (int t = 0; t < 3; ++t) {
        L.stats.steps[t] = (int64_t)cnt[kCSteps + t];
        L.stats.tracks[t] = (int64_t)cnt[kCTracks + t] + L.tracks0[t];
    }
    for (int p = 0; p < kNProc; ++p) L.stats.interactions[p] = (int64_t)cnt[kCProc + p];
    L.stats.escaped = (int64_t)cnt[kCEscaped];
    L.stats.killed = (int64_t)cnt[kCKilled];
    L.stats.rejection_exhausted = (int64_t)cnt[kCRej];
    L.stats.rk_substeps = (int64_t)cnt[kCRkSub];
    L.stats.rk_rejected = (int64_t)cnt[kCRkRej];
    L.stats.rk_lane_slots = (int64_t)cnt[kCRkSlots];
    L.stats.lane_slots = (int64_t)cnt[kCLaneSlots];
    L.stats.helper_steps = (int64_t)cnt[kCHelperSteps];
    L.stats.rk_parked = (int64_t)cnt[kCRkParked];
    L.stats.trace_records = (int64_t)std::min<unsigned long long>(tn, (unsigned long long)L.cfg.trace_cap);
    L.stats.e_in = L.e_in;
    double ed = 0.0, es = 0.0, ek = 0.0, np_ = 0.0, na = 0.0;
    for (int64_t e = 0; e < n_events; ++e) {
        es += L.ledger_h[4 * e + 0];
        ek += L.ledger_h[4 * e + 1];
        np_ += L.ledger_h[4 * e + 2];
        na += L.ledger_h[4 * e + 3];
    }
    if (!L.cfg.edep_on_device)
        for (size_t i = 0; i < ne; ++i) ed += edep_out[i];
    else
        ed = L.e_in + 2.0 * kMe * (na - np_) - es - ek;   // by the ledger identity
    L.stats.e_dep = ed;
    L.stats.e_escaped = es;
    L.stats.e_killed = ek;
    L.stats.n_pair = np_;
    L.stats.n_annih = na;
    // algorithmic track-state bytes: per step one slot read and the moving
    // fields (position, direction, energy, volume, step count) written back;
    // one slot written per secondary
    {
        const bool mixed = L.cfg.driver == GV_DRIVER_BATCHED && L.cfg.precision == GV_PMIX;
        const double per_step = mixed ? 60.0 + 48.0 : 77.0 + 64.0;
        const double per_child = mixed ? 60.0 : 77.0;
        double steps = 0.0, children = 0.0;
        for (int t = 0; t < 3; ++t) {
            steps += (double)L.stats.steps[t];
            children += (double)(L.stats.tracks[t] - L.tracks0[t]);
        }
        L.stats.alg_bytes = per_step * steps + per_child * children;
    }
    // track-state bytes the step kernels actually moved: one slot read per
    // track per launch, one slot written per survivor and per secondary
    if (L.cfg.driver == GV_DRIVER_BATCHED) {
        const double slot_bytes = L.cfg.precision == GV_PMIX ? 60.0 : 76.0;
        L.stats.state_bytes = (double)(cnt[kCLoads] + cnt[kCStores]) * slot_bytes;
    } else {  // the mixed pool carries a type byte
        L.stats.state_bytes = (L.plain_loads + L.plain_stores) * 77.0;
    }
    L.stats.autotune_ms = L.autotune_ms;
    L.stats.tuned = L.tuned ? 1 : 0;
    L.stats.queue_order = L.cfg.queue_order;
    L.stats.transport_ms = now_ms() - t0;
    return GV_OK;
}

int gv_transport(const gv_primary* primaries, int64_t n, uint64_t seed, double* edep_out)
{
    if (!edep_out) {
        if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
        return fail(GV_E_INVALID_ARG, "null edep_out");
    }
    int rc = gv_stage(primaries, n);
    if (rc) return rc;
    return gv_transport_staged(seed, edep_out);
}

int gv_stats(gv_stats_t* out)
{
    if (!out) return fail(GV_E_INVALID_ARG, "null stats");
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    *out = L.stats;
    return GV_OK;
}

int gv_ledger(double* out, int64_t n_events)
{
    if (!out) return fail(GV_E_INVALID_ARG, "null ledger");
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (n_events != L.last_events) return fail(GV_E_INVALID_ARG, "event count differs from the last transport");
    std::memcpy(out, L.ledger_h.data(), (size_t)n_events * 4 * sizeof(double));
    return GV_OK;
}

int gv_trace(gv_trace_rec* out, int64_t cap, int64_t* n_out)
{
    if (!out || !n_out || cap < 0) return fail(GV_E_INVALID_ARG, "null trace buffer");
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    const int64_t n = std::min<int64_t>(cap, L.stats.trace_records);
    if (n > 0) HIPCHK(hipMemcpy(out, L.trace.p, (size_t)n * sizeof(gv_trace_rec), hipMemcpyDeviceToHost));
    *n_out = n;
    return GV_OK;
}

int gv_escape_hist(uint64_t* out, int64_t n)
{
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (!out || n < kEhSize) return fail(GV_E_INVALID_ARG, "null output or fewer than 2400 entries");
    if (!L.esc_hist.p) {
        std::memset(out, 0, kEhSize * sizeof(uint64_t));
        return GV_OK;
    }
    HIPCHK(hipMemcpyAsync(out, L.esc_hist.p, kEhSize * sizeof(uint64_t), hipMemcpyDeviceToHost, stream()));
    HIPCHK(hipStreamSynchronize(stream()));
    return GV_OK;
}

int gv_alias_table(int32_t model, int32_t node, double* p, double* q, int32_t* alias, int32_t* valid)
{
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (model < 0 || model >= kAlNMod || node < 0 || node >= kAlNE || !p || !q || !alias || !valid)
        return fail(GV_E_INVALID_ARG, "model/node out of range or null output");
    const size_t idx = (size_t)model * kAlNE + node;
    double rec[kAlRec];
    hipStream_t s = stream();
    HIPCHK(hipMemcpyAsync(rec, L.al_rec64.p + idx * kAlRec, sizeof(rec), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(alias, L.al_alias.p + idx * kAlNX, kAlNX * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(valid, L.al_valid.p + idx, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int k = 0; k <= kAlNX; ++k) p[k] = rec[k];
    for (int k = 0; k < kAlNX; ++k) q[k] = rec[kAlNX + 1 + k];
    return GV_OK;
}

int gv_n_cells(int32_t* out)
{
    if (!out) return fail(GV_E_INVALID_ARG, "null");
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    *out = L.n_cells;
    return GV_OK;
}

void gv_finalize(void)
{
    if (L.busy) return;
    release_all();
}

int gv_compact3_noalloc(const int8_t* codes, int64_t n, int32_t block, int32_t* index, uint32_t* counts,
                        void* hip_stream)
{
    if (n < 0 || n > kNaMaxInputs) return fail(GV_E_INVALID_ARG, "n must be in [0, 2^24] (the scratch limit)");
    if (block != 64 && block != 128 && block != 256) return fail(GV_E_INVALID_ARG, "block must be 64, 128 or 256");
    if (!counts || (n > 0 && (!codes || !index))) return fail(GV_E_INVALID_ARG, "null device pointer");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(GV_E_INVALID_ARG, "device index beyond the supported range");
    NaDevice d;
    {
        std::lock_guard<std::mutex> lock(g_na_mutex);
        if (!g_na[dev].ptr) {
            void* p = nullptr;
            HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            int ncu = 0;
            HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
            g_na[dev].n_cu = ncu > 0 ? ncu : 256;
            g_na[dev].ptr = (uint64_t*)p;
        }
        d = g_na[dev];
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const long long nch = (n + block - 1) / block;
    const size_t words = 3 * (size_t)nch;
    const unsigned cg = (unsigned)std::max<size_t>(1, std::min<size_t>((words + 255) / 256, 1024));
    k_na_clear<<<cg, 256, 0, s>>>(d.ptr, words, counts);
    HIPCHK(hipGetLastError());
    if (n == 0) return GV_OK;
    uint32_t* ticket = (uint32_t*)d.ptr;
    uint64_t* status = d.ptr + kNaHeader;
    const unsigned grid = (unsigned)std::min<long long>(nch, (long long)d.n_cu * 4);
    if (block == 64) k_dbg_compact<64><<<grid, 64, 0, s>>>(codes, n, index, 3 * n, counts, ticket, status, 1u);
    else if (block == 128) k_dbg_compact<128><<<grid, 128, 0, s>>>(codes, n, index, 3 * n, counts, ticket, status, 1u);
    else k_dbg_compact<256><<<grid, 256, 0, s>>>(codes, n, index, 3 * n, counts, ticket, status, 1u);
    HIPCHK(hipGetLastError());
    return GV_OK;
}

int gv_debug_step(int32_t stage, int64_t n, gv_debug_io* io)
{
    if (!io || n < 0) return fail(GV_E_INVALID_ARG, "null io or negative n");
    if (!L.ready) return fail(GV_E_NOT_INIT, "gv_init has not succeeded");
    if (L.busy) return fail(GV_E_STATE, "transport in progress");
    if (n == 0) return GV_OK;
    hipStream_t s = stream();
    std::vector<void*> allocs;
    auto dalloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 1)) != hipSuccess) return nullptr;
        allocs.push_back(p);
        return p;
    };
    struct Free {
        std::vector<void*>* a;
        ~Free()
        {
            for (void* p : *a) (void)hipFree(p);
        }
    } freer{&allocs};
    auto up = [&](const void* h, size_t bytes) -> void* {
        void* d = dalloc(bytes);
        if (d && h) (void)hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s);
        return d;
    };
    const unsigned g = (unsigned)((n + 127) / 128);
    if (stage == GV_DBG_PHILOX) {
        if (!io->words || !io->words_out) return fail(GV_E_INVALID_ARG, "words");
        uint32_t* din = (uint32_t*)up(io->words, 24 * n);
        uint32_t* dout = (uint32_t*)dalloc(16 * n);
        if (!din || !dout) return fail(GV_E_HIP, "allocation failed");
        k_dbg_philox<<<g, 128, 0, s>>>(din, dout, n);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(io->words_out, dout, 16 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return GV_OK;
    }
    if (stage == GV_DBG_TABLE) {
        if (!io->values || io->material < 0 || io->material >= L.phys.n_mats || io->which < 0 || io->which > 12 ||
            n > L.phys.n_nodes)
            return fail(GV_E_INVALID_ARG, "table selection");
        // which: 0..11 = (type * 4 + column), 12 = node energies
        const int nn = L.phys.n_nodes;
        if (io->precision == GV_P64) {
            std::vector<double> h((size_t)nn * 3 * kCols * L.phys.n_mats);
            HIPCHK(hipMemcpy(h.data(), L.rec64.p, h.size() * sizeof(double), hipMemcpyDeviceToHost));
            std::vector<double> E(nn);
            HIPCHK(hipMemcpy(E.data(), L.E64.p, nn * sizeof(double), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i)
                io->values[i] = io->which == 12 ? E[i]
                                                : h[((size_t)(io->material * 3 + io->which / 4) * nn + i) * kCols +
                                                    io->which % 4];
        } else {
            std::vector<float> h((size_t)nn * 3 * kCols * L.phys.n_mats);
            HIPCHK(hipMemcpy(h.data(), L.rec32.p, h.size() * sizeof(float), hipMemcpyDeviceToHost));
            std::vector<float> E(nn);
            HIPCHK(hipMemcpy(E.data(), L.E32.p, nn * sizeof(float), hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i)
                io->values[i] = io->which == 12 ? E[i]
                                                : h[((size_t)(io->material * 3 + io->which / 4) * nn + i) * kCols +
                                                    io->which % 4];
        }
        return GV_OK;
    }
    if (stage == GV_DBG_GEOM) {
        if (!io->pos_in || !io->dir_in || !io->vol_in || !io->d_bnd || !io->vol || !io->vol_pre || !io->safety)
            return fail(GV_E_INVALID_ARG, "geom io");
        double* dp = (double*)up(io->pos_in, 24 * n);
        double* dd = (double*)up(io->dir_in, 24 * n);
        int* dv = (int*)up(io->vol_in, 4 * n);
        double* ob = (double*)dalloc(8 * n);
        int* on = (int*)dalloc(4 * n);
        int* ol = (int*)dalloc(4 * n);
        double* os = (double*)dalloc(8 * n);
        if (!dp || !dd || !dv || !ob || !on || !ol || !os) return fail(GV_E_HIP, "allocation failed");
        k_dbg_geom<<<g, 128, 0, s>>>(dp, dd, dv, ob, on, ol, os, n);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(io->d_bnd, ob, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->vol, on, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->vol_pre, ol, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->safety, os, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return GV_OK;
    }
    if (stage == GV_DBG_COMPACT) {
        if (!io->codes || !io->index || !io->counts) return fail(GV_E_INVALID_ARG, "compact io");
        for (int64_t i = 0; i < 3 * n; ++i)
            if (io->codes[i] < -1 || io->codes[i] > 2) return fail(GV_E_INVALID_ARG, "codes must be in [-1, 2]");
        if (n > (int64_t)1 << 28) return fail(GV_E_INVALID_ARG, "too many inputs");
        const int B = io->block;
        if (B != 64 && B != 128 && B != 256) return fail(GV_E_INVALID_ARG, "block must be 64, 128 or 256");
        int8_t* dc = (int8_t*)up(io->codes, 3 * n);
        int* dq = (int*)dalloc(sizeof(int) * 3 * 3 * n);
        uint32_t* dcnt = (uint32_t*)dalloc(16);
        uint32_t* dt = (uint32_t*)dalloc(16);
        const size_t nch = (size_t)((n + B - 1) / B);
        uint64_t* dst = (uint64_t*)dalloc(3 * nch * sizeof(uint64_t));
        if (!dc || !dq || !dcnt || !dt || !dst) return fail(GV_E_HIP, "allocation failed");
        HIPCHK(hipMemsetAsync(dcnt, 0, 16, s));
        HIPCHK(hipMemsetAsync(dt, 0, 16, s));
        HIPCHK(hipMemsetAsync(dst, 0, 3 * nch * sizeof(uint64_t), s));
        HIPCHK(hipMemsetAsync(dq, 0xFF, sizeof(int) * 9 * n, s));
        const unsigned grid = (unsigned)std::min<size_t>(nch, (size_t)L.n_cu * 4);
        if (B == 64) k_dbg_compact<64><<<grid, 64, 0, s>>>(dc, n, dq, 3 * n, dcnt, dt, dst, 1u);
        else if (B == 128) k_dbg_compact<128><<<grid, 128, 0, s>>>(dc, n, dq, 3 * n, dcnt, dt, dst, 1u);
        else k_dbg_compact<256><<<grid, 256, 0, s>>>(dc, n, dq, 3 * n, dcnt, dt, dst, 1u);
        HIPCHK(hipGetLastError());
        uint32_t hc[4];
        HIPCHK(hipMemcpyAsync(io->index, dq, sizeof(int) * 9 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(hc, dcnt, 16, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hc[3] & 2u) return fail(GV_E_STATE, "compaction look-back wait exceeded its bound");
        for (int q = 0; q < 3; ++q) io->counts[q] = hc[q];
        return GV_OK;
    }
    if (stage == GV_DBG_STEP || (stage >= GV_DBG_THRU_LIMIT && stage <= GV_DBG_THRU_ELOSS)) {
        const int stop = stage == GV_DBG_STEP ? 0 : stage - GV_DBG_THRU_LIMIT + kThruLimit;
        if (!io->type || !io->pos_in || !io->dir_in || !io->ekin_in || !io->event || !io->tid || !io->nstep)
            return fail(GV_E_INVALID_ARG, "step inputs");
        if (stop && !io->s_eloss) return fail(GV_E_INVALID_ARG, "step outputs: s_eloss");
        if (!io->pos || !io->dir || !io->ekin || !io->edep || !io->vol || !io->vol_pre || !io->limiter ||
            !io->process || !io->status || !io->n_children || !io->ch_type || !io->ch_ekin || !io->ch_dir ||
            !io->ch_tid || !io->step || !io->s_phys || !io->d_bnd || !io->safety)
            return fail(GV_E_INVALID_ARG, "step outputs");
        for (int64_t i = 0; i < n; ++i)
            if (io->type[i] < 0 || io->type[i] > 2 || !(io->ekin_in[i] > 0.0))
                return fail(GV_E_INVALID_ARG, "step input type/energy");
        DbgStepIO d;
        d.stop = stop;
        d.s_eloss = stop ? (double*)dalloc(8 * n) : nullptr;
        d.type = (const int*)up(io->type, 4 * n);
        d.pos_in = (const double*)up(io->pos_in, 24 * n);
        d.dir_in = (const double*)up(io->dir_in, 24 * n);
        d.ekin_in = (const double*)up(io->ekin_in, 8 * n);
        d.event = (const uint32_t*)up(io->event, 4 * n);
        d.tid = (const uint64_t*)up(io->tid, 8 * n);
        d.nstep = (const uint32_t*)up(io->nstep, 4 * n);
        d.pos = (double*)dalloc(24 * n);
        d.dir = (double*)dalloc(24 * n);
        d.ekin = (double*)dalloc(8 * n);
        d.edep = (double*)dalloc(8 * n);
        d.vol = (int*)dalloc(4 * n);
        d.vol_pre = (int*)dalloc(4 * n);
        d.lim = (int*)dalloc(4 * n);
        d.proc = (int*)dalloc(4 * n);
        d.status = (int*)dalloc(4 * n);
        d.nchild = (int*)dalloc(4 * n);
        d.ch_type = (int*)dalloc(8 * n);
        d.ch_ekin = (double*)dalloc(16 * n);
        d.ch_dir = (double*)dalloc(48 * n);
        d.ch_tid = (uint64_t*)dalloc(16 * n);
        d.step = (double*)dalloc(8 * n);
        d.s_phys = (double*)dalloc(8 * n);
        d.d_bnd = (double*)dalloc(8 * n);
        d.safety = (double*)dalloc(8 * n);
        for (void* p : allocs)
            if (!p) return fail(GV_E_HIP, "allocation failed");
        if (allocs.size() != (stop ? 26u : 25u)) return fail(GV_E_HIP, "allocation failed");
        if (io->precision == GV_P64)
            k_dbg_step<P64><<<g, 128, 0, s>>>(d, n, io->seed, tab_view<double>());
        else
            k_dbg_step<PMix><<<g, 128, 0, s>>>(d, n, io->seed, tab_view<float>());
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(io->pos, d.pos, 24 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->dir, d.dir, 24 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->ekin, d.ekin, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->edep, d.edep, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->vol, d.vol, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->vol_pre, d.vol_pre, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->limiter, d.lim, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->process, d.proc, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->status, d.status, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->n_children, d.nchild, 4 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->ch_type, d.ch_type, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->ch_ekin, d.ch_ekin, 16 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->ch_dir, d.ch_dir, 48 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->ch_tid, d.ch_tid, 16 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->step, d.step, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->s_phys, d.s_phys, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->d_bnd, d.d_bnd, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(io->safety, d.safety, 8 * n, hipMemcpyDeviceToHost, s));
        if (stop) HIPCHK(hipMemcpyAsync(io->s_eloss, d.s_eloss, 8 * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return GV_OK;
    }
    return fail(GV_E_INVALID_ARG, "unknown debug stage");
}

}  // extern "C"
