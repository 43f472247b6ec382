/*
 * gv.h -- C ABI of the MI355X (gfx950) basketised EM-shower stepping library.
 *
 * The library transports electrons, positrons and photons through a layered
 * detector (a 1-D stack of slabs or cylindrical shells inside an envelope inside
 * a vacuum world, optionally in a magnetic field: uniform, or the map of a finite
 * solenoid) and scores the energy
 * each event deposits in each cell.  It is the data-parallel hot path of the
 * GeantV method (arXiv 2005.00949): instead of following one track at a time,
 * every stage of a step runs over whole track populations (Sec. 2, "algorithm-
 * centric" stepping; stage order of Sec. 2.1.2), here as HIP kernels over
 * structure-of-arrays track state resident in HBM.
 *
 * Conventions for every function:
 *   * Return value: GV_OK (0) or one of the gv_status codes; gv_last_error()
 *     then returns a human-readable message (thread-local, valid until the
 *     next call from the same thread).
 *   * Pointers are host pointers unless stated otherwise.  The library copies
 *     what it needs before returning; the caller keeps ownership of every
 *     buffer it passes.
 *   * One context per process, bound to the HIP device that is current at
 *     gv_init.  Calls are not re-entrant (GV_E_STATE if a transport is running).
 *   * Units: cm, MeV, tesla.
 */
#ifndef GV_H
#define GV_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GV_MAX_ELEM 8
#define GV_MAX_MATS 16
#define GV_MAX_VOLS 1024

typedef enum {
    GV_OK = 0,
    GV_E_INVALID_ARG = 1,   /* null pointer, bad size, bad primary, bad config value */
    GV_E_GEOMETRY = 2,      /* stack bounds not increasing, material/cell out of range */
    GV_E_TABLES = 3,        /* table grid or cuts invalid, non-finite/non-positive table */
    GV_E_HIP = 4,           /* a HIP runtime call failed (message holds the HIP error) */
    GV_E_NOT_INIT = 5,      /* gv_init has not succeeded */
    GV_E_CAPACITY = 6,      /* track queues overflow even with one event in flight */
    GV_E_STATE = 7          /* call while a transport is running */
} gv_status;

enum { GV_AXIS_Z_SLABS = 0, GV_AXIS_R_SHELLS = 1 };
enum { GV_DRIVER_PLAIN = 0, GV_DRIVER_BATCHED = 1 };
enum { GV_P64 = 0, GV_PMIX = 1 };
/* Integration of charged tracks in the field (Sec. 3.6).  HELIX: closed-form
 * helix in the field at the step's start point (exact in a uniform field).
 * RK4: classic Runge-Kutta, ceil(s / (rk_frac * radius)) substeps, the field
 * taken at every stage point.  RK45: adaptive Dormand-Prince 5(4) with first-
 * same-as-last; a substep of length h has the error
 *   err = max(max_a |sum_j e_j kx_j[a]|, max_a |h sum_j e_j ku_j[a]|)
 * (e = 5th- minus 4th-order weights, kx / ku the position / direction stage
 * derivatives): the position error per unit length and the direction error.
 * A substep is accepted when err <= rk_tol.  The first attempt is
 * h = min(s, 0.8 (rk_tol / K)^(1/4) / |du/ds|), K = 8.1e-4 being the pair's
 * error constant on circular motion; then h is halved after a rejected
 * attempt and doubled after an accepted substep with err <= rk_tol / 16, and
 * never passes the end (powers of two: the substeps are an exact function of
 * s and the first attempt).  After rk_max_substeps attempts the step ends
 * where integration stopped. */
enum { GV_FIELD_HELIX = 0, GV_FIELD_RK4 = 1, GV_FIELD_RK45 = 2 };
/* Field maps.  UNIFORM: B everywhere.  SOLENOID: a finite solenoid along z
 * centred on the origin, coil radius sol_cm[0], half-length sol_cm[1],
 * central field B[2] (B[0] = B[1] = 0): on the axis the field of a uniform
 * current sheet, g(z) = B[2] f(z) / f(0) with
 * f(z) = (z+L)/sqrt(R^2+(z+L)^2) - (z-L)/sqrt(R^2+(z-L)^2); off the axis
 * B_r = -(r/2) g'(z), B_z = g(z) - (r^2/4) g''(z). */
enum { GV_MAP_UNIFORM = 0, GV_MAP_SOLENOID = 1 };
/* Order of tracks in the batched driver's queues between step launches.
 * ARRIVAL: each basket reserves its output range when it finishes (one
 * atomic add per queue), so queue order across baskets follows completion
 * order; within a basket it is slot order.  STABLE: output order is the
 * order of the input slots (single-pass look-back over the claimed baskets),
 * identical in every run.  Results are the same in both: a track's random
 * numbers are keyed by (event, track id, step), never by its queue slot. */
enum { GV_ORDER_ARRIVAL = 0, GV_ORDER_STABLE = 1 };
/* Accumulation of deposits and of the energy ledger.  FLOAT: FP64 atomic
 * adds, whose sums depend on arrival order in the last bits.  FIXED: each
 * deposit is rounded once to a whole number of 2^-40 MeV and summed with
 * integer atomics, so results are bit-identical for any basket size,
 * occupancy, inner steps and queue order (the reproducibility requirement of
 * Sec. 5.1 carried to the scores); converted to MeV on return. */
enum { GV_DEPOSIT_FLOAT = 0, GV_DEPOSIT_FIXED = 1 };
/* Final-state models that can sample from tables instead of by
 * composition-rejection (the two sampling methods of Sec. 3.5).  Table
 * sampling: a discrete variable picks one of the two primary-energy nodes
 * around E (20 per decade, 0.1 MeV - 100 GeV) with the linear weight in
 * ln E; Walker's alias table of that node picks one of 64 sub-intervals of a
 * transformed variable, inside which the tabulated linear density is sampled
 * exactly: four uniforms and no loop.  Bit m of gv_config.fs_alias. */
enum { GV_FS_COMPTON = 0, GV_FS_PAIR = 1, GV_FS_BREMS = 2, GV_FS_MOLLER = 3, GV_FS_BHABHA = 4 };

/* A material: density and elemental composition by mass fraction.  The
 * library derives electron density, radiation length (Tsai, unless X0_cm > 0),
 * mean excitation energy (Bragg additivity of I_elem_eV, unless I_eV > 0) and
 * plasma energy (density effect). */
typedef struct {
    double density;                 /* g/cm^3, > 0 */
    int32_t n_elem;                 /* 1..GV_MAX_ELEM */
    int32_t Z[GV_MAX_ELEM];
    double A[GV_MAX_ELEM];          /* g/mol */
    double w[GV_MAX_ELEM];          /* mass fractions, summing to 1 */
    double I_elem_eV[GV_MAX_ELEM];
    double I_eV;
    double X0_cm;
} gv_material;

/* Layered geometry (GeomQuery, Sec. 3.4, for a 1-D stack).  Volume ids:
 * 0 = vacuum world, 1..n_vol = stack volumes, -1 = outside the world.
 *   GV_AXIS_Z_SLABS : volume v is |x| <= env[0], |y| <= env[1],
 *                     z in [bounds[v-1], bounds[v]]; world box
 *                     |x| <= world[0], |y| <= world[1], z in [world[2], world[3]].
 *   GV_AXIS_R_SHELLS: volume v is r in [bounds[v-1], bounds[v]], |z| <= env[0]
 *                     (bounds[0] may be 0); world cylinder r <= world[0],
 *                     |z| <= world[1].
 * material[v-1] indexes the materials array (-1 = vacuum); cell[v-1] is the
 * scoring cell (-1 = none; every non-vacuum volume needs a cell). */
typedef struct {
    int32_t axis;
    int32_t n_vol;                  /* 1..GV_MAX_VOLS */
    const double* bounds;           /* n_vol + 1, strictly increasing */
    const int32_t* material;        /* n_vol */
    const int32_t* cell;            /* n_vol */
    double env[2];
    double world[4];
    double B[3];                    /* field, tesla (see field_map) */
    int32_t field_map;              /* GV_MAP_UNIFORM or GV_MAP_SOLENOID */
    int32_t reserved;               /* must be 0 */
    double sol_cm[2];               /* solenoid coil radius and half-length, > 0 for SOLENOID */
} gv_geometry;

/* Table grid and thresholds from which gv_init builds, on the device, the
 * per-material cross-section, restricted stopping-power and range tables
 * (log grid e_min * 10^(i / bins_per_decade), i < n_nodes; linear
 * interpolation in E; range by Gauss-Legendre quadrature of 1/S). */
typedef struct {
    double e_min_MeV;               /* first node, > 0 */
    double bins_per_decade;         /* > 0 */
    int32_t n_nodes;                /* 2..8192, last node >= highest primary energy */
    int32_t reserved;
    double t_cut_MeV;               /* delta-ray production threshold */
    double k_cut_MeV;               /* bremsstrahlung photon threshold */
    double t_track_MeV;             /* e+- tracking cut; gammas below are absorbed */
} gv_tables;

/* One primary track (64 bytes).  Events are 0..E-1 with E = 1 + max(event);
 * a primary's order of appearance within its event is its track id. */
typedef struct {
    int32_t pdg;                    /* 11 (e-), -11 (e+), 22 (gamma) */
    int32_t event;                  /* >= 0 */
    double ekin_MeV;                /* (0, last table node] */
    double pos_cm[3];
    double dir[3];                  /* |dir| within 1e-6 of 1; renormalised */
} gv_primary;

/* Run options (defaults apply until gv_configure is called). */
typedef struct {
    int32_t driver;                 /* GV_DRIVER_PLAIN (one kernel per stage, host loop) or
                                       GV_DRIVER_BATCHED (persistent kernel over per-type
                                       queues, graph-captured step loop); default BATCHED */
    int32_t precision;              /* GV_P64 or GV_PMIX; PLAIN supports GV_P64 only */
    int32_t basket;                 /* tracks per claimed basket, 64..4096 (power of 2), 0 = tuned */
    int32_t occupancy;              /* workgroups per CU of the persistent kernel, 0 = tuned */
    int32_t inner_steps;            /* max steps a track takes in registers per launch, 0 = tuned.
                                       Knobs left at 0 are chosen by the autotuner for batches
                                       of >= 4096 primaries (trial transports of a sample of
                                       the batch, choice cached per precision, order and batch
                                       size class), otherwise they take the defaults
                                       256 / 3 / 4 */
    int32_t graph_steps;            /* step launches per captured graph, 0 = default */
    int32_t field_method;           /* GV_FIELD_HELIX, GV_FIELD_RK4 or GV_FIELD_RK45 */
    int32_t edep_on_device;         /* edep_out of gv_transport is a device pointer */
    int64_t max_steps_per_track;    /* looper cap, default 2^20 (< 2^24) */
    int64_t capacity;               /* track slots per particle-type queue, 0 = default */
    int64_t max_events_in_flight;   /* 0 = all */
    double chord_tol_cm;            /* field: allowed bending deviation, default 1e-3 */
    double push_cm;                 /* field: push past a boundary, default 1e-7 */
    double rk_frac;                 /* RK4 substep as a fraction of the radius, default 0.05 */
    void* hip_stream;               /* hipStream_t to run on; NULL = the library's own */
    int64_t trace_cap;              /* > 0: record up to this many step records (tests) */
    int32_t queue_order;            /* GV_ORDER_ARRIVAL (default) or GV_ORDER_STABLE; batched driver */
    int32_t deposit_mode;           /* GV_DEPOSIT_FLOAT (default) or GV_DEPOSIT_FIXED */
    int32_t fs_alias;               /* bit m set (m = GV_FS_*): model m samples its final state
                                       from tables instead of by rejection; default 0 */
    int32_t reserved2;              /* must be 0 */
    double rk_tol;                  /* RK45 error tolerance, 0 = default 1e-5 */
    int32_t rk_max_substeps;        /* RK45 attempts per step, 1..2^20, 0 = default 16 */
    int32_t reserved3;              /* must be 0 */
} gv_config;

/* Counters of the last gv_transport. */
typedef struct {
    int64_t steps[3];               /* by type: gamma, e-, e+ (every propagation counts) */
    int64_t tracks[3];              /* tracks created, by type (primaries included) */
    int64_t interactions[8];        /* compton, pair, moller, bhabha, brems e-, brems e+,
                                       annihilation at rest, null (empty sampling interval) */
    int64_t escaped, killed, rejection_exhausted;
    int64_t iterations;             /* step launches */
    int64_t graph_replays;
    int64_t trace_records;
    int64_t overflow_restarts;
    double e_in, e_dep, e_escaped, e_killed;   /* MeV, all events */
    double n_pair, n_annih;
    double transport_ms;            /* wall time of gv_transport */
    double init_ms;                 /* wall time of gv_init (tables, uploads) */
    double kernel_ms;               /* summed duration of the step kernels (HIP events) */
    int64_t kernel_launches;        /* step-kernel launches timed into kernel_ms */
    double alg_bytes;               /* algorithmic track-state bytes: per step one slot read
                                       and the moving fields written back (PMix 60 + 48 B,
                                       FP64 77 + 64 B), plus one slot per secondary */
    int32_t driver, precision, basket, occupancy, inner_steps, graph_steps;
    int64_t capacity;
    double state_bytes;             /* track-state bytes the step kernels actually moved
                                       (slot reads + slot writes) */
    double autotune_ms;             /* time spent choosing basket/occupancy/inner steps
                                       before this transport (0 if a cached choice was used) */
    int32_t tuned;                  /* 1: basket/occupancy/inner steps left at 0 were set by
                                       the autotuner, 0: defaults or caller's values */
    int32_t queue_order;
    int32_t reserved;
    double tail_kernel_ms;          /* part of kernel_ms spent in the tail replays (batched
                                       driver): after the population peaked and fell below the
                                       tail threshold, or, in a window whose population never
                                       reaches the threshold, once a replay no longer raised it */
    int64_t rk_substeps;            /* RK45: accepted substeps */
    int64_t rk_rejected;            /* RK45: rejected attempts */
    int64_t rk_lane_slots;          /* RK45: 64 x the attempt rounds of every wavefront that
                                       integrates (inside a step: as many rounds as its lane
                                       with the most attempts; in the integration queue: every
                                       round while any of its lanes holds an integration);
                                       1 - (substeps + rejected) / lane_slots is the fraction
                                       of idle lanes in the integration loop */
    int64_t lane_slots;             /* batched driver: 64 x (step-loop iterations) summed over the
                                       wavefronts of every basket, a wavefront running as many
                                       iterations as its busiest lane; total steps / lane_slots is
                                       the lane use of the stepping loop (0 for the plain driver) */
    int64_t tail_steps;             /* steps taken in the launches counted in tail_kernel_ms */
    int64_t helper_steps;           /* of those, steps taken by the tail's vacuum helper kernel */
    int64_t rk_parked;              /* RK45 with arrival order: charged steps parked at their move
                                       in the integration queue (Sec. 3.6: lanes refilled as
                                       integrations finish); the rest integrate inside the step */
} gv_stats_t;

/* Step-record layout written when trace_cap > 0 (112 bytes). */
typedef struct {
    uint64_t tid;
    uint32_t event, nstep;
    int32_t type, limiter, vol_pre, vol_post, process, n_children;
    double pos[3], dir[3];
    double ekin, edep, step;
} gv_trace_rec;

/* gv_init -- set up materials, geometry and tables (the detector
 * description and physics tables that every stage reads: geometry of
 * Sec. 3.2 / 3.4 for a layered stack, the per-material cross-section,
 * stopping-power and range tables of Sec. 3.5's models).
 *   mats[n_mats]: host array, 1 <= n_mats <= GV_MAX_MATS; copied.
 *   geom: host record; its arrays are copied.  Validated: stack bounds
 *     strictly increasing and finite, material / cell ids in range, every
 *     material volume scored, envelope inside the world, field finite (a
 *     solenoid needs B along z and a positive radius and half-length).
 *   tables: the grid and thresholds from which the library builds every
 *     table on the device in FP64 (FP32 copies for the mixed policy).  The
 *     caller passes a grid, not table contents: the device computes the
 *     tables from the same closed forms as any other implementation would,
 *     so no table blob crosses the boundary.
 * Binds the context to the current HIP device and replaces any previous
 * context (and its staged batch).  Nothing is retained from the caller.
 * Errors: GV_E_INVALID_ARG (null pointer, count out of range, material
 * fractions), GV_E_GEOMETRY, GV_E_TABLES (grid, cuts, or a non-finite /
 * non-positive built value), GV_E_HIP, GV_E_STATE (called during a
 * transport).  On error no context remains. */
int gv_init(const gv_material* mats, int32_t n_mats, const gv_geometry* geom,
            const gv_tables* tables);

/* gv_configure -- replace the run options (host record, copied): driver
 * (per-stage plain FP64 stepping of Sec. 2.1.2, or the batched persistent
 * kernel over per-type queues that stands in for the scheduler of
 * Sec. 2.1.1), precision policy, basket / occupancy / inner steps (0 =
 * autotuned), field method (Sec. 3.6), stream, capacity, events in flight,
 * queue order, deposit mode (Sec. 5.1 reproducibility) and table sampling
 * per model (Sec. 3.5).  Every field is validated before any is applied.
 * Errors: GV_E_INVALID_ARG (null, out-of-range or reserved field set),
 * GV_E_NOT_INIT, GV_E_STATE; on error the previous options stay. */
int gv_configure(const gv_config* cfg);

/* gv_transport -- transport n primaries (the event server's injection,
 * Sec. 2.1 and 3.7.1) through every stage of Sec. 2.1.2 until all tracks
 * have stopped, escaped or reached the looper cap, and score the energy each
 * event deposits in each cell (per-event scoring of Sec. 3.8.1).
 *   primaries[n]: host array of gv_primary, copied; n >= 1.  Events are
 *     0..E-1 with E = 1 + max(event); a primary's order of appearance within
 *     its event is its track id.  Validation as for gv_stage.
 *   seed: run seed of the counter-based streams: Philox4x32-10 keyed by the
 *     seed, counter (event, track id, step, purpose) (the per-track streams
 *     of Sec. 5.1), so results do not depend on batching or scheduling.
 *   edep_out: caller-owned E x n_cells doubles, row-major [event][cell], in
 *     MeV; host memory unless gv_config.edep_on_device (then a device
 *     pointer on the library's device, written on the configured stream).
 *     Zero-filled, then accumulated; complete when the call returns.
 * Errors: GV_E_NOT_INIT, GV_E_INVALID_ARG, GV_E_CAPACITY (queues overflow
 * with one event in flight), GV_E_HIP, GV_E_STATE (re-entered, or the step
 * loop exceeded its launch bound).  On error edep_out is unspecified and the
 * counters of gv_stats describe the failed call. */
int gv_transport(const gv_primary* primaries, int64_t n, uint64_t seed, double* edep_out);

/* gv_stage / gv_transport_staged -- the same transport in two calls, so that
 * the primaries are made resident on the device once (the event server's
 * input buffer, Sec. 3.7.1) and transported many times with different seeds
 * or options.  gv_stage validates the primaries (pdg 11, -11 or 22; event
 * >= 0; 0 < ekin <= last table node; finite position; |dir| within 1e-6 of
 * 1), groups them by event (stable) and copies them to the device; the
 * caller's array is not retained.  gv_transport_staged transports the staged
 * batch; seed and edep_out as for gv_transport.  gv_init discards the staged
 * batch.  Errors: as gv_transport, plus GV_E_STATE if nothing is staged. */
int gv_stage(const gv_primary* primaries, int64_t n);
int gv_transport_staged(uint64_t seed, double* edep_out);

/* gv_stats -- counters of the last transport (the quantities the paper's
 * validation and performance sections report: steps and secondaries per
 * type, interactions per process, Sec. 4; stepping time, basket and
 * occupancy, Sec. 6.2; integration work and idle lanes, Sec. 3.6), copied
 * into the caller-owned *out.  Errors: GV_E_INVALID_ARG (null),
 * GV_E_NOT_INIT. */
int gv_stats(gv_stats_t* out);

/* gv_ledger -- per-event energy ledger of the last transport (energy that
 * left the scored cells: escaped and killed energy, and the conversion and
 * annihilation counts that change the rest-mass balance), so that
 *   sum T_primaries + 2 m (annihilations - conversions)
 *     = sum edep + escaped + killed   per event.
 * out: caller-owned n_events x 4 doubles (escaped MeV, killed MeV,
 * conversions, annihilations); n_events must equal the last transport's.
 * Errors: GV_E_INVALID_ARG, GV_E_NOT_INIT. */
int gv_ledger(double* out, int64_t n_events);

/* gv_trace -- step records of the last transport (trace_cap > 0): one
 * record per propagation, the per-track step history that the paper's
 * reproducibility test compares (Sec. 5.1).  out: caller-owned, cap
 * records; *n_out = records copied (records beyond trace_cap were dropped;
 * order is not defined).  Errors: GV_E_INVALID_ARG, GV_E_NOT_INIT, GV_E_HIP. */
int gv_trace(gv_trace_rec* out, int64_t cap, int64_t* n_out);

/* gv_n_cells -- number of scoring cells of the current geometry (the row
 * length of edep_out).  Errors: GV_E_INVALID_ARG, GV_E_NOT_INIT. */
int gv_n_cells(int32_t* out);

/* gv_escape_hist -- particles that left the world in the last transport,
 * counted per type (gamma, e-, e+), kinetic-energy bin (5 per decade from
 * 1 keV, 40 bins) and bin of the direction cosine with +z (20 bins on
 * [-1, 1]): the transmission / reflection spectra of single-slab set-ups
 * (Sec. 4).  Integer counts, so any arrival order gives the same histogram.
 * out: 3 x 40 x 20 uint64, row-major, caller-owned; n >= 2400.
 * Errors: GV_E_NOT_INIT, GV_E_INVALID_ARG, GV_E_HIP. */
int gv_escape_hist(uint64_t* out, int64_t n);

/* gv_alias_table -- test access to the final-state sampling table of one
 * model (GV_FS_*) at one node (0..120, energy 0.1 MeV * 10^(node/20)): the
 * sampling tables of Sec. 3.5, read back for comparison.  Outputs are
 * caller-owned: p[65] (density of the transformed variable at 65 points),
 * q[64] (alias thresholds), alias[64] (alias columns), *valid (node above
 * the model's threshold).  Errors: GV_E_NOT_INIT, GV_E_INVALID_ARG, GV_E_HIP. */
int gv_alias_table(int32_t model, int32_t node, double* p, double* q, int32_t* alias, int32_t* valid);

/* gv_finalize -- release every device allocation and the staged batch; the
 * context must be re-initialised before further use.  Does nothing while a
 * transport is running. */
void gv_finalize(void);

/* gv_last_error -- human-readable message of the last nonzero status on the
 * calling thread (thread-local storage owned by the library, valid until
 * that thread's next call). */
const char* gv_last_error(void);

/* ---------------- test entry points ---------------- */

enum {
    GV_DBG_STEP = 0,        /* one complete step of independent tracks */
    GV_DBG_PHILOX = 1,      /* raw Philox4x32-10 blocks */
    GV_DBG_COMPACT = 2,     /* stable three-way compaction (queue management) */
    GV_DBG_TABLE = 3,       /* read back a built table (node values) */
    GV_DBG_GEOM = 4,        /* distance to boundary, next volume, safety, locate */
    /* the step of GV_DBG_STEP ended after one of its stages (Sec. 2.1.2): */
    GV_DBG_THRU_LIMIT = 5,  /* ComputeIntLen: physics and continuous-loss lengths */
    GV_DBG_THRU_GEOM = 6,   /* GeomQuery: boundary distance and safety */
    GV_DBG_THRU_MOVE = 7,   /* Propagation: step length, limiter, moved and relocated track */
    GV_DBG_THRU_MSC = 8,    /* PostPropagation: multiple-scattering deflection */
    GV_DBG_THRU_ELOSS = 9   /* AlongStepAction: continuous energy loss and deposit */
};

/* Host arrays for the test entry point; which fields are read or written
 * depends on the stage:
 *   GV_DBG_STEP   in : type, pos[3n], dir[3n], ekin, event, tid, nstep, precision, seed
 *                 out: pos, dir, ekin, edep, vol, vol_pre, limiter, process, status,
 *                      n_children, ch_type[2n], ch_ekin[2n], ch_dir[6n], ch_tid[2n],
 *                      step, s_phys, d_bnd, safety
 *   GV_DBG_PHILOX in : words[6n] = counter(4), key(2);  out: words_out[4n]
 *   GV_DBG_COMPACT in: codes[3n] (output type 0..2 or -1 for the survivor and the
 *                      two child slots of each input), block;  out: index[3 * 3n]
 *                      (queue q at index + q*3n: input*4 + slot), counts[3]
 *   GV_DBG_TABLE  in : material, which (table id), precision;  out: values[n]
 *   GV_DBG_GEOM   in : pos, dir, vol (-2 = locate first);  out: d_bnd, vol (next),
 *                      vol_pre (located volume), safety
 *   GV_DBG_THRU_* in and out as GV_DBG_STEP, and out: s_eloss; outputs that the
 *                      stages run so far have not produced keep their initial
 *                      values (lengths 0, limiter and process -1, no children,
 *                      the input position, direction and energy) */
typedef struct {
    int32_t precision;
    int32_t block;
    int32_t material;
    int32_t which;
    uint64_t seed;
    const int32_t* type;
    const double* pos_in;
    const double* dir_in;
    const double* ekin_in;
    const uint32_t* event;
    const uint64_t* tid;
    const uint32_t* nstep;
    const int32_t* vol_in;
    const uint32_t* words;
    const int8_t* codes;
    double* pos;
    double* dir;
    double* ekin;
    double* edep;
    int32_t* vol;
    int32_t* vol_pre;
    int32_t* limiter;
    int32_t* process;
    int32_t* status;
    int32_t* n_children;
    int32_t* ch_type;
    double* ch_ekin;
    double* ch_dir;
    uint64_t* ch_tid;
    double* step;
    double* s_phys;
    double* d_bnd;
    double* safety;
    uint32_t* words_out;
    int32_t* index;
    int64_t* counts;
    double* values;
    double* s_eloss;
} gv_debug_io;

/* gv_debug_step -- test entry point: run one stage on n independent inputs
 * given as host arrays (copied to the device and back; the caller owns
 * every array in io):
 *   GV_DBG_STEP    one complete step of Sec. 2.1.2 (PreStep, ComputeIntLen,
 *                  GeomQuery, Propagation, PostPropagation, AlongStep,
 *                  PostStep) on arbitrary track states, with the outputs of
 *                  every stage (physics length, boundary distance, safety,
 *                  limiter, step length, post-step state, deposit,
 *                  secondaries), so that each stage's result can be checked
 *                  on its own against an independent implementation;
 *   GV_DBG_PHILOX  the counter-based generator of Sec. 3.3.2;
 *   GV_DBG_COMPACT the queue compaction of the stage baskets (Sec. 2.1.1);
 *   GV_DBG_TABLE   the built tables of Sec. 3.5;
 *   GV_DBG_GEOM    the geometry queries of Sec. 3.4;
 *   GV_DBG_THRU_*  the step of GV_DBG_STEP on the same inputs, ended after
 *                  the named stage of Sec. 2.1.2, so that each stage's own
 *                  outputs (ComputeIntLen and the continuous-loss limit of
 *                  Sec. 3.5, the field rule and propagation of Sec. 3.4 and
 *                  3.6, the deflection and loss of the along-step actions)
 *                  are compared with those of the reference ended at the same
 *                  stage; the discrete interaction and the stepping actions
 *                  are those of the whole step.
 * GV_DBG_TABLE: n = number of nodes.  Uses temporary device allocations.
 * Errors: GV_E_INVALID_ARG (unknown stage, null or invalid inputs),
 * GV_E_NOT_INIT, GV_E_STATE (during a transport, or a look-back wait gave
 * up), GV_E_HIP. */
int gv_debug_step(int32_t stage, int64_t n, gv_debug_io* io);

/* gv_compact3_noalloc -- the three-way stable compaction of GV_DBG_COMPACT
 * (queue management of the stage baskets) for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc.  It calls no hipMalloc, hipFree, hipMemset or
 * allocating library routine; its working memory (basket ticket and
 * look-back status words, 6 MiB) is a static array of the library, one copy
 * per device, held until the process ends, and cleared by a kernel at the
 * start of every call.  Calls that overlap on one device share that array
 * and race: serialise them (one stream, or events).  Does not need gv_init.
 *   codes: device array of 3n int8 in {-1, 0, 1, 2}: the output queue of the
 *     survivor and the two secondary slots of each input (-1 = none).
 *   n: 0 <= n <= 2^24 (the scratch limit); block: 64, 128 or 256.
 *   index: device array of 9n int32; queue q receives input*4 + slot, in
 *     input order then slot order, at index[q*3n ...]; entries past the
 *     queue's count are left unwritten.
 *   counts: device array of 4 uint32: the three queue sizes, then error
 *     flags (bit 1: a look-back wait gave up, bit 2: a code outside [-1, 2],
 *     which is dropped).
 *   hip_stream: hipStream_t to run on (NULL = the null stream).  The call
 *     only enqueues work: results are ready when the stream reaches them.
 * Errors (nothing enqueued): GV_E_INVALID_ARG (n out of range, block, null
 * pointer, device index >= 64), GV_E_HIP. */
int gv_compact3_noalloc(const int8_t* codes, int64_t n, int32_t block, int32_t* index, uint32_t* counts,
                        void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
