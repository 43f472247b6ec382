/*
 * oracle.h -- plain, slow, history-based FP64 reference of the basketised
 * EM-shower stepping method (GeantV, arXiv 2005.00949).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP library: only
 * the tests, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code with the HIP library.
 *
 * One track at a time, depth-first per event, threads over events.  Each step
 * follows the stage order of Sec. 2.1.2 (PreStep, ComputeIntLen, GeomQuery,
 * Propagation, PostPropagation = multiple scattering, AlongStepAction =
 * continuous loss, PostStepActions = discrete interaction, SteppingActions =
 * stop/kill/score), the field step rule of Sec. 3.4, and the per-track
 * counter-based random streams with collision-resistant daughter seeding of
 * Sec. 5.1.  The physics models are the EM "standard" set the paper names in
 * Sec. 3.5 reduced to textbook closed forms (Klein-Nishina, complete-screening
 * Bethe-Heitler and bremsstrahlung, Moller/Bhabha, restricted Bethe-Bloch,
 * Highland multiple scattering).
 *
 * Units: cm, MeV, tesla.
 */
#ifndef GV_ORACLE_H
#define GV_ORACLE_H
#include <stdint.h>

#define OR_MAX_ELEM 8
#define OR_MAX_MATS 16

enum { OR_GAMMA = 0, OR_ELECTRON = 1, OR_POSITRON = 2 };
enum { OR_AXIS_Z_SLABS = 0, OR_AXIS_R_SHELLS = 1 };
enum { OR_LIM_PHYS = 0, OR_LIM_ELOSS = 1, OR_LIM_GEOM = 2, OR_LIM_FIELD = 3 };
enum { OR_PROC_COMPTON = 0, OR_PROC_PAIR = 1, OR_PROC_MOLLER = 2, OR_PROC_BHABHA = 3,
       OR_PROC_BREMS_EM = 4, OR_PROC_BREMS_EP = 5, OR_PROC_ANNIH = 6, OR_PROC_NULL = 7,
       OR_NPROC = 8 };
/* random-stream purposes (low 8 bits of the fourth counter word) */
enum { OR_PURP_STEP = 0, OR_PURP_MSC = 1, OR_PURP_CHILD = 2, OR_PURP_ANNIH = 3,
       OR_PURP_FS0 = 16, OR_FS_MAX_ITER = 240 };
/* per-material table arrays */
enum { OR_T_COMPTON = 0, OR_T_PAIR, OR_T_MOLLER, OR_T_BREMS_EM, OR_T_S_EM, OR_T_R_EM,
       OR_T_BHABHA, OR_T_BREMS_EP, OR_T_S_EP, OR_T_R_EP, OR_NTAB };
enum { OR_FIELD_HELIX = 0, OR_FIELD_RK4 = 1, OR_FIELD_RK45 = 2 };
/* field maps: uniform B, or an analytic finite solenoid along z */
enum { OR_MAP_UNIFORM = 0, OR_MAP_SOLENOID = 1 };

#define OR_OUTSIDE (-1)

typedef struct {
    double density;                 /* g/cm^3 */
    int32_t n_elem;
    int32_t Z[OR_MAX_ELEM];
    double A[OR_MAX_ELEM];          /* g/mol */
    double w[OR_MAX_ELEM];          /* mass fractions */
    double I_elem_eV[OR_MAX_ELEM];  /* for Bragg additivity when I_eV == 0 */
    double I_eV;                    /* mean excitation energy; 0 => Bragg */
    double X0_cm;                   /* 0 => Tsai */
} or_material;

typedef struct {
    int32_t axis;                   /* OR_AXIS_* */
    int32_t n_vol;                  /* stack volumes 1..n_vol; 0 is the world */
    const double* bounds;           /* n_vol+1 strictly increasing (z or r) */
    const int32_t* material;        /* n_vol; -1 = vacuum */
    const int32_t* cell;            /* n_vol; -1 = not scored */
    double env[2];                  /* slabs: half-x, half-y; shells: half-z */
    double world[4];                /* slabs: half-x, half-y, z-lo, z-hi; shells: r, half-z */
    double B[3];                    /* tesla; the solenoid's central field is B[2] */
    int32_t field_map;              /* OR_MAP_* */
    int32_t pad;
    double sol[2];                  /* solenoid coil radius and half-length, cm */
} or_geometry;

typedef struct {
    double e_min;                   /* first table node (MeV) */
    double bins_per_decade;
    int32_t n_nodes;
    int32_t field_method;           /* OR_FIELD_* */
    double t_cut;                   /* delta-ray production threshold */
    double k_cut;                   /* bremsstrahlung photon threshold */
    double t_track;                 /* e+- tracking cut, gamma absorption */
    double chord_tol;               /* field: allowed bending deviation */
    double push;                    /* field: push past a boundary */
    double rk_frac;                 /* RK4 substep as a fraction of the radius */
    int64_t max_steps;              /* looper cap */
    int32_t fs_alias;               /* bit m set: model m samples from tables (OR_AL_*) */
    int32_t pad;
    double rk_tol;                  /* RK45: allowed error per substep (see or_rk45_move) */
    int32_t rk_max_sub;             /* RK45: substep attempts per step before it is cut short */
    int32_t pad2;
} or_config;

/* Histogram of escaping particles (single-slab observables, Sec. 4):
 * [type][energy bin][bin of the direction cosine with +z], counts.  Energy
 * bins: 5 per decade from 1 keV (40 bins); cosine bins: 20 on [-1, 1]. */
#define OR_EH_NE 40
#define OR_EH_NC 20
#define OR_EH_SIZE (3 * OR_EH_NE * OR_EH_NC)
int or_escape_hist(int64_t* out);   /* the histogram of the last or_transport */

/* Final-state models with a table (alias) sampler; bit m of fs_alias */
enum { OR_AL_COMPTON = 0, OR_AL_PAIR = 1, OR_AL_BREMS = 2, OR_AL_MOLLER = 3, OR_AL_BHABHA = 4,
       OR_AL_NMOD = 5 };
#define OR_AL_NX 64       /* sub-intervals of the transformed variable per node */
#define OR_AL_NPD 20      /* primary-energy nodes per decade */
#define OR_AL_NE 121      /* nodes 0.1 MeV .. 100 GeV */
#define OR_AL_E0 0.1

typedef struct {
    int32_t pdg;
    int32_t event;
    double ekin;
    double pos[3];
    double dir[3];
} or_primary;

typedef struct {
    uint64_t tid;
    uint32_t event;
    uint32_t nstep;
    int32_t type;
    int32_t limiter;
    int32_t vol_pre;
    int32_t vol_post;
    int32_t process;                /* -1 when no discrete interaction */
    int32_t n_children;
    double pos[3];
    double dir[3];
    double ekin;
    double edep;
    double step;
} or_trace;

enum { OR_C_STEPS_G = 0, OR_C_STEPS_EM, OR_C_STEPS_EP,
       OR_C_TRACKS_G, OR_C_TRACKS_EM, OR_C_TRACKS_EP,
       OR_C_PROC0,                      /* OR_NPROC interaction counters */
       OR_C_ESCAPED = OR_C_PROC0 + OR_NPROC, OR_C_KILLED, OR_C_REJ_EXHAUSTED,
       OR_C_TRACE_DROPPED, OR_C_RK_SUB, OR_C_RK_REJ, OR_NCOUNT };

/* ledger columns per event */
enum { OR_L_ESCAPED = 0, OR_L_KILLED, OR_L_NPAIR, OR_L_NANNIH, OR_NLEDGER };

/* setup: derives material constants and builds the tables; 0 on success */
int or_setup(const or_material* mats, int32_t n_mats, const or_geometry* geom, const or_config* cfg);
const char* or_error(void);

/* full transport of n primaries; edep is n_events x n_cells, ledger n_events x OR_NLEDGER */
int or_transport(const or_primary* prim, int64_t n, uint64_t seed, int32_t n_threads,
                 double* edep, double* ledger, int64_t* counters,
                 or_trace* trace, int64_t trace_cap, int64_t* trace_n);

/* one complete step of each of n independent tracks (no recursion into the
 * children): the single-step reference.  Outputs per input track: the state
 * after the step, the deposit, limiter/process/volume and up to two children
 * (type, ekin, dir, tid).  status[i]: 0 alive, 1 stopped, 2 escaped, 3 killed. */
int or_single_step(int64_t n, uint64_t seed,
                   const int32_t* type, const double* pos, const double* dir, const double* ekin,
                   const uint32_t* event, const uint64_t* tid, const uint32_t* nstep,
                   double* pos_out, double* dir_out, double* ekin_out, double* edep_out,
                   int32_t* vol_out, int32_t* vol_pre_out, int32_t* lim_out, int32_t* proc_out,
                   int32_t* status_out, int32_t* nchild_out,
                   int32_t* ch_type, double* ch_ekin, double* ch_dir, uint64_t* ch_tid,
                   double* s_out, double* sphys_out, double* dbnd_out, double* safety_out);

/* the same step ended after one stage of Sec. 2.1.2 (stop = 0: the whole
 * step, as or_single_step).  After ComputeIntLen: s_phys and s_eloss, the
 * track unmoved; after GeomQuery: also d_bnd and safety; after Propagation:
 * also the step length, limiter and the moved track (position, direction,
 * volume); after multiple scattering: the deflected direction; after the
 * continuous loss: the kinetic energy and deposit.  seloss_out may be NULL. */
enum { OR_STOP_LIMIT = 1, OR_STOP_GEOM = 2, OR_STOP_MOVE = 3, OR_STOP_MSC = 4, OR_STOP_ELOSS = 5 };
int or_stage_step(int32_t stop, int64_t n, uint64_t seed,
                  const int32_t* type, const double* pos, const double* dir, const double* ekin,
                  const uint32_t* event, const uint64_t* tid, const uint32_t* nstep,
                  double* pos_out, double* dir_out, double* ekin_out, double* edep_out,
                  int32_t* vol_out, int32_t* vol_pre_out, int32_t* lim_out, int32_t* proc_out,
                  int32_t* status_out, int32_t* nchild_out,
                  int32_t* ch_type, double* ch_ekin, double* ch_dir, uint64_t* ch_tid,
                  double* s_out, double* sphys_out, double* dbnd_out, double* safety_out, double* seloss_out);

/* ---- unit-level access for the pin tests ---- */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double or_u53(uint32_t wa, uint32_t wb);
double or_u32(uint32_t w);

/* table sampling: node energies, the tables of one node, one sample of the
 * transformed variable from four uniforms, and the samplers themselves */
double or_alias_node_energy(int32_t j);
int32_t or_alias_table(int32_t model, int32_t j, double* p, double* q, int32_t* alias);
double or_alias_pdf(int32_t model, double E, double xi);
double or_alias_var(int32_t model, double E, double xi);
double or_alias_xi(int32_t model, double E, const double u[4]);
int or_sample_compton_alias(double k, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_pair_alias(double k, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_brems_alias(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_moller_alias(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_bhabha_alias(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
double or_expo(uint32_t wa, uint32_t wb);
void or_stream(uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, uint32_t purpose,
               uint32_t out[4]);

double or_mat_electron_density(int32_t m);
double or_mat_X0(int32_t m);
double or_mat_I(int32_t m);
double or_mat_plasma_energy(int32_t m);
double or_xs_compton_per_electron(double k);       /* cm^2 */
double or_xs_compton(int32_t m, double k);         /* 1/cm */
double or_xs_pair(int32_t m, double k);
double or_xs_brems(int32_t m, double T);
double or_xs_moller(int32_t m, double T);
double or_xs_bhabha(int32_t m, double T);
double or_dedx_col(int32_t m, double T, int32_t positron, double t_cut);
double or_dedx_rad(int32_t m, double T, double k_cut);
double or_dedx_total(int32_t m, double T, int32_t positron);
double or_density_effect(int32_t m, double T);
int32_t or_n_nodes(void);
double or_node_energy(int32_t i);
double or_table_node(int32_t m, int32_t which, int32_t i);
double or_table_value(int32_t m, int32_t which, double T);
double or_range_inverse(int32_t m, int32_t positron, double r);
double or_gl_integrate(double (*f)(double), double a, double b);

int32_t or_locate(const double pos[3]);
double or_dist_out(int32_t vol, const double pos[3], const double dir[3], int32_t* next);
double or_safety(int32_t vol, const double pos[3]);

void or_helix_move(int32_t type, double ekin, const double B[3], double s, double pos[3], double dir[3]);
void or_rk4_move(int32_t type, double ekin, const double B[3], double s, int32_t nsub,
                 double pos[3], double dir[3]);

/* A magnetic field: uniform B, or a finite solenoid of coil radius sol[0]
 * and half-length sol[1] centred on the origin along z with central field
 * B[2] (axial field of a uniform current sheet, extended off the axis to
 * second order in r). */
typedef struct {
    int32_t map;                    /* OR_MAP_* */
    int32_t pad;
    double B[3];
    double sol[2];
} or_field;
void or_field_eval(const or_field* f, const double x[3], double B[3]);
/* classic RK4 with the field evaluated at every stage point */
void or_rk4_field_move(int32_t type, double ekin, const or_field* f, double s, int32_t nsub,
                       double pos[3], double dir[3]);
/* Adaptive Dormand-Prince 5(4) over a path length s (see or_sample.c for the
 * error measure and the step-size rule).  Returns the accepted substeps;
 * *n_rej gets the rejected ones and *s_done the length integrated, which is
 * below s only when max_sub attempts ran out. */
int32_t or_rk45_move(int32_t type, double ekin, const or_field* f, double s, double tol,
                     int32_t max_sub, double pos[3], double dir[3], double* s_done, int32_t* n_rej);
/* the Dormand-Prince 5(4) coefficients: a[7*7] (row i, column j < i), the
 * 5th-order weights b[7], the embedded 4th-order weights bh[7], nodes c[7] */
void or_dp45_tableau(double* a, double* b, double* bh, double* c);
double or_highland(int32_t m, double ekin, double s);
void or_rotate(double dir[3], double cos_t, double sin_t, double phi);

/* final-state samplers on a given key; return number of rejection iterations
 * used.  out[] layout documented in or_sample.c. */
int or_sample_compton(double k, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_pair(double k, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_brems(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_moller(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);
int or_sample_bhabha(double T, uint64_t seed, uint32_t event, uint64_t tid, uint32_t nstep, double out[4]);

#endif
