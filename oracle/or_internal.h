/* Internal declarations of the oracle (test infrastructure only). */
#ifndef GV_OR_INTERNAL_H
#define GV_OR_INTERNAL_H
#include <math.h>
#include <stdint.h>
#include "oracle.h"

/* CODATA 2018 */
#define OR_ME 0.51099895                 /* electron mass, MeV */
#define OR_RE 2.8179403262e-13           /* classical electron radius, cm */
#define OR_ALPHA (1.0 / 137.035999084)
#define OR_NA 6.02214076e23
#define OR_KB 2.99792458                 /* p[MeV] = OR_KB * B[T] * R[cm] */
#define OR_PI 3.14159265358979323846

typedef struct {
    int32_t n_mats;
    or_material mat[OR_MAX_MATS];
    double n_el[OR_MAX_MATS];     /* electrons / cm^3 */
    double X0[OR_MAX_MATS];       /* cm */
    double I[OR_MAX_MATS];        /* MeV */
    double hwp[OR_MAX_MATS];      /* plasma energy, MeV */
    int32_t axis, n_vol, n_cells;
    double* bounds;
    int32_t* vmat;
    int32_t* vcell;
    double env[2], world[4], B[3];
    or_field field;
    or_config cfg;
    double* node_E;
    double* tab[OR_MAX_MATS][OR_NTAB];
    double r_track[OR_MAX_MATS][2];
    int ready;
} or_ctx;

extern or_ctx G;

void or_set_error(const char* msg);
void or_build_alias(void);
void or_free_tables(void);
int or_build_tables(void);
int32_t or_vol_material(int32_t vol);
int32_t or_vol_cell(int32_t vol);

/* uniform pair of Box-Muller normals from two uniforms */
void or_box_muller(double ua, double ub, double* g1, double* g2);
#endif
