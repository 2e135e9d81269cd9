/* Plain FP64 CPU oracle of the three-dimensional D3Q6 VLBM with conservative
 * local grid refinement -- TEST INFRASTRUCTURE ONLY (see vlbm3_oracle.c). */
#ifndef VLBM3_ORACLE_H
#define VLBM3_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC3_BC_PERIODIC 0
#define ORC3_BC_OUTFLOW 1
#define ORC3_BC_REFLECT 2

typedef struct orc3 orc3;

/* Deliberate mistakes, planted only to show that the pins catch them. */
enum { ORC3_MUT_NONE = 0,
       ORC3_MUT_TAN_SLOPE_SIGN = 1,      /* hand-off: tangential slopes negated */
       ORC3_MUT_TAN_OFFSETS_SWAPPED = 2, /* hand-off: the two tangential offsets exchanged */
       ORC3_MUT_REFLUX_R2 = 3,           /* reflux weight 1 / r^2 instead of 1 / r^3 */
       ORC3_MUT_WALL_NO_FLIP = 4,        /* reflecting side without the normal-momentum flip */
       ORC3_MUT_MERGE_R2 = 5,            /* merge weight 1 / r^2 instead of 1 / r^3 */
       ORC3_MUT_SPLIT_SLOPE_SIGN = 6,    /* split slopes negated */
       ORC3_MUT_REGRID_RESTART_ALL = 7,  /* a regrid clears every previous-step sample */
       ORC3_MUT_REGRID_NEW_FACE_HISTORY = 8 }; /* a new interface keeps its ring cell's history */

/* Populations: index q * 5 + k, q in (+x, -x, +y, -y, +z, -z), k in
 * (rho, rho u, rho v, rho w, E). Level arrays are [comp][Nz][Ny][Nx]. */
void orc3_flux(double gamma, const double W[5], double Qx[5], double Qy[5], double Qz[5]);
void orc3_feq(double gamma, double c, const double W[5], double f[30]);
void orc3_collide(double gamma, double c, double beta, const double g[30], double fstar[30]);

/* bc[6]: sides -x, +x, -y, +y, -z, +z (periodic sides in pairs). */
orc3 *orc3_new(int nx0, int ny0, int nz0, double dx0, int r, int nlev, double gamma, double c,
               double beta, const int bc[6]);
void orc3_free(orc3 *o);
int orc3_set_mutation(orc3 *o, int mut);
/* boxes[n][7] = (level, i0, j0, k0, nx, ny, nz) in level cells, whole parent cells. */
int orc3_set_boxes(orc3 *o, const int *boxes, int nboxes);
int orc3_set_state(orc3 *o, int level, const double *U);   /* U[5][Nz][Ny][Nx]: covered cells */
int orc3_set_pop(orc3 *o, int level, const double *F);     /* F[30][Nz][Ny][Nx] */
int orc3_get_pop(const orc3 *o, int level, double *F);     /* NaN where not active */
int orc3_get_state(const orc3 *o, int level, double *U);   /* NaN where not active */
int orc3_active_mask(const orc3 *o, int level, unsigned char *mask);
int orc3_advance(orc3 *o, int ncoarse);
/* Replace the hierarchy, moving the state conservatively (Sec. 3.4): merge
 * exiting cells finest level first, split entering cells coarsest level first
 * (minmod slope per axis). An interface that exists before and after keeps
 * its temporal reconstruction; one the regrid creates starts flat. */
int orc3_regrid(orc3 *o, const int *boxes, int nboxes);
/* Refinement tags of the active level-l cells (Sec. 3.4, density-gradient
 * variant): tag when max over the axes of |rho(+1) - rho(-1)| / (2 rho)
 * exceeds thr, a neighbour that is not an active cell (periodic sides
 * wrapped) replaced by the cell itself. tags[Nz][Ny][Nx], 0 elsewhere. */
int orc3_tag(const orc3 *o, int level, double thr, unsigned char *tags);
void orc3_totals(const orc3 *o, double T[5], double ledger[5]);
int orc3_shape(const orc3 *o, int level, int shape[3]);     /* (Nx, Ny, Nz) */
const char *orc3_error(void);

#ifdef __cplusplus
}
#endif
#endif
