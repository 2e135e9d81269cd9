/*
 * Oracle for the vectorial lattice Boltzmann method (VLBM) with conservative
 * local grid refinement -- TEST INFRASTRUCTURE ONLY.
 *
 * This header belongs to the plain FP64 CPU oracle. Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load the oracle. The product
 * library never includes this header and shares no code with it.
 *
 * Conventions (paper, Sec. 2 "Vectorial LBM" and Sec. 3.2 "Extension to 2-D"):
 *   populations q: 0:+x  1:-x  2:+y  3:-y      (D2Q4, c_q = +-c e_alpha)
 *   components  k: 0:rho 1:rho u 2:rho v 3:rho E
 *   sides          0:west (x-) 1:east (x+) 2:south (y-) 3:north (y+)
 *   population arrays: F[(q*4+k)][y][x]  (row-major, x fastest)
 *   box = {level, i0, j0, nx, ny} in level-l cell indices.
 */
#ifndef VLBM_ORACLE_H
#define VLBM_ORACLE_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc orc;

enum { ORC_BC_PERIODIC = 0, ORC_BC_OUTFLOW = 1, ORC_BC_REFLECT = 2, ORC_BC_INFLOW = 3 };
enum { ORC_EOS_IDEAL = 0, ORC_EOS_STIFFENED = 1, ORC_EOS_VDW = 2 };
/* Deliberate mistakes, planted only to show that the pins catch them. */
enum { ORC_MUT_NONE = 0, ORC_MUT_REFLUX_END_LABEL = 1, ORC_MUT_RECON_SIGMA_SIGN = 2,
       ORC_MUT_REFLUX_LAST_ONLY = 3,
       ORC_MUT_REGRID_RESTART_ALL = 4,      /* a regrid clears every previous-step sample */
       ORC_MUT_REGRID_NEW_FACE_HISTORY = 5, /* a new interface keeps its ring cell's history */
       ORC_MUT_WALL_NO_FLIP = 6,            /* reflecting side without the normal-momentum flip */
       ORC_MUT_SENSOR_BOX_SUM = 7,          /* box filter as a sum instead of a mean */
       ORC_MUT_SENSOR_MAX_NORM = 8,         /* max over k of |s_k| instead of the RMS */
       ORC_MUT_SLOPE_RATIO_INVERTED = 9,    /* hand-off slope scaled by c_now / c_prev */
       ORC_MUT_TAG_ONE_SIDED = 10,          /* tag from rho(+1) - rho(0) instead of the central difference */
       ORC_MUT_FLUX_SENSOR_RMS = 11 };      /* eq. amr-sigma with the RMS over k instead of the max norm */
/* Planted mistake of the single-operation functions (EOS): 1 flips the sign
 * of the a rho^2 term inside the van der Waals pressure. Process-wide. */
void orc_set_function_mutation(int mut);

orc *orc_new(int nx0, int ny0, double dx0, int r, int nlev, double gamma, double c,
             double beta, const int bc[4], const double win[16]);
void orc_free(orc *o);
int orc_set_eos(orc *o, int eos, double a, double b);
int orc_set_mutation(orc *o, int mut);
/* Space/time-adaptive relaxation (eq. sensor-B): per-cell beta from the state
 * at the start of each step; c_sensor, beta_min, beta_max as stated there. */
int orc_set_sensor(orc *o, int on, double c_sensor, double beta_min, double beta_max);
/* beta of every cell of `level` at its last step (Ny x Nx; 0 where inactive). */
int orc_get_beta(const orc *o, int level, double *beta);
int orc_set_boxes(orc *o, const int *boxes, int nboxes);
int orc_regrid(orc *o, const int *boxes, int nboxes);
int orc_set_state(orc *o, int level, int i0, int j0, int nx, int ny, const double *U, long ld);
int orc_get_state(const orc *o, int level, int i0, int j0, int nx, int ny, double *U, long ld);
int orc_get_pop(const orc *o, int level, int i0, int j0, int nx, int ny, double *F, long ld);
int orc_set_pop(orc *o, int level, int i0, int j0, int nx, int ny, const double *F, long ld);
int orc_active_mask(const orc *o, int level, unsigned char *mask);
int orc_advance(orc *o, int ncoarse);
/* Adaptive time step: with on != 0, c = kappa * D * max(|u_alpha| + c_s) over
 * the active cells of every level at the start of every coarse step (ideal
 * gas only); the hand-off's temporal slope takes dt_now / dt_prev. */
int orc_set_time_stepping(orc *o, int on, double kappa);
double orc_time(const orc *o);        /* elapsed time since set_state */
double orc_link_speed(const orc *o);  /* c of the last coarse step */
void orc_totals(const orc *o, double T[4], double ledger[4]);
int orc_tag(const orc *o, int level, double thr, unsigned char *tags);
/* Refinement sensor of eq. (amr-sigma), s = max_k |s_k| per active cell of
 * `level` (out[Ny][Nx], 0 elsewhere), and its tags s > thr. */
int orc_flux_sensor(orc *o, int level, double *out);
int orc_tag_flux(orc *o, int level, double thr, unsigned char *tags);
const char *orc_error(void);

/* Single-operation entry points used by the unit pins. */
void orc_feq(double gamma, double c, int eos, double a, double b, const double W[4],
             double feq[16]);
void orc_flux(double gamma, int eos, double a, double b, const double W[4], double Qx[4],
              double Qy[4]);
void orc_collide(double gamma, double c, double beta, int eos, double a, double b,
                 const double g[16], double fstar[16]);
double orc_minmod(double a, double b);
double orc_recon_value(double out, double prev, double sigma, int r, int k, int j);
double orc_recon_value_scaled(double out, double prev, double sigma, int r, int k, int j, double ratio);
void orc_split_block(int r, const double fc[3][3], double *children);
double orc_merge_block(int r, const double *children);

#ifdef __cplusplus
}
#endif
#endif
