/*
 * Plain FP64 CPU oracle for the vectorial lattice Boltzmann method (VLBM) with
 * conservative local grid refinement -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library. The product path never links it, and the two share no code.
 *
 * Representation: every level l keeps dense arrays over the WHOLE domain at its
 * own resolution (Nx_l = nx0 r^l, Ny_l = ny0 r^l). A cell is covered at level l
 * when it lies in a level-l box, active when covered and not covered at level
 * l+1 (a "hole"), and only active cells are streamed, collided and counted.
 * The stored state at every time level is the post-collision population f*.
 *
 * What each part follows (paper):
 *   equilibrium                        Sec. 2.2, eq. (num-equilibrium)
 *   transport then BGK relaxation      Sec. 2.2, eq. (num-relaxation)
 *   sub-cycling, one link speed        Sec. 3.2 step 1, eq. (1d-dtratio)
 *   coarse-to-fine reconstruction      Sec. 3.2 step 3 eq. (1d-recon); Sec. 3.3
 *                                      eqs. (2d-recon-tanslope), (2d-recon)
 *   fine-to-coarse reflux              Sec. 3.2 step 4 eq. (1d-reflux); Sec. 3.3
 *                                      eq. (2d-reflux)
 *   merge / split                      Sec. 3.4, eqs. (amr-merge), (amr-slope),
 *                                      (amr-split)
 *   conserved totals                   Sec. 4.1.2 (mass sum over both grids)
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes): the reflux averages the values that cross the face DURING fine
 * sub-step k, i.e. post-collision values at its start; the first cycle after an
 * interface appears has no older coarse sample, so prev := out (slope 0); the
 * tangential slope uses the cells at L0 -+ tau when they are active at the
 * same level, else sigma = 0; a regrid leaves the reconstruction of every
 * interface that exists both before and after it unmodified (Sec. 3.4: the
 * operators run unchanged at whichever interfaces are active), so only the
 * interfaces it creates start with slope 0; relaxation is evaluated as
 * f + 2 beta (feq - f);
 * merges run finest level first and splits coarsest level first; split slopes
 * use neighbours covered at that level in the new hierarchy that hold data.
 *
 * Parity unpinned (conventions shared by design, conservation-neutral): the
 * tangential sigma neighbour rule, the split neighbour rule, the first-cycle
 * slope, and the density-gradient tagging indicator.
 */
#include "vlbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OMAXL 8

static const int CX[4] = {1, -1, 0, 0};
static const int CY[4] = {0, 0, 1, -1};
static const int OPP[4] = {1, 0, 3, 2};

static char g_err[256];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *orc_error(void) { return g_err; }

struct orc {
  int nx0, ny0, r, nlev;
  double dx0, gamma, c, beta;
  int eos;
  double eos_a, eos_b;
  int sensor;                        /* adaptive relaxation on (eq. sensor-B) */
  double c_sensor, beta_min, beta_max;
  double *beta_f[OMAXL];             /* per-cell beta of the level's last step */
  double qmax[4];                    /* max |Q_{alpha,k}| of the current coarse step */
  int adt;                           /* adaptive time step: c per coarse step */
  double kd;                         /* kappa * D */
  double c0;                         /* the parameter c (initial equilibria) */
  double c_last[OMAXL];              /* c of each level's last step */
  double time;                       /* elapsed time */
  int mut;
  int bc[4];
  double win[4][4];
  int Nx[OMAXL], Ny[OMAXL];
  double dx[OMAXL];
  double *F[OMAXL], *Fp[OMAXL], *G[OMAXL], *acc[OMAXL];
  double *accl[OMAXL]; /* last-sub-step-only variant (planted mistake) */
  unsigned char *cov[OMAXL];
  /* pok: per cell, bit q set when the cell's previous-step sample of
   * population q may serve as the hand-off's older coarse sample (eq. 1d-recon) */
  unsigned char *pok[OMAXL];
  double led[4], ledc[4];
};

/* ------------------------------------------------------------------ */
/* Neumaier compensated accumulation                                   */
/* ------------------------------------------------------------------ */
static void kadd(double *s, double *cmp, double v) {
  double t = *s + v;
  if (fabs(*s) >= fabs(v))
    *cmp += (*s - t) + v;
  else
    *cmp += (v - t) + *s;
  *s = t;
}

/* ------------------------------------------------------------------ */
/* Equation of state and Euler flux (Sec. 2.1: the EOS is generic)     */
/* ------------------------------------------------------------------ */
static int g_fmut = 0;
void orc_set_function_mutation(int mut) { g_fmut = mut; }

static double pressure(int eos, double gamma, double a, double b, double rho, double mx,
                       double my, double E) {
  double u = mx / rho;
  double v = my / rho;
  double eint = E - 0.5 * (mx * u + my * v); /* internal energy per volume */
  if (eos == ORC_EOS_STIFFENED) return (gamma - 1.0) * eint - gamma * a;
  if (eos == ORC_EOS_VDW && g_fmut == 1) /* planted mistake */
    return (gamma - 1.0) * (eint - a * rho * rho) / (1.0 - b * rho) - a * rho * rho;
  if (eos == ORC_EOS_VDW) return (gamma - 1.0) * (eint + a * rho * rho) / (1.0 - b * rho) - a * rho * rho;
  return (gamma - 1.0) * eint;
}

void orc_flux(double gamma, int eos, double a, double b, const double W[4], double Qx[4],
              double Qy[4]) {
  double rho = W[0], mx = W[1], my = W[2], E = W[3];
  double u = mx / rho;
  double v = my / rho;
  double p = pressure(eos, gamma, a, b, rho, mx, my, E);
  Qx[0] = mx;
  Qx[1] = mx * u + p;
  Qx[2] = my * u;
  Qx[3] = (E + p) * u;
  Qy[0] = my;
  Qy[1] = mx * v;
  Qy[2] = my * v + p;
  Qy[3] = (E + p) * v;
}

/* eq. (num-equilibrium): f_i^eq = W/(2D) + c_i . Q(W) / (2 c^2), D = 2. */
void orc_feq(double gamma, double c, int eos, double a, double b, const double W[4],
             double feq[16]) {
  double Qx[4], Qy[4];
  double h = 1.0 / (2.0 * c);
  orc_flux(gamma, eos, a, b, W, Qx, Qy);
  for (int k = 0; k < 4; ++k) {
    double w = 0.25 * W[k];
    feq[0 * 4 + k] = w + h * Qx[k];
    feq[1 * 4 + k] = w - h * Qx[k];
    feq[2 * 4 + k] = w + h * Qy[k];
    feq[3 * 4 + k] = w - h * Qy[k];
  }
}

/* eq. (num-relaxation), W = sum_i f_i; evaluated as f + 2 beta (feq - f). */
void orc_collide(double gamma, double c, double beta, int eos, double a, double b,
                 const double g[16], double fstar[16]) {
  double W[4], feq[16];
  for (int k = 0; k < 4; ++k) W[k] = ((g[0 * 4 + k] + g[1 * 4 + k]) + g[2 * 4 + k]) + g[3 * 4 + k];
  orc_feq(gamma, c, eos, a, b, W, feq);
  double tb = 2.0 * beta;
  for (int i = 0; i < 16; ++i) fstar[i] = g[i] + tb * (feq[i] - g[i]);
}

double orc_minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* eq. (2d-recon): out + (out - prev)(2k - r - 1)/(2r) + sigma (2j - r + 1)/(2r);
 * with a time step that changed since the parent's previous step, the
 * temporal term takes the ratio dt_now / dt_prev = c_prev / c_now. */
double orc_recon_value_scaled(double out, double prev, double sigma, int r, int k, int j, double ratio) {
  double ak = (double)(2 * k - r - 1) / (double)(2 * r);
  ak = ak * ratio;
  double bj = (double)(2 * j - r + 1) / (double)(2 * r);
  double B = out - prev;
  double v = out + B * ak;
  return v + sigma * bj;
}

double orc_recon_value(double out, double prev, double sigma, int r, int k, int j) {
  return orc_recon_value_scaled(out, prev, sigma, r, k, j, 1.0);
}

/* eq. (amr-slope) and (amr-split) for one population component. fc is the
 * 3x3 neighbourhood [y][x] centred on the parent; NaN marks a neighbour that is
 * not available (its axis slope is then 0). children is [r][r] (y, x). */
void orc_split_block(int r, const double fc[3][3], double *children) {
  double fi = fc[1][1];
  double sx = 0.0, sy = 0.0;
  if (!isnan(fc[1][0]) && !isnan(fc[1][2])) sx = orc_minmod(fi - fc[1][0], fc[1][2] - fi);
  if (!isnan(fc[0][1]) && !isnan(fc[2][1])) sy = orc_minmod(fi - fc[0][1], fc[2][1] - fi);
  for (int b = 0; b < r; ++b)
    for (int a = 0; a < r; ++a) {
      double xa = (double)(2 * a - r + 1) / (double)(2 * r);
      double xb = (double)(2 * b - r + 1) / (double)(2 * r);
      double v = fi + sx * xa;
      children[b * r + a] = v + sy * xb;
    }
}

/* eq. (amr-merge): plain average of the r^D children, summed row by row. */
double orc_merge_block(int r, const double *children) {
  double s = 0.0;
  for (int i = 0; i < r * r; ++i) s += children[i];
  return s / (double)(r * r);
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */
static size_t cidx(const orc *o, int l, int x, int y) { return (size_t)y * o->Nx[l] + x; }
static size_t pidx(const orc *o, int l, int qk, int x, int y) {
  return ((size_t)qk * o->Ny[l] + y) * o->Nx[l] + x;
}

/* Wrap (x,y) at level l by the periodic sides; return 0 if outside the domain. */
static int wrap(const orc *o, int l, int *x, int *y) {
  int Nx = o->Nx[l], Ny = o->Ny[l];
  if (*x < 0 || *x >= Nx) {
    if (o->bc[0] != ORC_BC_PERIODIC) return 0;
    *x = (*x % Nx + Nx) % Nx;
  }
  if (*y < 0 || *y >= Ny) {
    if (o->bc[2] != ORC_BC_PERIODIC) return 0;
    *y = (*y % Ny + Ny) % Ny;
  }
  return 1;
}

static int covered(const orc *o, int l, int x, int y) {
  if (l >= o->nlev) return 0;
  return o->cov[l][cidx(o, l, x, y)];
}
static int active(const orc *o, int l, int x, int y) {
  if (!covered(o, l, x, y)) return 0;
  if (l + 1 < o->nlev && o->cov[l + 1][cidx(o, l + 1, x * o->r, y * o->r)]) return 0;
  return 1;
}

orc *orc_new(int nx0, int ny0, double dx0, int r, int nlev, double gamma, double c,
             double beta, const int bc[4], const double win[16]) {
  if (nx0 < 1 || ny0 < 1 || r < 1 || nlev < 1 || nlev > OMAXL || !(c > 0.0)) {
    set_err("orc_new: bad arguments");
    return NULL;
  }
  if ((bc[0] == ORC_BC_PERIODIC) != (bc[1] == ORC_BC_PERIODIC) ||
      (bc[2] == ORC_BC_PERIODIC) != (bc[3] == ORC_BC_PERIODIC)) {
    set_err("orc_new: periodic sides must come in pairs");
    return NULL;
  }
  orc *o = (orc *)calloc(1, sizeof(orc));
  o->nx0 = nx0;
  o->ny0 = ny0;
  o->r = r;
  o->nlev = nlev;
  o->dx0 = dx0;
  o->gamma = gamma;
  o->c = c;
  o->c0 = c;
  for (int l = 0; l < OMAXL; ++l) o->c_last[l] = c;
  o->beta = beta;
  for (int s = 0; s < 4; ++s) {
    o->bc[s] = bc[s];
    for (int k = 0; k < 4; ++k) o->win[s][k] = win ? win[s * 4 + k] : 0.0;
  }
  long scale = 1;
  for (int l = 0; l < nlev; ++l) {
    o->Nx[l] = (int)(nx0 * scale);
    o->Ny[l] = (int)(ny0 * scale);
    o->dx[l] = dx0 / (double)scale;
    size_t nc = (size_t)o->Nx[l] * o->Ny[l];
    o->F[l] = (double *)calloc(16 * nc, sizeof(double));
    o->Fp[l] = (double *)calloc(16 * nc, sizeof(double));
    o->G[l] = (double *)calloc(16 * nc, sizeof(double));
    o->acc[l] = (double *)calloc(16 * nc, sizeof(double));
    o->accl[l] = (double *)calloc(16 * nc, sizeof(double));
    o->cov[l] = (unsigned char *)calloc(nc, 1);
    o->pok[l] = (unsigned char *)calloc(nc, 1);
    o->beta_f[l] = (double *)calloc(nc, sizeof(double));
    if (!o->F[l] || !o->Fp[l] || !o->G[l] || !o->acc[l] || !o->accl[l] || !o->cov[l] ||
        !o->pok[l] || !o->beta_f[l]) {
      set_err("orc_new: out of memory");
      orc_free(o);
      return NULL;
    }
    scale *= r;
  }
  memset(o->cov[0], 1, (size_t)o->Nx[0] * o->Ny[0]);
  return o;
}

void orc_free(orc *o) {
  if (!o) return;
  for (int l = 0; l < o->nlev; ++l) {
    free(o->F[l]);
    free(o->Fp[l]);
    free(o->G[l]);
    free(o->acc[l]);
    free(o->accl[l]);
    free(o->cov[l]);
    free(o->pok[l]);
    free(o->beta_f[l]);
  }
  free(o);
}

int orc_set_sensor(orc *o, int on, double c_sensor, double beta_min, double beta_max) {
  if (on && !(beta_min > 0.0 && beta_min <= beta_max && beta_max <= 1.0 && c_sensor >= 0.0)) {
    set_err("orc_set_sensor: need 0 < beta_min <= beta_max <= 1 and c_sensor >= 0");
    return -1;
  }
  o->sensor = on;
  o->c_sensor = c_sensor;
  o->beta_min = beta_min;
  o->beta_max = beta_max;
  return 0;
}

int orc_get_beta(const orc *o, int level, double *beta) {
  if (level < 0 || level >= o->nlev) {
    set_err("orc_get_beta: bad level");
    return -1;
  }
  memcpy(beta, o->beta_f[level], sizeof(double) * (size_t)o->Nx[level] * o->Ny[level]);
  return 0;
}

int orc_set_eos(orc *o, int eos, double a, double b) {
  o->eos = eos;
  o->eos_a = a;
  o->eos_b = b;
  return 0;
}

int orc_set_mutation(orc *o, int mut) {
  o->mut = mut;
  return 0;
}

/* Build coverage masks from boxes and check proper nesting: every cell covered
 * at level l >= 1 must have its parent's four neighbours covered at level l-1
 * (outside a non-periodic domain excepted), and boxes must consist of whole
 * parent cells. */
static int build_cov(const orc *o, const int *boxes, int nboxes, unsigned char **cov) {
  for (int l = 0; l < o->nlev; ++l) {
    size_t nc = (size_t)o->Nx[l] * o->Ny[l];
    memset(cov[l], l == 0 ? 1 : 0, nc);
  }
  for (int b = 0; b < nboxes; ++b) {
    int l = boxes[b * 5], i0 = boxes[b * 5 + 1], j0 = boxes[b * 5 + 2];
    int nx = boxes[b * 5 + 3], ny = boxes[b * 5 + 4];
    if (l < 1 || l >= o->nlev || nx <= 0 || ny <= 0 || i0 < 0 || j0 < 0 ||
        i0 + nx > o->Nx[l] || j0 + ny > o->Ny[l]) {
      set_err("box outside its level's domain");
      return -1;
    }
    if (i0 % o->r || j0 % o->r || nx % o->r || ny % o->r) {
      set_err("box not aligned to whole parent cells");
      return -1;
    }
    for (int y = j0; y < j0 + ny; ++y)
      for (int x = i0; x < i0 + nx; ++x) cov[l][(size_t)y * o->Nx[l] + x] = 1;
  }
  for (int l = 1; l < o->nlev; ++l) {
    for (int y = 0; y < o->Ny[l]; ++y)
      for (int x = 0; x < o->Nx[l]; ++x) {
        if (!cov[l][(size_t)y * o->Nx[l] + x]) continue;
        int px = x / o->r, py = y / o->r;
        for (int d = -1; d < 4; ++d) {
          int nx_ = px + (d < 0 ? 0 : CX[d]), ny_ = py + (d < 0 ? 0 : CY[d]);
          if (!wrap(o, l - 1, &nx_, &ny_)) continue;
          if (!cov[l - 1][(size_t)ny_ * o->Nx[l - 1] + nx_]) {
            set_err("hierarchy not properly nested");
            return -1;
          }
        }
      }
  }
  return 0;
}

int orc_set_boxes(orc *o, const int *boxes, int nboxes) {
  if (build_cov(o, boxes, nboxes, o->cov) != 0) return -1;
  for (int l = 0; l < o->nlev; ++l) memset(o->pok[l], 0, (size_t)o->Nx[l] * o->Ny[l]);
  return 0;
}

int orc_active_mask(const orc *o, int level, unsigned char *mask) {
  if (level < 0 || level >= o->nlev) return -1;
  for (int y = 0; y < o->Ny[level]; ++y)
    for (int x = 0; x < o->Nx[level]; ++x) mask[(size_t)y * o->Nx[level] + x] = (unsigned char)active(o, level, x, y);
  return 0;
}

static int check_rect(const orc *o, int level, int i0, int j0, int nx, int ny) {
  if (level < 0 || level >= o->nlev || i0 < 0 || j0 < 0 || nx < 0 || ny < 0 ||
      i0 + nx > o->Nx[level] || j0 + ny > o->Ny[level]) {
    set_err("rectangle outside the level's domain");
    return -1;
  }
  return 0;
}

/* Initial populations are the equilibrium of U (the paper is silent; standard). */
int orc_set_state(orc *o, int level, int i0, int j0, int nx, int ny, const double *U, long ld) {
  if (check_rect(o, level, i0, j0, nx, ny)) return -1;
  size_t plane = (size_t)ny * ld;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int gx = i0 + x, gy = j0 + y;
      if (!covered(o, level, gx, gy)) continue;
      double W[4], feq[16];
      for (int k = 0; k < 4; ++k) W[k] = U[k * plane + (size_t)y * ld + x];
      orc_feq(o->gamma, o->c0, o->eos, o->eos_a, o->eos_b, W, feq);
      for (int i = 0; i < 16; ++i) {
        o->F[level][pidx(o, level, i, gx, gy)] = feq[i];
        o->Fp[level][pidx(o, level, i, gx, gy)] = feq[i];
      }
      o->pok[level][cidx(o, level, gx, gy)] = 0;
    }
  for (int k = 0; k < 4; ++k) o->led[k] = o->ledc[k] = 0.0;
  o->time = 0.0;
  return 0;
}

int orc_set_pop(orc *o, int level, int i0, int j0, int nx, int ny, const double *Fin, long ld) {
  if (check_rect(o, level, i0, j0, nx, ny)) return -1;
  size_t plane = (size_t)ny * ld;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int gx = i0 + x, gy = j0 + y;
      if (!covered(o, level, gx, gy)) continue;
      for (int i = 0; i < 16; ++i) {
        double v = Fin[i * plane + (size_t)y * ld + x];
        o->F[level][pidx(o, level, i, gx, gy)] = v;
        o->Fp[level][pidx(o, level, i, gx, gy)] = v;
      }
      o->pok[level][cidx(o, level, gx, gy)] = 0;
    }
  for (int k = 0; k < 4; ++k) o->led[k] = o->ledc[k] = 0.0;
  return 0;
}

int orc_get_pop(const orc *o, int level, int i0, int j0, int nx, int ny, double *Fout, long ld) {
  if (check_rect(o, level, i0, j0, nx, ny)) return -1;
  size_t plane = (size_t)ny * ld;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int gx = i0 + x, gy = j0 + y;
      int act = active(o, level, gx, gy);
      for (int i = 0; i < 16; ++i)
        Fout[i * plane + (size_t)y * ld + x] = act ? o->F[level][pidx(o, level, i, gx, gy)] : NAN;
    }
  return 0;
}

int orc_get_state(const orc *o, int level, int i0, int j0, int nx, int ny, double *U, long ld) {
  if (check_rect(o, level, i0, j0, nx, ny)) return -1;
  size_t plane = (size_t)ny * ld;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      int gx = i0 + x, gy = j0 + y;
      int act = active(o, level, gx, gy);
      for (int k = 0; k < 4; ++k) {
        double w = NAN;
        if (act) {
          const double *F = o->F[level];
          w = ((F[pidx(o, level, 0 * 4 + k, gx, gy)] + F[pidx(o, level, 1 * 4 + k, gx, gy)]) +
               F[pidx(o, level, 2 * 4 + k, gx, gy)]) +
              F[pidx(o, level, 3 * 4 + k, gx, gy)];
        }
        U[k * plane + (size_t)y * ld + x] = w;
      }
    }
  return 0;
}

/* ------------------------------------------------------------------ */
/* One time step of level l (transport, then relaxation)               */
/* ------------------------------------------------------------------ */

/* Inbound population q at boundary edge cell (x,y) of level l through side s.
 * Readings: outflow copies the cell's own post-collision q (zero gradient);
 * reflect mirrors the outgoing population with the normal momentum negated;
 * inflow injects the equilibrium of the side's prescribed state. */
static void boundary_value(const orc *o, int l, int side, int q, int x, int y, double v[4]) {
  const double *F = o->F[l];
  if (o->bc[side] == ORC_BC_OUTFLOW) {
    for (int k = 0; k < 4; ++k) v[k] = F[pidx(o, l, q * 4 + k, x, y)];
  } else if (o->bc[side] == ORC_BC_REFLECT) {
    int qo = OPP[q];
    int kn = (side < 2) ? 1 : 2;
    for (int k = 0; k < 4; ++k) {
      double w = F[pidx(o, l, qo * 4 + k, x, y)];
      v[k] = (k == kn && o->mut != ORC_MUT_WALL_NO_FLIP) ? -w : w;
    }
  } else {
    double feq[16];
    orc_feq(o->gamma, o->c, o->eos, o->eos_a, o->eos_b, o->win[side], feq);
    for (int k = 0; k < 4; ++k) v[k] = feq[q * 4 + k];
  }
}

static int side_of(int q, int x_out_low) {
  /* q pointing +x enters through the west side, -x through east, +y south, -y north */
  (void)x_out_low;
  return q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 2 : 3;
}

/* Coarse-to-fine hand-off (eqs. 2d-recon-tanslope, 2d-recon) for the fine cell
 * (x,y) at level l whose upwind neighbour s lies in the coarser region. */
static void recon(const orc *o, int l, int q, int kstep, int x, int y, int sx, int sy, double v[4]) {
  int lp = l - 1, r = o->r;
  int px = sx / r, py = sy / r;
  const double *F = o->F[lp], *Fp = o->Fp[lp];
  int tx, ty, j;
  if (q < 2) {
    tx = 0;
    ty = 1;
    j = y - r * py;
  } else {
    tx = 1;
    ty = 0;
    j = x - r * px;
  }
  int mx_ = px - tx, my_ = py - ty, qx_ = px + tx, qy_ = py + ty;
  int have = wrap(o, lp, &mx_, &my_) && wrap(o, lp, &qx_, &qy_) && active(o, lp, mx_, my_) &&
             active(o, lp, qx_, qy_);
  int has_prev = (o->pok[lp][cidx(o, lp, px, py)] >> q) & 1;
  for (int k = 0; k < 4; ++k) {
    double out = F[pidx(o, lp, q * 4 + k, px, py)];
    double prev = has_prev ? Fp[pidx(o, lp, q * 4 + k, px, py)] : out;
    double sigma = 0.0;
    if (have) {
      double fm = F[pidx(o, lp, q * 4 + k, mx_, my_)];
      double fp = F[pidx(o, lp, q * 4 + k, qx_, qy_)];
      sigma = orc_minmod(out - fm, fp - out);
      if (o->mut == ORC_MUT_RECON_SIGMA_SIGN) sigma = -sigma;
    }
    const double ratio = o->mut == ORC_MUT_SLOPE_RATIO_INVERTED ? o->c / o->c_last[lp] : o->c_last[lp] / o->c;
    v[k] = orc_recon_value_scaled(out, prev, sigma, r, kstep, j, ratio);
  }
}

static void ledger_add(orc *o, double w, const double v[4], double sign) {
  for (int k = 0; k < 4; ++k) kadd(&o->led[k], &o->ledc[k], sign * (w * v[k]));
}

/* Qmax_k = max over the active cells of every level and both directions of
 * |Q_{alpha,k}(W)|, W = sum of the stored populations: the domain-wide
 * normalisation of eq. sensor-B, taken at the start of a coarse step, the one
 * instant at which the whole hierarchy holds one time level. */
static void sensor_qmax(orc *o) {
  for (int k = 0; k < 4; ++k) o->qmax[k] = 0.0;
  for (int l = 0; l < o->nlev; ++l) {
    const double *F = o->F[l];
    for (int y = 0; y < o->Ny[l]; ++y)
      for (int x = 0; x < o->Nx[l]; ++x) {
        if (!active(o, l, x, y)) continue;
        double Wc[4], Qx[4], Qy[4];
        for (int k = 0; k < 4; ++k)
          Wc[k] = ((F[pidx(o, l, 0 * 4 + k, x, y)] + F[pidx(o, l, 1 * 4 + k, x, y)]) +
                   F[pidx(o, l, 2 * 4 + k, x, y)]) + F[pidx(o, l, 3 * 4 + k, x, y)];
        orc_flux(o->gamma, o->eos, o->eos_a, o->eos_b, Wc, Qx, Qy);
        for (int k = 0; k < 4; ++k) {
          double m = fabs(Qx[k]) > fabs(Qy[k]) ? fabs(Qx[k]) : fabs(Qy[k]);
          if (m > o->qmax[k]) o->qmax[k] = m;
        }
      }
  }
}

/* Space/time-adaptive relaxation parameter (Sec. 2.2, eq. sensor-B) of every
 * active cell of level l, from the state at the start of its step
 * (W = sum of the stored populations; relaxation conserves it):
 *   s_k   = dx (div Q)_k / Qmax_k, with dx (div Q)_k by central differences,
 *           0.5 ((Qx_k(x+1) - Qx_k(x-1)) + (Qy_k(y+1) - Qy_k(y-1))), and
 *           Qmax_k of the coarse step (sensor_qmax; s_k = 0 where it is 0);
 *   a     = sqrt(0.25 (((s_0^2 + s_1^2) + s_2^2) + s_3^2))      (RMS over k);
 *   sbar  = mean of a over the active cells of the 3x3 block (box filter S);
 *   dil   = 0.5 ((u(x+1) - u(x-1)) + (v(y+1) - v(y-1))),
 *   vort  = 0.5 ((v(x+1) - v(x-1)) - (u(y+1) - u(y-1)))         (times dx);
 *   theta = dil^2 / (dil^2 + vort^2) where dil < 0 (compression), else 0
 *           (also 0 where dil^2 + vort^2 underflows to 0);
 *   beta  = beta_max - (beta_max - beta_min) clip(C sbar theta, 0, 1).
 * A neighbour that is not an active cell of the level (outside the domain on
 * a non-periodic side, coarser or finer) is replaced by the cell itself. */
static void sensor_beta(orc *o, int l) {
  const int Nx = o->Nx[l], Ny = o->Ny[l];
  const size_t nc = (size_t)Nx * Ny;
  const double *F = o->F[l];
  double *beta = o->beta_f[l];
  double *W = (double *)malloc(sizeof(double) * 4 * nc);
  double *a = (double *)malloc(sizeof(double) * nc);
  double *th = (double *)malloc(sizeof(double) * nc);
  const double *qmax = o->qmax;
  for (int y = 0; y < Ny; ++y)
    for (int x = 0; x < Nx; ++x) {
      if (!active(o, l, x, y)) continue;
      size_t c = cidx(o, l, x, y);
      for (int k = 0; k < 4; ++k)
        W[4 * c + k] = ((F[pidx(o, l, 0 * 4 + k, x, y)] + F[pidx(o, l, 1 * 4 + k, x, y)]) +
                        F[pidx(o, l, 2 * 4 + k, x, y)]) + F[pidx(o, l, 3 * 4 + k, x, y)];
    }
  for (int y = 0; y < Ny; ++y)
    for (int x = 0; x < Nx; ++x) {
      if (!active(o, l, x, y)) continue;
      size_t c = cidx(o, l, x, y);
      /* neighbours +x, -x, +y, -y (themselves where not active) */
      size_t nb[4];
      for (int d = 0; d < 4; ++d) {
        int xx = x + CX[d], yy = y + CY[d];
        nb[d] = (wrap(o, l, &xx, &yy) && active(o, l, xx, yy)) ? cidx(o, l, xx, yy) : c;
      }
      double Qx[4][4], Qy[4][4], u[4], v[4];
      for (int d = 0; d < 4; ++d) {
        orc_flux(o->gamma, o->eos, o->eos_a, o->eos_b, &W[4 * nb[d]], Qx[d], Qy[d]);
        u[d] = W[4 * nb[d] + 1] / W[4 * nb[d] + 0];
        v[d] = W[4 * nb[d] + 2] / W[4 * nb[d] + 0];
      }
      double sk[4];
      for (int k = 0; k < 4; ++k) {
        double dq = (Qx[0][k] - Qx[1][k]) + (Qy[2][k] - Qy[3][k]);
        sk[k] = qmax[k] > 0.0 ? (0.5 * dq) / qmax[k] : 0.0;
      }
      a[c] = sqrt(0.25 * (((sk[0] * sk[0] + sk[1] * sk[1]) + sk[2] * sk[2]) + sk[3] * sk[3]));
      if (o->mut == ORC_MUT_SENSOR_MAX_NORM) { /* planted mistake */
        a[c] = 0.0;
        for (int k = 0; k < 4; ++k) a[c] = fabs(sk[k]) > a[c] ? fabs(sk[k]) : a[c];
      }
      double dil = 0.5 * ((u[0] - u[1]) + (v[2] - v[3]));
      double vort = 0.5 * ((v[0] - v[1]) - (u[2] - u[3]));
      const double den = dil * dil + vort * vort;
      th[c] = (dil < 0.0 && den > 0.0) ? (dil * dil) / den : 0.0;
    }
  for (int y = 0; y < Ny; ++y)
    for (int x = 0; x < Nx; ++x) {
      if (!active(o, l, x, y)) continue;
      size_t c = cidx(o, l, x, y);
      double sum = 0.0;
      int n = 0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int xx = x + dx, yy = y + dy;
          if (!wrap(o, l, &xx, &yy) || !active(o, l, xx, yy)) continue;
          sum += a[cidx(o, l, xx, yy)];
          ++n;
        }
      double z = (o->c_sensor * (o->mut == ORC_MUT_SENSOR_BOX_SUM ? sum : sum / n)) * th[c];
      z = z < 0.0 ? 0.0 : z > 1.0 ? 1.0 : z;
      beta[c] = o->beta_max - (o->beta_max - o->beta_min) * z;
    }
  free(W);
  free(a);
  free(th);
}

static void advance_level(orc *o, int l, int kstep) {
  int Nx = o->Nx[l], Ny = o->Ny[l], r = o->r;
  double w2 = o->dx[l] * o->dx[l];
  double *F = o->F[l];
  if (o->sensor) sensor_beta(o, l);

  /* Values leaving level l during this step are the post-collision values at
   * its start: book them into the parent's reflux accumulator (eq. 2d-reflux)
   * or, at a non-periodic domain side, into the boundary ledger. */
  if (o->mut != ORC_MUT_REFLUX_END_LABEL) {
    for (int y = 0; y < Ny; ++y)
      for (int x = 0; x < Nx; ++x) {
        if (!active(o, l, x, y)) continue;
        for (int q = 0; q < 4; ++q) {
          int dx_ = x + CX[q], dy_ = y + CY[q];
          double v[4];
          for (int k = 0; k < 4; ++k) v[k] = F[pidx(o, l, q * 4 + k, x, y)];
          if (!wrap(o, l, &dx_, &dy_)) {
            ledger_add(o, w2, v, -1.0);
            continue;
          }
          if (l >= 1 && !covered(o, l, dx_, dy_)) {
            int px = dx_ / r, py = dy_ / r;
            for (int k = 0; k < 4; ++k) {
              size_t a = pidx(o, l - 1, q * 4 + k, px, py);
              o->acc[l - 1][a] += v[k];
              if (kstep == r) o->accl[l - 1][a] += v[k];
            }
          }
        }
      }
  } else {
    /* planted mistake: the boundary ledger is still booked at the start */
    for (int y = 0; y < Ny; ++y)
      for (int x = 0; x < Nx; ++x) {
        if (!active(o, l, x, y)) continue;
        for (int q = 0; q < 4; ++q) {
          int dx_ = x + CX[q], dy_ = y + CY[q];
          double v[4];
          for (int k = 0; k < 4; ++k) v[k] = F[pidx(o, l, q * 4 + k, x, y)];
          if (!wrap(o, l, &dx_, &dy_)) ledger_add(o, w2, v, -1.0);
        }
      }
  }

  /* Transport (exact shift) into G, with interface and boundary fills. */
  double *G = o->G[l];
  for (int y = 0; y < Ny; ++y)
    for (int x = 0; x < Nx; ++x) {
      if (!active(o, l, x, y)) continue;
      for (int q = 0; q < 4; ++q) {
        int sx = x - CX[q], sy = y - CY[q];
        double v[4];
        if (!wrap(o, l, &sx, &sy)) {
          boundary_value(o, l, side_of(q, 0), q, x, y, v);
          ledger_add(o, w2, v, +1.0);
        } else if (l + 1 < o->nlev && o->cov[l + 1][cidx(o, l + 1, sx * r, sy * r)]) {
          for (int k = 0; k < 4; ++k) {
            size_t a = pidx(o, l, q * 4 + k, x, y);
            const double *A = (o->mut == ORC_MUT_REFLUX_LAST_ONLY) ? o->accl[l] : o->acc[l];
            double scale = (o->mut == ORC_MUT_REFLUX_LAST_ONLY) ? (double)r : (double)(r * r);
            v[k] = A[a] / scale;
          }
        } else if (covered(o, l, sx, sy)) {
          for (int k = 0; k < 4; ++k) v[k] = F[pidx(o, l, q * 4 + k, sx, sy)];
        } else {
          recon(o, l, q, kstep, x, y, sx, sy, v);
        }
        for (int k = 0; k < 4; ++k) G[pidx(o, l, q * 4 + k, x, y)] = v[k];
      }
    }

  /* Planted mistake only: book the reflux with the values at the END of the
   * sub-step (the literal reading of the time labels). */
  /* (performed after relaxation below) */

  /* Relaxation, cell by cell. */
  for (int y = 0; y < Ny; ++y)
    for (int x = 0; x < Nx; ++x) {
      if (!active(o, l, x, y)) continue;
      double g[16], fs[16];
      for (int i = 0; i < 16; ++i) g[i] = G[pidx(o, l, i, x, y)];
      const double bx = o->sensor ? o->beta_f[l][cidx(o, l, x, y)] : o->beta;
      orc_collide(o->gamma, o->c, bx, o->eos, o->eos_a, o->eos_b, g, fs);
      for (int i = 0; i < 16; ++i) G[pidx(o, l, i, x, y)] = fs[i];
    }

  o->c_last[l] = o->c;
  /* Rotate: previous <- current <- new. */
  double *old = o->Fp[l];
  o->Fp[l] = o->F[l];
  o->F[l] = o->G[l];
  o->G[l] = old;
  for (int y = 0; y < Ny; ++y)
    for (int x = 0; x < Nx; ++x) o->pok[l][cidx(o, l, x, y)] = active(o, l, x, y) ? 0xF : 0;

  if (o->mut == ORC_MUT_REFLUX_END_LABEL && l >= 1) {
    F = o->F[l];
    for (int y = 0; y < Ny; ++y)
      for (int x = 0; x < Nx; ++x) {
        if (!active(o, l, x, y)) continue;
        for (int q = 0; q < 4; ++q) {
          int dx_ = x + CX[q], dy_ = y + CY[q];
          if (!wrap(o, l, &dx_, &dy_)) continue;
          if (!covered(o, l, dx_, dy_)) {
            int px = dx_ / r, py = dy_ / r;
            for (int k = 0; k < 4; ++k) o->acc[l - 1][pidx(o, l - 1, q * 4 + k, px, py)] += F[pidx(o, l, q * 4 + k, x, y)];
          }
        }
      }
  }
}

/* Recursive sub-cycle: level l+1 takes r steps of dt_l / r inside each step of
 * level l, then level l steps (Sec. 3.2 steps 1-4, Fig. 1). */
static void level_cycle(orc *o, int l, int kstep) {
  if (l + 1 < o->nlev) {
    size_t n = 16 * (size_t)o->Nx[l] * o->Ny[l];
    memset(o->acc[l], 0, n * sizeof(double));
    memset(o->accl[l], 0, n * sizeof(double));
    for (int kk = 1; kk <= o->r; ++kk) level_cycle(o, l + 1, kk);
  }
  advance_level(o, l, kstep);
}

/* Adaptive time step (acoustic scaling with a CFL-type link speed, read
 * from the step counts of Sec. 4 and the adaptive time stepping the paper
 * builds on): at the start of every coarse step
 *   c_n = (kappa D) max over the active cells of every level and both axes of
 *         |u_alpha| + c_s,  c_s = sqrt(gamma p / rho)  (ideal gas),
 * the same c on every level (dt_l = dx_l / c_n); the coarse step lasts
 * dx_0 / c_n. */
static double link_speed_now(const orc *o) {
  double m = 0.0;
  for (int l = 0; l < o->nlev; ++l) {
    const double *F = o->F[l];
    for (int y = 0; y < o->Ny[l]; ++y)
      for (int x = 0; x < o->Nx[l]; ++x) {
        if (!active(o, l, x, y)) continue;
        double W[4];
        for (int k = 0; k < 4; ++k)
          W[k] = ((F[pidx(o, l, 0 * 4 + k, x, y)] + F[pidx(o, l, 1 * 4 + k, x, y)]) +
                  F[pidx(o, l, 2 * 4 + k, x, y)]) + F[pidx(o, l, 3 * 4 + k, x, y)];
        double u = W[1] / W[0];
        double v = W[2] / W[0];
        double p = pressure(o->eos, o->gamma, o->eos_a, o->eos_b, W[0], W[1], W[2], W[3]);
        double cs = sqrt((o->gamma * p) / W[0]);
        double a = fabs(u) + cs, b = fabs(v) + cs;
        double s = a > b ? a : b;
        if (s > m) m = s;
      }
  }
  return o->kd * m;
}

int orc_advance(orc *o, int ncoarse) {
  for (int n = 0; n < ncoarse; ++n) {
    if (o->sensor) sensor_qmax(o);
    if (o->adt) o->c = link_speed_now(o);
    level_cycle(o, 0, 1);
    o->time += o->dx0 / o->c;
  }
  return 0;
}

int orc_set_time_stepping(orc *o, int on, double kappa) {
  if (on && !(kappa > 0.0)) {
    set_err("orc_set_time_stepping: kappa must be positive");
    return -1;
  }
  if (on && o->eos != ORC_EOS_IDEAL) {
    set_err("orc_set_time_stepping: ideal gas only");
    return -1;
  }
  o->adt = on;
  o->kd = kappa * 2.0;
  if (!on) { /* back to the parameter c, with no time-step change to carry */
    o->c = o->c0;
    for (int l = 0; l < OMAXL; ++l) o->c_last[l] = o->c0;
  }
  return 0;
}

double orc_time(const orc *o) { return o->time; }
double orc_link_speed(const orc *o) { return o->c; }

/* T_k = sum_l dx_l^2 sum_{active} sum_q f_{q,k}  (Sec. 4.1.2, 2-D form). */
void orc_totals(const orc *o, double T[4], double ledger[4]) {
  for (int k = 0; k < 4; ++k) {
    double s = 0.0, cs = 0.0;
    for (int l = 0; l < o->nlev; ++l) {
      double sl = 0.0, cl = 0.0;
      for (int y = 0; y < o->Ny[l]; ++y)
        for (int x = 0; x < o->Nx[l]; ++x) {
          if (!active(o, l, x, y)) continue;
          for (int q = 0; q < 4; ++q) kadd(&sl, &cl, o->F[l][pidx(o, l, q * 4 + k, x, y)]);
        }
      kadd(&s, &cs, o->dx[l] * o->dx[l] * (sl + cl));
    }
    T[k] = s + cs;
    if (ledger) ledger[k] = o->led[k] + o->ledc[k];
  }
}

/* ------------------------------------------------------------------ */
/* Regrid: merge exiting cells (finest level first), then split         */
/* entering cells (coarsest level first) -- Sec. 3.4, Fig. amr-flowchart */
/* ------------------------------------------------------------------ */
int orc_regrid(orc *o, const int *boxes, int nboxes) {
  int L = o->nlev, r = o->r;
  unsigned char *ncov[OMAXL];
  for (int l = 0; l < L; ++l) ncov[l] = (unsigned char *)malloc((size_t)o->Nx[l] * o->Ny[l]);
  int rc = build_cov(o, boxes, nboxes, ncov);
  if (rc != 0) {
    for (int l = 0; l < L; ++l) free(ncov[l]);
    return -1;
  }
  unsigned char **ocov = o->cov;
  /* 1. merges, finest level first: every block of r x r level-l cells that
   *    leaves level l is averaged into its parent at level l-1. */
  for (int l = L - 1; l >= 1; --l) {
    int Nxp = o->Nx[l - 1], Nyp = o->Ny[l - 1];
    for (int py = 0; py < Nyp; ++py)
      for (int px = 0; px < Nxp; ++px) {
        size_t c0 = cidx(o, l, px * r, py * r);
        if (!ocov[l][c0] || ncov[l][c0]) continue;
        for (int i = 0; i < 16; ++i) {
          double ch[64];
          for (int b = 0; b < r; ++b)
            for (int a = 0; a < r; ++a) ch[b * r + a] = o->F[l][pidx(o, l, i, px * r + a, py * r + b)];
          double m = orc_merge_block(r, ch);
          o->F[l - 1][pidx(o, l - 1, i, px, py)] = m;
          o->Fp[l - 1][pidx(o, l - 1, i, px, py)] = m;
        }
        o->pok[l - 1][cidx(o, l - 1, px, py)] = 0;
      }
  }
  /* 2. splits, coarsest level first: every level-(l+1) cell newly covered is
   *    produced from its parent with minmod slopes; a slope neighbour must be
   *    covered at level l in the new hierarchy and hold data (not a hole that
   *    stays a hole). */
  for (int l = 0; l + 1 < L; ++l) {
    int Nxp = o->Nx[l], Nyp = o->Ny[l];
    for (int py = 0; py < Nyp; ++py)
      for (int px = 0; px < Nxp; ++px) {
        size_t c0 = cidx(o, l + 1, px * r, py * r);
        if (!ncov[l + 1][c0] || ocov[l + 1][c0]) continue;
        int nbx[4], nby[4], avail[4];
        for (int d = 0; d < 4; ++d) {
          nbx[d] = px + CX[d];
          nby[d] = py + CY[d];
          avail[d] = wrap(o, l, &nbx[d], &nby[d]);
          if (avail[d]) {
            size_t ci = cidx(o, l, nbx[d], nby[d]);
            int cov_l = ncov[l][ci];
            int persistent_hole = 0;
            if (l + 1 < L) {
              size_t cc = cidx(o, l + 1, nbx[d] * r, nby[d] * r);
              persistent_hole = ocov[l + 1][cc] && ncov[l + 1][cc];
            }
            avail[d] = cov_l && !persistent_hole;
          }
        }
        for (int i = 0; i < 16; ++i) {
          double fc[3][3];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) fc[a][b] = NAN;
          fc[1][1] = o->F[l][pidx(o, l, i, px, py)];
          /* d: 0:+x 1:-x 2:+y 3:-y */
          if (avail[1]) fc[1][0] = o->F[l][pidx(o, l, i, nbx[1], nby[1])];
          if (avail[0]) fc[1][2] = o->F[l][pidx(o, l, i, nbx[0], nby[0])];
          if (avail[3]) fc[0][1] = o->F[l][pidx(o, l, i, nbx[3], nby[3])];
          if (avail[2]) fc[2][1] = o->F[l][pidx(o, l, i, nbx[2], nby[2])];
          double ch[64];
          orc_split_block(r, (const double(*)[3])fc, ch);
          for (int b = 0; b < r; ++b)
            for (int a = 0; a < r; ++a) {
              o->F[l + 1][pidx(o, l + 1, i, px * r + a, py * r + b)] = ch[b * r + a];
              o->Fp[l + 1][pidx(o, l + 1, i, px * r + a, py * r + b)] = ch[b * r + a];
            }
        }
        for (int b = 0; b < r; ++b)
          for (int a = 0; a < r; ++a) o->pok[l + 1][cidx(o, l + 1, px * r + a, py * r + b)] = 0;
      }
  }
  /* 3. interfaces. The hand-off across the face of level-l cell P towards a
   *    level-(l+1) hole P + c_q reads population q of P at the last two
   *    level-l steps. Where that face existed before the regrid (P active at
   *    level l, P + c_q covered at level l+1) it is kept, with the history P
   *    has (merged and split cells have none). A face the regrid creates has
   *    no older sample on that face yet: its first hand-off has slope 0, as
   *    for any interface that appears (Sec. 3.2 step 3). */
  for (int l = 0; l + 1 < L; ++l)
    for (int py = 0; py < o->Ny[l]; ++py)
      for (int px = 0; px < o->Nx[l]; ++px) {
        size_t ci = cidx(o, l, px, py);
        if (!o->pok[l][ci]) continue;
        const int act_new = ncov[l][ci] && !ncov[l + 1][cidx(o, l + 1, px * r, py * r)];
        const int act_old = ocov[l][ci] && !ocov[l + 1][cidx(o, l + 1, px * r, py * r)];
        if (!act_new) continue;
        for (int q = 0; q < 4; ++q) {
          int hx = px + CX[q], hy = py + CY[q];
          if (!wrap(o, l, &hx, &hy)) continue;
          const size_t hc = cidx(o, l + 1, hx * r, hy * r);
          const int face_new = ncov[l + 1][hc];
          const int face_old = act_old && ocov[l + 1][hc];
          if (face_new && !face_old && o->mut != ORC_MUT_REGRID_NEW_FACE_HISTORY)
            o->pok[l][ci] &= (unsigned char)~(1u << q);
        }
      }
  /* 4. adopt the new coverage */
  for (int l = 0; l < L; ++l) {
    if (o->mut == ORC_MUT_REGRID_RESTART_ALL) memset(o->pok[l], 0, (size_t)o->Nx[l] * o->Ny[l]);
    memcpy(o->cov[l], ncov[l], (size_t)o->Nx[l] * o->Ny[l]);
    free(ncov[l]);
  }
  return 0;
}

/* The refinement sensor of eq. (amr-sigma) (Sec. 3.4) on the active cells of
 * level l: s_k = dx (div Q)_k / max_{x,alpha} |Q_{alpha,k}| as for eq.
 * (sensor-B) -- central differences 0.5 ((Qx_k(x+1) - Qx_k(x-1)) +
 * (Qy_k(y+1) - Qy_k(y-1))), a neighbour that is not an active cell of the
 * level replaced by the cell itself, the max over the active cells of every
 * level and both directions (s_k = 0 where it is 0) -- combined with the
 * max norm s = max_k |s_k|. out[Ny][Nx], 0 on inactive cells. */
int orc_flux_sensor(orc *o, int level, double *out) {
  int l = level;
  if (l < 0 || l >= o->nlev) return -1;
  sensor_qmax(o);
  const double *F = o->F[l];
  for (int y = 0; y < o->Ny[l]; ++y)
    for (int x = 0; x < o->Nx[l]; ++x) {
      out[cidx(o, l, x, y)] = 0.0;
      if (!active(o, l, x, y)) continue;
      double Qx[4][4], Qy[4][4];
      for (int d = 0; d < 4; ++d) {
        int xx = x + CX[d], yy = y + CY[d];
        if (!wrap(o, l, &xx, &yy) || !active(o, l, xx, yy)) {
          xx = x;
          yy = y;
        }
        double Wn[4];
        for (int k = 0; k < 4; ++k)
          Wn[k] = ((F[pidx(o, l, 0 * 4 + k, xx, yy)] + F[pidx(o, l, 1 * 4 + k, xx, yy)]) +
                   F[pidx(o, l, 2 * 4 + k, xx, yy)]) + F[pidx(o, l, 3 * 4 + k, xx, yy)];
        orc_flux(o->gamma, o->eos, o->eos_a, o->eos_b, Wn, Qx[d], Qy[d]);
      }
      double smax = 0.0;
      for (int k = 0; k < 4; ++k) {
        double dq = (Qx[0][k] - Qx[1][k]) + (Qy[2][k] - Qy[3][k]);
        double sk = o->qmax[k] > 0.0 ? (0.5 * dq) / o->qmax[k] : 0.0;
        if (o->mut == ORC_MUT_FLUX_SENSOR_RMS) { /* planted mistake: accumulate squares */
          smax += 0.25 * sk * sk;
          continue;
        }
        if (fabs(sk) > smax) smax = fabs(sk);
      }
      if (o->mut == ORC_MUT_FLUX_SENSOR_RMS) smax = sqrt(smax);
      out[cidx(o, l, x, y)] = smax;
    }
  return 0;
}

/* Refinement tags from eq. (amr-sigma): s > thr on active level-l cells. */
int orc_tag_flux(orc *o, int level, double thr, unsigned char *tags) {
  int l = level;
  if (l < 0 || l >= o->nlev) return -1;
  size_t nc = (size_t)o->Nx[l] * o->Ny[l];
  double *s = (double *)malloc(sizeof(double) * nc);
  if (!s) return -1;
  orc_flux_sensor(o, l, s);
  for (size_t i = 0; i < nc; ++i) tags[i] = (unsigned char)(s[i] > thr);
  free(s);
  return 0;
}

/* Density-gradient tag on active level-l cells: max over axes of
 * |rho(+) - rho(-)| / (2 rho) > thr; a neighbour that is not active at level
 * l (or lies outside a non-periodic domain) is replaced by the cell itself. */
int orc_tag(const orc *o, int level, double thr, unsigned char *tags) {
  int l = level;
  if (l < 0 || l >= o->nlev) return -1;
  for (int y = 0; y < o->Ny[l]; ++y)
    for (int x = 0; x < o->Nx[l]; ++x) {
      tags[cidx(o, l, x, y)] = 0;
      if (!active(o, l, x, y)) continue;
      double rho[4];
      const double *F = o->F[l];
      double rc = ((F[pidx(o, l, 0, x, y)] + F[pidx(o, l, 4, x, y)]) + F[pidx(o, l, 8, x, y)]) +
                  F[pidx(o, l, 12, x, y)];
      for (int d = 0; d < 4; ++d) {
        int nx_ = x + CX[d], ny_ = y + CY[d];
        if (wrap(o, l, &nx_, &ny_) && active(o, l, nx_, ny_))
          rho[d] = ((F[pidx(o, l, 0, nx_, ny_)] + F[pidx(o, l, 4, nx_, ny_)]) + F[pidx(o, l, 8, nx_, ny_)]) +
                   F[pidx(o, l, 12, nx_, ny_)];
        else
          rho[d] = rc;
      }
      double gx = fabs(rho[0] - rho[1]) / (2.0 * rc);
      double gy = fabs(rho[2] - rho[3]) / (2.0 * rc);
      if (o->mut == ORC_MUT_TAG_ONE_SIDED) { /* planted mistake */
        gx = fabs(rho[0] - rc) / (2.0 * rc);
        gy = fabs(rho[2] - rc) / (2.0 * rc);
      }
      double g = gx > gy ? gx : gy;
      tags[cidx(o, l, x, y)] = (unsigned char)(g > thr);
    }
  return 0;
}
