/*
 * Plain FP64 CPU oracle of the three-dimensional D3Q6 VLBM with conservative
 * local grid refinement -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this library. The product path never links it, and the two share no code.
 *
 * D3Q6: six populations +-c e_alpha (alpha = x, y, z), each carrying the five
 * conserved components W = (rho, rho u, rho v, rho w, E). What each part
 * follows (paper):
 *   equilibrium W/(2D) + c_i . Q / (2 c^2), D = 3     Sec. 2.2 eq. (num-equilibrium)
 *   transport then BGK relaxation                     Sec. 2.2 eq. (num-relaxation)
 *   sub-cycling with one link speed                   Sec. 3.2 step 1
 *   coarse-to-fine hand-off                           Sec. 3.2 eq. (1d-recon) and
 *       Sec. 3.3 eqs. (2d-recon-tanslope), (2d-recon), one face at a time: a
 *       ring cell faces r^2 fine cells, and each of the two tangential axes
 *       adds its own minmod-limited correction at the fine cell's offset;
 *   fine-to-coarse reflux                             Sec. 3.3 eq. (2d-reflux):
 *       the plain average of the r^2 face cells' values over the r sub-steps,
 *       a weight of 1 / r^3;
 *   conserved totals                                  Sec. 4.1.2, dx^3 weights.
 *
 * Representation: every level keeps dense arrays over the whole domain at its
 * own resolution; a cell is covered at level l when it lies in a level-l box,
 * active when covered and not covered at level l+1. Stored values are the
 * post-collision populations f*. The readings are those of the 2-D oracle:
 * the reflux books the values at the start of each fine sub-step, the first
 * cycle of an interface has no older coarse sample (prev := out), a tangential
 * slope needs both tangential neighbours active at the parent's level (else
 * 0), relaxation is f + 2 beta (feq - f), and a regrid keeps the temporal
 * reconstruction of every interface that exists before and after it (only
 * the faces it creates start flat). Ideal gas; sides are periodic, outflow
 * (zero gradient) or reflecting.
 */
#include "vlbm3_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define O3MAXL 6

static const int C3X[6] = {1, -1, 0, 0, 0, 0};
static const int C3Y[6] = {0, 0, 1, -1, 0, 0};
static const int C3Z[6] = {0, 0, 0, 0, 1, -1};

static char g_err3[256];
static void set_err3(const char *m) { snprintf(g_err3, sizeof g_err3, "%s", m); }
const char *orc3_error(void) { return g_err3; }

struct orc3 {
  int n0[3], r, nlev;
  double dx0, gamma, c, beta;
  int bc[6];
  int N[O3MAXL][3];
  double dx[O3MAXL];
  double *F[O3MAXL], *Fp[O3MAXL], *G[O3MAXL], *acc[O3MAXL];
  unsigned char *cov[O3MAXL];
  /* pok: per cell, bit q set when the cell's previous-step sample of
   * population q may serve as the hand-off's older coarse sample */
  unsigned char *pok[O3MAXL];
  double led[5], ledc[5];
  int mut;
};

int orc3_set_mutation(orc3 *o, int mut) {
  o->mut = mut;
  return 0;
}

static void kadd3(double *s, double *cmp, double v) {
  double t = *s + v;
  if (fabs(*s) >= fabs(v))
    *cmp += (*s - t) + v;
  else
    *cmp += (v - t) + *s;
  *s = t;
}

/* ------------------------------------------------------------------ */
/* Single-cell physics (Sec. 2.1-2.2)                                  */
/* ------------------------------------------------------------------ */
void orc3_flux(double gamma, const double W[5], double Qx[5], double Qy[5], double Qz[5]) {
  double rho = W[0], mx = W[1], my = W[2], mz = W[3], E = W[4];
  double u = mx / rho;
  double v = my / rho;
  double w = mz / rho;
  double p = (gamma - 1.0) * (E - 0.5 * ((mx * u + my * v) + mz * w));
  Qx[0] = mx;
  Qx[1] = mx * u + p;
  Qx[2] = my * u;
  Qx[3] = mz * u;
  Qx[4] = (E + p) * u;
  Qy[0] = my;
  Qy[1] = mx * v;
  Qy[2] = my * v + p;
  Qy[3] = mz * v;
  Qy[4] = (E + p) * v;
  Qz[0] = mz;
  Qz[1] = mx * w;
  Qz[2] = my * w;
  Qz[3] = mz * w + p;
  Qz[4] = (E + p) * w;
}

void orc3_feq(double gamma, double c, const double W[5], double f[30]) {
  double Q[3][5];
  orc3_flux(gamma, W, Q[0], Q[1], Q[2]);
  double h = 1.0 / (2.0 * c);
  for (int k = 0; k < 5; ++k) {
    double share = W[k] / 6.0;
    for (int a = 0; a < 3; ++a) {
      f[(2 * a) * 5 + k] = share + h * Q[a][k];
      f[(2 * a + 1) * 5 + k] = share - h * Q[a][k];
    }
  }
}

void orc3_collide(double gamma, double c, double beta, const double g[30], double fstar[30]) {
  double W[5], feq[30];
  for (int k = 0; k < 5; ++k)
    W[k] = ((((g[0 * 5 + k] + g[1 * 5 + k]) + g[2 * 5 + k]) + g[3 * 5 + k]) + g[4 * 5 + k]) +
           g[5 * 5 + k];
  orc3_feq(gamma, c, W, feq);
  double tb = 2.0 * beta;
  for (int i = 0; i < 30; ++i) fstar[i] = g[i] + tb * (feq[i] - g[i]);
}

static double minmod3(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* ------------------------------------------------------------------ */
/* Grid helpers                                                        */
/* ------------------------------------------------------------------ */
static size_t ncell(const orc3 *o, int l) { return (size_t)o->N[l][0] * o->N[l][1] * o->N[l][2]; }
static size_t cid(const orc3 *o, int l, int x, int y, int z) {
  return ((size_t)z * o->N[l][1] + y) * o->N[l][0] + x;
}
static size_t pid(const orc3 *o, int l, int qk, int x, int y, int z) {
  return (size_t)qk * ncell(o, l) + cid(o, l, x, y, z);
}

/* Wrap (x,y,z) at level l by the periodic sides; 0 if outside the domain. */
static int wrap3(const orc3 *o, int l, int p[3]) {
  for (int a = 0; a < 3; ++a) {
    int n = o->N[l][a];
    if (p[a] < 0 || p[a] >= n) {
      if (o->bc[2 * a] != ORC3_BC_PERIODIC) return 0;
      p[a] = (p[a] % n + n) % n;
    }
  }
  return 1;
}
static int covered3(const orc3 *o, int l, int x, int y, int z) {
  if (l >= o->nlev) return 0;
  return o->cov[l][cid(o, l, x, y, z)];
}
static int active3(const orc3 *o, int l, int x, int y, int z) {
  if (!covered3(o, l, x, y, z)) return 0;
  if (l + 1 < o->nlev && o->cov[l + 1][cid(o, l + 1, x * o->r, y * o->r, z * o->r)]) return 0;
  return 1;
}

orc3 *orc3_new(int nx0, int ny0, int nz0, double dx0, int r, int nlev, double gamma, double c,
               double beta, const int bc[6]) {
  if (nx0 < 1 || ny0 < 1 || nz0 < 1 || r < 1 || nlev < 1 || nlev > O3MAXL || !(c > 0.0)) {
    set_err3("orc3_new: bad arguments");
    return NULL;
  }
  for (int a = 0; a < 3; ++a)
    if ((bc[2 * a] == ORC3_BC_PERIODIC) != (bc[2 * a + 1] == ORC3_BC_PERIODIC)) {
      set_err3("orc3_new: periodic sides must come in pairs");
      return NULL;
    }
  orc3 *o = (orc3 *)calloc(1, sizeof(orc3));
  o->n0[0] = nx0;
  o->n0[1] = ny0;
  o->n0[2] = nz0;
  o->r = r;
  o->nlev = nlev;
  o->dx0 = dx0;
  o->gamma = gamma;
  o->c = c;
  o->beta = beta;
  for (int s = 0; s < 6; ++s) o->bc[s] = bc[s];
  long scale = 1;
  for (int l = 0; l < nlev; ++l) {
    for (int a = 0; a < 3; ++a) o->N[l][a] = (int)(o->n0[a] * scale);
    o->dx[l] = dx0 / (double)scale;
    size_t nc = ncell(o, l);
    o->F[l] = (double *)calloc(30 * nc, sizeof(double));
    o->Fp[l] = (double *)calloc(30 * nc, sizeof(double));
    o->G[l] = (double *)calloc(30 * nc, sizeof(double));
    o->acc[l] = (double *)calloc(30 * nc, sizeof(double));
    o->cov[l] = (unsigned char *)calloc(nc, 1);
    o->pok[l] = (unsigned char *)calloc(nc, 1);
    if (!o->F[l] || !o->Fp[l] || !o->G[l] || !o->acc[l] || !o->cov[l] || !o->pok[l]) {
      set_err3("orc3_new: out of memory");
      orc3_free(o);
      return NULL;
    }
    scale *= r;
  }
  memset(o->cov[0], 1, ncell(o, 0));
  return o;
}

void orc3_free(orc3 *o) {
  if (!o) return;
  for (int l = 0; l < o->nlev; ++l) {
    free(o->F[l]);
    free(o->Fp[l]);
    free(o->G[l]);
    free(o->acc[l]);
    free(o->cov[l]);
    free(o->pok[l]);
  }
  free(o);
}

int orc3_shape(const orc3 *o, int level, int shape[3]) {
  if (level < 0 || level >= o->nlev) return -1;
  for (int a = 0; a < 3; ++a) shape[a] = o->N[level][a];
  return 0;
}

/* Coverage of every level from a box list into cov[], with the checks of
 * orc3_set_boxes; 0 on success. */
static int build_cov3(orc3 *o, const int *boxes, int nboxes, unsigned char **cov) {
  for (int l = 0; l < o->nlev; ++l) memset(cov[l], l == 0 ? 1 : 0, ncell(o, l));
  for (int b = 0; b < nboxes; ++b) {
    const int *B = boxes + 7 * b;
    int l = B[0];
    if (l < 1 || l >= o->nlev) {
      set_err3("box level outside 1..nlev-1");
      return -1;
    }
    for (int a = 0; a < 3; ++a) {
      if (B[4 + a] <= 0 || B[1 + a] < 0 || B[1 + a] + B[4 + a] > o->N[l][a]) {
        set_err3("box outside its level's domain");
        return -1;
      }
      if (B[1 + a] % o->r || B[4 + a] % o->r) {
        set_err3("box not aligned to whole parent cells");
        return -1;
      }
    }
    for (int z = B[3]; z < B[3] + B[6]; ++z)
      for (int y = B[2]; y < B[2] + B[5]; ++y)
        for (int x = B[1]; x < B[1] + B[4]; ++x) cov[l][cid(o, l, x, y, z)] = 1;
  }
  /* proper nesting: the parent of every covered cell and its six face
   * neighbours are covered one level up */
  for (int l = 1; l < o->nlev; ++l)
    for (int z = 0; z < o->N[l][2]; ++z)
      for (int y = 0; y < o->N[l][1]; ++y)
        for (int x = 0; x < o->N[l][0]; ++x) {
          if (!cov[l][cid(o, l, x, y, z)]) continue;
          for (int d = -1; d < 6; ++d) {
            int p[3] = {x / o->r + (d < 0 ? 0 : C3X[d]), y / o->r + (d < 0 ? 0 : C3Y[d]),
                        z / o->r + (d < 0 ? 0 : C3Z[d])};
            if (!wrap3(o, l - 1, p)) continue;
            if (!cov[l - 1][cid(o, l - 1, p[0], p[1], p[2])]) {
              set_err3("hierarchy not properly nested");
              return -1;
            }
          }
        }
  return 0;
}

int orc3_set_boxes(orc3 *o, const int *boxes, int nboxes) {
  if (build_cov3(o, boxes, nboxes, o->cov) != 0) {
    for (int m = 1; m < o->nlev; ++m) memset(o->cov[m], 0, ncell(o, m));
    return -1;
  }
  for (int l = 0; l < o->nlev; ++l) memset(o->pok[l], 0, ncell(o, l));
  return 0;
}

int orc3_active_mask(const orc3 *o, int level, unsigned char *mask) {
  if (level < 0 || level >= o->nlev) return -1;
  for (int z = 0; z < o->N[level][2]; ++z)
    for (int y = 0; y < o->N[level][1]; ++y)
      for (int x = 0; x < o->N[level][0]; ++x)
        mask[cid(o, level, x, y, z)] = (unsigned char)active3(o, level, x, y, z);
  return 0;
}

/* Initial populations are the equilibrium of U. */
int orc3_set_state(orc3 *o, int level, const double *U) {
  if (level < 0 || level >= o->nlev) return -1;
  size_t nc = ncell(o, level);
  for (size_t i = 0; i < nc; ++i) {
    if (!o->cov[level][i]) continue;
    double W[5], f[30];
    for (int k = 0; k < 5; ++k) W[k] = U[k * nc + i];
    orc3_feq(o->gamma, o->c, W, f);
    for (int j = 0; j < 30; ++j) o->F[level][j * nc + i] = o->Fp[level][j * nc + i] = f[j];
    o->pok[level][i] = 0;
  }
  for (int k = 0; k < 5; ++k) o->led[k] = o->ledc[k] = 0.0;
  return 0;
}

int orc3_set_pop(orc3 *o, int level, const double *Fin) {
  if (level < 0 || level >= o->nlev) return -1;
  size_t nc = ncell(o, level);
  for (size_t i = 0; i < nc; ++i) {
    if (!o->cov[level][i]) continue;
    for (int j = 0; j < 30; ++j) o->F[level][j * nc + i] = o->Fp[level][j * nc + i] = Fin[j * nc + i];
    o->pok[level][i] = 0;
  }
  for (int k = 0; k < 5; ++k) o->led[k] = o->ledc[k] = 0.0;
  return 0;
}

int orc3_get_pop(const orc3 *o, int level, double *Fout) {
  if (level < 0 || level >= o->nlev) return -1;
  size_t nc = ncell(o, level);
  for (int z = 0; z < o->N[level][2]; ++z)
    for (int y = 0; y < o->N[level][1]; ++y)
      for (int x = 0; x < o->N[level][0]; ++x) {
        size_t i = cid(o, level, x, y, z);
        int act = active3(o, level, x, y, z);
        for (int j = 0; j < 30; ++j) Fout[j * nc + i] = act ? o->F[level][j * nc + i] : NAN;
      }
  return 0;
}

int orc3_get_state(const orc3 *o, int level, double *U) {
  if (level < 0 || level >= o->nlev) return -1;
  size_t nc = ncell(o, level);
  const double *F = o->F[level];
  for (int z = 0; z < o->N[level][2]; ++z)
    for (int y = 0; y < o->N[level][1]; ++y)
      for (int x = 0; x < o->N[level][0]; ++x) {
        size_t i = cid(o, level, x, y, z);
        int act = active3(o, level, x, y, z);
        for (int k = 0; k < 5; ++k)
          U[k * nc + i] = act ? ((((F[(0 * 5 + k) * nc + i] + F[(1 * 5 + k) * nc + i]) +
                                   F[(2 * 5 + k) * nc + i]) + F[(3 * 5 + k) * nc + i]) +
                                 F[(4 * 5 + k) * nc + i]) + F[(5 * 5 + k) * nc + i]
                              : NAN;
      }
  return 0;
}

/* ------------------------------------------------------------------ */
/* One time step of level l (transport, then relaxation)               */
/* ------------------------------------------------------------------ */

/* Inbound population q at a boundary cell through the side it enters by.
 * Outflow copies the cell's own post-collision q (zero gradient); reflect
 * mirrors the outgoing population with the normal momentum negated. */
static void boundary3(const orc3 *o, int l, int side, int q, int x, int y, int z, double v[5]) {
  const double *F = o->F[l];
  if (o->bc[side] == ORC3_BC_OUTFLOW) {
    for (int k = 0; k < 5; ++k) v[k] = F[pid(o, l, q * 5 + k, x, y, z)];
  } else {
    int qo = q ^ 1, kn = 1 + q / 2;
    for (int k = 0; k < 5; ++k) {
      double w = F[pid(o, l, qo * 5 + k, x, y, z)];
      v[k] = (k == kn && o->mut != ORC3_MUT_WALL_NO_FLIP) ? -w : w;
    }
  }
}

/* Coarse-to-fine hand-off for fine cell p (level l) pulling q from s, which
 * lies in the coarser region: temporal term, then one tangential correction
 * per tangential axis, in axis order. */
static void recon3(const orc3 *o, int l, int q, int kstep, const int p[3], const int s[3],
                   double v[5]) {
  int lp = l - 1, r = o->r, n = q / 2;
  int P[3] = {s[0] / r, s[1] / r, s[2] / r};
  const double *F = o->F[lp], *Fp = o->Fp[lp];
  int has_prev = (o->pok[lp][cid(o, lp, P[0], P[1], P[2])] >> q) & 1;
  int ta[2], nt = 0;
  for (int a = 0; a < 3; ++a)
    if (a != n) ta[nt++] = a;
  int have[2];
  size_t im[2], ip[2];
  double bj[2];
  for (int t = 0; t < 2; ++t) {
    int a = ta[t];
    int m[3] = {P[0], P[1], P[2]}, pp[3] = {P[0], P[1], P[2]};
    m[a] -= 1;
    pp[a] += 1;
    have[t] = wrap3(o, lp, m) && wrap3(o, lp, pp) && active3(o, lp, m[0], m[1], m[2]) &&
              active3(o, lp, pp[0], pp[1], pp[2]);
    im[t] = have[t] ? cid(o, lp, m[0], m[1], m[2]) : 0;
    ip[t] = have[t] ? cid(o, lp, pp[0], pp[1], pp[2]) : 0;
    int j = p[a] - r * P[a];
    bj[t] = (double)(2 * j - r + 1) / (double)(2 * r);
  }
  if (o->mut == ORC3_MUT_TAN_OFFSETS_SWAPPED) {
    double b0 = bj[0];
    bj[0] = bj[1];
    bj[1] = b0;
  }
  double ak = (double)(2 * kstep - r - 1) / (double)(2 * r);
  size_t nc = ncell(o, lp), ci = cid(o, lp, P[0], P[1], P[2]);
  for (int k = 0; k < 5; ++k) {
    size_t pl = (size_t)(q * 5 + k) * nc;
    double out = F[pl + ci];
    double prev = has_prev ? Fp[pl + ci] : out;
    double val = out + (out - prev) * ak;
    for (int t = 0; t < 2; ++t) {
      double sigma = have[t] ? minmod3(out - F[pl + im[t]], F[pl + ip[t]] - out) : 0.0;
      if (o->mut == ORC3_MUT_TAN_SLOPE_SIGN) sigma = -sigma;
      val = val + sigma * bj[t];
    }
    v[k] = val;
  }
}

static void ledger3(orc3 *o, double w, const double v[5], double sign) {
  for (int k = 0; k < 5; ++k) kadd3(&o->led[k], &o->ledc[k], sign * (w * v[k]));
}

static void advance3(orc3 *o, int l, int kstep) {
  const int r = o->r;
  const double w3 = o->dx[l] * o->dx[l] * o->dx[l];
  const int *N = o->N[l];
  double *F = o->F[l];
  /* values leaving level l during this step (those at its start): the
   * parent's reflux accumulator, or the boundary ledger at a domain side */
  for (int z = 0; z < N[2]; ++z)
    for (int y = 0; y < N[1]; ++y)
      for (int x = 0; x < N[0]; ++x) {
        if (!active3(o, l, x, y, z)) continue;
        for (int q = 0; q < 6; ++q) {
          int d[3] = {x + C3X[q], y + C3Y[q], z + C3Z[q]};
          double v[5];
          for (int k = 0; k < 5; ++k) v[k] = F[pid(o, l, q * 5 + k, x, y, z)];
          if (!wrap3(o, l, d)) {
            ledger3(o, w3, v, -1.0);
            continue;
          }
          if (l >= 1 && !covered3(o, l, d[0], d[1], d[2]))
            for (int k = 0; k < 5; ++k)
              o->acc[l - 1][pid(o, l - 1, q * 5 + k, d[0] / r, d[1] / r, d[2] / r)] += v[k];
        }
      }
  /* transport (exact shift) into G with interface and boundary fills */
  double *G = o->G[l];
  const double r3 = o->mut == ORC3_MUT_REFLUX_R2 ? (double)(r * r) : (double)(r * r * r);
  for (int z = 0; z < N[2]; ++z)
    for (int y = 0; y < N[1]; ++y)
      for (int x = 0; x < N[0]; ++x) {
        if (!active3(o, l, x, y, z)) continue;
        for (int q = 0; q < 6; ++q) {
          int s[3] = {x - C3X[q], y - C3Y[q], z - C3Z[q]};
          double v[5];
          if (!wrap3(o, l, s)) {
            /* +alpha (q = 2a) enters through the -alpha side (side 2a), -alpha through +alpha */
            boundary3(o, l, q, q, x, y, z, v);
            ledger3(o, w3, v, +1.0);
          } else if (l + 1 < o->nlev && o->cov[l + 1][cid(o, l + 1, s[0] * r, s[1] * r, s[2] * r)]) {
            for (int k = 0; k < 5; ++k) v[k] = o->acc[l][pid(o, l, q * 5 + k, x, y, z)] / r3;
          } else if (covered3(o, l, s[0], s[1], s[2])) {
            for (int k = 0; k < 5; ++k) v[k] = F[pid(o, l, q * 5 + k, s[0], s[1], s[2])];
          } else {
            int p[3] = {x, y, z};
            recon3(o, l, q, kstep, p, s, v);
          }
          for (int k = 0; k < 5; ++k) G[pid(o, l, q * 5 + k, x, y, z)] = v[k];
        }
      }
  /* relaxation, cell by cell */
  size_t nc = ncell(o, l);
  for (int z = 0; z < N[2]; ++z)
    for (int y = 0; y < N[1]; ++y)
      for (int x = 0; x < N[0]; ++x) {
        if (!active3(o, l, x, y, z)) continue;
        size_t i = cid(o, l, x, y, z);
        double g[30], fs[30];
        for (int j = 0; j < 30; ++j) g[j] = G[j * nc + i];
        orc3_collide(o->gamma, o->c, o->beta, g, fs);
        for (int j = 0; j < 30; ++j) G[j * nc + i] = fs[j];
      }
  double *old = o->Fp[l];
  o->Fp[l] = o->F[l];
  o->F[l] = o->G[l];
  o->G[l] = old;
  for (int z = 0; z < N[2]; ++z)
    for (int y = 0; y < N[1]; ++y)
      for (int x = 0; x < N[0]; ++x)
        o->pok[l][cid(o, l, x, y, z)] = active3(o, l, x, y, z) ? 0x3F : 0;
}

/* Level l+1 takes r steps inside each step of level l, then level l steps. */
static void cycle3(orc3 *o, int l, int kstep) {
  if (l + 1 < o->nlev) {
    memset(o->acc[l], 0, 30 * ncell(o, l) * sizeof(double));
    for (int kk = 1; kk <= o->r; ++kk) cycle3(o, l + 1, kk);
  }
  advance3(o, l, kstep);
}

int orc3_advance(orc3 *o, int ncoarse) {
  for (int n = 0; n < ncoarse; ++n) cycle3(o, 0, 1);
  return 0;
}

/* T_k = sum_l dx_l^3 sum_active sum_q f_{q,k}, compensated. */
void orc3_totals(const orc3 *o, double T[5], double ledger[5]) {
  for (int k = 0; k < 5; ++k) {
    double s = 0.0, cs = 0.0;
    for (int l = 0; l < o->nlev; ++l) {
      double sl = 0.0, cl = 0.0;
      size_t nc = ncell(o, l);
      for (int z = 0; z < o->N[l][2]; ++z)
        for (int y = 0; y < o->N[l][1]; ++y)
          for (int x = 0; x < o->N[l][0]; ++x) {
            if (!active3(o, l, x, y, z)) continue;
            size_t i = cid(o, l, x, y, z);
            for (int q = 0; q < 6; ++q) kadd3(&sl, &cl, o->F[l][(size_t)(q * 5 + k) * nc + i]);
          }
      kadd3(&s, &cs, o->dx[l] * o->dx[l] * o->dx[l] * (sl + cl));
    }
    T[k] = s + cs;
    if (ledger) ledger[k] = o->led[k] + o->ledc[k];
  }
}

/* ------------------------------------------------------------------ */
/* Regrid: merge exiting cells (finest level first), then split         */
/* entering cells (coarsest level first) -- Sec. 3.4, eqs. (amr-merge),  */
/* (amr-slope), (amr-split) with D = 3                                   */
/* ------------------------------------------------------------------ */

/* eq. (amr-split), D = 3: child (a, b, g) along (x, y, z) of a parent with
 * value fi and minmod slopes s[3] gets fi + s_x xi_a + s_y xi_b + s_z xi_g,
 * added in axis order. */
static double split3_value(int r, double fi, const double s[3], int a, int b, int g) {
  double xa = (double)(2 * a - r + 1) / (double)(2 * r);
  double xb = (double)(2 * b - r + 1) / (double)(2 * r);
  double xg = (double)(2 * g - r + 1) / (double)(2 * r);
  double v = fi + s[0] * xa;
  v = v + s[1] * xb;
  return v + s[2] * xg;
}

int orc3_regrid(orc3 *o, const int *boxes, int nboxes) {
  const int L = o->nlev, r = o->r;
  unsigned char *ncov[O3MAXL];
  for (int l = 0; l < L; ++l) ncov[l] = (unsigned char *)malloc(ncell(o, l));
  if (build_cov3(o, boxes, nboxes, ncov) != 0) {
    for (int l = 0; l < L; ++l) free(ncov[l]);
    return -1;
  }
  unsigned char **ocov = o->cov;
  /* 1. merges, finest level first (eq. amr-merge): a parent whose r^3
   *    children leave level l gets their plain average, summed in raster
   *    order (z, y, x); both time levels get it. */
  for (int l = L - 1; l >= 1; --l) {
    const int *Np = o->N[l - 1];
    for (int pz = 0; pz < Np[2]; ++pz)
      for (int py = 0; py < Np[1]; ++py)
        for (int px = 0; px < Np[0]; ++px) {
          size_t c0 = cid(o, l, px * r, py * r, pz * r);
          if (!ocov[l][c0] || ncov[l][c0]) continue;
          size_t pc = cid(o, l - 1, px, py, pz);
          for (int i = 0; i < 30; ++i) {
            double sum = 0.0;
            for (int g = 0; g < r; ++g)
              for (int b = 0; b < r; ++b)
                for (int a = 0; a < r; ++a)
                  sum += o->F[l][pid(o, l, i, px * r + a, py * r + b, pz * r + g)];
            double m = sum / (o->mut == ORC3_MUT_MERGE_R2 ? (double)(r * r) : (double)(r * r * r));
            o->F[l - 1][(size_t)i * ncell(o, l - 1) + pc] = m;
            o->Fp[l - 1][(size_t)i * ncell(o, l - 1) + pc] = m;
          }
          o->pok[l - 1][pc] = 0;
        }
  }
  /* 2. splits, coarsest level first (eqs. amr-slope, amr-split): a slope
   *    neighbour must be covered at level l in the new hierarchy and hold
   *    data (not a hole before and after). */
  for (int l = 0; l + 1 < L; ++l) {
    const int *Np = o->N[l];
    for (int pz = 0; pz < Np[2]; ++pz)
      for (int py = 0; py < Np[1]; ++py)
        for (int px = 0; px < Np[0]; ++px) {
          size_t c0 = cid(o, l + 1, px * r, py * r, pz * r);
          if (!ncov[l + 1][c0] || ocov[l + 1][c0]) continue;
          size_t nb[6];
          int avail[6];
          for (int d = 0; d < 6; ++d) {
            int q[3] = {px + C3X[d], py + C3Y[d], pz + C3Z[d]};
            avail[d] = wrap3(o, l, q);
            if (avail[d]) {
              nb[d] = cid(o, l, q[0], q[1], q[2]);
              int persistent_hole = 0;
              if (l + 1 < L) {
                size_t cc = cid(o, l + 1, q[0] * r, q[1] * r, q[2] * r);
                persistent_hole = ocov[l + 1][cc] && ncov[l + 1][cc];
              }
              avail[d] = ncov[l][nb[d]] && !persistent_hole;
            }
          }
          size_t pc = cid(o, l, px, py, pz), ncl = ncell(o, l);
          for (int i = 0; i < 30; ++i) {
            const double *F = o->F[l] + (size_t)i * ncl;
            double fi = F[pc], sl[3];
            for (int a = 0; a < 3; ++a)
              sl[a] = (avail[2 * a] && avail[2 * a + 1]) ? minmod3(fi - F[nb[2 * a + 1]], F[nb[2 * a]] - fi) : 0.0;
            if (o->mut == ORC3_MUT_SPLIT_SLOPE_SIGN)
              for (int a = 0; a < 3; ++a) sl[a] = -sl[a];
            for (int g = 0; g < r; ++g)
              for (int b = 0; b < r; ++b)
                for (int a = 0; a < r; ++a) {
                  size_t ci = pid(o, l + 1, i, px * r + a, py * r + b, pz * r + g);
                  double v = split3_value(r, fi, sl, a, b, g);
                  o->F[l + 1][ci] = v;
                  o->Fp[l + 1][ci] = v;
                }
          }
          for (int g = 0; g < r; ++g)
            for (int b = 0; b < r; ++b)
              for (int a = 0; a < r; ++a)
                o->pok[l + 1][cid(o, l + 1, px * r + a, py * r + b, pz * r + g)] = 0;
        }
  }
  /* 3. interfaces: a face of level-l cell P towards a level-(l+1) hole P + c_q
   *    that existed before the regrid keeps P's history of population q (the
   *    reconstruction runs unmodified there, Sec. 3.4); a face the regrid
   *    creates starts flat (no older sample on that face). */
  for (int l = 0; l + 1 < L; ++l) {
    const int *Np = o->N[l];
    for (int pz = 0; pz < Np[2]; ++pz)
      for (int py = 0; py < Np[1]; ++py)
        for (int px = 0; px < Np[0]; ++px) {
          size_t ci = cid(o, l, px, py, pz);
          if (!o->pok[l][ci] || !ncov[l][ci]) continue;
          size_t ch = cid(o, l + 1, px * r, py * r, pz * r);
          if (ncov[l + 1][ch]) continue;
          const int act_old = ocov[l][ci] && !ocov[l + 1][ch];
          for (int q = 0; q < 6; ++q) {
            int h[3] = {px + C3X[q], py + C3Y[q], pz + C3Z[q]};
            if (!wrap3(o, l, h)) continue;
            size_t hc = cid(o, l + 1, h[0] * r, h[1] * r, h[2] * r);
            if (ncov[l + 1][hc] && !(act_old && ocov[l + 1][hc]) && o->mut != ORC3_MUT_REGRID_NEW_FACE_HISTORY)
              o->pok[l][ci] &= (unsigned char)~(1u << q);
          }
        }
  }
  /* 4. adopt the new coverage */
  for (int l = 0; l < L; ++l) {
    if (o->mut == ORC3_MUT_REGRID_RESTART_ALL) memset(o->pok[l], 0, ncell(o, l));
    memcpy(o->cov[l], ncov[l], ncell(o, l));
    free(ncov[l]);
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Refinement tags (Sec. 3.4, density-gradient variant)               */
/* ------------------------------------------------------------------ */

static double rho_at(const orc3 *o, int l, int x, int y, int z) {
  const double *F = o->F[l];
  const size_t nc = ncell(o, l), i = cid(o, l, x, y, z);
  return ((((F[0 * nc + i] + F[5 * nc + i]) + F[10 * nc + i]) + F[15 * nc + i]) + F[20 * nc + i]) +
         F[25 * nc + i];
}

int orc3_tag(const orc3 *o, int level, double thr, unsigned char *tags) {
  const int l = level;
  if (l < 0 || l >= o->nlev) return -1;
  for (int z = 0; z < o->N[l][2]; ++z)
    for (int y = 0; y < o->N[l][1]; ++y)
      for (int x = 0; x < o->N[l][0]; ++x) {
        const size_t i = cid(o, l, x, y, z);
        tags[i] = 0;
        if (!active3(o, l, x, y, z)) continue;
        const double rc = rho_at(o, l, x, y, z);
        double g = 0.0;
        for (int a = 0; a < 3; ++a) {
          double side[2];
          for (int s = 0; s < 2; ++s) {
            int p[3] = {x, y, z};
            p[a] += s == 0 ? 1 : -1;
            side[s] = (wrap3(o, l, p) && active3(o, l, p[0], p[1], p[2])) ? rho_at(o, l, p[0], p[1], p[2]) : rc;
          }
          const double ga = fabs(side[0] - side[1]) / (2.0 * rc);
          if (ga > g) g = ga;
        }
        tags[i] = (unsigned char)(g > thr);
      }
  return 0;
}
