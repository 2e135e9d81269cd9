/*
 * vlbm.h -- C ABI of libvlbm, the MI355X (gfx950) implementation of the
 * vectorial lattice Boltzmann method (VLBM) for the 2-D compressible Euler
 * equations with conservative, sub-cycled local grid refinement.
 *
 * Method (Hosseini, Straessle, Karlin, "Conservative local grid refinement for
 * the vectorial lattice Boltzmann method"):
 *   - D2Q4 vectorial populations f_q in R^4, q in {+x, -x, +y, -y}, carrying
 *     W = (rho, rho u, rho v, rho E); equilibrium of Sec. 2.2 eq.
 *     (num-equilibrium), exact streaming and BGK relaxation eq.
 *     (num-relaxation), ideal-gas pressure p = (gamma-1)(E - |m|^2/(2 rho)).
 *   - refinement ratio r, one link speed c on every level (Sec. 3.2 step 1);
 *     level l advances r steps of dt_l = dx_l / c per step of level l-1.
 *   - coarse-to-fine ghost populations from the mean-preserving temporal
 *     reconstruction with the minmod tangential slope (Sec. 3.3, eqs.
 *     2d-recon-tanslope and 2d-recon); fine-to-coarse populations from the
 *     reflux average over r fine cells and r sub-steps (eq. 2d-reflux).
 *   - regridding by merge (eq. amr-merge) and minmod split (eqs. amr-slope,
 *     amr-split) (Sec. 3.4).
 *
 * Conventions
 *   population index q: 0:+x 1:-x 2:+y 3:-y;  component k: 0:rho 1:rho u 2:rho v 3:rho E
 *   domain sides: 0:west (x-) 1:east (x+) 2:south (y-) 3:north (y+)
 *   level l has Nx_l = nx0 r^l by Ny_l = ny0 r^l cells of size dx_l = dx0 / r^l.
 *   A box {level, i0, j0, nx, ny} covers level-l cells [i0, i0+nx) x [j0, j0+ny);
 *   i0, j0, nx, ny must be multiples of r, and every covered cell's parent must
 *   have its four neighbours covered at level l-1 (proper nesting; neighbours
 *   outside a non-periodic side are exempt). Boxes of one level may touch or
 *   overlap (their union counts). A cell is ACTIVE on level l when covered at
 *   l and not covered at l+1; only active cells are advanced and counted.
 *   Host arrays are row-major with x fastest: U[4][ny][ld], F[16][ny][ld]
 *   with plane index q*4+k.
 *
 * Ownership and errors
 *   Every call returns a vlbm_status and never throws across the ABI. Host
 *   pointers are owned by the caller and used only during the call. Device
 *   memory is suballocated from a caller-bound pool (vlbm_bind_pool) or, when
 *   none is bound, allocated by the library; vlbm_destroy releases it. Table
 *   uploads go through a pinned host staging area of the context (4-64 MB,
 *   grown on demand, freed by vlbm_destroy). Host work of hierarchy changes
 *   (coverage, tile and task lists) runs on a pool of worker threads shared by
 *   every context of the process. Work is
 *   issued on the HIP stream given at creation (NULL: the default stream);
 *   vlbm_advance returns before the GPU finishes, every call that returns data
 *   to the host synchronises the stream first. A context must not be used from
 *   two host threads at once. vlbm_last_error() describes the last failure on
 *   the calling thread.
 */
#ifndef VLBM_H
#define VLBM_H

#define VLBM_MAX_LEVELS 8 /* levels of a hierarchy, level 0 included */
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vlbm_ctx vlbm_ctx;

typedef enum {
  VLBM_OK = 0,
  VLBM_EINVAL = -1,     /* bad argument */
  VLBM_ENOMEM = -2,     /* device pool or host allocation exhausted */
  VLBM_ENEST = -3,      /* hierarchy not properly nested or misaligned */
  VLBM_EUNSTABLE = -4,  /* rho <= 0, p <= 0 or NaN found by vlbm_check_health */
  VLBM_EDEVICE = -5,    /* a HIP runtime call failed */
  VLBM_ESTATE = -6      /* call out of order (e.g. advance before set_hierarchy) */
} vlbm_status;

enum { VLBM_BC_PERIODIC = 0, VLBM_BC_OUTFLOW = 1, VLBM_BC_REFLECT = 2, VLBM_BC_INFLOW = 3 };
enum { VLBM_FP64 = 0, VLBM_FP32 = 1, VLBM_FP32_STORAGE = 2 };
/* Equations of state p(rho, rho e), rho e = E - (m_x^2 + m_y^2) / (2 rho)
 * (Sec. 2.1 leaves the EOS generic; the coupling is EOS-blind):
 *   IDEAL      (gamma - 1) rho e
 *   STIFFENED  (gamma - 1) rho e - gamma a
 *   VDW        ((gamma - 1) (rho e + a rho^2)) / (1 - b rho) - a rho^2 */
enum { VLBM_EOS_IDEAL = 0, VLBM_EOS_STIFFENED = 1, VLBM_EOS_VDW = 2 };

/* Problem parameters (the paper's problem statement: base grid, ratio, EOS,
 * relaxation, link speed; Sec. 2.2 and 3.2).
 *   bc: per side. Periodic must be set on both sides of an axis. Outflow
 *       copies the edge cell's own post-collision inbound population; reflect
 *       returns the outgoing population with the normal momentum negated;
 *       inflow injects f^eq(w_inflow[side]).
 *   precision: VLBM_FP64 stores and relaxes populations in FP64;
 *       VLBM_FP32 stores and relaxes them in FP32 while the reconstruction,
 *       the reflux accumulators, the boundary ledger and the totals stay FP64;
 *       VLBM_FP32_STORAGE stores them in FP32 (same bytes as VLBM_FP32) but
 *       evaluates the relaxation in FP64, rounding once per stored value.
 *   beta in [0, 1] (0 switches relaxation off: pure streaming). */
typedef struct {
  int nx0, ny0;
  double dx0;
  int bc[4];
  double w_inflow[4][4];
  double gamma, c, beta;
  int r;
  int max_levels; /* number of levels including level 0, 1..8 */
  int precision;
  int eos;        /* VLBM_EOS_*; a zeroed struct is an ideal gas */
  double eos_a, eos_b; /* EOS constants a and b (b >= 0) */
} vlbm_params;

typedef struct {
  int level, i0, j0, nx, ny;
} vlbm_box;

/* Create a context. stream is a hipStream_t (NULL: default stream). */
vlbm_status vlbm_create(const vlbm_params *params, void *stream, vlbm_ctx **out);

/* Release all device memory the context owns and free it. NULL is a no-op. */
void vlbm_destroy(vlbm_ctx *ctx);

/* Suballocate every later device allocation of ctx from [dev, dev + bytes),
 * a device region owned by the caller (e.g. a torch tensor) that must outlive
 * the context. Must precede vlbm_set_hierarchy. */
vlbm_status vlbm_bind_pool(vlbm_ctx *ctx, void *dev, size_t bytes);

/* A caller's device allocator: alloc returns a block of at least `bytes`
 * bytes, 256-byte aligned, usable on the context's stream (NULL when it cannot:
 * the call that needed it returns VLBM_ENOMEM); release returns a block the
 * library has finished with (the context's stream has completed all work on
 * it). Both are called on the thread that made the library call. */
typedef void *(*vlbm_alloc_fn)(size_t bytes, void *user);
typedef void (*vlbm_free_fn)(void *ptr, void *user);

/* Take every later device allocation of ctx from the caller's allocator
 * (e.g. PyTorch's caching allocator on the context's stream), so that the
 * caller is the only allocator and a hierarchy can grow through regrids
 * without a preset pool size. Must precede vlbm_set_hierarchy and cannot be
 * combined with vlbm_bind_pool (VLBM_ESTATE). vlbm_destroy releases every
 * block still held. */
vlbm_status vlbm_bind_allocator(vlbm_ctx *ctx, vlbm_alloc_fn alloc, vlbm_free_fn release, void *user);

/* Device bytes a context with these parameters and boxes needs (admission
 * control, and the size of a pool that holds it): both time levels of every
 * frame, status and row tables, list and slot estimates, and the staging of
 * a whole-level read. Not included: the adaptive relaxation's planes
 * (vlbm_set_sensor) and frames that later regrids grow. Pure host
 * computation. */
size_t vlbm_footprint_bytes(const vlbm_params *params, const vlbm_box *boxes, int nboxes);

/* Install a static hierarchy (level-0 always covers the domain). Discards any
 * previous state; populations are undefined until vlbm_set_state. */
vlbm_status vlbm_set_hierarchy(vlbm_ctx *ctx, const vlbm_box *boxes, int nboxes);

/* Set the conserved state U[4][ny][ld] (host, FP64) of the level-l cells in
 * [i0, i0+nx) x [j0, j0+ny) that are covered at level l: f := f^eq(U)
 * (eq. num-equilibrium). Clears the previous-step samples of those cells and
 * the boundary ledger. */
vlbm_status vlbm_set_state(vlbm_ctx *ctx, int level, int i0, int j0, int nx, int ny,
                           const double *U, long ld);

/* Same with raw populations F[16][ny][ld] (host, FP64). */
vlbm_status vlbm_set_populations(vlbm_ctx *ctx, int level, int i0, int j0, int nx, int ny,
                                 const double *F, long ld);

/* Advance n coarse steps: each is the recursive sub-cycle of Sec. 3.2-3.3
 * (r steps of level l+1 per step of level l, reconstruction into fine ghosts,
 * reflux into coarse ring cells). Asynchronous on the context's stream. */
vlbm_status vlbm_advance(vlbm_ctx *ctx, int n_coarse_steps);

/* Read W = sum_q f_q (U[4][ny][ld], host, FP64) of active level-l cells in the
 * rectangle (Sec. 2.2: the conserved state is the sum of the populations;
 * Sec. 4.1.2 reads it on the active cells of each grid); other cells get NaN.
 * Synchronises. */
vlbm_status vlbm_get_state(vlbm_ctx *ctx, int level, int i0, int j0, int nx, int ny, double *U,
                           long ld);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as vlbm_get_state, staged through a static per-GPU device array of
 * VLBM_NOALLOC_STAGE_BYTES (32 MiB) instead of a staging buffer allocated per
 * call, and copied straight into U. Calls no hipMalloc, hipFree or other
 * allocating routine. The part of the rectangle inside the level's frame may
 * hold at most VLBM_NOALLOC_STAGE_BYTES / 32 cells (1 Mi cells, e.g. 1024 x
 * 1024); a larger one returns VLBM_EINVAL before any device work (read it in
 * pieces). The array's device address is looked up once per GPU, on the first
 * call of a context whose stream is on it. Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents: calls that overlap
 * in time on one GPU (two host threads, or two contexts on different streams)
 * race and must be serialised by the caller. Synchronises. */
#define VLBM_NOALLOC_STAGE_BYTES (32u << 20)
vlbm_status vlbm_get_state_noalloc(vlbm_ctx *ctx, int level, int i0, int j0, int nx, int ny, double *U,
                                   long ld);

/* Read the stored post-collision populations F[16][ny][ld] (FP64 on the host,
 * widened in the FP32 form) of active cells; others NaN. Synchronises. */
vlbm_status vlbm_get_populations(vlbm_ctx *ctx, int level, int i0, int j0, int nx, int ny,
                                 double *F, long ld);

/* Conserved totals (Sec. 4.1.2: the mass summed over the active cells of both
 * grids, each weighted by its cell size; here every component, in 2-D)
 * T_k = sum_l dx_l^2 sum_active sum_q f_{q,k} (FP64,
 * compensated, fixed summation order) and the boundary ledger: the net amount
 * of each component that entered through non-periodic sides since the last
 * set_state. T(t) - T(0) equals the ledger to round-off. Synchronises. */
vlbm_status vlbm_conserved_totals(vlbm_ctx *ctx, double totals[4], double ledger[4]);

/* Replace the hierarchy by boxes, moving the state conservatively (Sec. 3.4):
 * merge exiting cells finest level first (eq. amr-merge), then split entering
 * cells coarsest level first (eqs. amr-slope, amr-split). An interface that
 * exists before and after keeps its temporal reconstruction unmodified; a
 * face the regrid creates (and every merged or split cell) has no older
 * sample, so its first coarse-to-fine hand-off has no temporal slope.
 * Synchronises. */
vlbm_status vlbm_regrid(vlbm_ctx *ctx, const vlbm_box *boxes, int nboxes);

/* Refinement indicator of vlbm_tag and vlbm_tag_and_regrid (default
 * VLBM_TAG_DENSITY):
 *   VLBM_TAG_DENSITY  max over axes |rho(+1) - rho(-1)| / (2 rho) > threshold;
 *   VLBM_TAG_FLUX     the sensor of eq. amr-sigma (Sec. 3.4),
 *                     max_k |s_k| > threshold with s_k = dx (div Q)_k /
 *                     max_{x,alpha} |Q_{alpha,k}| (central differences; the
 *                     max over the active cells of every level).
 * Either way a missing or inactive neighbour is replaced by the cell itself.
 * VLBM_EINVAL for another kind. */
#define VLBM_TAG_DENSITY 0
#define VLBM_TAG_FLUX 1
vlbm_status vlbm_set_tag_indicator(vlbm_ctx *ctx, int kind);

/* Tags of active level-l cells by the context's indicator
 * (vlbm_set_tag_indicator). tags[Ny_l][Nx_l] (host). Synchronises. */
vlbm_status vlbm_tag(vlbm_ctx *ctx, int level, double threshold, unsigned char *tags);

/* Tag every level below the finest, dilate by `buffer` cells, cluster into
 * boxes with sides in [min_box, max_box] level-(l+1) cells and regrid
 * (Sec. 3.4, Fig. amr-flowchart). Synchronises. The tags, the tile lists and,
 * for VLBM_TAG_DENSITY, one FP64 density per frame element of the largest
 * level live in device scratch that the context keeps between calls (and
 * vlbm_tag shares); vlbm_destroy frees it. */
vlbm_status vlbm_tag_and_regrid(vlbm_ctx *ctx, double threshold, int buffer, int min_box,
                                int max_box);

/* Current boxes (up to cap) and their count. */
vlbm_status vlbm_get_boxes(vlbm_ctx *ctx, vlbm_box *boxes, int cap, int *nboxes);

/* Scan active cells for rho <= 0, p <= 0 or NaN; returns VLBM_EUNSTABLE if any. */
vlbm_status vlbm_check_health(vlbm_ctx *ctx);

/* Serialise populations, both previous-step samples, reflux/ledger state, the
 * hierarchy and the step counters into buf (size *bytes; with buf NULL only the
 * size is returned). vlbm_load restores it into a context created with equal
 * parameters. Resume is bitwise. Synchronise. */
vlbm_status vlbm_save(vlbm_ctx *ctx, void *buf, size_t *bytes);
vlbm_status vlbm_load(vlbm_ctx *ctx, const void *buf, size_t bytes);

/* Advance several contexts together, n_steps[i] coarse steps each, with the
 * phases of all contexts merged into shared launches (Sec. 3.2, Fig. 1: the
 * sub-cycle of the deepest context; a shallower one joins the phases of the
 * levels it has, and a fused finest level takes its two sub-steps in one
 * launch at its parent's second sub-step, shared with the other fused
 * levels there). All contexts must use the same stream, precision,
 * refinement ratio and launch tuning; either all or none use the adaptive
 * relaxation, and either all or none the adaptive time step (each with its
 * own constants and clock): VLBM_EINVAL otherwise. With the graph tuning flag
 * (1024), two coarse steps of the merged launches are captured once per
 * membership (the contexts, their launch tables and parities) as a hipGraph
 * of kernel nodes and replayed; up to 16 captures are cached, and destroying
 * a context drops those that hold it. Each context's results are
 * bit-identical to advancing it alone. Synchronises. */
vlbm_status vlbm_batch_advance(vlbm_ctx *const *ctxs, const int *n_steps, int nctx);

/* Launch tuning (no effect on results, which are identical for every
 * setting): tile_cells is the largest number of cells one workgroup advances
 * (64..2^20); flags: 1 non-temporal stores, 2 two cells per thread,
 * 4 XCD-contiguous workgroup order, 16 fused sub-steps: with r = 2 and at
 * least two levels, one launch advances the finest level by both sub-steps of
 * its parent's step, the intermediate time level kept in LDS (temporal
 * blocking of the sub-cycling of Sec. 3), 512 XCD-contiguous order for the
 * fused launches only, 1024 replay captured hipGraphs of two coarse steps
 * (vlbm_advance of four or more steps, and vlbm_batch_advance; the
 * environment variable VLBM_GRAPHS=1 sets it at creation), 2048 a level with
 * fewer than 4096 step tiles of tile_cells cells gets tiles of half the size
 * until it has that many or they reach 64 cells (levels too small to fill
 * the chip). Rebuilds the
 * launch tables; the
 * hierarchy and the time history are kept. VLBM_EINVAL for other values. */
vlbm_status vlbm_set_tuning(vlbm_ctx *ctx, int tile_cells, int flags);

/* Autotuner: time tile sizes {128, 256, 512, 1024} x workgroup orders x store
 * kinds (x fused sub-steps on or off, where they apply) on real
 * coarse steps of this context (every trial advances the solution by
 * 1 + steps_per_trial coarse steps) and keep the fastest. A context created
 * with a stream of its own then times the fastest with and without graph
 * replay (flag 1024; 2 + m and 4 + m more coarse steps, m = steps_per_trial
 * rounded up to an even number of at least 4) and keeps replay if it saves
 * more than 2%. Before that it times the fastest with and without flag 2048
 * (2 + 2 m coarse steps, m = steps_per_trial; not with the adaptive
 * relaxation) and keeps the flag if it saves more than 1%. The choice is cached
 * per geometry (base grid, ratio, precision, boxes) for the process, so a
 * repeated call advances nothing. Reports the choice in tile_cells/flags
 * (either may be NULL). */
vlbm_status vlbm_autotune(vlbm_ctx *ctx, int steps_per_trial, int *tile_cells, int *flags);

/* Space/time-adaptive relaxation parameter (Sec. 2.2, eq. sensor-B). With
 * on != 0 every step of every level first computes, per active cell and from
 * the state at the step's start (W = sum_q f_q):
 *   s_k   = dx (div Q)_k / max |Q_{alpha,k}|, by central differences, the max
 *           over both directions and the active cells of every level, taken
 *           once per coarse step from the state at its start, when the whole
 *           hierarchy holds one time level (s_k = 0 where that max is 0);
 *   sbar  = mean over the active cells of the 3x3 block of sqrt(mean_k s_k^2);
 *   theta = dil^2 / (dil^2 + vort^2) where the velocity divergence dil < 0
 *           (compression), else 0; vort = dv/dx - du/dy;
 *   beta  = beta_max - (beta_max - beta_min) clip(c_sensor sbar theta, 0, 1),
 * and relaxes the cell with that beta (vlbm_params.beta is then unused). A
 * neighbour that is not an active cell of the level stands in as the cell
 * itself in the differences and is left out of the mean. Arithmetic in FP64
 * for every precision. Needs 0 < beta_min <= beta_max <= 1 and c_sensor >= 0
 * (VLBM_EINVAL otherwise). While on, fused sub-steps (tuning flag 16) and two
 * cells per thread (flag 2) are not used, the step tiles are at most 32 x 8
 * cells whatever tile_cells says (each step workgroup computes its tile's
 * sensor in LDS), and each level holds 9 more FP64 planes of its frame (two
 * W sets and beta; not counted by vlbm_footprint_bytes). on = 0 returns to
 * the constant beta. Switching rebuilds the tile lists; it keeps the state
 * and the time history. */
vlbm_status vlbm_set_sensor(vlbm_ctx *ctx, int on, double c_sensor, double beta_min,
                            double beta_max);

/* Adaptive time step (the acoustic scaling dx/dt = c kept on every level,
 * with c chosen per coarse step; the paper builds on an adaptive time
 * stepping for the VLBM and states that the coupling conserves for any time
 * step). With on != 0, every coarse step starts with
 *   c_n = 2 kappa max(|u_alpha| + c_s), c_s = sqrt(gamma p / rho),
 * over the active cells of every level (a device reduction; no host sync),
 * relaxes and hands off with h = 1/(2 c_n), and a hand-off whose parent last
 * stepped in the previous coarse step scales its temporal slope by
 * dt_now / dt_prev = c_prev / c_n. kappa > 0; ideal gas only (VLBM_EINVAL
 * otherwise). set_state keeps building equilibria with vlbm_params.c; on = 0
 * returns to it. vlbm_batch_advance takes it when every context of the batch
 * uses it. The maximum is accumulated
 * by each level's last step launch of the previous coarse step from the
 * values it stores; after a host-side change of the state (set_state,
 * set_populations, regrid, tag_and_regrid, load, a new hierarchy or tuning)
 * the next advance first reads every level once to take it from memory. Both
 * give the same bits. */
vlbm_status vlbm_set_time_stepping(vlbm_ctx *ctx, int on, double kappa);

/* Elapsed time since set_state and the link speed of the last coarse step
 * (either pointer may be NULL). With a fixed c, time = steps * dx0 / c.
 * Synchronises. */
vlbm_status vlbm_time(vlbm_ctx *ctx, double *time, double *link_speed);

/* beta[ny][ld] (host) of the active level-l cells in the rectangle, as used
 * by the level's latest step with the adaptive relaxation on; other cells, and
 * every cell while it is off, get NaN (0 before the level's first step with
 * it). Synchronises. */
vlbm_status vlbm_get_beta(vlbm_ctx *ctx, int level, int i0, int j0, int nx, int ny, double *beta,
                          long ld);

/* Per-kernel timing of the step launches of vlbm_advance. With enable != 0
 * every launch records its own start and end (events of the AMD launch
 * extension: no extra work on the stream) and the accumulators restart at
 * zero; graph replay is bypassed meanwhile. enable = 0 stops recording and
 * keeps the totals. Launches of vlbm_batch_advance are not recorded. */
vlbm_status vlbm_set_profiling(vlbm_ctx *ctx, int enable);

/* Accumulated kernel time in ms, launch count and active cells advanced
 * (summed over the launches) per level and launch form, at index
 * 2 * level + f with f = 1 for fused two-sub-step launches of the finest level
 * (r = 2 hierarchy with tuning flag 16), which advance each cell by both
 * sub-steps of its parent's step. ms, calls and cells hold
 * 2 * VLBM_MAX_LEVELS entries each. Synchronises with the recorded
 * launches. */
vlbm_status vlbm_kernel_times(vlbm_ctx *ctx, double *ms, long *calls, double *cells);

/* Coarse steps taken since set_state. */
long vlbm_steps(const vlbm_ctx *ctx);

/* Number of active cells of a level (0 for an absent level). */
long vlbm_active_cells(const vlbm_ctx *ctx, int level);

/* Wait for all work of ctx. */
vlbm_status vlbm_sync(vlbm_ctx *ctx);

const char *vlbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
