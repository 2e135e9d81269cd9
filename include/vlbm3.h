/*
 * libvlbm, three-dimensional path: the D3Q6 vectorial lattice Boltzmann method
 * with conservative local grid refinement (static hierarchies and regrid), on
 * one GPU (gfx950).
 *
 * The method (paper):
 *   - Six populations f_i = +-c e_alpha (alpha = x, y, z), each carrying the
 *     five conserved components W = (rho, rho u, rho v, rho w, E); equilibrium
 *     f_i^eq = W/(2D) + c_i . Q(W) / (2 c^2) with D = 3 (Sec. 2.2 eq.
 *     num-equilibrium), exact-shift transport, BGK relaxation
 *     f* = f + 2 beta (f^eq - f) (eq. num-relaxation). Ideal gas.
 *   - Refinement: level l+1 takes r steps per step of level l (Sec. 3.2, one
 *     link speed c = dx/dt on every level). The coupling is that of Sec. 3.3
 *     applied face by face: a coarse ring cell hands its two stored samples
 *     to the r^2 fine cells it faces, out + (out - prev)(2k - r - 1)/(2r) plus
 *     one minmod-limited tangential correction per tangential axis at the fine
 *     cell's offset (eqs. 2d-recon-tanslope, 2d-recon); the coarse cell facing
 *     the patch receives the plain average of the r^2 face cells' outgoing
 *     values over the r sub-steps, a weight of 1/r^3 (eq. 2d-reflux).
 *
 * Conventions shared with include/vlbm.h: vlbm_status codes, vlbm_last_error,
 * every call returns a status and never throws, host arrays stay caller-owned,
 * device memory is the library's (and a pinned host buffer through which the
 * boundary ledger is read back, grown on demand and freed by vlbm3_destroy).
 * Calls that return data synchronise the context's stream; vlbm3_advance is
 * asynchronous. Host work of hierarchy changes runs on a pool of worker
 * threads shared by every context of the process.
 *
 * Host arrays: U[5][nz][ny][nx] (rho, rho u, rho v, rho w, E) and
 * F[30][nz][ny][nx] with plane index q * 5 + k, q in (+x, -x, +y, -y, +z, -z),
 * for the rectangle [i0, i0 + nx) x [j0, j0 + ny) x [k0, k0 + nz) of level-l
 * cells, FP64 on the host in every precision.
 */
#ifndef VLBM3_H
#define VLBM3_H

#include <stddef.h>

#include "vlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VLBM3_MAX_LEVELS 6

typedef struct vlbm3_ctx vlbm3_ctx;

/* nx0 x ny0 x nz0 level-0 cells of size dx0; r the refinement ratio (1..8);
 * max_levels 1..VLBM3_MAX_LEVELS; bc per side (-x, +x, -y, +y, -z, +z):
 * VLBM_BC_PERIODIC (on both sides of an axis), VLBM_BC_OUTFLOW (the edge
 * cell's own post-collision inbound population) or VLBM_BC_REFLECT (the
 * outgoing population with the normal momentum negated); beta in [0, 1].
 * precision as in include/vlbm.h: VLBM_FP64; VLBM_FP32_STORAGE (populations
 * stored in FP32, the cell update evaluated in FP64); VLBM_FP32 (stored and
 * updated in FP32). The hand-off, the reflux, the ledger, the audit and
 * regrid evaluate in FP64 in every form and round to the storage type. */
typedef struct {
  int nx0, ny0, nz0;
  double dx0;
  int bc[6];
  double gamma, c, beta;
  int r;
  int max_levels;
  int precision;
} vlbm3_params;

/* A box of level-l cells (level >= 1), made of whole parent cells. */
typedef struct {
  int level, i0, j0, k0, nx, ny, nz;
} vlbm3_box;

/* Create a context on stream (a hipStream_t; NULL: the default stream).
 * VLBM_EINVAL for bad parameters. */
vlbm_status vlbm3_create(const vlbm3_params *params, void *stream, vlbm3_ctx **out);

/* Take every later device allocation of ctx from the caller's allocator
 * (vlbm_alloc_fn / vlbm_free_fn of include/vlbm.h; e.g. PyTorch's caching
 * allocator on the context's stream), so that the caller is the only
 * allocator; blocks must be 256-byte aligned (others are handed back and
 * count as a failure). Must precede vlbm3_set_hierarchy (VLBM_ESTATE after
 * it); VLBM_EINVAL for a null function. Without it the library allocates
 * with hipMalloc. A failed allocation makes the call that needed it return
 * VLBM_ENOMEM. vlbm3_destroy releases every block through `release`. */
vlbm_status vlbm3_bind_allocator(vlbm3_ctx *ctx, vlbm_alloc_fn alloc, vlbm_free_fn release, void *user);

/* Release all device memory of ctx and free it. NULL is a no-op. */
void vlbm3_destroy(vlbm3_ctx *ctx);

/* Device bytes a context with these parameters and boxes needs. Pure host
 * computation; 0 for invalid input. */
size_t vlbm3_footprint_bytes(const vlbm3_params *params, const vlbm3_box *boxes, int nboxes);

/* Install a static hierarchy (level 0 covers the domain). Boxes of level l must
 * lie in the level's domain, be made of whole parent cells, and be properly
 * nested: the parent of every covered cell and its six face neighbours are
 * covered one level up (VLBM_ENEST otherwise). Discards any previous state. */
vlbm_status vlbm3_set_hierarchy(vlbm3_ctx *ctx, const vlbm3_box *boxes, int nboxes);

/* Replace the hierarchy by boxes, moving the state conservatively (Sec. 3.4
 * with D = 3): exiting cells are merged finest level first (eq. amr-merge, the
 * plain average of r^3 children, summed z, y, x), entering cells split
 * coarsest level first (eqs. amr-slope, amr-split, one minmod slope per axis
 * from neighbours covered at that level in the new hierarchy that hold data).
 * Merged and split cells get the same value in both time levels. An
 * interface that exists before and after keeps its temporal reconstruction;
 * a face the regrid creates starts with no temporal slope. The boundary
 * ledger is kept. Validation as vlbm3_set_hierarchy. Synchronises. */
vlbm_status vlbm3_regrid(vlbm3_ctx *ctx, const vlbm3_box *boxes, int nboxes);

/* Refinement tags of the active level-l cells (Sec. 3.4, density-gradient
 * variant): max over the three axes of |rho(+1) - rho(-1)| / (2 rho) >
 * threshold, a neighbour that is not an active cell of the level (periodic
 * sides wrapped) replaced by the cell itself. tags[Nz_l][Ny_l][Nx_l] (host,
 * caller-owned), 0 on cells that are not active. Synchronises. */
vlbm_status vlbm3_tag(vlbm3_ctx *ctx, int level, double threshold, unsigned char *tags);

/* Tag every present level below max_levels - 1, mark the parents of tagged
 * finer cells, dilate by `buffer` cells and cluster, coarsest level first,
 * into boxes of level l+1 on a grid of tiles of ceil(min_box / r) level-l
 * cells per axis (boxes of at most max_box level-(l+1) cells per axis, tiles
 * taken only where they and the cells beside their faces are covered, so the
 * boxes nest), then vlbm3_regrid to them (Sec. 3.4, Fig. amr-flowchart).
 * VLBM_EINVAL unless 0 <= buffer and 1 <= min_box <= max_box. Synchronises. */
vlbm_status vlbm3_tag_and_regrid(vlbm3_ctx *ctx, double threshold, int buffer, int min_box, int max_box);

/* The current boxes (up to cap of them) and their count. */
vlbm_status vlbm3_get_boxes(vlbm3_ctx *ctx, vlbm3_box *boxes, int cap, int *nboxes);

/* f := f^eq(U) on the covered cells of the rectangle; clears the previous-step
 * samples of those cells and the boundary ledger. */
vlbm_status vlbm3_set_state(vlbm3_ctx *ctx, int level, int i0, int j0, int k0, int nx, int ny,
                            int nz, const double *U);

/* The same with raw populations F. */
vlbm_status vlbm3_set_populations(vlbm3_ctx *ctx, int level, int i0, int j0, int k0, int nx,
                                  int ny, int nz, const double *F);

/* W = sum_q f_q of the active cells of the rectangle (NaN elsewhere). */
vlbm_status vlbm3_get_state(vlbm3_ctx *ctx, int level, int i0, int j0, int k0, int nx, int ny,
                            int nz, double *U);

/* The stored post-collision populations of the active cells (NaN elsewhere). */
vlbm_status vlbm3_get_populations(vlbm3_ctx *ctx, int level, int i0, int j0, int k0, int nx,
                                  int ny, int nz, double *F);

/* Advance n coarse steps (the recursive sub-cycle). Asynchronous. */
vlbm_status vlbm3_advance(vlbm3_ctx *ctx, int n_coarse_steps);

/* T_k = sum_l dx_l^3 sum_active sum_q f_{q,k} (compensated) and the boundary
 * ledger: what entered through non-periodic sides since the last set_state. */
vlbm_status vlbm3_conserved_totals(vlbm3_ctx *ctx, double totals[5], double ledger[5]);

/* Launch tuning, no effect on results: tile_cells (64..65536) bounds the cells
 * one workgroup advances; flags: 1 non-temporal stores (default: non-temporal
 * stores, 512-cell tiles in FP64, 1024-cell tiles in the FP32 forms).
 * Rebuilds the lists; state and history are kept. */
vlbm_status vlbm3_set_tuning(vlbm3_ctx *ctx, int tile_cells, int flags);

/* Per-level kernel timing of the step launches (launch-extension events),
 * as vlbm_set_profiling / vlbm_kernel_times; ms, calls, cells hold
 * VLBM3_MAX_LEVELS entries. */
vlbm_status vlbm3_set_profiling(vlbm3_ctx *ctx, int enable);
vlbm_status vlbm3_kernel_times(vlbm3_ctx *ctx, double *ms, long *calls, double *cells);

/* Checkpoint of the state: the boxes, every level's two time levels of
 * populations and step count, the coarse step count and the boundary
 * ledger's totals, into buf (caller-owned, *bytes long; with buf NULL only
 * the size needed is returned in *bytes). vlbm3_load restores it into a
 * context created with equal parameters (VLBM_EINVAL otherwise), under any
 * launch tuning; the run continues bit for bit as if never interrupted.
 * Both synchronise. */
vlbm_status vlbm3_save(vlbm3_ctx *ctx, void *buf, size_t *bytes);
vlbm_status vlbm3_load(vlbm3_ctx *ctx, const void *buf, size_t bytes);

/* Active cells of a level (0 if absent). */
long vlbm3_active_cells(const vlbm3_ctx *ctx, int level);

/* Wait for all work of ctx. */
vlbm_status vlbm3_sync(vlbm3_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
