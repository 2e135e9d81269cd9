// Internal definitions of libvlbm shared by its host and device translation
// units: device work descriptors and the launch entry points.
//
// Data layout (per level l, one "frame": the columns of the coverage's bounding
// box plus a ghost column on each side, over the runs of rows that hold the
// covered rows and their neighbour rows; rows between runs are not stored):
//   buffer b in {0,1}: 16 planes (q*4+k) of `plane` elements each; the element
//   of level cell (x,y) is  srow[y - fy0] * pitch + (x - fx0) + xoff  within a
//   plane, where srow numbers the stored rows in increasing y (so the rows
//   above and below an active cell are one pitch away).
//   Stored values are post-collision populations f*; the current time level of
//   level l lives in buf[steps_l & 1], the previous one in the other buffer.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vlbm {

// Work items executed by a tile's workgroup before it advances its cells.
enum TaskKind : int32_t {
  T_COPY = 0,     // ghost slot <- same-level cell (periodic image), population q
  T_OUTFLOW = 1,  // ghost slot <- own edge cell, population q; boundary ledger
  T_REFLECT = 2,  // ghost slot <- own edge cell, population opp(q), normal momentum negated; ledger
  T_INFLOW = 3,   // ghost slot <- f^eq_q(w_inflow[side]); ledger
  T_RECON = 4,    // ghost slot <- coarse-to-fine hand-off (eq. 2d-recon) from the parent ring cell
  T_REFLUX = 5,   // hole slot  <- reflux accumulator / r^2 (eq. 2d-reflux)
  T_CAPTURE = 6,  // reflux accumulator (=, or += after the first sub-step) sum_j f_q(R_j)
  // fused two-sub-step launches of the finest level (r = 2):
  T_RING = 7,      // sub-step 1 of a ring cell: global cell src -> LDS position dst of population q
  T_CAPTURE2 = 8,  // both sub-steps' captures: global R_0 src (stride n0), LDS R_0 n1 (stride j)
  T_NONE = -1,     // host-side only: the slot is an active cell, no task
  TASK_LEDGER = 0x100,  // flag: this task books the boundary ledger (owner tile)
  TASK_K2 = 0x200,      // flag: sub-step-2 ghost value into LDS position dst (boundary kinds:
                        // the tile cell at LDS position src for population q, n1 for q^1)
};

struct Task {      // 32 bytes
  int32_t kind;
  int32_t q;       // population written (ghost kinds) or captured
  int32_t dst;     // element offset of the ghost / hole slot in this level's planes
  int32_t src;     // element offset of the source cell (own level; parent level for RECON)
  int32_t n0;      // RECON: parent cell - tau (or -1); CAPTURE: stride between R_j; BC: side
  int32_t n1;      // RECON: parent cell + tau (or -1)
  int32_t j;       // RECON: tangential index j of the fine cell within its parent
  int32_t slot;    // REFLUX/CAPTURE: accumulator slot; BC: ledger slot
};

struct Tile {      // 32 bytes: a w x h rectangle of active cells
  int32_t off0;    // element offset of cell (x0, y0)
  int32_t w, h;
  int32_t task0, ntask;
  // fused tiles: ntask counts sub-step-1 ghost tasks, then follow nring ring
  // cells, nk2 sub-step-2 ghost tasks and ncap captures
  int32_t nring, nk2, ncap;
};

// Largest fused tile: FUSE_W x FUSE_H cells (both even). The LDS copy of the
// intermediate time level keeps, per population q, the tile's cells and the
// one ring side from which the tile pulls f_q: (w+1) x h positions for q = +-x,
// w x (h+1) for q = +-y, at most FUSE_POS each. Position of tile-relative cell
// (cx, cy) in the plane group of q:
//   +x: cy (w+1) + cx + 1   -x: cy (w+1) + cx   +y: (cy+1) w + cx   -y: cy w + cx
#ifndef VLBM_FUSE_W
#define VLBM_FUSE_W 64
#define VLBM_FUSE_H 4
#endif
constexpr int FUSE_W = VLBM_FUSE_W;
constexpr int FUSE_H = VLBM_FUSE_H;
constexpr int FUSE_POS = (FUSE_W + 1) * FUSE_H > FUSE_W * (FUSE_H + 1) ? (FUSE_W + 1) * FUSE_H
                                                                      : FUSE_W * (FUSE_H + 1);
#ifndef VLBM_FUSE_THREADS
#define VLBM_FUSE_THREADS 256
#endif
constexpr int FUSE_THREADS = VLBM_FUSE_THREADS;
static_assert(FUSE_W % 2 == 0 && FUSE_H % 2 == 0 && FUSE_W * FUSE_H <= FUSE_THREADS &&
                  2 * (FUSE_W + FUSE_H) <= FUSE_THREADS,
              "fused tile shape: one tile cell and one ring cell per thread at most");

// Equation of state p(rho, rho e) (Sec. 2.1 leaves it generic): kind 0 ideal
// gas (gamma-1) rho e; 1 stiffened gas (gamma-1) rho e - gamma a; 2 van der
// Waals ((gamma-1) (rho e + a rho rho)) / (1 - b rho) - a rho rho; with
// rho e = E - 0.5 (m_x u + m_y v) and ga = gamma * a.
template <class T>
struct EosT {
  int32_t kind;
  T gm1, a, b, ga;
};

enum StepFlags : int32_t {
  STEP_NT_STORES = 1,        // write the new time level with non-temporal stores
  STEP_TWO_CELLS = 2,        // two cells per thread, gathers issued together
  STEP_XCD_CONTIGUOUS = 4,   // map consecutive tiles to the same XCD
  STEP_F64_MATH = 8,         // FP32 storage, relaxation evaluated in FP64
  STEP_FUSE2 = 16,           // tuning: the finest level takes both sub-steps per launch
  STEP_FUSED_PHASE = 32,     // launch-uniform: this phase is a fused two-sub-step launch
  STEP_SENSOR = 64,          // launch-uniform: relax with the per-cell beta of the sensor planes
  STEP_ADAPTIVE_DT = 128,    // launch-uniform: h and the hand-off's time-step ratio from DynState
  STEP_CFL_EMIT = 256,       // launch-uniform: the level's last step launch of the coarse step folds
                             // the CFL term of its stored cells into cfl_next (emit_cfl)
  STEP_XCD_FUSED = 512,      // tuning: XCD-contiguous order for the fused launches only
  STEP_GRAPHS = 1024,        // tuning: replay captured graphs of two coarse steps (kernels unaffected)
  STEP_SMALL_TILES = 2048,   // tuning: a level with fewer than 4096 step tiles gets smaller tiles
};

// Device scalars of the adaptive time step, updated once per coarse step by
// launch_cfl_finalize (never by the host while steps are queued).
enum DynSlot : int32_t {
  DYN_C = 0,       // link speed of the current coarse step
  DYN_H = 1,       // 1 / (2 c)
  DYN_C_PREV = 2,  // link speed of the previous coarse step
  DYN_TIME = 3,    // elapsed time
  DYN_GAMMA = 4,   // gamma (sound speed)
  DYN_KD = 5,      // kappa * D
  DYN_DX0 = 6,     // level-0 cell size
  DYN_SLOTS = 8
};

// Adaptive relaxation planes of a level (FP64, `plane` elements each, same
// element offsets as the populations): two sets of W_0..W_3, one per parity
// of the level's step count (a step reads the set of its input time level
// and writes the other one), and beta of the last step. A W set spans four
// planes with the components of element o at 4 o .. 4 o + 3.
enum SensorPlane : int32_t { SEN_W0 = 0, SEN_W1 = 4, SEN_BETA = 8, SEN_PLANES = 9 };

// With the adaptive relaxation the step tiles are at most SEN_TW x SEN_TH
// cells. A step workgroup keeps in LDS the fluxes and velocities of the
// active cells within two cells of its tile (a (w + 4) x (h + 4) block) and
// the activity of the tile and its one-cell ring ((w + 2) x (h + 2)).
constexpr int SEN_TW = 32, SEN_TH = 8;
constexpr int SEN_BLOCK = (SEN_TW + 4) * (SEN_TH + 4);
constexpr int SEN_RING = (SEN_TW + 2) * (SEN_TH + 2);

// Neighbourhood mask of an active cell (32 bits per frame element): bit
// nb_bit(dx, dy) = (dy + 2) * 5 + (dx + 2), |dx|, |dy| <= 2, is set when
// level cell (x + dx, y + dy), periodic sides wrapped, is an active cell of
// the level (the centre bit always, the four corner bits never). Inactive
// cells hold 0.
__host__ __device__ constexpr int nb_bit(int dx, int dy) { return (dy + 2) * 5 + (dx + 2); }

// Everything the step kernel needs about one (context, level) at one phase of
// the schedule. Lives in device memory; a launch covers one or more of them.
struct LevelDesc {
  void *src;                 // current buffer of the level (ghost slots are written into it)
  void *dst;                 // next buffer of the level
  const void *pcur, *pprev;  // parent level: current and previous buffers (RECON)
  const Tile *tiles;
  const Task *tasks;
  double *acc_in;            // accumulators filled by the finer level (REFLUX reads)
  double *acc_out;           // parent's accumulators (CAPTURE writes)
  double *ledger;            // boundary ledger slots [slot][4]
  int64_t plane, pplane;     // elements per population plane (level, parent)
  int32_t pitch, ntiles, r;
  int32_t eos;               // equation of state kind (EosT)
  double rr;                 // r * r
  double w2;                 // dx_l^2 (ledger weight)
  double gm1, h, tb;         // gamma - 1, 1/(2c), 2 beta
  double eos_a, eos_b, eos_ga;  // EOS constants a, b and gamma * a
  double win[4][4];          // inflow conserved states per side
  // adaptive relaxation (eq. sensor-B); sen == nullptr when it is off
  double *sen;               // SEN_PLANES planes (SensorPlane)
  const double *wcur;        // the W set of this step's input time level
  double *wnext;             // the W set of its output
  const uint32_t *mask;      // neighbourhood masks (nb_bit), `plane` words
  unsigned long long *qmax;       // [4] max |Q_{alpha,k}| of this coarse step, as bits
  unsigned long long *qmax_next;  // [4] the next coarse step's, accumulated by its last steps
  int32_t clear_next;        // this phase is the context's first of the coarse step: qmax_next is
                             // cleared (stage 1) before it
  int32_t emit_qmax;         // this phase is the level's last of the coarse step: accumulate qmax_next
  int32_t fx0, fy0, xoff;    // frame origin (level cells)
  const int32_t *srow;       // frame row -> storage row (-1: not stored)
  const int32_t *yrow;       // storage row -> frame row
  int32_t Nx, Ny;            // level domain
  double c_sensor, beta_min, beta_max;
  // adaptive time step: the DynState scalars, and whether this phase's parent
  // last stepped in the previous coarse step (hand-off takes c_prev / c)
  const double *dyn;
  int32_t use_ratio;
  int32_t emit_cfl;               // this phase is the level's last of the coarse step: fold the CFL
                                  // term of every stored cell into *cfl_next
  unsigned long long *cfl_next;   // the next coarse step's CFL bound (bits), cleared by the finalize
};

// A run of workgroups of one launch that works on one LevelDesc. first_block
// and nblocks are multiples of 8 so that the XCD of a workgroup (blockIdx % 8)
// is also its index modulo 8 inside the segment.
struct Segment {
  const LevelDesc *d;
  int32_t first_block, nblocks;
};

// Launch-uniform parameters of one phase (level l, sub-step k of its parent).
// A launch over a single descriptor passes its address directly (d0 with
// nseg == 0); a batched launch passes a segment table instead.
struct StepLaunch {
  const LevelDesc *d0;
  const Segment *segs;
  int32_t nseg;
  int32_t nblocks;           // total workgroups
  int32_t first;             // CAPTURE: k == 1 (first sub-step of the parent's cycle)
  int32_t flags;             // STEP_* variants
  double ak;                 // (2k - r - 1) / (2r)
};

// Rectangle copy-in / copy-out and diagnostics.
struct RectArgs {
  void *buf0, *buf1;         // both buffers of the level (set: both written; get: buf0 read)
  const uint8_t *status;     // frame status (fw per stored row): 0 none, 1 active, 2 hole
  const int32_t *srow;       // frame row -> storage row (-1: not stored, no covered cell)
  double *host_stage;        // device staging [ncomp][ny][nx]
  int64_t plane;
  int32_t pitch, xoff, fx0, fy0, fw;
  int32_t x0, y0, nx, ny;    // rectangle in level cells
  double gm1, h;
  EosT<double> eos;
};

// Launchers (kernels.hip). All return hipError_t of the launch.
hipError_t launch_step(const StepLaunch &a, int fp32, hipStream_t s, hipEvent_t ev0 = nullptr,
                       hipEvent_t ev1 = nullptr);
// Adaptive relaxation: stage 0 (the input W set of every level and the coarse
// step's max |Q| from the stored populations, over the first-phase
// descriptors of every level; after any change of state) or stage 1 (one
// workgroup: clear qmax_next of every descriptor of the launch `a` that has
// clear_next, to run just before the step launch `a`).
hipError_t launch_sensor(const StepLaunch &a, int stage, int fp32, hipStream_t s);
// Adaptive time step: the CFL bound max(|u_alpha| + c_s) over the step tiles of
// the launch (every level at the coarse step's start) into *cmax (bits), then
// the one-thread update of the DynState scalars, which also clears *cmax.
hipError_t launch_cfl(const StepLaunch &a, int fp32, unsigned long long *cmax, const double *dyn,
                      hipStream_t s);
hipError_t launch_cfl_finalize(double *dyn, unsigned long long *cmax, hipStream_t s);
// Zero n 64-bit words of device memory on stream s (no memset node under capture).
hipError_t launch_clear_u64(unsigned long long *p, int n, hipStream_t s);
// Neighbourhood masks of a level frame from its status (fw bytes per stored
// row, 1 = active); srow / yrow map frame rows to storage rows and back.
hipError_t launch_sensor_mask(const uint8_t *status, uint32_t *mask, const int32_t *srow, const int32_t *yrow,
                              int fx0, int fy0, int fw, int fh, int nrows, int pitch, int xoff, int Nx,
                              int Ny, int per, hipStream_t s);
hipError_t launch_audit(const void *buf, const Tile *tiles, int ntiles, int64_t plane,
                        int pitch, int fp32, double *partial, hipStream_t s);
hipError_t launch_set_state(const RectArgs &a, int fp32, int raw_populations, hipStream_t s);
hipError_t launch_get(const RectArgs &a, int fp32, int populations, hipStream_t s);
hipError_t launch_health(const void *buf, const Tile *tiles, int ntiles, int64_t plane,
                         int pitch, int fp32, const EosT<double> &eos, int *flag, hipStream_t s);
// tags: indexed like the status (fw bytes per stored row), 1 on tagged active
// cells, else 0; rho: device scratch of fw * nrows doubles (the densities)
hipError_t launch_tag(const void *buf, const uint8_t *status, const int32_t *srow, const int32_t *yrow,
                      int64_t plane, int pitch, int xoff, int fx0, int fy0, int fw, int fh, int nrows,
                      int Nx, int Ny, int perx, int pery, int fp32, double thr, double *rho, uint8_t *tags,
                      hipStream_t s);

// Refinement sensor of eq. amr-sigma: flux_max folds max |Q_{alpha,k}| of a
// level's active cells (its step tiles) into qmax[4] (bits, zeroed by the
// caller before the first level); tag_flux tags, like launch_tag, the active
// cells whose max_k |s_k| exceeds thr.
hipError_t launch_flux_max(const void *buf, const Tile *tiles, int ntiles, int64_t plane, int pitch, int fp32,
                           const EosT<double> &eos, unsigned long long *qmax, hipStream_t s);
hipError_t launch_tag_flux(const void *buf, const uint8_t *status, const int32_t *srow, const int32_t *yrow,
                           int64_t plane, int pitch, int xoff, int fx0, int fy0, int fw, int fh, int nrows, int Nx,
                           int Ny, int perx, int pery, int fp32, const EosT<double> &eos,
                           const unsigned long long *qmax, double thr, uint8_t *tags, hipStream_t s);

// Clustering on the device. tag_parents: every tagged cell of a level-(l+1)
// frame (fw per stored row) tags its parent in the level-l tags. tile_hits:
// of the tile rows listed in trows (tiles of side T, ntx per tile row), the
// tiles within `buf` cells of a tag, appended to list[0 .. *count) in no
// particular order (at most cap entries stored).
hipError_t launch_tag_parents(const uint8_t *ftags, const int32_t *fyrow, int ffx0, int ffy0, int ffw,
                              int fnrows, uint8_t *ptags, const int32_t *psrow, int pfx0, int pfy0, int pfw,
                              int pfh, int r, hipStream_t s);
// masks: device scratch of nrows * ceil(Nx / 64) words (the rows' tags as bits).
hipError_t launch_tile_hits(const uint8_t *tags, const int32_t *srow, int fx0, int fy0, int fw, int fh, int nrows,
                            int Nx, int Ny, int perx, int pery, int T, int buf, int ntx, const int32_t *trows,
                            int ntrows, unsigned long long *masks, int32_t *list, int cap, int *count, hipStream_t s);

// Regrid kernels: a list of cell operations on level frames.
struct RegridOp {          // one coarse cell (merge) or one parent cell (split)
  int32_t dst;             // element offset of the destination (merge: parent cell;
                           // split: child (0,0) in the fine frame)
  int32_t src;             // merge: child (0,0) in the fine frame; split: parent cell
  int32_t nb[4];           // split: neighbour offsets +x,-x,+y,-y in the parent frame (-1: none)
};
struct RegridArgs {
  void *fine0, *fine1;     // fine frame buffers (merge reads current; split writes both)
  void *coarse0, *coarse1; // coarse frame buffers (merge writes both; split reads current)
  int fine_cur, coarse_cur;
  int64_t fplane, cplane;
  int32_t fpitch, cpitch;
  int32_t r;
  const RegridOp *ops;
  int32_t nops;
};
hipError_t launch_merge(const RegridArgs &a, int fp32, hipStream_t s);
hipError_t launch_split(const RegridArgs &a, int fp32, hipStream_t s);
hipError_t launch_copy_frame(const void *src, void *dst, const int32_t *pairs, int npairs,
                             int64_t splane, int64_t dplane, int fp32, hipStream_t s);
// Interfaces a regrid creates: population q (4 planes) of each listed cell
// copied from the current buffer into the other one; items[2i] element offset,
// items[2i+1] q.
hipError_t launch_restart_faces(const void *cur, void *other, const int32_t *items, int n,
                                int64_t plane, int fp32, hipStream_t s);

}  // namespace vlbm
