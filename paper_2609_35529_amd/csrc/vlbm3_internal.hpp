// Internal definitions of the three-dimensional (D3Q6) path of libvlbm: work
// descriptors shared by api3.hip and kernels3.hip.
//
// Data layout, per level l: one dense frame = bounding box of the level's
// coverage plus a one-cell ghost layer. Buffer b in {0, 1} holds 30 planes
// (q * 5 + k) of `plane` elements (double, or float in the FP32 forms); cell
// (x, y, z) of the level sits at element
//   ((z - fz0) * fh + (y - fy0)) * pitch + (x - fx0) + xoff
// of a plane, with rows of `pitch` elements (a multiple of 64) and the first
// interior column on a 128-byte line. The current time level of l lives in
// buf[steps_l & 1]; stored values are post-collision populations f*.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vlbm3 {

// Ghost and interface work executed by a tile's workgroup before its cells.
enum TaskKind3 : int32_t {
  K3_COPY = 0,      // ghost slot <- same-level cell (periodic image)
  K3_OUTFLOW = 1,   // ghost slot <- the edge cell's own population q; ledger
  K3_REFLECT = 2,   // ghost slot <- the edge cell's population q^1, normal momentum negated; ledger
  K3_RECON = 3,     // ghost slot <- coarse-to-fine hand-off from the parent ring cell
  K3_REFLUX = 4,    // hole slot  <- reflux accumulator / r^3
  K3_CAPTURE = 5,   // reflux accumulator (=, or += after the first sub-step) of r^2 face cells
  K3_LEDGER = 0x100,
};

struct Task3 {    // 48 bytes
  int32_t kind;   // TaskKind3 (| K3_LEDGER)
  int32_t q;      // population written (ghost kinds) or captured
  int32_t dst;    // element offset of the ghost / hole slot in this level's planes
  int32_t src;    // source cell (own level; parent level for RECON; first face cell for CAPTURE)
  int32_t n[4];   // RECON: parent cells -+ e_t1, -+ e_t2 (-1: no slope); CAPTURE: outer, inner stride
  int32_t j1, j2; // RECON: tangential indices of the fine cell in its parent (t1 < t2)
  int32_t slot;   // REFLUX / CAPTURE: accumulator slot; boundary kinds: ledger slot
  int32_t pad;
};

struct Tile3 {    // 32 bytes: w x h cells, rows of one z-slab
  int32_t off0;   // element offset of the first cell
  int32_t w, h;
  int32_t task0, ntask;
  int32_t pad[3];
};

struct Desc3 {
  void *src, *dst;            // current and next buffer of the level
  const void *pcur, *pprev;   // parent: current and previous buffers (RECON)
  const Tile3 *tiles;
  const Task3 *tasks;
  double *acc_in;             // accumulators the finer level filled (REFLUX)
  double *acc_out;            // the parent's accumulators (CAPTURE)
  double *ledger;             // boundary ledger slots [slot][5]
  int64_t plane, pplane, slab;
  int32_t pitch, ntiles, r, pad;
  double rrr;                 // r^3
  double w3;                  // dx_l^3
  double gm1, h, tb;          // gamma - 1, 1/(2c), 2 beta
};

enum StepFlags3 : int32_t {
  S3_NT_STORES = 1,  // tuning: non-temporal stores of the new time level
  S3_FP32 = 2,       // storage in float
  S3_F64_MATH = 4,   // with S3_FP32: the cell update evaluated in double
};

struct Launch3 {
  const Desc3 *d;
  int32_t nblocks, first, flags, pad;
  double ak;                  // (2k - r - 1) / (2r)
};

struct Rect3 {
  void *buf0, *buf1;          // set: both written; get: buf0 read
  const uint8_t *status;      // frame status: 0 none, 1 active, 2 hole
  double *stage;              // device staging [ncomp][nz][ny][nx]
  int64_t plane, slab;
  int32_t pitch, xoff, fx0, fy0, fz0, fw, fh;
  int32_t x0, y0, z0, nx, ny, nz;
  double gm1, h;
};

// Regrid: merge (dst: parent in the coarse frame, src: child (0,0,0) in the
// fine frame) or split (dst: child (0,0,0) in the fine frame, src: parent in
// the coarse frame, nb: parent's neighbours +x, -x, +y, -y, +z, -z or -1).
struct RegridOp3 {
  int32_t dst, src;
  int32_t nb[6];
};
struct RegridArgs3 {
  const void *fine_cur;           // merge: the fine level's current buffer (old frame)
  void *fine0, *fine1;            // split: both fine buffers (new frame)
  const void *coarse_cur;         // split: the coarse level's current buffer (new frame)
  void *coarse0, *coarse1;        // merge: both coarse buffers (old frame)
  int64_t fplane, fslab, cplane;
  int32_t fpitch, r;
  const RegridOp3 *ops;
  int32_t nops;
};
// fp32: float storage. Every launcher below takes it; their arithmetic is FP64.
hipError_t launch_merge3(const RegridArgs3 &a, int fp32, hipStream_t s);
hipError_t launch_split3(const RegridArgs3 &a, int fp32, hipStream_t s);
hipError_t launch_copy3_runs(const void *s0, const void *s1, void *d0, void *d1, const int32_t *runs,
                             int nruns, int64_t splane, int64_t dplane, int fp32, hipStream_t s);
// Interfaces a regrid creates: population q (5 planes) of each listed cell
// copied from the current buffer into the other one; items[2i] element
// offset, items[2i+1] q.
hipError_t launch_restart_faces3(const void *cur, void *other, const int32_t *items, int n, int64_t plane,
                                 int fp32, hipStream_t s);

// Refinement tags of one level frame (one byte per frame element).
struct Tag3Args {
  const void *buf;         // the level's current buffer
  const uint8_t *status;   // frame status: 1 active
  uint8_t *tags;           // out: fn0 x fn1 x fn2 bytes, frame order
  int64_t plane, slab;
  int32_t pitch, xoff;
  int32_t f0[3], fn[3], N[3];
  int32_t periodic;        // bit a: axis a is periodic
  double thr;
};
hipError_t launch_tag3(const Tag3Args &a, int fp32, hipStream_t s);

hipError_t launch_step3(const Launch3 &a, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr);
hipError_t launch_audit3(const void *buf, const Tile3 *tiles, int ntiles, int64_t plane, int pitch,
                         double *partial, int fp32, hipStream_t s);
hipError_t launch_set3(const Rect3 &a, int raw_populations, int fp32, hipStream_t s);
hipError_t launch_get3(const Rect3 &a, int populations, int fp32, hipStream_t s);

}  // namespace vlbm3
