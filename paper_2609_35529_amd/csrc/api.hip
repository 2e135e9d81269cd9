// Host side of libvlbm: hierarchy frames, tile and task lists, the recursive
// sub-cycle schedule, and the C ABI declared in include/vlbm.h.
//
// Schedule (paper Sec. 3.2, Fig. 1, and Sec. 3.3): one coarse step of level l
// runs r steps of level l+1 first, each of which recursively runs level l+2,
// then advances level l itself. Every level step is ONE launch of the fused
// step kernel: its workgroups fill their own ghost slots (periodic images,
// boundary values, reconstruction from the parent's two stored time levels,
// reflux from the accumulator the finer level filled), add this sub-step's
// outgoing edge values into the parent's reflux accumulators, then stream and
// relax their cells. Because the stored state is post-collision, a level's
// step needs its parent's samples at t_n and t_n - dt_{l-1} (both buffers of
// the parent) and its children's r sub-steps to have completed (for the reflux),
// which the finest-first order guarantees.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <functional>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/vlbm.h"
#include "host_util.hpp"
#include "vlbm_internal.hpp"

using namespace vlbm;

namespace {

thread_local std::string g_err;

vlbm_status fail(vlbm_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(expr)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(VLBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

constexpr int kMaxLevels = VLBM_MAX_LEVELS;

using vlbm_host::PhaseTimer;
const int CX[4] = {1, -1, 0, 0};
const int CY[4] = {0, 0, 1, -1};

int tile_cells_default() {
  const char *e = getenv("VLBM_TILE_CELLS");
  int v = e ? atoi(e) : 256;
  if (v < 64) v = 64;
  if (v > (1 << 20)) v = 1 << 20;
  return v;
}

// ----------------------------------------------------------------------------
// Device memory: first-fit suballocation of a caller-bound region, or hipMalloc.
// ----------------------------------------------------------------------------
struct DevMem {
  char *base = nullptr;
  size_t size = 0;
  bool bound = false;
  // caller's allocator (vlbm_bind_allocator): every block comes from it
  vlbm_alloc_fn ext_alloc = nullptr;
  vlbm_free_fn ext_free = nullptr;
  void *ext_user = nullptr;
  std::map<size_t, size_t> free_;     // offset -> length
  std::map<void *, size_t> live_;     // pointer -> length (bound region)
  std::unordered_map<void *, size_t> owned_;  // hipMalloc'ed blocks in use -> length
  // Released hipMalloc'ed blocks kept for reuse (hipFree synchronises the
  // device; a regrid reallocates dozens of small tables). All of a context's
  // device work runs on its one stream, so a block reused by a later
  // stream-ordered operation cannot overlap the work that used it before.
  std::multimap<size_t, void *> cache_;
  size_t cached_ = 0;
  static constexpr size_t kCacheBlock = size_t(16) << 20, kCacheTotal = size_t(64) << 20;

  static size_t round(size_t n) { return (n + 255) & ~size_t(255); }

  void bind(void *p, size_t n) {
    base = static_cast<char *>(p);
    size = n & ~size_t(255);
    bound = true;
    free_.clear();
    live_.clear();
    size_t lead = (256 - (reinterpret_cast<uintptr_t>(base) & 255)) & 255;
    if (lead < size) free_[lead] = size - lead;
  }

  void *alloc(size_t n) {
    n = round(std::max<size_t>(n, 256));
    if (ext_alloc) {
      void *p = ext_alloc(n, ext_user);
      if (!p) return nullptr;
      if (reinterpret_cast<uintptr_t>(p) & 255) {  // the layout needs 256-byte alignment
        ext_free(p, ext_user);
        return nullptr;
      }
      owned_[p] = n;
      return p;
    }
    if (!bound) {
      auto c = cache_.lower_bound(n);
      if (c != cache_.end() && c->first <= 2 * n) {
        void *p = c->second;
        owned_[p] = c->first;
        cached_ -= c->first;
        cache_.erase(c);
        return p;
      }
      void *p = nullptr;
      if (hipMalloc(&p, n) != hipSuccess) {
        drop_cache();
        if (hipMalloc(&p, n) != hipSuccess) return nullptr;
      }
      owned_[p] = n;
      return p;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        void *p = base + off;
        live_[p] = n;
        return p;
      }
    }
    return nullptr;
  }

  void release(void *p) {
    if (!p) return;
    if (ext_alloc) {
      auto it = owned_.find(p);
      if (it == owned_.end()) return;
      owned_.erase(it);
      ext_free(p, ext_user);
      return;
    }
    if (!bound) {
      auto it = owned_.find(p);
      if (it == owned_.end()) return;
      const size_t n = it->second;
      owned_.erase(it);
      if (n <= kCacheBlock && cached_ + n <= kCacheTotal) {
        cache_.insert({n, p});
        cached_ += n;
      } else {
        (void)hipFree(p);
      }
      return;
    }
    auto it = live_.find(p);
    if (it == live_.end()) return;
    size_t off = static_cast<char *>(p) - base, len = it->second;
    live_.erase(it);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + len == nx->first) {
      len += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += len;
        return;
      }
    }
    free_[off] = len;
  }

  void drop_cache() {
    for (auto &kv : cache_) (void)hipFree(kv.second);
    cache_.clear();
    cached_ = 0;
  }

  void release_all() {
    for (auto &kv : owned_) {
      if (ext_alloc)
        ext_free(kv.first, ext_user);
      else
        (void)hipFree(kv.first);
    }
    owned_.clear();
    drop_cache();
    if (bound) bind(base, size);
  }
};

// Sorted, disjoint runs of level rows [y0, y1).
using Runs = std::vector<std::pair<int, int>>;

struct Level {
  bool present = false;
  int Nx = 0, Ny = 0;
  double dx = 0.0;
  // Frame: the columns of the coverage's bounding box plus one ghost column on
  // each side, over row runs that hold every covered row and its neighbour rows
  // (the ghost ring). Rows between runs are not stored: a level made of
  // separate bands (two shear layers, say) stores only the bands. Stored rows
  // follow each other in storage in increasing y, so the rows above and below
  // an active cell are one pitch away.
  int fx0 = 0, fy0 = 0, fw = 0, fh = 0;  // column and row range of the frame
  Runs runs;                              // stored rows
  std::vector<int32_t> srow;              // frame row (y - fy0) -> storage row, -1 if not stored
  std::vector<int32_t> yrow;              // storage row -> frame row (y - fy0)
  int nrows = 0;                          // stored rows
  int32_t *dsrow = nullptr, *dyrow = nullptr;  // device copies of srow and yrow
  int pitch = 0, xoff = 0;
  int64_t plane = 0;
  void *buf[2] = {nullptr, nullptr};
  uint8_t *dstatus = nullptr;
  void *dtables = nullptr;  // one block: dstatus, dsrow, dyrow and the tile, task and slot tables
  std::vector<uint8_t> cov;     // per frame cell: covered at this level
  std::vector<uint8_t> status;  // 0 none, 1 active, 2 hole
  std::vector<Tile> tiles;
  std::vector<Task> tasks;
  Tile *dtiles = nullptr;
  Task *dtasks = nullptr;
  // fused two-sub-step launch (finest level, r = 2): tiles of at most
  // FUSE_W x FUSE_H cells and their task lists
  std::vector<Tile> ftiles;
  std::vector<Task> ftasks;
  Tile *dftiles = nullptr;
  Task *dftasks = nullptr;
  double *dacc = nullptr;       // reflux accumulators of ring cells of this level
  int nacc = 0;
  double *dledger = nullptr;
  int nledger = 0;
  double *dpartial = nullptr;
  long steps = 0;  // buffer flips so far; its parity selects the current buffer
  // adaptive relaxation planes (SensorPlane, SEN_PLANES x sen_plane doubles)
  // and neighbour masks (sen_plane bytes), allocated while the sensor is on
  double *dsen = nullptr;
  uint32_t *dmask = nullptr;
  int64_t sen_plane = 0;
  std::vector<int64_t> reflux_key;  // per reflux slot: (y * Nx + x) * 4 + q of its ring cell

  // (x, y) must lie in the frame (in_frame)
  int64_t off(int x, int y) const {
    return (int64_t)srow[y - fy0] * pitch + (x - fx0) + xoff;
  }
  bool stored(int y) const { return y >= fy0 && y < fy0 + fh && srow[y - fy0] >= 0; }
  bool in_frame(int x, int y) const { return x >= fx0 && x < fx0 + fw && stored(y); }
  // index of frame cell (x, y) in the host arrays (cov, status: fw per stored row)
  size_t fidx(int x, int y) const { return (size_t)srow[y - fy0] * fw + (x - fx0); }
  int cur() const { return (int)(steps & 1); }
};

}  // namespace

namespace {
// One launch of a coarse step: segments [seg0, seg0 + nseg) of the segment
// table (parity e adds e times the table's half length).
struct LaunchRec {
  int32_t seg0 = 0, nseg = 0, nblocks = 0;
  int32_t first = 0;         // CAPTURE: first sub-step of the parent's cycle (step tiles)
  double ak = 0.0;           // reconstruction weight of the step tiles' sub-step
  int32_t fused_kernel = 0;  // launched as the fused kernel
  int32_t prof_key = 0;      // 2 * level + fused, for per-kernel timing
  double cells = 0.0;        // active cells the launch advances
  int32_t emit_cfl = 0;      // adaptive time step: the level's last launch of the coarse step
};
}  // namespace

struct vlbm_ctx {
  vlbm_params p{};
  hipStream_t stream = nullptr;
  double *noalloc_stage = nullptr;  // its GPU's static staging array (vlbm_get_state_noalloc)
  bool fp32 = false;
  size_t esz = 8;
  DevMem mem;
  Level lv[kMaxLevels];
  int nlev = 1;  // levels present (0..nlev-1)
  std::vector<vlbm_box> boxes;
  bool have_hierarchy = false;
  long coarse_steps = 0;
  int tile_cells = 256;
  int step_flags = 0;
  int *dflag = nullptr;
  double gm1 = 0, h = 0, tb = 0;
  EosT<double> eos{};
  // space/time-adaptive relaxation parameter (eq. sensor-B)
  bool sensor = false;
  double c_sensor = 1.0, beta_min = 1.0, beta_max = 1.0;
  unsigned long long *dqmax = nullptr;  // [2][4]: max |Q| per coarse-step parity, as bits
  bool sensor_stale = true;  // W planes and this coarse step's max |Q| need stage 0
  bool cfl_stale = true;     // the state changed since the last step launches: the CFL bound needs
                             // the full pass
  // adaptive time step: DynState scalars and the CFL max slot (device)
  bool adt = false;
  double *ddyn = nullptr;
  unsigned long long *dcmax = nullptr;
  int32_t s0_seg0 = 0, s0_nseg = 0, s0_nblocks = 0;  // stage 0: segments over every level
  double ledger_carry[4] = {0, 0, 0, 0}, ledger_carry_c[4] = {0, 0, 0, 0};
  // schedule tables: phases of one coarse step and their descriptors for the
  // two parities of the coarse step counter relative to table_base
  std::vector<std::pair<int, int>> phases;  // (level, k)
  std::vector<int32_t> phase_blocks;
  std::vector<LevelDesc> hdesc;  // host copy of the descriptor table
  LevelDesc *ddesc = nullptr;
  Segment *dseg = nullptr;
  long table_base = 0;
  long tables_version = 0;  // bumped by every rebuild of the launch tables
  long flips[kMaxLevels] = {};  // buffer flips of each level per coarse step
  bool use_graphs = false;
  hipGraphExec_t graph = nullptr;  // two coarse steps from an even table parity
  // per-kernel timing (vlbm_set_profiling): start and end events of every
  // step launch, read back in batches
  bool prof = false;
  std::vector<hipEvent_t> pev;  // event pool, two per pending launch
  std::vector<std::pair<int, double>> pend;  // pending launches: (2 * level + fused, cells)
  double prof_ms[2 * kMaxLevels] = {};
  long prof_calls[2 * kMaxLevels] = {};
  double prof_cells[2 * kMaxLevels] = {};
  // launches of one coarse step and their segment table (both parities)
  std::vector<LaunchRec> launches;
  std::vector<Segment> hseg;
  int nseg_table = 0;
  long graph_key = -1;
  // device scratch of tag_and_regrid (tags per level, tile bits and lists,
  // counts), kept between calls and grown on demand: slot -> (pointer, bytes)
  std::vector<std::pair<void *, size_t>> tag_scratch;
  int tag_kind = VLBM_TAG_DENSITY;              // refinement indicator (vlbm_set_tag_indicator)
  unsigned long long *dflux_qmax = nullptr;     // [4] its domain-wide flux maxima (bits)
  void *scratch_slot(size_t slot, size_t bytes) {
    if (tag_scratch.size() <= slot) tag_scratch.resize(slot + 1, {nullptr, 0});
    auto &e = tag_scratch[slot];
    if (e.second < bytes) {
      mem.release(e.first);
      e.first = mem.alloc(std::max<size_t>(bytes, 256));
      e.second = e.first ? bytes : 0;
    }
    return e.first;
  }

  // pinned host staging of table uploads (stage_h2d)
  char *stage = nullptr;
  size_t stage_cap = 0, stage_used = 0;

  bool perx() const { return p.bc[0] == VLBM_BC_PERIODIC; }
  bool pery() const { return p.bc[2] == VLBM_BC_PERIODIC; }
  bool wrap(int l, int &x, int &y) const {
    const Level &L = lv[l];
    if (x < 0 || x >= L.Nx) {
      if (!perx()) return false;
      x = ((x % L.Nx) + L.Nx) % L.Nx;
    }
    if (y < 0 || y >= L.Ny) {
      if (!pery()) return false;
      y = ((y % L.Ny) + L.Ny) % L.Ny;
    }
    return true;
  }
  // (x, y) must be in-domain coordinates of level l.
  bool covered(int l, int x, int y) const {
    if (l >= kMaxLevels || !lv[l].present) return false;
    const Level &L = lv[l];
    if (!L.in_frame(x, y)) return false;
    return L.cov[L.fidx(x, y)] != 0;
  }
  bool active(int l, int x, int y) const {
    if (!covered(l, x, y)) return false;
    if (l + 1 < kMaxLevels && covered(l + 1, x * p.r, y * p.r)) return false;
    return true;
  }
};

namespace {

void drop_batch_graphs(vlbm_ctx *c);  // captured batches that hold c (vlbm_batch_advance)

void free_level(vlbm_ctx *c, Level &L) {
  c->mem.release(L.buf[0]);
  c->mem.release(L.buf[1]);
  c->mem.release(L.dtables);  // status, row maps, tiles, tasks, slots (upload_level)
  c->mem.release(L.dsen);
  c->mem.release(L.dmask);
  long steps = L.steps;
  L = Level();
  L.steps = steps;
}

// --------------------------------------------------------------------------
// Hierarchy geometry (host)
// --------------------------------------------------------------------------
struct Geometry {
  bool present[kMaxLevels] = {};
  int bx0[kMaxLevels], by0[kMaxLevels], bx1[kMaxLevels], by1[kMaxLevels];
  Runs rows[kMaxLevels];  // rows each level's frame stores
};

// Runs closer than kRowGap rows are stored as one (fewer runs, little memory).
constexpr int kRowGap = 16;
// Rows a growing level adds beyond those it needs (a regrid that moves a band
// by a few rows then reuses the frame).
constexpr int kRowPad = 16;

Runs merge_runs(Runs v) {
  std::sort(v.begin(), v.end());
  Runs out;
  for (const auto &r : v) {
    if (!out.empty() && r.first <= out.back().second + kRowGap)
      out.back().second = std::max(out.back().second, r.second);
    else
      out.push_back(r);
  }
  return out;
}

// every run of `inner` lies inside a run of `outer`
bool runs_cover(const Runs &outer, const Runs &inner) {
  size_t j = 0;
  for (const auto &r : inner) {
    while (j < outer.size() && outer[j].second < r.second) ++j;
    if (j == outer.size() || outer[j].first > r.first) return false;
  }
  return true;
}

vlbm_status check_boxes(const vlbm_params &p, const vlbm_box *boxes, int n, Geometry &g) {
  for (int l = 0; l < kMaxLevels; ++l) {
    g.present[l] = false;
    g.bx0[l] = g.by0[l] = 1 << 30;
    g.bx1[l] = g.by1[l] = -(1 << 30);
  }
  g.present[0] = true;
  g.bx0[0] = 0;
  g.by0[0] = 0;
  g.bx1[0] = p.nx0;
  g.by1[0] = p.ny0;
  for (int l = 0; l < kMaxLevels; ++l) g.rows[l].clear();
  g.rows[0].push_back({-1, p.ny0 + 1});
  if (n < 0 || (n > 0 && !boxes)) return fail(VLBM_EINVAL, "bad box list");
  for (int b = 0; b < n; ++b) {
    const vlbm_box &B = boxes[b];
    if (B.level < 1 || B.level >= p.max_levels)
      return fail(VLBM_EINVAL, "box %d: level %d outside 1..%d", b, B.level, p.max_levels - 1);
    long s = 1;
    for (int i = 0; i < B.level; ++i) s *= p.r;
    long Nx = p.nx0 * s, Ny = p.ny0 * s;
    if (B.nx <= 0 || B.ny <= 0 || B.i0 < 0 || B.j0 < 0 || B.i0 + (long)B.nx > Nx ||
        B.j0 + (long)B.ny > Ny)
      return fail(VLBM_EINVAL, "box %d lies outside its level's domain", b);
    if (B.i0 % p.r || B.j0 % p.r || B.nx % p.r || B.ny % p.r)
      return fail(VLBM_ENEST, "box %d is not made of whole parent cells (ratio %d)", b, p.r);
    int l = B.level;
    g.present[l] = true;
    g.bx0[l] = std::min(g.bx0[l], B.i0);
    g.by0[l] = std::min(g.by0[l], B.j0);
    g.bx1[l] = std::max(g.bx1[l], B.i0 + B.nx);
    g.by1[l] = std::max(g.by1[l], B.j0 + B.ny);
    g.rows[l].push_back({B.j0 - 1, B.j0 + B.ny + 1});
  }
  for (int l = 1; l < kMaxLevels; ++l)
    if (g.present[l] && !g.present[l - 1])
      return fail(VLBM_ENEST, "level %d has boxes but level %d has none", l, l - 1);
  for (int l = 0; l < kMaxLevels; ++l) g.rows[l] = merge_runs(std::move(g.rows[l]));
  return VLBM_OK;
}

// A level that persists through a regrid keeps its frame when the new
// coverage fits in it; otherwise its frame grows to hold old and new rows
// (new rows padded by kRowPad), so a slowly moving band reallocates rarely.
void grow_geometry(Geometry &g, int l, const Level &O, int Ny) {
  if (!g.present[l] || !O.present) return;
  g.bx0[l] = std::min(g.bx0[l], O.fx0 + 1);
  g.bx1[l] = std::max(g.bx1[l], O.fx0 + O.fw - 1);
  g.by0[l] = std::min(g.by0[l], O.fy0 + 1);
  g.by1[l] = std::max(g.by1[l], O.fy0 + O.fh - 1);
  if (runs_cover(O.runs, g.rows[l])) {
    g.rows[l] = O.runs;
    return;
  }
  Runs v = O.runs;
  for (const auto &r : g.rows[l])
    v.push_back({std::max(-1, r.first - kRowPad), std::min(Ny + 1, r.second + kRowPad)});
  g.rows[l] = merge_runs(std::move(v));
}

void frame_of(const vlbm_params &p, size_t esz, const Geometry &g, int l, Level &L) {
  long s = 1;
  for (int i = 0; i < l; ++i) s *= p.r;
  L.Nx = (int)(p.nx0 * s);
  L.Ny = (int)(p.ny0 * s);
  L.dx = p.dx0 / (double)s;
  L.present = g.present[l];
  L.runs.clear();
  L.srow.clear();
  L.yrow.clear();
  L.nrows = 0;
  if (!L.present) {
    L.fx0 = L.fy0 = L.fw = L.fh = L.pitch = L.xoff = 0;
    L.plane = 0;
    return;
  }
  L.fx0 = g.bx0[l] - 1;
  L.fw = g.bx1[l] - g.bx0[l] + 2;
  L.runs = g.rows[l];
  L.fy0 = L.runs.front().first;
  L.fh = L.runs.back().second - L.fy0;
  L.srow.assign(L.fh, -1);
  for (const auto &r : L.runs)
    for (int y = r.first; y < r.second; ++y) {
      L.srow[y - L.fy0] = (int32_t)L.yrow.size();
      L.yrow.push_back(y - L.fy0);
    }
  L.nrows = (int)L.yrow.size();
  // The first interior column starts on a 128-byte line; rows are padded to 64
  // elements and every population plane to a multiple of 4 KiB. Measured on
  // MI355X for a 4096^2 FP64 frame: a plane stride of 512 B mod 4 KiB runs the
  // step kernel at 4.4 TB/s, 4 KiB-aligned planes at 5.1-5.25 TB/s.
  const int align = (int)(128 / esz);
  L.xoff = align - 1;
  L.pitch = (L.fw + L.xoff + 63) / 64 * 64;
  const int64_t pa = 4096 / (int64_t)esz;
  L.plane = ((int64_t)L.pitch * L.nrows + pa - 1) / pa * pa;
}

size_t level_bytes(const Level &L, size_t esz) { return (size_t)L.plane * 16 * esz; }

int align_up(int v, int a) { return (v + a - 1) / a * a; }  // v >= 0

// Build coverage, check nesting, build status, tiles and tasks for all levels.
// What fills the slot from which active cell (x, y) of level l pulls f_q
// (t.kind == T_NONE: an active cell of the same level, read in place). t.dst is
// the slot's element offset; slots of BC and REFLUX tasks are assigned by the
// caller.
vlbm_status ghost_task(const vlbm_ctx *c, int l, int x, int y, int q, Task &t) {
  const vlbm_params &p = c->p;
  const int r = p.r;
  const Level &L = c->lv[l];
  const int sx = x - CX[q], sy = y - CY[q];
  int wx = sx, wy = sy;
  t = Task{};
  t.kind = T_NONE;
  t.q = q;
  t.dst = (int32_t)L.off(sx, sy);
  t.n0 = t.n1 = -1;
  // A level's status holds its coverage and that of the next finer level
  // (proper nesting): 1 active, 2 under a finer box (covered at l + 1), 0 not
  // covered; cells outside the frame are not covered.
  auto status = [&](int lv, int ax, int ay) -> int {
    const Level &A = c->lv[lv];
    return A.in_frame(ax, ay) ? A.status[A.fidx(ax, ay)] : 0;
  };
  int s;
  if (!c->wrap(l, wx, wy)) {
    const int side = q;  // +x enters through west (0), -x east (1), +y south (2), -y north (3)
    const int bc = p.bc[side];
    t.kind = (bc == VLBM_BC_OUTFLOW ? T_OUTFLOW : bc == VLBM_BC_REFLECT ? T_REFLECT : T_INFLOW) | TASK_LEDGER;
    t.src = (int32_t)L.off(x, y);
    t.n0 = side;
  } else if ((s = status(l, wx, wy)) == 2) {
    t.kind = T_REFLUX;
  } else if (s == 1) {
    if (wx != sx || wy != sy) {
      t.kind = T_COPY;
      t.src = (int32_t)L.off(wx, wy);
    }
  } else {
    if (l == 0) return fail(VLBM_ENEST, "internal: level-0 cell without source");
    const Level &PL = c->lv[l - 1];
    int px = wx / r, py = wy / r;
    if (status(l - 1, px, py) != 1)
      return fail(VLBM_ENEST, "level %d cell (%d,%d): parent ring cell inactive", l, x, y);
    t.kind = T_RECON;
    t.src = (int32_t)PL.off(px, py);
    int tx = q < 2 ? 0 : 1, ty = q < 2 ? 1 : 0;
    t.j = q < 2 ? (y - r * py) : (x - r * px);
    int mx = px - tx, my = py - ty, qx = px + tx, qy = py + ty;
    bool have = c->wrap(l - 1, mx, my) && c->wrap(l - 1, qx, qy) && status(l - 1, mx, my) == 1 &&
                status(l - 1, qx, qy) == 1;
    if (have) {
      t.n0 = (int32_t)PL.off(mx, my);
      t.n1 = (int32_t)PL.off(qx, qy);
    }
  }
  return VLBM_OK;
}

// Lists of the fused two-sub-step launch of level l (the finest, r = 2).
// Active cells are cut into rectangles of at most FUSE_W x FUSE_H cells
// aligned to a FUSE_W x FUSE_H grid from the frame's first interior cell.
// Coverage of the finest level is a union of r x r blocks aligned like that
// cell, and both sides are even, so every rectangle is too: both cells of a reflux
// capture lie in one tile. LDS positions follow the per-population layout of
// the fused kernel (see FUSE_POS). Per tile, in this order:
//   ntask  sub-step-1 ghost tasks of every cell whose sub-step-1 value the tile
//          needs (its own cells, which book the ledger, and the sources of its
//          ring positions, which do not);
//   nring  ring positions holding an active cell (T_RING: global source cell,
//          the periodic partner for a wrapped position; LDS destination);
//   nk2    sub-step-2 ghost values of the remaining ring positions (TASK_K2:
//          boundary tasks read the tile cell's LDS value, RECON reads the parent);
//   ncap   reflux captures whose first cell R_0 lies in the tile (T_CAPTURE2).
// A ring position touches exactly one tile cell, which pulls exactly one
// population from it, so every ring entry is that one (cell, q) pair.
vlbm_status build_fused(vlbm_ctx *c, int l, const std::unordered_map<int64_t, int> &bc_slot,
                        const std::vector<std::pair<int64_t, Task>> &caps) {
  Level &L = c->lv[l];
  // rectangles: per row, runs of active cells cut at the FUSE_W grid; equal
  // runs on consecutive rows of one FUSE_H band stack into one rectangle
  struct Rect { int x0, y0, w, h; };
  std::vector<Rect> rects;
  std::map<std::pair<int, int>, int> open;  // (x0, w) -> index in rects (current band)
  for (int y = L.fy0 + 1; y < L.fy0 + L.fh - 1; ++y) {
    if ((y - L.fy0 - 1) % FUSE_H == 0) open.clear();
    if (!L.stored(y)) continue;  // no active cell (rectangles need consecutive rows)
    std::map<std::pair<int, int>, int> next;
    int x = L.fx0 + 1;
    const int xe = L.fx0 + L.fw - 1;
    while (x < xe) {
      if (L.status[L.fidx(x, y)] != 1) {
        ++x;
        continue;
      }
      const int xa = x;
      const int cut = L.fx0 + 1 + ((x - L.fx0 - 1) / FUSE_W + 1) * FUSE_W;
      while (x < xe && x < cut && L.status[L.fidx(x, y)] == 1) ++x;
      const std::pair<int, int> key{xa, x - xa};
      auto it = open.find(key);
      if (it != open.end() && rects[it->second].y0 + rects[it->second].h == y) {
        rects[it->second].h += 1;
        next[key] = it->second;
      } else {
        rects.push_back({xa, y, x - xa, 1});
        next[key] = (int)rects.size() - 1;
      }
    }
    open.swap(next);
  }
  std::sort(rects.begin(), rects.end(), [](const Rect &a, const Rect &b) {
    return a.y0 != b.y0 ? a.y0 < b.y0 : a.x0 < b.x0;
  });
  std::vector<int32_t> owner(L.cov.size(), -1);
  for (size_t t = 0; t < rects.size(); ++t)
    for (int yy = 0; yy < rects[t].h; ++yy)
      for (int xx = 0; xx < rects[t].w; ++xx) owner[L.fidx(rects[t].x0 + xx, rects[t].y0 + yy)] = (int32_t)t;
  std::vector<std::vector<Task>> capt(rects.size());
  // LDS position of cell (x, y) in the plane group of population q, for tile R
  auto pos = [](const Rect &R, int q, int x, int y) -> int32_t {
    const int cx = x - R.x0, cy = y - R.y0;
    switch (q) {
      case 0: return cy * (R.w + 1) + cx + 1;
      case 1: return cy * (R.w + 1) + cx;
      case 2: return (cy + 1) * R.w + cx;
      default: return cy * R.w + cx;
    }
  };
  for (const auto &ct : caps) {
    const int x = (int)(ct.first % L.Nx), y = (int)(ct.first / L.Nx);
    const int t = owner[L.fidx(x, y)];
    const Rect &R = rects[t];
    Task u = ct.second;
    u.kind = T_CAPTURE2;
    u.n1 = pos(R, u.q, x, y);
    u.j = u.q < 2 ? R.w + 1 : 1;
    const int x1 = x + (u.q < 2 ? 0 : 1), y1 = y + (u.q < 2 ? 1 : 0);
    if (x1 >= R.x0 + R.w || y1 >= R.y0 + R.h)
      return fail(VLBM_ENEST, "internal: reflux capture split across fused tiles");
    capt[t].push_back(u);
  }
  std::vector<uint8_t> mark(L.cov.size(), 0);
  std::vector<size_t> marked;
  L.ftiles.clear();
  L.ftasks.clear();
  for (size_t ti = 0; ti < rects.size(); ++ti) {
    const Rect &R = rects[ti];
    auto in_tile = [&](int x, int y) { return x >= R.x0 && y >= R.y0 && x < R.x0 + R.w && y < R.y0 + R.h; };
    std::vector<std::pair<int, int>> src_cells;  // ring sources outside the tile
    std::vector<Task> ring, k2;
    for (int y = R.y0; y < R.y0 + R.h; ++y)
      for (int x = R.x0; x < R.x0 + R.w; ++x) {
        if (x > R.x0 && x < R.x0 + R.w - 1 && y > R.y0 && y < R.y0 + R.h - 1) continue;
        for (int q = 0; q < 4; ++q) {
          const int sx = x - CX[q], sy = y - CY[q];
          if (in_tile(sx, sy)) continue;
          Task t{};
          vlbm_status gs = ghost_task(c, l, x, y, q, t);
          if (gs) return gs;
          const int kind = t.kind == T_NONE ? T_NONE : t.kind & 0xFF;
          Task u = t;
          u.dst = pos(R, q, sx, sy);
          if (kind == T_NONE || kind == T_COPY) {
            int wx = sx, wy = sy;
            c->wrap(l, wx, wy);
            u.kind = T_RING;
            u.src = (int32_t)L.off(wx, wy);
            ring.push_back(u);
            if (!in_tile(wx, wy)) {
              const size_t fi = L.fidx(wx, wy);
              if (!mark[fi]) {
                mark[fi] = 1;
                marked.push_back(fi);
                src_cells.push_back({wx, wy});
              }
            }
          } else if (kind == T_RECON) {
            u.kind = T_RECON | TASK_K2;
            k2.push_back(u);
          } else if (kind == T_OUTFLOW || kind == T_REFLECT || kind == T_INFLOW) {
            auto it = bc_slot.find(((int64_t)y * L.Nx + x) * 4 + q);
            if (it == bc_slot.end()) return fail(VLBM_ENEST, "internal: no ledger slot for a fused boundary task");
            u.kind = kind | TASK_K2 | TASK_LEDGER;
            u.src = pos(R, q, x, y);
            u.n1 = pos(R, q ^ 1, x, y);
            u.slot = it->second;
            k2.push_back(u);
          } else {
            return fail(VLBM_ENEST, "internal: reflux slot on the finest level");
          }
        }
      }
    for (size_t fi : marked) mark[fi] = 0;
    marked.clear();
    // sub-step-1 ghost tasks: tile cells (with ledger) then ring sources (without)
    Tile tl{};
    tl.off0 = (int32_t)L.off(R.x0, R.y0);
    tl.w = R.w;
    tl.h = R.h;
    tl.task0 = (int32_t)L.ftasks.size();
    auto add_cell = [&](int x, int y, bool own) -> vlbm_status {
      const size_t ci = L.fidx(x, y);
      if (L.status[ci - 1] == 1 && L.status[ci + 1] == 1 && L.status[ci - L.fw] == 1 &&
          L.status[ci + L.fw] == 1)
        return VLBM_OK;
      for (int q = 0; q < 4; ++q) {
        Task t{};
        vlbm_status gs = ghost_task(c, l, x, y, q, t);
        if (gs) return gs;
        if (t.kind == T_NONE) continue;
        const int kind = t.kind & 0xFF;
        if (kind == T_REFLUX) return fail(VLBM_ENEST, "internal: reflux slot on the finest level");
        if (kind == T_OUTFLOW || kind == T_REFLECT || kind == T_INFLOW) {
          auto it = bc_slot.find(((int64_t)y * L.Nx + x) * 4 + q);
          if (it == bc_slot.end()) return fail(VLBM_ENEST, "internal: no ledger slot for a fused boundary task");
          t.slot = it->second;
          if (!own) t.kind &= ~TASK_LEDGER;
        }
        L.ftasks.push_back(t);
      }
      return VLBM_OK;
    };
    for (int y = R.y0; y < R.y0 + R.h; ++y)
      for (int x = R.x0; x < R.x0 + R.w; ++x) {
        vlbm_status as = add_cell(x, y, true);
        if (as) return as;
      }
    for (auto &sc : src_cells) {
      vlbm_status as = add_cell(sc.first, sc.second, false);
      if (as) return as;
    }
    tl.ntask = (int32_t)L.ftasks.size() - tl.task0;
    tl.nring = (int32_t)ring.size();
    tl.nk2 = (int32_t)k2.size();
    tl.ncap = (int32_t)capt[ti].size();
    L.ftasks.insert(L.ftasks.end(), ring.begin(), ring.end());
    L.ftasks.insert(L.ftasks.end(), k2.begin(), k2.end());
    L.ftasks.insert(L.ftasks.end(), capt[ti].begin(), capt[ti].end());
    if (R.w > FUSE_W || R.h > FUSE_H || R.x0 % 2 || R.y0 % 2 || R.w % 2 || R.h % 2)
      return fail(VLBM_ENEST, "internal: fused tile %dx%d at (%d,%d) not block aligned", R.w, R.h, R.x0, R.y0);
    L.ftiles.push_back(tl);
  }
  return VLBM_OK;
}

// An entry point's body that builds host tables: an exception (host memory
// exhausted) becomes a status, not a throw across the C ABI.
template <class F>
vlbm_status guarded(F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return fail(VLBM_ENOMEM, "host memory exhausted");
  } catch (...) {
    return fail(VLBM_EINVAL, "internal error in a host section");
  }
}

// Run f(i) for i in [0, n) on the process's worker pool and this thread
// (independent items, in any order and concurrency). The status of the lowest
// failing index is returned, with its message (messages are per thread).
vlbm_status run_parallel(int n, const std::function<vlbm_status(int)> &f) {
  if (n <= 1) return n == 1 ? f(0) : VLBM_OK;
  std::vector<vlbm_status> st(n, VLBM_OK);
  std::vector<std::string> err(n);
  vlbm_host::Pool::get().run(n, [&](int i) {
    try {  // no exception leaves a section (nor the C ABI above it)
      st[i] = f(i);
    } catch (const std::bad_alloc &) {
      st[i] = fail(VLBM_ENOMEM, "host memory exhausted");
    } catch (...) {
      st[i] = fail(VLBM_EINVAL, "internal error in a host section");
    }
    if (st[i]) err[i] = g_err;
  });
  for (int i = 0; i < n; ++i)
    if (st[i]) {
      g_err = err[i];
      return st[i];
    }
  return VLBM_OK;
}

// Coverage, proper nesting and cell status of every present level of c, from
// the boxes.
vlbm_status build_coverage(vlbm_ctx *c, const vlbm_box *boxes, int n) {
  PhaseTimer tm("build_coverage");
  const vlbm_params &p = c->p;
  const int r = p.r;
  int nlev = 0;
  while (nlev < kMaxLevels && c->lv[nlev].present) ++nlev;
  // coverage, one level per thread
  std::vector<std::vector<int>> of_level(nlev + 1);  // box indices per level
  for (int b = 0; b < n; ++b)
    if (boxes[b].level >= 0 && boxes[b].level < nlev) of_level[boxes[b].level].push_back(b);
  vlbm_status cst = run_parallel(nlev, [&](int l) -> vlbm_status {
    Level &L = c->lv[l];
    L.cov.assign((size_t)L.fw * L.nrows, 0);
    if (l == 0)
      for (int y = 0; y < L.Ny; ++y) memset(&L.cov[L.fidx(0, y)], 1, L.Nx);
    for (int b : of_level[l])
      for (int y = boxes[b].j0; y < boxes[b].j0 + boxes[b].ny; ++y)
        memset(&L.cov[L.fidx(boxes[b].i0, y)], 1, boxes[b].nx);
    return VLBM_OK;
  });
  if (cst) return cst;
  // proper nesting: a covered cell's parent and the parent's 4 neighbours are
  // covered. Per box: its parent rectangle, widened by one cell along x on its
  // rows and along y on its columns (wrapped on periodic axes; cells outside a
  // non-periodic side are exempt).
  for (int b = 0; b < n; ++b) {
    const int l = boxes[b].level;
    if (l < 1) continue;
    const Level &PL = c->lv[l - 1];
    const int x0 = boxes[b].i0 / r, x1 = (boxes[b].i0 + boxes[b].nx) / r;
    const int y0 = boxes[b].j0 / r, y1 = (boxes[b].j0 + boxes[b].ny) / r;
    auto need = [&](int qx, int qy, int px, int py) -> vlbm_status {
      int wx = qx, wy = qy;
      if (!c->wrap(l - 1, wx, wy) || c->covered(l - 1, wx, wy)) return VLBM_OK;
      return fail(VLBM_ENEST, "level %d cell (%d,%d): parent neighbour (%d,%d) not covered at level %d",
                  l, px * r, py * r, wx, wy, l - 1);
    };
    for (int y = y0; y < y1; ++y) {
      if (PL.in_frame(x0, y) && PL.in_frame(x1 - 1, y)) {
        const uint8_t *row = &PL.cov[PL.fidx(x0, y)];
        const void *z = memchr(row, 0, x1 - x0);
        if (z) {
          const int x = x0 + (int)(static_cast<const uint8_t *>(z) - row);
          return need(x, y, x, y);
        }
      } else {
        for (int x = x0; x < x1; ++x) {
          vlbm_status st = need(x, y, x, y);
          if (st) return st;
        }
      }
      vlbm_status st = need(x0 - 1, y, x0, y);
      if (!st) st = need(x1, y, x1 - 1, y);
      if (st) return st;
    }
    for (int x = x0; x < x1; ++x) {
      vlbm_status st = need(x, y0 - 1, x, y0);
      if (!st) st = need(x, y1, x, y1 - 1);
      if (st) return st;
    }
  }
  tm.mark("coverage+nesting");
  // status: covered cells are active (1), those under a finer box are holes
  // (2); one level per thread
  cst = run_parallel(nlev, [&](int l) -> vlbm_status {
    Level &L = c->lv[l];
    L.status = L.cov;
    for (int b : of_level[l + 1]) {
      const int x0 = boxes[b].i0 / r, x1 = (boxes[b].i0 + boxes[b].nx) / r;
      for (int y = boxes[b].j0 / r; y < (boxes[b].j0 + boxes[b].ny) / r; ++y)
        memset(&L.status[L.fidx(x0, y)], 2, x1 - x0);
    }
    return VLBM_OK;
  });
  if (cst) return cst;
  tm.mark("status");
  return VLBM_OK;
}

// Tiles, ghost tasks, reflux and ledger slots, captures and fused lists of
// every present level of c (after build_coverage). Reads the levels' frames,
// coverage and status; writes only their lists.
vlbm_status build_task_lists(vlbm_ctx *c) {
  PhaseTimer tm("build_task_lists");
  const int r = c->p.r;
  int nlev = 0;
  while (nlev < kMaxLevels && c->lv[nlev].present) ++nlev;
  // Per level, two passes; the levels of a pass run on threads of their own.
  // Pass A: tiles, cell -> tile map, ghost tasks, reflux and ledger slots.
  // Pass B (needs the parent's reflux slots): captures, task order, fused lists.
  struct Work {
    // cell -> tile: per stored row, the tiles crossing it as frame-column
    // ranges [x0, x1), ordered by x0 (rows row0[s] .. row0[s + 1] of own)
    struct Own {
      int32_t x0, x1, tile;
    };
    std::vector<int32_t> row0;
    std::vector<Own> own;
    int32_t owner(const Level &L, int64_t fi) const {  // fi: frame index of an active cell
      const int s = (int)(fi / L.fw), fx = (int)(fi % L.fw);
      const Own *b = own.data() + row0[s], *e = own.data() + row0[s + 1];
      const Own *it = std::upper_bound(b, e, fx, [](int v, const Own &o) { return v < o.x0; });
      return (it != b && fx < (it - 1)->x1) ? (it - 1)->tile : -1;
    }
    std::vector<std::pair<int, Task>> tk;       // (tile, task)
    std::unordered_map<int64_t, int> bc_slot;   // (cell, q) -> ledger slot (fused level)
    std::vector<std::pair<int64_t, Task>> caps; // (cell R_0 as y * Nx + x, capture) (fused level)
    bool fuse = false;
    vlbm_status st = VLBM_OK;
    std::string err;
  };
  std::vector<Work> W(nlev);
  const int TCfull = c->tile_cells;
  auto passA = [&](int l) -> vlbm_status {
    PhaseTimer lt(l == 0 ? "passA l0" : l == 1 ? "passA l1" : l == 2 ? "passA l2" : "passA l3+");
    Level &L = c->lv[l];
    Work &w = W[l];
    // tiles: runs of active cells per row, stacked into rectangles of <= TC cells
    const bool sen_tiles = c->sensor;
    struct Open { int xa, xb, y0, h; };
    std::vector<Open> open, nopen;
    std::vector<std::pair<int, int>> rect_xy;  // (x0, y0) of each emitted tile
    // With STEP_SMALL_TILES, a level too small to fill the chip with tiles of
    // TCfull cells (fewer than 4096 of them) gets tiles of half the size,
    // down to 64 cells.
    const int kMinTiles = (c->step_flags & STEP_SMALL_TILES) ? 4096 : 0;
    for (int TC = TCfull;; TC /= 2) {
    L.tiles.clear();
    rect_xy.clear();
    open.clear();
    auto emit = [&](const Open &o) {
      // split wide rectangles (h == 1) into chunks of at most TC cells
      for (int x = o.xa; x < o.xb; x += TC) {
        Tile u{};
        u.w = std::min(TC, o.xb - x);
        u.h = o.h;
        u.off0 = (int32_t)L.off(x, o.y0);
        L.tiles.push_back(u);
        rect_xy.push_back({x, o.y0});
      }
    };
    for (int y = L.fy0; y < L.fy0 + L.fh; ++y) {
      nopen.clear();
      if (!L.stored(y)) {  // no active cell: close every open rectangle
        for (const Open &o : open) emit(o);
        open.clear();
        continue;
      }
      const uint8_t *row = &L.status[L.fidx(L.fx0, y)];
      size_t j = 0;  // open rectangles are ordered by xa, like the runs of a row
      int x = 0;
      constexpr uint64_t ones = 0x0101010101010101ull;
      while (x < L.fw) {
        if (row[x] != 1) {  // to the next active cell
          const void *nx = memchr(row + x, 1, L.fw - x);
          if (!nx) break;
          x = (int)(static_cast<const uint8_t *>(nx) - row);
        }
        const int xa = x;
        for (uint64_t v; x + 8 <= L.fw && (memcpy(&v, row + x, 8), v == ones);) x += 8;
        while (x < L.fw && row[x] == 1) ++x;
        // with the adaptive relaxation, runs are cut on a SEN_TW grid from the
        // frame's first interior column and stacked at most SEN_TH high
        for (int ca = L.fx0 + xa; ca < L.fx0 + x;) {
          const int cb = sen_tiles ? std::min(L.fx0 + x, L.fx0 + 1 + ((ca - L.fx0 - 1) / SEN_TW + 1) * SEN_TW)
                                   : L.fx0 + x;
          const int a = ca, b = cb, maxh = sen_tiles ? SEN_TH : std::max(1, TC / (b - a));
          ca = cb;
          while (j < open.size() && open[j].xa < a) emit(open[j++]);
          if (j < open.size() && open[j].xa == a && open[j].xb == b) {
            if (open[j].h < maxh) {
              nopen.push_back({a, b, open[j].y0, open[j].h + 1});
              ++j;
              continue;
            }
            emit(open[j++]);
          }
          nopen.push_back({a, b, y, 1});
        }
      }
      while (j < open.size()) emit(open[j++]);
      open.swap(nopen);
    }
    for (const Open &o : open) emit(o);
    if (sen_tiles || TC <= 64 || (int64_t)L.tiles.size() >= kMinTiles) break;
    }
    // order tiles by (y0, x0) for locality
    std::vector<int> order(L.tiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      return rect_xy[a].second != rect_xy[b].second ? rect_xy[a].second < rect_xy[b].second
                                                    : rect_xy[a].first < rect_xy[b].first;
    });
    std::vector<Tile> sorted(order.size());
    std::vector<std::pair<int, int>> sxy(order.size());
    for (size_t i = 0; i < order.size(); ++i) {
      sorted[i] = L.tiles[order[i]];
      sxy[i] = rect_xy[order[i]];
    }
    L.tiles.swap(sorted);
    rect_xy.swap(sxy);
    lt.mark("tiles");
    // cell -> tile: the tiles crossing each stored row
    {
      const int nt = (int)L.tiles.size();
      w.row0.assign((size_t)L.nrows + 1, 0);
      for (int t = 0; t < nt; ++t)
        for (int yy = 0; yy < L.tiles[t].h; ++yy) w.row0[L.srow[rect_xy[t].second + yy - L.fy0] + 1] += 1;
      for (int s2 = 0; s2 < L.nrows; ++s2) w.row0[s2 + 1] += w.row0[s2];
      w.own.resize(w.row0[L.nrows]);
      std::vector<int32_t> at(w.row0.begin(), w.row0.end() - 1);
      for (int t = 0; t < nt; ++t) {
        const int x0 = rect_xy[t].first - L.fx0;
        for (int yy = 0; yy < L.tiles[t].h; ++yy)
          w.own[at[L.srow[rect_xy[t].second + yy - L.fy0]]++] = {x0, x0 + L.tiles[t].w, t};
      }
      for (int s2 = 0; s2 < L.nrows; ++s2)
        std::sort(w.own.begin() + w.row0[s2], w.own.begin() + w.row0[s2 + 1],
                  [](const Work::Own &a, const Work::Own &b) { return a.x0 < b.x0; });
    }
    vlbm_status st = VLBM_OK;
    lt.mark("owner");
    // ghost tasks, found per band of rows in parallel, then numbered in row order
    L.reflux_key.clear();
    L.nledger = 0;
    // the finest level of a two-level-or-deeper hierarchy with r = 2 also gets
    // the lists of the fused two-sub-step launch
    w.fuse = (c->step_flags & STEP_FUSE2) && l >= 1 && l == nlev - 1 && r == 2;
    const int fw = L.fw, ya = L.fy0 + 1, yb = L.fy0 + L.fh - 1;
    // 1. active cells with a non-active upwind neighbour, per band of rows
    const int B = std::max(1, std::min({8, (yb - ya) / 16, (int)(L.cov.size() >> 18)}));
    std::vector<std::vector<int32_t>> edge(B);  // frame indices, row order
    st = run_parallel(B, [&](int b) -> vlbm_status {
      constexpr uint64_t ones = 0x0101010101010101ull;
      auto all8 = [&](const uint8_t *p) {
        uint64_t v;
        memcpy(&v, p, 8);
        return v == ones;
      };
      for (int y = ya + (int)((int64_t)(yb - ya) * b / B); y < ya + (int)((int64_t)(yb - ya) * (b + 1) / B); ++y) {
        if (!L.stored(y)) continue;
        const size_t r0 = L.fidx(L.fx0, y);
        const uint8_t *sr = &L.status[r0];
        for (int xi = 1; xi < fw - 1;) {
          if (sr[xi] != 1) {  // to the next active cell
            const void *nx = memchr(sr + xi, 1, fw - 1 - xi);
            if (!nx) break;
            xi = (int)(static_cast<const uint8_t *>(nx) - sr);
          }
          // (the rows of an active cell's neighbours are stored next to its row)
          // eight interior cells at once: cells xi - 1 .. xi + 8 of the row and
          // xi .. xi + 7 of the rows below and above active
          if (xi + 8 < fw && all8(sr + xi - 1) && all8(sr + xi + 1) && all8(sr + xi - fw) && all8(sr + xi + fw)) {
            xi += 8;
            continue;
          }
          // interior cell: all four upwind neighbours active at this level (hence
          // inside the domain) -> plain pulls, no task
          if (!(sr[xi - 1] == 1 && sr[xi + 1] == 1 && sr[xi - fw] == 1 && sr[xi + fw] == 1))
            edge[b].push_back((int32_t)(r0 + xi));
          ++xi;
        }
      }
      return VLBM_OK;
    });
    if (st) return st;
    std::vector<int32_t> cells;
    for (auto &e : edge) cells.insert(cells.end(), e.begin(), e.end());
    lt.mark("edges");
    // 2. their ghost tasks, in equal shares of the cell list
    const int E = std::max(1, std::min(8, (int)(cells.size() / 512)));
    struct Band {
      std::vector<std::pair<int, Task>> tk;
      std::vector<int64_t> key;  // (cell, q) of each task
    };
    std::vector<Band> bands(E);
    st = run_parallel(E, [&](int b) -> vlbm_status {
      Band &bd = bands[b];
      const size_t i0 = cells.size() * b / E, i1 = cells.size() * (b + 1) / E;
      for (size_t i = i0; i < i1; ++i) {
        const int x = L.fx0 + cells[i] % fw, y = L.fy0 + L.yrow[cells[i] / fw];
        const int tile = w.owner(L, cells[i]);
        for (int q = 0; q < 4; ++q) {
          // an active upwind cell of this level is read in place (no task);
          // the rows next to an active cell are stored next to its row
          if (L.status[cells[i] - CX[q] - (int64_t)CY[q] * fw] == 1) continue;
          Task t{};
          vlbm_status gs = ghost_task(c, l, x, y, q, t);
          if (gs) return gs;
          if (t.kind == T_NONE) continue;
          bd.tk.push_back({tile, t});
          bd.key.push_back(((int64_t)y * L.Nx + x) * 4 + q);
        }
      }
      return VLBM_OK;
    });
    if (st) return st;
    lt.mark("tasks");
    size_t ntk = 0;
    for (const Band &bd : bands) ntk += bd.tk.size();
    w.tk.reserve(ntk);
    for (Band &bd : bands)
      for (size_t i = 0; i < bd.tk.size(); ++i) {
        Task &t = bd.tk[i].second;
        const int kind = t.kind & 0xFF;
        if (kind == T_OUTFLOW || kind == T_REFLECT || kind == T_INFLOW) {
          t.slot = L.nledger++;
          if (w.fuse) w.bc_slot[bd.key[i]] = t.slot;
        } else if (kind == T_REFLUX) {
          const int slot = (int)L.reflux_key.size();
          L.reflux_key.push_back(bd.key[i]);
          t.slot = slot;
        }
        w.tk.push_back(bd.tk[i]);
      }
    L.nacc = (int)L.reflux_key.size();
    return VLBM_OK;
  };
  auto passB = [&](int l) -> vlbm_status {
    PhaseTimer lt(l == 0 ? "passB l0" : l == 1 ? "passB l1" : l == 2 ? "passB l2" : "passB l3+");
    Level &L = c->lv[l];
    Work &w = W[l];
    std::vector<std::pair<int, Task>> &tk = w.tk;
    // captures: values leaving level l towards the parent's ring cells. One
    // per reflux slot (ring cell P, population q) of the parent: the r fine
    // cells streaming q into P are the children of the hole P - c_q on its
    // face towards P (all active: by proper nesting no finer level reaches
    // there). R_0 is the first of them in row order, and captures are kept in
    // the order of their R_0 (row, column) and q.
    if (l >= 1) {
      const Level &PL = c->lv[l - 1];
      struct Cap {
        int x, y, q, slot;
      };
      std::vector<Cap> caps(PL.reflux_key.size());
      for (size_t slot = 0; slot < PL.reflux_key.size(); ++slot) {
        const int64_t key = PL.reflux_key[slot];
        const int q = (int)(key & 3);
        const int64_t cell = key >> 2;
        int hx = (int)(cell % PL.Nx) - CX[q], hy = (int)(cell / PL.Nx) - CY[q];
        c->wrap(l - 1, hx, hy);
        const int x = hx * r + (q == 0 ? r - 1 : 0), y = hy * r + (q == 2 ? r - 1 : 0);
        const int x1 = x + (q < 2 ? 0 : r - 1), y1 = y + (q < 2 ? r - 1 : 0);
        if (!L.in_frame(x, y) || !L.in_frame(x1, y1) || L.status[L.fidx(x, y)] != 1 ||
            L.status[L.fidx(x1, y1)] != 1)
          return fail(VLBM_ENEST, "internal: level %d reflux face without active fine cells", l - 1);
        caps[slot] = {x, y, q, (int)slot};
      }
      std::sort(caps.begin(), caps.end(), [](const Cap &a, const Cap &b) {
        return a.y != b.y ? a.y < b.y : a.x != b.x ? a.x < b.x : a.q < b.q;
      });
      tk.reserve(tk.size() + caps.size());
      for (const Cap &cd : caps) {
        Task t{};
        t.kind = T_CAPTURE;
        t.q = cd.q;
        t.src = (int32_t)L.off(cd.x, cd.y);
        t.n0 = cd.q < 2 ? L.pitch : 1;
        t.n1 = -1;
        t.j = r - 1;  // captured cells beyond the first (the device reads r)
        t.slot = cd.slot;
        tk.push_back({w.owner(L, L.fidx(cd.x, cd.y)), t});
        if (w.fuse) w.caps.push_back({(int64_t)cd.y * L.Nx + cd.x, t});
      }
    }
    lt.mark("captures");
    // tasks grouped by tile, in their order of discovery (a counting sort)
    const size_t nt = L.tiles.size();
    std::vector<int32_t> start(nt + 1, 0);
    for (const auto &e : tk) start[e.first + 1] += 1;
    for (size_t t = 0; t < nt; ++t) {
      L.tiles[t].ntask = start[t + 1];
      start[t + 1] += start[t];
      L.tiles[t].task0 = L.tiles[t].ntask ? start[t] : 0;
    }
    L.tasks.resize(tk.size());
    for (const auto &e : tk) L.tasks[start[e.first]++] = e.second;
    L.ftiles.clear();
    L.ftasks.clear();
    if (w.fuse) return build_fused(c, l, w.bc_slot, w.caps);
    return VLBM_OK;
  };
  // Run one pass over all levels, each on its own thread (level 0 on this one).
  auto run_pass = [&](const std::function<vlbm_status(int)> &pass) { return run_parallel(nlev, pass); };
  vlbm_status st = run_pass(passA);
  tm.mark("tiles+tasks");
  if (!st) st = run_pass(passB);
  tm.mark("captures+order+fused");
  return st;
}

vlbm_status build_lists(vlbm_ctx *c, const vlbm_box *boxes, int n) {
  vlbm_status st = build_coverage(c, boxes, n);
  return st ? st : build_task_lists(c);
}

// Pinned host staging of uploads: n bytes of the context's staging area that
// no copy in flight reads (the caller fills them and copies from them on the
// context's stream), or nullptr when n exceeds kStageMax or no pinned memory
// can be had. The area is used front to back and restarts after a
// synchronisation of the stream when a request does not fit; it grows to the
// largest request up to kStageMax.
constexpr size_t kStageMin = size_t(4) << 20, kStageMax = size_t(64) << 20;
char *stage_reserve(vlbm_ctx *c, size_t n, hipError_t &e) {
  e = hipSuccess;
  const size_t need = (std::max<size_t>(n, 1) + 255) & ~size_t(255);
  if (need > kStageMax) return nullptr;
  if (c->stage_used + need > c->stage_cap) {
    e = hipStreamSynchronize(c->stream);  // the stream has read the area
    if (e != hipSuccess) return nullptr;
    c->stage_used = 0;
    if (need > c->stage_cap) {
      const size_t cap = std::min(kStageMax, std::max({need, kStageMin, 2 * c->stage_cap}));
      if (c->stage) (void)hipHostFree(c->stage);
      c->stage = nullptr;
      c->stage_cap = 0;
      void *h = nullptr;
      if (hipHostMalloc(&h, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      c->stage = static_cast<char *>(h);
      c->stage_cap = cap;
    }
  }
  char *h = c->stage + c->stage_used;
  c->stage_used += need;
  return h;
}

// Host-to-device copy of n bytes, asynchronous on the context's stream: the
// source may change as soon as this returns. Through the staging area (a DMA
// enqueue instead of a staged pageable copy); beyond it, from the pageable
// source, followed by a synchronisation.
hipError_t stage_h2d(vlbm_ctx *c, void *dst, const void *src, size_t n) {
  if (n == 0) return hipSuccess;
  hipError_t e;
  char *h = stage_reserve(c, n, e);
  if (e != hipSuccess) return e;
  if (!h) {
    e = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, c->stream);
    return e == hipSuccess ? hipStreamSynchronize(c->stream) : e;
  }
  memcpy(h, src, n);
  return hipMemcpyAsync(dst, h, n, hipMemcpyHostToDevice, c->stream);
}

vlbm_status upload_level(vlbm_ctx *c, Level &L, bool alloc_buffers) {
  auto &M = c->mem;
  if (alloc_buffers) {
    size_t nb = level_bytes(L, c->esz);
    L.buf[0] = M.alloc(nb);
    L.buf[1] = M.alloc(nb);
    if (!L.buf[0] || !L.buf[1]) return fail(VLBM_ENOMEM, "population buffers (%zu bytes)", nb);
    HIPCHK(hipMemsetAsync(L.buf[0], 0, nb, c->stream));
    HIPCHK(hipMemsetAsync(L.buf[1], 0, nb, c->stream));
  }
  // Every table of the level lives in one device block, written by one copy
  // of its host image (reflux accumulators and ledger slots zeroed by it).
  struct Part {
    void **dst;
    const void *src;  // bytes copied; the rest of the part is zeroed
    size_t nsrc, n;
  };
  const bool fused = !L.ftiles.empty();
  const Part parts[] = {
      {(void **)&L.dstatus, L.status.data(), L.status.size(), L.status.size()},
      {(void **)&L.dsrow, L.srow.data(), sizeof(int32_t) * L.srow.size(), sizeof(int32_t) * std::max<size_t>(1, L.srow.size())},
      {(void **)&L.dyrow, L.yrow.data(), sizeof(int32_t) * L.yrow.size(), sizeof(int32_t) * std::max<size_t>(1, L.yrow.size())},
      {(void **)&L.dtiles, L.tiles.data(), sizeof(Tile) * L.tiles.size(), sizeof(Tile) * std::max<size_t>(1, L.tiles.size())},
      {(void **)&L.dtasks, L.tasks.data(), sizeof(Task) * L.tasks.size(), sizeof(Task) * std::max<size_t>(1, L.tasks.size())},
      {(void **)&L.dacc, nullptr, 0, sizeof(double) * 4 * std::max(1, L.nacc)},
      {(void **)&L.dledger, nullptr, 0, sizeof(double) * 4 * std::max(1, L.nledger)},
      {(void **)&L.dpartial, nullptr, 0, sizeof(double) * 4 * std::max<size_t>(1, L.tiles.size())},
      {fused ? (void **)&L.dftiles : nullptr, L.ftiles.data(), sizeof(Tile) * L.ftiles.size(), sizeof(Tile) * L.ftiles.size()},
      {fused ? (void **)&L.dftasks : nullptr, L.ftasks.data(), sizeof(Task) * L.ftasks.size(),
       sizeof(Task) * std::max<size_t>(1, L.ftasks.size())},
  };
  size_t at[sizeof parts / sizeof parts[0]], total = 0;
  for (size_t i = 0; i < sizeof parts / sizeof parts[0]; ++i) {
    at[i] = total;
    if (parts[i].dst) total += (std::max<size_t>(parts[i].n, 1) + 255) & ~size_t(255);
  }
  L.dtables = M.alloc(total);
  if (!L.dtables) return fail(VLBM_ENOMEM, "level tables (%zu bytes)", total);
  hipError_t e;
  char *img = stage_reserve(c, total, e);
  if (e != hipSuccess) return fail(VLBM_EDEVICE, "%s", hipGetErrorString(e));
  std::vector<char> pageable;
  if (!img) {
    pageable.resize(total);
    img = pageable.data();
  }
  for (size_t i = 0; i < sizeof parts / sizeof parts[0]; ++i) {
    const Part &q = parts[i];
    if (!q.dst) continue;
    *q.dst = static_cast<char *>(L.dtables) + at[i];
    if (q.nsrc) memcpy(img + at[i], q.src, q.nsrc);
    if (q.n > q.nsrc) memset(img + at[i] + q.nsrc, 0, q.n - q.nsrc);
  }
  HIPCHK(hipMemcpyAsync(L.dtables, img, total, hipMemcpyHostToDevice, c->stream));
  if (!pageable.empty()) HIPCHK(hipStreamSynchronize(c->stream));
  return VLBM_OK;  // the caller's build_tables synchronises
}

// Phases of one coarse step in execution order: level l+1 takes r steps
// before each step of level l (finest first). With `fused` the finest level's
// r = 2 sub-steps of one parent step form one phase, k = 0.
void schedule(int l, int k, int nlev, int r, std::vector<std::pair<int, int>> &out,
              bool fused = false) {
  if (l + 1 < nlev) {
    if (fused && l + 2 == nlev)
      out.push_back({l + 1, 0});
    else
      for (int kk = 1; kk <= r; ++kk) schedule(l + 1, kk, nlev, r, out, fused);
  }
  out.push_back({l, k});
}

// Whether the finest level runs fused two-sub-step launches.
// Whether the finest level runs fused two-sub-step launches (never with the
// adaptive relaxation, whose second sub-step needs a level-wide maximum of the
// intermediate time level).
bool fused_active(const vlbm_ctx *c) {
  return (c->step_flags & STEP_FUSE2) && !c->sensor && c->nlev >= 2 &&
         !c->lv[c->nlev - 1].ftiles.empty();
}

// Allocate (sensor on) or release (off) the adaptive relaxation planes of
// every present level (new planes start at zero) and rebuild the neighbour
// masks from the current status. The W planes and maxima then need stage 0.
vlbm_status ensure_sensor(vlbm_ctx *c) {
  c->sensor_stale = true;
  c->cfl_stale = true;
  for (int l = 0; l < kMaxLevels; ++l) {
    Level &L = c->lv[l];
    const bool want = c->sensor && L.present && l < c->nlev;
    if (L.dsen && (!want || L.sen_plane != L.plane)) {
      c->mem.release(L.dsen);
      c->mem.release(L.dmask);
      L.dsen = nullptr;
      L.dmask = nullptr;
      L.sen_plane = 0;
    }
    if (!want) continue;
    if (!L.dsen) {
      const size_t nb = sizeof(double) * SEN_PLANES * (size_t)L.plane;
      L.dsen = static_cast<double *>(c->mem.alloc(nb));
      L.dmask = static_cast<uint32_t *>(c->mem.alloc(sizeof(uint32_t) * (size_t)L.plane));
      if (!L.dsen || !L.dmask) return fail(VLBM_ENOMEM, "adaptive relaxation planes (%zu bytes)", nb);
      L.sen_plane = L.plane;
      HIPCHK(hipMemsetAsync(L.dsen, 0, nb, c->stream));
    }
    HIPCHK(hipMemsetAsync(L.dmask, 0, sizeof(uint32_t) * (size_t)L.plane, c->stream));
    HIPCHK(launch_sensor_mask(L.dstatus, L.dmask, L.dsrow, L.dyrow, L.fx0, L.fy0, L.fw, L.fh, L.nrows,
                              L.pitch, L.xoff, L.Nx, L.Ny, (c->perx() ? 1 : 0) | (c->pery() ? 2 : 0),
                              c->stream));
  }
  if (!c->sensor) {
    c->mem.release(c->dqmax);
    c->dqmax = nullptr;
    return VLBM_OK;
  }
  if (!c->dqmax) c->dqmax = static_cast<unsigned long long *>(c->mem.alloc(8 * sizeof(unsigned long long)));
  if (!c->dqmax) return fail(VLBM_ENOMEM, "adaptive relaxation maxima");
  return VLBM_OK;
}


// Descriptor of level l at flip counts st (fused: its fused two-sub-step tiles).
LevelDesc make_desc(const vlbm_ctx *c, int l, const long *st, bool fused = false) {
  const Level &L = c->lv[l];
  LevelDesc a{};
  a.src = L.buf[st[l] & 1];
  a.dst = L.buf[(st[l] + 1) & 1];
  if (l > 0) {
    const Level &P = c->lv[l - 1];
    a.pcur = P.buf[st[l - 1] & 1];
    a.pprev = P.buf[(st[l - 1] + 1) & 1];
    a.pplane = P.plane;
    a.acc_out = P.dacc;
  }
  a.tiles = fused ? L.dftiles : L.dtiles;
  a.tasks = fused ? L.dftasks : L.dtasks;
  a.acc_in = L.dacc;
  a.ledger = L.dledger;
  a.plane = L.plane;
  a.pitch = L.pitch;
  a.ntiles = (int32_t)(fused ? L.ftiles.size() : L.tiles.size());
  a.r = c->p.r;
  a.rr = (double)(c->p.r * c->p.r);
  a.w2 = L.dx * L.dx;
  a.gm1 = c->gm1;
  a.h = c->h;
  a.tb = c->tb;
  a.eos = c->eos.kind;
  a.eos_a = c->eos.a;
  a.eos_b = c->eos.b;
  a.eos_ga = c->eos.ga;
  for (int s2 = 0; s2 < 4; ++s2)
    for (int k = 0; k < 4; ++k) a.win[s2][k] = c->p.w_inflow[s2][k];
  if (c->sensor && !fused) {
    a.sen = L.dsen;  // qmax, qmax_next, clear_next, emit_qmax: per phase (build_tables)
    a.mask = L.dmask;
    a.fx0 = L.fx0;
    a.fy0 = L.fy0;
    a.xoff = L.xoff;
    a.srow = L.dsrow;
    a.yrow = L.dyrow;
    a.Nx = L.Nx;
    a.Ny = L.Ny;
    a.c_sensor = c->c_sensor;
    a.beta_min = c->beta_min;
    a.beta_max = c->beta_max;
  }
  return a;
}

void drop_graph(vlbm_ctx *c) {
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
  c->graph_key = -1;
}

double ak_of(int k, int r) { return (double)(2 * k - r - 1) / (double)(2 * r); }

long tile_cells_sum(const Level &L, bool fused, size_t t0, size_t t1) {
  const std::vector<Tile> &T = fused ? L.ftiles : L.tiles;
  long n = 0;
  for (size_t t = t0; t < std::min(t1, T.size()); ++t) n += (long)T[t].w * T[t].h;
  return n;
}

// (Re)build the descriptor tables after any change of buffers, lists or
// step counters: one descriptor per phase and parity (e * P + p), one launch
// per phase, each a run of segments of the segment table.
vlbm_status build_tables(vlbm_ctx *c) {
  drop_graph(c);
  c->tables_version += 1;
  vlbm_status sst = ensure_sensor(c);
  if (sst) return sst;
  c->phases.clear();
  schedule(0, 1, c->nlev, c->p.r, c->phases, fused_active(c));
  const size_t P = c->phases.size();
  if (c->sensor)  // the SEN step keeps its tile's neighbourhood in LDS
    for (int l = 0; l < c->nlev; ++l)
      for (const Tile &t : c->lv[l].tiles)
        if (t.w > SEN_TW || t.h > SEN_TH) return fail(VLBM_EINVAL, "internal: tile larger than the sensor's LDS");
  // buffer flips of each level per coarse step: one per phase
  for (int l = 0; l < kMaxLevels; ++l) c->flips[l] = 0;
  for (const auto &ph : c->phases) c->flips[ph.first] += 1;
  auto nb8 = [](long n) { return (int32_t)((n + 7) / 8 * 8); };
  std::vector<LevelDesc> descs(2 * P);
  c->launches.clear();
  std::vector<std::pair<int, int>> seg_desc;  // per parity-0 segment: (desc index e=0, nblocks)
  std::vector<int> seg_desc1;                 // the same segment's desc index for e=1
  c->phase_blocks.assign(P, 0);
  for (int e = 0; e < 2; ++e) {
    long st[kMaxLevels];
    for (int l = 0; l < kMaxLevels; ++l) st[l] = c->lv[l].steps + e * c->flips[l];
    for (size_t p = 0; p < P; ++p) {
      const int l = c->phases[p].first, k = c->phases[p].second;
      const bool fused = k == 0;
      descs[e * P + p] = make_desc(c, l, st, fused);
      if (c->adt) {
        // the hand-off scales its temporal slope when the parent's previous
        // step belongs to the previous coarse step
        LevelDesc &D = descs[e * P + p];
        D.dyn = c->ddyn;
        bool parent_stepped = false;
        for (size_t q2 = 0; q2 < p; ++q2)
          if (c->phases[q2].first == l - 1) parent_stepped = true;
        D.use_ratio = (l > 0 && !parent_stepped) ? 1 : 0;
        bool later = false;
        for (size_t q2 = p + 1; q2 < P; ++q2)
          if (c->phases[q2].first == l) later = true;
        D.emit_cfl = later ? 0 : 1;
        D.cfl_next = c->dcmax;
      }
      if (descs[e * P + p].sen) {
        LevelDesc &D = descs[e * P + p];
        D.qmax = c->dqmax + 4 * e;
        D.qmax_next = c->dqmax + 4 * (e ^ 1);
        D.clear_next = p == 0;
        const Level &L = c->lv[l];
        const bool odd = (st[l] & 1) != 0;
        D.wcur = L.dsen + (odd ? SEN_W1 : SEN_W0) * L.plane;
        D.wnext = L.dsen + (odd ? SEN_W0 : SEN_W1) * L.plane;
        size_t last = p;
        for (size_t q = p + 1; q < P; ++q)
          if (c->phases[q].first == l) last = q;
        D.emit_qmax = last == p;
      }
      const int nb = nb8(fused ? c->lv[l].ftiles.size() : c->lv[l].tiles.size());
      c->phase_blocks[p] = nb;
      if (e == 0) {
        LaunchRec a{};
        a.seg0 = (int)seg_desc.size();
        seg_desc.push_back({(int)(e * P + p), nb});
        a.nseg = 1;
        a.first = k == 1;
        a.ak = ak_of(k, c->p.r);
        a.fused_kernel = fused;
        a.prof_key = 2 * l + (fused ? 1 : 0);
        a.cells = (double)tile_cells_sum(c->lv[l], fused, 0, SIZE_MAX);
        a.emit_cfl = descs[e * P + p].emit_cfl;
        c->launches.push_back(a);
      } else {
        seg_desc1.push_back((int)(e * P + p));
      }
      st[l] += 1;
    }
  }
  c->s0_seg0 = (int32_t)seg_desc.size();
  c->s0_nseg = 0;
  c->s0_nblocks = 0;
  if (c->sensor || c->adt) {
    // one segment per level over every level's cells as at the coarse step's
    // start (the sensor's stage 0, the adaptive time step's CFL bound): the
    // descriptor of the level's first phase, fused or not (its tiles cover
    // the level's active cells either way)
    for (int l = 0; l < c->nlev; ++l) {
      size_t p0 = 0;
      while (p0 < P && c->phases[p0].first != l) ++p0;
      if (p0 == P) return fail(VLBM_EINVAL, "internal: level without a phase");
      const bool fz = c->phases[p0].second == 0;
      seg_desc.push_back({(int)p0, nb8(fz ? c->lv[l].ftiles.size() : c->lv[l].tiles.size())});
      seg_desc1.push_back((int)(P + p0));
      c->s0_nseg += 1;
    }
  }
  const size_t NS = seg_desc.size();
  if (seg_desc1.size() != NS) return fail(VLBM_EINVAL, "internal: launch tables differ between parities");
  c->mem.release(c->ddesc);
  c->mem.release(c->dseg);
  c->ddesc = static_cast<LevelDesc *>(c->mem.alloc(sizeof(LevelDesc) * descs.size()));
  c->dseg = static_cast<Segment *>(c->mem.alloc(sizeof(Segment) * std::max<size_t>(1, 2 * NS)));
  if (!c->ddesc || !c->dseg) return fail(VLBM_ENOMEM, "schedule tables");
  // segments of one launch are laid out back to back, first_block running on
  std::vector<Segment> segs(2 * NS);
  auto lay = [&](int seg0, int nseg) {
    int32_t fb = 0;
    for (int i = seg0; i < seg0 + nseg; ++i) {
      segs[i] = {c->ddesc + seg_desc[i].first, fb, seg_desc[i].second};
      segs[NS + i] = {c->ddesc + seg_desc1[i], fb, seg_desc[i].second};
      fb += seg_desc[i].second;
    }
    return fb;
  };
  for (const LaunchRec &a : c->launches) lay(a.seg0, a.nseg);
  c->s0_nblocks = lay(c->s0_seg0, c->s0_nseg);
  for (LaunchRec &a : c->launches) {
    a.nblocks = 0;
    for (int i = a.seg0; i < a.seg0 + a.nseg; ++i) a.nblocks += seg_desc[i].second;
  }
  c->nseg_table = (int)NS;
  c->hseg = segs;
  c->hdesc = descs;
  HIPCHK(stage_h2d(c, c->ddesc, descs.data(), sizeof(LevelDesc) * descs.size()));
  HIPCHK(stage_h2d(c, c->dseg, segs.data(), sizeof(Segment) * segs.size()));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->table_base = c->coarse_steps;
  return VLBM_OK;
}



// Read back the pending launch timings into the accumulators.
vlbm_status prof_flush(vlbm_ctx *c) {
  if (c->pend.empty()) return VLBM_OK;
  HIPCHK(hipEventSynchronize(c->pev[2 * c->pend.size() - 1]));
  for (size_t i = 0; i < c->pend.size(); ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, c->pev[2 * i], c->pev[2 * i + 1]));
    c->prof_ms[c->pend[i].first] += ms;
    c->prof_calls[c->pend[i].first] += 1;
    c->prof_cells[c->pend[i].first] += c->pend[i].second;
  }
  c->pend.clear();
  return VLBM_OK;
}

// Launch every launch of one coarse step of table parity e.
vlbm_status launch_coarse_step(vlbm_ctx *c, int e) {
  // this coarse step's link speed from the bound of the state at its start,
  // which the previous coarse step's last launches (or cfl_init) left in dcmax
  if (c->adt) HIPCHK(launch_cfl_finalize(c->ddyn, c->dcmax, c->stream));
  for (size_t ri = 0; ri < c->launches.size(); ++ri) {
    const LaunchRec &r = c->launches[ri];
    if (c->sensor && ri == 0 && c->hdesc[e * c->phases.size()].emit_qmax) {
      // the first phase also accumulates the next Qmax: clear its slot first
      StepLaunch a{};
      a.d0 = c->hseg[e * c->nseg_table + r.seg0].d;
      a.nblocks = 1;
      HIPCHK(launch_sensor(a, 1, c->fp32, c->stream));
    }
    if (r.nblocks <= 0) continue;
    StepLaunch a{};
    const int s0 = e * c->nseg_table + r.seg0;
    if (r.nseg == 1) {
      a.d0 = c->hseg[s0].d;
      a.nseg = 0;
    } else {
      a.segs = c->dseg + s0;
      a.nseg = r.nseg;
    }
    a.nblocks = r.nblocks;
    a.first = r.first;
    a.flags = c->step_flags | (r.fused_kernel ? STEP_FUSED_PHASE : 0) | (c->adt ? STEP_ADAPTIVE_DT : 0);
    if (r.fused_kernel && (c->step_flags & STEP_XCD_FUSED)) a.flags |= STEP_XCD_CONTIGUOUS;
    if (c->adt && r.emit_cfl) a.flags |= STEP_CFL_EMIT;
    a.ak = r.ak;
    if (c->sensor && !r.fused_kernel) a.flags |= STEP_SENSOR;  // per-cell beta
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof) {
      if (c->pend.size() >= 4096) {
        vlbm_status st = prof_flush(c);
        if (st) return st;
      }
      const size_t i = 2 * c->pend.size();
      while (c->pev.size() < i + 2) {
        hipEvent_t ev;
        HIPCHK(hipEventCreate(&ev));
        c->pev.push_back(ev);
      }
      e0 = c->pev[i];
      e1 = c->pev[i + 1];
      c->pend.push_back({r.prof_key, r.cells});
    }
    HIPCHK(launch_step(a, c->fp32, c->stream, e0, e1));
  }
  return VLBM_OK;
}

// Stage 0 before a coarse step of table parity e: W planes of every level and
// the coarse step's max |Q| from the stored populations (both slots cleared
// first; eager, never inside a graph).
vlbm_status sensor_init(vlbm_ctx *c, int e) {
  if (!c->sensor || !c->sensor_stale) return VLBM_OK;
  HIPCHK(launch_clear_u64(c->dqmax, 8, c->stream));
  StepLaunch a{};
  const int s0 = e * c->nseg_table + c->s0_seg0;
  if (c->s0_nseg == 1) {
    a.d0 = c->hseg[s0].d;
  } else {
    a.segs = c->dseg + s0;
    a.nseg = c->s0_nseg;
  }
  a.nblocks = c->s0_nblocks;
  HIPCHK(launch_sensor(a, 0, c->fp32, c->stream));
  c->sensor_stale = false;
  return VLBM_OK;
}

// The CFL bound of the stored state, before a coarse step of table parity e,
// after the host changed the state (eager, never inside a graph); the step
// launches keep it current from then on.
vlbm_status cfl_init(vlbm_ctx *c, int e) {
  if (!c->adt || !c->cfl_stale) return VLBM_OK;
  HIPCHK(launch_clear_u64(c->dcmax, 1, c->stream));
  StepLaunch a{};
  const int s0 = e * c->nseg_table + c->s0_seg0;
  if (c->s0_nseg == 1) {
    a.d0 = c->hseg[s0].d;
  } else {
    a.segs = c->dseg + s0;
    a.nseg = c->s0_nseg;
  }
  a.nblocks = c->s0_nblocks;
  HIPCHK(launch_cfl(a, c->fp32, c->dcmax, c->ddyn, c->stream));
  c->cfl_stale = false;
  return VLBM_OK;
}

void count_steps(vlbm_ctx *c, long n) {
  for (int l = 0; l < c->nlev; ++l) c->lv[l].steps += n * c->flips[l];
  c->coarse_steps += n;
}

int table_parity(const vlbm_ctx *c) { return (int)((c->coarse_steps - c->table_base) & 1); }

// Capture two coarse steps (table parities 0 then 1) into a graph.
vlbm_status ensure_graph(vlbm_ctx *c) {
  if (c->graph) return VLBM_OK;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  vlbm_status st = launch_coarse_step(c, 0);
  if (!st) st = launch_coarse_step(c, 1);
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (st) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(VLBM_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->graph = nullptr;
    return fail(VLBM_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  }
  return VLBM_OK;
}

vlbm_status advance_impl(vlbm_ctx *c, long n) {
  if (n > 0) {
    vlbm_status st = sensor_init(c, table_parity(c));
    if (!st) st = cfl_init(c, table_parity(c));
    if (st) return st;
  }
  const bool graphs = c->use_graphs && !c->prof && c->stream != nullptr && n >= 4;
  while (n > 0) {
    const int e = table_parity(c);
    if (graphs && e == 0 && n >= 2) {
      vlbm_status st = ensure_graph(c);
      if (st) return st;
      while (n >= 2) {
        HIPCHK(hipGraphLaunch(c->graph, c->stream));
        count_steps(c, 2);
        n -= 2;
      }
      continue;
    }
    vlbm_status st = launch_coarse_step(c, e);
    if (st) return st;
    count_steps(c, 1);
    n -= 1;
  }
  return VLBM_OK;
}

vlbm_status check_rect(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny) {
  if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
  if (level < 0 || level >= c->p.max_levels) return fail(VLBM_EINVAL, "bad level %d", level);
  long s = 1;
  for (int i = 0; i < level; ++i) s *= c->p.r;
  if (i0 < 0 || j0 < 0 || nx < 0 || ny < 0 || i0 + (long)nx > c->p.nx0 * s ||
      j0 + (long)ny > c->p.ny0 * s)
    return fail(VLBM_EINVAL, "rectangle outside level %d", level);
  return VLBM_OK;
}

// Clip a rectangle to a level's frame; returns false if empty.
bool clip_to_frame(const Level &L, int &i0, int &j0, int &nx, int &ny, int &ox, int &oy) {
  int x0 = std::max(i0, L.fx0), y0 = std::max(j0, L.fy0);
  int x1 = std::min(i0 + nx, L.fx0 + L.fw), y1 = std::min(j0 + ny, L.fy0 + L.fh);
  ox = x0 - i0;
  oy = y0 - j0;
  if (x1 <= x0 || y1 <= y0) return false;
  i0 = x0;
  j0 = y0;
  nx = x1 - x0;
  ny = y1 - y0;
  return true;
}

vlbm_status rect_io(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny, double *host, long ld,
                    int ncomp, bool write, bool raw) {
  vlbm_status st = check_rect(c, level, i0, j0, nx, ny);
  if (st) return st;
  if (ld < nx) return fail(VLBM_EINVAL, "ld < nx");
  Level &L = c->lv[level];
  const size_t full_plane = (size_t)ny * ld;
  if (!write) {  // defaults: NaN everywhere, then fill the part inside the frame
    for (int k = 0; k < ncomp; ++k)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) host[k * full_plane + (size_t)y * ld + x] = NAN;
  }
  if (!L.present) return VLBM_OK;
  int ci0 = i0, cj0 = j0, cnx = nx, cny = ny, ox = 0, oy = 0;
  if (!clip_to_frame(L, ci0, cj0, cnx, cny, ox, oy)) return VLBM_OK;
  const size_t n = (size_t)cnx * cny;
  double *stage = static_cast<double *>(c->mem.alloc(sizeof(double) * ncomp * n));
  if (!stage) return fail(VLBM_ENOMEM, "staging buffer");
  std::vector<double> tmp(ncomp * n);
  RectArgs a{};
  a.buf0 = write ? L.buf[0] : L.buf[L.cur()];
  a.buf1 = L.buf[1];
  a.status = L.dstatus;
  a.host_stage = stage;
  a.plane = L.plane;
  a.pitch = L.pitch;
  a.xoff = L.xoff;
  a.fx0 = L.fx0;
  a.fy0 = L.fy0;
  a.fw = L.fw;
  a.srow = L.dsrow;
  a.x0 = ci0;
  a.y0 = cj0;
  a.nx = cnx;
  a.ny = cny;
  a.gm1 = c->gm1;
  a.h = c->h;
  a.eos = c->eos;
  hipError_t e = hipSuccess;
  if (write) {
    for (int k = 0; k < ncomp; ++k)
      for (int y = 0; y < cny; ++y)
        memcpy(&tmp[k * n + (size_t)y * cnx], &host[k * full_plane + (size_t)(y + oy) * ld + ox],
               sizeof(double) * cnx);
    e = hipMemcpyAsync(stage, tmp.data(), sizeof(double) * ncomp * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_set_state(a, c->fp32, raw ? 1 : 0, c->stream);
    c->sensor_stale = true;
    c->cfl_stale = true;
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    e = launch_get(a, c->fp32, ncomp == 16 ? 1 : 0, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tmp.data(), stage, sizeof(double) * ncomp * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
      for (int k = 0; k < ncomp; ++k)
        for (int y = 0; y < cny; ++y)
          memcpy(&host[k * full_plane + (size_t)(y + oy) * ld + ox], &tmp[k * n + (size_t)y * cnx],
                 sizeof(double) * cnx);
  }
  c->mem.release(stage);
  if (e != hipSuccess) return fail(VLBM_EDEVICE, "state transfer: %s", hipGetErrorString(e));
  return VLBM_OK;
}

}  // namespace

// Static staging of vlbm_get_state_noalloc: every GPU the library runs on holds
// its own copy of this array until the process ends. In host code `scratch`
// only names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (scratch_address) and is the only form passed to
// kernels and copies.
static __device__ __align__(256) double scratch[VLBM_NOALLOC_STAGE_BYTES / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_addr;  // device -> address of its `scratch`

// Address of `scratch` on device dev, looked up once per device with dev current.
vlbm_status scratch_address(int dev, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return VLBM_OK;
  }
  int cur = 0;
  HIPCHK(hipGetDevice(&cur));
  if (cur != dev) HIPCHK(hipSetDevice(dev));
  double *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (cur != dev) HIPCHK(hipSetDevice(cur));
  if (e != hipSuccess || !ptr)
    return fail(VLBM_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
  g_scratch_addr[dev] = ptr;
  *out = ptr;
  return VLBM_OK;
}

vlbm_status reset_time(vlbm_ctx *c) {
  if (!c->adt) return VLBM_OK;
  const double zero = 0.0;
  HIPCHK(hipMemcpyAsync(c->ddyn + DYN_TIME, &zero, sizeof zero, hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return VLBM_OK;
}

vlbm_status reset_ledgers(vlbm_ctx *c) {
  for (int k = 0; k < 4; ++k) c->ledger_carry[k] = c->ledger_carry_c[k] = 0.0;
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->lv[l];
    HIPCHK(hipMemsetAsync(L.dledger, 0, sizeof(double) * 4 * std::max(1, L.nledger), c->stream));
  }
  return VLBM_OK;
}

void kadd(double &s, double &cmp, double v) {
  double t = s + v;
  if (std::fabs(s) >= std::fabs(v))
    cmp += (s - t) + v;
  else
    cmp += (v - t) + s;
  s = t;
}

bool same_frame(const Level &a, const Level &b) {
  return a.present && b.present && a.fx0 == b.fx0 && a.fy0 == b.fy0 && a.fw == b.fw &&
         a.fh == b.fh && a.pitch == b.pitch && a.plane == b.plane && a.xoff == b.xoff && a.runs == b.runs;
}

// Move the sum of every ledger slot into the host-side carry (before the slots
// are rebuilt by a regrid).
vlbm_status carry_ledgers(vlbm_ctx *c) {
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->lv[l];
    if (!L.nledger) continue;
    std::vector<double> led(4 * (size_t)L.nledger);
    HIPCHK(hipMemcpyAsync(led.data(), L.dledger, sizeof(double) * led.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int t = 0; t < L.nledger; ++t)
      for (int k = 0; k < 4; ++k) kadd(c->ledger_carry[k], c->ledger_carry_c[k], led[4 * t + k]);
  }
  return VLBM_OK;
}

// Conservative regrid (paper Sec. 3.4): merge exiting cells finest level
// first (eq. amr-merge) in the old frames, move the surviving data into the new
// frames, then split entering cells coarsest level first (eqs. amr-slope,
// amr-split). Merged and split cells get the same value in both time levels,
// so their first hand-off has no temporal slope. A split slope uses a
// neighbour only if it is covered at that level in the new hierarchy and holds
// data (i.e. it is not a hole both before and after).
//
// Interfaces: the reconstruction of a face that exists before and after the
// regrid runs unmodified (Sec. 3.4), with the ring cell's two stored time
// levels. A face the regrid creates (ring cell P, population q towards the new
// hole) has no older sample on that face: population q of P gets its current
// value in the other buffer too, so its first hand-off is flat. A level that
// ran fused before the regrid (the finest, whose other buffer is not its
// previous sub-step) had no finer level, so all of its faces are new.
vlbm_status regrid_impl(vlbm_ctx *c, const vlbm_box *boxes, int nboxes) {
  PhaseTimer tm("regrid");
  Geometry g;
  vlbm_status st = check_boxes(c->p, boxes, nboxes, g);
  if (st) return st;
  // Frames only grow while a level persists: when the new coverage fits in the
  // current frame the frame (and its buffers) is kept, so a moving refinement
  // zone does not reallocate every regrid.
  for (int l = 1; l < kMaxLevels; ++l) grow_geometry(g, l, c->lv[l], c->lv[l].Ny);
  vlbm_ctx *t = new vlbm_ctx();
  t->p = c->p;
  t->esz = c->esz;
  t->tile_cells = c->tile_cells;
  t->step_flags = c->step_flags;
  t->sensor = c->sensor;  // tile shapes follow it
  int nlev = 0;
  for (int l = 0; l < kMaxLevels; ++l) {
    frame_of(c->p, c->esz, g, l, t->lv[l]);
    if (g.present[l]) nlev = l + 1;
    if (t->lv[l].plane >= (int64_t(1) << 31)) {
      delete t;
      return fail(VLBM_EINVAL, "level %d frame too large for 32-bit offsets", l);
    }
  }
  st = build_coverage(t, boxes, nboxes);
  if (st) {
    delete t;
    return st;
  }
  const int r = c->p.r;
  // The new levels' task lists depend on their coverage alone: they are built
  // while other threads plan the merges and splits (per level and kind, in
  // bands of the r-aligned rows of the frame the ops live in; a level's ops
  // in row order), and the device is touched only after both are done (a
  // failure leaves the installed hierarchy as it was).
  struct PlanItem {
    bool split;
    int l, y0, y1;  // rows [y0, y1), y0 r-aligned
    std::vector<RegridOp> ops;
  };
  std::vector<PlanItem> items;
  auto bands = [&](bool split, int l, const Level &L) {
    const int ya = align_up(L.fy0 + 1, r), yb = L.fy0 + L.fh - 1;
    if (ya >= yb) return;
    const int k = (yb - ya + r - 1) / r;  // r-aligned rows
    const int nb = std::max(1, std::min(8, (int)(((int64_t)k * L.fw) >> 15)));
    for (int i = 0; i < nb; ++i)
      items.push_back({split, l, ya + (int)((int64_t)k * i / nb) * r, std::min(yb, ya + (int)((int64_t)k * (i + 1) / nb) * r), {}});
  };
  for (int l = c->nlev - 1; l >= 1; --l) bands(false, l, c->lv[l]);
  for (int l = 0; l + 1 < nlev; ++l) bands(true, l, t->lv[l + 1]);
  // coverage row y of level l of context x (null: none stored), indexed by
  // x - fx0 over [fx0, fx0 + fw)
  auto cov_row = [](const vlbm_ctx *x, int l, int y) -> const uint8_t * {
    if (l >= kMaxLevels || !x->lv[l].present || !x->lv[l].stored(y)) return nullptr;
    const Level &L = x->lv[l];
    return &L.cov[L.fidx(L.fx0, y)];
  };
  auto in_row = [](const vlbm_ctx *x, int l, const uint8_t *row, int xx) {
    const Level &L = x->lv[l];
    return row && xx >= L.fx0 && xx < L.fx0 + L.fw && row[xx - L.fx0];
  };
  auto plan = [&](PlanItem &it) {
    const int l = it.l;
    if (!it.split) {
      // merges, inside the old frames: a covered cell of level l >= 1 on the
      // r-grid whose coverage the new hierarchy drops
      const Level &F = c->lv[l], &C = c->lv[l - 1];
      for (int y = it.y0; y < it.y1; y += r) {
        const uint8_t *fo = cov_row(c, l, y), *fn = cov_row(t, l, y);
        if (!fo) continue;
        for (int x = align_up(F.fx0 + 1, r); x < F.fx0 + F.fw - 1; x += r) {
          if (!fo[x - F.fx0] || in_row(t, l, fn, x)) continue;
          RegridOp op{};
          op.dst = (int32_t)C.off(x / r, y / r);
          op.src = (int32_t)F.off(x, y);
          op.nb[0] = op.nb[1] = op.nb[2] = op.nb[3] = -1;
          it.ops.push_back(op);
        }
      }
      return;
    }
    // splits, inside the new frames: a newly covered cell of level l + 1 on
    // the r-grid, from its parent and the parent's slope neighbours
    const Level &Cn = t->lv[l], &Fn = t->lv[l + 1];
    for (int y = it.y0; y < it.y1; y += r) {
      const uint8_t *fn = cov_row(t, l + 1, y), *fo = cov_row(c, l + 1, y);
      if (!fn) continue;
      for (int x = align_up(Fn.fx0 + 1, r); x < Fn.fx0 + Fn.fw - 1; x += r) {
        if (!fn[x - Fn.fx0] || in_row(c, l + 1, fo, x)) continue;
        const int px = x / r, py = y / r;
        RegridOp op{};
        op.src = (int32_t)Cn.off(px, py);
        op.dst = (int32_t)Fn.off(x, y);
        for (int d = 0; d < 4; ++d) {
          int nx = px + CX[d], ny = py + CY[d];
          op.nb[d] = -1;
          if (!t->wrap(l, nx, ny)) continue;
          const bool persistent_hole = c->covered(l + 1, nx * r, ny * r) && t->covered(l + 1, nx * r, ny * r);
          if (t->covered(l, nx, ny) && !persistent_hole) op.nb[d] = (int32_t)Cn.off(nx, ny);
        }
        it.ops.push_back(op);
      }
    }
  };
  vlbm_status lst = run_parallel(1 + (int)items.size(), [&](int i) -> vlbm_status {
    if (i == 0) return build_task_lists(t);
    plan(items[i - 1]);
    return VLBM_OK;
  });
  std::vector<std::vector<RegridOp>> merge_ops(kMaxLevels), split_ops(kMaxLevels);
  for (PlanItem &it : items) {
    std::vector<RegridOp> &v = it.split ? split_ops[it.l] : merge_ops[it.l];
    v.insert(v.end(), it.ops.begin(), it.ops.end());
  }
  if (lst) {
    delete t;
    return lst;
  }
  tm.mark("lists+plans");
  auto done = [&](vlbm_status s2) {
    delete t;
    return s2;
  };
  if (hipStreamSynchronize(c->stream) != hipSuccess) return done(fail(VLBM_EDEVICE, "sync"));
  st = carry_ledgers(c);
  if (st) return done(st);
  RegridOp *dops = nullptr;
  auto upload_ops = [&](const std::vector<RegridOp> &ops) -> vlbm_status {
    c->mem.release(dops);
    dops = static_cast<RegridOp *>(c->mem.alloc(sizeof(RegridOp) * std::max<size_t>(1, ops.size())));
    if (!dops) return fail(VLBM_ENOMEM, "regrid op list");
    if (!ops.empty())
      HIPCHK(stage_h2d(c, dops, ops.data(), sizeof(RegridOp) * ops.size()));
    return VLBM_OK;
  };
  // 1. merges, finest level first, inside the old frames
  for (int l = c->nlev - 1; l >= 1; --l) {
    Level &F = c->lv[l], &C = c->lv[l - 1];
    const std::vector<RegridOp> &ops = merge_ops[l];
    if (ops.empty()) continue;
    st = upload_ops(ops);
    if (st) return done(st);
    RegridArgs a{};
    a.fine0 = F.buf[0];
    a.fine1 = F.buf[1];
    a.coarse0 = C.buf[0];
    a.coarse1 = C.buf[1];
    a.fine_cur = F.cur();
    a.coarse_cur = C.cur();
    a.fplane = F.plane;
    a.cplane = C.plane;
    a.fpitch = F.pitch;
    a.cpitch = C.pitch;
    a.r = r;
    a.ops = dops;
    a.nops = (int32_t)ops.size();
    HIPCHK(launch_merge(a, c->fp32, c->stream));
  }
  // 2. new frames: keep identical ones, otherwise allocate and copy the overlap
  for (int l = 0; l < kMaxLevels; ++l) {
    Level &O = c->lv[l], &N = t->lv[l];
    N.steps = O.present ? O.steps : 0;
    if (!N.present) continue;
    if (same_frame(O, N)) {
      N.buf[0] = O.buf[0];
      N.buf[1] = O.buf[1];
      O.buf[0] = O.buf[1] = nullptr;
      continue;
    }
    size_t nb = level_bytes(N, c->esz);
    N.buf[0] = c->mem.alloc(nb);
    N.buf[1] = c->mem.alloc(nb);
    if (!N.buf[0] || !N.buf[1]) return done(fail(VLBM_ENOMEM, "population buffers (%zu bytes)", nb));
    HIPCHK(hipMemsetAsync(N.buf[0], 0, nb, c->stream));
    HIPCHK(hipMemsetAsync(N.buf[1], 0, nb, c->stream));
    if (!O.present) continue;
    int x0 = std::max(O.fx0, N.fx0), y0 = std::max(O.fy0, N.fy0);
    int x1 = std::min(O.fx0 + O.fw, N.fx0 + N.fw), y1 = std::min(O.fy0 + O.fh, N.fy0 + N.fh);
    if (x1 <= x0 || y1 <= y0) continue;
    // rows stored by both frames, in runs that are contiguous in both
    for (int ya = y0; ya < y1;) {
      if (!O.stored(ya) || !N.stored(ya)) {
        ++ya;
        continue;
      }
      int yb = ya + 1;
      while (yb < y1 && O.stored(yb) && N.stored(yb)) ++yb;
      for (int b = 0; b < 2; ++b)
        for (int i = 0; i < 16; ++i) {
          char *dst = static_cast<char *>(N.buf[b]) + (i * N.plane + N.off(x0, ya)) * c->esz;
          const char *src = static_cast<const char *>(O.buf[b]) + (i * O.plane + O.off(x0, ya)) * c->esz;
          HIPCHK(hipMemcpy2DAsync(dst, N.pitch * c->esz, src, O.pitch * c->esz, (x1 - x0) * c->esz,
                                  yb - ya, hipMemcpyDeviceToDevice, c->stream));
        }
      ya = yb;
    }
  }
  // 3. splits, coarsest level first, inside the new frames
  for (int l = 0; l + 1 < nlev; ++l) {
    Level &Cn = t->lv[l], &Fn = t->lv[l + 1];
    const std::vector<RegridOp> &ops = split_ops[l];
    if (ops.empty()) continue;
    st = upload_ops(ops);
    if (st) return done(st);
    RegridArgs a{};
    a.fine0 = Fn.buf[0];
    a.fine1 = Fn.buf[1];
    a.coarse0 = Cn.buf[0];
    a.coarse1 = Cn.buf[1];
    a.fine_cur = (int)(Fn.steps & 1);
    a.coarse_cur = (int)(Cn.steps & 1);
    a.fplane = Fn.plane;
    a.cplane = Cn.plane;
    a.fpitch = Fn.pitch;
    a.cpitch = Cn.pitch;
    a.r = r;
    a.ops = dops;
    a.nops = (int32_t)ops.size();
    HIPCHK(launch_split(a, c->fp32, c->stream));
  }
  // 4. faces the regrid creates start flat (reflux keys name the faces:
  //    ring cell P and the population P pulls from the hole, the opposite of
  //    the one handed off into the hole)
  std::vector<int32_t *> face_lists;
  for (int l = 0; l + 1 < nlev; ++l) {
    Level &N = t->lv[l];
    const Level &O = c->lv[l];
    std::vector<int64_t> old_keys(O.reflux_key);
    std::sort(old_keys.begin(), old_keys.end());
    std::vector<int32_t> items;
    for (int64_t key : N.reflux_key) {
      if (std::binary_search(old_keys.begin(), old_keys.end(), key)) continue;
      const int q = (int)(key & 3);
      const int64_t cell = key >> 2;
      items.push_back((int32_t)N.off((int)(cell % N.Nx), (int)(cell / N.Nx)));
      items.push_back(q ^ 1);
    }
    if (items.empty()) continue;
    int32_t *d = static_cast<int32_t *>(c->mem.alloc(sizeof(int32_t) * items.size()));
    if (!d) return done(fail(VLBM_ENOMEM, "regrid face list"));
    face_lists.push_back(d);
    HIPCHK(stage_h2d(c, d, items.data(), sizeof(int32_t) * items.size()));
    const int cur = (int)(N.steps & 1);
    HIPCHK(launch_restart_faces(N.buf[cur], N.buf[cur ^ 1], d, (int)(items.size() / 2), N.plane, c->fp32,
                                c->stream));
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return done(fail(VLBM_EDEVICE, "regrid kernels failed"));
  for (int32_t *d : face_lists) c->mem.release(d);
  tm.mark("merge/copy/split");
  c->mem.release(dops);
  // 4. install the new hierarchy
  for (int l = 0; l < kMaxLevels; ++l) {
    free_level(c, c->lv[l]);
    c->lv[l] = std::move(t->lv[l]);
  }
  delete t;
  c->nlev = nlev;
  for (int l = 0; l < c->nlev; ++l) {
    st = upload_level(c, c->lv[l], false);
    if (st) return st;
  }
  c->boxes.assign(boxes, boxes + nboxes);
  st = build_tables(c);
  tm.mark("upload");
  return st;
}

int level_nx(const vlbm_ctx *c, int l);
int level_ny(const vlbm_ctx *c, int l);

// Coverage of one level (the boxes just made for it) as merged column
// intervals [x0, x1) per row y0 + i; other rows hold none.
struct CovMap {
  bool all = false;
  int y0 = 0;
  std::vector<std::vector<std::pair<int, int>>> rows;
  // [xa, xb) of in-domain row y covered
  bool span(int y, int xa, int xb) const {
    if (all) return true;
    const int i = y - y0;
    if (i < 0 || i >= (int)rows.size()) return false;
    const auto &v = rows[i];
    auto it = std::upper_bound(v.begin(), v.end(), std::make_pair(xa, INT32_MAX));
    if (it == v.begin()) return false;
    --it;
    return it->first <= xa && it->second >= xb;
  }
  static CovMap of_boxes(const vlbm_box *b, size_t n) {
    CovMap m;
    int ya = INT32_MAX, yb = INT32_MIN;
    for (size_t i = 0; i < n; ++i) {
      ya = std::min(ya, b[i].j0);
      yb = std::max(yb, b[i].j0 + b[i].ny);
    }
    if (!n) return m;
    m.y0 = ya;
    m.rows.resize(yb - ya);
    for (size_t i = 0; i < n; ++i)
      for (int y = b[i].j0; y < b[i].j0 + b[i].ny; ++y) m.rows[y - ya].push_back({b[i].i0, b[i].i0 + b[i].nx});
    for (auto &v : m.rows) {
      std::sort(v.begin(), v.end());
      std::vector<std::pair<int, int>> out;
      for (const auto &iv : v) {
        if (!out.empty() && iv.first <= out.back().second)
          out.back().second = std::max(out.back().second, iv.second);
        else
          out.push_back(iv);
      }
      v.swap(out);
    }
    return m;
  }
};

// Clustering for tag_and_regrid, level l: `hits` (sorted) are the tiles of a
// grid of side T = ceil(min_box / r) level-l cells that hold a cell within the
// dilation buffer of a tag (computed on the device). A hit tile is kept when
// it and the ring of cells around it are covered at level l (cells outside a
// non-periodic side exempt, periodic axes wrapped), which keeps the new
// level properly nested. Kept tiles merge greedily into rectangles: runs of
// at most maxT tiles along a tile row, stacked while the run below is
// identical, with sides of at most max_box level-(l+1) cells.
void cluster_level(vlbm_ctx *c, int l, const std::vector<int32_t> &hits, const CovMap &cov, int min_box,
                   int max_box, std::vector<vlbm_box> &out) {
  const int r = c->p.r;
  const int Nx = level_nx(c, l), Ny = level_ny(c, l);
  const bool px = c->perx(), py = c->pery();
  const int T = std::max(1, (min_box + r - 1) / r);
  const int maxT = std::max(1, max_box / (T * r));
  const int ntx = (Nx + T - 1) / T, nty = (Ny + T - 1) / T;
  // [xa, xb) of row y covered, y possibly outside the domain (wrapped on a
  // periodic axis, exempt on another)
  auto row_ok = [&](int y, int xa, int xb) {
    if (y < 0 || y >= Ny) {
      if (!py) return true;
      y = (y + Ny) % Ny;
    }
    return cov.span(y, xa, xb);
  };
  auto cell_ok = [&](int x, int y) {
    if (x < 0 || x >= Nx) {
      if (!px) return true;
      x = (x + Nx) % Nx;
    }
    return row_ok(y, x, x + 1);
  };
  auto allowed_slow = [&](int tx, int ty) {
    const int x0 = tx * T, y0 = ty * T, x1 = std::min(Nx, x0 + T), y1 = std::min(Ny, y0 + T);
    for (int y = y0; y < y1; ++y)
      if (!row_ok(y, x0, x1) || !cell_ok(x0 - 1, y) || !cell_ok(x1, y)) return false;
    return row_ok(y0 - 1, x0, x1) && row_ok(y1, x0, x1);
  };
  // Per tile row, the columns covered on every row of the tile (mid) and on
  // the rows just above and below (edge), as merged intervals; a tile away
  // from the x sides is allowed iff [x0 - 1, x1 + 1) lies in mid and
  // [x0, x1) in both edges, the same test as allowed_slow.
  using Iv = std::vector<std::pair<int, int>>;
  auto row_iv = [&](int y, Iv &out) {  // coverage of row y, wrapped or exempt outside
    out.clear();
    if (y < 0 || y >= Ny) {
      if (!py) {
        out.push_back({INT32_MIN, INT32_MAX});
        return;
      }
      y = (y + Ny) % Ny;
    }
    if (cov.all) {
      out.push_back({INT32_MIN, INT32_MAX});
      return;
    }
    const int i = y - cov.y0;
    if (i >= 0 && i < (int)cov.rows.size()) out = cov.rows[i];
  };
  auto intersect = [](const Iv &a, const Iv &b, Iv &out) {
    out.clear();
    size_t i = 0, j = 0;
    while (i < a.size() && j < b.size()) {
      const int lo = std::max(a[i].first, b[j].first), hi = std::min(a[i].second, b[j].second);
      if (lo < hi) out.push_back({lo, hi});
      if (a[i].second < b[j].second) ++i; else ++j;
    }
  };
  auto inside = [](const Iv &v, int xa, int xb) {  // [xa, xb) within one interval of v
    auto it = std::upper_bound(v.begin(), v.end(), std::make_pair(xa, INT32_MAX));
    if (it == v.begin()) return false;
    --it;
    return it->first <= xa && it->second >= xb;
  };
  Iv mid, top, bot, tmp, cur;
  int row_ty = -1;
  auto allowed = [&](int tx, int ty) {
    const int x0 = tx * T, x1 = std::min(Nx, x0 + T);
    if (x0 == 0 || x1 >= Nx) return allowed_slow(tx, ty);
    if (ty != row_ty) {
      row_ty = ty;
      const int y0 = ty * T, y1 = std::min(Ny, y0 + T);
      row_iv(y0, mid);
      for (int y = y0 + 1; y < y1 && !mid.empty(); ++y) {
        row_iv(y, cur);
        intersect(mid, cur, tmp);
        mid.swap(tmp);
      }
      row_iv(y0 - 1, top);
      row_iv(y1, bot);
    }
    return inside(mid, x0 - 1, x1 + 1) && inside(top, x0, x1) && inside(bot, x0, x1);
  };
  struct Run { int a, b, y0, h; };
  std::vector<Run> open, next;
  auto emit = [&](const Run &u) {
    int x0 = u.a * T, x1 = std::min(Nx, u.b * T), y0 = u.y0 * T, y1 = std::min(Ny, (u.y0 + u.h) * T);
    out.push_back({l + 1, x0 * r, y0 * r, (x1 - x0) * r, (y1 - y0) * r});
  };
  // one tile row: its runs of kept tiles; then the open rectangles continue
  // (identical run below, room to grow) or are emitted
  // (the runs of a row are disjoint and both lists are ordered by a, so the
  // run of the new row that starts where an open rectangle does is found by
  // one merged pass)
  auto close_row = [&](int ty) {
    size_t j = 0;
    for (auto &o : open) {
      while (j < next.size() && next[j].a < o.a) ++j;
      if (j < next.size() && next[j].a == o.a && next[j].b == o.b && next[j].h == 1 && o.h < maxT) {
        next[j].y0 = o.y0;
        next[j].h = o.h + 1;
      } else {
        emit(o);
      }
    }
    open.swap(next);
    next.clear();
    (void)ty;
  };
  size_t i = 0;
  int last_ty = -2;
  while (i < hits.size()) {
    const int ty = (int)(hits[i] / ntx);
    if (ty != last_ty + 1 && !open.empty()) close_row(last_ty + 1);  // an empty tile row between
    // kept tiles of this row, in order, cut into runs of at most maxT
    int run_a = -1, run_b = -1;
    for (; i < hits.size() && hits[i] / ntx == ty; ++i) {
      const int tx = (int)(hits[i] % ntx);
      if (!allowed(tx, ty)) continue;
      if (run_a >= 0 && tx == run_b && run_b - run_a < maxT) {
        run_b = tx + 1;
        continue;
      }
      if (run_a >= 0) next.push_back({run_a, run_b, ty, 1});
      run_a = tx;
      run_b = tx + 1;
    }
    if (run_a >= 0) next.push_back({run_a, run_b, ty, 1});
    close_row(ty);
    last_ty = ty;
  }
  next.clear();
  close_row(nty);  // emits whatever is still open
}

int level_nx(const vlbm_ctx *c, int l) {
  long s = 1;
  for (int i = 0; i < l; ++i) s *= c->p.r;
  return (int)(c->p.nx0 * s);
}
int level_ny(const vlbm_ctx *c, int l) {
  long s = 1;
  for (int i = 0; i < l; ++i) s *= c->p.r;
  return (int)(c->p.ny0 * s);
}

// Refinement tags of the present levels l with dtag[l] set, into dtag[l]
// (device, indexed like each level's status): the density-gradient indicator,
// or the sensor of eq. amr-sigma, whose flux maxima run over every level.
// Scratch slot of the density plane (tag_and_regrid numbers its own slots
// from 0, a few per level).
constexpr size_t kRhoSlot = 64;

hipError_t launch_level_tags(vlbm_ctx *c, double thr, const std::vector<uint8_t *> &dtag) {
  hipError_t e = hipSuccess;
  if (c->tag_kind == VLBM_TAG_FLUX) {
    if (!c->dflux_qmax) c->dflux_qmax = static_cast<unsigned long long *>(c->mem.alloc(4 * sizeof(unsigned long long)));
    if (!c->dflux_qmax) return hipErrorOutOfMemory;
    e = launch_clear_u64(c->dflux_qmax, 4, c->stream);
    for (int l = 0; l < c->nlev && e == hipSuccess; ++l) {
      const Level &L = c->lv[l];
      e = launch_flux_max(L.buf[L.cur()], L.dtiles, (int)L.tiles.size(), L.plane, L.pitch, c->fp32, c->eos,
                          c->dflux_qmax, c->stream);
    }
  }
  for (int l = 0; l < (int)dtag.size() && l < c->nlev && e == hipSuccess; ++l) {
    if (!dtag[l]) continue;
    const Level &L = c->lv[l];
    if (c->tag_kind == VLBM_TAG_FLUX)
      e = launch_tag_flux(L.buf[L.cur()], L.dstatus, L.dsrow, L.dyrow, L.plane, L.pitch, L.xoff, L.fx0, L.fy0,
                          L.fw, L.fh, L.nrows, L.Nx, L.Ny, c->perx(), c->pery(), c->fp32, c->eos, c->dflux_qmax,
                          thr, dtag[l], c->stream);
    else {
      // the density plane: one scratch slot of its own, shared by the levels
      // (their launches follow each other on the stream)
      double *rho = static_cast<double *>(c->scratch_slot(kRhoSlot, sizeof(double) * (size_t)L.fw * L.nrows));
      if (!rho) return hipErrorOutOfMemory;
      e = launch_tag(L.buf[L.cur()], L.dstatus, L.dsrow, L.dyrow, L.plane, L.pitch, L.xoff, L.fx0, L.fy0, L.fw,
                     L.fh, L.nrows, L.Nx, L.Ny, c->perx(), c->pery(), c->fp32, thr, rho, dtag[l], c->stream);
    }
  }
  return e;
}

// Refinement tags of level l's active cells, indexed like its status (fw
// bytes per stored row).
vlbm_status tag_frame(vlbm_ctx *c, int l, double thr, std::vector<uint8_t> &ft) {
  const Level &L = c->lv[l];
  const size_t n = (size_t)L.fw * L.nrows;
  ft.assign(n, 0);
  uint8_t *d = static_cast<uint8_t *>(c->mem.alloc(n));
  if (!d) return fail(VLBM_ENOMEM, "tag buffer");
  std::vector<uint8_t *> dtag(l + 1, nullptr);
  dtag[l] = d;
  hipError_t e = launch_level_tags(c, thr, dtag);
  if (e == hipSuccess) e = hipMemcpyAsync(ft.data(), d, n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->mem.release(d);
  if (e == hipErrorOutOfMemory) return fail(VLBM_ENOMEM, "tag scratch");
  if (e != hipSuccess) return fail(VLBM_EDEVICE, "tag: %s", hipGetErrorString(e));
  return VLBM_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *vlbm_last_error(void) { return g_err.c_str(); }
}  // extern "C"

// The three-dimensional path (api3.hip) reports through the same message.
namespace vlbm {
void set_error_message(const char *msg) { g_err = msg; }
}  // namespace vlbm

extern "C" {

vlbm_status vlbm_create(const vlbm_params *params, void *stream, vlbm_ctx **out) {
  if (!params || !out) return fail(VLBM_EINVAL, "null argument");
  const vlbm_params &p = *params;
  if (p.nx0 < 1 || p.ny0 < 1 || !(p.dx0 > 0) || p.r < 1 || p.r > 8 || p.max_levels < 1 ||
      p.max_levels > kMaxLevels || !(p.c > 0) || !(p.beta >= 0 && p.beta <= 1) ||
      !(p.gamma > 1) ||
      (p.precision != VLBM_FP64 && p.precision != VLBM_FP32 && p.precision != VLBM_FP32_STORAGE) ||
      p.eos < VLBM_EOS_IDEAL || p.eos > VLBM_EOS_VDW || !(p.eos_b >= 0.0) || !std::isfinite(p.eos_a))
    return fail(VLBM_EINVAL, "invalid parameters");
  for (int s = 0; s < 4; ++s)
    if (p.bc[s] < 0 || p.bc[s] > 3) return fail(VLBM_EINVAL, "invalid boundary condition");
  if ((p.bc[0] == VLBM_BC_PERIODIC) != (p.bc[1] == VLBM_BC_PERIODIC) ||
      (p.bc[2] == VLBM_BC_PERIODIC) != (p.bc[3] == VLBM_BC_PERIODIC))
    return fail(VLBM_EINVAL, "periodic sides must come in pairs");
  long s = 1;
  for (int i = 1; i < p.max_levels; ++i) s *= p.r;
  if ((double)p.nx0 * s + 2 > 2e9 || (double)p.ny0 * s + 2 > 2e9)
    return fail(VLBM_EINVAL, "finest level too large");
  vlbm_ctx *c = new vlbm_ctx();
  c->p = p;
  c->stream = static_cast<hipStream_t>(stream);
  c->fp32 = p.precision != VLBM_FP64;
  if (p.precision == VLBM_FP32_STORAGE) c->step_flags |= STEP_F64_MATH;
  c->esz = c->fp32 ? 4 : 8;
  c->tile_cells = tile_cells_default();
  if (const char *e = getenv("VLBM_NT_STORES")) c->step_flags |= atoi(e) ? STEP_NT_STORES : 0;
  if (const char *e = getenv("VLBM_TWO_CELLS")) c->step_flags |= atoi(e) ? STEP_TWO_CELLS : 0;
  if (const char *e = getenv("VLBM_XCD_CONTIGUOUS")) c->step_flags |= atoi(e) ? STEP_XCD_CONTIGUOUS : 0;
  if (const char *e = getenv("VLBM_GRAPHS")) c->step_flags |= atoi(e) ? STEP_GRAPHS : 0;
  c->use_graphs = (c->step_flags & STEP_GRAPHS) != 0;
  c->gm1 = p.gamma - 1.0;
  c->eos = EosT<double>{p.eos, p.gamma - 1.0, p.eos_a, p.eos_b, p.gamma * p.eos_a};
  c->h = 1.0 / (2.0 * p.c);
  c->tb = 2.0 * p.beta;
  *out = c;
  return VLBM_OK;
}

void vlbm_destroy(vlbm_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  drop_batch_graphs(c);
  for (hipEvent_t ev : c->pev) (void)hipEventDestroy(ev);
  for (int l = 0; l < kMaxLevels; ++l) free_level(c, c->lv[l]);
  c->mem.release(c->ddesc);
  c->mem.release(c->dseg);
  c->mem.release(c->dflag);
  c->mem.release(c->dqmax);
  c->mem.release(c->ddyn);
  c->mem.release(c->dcmax);
  for (auto &e : c->tag_scratch) c->mem.release(e.first);
  c->mem.release(c->dflux_qmax);
  c->mem.release_all();
  if (c->stage) (void)hipHostFree(c->stage);
  delete c;
}

vlbm_status vlbm_bind_pool(vlbm_ctx *c, void *dev, size_t bytes) {
  if (!c || !dev || bytes < 4096) return fail(VLBM_EINVAL, "bad pool");
  if (c->have_hierarchy || c->mem.ext_alloc) return fail(VLBM_ESTATE, "bind the pool before set_hierarchy");
  c->mem.bind(dev, bytes);
  return VLBM_OK;
}

vlbm_status vlbm_bind_allocator(vlbm_ctx *c, vlbm_alloc_fn alloc, vlbm_free_fn release, void *user) {
  if (!c || !alloc || !release) return fail(VLBM_EINVAL, "null allocator");
  if (c->have_hierarchy || c->mem.bound || !c->mem.owned_.empty())
    return fail(VLBM_ESTATE, "bind the allocator before set_hierarchy");
  c->mem.drop_cache();
  c->mem.ext_alloc = alloc;
  c->mem.ext_free = release;
  c->mem.ext_user = user;
  return VLBM_OK;
}

size_t vlbm_footprint_bytes(const vlbm_params *params, const vlbm_box *boxes, int nboxes) {
  if (!params) return 0;
  Geometry g;
  if (check_boxes(*params, boxes, nboxes, g) != VLBM_OK) return 0;
  size_t esz = params->precision == VLBM_FP32 ? 4 : 8, total = 0, stage = 0;
  for (int l = 0; l < kMaxLevels && g.present[l]; ++l) {
    Level L;
    frame_of(*params, esz, g, l, L);
    size_t cells = (size_t)L.fw * L.nrows;
    total += DevMem::round(level_bytes(L, esz)) * 2;  // two time levels
    total += DevMem::round(cells);                    // status
    total += DevMem::round(sizeof(int32_t) * ((size_t)L.fh + L.nrows));  // row tables
    stage = std::max(stage, DevMem::round(sizeof(double) * 16 * cells));  // a whole-level read
    // tiles, tasks, accumulators, ledger, partials: bounded by the perimeter
    size_t perim = 2 * ((size_t)L.fw * L.runs.size() + L.nrows) * 4 + 64;
    total += DevMem::round(sizeof(Task) * perim * 2) + DevMem::round(sizeof(double) * 4 * perim * 2);
    total += DevMem::round((cells / 64 + 64) * (sizeof(Tile) + 4 * sizeof(double)));
  }
  return total + stage + (1 << 20);
}

}  // extern "C"

namespace {
// A level's frame as a checkpoint records it: columns [bx0, bx1) of the
// coverage's bounding box and the stored row runs.
struct FrameSpec {
  int bx0 = 0, bx1 = 0;
  Runs rows;
};

// Install a hierarchy; with specs (one per level, a checkpoint's frames) every
// level takes exactly that frame, which must hold its boxes.
vlbm_status set_hierarchy_impl(vlbm_ctx *c, const vlbm_box *boxes, int nboxes, const FrameSpec *specs) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  Geometry g;
  vlbm_status st = check_boxes(c->p, boxes, nboxes, g);
  if (st) return st;
  if (specs)
    for (int l = 0; l < kMaxLevels; ++l) {
      if (!g.present[l]) continue;
      const FrameSpec &f = specs[l];
      if (f.rows.empty() || f.bx0 > g.bx0[l] || f.bx1 < g.bx1[l] || !runs_cover(f.rows, g.rows[l]))
        return fail(VLBM_EINVAL, "checkpoint frame of level %d does not hold its boxes", l);
      g.bx0[l] = f.bx0;
      g.bx1[l] = f.bx1;
      g.rows[l] = f.rows;
    }
  // Build every host table on a scratch context first: a rejected hierarchy
  // leaves the installed one untouched and touches no device state.
  vlbm_ctx *t = new vlbm_ctx();
  t->p = c->p;
  t->esz = c->esz;
  t->tile_cells = c->tile_cells;
  t->step_flags = c->step_flags;
  t->sensor = c->sensor;  // tile shapes follow it
  int nlev = 0;
  for (int l = 0; l < kMaxLevels; ++l) {
    frame_of(c->p, c->esz, g, l, t->lv[l]);
    if (g.present[l]) nlev = l + 1;
    if (t->lv[l].plane >= (int64_t(1) << 31)) {
      delete t;
      return fail(VLBM_EINVAL, "level %d frame too large for 32-bit offsets", l);
    }
  }
  st = build_lists(t, boxes, nboxes);
  if (st) {
    delete t;
    return st;
  }
  vlbm_status sync = VLBM_OK;
  if (hipStreamSynchronize(c->stream) != hipSuccess) sync = fail(VLBM_EDEVICE, "stream sync failed");
  if (sync) {
    delete t;
    return sync;
  }
  for (int l = 0; l < kMaxLevels; ++l) {
    free_level(c, c->lv[l]);
    c->lv[l] = std::move(t->lv[l]);
    c->lv[l].steps = 0;
  }
  delete t;
  c->nlev = nlev;
  for (int l = 0; l < c->nlev; ++l) {
    st = upload_level(c, c->lv[l], true);
    if (st) return st;
  }
  if (!c->dflag) c->dflag = static_cast<int *>(c->mem.alloc(256));
  c->boxes.assign(boxes, boxes + nboxes);
  c->have_hierarchy = true;
  c->coarse_steps = 0;
  return build_tables(c);
}
}  // namespace

extern "C" {

vlbm_status vlbm_set_hierarchy(vlbm_ctx *c, const vlbm_box *boxes, int nboxes) {
  return guarded([&]() -> vlbm_status {
    return set_hierarchy_impl(c, boxes, nboxes, nullptr);
  });
}

vlbm_status vlbm_set_state(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny,
                           const double *U, long ld) {
  if (!U) return fail(VLBM_EINVAL, "null U");
  vlbm_status st = rect_io(c, level, i0, j0, nx, ny, const_cast<double *>(U), ld, 4, true, false);
  if (st) return st;
  c->table_base -= c->coarse_steps;  // keep the table parity while restarting the count
  c->coarse_steps = 0;
  st = reset_time(c);
  return st ? st : reset_ledgers(c);
}

vlbm_status vlbm_set_populations(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny,
                                 const double *F, long ld) {
  if (!F) return fail(VLBM_EINVAL, "null F");
  vlbm_status st = rect_io(c, level, i0, j0, nx, ny, const_cast<double *>(F), ld, 16, true, true);
  if (st) return st;
  c->table_base -= c->coarse_steps;
  c->coarse_steps = 0;
  st = reset_time(c);
  return st ? st : reset_ledgers(c);
}

vlbm_status vlbm_get_state(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny, double *U,
                           long ld) {
  if (!U) return fail(VLBM_EINVAL, "null U");
  return rect_io(c, level, i0, j0, nx, ny, U, ld, 4, false, false);
}

vlbm_status vlbm_get_state_noalloc(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny, double *U,
                                   long ld) {
  if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
  if (!U) return fail(VLBM_EINVAL, "null U");
  vlbm_status st = check_rect(c, level, i0, j0, nx, ny);
  if (st) return st;
  if (ld < nx) return fail(VLBM_EINVAL, "ld < nx");
  if (!c->noalloc_stage) {  // first call of this context: its GPU's array (looked up once per GPU)
    hipDevice_t dev = 0;
    HIPCHK(hipStreamGetDevice(c->stream, &dev));
    st = scratch_address((int)dev, &c->noalloc_stage);
    if (st) return st;
  }
  Level &L = c->lv[level];
  int ci0 = i0, cj0 = j0, cnx = nx, cny = ny, ox = 0, oy = 0;
  const bool any = L.present && clip_to_frame(L, ci0, cj0, cnx, cny, ox, oy);
  const size_t n = any ? (size_t)cnx * cny : 0;
  if (n * 4 * sizeof(double) > VLBM_NOALLOC_STAGE_BYTES)
    return fail(VLBM_EINVAL, "rectangle part inside the frame has %zu cells; the static staging holds %zu",
                n, (size_t)VLBM_NOALLOC_STAGE_BYTES / (4 * sizeof(double)));
  const size_t full_plane = (size_t)ny * ld;
  for (int k = 0; k < 4; ++k)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) U[k * full_plane + (size_t)y * ld + x] = NAN;
  if (!any) return VLBM_OK;
  RectArgs a{};
  a.buf0 = L.buf[L.cur()];
  a.buf1 = L.buf[1];
  a.status = L.dstatus;
  a.host_stage = c->noalloc_stage;
  a.plane = L.plane;
  a.pitch = L.pitch;
  a.xoff = L.xoff;
  a.fx0 = L.fx0;
  a.fy0 = L.fy0;
  a.fw = L.fw;
  a.srow = L.dsrow;
  a.x0 = ci0;
  a.y0 = cj0;
  a.nx = cnx;
  a.ny = cny;
  a.gm1 = c->gm1;
  a.h = c->h;
  a.eos = c->eos;
  HIPCHK(launch_get(a, c->fp32, 0, c->stream));
  for (int k = 0; k < 4; ++k)
    HIPCHK(hipMemcpy2DAsync(U + k * full_plane + (size_t)oy * ld + ox, sizeof(double) * ld,
                            c->noalloc_stage + k * n, sizeof(double) * cnx, sizeof(double) * cnx, cny,
                            hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return VLBM_OK;
}

vlbm_status vlbm_get_populations(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny,
                                 double *F, long ld) {
  if (!F) return fail(VLBM_EINVAL, "null F");
  return rect_io(c, level, i0, j0, nx, ny, F, ld, 16, false, false);
}

vlbm_status vlbm_advance(vlbm_ctx *c, int n) {
  if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
  if (n < 0) return fail(VLBM_EINVAL, "negative step count");
  return advance_impl(c, n);
}

vlbm_status vlbm_conserved_totals(vlbm_ctx *c, double totals[4], double ledger[4]) {
  if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
  double T[4] = {0, 0, 0, 0}, Tc[4] = {0, 0, 0, 0}, G[4] = {0, 0, 0, 0}, Gc[4] = {0, 0, 0, 0};
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->lv[l];
    const int nt = (int)L.tiles.size();
    HIPCHK(launch_audit(L.buf[L.cur()], L.dtiles, nt, L.plane, L.pitch, c->fp32, L.dpartial, c->stream));
    std::vector<double> part(4 * (size_t)std::max(nt, 1)), led(4 * (size_t)std::max(L.nledger, 1));
    if (nt) HIPCHK(hipMemcpyAsync(part.data(), L.dpartial, sizeof(double) * 4 * nt, hipMemcpyDeviceToHost, c->stream));
    if (L.nledger)
      HIPCHK(hipMemcpyAsync(led.data(), L.dledger, sizeof(double) * 4 * L.nledger, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < 4; ++k) {
      double s = 0, sc = 0;
      for (int t = 0; t < nt; ++t) kadd(s, sc, part[4 * t + k]);
      kadd(T[k], Tc[k], L.dx * L.dx * (s + sc));
      for (int t = 0; t < L.nledger; ++t) kadd(G[k], Gc[k], led[4 * t + k]);
    }
  }
  for (int k = 0; k < 4; ++k) {
    kadd(G[k], Gc[k], c->ledger_carry[k]);
    kadd(G[k], Gc[k], c->ledger_carry_c[k]);
    if (totals) totals[k] = T[k] + Tc[k];
    if (ledger) ledger[k] = G[k] + Gc[k];
  }
  return VLBM_OK;
}

vlbm_status vlbm_check_health(vlbm_ctx *c) {
  if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
  HIPCHK(hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
  for (int l = 0; l < c->nlev; ++l) {
    Level &L = c->lv[l];
    HIPCHK(launch_health(L.buf[L.cur()], L.dtiles, (int)L.tiles.size(), L.plane, L.pitch, c->fp32,
                         c->eos, c->dflag, c->stream));
  }
  int flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (flag) return fail(VLBM_EUNSTABLE, "non-physical state (rho <= 0, p <= 0 or NaN)");
  return VLBM_OK;
}

vlbm_status vlbm_tag(vlbm_ctx *c, int level, double thr, unsigned char *tags) {
  if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
  if (level < 0 || level >= c->p.max_levels || !tags) return fail(VLBM_EINVAL, "bad tag request");
  const Level &L = c->lv[level];
  const int Nx = level_nx(c, level), Ny = level_ny(c, level);
  memset(tags, 0, (size_t)Nx * Ny);
  if (!L.present) return VLBM_OK;
  std::vector<uint8_t> ft;
  vlbm_status st = tag_frame(c, level, thr, ft);
  if (st) return st;
  for (int sr = 0; sr < L.nrows; ++sr) {  // stored rows inside the level; interior columns
    const int y = L.fy0 + L.yrow[sr];
    if (y >= 0 && y < Ny) memcpy(&tags[(size_t)y * Nx + L.fx0 + 1], &ft[(size_t)sr * L.fw + 1], L.fw - 2);
  }
  return VLBM_OK;
}

vlbm_status vlbm_set_tag_indicator(vlbm_ctx *c, int kind) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  if (kind != VLBM_TAG_DENSITY && kind != VLBM_TAG_FLUX) return fail(VLBM_EINVAL, "unknown tag indicator %d", kind);
  c->tag_kind = kind;
  return VLBM_OK;
}

vlbm_status vlbm_get_boxes(vlbm_ctx *c, vlbm_box *boxes, int cap, int *nboxes) {
  if (!c || !nboxes) return fail(VLBM_EINVAL, "null argument");
  *nboxes = (int)c->boxes.size();
  for (int i = 0; i < cap && i < (int)c->boxes.size(); ++i) boxes[i] = c->boxes[i];
  return VLBM_OK;
}

vlbm_status vlbm_regrid(vlbm_ctx *c, const vlbm_box *boxes, int nboxes) {
  return guarded([&]() -> vlbm_status {
    if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
    // The same boxes again: nothing is merged or split and every interface is
    // kept, so the hierarchy, its lists and both time levels stay as they are.
    if (nboxes >= 0 && (size_t)nboxes == c->boxes.size() && (nboxes == 0 || boxes)) {
      bool same = true;
      for (int b = 0; b < nboxes && same; ++b) {
        const vlbm_box &u = boxes[b], &v = c->boxes[b];
        same = u.level == v.level && u.i0 == v.i0 && u.j0 == v.j0 && u.nx == v.nx && u.ny == v.ny;
      }
      if (same) return VLBM_OK;
    }
    return regrid_impl(c, boxes, nboxes);
  });
}

vlbm_status vlbm_tag_and_regrid(vlbm_ctx *c, double thr, int buffer, int min_box, int max_box) {
  return guarded([&]() -> vlbm_status {
    if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
    if (buffer < 0 || min_box < 1 || max_box < min_box) return fail(VLBM_EINVAL, "bad clustering sizes");
    PhaseTimer tm("tag_and_regrid");
    const int ML = c->p.max_levels;
    if (ML < 2) return VLBM_OK;
    const int r = c->p.r;
    const int nclu = std::min(c->nlev, ML - 1);  // levels whose tags make the next level's boxes
    // 1. tags of every present level on the device (indexed like each level's
    //    status); a tagged cell also tags its parent, finest level first, so
    //    refined features keep their levels. Scratch: slots of the context's
    //    tag scratch (kept between calls).
    size_t next_slot = 0;
    auto dalloc = [&](size_t n) -> void * { return c->scratch_slot(next_slot++, n); };
    auto release = [&]() {};
    if (getenv("VLBM_TIMING")) {  // separate the regrid's own time from the steps queued before it
      HIPCHK(hipStreamSynchronize(c->stream));
      tm.mark("queued steps");
    }
    std::vector<uint8_t *> dtag(c->nlev, nullptr);
    for (int l = 0; l < c->nlev; ++l) {
      const Level &L = c->lv[l];
      dtag[l] = static_cast<uint8_t *>(dalloc((size_t)L.fw * L.nrows));
      if (!dtag[l]) {
        release();
        return fail(VLBM_ENOMEM, "tag buffer");
      }
    }
    hipError_t e = launch_level_tags(c, thr, dtag);
    for (int l = c->nlev - 1; l >= 1 && e == hipSuccess; --l) {
      const Level &F = c->lv[l], &P = c->lv[l - 1];
      e = launch_tag_parents(dtag[l], F.dyrow, F.fx0, F.fy0, F.fw, F.nrows, dtag[l - 1], P.dsrow, P.fx0, P.fy0,
                             P.fw, P.fh, r, c->stream);
    }
    // 2. per clustered level, the tiles within `buffer` of a tag, listed on the
    //    device (few tiles of a large level are hit); only tile rows within
    //    `buffer` of a stored frame row can hold one
    const int T = std::max(1, (min_box + r - 1) / r);
    std::vector<int32_t *> dlist(nclu, nullptr);
    std::vector<int> cap(nclu, 0);
    int *dcount = static_cast<int *>(dalloc(sizeof(int) * std::max(nclu, 1)));
    if (!dcount) {
      release();
      return fail(VLBM_ENOMEM, "tile lists");
    }
    if (e == hipSuccess) e = hipMemsetAsync(dcount, 0, sizeof(int) * std::max(nclu, 1), c->stream);
    std::vector<std::vector<int32_t>> trows(nclu);
    for (int l = 0; l < nclu && e == hipSuccess; ++l) {
      const Level &L = c->lv[l];
      const int ntx = (L.Nx + T - 1) / T, nty = (L.Ny + T - 1) / T;
      std::vector<uint8_t> want(nty, 0);
      for (const auto &run : L.runs) {
        const int ya = std::max(0, run.first) - buffer, yb = std::min(L.Ny, run.second) + buffer;
        if (c->pery() && yb - ya >= L.Ny) {
          std::fill(want.begin(), want.end(), 1);
          break;
        }
        for (int y = ya; y < yb; ++y) {
          int wy = y;
          if (wy < 0 || wy >= L.Ny) {
            if (!c->pery()) continue;
            wy = (wy + L.Ny) % L.Ny;
          }
          want[wy / T] = 1;
        }
      }
      for (int ty = 0; ty < nty; ++ty)
        if (want[ty]) trows[l].push_back(ty);
      const int64_t ntiles = (int64_t)ntx * (int64_t)trows[l].size();
      if (ntiles >= (int64_t(1) << 31)) {
        release();
        return fail(VLBM_EINVAL, "clustering grid of level %d too large", l);
      }
      cap[l] = (int)ntiles;
      dlist[l] = static_cast<int32_t *>(dalloc(sizeof(int32_t) * (size_t)std::max<int64_t>(ntiles, 1)));
      int32_t *dtrows = static_cast<int32_t *>(dalloc(sizeof(int32_t) * std::max<size_t>(trows[l].size(), 1)));
      auto *dmasks = static_cast<unsigned long long *>(
          dalloc(sizeof(unsigned long long) * (size_t)std::max(L.nrows, 1) * (size_t)((L.Nx + 63) / 64)));
      if (!dlist[l] || !dtrows || !dmasks) {
        release();
        return fail(VLBM_ENOMEM, "tile lists");
      }
      if (!trows[l].empty())
        e = stage_h2d(c, dtrows, trows[l].data(), sizeof(int32_t) * trows[l].size());
      if (e == hipSuccess)
        e = launch_tile_hits(dtag[l], L.dsrow, L.fx0, L.fy0, L.fw, L.fh, L.nrows, L.Nx, L.Ny, c->perx(), c->pery(),
                             T, buffer, ntx, dtrows, (int)trows[l].size(), dmasks, dlist[l], cap[l], dcount + l,
                             c->stream);
    }
    std::vector<int> count(std::max(nclu, 1), 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(count.data(), dcount, sizeof(int) * std::max(nclu, 1), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<std::vector<int32_t>> hits(nclu);
    for (int l = 0; l < nclu && e == hipSuccess; ++l) {
      hits[l].resize(std::min(count[l], cap[l]));
      if (!hits[l].empty())
        e = hipMemcpyAsync(hits[l].data(), dlist[l], sizeof(int32_t) * hits[l].size(), hipMemcpyDeviceToHost,
                           c->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    release();
    if (e == hipErrorOutOfMemory) return fail(VLBM_ENOMEM, "tag scratch");
    if (e != hipSuccess) return fail(VLBM_EDEVICE, "tag and cluster: %s", hipGetErrorString(e));
    tm.mark("tags+tiles");
    // 3. boxes, level by level: each level's kept tiles must lie in the
    //    coverage of the boxes just made for it
    std::vector<vlbm_box> boxes;
    CovMap cov;
    cov.all = true;
    for (int l = 0; l < nclu; ++l) {
      const size_t before = boxes.size();
      // the hits in tile order: a bit per tile of the scanned tile rows (the
      // device appends them a wavefront at a time, in any order)
      {
        const Level &L = c->lv[l];
        const int ntx = (L.Nx + T - 1) / T, nty = (L.Ny + T - 1) / T;
        std::vector<int32_t> row_of(nty, -1);
        for (size_t k = 0; k < trows[l].size(); ++k) row_of[trows[l][k]] = (int32_t)k;
        const int64_t nbit = (int64_t)ntx * (int64_t)trows[l].size();
        std::vector<uint64_t> bits((size_t)((nbit + 63) / 64), 0);
        for (int32_t h : hits[l]) {
          if (h < 0 || h / ntx >= nty || row_of[h / ntx] < 0) continue;  // only scanned tiles are listed
          const int64_t k = (int64_t)row_of[h / ntx] * ntx + h % ntx;
          bits[(size_t)(k >> 6)] |= 1ull << (k & 63);
        }
        size_t n = 0;
        for (size_t wi = 0; wi < bits.size(); ++wi)
          for (uint64_t w = bits[wi]; w; w &= w - 1) {
            const int64_t k = (int64_t)wi * 64 + __builtin_ctzll(w);
            hits[l][n++] = trows[l][(size_t)(k / ntx)] * ntx + (int32_t)(k % ntx);
          }
        hits[l].resize(n);
      }
      cluster_level(c, l, hits[l], cov, min_box, max_box, boxes);
      static const char *const kClu[] = {"cluster l0", "cluster l1", "cluster l2", "cluster l3+"};
      tm.mark(kClu[std::min(l, 3)]);
      if (boxes.size() == before || l + 2 >= ML) break;
      cov = CovMap::of_boxes(boxes.data() + before, boxes.size() - before);
    }
    tm.mark("cluster");
    return vlbm_regrid(c, boxes.data(), (int)boxes.size());
  });
}

// Checkpoint layout: header; boxes; per present level its frame {bx0, bx1,
// number of row runs, the runs}; then per present level {steps, nacc,
// nledger, both buffers, reflux accumulators, ledger slots}. The header
// carries the ledger carry and, for the adaptive time step, the link speeds
// of the current and previous coarse step and the elapsed time.
struct CkptHeader {
  char magic[8];
  vlbm_params p;
  int32_t nboxes, nlev;
  int64_t coarse_steps;
  double carry[4], carry_c[4];
  int32_t adt, pad;
  double dyn_c, dyn_c_prev, dyn_time;
};

vlbm_status vlbm_save(vlbm_ctx *c, void *buf, size_t *bytes) {
  if (!c || !c->have_hierarchy || !bytes) return fail(VLBM_ESTATE, "nothing to save");
  size_t need = sizeof(CkptHeader) + sizeof(vlbm_box) * c->boxes.size();
  for (int l = 0; l < c->nlev; ++l) {
    const Level &L = c->lv[l];
    need += 3 * sizeof(int32_t) + 2 * sizeof(int32_t) * L.runs.size();
    need += sizeof(int64_t) + 2 * sizeof(int32_t) + 2 * level_bytes(L, c->esz) +
            sizeof(double) * 4 * ((size_t)L.nacc + L.nledger);
  }
  if (!buf) {
    *bytes = need;
    return VLBM_OK;
  }
  if (*bytes < need) return fail(VLBM_EINVAL, "checkpoint buffer too small (%zu < %zu)", *bytes, need);
  char *p = static_cast<char *>(buf);
  auto put = [&](const void *v, size_t n) {
    memcpy(p, v, n);
    p += n;
  };
  CkptHeader h{};
  memcpy(h.magic, "VLBMCK2", 8);
  h.p = c->p;
  h.nboxes = (int32_t)c->boxes.size();
  h.nlev = c->nlev;
  h.coarse_steps = c->coarse_steps;
  for (int k = 0; k < 4; ++k) {
    h.carry[k] = c->ledger_carry[k];
    h.carry_c[k] = c->ledger_carry_c[k];
  }
  h.adt = c->adt ? 1 : 0;
  if (c->adt) {
    double dyn[DYN_SLOTS];
    HIPCHK(hipMemcpyAsync(dyn, c->ddyn, sizeof dyn, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    h.dyn_c = dyn[DYN_C];
    h.dyn_c_prev = dyn[DYN_C_PREV];
    h.dyn_time = dyn[DYN_TIME];
  }
  put(&h, sizeof h);
  put(c->boxes.data(), sizeof(vlbm_box) * c->boxes.size());
  for (int l = 0; l < c->nlev; ++l) {
    const Level &L = c->lv[l];
    const int32_t fr[3] = {L.fx0 + 1, L.fx0 + L.fw - 1, (int32_t)L.runs.size()};
    put(fr, sizeof fr);
    for (const auto &r : L.runs) {
      const int32_t rr[2] = {r.first, r.second};
      put(rr, sizeof rr);
    }
  }
  for (int l = 0; l < c->nlev; ++l) {
    const Level &L = c->lv[l];
    const int64_t steps = L.steps;
    const int32_t counts[2] = {L.nacc, L.nledger};
    put(&steps, sizeof steps);
    put(counts, sizeof counts);
    const size_t nb = level_bytes(L, c->esz);
    for (int b = 0; b < 2; ++b) {
      HIPCHK(hipMemcpyAsync(p, L.buf[b], nb, hipMemcpyDeviceToHost, c->stream));
      p += nb;
    }
    if (L.nacc) HIPCHK(hipMemcpyAsync(p, L.dacc, sizeof(double) * 4 * L.nacc, hipMemcpyDeviceToHost, c->stream));
    p += sizeof(double) * 4 * L.nacc;
    if (L.nledger)
      HIPCHK(hipMemcpyAsync(p, L.dledger, sizeof(double) * 4 * L.nledger, hipMemcpyDeviceToHost, c->stream));
    p += sizeof(double) * 4 * L.nledger;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  *bytes = need;
  return VLBM_OK;
}

// Every read is checked against the buffer's size before it is made; a
// checkpoint that does not fit the context (parameters, time stepping mode,
// levels, frames, slot counts) is refused with VLBM_EINVAL.
vlbm_status vlbm_load(vlbm_ctx *c, const void *buf, size_t bytes) {
  return guarded([&]() -> vlbm_status {
    if (!c || !buf) return fail(VLBM_EINVAL, "bad checkpoint");
    const char *const base = static_cast<const char *>(buf);
    size_t at = 0;
    auto take = [&](void *v, size_t n) -> bool {
      if (n > bytes - at) return false;
      memcpy(v, base + at, n);
      at += n;
      return true;
    };
    CkptHeader h;
    if (bytes < sizeof h || !take(&h, sizeof h) || memcmp(h.magic, "VLBMCK2", 8) != 0)
      return fail(VLBM_EINVAL, "not a checkpoint");
    {
      const vlbm_params &a = h.p, &b = c->p;
      bool same = a.nx0 == b.nx0 && a.ny0 == b.ny0 && a.dx0 == b.dx0 && a.gamma == b.gamma &&
                  a.c == b.c && a.beta == b.beta && a.r == b.r && a.max_levels == b.max_levels &&
                  a.precision == b.precision && a.eos == b.eos && a.eos_a == b.eos_a && a.eos_b == b.eos_b;
      for (int s = 0; s < 4; ++s) {
        same = same && a.bc[s] == b.bc[s];
        for (int k = 0; k < 4; ++k) same = same && a.w_inflow[s][k] == b.w_inflow[s][k];
      }
      if (!same) return fail(VLBM_EINVAL, "checkpoint parameters differ from the context's");
    }
    if ((h.adt != 0) != c->adt)
      return fail(VLBM_EINVAL, "checkpoint taken with the adaptive time step %s, context has it %s",
                  h.adt ? "on" : "off", c->adt ? "on" : "off");
    if (h.nboxes < 0 || h.nlev < 1 || h.nlev > kMaxLevels || h.coarse_steps < 0 ||
        (size_t)h.nboxes > (bytes - at) / sizeof(vlbm_box))
      return fail(VLBM_EINVAL, "corrupt checkpoint header");
    std::vector<vlbm_box> boxes(h.nboxes);
    if (h.nboxes) take(boxes.data(), sizeof(vlbm_box) * h.nboxes);
    FrameSpec specs[kMaxLevels];
    for (int l = 0; l < h.nlev; ++l) {
      int32_t fr[3];
      if (!take(fr, sizeof fr)) return fail(VLBM_EINVAL, "truncated checkpoint");
      if (fr[2] < 1 || fr[0] >= fr[1] || (size_t)fr[2] > (bytes - at) / (2 * sizeof(int32_t)))
        return fail(VLBM_EINVAL, "corrupt checkpoint frame (level %d)", l);
      specs[l].bx0 = fr[0];
      specs[l].bx1 = fr[1];
      for (int i = 0; i < fr[2]; ++i) {
        int32_t rr[2];
        take(rr, sizeof rr);
        if (rr[0] >= rr[1] || (!specs[l].rows.empty() && rr[0] <= specs[l].rows.back().second))
          return fail(VLBM_EINVAL, "corrupt checkpoint frame (level %d)", l);
        specs[l].rows.push_back({rr[0], rr[1]});
      }
    }
    vlbm_status st = set_hierarchy_impl(c, boxes.data(), h.nboxes, specs);
    if (st) return st;
    if (c->nlev != h.nlev) return fail(VLBM_EINVAL, "checkpoint level count mismatch");
    for (int l = 0; l < c->nlev; ++l) {
      Level &L = c->lv[l];
      int64_t steps;
      int32_t counts[2];
      if (!take(&steps, sizeof steps) || !take(counts, sizeof counts)) return fail(VLBM_EINVAL, "truncated checkpoint");
      if (steps < 0 || counts[0] != L.nacc || counts[1] != L.nledger)
        return fail(VLBM_EINVAL, "checkpoint level %d does not match its hierarchy", l);
      const size_t nb = level_bytes(L, c->esz);
      const size_t slots = sizeof(double) * 4 * ((size_t)L.nacc + L.nledger);
      if (bytes - at < 2 * nb || bytes - at - 2 * nb < slots) return fail(VLBM_EINVAL, "truncated checkpoint");
      L.steps = steps;
      for (int b = 0; b < 2; ++b) {
        HIPCHK(hipMemcpyAsync(L.buf[b], base + at, nb, hipMemcpyHostToDevice, c->stream));
        at += nb;
      }
      if (L.nacc) HIPCHK(hipMemcpyAsync(L.dacc, base + at, sizeof(double) * 4 * L.nacc, hipMemcpyHostToDevice, c->stream));
      at += sizeof(double) * 4 * L.nacc;
      if (L.nledger)
        HIPCHK(hipMemcpyAsync(L.dledger, base + at, sizeof(double) * 4 * L.nledger, hipMemcpyHostToDevice, c->stream));
      at += sizeof(double) * 4 * L.nledger;
    }
    if (c->adt) {
      double dyn[DYN_SLOTS];
      HIPCHK(hipMemcpyAsync(dyn, c->ddyn, sizeof dyn, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      dyn[DYN_C] = h.dyn_c;
      dyn[DYN_H] = 1.0 / (2.0 * h.dyn_c);
      dyn[DYN_C_PREV] = h.dyn_c_prev;
      dyn[DYN_TIME] = h.dyn_time;
      HIPCHK(hipMemcpyAsync(c->ddyn, dyn, sizeof dyn, hipMemcpyHostToDevice, c->stream));
      c->cfl_stale = true;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    c->coarse_steps = h.coarse_steps;
    for (int k = 0; k < 4; ++k) {
      c->ledger_carry[k] = h.carry[k];
      c->ledger_carry_c[k] = h.carry_c[k];
    }
    return build_tables(c);
  });
}

}  // extern "C"

namespace {

// A merged batch of contexts: the launches of one coarse step for both table
// parities e (relative to the batch's start). A phase of the merged schedule
// (the deepest context's, unfused) is one step-kernel launch over the
// segments of every context that steps that level there, plus one fused-
// kernel launch over the fused finest levels placed at its second sub-step.
struct BatchLaunch {
  int32_t seg0 = 0, nseg = 0, nblocks = 0, flags = 0, first = 0;
  double ak = 0.0;
  bool sensor_clear = false;
};
struct BatchPlan {
  std::vector<Segment> segs;
  std::vector<BatchLaunch> launches[2];
  std::vector<vlbm_ctx *> adt_ctx;  // contexts whose link speed is updated every coarse step
  Segment *dseg = nullptr;
};

vlbm_status plan_batch(vlbm_ctx *const *ctxs, const std::vector<int> &act, BatchPlan &bp) {
  vlbm_ctx *c0 = ctxs[act[0]];
  const int r = c0->p.r;
  int D = 0;
  for (int i : act) D = std::max(D, ctxs[i]->nlev);
  std::vector<std::pair<int, int>> ph;
  schedule(0, 1, D, r, ph);
  const size_t P = ph.size();
  // per context and merged phase: its own phase index there (-1: none), and
  // whether that is its fused finest level (taken at the second sub-step)
  std::vector<std::vector<int>> occ(act.size());
  for (size_t a = 0; a < act.size(); ++a) {
    vlbm_ctx *c = ctxs[act[a]];
    std::vector<std::vector<int>> idx(kMaxLevels);
    for (size_t p = 0; p < c->phases.size(); ++p) idx[c->phases[p].first].push_back((int)p);
    std::vector<int> seen(kMaxLevels, 0);
    const bool fz = fused_active(c);
    for (size_t p = 0; p < P; ++p) {
      const int l = ph[p].first;
      int pi = -1;
      if (l < c->nlev) {
        if (fz && l == c->nlev - 1) {
          // the fused launch replaces this level's sub-steps k = 1, 2
          if (ph[p].second == r) pi = idx[l][seen[l]++];
        } else {
          pi = idx[l][seen[l]++];
        }
      }
      occ[a].push_back(pi);
    }
    for (int l = 0; l < c->nlev; ++l)
      if (seen[l] != (int)idx[l].size())
        return fail(VLBM_EINVAL, "internal: batched schedule does not cover context %d", act[a]);
  }
  for (int i : act)
    if (ctxs[i]->adt) bp.adt_ctx.push_back(ctxs[i]);
  for (int e = 0; e < 2; ++e)
    for (size_t p = 0; p < P; ++p)
      for (int fused = 0; fused < 2; ++fused) {
        BatchLaunch L;
        L.seg0 = (int32_t)bp.segs.size();
        int32_t fb = 0;
        bool cfl_emit = false, clear = false;
        for (size_t a = 0; a < act.size(); ++a) {
          vlbm_ctx *c = ctxs[act[a]];
          const int pi = occ[a][p];
          if (pi < 0 || c->phase_blocks[pi] == 0) continue;
          if ((c->phases[pi].second == 0) != (fused == 1)) continue;
          const int ei = table_parity(c) ^ e;
          const size_t Pi = c->phases.size();
          bp.segs.push_back({c->ddesc + ei * Pi + pi, fb, c->phase_blocks[pi]});
          fb += c->phase_blocks[pi];
          const LevelDesc &D0 = c->hdesc[ei * Pi + pi];
          cfl_emit |= c->adt && D0.emit_cfl;
          // a context whose first phase this is, and which also accumulates
          // the next Qmax in it, has its slot cleared first
          clear |= c->sensor && pi == 0 && c->hdesc[ei * Pi].emit_qmax;
        }
        L.nseg = (int32_t)bp.segs.size() - L.seg0;
        if (L.nseg == 0) continue;
        L.nblocks = fb;
        L.first = fused ? 0 : ph[p].second == 1;
        L.ak = ak_of(fused ? 0 : ph[p].second, r);
        L.flags = c0->step_flags | (fused ? STEP_FUSED_PHASE : 0);
        if (fused && (c0->step_flags & STEP_XCD_FUSED)) L.flags |= STEP_XCD_CONTIGUOUS;
        if (c0->adt) L.flags |= STEP_ADAPTIVE_DT | (cfl_emit ? STEP_CFL_EMIT : 0);
        if (c0->sensor && !fused) L.flags |= STEP_SENSOR;
        L.sensor_clear = clear;
        bp.launches[e].push_back(L);
      }
  return VLBM_OK;
}

// The launches of one coarse step of relative parity e.
hipError_t launch_batch_step(const BatchPlan &bp, int e, int fp32, hipStream_t s) {
  hipError_t err = hipSuccess;
  // adaptive time step: every context's link speed for this coarse step, from
  // the bound its previous coarse step's last launches left
  for (vlbm_ctx *c : bp.adt_ctx)
    if (err == hipSuccess) err = launch_cfl_finalize(c->ddyn, c->dcmax, s);
  for (const BatchLaunch &L : bp.launches[e]) {
    if (err != hipSuccess) break;
    StepLaunch a{};
    a.segs = bp.dseg + L.seg0;
    a.nseg = L.nseg;
    a.nblocks = L.nblocks;
    a.first = L.first;
    a.flags = L.flags;
    a.ak = L.ak;
    if (L.sensor_clear) err = launch_sensor(a, 1, fp32, s);
    if (err == hipSuccess) err = launch_step(a, fp32, s);
  }
  return err;
}

// Captured batches: two coarse steps (relative parities 0 and 1) of a fixed
// list of contexts, each at the table version and parity it had at capture.
struct BatchGraph {
  std::vector<long> key;  // per context: pointer, tables_version, table parity
  std::vector<vlbm_ctx *> ctxs;
  vlbm_ctx *owner = nullptr;  // whose memory holds the segment table
  BatchPlan plan;
  hipGraphExec_t exec = nullptr;
  long last_use = 0;
};
std::mutex g_batch_mu;
std::vector<BatchGraph> g_batch_graphs;
long g_batch_clock = 0;
constexpr size_t kBatchGraphs = 16;

void release_batch_graph(BatchGraph &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  if (g.owner) g.owner->mem.release(g.plan.dseg);
  g.plan.dseg = nullptr;
}

// Forget every captured batch that holds c (called before c goes away).
void drop_batch_graphs(vlbm_ctx *c) {
  std::lock_guard<std::mutex> lock(g_batch_mu);
  for (size_t i = 0; i < g_batch_graphs.size();) {
    BatchGraph &g = g_batch_graphs[i];
    if (std::find(g.ctxs.begin(), g.ctxs.end(), c) != g.ctxs.end()) {
      release_batch_graph(g);
      g_batch_graphs.erase(g_batch_graphs.begin() + i);
    } else {
      ++i;
    }
  }
}

std::vector<long> batch_key(vlbm_ctx *const *ctxs, const std::vector<int> &act) {
  std::vector<long> key;
  for (int i : act) {
    key.push_back((long)reinterpret_cast<uintptr_t>(ctxs[i]));
    key.push_back(ctxs[i]->tables_version);
    key.push_back(table_parity(ctxs[i]));
  }
  return key;
}

}  // namespace

extern "C" {

vlbm_status vlbm_batch_advance(vlbm_ctx *const *ctxs, const int *n_steps, int nctx) {
  if (nctx <= 0) return VLBM_OK;
  if (!ctxs || !n_steps) return fail(VLBM_EINVAL, "null argument");
  vlbm_ctx *c0 = ctxs[0];
  for (int i = 0; i < nctx; ++i) {
    vlbm_ctx *c = ctxs[i];
    if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "context %d has no hierarchy", i);
    if (n_steps[i] < 0) return fail(VLBM_EINVAL, "negative step count");
    if (c->stream != c0->stream || c->p.precision != c0->p.precision || c->p.r != c0->p.r)
      return fail(VLBM_EINVAL, "batched contexts must share stream, precision and ratio");
    if ((c->step_flags & ~STEP_F64_MATH) != (c0->step_flags & ~STEP_F64_MATH))
      return fail(VLBM_EINVAL, "batched contexts must share their launch tuning");
    if (c->sensor != c0->sensor)
      return fail(VLBM_EINVAL, "batched contexts must all use the adaptive relaxation, or none");
    if (c->adt != c0->adt)
      return fail(VLBM_EINVAL, "batched contexts must all use the adaptive time step, or none");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return fail(VLBM_EINVAL, "context %d listed twice", i);
  }
  std::vector<long> rem(n_steps, n_steps + nctx);
  for (;;) {
    std::vector<int> act;
    long m = 0;
    for (int i = 0; i < nctx; ++i)
      if (rem[i] > 0) {
        act.push_back(i);
        m = m == 0 ? rem[i] : std::min(m, rem[i]);
      }
    if (act.empty()) break;
    if (act.size() == 1) {
      vlbm_status st = advance_impl(ctxs[act[0]], m);
      if (st) return st;
      rem[act[0]] -= m;
      continue;
    }
    for (int i : act) {  // adaptive relaxation stage 0 and the CFL bound where the state changed
      vlbm_status st = sensor_init(ctxs[i], table_parity(ctxs[i]));
      if (!st) st = cfl_init(ctxs[i], table_parity(ctxs[i]));
      if (st) return st;
    }
    vlbm_ctx *lead = ctxs[act[0]];
    const bool graphs = lead->use_graphs && lead->stream != nullptr && m >= 4;
    long done = 0;
    if (graphs) {
      // replay a captured pair of coarse steps (capturing it the first time)
      std::lock_guard<std::mutex> lock(g_batch_mu);
      const std::vector<long> key = batch_key(ctxs, act);
      BatchGraph *g = nullptr;
      for (BatchGraph &b : g_batch_graphs)
        if (b.key == key) g = &b;
      if (!g) {
        if (g_batch_graphs.size() >= kBatchGraphs) {  // evict the least recently used
          auto it = std::min_element(g_batch_graphs.begin(), g_batch_graphs.end(),
                                     [](const BatchGraph &x, const BatchGraph &y) { return x.last_use < y.last_use; });
          release_batch_graph(*it);
          g_batch_graphs.erase(it);
        }
        BatchGraph nb;
        nb.key = key;
        for (int i : act) nb.ctxs.push_back(ctxs[i]);
        nb.owner = lead;
        vlbm_status st = plan_batch(ctxs, act, nb.plan);
        if (st) return st;
        nb.plan.dseg = static_cast<Segment *>(lead->mem.alloc(sizeof(Segment) * std::max<size_t>(1, nb.plan.segs.size())));
        if (!nb.plan.dseg) return fail(VLBM_ENOMEM, "batch segment table");
        HIPCHK(hipMemcpyAsync(nb.plan.dseg, nb.plan.segs.data(), sizeof(Segment) * nb.plan.segs.size(),
                              hipMemcpyHostToDevice, lead->stream));
        HIPCHK(hipStreamSynchronize(lead->stream));
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(lead->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = launch_batch_step(nb.plan, 0, lead->fp32, lead->stream);
        if (err == hipSuccess) err = launch_batch_step(nb.plan, 1, lead->fp32, lead->stream);
        const hipError_t ec = hipStreamEndCapture(lead->stream, &graph);
        if (err == hipSuccess) err = ec;
        if (err == hipSuccess) err = hipGraphInstantiate(&nb.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (err != hipSuccess) {
          release_batch_graph(nb);
          return fail(VLBM_EDEVICE, "batched graph: %s", hipGetErrorString(err));
        }
        g_batch_graphs.push_back(std::move(nb));
        g = &g_batch_graphs.back();
      }
      g->last_use = ++g_batch_clock;
      for (; done + 2 <= m; done += 2) HIPCHK(hipGraphLaunch(g->exec, lead->stream));
      if (done < m) {  // an odd last coarse step, relative parity 0, eagerly
        HIPCHK(launch_batch_step(g->plan, 0, lead->fp32, lead->stream));
        done += 1;
      }
    } else {
      BatchPlan bp;
      vlbm_status st = plan_batch(ctxs, act, bp);
      if (st) return st;
      bp.dseg = static_cast<Segment *>(lead->mem.alloc(sizeof(Segment) * std::max<size_t>(1, bp.segs.size())));
      if (!bp.dseg) return fail(VLBM_ENOMEM, "batch segment table");
      HIPCHK(hipMemcpyAsync(bp.dseg, bp.segs.data(), sizeof(Segment) * bp.segs.size(), hipMemcpyHostToDevice,
                            lead->stream));
      hipError_t err = hipSuccess;
      for (; done < m && err == hipSuccess; ++done) err = launch_batch_step(bp, (int)(done & 1), lead->fp32, lead->stream);
      if (err == hipSuccess) err = hipStreamSynchronize(lead->stream);
      lead->mem.release(bp.dseg);
      if (err != hipSuccess) return fail(VLBM_EDEVICE, "batched launch: %s", hipGetErrorString(err));
    }
    for (int i : act) {
      count_steps(ctxs[i], m);
      rem[i] -= m;
    }
  }
  return VLBM_OK;
}

vlbm_status vlbm_set_tuning(vlbm_ctx *c, int tile_cells, int flags) {
  return guarded([&]() -> vlbm_status {
    if (!c) return fail(VLBM_EINVAL, "null context");
    if (tile_cells < 64 || tile_cells > (1 << 20) ||
        (flags & ~(STEP_NT_STORES | STEP_TWO_CELLS | STEP_XCD_CONTIGUOUS | STEP_FUSE2 | STEP_XCD_FUSED | STEP_GRAPHS |
                   STEP_SMALL_TILES)))
      return fail(VLBM_EINVAL, "bad tuning (tile_cells %d, flags %d)", tile_cells, flags);
    c->tile_cells = tile_cells;
    c->step_flags = flags | (c->step_flags & STEP_F64_MATH);
    c->use_graphs = (flags & STEP_GRAPHS) != 0;
    if (!c->have_hierarchy) return VLBM_OK;
    // same hierarchy and time history, new tile decomposition
    std::vector<vlbm_box> boxes = c->boxes;
    return regrid_impl(c, boxes.data(), (int)boxes.size());
  });
}

// Tuning cache: one entry per geometry (base grid, ratio, precision, boxes).
static std::map<std::string, std::pair<int, int>> g_tuned;

static std::string tuning_key(const vlbm_ctx *c) {
  std::string k = std::to_string(c->p.nx0) + "x" + std::to_string(c->p.ny0) + "r" +
                  std::to_string(c->p.r) + "p" + std::to_string(c->p.precision) +
                  (c->sensor ? "s" : "") + (c->adt ? "a" : "");
  for (const vlbm_box &b : c->boxes)
    k += ":" + std::to_string(b.level) + "," + std::to_string(b.i0) + "," + std::to_string(b.j0) +
         "," + std::to_string(b.nx) + "," + std::to_string(b.ny);
  return k;
}

namespace {
// One timed autotuning trial: install (tile_cells, flags), advance `warm`
// untimed coarse steps, then time `steps` of them between two events.
vlbm_status time_trial(vlbm_ctx *c, int tile_cells, int flags, int warm, int steps, hipEvent_t e0,
                       hipEvent_t e1, float *ms) {
  vlbm_status st = vlbm_set_tuning(c, tile_cells, flags);
  if (!st) st = advance_impl(c, warm);
  if (!st && hipEventRecord(e0, c->stream) != hipSuccess) st = fail(VLBM_EDEVICE, "event");
  if (!st) st = advance_impl(c, steps);
  if (!st && hipEventRecord(e1, c->stream) != hipSuccess) st = fail(VLBM_EDEVICE, "event");
  if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    st = fail(VLBM_EDEVICE, "event timing");
  return st;
}
}  // namespace

vlbm_status vlbm_autotune(vlbm_ctx *c, int steps_per_trial, int *tile_cells, int *flags) {
  return guarded([&]() -> vlbm_status {
    if (!c || !c->have_hierarchy) return fail(VLBM_ESTATE, "no hierarchy installed");
    if (steps_per_trial < 1) return fail(VLBM_EINVAL, "steps_per_trial < 1");
    const std::string key = tuning_key(c);
    auto hit = g_tuned.find(key);
    vlbm_status st;
    if (hit == g_tuned.end()) {
      const int tiles[] = {128, 256, 512, 1024};
      const bool can_fuse = c->p.r == 2 && c->nlev >= 2 && !c->sensor;
      // workgroup order x store kind (x fused sub-steps where they apply)
      std::vector<int> orders;
      for (int fuse : {0, (int)STEP_FUSE2})
        for (int nt : {0, (int)STEP_NT_STORES})
          for (int xcd : {0, (int)STEP_XCD_CONTIGUOUS})
            if (!fuse || can_fuse) orders.push_back(fuse | nt | xcd);
      const int norders = (int)orders.size();
      float best = 1e30f;
      std::pair<int, int> choice{c->tile_cells, c->step_flags};
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      for (int tcell : tiles)
        for (int oi = 0; oi < norders; ++oi) {
          const int ord = orders[oi];
          const int fl = (c->step_flags & ~(STEP_XCD_CONTIGUOUS | STEP_FUSE2 | STEP_NT_STORES | STEP_F64_MATH |
                                            STEP_GRAPHS | STEP_SMALL_TILES)) | ord;
          float ms = 0.f;
          st = time_trial(c, tcell, fl, 1, steps_per_trial, e0, e1, &ms);
          if (st) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return st;
          }
          if (ms < best) {
            best = ms;
            choice = {tcell, fl};
          }
        }
      // smaller tiles on levels with few tiles (STEP_SMALL_TILES), kept only
      // if it saves more than 1%
      if (!c->sensor) {
        float base = 0.f, small = 0.f;
        st = time_trial(c, choice.first, choice.second, 1, steps_per_trial, e0, e1, &base);
        if (!st) st = time_trial(c, choice.first, choice.second | STEP_SMALL_TILES, 1, steps_per_trial, e0, e1, &small);
        if (st) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return st;
        }
        if (small < 0.99f * base) choice.second |= STEP_SMALL_TILES;
      }
      // graph replay of the chosen launches (an even number of steps, at least
      // four, so that every step of the trial is replayed) where the context has
      // a stream of its own; kept only if it saves more than 2%
      if (c->stream != nullptr && !c->prof) {
        const int gsteps = std::max(4, (steps_per_trial + 1) & ~1);
        float plain = 0.f, graphed = 0.f;
        st = time_trial(c, choice.first, choice.second, 2, gsteps, e0, e1, &plain);
        if (!st) st = time_trial(c, choice.first, choice.second | STEP_GRAPHS, 4, gsteps, e0, e1, &graphed);
        if (st) {
          (void)hipEventDestroy(e0);
          (void)hipEventDestroy(e1);
          return st;
        }
        if (graphed < 0.98f * plain) choice.second |= STEP_GRAPHS;
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      hit = g_tuned.emplace(key, choice).first;
    }
    st = vlbm_set_tuning(c, hit->second.first, hit->second.second);
    if (st) return st;
    if (tile_cells) *tile_cells = c->tile_cells;
    if (flags) *flags = c->step_flags & ~STEP_F64_MATH;
    return VLBM_OK;
  });
}

vlbm_status vlbm_set_sensor(vlbm_ctx *c, int on, double c_sensor, double beta_min, double beta_max) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  if (on && !(beta_min > 0.0 && beta_min <= beta_max && beta_max <= 1.0 && c_sensor >= 0.0))
    return fail(VLBM_EINVAL, "adaptive relaxation needs 0 < beta_min <= beta_max <= 1 and C >= 0");
  const bool was = c->sensor;
  c->sensor = on != 0;
  if (c->sensor) {
    c->c_sensor = c_sensor;
    c->beta_min = beta_min;
    c->beta_max = beta_max;
  }
  if (!c->have_hierarchy) return VLBM_OK;
  if (was != c->sensor) {
    // the step tiles change shape (SEN_TW x SEN_TH with the sensor): same
    // hierarchy and time history, new lists
    std::vector<vlbm_box> boxes = c->boxes;
    return regrid_impl(c, boxes.data(), (int)boxes.size());
  }
  // same buffers and time history; descriptors, planes and fusion follow the setting
  return build_tables(c);
}

vlbm_status vlbm_set_time_stepping(vlbm_ctx *c, int on, double kappa) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  if (on && !(kappa > 0.0)) return fail(VLBM_EINVAL, "adaptive time step needs kappa > 0");
  if (on && c->eos.kind != VLBM_EOS_IDEAL) return fail(VLBM_EINVAL, "adaptive time step: ideal gas only");
  HIPCHK(hipStreamSynchronize(c->stream));
  c->adt = on != 0;
  c->cfl_stale = true;
  if (c->adt) {
    if (!c->ddyn) c->ddyn = static_cast<double *>(c->mem.alloc(sizeof(double) * DYN_SLOTS));
    if (!c->dcmax) c->dcmax = static_cast<unsigned long long *>(c->mem.alloc(sizeof(unsigned long long)));
    if (!c->ddyn || !c->dcmax) return fail(VLBM_ENOMEM, "adaptive time step scalars");
    double dyn[DYN_SLOTS] = {};
    dyn[DYN_C] = c->p.c;
    dyn[DYN_H] = c->h;
    dyn[DYN_C_PREV] = c->p.c;
    dyn[DYN_TIME] = (double)c->coarse_steps * (c->p.dx0 / c->p.c);
    dyn[DYN_GAMMA] = c->p.gamma;
    dyn[DYN_KD] = kappa * 2.0;
    dyn[DYN_DX0] = c->p.dx0;
    const unsigned long long zero = 0;
    HIPCHK(hipMemcpyAsync(c->ddyn, dyn, sizeof dyn, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->dcmax, &zero, sizeof zero, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  if (!c->have_hierarchy) return VLBM_OK;
  return build_tables(c);
}

vlbm_status vlbm_time(vlbm_ctx *c, double *time, double *link_speed) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  double t = (double)c->coarse_steps * (c->p.dx0 / c->p.c), cs = c->p.c;
  if (c->adt) {
    double dyn[DYN_SLOTS];
    HIPCHK(hipMemcpyAsync(dyn, c->ddyn, sizeof dyn, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    t = dyn[DYN_TIME];
    cs = dyn[DYN_C];
  }
  if (time) *time = t;
  if (link_speed) *link_speed = cs;
  return VLBM_OK;
}

vlbm_status vlbm_get_beta(vlbm_ctx *c, int level, int i0, int j0, int nx, int ny, double *beta,
                          long ld) {
  if (!beta) return fail(VLBM_EINVAL, "null beta");
  vlbm_status st = check_rect(c, level, i0, j0, nx, ny);
  if (st) return st;
  if (ld < nx) return fail(VLBM_EINVAL, "ld < nx");
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) beta[(size_t)y * ld + x] = NAN;
  const Level &L = c->lv[level];
  if (!L.present || !L.dsen) return VLBM_OK;
  int ci0 = i0, cj0 = j0, cnx = nx, cny = ny, ox = 0, oy = 0;
  if (!clip_to_frame(L, ci0, cj0, cnx, cny, ox, oy)) return VLBM_OK;
  std::vector<double> rows((size_t)cnx * cny);
  for (int y = 0; y < cny;) {  // runs of stored rows
    if (!L.stored(cj0 + y)) {
      ++y;
      continue;
    }
    int y1 = y + 1;
    while (y1 < cny && L.stored(cj0 + y1)) ++y1;
    HIPCHK(hipMemcpy2DAsync(rows.data() + (size_t)y * cnx, sizeof(double) * cnx,
                            L.dsen + SEN_BETA * L.plane + L.off(ci0, cj0 + y), sizeof(double) * L.pitch,
                            sizeof(double) * cnx, y1 - y, hipMemcpyDeviceToHost, c->stream));
    y = y1;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  for (int y = 0; y < cny; ++y)
    for (int x = 0; x < cnx; ++x)
      if (L.stored(cj0 + y) && L.status[L.fidx(ci0 + x, cj0 + y)] == 1)
        beta[(size_t)(y + oy) * ld + x + ox] = rows[(size_t)y * cnx + x];
  return VLBM_OK;
}

vlbm_status vlbm_set_profiling(vlbm_ctx *c, int enable) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  vlbm_status st = prof_flush(c);
  if (st) return st;
  c->prof = enable != 0;
  if (c->prof)
    for (int i = 0; i < 2 * kMaxLevels; ++i) {
      c->prof_ms[i] = 0.0;
      c->prof_calls[i] = 0;
      c->prof_cells[i] = 0.0;
    }
  return VLBM_OK;
}

vlbm_status vlbm_kernel_times(vlbm_ctx *c, double *ms, long *calls, double *cells) {
  if (!c || !ms || !calls || !cells) return fail(VLBM_EINVAL, "null argument");
  vlbm_status st = prof_flush(c);
  if (st) return st;
  for (int i = 0; i < 2 * kMaxLevels; ++i) {
    ms[i] = c->prof_ms[i];
    calls[i] = c->prof_calls[i];
    cells[i] = c->prof_cells[i];
  }
  return VLBM_OK;
}

long vlbm_steps(const vlbm_ctx *c) { return c ? c->coarse_steps : -1; }

long vlbm_active_cells(const vlbm_ctx *c, int level) {
  if (!c || !c->have_hierarchy || level < 0 || level >= kMaxLevels || !c->lv[level].present) return 0;
  long n = 0;
  for (const Tile &t : c->lv[level].tiles) n += (long)t.w * t.h;
  return n;
}

vlbm_status vlbm_sync(vlbm_ctx *c) {
  if (!c) return fail(VLBM_EINVAL, "null context");
  HIPCHK(hipStreamSynchronize(c->stream));
  return VLBM_OK;
}

}  // extern "C"
