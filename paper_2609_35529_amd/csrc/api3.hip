// Host side of the three-dimensional (D3Q6) path of libvlbm: level frames,
// tile and task lists, the recursive sub-cycle schedule and the C ABI declared
// in include/vlbm3.h.
//
// Schedule (paper Sec. 3.2, Fig. 1): one coarse step of level l runs r steps
// of level l+1, each recursively running level l+2, then advances level l.
// Every level step is one launch of step3_kernel. Its workgroups fill the
// ghost slots their own cells read: periodic images, boundary values, the
// hand-off from the parent's two stored time levels (one tangential slope per
// tangential axis) and the reflux average of the finer level's face values.
// They also add this sub-step's outgoing face values into the parent's reflux
// accumulators, then stream and relax their cells.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/vlbm3.h"
#include "host_util.hpp"
#include "vlbm3_internal.hpp"

namespace vlbm {
void set_error_message(const char *msg);
}

using namespace vlbm3;
using vlbm_host::PhaseTimer;

namespace {

vlbm_status fail3(vlbm_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  vlbm::set_error_message(buf);
  return st;
}

// An entry point's body that runs host sections on the worker pool: an
// exception (host memory exhausted) becomes a status, not a throw across the
// C ABI.
template <class F>
vlbm_status guard3(F &&f) {
  try {
    return f();
  } catch (const std::bad_alloc &) {
    return fail3(VLBM_ENOMEM, "host memory exhausted");
  } catch (...) {
    return fail3(VLBM_EINVAL, "internal error in a host section");
  }
}

#define HIPCHK3(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail3(VLBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

// ptr := n bytes of the context's device memory, or VLBM_ENOMEM.
#define ALLOC3(ptr, n)                                                                       \
  do {                                                                                       \
    const size_t n_ = (n);                                                                   \
    (ptr) = static_cast<std::remove_reference_t<decltype(ptr)>>(c->mem.alloc(n_));           \
    if (!(ptr)) return fail3(VLBM_ENOMEM, "device memory (%zu bytes)", n_);                  \
  } while (0)

constexpr int kL = VLBM3_MAX_LEVELS;
const int E3[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

// An allocator whose resize leaves new elements uninitialised: the frame-sized
// host arrays (hundreds of MB on a large level) are then written once, by
// their builders, in parallel.
template <class T>
struct NoInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInit<U>;
  };
  NoInit() = default;
  template <class U>
  NoInit(const NoInit<U> &) noexcept {}
  template <class U>
  void construct(U *q) noexcept {
    ::new (static_cast<void *>(q)) U;
  }
  template <class U, class... A>
  void construct(U *q, A &&...a) {
    ::new (static_cast<void *>(q)) U(std::forward<A>(a)...);
  }
};
using Bytes = std::vector<uint8_t, NoInit<uint8_t>>;

struct Level3 {
  bool present = false;
  int N[3] = {0, 0, 0};
  double dx = 0.0;
  int f0[3] = {0, 0, 0}, fn[3] = {0, 0, 0};  // frame origin and extent (bbox + ghost layer)
  int pitch = 0, xoff = 0;
  int esz = 8;  // bytes per stored element
  int64_t slab = 0, plane = 0;
  void *buf[2] = {nullptr, nullptr};
  Bytes cov;     // per frame cell: covered at this level
  Bytes status;  // 0 none, 1 active, 2 hole
  uint8_t *dstatus = nullptr;
  std::vector<Tile3> tiles;
  std::vector<Task3> tasks;
  Tile3 *dtiles = nullptr;
  Task3 *dtasks = nullptr;
  double *dacc = nullptr;
  int nacc = 0;
  double *dledger = nullptr;
  int nledger = 0;
  double *dpartial = nullptr;
  long steps = 0;
  // interfaces towards the finer level, sorted: (linear index of the ring
  // cell in the level domain) * 6 + the population it hands into the hole
  std::vector<int64_t> face_key;

  bool in_frame(const int p[3]) const {
    for (int a = 0; a < 3; ++a)
      if (p[a] < f0[a] || p[a] >= f0[a] + fn[a]) return false;
    return true;
  }
  size_t fidx(const int p[3]) const {
    return ((size_t)(p[2] - f0[2]) * fn[1] + (p[1] - f0[1])) * fn[0] + (p[0] - f0[0]);
  }
  int64_t off(const int p[3]) const {
    return ((int64_t)(p[2] - f0[2]) * fn[1] + (p[1] - f0[1])) * pitch + (p[0] - f0[0]) + xoff;
  }
  int64_t stride(int a) const { return a == 0 ? 1 : a == 1 ? (int64_t)pitch : slab; }
  int cur() const { return (int)(steps & 1); }
};

// Device memory of a context: from the caller's allocator after
// vlbm3_bind_allocator, else hipMalloc. Blocks are 256-byte aligned.
struct Alloc3 {
  vlbm_alloc_fn a = nullptr;
  vlbm_free_fn f = nullptr;
  void *user = nullptr;
  void *alloc(size_t n) {
    n = (std::max<size_t>(n, 256) + 255) & ~size_t(255);
    if (a) {
      void *q = a(n, user);
      if (q && (reinterpret_cast<uintptr_t>(q) & 255)) {
        f(q, user);
        return nullptr;
      }
      return q;
    }
    void *q = nullptr;
    return hipMalloc(&q, n) == hipSuccess ? q : nullptr;
  }
  void release(void *q) {
    if (!q) return;
    if (f)
      f(q, user);
    else
      (void)hipFree(q);
  }
};

void dfree(Alloc3 &m, void *&p) {
  m.release(p);
  p = nullptr;
}
template <class T>
void dfree(Alloc3 &m, T *&p) {
  void *v = p;
  dfree(m, v);
  p = nullptr;
}

// f(lo, hi) over up to 16 contiguous ranges of [0, n), on the process's
// worker pool and the calling thread; ranges hold at least `grain` items.
template <class F>
void par_ranges(size_t n, size_t grain, const F &f) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const int nw = (int)std::max<size_t>(1, std::min<size_t>({16, hw, (n + grain - 1) / std::max<size_t>(1, grain)}));
  vlbm_host::Pool::get().run(nw, [&](int w) { f(n * w / nw, n * (w + 1) / nw); });
}

// Items of f(i, out) for i in [0, n), each appending to `out`, computed on
// the worker pool in contiguous ranges and concatenated in order of i.
template <class T, class F>
std::vector<T> par_collect(size_t n, const F &f) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const int nw = (int)std::max<size_t>(1, std::min<size_t>({16, hw, n}));
  std::vector<std::vector<T>> part(nw);
  vlbm_host::Pool::get().run(nw, [&](int w) {
    for (size_t i = n * w / nw; i < n * (w + 1) / nw; ++i) f(i, part[w]);
  });
  std::vector<T> out;
  size_t total = 0;
  for (const auto &v : part) total += v.size();
  out.reserve(total);
  for (const auto &v : part) out.insert(out.end(), v.begin(), v.end());
  return out;
}

}  // namespace

struct vlbm3_ctx {
  vlbm3_params p{};
  hipStream_t stream = nullptr;
  Level3 lv[kL];
  int nlev = 1;
  bool have_hierarchy = false;
  long coarse_steps = 0;
  // measured on MI355X (256^3 blast): with non-temporal stores, FP64 runs the
  // step at 0.57 of HBM peak with 512-cell tiles (0.50 at 256, 0.23 at 64),
  // the FP32 forms at 0.58-0.62 with 1024-cell tiles (0.48-0.54 at 512)
  int tile_cells = 512;
  int flags = S3_NT_STORES;
  int fp32 = 0;    // float storage
  int sflags = 0;  // S3_FP32 | S3_F64_MATH of the precision
  double gm1 = 0, h = 0, tb = 0;
  std::vector<vlbm3_box> boxes;
  std::vector<std::pair<int, int>> phases;  // (level, k)
  long flips[kL] = {};
  Desc3 *ddesc = nullptr;
  long table_base = 0;
  Alloc3 mem;
  bool prof = false;
  std::vector<hipEvent_t> pev;
  std::vector<std::pair<int, double>> pend;
  double prof_ms[kL] = {}, prof_cells[kL] = {};
  long prof_calls[kL] = {};
  // pinned host buffer for reading the ledger slots back (grown on demand)
  double *pin = nullptr;
  size_t pin_cap = 0;  // doubles
  double *pinned(size_t n) {
    if (n > pin_cap) {
      if (pin) (void)hipHostFree(pin);
      pin = nullptr;
      pin_cap = 0;
      void *h = nullptr;
      if (hipHostMalloc(&h, sizeof(double) * n, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      pin = static_cast<double *>(h);
      pin_cap = n;
    }
    return pin;
  }

  bool periodic(int a) const { return p.bc[2 * a] == VLBM_BC_PERIODIC; }
  // wrap p (level l) by the periodic axes; false if outside a non-periodic side
  bool wrap(int l, int q[3]) const {
    for (int a = 0; a < 3; ++a) {
      const int n = lv[l].N[a];
      if (q[a] < 0 || q[a] >= n) {
        if (!periodic(a)) return false;
        q[a] = ((q[a] % n) + n) % n;
      }
    }
    return true;
  }
  // q: in-domain coordinates of level l
  bool covered(int l, const int q[3]) const {
    if (l >= nlev || !lv[l].present) return false;
    const Level3 &L = lv[l];
    if (!L.in_frame(q)) return false;
    return L.cov[L.fidx(q)] != 0;
  }
  bool active(int l, const int q[3]) const {
    if (!covered(l, q)) return false;
    const int r = p.r;
    const int c[3] = {q[0] * r, q[1] * r, q[2] * r};
    return !covered(l + 1, c);
  }
};

namespace {

void free_level3(Alloc3 &m, Level3 &L) {
  dfree(m, L.buf[0]);
  dfree(m, L.buf[1]);
  dfree(m, L.dstatus);
  dfree(m, L.dtiles);
  dfree(m, L.dtasks);
  dfree(m, L.dacc);
  dfree(m, L.dledger);
  dfree(m, L.dpartial);
  L = Level3();
}

void free_lists3(Alloc3 &m, Level3 &L) {
  dfree(m, L.dtiles);
  dfree(m, L.dtasks);
  dfree(m, L.dacc);
  dfree(m, L.dledger);
  dfree(m, L.dpartial);
}

vlbm_status check_params3(const vlbm3_params &p) {
  if (p.nx0 < 1 || p.ny0 < 1 || p.nz0 < 1 || !(p.dx0 > 0) || p.r < 1 || p.r > 8 || p.max_levels < 1 ||
      p.max_levels > kL || !(p.c > 0) || !(p.gamma > 1) || p.beta < 0 || p.beta > 1 ||
      (p.precision != VLBM_FP64 && p.precision != VLBM_FP32 && p.precision != VLBM_FP32_STORAGE))
    return fail3(VLBM_EINVAL, "bad parameters");
  for (int a = 0; a < 3; ++a) {
    const int b0 = p.bc[2 * a], b1 = p.bc[2 * a + 1];
    if (b0 < 0 || b0 > 2 || b1 < 0 || b1 > 2) return fail3(VLBM_EINVAL, "bad boundary kind (3-D: periodic, outflow, reflect)");
    if ((b0 == VLBM_BC_PERIODIC) != (b1 == VLBM_BC_PERIODIC))
      return fail3(VLBM_EINVAL, "periodic sides must come in pairs");
  }
  return VLBM_OK;
}

struct Geom3 {
  bool present[kL] = {};
  int lo[kL][3], hi[kL][3];
  int nlev = 1;
};

vlbm_status check_boxes3(const vlbm3_params &p, const vlbm3_box *boxes, int n, Geom3 &g) {
  if (n < 0 || (n > 0 && !boxes)) return fail3(VLBM_EINVAL, "bad box list");
  for (int l = 0; l < kL; ++l)
    for (int a = 0; a < 3; ++a) {
      g.lo[l][a] = 1 << 30;
      g.hi[l][a] = -(1 << 30);
    }
  g.present[0] = true;
  const int n0[3] = {p.nx0, p.ny0, p.nz0};
  for (int a = 0; a < 3; ++a) {
    g.lo[0][a] = 0;
    g.hi[0][a] = n0[a];
  }
  g.nlev = 1;
  for (int b = 0; b < n; ++b) {
    const vlbm3_box &B = boxes[b];
    if (B.level < 1 || B.level >= p.max_levels)
      return fail3(VLBM_EINVAL, "box %d: level %d outside 1..%d", b, B.level, p.max_levels - 1);
    long s = 1;
    for (int i = 0; i < B.level; ++i) s *= p.r;
    const int lo[3] = {B.i0, B.j0, B.k0}, ext[3] = {B.nx, B.ny, B.nz};
    for (int a = 0; a < 3; ++a) {
      if (ext[a] <= 0 || lo[a] < 0 || lo[a] + (long)ext[a] > n0[a] * s)
        return fail3(VLBM_EINVAL, "box %d lies outside its level's domain", b);
      if (lo[a] % p.r || ext[a] % p.r)
        return fail3(VLBM_ENEST, "box %d is not made of whole parent cells (ratio %d)", b, p.r);
    }
    const int l = B.level;
    g.present[l] = true;
    g.nlev = std::max(g.nlev, l + 1);
    for (int a = 0; a < 3; ++a) {
      g.lo[l][a] = std::min(g.lo[l][a], lo[a]);
      g.hi[l][a] = std::max(g.hi[l][a], lo[a] + ext[a]);
    }
  }
  for (int l = 1; l < kL; ++l)
    if (g.present[l] && !g.present[l - 1])
      return fail3(VLBM_ENEST, "level %d has boxes but level %d has none", l, l - 1);
  return VLBM_OK;
}

void frame3(const vlbm3_params &p, const Geom3 &g, int l, Level3 &L) {
  long s = 1;
  for (int i = 0; i < l; ++i) s *= p.r;
  const int n0[3] = {p.nx0, p.ny0, p.nz0};
  for (int a = 0; a < 3; ++a) L.N[a] = (int)(n0[a] * s);
  L.dx = p.dx0 / (double)s;
  L.present = g.present[l];
  if (!L.present) return;
  for (int a = 0; a < 3; ++a) {
    L.f0[a] = g.lo[l][a] - 1;
    L.fn[a] = g.hi[l][a] - g.lo[l][a] + 2;
  }
  // first interior column on a 128-byte line; rows padded to 64 elements;
  // planes to a multiple of 4 KiB
  L.esz = p.precision == VLBM_FP64 ? 8 : 4;
  L.xoff = 128 / L.esz - 1;
  L.pitch = (L.fn[0] + L.xoff + 63) / 64 * 64;
  L.slab = (int64_t)L.pitch * L.fn[1];
  const int64_t pa = 4096 / L.esz;
  L.plane = (L.slab * L.fn[2] + pa - 1) / pa * pa;
}

size_t level_bytes3(const Level3 &L) { return (size_t)L.plane * 30 * L.esz; }

// What fills the slot from which active cell x of level l pulls population q
// (returns false: an active cell of the same level, read in place).
vlbm_status ghost_task3(const vlbm3_ctx *c, int l, const int x[3], int q, Task3 &t, bool &needed) {
  const Level3 &L = c->lv[l];
  const int r = c->p.r;
  int s[3] = {x[0] - E3[q][0], x[1] - E3[q][1], x[2] - E3[q][2]};
  int w[3] = {s[0], s[1], s[2]};
  t = Task3{};
  t.q = q;
  t.n[0] = t.n[1] = t.n[2] = t.n[3] = -1;
  if (!L.in_frame(s)) return fail3(VLBM_ENEST, "internal: ghost slot outside the frame");
  t.dst = (int32_t)L.off(s);
  needed = true;
  if (!c->wrap(l, w)) {
    const int side = q;  // +alpha enters through the -alpha side, -alpha through +alpha
    t.kind = (c->p.bc[side] == VLBM_BC_OUTFLOW ? K3_OUTFLOW : K3_REFLECT) | K3_LEDGER;
    t.src = (int32_t)L.off(x);
    return VLBM_OK;
  }
  const int wc[3] = {w[0] * r, w[1] * r, w[2] * r};
  if (c->covered(l + 1, wc)) {
    t.kind = K3_REFLUX;
    return VLBM_OK;
  }
  if (c->covered(l, w)) {
    if (w[0] == s[0] && w[1] == s[1] && w[2] == s[2]) {
      needed = false;
      return VLBM_OK;
    }
    t.kind = K3_COPY;
    t.src = (int32_t)L.off(w);
    return VLBM_OK;
  }
  if (l == 0) return fail3(VLBM_ENEST, "internal: level-0 cell without a source");
  const Level3 &PL = c->lv[l - 1];
  int P[3] = {w[0] / r, w[1] / r, w[2] / r};
  if (!c->active(l - 1, P)) return fail3(VLBM_ENEST, "level %d: parent ring cell inactive", l);
  t.kind = K3_RECON;
  t.src = (int32_t)PL.off(P);
  const int n = q / 2;
  int ti = 0;
  for (int a = 0; a < 3; ++a) {
    if (a == n) continue;
    int m[3] = {P[0], P[1], P[2]}, pp[3] = {P[0], P[1], P[2]};
    m[a] -= 1;
    pp[a] += 1;
    const bool have = c->wrap(l - 1, m) && c->wrap(l - 1, pp) && c->active(l - 1, m) && c->active(l - 1, pp);
    if (have) {
      t.n[2 * ti] = (int32_t)PL.off(m);
      t.n[2 * ti + 1] = (int32_t)PL.off(pp);
    }
    const int j = x[a] - r * P[a];
    if (ti == 0)
      t.j1 = j;
    else
      t.j2 = j;
    ++ti;
  }
  return VLBM_OK;
}

// Cell -> tile of one level: per frame row (z, y), the tiles crossing it as
// frame-column ranges [x0, x1), ordered by x0.
struct TileRows3 {
  struct Ent {
    int32_t x0, x1, tile;
  };
  std::vector<int32_t> row0;  // row i holds ent[row0[i] .. row0[i + 1])
  std::vector<Ent> ent;
  int32_t tile_of(const Level3 &L, const int p[3]) const {  // p: an active cell
    const size_t row = (size_t)(p[2] - L.f0[2]) * L.fn[1] + (p[1] - L.f0[1]);
    const int fx = p[0] - L.f0[0];
    const Ent *b = ent.data() + row0[row], *e = ent.data() + row0[row + 1];
    const Ent *it = std::upper_bound(b, e, fx, [](int v, const Ent &o) { return v < o.x0; });
    return (it != b && fx < (it - 1)->x1) ? (it - 1)->tile : -1;
  }
};

// Frame position (fx, fy, fz) of a tile's first cell.
void tile_origin3(const Level3 &L, const Tile3 &T, int f[3]) {
  const int64_t rel = T.off0 - L.xoff;
  f[2] = (int)(rel / L.slab);
  f[1] = (int)((rel - (int64_t)f[2] * L.slab) / L.pitch);
  f[0] = (int)(rel - (int64_t)f[2] * L.slab - (int64_t)f[1] * L.pitch);
}

// Tiles of the z-slabs [za, zb) of level l into `tiles`: runs of active cells
// along x (cut at tc cells), equal runs on consecutive rows stacked while the
// tile holds at most tc cells.
void build_tile_slabs3(vlbm3_ctx *c, int l, int za, int zb, int tc, std::vector<Tile3> &tiles) {
  Level3 &L = c->lv[l];
  struct Open {
    int xa, w, ti;  // run start (frame column), width, tile growing on the previous row
  };
  std::vector<Open> open, next;  // ordered by xa (the runs of a row are disjoint)
  const int xe = L.fn[0] - 1;
  for (int z = za; z < zb; ++z) {
    open.clear();
    for (int y = L.f0[1] + 1; y < L.f0[1] + L.fn[1] - 1; ++y) {
      next.clear();
      const int p0[3] = {L.f0[0], y, z};
      const uint8_t *row = &L.status[L.fidx(p0)];
      size_t j = 0;
      for (int x = 1; x < xe;) {
        if (row[x] != 1) {  // to the next active cell
          const void *nx = memchr(row + x, 1, xe - x);
          if (!nx) break;
          x = (int)(static_cast<const uint8_t *>(nx) - row);
        }
        const int xa = x;
        while (x < xe && x - xa < tc && row[x] == 1) ++x;
        const int w = x - xa;
        while (j < open.size() && open[j].xa < xa) ++j;
        int ti;
        if (j < open.size() && open[j].xa == xa && open[j].w == w && (tiles[open[j].ti].h + 1) * w <= tc) {
          ti = open[j].ti;
          tiles[ti].h += 1;
        } else {
          Tile3 t{};
          const int q0[3] = {L.f0[0] + xa, y, z};
          t.off0 = (int32_t)L.off(q0);
          t.w = w;
          t.h = 1;
          tiles.push_back(t);
          ti = (int)tiles.size() - 1;
        }
        next.push_back({xa, w, ti});
      }
      open.swap(next);
    }
  }
}

void build_tiles3(vlbm3_ctx *c, int l, TileRows3 &own) {
  Level3 &L = c->lv[l];
  L.tiles.clear();
  const int tc = c->tile_cells;
  // z-slabs are independent: ranges of them on worker threads, each with its
  // own tile list, then concatenated in z order
  const int nz = std::max(0, L.fn[2] - 2);
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const int nw = (int)std::max<size_t>(1, std::min<size_t>({16, hw, (size_t)std::max(nz, 1)}));
  std::vector<std::vector<Tile3>> part(nw);
  vlbm_host::Pool::get().run(nw, [&](int w) {
    build_tile_slabs3(c, l, L.f0[2] + 1 + (int)((size_t)nz * w / nw), L.f0[2] + 1 + (int)((size_t)nz * (w + 1) / nw),
                      tc, part[w]);
  });
  for (const auto &v : part) L.tiles.insert(L.tiles.end(), v.begin(), v.end());
  // the tiles crossing each frame row
  const size_t nrows = (size_t)L.fn[1] * L.fn[2];
  own.row0.assign(nrows + 1, 0);
  for (const Tile3 &T : L.tiles) {
    int f[3];
    tile_origin3(L, T, f);
    for (int cy = 0; cy < T.h; ++cy) own.row0[(size_t)f[2] * L.fn[1] + f[1] + cy + 1] += 1;
  }
  for (size_t i = 0; i < nrows; ++i) own.row0[i + 1] += own.row0[i];
  own.ent.resize(own.row0[nrows]);
  std::vector<int32_t> at(own.row0.begin(), own.row0.end() - 1);
  for (size_t ti = 0; ti < L.tiles.size(); ++ti) {
    const Tile3 &T = L.tiles[ti];
    int f[3];
    tile_origin3(L, T, f);
    for (int cy = 0; cy < T.h; ++cy)
      own.ent[at[(size_t)f[2] * L.fn[1] + f[1] + cy]++] = {f[0], f[0] + T.w, (int32_t)ti};
  }
  // a row's entries come in tile order (tiles that started on earlier rows
  // first): ordered by x0 row by row
  par_ranges(nrows, 4096, [&](size_t i0, size_t i1) {
    for (size_t i = i0; i < i1; ++i)
      if (own.row0[i + 1] - own.row0[i] > 1)
        std::sort(own.ent.begin() + own.row0[i], own.ent.begin() + own.row0[i + 1],
                  [](const TileRows3::Ent &a, const TileRows3::Ent &b) { return a.x0 < b.x0; });
  });
}

struct RefluxKey3 {
  int hole[3];  // hole cell H of level l (wrapped, in-domain)
  int q;
  int slot;
};

// Tiles, tasks, accumulator and ledger slots of every level (coarse to fine:
// a level's reflux slots define the captures of the next finer level).
vlbm_status build_lists3(vlbm3_ctx *c) {
  std::vector<RefluxKey3> caps_from_parent;
  const int r = c->p.r;
  for (int l = 0; l < c->nlev; ++l) {
    PhaseTimer lt(l == 0 ? "lists3 l0" : l == 1 ? "lists3 l1" : l == 2 ? "lists3 l2" : "lists3 l3+");
    Level3 &L = c->lv[l];
    TileRows3 own;
    build_tiles3(c, l, own);
    lt.mark("tiles");
    std::vector<std::vector<Task3>> per(L.tiles.size());
    std::vector<RefluxKey3> refl;
    L.nacc = 0;
    L.nledger = 0;
    // Ghost tasks of the tiles, on worker threads over contiguous tile ranges:
    // a tile's reflux and ledger slots are numbered locally first, then
    // renumbered in tile order below, so the lists do not depend on the
    // threading.
    std::vector<std::vector<RefluxKey3>> trefl(L.tiles.size());
    std::vector<int> tled(L.tiles.size(), 0);
    auto tile_tasks = [&](size_t ti) -> vlbm_status {
      const Tile3 &T = L.tiles[ti];
      int nacc = 0, nled = 0;
      // tile cells: decode the first cell's coordinates once
      const int64_t rel = T.off0 - L.xoff;
      const int fz = (int)(rel / L.slab);
      const int fy = (int)((rel - (int64_t)fz * L.slab) / L.pitch);
      const int fx = (int)(rel - (int64_t)fz * L.slab - (int64_t)fy * L.pitch);
      // Status offsets of the six upwind neighbours (an active cell's
      // neighbours all lie in the frame, whose ghost layer surrounds them).
      const int64_t sy = L.fn[0], sz = (int64_t)L.fn[0] * L.fn[1];
      const int64_t up[6] = {-1, 1, -sy, sy, -sz, sz};  // cell - e_q
      constexpr uint64_t ones = 0x0101010101010101ull;
      auto all8 = [](const uint8_t *p) {
        uint64_t v;
        memcpy(&v, p, 8);
        return v == ones;
      };
      for (int cy = 0; cy < T.h; ++cy) {
        const uint8_t *st = &L.status[((size_t)fz * L.fn[1] + fy + cy) * L.fn[0] + fx];
        for (int cx = 0; cx < T.w;) {
          // eight interior cells at once: cells cx - 1 .. cx + 8 of the row and
          // cx .. cx + 7 of the four rows around it active
          if (cx + 8 <= T.w && fx + cx + 8 < L.fn[0] && all8(st + cx - 1) && all8(st + cx + 1) &&
              all8(st + cx - sy) && all8(st + cx + sy) && all8(st + cx - sz) && all8(st + cx + sz)) {
            cx += 8;
            continue;
          }
          const uint8_t *sc = st + cx;
          ++cx;
          if (sc[-1] == 1 && sc[1] == 1 && sc[-sy] == 1 && sc[sy] == 1 && sc[-sz] == 1 && sc[sz] == 1) continue;
          const int x[3] = {L.f0[0] + fx + cx - 1, L.f0[1] + fy + cy, L.f0[2] + fz};
          for (int q = 0; q < 6; ++q) {
            if (sc[up[q]] == 1) continue;  // an active cell of this level, read in place
            Task3 t;
            bool needed = false;
            vlbm_status st = ghost_task3(c, l, x, q, t, needed);
            if (st) return st;
            if (!needed) continue;
            const int kind = t.kind & 0xFF;
            if (kind == K3_REFLUX) {
              t.slot = nacc++;
              int w[3] = {x[0] - E3[q][0], x[1] - E3[q][1], x[2] - E3[q][2]};
              c->wrap(l, w);
              trefl[ti].push_back({{w[0], w[1], w[2]}, q, t.slot});
            } else if (kind == K3_OUTFLOW || kind == K3_REFLECT) {
              t.slot = nled++;
            }
            per[ti].push_back(t);
          }
        }
      }
      tled[ti] = nled;
      return VLBM_OK;
    };
    {
      const size_t nt = L.tiles.size();
      const int nw = (int)std::max<size_t>(1, std::min<size_t>({16, std::max(1u, std::thread::hardware_concurrency()),
                                                                (nt + 255) / 256}));
      std::vector<vlbm_status> wst(nw, VLBM_OK);
      std::vector<std::string> wmsg(nw);
      auto work = [&](int w) {
        for (size_t ti = nt * w / nw; ti < nt * (w + 1) / nw; ++ti) {
          vlbm_status st = tile_tasks(ti);
          if (st) {
            wst[w] = st;
            wmsg[w] = vlbm_last_error();  // the message lives in the worker's thread
            return;
          }
        }
      };
      vlbm_host::Pool::get().run(nw, work);
      for (int w = 0; w < nw; ++w)
        if (wst[w]) return fail3(wst[w], "%s", wmsg[w].c_str());
    }
    lt.mark("tasks");
    // slots in tile order: each tile's first reflux and ledger slot from a
    // prefix over the tiles, then its tasks renumbered on the pool
    {
      const size_t nt = L.tiles.size();
      std::vector<int> acc0(nt + 1, 0), led0(nt + 1, 0);
      for (size_t ti = 0; ti < nt; ++ti) {
        acc0[ti + 1] = acc0[ti] + (int)trefl[ti].size();
        led0[ti + 1] = led0[ti] + tled[ti];
      }
      refl.resize(acc0[nt]);
      par_ranges(nt, 64, [&](size_t t0, size_t t1) {
        for (size_t ti = t0; ti < t1; ++ti) {
          for (Task3 &t : per[ti]) {
            const int kind = t.kind & 0xFF;
            if (kind == K3_REFLUX)
              t.slot += acc0[ti];
            else if (kind == K3_OUTFLOW || kind == K3_REFLECT)
              t.slot += led0[ti];
          }
          for (size_t j = 0; j < trefl[ti].size(); ++j) {
            RefluxKey3 k = trefl[ti][j];
            k.slot += acc0[ti];
            refl[acc0[ti] + j] = k;
          }
        }
      });
      L.nacc = acc0[nt];
      L.nledger = led0[nt];
    }
    lt.mark("slots");
    // captures of this level for the parent's reflux slots
    if (l > 0) {
      // found on the pool in order of the parent's slots (a failure is
      // reported as its tile -1 - code), then appended to their tiles
      struct Cap {
        int32_t ti;
        Task3 t;
      };
      const std::vector<Cap> caps = par_collect<Cap>(caps_from_parent.size(), [&](size_t i, std::vector<Cap> &out) {
        const RefluxKey3 &k = caps_from_parent[i];
        const int q = k.q, n = q / 2;
        // the fine cells of hole H on its face towards the ring cell (which
        // lies at H + e_q): normal index r-1 for a + population, 0 for -
        int R0[3];
        for (int a = 0; a < 3; ++a) R0[a] = k.hole[a] * r;
        if (q % 2 == 0) R0[n] += r - 1;
        int ta[2], nt = 0;
        for (int a = 0; a < 3; ++a)
          if (a != n) ta[nt++] = a;
        Task3 t{};
        if (!L.in_frame(R0)) {
          out.push_back({-1, t});
          return;
        }
        t.kind = K3_CAPTURE;
        t.q = q;
        t.src = (int32_t)L.off(R0);
        t.n[0] = (int32_t)L.stride(ta[1]);  // outer (raster order: the higher axis)
        t.n[1] = (int32_t)L.stride(ta[0]);  // inner
        t.n[2] = t.n[3] = -1;
        t.slot = k.slot;
        for (int a2 = 0; a2 < r; ++a2)
          for (int b2 = 0; b2 < r; ++b2) {
            int Rc[3] = {R0[0], R0[1], R0[2]};
            Rc[ta[1]] += a2;
            Rc[ta[0]] += b2;
            if (!L.in_frame(Rc) || L.status[L.fidx(Rc)] != 1) {
              out.push_back({-2, t});
              return;
            }
          }
        const int32_t ti = own.tile_of(L, R0);
        out.push_back({ti < 0 ? -3 : ti, t});
      });
      for (const Cap &cp : caps) {
        if (cp.ti == -1) return fail3(VLBM_ENEST, "internal: capture outside the fine frame");
        if (cp.ti == -2) return fail3(VLBM_ENEST, "level %d: reflux face cell not active (nesting)", l);
        if (cp.ti == -3) return fail3(VLBM_ENEST, "internal: capture without a tile");
        per[cp.ti].push_back(cp.t);
      }
    }
    lt.mark("captures");
    L.face_key.clear();
    L.face_key.reserve(refl.size());
    for (const RefluxKey3 &k : refl) {
      int ring[3] = {k.hole[0] + E3[k.q][0], k.hole[1] + E3[k.q][1], k.hole[2] + E3[k.q][2]};
      c->wrap(l, ring);
      L.face_key.push_back((((int64_t)ring[2] * L.N[1] + ring[1]) * L.N[0] + ring[0]) * 6 + (k.q ^ 1));
    }
    lt.mark("face keys");
    std::sort(L.face_key.begin(), L.face_key.end());
    lt.mark("face sort");
    caps_from_parent.swap(refl);
    // tasks grouped by tile, in tile order: offsets by a prefix, copies on
    // the pool
    {
      const size_t nt = L.tiles.size();
      size_t ntask = 0;
      for (size_t ti = 0; ti < nt; ++ti) {
        L.tiles[ti].task0 = (int32_t)ntask;
        L.tiles[ti].ntask = (int32_t)per[ti].size();
        ntask += per[ti].size();
      }
      L.tasks.resize(ntask);
      par_ranges(nt, 64, [&](size_t t0, size_t t1) {
        for (size_t ti = t0; ti < t1; ++ti)
          std::copy(per[ti].begin(), per[ti].end(), L.tasks.begin() + L.tiles[ti].task0);
      });
    }
    lt.mark("faces+order");
  }
  if (!caps_from_parent.empty()) return fail3(VLBM_ENEST, "internal: reflux slots on the finest level");
  return VLBM_OK;
}

template <class T>
vlbm_status upload3(vlbm3_ctx *c, T *&dst, const std::vector<T> &v, size_t min_elems = 1) {
  dfree(c->mem, dst);
  const size_t n = std::max(v.size(), min_elems);
  ALLOC3(dst, sizeof(T) * n);
  if (!v.empty()) HIPCHK3(hipMemcpyAsync(dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, c->stream));
  return VLBM_OK;
}

vlbm_status upload_lists3(vlbm3_ctx *c) {
  for (int l = 0; l < c->nlev; ++l) {
    Level3 &L = c->lv[l];
    vlbm_status st = upload3(c, L.dtiles, L.tiles);
    if (!st) st = upload3(c, L.dtasks, L.tasks);
    if (st) return st;
    dfree(c->mem, L.dacc);
    dfree(c->mem, L.dledger);
    dfree(c->mem, L.dpartial);
    ALLOC3(L.dacc, sizeof(double) * 5 * std::max(1, L.nacc));
    ALLOC3(L.dledger, sizeof(double) * 5 * std::max(1, L.nledger));
    ALLOC3(L.dpartial, sizeof(double) * 5 * std::max<size_t>(1, L.tiles.size()));
    HIPCHK3(hipMemsetAsync(L.dacc, 0, sizeof(double) * 5 * std::max(1, L.nacc), c->stream));
    HIPCHK3(hipMemsetAsync(L.dledger, 0, sizeof(double) * 5 * std::max(1, L.nledger), c->stream));
  }
  HIPCHK3(hipStreamSynchronize(c->stream));
  return VLBM_OK;
}

void schedule3(int l, int k, int nlev, int r, std::vector<std::pair<int, int>> &out) {
  if (l + 1 < nlev)
    for (int kk = 1; kk <= r; ++kk) schedule3(l + 1, kk, nlev, r, out);
  out.push_back({l, k});
}

double ak3(int k, int r) { return (double)(2 * k - r - 1) / (double)(2 * r); }

// Descriptors of every phase for the two parities of the coarse step count
// relative to table_base (buffers alternate).
vlbm_status build_tables3(vlbm3_ctx *c) {
  c->phases.clear();
  schedule3(0, 1, c->nlev, c->p.r, c->phases);
  const size_t P = c->phases.size();
  for (int l = 0; l < kL; ++l) c->flips[l] = 0;
  for (const auto &ph : c->phases) c->flips[ph.first] += 1;
  std::vector<Desc3> descs(2 * P);
  for (int e = 0; e < 2; ++e) {
    long st[kL];
    for (int l = 0; l < kL; ++l) st[l] = c->lv[l].steps + e * c->flips[l];
    for (size_t p = 0; p < P; ++p) {
      const int l = c->phases[p].first;
      const Level3 &L = c->lv[l];
      Desc3 a{};
      a.src = L.buf[st[l] & 1];
      a.dst = L.buf[(st[l] + 1) & 1];
      if (l > 0) {
        const Level3 &PL = c->lv[l - 1];
        a.pcur = PL.buf[st[l - 1] & 1];
        a.pprev = PL.buf[(st[l - 1] + 1) & 1];
        a.pplane = PL.plane;
        a.acc_out = PL.dacc;
      }
      a.tiles = L.dtiles;
      a.tasks = L.dtasks;
      a.acc_in = L.dacc;
      a.ledger = L.dledger;
      a.plane = L.plane;
      a.slab = L.slab;
      a.pitch = L.pitch;
      a.ntiles = (int32_t)L.tiles.size();
      a.r = c->p.r;
      a.rrr = (double)(c->p.r * c->p.r * c->p.r);
      a.w3 = L.dx * L.dx * L.dx;
      a.gm1 = c->gm1;
      a.h = c->h;
      a.tb = c->tb;
      descs[e * P + p] = a;
      st[l] += 1;
    }
  }
  dfree(c->mem, c->ddesc);
  ALLOC3(c->ddesc, sizeof(Desc3) * descs.size());
  HIPCHK3(hipMemcpyAsync(c->ddesc, descs.data(), sizeof(Desc3) * descs.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK3(hipStreamSynchronize(c->stream));
  c->table_base = c->coarse_steps;
  return VLBM_OK;
}

vlbm_status prof_flush3(vlbm3_ctx *c) {
  if (c->pend.empty()) return VLBM_OK;
  HIPCHK3(hipEventSynchronize(c->pev[2 * c->pend.size() - 1]));
  for (size_t i = 0; i < c->pend.size(); ++i) {
    float ms = 0.f;
    HIPCHK3(hipEventElapsedTime(&ms, c->pev[2 * i], c->pev[2 * i + 1]));
    c->prof_ms[c->pend[i].first] += ms;
    c->prof_calls[c->pend[i].first] += 1;
    c->prof_cells[c->pend[i].first] += c->pend[i].second;
  }
  c->pend.clear();
  return VLBM_OK;
}

vlbm_status coarse_step3(vlbm3_ctx *c) {
  const int e = (int)((c->coarse_steps - c->table_base) & 1);
  const size_t P = c->phases.size();
  for (size_t p = 0; p < P; ++p) {
    const int l = c->phases[p].first, k = c->phases[p].second;
    Launch3 a{};
    a.d = c->ddesc + e * P + p;
    a.nblocks = (int32_t)c->lv[l].tiles.size();
    a.first = k == 1;
    a.flags = c->flags | c->sflags;
    a.ak = ak3(k, c->p.r);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof) {
      if (c->pend.size() >= 4096) {
        vlbm_status st = prof_flush3(c);
        if (st) return st;
      }
      const size_t i = 2 * c->pend.size();
      while (c->pev.size() < i + 2) {
        hipEvent_t ev;
        HIPCHK3(hipEventCreate(&ev));
        c->pev.push_back(ev);
      }
      e0 = c->pev[i];
      e1 = c->pev[i + 1];
      double cells = 0;
      for (const Tile3 &t : c->lv[l].tiles) cells += (double)t.w * t.h;
      c->pend.push_back({l, cells});
    }
    HIPCHK3(launch_step3(a, c->stream, e0, e1));
  }
  for (int l = 0; l < c->nlev; ++l) c->lv[l].steps += c->flips[l];
  c->coarse_steps += 1;
  return VLBM_OK;
}

vlbm_status check_rect3(vlbm3_ctx *c, int level, const int lo[3], const int ext[3]) {
  if (!c || !c->have_hierarchy) return fail3(VLBM_ESTATE, "no hierarchy installed");
  if (level < 0 || level >= c->p.max_levels) return fail3(VLBM_EINVAL, "bad level %d", level);
  const Level3 &L = c->lv[level];
  long s = 1;
  for (int i = 0; i < level; ++i) s *= c->p.r;
  const int n0[3] = {c->p.nx0, c->p.ny0, c->p.nz0};
  for (int a = 0; a < 3; ++a)
    if (lo[a] < 0 || ext[a] < 0 || lo[a] + (long)ext[a] > n0[a] * s)
      return fail3(VLBM_EINVAL, "rectangle outside level %d", level);
  (void)L;
  return VLBM_OK;
}

vlbm_status rect_io3(vlbm3_ctx *c, int level, const int lo[3], const int ext[3], double *host, int ncomp,
                     bool write, bool raw) {
  vlbm_status st = check_rect3(c, level, lo, ext);
  if (st) return st;
  const size_t full = (size_t)ext[0] * ext[1] * ext[2];
  if (!write)
    for (size_t i = 0; i < full * ncomp; ++i) host[i] = NAN;
  Level3 &L = c->lv[level];
  if (!L.present || full == 0) return VLBM_OK;
  // clip to the frame
  int clo[3], cext[3], o[3];
  for (int a = 0; a < 3; ++a) {
    const int x0 = std::max(lo[a], L.f0[a]), x1 = std::min(lo[a] + ext[a], L.f0[a] + L.fn[a]);
    if (x1 <= x0) return VLBM_OK;
    clo[a] = x0;
    cext[a] = x1 - x0;
    o[a] = x0 - lo[a];
  }
  const size_t n = (size_t)cext[0] * cext[1] * cext[2];
  double *stage = nullptr;
  ALLOC3(stage, sizeof(double) * ncomp * n);
  std::vector<double> tmp(ncomp * n);
  Rect3 a{};
  a.buf0 = write ? L.buf[0] : L.buf[L.cur()];
  a.buf1 = L.buf[1];
  a.status = L.dstatus;
  a.stage = stage;
  a.plane = L.plane;
  a.slab = L.slab;
  a.pitch = L.pitch;
  a.xoff = L.xoff;
  a.fx0 = L.f0[0];
  a.fy0 = L.f0[1];
  a.fz0 = L.f0[2];
  a.fw = L.fn[0];
  a.fh = L.fn[1];
  a.x0 = clo[0];
  a.y0 = clo[1];
  a.z0 = clo[2];
  a.nx = cext[0];
  a.ny = cext[1];
  a.nz = cext[2];
  a.gm1 = c->gm1;
  a.h = c->h;
  auto hidx = [&](int k, int x, int y, int z) {
    return (size_t)k * full + ((size_t)(z + o[2]) * ext[1] + (y + o[1])) * ext[0] + (x + o[0]);
  };
  hipError_t e = hipSuccess;
  if (write) {
    for (int k = 0; k < ncomp; ++k)
      for (int z = 0; z < cext[2]; ++z)
        for (int y = 0; y < cext[1]; ++y)
          memcpy(&tmp[(size_t)k * n + ((size_t)z * cext[1] + y) * cext[0]], &host[hidx(k, 0, y, z)],
                 sizeof(double) * cext[0]);
    e = hipMemcpyAsync(stage, tmp.data(), sizeof(double) * ncomp * n, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = launch_set3(a, raw ? 1 : 0, c->fp32, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  } else {
    e = launch_get3(a, ncomp == 30 ? 1 : 0, c->fp32, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(tmp.data(), stage, sizeof(double) * ncomp * n, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
      for (int k = 0; k < ncomp; ++k)
        for (int z = 0; z < cext[2]; ++z)
          for (int y = 0; y < cext[1]; ++y)
            memcpy(&host[hidx(k, 0, y, z)], &tmp[(size_t)k * n + ((size_t)z * cext[1] + y) * cext[0]],
                   sizeof(double) * cext[0]);
  }
  c->mem.release(stage);
  if (e != hipSuccess) return fail3(VLBM_EDEVICE, "state transfer: %s", hipGetErrorString(e));
  return VLBM_OK;
}

vlbm_status restart_count3(vlbm3_ctx *c) {
  c->table_base -= c->coarse_steps;  // keep the table parity while restarting the count
  c->coarse_steps = 0;
  for (int l = 0; l < c->nlev; ++l) {
    Level3 &L = c->lv[l];
    HIPCHK3(hipMemsetAsync(L.dledger, 0, sizeof(double) * 5 * std::max(1, L.nledger), c->stream));
  }
  return VLBM_OK;
}

void kadd3(double &s, double &cmp, double v) {
  const double t = s + v;
  if (std::fabs(s) >= std::fabs(v))
    cmp += (s - t) + v;
  else
    cmp += (v - t) + s;
  s = t;
}

// The boundary ledger of every level, summed as vlbm3_conserved_totals sums
// it (compensated, level by level, slot by slot), without the audit of the
// populations.
vlbm_status ledger_sum3(vlbm3_ctx *c, double ledger[5]) {
  double ls[5] = {}, lc[5] = {};
  // every level's slots into one pinned buffer (a face of a 256^3 level has
  // some 400,000 slots: 16 MB that a pageable copy takes milliseconds over)
  size_t at[kL] = {}, total = 0;
  for (int l = 0; l < c->nlev; ++l) {
    at[l] = total;
    total += 5 * (size_t)c->lv[l].nledger;
  }
  std::vector<double> pageable;
  double *h = c->pinned(std::max<size_t>(total, 1));
  if (!h) {
    pageable.resize(std::max<size_t>(total, 1));
    h = pageable.data();
  }
  for (int l = 0; l < c->nlev; ++l) {
    const Level3 &L = c->lv[l];
    if (!L.nledger) continue;
    HIPCHK3(hipMemcpyAsync(h + at[l], L.dledger, sizeof(double) * 5 * L.nledger, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCHK3(hipStreamSynchronize(c->stream));
  for (int l = 0; l < c->nlev; ++l)
    for (int k = 0; k < 5; ++k)
      for (int t = 0; t < c->lv[l].nledger; ++t) kadd3(ls[k], lc[k], h[at[l] + 5 * (size_t)t + k]);
  for (int k = 0; k < 5; ++k) ledger[k] = ls[k] + lc[k];
  return VLBM_OK;
}

bool wrap_in(const vlbm3_params &p, const Level3 *lv, int l, int q[3]) {
  for (int a = 0; a < 3; ++a) {
    const int n = lv[l].N[a];
    if (q[a] < 0 || q[a] >= n) {
      if (p.bc[2 * a] != VLBM_BC_PERIODIC) return false;
      q[a] = ((q[a] % n) + n) % n;
    }
  }
  return true;
}

bool cov_in(const Level3 *lv, int nlev, int l, const int q[3]) {
  if (l >= nlev || !lv[l].present || !lv[l].in_frame(q)) return false;
  return lv[l].cov[lv[l].fidx(q)] != 0;
}

// Frames, coverage and status of the hierarchy `boxes` into lv[0..kL), with
// every host-side check (alignment, range, proper nesting). No device work.
vlbm_status build_geometry3(const vlbm3_params &p, const vlbm3_box *boxes, int nboxes, Level3 *lv, int &nlev) {
  Geom3 g;
  vlbm_status st = check_boxes3(p, boxes, nboxes, g);
  if (st) return st;
  nlev = g.nlev;
  for (int l = 0; l < kL; ++l) {
    lv[l] = Level3();
    frame3(p, g, l, lv[l]);
    if (lv[l].present && lv[l].plane >= (int64_t(1) << 31))
      return fail3(VLBM_EINVAL, "level %d frame too large for 32-bit offsets", l);
  }
  // coverage, on the pool by frame planes: each thread clears its planes and
  // fills the part of every box (level 0: the domain) that lies in them
  for (int l = 0; l < nlev; ++l) {
    Level3 &L = lv[l];
    const size_t slab = (size_t)L.fn[0] * L.fn[1];
    L.cov.resize(slab * L.fn[2]);
    par_ranges((size_t)L.fn[2], 1, [&](size_t z0, size_t z1) {
      memset(L.cov.data() + z0 * slab, 0, (z1 - z0) * slab);
      const int za = L.f0[2] + (int)z0, zb = L.f0[2] + (int)z1;  // frame planes [za, zb)
      auto fill = [&](const int lo[3], const int ext[3]) {
        for (int z = std::max(lo[2], za); z < std::min(lo[2] + ext[2], zb); ++z)
          for (int y = lo[1]; y < lo[1] + ext[1]; ++y) {
            int p0[3] = {lo[0], y, z};
            memset(&L.cov[L.fidx(p0)], 1, ext[0]);
          }
      };
      if (l == 0) {
        const int lo[3] = {0, 0, 0};
        fill(lo, L.N);
      } else {
        for (int b = 0; b < nboxes; ++b)
          if (boxes[b].level == l) {
            const int lo[3] = {boxes[b].i0, boxes[b].j0, boxes[b].k0};
            const int ext[3] = {boxes[b].nx, boxes[b].ny, boxes[b].nz};
            fill(lo, ext);
          }
      }
    });
  }
  // proper nesting: the parent of every covered cell and its face neighbours
  const int r = p.r;
  std::vector<uint8_t> bad(nboxes > 0 ? nboxes : 1, 0);
  par_ranges((size_t)std::max(nboxes, 0), 4, [&](size_t b0, size_t b1) {
    for (size_t b = b0; b < b1; ++b) {
      const vlbm3_box &B = boxes[b];
      const int l = B.level;
      for (int pz = B.k0 / r; pz < (B.k0 + B.nz) / r && !bad[b]; ++pz)
        for (int py = B.j0 / r; py < (B.j0 + B.ny) / r && !bad[b]; ++py)
          for (int px = B.i0 / r; px < (B.i0 + B.nx) / r && !bad[b]; ++px)
            for (int d = -1; d < 6; ++d) {
              int P[3] = {px + (d < 0 ? 0 : E3[d][0]), py + (d < 0 ? 0 : E3[d][1]), pz + (d < 0 ? 0 : E3[d][2])};
              if (!wrap_in(p, lv, l - 1, P)) continue;
              if (!cov_in(lv, nlev, l - 1, P)) {
                bad[b] = 1;
                break;
              }
            }
    }
  });
  for (int b = 0; b < nboxes; ++b)
    if (bad[b]) return fail3(VLBM_ENEST, "box %d: hierarchy not properly nested", b);
  // status: covered cells are active (1); those under a level-(l+1) box,
  // whose parent cells form a block of whole level-l cells, are holes (2)
  for (int l = 0; l < nlev; ++l) {
    Level3 &L = lv[l];
    const size_t slab = (size_t)L.fn[0] * L.fn[1];
    L.status.resize(L.cov.size());
    par_ranges((size_t)L.fn[2], 1, [&](size_t z0, size_t z1) {
      memcpy(L.status.data() + z0 * slab, L.cov.data() + z0 * slab, (z1 - z0) * slab);
      const int za = L.f0[2] + (int)z0, zb = L.f0[2] + (int)z1;
      for (int b = 0; b < nboxes; ++b) {
        const vlbm3_box &B = boxes[b];
        if (B.level != l + 1) continue;
        for (int z = std::max(B.k0 / r, za); z < std::min((B.k0 + B.nz) / r, zb); ++z)
          for (int y = B.j0 / r; y < (B.j0 + B.ny) / r; ++y) {
            const int p0[3] = {B.i0 / r, y, z};
            memset(&L.status[L.fidx(p0)], 2, B.nx / r);
          }
      }
    });
  }
  return VLBM_OK;
}

}  // namespace

namespace {

// --------------------------------------------------------------------------
// Tagging and clustering (Sec. 3.4, Fig. amr-flowchart, in 3-D)
// --------------------------------------------------------------------------
struct TagMap3 {  // one byte per frame cell of a level, frame order
  int o[3] = {0, 0, 0}, n[3] = {0, 0, 0};
  std::vector<uint8_t> t;
  uint8_t &at(int x, int y, int z) { return t[((size_t)(z - o[2]) * n[1] + (y - o[1])) * n[0] + (x - o[0])]; }
};

struct CovMap3 {  // coverage of a level over a box of its cells (all: everything)
  bool all = true;
  int o[3] = {0, 0, 0}, n[3] = {0, 0, 0};
  std::vector<uint8_t> m;
  bool at(int x, int y, int z) const {
    if (all) return true;
    const int p[3] = {x - o[0], y - o[1], z - o[2]};
    for (int a = 0; a < 3; ++a)
      if (p[a] < 0 || p[a] >= n[a]) return false;
    return m[((size_t)p[2] * n[1] + p[1]) * n[0] + p[0]] != 0;
  }
};

// Tags of every active cell of level l's frame (device kernel, then to host).
vlbm_status tag_frame3(vlbm3_ctx *c, int l, double thr, TagMap3 &T) {
  const Level3 &L = c->lv[l];
  const size_t n = (size_t)L.fn[0] * L.fn[1] * L.fn[2];
  for (int a = 0; a < 3; ++a) {
    T.o[a] = L.f0[a];
    T.n[a] = L.fn[a];
  }
  T.t.assign(n, 0);
  uint8_t *dt = nullptr;
  ALLOC3(dt, n);
  Tag3Args a{};
  a.buf = L.buf[L.cur()];
  a.status = L.dstatus;
  a.tags = dt;
  a.plane = L.plane;
  a.slab = L.slab;
  a.pitch = L.pitch;
  a.xoff = L.xoff;
  for (int k = 0; k < 3; ++k) {
    a.f0[k] = L.f0[k];
    a.fn[k] = L.fn[k];
    a.N[k] = L.N[k];
    a.periodic |= c->periodic(k) ? 1 << k : 0;
  }
  a.thr = thr;
  hipError_t e = launch_tag3(a, c->fp32, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(T.t.data(), dt, n, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->mem.release(dt);
  if (e != hipSuccess) return fail3(VLBM_EDEVICE, "tags: %s", hipGetErrorString(e));
  return VLBM_OK;
}

// Tiles of T cells (per axis) of level l reached by a range [a, b] of cells
// along an axis of n cells (periodic: wrapped), appended to v.
void tiles_in3(int a, int b, int n, int T, bool periodic, std::vector<int> &v) {
  v.clear();
  if (periodic && b - a + 1 >= n) a = 0, b = n - 1, periodic = false;
  if (!periodic) {
    a = std::max(a, 0);
    b = std::min(b, n - 1);
    for (int t = a / T; a <= b && t <= b / T; ++t) v.push_back(t);
    return;
  }
  const int am = ((a % n) + n) % n, bm = ((b % n) + n) % n;
  if (am <= bm) {
    for (int t = am / T; t <= bm / T; ++t) v.push_back(t);
  } else {  // wraps: [am, n) and [0, bm]
    for (int t = 0; t <= bm / T; ++t) v.push_back(t);
    for (int t = am / T; t <= (n - 1) / T; ++t)
      if (v.empty() || t > v.back()) v.push_back(t);
  }
}

// Boxes of level l+1 over the tagged cells of level l, dilated by `buffer`
// cells: a grid of tiles of T = ceil(min_box / r) level-l cells per axis; a
// tile is taken when the dilation reaches it and it, and the cells beside
// its six faces, are covered at level l (so the boxes nest); taken tiles are
// merged greedily into runs of at most maxT tiles along x, stacked along y
// while identical, then along z while identical.
void cluster_level3(const vlbm3_ctx *c, int l, const TagMap3 &tags, const CovMap3 &cov, int buffer,
                    int min_box, int max_box, std::vector<vlbm3_box> &out) {
  const int r = c->p.r;
  const Level3 &L = c->lv[l];
  const int T = std::max(1, (min_box + r - 1) / r);
  const int maxT = std::max(1, max_box / (T * r));
  int nt[3];
  bool per[3];
  for (int a = 0; a < 3; ++a) {
    nt[a] = (L.N[a] + T - 1) / T;
    per[a] = c->periodic(a);
  }
  auto tid = [&](int tx, int ty, int tz) { return ((size_t)tz * nt[1] + ty) * nt[0] + tx; };
  std::vector<uint8_t> hit((size_t)nt[0] * nt[1] * nt[2], 0);
  std::vector<int> xs, ys, zs;
  for (int fz = 0; fz < tags.n[2]; ++fz)
    for (int fy = 0; fy < tags.n[1]; ++fy) {
      const uint8_t *row = &tags.t[((size_t)fz * tags.n[1] + fy) * tags.n[0]];
      const int y = tags.o[1] + fy, z = tags.o[2] + fz;
      bool any = false;
      int fx = 0;
      while (fx < tags.n[0]) {
        if (!row[fx]) {  // to the next tagged cell (tags are 0 or 1)
          const void *nx = memchr(row + fx, 1, tags.n[0] - fx);
          if (!nx) break;
          fx = (int)(static_cast<const uint8_t *>(nx) - row);
        }
        const int xa = fx;
        while (fx < tags.n[0] && row[fx]) ++fx;
        if (!any) {
          tiles_in3(y - buffer, y + buffer, L.N[1], T, per[1], ys);
          tiles_in3(z - buffer, z + buffer, L.N[2], T, per[2], zs);
          any = true;
        }
        tiles_in3(tags.o[0] + xa - buffer, tags.o[0] + fx - 1 + buffer, L.N[0], T, per[0], xs);
        for (int tz : zs)
          for (int ty : ys)
            for (int tx : xs) hit[tid(tx, ty, tz)] = 1;
      }
    }
  // covered at level l; true outside a non-periodic side
  auto covered_at = [&](int x, int y, int z) {
    int p[3] = {x, y, z};
    for (int a = 0; a < 3; ++a)
      if (p[a] < 0 || p[a] >= L.N[a]) {
        if (!per[a]) return true;
        p[a] = (p[a] + L.N[a]) % L.N[a];
      }
    return cov.at(p[0], p[1], p[2]);
  };
  std::vector<uint8_t> mark(hit.size(), 0);
  for (int tz = 0; tz < nt[2]; ++tz)
    for (int ty = 0; ty < nt[1]; ++ty)
      for (int tx = 0; tx < nt[0]; ++tx) {
        if (!hit[tid(tx, ty, tz)]) continue;
        bool ok = true;
        if (!cov.all) {
          const int lo[3] = {tx * T, ty * T, tz * T};
          const int hi[3] = {std::min(L.N[0], lo[0] + T), std::min(L.N[1], lo[1] + T),
                             std::min(L.N[2], lo[2] + T)};
          for (int z = lo[2] - 1; ok && z <= hi[2]; ++z)
            for (int y = lo[1] - 1; ok && y <= hi[1]; ++y)
              for (int x = lo[0] - 1; ok && x <= hi[0]; ++x) {
                const int outside = (x < lo[0] || x >= hi[0]) + (y < lo[1] || y >= hi[1]) + (z < lo[2] || z >= hi[2]);
                if (outside <= 1) ok = covered_at(x, y, z);  // the tile and its face layers
              }
        }
        mark[tid(tx, ty, tz)] = ok;
      }
  // greedy merge: x runs, stacked along y, then along z
  struct Rect { int a, b, y0, h; };
  struct Box { int a, b, y0, h, z0, d; };
  std::vector<Box> open, next;
  auto emit = [&](const Box &u) {
    const int x0 = u.a * T, x1 = std::min(L.N[0], u.b * T);
    const int y0 = u.y0 * T, y1 = std::min(L.N[1], (u.y0 + u.h) * T);
    const int z0 = u.z0 * T, z1 = std::min(L.N[2], (u.z0 + u.d) * T);
    out.push_back({l + 1, x0 * r, y0 * r, z0 * r, (x1 - x0) * r, (y1 - y0) * r, (z1 - z0) * r});
  };
  for (int tz = 0; tz <= nt[2]; ++tz) {
    std::vector<Rect> rects;
    if (tz < nt[2]) {  // the slab's rectangles
      std::vector<Rect> ro, rn;
      for (int ty = 0; ty <= nt[1]; ++ty) {
        rn.clear();
        if (ty < nt[1]) {
          int tx = 0;
          while (tx < nt[0]) {
            if (!mark[tid(tx, ty, tz)]) {
              ++tx;
              continue;
            }
            const int a = tx;
            while (tx < nt[0] && mark[tid(tx, ty, tz)] && tx - a < maxT) ++tx;
            rn.push_back({a, tx, ty, 1});
          }
        }
        for (const Rect &o : ro) {
          bool cont = false;
          for (Rect &q : rn)
            if (q.a == o.a && q.b == o.b && q.h == 1 && o.h < maxT) {
              q.y0 = o.y0;
              q.h = o.h + 1;
              cont = true;
              break;
            }
          if (!cont) rects.push_back(o);
        }
        ro = rn;
      }
    }
    next.clear();
    for (const Box &o : open) {
      bool cont = false;
      for (Rect &q : rects)
        if (q.a == o.a && q.b == o.b && q.y0 == o.y0 && q.h == o.h && o.d < maxT) {
          next.push_back({o.a, o.b, o.y0, o.h, o.z0, o.d + 1});
          q.h = -1;  // taken
          cont = true;
          break;
        }
      if (!cont) emit(o);
    }
    for (const Rect &q : rects)
      if (q.h > 0) next.push_back({q.a, q.b, q.y0, q.h, tz, 1});
    open.swap(next);
  }
}

// Parents of tagged level-(l+1) cells are tagged at level l (so a refined
// zone keeps its parent refined), then levels are clustered coarsest first,
// each inside the coverage of the boxes just made one level up.
void cluster_hierarchy3(const vlbm3_ctx *c, std::vector<TagMap3> &tags, int buffer, int min_box, int max_box,
                        std::vector<vlbm3_box> &boxes) {
  const int r = c->p.r, ML = c->p.max_levels;
  PhaseTimer tm("cluster3");
  for (int l = ML - 1; l >= 1; --l) {
    TagMap3 &F = tags[l], &P = tags[l - 1];
    if (F.t.empty() || P.t.empty()) continue;
    // on the pool by parent planes: the fine planes of a parent plane are its
    // r children planes, so no two threads mark the same parent cell
    auto fdiv = [r](int a) { return a >= 0 ? a / r : -((-a + r - 1) / r); };  // floor(a / r)
    const int pz0 = fdiv(F.o[2]), pz1 = fdiv(F.o[2] + F.n[2] - 1) + 1;
    par_ranges((size_t)(pz1 - pz0), 1, [&](size_t i0, size_t i1) {
    for (int fz = std::max(0, (pz0 + (int)i0) * r - F.o[2]); fz < std::min(F.n[2], (pz0 + (int)i1) * r - F.o[2]); ++fz)
      for (int fy = 0; fy < F.n[1]; ++fy) {
        const uint8_t *row = &F.t[((size_t)fz * F.n[1] + fy) * F.n[0]];
        for (int fx = 0; fx < F.n[0]; ++fx) {
          if (!row[fx]) {  // to the next tagged cell (tags are 0 or 1)
            const void *nx = memchr(row + fx, 1, F.n[0] - fx);
            if (!nx) break;
            fx = (int)(static_cast<const uint8_t *>(nx) - row);
          }
          const int p[3] = {(F.o[0] + fx) / r, (F.o[1] + fy) / r, (F.o[2] + fz) / r};
          bool in = true;
          for (int a = 0; a < 3; ++a) in = in && p[a] >= P.o[a] && p[a] < P.o[a] + P.n[a];
          if (in) P.at(p[0], p[1], p[2]) = 1;
        }
      }
    });
  }
  tm.mark("parents");
  CovMap3 cov;
  for (int l = 0; l + 1 < ML; ++l) {
    if (tags[l].t.empty()) break;
    const size_t before = boxes.size();
    cluster_level3(c, l, tags[l], cov, buffer, min_box, max_box, boxes);
    tm.mark(l == 0 ? "level 0" : l == 1 ? "level 1" : "level 2+");
    if (boxes.size() == before || l + 2 >= ML) break;
    CovMap3 nc;  // coverage of level l+1 over the bounding box of its new boxes
    nc.all = false;
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (size_t b = before; b < boxes.size(); ++b) {
      const int bl[3] = {boxes[b].i0, boxes[b].j0, boxes[b].k0}, bn[3] = {boxes[b].nx, boxes[b].ny, boxes[b].nz};
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], bl[a]);
        hi[a] = std::max(hi[a], bl[a] + bn[a]);
      }
    }
    for (int a = 0; a < 3; ++a) {
      nc.o[a] = lo[a];
      nc.n[a] = hi[a] - lo[a];
    }
    nc.m.assign((size_t)nc.n[0] * nc.n[1] * nc.n[2], 0);
    for (size_t b = before; b < boxes.size(); ++b)
      for (int z = boxes[b].k0; z < boxes[b].k0 + boxes[b].nz; ++z)
        for (int y = boxes[b].j0; y < boxes[b].j0 + boxes[b].ny; ++y)
          memset(&nc.m[((size_t)(z - lo[2]) * nc.n[1] + (y - lo[1])) * nc.n[0] + boxes[b].i0 - lo[0]], 1,
                 boxes[b].nx);
    cov = std::move(nc);
  }
}

}  // namespace

extern "C" {

vlbm_status vlbm3_create(const vlbm3_params *params, void *stream, vlbm3_ctx **out) {
  if (!params || !out) return fail3(VLBM_EINVAL, "null argument");
  vlbm_status st = check_params3(*params);
  if (st) return st;
  vlbm3_ctx *c = new vlbm3_ctx();
  c->p = *params;
  c->stream = static_cast<hipStream_t>(stream);
  c->gm1 = c->p.gamma - 1.0;
  c->h = 1.0 / (2.0 * c->p.c);
  c->tb = 2.0 * c->p.beta;
  c->fp32 = c->p.precision != VLBM_FP64;
  c->sflags = !c->fp32 ? 0 : S3_FP32 | (c->p.precision == VLBM_FP32_STORAGE ? S3_F64_MATH : 0);
  c->tile_cells = c->fp32 ? 1024 : 512;
  *out = c;
  return VLBM_OK;
}

vlbm_status vlbm3_bind_allocator(vlbm3_ctx *c, vlbm_alloc_fn alloc, vlbm_free_fn release, void *user) {
  if (!c || !alloc || !release) return fail3(VLBM_EINVAL, "null argument");
  if (c->have_hierarchy) return fail3(VLBM_ESTATE, "bind the allocator before installing a hierarchy");
  c->mem.a = alloc;
  c->mem.f = release;
  c->mem.user = user;
  return VLBM_OK;
}

void vlbm3_destroy(vlbm3_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t ev : c->pev) (void)hipEventDestroy(ev);
  for (int l = 0; l < kL; ++l) free_level3(c->mem, c->lv[l]);
  dfree(c->mem, c->ddesc);
  if (c->pin) (void)hipHostFree(c->pin);
  delete c;
}

size_t vlbm3_footprint_bytes(const vlbm3_params *params, const vlbm3_box *boxes, int nboxes) {
  if (!params || check_params3(*params)) return 0;
  Geom3 g;
  if (check_boxes3(*params, boxes, nboxes, g)) return 0;
  size_t total = 0;
  for (int l = 0; l < g.nlev; ++l) {
    Level3 L;
    frame3(*params, g, l, L);
    if (!L.present) continue;
    const size_t cells = (size_t)L.fn[0] * L.fn[1] * L.fn[2];
    total += 2 * level_bytes3(L) + cells;  // buffers and status
    total += cells * 3;                    // tiles, tasks and slots (bounded estimate)
  }
  return total;
}

vlbm_status vlbm3_set_hierarchy(vlbm3_ctx *c, const vlbm3_box *boxes, int nboxes) {
  return guard3([&]() -> vlbm_status {
    if (!c) return fail3(VLBM_EINVAL, "null context");
    Level3 nl[kL];
    int nnlev = 1;
    vlbm_status st = build_geometry3(c->p, boxes, nboxes, nl, nnlev);
    if (st) return st;
    HIPCHK3(hipStreamSynchronize(c->stream));
    for (int l = 0; l < kL; ++l) free_level3(c->mem, c->lv[l]);
    c->have_hierarchy = false;
    for (int l = 0; l < kL; ++l) c->lv[l] = std::move(nl[l]);
    c->nlev = nnlev;
    st = build_lists3(c);
    if (st) {
      for (int m = 0; m < kL; ++m) free_level3(c->mem, c->lv[m]);
      return st;
    }
    for (int l = 0; l < c->nlev; ++l) {
      Level3 &L = c->lv[l];
      const size_t nb = level_bytes3(L);
      ALLOC3(L.buf[0], nb);
      ALLOC3(L.buf[1], nb);
      HIPCHK3(hipMemsetAsync(L.buf[0], 0, nb, c->stream));
      HIPCHK3(hipMemsetAsync(L.buf[1], 0, nb, c->stream));
      ALLOC3(L.dstatus, L.status.size());
      HIPCHK3(hipMemcpyAsync(L.dstatus, L.status.data(), L.status.size(), hipMemcpyHostToDevice, c->stream));
      L.steps = 0;
    }
    st = upload_lists3(c);
    if (st) return st;
    c->boxes.assign(boxes, boxes + nboxes);
    c->have_hierarchy = true;
    c->coarse_steps = 0;
    return build_tables3(c);
  });
}

vlbm_status vlbm3_regrid(vlbm3_ctx *c, const vlbm3_box *boxes, int nboxes) {
  return guard3([&]() -> vlbm_status {
    if (!c || !c->have_hierarchy) return fail3(VLBM_ESTATE, "no hierarchy installed");
    PhaseTimer tm("regrid3");
    Level3 nl[kL];
    int nnlev = 1;
    vlbm_status st = build_geometry3(c->p, boxes, nboxes, nl, nnlev);
    if (st) return st;
    tm.mark("geometry");
    const int r = c->p.r, onlev = c->nlev;
    // the boundary ledger survives the rebuild of its slots
    double led[5] = {};
    st = ledger_sum3(c, led);
    if (st) return st;
    tm.mark("ledger");
    auto old_cov = [&](int l, const int q[3]) { return cov_in(c->lv, onlev, l, q); };
    auto new_cov = [&](int l, const int q[3]) { return cov_in(nl, nnlev, l, q); };
    // coverage row (y, z) of level l of `lv` (null: not in its frame), indexed
    // by x - f0[0] over the frame's columns
    auto cov_row = [](const Level3 *lv, int nlev, int l, int y, int z) -> const uint8_t * {
      if (l >= nlev || !lv[l].present) return nullptr;
      const Level3 &L = lv[l];
      if (y < L.f0[1] || y >= L.f0[1] + L.fn[1] || z < L.f0[2] || z >= L.f0[2] + L.fn[2]) return nullptr;
      const int q[3] = {L.f0[0], y, z};
      return &L.cov[L.fidx(q)];
    };
    auto in_row = [](const Level3 *lv, int l, const uint8_t *row, int x) {
      const Level3 &L = lv[l];
      return row && x >= L.f0[0] && x < L.f0[0] + L.fn[0] && row[x - L.f0[0]];
    };
    std::vector<void *> scratch;  // device op lists, freed after the final sync
    auto upload_ops = [&](const std::vector<RegridOp3> &ops, RegridOp3 *&d) -> vlbm_status {
      ALLOC3(d, sizeof(RegridOp3) * std::max<size_t>(1, ops.size()));
      scratch.push_back(d);
      if (!ops.empty()) HIPCHK3(hipMemcpyAsync(d, ops.data(), sizeof(RegridOp3) * ops.size(), hipMemcpyHostToDevice, c->stream));
      return VLBM_OK;
    };
    // 1. merges, finest level first, in the old frames (eq. amr-merge)
    for (int l = onlev - 1; l >= 1; --l) {
      const Level3 &F = c->lv[l];
      Level3 &Cl = c->lv[l - 1];
      const int nzs = (F.fn[2] - 2 + r - 1) / r;  // r-grid planes (the frame's first interior cell is aligned)
      const std::vector<RegridOp3> ops = par_collect<RegridOp3>((size_t)std::max(nzs, 0), [&](size_t iz, std::vector<RegridOp3> &out) {
        const int z = F.f0[2] + 1 + (int)iz * r;
        for (int y = F.f0[1] + 1; y < F.f0[1] + F.fn[1] - 1; y += r) {
          const uint8_t *fo = cov_row(c->lv, onlev, l, y, z), *fn = cov_row(nl, nnlev, l, y, z);
          for (int x = F.f0[0] + 1; x < F.f0[0] + F.fn[0] - 1; x += r) {
            if (!fo[x - F.f0[0]] || in_row(nl, l, fn, x)) continue;
            const int q[3] = {x, y, z};
            const int P[3] = {x / r, y / r, z / r};
            RegridOp3 o{};
            o.dst = (int32_t)Cl.off(P);
            o.src = (int32_t)F.off(q);
            out.push_back(o);
          }
        }
      });
      tm.mark("merge plan");
      if (ops.empty()) continue;
      RegridArgs3 a{};
      a.fine_cur = F.buf[F.cur()];
      a.coarse0 = Cl.buf[0];
      a.coarse1 = Cl.buf[1];
      a.fplane = F.plane;
      a.fslab = F.slab;
      a.fpitch = F.pitch;
      a.cplane = Cl.plane;
      a.r = r;
      RegridOp3 *d = nullptr;
      st = upload_ops(ops, d);
      if (st) return st;
      a.ops = d;
      a.nops = (int32_t)ops.size();
      HIPCHK3(launch_merge3(a, c->fp32, c->stream));
    }
    tm.mark("merges");
    // 2. new frames: surviving cells move over (both time levels); a level
    //    whose frame is unchanged keeps its buffers
    for (int l = 0; l < nnlev; ++l) {
      Level3 &N = nl[l];
      Level3 *O = l < onlev ? &c->lv[l] : nullptr;
      N.steps = O ? O->steps : 0;
      if (O && O->present && O->plane == N.plane && O->pitch == N.pitch && O->slab == N.slab &&
          O->f0[0] == N.f0[0] && O->f0[1] == N.f0[1] && O->f0[2] == N.f0[2] && O->fn[0] == N.fn[0] &&
          O->fn[1] == N.fn[1] && O->fn[2] == N.fn[2]) {
        N.buf[0] = O->buf[0];
        N.buf[1] = O->buf[1];
        O->buf[0] = O->buf[1] = nullptr;
        continue;
      }
      const size_t nb = level_bytes3(N);
      ALLOC3(N.buf[0], nb);
      ALLOC3(N.buf[1], nb);
      HIPCHK3(hipMemsetAsync(N.buf[0], 0, nb, c->stream));
      HIPCHK3(hipMemsetAsync(N.buf[1], 0, nb, c->stream));
      if (!O || !O->present) continue;
      const std::vector<int32_t> runs = par_collect<int32_t>((size_t)std::max(N.fn[2] - 2, 0), [&](size_t iz, std::vector<int32_t> &out) {
        const int z = N.f0[2] + 1 + (int)iz;
        for (int y = N.f0[1] + 1; y < N.f0[1] + N.fn[1] - 1; ++y) {
          int x = N.f0[0] + 1;
          const int xe = N.f0[0] + N.fn[0] - 1;
          while (x < xe) {
            const int q[3] = {x, y, z};
            if (!(N.cov[N.fidx(q)] && O->in_frame(q) && O->cov[O->fidx(q)])) {
              ++x;
              continue;
            }
            const int xa = x;
            while (x < xe) {
              const int qq[3] = {x, y, z};
              if (!(N.cov[N.fidx(qq)] && O->in_frame(qq) && O->cov[O->fidx(qq)])) break;
              ++x;
            }
            const int qa[3] = {xa, y, z};
            out.push_back((int32_t)O->off(qa));
            out.push_back((int32_t)N.off(qa));
            out.push_back(x - xa);
          }
        }
      });
      if (runs.empty()) continue;
      int32_t *druns = nullptr;
      ALLOC3(druns, sizeof(int32_t) * runs.size());
      scratch.push_back(druns);
      HIPCHK3(hipMemcpyAsync(druns, runs.data(), sizeof(int32_t) * runs.size(), hipMemcpyHostToDevice, c->stream));
      HIPCHK3(launch_copy3_runs(O->buf[0], O->buf[1], N.buf[0], N.buf[1], druns, (int)(runs.size() / 3), O->plane,
                                N.plane, c->fp32, c->stream));
    }
    tm.mark("frames");
    // 3. splits, coarsest level first, in the new frames (eqs. amr-slope,
    //    amr-split); a slope neighbour is covered at that level in the new
    //    hierarchy and holds data (not a hole before and after)
    for (int l = 0; l + 1 < nnlev; ++l) {
      Level3 &Cl = nl[l], &F = nl[l + 1];
      const int nzs = (F.fn[2] - 2 + r - 1) / r;
      const std::vector<RegridOp3> ops = par_collect<RegridOp3>((size_t)std::max(nzs, 0), [&](size_t iz, std::vector<RegridOp3> &out) {
        const int z = F.f0[2] + 1 + (int)iz * r;
        for (int y = F.f0[1] + 1; y < F.f0[1] + F.fn[1] - 1; y += r) {
          const uint8_t *fn = cov_row(nl, nnlev, l + 1, y, z), *fo = cov_row(c->lv, onlev, l + 1, y, z);
          for (int x = F.f0[0] + 1; x < F.f0[0] + F.fn[0] - 1; x += r) {
            if (!fn[x - F.f0[0]] || in_row(c->lv, l + 1, fo, x)) continue;
            const int q[3] = {x, y, z};
            const int P[3] = {x / r, y / r, z / r};
            RegridOp3 o{};
            o.dst = (int32_t)F.off(q);
            o.src = (int32_t)Cl.off(P);
            for (int d = 0; d < 6; ++d) {
              int nbq[3] = {P[0] + E3[d][0], P[1] + E3[d][1], P[2] + E3[d][2]};
              o.nb[d] = -1;
              if (!wrap_in(c->p, nl, l, nbq) || !new_cov(l, nbq)) continue;
              const int ch[3] = {nbq[0] * r, nbq[1] * r, nbq[2] * r};
              if (old_cov(l + 1, ch) && new_cov(l + 1, ch)) continue;  // a hole before and after
              o.nb[d] = (int32_t)Cl.off(nbq);
            }
            out.push_back(o);
          }
        }
      });
      if (ops.empty()) continue;
      RegridArgs3 a{};
      a.coarse_cur = Cl.buf[Cl.cur()];
      a.fine0 = F.buf[0];
      a.fine1 = F.buf[1];
      a.fplane = F.plane;
      a.fslab = F.slab;
      a.fpitch = F.pitch;
      a.cplane = Cl.plane;
      a.r = r;
      RegridOp3 *d = nullptr;
      st = upload_ops(ops, d);
      if (st) return st;
      a.ops = d;
      a.nops = (int32_t)ops.size();
      HIPCHK3(launch_split3(a, c->fp32, c->stream));
    }
    HIPCHK3(hipStreamSynchronize(c->stream));
    for (void *p : scratch) c->mem.release(p);
    scratch.clear();
    tm.mark("splits+sync");
    // 4. install the new hierarchy and rebuild its lists
    std::vector<int64_t> old_faces[kL];
    for (int l = 0; l < onlev; ++l) old_faces[l].swap(c->lv[l].face_key);
    for (int l = 0; l < kL; ++l) free_level3(c->mem, c->lv[l]);
    for (int l = 0; l < kL; ++l) c->lv[l] = std::move(nl[l]);
    c->nlev = nnlev;
    st = build_lists3(c);
    if (st) return st;
    tm.mark("lists");
    // 5. an interface that exists before and after keeps its reconstruction
    //    unmodified (Sec. 3.4); a face the regrid creates starts flat: the
    //    population its ring cell hands into the new hole gets the current
    //    value in the other buffer too
    for (int l = 0; l + 1 < c->nlev; ++l) {
      Level3 &N = c->lv[l];
      std::vector<int32_t> items;
      for (int64_t key : N.face_key) {
        if (std::binary_search(old_faces[l].begin(), old_faces[l].end(), key)) continue;
        const int64_t cell = key / 6;
        const int p[3] = {(int)(cell % N.N[0]), (int)(cell / N.N[0] % N.N[1]), (int)(cell / ((int64_t)N.N[0] * N.N[1]))};
        items.push_back((int32_t)N.off(p));
        items.push_back((int32_t)(key % 6));
      }
      if (items.empty()) continue;
      int32_t *d = nullptr;
      ALLOC3(d, sizeof(int32_t) * items.size());
      scratch.push_back(d);
      HIPCHK3(hipMemcpyAsync(d, items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice, c->stream));
      HIPCHK3(launch_restart_faces3(N.buf[N.cur()], N.buf[N.cur() ^ 1], d, (int)(items.size() / 2), N.plane,
                                    c->fp32, c->stream));
    }
    HIPCHK3(hipStreamSynchronize(c->stream));
    for (void *p : scratch) c->mem.release(p);
    for (int l = 0; l < c->nlev; ++l) {
      Level3 &L = c->lv[l];
      ALLOC3(L.dstatus, L.status.size());
      HIPCHK3(hipMemcpyAsync(L.dstatus, L.status.data(), L.status.size(), hipMemcpyHostToDevice, c->stream));
    }
    st = upload_lists3(c);
    if (st) return st;
    for (int l = 0; l < c->nlev; ++l)
      if (c->lv[l].nledger > 0) {
        HIPCHK3(hipMemcpy(c->lv[l].dledger, led, sizeof led, hipMemcpyHostToDevice));
        break;
      }
    c->boxes.assign(boxes, boxes + nboxes);
    st = build_tables3(c);
    tm.mark("faces+upload");
    return st;
  });
}

vlbm_status vlbm3_set_state(vlbm3_ctx *c, int level, int i0, int j0, int k0, int nx, int ny, int nz,
                            const double *U) {
  if (!U) return fail3(VLBM_EINVAL, "null U");
  const int lo[3] = {i0, j0, k0}, ext[3] = {nx, ny, nz};
  vlbm_status st = rect_io3(c, level, lo, ext, const_cast<double *>(U), 5, true, false);
  return st ? st : restart_count3(c);
}

vlbm_status vlbm3_set_populations(vlbm3_ctx *c, int level, int i0, int j0, int k0, int nx, int ny, int nz,
                                  const double *F) {
  if (!F) return fail3(VLBM_EINVAL, "null F");
  const int lo[3] = {i0, j0, k0}, ext[3] = {nx, ny, nz};
  vlbm_status st = rect_io3(c, level, lo, ext, const_cast<double *>(F), 30, true, true);
  return st ? st : restart_count3(c);
}

vlbm_status vlbm3_get_state(vlbm3_ctx *c, int level, int i0, int j0, int k0, int nx, int ny, int nz,
                            double *U) {
  if (!U) return fail3(VLBM_EINVAL, "null U");
  const int lo[3] = {i0, j0, k0}, ext[3] = {nx, ny, nz};
  return rect_io3(c, level, lo, ext, U, 5, false, false);
}

vlbm_status vlbm3_get_populations(vlbm3_ctx *c, int level, int i0, int j0, int k0, int nx, int ny, int nz,
                                  double *F) {
  if (!F) return fail3(VLBM_EINVAL, "null F");
  const int lo[3] = {i0, j0, k0}, ext[3] = {nx, ny, nz};
  return rect_io3(c, level, lo, ext, F, 30, false, false);
}

vlbm_status vlbm3_advance(vlbm3_ctx *c, int n) {
  if (!c || !c->have_hierarchy) return fail3(VLBM_ESTATE, "no hierarchy installed");
  if (n < 0) return fail3(VLBM_EINVAL, "negative step count");
  for (int i = 0; i < n; ++i) {
    vlbm_status st = coarse_step3(c);
    if (st) return st;
  }
  return VLBM_OK;
}

vlbm_status vlbm3_conserved_totals(vlbm3_ctx *c, double totals[5], double ledger[5]) {
  if (!c || !c->have_hierarchy) return fail3(VLBM_ESTATE, "no hierarchy installed");
  if (!totals) return fail3(VLBM_EINVAL, "null totals");
  double s[5] = {}, cs[5] = {}, ls[5] = {}, lc[5] = {};
  for (int l = 0; l < c->nlev; ++l) {
    Level3 &L = c->lv[l];
    const int nt = (int)L.tiles.size();
    HIPCHK3(launch_audit3(L.buf[L.cur()], L.dtiles, nt, L.plane, L.pitch, L.dpartial, c->fp32, c->stream));
    std::vector<double> part(5 * (size_t)std::max(nt, 1)), led(5 * (size_t)std::max(1, L.nledger));
    if (nt) HIPCHK3(hipMemcpyAsync(part.data(), L.dpartial, sizeof(double) * 5 * nt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(hipMemcpyAsync(led.data(), L.dledger, sizeof(double) * led.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK3(hipStreamSynchronize(c->stream));
    const double w3 = L.dx * L.dx * L.dx;
    for (int k = 0; k < 5; ++k) {
      double sl = 0.0, cl = 0.0;
      for (int t = 0; t < nt; ++t) kadd3(sl, cl, part[5 * (size_t)t + k]);
      kadd3(s[k], cs[k], w3 * (sl + cl));
      for (int t = 0; t < L.nledger; ++t) kadd3(ls[k], lc[k], led[5 * (size_t)t + k]);
    }
  }
  for (int k = 0; k < 5; ++k) {
    totals[k] = s[k] + cs[k];
    if (ledger) ledger[k] = ls[k] + lc[k];
  }
  return VLBM_OK;
}

vlbm_status vlbm3_set_tuning(vlbm3_ctx *c, int tile_cells, int flags) {
  if (!c) return fail3(VLBM_EINVAL, "null context");
  if (tile_cells < 64 || tile_cells > 65536 || (flags & ~S3_NT_STORES))
    return fail3(VLBM_EINVAL, "bad tuning (tile_cells %d, flags %d)", tile_cells, flags);
  c->tile_cells = tile_cells;
  c->flags = flags;
  if (!c->have_hierarchy) return VLBM_OK;
  HIPCHK3(hipStreamSynchronize(c->stream));
  // the accumulators hold nothing between coarse steps and the ledger is
  // carried through the rebuild
  double led[5] = {};
  vlbm_status st = ledger_sum3(c, led);
  if (st) return st;
  for (int l = 0; l < c->nlev; ++l) free_lists3(c->mem, c->lv[l]);
  st = guard3([&] { return build_lists3(c); });
  if (!st) st = upload_lists3(c);
  if (st) return st;
  // put the carried ledger into the first slot that exists
  for (int l = 0; l < c->nlev; ++l)
    if (c->lv[l].nledger > 0) {
      HIPCHK3(hipMemcpy(c->lv[l].dledger, led, sizeof led, hipMemcpyHostToDevice));
      break;
    }
  return build_tables3(c);  // descriptors for the current buffers
}

vlbm_status vlbm3_set_profiling(vlbm3_ctx *c, int enable) {
  if (!c) return fail3(VLBM_EINVAL, "null context");
  vlbm_status st = prof_flush3(c);
  if (st) return st;
  c->prof = enable != 0;
  if (c->prof)
    for (int i = 0; i < kL; ++i) {
      c->prof_ms[i] = 0.0;
      c->prof_calls[i] = 0;
      c->prof_cells[i] = 0.0;
    }
  return VLBM_OK;
}

vlbm_status vlbm3_kernel_times(vlbm3_ctx *c, double *ms, long *calls, double *cells) {
  if (!c || !ms || !calls || !cells) return fail3(VLBM_EINVAL, "null argument");
  vlbm_status st = prof_flush3(c);
  if (st) return st;
  for (int i = 0; i < kL; ++i) {
    ms[i] = c->prof_ms[i];
    calls[i] = c->prof_calls[i];
    cells[i] = c->prof_cells[i];
  }
  return VLBM_OK;
}

vlbm_status vlbm3_tag(vlbm3_ctx *c, int level, double threshold, unsigned char *tags) {
  if (!c || !tags) return fail3(VLBM_EINVAL, "null argument");
  if (!c->have_hierarchy) return fail3(VLBM_ESTATE, "no hierarchy installed");
  if (level < 0 || level >= kL) return fail3(VLBM_EINVAL, "bad level");
  const Level3 &L = c->lv[level];
  const size_t nall = (size_t)L.N[0] * L.N[1] * L.N[2];
  if (level < c->nlev && L.present) {
    TagMap3 T;
    vlbm_status st = tag_frame3(c, level, threshold, T);
    if (st) return st;
    memset(tags, 0, nall);
    for (int z = 0; z < L.N[2]; ++z)
      for (int y = 0; y < L.N[1]; ++y)
        for (int x = 0; x < L.N[0]; ++x) {
          const int p[3] = {x, y, z};
          if (L.in_frame(p)) tags[((size_t)z * L.N[1] + y) * L.N[0] + x] = T.t[L.fidx(p)];
        }
  } else {
    long s = 1;
    for (int i = 0; i < level; ++i) s *= c->p.r;
    memset(tags, 0, (size_t)c->p.nx0 * s * c->p.ny0 * s * c->p.nz0 * s);
  }
  return VLBM_OK;
}

vlbm_status vlbm3_tag_and_regrid(vlbm3_ctx *c, double threshold, int buffer, int min_box, int max_box) {
  return guard3([&]() -> vlbm_status {
    if (!c) return fail3(VLBM_EINVAL, "null context");
    if (!c->have_hierarchy) return fail3(VLBM_ESTATE, "no hierarchy installed");
    if (buffer < 0 || min_box < 1 || max_box < min_box) return fail3(VLBM_EINVAL, "bad clustering sizes");
    const int ML = c->p.max_levels;
    if (ML < 2) return VLBM_OK;
    PhaseTimer tm("tag_and_regrid3");
    std::vector<TagMap3> tags(ML);
    for (int l = 0; l < c->nlev; ++l) {
      if (!c->lv[l].present) continue;
      vlbm_status st = tag_frame3(c, l, threshold, tags[l]);
      if (st) return st;
    }
    tm.mark("tags");
    std::vector<vlbm3_box> boxes;
    cluster_hierarchy3(c, tags, buffer, min_box, max_box, boxes);
    tm.mark("cluster");
    return vlbm3_regrid(c, boxes.data(), (int)boxes.size());
  });
}

vlbm_status vlbm3_get_boxes(vlbm3_ctx *c, vlbm3_box *boxes, int cap, int *nboxes) {
  if (!c || !nboxes || cap < 0 || (cap > 0 && !boxes)) return fail3(VLBM_EINVAL, "bad argument");
  *nboxes = (int)c->boxes.size();
  for (int i = 0; i < std::min(cap, *nboxes); ++i) boxes[i] = c->boxes[i];
  return VLBM_OK;
}

// Checkpoint: header, boxes, per present level {step count, both buffers}.
// The reflux accumulators hold nothing between coarse steps, and the
// boundary ledger is kept as its five totals, so a checkpoint loads under any
// launch tuning.
struct Ckpt3Header {
  char magic[8];
  vlbm3_params p;
  int32_t nboxes, nlev;
  int64_t coarse_steps;
  double ledger[5];
};

vlbm_status vlbm3_save(vlbm3_ctx *c, void *buf, size_t *bytes) {
  if (!c || !bytes) return fail3(VLBM_EINVAL, "null argument");
  if (!c->have_hierarchy) return fail3(VLBM_ESTATE, "nothing to save");
  size_t need = sizeof(Ckpt3Header) + sizeof(vlbm3_box) * c->boxes.size();
  for (int l = 0; l < c->nlev; ++l) need += sizeof(int64_t) + 2 * level_bytes3(c->lv[l]);
  if (!buf) {
    *bytes = need;
    return VLBM_OK;
  }
  if (*bytes < need) return fail3(VLBM_EINVAL, "checkpoint buffer too small (%zu < %zu)", *bytes, need);
  Ckpt3Header h{};
  memcpy(h.magic, "VLBM3C1", 8);
  h.p = c->p;
  h.nboxes = (int32_t)c->boxes.size();
  h.nlev = c->nlev;
  h.coarse_steps = c->coarse_steps;
  double tot[5];
  vlbm_status st = vlbm3_conserved_totals(c, tot, h.ledger);
  if (st) return st;
  char *p = static_cast<char *>(buf);
  memcpy(p, &h, sizeof h);
  p += sizeof h;
  memcpy(p, c->boxes.data(), sizeof(vlbm3_box) * c->boxes.size());
  p += sizeof(vlbm3_box) * c->boxes.size();
  for (int l = 0; l < c->nlev; ++l) {
    const Level3 &L = c->lv[l];
    const int64_t steps = L.steps;
    memcpy(p, &steps, sizeof steps);
    p += sizeof steps;
    const size_t nb = level_bytes3(L);
    for (int b = 0; b < 2; ++b) {
      HIPCHK3(hipMemcpyAsync(p, L.buf[b], nb, hipMemcpyDeviceToHost, c->stream));
      p += nb;
    }
  }
  HIPCHK3(hipStreamSynchronize(c->stream));
  *bytes = need;
  return VLBM_OK;
}

vlbm_status vlbm3_load(vlbm3_ctx *c, const void *buf, size_t bytes) {
  if (!c || !buf || bytes < sizeof(Ckpt3Header)) return fail3(VLBM_EINVAL, "bad checkpoint");
  const char *p = static_cast<const char *>(buf);
  Ckpt3Header h;
  memcpy(&h, p, sizeof h);
  p += sizeof h;
  if (memcmp(h.magic, "VLBM3C1", 8) != 0) return fail3(VLBM_EINVAL, "not a 3-D checkpoint");
  {
    const vlbm3_params &a = h.p, &b = c->p;
    bool same = a.nx0 == b.nx0 && a.ny0 == b.ny0 && a.nz0 == b.nz0 && a.dx0 == b.dx0 && a.gamma == b.gamma &&
                a.c == b.c && a.beta == b.beta && a.r == b.r && a.max_levels == b.max_levels &&
                a.precision == b.precision;
    for (int s2 = 0; s2 < 6; ++s2) same = same && a.bc[s2] == b.bc[s2];
    if (!same) return fail3(VLBM_EINVAL, "checkpoint parameters differ from the context's");
  }
  if (h.nboxes < 0 || sizeof h + sizeof(vlbm3_box) * (size_t)h.nboxes > bytes)
    return fail3(VLBM_EINVAL, "truncated checkpoint");
  std::vector<vlbm3_box> boxes(h.nboxes);
  memcpy(boxes.data(), p, sizeof(vlbm3_box) * h.nboxes);
  p += sizeof(vlbm3_box) * h.nboxes;
  vlbm_status st = vlbm3_set_hierarchy(c, boxes.data(), h.nboxes);
  if (st) return st;
  if (c->nlev != h.nlev) return fail3(VLBM_EINVAL, "checkpoint level count mismatch");
  for (int l = 0; l < c->nlev; ++l) {
    Level3 &L = c->lv[l];
    const size_t nb = level_bytes3(L);
    if ((size_t)(p - static_cast<const char *>(buf)) + sizeof(int64_t) + 2 * nb > bytes)
      return fail3(VLBM_EINVAL, "truncated checkpoint");
    int64_t steps;
    memcpy(&steps, p, sizeof steps);
    p += sizeof steps;
    L.steps = steps;
    for (int b = 0; b < 2; ++b) {
      HIPCHK3(hipMemcpyAsync(L.buf[b], p, nb, hipMemcpyHostToDevice, c->stream));
      p += nb;
    }
  }
  // the ledger totals into the first slot that exists (the others start at 0)
  for (int l = 0; l < c->nlev; ++l)
    if (c->lv[l].nledger > 0) {
      HIPCHK3(hipMemcpyAsync(c->lv[l].dledger, h.ledger, sizeof h.ledger, hipMemcpyHostToDevice, c->stream));
      break;
    }
  HIPCHK3(hipStreamSynchronize(c->stream));
  c->coarse_steps = h.coarse_steps;
  return build_tables3(c);
}

long vlbm3_active_cells(const vlbm3_ctx *c, int level) {
  if (!c || !c->have_hierarchy || level < 0 || level >= kL || !c->lv[level].present) return 0;
  long n = 0;
  for (const Tile3 &t : c->lv[level].tiles) n += (long)t.w * t.h;
  return n;
}

vlbm_status vlbm3_sync(vlbm3_ctx *c) {
  if (!c) return fail3(VLBM_EINVAL, "null context");
  HIPCHK3(hipStreamSynchronize(c->stream));
  return VLBM_OK;
}

}  // extern "C"
