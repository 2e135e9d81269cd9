// Host-only check of the 3-D hierarchy code (built with AddressSanitizer by
// tests/test_host_lists.py; no GPU): synthetic tag maps (a spherical shell, a
// plane across the periodic seam, sparse random cells) are clustered into
// level-1 boxes, which must be accepted by the hierarchy builder (nesting),
// cover every tag dilated by the buffer and respect max_box; the tile and
// task lists of the new hierarchy are built on worker threads and must cover
// every active cell exactly once. The device launchers are stubs that are
// never reached.
#include "../../paper_2609_35529_amd/csrc/api3.hip"
#include <cstdio>
#include <random>
#include <string>

namespace vlbm {
static std::string g_last;
void set_error_message(const char *msg) { g_last = msg; }
}  // namespace vlbm
extern "C" const char *vlbm_last_error(void) { return vlbm::g_last.c_str(); }
namespace vlbm {
}  // namespace vlbm
namespace vlbm3 {
hipError_t launch_step3(const Launch3 &, hipStream_t, hipEvent_t, hipEvent_t) { return hipErrorUnknown; }
hipError_t launch_audit3(const void *, const Tile3 *, int, int64_t, int, double *, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_set3(const Rect3 &, int, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_get3(const Rect3 &, int, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_merge3(const RegridArgs3 &, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_split3(const RegridArgs3 &, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_copy3_runs(const void *, const void *, void *, void *, const int32_t *, int, int64_t, int64_t, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_restart_faces3(const void *, void *, const int32_t *, int, int64_t, int, hipStream_t) { return hipErrorUnknown; }
hipError_t launch_tag3(const Tag3Args &, int, hipStream_t) { return hipErrorUnknown; }
}  // namespace vlbm3

using namespace vlbm3;

static int run(int nx, int ny, int nz, int ML, int per, int buffer, int minb, int maxb, int seed, int shape) {
  vlbm3_params p{};
  p.nx0 = nx; p.ny0 = ny; p.nz0 = nz; p.dx0 = 1.0 / nx; p.r = 2; p.max_levels = ML; p.c = 4; p.beta = 0.5; p.gamma = 1.4;
  for (int s = 0; s < 6; ++s) p.bc[s] = per ? 0 : 1;
  vlbm3_ctx *c = new vlbm3_ctx();
  c->p = p;
  // level 0 only, frames from a geometry with no boxes
  int nlev = 1;
  if (build_geometry3(p, nullptr, 0, c->lv, nlev)) { printf("geom fail\n"); return 1; }
  c->nlev = nlev;
  std::vector<TagMap3> tags(ML);
  const Level3 &L = c->lv[0];
  for (int a = 0; a < 3; ++a) { tags[0].o[a] = L.f0[a]; tags[0].n[a] = L.fn[a]; }
  tags[0].t.assign((size_t)L.fn[0] * L.fn[1] * L.fn[2], 0);
  std::mt19937 rng(seed);
  std::vector<std::array<int, 3>> tagged;
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        bool t = false;
        if (shape == 0) {  // spherical shell
          double dx = x - nx * 0.5, dy = y - ny * 0.4, dz = z - nz * 0.6, rr = sqrt(dx * dx + dy * dy + dz * dz);
          t = fabs(rr - nx * 0.25) < 1.0;
        } else if (shape == 1) {  // a plane across the periodic seam
          t = x == 0 || x == nx - 1;
        } else {  // random sparse
          t = (rng() % 97) == 0;
        }
        if (t) { tags[0].at(x, y, z) = 1; tagged.push_back({x, y, z}); }
      }
  std::vector<vlbm3_box> boxes;
  cluster_hierarchy3(c, tags, buffer, minb, maxb, boxes);
  // accepted by the hierarchy builder
  Level3 nl[kL];
  int nn = 1;
  vlbm_status st = build_geometry3(p, boxes.data(), (int)boxes.size(), nl, nn);
  if (st) { printf("  REJECTED: %s\n", vlbm::g_last.c_str()); return 1; }
  vlbm3_ctx *t = new vlbm3_ctx();
  t->p = p;
  t->nlev = nn;
  t->tile_cells = 256;
  for (int l = 0; l < kL; ++l) t->lv[l] = std::move(nl[l]);
  if (build_lists3(t)) { printf("  LISTS FAILED: %s\n", vlbm::g_last.c_str()); return 1; }
  for (int l = 0; l < nn; ++l) {
    const Level3 &L = t->lv[l];
    std::vector<int> hit(L.status.size(), 0);
    for (const Tile3 &tl : L.tiles) {
      const int64_t rel = tl.off0 - L.xoff;
      const int fz = (int)(rel / L.slab), fy = (int)((rel - (int64_t)fz * L.slab) / L.pitch);
      const int fx = (int)(rel - (int64_t)fz * L.slab - (int64_t)fy * L.pitch);
      for (int cy = 0; cy < tl.h; ++cy)
        for (int cx = 0; cx < tl.w; ++cx) hit[((size_t)fz * L.fn[1] + fy + cy) * L.fn[0] + fx + cx] += 1;
    }
    for (size_t i = 0; i < hit.size(); ++i)
      if (hit[i] != (L.status[i] == 1 ? 1 : 0)) { printf("  TILES DO NOT COVER level %d\n", l); return 1; }
  }
  delete t;
  // every dilated tag (within buffer per axis, Chebyshev) is covered at level 1
  std::vector<uint8_t> cov1((size_t)nx * ny * nz, 0);
  for (auto &b : boxes)
    if (b.level == 1)
      for (int z = b.k0 / 2; z < (b.k0 + b.nz) / 2; ++z)
        for (int y = b.j0 / 2; y < (b.j0 + b.ny) / 2; ++y)
          for (int x = b.i0 / 2; x < (b.i0 + b.nx) / 2; ++x) cov1[((size_t)z * ny + y) * nx + x] = 1;
  long miss = 0, total = 0;
  for (auto &t : tagged)
    for (int dz = -buffer; dz <= buffer; ++dz)
      for (int dy = -buffer; dy <= buffer; ++dy)
        for (int dx = -buffer; dx <= buffer; ++dx) {
          int q[3] = {t[0] + dx, t[1] + dy, t[2] + dz}, n[3] = {nx, ny, nz};
          bool in = true;
          for (int a = 0; a < 3; ++a)
            if (q[a] < 0 || q[a] >= n[a]) {
              if (per) q[a] = (q[a] + n[a]) % n[a]; else in = false;
            }
          if (!in) continue;
          ++total;
          if (!cov1[((size_t)q[2] * ny + q[1]) * nx + q[0]]) ++miss;
        }
  int maxext = 0;
  for (auto &b : boxes) maxext = std::max({maxext, b.nx, b.ny, b.nz});
  printf("  shape %d per %d: %zu tagged, %zu boxes, max extent %d (max_box %d), uncovered dilated %ld of %ld\n", shape,
         per, tagged.size(), boxes.size(), maxext, maxb, miss, total);
  return miss != 0 || maxext > maxb;
}

int main() {
  int bad = 0;
  for (int shape = 0; shape < 3; ++shape)
    for (int per = 0; per < 2; ++per) bad |= run(40, 36, 32, 2, per, 2, 8, 32, shape + 7, shape);
  bad |= run(48, 48, 48, 3, 1, 1, 4, 16, 3, 0);
  printf(bad ? "FAIL\n" : "ok\n");
  return bad;
}
