// Drives the host tessellation stage through its C interface on random,
// degenerate and invalid inputs; built together with the stage under
// AddressSanitizer and UndefinedBehaviorSanitizer, so any out-of-bounds
// access, leak, use after free, overflow or misaligned access aborts it.
// Every mesh is also checked for the partition identity (cell areas sum to
// the box area) so that the run does real work on every path.
#include "rich_tess.h"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

static uint64_t g_state = 0x9e3779b97f4a7c15ull;
static double uni() {  // splitmix64 -> [0, 1)
  uint64_t z = (g_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (z >> 11) * (1.0 / 9007199254740992.0);
}

static int g_fail = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      g_fail = 1;                                                       \
    }                                                                   \
  } while (0)

static void build_and_check(const std::vector<double>& x, const std::vector<double>& y,
                            const double box[4], uint32_t bc, int threads, const char* what) {
  rich_mesh_host m{};
  int st = rich_tess_build(x.data(), y.data(), (int64_t)x.size(), box, bc, threads, &m);
  if (st != 0) {
    std::fprintf(stderr, "%s: status %d\n", what, st);
    g_fail = 1;
    return;
  }
  double a = 0.0;
  for (int64_t i = 0; i < m.n_cells; ++i) a += m.area[i];
  double want = (box[2] - box[0]) * (box[3] - box[1]);
  CHECK(std::fabs(a - want) < 1e-10 * want);
  CHECK(m.off[m.n_cells] == m.n_csr && m.eoff[m.n_cells] == m.n_edges);
  for (int64_t k = 0; k < m.n_csr; ++k) CHECK(m.idx[k] >= 0 && m.idx[k] < 2 * m.n_edges);
  std::printf("%-28s n=%lld edges=%lld ok\n", what, (long long)m.n_cells, (long long)m.n_edges);
  rich_tess_free(&m);
}

int main() {
  const double unit[4] = {0.0, 0.0, 1.0, 1.0};
  const double rect[4] = {-1.0, 0.5, 2.0, 1.5};
  for (uint32_t bc = 0; bc < 2; ++bc) {
    for (int n : {1, 2, 3, 7, 2000}) {
      std::vector<double> x(n), y(n);
      for (int i = 0; i < n; ++i) {
        x[i] = 0.001 + 0.998 * uni();
        y[i] = 0.001 + 0.998 * uni();
      }
      build_and_check(x, y, unit, bc, n > 100 ? 4 : 1, bc ? "random periodic" : "random walls");
    }
    // square lattice (co-circular quadruples everywhere) in a rectangle
    std::vector<double> x, y;
    for (int j = 0; j < 17; ++j)
      for (int i = 0; i < 40; ++i) {
        x.push_back(rect[0] + (i + 0.5) * 3.0 / 40);
        y.push_back(rect[1] + (j + 0.5) / 17.0);
      }
    build_and_check(x, y, rect, bc, 2, "square lattice");
    // points hugging the walls
    x.clear();
    y.clear();
    for (int i = 0; i < 500; ++i) {
      double t = uni();
      x.push_back(i % 2 ? 1e-9 + 1e-9 * t : 1.0 - 1e-9 - 1e-9 * t);
      y.push_back(0.001 + 0.998 * uni());
    }
    build_and_check(x, y, unit, bc, 3, "near walls");
  }
  // the step adapter: several meshes in flight, released out of order
  rich_tess_ctx* ctx = rich_tess_ctx_create(2);
  std::vector<double> x(300), y(300);
  for (int i = 0; i < 300; ++i) {
    x[i] = uni();
    y[i] = uni();
  }
  rich_tess_view v[3];
  for (auto& w : v) CHECK(rich_tess_callback(ctx, x.data(), y.data(), 300, unit, 1, &w) == 0);
  rich_tess_release(ctx, &v[1]);
  rich_tess_release(ctx, &v[0]);
  rich_tess_release(ctx, &v[2]);
  rich_tess_ctx_destroy(ctx);
  // Lloyd, triangles, Hilbert order
  CHECK(rich_tess_lloyd(x.data(), y.data(), 300, unit, 1, 3, 2) == 0);
  rich_tri_host t{};
  CHECK(rich_tess_triangles(x.data(), y.data(), 300, unit, 0, &t) == 0);
  for (int64_t k = 0; k < 3 * t.n_tri; ++k) CHECK(t.tri[k] >= 0 && t.tri[k] < t.n_pts);
  rich_tess_free_tri(&t);
  std::vector<int64_t> perm(300);
  CHECK(rich_tess_hilbert_order(x.data(), y.data(), 300, unit, perm.data()) == 0);
  // invalid inputs: each must be refused with a negative status and a zeroed mesh
  rich_mesh_host m{};
  std::vector<double> bx = {0.5, 1.5}, by = {0.5, 0.5};
  CHECK(rich_tess_build(bx.data(), by.data(), 2, unit, 0, 1, &m) < 0 && m.area == nullptr);
  bx = {0.5, NAN};
  CHECK(rich_tess_build(bx.data(), by.data(), 2, unit, 1, 1, &m) < 0 && m.area == nullptr);
  CHECK(rich_tess_build(bx.data(), by.data(), 0, unit, 0, 1, &m) < 0);
  const double flat[4] = {0.0, 0.0, 1.0, 0.0};
  bx = {0.5, 0.25};
  CHECK(rich_tess_build(bx.data(), by.data(), 2, flat, 0, 1, &m) < 0);
  rich_tess_free(&m);
  std::printf(g_fail ? "FAILED\n" : "ALL OK\n");
  return g_fail;
}
