// Host input stage: Delaunay triangulation by point insertion with exact
// predicates, Voronoi diagram read off the triangulation, ghost points for
// reflecting walls and periodic boxes, and the flat mesh arrays (cells, edges,
// CSR) consumed by the device path and by the oracle.
//
// Paper section 2.1 ("Tessellation Creation") describes the method: points are
// inserted one after another, each insertion checks which triangles have the
// new point inside their circumcircle, and the orientation / in-circle signs
// are computed exactly whenever round-off could change them (adaptive
// arithmetic: a floating-point evaluation with a rigorous error bound, and an
// exact evaluation with floating-point expansions only when the bound cannot
// decide).  The Voronoi diagram is then obtained from the triangulation in
// linear time.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared -pthread.  The
// exact arithmetic relies on IEEE double rounding with no contraction of
// a*b+c into a fused multiply-add and no reassociation.

#include "rich_tess.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Exact arithmetic on floating-point expansions.
//
// An expansion is a sum of doubles whose components do not overlap and are
// stored in increasing order of magnitude; its sign is the sign of its last
// (largest) nonzero component.  The error-free transformations below are the
// classical ones: the sum a+b and the product a*b are each represented exactly
// by a rounded result plus an error term (Knuth's two-sum; Dekker's product
// with Veltkamp splitting).
// ---------------------------------------------------------------------------

constexpr double kEps = 1.1102230246251565e-16;  // 2^-53, unit round-off
constexpr double kSplitter = 134217729.0;        // 2^27 + 1

inline void two_sum(double a, double b, double& x, double& y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}

inline void split(double a, double& hi, double& lo) {
  double c = kSplitter * a;
  double big = c - a;
  hi = c - big;
  lo = a - hi;
}

inline void two_prod(double a, double b, double& x, double& y) {
  x = a * b;
  double ahi, alo, bhi, blo;
  split(a, ahi, alo);
  split(b, bhi, blo);
  double e1 = x - ahi * bhi;
  double e2 = e1 - alo * bhi;
  double e3 = e2 - ahi * blo;
  y = alo * blo - e3;
}

using Exp = std::vector<double>;

// h = e + b, zero components removed.
void exp_grow(const Exp& e, double b, Exp& h) {
  h.clear();
  double q = b;
  for (double ek : e) {
    double qn, r;
    two_sum(q, ek, qn, r);
    if (r != 0.0) h.push_back(r);
    q = qn;
  }
  if (q != 0.0 || h.empty()) h.push_back(q);
}

// h = e + f
void exp_add(const Exp& e, const Exp& f, Exp& h) {
  Exp cur = e, tmp;
  for (double fk : f) {
    exp_grow(cur, fk, tmp);
    cur.swap(tmp);
  }
  h.swap(cur);
}

// h = e * b
void exp_scale(const Exp& e, double b, Exp& h) {
  h.clear();
  double q, r;
  two_prod(e[0], b, q, r);
  if (r != 0.0) h.push_back(r);
  for (size_t i = 1; i < e.size(); ++i) {
    double big, small;
    two_prod(e[i], b, big, small);
    double q2, r1;
    two_sum(q, small, q2, r1);
    if (r1 != 0.0) h.push_back(r1);
    double q3, r2;
    two_sum(big, q2, q3, r2);
    if (r2 != 0.0) h.push_back(r2);
    q = q3;
  }
  if (q != 0.0 || h.empty()) h.push_back(q);
}

// h = e * f
void exp_mul(const Exp& e, const Exp& f, Exp& h) {
  Exp acc{0.0}, part, tmp;
  for (double fk : f) {
    if (fk == 0.0) continue;
    exp_scale(e, fk, part);
    exp_add(acc, part, tmp);
    acc.swap(tmp);
  }
  h.swap(acc);
}

Exp exp_neg(const Exp& e) {
  Exp r(e);
  for (double& v : r) v = -v;
  return r;
}

int exp_sign(const Exp& e) {
  for (size_t i = e.size(); i-- > 0;) {
    if (e[i] > 0.0) return 1;
    if (e[i] < 0.0) return -1;
  }
  return 0;
}

// exact difference a - b as an expansion
Exp exp_diff(double a, double b) {
  double x, y;
  two_sum(a, -b, x, y);
  Exp r;
  if (y != 0.0) r.push_back(y);
  r.push_back(x);
  return r;
}

int orient_exact(double ax, double ay, double bx, double by, double cx, double cy) {
  Exp acx = exp_diff(ax, cx), bcy = exp_diff(by, cy);
  Exp acy = exp_diff(ay, cy), bcx = exp_diff(bx, cx);
  Exp l, r, d;
  exp_mul(acx, bcy, l);
  exp_mul(acy, bcx, r);
  exp_add(l, exp_neg(r), d);
  return exp_sign(d);
}

int incircle_exact(double ax, double ay, double bx, double by, double cx,
                   double cy, double dx, double dy) {
  Exp adx = exp_diff(ax, dx), ady = exp_diff(ay, dy);
  Exp bdx = exp_diff(bx, dx), bdy = exp_diff(by, dy);
  Exp cdx = exp_diff(cx, dx), cdy = exp_diff(cy, dy);
  auto lift = [](const Exp& u, const Exp& v) {
    Exp uu, vv, s;
    exp_mul(u, u, uu);
    exp_mul(v, v, vv);
    exp_add(uu, vv, s);
    return s;
  };
  auto cross = [](const Exp& u1, const Exp& v2, const Exp& u2, const Exp& v1) {
    // u1*v2 - u2*v1
    Exp p, q, s;
    exp_mul(u1, v2, p);
    exp_mul(u2, v1, q);
    exp_add(p, exp_neg(q), s);
    return s;
  };
  Exp al = lift(adx, ady), bl = lift(bdx, bdy), cl = lift(cdx, cdy);
  Exp t1, t2, t3, s12, det;
  exp_mul(al, cross(bdx, cdy, cdx, bdy), t1);
  exp_mul(bl, cross(cdx, ady, adx, cdy), t2);
  exp_mul(cl, cross(adx, bdy, bdx, ady), t3);
  exp_add(t1, t2, s12);
  exp_add(s12, t3, det);
  return exp_sign(det);
}

// Error bounds of the floating-point evaluations (derived in the comments of
// orient() and incircle()); generous constants only cost extra exact calls.
constexpr double kOrientBound = 5.0 * kEps;
constexpr double kInCircleBound = 16.0 * kEps;

// Each of the two products carries at most ~3 eps relative error (two
// rounded differences and one rounded product), the final difference one
// more eps of the result, which is bounded by |l| + |r|.
inline int orient(double ax, double ay, double bx, double by, double cx,
                  double cy, int64_t* n_exact) {
  double l = (ax - cx) * (by - cy);
  double r = (ay - cy) * (bx - cx);
  double det = l - r;
  double bound = kOrientBound * (std::fabs(l) + std::fabs(r));
  if (det > bound) return 1;
  if (-det > bound) return -1;
  ++*n_exact;
  return orient_exact(ax, ay, bx, by, cx, cy);
}

// Lifted terms carry ~4 eps, the 2x2 minors ~4 eps of their permanent, the
// products ~9 eps and the two final sums 2 eps of the permanent: 11 eps in
// total to first order.
inline int incircle(double ax, double ay, double bx, double by, double cx,
                    double cy, double dx, double dy, int64_t* n_exact) {
  double adx = ax - dx, ady = ay - dy;
  double bdx = bx - dx, bdy = by - dy;
  double cdx = cx - dx, cdy = cy - dy;
  double bc1 = bdx * cdy, bc2 = cdx * bdy;
  double ca1 = cdx * ady, ca2 = adx * cdy;
  double ab1 = adx * bdy, ab2 = bdx * ady;
  double al = adx * adx + ady * ady;
  double bl = bdx * bdx + bdy * bdy;
  double cl = cdx * cdx + cdy * cdy;
  double det = al * (bc1 - bc2) + bl * (ca1 - ca2) + cl * (ab1 - ab2);
  double perm = (std::fabs(bc1) + std::fabs(bc2)) * al +
                (std::fabs(ca1) + std::fabs(ca2)) * bl +
                (std::fabs(ab1) + std::fabs(ab2)) * cl;
  double bound = kInCircleBound * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  ++*n_exact;
  return incircle_exact(ax, ay, bx, by, cx, cy, dx, dy);
}

// ---------------------------------------------------------------------------
// Hilbert curve index of a point of a 2^16 x 2^16 grid (the classical
// quadrant-recursive construction: at each level the quadrant number is
// appended and the coordinates are rotated / reflected into the sub-square's
// canonical orientation).
// ---------------------------------------------------------------------------
uint64_t hilbert_index(uint32_t x, uint32_t y) {
  const uint32_t n = 1u << 16;
  uint64_t d = 0;
  for (uint32_t s = n >> 1; s > 0; s >>= 1) {
    uint32_t rx = (x & s) ? 1u : 0u;
    uint32_t ry = (y & s) ? 1u : 0u;
    d += static_cast<uint64_t>(s) * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - (x & (s - 1));
        y = s - 1 - (y & (s - 1));
      } else {
        x &= (s - 1);
        y &= (s - 1);
      }
      std::swap(x, y);
    } else {
      x &= (s - 1);
      y &= (s - 1);
    }
  }
  return d;
}

uint32_t grid_coord(double v, double lo, double hi) {
  double t = (v - lo) / (hi - lo);
  if (!(t > 0.0)) t = 0.0;
  if (t >= 1.0) t = 1.0 - 1e-16;
  return static_cast<uint32_t>(t * 65536.0);
}

void hilbert_sort(const double* x, const double* y, int64_t n, double x0,
                  double y0, double x1, double y1, std::vector<int64_t>& perm) {
  std::vector<std::pair<uint64_t, int64_t>> keys(n);
  for (int64_t i = 0; i < n; ++i)
    keys[i] = {hilbert_index(grid_coord(x[i], x0, x1), grid_coord(y[i], y0, y1)), i};
  std::sort(keys.begin(), keys.end());
  perm.resize(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = keys[i].second;
}

// ---------------------------------------------------------------------------
// Incremental Delaunay triangulation with edge flips.
//
// Triangles are stored counter-clockwise; tn[3t+k] is the triangle across the
// edge opposite vertex tv[3t+k] (-1 if none).  Three far "super" vertices
// enclose all points, so every inserted point falls strictly inside.
// ---------------------------------------------------------------------------
struct Delaunay {
  std::vector<double> X, Y;
  std::vector<int32_t> tv, tn;
  int32_t ntri = 0;
  int32_t last = 0;
  int32_t nsuper0 = 0;  // index of the first super vertex
  int64_t n_exact = 0;
  std::vector<std::pair<int32_t, int32_t>> stack;

  int o(int a, int b, int c) {
    return orient(X[a], Y[a], X[b], Y[b], X[c], Y[c], &n_exact);
  }
  int ic(int a, int b, int c, int d) {
    return incircle(X[a], Y[a], X[b], Y[b], X[c], Y[c], X[d], Y[d], &n_exact);
  }

  int32_t new_tri(int a, int b, int c, int na, int nb, int nc) {
    int32_t t = ntri++;
    tv[3 * t] = a; tv[3 * t + 1] = b; tv[3 * t + 2] = c;
    tn[3 * t] = na; tn[3 * t + 1] = nb; tn[3 * t + 2] = nc;
    return t;
  }
  void set_tri(int32_t t, int a, int b, int c, int na, int nb, int nc) {
    tv[3 * t] = a; tv[3 * t + 1] = b; tv[3 * t + 2] = c;
    tn[3 * t] = na; tn[3 * t + 1] = nb; tn[3 * t + 2] = nc;
  }
  void replace_nb(int32_t t, int32_t old_n, int32_t new_n) {
    if (t < 0) return;
    for (int k = 0; k < 3; ++k)
      if (tn[3 * t + k] == old_n) { tn[3 * t + k] = new_n; return; }
  }

  // Triangle containing point p (inside or on its boundary): visibility walk.
  int32_t locate(int p) {
    int32_t t = last;
    int rot = 0;
    int64_t steps = 0;
    const int64_t limit = 4 * static_cast<int64_t>(ntri) + 64;
    while (true) {
      int moved = -1;
      for (int s = 0; s < 3; ++s) {
        int k = (s + rot) % 3;
        int a = tv[3 * t + (k + 1) % 3], b = tv[3 * t + (k + 2) % 3];
        if (o(a, b, p) < 0) { moved = k; break; }
      }
      if (moved < 0) return t;
      t = tn[3 * t + moved];
      rot = (rot + 1) % 3;
      if (t < 0 || ++steps > limit) break;
    }
    // Fallback (never expected): scan all triangles.
    for (int32_t u = 0; u < ntri; ++u) {
      int a = tv[3 * u], b = tv[3 * u + 1], c = tv[3 * u + 2];
      if (o(b, c, p) >= 0 && o(c, a, p) >= 0 && o(a, b, p) >= 0) return u;
    }
    return -1;
  }

  // Restore the Delaunay property around the new point p.  Stack entries are
  // (triangle, index of p in it); the edge opposite p is tested against the
  // vertex of the neighbouring triangle across it, and flipped if that vertex
  // lies inside the circumcircle.
  void legalize() {
    while (!stack.empty()) {
      auto [t, k] = stack.back();
      stack.pop_back();
      int p = tv[3 * t + k];
      int a = tv[3 * t + (k + 1) % 3], b = tv[3 * t + (k + 2) % 3];
      int32_t u = tn[3 * t + k];
      if (u < 0) continue;
      int m = 0;
      while (m < 3 && tn[3 * u + m] != t) ++m;
      if (m == 3) continue;  // inconsistent adjacency (not expected)
      int d = tv[3 * u + m];
      if (ic(p, a, b, d) <= 0) continue;
      int32_t n_bp = tn[3 * t + (k + 1) % 3];
      int32_t n_pa = tn[3 * t + (k + 2) % 3];
      int32_t n_ad = tn[3 * u + (m + 1) % 3];
      int32_t n_db = tn[3 * u + (m + 2) % 3];
      set_tri(t, p, a, d, n_ad, u, n_pa);
      set_tri(u, p, d, b, n_db, n_bp, t);
      replace_nb(n_ad, u, t);
      replace_nb(n_bp, t, u);
      stack.push_back({t, 0});
      stack.push_back({u, 0});
    }
  }

  // Returns 0 on success, -1 for a duplicate point or location failure.
  int insert(int p) {
    int32_t t = locate(p);
    if (t < 0) return -1;
    int v0 = tv[3 * t], v1 = tv[3 * t + 1], v2 = tv[3 * t + 2];
    int oo[3] = {o(v1, v2, p), o(v2, v0, p), o(v0, v1, p)};
    int nz = (oo[0] == 0) + (oo[1] == 0) + (oo[2] == 0);
    if (nz >= 2) return -1;  // coincides with a vertex
    if (nz == 0) {
      int32_t n0 = tn[3 * t], n1 = tn[3 * t + 1], n2 = tn[3 * t + 2];
      int32_t t1 = ntri, t2 = ntri + 1;
      set_tri(t, p, v1, v2, n0, t1, t2);
      new_tri(v0, p, v2, t, n1, t2);
      new_tri(v0, v1, p, t, t1, n2);
      replace_nb(n1, t, t1);
      replace_nb(n2, t, t2);
      stack.push_back({t, 0});
      stack.push_back({t1, 1});
      stack.push_back({t2, 2});
      last = t2;
    } else {
      int k = (oo[0] == 0) ? 0 : (oo[1] == 0 ? 1 : 2);
      int c = tv[3 * t + k];
      int a = tv[3 * t + (k + 1) % 3], b = tv[3 * t + (k + 2) % 3];
      int32_t u = tn[3 * t + k];
      if (u < 0) return -1;
      int m = 0;
      while (m < 3 && tn[3 * u + m] != t) ++m;
      if (m == 3) return -1;
      int d = tv[3 * u + m];
      int32_t n_bc = tn[3 * t + (k + 1) % 3];
      int32_t n_ca = tn[3 * t + (k + 2) % 3];
      int32_t n_ad = tn[3 * u + (m + 1) % 3];
      int32_t n_db = tn[3 * u + (m + 2) % 3];
      int32_t T1 = t, T3 = u, T2 = ntri, T4 = ntri + 1;
      set_tri(T1, p, c, a, n_ca, T2, T4);
      new_tri(p, a, d, n_ad, T3, T1);   // T2
      set_tri(T3, p, d, b, n_db, T4, T2);
      new_tri(p, b, c, n_bc, T1, T3);   // T4
      replace_nb(n_bc, t, T4);
      replace_nb(n_ad, u, T2);
      stack.push_back({T1, 0});
      stack.push_back({T2, 0});
      stack.push_back({T3, 0});
      stack.push_back({T4, 0});
      last = T4;
    }
    legalize();
    return 0;
  }

  // Triangulate points (X,Y)[0..npts) inserted in `order`.
  int build(const std::vector<int64_t>& order) {
    int npts = static_cast<int>(X.size());
    double xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
    for (int i = 1; i < npts; ++i) {
      xmin = std::min(xmin, X[i]); xmax = std::max(xmax, X[i]);
      ymin = std::min(ymin, Y[i]); ymax = std::max(ymax, Y[i]);
    }
    double cx = 0.5 * (xmin + xmax), cy = 0.5 * (ymin + ymax);
    double D = std::max(xmax - xmin, ymax - ymin);
    if (!(D > 0.0)) D = 1.0;
    const double M = 64.0 * D;
    nsuper0 = npts;
    X.push_back(cx - 2.0 * M); Y.push_back(cy - M);
    X.push_back(cx + 2.0 * M); Y.push_back(cy - M);
    X.push_back(cx);           Y.push_back(cy + 2.0 * M);
    size_t cap = 3 + 2 * static_cast<size_t>(npts) + 8;
    tv.assign(3 * cap, -1);
    tn.assign(3 * cap, -1);
    ntri = 0;
    new_tri(npts, npts + 1, npts + 2, -1, -1, -1);
    last = 0;
    stack.reserve(64);
    for (int64_t q : order)
      if (insert(static_cast<int>(q)) != 0) return -1;
    return 0;
  }
};

// ---------------------------------------------------------------------------
// Ghost points and the full mesh build
// ---------------------------------------------------------------------------

struct Box {
  double x0, y0, x1, y1;
  double lx() const { return x1 - x0; }
  double ly() const { return y1 - y0; }
};

inline double wrap(double v, double lo, double hi) {
  double L = hi - lo;
  if (v < lo - L || v >= hi + L) v = lo + std::fmod(v - lo, L);
  while (v < lo) v += L;
  while (v >= hi) v -= L;
  return v;
}

// periodic shift (sx,sy) <-> code 1..8
inline int shift_code(int sx, int sy) {
  int k = (sx + 1) * 3 + (sy + 1);  // 0..8, 4 is (0,0)
  return k < 4 ? k + 1 : k;         // skip (0,0)
}
inline void code_shift(int code, int& sx, int& sy) {
  int k = code <= 4 ? code - 1 : code;
  sx = k / 3 - 1;
  sy = k % 3 - 1;
}

// neighbour cell index and ghost code packed into one int32 (code in the top
// four bits)
inline int32_t pack_nb(int32_t cell, int code) {
  uint32_t u = static_cast<uint32_t>(cell) |
               (static_cast<uint32_t>(code) << RICH_CODE_SHIFT);
  int32_t r;
  std::memcpy(&r, &u, sizeof(r));
  return r;
}

constexpr double kPi = 3.14159265358979323846;

struct Triangulation {
  Delaunay dt;
  int64_t n = 0;                 // real points
  std::vector<int32_t> gsrc;     // ghost -> source real point
  std::vector<int8_t> gcode;     // ghost -> code (periodic shift / wall)
  double band = 0.0;
  int32_t rebuilds = 0;
};

template <class F>
void parallel_for(int64_t n, int nthreads, F&& f) {
  if (nthreads <= 1 || n < 4096) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    th.emplace_back([&f, b, e] { f(b, e); });
  }
  for (auto& x : th) x.join();
}

void circumcenter(double ax, double ay, double bx, double by, double cx,
                  double cy, double& ox, double& oy) {
  double bxr = bx - ax, byr = by - ay, cxr = cx - ax, cyr = cy - ay;
  double d = 2.0 * (bxr * cyr - byr * cxr);
  double b2 = bxr * bxr + byr * byr, c2 = cxr * cxr + cyr * cyr;
  ox = ax + (cyr * b2 - byr * c2) / d;
  oy = ay + (bxr * c2 - cxr * b2) / d;
}

// Build the ghost-augmented triangulation, widening the band until every
// triangle touching a real point has its circumcircle inside box + band.
int triangulate(const double* px, const double* py, int64_t n, const Box& box,
                uint32_t bc, int nthreads, Triangulation& T,
                std::vector<double>& ccx, std::vector<double>& ccy,
                std::vector<int32_t>& vtri) {
  T.n = n;
  const double area = box.lx() * box.ly();
  double band = 4.0 * std::sqrt(area / static_cast<double>(n));
  const double band_max = 1.0001 * std::max(box.lx(), box.ly());
  band = std::min(band, band_max);
  T.rebuilds = 0;
  for (;;) {
    Delaunay& D = T.dt;
    D = Delaunay();
    T.gsrc.clear();
    T.gcode.clear();
    D.X.assign(px, px + n);
    D.Y.assign(py, py + n);
    const double ex0 = box.x0 - band, ex1 = box.x1 + band;
    const double ey0 = box.y0 - band, ey1 = box.y1 + band;
    auto inside_ext = [&](double x, double y) {
      return x >= ex0 && x <= ex1 && y >= ey0 && y <= ey1;
    };
    for (int64_t i = 0; i < n; ++i) {
      double x = px[i], y = py[i];
      if (bc == RICH_BC_PERIODIC) {
        for (int sx = -1; sx <= 1; ++sx)
          for (int sy = -1; sy <= 1; ++sy) {
            if (sx == 0 && sy == 0) continue;
            double gx = x + sx * box.lx(), gy = y + sy * box.ly();
            if (inside_ext(gx, gy)) {
              D.X.push_back(gx); D.Y.push_back(gy);
              T.gsrc.push_back(static_cast<int32_t>(i));
              T.gcode.push_back(static_cast<int8_t>(shift_code(sx, sy)));
            }
          }
      } else {
        double mx[4] = {2 * box.x0 - x, 2 * box.x1 - x, x, x};
        double my[4] = {y, y, 2 * box.y0 - y, 2 * box.y1 - y};
        for (int w = 0; w < 4; ++w)
          if (inside_ext(mx[w], my[w])) {
            D.X.push_back(mx[w]); D.Y.push_back(my[w]);
            T.gsrc.push_back(static_cast<int32_t>(i));
            T.gcode.push_back(static_cast<int8_t>(RICH_CODE_WALL_X0 + w));
          }
      }
    }
    const int64_t npts = static_cast<int64_t>(D.X.size());
    if (npts >= (int64_t(1) << 30)) return RICH_TESS_E_NOMEM;
    std::vector<int64_t> order;
    hilbert_sort(D.X.data(), D.Y.data(), npts, ex0, ey0, ex1, ey1, order);
    if (D.build(order) != 0) return RICH_TESS_E_MESH;

    // circumcentres of all triangles, vertex -> triangle map
    const int32_t ntri = D.ntri;
    ccx.assign(ntri, 0.0);
    ccy.assign(ntri, 0.0);
    parallel_for(ntri, nthreads, [&](int64_t b, int64_t e) {
      for (int64_t t = b; t < e; ++t) {
        int a = D.tv[3 * t], bb = D.tv[3 * t + 1], c = D.tv[3 * t + 2];
        circumcenter(D.X[a], D.Y[a], D.X[bb], D.Y[bb], D.X[c], D.Y[c], ccx[t], ccy[t]);
      }
    });
    vtri.assign(npts + 3, -1);
    for (int32_t t = 0; t < ntri; ++t)
      for (int k = 0; k < 3; ++k) vtri[D.tv[3 * t + k]] = t;

    // verification.  Once the band spans the whole box every first-ring
    // image (periodic) or single mirror (walls) is present, and only the
    // absence of super vertices is checked.
    const bool complete = band >= band_max;
    std::atomic<int> bad{0};
    const double tol = 1e-9 * std::max(box.lx(), box.ly());
    parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e && !bad.load(std::memory_order_relaxed); ++i) {
        int32_t t0 = vtri[i], t = t0;
        if (t0 < 0) { bad = 2; return; }
        int guard = 0;
        do {
          int k = 0;
          while (k < 3 && D.tv[3 * t + k] != i) ++k;
          if (k == 3) { bad = 2; return; }
          for (int q = 0; q < 3; ++q)
            if (D.tv[3 * t + q] >= D.nsuper0) { bad = 1; return; }
          int a = D.tv[3 * t];
          double R = std::hypot(ccx[t] - D.X[a], ccy[t] - D.Y[a]);
          if (!complete && (ccx[t] - R < ex0 + tol || ccx[t] + R > ex1 - tol ||
              ccy[t] - R < ey0 + tol || ccy[t] + R > ey1 - tol)) {
            bad = 1;
            return;
          }
          t = D.tn[3 * t + (k + 1) % 3];
          if (t < 0 || ++guard > 1000000) { bad = 2; return; }
        } while (t != t0);
      }
    });
    if (bad.load() == 2) return RICH_TESS_E_MESH;
    if (bad.load() == 0) break;
    if (band >= band_max) return RICH_TESS_E_MESH;
    band = std::min(2.0 * band, band_max);
    ++T.rebuilds;
  }
  T.band = band;
  return RICH_TESS_OK;
}

template <class T>
T* alloc_copy(const std::vector<T>& v) {
  T* p = static_cast<T*>(std::malloc(std::max<size_t>(1, v.size()) * sizeof(T)));
  if (p && !v.empty()) std::memcpy(p, v.data(), v.size() * sizeof(T));
  return p;
}

int check_inputs(const double* px, const double* py, int64_t n,
                 const double* box, uint32_t bc) {
  if (!px || !py || !box || n < 1) return RICH_TESS_E_INVAL;
  if (n > RICH_CELL_MASK) return RICH_TESS_E_INVAL;
  if (!(box[2] > box[0]) || !(box[3] > box[1])) return RICH_TESS_E_INVAL;
  if (bc != RICH_BC_WALLS && bc != RICH_BC_PERIODIC) return RICH_TESS_E_INVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(px[i]) || !std::isfinite(py[i])) return RICH_TESS_E_INVAL;
    if (bc == RICH_BC_WALLS &&
        !(px[i] > box[0] && px[i] < box[2] && py[i] > box[1] && py[i] < box[3]))
      return RICH_TESS_E_INVAL;
  }
  return RICH_TESS_OK;
}

int build_mesh(const double* pxin, const double* pyin, int64_t n,
               const double* boxv, uint32_t bc, int nthreads,
               rich_mesh_host* out) {
  std::memset(out, 0, sizeof(*out));
  int st = check_inputs(pxin, pyin, n, boxv, bc);
  if (st) return st;
  if (nthreads <= 0) nthreads = std::max(1u, std::thread::hardware_concurrency());
  Box box{boxv[0], boxv[1], boxv[2], boxv[3]};
  std::vector<double> px(pxin, pxin + n), py(pyin, pyin + n);
  if (bc == RICH_BC_PERIODIC)
    for (int64_t i = 0; i < n; ++i) {
      px[i] = wrap(px[i], box.x0, box.x1);
      py[i] = wrap(py[i], box.y0, box.y1);
    }
  Triangulation T;
  std::vector<double> ccx, ccy;
  std::vector<int32_t> vtri;
  auto clock0 = std::chrono::steady_clock::now();
  st = triangulate(px.data(), py.data(), n, box, bc, nthreads, T, ccx, ccy, vtri);
  if (st) return st;
  auto clock1 = std::chrono::steady_clock::now();
  const Delaunay& D = T.dt;

  // 1. fan sizes
  std::vector<int64_t> poff(n + 1, 0);
  parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t t0 = vtri[i], t = t0;
      int64_t deg = 0;
      do {
        int k = 0;
        while (D.tv[3 * t + k] != i) ++k;
        t = D.tn[3 * t + (k + 1) % 3];
        ++deg;
      } while (t != t0);
      poff[i + 1] = deg;
    }
  });
  for (int64_t i = 0; i < n; ++i) poff[i + 1] += poff[i];
  const int64_t nslot = poff[n];

  // 2. polygons: neighbour, length, midpoint per slot; area and centroid
  std::vector<int32_t> s_nb(nslot);    // neighbour point id (real or ghost)
  std::vector<double> s_len(nslot), s_fx(nslot), s_fy(nslot);
  std::vector<double> area(n), sx(n), sy(n);
  parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
    std::vector<double> vx, vy;
    for (int64_t i = b; i < e; ++i) {
      vx.clear(); vy.clear();
      int32_t t0 = vtri[i], t = t0;
      int64_t s = poff[i];
      do {
        int k = 0;
        while (D.tv[3 * t + k] != i) ++k;
        vx.push_back(ccx[t]);
        vy.push_back(ccy[t]);
        s_nb[s++] = D.tv[3 * t + (k + 2) % 3];
        t = D.tn[3 * t + (k + 1) % 3];
      } while (t != t0);
      const size_t m = vx.size();
      double A2 = 0.0, cxs = 0.0, cys = 0.0;
      for (size_t q = 0; q < m; ++q) {
        size_t q1 = (q + 1) % m;
        double ax = vx[q] - px[i], ay = vy[q] - py[i];
        double bx = vx[q1] - px[i], by = vy[q1] - py[i];
        double cr = ax * by - ay * bx;
        A2 += cr;
        cxs += (ax + bx) * cr;
        cys += (ay + by) * cr;
        int64_t sl = poff[i] + static_cast<int64_t>(q);
        s_len[sl] = std::hypot(vx[q1] - vx[q], vy[q1] - vy[q]);
        s_fx[sl] = 0.5 * (vx[q] + vx[q1]);
        s_fy[sl] = 0.5 * (vy[q] + vy[q1]);
      }
      area[i] = 0.5 * A2;
      sx[i] = px[i] + cxs / (3.0 * A2);
      sy[i] = py[i] + cys / (3.0 * A2);
    }
  });

  // 3. classify slots: neighbour cell, code, kept?, owned?
  std::vector<int32_t> s_cell(nslot);
  std::vector<int8_t> s_code(nslot), s_keep(nslot), s_own(nslot);
  std::atomic<int> bad{0};
  std::atomic<int64_t> dropped{0};
  parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
    int64_t drop_local = 0;
    for (int64_t i = b; i < e; ++i) {
      double Ri = std::sqrt(area[i] / kPi);
      for (int64_t s = poff[i]; s < poff[i + 1]; ++s) {
        int32_t q = s_nb[s];
        int32_t cell;
        int code;
        if (q < n) {
          cell = q;
          code = 0;
        } else if (q - n < static_cast<int64_t>(T.gsrc.size())) {
          cell = T.gsrc[q - n];
          code = T.gcode[q - n];
        } else {
          bad = 1;
          continue;
        }
        double Rj = std::sqrt(area[cell] / kPi);
        bool keep = s_len[s] >= 1e-12 * 0.5 * (Ri + Rj);
        // A point, another point and their mirror images across one wall
        // are concyclic (isosceles trapezoid), so the triangulation may join
        // a cell to the mirror image of another cell.  The Voronoi edge of
        // that pair has length zero exactly; rounding in the circumcentres
        // of such thin triangles can leave it above the threshold, so it is
        // dropped whatever its computed length.
        if (code >= RICH_CODE_WALL_X0 && cell != i) keep = false;
        if (!keep) ++drop_local;
        bool own;
        if (code >= RICH_CODE_WALL_X0) own = true;
        else if (cell != i) own = i < cell;
        else own = code >= 5;  // a cell bordering its own periodic image
        s_cell[s] = cell;
        s_code[s] = static_cast<int8_t>(code);
        s_keep[s] = keep;
        s_own[s] = keep && own;
      }
    }
    dropped += drop_local;
  });
  if (bad.load()) return RICH_TESS_E_MESH;

  // 4. edges, sorted by owner e_i, in polygon order
  std::vector<int32_t> eoff(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = 0;
    for (int64_t s = poff[i]; s < poff[i + 1]; ++s) c += s_own[s];
    eoff[i + 1] = eoff[i] + c;
  }
  const int64_t ne = eoff[n];
  std::vector<int32_t> e_i(ne), e_j(ne);
  std::vector<double> e_len(ne), e_fx(ne), e_fy(ne);
  std::vector<int32_t> s_edge(nslot, -1);
  parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t k = eoff[i];
      for (int64_t s = poff[i]; s < poff[i + 1]; ++s) {
        if (!s_own[s]) continue;
        e_i[k] = static_cast<int32_t>(i);
        e_j[k] = pack_nb(s_cell[s], s_code[s]);
        e_len[k] = s_len[s];
        e_fx[k] = s_fx[s];
        e_fy[k] = s_fy[s];
        s_edge[s] = k;
        ++k;
      }
    }
  });

  // 5. CSR over kept slots; non-owned slots find the owner's edge
  std::vector<int32_t> off(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = 0;
    for (int64_t s = poff[i]; s < poff[i + 1]; ++s) c += s_keep[s];
    off[i + 1] = off[i] + c;
  }
  const int64_t ncsr = off[n];
  std::vector<int32_t> idx(ncsr);
  parallel_for(n, nthreads, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) {
      int32_t k = off[i];
      for (int64_t s = poff[i]; s < poff[i + 1]; ++s) {
        if (!s_keep[s]) continue;
        if (s_own[s]) {
          idx[k++] = 2 * s_edge[s];
          continue;
        }
        int32_t j = s_cell[s];
        int want_code = s_code[s] == 0 ? 0 : 9 - s_code[s];
        int32_t want = pack_nb(static_cast<int32_t>(i), want_code);
        int32_t found = -1;
        for (int32_t q = eoff[j]; q < eoff[j + 1]; ++q)
          if (e_j[q] == want) { found = q; break; }
        if (found < 0) { bad = 1; idx[k++] = 0; continue; }
        idx[k++] = 2 * found + 1;
      }
    }
  });
  if (bad.load()) return RICH_TESS_E_MESH;

  out->n_cells = n;
  out->n_edges = ne;
  out->n_csr = ncsr;
  out->px = alloc_copy(px);
  out->py = alloc_copy(py);
  out->sx = alloc_copy(sx);
  out->sy = alloc_copy(sy);
  out->area = alloc_copy(area);
  out->e_i = alloc_copy(e_i);
  out->e_j = alloc_copy(e_j);
  out->e_len = alloc_copy(e_len);
  out->e_fx = alloc_copy(e_fx);
  out->e_fy = alloc_copy(e_fy);
  out->off = alloc_copy(off);
  out->idx = alloc_copy(idx);
  out->eoff = alloc_copy(eoff);
  out->box[0] = box.x0; out->box[1] = box.y0;
  out->box[2] = box.x1; out->box[3] = box.y1;
  out->bc = bc;
  out->n_ghosts = static_cast<int64_t>(T.gsrc.size());
  out->n_dropped = dropped.load();
  out->band = T.band;
  out->n_rebuilds = T.rebuilds;
  out->n_exact = D.n_exact;
  auto clock2 = std::chrono::steady_clock::now();
  out->t_triangulate = std::chrono::duration<double>(clock1 - clock0).count();
  out->t_voronoi = std::chrono::duration<double>(clock2 - clock1).count();
  if (!out->px || !out->py || !out->sx || !out->sy || !out->area || !out->e_i ||
      !out->e_j || !out->e_len || !out->e_fx || !out->e_fy || !out->off ||
      !out->idx || !out->eoff) {
    rich_tess_free(out);
    return RICH_TESS_E_NOMEM;
  }
  return RICH_TESS_OK;
}

}  // namespace

extern "C" {

int rich_tess_build(const double* px, const double* py, int64_t n,
                    const double box[4], uint32_t bc, int32_t n_threads,
                    rich_mesh_host* out) {
  if (!out) return RICH_TESS_E_INVAL;
  try {
    int st = build_mesh(px, py, n, box, bc, n_threads, out);
    if (st) {
      rich_tess_free(out);
      std::memset(out, 0, sizeof(*out));
    }
    return st;
  } catch (const std::bad_alloc&) {
    rich_tess_free(out);
    std::memset(out, 0, sizeof(*out));
    return RICH_TESS_E_NOMEM;
  } catch (...) {
    rich_tess_free(out);
    std::memset(out, 0, sizeof(*out));
    return RICH_TESS_E_MESH;
  }
}

void rich_tess_free(rich_mesh_host* m) {
  if (!m) return;
  void* ptrs[] = {m->px, m->py, m->sx, m->sy, m->area, m->e_i, m->e_j,
                  m->e_len, m->e_fx, m->e_fy, m->off, m->idx, m->eoff};
  for (void* p : ptrs) std::free(p);
  m->px = m->py = m->sx = m->sy = m->area = nullptr;
  m->e_i = m->e_j = nullptr;
  m->e_len = m->e_fx = m->e_fy = nullptr;
  m->off = m->idx = m->eoff = nullptr;
}

int rich_tess_triangles(const double* pxin, const double* pyin, int64_t n,
                        const double boxv[4], uint32_t bc, rich_tri_host* out) {
  if (!out) return RICH_TESS_E_INVAL;
  std::memset(out, 0, sizeof(*out));
  try {
    int st = check_inputs(pxin, pyin, n, boxv, bc);
    if (st) return st;
    Box box{boxv[0], boxv[1], boxv[2], boxv[3]};
    std::vector<double> px(pxin, pxin + n), py(pyin, pyin + n);
    if (bc == RICH_BC_PERIODIC)
      for (int64_t i = 0; i < n; ++i) {
        px[i] = wrap(px[i], box.x0, box.x1);
        py[i] = wrap(py[i], box.y0, box.y1);
      }
    Triangulation T;
    std::vector<double> ccx, ccy;
    std::vector<int32_t> vtri;
    st = triangulate(px.data(), py.data(), n, box, bc, 1, T, ccx, ccy, vtri);
    if (st) return st;
    const Delaunay& D = T.dt;
    std::vector<int32_t> tri;
    for (int32_t t = 0; t < D.ntri; ++t) {
      int a = D.tv[3 * t], b = D.tv[3 * t + 1], c = D.tv[3 * t + 2];
      if (a >= D.nsuper0 || b >= D.nsuper0 || c >= D.nsuper0) continue;
      if (a < n || b < n || c < n) {
        tri.push_back(a); tri.push_back(b); tri.push_back(c);
      }
    }
    const int64_t npts = D.nsuper0;
    std::vector<int32_t> gs(npts, -1);
    for (size_t g = 0; g < T.gsrc.size(); ++g) gs[n + g] = T.gsrc[g];
    std::vector<double> X(D.X.begin(), D.X.begin() + npts), Y(D.Y.begin(), D.Y.begin() + npts);
    out->n_pts = npts;
    out->n_tri = static_cast<int64_t>(tri.size() / 3);
    out->x = alloc_copy(X);
    out->y = alloc_copy(Y);
    out->ghost_src = alloc_copy(gs);
    out->tri = alloc_copy(tri);
    return RICH_TESS_OK;
  } catch (...) {
    rich_tess_free_tri(out);
    return RICH_TESS_E_NOMEM;
  }
}

void rich_tess_free_tri(rich_tri_host* t) {
  if (!t) return;
  std::free(t->x);
  std::free(t->y);
  std::free(t->ghost_src);
  std::free(t->tri);
  std::memset(t, 0, sizeof(*t));
}

int rich_tess_orient2d(const double a[2], const double b[2], const double c[2]) {
  int64_t ne = 0;
  return orient(a[0], a[1], b[0], b[1], c[0], c[1], &ne);
}

int rich_tess_incircle(const double a[2], const double b[2], const double c[2],
                       const double d[2]) {
  int64_t ne = 0;
  return incircle(a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1], &ne);
}

int rich_tess_hilbert_order(const double* px, const double* py, int64_t n,
                            const double box[4], int64_t* perm_out) {
  if (!px || !py || !box || !perm_out || n < 0) return RICH_TESS_E_INVAL;
  try {
    std::vector<int64_t> perm;
    hilbert_sort(px, py, n, box[0], box[1], box[2], box[3], perm);
    std::memcpy(perm_out, perm.data(), n * sizeof(int64_t));
    return RICH_TESS_OK;
  } catch (...) {
    return RICH_TESS_E_NOMEM;
  }
}

int rich_tess_lloyd(double* px, double* py, int64_t n, const double box[4],
                    uint32_t bc, int32_t iters, int32_t n_threads) {
  if (!px || !py || !box || iters < 0) return RICH_TESS_E_INVAL;
  for (int32_t it = 0; it < iters; ++it) {
    rich_mesh_host m;
    int st = rich_tess_build(px, py, n, box, bc, n_threads, &m);
    if (st) return st;
    for (int64_t i = 0; i < n; ++i) {
      double x = m.sx[i], y = m.sy[i];
      if (bc == RICH_BC_PERIODIC) {
        x = wrap(x, box[0], box[2]);
        y = wrap(y, box[1], box[3]);
      }
      px[i] = x;
      py[i] = y;
    }
    rich_tess_free(&m);
  }
  return RICH_TESS_OK;
}

struct rich_tess_ctx {
  int32_t n_threads = 0;
  std::vector<rich_mesh_host*> out;
};

rich_tess_ctx* rich_tess_ctx_create(int32_t n_threads) {
  try {
    rich_tess_ctx* c = new rich_tess_ctx;
    c->n_threads = n_threads;
    return c;
  } catch (...) {
    return nullptr;
  }
}

void rich_tess_ctx_destroy(rich_tess_ctx* ctx) {
  if (!ctx) return;
  for (rich_mesh_host* m : ctx->out) {
    rich_tess_free(m);
    delete m;
  }
  delete ctx;
}

int rich_tess_callback(void* user, const double* px, const double* py, int64_t n,
                       const double box[4], uint32_t bc, rich_tess_view* v) {
  rich_tess_ctx* ctx = static_cast<rich_tess_ctx*>(user);
  if (!ctx || !v) return RICH_TESS_E_INVAL;
  rich_mesh_host* m = nullptr;
  try {
    m = new rich_mesh_host;
    ctx->out.push_back(m);
  } catch (...) {
    delete m;
    return RICH_TESS_E_NOMEM;
  }
  int st = rich_tess_build(px, py, n, box, bc, ctx->n_threads, m);
  if (st) {
    ctx->out.pop_back();
    delete m;
    return st;
  }
  v->n_cells = m->n_cells;
  v->n_edges = m->n_edges;
  v->n_csr = m->n_csr;
  v->px = m->px; v->py = m->py; v->sx = m->sx; v->sy = m->sy; v->area = m->area;
  v->e_i = m->e_i; v->e_j = m->e_j;
  v->e_len = m->e_len; v->e_fx = m->e_fx; v->e_fy = m->e_fy;
  v->off = m->off; v->idx = m->idx; v->eoff = m->eoff;
  return RICH_TESS_OK;
}

void rich_tess_release(void* user, rich_tess_view* v) {
  rich_tess_ctx* ctx = static_cast<rich_tess_ctx*>(user);
  if (!ctx || !v) return;
  for (size_t k = 0; k < ctx->out.size(); ++k)
    if (ctx->out[k]->px == v->px) {
      rich_tess_free(ctx->out[k]);
      delete ctx->out[k];
      ctx->out.erase(ctx->out.begin() + k);
      break;
    }
  std::memset(v, 0, sizeof(*v));
}

}  // extern "C"
