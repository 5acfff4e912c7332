// One stage of RICH's moving-mesh Godunov scheme (Yalinewich, Steinberg &
// Sari) as a single kernel per tile of T consecutive cells (cells come in
// Hilbert order, so a tile is a compact patch of the mesh).  Nothing but the
// stage's inputs is read from HBM and nothing but its outputs is written:
//
//   1. the tile's cells: point, area, centroid and source totals give the
//      primitives (A1) and the point velocity (A2, section 6) into LDS; each
//      cell's CSR entries and edges are loaded once and kept in registers;
//      neighbours outside the tile (the 1-ring halo) go into an LDS hash
//   2. the 1-ring cells: the same, and their own neighbours outside the
//      tile and the 1-ring (the 2-ring) go into the hash
//   3. the 2-ring cells: primitives only
//   4. the Green-Gauss gradient (section 2.2, eq. slope), the shock detector
//      and the limiter (section 2.2) of every tile and 1-ring cell, from LDS
//   5. every tile cell computes the flux of each of its edges (A5-A7:
//      extrapolation to the edge centre, the frame of the moving edge of
//      section 5, HLLC or exact Riemann solver of section 2.4, the lab-frame
//      flux) and sums them in the order of its CSR entries (A8), then writes
//      its updated totals and point.
//
// Every edge flux is computed by both of its cells with the edge's first
// cell (e_i) on the left, from the same inputs with the same code, so the two
// results are equal bit for bit and the stage conserves exactly what the
// arithmetic of one flux conserves.  A halo cell's reconstruction is the
// same function of the same inputs in every tile that needs it, so the
// result does not depend on the tile size, the grid or a batch's make-up.
// A tile whose halo exceeds the LDS capacity reads the missing cells'
// primitives, or rebuilds their reconstruction, from global memory with the
// same functions.
#pragma once

#include "rich_device.hpp"

namespace rich {

template <int T>
struct TileCfg {
  static constexpr int kNH = T / 2;              // halo lanes: one 1-ring cell each
  static constexpr int kThreads = T + kNH;       // tile lanes, then halo lanes
  static constexpr int kHalo1 = kNH;             // 1-ring cells (each with a record)
  static constexpr int kHalo = kNH + 5 * T / 8;  // 1-ring and 2-ring cells with primitives
  static constexpr int kHash = 2 * T;            // hash of the halo cell ids
  static constexpr int kLogHash = T == 128 ? 8 : (T == 256 ? 9 : 10);
  static constexpr int kS = T + kHalo;           // LDS slots with point and primitives
  static constexpr int kR = T + kHalo1;          // LDS slots with a reconstruction record
  static_assert(T == 128 || T == 256 || T == 512, "tile of 128, 256 or 512 cells");
};

constexpr int kMaxE = 8;  // CSR entries of a cell kept in registers (the rest reloaded)

// One CSR entry of a cell, decoded.  ew: the entry word (2 * edge + side).
// nbc: neighbour id in the low 28 bits, the edge's ghost code in the top 4
// (as e_j).  ref: bits 0..15 the neighbour's LDS slot (0xFFFF: not in LDS),
// bit 17 set for a valid entry.  The edge's geometry (Geo: midpoint in the
// frame of e_i, length) is loaded where it is used.
struct Ent {
  int ew;
  int nbc;
  int ref;
};
struct Geo {
  double fx, fy, L;
};
constexpr int kNoSlot = 0xFFFF;

__device__ __forceinline__ int ent_code(const Ent& e) { return (int)((uint32_t)e.nbc >> 28); }
__device__ __forceinline__ int ent_nb(const Ent& e) { return (int)((uint32_t)e.nbc & kCellMask); }
__device__ __forceinline__ int ent_side(const Ent& e) { return e.ew & 1; }
__device__ __forceinline__ int ent_edge(const Ent& e) { return e.ew >> 1; }
__device__ __forceinline__ bool ent_valid(const Ent& e) { return (e.ref >> 17) & 1; }
__device__ __forceinline__ int ent_slot(const Ent& e) { return e.ref & 0xFFFF; }
__device__ __forceinline__ bool ent_wall(const Ent& e) {
  return ent_side(e) == 0 && ent_code(e) >= 9;
}
__device__ __forceinline__ void ent_set_slot(Ent& e, int slot) {
  e.ref = (e.ref & ~0xFFFF) | (slot & 0xFFFF);
}
__device__ __forceinline__ Geo geo_load(const RunDesc& d, const Ent& e) {
  const double2 a = reinterpret_cast<const double2*>(d.edges + ent_edge(e))[0];
  const double L = reinterpret_cast<const double*>(d.edges + ent_edge(e))[2];
  return Geo{a.x, a.y, L};
}

// Decode CSR entry word `entry` of cell i (its edge record er already
// loaded).  Indices from the mesh are range-checked; a bad one sets `bad`
// and yields an invalid entry.
__device__ __forceinline__ Ent ent_decode(const RunDesc& d, int i, int entry, const EdgeRec& er,
                                          bool in_range, bool& bad) {
  Ent e;
  const int side = entry & 1;
  const int code = (int)(er.j >> 28);
  int nb = side == 0 ? (int)(er.j & kCellMask) : er.i;
  bool ok = in_range;
  if (side == 0 && code >= 9) nb = i;  // a wall: the cell's own mirror image
  if (nb < 0 || nb >= d.n) {
    ok = false;
    nb = i;
  }
  if (in_range && !ok) bad = true;
  e.ew = in_range ? entry : 0;
  e.nbc = (int)((uint32_t)nb | ((uint32_t)code << 28));
  e.ref = kNoSlot | (ok ? (1 << 17) : 0);
  return e;
}

// Load and decode CSR entry k of cell i (k in [off[i], off[i+1])), with its
// edge's geometry.
__device__ __forceinline__ Ent ent_load(const RunDesc& d, int i, int k, Geo& g, bool& bad) {
  const int entry = d.idx[k];
  const int e = entry >> 1;
  const bool in_range = e >= 0 && e < d.n_edges;
  if (!in_range) bad = true;
  EdgeRec er{0.0, 0.0, 0.0, i, 0u};
  if (in_range) er = load_edge(d, e);
  g = Geo{er.fx, er.fy, er.L};
  return ent_decode(d, i, entry, er, in_range, bad);
}

// ---------------------------------------------------------------------------
// per-cell quantities (A1, A2) and the reconstruction (A3, A4)
// ---------------------------------------------------------------------------
struct Own {
  double rx, ry, A, sx, sy;    // point, area, centroid
  double rho, vx, vy, p, c, R;  // primitives, sound speed, radius sqrt(A/pi)
  double wx, wy;               // point velocity
  bool rounded;                // the cell-rounding correction applied
};

__device__ __forceinline__ void own_from(const RunDesc& d, double M, double Px, double Py,
                                         double E, Own& o) {
  prim_from(d, o.A, M, Px, Py, E, o.rho, o.vx, o.vy, o.p);
  o.c = sqrt(d.gamma * o.p / o.rho);
  o.R = sqrt(o.A / kPi);
  o.wx = 0.0;
  o.wy = 0.0;
  o.rounded = false;
  if (d.motion) {
    // section 6: Lagrangian motion plus the cell-rounding correction
    o.wx = o.vx;
    o.wy = o.vy;
    const double dx = o.sx - o.rx, dy = o.sy - o.ry;
    const double dd = sqrt(dx * dx + dy * dy);
    if (dd > d.eta * o.R) {
      o.wx += d.chi * o.c * dx / dd;
      o.wy += d.chi * o.c * dy / dd;
      o.rounded = true;
    }
  }
}

__device__ __forceinline__ void own_load(const RunDesc& d, int i, Own& o, double q[4]) {
  load_cell(d, i, o.rx, o.ry, o.A, o.sx, o.sy);
  q[0] = d.sM[i];
  q[1] = d.sPx[i];
  q[2] = d.sPy[i];
  q[3] = d.sE[i];
}

// The neighbour across entry e as the cell sees it: its point and the edge
// midpoint in the cell's frame and its primitives.  prim_of(nb, slot, pj,
// rjx, rjy) supplies a real neighbour's primitives and point.
template <class PrimOf>
__device__ __forceinline__ void nb_view(const RunDesc& d, const Own& o, const Ent& e,
                                        const Geo& ge, PrimOf&& prim_of, double pj[4],
                                        double& rjx, double& rjy, double& fx, double& fy) {
  const int code = ent_code(e);
  if (ent_wall(e)) {
    pj[0] = o.rho;
    mirror_vec(code, o.vx, o.vy, pj[1], pj[2]);
    pj[3] = o.p;
    mirror_point(d, code, o.rx, o.ry, rjx, rjy);
    fx = ge.fx;
    fy = ge.fy;
    return;
  }
  double shx, shy;
  shift_of(d, code, shx, shy);
  fx = ge.fx;
  fy = ge.fy;
  if (ent_side(e)) {
    shx = -shx;
    shy = -shy;
    fx += shx;
    fy += shy;
  }
  prim_of(ent_nb(e), ent_slot(e), pj, rjx, rjy);
  rjx += shx;
  rjy += shy;
}

// Reconstruction record of a cell: primitives, limited gradients, point
// velocity, centroid and point.
struct Rec {
  double phi[4];  // rho, vx, vy, p
  double g[8];    // limited d/dx, d/dy of rho, vx, vy, p
  double wx, wy, sx, sy, rx, ry;
};

// For m = 0 .. nreg-1 (nreg <= kMaxE, the loop unrolled so that m is a
// constant): f(m, geometry of E[m]) for a valid entry, skip(m) otherwise.
// Each entry's edge geometry is loaded D entries ahead of its use.
template <int D, class F, class Skip>
__device__ __forceinline__ void geo_walk(const RunDesc& d, const Ent E[kMaxE], int nreg, F&& f,
                                         Skip&& skip) {
  Geo GQ[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    GQ[k] = Geo{0.0, 0.0, 0.0};
    if (k < nreg && ent_valid(E[k])) GQ[k] = geo_load(d, E[k]);
  }
#pragma unroll
  for (int m = 0; m < kMaxE; ++m) {
    if (m < nreg) {
      const Geo ge = GQ[m % D];
      const int m2 = m + D < kMaxE ? m + D : m;  // a constant once unrolled
      if (m + D < nreg && ent_valid(E[m2])) GQ[m % D] = geo_load(d, E[m2]);
      if (ent_valid(E[m])) f(m, ge);
      else skip(m);
    } else {
      skip(m);
    }
    // one scheduling region per entry: the loads of later entries are not
    // hoisted here, where they would hold registers for the whole walk
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Primitives of the neighbour across entry e (the mirrored cell for a wall).
template <class PrimOf>
__device__ __forceinline__ void nb_prims(const RunDesc& d, const Own& o, const Ent& e,
                                         PrimOf&& prim_of, double pj[4]) {
  if (ent_wall(e)) {
    pj[0] = o.rho;
    mirror_vec(ent_code(e), o.vx, o.vy, pj[1], pj[2]);
    pj[3] = o.p;
    return;
  }
  double rx, ry;
  prim_of(ent_nb(e), ent_slot(e), pj, rx, ry);
}

// A3 + A4 for one cell.  Its CSR entries k0 .. k0+ne-1 are taken in order:
// the first nreg from the registers E (their edge geometry loaded here in one
// batch), the rest reloaded from memory, resolve(e) giving a reloaded entry
// its slot.  prim_of as in nb_view.  Writes the limited gradient into G and
// returns the debug bits (shock flag, rounding, alpha < 1 per field).
template <class Resolve, class PrimOf>
__device__ __forceinline__ int recon(const RunDesc& d, const Own& o, const Ent E[kMaxE], int nreg,
                                     int ci, int k0, int ne, Resolve&& resolve,
                                     PrimOf&& prim_of, bool& bad, double G[8]) {
  const double phi[4] = {o.rho, o.vx, o.vy, o.p};
  double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double pmax[4] = {o.rho, o.vx, o.vy, o.p}, pmin[4] = {o.rho, o.vx, o.vy, o.p};
  bool pflag = false;
  // eq. (slope) with r_ij = r_i - r_j and c_ij from the midpoint of the two
  // points to the edge centre; each term rounded before it is added.  The
  // edge centre relative to the centroid (dx, dy) is kept for the limiter.
  auto term = [&](const Ent& e, const Geo& ge, double& dx, double& dy) {
    double pj[4], rjx, rjy, fx, fy;
    nb_view(d, o, e, ge, prim_of, pj, rjx, rjy, fx, fy);
    const double rx = o.rx - rjx, ry = o.ry - rjy;
    const double inv_r = rsqrt(rx * rx + ry * ry);
    const double cx = fx - 0.5 * (o.rx + rjx), cy = fy - 0.5 * (o.ry + rjy);
    const double ux = cx * inv_r, uy = cy * inv_r, nx = rx * inv_r, ny = ry * inv_r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double dphi = pj[q] - phi[q];
      const double mean = 0.5 * (phi[q] + pj[q]);
      g[2 * q] += ge.L * (dphi * ux - mean * nx);
      g[2 * q + 1] += ge.L * (dphi * uy - mean * ny);
      pmax[q] = fmax(pmax[q], pj[q]);
      pmin[q] = fmin(pmin[q], pj[q]);
    }
    if (pressure_jump(d.delta_p, o.p, pj[3])) pflag = true;
    dx = fx - o.sx;
    dy = fy - o.sy;
  };
  double DX[kMaxE], DY[kMaxE];
  geo_walk<2>(d, E, nreg, [&](int m, const Geo& ge) { term(E[m], ge, DX[m], DY[m]); },
           [&](int m) {
             DX[m] = 0.0;
             DY[m] = 0.0;
           });
  auto reload = [&](int k, Geo& ge) {
    Ent e = ent_load(d, ci, k, ge, bad);
    if (ent_valid(e)) resolve(e);
    return e;
  };
#pragma unroll 1
  for (int k = k0 + nreg; k < k0 + ne; ++k) {
    Geo ge;
    const Ent e = reload(k, ge);
    double dx, dy;
    if (ent_valid(e)) term(e, ge, dx, dy);
  }
  const double rA = 1.0 / o.A;
#pragma unroll
  for (int q = 0; q < 8; ++q) G[q] = g[q] * rA;
  const bool shock = pflag || (-(G[2] + G[5]) > d.delta_v * o.c / o.R);

  double alpha[4] = {1.0, 1.0, 1.0, 1.0};
  int local = -1;
  if (d.limiter == 0) local = shock ? 1 : 0;
  if (d.limiter == 1) local = 0;
  if (d.limiter == 2) local = 1;
  if (d.limiter == 4) alpha[0] = alpha[1] = alpha[2] = alpha[3] = 0.0;
  if (local == 0) {
    // global limiter: min_j psi_ij is attained at the largest positive and
    // the most negative projected change
    double dmax[4] = {0, 0, 0, 0}, dmin[4] = {0, 0, 0, 0};
    auto bound = [&](double dx, double dy) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double dphi = G[2 * q] * dx + G[2 * q + 1] * dy;
        dmax[q] = fmax(dmax[q], dphi);
        dmin[q] = fmin(dmin[q], dphi);
      }
    };
#pragma unroll
    for (int m = 0; m < kMaxE; ++m)
      if (m < nreg && ent_valid(E[m])) bound(DX[m], DY[m]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll 1
    for (int k = k0 + nreg; k < k0 + ne; ++k) {
      Geo ge;
      const Ent e = reload(k, ge);
      if (!ent_valid(e)) continue;
      double pj[4], rjx, rjy, fx, fy;
      nb_view(d, o, e, ge, prim_of, pj, rjx, rjy, fx, fy);
      bound(fx - o.sx, fy - o.sy);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (dmax[q] > 0.0) alpha[q] = fmin(alpha[q], (pmax[q] - phi[q]) / dmax[q]);
      if (dmin[q] < 0.0) alpha[q] = fmin(alpha[q], (pmin[q] - phi[q]) / dmin[q]);
    }
  } else if (local == 1) {
    auto psi_min = [&](const double pj[4], double dx, double dy) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double dphi = G[2 * q] * dx + G[2 * q + 1] * dy;
        const double psi = (dphi != 0.0) ? fmax(d.theta * (pj[q] - phi[q]) / dphi, 0.0) : 1.0;
        alpha[q] = fmin(alpha[q], psi);
      }
    };
#pragma unroll
    for (int m = 0; m < kMaxE; ++m) {
      if (m < nreg && ent_valid(E[m])) {
        double pj[4];
        nb_prims(d, o, E[m], prim_of, pj);
        psi_min(pj, DX[m], DY[m]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll 1
    for (int k = k0 + nreg; k < k0 + ne; ++k) {
      Geo ge;
      const Ent e = reload(k, ge);
      if (!ent_valid(e)) continue;
      double pj[4], rjx, rjy, fx, fy;
      nb_view(d, o, e, ge, prim_of, pj, rjx, rjy, fx, fy);
      psi_min(pj, fx - o.sx, fy - o.sy);
    }
  }
  int bits = (shock ? 1 : 0) | (o.rounded ? 2 : 0);
#pragma unroll
  for (int q = 0; q < 8; ++q) G[q] *= alpha[q / 2];
#pragma unroll
  for (int q = 0; q < 4; ++q) bits |= (alpha[q] < 1.0 ? 4 << q : 0);
  return bits;
}

// Extrapolated fluxes (section 2.3): the primitives advanced by hh with the
// time derivatives the limited gradients give in the primitive Euler
// equations, following the cell's point (v - w).
__device__ __forceinline__ void advance_half(double gamma, double hh, Rec& r) {
  const double* g = r.g;
  const double rho = r.phi[0], vx = r.phi[1], vy = r.phi[2], p = r.phi[3];
  const double ux = vx - r.wx, uy = vy - r.wy;
  const double div = g[2] + g[5];
  const double rho_t = -(ux * g[0] + uy * g[1]) - rho * div;
  const double vx_t = -(ux * g[2] + uy * g[3]) - g[6] / rho;
  const double vy_t = -(ux * g[4] + uy * g[5]) - g[7] / rho;
  const double p_t = -(ux * g[6] + uy * g[7]) - gamma * p * div;
  r.phi[0] = rho + hh * rho_t;
  r.phi[1] = vx + hh * vx_t;
  r.phi[2] = vy + hh * vy_t;
  r.phi[3] = p + hh * p_t;
}

// ---------------------------------------------------------------------------
// A5-A7 for one edge with its first cell on the left: extrapolation to the
// edge centre, boost into the frame of the moving edge and rotation onto its
// normal, Riemann solve, lab-frame flux times the edge length.
// ---------------------------------------------------------------------------
// One side of an edge: the state extrapolated to the edge centre, the
// cell's point velocity and its point (the second cell's shifted by the
// edge's periodic image code).
struct Side {
  double ph[4];
  double wx, wy, rx, ry;
};

// phi + g . (f - s): the cell's primitives extrapolated to the edge centre
// (fx, fy) from its centroid (sx, sy)
__device__ __forceinline__ void face_of(const double phi[4], const double g[8], double sx,
                                        double sy, double fx, double fy, double ph[4]) {
  const double dx = fx - sx, dy = fy - sy;
#pragma unroll
  for (int q = 0; q < 4; ++q) ph[q] = phi[q] + g[2 * q] * dx + g[2 * q + 1] * dy;
}

// The Riemann problem of the edge from its two sides (b unused for a wall)
// and the lab-frame flux times the length.  Returns false when the exact
// solver meets a vacuum.
template <int RIEMANN>
__device__ __forceinline__ bool flux_core(const RunDesc& d, int code, double fx, double fy,
                                          double L, const Side& a, const Side& b, double LF[4],
                                          uint8_t* br) {
  double nx, ny, wex, wey;
  double WL[4], WR[4];
  if (code >= 9) {
    // reflecting wall: the ghost is the mirror image of the cell's own
    // extrapolated state; the edge moves only along the wall
    nx = (code == 9) ? -1.0 : (code == 10 ? 1.0 : 0.0);
    ny = (code == 11) ? -1.0 : (code == 12 ? 1.0 : 0.0);
    const double tx = -ny, ty = nx;
    const double wn = a.wx * nx + a.wy * ny;
    wex = a.wx - wn * nx;
    wey = a.wy - wn * ny;
    const double vx = a.ph[1] - wex, vy = a.ph[2] - wey;
    WL[0] = a.ph[0]; WL[1] = vx * nx + vy * ny; WL[2] = vx * tx + vy * ty; WL[3] = a.ph[3];
    WR[0] = a.ph[0]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = a.ph[3];
  } else {
    const double dx = b.rx - a.rx, dy = b.ry - a.ry;
    const double inv_dist = rsqrt(dx * dx + dy * dy);
    nx = dx * inv_dist;
    ny = dy * inv_dist;
    const double tx = -ny, ty = nx;
    const double cx = fx - 0.5 * (a.rx + b.rx), cy = fy - 0.5 * (a.ry + b.ry);
    // edge velocity (section 5): mean of the two point velocities plus the
    // normal part that keeps the edge on the bisector
    const double s = ((a.wx - b.wx) * cx + (a.wy - b.wy) * cy) * inv_dist;
    wex = 0.5 * (a.wx + b.wx) + s * nx;
    wey = 0.5 * (a.wy + b.wy) + s * ny;
    const double vlx = a.ph[1] - wex, vly = a.ph[2] - wey;
    const double vrx = b.ph[1] - wex, vry = b.ph[2] - wey;
    WL[0] = a.ph[0]; WL[1] = vlx * nx + vly * ny; WL[2] = vlx * tx + vly * ty; WL[3] = a.ph[3];
    WR[0] = b.ph[0]; WR[1] = vrx * nx + vry * ny; WR[2] = vrx * tx + vry * ty; WR[3] = b.ph[3];
  }
  double F[4];
  bool ok = true;
  if (RIEMANN == 1) {
    if (!exact_flux(d.gamma, d.rgm1, WL, WR, F, br)) ok = false;
  } else {
    hllc(d.gamma, d.rgm1, WL, WR, F, br);
  }
  // back to the lab frame: rotate, then the Galilean transform of the flux
  // through a surface moving with (wex, wey)
  const double tx = -ny, ty = nx;
  const double fpx = F[1] * nx + F[2] * tx, fpy = F[1] * ny + F[2] * ty;
  const double fm = F[0];
  LF[0] = L * fm;
  LF[1] = L * (fpx + fm * wex);
  LF[2] = L * (fpy + fm * wey);
  LF[3] = L * (F[3] + fpx * wex + fpy * wey + 0.5 * (wex * wex + wey * wey) * fm);
  return ok;
}

// The sides of an edge from two full records (a the edge's first cell, b
// the second as stored, shifted here by the edge's image code).
__device__ __forceinline__ void sides_of(const RunDesc& d, int code, double fx, double fy,
                                         const Rec& a, const Rec& b, Side& A, Side& B) {
  face_of(a.phi, a.g, a.sx, a.sy, fx, fy, A.ph);
  A.wx = a.wx; A.wy = a.wy; A.rx = a.rx; A.ry = a.ry;
  if (code < 9) {
    double shx, shy;
    shift_of(d, code, shx, shy);
    face_of(b.phi, b.g, b.sx + shx, b.sy + shy, fx, fy, B.ph);
    B.wx = b.wx; B.wy = b.wy; B.rx = b.rx + shx; B.ry = b.ry + shy;
  } else {
    B = A;
  }
}

template <int RIEMANN>
__device__ __forceinline__ bool flux_lr(const RunDesc& d, int code, double fx, double fy,
                                        double L, const Rec& a, const Rec& b, double LF[4],
                                        uint8_t* br) {
  Side A, B;
  sides_of(d, code, fx, fy, a, b, A, B);
  return flux_core<RIEMANN>(d, code, fx, fy, L, A, B, LF, br);
}

// ---------------------------------------------------------------------------
// global-memory versions (a halo cell the LDS does not hold)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void prim_global(const RunDesc& d, int j, double pj[4], double& rx,
                                            double& ry) {
  double A;
  load_point_area(d, j, rx, ry, A);
  prim_from(d, A, d.sM[j], d.sPx[j], d.sPy[j], d.sE[j], pj[0], pj[1], pj[2], pj[3]);
}

// The whole record of cell j from global memory: the same functions on the
// same inputs as the LDS path, so the same bits.
__device__ __noinline__ void rec_global(const RunDesc& d, int j, Rec& r, bool& bad) {
  Own o;
  double q[4];
  own_load(d, j, o, q);
  own_from(d, q[0], q[1], q[2], q[3], o);
  int k0 = d.off[j], k1 = d.off[j + 1];
  if (k0 < 0 || k1 < k0 || k1 > d.n_csr) {
    bad = true;
    k1 = k0;
  }
  auto pg = [&](int nb, int, double pj[4], double& rx, double& ry) {
    prim_global(d, nb, pj, rx, ry);
  };
  const Ent none[kMaxE] = {};
  recon(d, o, none, 0, j, k0, k1 - k0, [](Ent&) {}, pg, bad, r.g);
  r.phi[0] = o.rho; r.phi[1] = o.vx; r.phi[2] = o.vy; r.phi[3] = o.p;
  r.wx = o.wx; r.wy = o.wy; r.sx = o.sx; r.sy = o.sy; r.rx = o.rx; r.ry = o.ry;
}

// ---------------------------------------------------------------------------
// block-wide helpers
// ---------------------------------------------------------------------------
template <int T>
__device__ __forceinline__ int hash_pos(int key) {
  return (int)(((uint32_t)key * 2654435761u) >> (32 - TileCfg<T>::kLogHash));
}

// Insert key; returns its position or -1 if the table is full.
template <int T>
__device__ __forceinline__ int hash_insert(int* skey, int key) {
  constexpr int H = TileCfg<T>::kHash;
  int h = hash_pos<T>(key);
#pragma unroll 1
  for (int probe = 0; probe < H; ++probe) {
    const int old = atomicCAS(&skey[h], -1, key);
    if (old == -1 || old == key) return h;
    h = (h + 1) & (H - 1);
  }
  return -1;
}

template <int T>
__device__ __forceinline__ int hash_find(const int* skey, int key) {
  constexpr int H = TileCfg<T>::kHash;
  int h = hash_pos<T>(key);
#pragma unroll 1
  for (int probe = 0; probe < H; ++probe) {
    const int k = skey[h];
    if (k == key) return h;
    if (k == -1) return -1;
    h = (h + 1) & (H - 1);
  }
  return -1;
}

// Exclusive prefix sum over the block (TileCfg<T>::kThreads lanes) of one int
// per lane; total gets the sum.  sbuf holds one int per wave.  Contains
// barriers.
template <int T>
__device__ __forceinline__ int block_scan(int v, int* sbuf, int& total) {
  constexpr int W = TileCfg<T>::kThreads / 64;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sbuf[w] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int s = sbuf[k];
    base += k < w ? s : 0;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

// Number the keys of the hash that have no slot yet (sval == -1): slot
// first + rank, or -2 (not held in LDS) from rank `cap` on; their ids go to
// shid[base + rank].  Returns the number of keys given a slot; all gets the
// number of keys numbered.  Contains barriers.
template <int T>
__device__ __forceinline__ int hash_compact(const int* skey, int* sval, int* shid, int* sbuf,
                                            int first, int base, int cap, int& all) {
  constexpr int H = TileCfg<T>::kHash, NT = TileCfg<T>::kThreads;
  constexpr int PER = (H + NT - 1) / NT;
  const int tid = (int)threadIdx.x;
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int h = tid * PER + k;
    if (h < H) cnt += (skey[h] != -1 && sval[h] == -1) ? 1 : 0;
  }
  int total = 0;
  int rank = block_scan<T>(cnt, sbuf, total);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int h = tid * PER + k;
    if (h >= H) break;
    const int key = skey[h];
    if (key != -1 && sval[h] == -1) {
      if (rank < cap) {
        sval[h] = first + rank;
        shid[base + rank] = key;
      } else {
        sval[h] = -2;
      }
      ++rank;
    }
  }
  __syncthreads();
  all = total;
  return min(total, cap);
}

// ---------------------------------------------------------------------------
// the stage kernel
// ---------------------------------------------------------------------------
template <int T>
struct TileLds {
  double P[6][TileCfg<T>::kS];   // px, py, rho, vx, vy, p
  double R[12][TileCfg<T>::kR];  // limited gradient (8), wx, wy, sx, sy
  int key[TileCfg<T>::kHash];    // hash of halo cell ids (-1: empty)
  int val[TileCfg<T>::kHash];    // their slots (-1: none yet, -2: not in LDS)
  int hid[TileCfg<T>::kHalo];    // halo cell of slot T + k
  int buf[TileCfg<T>::kThreads / 64];
  int full;                      // an insert found the hash full
};

// The first nreg (at most kMaxE) CSR entries of cell i from k0 on, level by
// level (all entry words, then all edge records), so that a lane waits for
// two round trips instead of two per entry.
__device__ __forceinline__ void ents_load(const RunDesc& d, int i, int k0, int nreg,
                                          Ent E[kMaxE], bool& bad) {
  int ent[kMaxE];
#pragma unroll
  for (int m = 0; m < kMaxE; ++m) ent[m] = m < nreg ? d.idx[k0 + m] : 0;
  bool inr[kMaxE];
#pragma unroll
  for (int m = 0; m < kMaxE; ++m) {
    const int e = ent[m] >> 1;
    inr[m] = m < nreg && e >= 0 && e < d.n_edges;
    if (m < nreg && !inr[m]) bad = true;
  }
#pragma unroll
  for (int m = 0; m < kMaxE; ++m) {
    EdgeRec er{0.0, 0.0, 0.0, i, 0u};
    if (inr[m]) er = load_edge(d, ent[m] >> 1);
    E[m] = ent_decode(d, i, ent[m], er, inr[m], bad);
    if (m >= nreg) E[m].ref = kNoSlot;  // not an entry
  }
}

// Entry m of the register array E, by selects over constant indices (a
// dynamic index would move the array to scratch memory).
__device__ __forceinline__ Ent ent_pick(const Ent E[kMaxE], int m) {
  Ent e = E[0];
#pragma unroll
  for (int k = 1; k < kMaxE; ++k)
    if (m == k) e = E[k];
  return e;
}

// Slot marker: the neighbour's hash position, to be turned into its slot.
constexpr int kPosMark = 0x4000;

template <int T>
__device__ __forceinline__ int halo_insert_slot(TileLds<T>& s, int nb, int c0, int nt) {
  if (nb >= c0 && nb < c0 + nt) return nb - c0;
  const int pos = hash_insert<T>(s.key, nb);
  if (pos < 0) s.full = 1;
  return pos < 0 ? kNoSlot : (kPosMark | pos);
}
template <int T>
__device__ __forceinline__ int slot_resolve(const TileLds<T>& s, int slot) {
  if (slot == kNoSlot || !(slot & kPosMark)) return slot;
  const int v = s.val[slot & (kPosMark - 1)];
  return v >= 0 ? v : kNoSlot;
}
// Slot of neighbour nb after both numberings (entries reloaded from memory).
template <int T>
__device__ __forceinline__ int slot_find(const TileLds<T>& s, int nb, int c0, int nt) {
  if (nb >= c0 && nb < c0 + nt) return nb - c0;
  const int pos = hash_find<T>(s.key, nb);
  if (pos < 0) return kNoSlot;
  const int v = s.val[pos];
  return v >= 0 ? v : kNoSlot;
}

template <int T>
__device__ __forceinline__ void lds_rec(const TileLds<T>& s, int slot, Rec& r) {
  r.rx = s.P[0][slot];
  r.ry = s.P[1][slot];
#pragma unroll
  for (int q = 0; q < 4; ++q) r.phi[q] = s.P[2 + q][slot];
#pragma unroll
  for (int q = 0; q < 8; ++q) r.g[q] = s.R[q][slot];
  r.wx = s.R[8][slot];
  r.wy = s.R[9][slot];
  r.sx = s.R[10][slot];
  r.sy = s.R[11][slot];
}

// One side of an edge read from LDS slot sl and extrapolated to the edge
// centre; shx, shy shift the cell into the frame of the edge's first cell.
// The same arithmetic as sides_of on a full record.
template <int T>
__device__ __forceinline__ void lds_side(const RunDesc& d, const TileLds<T>& s, int sl, double hh,
                                         double fx, double fy, double shx, double shy, Side& S) {
  Rec r;
  lds_rec<T>(s, sl, r);
  if (d.integrator == 1) advance_half(d.gamma, hh, r);
  face_of(r.phi, r.g, r.sx + shx, r.sy + shy, fx, fy, S.ph);
  S.wx = r.wx;
  S.wy = r.wy;
  S.rx = r.rx + shx;
  S.ry = r.ry + shy;
}

template <int T>
__device__ __forceinline__ void lds_put_own(TileLds<T>& s, int sl, const Own& o) {
  s.P[0][sl] = o.rx;
  s.P[1][sl] = o.ry;
  s.P[2][sl] = o.rho;
  s.P[3][sl] = o.vx;
  s.P[4][sl] = o.vy;
  s.P[5][sl] = o.p;
  s.R[8][sl] = o.wx;
  s.R[9][sl] = o.wy;
  s.R[10][sl] = o.sx;
  s.R[11][sl] = o.sy;
}

// The flux of one CSR entry of cell `me` (neighbour record nb, unused for a
// wall), added to acc with the entry's sign; the Riemann branch record goes
// to br.  Returns false when the exact solver meets a vacuum.  The edge's
// first cell (e_i) is always the left state.
template <int RIEMANN, bool DBG>
__device__ __forceinline__ bool entry_flux(const RunDesc& d, const Ent& e, const Geo& ge,
                                           const Rec& me, const Rec& nb, double acc[4],
                                           uint8_t& br) {
  const bool swap = ent_side(e) != 0;
  double LF[4];
  const bool okf = swap ? flux_lr<RIEMANN>(d, ent_code(e), ge.fx, ge.fy, ge.L, nb, me, LF,
                                           DBG ? &br : nullptr)
                        : flux_lr<RIEMANN>(d, ent_code(e), ge.fx, ge.fy, ge.L, me, nb, LF,
                                           DBG ? &br : nullptr);
  const double sg = swap ? -1.0 : 1.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] += sg * LF[c];
  return okf;
}

// A8: Q_out = Q_base - h sum(+/- L F), plus the external source of the
// stage's own totals; x_out = x_base + h w, wrapped into a periodic box.
// b holds the base totals and point (M, Px, Py, E, x, y).  Sets ok = false on
// a produced state that fails the physical checks.
__device__ __forceinline__ void cell_update(const RunDesc& d, int i, double h, const double acc[4],
                                            const double b[6], double wx, double wy, bool& ok) {
  double M = b[0] - h * acc[0];
  double Px = b[1] - h * acc[1];
  double Py = b[2] - h * acc[2];
  double En = b[3] - h * acc[3];
  double gx = d.gx, gy = d.gy;
  if (d.ax != nullptr) {  // the cell's own acceleration
    gx += d.ax[i];
    gy += d.ay[i];
  }
  if (gx != 0.0 || gy != 0.0) {
    // external acceleration (section 2.3): h (0, M g, P.g) of the stage's
    // source totals
    const double sm = d.sM[i], spx = d.sPx[i], spy = d.sPy[i];
    Px += h * (sm * gx);
    Py += h * (sm * gy);
    En += h * (spx * gx + spy * gy);
  }
  double x = b[4] + h * wx;
  double y = b[5] + h * wy;
  if (d.bc == RICH_BOUNDARY_PERIODIC) {
    const double Lx = d.x1 - d.x0, Ly = d.y1 - d.y0;
    if (x < d.x0) x += Lx;
    if (x >= d.x1) x -= Lx;
    if (y < d.y0) y += Ly;
    if (y >= d.y1) y -= Ly;
    if (!(x >= d.x0 && x < d.x1 && y >= d.y0 && y < d.y1)) ok = false;
  }
  d.oM[i] = M;
  d.oPx[i] = Px;
  d.oPy[i] = Py;
  d.oE[i] = En;
  d.ox[i] = x;
  d.oy[i] = y;
  const double eint = En - 0.5 * (Px * Px + Py * Py) / M;
  if (!(M > 0.0) || !(eint > 0.0) || !isfinite(En) || !isfinite(Px) || !isfinite(Py) ||
      !isfinite(x) || !isfinite(y))
    ok = false;
}

__device__ __forceinline__ void base_load(const RunDesc& d, int i, double b[6]) {
  b[0] = d.bM[i];
  b[1] = d.bPx[i];
  b[2] = d.bPy[i];
  b[3] = d.bE[i];
  b[4] = d.bx[i];
  b[5] = d.by[i];
}

__device__ __forceinline__ double stage_h(const RunDesc& d) {
  return d.h_dev != nullptr ? d.h_factor * (*d.h_dev) : d.h;
}

// A tile whose halo does not fit the LDS: every cell rebuilds its own
// record and its neighbours' from global memory (the same functions on the
// same inputs as the LDS path, hence the same bits).  No barriers.
template <int RIEMANN, bool DBG>
__device__ __forceinline__ void tile_global(const RunDesc& d, int c0, int nt,
                                            uint8_t* __restrict__ dbg_cell,
                                            uint8_t* __restrict__ dbg_edge) {
  const int tid = (int)threadIdx.x;
  if (tid >= nt) return;
  const int i = c0 + tid;
  bool bad = false;
  Own o;
  double q[4];
  own_load(d, i, o, q);
  if (!(o.A > 0.0 && o.A < INFINITY)) bad = true;
  own_from(d, q[0], q[1], q[2], q[3], o);
  int k0 = d.off[i], k1 = d.off[i + 1];
  if (k0 < 0 || k1 < k0 || k1 > d.n_csr) {
    bad = true;
    k1 = k0;
  }
  auto pg = [&](int nb, int, double pj[4], double& rx, double& ry) {
    prim_global(d, nb, pj, rx, ry);
  };
  const Ent none[kMaxE] = {};
  Rec me;
  const int bits = recon(d, o, none, 0, i, k0, k1 - k0, [](Ent&) {}, pg, bad, me.g);
  if constexpr (DBG) dbg_cell[i] = (uint8_t)bits;
  const double h = stage_h(d);
  me.phi[0] = o.rho; me.phi[1] = o.vx; me.phi[2] = o.vy; me.phi[3] = o.p;
  me.wx = o.wx; me.wy = o.wy; me.sx = o.sx; me.sy = o.sy; me.rx = o.rx; me.ry = o.ry;
  if (d.integrator == 1) advance_half(d.gamma, 0.5 * h, me);
  bool ok = true;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = k0; k < k1; ++k) {
    Geo ge;
    const Ent e = ent_load(d, i, k, ge, bad);
    if (!ent_valid(e)) continue;
    Rec nb = me;
    if (!ent_wall(e)) {
      rec_global(d, ent_nb(e), nb, bad);
      if (d.integrator == 1) advance_half(d.gamma, 0.5 * h, nb);
    }
    uint8_t br = 0;
    const bool okf = entry_flux<RIEMANN, DBG>(d, e, ge, me, nb, acc, br);
    if (!okf) ok = false;
    if constexpr (DBG) {
      if (ent_side(e) == 0) dbg_edge[ent_edge(e)] = (uint8_t)(br | (okf ? 0 : 8));
    }
  }
  double b[6];
  base_load(d, i, b);
  cell_update(d, i, h, acc, b, o.wx, o.wy, ok);
  if (!ok || bad) atomicOr(d.flag, RICH_FLAG_DOMAIN);
}

// One tile: cells [lt*T, min((lt+1)*T, n)) of run d (run index `run` in a
// batch).  Lanes 0..T-1 hold the tile's cells, lanes T.. (the halo lanes)
// its 1-ring cells, each lane one cell with its CSR entries in registers; a
// tile whose 1-ring has more cells than there are halo lanes goes to the
// overflow pass.  Each phase ends in a barrier.
template <int T, int RIEMANN, bool DBG>
__device__ __forceinline__ void stage_tile(const RunDesc& d, int run, int lt, TileLds<T>& s,
                                           uint8_t* __restrict__ dbg_cell,
                                           uint8_t* __restrict__ dbg_edge) {
  using C = TileCfg<T>;
  constexpr int NH = C::kNH;
  const int tid = (int)threadIdx.x;
  const bool tile = tid < T;
  const int hl = tid - T;  // halo lane
  const int c0 = lt * T;
  const int nt = min(T, d.n - c0);
  const bool act = tile && tid < nt;
  bool bad = false;

  // The lane's cell: a tile cell (pass 0) or a 1-ring cell (pass 1).
  Own o;
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  Ent E[kMaxE];
  int ci = act ? c0 + tid : c0, slot = tid, k0 = 0, ne = 0;
  bool has = act;
  int nh1 = 0, nh2 = 0;

  if (!tile) {
    for (int k = hl; k < C::kHash; k += NH) {
      s.key[k] = -1;
      s.val[k] = -1;
    }
    if (hl == 0) s.full = 0;
  }
  // passes 0 (tile lanes: the tile's cells) and 1 (halo lanes: the 1-ring)
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const bool mine = (pass == 0) == tile;
    if (mine && has) {
      own_load(d, ci, o, q);
      if (!(o.A > 0.0 && o.A < INFINITY)) bad = true;  // a mesh cell without a volume
      int a = d.off[ci], e1 = d.off[ci + 1];
      if (a < 0 || e1 < a || e1 > d.n_csr) {
        bad = true;
        e1 = a;
      }
      k0 = a;
      ne = e1 - a;
      ents_load(d, ci, k0, min(ne, kMaxE), E, bad);
      own_from(d, q[0], q[1], q[2], q[3], o);
      lds_put_own<T>(s, slot, o);
    }
    if (pass == 0) __syncthreads();  // the hash is clear
    if (mine && has) {
#pragma unroll
      for (int m = 0; m < kMaxE; ++m)
        if (m < ne && ent_valid(E[m]) && !ent_wall(E[m]))
          ent_set_slot(E[m], halo_insert_slot<T>(s, ent_nb(E[m]), c0, nt));
#pragma unroll 1
      for (int k = k0 + kMaxE; k < k0 + ne; ++k) {
        Geo ge;
        const Ent e = ent_load(d, ci, k, ge, bad);
        if (ent_valid(e) && !ent_wall(e)) (void)halo_insert_slot<T>(s, ent_nb(e), c0, nt);
      }
    }
    __syncthreads();
    int all = 0;
    if (pass == 0) {
      nh1 = hash_compact<T>(s.key, s.val, s.hid, s.buf, T, 0, C::kHalo1, all);
      if (all > nh1 || s.full) {
        // the 1-ring does not fit: the tile goes on the overflow list, whose
        // tiles k_stage_overflow computes from global memory
        if (tid == 0) {
          const int k = atomicAdd(d.ovf_count, 1);
          d.ovf_list[k] = make_int2(run, lt);
        }
        __syncthreads();
        return;
      }
    } else {
      nh2 = hash_compact<T>(s.key, s.val, s.hid, s.buf, T + nh1, nh1, C::kHalo - nh1, all);
    }
    if (mine && has) {
#pragma unroll
      for (int m = 0; m < kMaxE; ++m)
        if (m < ne) ent_set_slot(E[m], slot_resolve<T>(s, ent_slot(E[m])));
    }
    if (pass == 0 && !tile) {
      has = hl < nh1;
      ci = has ? s.hid[hl] : c0;
      slot = T + hl;
    }
  }

  // the 2-ring: points and primitives
  if (!tile) {
#pragma unroll
    for (int r = 0; r < (C::kHalo + NH - 1) / NH; ++r) {
      const int k = hl + r * NH;
      if (k < nh2) {
        double pj[4], rx, ry;
        prim_global(d, s.hid[nh1 + k], pj, rx, ry);
        const int sl = T + nh1 + k;
        s.P[0][sl] = rx;
        s.P[1][sl] = ry;
#pragma unroll
        for (int c = 0; c < 4; ++c) s.P[2 + c][sl] = pj[c];
      }
    }
  }
  __syncthreads();

  // reconstruction of the lane's cell (a tile cell or a 1-ring cell)
  auto prim_of = [&](int nb, int sl, double pj[4], double& rx, double& ry) {
    if (sl != kNoSlot) {
      rx = s.P[0][sl];
      ry = s.P[1][sl];
#pragma unroll
      for (int c = 0; c < 4; ++c) pj[c] = s.P[2 + c][sl];
    } else {
      prim_global(d, nb, pj, rx, ry);
    }
  };
  auto resolve = [&](Ent& e) {
    if (!ent_wall(e)) ent_set_slot(e, slot_find<T>(s, ent_nb(e), c0, nt));
  };
  if (has) {
    double G[8];
    const int bits = recon(d, o, E, min(ne, kMaxE), ci, k0, ne, resolve, prim_of, bad, G);
#pragma unroll
    for (int k = 0; k < 8; ++k) s.R[k][slot] = G[k];
    if constexpr (DBG) {
      if (act) dbg_cell[c0 + tid] = (uint8_t)bits;
    }
  }
  __syncthreads();

  // fluxes of the tile cells' edges and the update; every neighbour of a
  // tile cell is in the tile or the 1-ring, whose records are in LDS next to
  // the cell's own: the edge's first cell (e_i) is the left record
  if (act) {
    const int i = c0 + tid;
    const double h = stage_h(d);
    bool ok = true;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto flux_entry = [&](const Ent& e, const Geo& ge) {
      int sl = ent_wall(e) ? tid : ent_slot(e);
      if (sl == kNoSlot) {  // cannot happen: every neighbour has a slot
        bad = true;
        sl = tid;
      }
      const bool swap = ent_side(e) != 0;
      const int code = ent_code(e);
      Side A, B;
      lds_side<T>(d, s, swap ? sl : tid, 0.5 * h, ge.fx, ge.fy, 0.0, 0.0, A);
      __builtin_amdgcn_sched_barrier(0);
      if (code < 9) {
        double shx, shy;
        shift_of(d, code, shx, shy);
        lds_side<T>(d, s, swap ? tid : sl, 0.5 * h, ge.fx, ge.fy, shx, shy, B);
      } else {
        B = A;
      }
      __builtin_amdgcn_sched_barrier(0);
      double LF[4];
      uint8_t br = 0;
      const bool okf = flux_core<RIEMANN>(d, code, ge.fx, ge.fy, ge.L, A, B, LF,
                                          DBG ? &br : nullptr);
      if (!okf) ok = false;
      const double sg = swap ? -1.0 : 1.0;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += sg * LF[c];
      if constexpr (DBG) {
        if (!swap) dbg_edge[ent_edge(e)] = (uint8_t)(br | (okf ? 0 : 8));
      }
    };
    const int nreg = min(ne, kMaxE);
    double b[6];
    base_load(d, i, b);
    if constexpr (RIEMANN == 0) {
      // HLLC: the entries unrolled (constant register indices)
      geo_walk<1>(d, E, nreg, [&](int m, const Geo& ge) { flux_entry(E[m], ge); }, [](int) {});
    } else {
      // the exact solver is large: one copy of it in a loop over the entries
      // (picked from the registers), each entry's geometry loaded one ahead
      Geo gn{0.0, 0.0, 0.0};
      if (nreg > 0 && ent_valid(E[0])) gn = geo_load(d, E[0]);
#pragma unroll 1
      for (int m = 0; m < nreg; ++m) {
        const Ent e = ent_pick(E, m);
        const Geo ge = gn;
        if (m + 1 < nreg) {
          const Ent en = ent_pick(E, m + 1);
          if (ent_valid(en)) gn = geo_load(d, en);
        }
        if (ent_valid(e)) flux_entry(e, ge);
      }
    }
#pragma unroll 1
    for (int k = k0 + kMaxE; k < k0 + ne; ++k) {
      Geo ge;
      Ent e = ent_load(d, i, k, ge, bad);
      if (!ent_valid(e)) continue;
      resolve(e);
      flux_entry(e, ge);
    }
    cell_update(d, i, h, acc, b, s.R[8][tid], s.R[9][tid], ok);
    if (!ok) bad = true;
  }
  if (bad) atomicOr(d.flag, RICH_FLAG_DOMAIN);
  __syncthreads();  // the next tile reuses the LDS
}

// One stage over n_tiles tiles of T cells: a single run (one), or a batch
// whose tile k belongs to run tiles[k].x as its local tile tiles[k].y.
// Blocks of T + T/2 lanes stride over the tiles in XCD-contiguous order.
template <int T, int RIEMANN, bool BATCH, bool DBG = false>
__global__ __launch_bounds__(TileCfg<T>::kThreads, 3) void k_stage(
    RunDesc one, const RunDesc* __restrict__ descs, const int2* __restrict__ tiles, int n_tiles,
    uint8_t* __restrict__ dbg_cell, uint8_t* __restrict__ dbg_edge) {
  __shared__ TileLds<T> s;
  if (blockDim.x != TileCfg<T>::kThreads) {
    // a launch with the wrong block shape has no halo lanes: report it on
    // the first tile's run and do nothing
    if (threadIdx.x == 0 && blockIdx.x == 0 && n_tiles > 0)
      atomicOr(BATCH ? descs[tiles[0].x].flag : one.flag, RICH_FLAG_DOMAIN);
    return;
  }
  for (int b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    const int tt = xcd_tile(b, n_tiles);
    if constexpr (BATCH) {
      const int2 tr = tiles[tt];
      stage_tile<T, RIEMANN, DBG>(descs[tr.x], tr.x, tr.y, s, dbg_cell, dbg_edge);
    } else {
      // the descriptor read through a pointer the compiler cannot trace to
      // the kernel arguments, so that its fields are loaded where they are
      // used instead of being held (and spilled) for the whole kernel
      const RunDesc* dp = &one;
      asm volatile("" : "+s"(dp));
      stage_tile<T, RIEMANN, DBG>(*dp, 0, tt, s, dbg_cell, dbg_edge);
    }
  }
}

// The tiles k_stage put on the overflow list (*ovf_count entries of
// (run, local tile) at ovf_list), each cell from global memory.
template <int T, int RIEMANN, bool BATCH, bool DBG = false>
__global__ __launch_bounds__(T) void k_stage_overflow(RunDesc one,
                                                      const RunDesc* __restrict__ descs,
                                                      const int* __restrict__ ovf_count,
                                                      const int2* __restrict__ ovf_list,
                                                      uint8_t* __restrict__ dbg_cell,
                                                      uint8_t* __restrict__ dbg_edge) {
  const int cnt = *ovf_count;
  for (int b = blockIdx.x; b < cnt; b += gridDim.x) {
    const int2 tr = ovf_list[b];
    const RunDesc& d = BATCH ? descs[tr.x] : one;
    const int c0 = tr.y * T;
    tile_global<RIEMANN, DBG>(d, c0, min(T, d.n - c0), dbg_cell, dbg_edge);
  }
}

}  // namespace rich
