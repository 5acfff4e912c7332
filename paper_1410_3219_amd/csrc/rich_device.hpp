// Device-side building blocks of one stage of RICH's moving-mesh Godunov
// scheme (Yalinewich, Steinberg & Sari) for gfx950: primitive recovery, point
// velocity (section 6), Green-Gauss gradient (section 2.2, eq. slope), the
// global/local limiter switch (section 2.2), extrapolation to the edge centre
// (section 2.2), the HLLC and exact Riemann solvers (section 2.4) in the frame
// of the moving edge (section 1, section 5), and the lab-frame flux.
//
// Arithmetic is FP64 throughout, without fast-math: every division written
// with '/' and every sqrt is the correctly rounded IEEE operation.  The
// divisions of the hot paths (rcp, ddiv below) are the hardware reciprocal
// refined by Newton steps, within about an ulp of the quotient; the inverse
// distances of the gradient terms, of the edge normals and of the rounding
// correction are reciprocal square roots (rsqrt), accurate to a few units in
// the last place.  The oracle divides correctly rounded there, and the
// differences stay at rounding level.  Floating-point
// contraction is per source expression (-ffp-contract=on), so every call of
// these functions on the same inputs produces the same bits, wherever it is
// inlined: a cell or an edge computed by two different tiles agrees bitwise.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rich.h"

namespace rich {

constexpr double kPi = 3.14159265358979323846;
constexpr uint32_t kCellMask = 0x0FFFFFFFu;
constexpr int kRecDoubles = 16;  // reconstruction record: 128 bytes per cell

// Everything one stage of one run needs (device pointers).  Passed by value
// as a kernel argument for a single run, stored in device memory for a batch.
struct RunDesc {
  // mesh
  const rich_cell* cells;
  const rich_edge* edges;
  const int32_t *off, *idx, *eoff;
  // state
  const double *sM, *sPx, *sPy, *sE;              // primitives come from here
  const double *bM, *bPx, *bPy, *bE, *bx, *by;    // base of the update
  double *oM, *oPx, *oPy, *oE, *ox, *oy;          // result
  // workspace of this run
  double* rec;       // [n][16] records
  double* cfl_blocks;   // Courant minimum of each cell-kernel block, or null
  const double* h_dev;  // if set, the step is h_factor * (*h_dev) (device dt)
  double h_factor;
  int32_t* flag;     // status word
  unsigned long long* cfl_min;  // bit pattern of the smallest R/(c+|v-w|)
  // geometry and parameters
  double x0, y0, x1, y1, Lx, Ly;
  double h, gamma, theta, delta_v, delta_p, chi, eta, cfl;
  double rgm1;  // 1 / (gamma - 1)
  double gx, gy;  // uniform external acceleration
  const double *ax, *ay;  // per-cell acceleration added to (gx, gy), or null
  int32_t n, n_edges, n_csr, bc;
  int32_t riemann, motion, limiter, integrator;
};

// Record layout (doubles): 0..3 rho, vx, vy, p of the limited linear
// reconstruction evaluated at the cell's point (the cell averages moved from
// the centroid s to the point r along the limited gradient, so that the value
// at an edge midpoint f is rec + G (f - r)); 4..11 limited gradients (d/dx,
// d/dy of rho, vx, vy, p); 12..13 point velocity; 14..15 the point itself.
// The flux pass thus needs no mesh cell data.
enum { R_RHO = 0, R_VX, R_VY, R_P, R_G = 4, R_WX = 12, R_WY, R_PX, R_PY };

// ---------------------------------------------------------------------------
// mesh records: 16-byte loads
// ---------------------------------------------------------------------------
struct EdgeRec {
  double fx, fy, L;
  int i;
  uint32_t j;
};
__device__ __forceinline__ EdgeRec load_edge(const RunDesc& d, int e) {
  const double2 a = reinterpret_cast<const double2*>(d.edges + e)[0];
  const int4 b = reinterpret_cast<const int4*>(d.edges + e)[1];
  EdgeRec r;
  r.fx = a.x;
  r.fy = a.y;
  r.L = __hiloint2double(b.y, b.x);
  r.i = b.z;
  r.j = (uint32_t)b.w;
  return r;
}
// point of cell c (one load); point and area (two); all (three)
__device__ __forceinline__ void load_point(const RunDesc& d, int c, double& px, double& py) {
  const double2 a = reinterpret_cast<const double2*>(d.cells + c)[0];
  px = a.x;
  py = a.y;
}
__device__ __forceinline__ void load_point_area(const RunDesc& d, int c, double& px, double& py,
                                                double& area) {
  const double2* p = reinterpret_cast<const double2*>(d.cells + c);
  const double2 a = p[0], b = p[1];
  px = a.x;
  py = a.y;
  area = b.x;
}
__device__ __forceinline__ void load_cell(const RunDesc& d, int c, double& px, double& py,
                                          double& area, double& sx, double& sy) {
  const double2* p = reinterpret_cast<const double2*>(d.cells + c);
  const double2 a = p[0], b = p[1], g = p[2];
  px = a.x;
  py = a.y;
  area = b.x;
  sx = b.y;
  sy = g.x;
}

// ---------------------------------------------------------------------------
// mesh access
// ---------------------------------------------------------------------------
// Image shift of a ghost code: codes 1..4 are k = code - 1 and 5..8 are
// k = code of the 3x3 grid of images, shifted by (k/3 - 1, k%3 - 1) box
// lengths; code 0 and the wall codes have none.  Each code's two offsets are
// read from 2-bit fields (offset + 1) of two constants instead of dividing.
__device__ __forceinline__ void shift_of(const RunDesc& d, int code, double& shx,
                                         double& shy) {
  constexpr uint32_t kOffX = 0x5556a501u, kOffY = 0x55564891u;
  const uint32_t sh = 2u * ((uint32_t)code & 15u);
  shx = (double)((int)((kOffX >> sh) & 3u) - 1) * d.Lx;
  shy = (double)((int)((kOffY >> sh) & 3u) - 1) * d.Ly;
}

// Both coordinates are always computed and selected, so that the compiler
// keeps them in registers (conditional stores to one of two outputs are
// otherwise merged into a dynamically indexed stack slot).
__device__ __forceinline__ void mirror_point(const RunDesc& d, int code, double x,
                                             double y, double& mx, double& my) {
  const double ax = 2.0 * (code == 9 ? d.x0 : d.x1) - x;
  const double ay = 2.0 * (code == 11 ? d.y0 : d.y1) - y;
  mx = (code == 9 || code == 10) ? ax : x;
  my = (code == 11 || code == 12) ? ay : y;
}

__device__ __forceinline__ void mirror_vec(int code, double vx, double vy, double& mx,
                                           double& my) {
  mx = (code == 9 || code == 10) ? -vx : vx;
  my = (code == 11 || code == 12) ? -vy : vy;
}

// The neighbour across one CSR entry of cell i: the edge's data and the
// neighbour's index and image shift.  Indices read from the mesh are
// range-checked.
struct NbE {
  int j, wall;
  double shx, shy, fx, fy, L;
};

__device__ __forceinline__ NbE nb_edge(const RunDesc& d, int i, int entry, bool& bad) {
  NbE v;
  int e = entry >> 1;
  const int side = entry & 1;
  if (e < 0 || e >= d.n_edges) {
    bad = true;
    e = 0;
  }
  const EdgeRec er = load_edge(d, e);
  const uint32_t ej = er.j;
  const int code = (int)(ej >> 28);
  v.L = er.L;
  v.fx = er.fx;
  v.fy = er.fy;
  shift_of(d, code, v.shx, v.shy);
  v.wall = 0;
  if (side == 0) {
    if (code >= 9) {
      v.wall = code;
      v.j = i;
      return v;
    }
    v.j = (int)(ej & kCellMask);
  } else {
    v.j = er.i;
    v.shx = -v.shx;
    v.shy = -v.shy;
    v.fx += v.shx;
    v.fy += v.shy;
  }
  if (v.j < 0 || v.j >= d.n) {
    bad = true;
    v.j = i;
  }
  return v;
}

// ---------------------------------------------------------------------------
// arithmetic helpers
// ---------------------------------------------------------------------------
#ifndef RICH_NOCANON
#define RICH_NOCANON 1
#endif
#ifndef RICH_FASTDIV
#define RICH_FASTDIV 1
#endif
// Larger / smaller of two doubles, as fmax / fmin (a NaN operand yields the
// other one).  fmax and fmin first quiet each operand the compiler cannot
// prove already canonical (one extra instruction per operand); the hardware
// instruction alone does the same for every operand that is not a
// signalling NaN, and none of the stage's values is one.
__device__ __forceinline__ double dmax(double a, double b) {
#if RICH_NOCANON
  double r;
  asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
#else
  return fmax(a, b);
#endif
}
__device__ __forceinline__ double dmin(double a, double b) {
#if RICH_NOCANON
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
  return r;
#else
  return fmin(a, b);
#endif
}

// 1/b: the hardware estimate refined by two Newton steps
// r <- r + r (1 - b r), each squaring the relative error, so the result is
// within an ulp or so of the correctly rounded reciprocal for every finite
// nonzero b whose reciprocal is a normal number.
__device__ __forceinline__ double rcp(double b) {
#if RICH_FASTDIV
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / b;
#endif
}
// a/b: a times the reciprocal, then one correction with the exact residual
// a - b q (an fma), which brings the quotient to within an ulp of a/b.
__device__ __forceinline__ double ddiv(double a, double b) {
#if RICH_FASTDIV
  const double r = rcp(b);
  const double q = a * r;
  return fma(r, fma(-b, q, a), q);
#else
  return a / b;
#endif
}

// ---------------------------------------------------------------------------
// A1: primitives of cell j from the extensive totals (ideal gas)
// ---------------------------------------------------------------------------
// Two reciprocals instead of four divisions: the results may differ from the
// quotients in the last bit.
__device__ __forceinline__ void prim_from(const RunDesc& d, double A, double M, double Px,
                                          double Py, double E, double& rho, double& vx,
                                          double& vy, double& p) {
  const double rA = rcp(A);
  const double rM = rcp(M);
  rho = M * rA;
  vx = Px * rM;
  vy = Py * rM;
  p = (d.gamma - 1.0) * (E * rA - 0.5 * rho * (vx * vx + vy * vy));
}
__device__ __forceinline__ void prim_of(const RunDesc& d, int j, double area, double& rho,
                                        double& vx, double& vy, double& p) {
  prim_from(d, area, d.sM[j], d.sPx[j], d.sPy[j], d.sE[j], rho, vx, vy, p);
}

// A2 (section 6) and the Courant ratio of section 2.3 for one cell: sound
// speed c, effective radius R = sqrt(A/pi), point velocity w (Lagrangian
// motion plus the cell-rounding correction chi c (s - r)/|s - r| when the
// centroid s lies more than eta R from the point r; w = 0 without motion)
// and R / (c + |v - w|).  Shared by the cell pass and the Courant kernel,
// which must agree bitwise.
struct Kin {
  double c, R, wx, wy;
  bool rounded;
};
__device__ __forceinline__ Kin kinematics(const RunDesc& d, double A, double rho, double vx,
                                          double vy, double p, double rix, double riy,
                                          double six, double siy) {
  constexpr double kInvPi = 0.31830988618379067154;
  Kin k;
  k.c = sqrt(d.gamma * ddiv(p, rho));
  k.R = sqrt(A * kInvPi);
  k.wx = 0.0;
  k.wy = 0.0;
  k.rounded = false;
  if (d.motion) {
    k.wx = vx;
    k.wy = vy;
    // |s - r| > eta R compared in squares; 1/|s - r| as one reciprocal
    // square root
    const double dx = six - rix, dy = siy - riy;
    const double dd2 = dx * dx + dy * dy;
    const double er = d.eta * k.R;
    if (dd2 > er * er) {
      const double s = d.chi * k.c * rsqrt(dd2);
      k.wx += s * dx;
      k.wy += s * dy;
      k.rounded = true;
    }
  }
  return k;
}
__device__ __forceinline__ double courant_ratio(const Kin& k, double vx, double vy) {
  const double ux = vx - k.wx, uy = vy - k.wy;
  const double cs = k.c + sqrt(ux * ux + uy * uy);
  const double ti = ddiv(k.R, cs);
  return (ti > 0.0 && isfinite(ti)) ? ti : 0.0;
}

// Pressure-ratio test of the shock detector, min(pi/pj, pj/pi) < delta_p,
// without a division (both pressures positive).
__device__ __forceinline__ bool pressure_jump(double delta_p, double pi, double pj) {
  return pi > pj ? (pj < delta_p * pi) : (pj > pi ? (pi < delta_p * pj) : (delta_p > 1.0));
}

// ---------------------------------------------------------------------------
// Riemann solvers in the edge frame (section 2.4).  W = (rho, u, vt, p).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void phys_flux(double g, double rgm1, const double* W, double* F) {
  const double rho = W[0], u = W[1], vt = W[2], pr = W[3];
  const double E = pr * rgm1 + 0.5 * rho * (u * u + vt * vt);
  F[0] = rho * u;
  F[1] = rho * u * u + pr;
  F[2] = rho * u * vt;
  F[3] = u * (E + pr);
}

// HLLC with Davis wave-speed bounds; star fluxes are the physical fluxes of
// the star states (identical to the Rankine-Hugoniot form).
// br (debug record, may be null): bit 0 = (0 <= S_L), bit 1 = (0 <= S*),
// bit 2 = (0 < S_R), the three comparisons that pick the flux.
__device__ inline void hllc(double g, double rgm1, const double* WL, const double* WR,
                            double* F, uint8_t* br = nullptr) {
  const double rl = WL[0], ul = WL[1], pl = WL[3];
  const double rr = WR[0], ur = WR[1], pr = WR[3];
  const double cl = sqrt(g * ddiv(pl, rl)), cr = sqrt(g * ddiv(pr, rr));
  const double sl = dmin(ul - cl, ur - cr);
  const double sr = dmax(ul + cl, ur + cr);
  const double ss = ddiv(pr - pl + rl * ul * (sl - ul) - rr * ur * (sr - ur),
                         rl * (sl - ul) - rr * (sr - ur));
  if (br != nullptr)
    *br = (uint8_t)((0.0 <= sl ? 1 : 0) | (0.0 <= ss ? 2 : 0) | (0.0 < sr ? 4 : 0));
  if (0.0 <= sl) {
    phys_flux(g, rgm1, WL, F);
    return;
  }
  if (!(0.0 <= ss) && !(0.0 < sr)) {
    phys_flux(g, rgm1, WR, F);
    return;
  }
  const bool left = (0.0 <= ss);
  const double* W = left ? WL : WR;
  const double sk = left ? sl : sr;
  const double rho = W[0], u = W[1], vt = W[2], pk = W[3];
  const double E = pk * rgm1 + 0.5 * rho * (u * u + vt * vt);
  const double rs = ddiv(rho * (sk - u), sk - ss);
  const double ps = pk + rho * (sk - u) * (ss - u);
  const double Es = rs * (ddiv(E, rho) + (ss - u) * (ss + ddiv(pk, rho * (sk - u))));
  F[0] = rs * ss;
  F[1] = rs * ss * ss + ps;
  F[2] = rs * ss * vt;
  F[3] = (Es + ps) * ss;
}

// Exact solver: star pressure by Newton iteration on
// f_L(p) + f_R(p) + u_R - u_L = 0 (shock branch for p > p_K, rarefaction
// branch otherwise), primitive-variable initial guess clipped at 1e-14,
// relative change 1e-14 or 50 iterations; the solution sampled at x/t = 0.
__device__ __forceinline__ void pfun(double g, double ps, double rk, double pk, double ck,
                                     double& f, double& fd) {
  if (ps > pk) {
    const double A = 2.0 / ((g + 1.0) * rk), B = (g - 1.0) / (g + 1.0) * pk;
    const double q = sqrt(A / (ps + B));
    f = (ps - pk) * q;
    fd = q * (1.0 - 0.5 * (ps - pk) / (B + ps));
  } else {
    const double pr = ps / pk;
    f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
    fd = 1.0 / (rk * ck) * pow(pr, -(g + 1.0) / (2.0 * g));
  }
}

// br (debug record, may be null): bit 1 = (0 <= u*), the side of the contact
// sampled at x/t = 0; bit 3 = the states would create a vacuum.
__device__ inline bool exact_flux(double g, double rgm1, const double* WL, const double* WR,
                                  double* F, uint8_t* br = nullptr) {
  const double rl = WL[0], ul = WL[1], pl = WL[3];
  const double rr = WR[0], ur = WR[1], pr = WR[3];
  const double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  if (2.0 / (g - 1.0) * (cl + cr) <= ur - ul) {
    F[0] = F[1] = F[2] = F[3] = 0.0;
    if (br != nullptr) *br = 8;
    return false;
  }
  const double tiny = 1e-14;
  double ps = 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr);
  if (ps < tiny) ps = tiny;
  for (int it = 1; it <= 50; ++it) {
    double fl, fld, fr, frd;
    pfun(g, ps, rl, pl, cl, fl, fld);
    pfun(g, ps, rr, pr, cr, fr, frd);
    double pn = ps - (fl + fr + ur - ul) / (fld + frd);
    if (pn < tiny) pn = tiny;
    const double change = 2.0 * fabs(pn - ps) / (pn + ps);
    ps = pn;
    if (change < 1e-14) break;
  }
  double fl, fld, fr, frd;
  pfun(g, ps, rl, pl, cl, fl, fld);
  pfun(g, ps, rr, pr, cr, fr, frd);
  const double us = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  if (br != nullptr) *br = (uint8_t)(0.0 <= us ? 2 : 0);
  // sample at x/t = 0
  const double g1 = (g - 1.0) / (2.0 * g), g2 = (g + 1.0) / (2.0 * g);
  const double g3 = 2.0 * g / (g - 1.0), g4 = 2.0 / (g - 1.0), g5 = 2.0 / (g + 1.0);
  const double g6 = (g - 1.0) / (g + 1.0), g7 = (g - 1.0) / 2.0;
  double W[4];
  if (0.0 <= us) {
    W[2] = WL[2];
    if (ps > pl) {
      const double s = ul - cl * sqrt(g2 * ps / pl + g1);
      if (0.0 <= s) {
        W[0] = rl; W[1] = ul; W[3] = pl;
      } else {
        W[0] = rl * (ps / pl + g6) / (g6 * ps / pl + 1.0); W[1] = us; W[3] = ps;
      }
    } else if (0.0 <= ul - cl) {
      W[0] = rl; W[1] = ul; W[3] = pl;
    } else {
      const double cml = cl * pow(ps / pl, g1);
      if (0.0 > us - cml) {
        W[0] = rl * pow(ps / pl, 1.0 / g); W[1] = us; W[3] = ps;
      } else {
        const double cc = g5 * (cl + g7 * ul);
        W[0] = rl * pow(cc / cl, g4);
        W[1] = g5 * (cl + g7 * ul);
        W[3] = pl * pow(cc / cl, g3);
      }
    }
  } else {
    W[2] = WR[2];
    if (ps > pr) {
      const double s = ur + cr * sqrt(g2 * ps / pr + g1);
      if (0.0 >= s) {
        W[0] = rr; W[1] = ur; W[3] = pr;
      } else {
        W[0] = rr * (ps / pr + g6) / (g6 * ps / pr + 1.0); W[1] = us; W[3] = ps;
      }
    } else if (0.0 >= ur + cr) {
      W[0] = rr; W[1] = ur; W[3] = pr;
    } else {
      const double cmr = cr * pow(ps / pr, g1);
      if (0.0 <= us + cmr) {
        W[0] = rr * pow(ps / pr, 1.0 / g); W[1] = us; W[3] = ps;
      } else {
        const double cc = g5 * (cr - g7 * ur);
        W[0] = rr * pow(cc / cr, g4);
        W[1] = g5 * (-cr + g7 * ur);
        W[3] = pr * pow(cc / cr, g3);
      }
    }
  }
  phys_flux(g, rgm1, W, F);
  return true;
}

// ---------------------------------------------------------------------------
// A5-A7 for one edge: extrapolation, frame of the moving edge, Riemann solve,
// lab-frame flux times the edge length.  Returns false on a bad index or a
// vacuum in the exact solver.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void load_rec(const double* __restrict__ rec, int c, double* r) {
  const double2* p = reinterpret_cast<const double2*>(rec + (size_t)c * kRecDoubles);
#pragma unroll
  for (int k = 0; k < kRecDoubles / 2; ++k) {
    double2 v = p[k];
    r[2 * k] = v.x;
    r[2 * k + 1] = v.y;
  }
}

// The flux of edge e = (i, ej) with midpoint (fx, fy), length L, from the
// records of both sides (rj unused for a wall), which carry the points.  br,
// when not null, receives the Riemann solver's branch record.
template <int RIEMANN>
__device__ inline bool edge_flux_at(const RunDesc& d, int i, uint32_t ej, double fx, double fy,
                                    double L, const double* ri, const double* rj_in, double* LF,
                                    uint8_t* br = nullptr) {
  bool ok = true;
  const int code = (int)(ej >> 28);
  const double rix = ri[R_PX], riy = ri[R_PY];
  double phL[4], phR[4];
  {
    const double dx = fx - rix, dy = fy - riy;
#pragma unroll
    for (int q = 0; q < 4; ++q) phL[q] = ri[q] + ri[R_G + 2 * q] * dx + ri[R_G + 2 * q + 1] * dy;
  }
  double nx, ny, wex, wey;
  double WL[4], WR[4];
  if (code >= 9) {
    nx = (code == 9) ? -1.0 : (code == 10 ? 1.0 : 0.0);
    ny = (code == 11) ? -1.0 : (code == 12 ? 1.0 : 0.0);
    const double tx = -ny, ty = nx;
    const double wn = ri[R_WX] * nx + ri[R_WY] * ny;
    wex = ri[R_WX] - wn * nx;
    wey = ri[R_WY] - wn * ny;
    const double vx = phL[1] - wex, vy = phL[2] - wey;
    WL[0] = phL[0]; WL[1] = vx * nx + vy * ny; WL[2] = vx * tx + vy * ty; WL[3] = phL[3];
    WR[0] = phL[0]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = phL[3];
  } else {
    int j = (int)(ej & kCellMask);
    if (j >= d.n) {
      ok = false;
      j = i;
    }
    const double* rj = rj_in;
    double shx, shy;
    shift_of(d, code, shx, shy);
    const double rjx = rj[R_PX] + shx, rjy = rj[R_PY] + shy;
    {
      const double dx = fx - rjx, dy = fy - rjy;
#pragma unroll
      for (int q = 0; q < 4; ++q) phR[q] = rj[q] + rj[R_G + 2 * q] * dx + rj[R_G + 2 * q + 1] * dy;
    }
    const double dx = rjx - rix, dy = rjy - riy;
    const double inv_dist = rsqrt(dx * dx + dy * dy);
    nx = dx * inv_dist;
    ny = dy * inv_dist;
    const double tx = -ny, ty = nx;
    const double cx = fx - 0.5 * (rix + rjx), cy = fy - 0.5 * (riy + rjy);
    const double wix = ri[R_WX], wiy = ri[R_WY], wjx = rj[R_WX], wjy = rj[R_WY];
    const double a = ((wix - wjx) * cx + (wiy - wjy) * cy) * inv_dist;
    wex = 0.5 * (wix + wjx) + a * nx;
    wey = 0.5 * (wiy + wjy) + a * ny;
    const double vlx = phL[1] - wex, vly = phL[2] - wey;
    const double vrx = phR[1] - wex, vry = phR[2] - wey;
    WL[0] = phL[0]; WL[1] = vlx * nx + vly * ny; WL[2] = vlx * tx + vly * ty; WL[3] = phL[3];
    WR[0] = phR[0]; WR[1] = vrx * nx + vry * ny; WR[2] = vrx * tx + vry * ty; WR[3] = phR[3];
  }
  double F[4];
  if (RIEMANN == 1) {
    if (!exact_flux(d.gamma, d.rgm1, WL, WR, F, br)) ok = false;
  } else {
    hllc(d.gamma, d.rgm1, WL, WR, F, br);
  }
  const double tx = -ny, ty = nx;
  const double fpx = F[1] * nx + F[2] * tx, fpy = F[1] * ny + F[2] * ty;
  const double fm = F[0];
  const double fmx = fpx + fm * wex;
  const double fmy = fpy + fm * wey;
  const double fe = F[3] + fpx * wex + fpy * wey + 0.5 * (wex * wex + wey * wey) * fm;
  LF[0] = L * fm;
  LF[1] = L * fmx;
  LF[2] = L * fmy;
  LF[3] = L * fe;
  return ok;
}

template <int RIEMANN>
__device__ inline bool edge_flux(const RunDesc& d, int e, const double* ri, const double* rj_in,
                                 double* LF) {
  const EdgeRec er = load_edge(d, e);
  return edge_flux_at<RIEMANN>(d, er.i, er.j, er.fx, er.fy, er.L, ri, rj_in, LF);
}

}  // namespace rich
