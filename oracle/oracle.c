/*
 * oracle.c -- plain, serial, FP64 reference of one stage of RICH's moving-mesh
 * Godunov scheme.  TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
 * check and the CPU baseline of the benchmark, never by the product path.
 *
 * Each function follows a passage of the paper (Yalinewich, Steinberg & Sari,
 * "RICH: Open Source Hydrodynamic Simulation on a Moving Voronoi Mesh"):
 *   or_primitives      state of a cell from its extensive totals
 *   or_point_velocity  section 6: Lagrangian motion plus the cell-rounding
 *                      correction (parameters chi, eta)
 *   or_gradients       section 2.2, eq. (slope): Green-Gauss gradient
 *   or_limiter         section 2.2: global (AREPO) limiter, local (TESS)
 *                      limiter with theta, and the shock detector that
 *                      switches between them (delta_v, delta_p)
 *   or_edge_fluxes     section 2.2 (linear extrapolation to the edge centre),
 *                      section 1 / section 5 (flux computed in the frame of
 *                      the moving edge), section 2.4 (HLLC or exact solver)
 *   or_area_rate       section 5, eq. (areachange)
 *   or_stage           one conservative update (section 2.3)
 *   or_cfl_dt          section 2.3 (Courant condition, number 0.3)
 *   or_voronoi         section 2.1: the Voronoi cells of the mesh points, by
 *                      clipping against every other point (input stage)
 *
 * Readings of points the paper leaves open are listed where they are used.
 * Build: gcc -O2 -std=c99 -ffp-contract=off (no fast-math).
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ---------------------------------------------------------------------- */
/* mesh access                                                             */
/* ---------------------------------------------------------------------- */

static int32_t nb_cell(int32_t ej) { return (int32_t)((uint32_t)ej & 0x0FFFFFFFu); }
static int nb_code(int32_t ej) { return (int)((uint32_t)ej >> 28); }
static int is_wall(int code) { return code >= 9 && code <= 12; }

/* periodic image shift (in box lengths) of code 1..8 */
static void code_shift(int code, double* sx, double* sy) {
  int k = code <= 4 ? code - 1 : code;
  *sx = (double)(k / 3 - 1);
  *sy = (double)(k % 3 - 1);
}

/* mirror of a point across wall `code` */
static void mirror_point(const or_mesh* m, int code, double x, double y,
                         double* mx, double* my) {
  *mx = x;
  *my = y;
  if (code == 9) *mx = 2.0 * m->box[0] - x;
  if (code == 10) *mx = 2.0 * m->box[2] - x;
  if (code == 11) *my = 2.0 * m->box[1] - y;
  if (code == 12) *my = 2.0 * m->box[3] - y;
}

/* mirror of a vector across wall `code`: the normal component reverses */
static void mirror_vec(int code, double vx, double vy, double* mx, double* my) {
  *mx = (code == 9 || code == 10) ? -vx : vx;
  *my = (code == 11 || code == 12) ? -vy : vy;
}

/* The neighbour across one CSR entry of cell i, seen in i's frame. */
typedef struct {
  int32_t e;      /* edge id                                   */
  int side;       /* 0: i is e_i, 1: i is e_j                  */
  int wall;       /* wall code (9..12) or 0                    */
  int32_t j;      /* neighbour cell (i itself for a wall)      */
  double rx, ry;  /* neighbour point                           */
  double sx, sy;  /* neighbour centroid (not used for walls)   */
  double fx, fy;  /* edge midpoint                             */
  double L;       /* edge length                               */
} nb_view;

static void view(const or_mesh* m, int64_t i, int32_t entry, nb_view* v) {
  int32_t e = entry >> 1;
  int side = entry & 1;
  int32_t ej = m->e_j[e];
  int code = nb_code(ej);
  double shx = 0.0, shy = 0.0;
  if (code >= 1 && code <= 8) {
    double a, b;
    code_shift(code, &a, &b);
    shx = a * (m->box[2] - m->box[0]);
    shy = b * (m->box[3] - m->box[1]);
  }
  v->e = e;
  v->side = side;
  v->L = m->e_len[e];
  v->wall = 0;
  if (side == 0) {
    v->fx = m->e_fx[e];
    v->fy = m->e_fy[e];
    if (is_wall(code)) {
      v->wall = code;
      v->j = (int32_t)i;
      mirror_point(m, code, m->px[i], m->py[i], &v->rx, &v->ry);
      v->sx = v->rx;
      v->sy = v->ry;
    } else {
      int32_t j = nb_cell(ej);
      v->j = j;
      v->rx = m->px[j] + shx;
      v->ry = m->py[j] + shy;
      v->sx = m->sx[j] + shx;
      v->sy = m->sy[j] + shy;
    }
  } else {
    int32_t j = m->e_i[e];
    v->j = j;
    v->rx = m->px[j] - shx;
    v->ry = m->py[j] - shy;
    v->sx = m->sx[j] - shx;
    v->sy = m->sy[j] - shy;
    v->fx = m->e_fx[e] - shx;
    v->fy = m->e_fy[e] - shy;
  }
}

/* primitive values (rho, vx, vy, p) of the neighbour in a view */
static void nb_prim(const or_mesh* m, const double* prim, int64_t i,
                    const nb_view* v, double* phi) {
  int64_t n = m->n_cells;
  if (v->wall) {
    phi[0] = prim[0 * n + i];
    mirror_vec(v->wall, prim[1 * n + i], prim[2 * n + i], &phi[1], &phi[2]);
    phi[3] = prim[3 * n + i];
  } else {
    phi[0] = prim[0 * n + v->j];
    phi[1] = prim[1 * n + v->j];
    phi[2] = prim[2 * n + v->j];
    phi[3] = prim[3 * n + v->j];
  }
}

/* ---------------------------------------------------------------------- */
/* A1: primitives.  Q holds totals over the cell (mass, momentum, total    */
/* energy); the primitives are those totals divided by the cell area.      */
/* Ideal gas: p = (gamma-1) * internal energy density, c = sqrt(gamma p/rho) */
/* ---------------------------------------------------------------------- */
/* Threads the per-cell and per-edge loops run on: 1 in the serial build
 * (the reference), the OpenMP team size in the parallel build of the same
 * source (used only to time the oracle on all host cores; each iteration
 * writes only its own cell or edge, so both builds give the same bits). */
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int or_primitives(const or_mesh* m, const double* Q, const or_params* p, double* prim) {
  int64_t n = m->n_cells;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double A = m->area[i];
    double M = Q[i], Px = Q[n + i], Py = Q[2 * n + i], E = Q[3 * n + i];
    double rho = M / A;
    double vx = Px / M, vy = Py / M;
    double pr = (p->gamma - 1.0) * (E / A - 0.5 * rho * (vx * vx + vy * vy));
    prim[i] = rho;
    prim[n + i] = vx;
    prim[2 * n + i] = vy;
    prim[3 * n + i] = pr;
    prim[4 * n + i] = sqrt(p->gamma * pr / rho);
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* A2: mesh-point velocity (section 6).  Lagrangian motion w = v, plus a    */
/* velocity chi * c_s towards the cell's centre of mass when the point is   */
/* farther than eta * R from it; R = sqrt(A/pi) is the cell radius.         */
/* ---------------------------------------------------------------------- */
int or_point_velocity(const or_mesh* m, const double* prim, const or_params* p,
                      double* w) {
  int64_t n = m->n_cells;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    if (p->motion == 0) {
      w[i] = 0.0;
      w[n + i] = 0.0;
      continue;
    }
    double wx = prim[n + i], wy = prim[2 * n + i];
    double dx = m->sx[i] - m->px[i], dy = m->sy[i] - m->py[i];
    double d = sqrt(dx * dx + dy * dy);
    double R = sqrt(m->area[i] / OR_PI);
    if (d > p->eta * R) {
      double c = prim[4 * n + i];
      wx += p->chi * c * dx / d;
      wy += p->chi * c * dy / d;
    }
    w[i] = wx;
    w[n + i] = wy;
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* A3: Green-Gauss gradient, eq. (slope):                                   */
/*   grad_i = (1/A_i) sum_j L_ij ( [phi_j - phi_i] c_ij/|r_ij|              */
/*                                 - (phi_i + phi_j)/2 * r_ij/|r_ij| )      */
/* with r_ij = r_i - r_j and c_ij the vector from the midpoint of the two   */
/* points to the edge centre (the reading under which a linear field gets   */
/* its exact gradient).  Wall neighbours are mirror images of the cell.     */
/* ---------------------------------------------------------------------- */
int or_gradients(const or_mesh* m, const double* prim, double* grad) {
  int64_t n = m->n_cells;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double phi_i[4] = {prim[i], prim[n + i], prim[2 * n + i], prim[3 * n + i]};
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t k = m->off[i]; k < m->off[i + 1]; ++k) {
      nb_view v;
      view(m, i, m->idx[k], &v);
      double phi_j[4];
      nb_prim(m, prim, i, &v, phi_j);
      double rx = m->px[i] - v.rx, ry = m->py[i] - v.ry;
      double r = sqrt(rx * rx + ry * ry);
      double cx = v.fx - 0.5 * (m->px[i] + v.rx);
      double cy = v.fy - 0.5 * (m->py[i] + v.ry);
      for (int q = 0; q < 4; ++q) {
        double dphi = phi_j[q] - phi_i[q];
        double mean = 0.5 * (phi_i[q] + phi_j[q]);
        g[2 * q] += v.L * (dphi * cx / r - mean * rx / r);
        g[2 * q + 1] += v.L * (dphi * cy / r - mean * ry / r);
      }
    }
    for (int q = 0; q < 8; ++q) grad[(int64_t)q * n + i] = g[q] / m->area[i];
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* A4: slope limiter (section 2.2).                                         */
/* Global (AREPO): psi_ij = (phi_max - phi_i)/dphi_ij if dphi_ij > 0,       */
/*   (phi_min - phi_i)/dphi_ij if dphi_ij < 0, 1 if dphi_ij = 0, where      */
/*   dphi_ij = grad_i . (edge centre - centre of mass) is the unlimited      */
/*   change to the edge; phi_max / phi_min run over the neighbours and the  */
/*   cell itself (so that alpha stays in [0, 1]).                           */
/* Local (TESS): psi_ij = max(theta (phi_j - phi_i)/dphi_ij, 0), 1 if       */
/*   dphi_ij = 0.                                                           */
/* alpha_i = min(1, min_j psi_ij), per reconstructed variable.              */
/* Shock detector: a cell uses the local limiter for all variables when     */
/*   -(div v) > delta_v c_s / R  or when for some neighbour the smaller of  */
/*   the two pressures divided by the larger is below delta_p; the          */
/*   divergence comes from the unlimited gradients.                         */
/* ---------------------------------------------------------------------- */
int or_limiter(const or_mesh* m, const double* prim, const double* grad,
               const or_params* p, double* alpha, int32_t* flag) {
  int64_t n = m->n_cells;
  #pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double phi_i[4] = {prim[i], prim[n + i], prim[2 * n + i], prim[3 * n + i]};
    double G[8];
    for (int q = 0; q < 8; ++q) G[q] = grad[(int64_t)q * n + i];
    double ci = prim[4 * n + i];
    double R = sqrt(m->area[i] / OR_PI);

    int shock = (-(G[2] + G[5]) > p->delta_v * ci / R);
    double pmax[4], pmin[4];
    for (int q = 0; q < 4; ++q) pmax[q] = pmin[q] = phi_i[q];
    for (int32_t k = m->off[i]; k < m->off[i + 1]; ++k) {
      nb_view v;
      view(m, i, m->idx[k], &v);
      double phi_j[4];
      nb_prim(m, prim, i, &v, phi_j);
      for (int q = 0; q < 4; ++q) {
        if (phi_j[q] > pmax[q]) pmax[q] = phi_j[q];
        if (phi_j[q] < pmin[q]) pmin[q] = phi_j[q];
      }
      double pi_ = phi_i[3], pj = phi_j[3];
      double ratio = 1.0;
      if (pj > pi_) ratio = pi_ / pj;
      if (pi_ > pj) ratio = pj / pi_;
      if (p->delta_p > ratio) shock = 1;
    }
    if (flag) flag[i] = shock;

    int local;
    switch (p->limiter) {
      case 0: local = shock; break;
      case 1: local = 0; break;
      case 2: local = 1; break;
      default: local = -1; break;
    }
    for (int q = 0; q < 4; ++q) {
      double a = 1.0;
      if (p->limiter == 4) a = 0.0;
      if (local >= 0) {
        for (int32_t k = m->off[i]; k < m->off[i + 1]; ++k) {
          nb_view v;
          view(m, i, m->idx[k], &v);
          double phi_j[4];
          nb_prim(m, prim, i, &v, phi_j);
          double dphi = G[2 * q] * (v.fx - m->sx[i]) + G[2 * q + 1] * (v.fy - m->sy[i]);
          double psi;
          if (local) {
            psi = (dphi != 0.0) ? fmax(p->theta * (phi_j[q] - phi_i[q]) / dphi, 0.0) : 1.0;
          } else if (dphi > 0.0) {
            psi = (pmax[q] - phi_i[q]) / dphi;
          } else if (dphi < 0.0) {
            psi = (pmin[q] - phi_i[q]) / dphi;
          } else {
            psi = 1.0;
          }
          if (psi < a) a = psi;
        }
      }
      alpha[(int64_t)q * n + i] = a;
    }
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Riemann solvers in the frame of the edge (section 2.4).                  */
/* W = (rho, u, vt, p); u along the edge normal, vt the passive tangential  */
/* velocity.  Flux = (rho u, rho u^2 + p, rho u vt, u (E + p)) with          */
/* E = p/(gamma-1) + rho (u^2 + vt^2)/2.                                    */
/* ---------------------------------------------------------------------- */
static void phys_flux(double g, const double* W, double* F) {
  double rho = W[0], u = W[1], vt = W[2], pr = W[3];
  double E = pr / (g - 1.0) + 0.5 * rho * (u * u + vt * vt);
  F[0] = rho * u;
  F[1] = rho * u * u + pr;
  F[2] = rho * u * vt;
  F[3] = u * (E + pr);
}

/* HLLC (Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics,
 * ch. 10).  Wave speeds S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L,
 * u_R + c_R) use only the sound speeds; S* from the momentum balance across
 * both outer waves; the star-region flux is the flux of the star state with
 * pressure p*_K = p_K + rho_K (S_K - u_K)(S* - u_K), which equals the
 * Rankine-Hugoniot form F_K + S_K (U*_K - U_K). */
static void hllc_speeds(double g, const double* WL, const double* WR, double* sl,
                        double* ss, double* sr) {
  double rl = WL[0], ul = WL[1], pl = WL[3];
  double rr = WR[0], ur = WR[1], pr = WR[3];
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  *sl = fmin(ul - cl, ur - cr);
  *sr = fmax(ul + cl, ur + cr);
  *ss = (pr - pl + rl * ul * (*sl - ul) - rr * ur * (*sr - ur)) /
        (rl * (*sl - ul) - rr * (*sr - ur));
}

void or_hllc(double g, const double* WL, const double* WR, double* F) {
  double sl, ss, sr;
  hllc_speeds(g, WL, WR, &sl, &ss, &sr);
  /* branch order: 0 <= S_L -> F_L; 0 <= S* -> F*_L; 0 < S_R -> F*_R; F_R */
  if (0.0 <= sl) {
    phys_flux(g, WL, F);
    return;
  }
  if (!(0.0 <= ss) && !(0.0 < sr)) {
    phys_flux(g, WR, F);
    return;
  }
  const double* W = (0.0 <= ss) ? WL : WR;
  double sk = (0.0 <= ss) ? sl : sr;
  double rho = W[0], u = W[1], vt = W[2], pk = W[3];
  double E = pk / (g - 1.0) + 0.5 * rho * (u * u + vt * vt);
  double rs = rho * (sk - u) / (sk - ss);
  double ps = pk + rho * (sk - u) * (ss - u);
  double Es = rs * (E / rho + (ss - u) * (ss + pk / (rho * (sk - u))));
  F[0] = rs * ss;
  F[1] = rs * ss * ss + ps;
  F[2] = rs * ss * vt;
  F[3] = (Es + ps) * ss;
}

/* Exact solver (Toro ch. 4): the star pressure solves
 *   f_L(p) + f_R(p) + (u_R - u_L) = 0,
 * f_K(p) = (p - p_K) sqrt(A_K / (p + B_K))            (shock,  p > p_K)
 *        = 2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2gamma)) - 1)  (rarefaction),
 * A_K = 2/((gamma+1) rho_K), B_K = (gamma-1)/(gamma+1) p_K.  Newton from the
 * primitive-variable guess (clipped at 1e-14), stopped when the relative change
 * falls below 1e-14 or after 50 iterations. */
static void pfun(double g, double pstar, double rk, double pk, double ck,
                 double* f, double* fd) {
  if (pstar > pk) {
    double A = 2.0 / ((g + 1.0) * rk), B = (g - 1.0) / (g + 1.0) * pk;
    double q = sqrt(A / (pstar + B));
    *f = (pstar - pk) * q;
    *fd = q * (1.0 - 0.5 * (pstar - pk) / (B + pstar));
  } else {
    double pr = pstar / pk;
    *f = 2.0 * ck / (g - 1.0) * (pow(pr, (g - 1.0) / (2.0 * g)) - 1.0);
    *fd = 1.0 / (rk * ck) * pow(pr, -(g + 1.0) / (2.0 * g));
  }
}

static int star_state(double g, const double* WL, const double* WR, double* ps,
                      double* us) {
  double rl = WL[0], ul = WL[1], pl = WL[3];
  double rr = WR[0], ur = WR[1], pr = WR[3];
  double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
  if (2.0 / (g - 1.0) * (cl + cr) <= ur - ul) return -1;
  const double tiny = 1e-14;
  double p = 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr);
  if (p < tiny) p = tiny;
  int it = 0;
  for (it = 1; it <= 50; ++it) {
    double fl, fld, fr, frd;
    pfun(g, p, rl, pl, cl, &fl, &fld);
    pfun(g, p, rr, pr, cr, &fr, &frd);
    double pn = p - (fl + fr + ur - ul) / (fld + frd);
    if (pn < tiny) pn = tiny;
    double change = 2.0 * fabs(pn - p) / (pn + p);
    p = pn;
    if (change < 1e-14) break;
  }
  double fl, fld, fr, frd;
  pfun(g, p, rl, pl, cl, &fl, &fld);
  pfun(g, p, rr, pr, cr, &fr, &frd);
  *ps = p;
  *us = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  return it;
}

/* Sample the self-similar solution at x/t = xi (Toro ch. 4 sampling). */
static void sample(double g, const double* WL, const double* WR, double ps,
                   double us, double xi, double* W) {
  double g1 = (g - 1.0) / (2.0 * g), g2 = (g + 1.0) / (2.0 * g);
  double g3 = 2.0 * g / (g - 1.0), g4 = 2.0 / (g - 1.0), g5 = 2.0 / (g + 1.0);
  double g6 = (g - 1.0) / (g + 1.0), g7 = (g - 1.0) / 2.0;
  if (xi <= us) { /* left of the contact */
    double rl = WL[0], ul = WL[1], pl = WL[3];
    double cl = sqrt(g * pl / rl);
    W[2] = WL[2];
    if (ps > pl) { /* left shock */
      double sl = ul - cl * sqrt(g2 * ps / pl + g1);
      if (xi <= sl) {
        W[0] = rl; W[1] = ul; W[3] = pl;
      } else {
        W[0] = rl * (ps / pl + g6) / (g6 * ps / pl + 1.0);
        W[1] = us; W[3] = ps;
      }
    } else { /* left rarefaction */
      double shl = ul - cl;
      if (xi <= shl) {
        W[0] = rl; W[1] = ul; W[3] = pl;
      } else {
        double cml = cl * pow(ps / pl, g1);
        double stl = us - cml;
        if (xi > stl) {
          W[0] = rl * pow(ps / pl, 1.0 / g);
          W[1] = us; W[3] = ps;
        } else {
          double c = g5 * (cl + g7 * (ul - xi));
          W[0] = rl * pow(c / cl, g4);
          W[1] = g5 * (cl + g7 * ul + xi);
          W[3] = pl * pow(c / cl, g3);
        }
      }
    }
  } else { /* right of the contact */
    double rr = WR[0], ur = WR[1], pr = WR[3];
    double cr = sqrt(g * pr / rr);
    W[2] = WR[2];
    if (ps > pr) { /* right shock */
      double sr = ur + cr * sqrt(g2 * ps / pr + g1);
      if (xi >= sr) {
        W[0] = rr; W[1] = ur; W[3] = pr;
      } else {
        W[0] = rr * (ps / pr + g6) / (g6 * ps / pr + 1.0);
        W[1] = us; W[3] = ps;
      }
    } else { /* right rarefaction */
      double shr = ur + cr;
      if (xi >= shr) {
        W[0] = rr; W[1] = ur; W[3] = pr;
      } else {
        double cmr = cr * pow(ps / pr, g1);
        double str = us + cmr;
        if (xi <= str) {
          W[0] = rr * pow(ps / pr, 1.0 / g);
          W[1] = us; W[3] = ps;
        } else {
          double c = g5 * (cr - g7 * (ur - xi));
          W[0] = rr * pow(c / cr, g4);
          W[1] = g5 * (-cr + g7 * ur + xi);
          W[3] = pr * pow(c / cr, g3);
        }
      }
    }
  }
}

int or_exact_sample(double g, const double* WL, const double* WR, double xi, double* W) {
  double ps, us;
  int it = star_state(g, WL, WR, &ps, &us);
  if (it < 0) return -1;
  sample(g, WL, WR, ps, us, xi, W);
  return it;
}

int or_exact(double g, const double* WL, const double* WR, double* F, double* star) {
  double ps, us;
  int it = star_state(g, WL, WR, &ps, &us);
  if (it < 0) {
    F[0] = F[1] = F[2] = F[3] = NAN;
    return -1;
  }
  if (star) {
    star[0] = ps;
    star[1] = us;
  }
  double W[4];
  sample(g, WL, WR, ps, us, 0.0, W);
  phys_flux(g, W, F);
  return it;
}

/* ---------------------------------------------------------------------- */
/* A5-A7: per-edge flux.                                                    */
/* Extrapolation (section 2.2): phi_face = phi_i + (alpha grad)_i . (f - s_i) */
/* with f the edge centre and s_i the cell's centre of mass.                */
/* Edge velocity (section 5): the edge lies on the perpendicular bisector   */
/* of the two points; its velocity at the edge centre is                    */
/*   w_e = (w_i + w_j)/2 + [(w_i - w_j) . c_ij / |r_j - r_i|] n,            */
/* n = (r_j - r_i)/|r_j - r_i|, whose normal component is the integrand of  */
/* eq. (areachange).  The states are boosted by -w_e, rotated into (n, t),  */
/* the 1D Riemann problem is solved, and the flux through the moving edge   */
/* is transformed back to the lab frame:                                    */
/*   F_M = F'_m,  F_P = F'_P + F'_m w_e,  F_E = F'_E + F'_P . w_e + |w_e|^2 F'_m / 2. */
/* Reflecting wall: the ghost is the mirror image of the cell, so the right */
/* state is the left one with its normal velocity reversed, and the edge    */
/* moves only tangentially (w_e = tangential part of w_i).                  */
/* ---------------------------------------------------------------------- */
static void face_state(const double* prim, const double* lgrad, int64_t n, int64_t i,
                       double dx, double dy, double* phi) {
  for (int q = 0; q < 4; ++q)
    phi[q] = prim[(int64_t)q * n + i] + lgrad[(int64_t)(2 * q) * n + i] * dx +
             lgrad[(int64_t)(2 * q + 1) * n + i] * dy;
}

/* The Riemann states of edge e in its own frame (WL on e_i's side), the
 * edge normal (nx, ny) and the edge velocity (wex, wey). */
static void edge_frame(const or_mesh* m, const double* prim, const double* lgrad,
                       const double* w, int64_t e, double* WL, double* WR, double* nx_out,
                       double* ny_out, double* wex_out, double* wey_out) {
  int64_t n = m->n_cells;
  double Lx = m->box[2] - m->box[0], Ly = m->box[3] - m->box[1];
  int64_t i = m->e_i[e];
  int code = nb_code(m->e_j[e]);
  double fx = m->e_fx[e], fy = m->e_fy[e];
  double phiL[4], phiR[4];
  face_state(prim, lgrad, n, i, fx - m->sx[i], fy - m->sy[i], phiL);
  double nx, ny, wex, wey;
  if (is_wall(code)) {
    nx = (code == 9) ? -1.0 : (code == 10 ? 1.0 : 0.0);
    ny = (code == 11) ? -1.0 : (code == 12 ? 1.0 : 0.0);
    double tx = -ny, ty = nx;
    double wn = w[i] * nx + w[n + i] * ny;
    wex = w[i] - wn * nx;
    wey = w[n + i] - wn * ny;
    double vx = phiL[1] - wex, vy = phiL[2] - wey;
    WL[0] = phiL[0]; WL[1] = vx * nx + vy * ny; WL[2] = vx * tx + vy * ty; WL[3] = phiL[3];
    WR[0] = phiL[0]; WR[1] = -WL[1]; WR[2] = WL[2]; WR[3] = phiL[3];
  } else {
    int64_t j = nb_cell(m->e_j[e]);
    double shx = 0.0, shy = 0.0;
    if (code >= 1 && code <= 8) {
      double a, b;
      code_shift(code, &a, &b);
      shx = a * Lx;
      shy = b * Ly;
    }
    double rjx = m->px[j] + shx, rjy = m->py[j] + shy;
    double sjx = m->sx[j] + shx, sjy = m->sy[j] + shy;
    face_state(prim, lgrad, n, j, fx - sjx, fy - sjy, phiR);
    double dx = rjx - m->px[i], dy = rjy - m->py[i];
    double d = sqrt(dx * dx + dy * dy);
    nx = dx / d;
    ny = dy / d;
    double tx = -ny, ty = nx;
    double cx = fx - 0.5 * (m->px[i] + rjx), cy = fy - 0.5 * (m->py[i] + rjy);
    double wix = w[i], wiy = w[n + i], wjx = w[j], wjy = w[n + j];
    double a = ((wix - wjx) * cx + (wiy - wjy) * cy) / d;
    wex = 0.5 * (wix + wjx) + a * nx;
    wey = 0.5 * (wiy + wjy) + a * ny;
    double vlx = phiL[1] - wex, vly = phiL[2] - wey;
    double vrx = phiR[1] - wex, vry = phiR[2] - wey;
    WL[0] = phiL[0]; WL[1] = vlx * nx + vly * ny; WL[2] = vlx * tx + vly * ty; WL[3] = phiL[3];
    WR[0] = phiR[0]; WR[1] = vrx * nx + vry * ny; WR[2] = vrx * tx + vry * ty; WR[3] = phiR[3];
  }
  *nx_out = nx;
  *ny_out = ny;
  *wex_out = wex;
  *wey_out = wey;
}

int or_edge_fluxes(const or_mesh* m, const double* prim, const double* lgrad,
                   const double* w, const or_params* p, double* flux) {
  int64_t ne = m->n_edges;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t e = 0; e < ne; ++e) {
    double WL[4], WR[4], nx, ny, wex, wey;
    edge_frame(m, prim, lgrad, w, e, WL, WR, &nx, &ny, &wex, &wey);
    double F[4];
    if (p->riemann == 1) {
      if (or_exact(p->gamma, WL, WR, F, NULL) < 0) bad = 1;
    } else {
      or_hllc(p->gamma, WL, WR, F);
    }
    double tx = -ny, ty = nx;
    double fpx = F[1] * nx + F[2] * tx, fpy = F[1] * ny + F[2] * ty;
    flux[e] = F[0];
    flux[ne + e] = fpx + F[0] * wex;
    flux[2 * ne + e] = fpy + F[0] * wey;
    flux[3 * ne + e] = F[3] + fpx * wex + fpy * wey + 0.5 * (wex * wex + wey * wey) * F[0];
  }
  return bad ? OR_E_DOMAIN : OR_OK;
}

/* The quantities whose signs pick the Riemann solver's branch on every edge
 * (section 2.4), for comparing branch records: HLLC S_L, S*, S_R; exact
 * solver NaN, u*, NaN; and a velocity scale |u_L| + c_L + |u_R| + c_R of the
 * edge's two states. */
int or_edge_waves(const or_mesh* m, const double* prim, const double* lgrad,
                  const double* w, const or_params* p, double* waves) {
  int64_t ne = m->n_edges;
  int bad = 0;
  for (int64_t e = 0; e < ne; ++e) {
    double WL[4], WR[4], nx, ny, wex, wey;
    edge_frame(m, prim, lgrad, w, e, WL, WR, &nx, &ny, &wex, &wey);
    double sl = NAN, ss = NAN, sr = NAN;
    if (p->riemann == 1) {
      double F[4], star[2] = {NAN, NAN};
      if (or_exact(p->gamma, WL, WR, F, star) < 0) bad = 1;
      ss = star[1];
    } else {
      hllc_speeds(p->gamma, WL, WR, &sl, &ss, &sr);
    }
    waves[e] = sl;
    waves[ne + e] = ss;
    waves[2 * ne + e] = sr;
    waves[3 * ne + e] = fabs(WL[1]) + sqrt(p->gamma * WL[3] / WL[0]) + fabs(WR[1]) +
                        sqrt(p->gamma * WR[3] / WR[0]);
  }
  return bad ? OR_E_DOMAIN : OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Eq. (areachange), section 5, read with r_ij = r_j - r_i (the sign under  */
/* which it equals the rate of change of the cell area):                    */
/*   dA_i/dt = - sum_j L_ij ( [w_j - w_i] . c_ij/|r_ij|                     */
/*                            - (w_i + w_j)/2 . r_ij/|r_ij| ).              */
/* ---------------------------------------------------------------------- */
int or_area_rate(const or_mesh* m, const double* w, double* adot) {
  int64_t n = m->n_cells;
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (int32_t k = m->off[i]; k < m->off[i + 1]; ++k) {
      nb_view v;
      view(m, i, m->idx[k], &v);
      double wjx, wjy;
      if (v.wall) {
        mirror_vec(v.wall, w[i], w[n + i], &wjx, &wjy);
      } else {
        wjx = w[v.j];
        wjy = w[n + v.j];
      }
      double rx = v.rx - m->px[i], ry = v.ry - m->py[i];
      double r = sqrt(rx * rx + ry * ry);
      double cx = v.fx - 0.5 * (m->px[i] + v.rx);
      double cy = v.fy - 0.5 * (m->py[i] + v.ry);
      double t1 = ((wjx - w[i]) * cx + (wjy - w[n + i]) * cy) / r;
      double t2 = (0.5 * (w[i] + wjx) * rx + 0.5 * (w[n + i] + wjy) * ry) / r;
      s -= v.L * (t1 - t2);
    }
    adot[i] = s;
  }
  return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* One stage (section 2.3): primitives of Qsrc on this mesh, point          */
/* velocities, gradients, limiter, fluxes through every edge, then          */
/*   Qout_i = Qbase_i - h sum_{edges of i} (+/-) L_e F_e                    */
/* summed in the cell's CSR order (+ when i is the edge's first side), and  */
/*   Xout_i = Xbase_i + h w_i  (wrapped into a periodic box).               */
/* ---------------------------------------------------------------------- */
static double wrap(double v, double lo, double hi) {
  double L = hi - lo;
  while (v < lo) v += L;
  while (v >= hi) v -= L;
  return v;
}

/* ---------------------------------------------------------------------- */
/* Extrapolated fluxes (section 2.3): the spatial derivatives are put into  */
/* the hydrodynamic equations to get the time derivatives of the            */
/* primitives, and the values are advanced by half a step before they are   */
/* extrapolated to the edges.  Reading: the primitive Euler equations with  */
/* the limited gradients, the time derivative taken along the motion of the */
/* cell's point w (so the advection uses v - w):                            */
/*   d rho/dt = -(v - w).grad rho - rho div v                               */
/*   d v/dt   = -((v - w).grad) v - grad p / rho                            */
/*   d p/dt   = -(v - w).grad p - gamma p div v                             */
/* ---------------------------------------------------------------------- */
static void half_step_primitives(const or_mesh* m, const double* prim, const double* lgrad,
                                 const double* w, double gamma, double half_h,
                                 double* out) {
  int64_t n = m->n_cells;
  memcpy(out, prim, sizeof(double) * 5 * (size_t)n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double rho = prim[i], vx = prim[n + i], vy = prim[2 * n + i], pr = prim[3 * n + i];
    double ux = vx - w[i], uy = vy - w[n + i];
    double drx = lgrad[i], dry = lgrad[n + i];
    double dvxx = lgrad[2 * n + i], dvxy = lgrad[3 * n + i];
    double dvyx = lgrad[4 * n + i], dvyy = lgrad[5 * n + i];
    double dpx = lgrad[6 * n + i], dpy = lgrad[7 * n + i];
    double div = dvxx + dvyy;
    double rho_t = -(ux * drx + uy * dry) - rho * div;
    double vx_t = -(ux * dvxx + uy * dvxy) - dpx / rho;
    double vy_t = -(ux * dvyx + uy * dvyy) - dpy / rho;
    double p_t = -(ux * dpx + uy * dpy) - gamma * pr * div;
    out[i] = rho + half_h * rho_t;
    out[n + i] = vx + half_h * vx_t;
    out[2 * n + i] = vy + half_h * vy_t;
    out[3 * n + i] = pr + half_h * p_t;
  }
}

static int stage(const or_mesh* m, const double* Qsrc, const double* Qbase,
                 const double* Xbase, double h, const or_params* p, const double* ax,
                 const double* ay, double* Qout, double* Xout, double* d_prim, double* d_w,
                 double* d_alpha, int32_t* d_flag, double* d_flux) {
  if (!m || !Qsrc || !Qbase || !Xbase || !p || !Qout || !Xout) return OR_E_INVAL;
  if ((ax == NULL) != (ay == NULL)) return OR_E_INVAL;
  int64_t n = m->n_cells, ne = m->n_edges;
  double* prim = malloc(sizeof(double) * 5 * (size_t)n);
  double* w = malloc(sizeof(double) * 2 * (size_t)n);
  double* grad = malloc(sizeof(double) * 8 * (size_t)n);
  double* alpha = malloc(sizeof(double) * 4 * (size_t)n);
  int32_t* flag = malloc(sizeof(int32_t) * (size_t)n);
  double* flux = malloc(sizeof(double) * 4 * (size_t)(ne > 0 ? ne : 1));
  if (!prim || !w || !grad || !alpha || !flag || !flux) {
    free(prim); free(w); free(grad); free(alpha); free(flag); free(flux);
    return OR_E_INVAL;
  }
  or_primitives(m, Qsrc, p, prim);
  or_point_velocity(m, prim, p, w);
  or_gradients(m, prim, grad);
  or_limiter(m, prim, grad, p, alpha, flag);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int q = 0; q < 8; ++q) grad[(int64_t)q * n + i] *= alpha[(int64_t)(q / 2) * n + i];
  const double* fprim = prim;
  double* prim_h = NULL;
  if (p->integrator == 1) {
    prim_h = malloc(sizeof(double) * 5 * (size_t)n);
    if (!prim_h) {
      free(prim); free(w); free(grad); free(alpha); free(flag); free(flux);
      return OR_E_INVAL;
    }
    half_step_primitives(m, prim, grad, w, p->gamma, 0.5 * h, prim_h);
    fprim = prim_h;
  }
  int st = or_edge_fluxes(m, fprim, grad, w, p, flux);
  free(prim_h);

  int dom = 0;
#pragma omp parallel for schedule(static) reduction(| : dom)
  for (int64_t i = 0; i < n; ++i) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t k = m->off[i]; k < m->off[i + 1]; ++k) {
      int32_t e = m->idx[k] >> 1;
      double sgn = (m->idx[k] & 1) ? -1.0 : 1.0;
      for (int q = 0; q < 4; ++q) acc[q] += sgn * m->e_len[e] * flux[(int64_t)q * ne + e];
    }
    for (int q = 0; q < 4; ++q) Qout[(int64_t)q * n + i] = Qbase[(int64_t)q * n + i] - h * acc[q];
    /* External acceleration (section 2.3): the source only needs first-order
     * accuracy in time, because the time-centred composition makes it second
     * order.  Reading: each stage adds h * S(Q_src), with S = (0, M g, P.g)
     * from the stage's source totals (the force on the cell and its work);
     * g is the uniform acceleration plus the cell's own (ax, ay) if given. */
    double gx = p->gx, gy = p->gy;
    if (ax) {
      gx += ax[i];
      gy += ay[i];
    }
    if (gx != 0.0 || gy != 0.0) {
      double sm = Qsrc[i], spx = Qsrc[n + i], spy = Qsrc[2 * n + i];
      Qout[n + i] += h * (sm * gx);
      Qout[2 * n + i] += h * (sm * gy);
      Qout[3 * n + i] += h * (spx * gx + spy * gy);
    }
    double x = Xbase[i] + h * w[i], y = Xbase[n + i] + h * w[n + i];
    if (m->bc == 1) {
      x = wrap(x, m->box[0], m->box[2]);
      y = wrap(y, m->box[1], m->box[3]);
    }
    Xout[i] = x;
    Xout[n + i] = y;
    double M = Qout[i], Px = Qout[n + i], Py = Qout[2 * n + i], E = Qout[3 * n + i];
    double eint = E - 0.5 * (Px * Px + Py * Py) / M;
    if (!(M > 0.0) || !(eint > 0.0) || !isfinite(E) || !isfinite(Px) ||
        !isfinite(Py) || !isfinite(x) || !isfinite(y))
      dom = 1;
  }
  if (dom) st = OR_E_DOMAIN;
  if (d_prim) memcpy(d_prim, prim, sizeof(double) * 5 * (size_t)n);
  if (d_w) memcpy(d_w, w, sizeof(double) * 2 * (size_t)n);
  if (d_alpha) memcpy(d_alpha, alpha, sizeof(double) * 4 * (size_t)n);
  if (d_flag) memcpy(d_flag, flag, sizeof(int32_t) * (size_t)n);
  if (d_flux) memcpy(d_flux, flux, sizeof(double) * 4 * (size_t)ne);
  free(prim); free(w); free(grad); free(alpha); free(flag); free(flux);
  return st;
}

int or_stage(const or_mesh* m, const double* Qsrc, const double* Qbase,
             const double* Xbase, double h, const or_params* p, double* Qout,
             double* Xout, double* d_prim, double* d_w, double* d_alpha,
             int32_t* d_flag, double* d_flux) {
  return stage(m, Qsrc, Qbase, Xbase, h, p, NULL, NULL, Qout, Xout, d_prim, d_w, d_alpha,
               d_flag, d_flux);
}

int or_stage_accel(const or_mesh* m, const double* Qsrc, const double* Qbase,
                   const double* Xbase, double h, const or_params* p, const double* ax,
                   const double* ay, double* Qout, double* Xout) {
  if (!ax || !ay) return OR_E_INVAL;
  return stage(m, Qsrc, Qbase, Xbase, h, p, ax, ay, Qout, Xout, NULL, NULL, NULL, NULL, NULL);
}

/* ---------------------------------------------------------------------- */
/* A0: Courant condition (section 2.3; the paper gives the number, 0.3 by   */
/* default, but not the formula): dt = cfl * min_i R_i / (c_i + |v_i - w_i|) */
/* ---------------------------------------------------------------------- */
int or_cfl_dt(const or_mesh* m, const double* Q, const or_params* p, double* dt) {
  int64_t n = m->n_cells;
  double* prim = malloc(sizeof(double) * 5 * (size_t)n);
  double* w = malloc(sizeof(double) * 2 * (size_t)n);
  if (!prim || !w) {
    free(prim); free(w);
    return OR_E_INVAL;
  }
  or_primitives(m, Q, p, prim);
  or_point_velocity(m, prim, p, w);
  double best = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    double R = sqrt(m->area[i] / OR_PI);
    double ux = prim[n + i] - w[i], uy = prim[2 * n + i] - w[n + i];
    double s = prim[4 * n + i] + sqrt(ux * ux + uy * uy);
    double t = R / s;
    /* a cell with no positive finite Courant time (no real sound speed, or
       a gas at rest with zero pressure) leaves the step undefined */
    if (!(t > 0.0) || !isfinite(t)) t = 0.0;
    if (t < best) best = t;
  }
  *dt = p->cfl * best;
  free(prim);
  free(w);
  return isfinite(*dt) && *dt > 0.0 ? OR_OK : OR_E_DOMAIN;
}

/* ---------------------------------------------------------------------- */
/* Voronoi mesh by definition (section 2.1)                                 */
/* ---------------------------------------------------------------------- */

/* A convex polygon around the point, in coordinates relative to it, and the
   neighbour label of the edge from vertex k to vertex k+1. */
#define OR_VMAX 256
typedef struct {
  int nv;
  double x[OR_VMAX], y[OR_VMAX];
  int32_t lab[OR_VMAX];
} or_poly;

/* Keeps the part of the polygon where (x, y) . (ax, ay) <= b, labelling the
   new edge `lab`.  Sutherland-Hodgman for one half-plane. */
static int or_clip(or_poly* P, double ax, double ay, double b, int32_t lab) {
  or_poly Q;
  Q.nv = 0;
  int any_out = 0;
  for (int k = 0; k < P->nv; ++k)
    if (P->x[k] * ax + P->y[k] * ay - b > 0.0) any_out = 1;
  if (!any_out) return 0;
  for (int k = 0; k < P->nv; ++k) {
    int k1 = (k + 1) % P->nv;
    double s0 = P->x[k] * ax + P->y[k] * ay - b;
    double s1 = P->x[k1] * ax + P->y[k1] * ay - b;
    if (s0 <= 0.0) {
      if (Q.nv >= OR_VMAX) return -1;
      Q.x[Q.nv] = P->x[k]; Q.y[Q.nv] = P->y[k]; Q.lab[Q.nv] = P->lab[k]; ++Q.nv;
    }
    if ((s0 <= 0.0) != (s1 <= 0.0)) {
      /* the edge k -> k1 crosses the line: new vertex there */
      double t = s0 / (s0 - s1);
      if (Q.nv >= OR_VMAX) return -1;
      Q.x[Q.nv] = P->x[k] + t * (P->x[k1] - P->x[k]);
      Q.y[Q.nv] = P->y[k] + t * (P->y[k1] - P->y[k]);
      /* leaving the kept side: the new edge follows this vertex;
         entering it: the old edge's label continues */
      Q.lab[Q.nv] = s0 <= 0.0 ? lab : P->lab[k];
      ++Q.nv;
    }
  }
  *P = Q;
  return 0;
}

int or_voronoi(int64_t n, const double* px, const double* py, const double* box,
               uint32_t bc, int32_t max_fan, double* area, double* sx, double* sy,
               int32_t* deg, int32_t* nb, double* len, double* fx, double* fy) {
  if (n < 1 || !px || !py || !box || max_fan < 1 || !area || !sx || !sy || !deg || !nb ||
      !len || !fx || !fy)
    return OR_E_INVAL;
  const double Lx = box[2] - box[0], Ly = box[3] - box[1];
  if (!(Lx > 0.0) || !(Ly > 0.0) || (bc != 0 && bc != 1)) return OR_E_INVAL;
  or_poly* P = malloc(sizeof(or_poly));
  int32_t* fan = malloc(sizeof(int32_t) * (size_t)n * OR_VMAX);
  double* vx = malloc(sizeof(double) * (size_t)n * OR_VMAX);
  double* vy = malloc(sizeof(double) * (size_t)n * OR_VMAX);
  int32_t* nv = malloc(sizeof(int32_t) * (size_t)n);
  if (!P || !fan || !vx || !vy || !nv) {
    free(P); free(fan); free(vx); free(vy); free(nv);
    return OR_E_INVAL;
  }
  int st = OR_OK;
  for (int64_t i = 0; i < n && st == OR_OK; ++i) {
    const double xi = px[i], yi = py[i];
    /* the region the cell cannot leave, counter-clockwise from its lower
       left corner: the box (walls), or the bisectors with the point's own
       nearest images (periodic) */
    double hx0, hx1, hy0, hy1;
    int32_t lb, lr, lt, ll;
    if (bc == 0) {
      hx0 = box[0] - xi; hx1 = box[2] - xi; hy0 = box[1] - yi; hy1 = box[3] - yi;
      lb = (int32_t)((uint32_t)i | (11u << 28));   /* y0 wall */
      lr = (int32_t)((uint32_t)i | (10u << 28));   /* x1 wall */
      lt = (int32_t)((uint32_t)i | (12u << 28));   /* y1 wall */
      ll = (int32_t)((uint32_t)i | (9u << 28));    /* x0 wall */
    } else {
      hx0 = -0.5 * Lx; hx1 = 0.5 * Lx; hy0 = -0.5 * Ly; hy1 = 0.5 * Ly;
      /* image code of shift (sx, sy): k = 3 (sx + 1) + (sy + 1), skipping 4 */
      lb = (int32_t)((uint32_t)i | (4u << 28));    /* shift (0, -1) */
      lr = (int32_t)((uint32_t)i | (7u << 28));    /* shift (1, 0) */
      lt = (int32_t)((uint32_t)i | (5u << 28));    /* shift (0, 1) */
      ll = (int32_t)((uint32_t)i | (2u << 28));    /* shift (-1, 0) */
    }
    P->nv = 4;
    P->x[0] = hx0; P->y[0] = hy0; P->lab[0] = lb;
    P->x[1] = hx1; P->y[1] = hy0; P->lab[1] = lr;
    P->x[2] = hx1; P->y[2] = hy1; P->lab[2] = lt;
    P->x[3] = hx0; P->y[3] = hy1; P->lab[3] = ll;
    for (int64_t j = 0; j < n && st == OR_OK; ++j) {
      for (int sxs = -1; sxs <= 1; ++sxs)
        for (int sys = -1; sys <= 1; ++sys) {
          if (bc == 0 && (sxs != 0 || sys != 0)) continue;
          if (j == i && sxs == 0 && sys == 0) continue;
          /* image of point j, relative to point i */
          double dx = px[j] + sxs * Lx - xi, dy = py[j] + sys * Ly - yi;
          int k = 3 * (sxs + 1) + (sys + 1);
          uint32_t code = bc == 0 ? 0u : (uint32_t)(k < 4 ? k + 1 : (k == 4 ? 0 : k));
          int32_t lab = (int32_t)((uint32_t)j | (code << 28));
          /* nearer to i than to the image: x . d <= |d|^2 / 2 */
          if (or_clip(P, dx, dy, 0.5 * (dx * dx + dy * dy), lab) != 0) st = OR_E_INVAL;
        }
    }
    if (st != OR_OK) break;
    if (P->nv < 3 || P->nv > OR_VMAX) { st = OR_E_INVAL; break; }
    /* area and centroid by the shoelace sums over the triangles fanned
       from the point */
    double A2 = 0.0, cx = 0.0, cy = 0.0;
    for (int k = 0; k < P->nv; ++k) {
      int k1 = (k + 1) % P->nv;
      double cr = P->x[k] * P->y[k1] - P->y[k] * P->x[k1];
      A2 += cr;
      cx += (P->x[k] + P->x[k1]) * cr;
      cy += (P->y[k] + P->y[k1]) * cr;
    }
    area[i] = 0.5 * A2;
    sx[i] = xi + cx / (3.0 * A2);
    sy[i] = yi + cy / (3.0 * A2);
    nv[i] = P->nv;
    for (int k = 0; k < P->nv; ++k) {
      fan[i * OR_VMAX + k] = P->lab[k];
      vx[i * OR_VMAX + k] = xi + P->x[k];
      vy[i * OR_VMAX + k] = yi + P->y[k];
    }
  }
  /* edges, without the degenerate ones */
  for (int64_t i = 0; i < n && st == OR_OK; ++i) {
    const double Ri = sqrt(area[i] / OR_PI);
    int32_t d = 0;
    for (int k = 0; k < nv[i]; ++k) {
      int k1 = (k + 1) % nv[i];
      double ax = vx[i * OR_VMAX + k], ay = vy[i * OR_VMAX + k];
      double bx = vx[i * OR_VMAX + k1], by = vy[i * OR_VMAX + k1];
      double L = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
      int32_t lab = fan[i * OR_VMAX + k];
      int64_t j = (int64_t)((uint32_t)lab & 0x0FFFFFFFu);
      double Rj = sqrt(area[j] / OR_PI);
      if (!(L >= 1e-12 * 0.5 * (Ri + Rj))) continue;
      if (d >= max_fan) { st = OR_E_INVAL; break; }
      nb[i * max_fan + d] = lab;
      len[i * max_fan + d] = L;
      fx[i * max_fan + d] = 0.5 * (ax + bx);
      fy[i * max_fan + d] = 0.5 * (ay + by);
      ++d;
    }
    deg[i] = d;
  }
  free(P); free(fan); free(vx); free(vy); free(nv);
  return st;
}
