/*
 * oracle.h -- plain, serial, FP64 reference of one stage of the moving-mesh
 * Godunov scheme of RICH (Yalinewich, Steinberg & Sari).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code, header,
 * table or helper with the device path; both read the same mesh arrays
 * produced by the host tessellation stage.
 *
 * Conventions (layout of the arrays the host stage produces):
 *   cells    px,py points; sx,sy centroids; area
 *   edges    e_i (real cell), e_j (neighbour cell in the low 28 bits, ghost
 *            code in the top 4: 0 interior, 1..8 periodic image shift,
 *            9..12 reflecting wall x0,x1,y0,y1), e_len, e_fx/e_fy (midpoint,
 *            in e_i's frame)
 *   CSR      off[n+1], idx = 2*edge + side (side 1: the cell is e_j)
 * State arrays are planar: Q[4*n] = M | Px | Py | E (extensive totals over the
 * cell), X[2*n] = x | y.
 *
 * Parity unpinned.  Where the paper leaves a choice open, the oracle takes
 * one reading and the device path takes the same; no fact of the paper or of
 * the mathematics distinguishes it from the alternatives, so only the shared
 * reading pins these (every other function is pinned by a test that does
 * not re-run the oracle's own formula):
 *   - which variables are reconstructed: the primitives rho, p, vx, vy,
 *     limited one by one (section 2.2 names them, not the alternatives);
 *   - the reconstruction starts at the centroid s_i with the cell's value,
 *     although the gradient belongs to the point r_i (section 2.2);
 *   - the shock detector beyond its special cases (section 2.2: the
 *     compression test per cell with the unlimited gradient, strict
 *     inequalities, the pressure-ratio test over all neighbours);
 *   - the HLLC wave-speed estimates (Davis bounds; section 2.4 does not
 *     state them);
 *   - the on/off shape of the cell-rounding correction (section 6 gives its
 *     parameters, not its form near d = eta R).
 * The wall ghost (mirrored point, state, extrapolated edge state and edge
 * velocity) is pinned by the method of images: a walled run equals the
 * periodic run of the points and their mirror images.
 */
#ifndef RICH_ORACLE_H
#define RICH_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct or_mesh {
  int64_t n_cells, n_edges;
  const double *px, *py, *sx, *sy, *area;
  const int32_t *e_i, *e_j;
  const double *e_len, *e_fx, *e_fy;
  const int32_t *off, *idx;
  double box[4];
  uint32_t bc;
} or_mesh;

typedef struct or_params {
  double gamma;    /* adiabatic index                                    */
  double cfl;      /* Courant number (paper default 0.3)                 */
  double theta;    /* local-limiter factor (0.5)                         */
  double delta_v;  /* shock-detector compression threshold (0.2)        */
  double delta_p;  /* shock-detector pressure-ratio threshold (0.7)     */
  double chi;      /* cell-rounding speed in units of c_s (0.15)        */
  double eta;      /* cell-rounding offset threshold in units of R (0.02) */
  int32_t riemann; /* 0 HLLC, 1 exact                                   */
  int32_t motion;  /* 0 static (Eulerian), 1 Lagrangian + cell rounding */
  int32_t limiter; /* 0 switching (paper default), 1 global only, 2 local
                      only, 3 unlimited, 4 first order                  */
  double gx, gy;   /* uniform external acceleration (0 for pure hydro)  */
  int32_t integrator; /* 0 time-centred fluxes (the paper's), 1 extrapolated
                         fluxes (AREPO's, section 2.3)                     */
} or_params;

/* status codes */
#define OR_OK 0
#define OR_E_INVAL -1
#define OR_E_DOMAIN -4

/* A1: primitives of extensive Q on the mesh: prim[5n] = rho|vx|vy|p|c */
int or_primitives(const or_mesh* m, const double* Q, const or_params* p, double* prim);

/* A2: mesh-point velocities w[2n] from primitives (paper section 6). */
int or_point_velocity(const or_mesh* m, const double* prim, const or_params* p,
                      double* w);

/* A3: unlimited Green-Gauss gradients (eq. slope) of rho, vx, vy, p:
 * grad[8n] = drho/dx | drho/dy | dvx/dx | dvx/dy | dvy/dx | dvy/dy | dp/dx | dp/dy */
int or_gradients(const or_mesh* m, const double* prim, double* grad);

/* A4: limiter factors alpha[4n] and per-cell shock flags (bit 0) */
int or_limiter(const or_mesh* m, const double* prim, const double* grad,
               const or_params* p, double* alpha, int32_t* flag);

/* A5-A7: lab-frame flux per unit length through every edge, flux[4E] planar
 * (mass | x-momentum | y-momentum | energy), oriented from e_i to e_j.
 * lgrad is the limited gradient (alpha * grad), w the point velocities. */
int or_edge_fluxes(const or_mesh* m, const double* prim, const double* lgrad,
                   const double* w, const or_params* p, double* flux);

/* Branch quantities of the Riemann solver on every edge (section 2.4), for
 * comparing branch records, waves[4E] planar: HLLC S_L | S* | S_R | scale;
 * exact solver NaN | u* | NaN | scale; scale = |u_L| + c_L + |u_R| + c_R. */
int or_edge_waves(const or_mesh* m, const double* prim, const double* lgrad,
                  const double* w, const or_params* p, double* waves);

/* Area change rate of every cell implied by the edge velocities (eq. areachange) */
int or_area_rate(const or_mesh* m, const double* w, double* adot);

/* Threads the per-cell and per-edge loops run on (1 in the serial build;
 * the OpenMP team size in the parallel build used to time the oracle on all
 * host cores; both builds give the same bits). */
int or_threads(void);

/* One stage: Qout = Qbase - h * sum_edges(L F), Xout = Xbase + h w.
 * Optional diagnostics (may be NULL): prim[5n], w[2n], alpha[4n], flag[n],
 * flux[4E]. Returns OR_E_DOMAIN if a produced cell has M<=0, internal energy
 * <= 0 or a non-finite value (outputs are still written). */
int or_stage(const or_mesh* m, const double* Qsrc, const double* Qbase,
             const double* Xbase, double h, const or_params* p, double* Qout,
             double* Xout, double* d_prim, double* d_w, double* d_alpha,
             int32_t* d_flag, double* d_flux);

/* or_stage with a per-cell external acceleration: cell i is accelerated by
 * (p->gx + ax[i], p->gy + ay[i]) (section 2.3's source term, from the
 * stage's source totals). */
int or_stage_accel(const or_mesh* m, const double* Qsrc, const double* Qbase,
                   const double* Xbase, double h, const or_params* p, const double* ax,
                   const double* ay, double* Qout, double* Xout);

/* Courant time step of the state Q on mesh m (A0). */
int or_cfl_dt(const or_mesh* m, const double* Q, const or_params* p, double* dt);

/* Voronoi mesh of the points by its definition (section 2.1): cell i is the
 * set of points of the box nearer to (px_i, py_i) than to any other point
 * (walls: the box bounds the cell, which is what the mirror images of the
 * point across the walls give; periodic box: every periodic image of every
 * point counts).  O(n^2) half-plane clipping, for small n.
 * Outputs: area[n], centroid sx[n], sy[n], deg[n] and, for cell i, slots
 * i*max_fan .. i*max_fan+deg[i]-1, counter-clockwise: nb (neighbour cell |
 * code << 28: 0 interior, 1..8 periodic image, 9..12 wall x0 x1 y0 y1), len,
 * fx, fy (edge midpoint).  Edges shorter than 1e-12 (R_i + R_j) / 2 with
 * R = sqrt(area / pi) are left out.  Returns OR_E_INVAL for bad arguments or
 * a cell with more than max_fan edges. */
int or_voronoi(int64_t n, const double* px, const double* py, const double* box,
               uint32_t bc, int32_t max_fan, double* area, double* sx, double* sy,
               int32_t* deg, int32_t* nb, double* len, double* fx, double* fy);

/* One-dimensional Riemann problem in the frame of an edge.  States are
 * (rho, u, vt, p): density, normal velocity, tangential velocity, pressure.
 * Flux out: (mass, normal momentum, tangential momentum, energy). */
void or_hllc(double gamma, const double* WL, const double* WR, double* F);
/* Exact solver: flux at x/t = 0; star[2] = (p*, u*) if non-NULL; returns the
 * Newton iteration count, or -1 when the states would create a vacuum. */
int or_exact(double gamma, const double* WL, const double* WR, double* F, double* star);
/* Sample the exact solution at x/t = xi: W = (rho, u, vt, p). */
int or_exact_sample(double gamma, const double* WL, const double* WR, double xi,
                    double* W);

#ifdef __cplusplus
}
#endif
#endif
