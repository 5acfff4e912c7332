/*
 * rich_tess.h -- host input stage: Voronoi tessellation of the mesh-generating
 * points, produced as flat arrays that both the device path and the oracle
 * consume.
 *
 * Method (paper section 2.1, "Tessellation Creation"): the Delaunay
 * triangulation is built by inserting the points one after another and
 * restoring the empty-circumcircle property after each insertion; the
 * orientation and in-circle signs are decided exactly (floating-point filter
 * with an error bound, exact expansion arithmetic when the filter cannot
 * decide); the Voronoi diagram is then read off the triangulation in linear
 * time (circumcentres become Voronoi vertices, each Delaunay edge becomes a
 * Voronoi edge).
 *
 * Boundaries are handled with ghost points: mirror images of points across
 * each reflecting wall, or periodic images, inside a band around the box.
 * The band is widened until every triangle incident to a real point has its
 * circumcircle inside the band, so the cells of the real points are exactly
 * those of the infinite mirrored / periodic point set.
 *
 * This library is host-only C++ (no HIP).  All functions are thread-compatible
 * (no global state) and never throw across the ABI.
 */
#ifndef RICH_TESS_H
#define RICH_TESS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary kinds (rich_mesh_host.bc). */
#define RICH_BC_WALLS    0u  /* four reflecting walls                 */
#define RICH_BC_PERIODIC 1u  /* doubly periodic box                   */

/* Ghost codes stored in the top 4 bits of e_j (see rich_mesh_host).        */
/*   0           : interior edge, neighbour is cell (e_j & RICH_CELL_MASK)  */
/*   1..8        : periodic edge; neighbour is that cell's image shifted by */
/*                 (sx*Lx, sy*Ly) relative to e_i's frame, with             */
/*                 code-1 = (sx+1)*3 + (sy+1) skipping the (0,0) entry,     */
/*                 i.e. codes enumerate (sx,sy) in the order                */
/*                 (-1,-1) (-1,0) (-1,1) (0,-1) (0,1) (1,-1) (1,0) (1,1)    */
/*   9,10,11,12  : reflecting wall x=x0, x=x1, y=y0, y=y1; the neighbour is */
/*                 the mirror image of e_i itself                            */
#define RICH_CELL_MASK   0x0FFFFFFF
#define RICH_CODE_SHIFT  28
#define RICH_CODE_WALL_X0 9
#define RICH_CODE_WALL_X1 10
#define RICH_CODE_WALL_Y0 11
#define RICH_CODE_WALL_Y1 12

/* Status codes (shared numbering with rich.h). */
#define RICH_TESS_OK        0
#define RICH_TESS_E_INVAL  -1  /* null pointer, n < 1, bad box, point outside box */
#define RICH_TESS_E_NOMEM  -2
#define RICH_TESS_E_MESH   -5  /* duplicate points or tessellation failure       */

/*
 * Mesh arrays.  Cells keep the caller's point order (cell i is point i).
 *   px,py   [n_cells]  mesh-generating points (periodic: wrapped into box)
 *   sx,sy   [n_cells]  cell centroids, in the frame of the point (periodic
 *                      centroids may lie slightly outside the box)
 *   area    [n_cells]  cell areas
 *   e_i,e_j [n_edges]  edge sides; e_i is a real cell, e_j packs the
 *                      neighbour cell (low 28 bits) and the ghost code
 *                      (top 4 bits).  Interior and periodic edges satisfy
 *                      e_i <= (e_j & mask); edges are sorted by e_i.
 *   e_len   [n_edges]  Voronoi edge length L_ij
 *   e_fx,e_fy          Voronoi edge midpoint, in e_i's frame
 *   off   [n_cells+1]  CSR offsets into idx
 *   idx   [n_csr]      2*edge + side; side 0: the cell is e_i, side 1: the
 *                      cell is e_j.  Each cell's entries follow its Voronoi
 *                      polygon counter-clockwise.  Wall edges appear once.
 *   eoff  [n_cells+1]  eoff[c] = first edge with e_i >= c
 * Edges shorter than 1e-12 * (R_i + R_j)/2 (R = sqrt(area/pi)), which come
 * from co-circular point sets, are dropped, and so is every edge between a
 * cell and the mirror image of another cell (two points and their mirrors
 * across one wall are co-circular, so such an edge has zero length exactly).
 */
typedef struct rich_mesh_host {
  int64_t n_cells, n_edges, n_csr;
  double *px, *py, *sx, *sy, *area;
  int32_t *e_i, *e_j;
  double *e_len, *e_fx, *e_fy;
  int32_t *off, *idx, *eoff;
  double box[4];      /* x0, y0, x1, y1 */
  uint32_t bc;
  /* diagnostics */
  int64_t n_ghosts;   /* ghost points inserted                  */
  int64_t n_dropped;  /* zero-length edges dropped              */
  double band;        /* ghost band width finally used          */
  int32_t n_rebuilds; /* band widenings                         */
  int64_t n_exact;    /* predicate calls decided exactly        */
  double t_triangulate; /* seconds: ghosts + Delaunay + checks  */
  double t_voronoi;     /* seconds: cells, edges, CSR           */
} rich_mesh_host;

/*
 * Build the mesh of points (px[i], py[i]), i < n, inside box = {x0,y0,x1,y1}.
 * Walls: every point must lie strictly inside the box.  Periodic: points are
 * wrapped into [x0,x1) x [y0,y1) first.  n_threads <= 0 picks the hardware
 * concurrency.  On success *out owns malloc'd arrays; release them with
 * rich_tess_free.  On failure *out is zeroed and a negative status returned.
 */
int rich_tess_build(const double* px, const double* py, int64_t n,
                    const double box[4], uint32_t bc, int32_t n_threads,
                    rich_mesh_host* out);

/* Release the arrays of a mesh built by rich_tess_build (safe on zeroed). */
void rich_tess_free(rich_mesh_host* m);

/*
 * Triangulation (for verification): the Delaunay triangles of real and ghost
 * points that touch at least one real point.  Points 0..n-1 are the real
 * points (wrapped), n..n_pts-1 ghosts.  Arrays are malloc'd; free with
 * rich_tess_free_tri.
 */
typedef struct rich_tri_host {
  int64_t n_pts, n_tri;
  double *x, *y;        /* [n_pts]    */
  int32_t *ghost_src;   /* [n_pts]    real point a ghost copies (-1 for real) */
  int32_t *tri;         /* [3*n_tri]  counter-clockwise vertex ids */
} rich_tri_host;
int rich_tess_triangles(const double* px, const double* py, int64_t n,
                        const double box[4], uint32_t bc, rich_tri_host* out);
void rich_tess_free_tri(rich_tri_host* t);

/* Exact predicates, exported for tests: sign of orient2d(a,b,c) (>0 when
 * counter-clockwise) and of incircle(a,b,c,d) (>0 when d lies inside the
 * circle through the counter-clockwise triangle a,b,c). */
int rich_tess_orient2d(const double a[2], const double b[2], const double c[2]);
int rich_tess_incircle(const double a[2], const double b[2], const double c[2],
                       const double d[2]);

/* Permutation sorting points along a Hilbert curve over the box (2^16 cells
 * per axis); perm_out[k] is the index of the k-th point. */
int rich_tess_hilbert_order(const double* px, const double* py, int64_t n,
                            const double box[4], int64_t* perm_out);

/* Lloyd relaxation: `iters` times, move every point to its cell centroid
 * (periodic: wrapped back into the box).  Points are updated in place. */
int rich_tess_lloyd(double* px, double* py, int64_t n, const double box[4],
                    uint32_t bc, int32_t iters, int32_t n_threads);

/*
 * Adapter for the time-centred step of the device path: rich_tess_callback
 * and rich_tess_release have the signatures of rich_tess_fn and
 * rich_tess_release_fn in rich.h, and rich_tess_view has the field layout of
 * rich_host_mesh_view there.  `user` must be a rich_tess_ctx; each mesh the
 * callback hands out stays valid until released.
 */
typedef struct rich_tess_view {
  int64_t n_cells, n_edges, n_csr;
  const double *px, *py, *sx, *sy, *area;
  const int32_t *e_i, *e_j;
  const double *e_len, *e_fx, *e_fy;
  const int32_t *off, *idx, *eoff;
} rich_tess_view;
typedef struct rich_tess_ctx rich_tess_ctx;
rich_tess_ctx* rich_tess_ctx_create(int32_t n_threads);
void rich_tess_ctx_destroy(rich_tess_ctx* ctx);
int rich_tess_callback(void* user, const double* px, const double* py, int64_t n,
                       const double box[4], uint32_t bc, rich_tess_view* out);
void rich_tess_release(void* user, rich_tess_view* v);

#ifdef __cplusplus
}
#endif
#endif /* RICH_TESS_H */
