/*
 * rich.h -- C-ABI of the device path (librich.so): one stage and one
 * time-centred step of the moving-mesh Godunov scheme of RICH (Yalinewich,
 * Steinberg & Sari) on an MI355X (gfx950), for one run or a batch of
 * independent runs; the Courant step, the area change rate of the cells, and
 * the rebuild of the Voronoi mesh of moved points on the device.
 *
 * Every step of the stage runs in HIP kernels; this header carries no HIP or
 * torch types: device pointers are plain pointers and the stream is passed as
 * an opaque `void*` (a hipStream_t; NULL is the null stream).  The caller owns
 * all memory it passes in; the library never frees or keeps it.
 *
 * Data layout (device memory, FP64 values, int32 indices): the mesh is the
 * host tessellation stage's (rich_tess.h) with its cells and edges as
 * records (rich_cell, rich_edge below; rich_mesh_pack builds them) and its
 * CSR arrays as they are, or the same layout written by rich_retess; the state of a run is the extensive cell totals M,
 * Px, Py, E (mass, momentum, total energy integrated over each cell) and the
 * mesh-generating points x, y, each a row of n_cells doubles.
 *
 * Status codes: every function returns RICH_OK (0) or a negative code; no
 * C++ exception crosses the ABI.  rich_stage and rich_stage_batch only
 * enqueue work on the stream; their domain checks are read back with
 * rich_stage_flags / rich_batch_flags(_async).
 *
 * Threads: calls from several host threads may run concurrently as long as
 * each uses its own workspace, rich_ctx and stream; the kernel timing
 * switch (rich_profile_*) is process-wide and not thread-safe.
 */
#ifndef RICH_H
#define RICH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RICH_OK         0
#define RICH_E_INVAL   -1  /* null pointer, size mismatch, h/dt <= 0 or not finite */
#define RICH_E_NOMEM   -2  /* workspace too small, allocation failed          */
#define RICH_E_DEVICE  -3  /* HIP runtime error                               */
#define RICH_E_DOMAIN  -4  /* a cell got M <= 0, internal energy <= 0, a non-finite
                              value, or the exact solver met a vacuum          */
#define RICH_E_MESH    -5  /* invalid mesh or tessellation failure             */

/* Per-run flag bits reported by rich_stage_flags. */
#define RICH_FLAG_DOMAIN 1  /* a produced cell failed the physical checks, or
                               the mesh gave a cell a non-positive area or an
                               entry out of range */
#define RICH_FLAG_VACUUM 2  /* exact Riemann solver: states create a vacuum */

/* Boundary kinds (same values as rich_tess.h). */
#define RICH_BOUNDARY_WALLS    0u
#define RICH_BOUNDARY_PERIODIC 1u

/*
 * Device layout of a mesh: one record per cell and one per edge, so that a
 * gather of a neighbour's geometry or of an edge takes two 16-byte loads.
 * The values are those of the host stage's arrays (rich_tess.h), rearranged
 * bit for bit by rich_mesh_pack.
 *   rich_cell  px, py  mesh-generating point
 *              area    cell area
 *              sx, sy  centroid (in the frame of the point)
 *   rich_edge  fx, fy  Voronoi edge midpoint (in the frame of cell i)
 *              len     edge length
 *              i       first cell (edges sorted by i)
 *              j       neighbour cell (low 28 bits) and ghost code (top 4
 *                      bits), as e_j of the host stage
 * Both arrays must be 16-byte aligned.
 */
typedef struct rich_cell {
  double px, py, area, sx, sy, pad;
} rich_cell;
typedef struct rich_edge {
  double fx, fy, len;
  int32_t i, j;
} rich_edge;

/* Mesh of one run (device pointers, borrowed).  off[n_cells+1], idx[n_csr]
 * (2*edge + side, each cell's entries counter-clockwise) and eoff[n_cells+1]
 * (first edge of each cell) as in the host stage. */
typedef struct rich_mesh {
  int64_t n_cells, n_edges, n_csr;
  const rich_cell* cells;
  const rich_edge* edges;
  const int32_t *off, *idx, *eoff;
  double box[4];  /* x0, y0, x1, y1 */
  uint32_t bc;    /* RICH_BOUNDARY_* */
} rich_mesh;

/* State of one run (device pointers, borrowed). */
typedef struct rich_state {
  double *M, *Px, *Py, *E;  /* extensive totals per cell */
  double *x, *y;            /* mesh-generating points    */
  int64_t n_cells;
} rich_state;

/* Scheme parameters.  Paper defaults: theta 0.5, delta_v 0.2, delta_p 0.7
 * (section 2.2), Courant number 0.3 (section 2.3), chi 0.15, eta 0.02
 * (section 6). */
typedef struct rich_params {
  double gamma;    /* adiabatic index of the ideal gas                     */
  double cfl;      /* Courant number                                       */
  double theta;    /* local (TESS) limiter factor                          */
  double delta_v;  /* shock detector: compression threshold                */
  double delta_p;  /* shock detector: pressure-ratio threshold             */
  double chi;      /* cell rounding: correction speed in units of c_s      */
  double eta;      /* cell rounding: offset threshold in units of the cell radius */
  int32_t riemann; /* 0 HLLC (section 2.4), 1 exact                        */
  int32_t motion;  /* 0 static mesh, 1 Lagrangian with cell rounding (section 6) */
  int32_t limiter; /* 0 global/local switch on the shock detector (section 2.2),
                      1 global only, 2 local only, 3 unlimited, 4 first order */
  double gx, gy;   /* uniform external acceleration; each stage adds h times
                      (0, M g, P.g) of its source totals (section 2.3: the
                      time-centred scheme makes a first-order source second
                      order); 0 for pure hydrodynamics */
  int32_t integrator; /* 0 time-centred fluxes (the paper's scheme: two
                      stages per step); 1 extrapolated fluxes (AREPO's,
                      section 2.3: one stage per step, whose face states are
                      advanced half a step with the time derivatives the
                      limited gradients give in the primitive Euler
                      equations, following each cell's point; the source
                      term is then first order in time) */
} rich_params;

/* Fill p with the paper's defaults for adiabatic index gamma. */
void rich_params_default(rich_params* p, double gamma);

/* Workspace bytes one stage of a run with n_cells cells needs (scratch for
 * the per-cell reconstruction records, the Courant minimum and the flag word).
 * The workspace is caller-allocated device memory, 256-byte aligned. */
int rich_workspace_size(int64_t n_cells, size_t* bytes);

/*
 * One stage (section 2.3): on mesh m, with primitives taken from src,
 *   out.{M,Px,Py,E}_i = base.{M,Px,Py,E}_i - h * sum over the cell's edges of
 *                       (+/-) L_e F_e
 *   out.{x,y}_i       = base.{x,y}_i + h * w_i   (wrapped into a periodic box)
 * where F_e is the flux through the moving edge (sections 2.2-2.4, 5, 6).
 * src and base are never written; out may alias neither.  Enqueued on
 * `stream`; returns RICH_E_INVAL for bad arguments without enqueuing.
 * The domain checks of the produced state are reported by rich_stage_flags.
 */
int rich_stage(const rich_mesh* m, const rich_state* src, const rich_state* base,
               rich_state* out, double h, const rich_params* p, void* ws,
               size_t ws_bytes, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rich_stage
 * without a caller workspace.  The stage's scratch (the per-cell
 * reconstruction records, the Courant minimum and the flag word) is a
 * library-owned device array of fixed size, one per GPU, held from the
 * library's first use on that GPU until the process ends; its address is
 * looked up on the first call on each device.  Nothing is allocated and no
 * memset is enqueued (the flag word is cleared by the stage's own kernel).
 * Arguments, results and errors are those of rich_stage, and the results
 * equal rich_stage's bit for bit, with these differences:
 *   - meshes of more than RICH_NOALLOC_MAX_CELLS cells return RICH_E_NOMEM
 *     without enqueuing;
 *   - flag_out (caller-owned device int32, may be null) receives the stage's
 *     RICH_FLAG_* word when the stage completes (in place of
 *     rich_stage_flags, which needs a workspace);
 *   - every call on one GPU shares that GPU's scratch, which keeps the last
 *     call's contents: calls that overlap on one GPU (concurrent streams or
 *     host threads) race and must be serialised by the caller;
 *   - RICH_E_DEVICE if the scratch's address cannot be looked up.
 */
#define RICH_NOALLOC_MAX_CELLS 1048576
int rich_stage_noalloc(const rich_mesh* m, const rich_state* src, const rich_state* base,
                       rich_state* out, double h, const rich_params* p, int32_t* flag_out,
                       void* stream);

/*
 * rich_stage with a per-cell external acceleration (section 2.3's source
 * term): cell i is accelerated by (p->gx + ax[i], p->gy + ay[i]), and the
 * stage adds h (0, M g_i, P.g_i) of its source totals, as for the uniform
 * one.  ax, ay: device arrays of n_cells doubles, caller-owned, read only;
 * RICH_E_INVAL when null.  Otherwise as rich_stage.
 */
int rich_stage_accel(const rich_mesh* m, const rich_state* src, const rich_state* base,
                     rich_state* out, double h, const rich_params* p, const double* ax,
                     const double* ay, void* ws, size_t ws_bytes, void* stream);

/*
 * rich_stage with a record of the decisions the scheme takes (for comparing
 * branches with an independent implementation; its outputs equal rich_stage's
 * bit for bit).  Device arrays, caller-owned:
 *   cell_bits[n_cells]  bit 0  shock flag of the switching limiter (section
 *                              2.2: compression or pressure jump)
 *                       bit 1  cell-rounding correction applied (section 6:
 *                              centroid offset above eta R)
 *                       bits 2-5  alpha < 1 for rho, vx, vy, p (section 2.2)
 *   edge_bits[n_edges]  HLLC (section 2.4): bit 0 = (0 <= S_L),
 *                       bit 1 = (0 <= S*), bit 2 = (0 < S_R); exact solver:
 *                       bit 1 = (0 <= u*), the side of the contact sampled;
 *                       bit 3 = no flux could be formed (vacuum, bad index)
 * The edge record is taken by a separate launch after the cell pass; the
 * arithmetic is the stage's own.  RICH_E_INVAL for null record pointers.
 */
int rich_stage_debug(const rich_mesh* m, const rich_state* src, const rich_state* base,
                     rich_state* out, double h, const rich_params* p, void* ws,
                     size_t ws_bytes, uint8_t* cell_bits, uint8_t* edge_bits, void* stream);

/* Synchronise `stream` and return the flag word of the last stage that used
 * workspace ws (RICH_FLAG_* bits; 0 when all produced cells are valid). */
int rich_stage_flags(void* ws, void* stream, int32_t* flags);

/*
 * Courant time step (section 2.3): dt = cfl * min_i R_i / (c_i + |v_i - w_i|),
 * R_i = sqrt(A_i / pi).  Synchronises `stream` and writes the host double *dt.
 */
int rich_cfl_dt(const rich_mesh* m, const rich_state* s, const rich_params* p,
                double* dt, void* ws, size_t ws_bytes, void* stream);

/*
 * Area change rate of every cell that the moving edges imply (section 5, eq.
 * areachange): adot[i] = dA_i/dt with the point velocities w of state s on
 * mesh m (section 6).  The actual change of a cell's area over a step differs
 * from h * adot at second order: that difference is the paper's area
 * inconsistency.  adot is a device array of m->n_cells doubles.  Enqueued on
 * `stream`; a bad CSR entry sets RICH_FLAG_DOMAIN (rich_stage_flags).
 */
int rich_area_rate(const rich_mesh* m, const rich_state* s, const rich_params* p,
                   double* adot, void* ws, size_t ws_bytes, void* stream);

/*
 * Courant step fused into a stage, with no host round trip (sections 2.3 and
 * 2.2): the cell pass of this stage also takes the Courant minimum of src
 * (the same quantity rich_cfl_dt reduces), a one-block reduction writes
 * dt = cfl * minimum into workspace ws, and the stage is then rich_stage with
 * h = h_factor * dt read from device memory.  A time-centred step is
 *   rich_stage_courant(m, s, s, half, 0.5, p, ws, ...)
 *   (tessellate the half-step points)
 *   rich_stage_dt_of(m', half, s, out, 1.0, ws, p, ws, ...)
 * with results bitwise equal to rich_cfl_dt followed by rich_stage with
 * h = dt / 2 and h = dt.  Enqueued on `stream`; nothing synchronises.
 * Arguments are those of rich_stage; h_factor must be finite and >= 0, and
 * p->cfl positive.  Returns RICH_E_INVAL, without enqueuing, for integrator 1
 * (its cell pass needs the step before the minimum exists).  A dt that is
 * not positive and finite sets RICH_FLAG_DOMAIN in this stage's flag word.
 */
int rich_stage_courant(const rich_mesh* m, const rich_state* src, const rich_state* base,
                       rich_state* out, double h_factor, const rich_params* p, void* ws,
                       size_t ws_bytes, void* stream);

/*
 * rich_stage with h = h_factor * dt, where dt is the value the last
 * rich_stage_courant on workspace dt_ws wrote (read on the device when the
 * kernels run, so the call may be enqueued before that value exists).
 * dt_ws may be ws itself: a stage leaves the dt slot of its workspace alone.
 */
int rich_stage_dt_of(const rich_mesh* m, const rich_state* src, const rich_state* base,
                     rich_state* out, double h_factor, const void* dt_ws,
                     const rich_params* p, void* ws, size_t ws_bytes, void* stream);

/* Synchronise `stream` and copy the dt the last rich_stage_courant on ws
 * wrote to the host double *dt; RICH_E_DOMAIN if it is not positive and
 * finite. */
int rich_stage_dt(void* ws, void* stream, double* dt);

/*
 * Batched stage over n independent runs of any sizes, in one launch per
 * kernel phase: meshes[r], src[r], base[r], out[r], h[r], params[r] as for
 * rich_stage (host arrays of pointers to host structs holding device
 * pointers).  ws is one device workspace of rich_batch_workspace_size bytes.
 * The per-run results are bitwise identical to n separate rich_stage calls.
 */
int rich_batch_workspace_size(int32_t n, const int64_t* n_cells, size_t* bytes);
int rich_stage_batch(int32_t n, const rich_mesh* const* meshes,
                     const rich_state* const* src, const rich_state* const* base,
                     rich_state* const* out, const double* h,
                     const rich_params* const* params, void* ws, size_t ws_bytes,
                     void* stream);
/* rich_stage_batch with a per-cell external acceleration (section 2.3 source
 * term, as rich_stage_accel): ax[r], ay[r] are device arrays of
 * meshes[r]->n_cells doubles added to params[r]'s uniform (gx, gy), or both
 * NULL for a run without a field (a run with one of the two NULL is
 * RICH_E_INVAL, as are NULL ax or ay themselves).  Host arrays of n device
 * pointers, caller-owned.  The per-run results are bitwise identical to n
 * separate rich_stage_accel (or, for runs without a field, rich_stage) calls. */
int rich_stage_batch_accel(int32_t n, const rich_mesh* const* meshes,
                           const rich_state* const* src, const rich_state* const* base,
                           rich_state* const* out, const double* h,
                           const rich_params* const* params, const double* const* ax,
                           const double* const* ay, void* ws, size_t ws_bytes, void* stream);
/*
 * The same batched stage in two calls, so that its launches can be replayed
 * (for example captured once in a HIP graph and launched many times):
 *   rich_stage_batch_prepare  validates the runs exactly as rich_stage_batch,
 *                             enqueues on `stream` the upload of the run
 *                             descriptors and launch plans into ws, and fills
 *                             *plan (host struct, no pointers) with the launch
 *                             sizes; ws then holds everything the launch reads;
 *   rich_stage_batch_launch   enqueues the kernels of the stage (no copies, no
 *                             memsets, no allocation, no host synchronisation).
 * A launch reads the device and host memory named when the plan was made, so
 * every replay runs the stage again on whatever those buffers then hold.
 * A plan is valid on its workspace until the next prepare on that
 * workspace, which overwrites the descriptors: rich_stage_batch_launch
 * returns RICH_E_INVAL for any plan but the last one prepared on ws (a graph
 * that captured a launch replays whatever the workspace then holds, so
 * prepare nothing else on it while the graph is in use).
 * rich_stage_batch is prepare followed by launch.  Kernel timing must be off
 * while a launch is captured.
 */
typedef struct rich_batch_plan {
  int32_t n_runs;
  int32_t n_cell_tiles;     /* tiles of the cell kernel over all runs          */
  int32_t n_flux_tiles[2];  /* flux tiles of the HLLC runs, of the exact runs  */
  int32_t n_group[2];       /* number of HLLC runs, of exact-solver runs        */
  int32_t grid_cell;        /* blocks of the cell kernel (one per tile)        */
  int32_t grid_flux[2];     /* blocks of the two flux kernels (one per tile)   */
  int32_t flux_tile;        /* cells per flux tile (edge-tile shape)           */
  int32_t courant;          /* 1: the stage computes each run's step          */
  int64_t serial;           /* identifies the prepare that made the plan       */
  int64_t table_offset;     /* bytes from ws to the tile -> run tables         */
} rich_batch_plan;
int rich_stage_batch_prepare(int32_t n, const rich_mesh* const* meshes,
                             const rich_state* const* src, const rich_state* const* base,
                             rich_state* const* out, const double* h,
                             const rich_params* const* params, void* ws, size_t ws_bytes,
                             void* stream, rich_batch_plan* plan);
int rich_stage_batch_launch(const rich_batch_plan* plan, void* ws, void* stream);
/* As rich_stage_batch_prepare, with flux tiles of `tile` cells (128, 256 or
 * 512; rich_stage_batch_prepare takes 256).  A tile is a group of
 * consecutive cells whose owned edges one workgroup solves; the results do
 * not depend on it, bit for bit (each edge's flux is computed with the same
 * arithmetic wherever it is computed, and each cell sums its edges in CSR
 * order). */
int rich_stage_batch_prepare_tile(int32_t n, const rich_mesh* const* meshes,
                                  const rich_state* const* src, const rich_state* const* base,
                                  rich_state* const* out, const double* h,
                                  const rich_params* const* params, int32_t tile, void* ws,
                                  size_t ws_bytes, void* stream, rich_batch_plan* plan);
/* A batched stage whose steps are taken on the device, per run, from the
 * Courant condition of section 2.3 (the batched form of rich_stage_courant /
 * rich_stage_dt_of), prepared as rich_stage_batch_prepare_tile and launched
 * with rich_stage_batch_launch; a step of every run then needs no host
 * round trip, and both of its stages can be captured in one graph.
 *   dt_ws == NULL  the stage computes run r's step
 *                  dt_r = params[r]->cfl * min over cells of R/(c + |v - w|)
 *                  from src[r] in its cell pass, keeps it in ws (slot r,
 *                  read with rich_batch_dt) and applies h_r = factor[r] * dt_r
 *                  (factor 0.5 for the first stage of a time-centred step).
 *                  Runs with params[r]->integrator == 1 are RICH_E_INVAL
 *                  (their cell pass reads the step).  A step that is not a
 *                  positive finite number sets the run's domain flag.
 *   dt_ws != NULL  h_r = factor[r] * dt_r, with dt_r slot r of the batch
 *                  workspace dt_ws of an earlier Courant stage over the same
 *                  runs in the same order (dt_ws may be ws itself: a stage
 *                  leaves the slots of the steps alone).
 * factor[r] finite and >= 0.  Each run's step and result are bitwise those
 * of rich_stage_courant / rich_stage_dt_of on that run alone. */
int rich_stage_batch_prepare_courant(int32_t n, const rich_mesh* const* meshes,
                                     const rich_state* const* src,
                                     const rich_state* const* base, rich_state* const* out,
                                     const double* factor, const rich_params* const* params,
                                     int32_t tile, const void* dt_ws, void* ws, size_t ws_bytes,
                                     void* stream, rich_batch_plan* plan);
/* Synchronise `stream` and copy the n per-run steps the last Courant stage on
 * the batch workspace ws computed into the host array dt. */
int rich_batch_dt(int32_t n, void* ws, void* stream, double* dt);
/* Autotune the edge-tile shape of a batched stage: prepares and times (HIP
 * events, `reps` launches after one warm-up) the stage with each tile of
 * 128, 256 and 512 cells on these runs, writing the mean milliseconds per
 * launch into ms[3] and the fastest tile into *best_tile.  Runs the stage
 * 3 * (reps + 1) times (out is written each time; src and base are only
 * read) and synchronises `stream`. */
int rich_stage_batch_autotune(int32_t n, const rich_mesh* const* meshes,
                              const rich_state* const* src, const rich_state* const* base,
                              rich_state* const* out, const double* h,
                              const rich_params* const* params, int32_t reps, void* ws,
                              size_t ws_bytes, void* stream, int32_t* best_tile, double* ms);

/* Synchronise and read the n per-run flag words of the last batched stage. */
int rich_batch_flags(int32_t n, void* ws, void* stream, int32_t* flags);
/* Enqueue on stream a copy of the same n flag words into host_flags and
 * return without waiting: the words are there once the stream has passed
 * the copy (an event recorded after it).  host_flags should be pinned host
 * memory (hipHostMalloc); other memory makes the copy synchronous. */
int rich_batch_flags_async(int32_t n, void* ws, void* stream, int32_t* host_flags);

/*
 * One step (section 2.3) of one run.  Time-centred fluxes (integrator 0),
 * with a moving mesh:
 *   1. stage(mesh_n, Q^n, Q^n, x^n, dt/2)        -> Q^{n+1/2}, x^{n+1/2}
 *   2. tessellate x^{n+1/2}                       -> mesh_{n+1/2}
 *   3. stage(mesh_{n+1/2}, Q^{n+1/2}, Q^n, x^n, dt) -> Q^{n+1}, x^{n+1}
 *   4. tessellate x^{n+1}                         -> mesh_{n+1}
 * The tessellation is the caller's host function `tess` (the host input
 * stage); it receives host point arrays and must fill *out with host mesh
 * arrays that stay valid until `release` is called on it.  The library
 * uploads them into its own device buffers (owned by ctx).  With a static
 * mesh (params->motion == 0) no tessellation happens.  Extrapolated fluxes
 * (integrator 1): stage(mesh_n, Q^n, Q^n, x^n, dt) -> Q^{n+1}, x^{n+1}, then
 * one tessellation.
 * The state is committed only on success; on RICH_E_DOMAIN it is unchanged.
 */
typedef struct rich_host_mesh_view {
  int64_t n_cells, n_edges, n_csr;
  const double *px, *py, *sx, *sy, *area;
  const int32_t *e_i, *e_j;
  const double *e_len, *e_fx, *e_fy;
  const int32_t *off, *idx, *eoff;
} rich_host_mesh_view;
/* Host helper: rearrange a host mesh's cell and edge arrays into the device
 * records (host memory: cells[n_cells], edges[n_edges], caller-owned). */
int rich_mesh_pack(const rich_host_mesh_view* hm, rich_cell* cells, rich_edge* edges);
typedef int (*rich_tess_fn)(void* user, const double* px, const double* py,
                            int64_t n, const double box[4], uint32_t bc,
                            rich_host_mesh_view* out);
typedef void (*rich_tess_release_fn)(void* user, rich_host_mesh_view* m);

typedef struct rich_ctx rich_ctx;  /* device buffers of one run's step driver */
int rich_ctx_create(rich_ctx** ctx);
void rich_ctx_destroy(rich_ctx* ctx);
/* Upload a host mesh as the run's current mesh. */
int rich_ctx_set_mesh(rich_ctx* ctx, const rich_host_mesh_view* hm,
                      const double box[4], uint32_t bc, void* stream);
/* Device view of the run's current mesh. */
int rich_ctx_mesh(rich_ctx* ctx, rich_mesh* out);
/* With on = 1, rich_step rebuilds each mesh on the device (rich_retess, with
 * the previous mesh as the candidate source) and calls the host stage `tess`
 * only for a mesh the device does not certify; on = 0 (the default) always
 * uses the host stage.  rich_ctx_tess_counts reports how many meshes were
 * built each way since the context was created. */
int rich_ctx_set_device_tess(rich_ctx* ctx, int32_t on);
int rich_ctx_tess_counts(rich_ctx* ctx, int64_t* device, int64_t* host_fallback);
int rich_step(rich_ctx* ctx, rich_state* state, double dt, const rich_params* p,
              rich_tess_fn tess, rich_tess_release_fn release, void* tess_user,
              void* stream);
/* rich_step with a per-cell external acceleration in every stage (as
 * rich_stage_accel): cell i, which keeps its index through the step, is
 * accelerated by (p->gx + ax[i], p->gy + ay[i]).  ax, ay: device arrays of
 * n_cells doubles, caller-owned; RICH_E_INVAL when null. */
int rich_step_accel(rich_ctx* ctx, rich_state* state, double dt, const rich_params* p,
                    const double* ax, const double* ay, rich_tess_fn tess,
                    rich_tess_release_fn release, void* tess_user, void* stream);

/*
 * One step (section 2.3) of n independent runs at once: the same chain as
 * rich_step for every run (each with its own integrator), with each stage
 * issued as one batched stage over the runs that take it (rich_stage_batch)
 * and the host tessellations of the runs spread over n_threads host threads
 * in between.
 *   ctxs[r]       run r's driver (current mesh set with rich_ctx_set_mesh);
 *                 its device buffers are grown as needed
 *   states[r]     host struct of device pointers: Q^n, x^n in, Q^{n+1},
 *                 x^{n+1} out (committed only when status[r] == RICH_OK)
 *   dt[r], params[r]
 *   tess, release as for rich_step; tess is called with tess_users[r] for
 *                 run r, from up to n_threads threads at once (calls for
 *                 different runs must be safe to run concurrently, which
 *                 holds for rich_tess_callback with one rich_tess_ctx per
 *                 run); both may be NULL when no run moves its mesh
 *   status[r]     out: RICH_OK, or this run's error (E_INVAL, E_NOMEM,
 *                 E_DOMAIN, E_MESH); a failing run leaves its state and
 *                 current mesh unchanged and never alters another run
 *   ws            one device workspace of rich_batch_workspace_size bytes
 *                 for the runs' cell counts
 * Returns RICH_OK when every run succeeded, else the status of the first
 * failing run.  When the call as a whole fails (workspace too small, a HIP
 * error), that status is returned and written to every run not yet failed:
 * status[r] == RICH_OK always means run r was committed.  Synchronises
 * stream.
 * The results are bitwise identical to n separate rich_step calls.
 */
int rich_step_batch(int32_t n, rich_ctx* const* ctxs, rich_state* const* states,
                    const double* dt, const rich_params* const* params,
                    rich_tess_fn tess, rich_tess_release_fn release,
                    void* const* tess_users, int32_t n_threads, int32_t* status,
                    void* ws, size_t ws_bytes, void* stream);
/* rich_step_batch with a per-cell external acceleration in every stage of
 * the runs that carry one (as rich_step_accel): ax[r], ay[r] are device
 * arrays of run r's n_cells doubles, or both NULL for a run without a field
 * (a run with only one of them NULL fails with status RICH_E_INVAL; NULL ax
 * or ay themselves fail the call with RICH_E_INVAL).  Host arrays of n device
 * pointers, caller-owned.  The results are bitwise identical to n separate
 * rich_step_accel (or rich_step) calls. */
int rich_step_batch_accel(int32_t n, rich_ctx* const* ctxs, rich_state* const* states,
                          const double* dt, const rich_params* const* params,
                          const double* const* ax, const double* const* ay, rich_tess_fn tess,
                          rich_tess_release_fn release, void* const* tess_users,
                          int32_t n_threads, int32_t* status, void* ws, size_t ws_bytes,
                          void* stream);

/*
 * Device re-tessellation (section 2.1: the mesh is the Voronoi tessellation
 * of the mesh points, rebuilt after every move).  The Voronoi cell of each
 * new point is found by clipping, on the device, the box (walls) or the
 * square bounded by the point's own periodic images against the bisectors
 * with candidate points: the neighbours and neighbours' neighbours of the
 * cell in a previous mesh `prev` of the same points (periodic: the nearest
 * image of each candidate).  A cell that keeps its previous neighbours
 * (each vertex of two consecutive ones inside every other candidate's half
 * plane, by a margin of 1e-9 of the squared lengths) is taken from that
 * ring directly; only the others are clipped.  The result has the input
 * stage's layout and
 * rules: the same neighbour codes, edges shorter than 1e-12 (R_i + R_j)/2
 * dropped, an edge owned by the lower-numbered cell (a wall edge by its
 * cell; an edge with the cell's own periodic image by the side with code
 * >= 5), each cell's edges and CSR entries counter-clockwise.  The order of
 * a cell's entries may start elsewhere than the host stage's, so stage
 * results on the two meshes agree to rounding, not bitwise.
 *
 * The tessellation is certified on the device: every kept edge must be seen
 * by both of its cells with the same length and midpoint (each edge's owner
 * checks it, and the counts of kept and owned edges must agree), and the
 * cell areas must sum to the box area.  Each clipped cell contains the true cell, so together these
 * fail when a true neighbour was missing from the candidates (points moved
 * further than the previous mesh's second ring).  Then a RICH_RETESS_*
 * bit is set, the output mesh is left with no edges (a stage on it reads no
 * edge), and the caller rebuilds the mesh on the host (rich_tess_build).
 */
#define RICH_RETESS_POINT    1   /* a point outside the box or not finite       */
#define RICH_RETESS_FAN      2   /* a cell with more than 16 candidates (previous
                                    neighbours and entrants) or 20 edges         */
#define RICH_RETESS_CLIP     4   /* a clip left nothing, or parallel bisectors  */
#define RICH_RETESS_ASYM     8   /* an edge not seen alike from both cells      */
#define RICH_RETESS_AREA    16   /* cell areas do not sum to the box area       */
#define RICH_RETESS_CAP     32   /* more edges than the output capacity         */

/* Device buffers of a re-tessellated mesh (caller-allocated, sizes from
 * rich_retess_capacity). */
typedef struct rich_mesh_bufs {
  int64_t n_cells;
  int64_t cap_edges;     /* entries of edges[]                        */
  int64_t cap_csr;       /* entries of idx[]                          */
  rich_cell* cells;      /* [n_cells], 16-byte aligned                */
  rich_edge* edges;      /* [cap_edges], 16-byte aligned              */
  int32_t* off;          /* [n_cells + 1]                             */
  int32_t* idx;          /* [cap_csr]                                 */
  int32_t* eoff;         /* [n_cells + 1]                             */
} rich_mesh_bufs;

/* Edge and CSR capacities that hold any mesh of n_cells cells (at most
 * 3 n interior edges plus the wall edges). */
int rich_retess_capacity(int64_t n_cells, int64_t* cap_edges, int64_t* cap_csr);

/* Workspace bytes of rich_retess for n_cells cells (256-byte aligned device
 * memory).  Its first 64 bytes are the result header (rich_retess_result);
 * the caller zeroes them once when allocating it. */
int rich_retess_workspace_size(int64_t n_cells, size_t* bytes);

/* Re-tessellate: new points (x, y) (device arrays of prev->n_cells; walls:
 * strictly inside the box, periodic: inside [x0, x1) x [y0, y1), as a stage
 * leaves them) with candidates from mesh `prev`, into `out`.  prev and out
 * must not share memory.  Enqueued on `stream`; RICH_E_INVAL without
 * enqueuing for bad arguments (a periodic box needs at least 16 cells). */
int rich_retess(const rich_mesh* prev, const double* x, const double* y,
                const rich_mesh_bufs* out, void* ws, size_t ws_bytes, void* stream);

/* The stage's view of `out` after rich_retess: n_edges and n_csr are the
 * capacities (the kernels use them as bounds only), box and bc as given. */
int rich_retess_view(const rich_mesh_bufs* out, const double box[4], uint32_t bc,
                     rich_mesh* m);

/* Many re-tessellations at once, one launch per kernel for all n runs: run
 * r as rich_retess(prev[r], x[r], y[r], out[r], ws[r], ws_bytes[r]), each
 * run with its own workspace and output buffers.  bws is device memory of
 * rich_retess_batch_workspace_size bytes, 256-byte aligned; the runs'
 * descriptors are copied into it on `stream` from a pinned staging buffer
 * of the library (the call does not wait on the stream), then the kernels
 * are enqueued.  Any run's bad arguments fail the whole call with that
 * run's status, before anything is enqueued.  The results are read with
 * rich_retess_batch_result (or per run with rich_retess_result), or the
 * runs' flags without a wait with rich_retess_batch_flags_async. */
int rich_retess_batch_workspace_size(int32_t n, size_t* bytes);
int rich_retess_batch(int32_t n, const rich_mesh* const* prev, const double* const* x,
                      const double* const* y, const rich_mesh_bufs* const* out,
                      void* const* ws, const size_t* ws_bytes, void* bws, size_t bws_bytes,
                      void* stream);

typedef struct rich_retess_info {
  int32_t flags;      /* RICH_RETESS_* bits of the last rich_retess on ws   */
  int32_t sticky;     /* OR of the flags of every call since ws was zeroed  */
  int64_t n_edges;    /* edges and CSR entries of the last mesh             */
  int64_t n_csr;
  int64_t n_dropped;  /* degenerate edges left out                          */
  double area_sum;    /* sum of the cell areas (a check value, summed in a
                         fixed order: the same bits on every call)         */
  int64_t n_clipped;  /* cells that did not keep their previous ring (or
                         were not proved to) and were clipped              */
} rich_retess_info;

/* Synchronise `stream` and read the header of ws.  Returns RICH_E_MESH when
 * the last call's flags are set, else RICH_OK. */
int rich_retess_result(void* ws, void* stream, rich_retess_info* info);
/* Synchronise `stream` and read the results of the last rich_retess_batch on
 * bws: info[r] and status[r] (RICH_E_MESH when run r's flags are set) for
 * its n runs. */
int rich_retess_batch_result(int32_t n, void* bws, void* stream, rich_retess_info* info,
                             int32_t* status);
/* Enqueue on `stream` a copy of the RICH_RETESS_* flags of the last
 * rich_retess_batch on bws (n runs, in the batch's order) into host_flags[n]
 * (caller-owned host memory; pinned memory keeps the copy asynchronous).
 * The values are valid once the stream has passed this point (an event
 * recorded after the call has completed); nonzero flags mean the run's mesh
 * was not built (RICH_E_MESH from rich_retess_batch_result).  For serving
 * loops that poll events instead of synchronising.  RICH_E_INVAL for a null
 * pointer or n <= 0. */
int rich_retess_batch_flags_async(int32_t n, void* bws, void* stream, int32_t* host_flags);

/*
 * Kernel timing for benchmarks.  While enabled, every stage records HIP
 * events on its launch stream around each of its kernels ("k_cell",
 * "k_flux", or "k_stage" for the fused variant); rich_profile_read
 * synchronises those events, returns the summed duration in milliseconds
 * and the number of launches of the named kernel since the last read, and
 * forgets them.  Not thread-safe; off by default.
 */
int rich_profile_enable(int on);
int rich_profile_read(const char* kernel, double* total_ms, int64_t* launches);

/* Human-readable name of a status code. */
const char* rich_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* RICH_H */
