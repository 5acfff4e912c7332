// Kernels and C-ABI of one stage of RICH's moving-mesh Godunov scheme on
// gfx950 (MI355X).  See rich.h for the interface, rich_fused.hpp for the
// stage kernel and rich_device.hpp for the per-cell and per-edge arithmetic.
//
// One stage is one kernel over tiles of consecutive cells (cells come in
// Hilbert order, so a tile is a compact patch of the mesh): each tile
// reconstructs its cells and their two-ring halo in LDS and then every cell
// sums the fluxes of its edges in CSR order (k_stage).  Tiles whose halo does
// not fit the LDS are finished from global memory by k_stage_overflow.  The
// Courant step (k_cfl, k_cfl_final) is a separate light pass, since the
// update of every cell needs the minimum over all of them.
//
// No atomics touch the state: the sum order is fixed by the CSR, so the
// result does not depend on the tile size, the grid or the batch.
//
// Tiles are mapped to blocks so that each of the 8 XCDs (each with its own
// L2) processes one contiguous range of tiles: neighbouring tiles, whose
// cells are each other's halo, then share an L2.
//
// All HIP code is built with packed-FP32 instructions disabled and without
// fast-math; nothing here writes through the scalar cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "rich.h"
#include "rich_device.hpp"
#include "rich_fused.hpp"

static_assert(sizeof(rich_cell) == 48, "rich_cell is three 16-byte chunks");
static_assert(sizeof(rich_edge) == 32, "rich_edge is two 16-byte chunks");

namespace rich {

constexpr size_t kHeader = 256;  // per-run workspace header

// ---------------------------------------------------------------------------
// workspace header: flag word and Courant minimum
// ---------------------------------------------------------------------------
__global__ void k_clear(int32_t* flag, unsigned long long* cfl_min, int32_t* ovf_count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *flag = 0;
    *cfl_min = 0x7FF0000000000000ull;  // +inf
    *ovf_count = 0;
  }
}

__global__ void k_clear_batch(const RunDesc* __restrict__ descs, int n_runs,
                              int32_t* ovf_counts) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_runs) {
    *descs[r].flag = 0;
    *descs[r].cfl_min = 0x7FF0000000000000ull;
  }
  if (r < 2) ovf_counts[r] = 0;
}

// ---------------------------------------------------------------------------
// A0: Courant step, min over cells of R/(c + |v - w|).  Two levels: each
// block of a bounded grid reduces its cells to one value in scratch, then a
// single block reduces those (min is order-free, so the result is
// deterministic).  A cell whose ratio is not a positive number makes the
// minimum 0, which the host reports as a domain error.
// ---------------------------------------------------------------------------
constexpr int kCflThreads = 256;
constexpr int kCflMaxBlocks = 16384;  // one cell per thread up to 4.19M cells, then strides

__device__ __forceinline__ double block_min(double t, double* smin) {
  for (int o = 32; o > 0; o >>= 1) t = fmin(t, __shfl_xor(t, o));
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = t;
  __syncthreads();
  double m = smin[0];
  for (int w = 1; w < kCflThreads / 64; ++w) m = fmin(m, smin[w]);
  return m;
}

// Area change rate of every cell implied by its edges' velocities (section 5,
// eq. areachange): each edge moves along its normal with the edge velocity of
// the moving frame, so dA_i/dt = -sum_j L_ij ((w_j - w_i).c_ij - (w_i + w_j)/2 .
// r_ij) / |r_ij| with r_ij from point i to the neighbour (image or mirror) and
// c_ij from their midpoint to the edge centre.  The point velocities come
// from k_wvel (w[2i], w[2i+1]).
__global__ __launch_bounds__(kCflThreads) void k_wvel(RunDesc d, double* w) {
  const int i = blockIdx.x * kCflThreads + threadIdx.x;
  if (i >= d.n) return;
  Own o;
  double q[4];
  own_load(d, i, o, q);
  own_from(d, q[0], q[1], q[2], q[3], o);
  w[2 * (size_t)i] = o.wx;
  w[2 * (size_t)i + 1] = o.wy;
}

__global__ __launch_bounds__(kCflThreads) void k_adot(RunDesc d, const double* w,
                                                      double* adot) {
  const int i = blockIdx.x * kCflThreads + threadIdx.x;
  if (i >= d.n) return;
  double rix, riy;
  load_point(d, i, rix, riy);
  const double wix = w[2 * (size_t)i], wiy = w[2 * (size_t)i + 1];
  int k0 = d.off[i], k1 = d.off[i + 1];
  bool bad = false;
  if (k0 < 0 || k1 < k0 || k1 > d.n_csr) {
    bad = true;
    k1 = k0;
  }
  double s = 0.0;
  for (int k = k0; k < k1; ++k) {
    const NbE v = nb_edge(d, i, d.idx[k], bad);
    double rjx, rjy, wjx, wjy;
    if (v.wall) {
      mirror_point(d, v.wall, rix, riy, rjx, rjy);
      mirror_vec(v.wall, wix, wiy, wjx, wjy);
    } else {
      load_point(d, v.j, rjx, rjy);
      rjx += v.shx;
      rjy += v.shy;
      wjx = w[2 * (size_t)v.j];
      wjy = w[2 * (size_t)v.j + 1];
    }
    const double rx = rjx - rix, ry = rjy - riy;
    const double r = sqrt(rx * rx + ry * ry);
    const double cx = v.fx - 0.5 * (rix + rjx), cy = v.fy - 0.5 * (riy + rjy);
    const double t1 = ((wjx - wix) * cx + (wjy - wiy) * cy) / r;
    const double t2 = (0.5 * (wix + wjx) * rx + 0.5 * (wiy + wjy) * ry) / r;
    s -= v.L * (t1 - t2);
  }
  adot[i] = s;
  if (bad) atomicOr(d.flag, RICH_FLAG_DOMAIN);
}

__global__ __launch_bounds__(kCflThreads) void k_cfl(RunDesc d, double* block_out) {
  __shared__ double smin[kCflThreads / 64];
  double t = INFINITY;
  for (int i = blockIdx.x * kCflThreads + threadIdx.x; i < d.n; i += gridDim.x * kCflThreads) {
    double pxi, pyi, A, sxi, syi;
    load_cell(d, i, pxi, pyi, A, sxi, syi);
    double rho, vx, vy, p;
    prim_of(d, i, A, rho, vx, vy, p);
    const double c = sqrt(d.gamma * p / rho);
    const double R = sqrt(A / kPi);
    double wx = 0.0, wy = 0.0;
    if (d.motion) {
      wx = vx;
      wy = vy;
      const double dx = sxi - pxi, dy = syi - pyi;
      const double dd = sqrt(dx * dx + dy * dy);
      if (dd > d.eta * R) {
        wx += d.chi * c * dx / dd;
        wy += d.chi * c * dy / dd;
      }
    }
    const double ux = vx - wx, uy = vy - wy;
    const double s = c + sqrt(ux * ux + uy * uy);
    double ti = R / s;
    if (!(ti > 0.0) || !isfinite(ti)) ti = 0.0;
    t = fmin(t, ti);
  }
  const double m = block_min(t, smin);
  if (threadIdx.x == 0) block_out[blockIdx.x] = m;
}

constexpr int kCflFinalThreads = 1024;
// The minimum of the block minima, as a bit pattern in *out; with dt_out
// also dt = cfl * minimum in *dt_out, and the domain flag when that is not
// a positive number.
__global__ __launch_bounds__(kCflFinalThreads) void k_cfl_final(const double* block_in, int nb,
                                                                unsigned long long* out,
                                                                double cfl, double* dt_out,
                                                                int32_t* flag) {
  __shared__ double smin[kCflFinalThreads / 64];
  // four independent minima per thread, so the loads of a thread overlap
  double t0 = INFINITY, t1 = INFINITY, t2 = INFINITY, t3 = INFINITY;
  int b = threadIdx.x;
  for (; b + 3 * kCflFinalThreads < nb; b += 4 * kCflFinalThreads) {
    t0 = fmin(t0, block_in[b]);
    t1 = fmin(t1, block_in[b + kCflFinalThreads]);
    t2 = fmin(t2, block_in[b + 2 * kCflFinalThreads]);
    t3 = fmin(t3, block_in[b + 3 * kCflFinalThreads]);
  }
  for (; b < nb; b += kCflFinalThreads) t0 = fmin(t0, block_in[b]);
  double t = fmin(fmin(t0, t1), fmin(t2, t3));
  for (int o = 32; o > 0; o >>= 1) t = fmin(t, __shfl_xor(t, o));
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smin[0];
    for (int w = 1; w < kCflFinalThreads / 64; ++w) m = fmin(m, smin[w]);
    *out = (unsigned long long)__double_as_longlong(m);
    if (dt_out != nullptr) {
      const double dt = cfl * m;
      *dt_out = dt;
      if (!(dt > 0.0) || !isfinite(dt)) atomicOr(flag, RICH_FLAG_DOMAIN);
    }
  }
}

}  // namespace rich

// ===========================================================================
// Host side
// ===========================================================================
using rich::RunDesc;

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? RICH_OK : RICH_E_DEVICE; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Workspace of one run: a 256-byte header (flag word @0, Courant minimum @8,
// device dt @16, overflow count @24), the overflow list (one (run, tile)
// pair per tile of the smallest tile size), the Courant block minima, and
// the point velocities of the area-rate call.
constexpr size_t kDtOffset = 16;
constexpr size_t kOvfOffset = 24;
constexpr int kMinTile = 128;
struct RunWs {
  size_t ovf, cfl, w, total;
};
RunWs run_ws(int64_t n) {
  RunWs L;
  size_t o = rich::kHeader;
  L.ovf = o;
  o += align_up(sizeof(int2) * (size_t)((n + kMinTile - 1) / kMinTile), 256);
  L.cfl = o;
  o += align_up(sizeof(double) * (size_t)std::min<int64_t>(
                                     (n + rich::kCflThreads - 1) / rich::kCflThreads,
                                     rich::kCflMaxBlocks), 256);
  L.w = o;
  o += align_up(2 * sizeof(double) * (size_t)n, 256);
  L.total = o;
  return L;
}
size_t run_ws_bytes(int64_t n) { return run_ws(n).total; }

bool valid_mesh(const rich_mesh* m) {
  return m && m->n_cells > 0 && m->n_cells <= (int64_t)rich::kCellMask && m->n_edges >= 0 &&
         m->n_edges < (int64_t)INT32_MAX / 2 && m->n_csr >= 0 && m->n_csr < (int64_t)INT32_MAX &&
         m->cells && (reinterpret_cast<uintptr_t>(m->cells) & 15) == 0 && m->off && m->eoff &&
         (m->n_edges == 0 ||
          (m->edges && (reinterpret_cast<uintptr_t>(m->edges) & 15) == 0)) &&
         (m->n_csr == 0 || m->idx) && m->box[2] > m->box[0] && m->box[3] > m->box[1] &&
         (m->bc == RICH_BOUNDARY_WALLS || m->bc == RICH_BOUNDARY_PERIODIC);
}

bool valid_state(const rich_state* s, int64_t n, bool need_points) {
  return s && s->n_cells == n && s->M && s->Px && s->Py && s->E &&
         (!need_points || (s->x && s->y));
}

bool valid_params(const rich_params* p) {
  return p && p->gamma > 1.0 && std::isfinite(p->gamma) && p->riemann >= 0 && p->riemann <= 1 &&
         p->motion >= 0 && p->motion <= 1 && p->limiter >= 0 && p->limiter <= 4 &&
         std::isfinite(p->gx) && std::isfinite(p->gy) && p->integrator >= 0 &&
         p->integrator <= 1;
}

RunDesc make_desc(const rich_mesh* m, const rich_state* src, const rich_state* base,
                  rich_state* out, double h, const rich_params* p, char* ws) {
  RunDesc d;
  std::memset(&d, 0, sizeof(d));
  d.cells = m->cells;
  d.edges = m->edges;
  d.off = m->off; d.idx = m->idx; d.eoff = m->eoff;
  d.sM = src->M; d.sPx = src->Px; d.sPy = src->Py; d.sE = src->E;
  if (base) {
    d.bM = base->M; d.bPx = base->Px; d.bPy = base->Py; d.bE = base->E;
    d.bx = base->x; d.by = base->y;
  }
  if (out) {
    d.oM = out->M; d.oPx = out->Px; d.oPy = out->Py; d.oE = out->E;
    d.ox = out->x; d.oy = out->y;
  }
  const RunWs L = run_ws(m->n_cells);
  d.flag = reinterpret_cast<int32_t*>(ws);
  d.cfl_min = reinterpret_cast<unsigned long long*>(ws + 8);
  d.ovf_count = reinterpret_cast<int32_t*>(ws + kOvfOffset);
  d.ovf_list = reinterpret_cast<int2*>(ws + L.ovf);
  d.rec = reinterpret_cast<double*>(ws + L.w);
  d.x0 = m->box[0]; d.y0 = m->box[1]; d.x1 = m->box[2]; d.y1 = m->box[3];
  d.Lx = m->box[2] - m->box[0];
  d.Ly = m->box[3] - m->box[1];
  d.h = h;
  d.gamma = p->gamma; d.theta = p->theta; d.delta_v = p->delta_v; d.delta_p = p->delta_p;
  d.chi = p->chi; d.eta = p->eta; d.cfl = p->cfl;
  d.rgm1 = 1.0 / (p->gamma - 1.0);
  d.gx = p->gx;
  d.gy = p->gy;
  d.n = (int32_t)m->n_cells;
  d.n_edges = (int32_t)m->n_edges;
  d.n_csr = (int32_t)m->n_csr;
  d.bc = (int32_t)m->bc;
  d.riemann = p->riemann; d.motion = p->motion; d.limiter = p->limiter;
  d.integrator = p->integrator;
  return d;
}

// ---------------------------------------------------------------------------
// kernel timing: event pairs recorded around launches while enabled
// ---------------------------------------------------------------------------
struct ProfEntry {
  std::string name;
  hipEvent_t a, b;
};
struct Profiler {
  bool on = false;
  std::vector<ProfEntry> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler& profiler() {
  static Profiler p;
  return p;
}

// Records the start event of a kernel; returns the index to close, or -1.
int prof_begin(const char* name, hipStream_t st) {
  Profiler& P = profiler();
  if (!P.on) return -1;
  ProfEntry e{name, P.get(), P.get()};
  if (!e.a || !e.b) return -1;
  (void)hipEventRecord(e.a, st);
  P.pending.push_back(e);
  return (int)P.pending.size() - 1;
}
void prof_end(int k, hipStream_t st) {
  if (k >= 0) (void)hipEventRecord(profiler().pending[k].b, st);
}

#ifndef RICH_STAGE_TILE
#define RICH_STAGE_TILE 256
#endif
constexpr int kStageTile = RICH_STAGE_TILE;   // cells per tile of the fused stage kernel

// Courant step on the device: per-block minima of R/(c + |v - w|) into
// d.cfl_blocks, then dt = cfl * minimum into *d.h_dev (the workspace's dt
// slot), before the stage that reads it.
int launch_courant(const RunDesc& d, hipStream_t st) {
  const int nb = std::min<int>((d.n + rich::kCflThreads - 1) / rich::kCflThreads,
                               rich::kCflMaxBlocks);
  int pc = prof_begin("k_cfl", st);
  hipLaunchKernelGGL(rich::k_cfl, dim3(nb), dim3(rich::kCflThreads), 0, st, d, d.cfl_blocks);
  hipLaunchKernelGGL(rich::k_cfl_final, dim3(1), dim3(rich::kCflFinalThreads), 0, st,
                     (const double*)d.cfl_blocks, nb, d.cfl_min, d.cfl,
                     const_cast<double*>(d.h_dev), d.flag);
  prof_end(pc, st);
  return RICH_OK;
}

constexpr int kOverflowGrid = 256;  // blocks of the overflow pass (most exit at once)

int launch_stage(const RunDesc& d, int riemann, hipStream_t st, uint8_t* dbg_cell = nullptr,
                 uint8_t* dbg_edge = nullptr) {
  constexpr int T = kStageTile;
  const int n_tiles = (d.n + T - 1) / T;
  const int og = std::min(n_tiles, kOverflowGrid);
  hipLaunchKernelGGL(rich::k_clear, dim3(1), dim3(64), 0, st, d.flag, d.cfl_min, d.ovf_count);
  if (d.cfl_blocks != nullptr) launch_courant(d, st);
  const bool dbg = dbg_cell != nullptr;
  int pf = prof_begin("k_stage", st);
  if (riemann == 1) {
    if (dbg)
      hipLaunchKernelGGL((rich::k_stage<T, 1, false, true>), dim3(n_tiles), dim3(rich::TileCfg<T>::kThreads), 0, st, d,
                         (const RunDesc*)nullptr, (const int2*)nullptr, n_tiles, dbg_cell,
                         dbg_edge);
    else
      hipLaunchKernelGGL((rich::k_stage<T, 1, false>), dim3(n_tiles), dim3(rich::TileCfg<T>::kThreads), 0, st, d,
                         (const RunDesc*)nullptr, (const int2*)nullptr, n_tiles,
                         (uint8_t*)nullptr, (uint8_t*)nullptr);
  } else {
    if (dbg)
      hipLaunchKernelGGL((rich::k_stage<T, 0, false, true>), dim3(n_tiles), dim3(rich::TileCfg<T>::kThreads), 0, st, d,
                         (const RunDesc*)nullptr, (const int2*)nullptr, n_tiles, dbg_cell,
                         dbg_edge);
    else
      hipLaunchKernelGGL((rich::k_stage<T, 0, false>), dim3(n_tiles), dim3(rich::TileCfg<T>::kThreads), 0, st, d,
                         (const RunDesc*)nullptr, (const int2*)nullptr, n_tiles,
                         (uint8_t*)nullptr, (uint8_t*)nullptr);
  }
  prof_end(pf, st);
  const int* oc = d.ovf_count;
  const int2* ol = d.ovf_list;
  const RunDesc* nd = nullptr;
  if (riemann == 1) {
    if (dbg)
      hipLaunchKernelGGL((rich::k_stage_overflow<T, 1, false, true>), dim3(og), dim3(T), 0, st, d,
                         nd, oc, ol, dbg_cell, dbg_edge);
    else
      hipLaunchKernelGGL((rich::k_stage_overflow<T, 1, false>), dim3(og), dim3(T), 0, st, d, nd,
                         oc, ol, (uint8_t*)nullptr, (uint8_t*)nullptr);
  } else {
    if (dbg)
      hipLaunchKernelGGL((rich::k_stage_overflow<T, 0, false, true>), dim3(og), dim3(T), 0, st, d,
                         nd, oc, ol, dbg_cell, dbg_edge);
    else
      hipLaunchKernelGGL((rich::k_stage_overflow<T, 0, false>), dim3(og), dim3(T), 0, st, d, nd,
                         oc, ol, (uint8_t*)nullptr, (uint8_t*)nullptr);
  }
  return hip_status(hipGetLastError());
}

}  // namespace

// ---------------------------------------------------------------------------
// batch workspace: a fixed part that depends on the number of runs only
// (descriptors, flag words, Courant minima, the two overflow counts), then
// the tile table and the two overflow lists, each with room for the tiles
// of the smallest tile size
// ---------------------------------------------------------------------------
struct BatchLayout {
  size_t desc, flags, cfl, ovfc, tiles, ovf[2], total;
  int64_t max_tiles;
};

BatchLayout batch_layout(int32_t n, const int64_t* n_cells) {
  BatchLayout L;
  size_t o = 0;
  L.desc = o;
  o += align_up((size_t)n * sizeof(RunDesc), 256);
  L.flags = o;
  o += align_up((size_t)n * sizeof(int32_t), 256);
  L.cfl = o;
  o += align_up((size_t)n * sizeof(unsigned long long), 256);
  L.ovfc = o;
  o += 256;
  L.max_tiles = 0;
  if (n_cells)
    for (int32_t r = 0; r < n; ++r) L.max_tiles += (n_cells[r] + kMinTile - 1) / kMinTile;
  const size_t tb = align_up(sizeof(int2) * (size_t)L.max_tiles, 256);
  L.tiles = o;
  o += tb;
  L.ovf[0] = o;
  o += tb;
  L.ovf[1] = o;
  o += tb;
  L.total = o;
  return L;
}

struct Staging {
  struct Buf {
    void* p = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
  };
  Buf bufs[4];
  int next = 0;
  void* get(size_t bytes, hipEvent_t* ev) {
    Buf& b = bufs[next];
    next = (next + 1) % 4;
    if (b.done) (void)hipEventSynchronize(b.done);
    if (b.cap < bytes) {
      if (b.p) (void)hipHostFree(b.p);
      b.p = nullptr;
      b.cap = 0;
      if (hipHostMalloc(&b.p, bytes, 0) != hipSuccess) return nullptr;
      b.cap = bytes;
    }
    if (!b.done && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
      return nullptr;
    *ev = b.done;
    return b.p;
  }
};
Staging& staging() {
  static Staging s;
  return s;
}
std::mutex& staging_lock() {
  static std::mutex m;
  return m;
}

// Copy two host blocks into device memory through the pinned ring, on
// stream st.  The whole sequence (pick a buffer, fill it, enqueue the
// copies, record the buffer's event) holds one lock, so host threads that
// launch batches concurrently never share a buffer in flight.
int upload_staged(void* dst1, const void* src1, size_t b1, void* dst2, const void* src2,
                  size_t b2, hipStream_t st) {
  std::lock_guard<std::mutex> g(staging_lock());
  hipEvent_t ev = nullptr;
  char* host = static_cast<char*>(staging().get(b1 + b2, &ev));
  if (!host) return RICH_E_NOMEM;
  std::memcpy(host, src1, b1);
  std::memcpy(host + b1, src2, b2);
  if (hipMemcpyAsync(dst1, host, b1, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dst2, host + b1, b2, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(ev, st) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}

int resident_blocks(const void* kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 1024;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess ||
      per < 1)
    per = 1;
  return cus * per;
}

// ---------------------------------------------------------------------------
// step driver: device buffers owned by a rich_ctx
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool ensure(size_t bytes) {
    if (bytes <= cap) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
    cap = std::max<size_t>(bytes, 256);
    return true;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

struct DevMesh {
  DevBuf b[5];  // cells edges off idx eoff
  std::vector<rich_cell> hc;  // host staging of the packed records
  std::vector<rich_edge> he;
  int64_t n = 0, ne = 0, nc = 0;
  double box[4] = {0, 0, 1, 1};
  uint32_t bc = 0;
  bool set = false;

  int upload(const rich_host_mesh_view* hm, const double* bx, uint32_t bcv, hipStream_t st) {
    int rc = upload_async(hm, bx, bcv, st);
    if (rc) return rc;
    return hipStreamSynchronize(st) == hipSuccess ? RICH_OK : RICH_E_DEVICE;
  }
  // Enqueues the copies; the host arrays (and this object's staging) must
  // stay valid until the stream has passed them.
  int upload_async(const rich_host_mesh_view* hm, const double* bx, uint32_t bcv,
                   hipStream_t st) {
    const int64_t n_ = hm->n_cells, ne_ = hm->n_edges, nc_ = hm->n_csr;
    try {
      hc.resize((size_t)n_);
      he.resize((size_t)std::max<int64_t>(ne_, 0));
    } catch (...) {
      return RICH_E_NOMEM;
    }
    int rc = rich_mesh_pack(hm, hc.data(), he.data());
    if (rc) return rc;
    const void* src[5] = {hc.data(), he.data(), hm->off, hm->idx, hm->eoff};
    const size_t bytes[5] = {sizeof(rich_cell) * (size_t)n_, sizeof(rich_edge) * (size_t)ne_,
                             4 * (size_t)(n_ + 1), 4 * (size_t)nc_, 4 * (size_t)(n_ + 1)};
    for (int k = 0; k < 5; ++k) {
      if (bytes[k] && !src[k]) return RICH_E_INVAL;
      if (!b[k].ensure(bytes[k])) return RICH_E_NOMEM;
      if (bytes[k] &&
          hipMemcpyAsync(b[k].p, src[k], bytes[k], hipMemcpyHostToDevice, st) != hipSuccess)
        return RICH_E_DEVICE;
    }
    n = n_;
    ne = ne_;
    nc = nc_;
    std::memcpy(box, bx, sizeof(box));
    bc = bcv;
    set = true;
    return RICH_OK;
  }
  void view(rich_mesh* m) const {
    m->n_cells = n;
    m->n_edges = ne;
    m->n_csr = nc;
    m->cells = (const rich_cell*)b[0].p;
    m->edges = (const rich_edge*)b[1].p;
    m->off = (const int32_t*)b[2].p;
    m->idx = (const int32_t*)b[3].p;
    m->eoff = (const int32_t*)b[4].p;
    std::memcpy(m->box, box, sizeof(box));
    m->bc = bc;
  }
  void release() {
    for (auto& x : b) x.release();
    std::vector<rich_cell>().swap(hc);
    std::vector<rich_edge>().swap(he);
    set = false;
  }
};

struct rich_ctx {
  DevMesh cur, spare, third;
  DevBuf Qh, Xh, Qn, Xn, ws;
  void* hostX = nullptr;
  size_t hostX_cap = 0;
  // device re-tessellation with the host stage as fallback
  bool device_tess = false;
  DevBuf rws;                 // rich_retess workspace (header zeroed at allocation)
  DevBuf bws;                 // descriptors of a batched rebuild this context leads
  int64_t n_device = 0, n_fallback = 0;
};

namespace {

rich_state state_view(DevBuf& Q, DevBuf& X, int64_t n) {
  rich_state s;
  double* q = (double*)Q.p;
  double* x = (double*)X.p;
  s.M = q; s.Px = q + n; s.Py = q + 2 * n; s.E = q + 3 * n;
  s.x = x; s.y = x + n;
  s.n_cells = n;
  return s;
}

// Buffers of a device rebuild of run c's n-cell mesh into dst, described in out.
int retess_prepare(rich_ctx* c, int64_t n, DevMesh& dst, hipStream_t st, rich_mesh_bufs& out) {
  int64_t ce = 0, cc = 0;
  size_t wsb = 0;
  if (rich_retess_capacity(n, &ce, &cc) || rich_retess_workspace_size(n, &wsb))
    return RICH_E_INVAL;
  const size_t bytes[5] = {sizeof(rich_cell) * (size_t)n, sizeof(rich_edge) * (size_t)ce,
                           4 * (size_t)(n + 1), 4 * (size_t)cc, 4 * (size_t)(n + 1)};
  for (int k = 0; k < 5; ++k)
    if (!dst.b[k].ensure(bytes[k])) return RICH_E_NOMEM;
  if (c->rws.cap < wsb) {
    if (!c->rws.ensure(wsb)) return RICH_E_NOMEM;
    if (hipMemsetAsync(c->rws.p, 0, 256, st) != hipSuccess) return RICH_E_DEVICE;
  }
  out.n_cells = n;
  out.cap_edges = (int64_t)(dst.b[1].cap / sizeof(rich_edge));
  out.cap_csr = std::min<int64_t>((int64_t)(dst.b[3].cap / 4), (int64_t)INT32_MAX - 1);
  out.cells = (rich_cell*)dst.b[0].p;
  out.edges = (rich_edge*)dst.b[1].p;
  out.off = (int32_t*)dst.b[2].p;
  out.idx = (int32_t*)dst.b[3].p;
  out.eoff = (int32_t*)dst.b[4].p;
  dst.set = false;
  return RICH_OK;
}

// Take a certified rebuilt mesh (counts in info) into dst.
void retess_adopt(const rich_mesh& prev, const rich_retess_info& info, DevMesh& dst) {
  dst.n = prev.n_cells;
  dst.ne = info.n_edges;
  dst.nc = info.n_csr;
  std::memcpy(dst.box, prev.box, sizeof(dst.box));
  dst.bc = prev.bc;
  dst.set = true;
}

// The mesh of points (x, y) (device) into dst, rebuilt on the device with
// candidates from prev.  RICH_E_MESH when the result is not certified.
int retess_into(rich_ctx* c, const rich_mesh& prev, const double* x, const double* y,
                DevMesh& dst, hipStream_t st) {
  rich_mesh_bufs out;
  int rc = retess_prepare(c, prev.n_cells, dst, st, out);
  if (rc) return rc;
  if ((rc = rich_retess(&prev, x, y, &out, c->rws.p, c->rws.cap, st))) return rc;
  rich_retess_info info;
  if ((rc = rich_retess_result(c->rws.p, st, &info))) return rc;
  retess_adopt(prev, info, dst);
  return RICH_OK;
}

int tessellate_into(rich_ctx* c, DevMesh& dst, const double* dx, int64_t n, const double* box,
                    uint32_t bc, rich_tess_fn tess, rich_tess_release_fn release, void* user,
                    hipStream_t st) {
  const size_t bytes = 2 * (size_t)n * sizeof(double);
  if (c->hostX_cap < bytes) {
    if (c->hostX) (void)hipHostFree(c->hostX);
    c->hostX = nullptr;
    c->hostX_cap = 0;
    if (hipHostMalloc(&c->hostX, bytes, 0) != hipSuccess) return RICH_E_NOMEM;
    c->hostX_cap = bytes;
  }
  if (hipMemcpyAsync(c->hostX, dx, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return RICH_E_DEVICE;
  const double* hx = (const double*)c->hostX;
  rich_host_mesh_view hv;
  std::memset(&hv, 0, sizeof(hv));
  if (tess(user, hx, hx + n, n, box, bc, &hv) != 0) return RICH_E_MESH;
  int rc = RICH_E_MESH;
  if (hv.n_cells == n) rc = dst.upload(&hv, box, bc, st);
  release(user, &hv);
  return rc;
}

}  // namespace

extern "C" {

void rich_params_default(rich_params* p, double gamma) {
  if (!p) return;
  p->gamma = gamma;
  p->cfl = 0.3;
  p->theta = 0.5;
  p->delta_v = 0.2;
  p->delta_p = 0.7;
  p->chi = 0.15;
  p->eta = 0.02;
  p->riemann = 0;
  p->motion = 1;
  p->limiter = 0;
  p->gx = 0.0;
  p->gy = 0.0;
  p->integrator = 0;
}

int rich_workspace_size(int64_t n_cells, size_t* bytes) {
  if (!bytes || n_cells <= 0 || n_cells > (int64_t)rich::kCellMask) return RICH_E_INVAL;
  *bytes = run_ws_bytes(n_cells);
  return RICH_OK;
}

int rich_stage(const rich_mesh* m, const rich_state* src, const rich_state* base,
               rich_state* out, double h, const rich_params* p, void* ws, size_t ws_bytes,
               void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !ws) return RICH_E_INVAL;
  const int64_t n = m->n_cells;
  if (!valid_state(src, n, false) || !valid_state(base, n, true) || !valid_state(out, n, true))
    return RICH_E_INVAL;
  if (!std::isfinite(h) || h < 0.0) return RICH_E_INVAL;
  if (out->M == src->M || out->M == base->M || out->x == base->x) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(n) || (reinterpret_cast<uintptr_t>(ws) & 255)) return RICH_E_NOMEM;
  RunDesc d = make_desc(m, src, base, out, h, p, static_cast<char*>(ws));
  return launch_stage(d, p->riemann, static_cast<hipStream_t>(stream));
}

int rich_stage_accel(const rich_mesh* m, const rich_state* src, const rich_state* base,
                     rich_state* out, double h, const rich_params* p, const double* ax,
                     const double* ay, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !ws || !ax || !ay) return RICH_E_INVAL;
  const int64_t n = m->n_cells;
  if (!valid_state(src, n, false) || !valid_state(base, n, true) || !valid_state(out, n, true))
    return RICH_E_INVAL;
  if (!std::isfinite(h) || h < 0.0) return RICH_E_INVAL;
  if (out->M == src->M || out->M == base->M || out->x == base->x) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(n) || (reinterpret_cast<uintptr_t>(ws) & 255)) return RICH_E_NOMEM;
  RunDesc d = make_desc(m, src, base, out, h, p, static_cast<char*>(ws));
  d.ax = ax;
  d.ay = ay;
  return launch_stage(d, p->riemann, static_cast<hipStream_t>(stream));
}

int rich_stage_debug(const rich_mesh* m, const rich_state* src, const rich_state* base,
                     rich_state* out, double h, const rich_params* p, void* ws,
                     size_t ws_bytes, uint8_t* cell_bits, uint8_t* edge_bits, void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !ws || !cell_bits || !edge_bits) return RICH_E_INVAL;
  const int64_t n = m->n_cells;
  if (!valid_state(src, n, false) || !valid_state(base, n, true) || !valid_state(out, n, true))
    return RICH_E_INVAL;
  if (!std::isfinite(h) || h < 0.0) return RICH_E_INVAL;
  if (out->M == src->M || out->M == base->M || out->x == base->x) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(n) || (reinterpret_cast<uintptr_t>(ws) & 255)) return RICH_E_NOMEM;
  RunDesc d = make_desc(m, src, base, out, h, p, static_cast<char*>(ws));
  return launch_stage(d, p->riemann, static_cast<hipStream_t>(stream), cell_bits, edge_bits);
}

namespace {
int stage_with_device_dt(const rich_mesh* m, const rich_state* src, const rich_state* base,
                         rich_state* out, double h_factor, const void* dt_ws, bool courant,
                         const rich_params* p, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !ws || (!courant && !dt_ws)) return RICH_E_INVAL;
  const int64_t n = m->n_cells;
  if (!valid_state(src, n, false) || !valid_state(base, n, true) || !valid_state(out, n, true))
    return RICH_E_INVAL;
  if (!std::isfinite(h_factor) || h_factor < 0.0) return RICH_E_INVAL;
  if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return RICH_E_INVAL;
  if (out->M == src->M || out->M == base->M || out->x == base->x) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(n) || (reinterpret_cast<uintptr_t>(ws) & 255)) return RICH_E_NOMEM;
  if (dt_ws && (reinterpret_cast<uintptr_t>(dt_ws) & 255)) return RICH_E_INVAL;
  char* w = static_cast<char*>(ws);
  RunDesc d = make_desc(m, src, base, out, 0.0, p, w);
  d.h_factor = h_factor;
  if (courant) {
    d.cfl_blocks = reinterpret_cast<double*>(w + run_ws(n).cfl);
    d.h_dev = reinterpret_cast<const double*>(w + kDtOffset);
  } else {
    d.h_dev = reinterpret_cast<const double*>(static_cast<const char*>(dt_ws) + kDtOffset);
  }
  return launch_stage(d, p->riemann, static_cast<hipStream_t>(stream));
}
}  // namespace

int rich_stage_courant(const rich_mesh* m, const rich_state* src, const rich_state* base,
                       rich_state* out, double h_factor, const rich_params* p, void* ws,
                       size_t ws_bytes, void* stream) {
  return stage_with_device_dt(m, src, base, out, h_factor, nullptr, true, p, ws, ws_bytes,
                              stream);
}

int rich_stage_dt_of(const rich_mesh* m, const rich_state* src, const rich_state* base,
                     rich_state* out, double h_factor, const void* dt_ws, const rich_params* p,
                     void* ws, size_t ws_bytes, void* stream) {
  return stage_with_device_dt(m, src, base, out, h_factor, dt_ws, false, p, ws, ws_bytes,
                              stream);
}

int rich_stage_dt(void* ws, void* stream, double* dt) {
  if (!ws || !dt) return RICH_E_INVAL;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RICH_E_DEVICE;
  if (hipMemcpy(dt, static_cast<char*>(ws) + kDtOffset, sizeof(double), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return RICH_E_DEVICE;
  return (std::isfinite(*dt) && *dt > 0.0) ? RICH_OK : RICH_E_DOMAIN;
}

int rich_stage_flags(void* ws, void* stream, int32_t* flags) {
  if (!ws || !flags) return RICH_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess) return RICH_E_DEVICE;
  if (hipMemcpy(flags, ws, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}

int rich_area_rate(const rich_mesh* m, const rich_state* s, const rich_params* p, double* adot,
                   void* ws, size_t ws_bytes, void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !adot || !ws) return RICH_E_INVAL;
  if (!valid_state(s, m->n_cells, false)) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(m->n_cells) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return RICH_E_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  RunDesc d = make_desc(m, s, nullptr, nullptr, 0.0, p, static_cast<char*>(ws));
  const int nb = (d.n + rich::kCflThreads - 1) / rich::kCflThreads;
  // the point velocities into the workspace, then the rates
  hipLaunchKernelGGL(rich::k_clear, dim3(1), dim3(64), 0, st, d.flag, d.cfl_min, d.ovf_count);
  hipLaunchKernelGGL(rich::k_wvel, dim3(nb), dim3(rich::kCflThreads), 0, st, d, d.rec);
  hipLaunchKernelGGL(rich::k_adot, dim3(nb), dim3(rich::kCflThreads), 0, st, d,
                     (const double*)d.rec, adot);
  return hip_status(hipGetLastError());
}

int rich_cfl_dt(const rich_mesh* m, const rich_state* s, const rich_params* p, double* dt,
                void* ws, size_t ws_bytes, void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !dt || !ws) return RICH_E_INVAL;
  if (!valid_state(s, m->n_cells, false)) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(m->n_cells) || (reinterpret_cast<uintptr_t>(ws) & 255))
    return RICH_E_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  RunDesc d = make_desc(m, s, nullptr, nullptr, 0.0, p, static_cast<char*>(ws));
  const int nb = std::min<int>((d.n + rich::kCflThreads - 1) / rich::kCflThreads,
                               rich::kCflMaxBlocks);
  double* blocks = reinterpret_cast<double*>(static_cast<char*>(ws) + run_ws(d.n).cfl);
  hipLaunchKernelGGL(rich::k_cfl, dim3(nb), dim3(rich::kCflThreads), 0, st, d, blocks);
  hipLaunchKernelGGL(rich::k_cfl_final, dim3(1), dim3(rich::kCflFinalThreads), 0, st,
                     (const double*)blocks, nb, d.cfl_min, 0.0, (double*)nullptr,
                     (int32_t*)nullptr);
  if (hipGetLastError() != hipSuccess) return RICH_E_DEVICE;
  unsigned long long bits = 0;
  if (hipStreamSynchronize(st) != hipSuccess) return RICH_E_DEVICE;
  if (hipMemcpy(&bits, d.cfl_min, sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess)
    return RICH_E_DEVICE;
  double mn;
  std::memcpy(&mn, &bits, sizeof(mn));
  *dt = p->cfl * mn;
  return (std::isfinite(*dt) && *dt > 0.0) ? RICH_OK : RICH_E_DOMAIN;
}


int rich_batch_workspace_size(int32_t n, const int64_t* n_cells, size_t* bytes) {
  if (n <= 0 || !n_cells || !bytes) return RICH_E_INVAL;
  for (int32_t r = 0; r < n; ++r)
    if (n_cells[r] <= 0 || n_cells[r] > (int64_t)rich::kCellMask) return RICH_E_INVAL;
  *bytes = batch_layout(n, n_cells).total;
  return RICH_OK;
}

int rich_stage_batch_prepare(int32_t n, const rich_mesh* const* meshes,
                             const rich_state* const* src, const rich_state* const* base,
                             rich_state* const* out, const double* h,
                             const rich_params* const* params, void* ws, size_t ws_bytes,
                             void* stream, rich_batch_plan* plan) {
  return rich_stage_batch_prepare_tile(n, meshes, src, base, out, h, params, kStageTile, ws,
                                       ws_bytes, stream, plan);
}

namespace {

// The batched stage's validation and upload; ax, ay (either both null or both
// set) hold each run's per-cell acceleration, null entries meaning none.
int batch_prepare(int32_t n, const rich_mesh* const* meshes, const rich_state* const* src,
                  const rich_state* const* base, rich_state* const* out, const double* h,
                  const rich_params* const* params, const double* const* ax,
                  const double* const* ay, int32_t tile, void* ws, size_t ws_bytes,
                  void* stream, rich_batch_plan* plan) {
  if (n <= 0 || !meshes || !src || !base || !out || !h || !params || !ws || !plan)
    return RICH_E_INVAL;
  if ((ax == nullptr) != (ay == nullptr)) return RICH_E_INVAL;
  if (ax)
    for (int32_t r = 0; r < n; ++r)
      if ((ax[r] == nullptr) != (ay[r] == nullptr)) return RICH_E_INVAL;
  if (tile != 128 && tile != 256 && tile != 512) return RICH_E_INVAL;
  std::memset(plan, 0, sizeof(*plan));
  std::vector<int64_t> nc(n);
  for (int32_t r = 0; r < n; ++r) {
    const rich_mesh* m = meshes[r];
    if (!valid_mesh(m) || !valid_params(params[r])) return RICH_E_INVAL;
    const int64_t cnt = m->n_cells;
    if (!valid_state(src[r], cnt, false) || !valid_state(base[r], cnt, true) ||
        !valid_state(out[r], cnt, true))
      return RICH_E_INVAL;
    if (!std::isfinite(h[r]) || h[r] < 0.0) return RICH_E_INVAL;
    if (out[r]->M == src[r]->M || out[r]->M == base[r]->M || out[r]->x == base[r]->x)
      return RICH_E_INVAL;
    nc[r] = cnt;
  }
  if (reinterpret_cast<uintptr_t>(ws) & 255) return RICH_E_NOMEM;
  BatchLayout L = batch_layout(n, nc.data());
  if (ws_bytes < L.total) return RICH_E_NOMEM;
  char* w = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);

  // descriptors (each run's overflow count and list are its solver group's)
  // and the tile table: the HLLC runs' tiles, then the exact-solver runs'
  std::vector<RunDesc> descs(n);
  std::vector<int32_t> g[2];
  for (int32_t r = 0; r < n; ++r) g[params[r]->riemann == 1 ? 1 : 0].push_back(r);
  std::vector<int2> tiles;
  int64_t nt[2] = {0, 0};
  for (int k = 0; k < 2; ++k)
    for (int32_t r : g[k]) {
      const int64_t t = (nc[r] + tile - 1) / tile;
      for (int64_t q = 0; q < t; ++q) tiles.push_back(make_int2(r, (int)q));
      nt[k] += t;
    }
  if (nt[0] + nt[1] > L.max_tiles || nt[0] + nt[1] > INT32_MAX / 2) return RICH_E_INVAL;
  for (int32_t r = 0; r < n; ++r) {
    RunDesc d = make_desc(meshes[r], src[r], base[r], out[r], h[r], params[r], w);
    const int k = params[r]->riemann == 1 ? 1 : 0;
    d.flag = reinterpret_cast<int32_t*>(w + L.flags) + r;
    d.cfl_min = reinterpret_cast<unsigned long long*>(w + L.cfl) + r;
    d.ovf_count = reinterpret_cast<int32_t*>(w + L.ovfc) + k;
    d.ovf_list = reinterpret_cast<int2*>(w + L.ovf[k]);
    d.rec = nullptr;
    if (ax) {
      d.ax = ax[r];
      d.ay = ay[r];
    }
    descs[r] = d;
  }
  const size_t db = (size_t)n * sizeof(RunDesc), tb = tiles.size() * sizeof(int2);
  const int up = upload_staged(w + L.desc, descs.data(), db, w + L.tiles, tiles.data(), tb, st);
  if (up) return up;

  const int ti = tile == 128 ? 0 : (tile == 256 ? 1 : 2);
  static const int grids[3][2] = {
      {resident_blocks(reinterpret_cast<const void*>(&rich::k_stage<128, 0, true>), rich::TileCfg<128>::kThreads),
       resident_blocks(reinterpret_cast<const void*>(&rich::k_stage<128, 1, true>), rich::TileCfg<128>::kThreads)},
      {resident_blocks(reinterpret_cast<const void*>(&rich::k_stage<256, 0, true>), rich::TileCfg<256>::kThreads),
       resident_blocks(reinterpret_cast<const void*>(&rich::k_stage<256, 1, true>), rich::TileCfg<256>::kThreads)},
      {resident_blocks(reinterpret_cast<const void*>(&rich::k_stage<512, 0, true>), rich::TileCfg<512>::kThreads),
       resident_blocks(reinterpret_cast<const void*>(&rich::k_stage<512, 1, true>), rich::TileCfg<512>::kThreads)}};
  plan->n_runs = n;
  plan->tile = tile;
  for (int k = 0; k < 2; ++k) {
    plan->n_tiles[k] = (int32_t)nt[k];
    plan->n_group[k] = (int32_t)g[k].size();
    plan->grid[k] = (int32_t)std::min<int64_t>(nt[k], grids[ti][k]);
    plan->ovf_off[k] = (int64_t)L.ovf[k];
  }
  plan->tiles_off[0] = (int64_t)L.tiles;
  plan->tiles_off[1] = (int64_t)(L.tiles + sizeof(int2) * (size_t)nt[0]);
  plan->ovfc_off = (int64_t)L.ovfc;
  return RICH_OK;
}

}  // namespace

int rich_stage_batch_prepare_tile(int32_t n, const rich_mesh* const* meshes,
                                  const rich_state* const* src, const rich_state* const* base,
                                  rich_state* const* out, const double* h,
                                  const rich_params* const* params, int32_t tile, void* ws,
                                  size_t ws_bytes, void* stream, rich_batch_plan* plan) {
  return batch_prepare(n, meshes, src, base, out, h, params, nullptr, nullptr, tile, ws,
                       ws_bytes, stream, plan);
}

extern "C++" {
namespace {
template <int T>
void launch_stage_batch(int k, int grid, int n_tiles, hipStream_t st, const RunDesc& dummy,
                        const RunDesc* dd, const int2* tiles, const int* oc, const int2* ol) {
  const int og = std::min(n_tiles, kOverflowGrid);
  uint8_t* nb = nullptr;
  if (k == 0) {
    hipLaunchKernelGGL((rich::k_stage<T, 0, true>), dim3(grid), dim3(rich::TileCfg<T>::kThreads), 0, st, dummy, dd, tiles,
                       n_tiles, nb, nb);
    hipLaunchKernelGGL((rich::k_stage_overflow<T, 0, true>), dim3(og), dim3(T), 0, st, dummy, dd,
                       oc, ol, nb, nb);
  } else {
    hipLaunchKernelGGL((rich::k_stage<T, 1, true>), dim3(grid), dim3(rich::TileCfg<T>::kThreads), 0, st, dummy, dd, tiles,
                       n_tiles, nb, nb);
    hipLaunchKernelGGL((rich::k_stage_overflow<T, 1, true>), dim3(og), dim3(T), 0, st, dummy, dd,
                       oc, ol, nb, nb);
  }
}
}  // namespace
}  // extern "C++"

int rich_stage_batch_launch(const rich_batch_plan* plan, void* ws, void* stream) {
  if (!plan || !ws || plan->n_runs <= 0 || plan->n_tiles[0] + plan->n_tiles[1] <= 0)
    return RICH_E_INVAL;
  if (plan->tile != 128 && plan->tile != 256 && plan->tile != 512) return RICH_E_INVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return RICH_E_NOMEM;
  const int32_t n = plan->n_runs;
  const BatchLayout L = batch_layout(n, nullptr);   // the fixed part's offsets
  char* w = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const RunDesc* dd = reinterpret_cast<const RunDesc*>(w + L.desc);
  int32_t* ovfc = reinterpret_cast<int32_t*>(w + plan->ovfc_off);
  RunDesc dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  hipLaunchKernelGGL(rich::k_clear_batch, dim3((n + 255) / 256), dim3(256), 0, st, dd, n, ovfc);
  int pf = prof_begin("k_stage", st);
  for (int k = 0; k < 2; ++k) {
    if (plan->n_tiles[k] <= 0 || plan->grid[k] <= 0) continue;
    const int2* tiles = reinterpret_cast<const int2*>(w + plan->tiles_off[k]);
    const int2* ol = reinterpret_cast<const int2*>(w + plan->ovf_off[k]);
    const int* oc = ovfc + k;
    switch (plan->tile) {
      case 128: launch_stage_batch<128>(k, plan->grid[k], plan->n_tiles[k], st, dummy, dd, tiles, oc, ol); break;
      case 256: launch_stage_batch<256>(k, plan->grid[k], plan->n_tiles[k], st, dummy, dd, tiles, oc, ol); break;
      default: launch_stage_batch<512>(k, plan->grid[k], plan->n_tiles[k], st, dummy, dd, tiles, oc, ol); break;
    }
  }
  prof_end(pf, st);
  return hip_status(hipGetLastError());
}

int rich_stage_batch_autotune(int32_t n, const rich_mesh* const* meshes,
                              const rich_state* const* src, const rich_state* const* base,
                              rich_state* const* out, const double* h,
                              const rich_params* const* params, int32_t reps, void* ws,
                              size_t ws_bytes, void* stream, int32_t* best_tile, double* ms) {
  if (!best_tile || !ms || reps <= 0) return RICH_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  static const int32_t tiles[3] = {128, 256, 512};
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return RICH_E_DEVICE;
  }
  int rc = RICH_OK;
  double best = 0.0;
  *best_tile = 0;
  for (int k = 0; k < 3 && rc == RICH_OK; ++k) {
    rich_batch_plan plan;
    rc = rich_stage_batch_prepare_tile(n, meshes, src, base, out, h, params, tiles[k], ws,
                                       ws_bytes, stream, &plan);
    if (rc) break;
    if ((rc = rich_stage_batch_launch(&plan, ws, stream))) break;   // warm-up
    if (hipEventRecord(a, st) != hipSuccess) { rc = RICH_E_DEVICE; break; }
    for (int r = 0; r < reps && rc == RICH_OK; ++r) rc = rich_stage_batch_launch(&plan, ws, stream);
    if (rc) break;
    float t = 0.0f;
    if (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&t, a, b) != hipSuccess) {
      rc = RICH_E_DEVICE;
      break;
    }
    ms[k] = (double)t / reps;
    if (*best_tile == 0 || ms[k] < best) {
      best = ms[k];
      *best_tile = tiles[k];
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return rc;
}

int rich_stage_batch(int32_t n, const rich_mesh* const* meshes, const rich_state* const* src,
                     const rich_state* const* base, rich_state* const* out, const double* h,
                     const rich_params* const* params, void* ws, size_t ws_bytes,
                     void* stream) {
  rich_batch_plan plan;
  const int rc = rich_stage_batch_prepare(n, meshes, src, base, out, h, params, ws, ws_bytes,
                                          stream, &plan);
  if (rc) return rc;
  return rich_stage_batch_launch(&plan, ws, stream);
}

int rich_stage_batch_accel(int32_t n, const rich_mesh* const* meshes,
                           const rich_state* const* src, const rich_state* const* base,
                           rich_state* const* out, const double* h,
                           const rich_params* const* params, const double* const* ax,
                           const double* const* ay, void* ws, size_t ws_bytes, void* stream) {
  if (!ax || !ay) return RICH_E_INVAL;
  rich_batch_plan plan;
  const int rc = batch_prepare(n, meshes, src, base, out, h, params, ax, ay, kStageTile, ws,
                               ws_bytes, stream, &plan);
  if (rc) return rc;
  return rich_stage_batch_launch(&plan, ws, stream);
}

int rich_batch_flags(int32_t n, void* ws, void* stream, int32_t* flags) {
  if (n <= 0 || !ws || !flags) return RICH_E_INVAL;
  std::vector<int64_t> one(n, 1);
  BatchLayout L = batch_layout(n, one.data());
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RICH_E_DEVICE;
  if (hipMemcpy(flags, static_cast<char*>(ws) + L.flags, (size_t)n * sizeof(int32_t),
                hipMemcpyDeviceToHost) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}


int rich_batch_flags_async(int32_t n, void* ws, void* stream, int32_t* host_flags) {
  if (n <= 0 || !ws || !host_flags) return RICH_E_INVAL;
  std::vector<int64_t> one(n, 1);
  BatchLayout L = batch_layout(n, one.data());
  if (hipMemcpyAsync(host_flags, static_cast<char*>(ws) + L.flags, (size_t)n * sizeof(int32_t),
                     hipMemcpyDeviceToHost, static_cast<hipStream_t>(stream)) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}

int rich_mesh_pack(const rich_host_mesh_view* hm, rich_cell* cells, rich_edge* edges) {
  if (!hm || hm->n_cells <= 0 || hm->n_edges < 0 || !cells || (hm->n_edges > 0 && !edges))
    return RICH_E_INVAL;
  if (!hm->px || !hm->py || !hm->sx || !hm->sy || !hm->area) return RICH_E_INVAL;
  if (hm->n_edges > 0 &&
      (!hm->e_i || !hm->e_j || !hm->e_len || !hm->e_fx || !hm->e_fy))
    return RICH_E_INVAL;
  for (int64_t c = 0; c < hm->n_cells; ++c) {
    rich_cell& r = cells[c];
    r.px = hm->px[c];
    r.py = hm->py[c];
    r.area = hm->area[c];
    r.sx = hm->sx[c];
    r.sy = hm->sy[c];
    r.pad = 0.0;
  }
  for (int64_t e = 0; e < hm->n_edges; ++e) {
    rich_edge& r = edges[e];
    r.fx = hm->e_fx[e];
    r.fy = hm->e_fy[e];
    r.len = hm->e_len[e];
    r.i = hm->e_i[e];
    r.j = hm->e_j[e];
  }
  return RICH_OK;
}

int rich_ctx_create(rich_ctx** ctx) {
  if (!ctx) return RICH_E_INVAL;
  try {
    *ctx = new rich_ctx;
  } catch (...) {
    return RICH_E_NOMEM;
  }
  return RICH_OK;
}

void rich_ctx_destroy(rich_ctx* ctx) {
  if (!ctx) return;
  ctx->cur.release();
  ctx->spare.release();
  ctx->third.release();
  ctx->rws.release();
  ctx->bws.release();
  ctx->Qh.release(); ctx->Xh.release(); ctx->Qn.release(); ctx->Xn.release();
  ctx->ws.release();
  if (ctx->hostX) (void)hipHostFree(ctx->hostX);
  delete ctx;
}

int rich_ctx_set_mesh(rich_ctx* ctx, const rich_host_mesh_view* hm, const double box[4],
                      uint32_t bc, void* stream) {
  if (!ctx || !hm || !box || hm->n_cells <= 0 || hm->n_cells > (int64_t)rich::kCellMask ||
      hm->n_edges < 0 || hm->n_csr < 0)
    return RICH_E_INVAL;
  return ctx->cur.upload(hm, box, bc, static_cast<hipStream_t>(stream));
}

int rich_ctx_mesh(rich_ctx* ctx, rich_mesh* out) {
  if (!ctx || !out || !ctx->cur.set) return RICH_E_INVAL;
  ctx->cur.view(out);
  return RICH_OK;
}

namespace {
// The mesh of state s's points into dst: on the device from `prev` when the
// context asks for it, with the host stage when that is off or the device
// result is not certified.
int mesh_of(rich_ctx* ctx, const rich_mesh& prev, const rich_state& s, DevMesh& dst,
            rich_tess_fn tess, rich_tess_release_fn release, void* tess_user, hipStream_t st) {
  if (ctx->device_tess) {
    // RICH_E_INVAL: a run the device rebuild does not take (a periodic box
    // of under 16 cells); RICH_E_MESH: a mesh it did not certify
    const int rc = retess_into(ctx, prev, s.x, s.y, dst, st);
    if (rc == RICH_OK) {
      ++ctx->n_device;
      return RICH_OK;
    }
    if (rc != RICH_E_MESH && rc != RICH_E_INVAL) return rc;
    ++ctx->n_fallback;
  }
  return tessellate_into(ctx, dst, s.x, prev.n_cells, ctx->cur.box, ctx->cur.bc, tess, release,
                         tess_user, st);
}
}  // namespace

int rich_ctx_set_device_tess(rich_ctx* ctx, int32_t on) {
  if (!ctx || (on != 0 && on != 1)) return RICH_E_INVAL;
  ctx->device_tess = on == 1;
  return RICH_OK;
}

int rich_ctx_tess_counts(rich_ctx* ctx, int64_t* device, int64_t* host_fallback) {
  if (!ctx || !device || !host_fallback) return RICH_E_INVAL;
  *device = ctx->n_device;
  *host_fallback = ctx->n_fallback;
  return RICH_OK;
}

namespace {
// One stage of a step, with the per-cell acceleration when given.
int step_stage(const rich_mesh* m, const rich_state* src, const rich_state* base,
               rich_state* out, double h, const rich_params* p, const double* ax,
               const double* ay, void* ws, size_t ws_bytes, void* stream) {
  return ax ? rich_stage_accel(m, src, base, out, h, p, ax, ay, ws, ws_bytes, stream)
            : rich_stage(m, src, base, out, h, p, ws, ws_bytes, stream);
}

int step_impl(rich_ctx* ctx, rich_state* state, double dt, const rich_params* p,
              const double* ax, const double* ay, rich_tess_fn tess,
              rich_tess_release_fn release, void* tess_user, void* stream) {
  if (!ctx || !state || !valid_params(p) || !ctx->cur.set) return RICH_E_INVAL;
  if (!std::isfinite(dt) || !(dt > 0.0)) return RICH_E_INVAL;
  if (p->motion && (!tess || !release)) return RICH_E_INVAL;
  const int64_t n = ctx->cur.n;
  if (!valid_state(state, n, true)) return RICH_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  size_t wsb = run_ws_bytes(n);
  if (!ctx->Qh.ensure(32 * (size_t)n) || !ctx->Xh.ensure(16 * (size_t)n) ||
      !ctx->Qn.ensure(32 * (size_t)n) || !ctx->Xn.ensure(16 * (size_t)n) ||
      !ctx->ws.ensure(wsb))
    return RICH_E_NOMEM;
  rich_state half = state_view(ctx->Qh, ctx->Xh, n);
  rich_state next = state_view(ctx->Qn, ctx->Xn, n);
  rich_mesh m;
  ctx->cur.view(&m);
  rich_mesh mh = m;
  int rc;
  int32_t flags = 0;
  if (p->integrator == 1) {
    // extrapolated fluxes: one stage on the start-of-step mesh
    rc = step_stage(&m, state, state, &next, dt, p, ax, ay, ctx->ws.p, ctx->ws.cap, stream);
    if (rc) return rc;
  } else {
    rc = step_stage(&m, state, state, &half, 0.5 * dt, p, ax, ay, ctx->ws.p, ctx->ws.cap,
                    stream);
    if (rc) return rc;
    if ((rc = rich_stage_flags(ctx->ws.p, stream, &flags))) return rc;
    if (flags) return RICH_E_DOMAIN;
    if (p->motion) {
      rc = mesh_of(ctx, m, half, ctx->spare, tess, release, tess_user, st);
      if (rc) return rc;
      ctx->spare.view(&mh);
    }
    rc = step_stage(&mh, &half, state, &next, dt, p, ax, ay, ctx->ws.p, ctx->ws.cap, stream);
    if (rc) return rc;
  }
  if ((rc = rich_stage_flags(ctx->ws.p, stream, &flags))) return rc;
  if (flags) return RICH_E_DOMAIN;
  if (p->motion) {
    // the new mesh goes into the third buffers (the device rebuild reads the
    // half-step mesh from the spare ones), which then become current
    rc = mesh_of(ctx, p->integrator == 1 ? m : mh, next, ctx->third, tess, release, tess_user,
                 st);
    if (rc) return rc;
    std::swap(ctx->cur, ctx->third);
  }
  // commit
  const double* sq[6] = {next.M, next.Px, next.Py, next.E, next.x, next.y};
  double* dq[6] = {state->M, state->Px, state->Py, state->E, state->x, state->y};
  for (int k = 0; k < 6; ++k)
    if (hipMemcpyAsync(dq[k], sq[k], 8 * (size_t)n, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return RICH_E_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return RICH_E_DEVICE;
  return RICH_OK;
}
}  // namespace

int rich_step(rich_ctx* ctx, rich_state* state, double dt, const rich_params* p,
              rich_tess_fn tess, rich_tess_release_fn release, void* tess_user, void* stream) {
  return step_impl(ctx, state, dt, p, nullptr, nullptr, tess, release, tess_user, stream);
}

int rich_step_accel(rich_ctx* ctx, rich_state* state, double dt, const rich_params* p,
                    const double* ax, const double* ay, rich_tess_fn tess,
                    rich_tess_release_fn release, void* tess_user, void* stream) {
  if (!ax || !ay) return RICH_E_INVAL;
  return step_impl(ctx, state, dt, p, ax, ay, tess, release, tess_user, stream);
}

namespace {

// The batched step; ax, ay (both null, or host arrays of n device pointers)
// hold each run's per-cell acceleration, null entries meaning none.
int step_batch_impl(int32_t n, rich_ctx* const* ctxs, rich_state* const* states,
                    const double* dt, const rich_params* const* params,
                    const double* const* ax, const double* const* ay, rich_tess_fn tess,
                    rich_tess_release_fn release, void* const* tess_users, int32_t n_threads,
                    int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (n <= 0 || !ctxs || !states || !dt || !params || !status || !ws) return RICH_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<int64_t> nc(n, 1);
  bool any_motion = false;
  for (int32_t r = 0; r < n; ++r) {
    status[r] = RICH_OK;
    rich_ctx* c = ctxs[r];
    if (!c || !c->cur.set || !valid_params(params[r]) || !std::isfinite(dt[r]) ||
        !(dt[r] > 0.0) || !valid_state(states[r], c->cur.n, true) ||
        (ax && (ax[r] == nullptr) != (ay[r] == nullptr))) {
      status[r] = RICH_E_INVAL;
      continue;
    }
    if (params[r]->motion) {
      if (!tess || !release || !tess_users) {
        status[r] = RICH_E_INVAL;
        continue;
      }
      any_motion = true;
    }
    nc[r] = c->cur.n;
    const size_t cn = (size_t)nc[r];
    if (!c->Qh.ensure(32 * cn) || !c->Xh.ensure(16 * cn) || !c->Qn.ensure(32 * cn) ||
        !c->Xn.ensure(16 * cn))
      status[r] = RICH_E_NOMEM;
  }
  // a failure of the call as a whole: no run still pending is committed
  auto fail_all = [&](int e) {
    for (int32_t r = 0; r < n; ++r)
      if (!status[r]) status[r] = e;
    return e;
  };
  size_t need = 0;
  int rc = rich_batch_workspace_size(n, nc.data(), &need);
  if (rc) return fail_all(rc);
  if (ws_bytes < need) return fail_all(RICH_E_NOMEM);

  std::vector<rich_state> half(n), next(n);
  std::vector<rich_mesh> mesh(n);
  for (int32_t r = 0; r < n; ++r) {
    if (status[r]) continue;
    half[r] = state_view(ctxs[r]->Qh, ctxs[r]->Xh, nc[r]);
    next[r] = state_view(ctxs[r]->Qn, ctxs[r]->Xn, nc[r]);
    ctxs[r]->cur.view(&mesh[r]);
  }

  // One batched stage over the runs still alive; flagged runs drop out.
  auto stage = [&](bool second) -> int {
    std::vector<int32_t> live;
    for (int32_t r = 0; r < n; ++r)
      if (!status[r] && !(second && params[r]->integrator == 1)) live.push_back(r);
    if (live.empty()) return RICH_OK;
    const size_t m = live.size();
    std::vector<const rich_mesh*> mp(m);
    std::vector<const rich_state*> sp(m), bp(m);
    std::vector<rich_state*> op(m);
    std::vector<double> h(m);
    std::vector<const rich_params*> pp(m);
    std::vector<const double*> axk(m, nullptr), ayk(m, nullptr);
    for (size_t k = 0; k < m; ++k) {
      const int32_t r = live[k];
      const bool one = params[r]->integrator == 1;  // extrapolated fluxes: one stage
      if (ax) {
        axk[k] = ax[r];
        ayk[k] = ay[r];
      }
      mp[k] = &mesh[r];
      sp[k] = second ? &half[r] : states[r];
      bp[k] = states[r];
      op[k] = (second || one) ? &next[r] : &half[r];
      h[k] = (second || one) ? dt[r] : 0.5 * dt[r];
      pp[k] = params[r];
    }
    rich_batch_plan plan;
    int e = batch_prepare((int32_t)m, mp.data(), sp.data(), bp.data(), op.data(), h.data(),
                          pp.data(), ax ? axk.data() : nullptr, ax ? ayk.data() : nullptr,
                          kStageTile, ws, ws_bytes, stream, &plan);
    if (!e) e = rich_stage_batch_launch(&plan, ws, stream);
    if (e) return e;
    std::vector<int32_t> fl(m, 0);
    if ((e = rich_batch_flags((int32_t)m, ws, stream, fl.data()))) return e;
    for (size_t k = 0; k < m; ++k)
      if (fl[k]) status[live[k]] = RICH_E_DOMAIN;
    return RICH_OK;
  };

  // Host tessellation of the points xs[r] of every live moving run into its
  // spare mesh: device->host copies, then the runs spread over n_threads
  // host threads (each call with its own run's tess_users[r]), then the
  // uploads, one synchronisation, and the host arrays released.
  // Runs whose context asks for it are rebuilt on the device first (all
  // enqueued, then one synchronisation); a mesh the device does not certify
  // joins the host tessellations.
  std::vector<rich_host_mesh_view> hv(n);
  auto retessellate = [&](const std::vector<rich_state>& xs, bool half_step) -> int {
    std::vector<int32_t> todo, dev;
    for (int32_t r = 0; r < n; ++r)
      if (!status[r] && params[r]->motion && !(half_step && params[r]->integrator == 1))
        (ctxs[r]->device_tess ? dev : todo).push_back(r);
    auto dst_of = [&](int32_t r) -> DevMesh& {
      return half_step ? ctxs[r]->spare : ctxs[r]->third;
    };
    if (!dev.empty()) {
      // one batched rebuild of every device run; runs whose arguments the
      // device path does not take (a periodic box of under 16 cells) and
      // uncertified meshes go to the host stage
      const size_t m = dev.size();
      std::vector<rich_mesh_bufs> ob(m);
      std::vector<const rich_mesh*> pp(m);
      std::vector<const rich_mesh_bufs*> op(m);
      std::vector<const double*> xp(m), yp(m);
      std::vector<void*> wp(m);
      std::vector<size_t> wb(m);
      for (size_t k = 0; k < m; ++k) {
        const int32_t r = dev[k];
        const int e = retess_prepare(ctxs[r], nc[r], dst_of(r), st, ob[k]);
        if (e) return e;
        pp[k] = &mesh[r];
        op[k] = &ob[k];
        xp[k] = xs[r].x;
        yp[k] = xs[r].y;
        wp[k] = ctxs[r]->rws.p;
        wb[k] = ctxs[r]->rws.cap;
      }
      size_t bb = 0;
      rich_ctx* owner = ctxs[dev[0]];   // holds the batch descriptors for this call
      int e = rich_retess_batch_workspace_size((int32_t)m, &bb);
      if (e) return e;
      if (!owner->bws.ensure(bb)) return RICH_E_NOMEM;
      e = rich_retess_batch((int32_t)m, pp.data(), xp.data(), yp.data(), op.data(), wp.data(),
                            wb.data(), owner->bws.p, owner->bws.cap, st);
      std::vector<rich_retess_info> info(m);
      std::vector<int32_t> rs(m, RICH_E_MESH);
      if (e == RICH_OK) {
        if ((e = rich_retess_batch_result((int32_t)m, owner->bws.p, st, info.data(), rs.data())))
          return e;
      } else if (e != RICH_E_INVAL) {
        return e;
      }
      for (size_t k = 0; k < m; ++k) {
        const int32_t r = dev[k];
        if (rs[k] == RICH_OK) {
          retess_adopt(mesh[r], info[k], dst_of(r));
          ++ctxs[r]->n_device;
        } else {
          ++ctxs[r]->n_fallback;
          todo.push_back(r);
        }
      }
    }
    if (todo.empty()) return RICH_OK;
    for (int32_t r : todo) {
      rich_ctx* c = ctxs[r];
      const size_t bytes = 2 * (size_t)nc[r] * sizeof(double);
      if (c->hostX_cap < bytes) {
        if (c->hostX) (void)hipHostFree(c->hostX);
        c->hostX = nullptr;
        c->hostX_cap = 0;
        if (hipHostMalloc(&c->hostX, bytes, 0) != hipSuccess) {
          status[r] = RICH_E_NOMEM;
          continue;
        }
        c->hostX_cap = bytes;
      }
      if (hipMemcpyAsync(c->hostX, xs[r].x, bytes, hipMemcpyDeviceToHost, st) != hipSuccess)
        return RICH_E_DEVICE;
    }
    if (hipStreamSynchronize(st) != hipSuccess) return RICH_E_DEVICE;
    std::atomic<size_t> next_job{0};
    auto worker = [&]() {
      for (;;) {
        const size_t k = next_job.fetch_add(1);
        if (k >= todo.size()) return;
        const int32_t r = todo[k];
        if (status[r]) continue;
        const double* hx = static_cast<const double*>(ctxs[r]->hostX);
        std::memset(&hv[r], 0, sizeof(hv[r]));
        const int t = tess(tess_users[r], hx, hx + nc[r], nc[r], ctxs[r]->cur.box,
                           ctxs[r]->cur.bc, &hv[r]);
        if (t != 0) {
          status[r] = RICH_E_MESH;
        } else if (hv[r].n_cells != nc[r]) {
          release(tess_users[r], &hv[r]);
          status[r] = RICH_E_MESH;
        }
      }
    };
    const int nt = std::max(1, std::min<int>(n_threads > 0 ? n_threads : 1, (int)todo.size()));
    std::vector<std::thread> pool;
    try {
      for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    } catch (...) {
      // fewer threads: the calling thread still drains the queue
    }
    worker();
    for (auto& t : pool) t.join();
    int err = RICH_OK;
    std::vector<int32_t> uploaded;
    for (int32_t r : todo) {
      if (status[r]) continue;
      const int u = dst_of(r).upload_async(&hv[r], ctxs[r]->cur.box, ctxs[r]->cur.bc, st);
      if (u) {
        status[r] = u;
        if (u == RICH_E_DEVICE) err = u;
      }
      uploaded.push_back(r);   // released after the synchronisation below
    }
    const bool synced = hipStreamSynchronize(st) == hipSuccess;
    for (int32_t r : uploaded) release(tess_users[r], &hv[r]);
    if (!synced) return RICH_E_DEVICE;
    return err;
  };

  if ((rc = stage(false))) return fail_all(rc);
  bool any_two = false;   // runs with a second stage (time-centred fluxes)
  for (int32_t r = 0; r < n; ++r)
    if (!status[r] && params[r]->integrator == 0) any_two = true;
  if (any_motion && any_two) {
    if ((rc = retessellate(half, true))) return fail_all(rc);
    for (int32_t r = 0; r < n; ++r)
      if (!status[r] && params[r]->motion && params[r]->integrator == 0)
        ctxs[r]->spare.view(&mesh[r]);
  }
  if ((rc = stage(true))) return fail_all(rc);
  // the final meshes go into the third buffers (a device rebuild reads the
  // half-step mesh from the spare ones); a run's current mesh is replaced
  // only once its whole step has succeeded
  if (any_motion && (rc = retessellate(next, false))) return fail_all(rc);
  for (int32_t r = 0; r < n; ++r) {
    if (status[r]) continue;
    const size_t b = 8 * (size_t)nc[r];
    const double* sq[6] = {next[r].M, next[r].Px, next[r].Py, next[r].E, next[r].x, next[r].y};
    double* dq[6] = {states[r]->M, states[r]->Px, states[r]->Py, states[r]->E, states[r]->x,
                     states[r]->y};
    for (int k = 0; k < 6; ++k)
      if (hipMemcpyAsync(dq[k], sq[k], b, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail_all(RICH_E_DEVICE);
  }
  if (hipStreamSynchronize(st) != hipSuccess) return fail_all(RICH_E_DEVICE);
  for (int32_t r = 0; r < n; ++r)
    if (!status[r] && params[r]->motion) std::swap(ctxs[r]->cur, ctxs[r]->third);
  for (int32_t r = 0; r < n; ++r)
    if (status[r]) return status[r];
  return RICH_OK;
}

}  // namespace

int rich_step_batch(int32_t n, rich_ctx* const* ctxs, rich_state* const* states,
                    const double* dt, const rich_params* const* params, rich_tess_fn tess,
                    rich_tess_release_fn release, void* const* tess_users, int32_t n_threads,
                    int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  return step_batch_impl(n, ctxs, states, dt, params, nullptr, nullptr, tess, release,
                         tess_users, n_threads, status, ws, ws_bytes, stream);
}

int rich_step_batch_accel(int32_t n, rich_ctx* const* ctxs, rich_state* const* states,
                          const double* dt, const rich_params* const* params,
                          const double* const* ax, const double* const* ay, rich_tess_fn tess,
                          rich_tess_release_fn release, void* const* tess_users,
                          int32_t n_threads, int32_t* status, void* ws, size_t ws_bytes,
                          void* stream) {
  if (!ax || !ay) return RICH_E_INVAL;
  return step_batch_impl(n, ctxs, states, dt, params, ax, ay, tess, release, tess_users,
                         n_threads, status, ws, ws_bytes, stream);
}

int rich_profile_enable(int on) {
  profiler().on = on != 0;
  return RICH_OK;
}

int rich_profile_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return RICH_E_INVAL;
  Profiler& P = profiler();
  double sum = 0.0;
  int64_t cnt = 0;
  std::vector<ProfEntry> keep;
  for (auto& e : P.pending) {
    if (e.name != kernel) {
      keep.push_back(e);
      continue;
    }
    if (hipEventSynchronize(e.b) != hipSuccess) return RICH_E_DEVICE;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return RICH_E_DEVICE;
    sum += ms;
    ++cnt;
    P.pool.push_back(e.a);
    P.pool.push_back(e.b);
  }
  P.pending.swap(keep);
  *total_ms = sum;
  *launches = cnt;
  return RICH_OK;
}

const char* rich_strerror(int status) {
  switch (status) {
    case RICH_OK: return "ok";
    case RICH_E_INVAL: return "invalid argument";
    case RICH_E_NOMEM: return "workspace too small or allocation failed";
    case RICH_E_DEVICE: return "HIP runtime error";
    case RICH_E_DOMAIN: return "unphysical state produced (mass, internal energy or non-finite)";
    case RICH_E_MESH: return "invalid mesh or tessellation failure";
    default: return "unknown status";
  }
}

}  // extern "C"
