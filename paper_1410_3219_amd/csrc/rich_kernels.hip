// Kernels and C-ABI of one stage of RICH's moving-mesh Godunov scheme on
// gfx950 (MI355X).  See rich.h for the interface and rich_device.hpp for the
// per-cell and per-edge arithmetic.
//
// One stage is two kernels over tiles of kTile consecutive cells (cells come
// in Hilbert order, so a tile is a compact patch of the mesh):
//   k_cell  one thread per cell: primitives, point velocity, gradient and
//           limiter (A1-A4); writes a 128-byte record per cell.
//   k_flux  one block per tile: the fluxes of the edges the tile owns (edges
//           are sorted by their first cell) are computed once each and kept
//           in LDS; then every cell sums the fluxes of its edges in CSR order
//           (fluxes of edges owned by another tile are recomputed, bitwise
//           identical), and writes the updated state and point (A5-A8).
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
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "rich.h"
#include "rich_device.hpp"

namespace rich {

constexpr int kTile = 256;      // cells per tile = threads per block
constexpr int kEdgeCap = 1024;  // owned-edge fluxes kept in LDS per tile
constexpr int kNumXcd = 8;
constexpr size_t kHeader = 256;  // per-run workspace header

// block -> tile, so that XCD x (blocks x, x+8, ...) gets one contiguous range
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / kNumXcd, rem = nb % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return x * q + min(x, rem) + k;
}

// run owning global tile t (tile_start is an exclusive prefix, n_runs + 1)
__device__ __forceinline__ int find_run(const int32_t* __restrict__ tile_start, int n_runs,
                                        int t) {
  int lo = 0, hi = n_runs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (tile_start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// workspace header: flag word and Courant minimum
// ---------------------------------------------------------------------------
__global__ void k_clear(int32_t* flag, unsigned long long* cfl_min) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *flag = 0;
    *cfl_min = 0x7FF0000000000000ull;  // +inf
  }
}

__global__ void k_clear_batch(const RunDesc* __restrict__ descs, int n_runs) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_runs) {
    *descs[r].flag = 0;
    *descs[r].cfl_min = 0x7FF0000000000000ull;
  }
}

// ---------------------------------------------------------------------------
// A1-A4: one thread per cell
// ---------------------------------------------------------------------------
template <bool BATCH>
__global__ __launch_bounds__(kTile) void k_cell(RunDesc one, const RunDesc* __restrict__ descs,
                                                const int32_t* __restrict__ tile_start,
                                                int n_runs, int n_tiles) {
  for (int b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    const int t = BATCH ? b : xcd_tile(b, n_tiles);
    const int r = BATCH ? find_run(tile_start, n_runs, t) : 0;
    const RunDesc& d = BATCH ? descs[r] : one;
    const int c0 = (t - (BATCH ? tile_start[r] : 0)) * kTile;
    const int i = c0 + (int)threadIdx.x;
    if (i < d.n) {
      double rec[kRecDoubles];
      if (!cell_record(d, i, rec)) atomicOr(d.flag, RICH_FLAG_DOMAIN);
      double2* dst = reinterpret_cast<double2*>(d.rec + (size_t)i * kRecDoubles);
#pragma unroll
      for (int k = 0; k < kRecDoubles / 2; ++k) dst[k] = make_double2(rec[2 * k], rec[2 * k + 1]);
    }
  }
}

// ---------------------------------------------------------------------------
// A5-A8: one block per tile
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wrap_once(double v, double lo, double hi) {
  const double L = hi - lo;
  if (v < lo) v += L;
  if (v >= hi) v -= L;
  return v;
}

template <int RIEMANN>
__device__ __forceinline__ bool flux_of_edge(const RunDesc& d, int e, double* LF) {
  double ri[kRecDoubles], rj[kRecDoubles];
  if (e < 0 || e >= d.n_edges) {
    LF[0] = LF[1] = LF[2] = LF[3] = 0.0;
    return false;
  }
  const int i = d.e_i[e];
  const uint32_t ej = (uint32_t)d.e_j[e];
  if (i < 0 || i >= d.n) {
    LF[0] = LF[1] = LF[2] = LF[3] = 0.0;
    return false;
  }
  load_rec(d.rec, i, ri);
  if ((ej >> 28) < 9) {
    int j = (int)(ej & kCellMask);
    if (j >= d.n) j = i;
    load_rec(d.rec, j, rj);
  }
  return edge_flux<RIEMANN>(d, e, ri, rj, LF);
}

template <int RIEMANN, bool BATCH>
__global__ __launch_bounds__(kTile) void k_flux(RunDesc one, const RunDesc* __restrict__ descs,
                                                const int32_t* __restrict__ tile_start,
                                                int n_runs, int n_tiles) {
  __shared__ double sF[4][kEdgeCap];
  for (int b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    const int t = BATCH ? b : xcd_tile(b, n_tiles);
    const int r = BATCH ? find_run(tile_start, n_runs, t) : 0;
    const RunDesc& d = BATCH ? descs[r] : one;
    const int c0 = (t - (BATCH ? tile_start[r] : 0)) * kTile;
    const int c1 = min(c0 + kTile, d.n);
    const int e0 = d.eoff[c0];
    const int ne = min(d.eoff[c1] - e0, kEdgeCap);
    bool ok = true;
    for (int k = (int)threadIdx.x; k < ne; k += kTile) {
      double LF[4];
      if (!flux_of_edge<RIEMANN>(d, e0 + k, LF)) ok = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) sF[q][k] = LF[q];
    }
    __syncthreads();
    const int i = c0 + (int)threadIdx.x;
    if (i < c1) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int k0 = d.off[i], k1 = d.off[i + 1];
      if (k0 < 0 || k1 < k0 || k1 > d.n_csr) {
        ok = false;
        k1 = k0;
      }
      for (int k = k0; k < k1; ++k) {
        const int entry = d.idx[k];
        const int e = entry >> 1;
        double LF[4];
        if (e >= e0 && e < e0 + ne) {
#pragma unroll
          for (int q = 0; q < 4; ++q) LF[q] = sF[q][e - e0];
        } else if (e >= 0 && e < d.n_edges) {
          if (!flux_of_edge<RIEMANN>(d, e, LF)) ok = false;
        } else {
          ok = false;
          LF[0] = LF[1] = LF[2] = LF[3] = 0.0;
        }
        if (entry & 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] -= LF[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += LF[q];
        }
      }
      const double h = d.h;
      const double M = d.bM[i] - h * acc[0];
      const double Px = d.bPx[i] - h * acc[1];
      const double Py = d.bPy[i] - h * acc[2];
      const double E = d.bE[i] - h * acc[3];
      const double* rec = d.rec + (size_t)i * kRecDoubles;
      double x = d.bx[i] + h * rec[R_WX];
      double y = d.by[i] + h * rec[R_WY];
      if (d.bc == RICH_BOUNDARY_PERIODIC) {
        x = wrap_once(x, d.x0, d.x1);
        y = wrap_once(y, d.y0, d.y1);
        if (!(x >= d.x0 && x < d.x1 && y >= d.y0 && y < d.y1)) ok = false;
      }
      d.oM[i] = M;
      d.oPx[i] = Px;
      d.oPy[i] = Py;
      d.oE[i] = E;
      d.ox[i] = x;
      d.oy[i] = y;
      const double eint = E - 0.5 * (Px * Px + Py * Py) / M;
      if (!(M > 0.0) || !(eint > 0.0) || !isfinite(E) || !isfinite(Px) || !isfinite(Py) ||
          !isfinite(x) || !isfinite(y))
        ok = false;
    }
    if (!ok) atomicOr(d.flag, RICH_FLAG_DOMAIN);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// A0: Courant step, min over cells of R/(c + |v - w|)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_cfl(RunDesc d) {
  __shared__ double smin[kTile / 64];
  const int i = blockIdx.x * kTile + threadIdx.x;
  double t = INFINITY;
  if (i < d.n) {
    double rho, vx, vy, p;
    prim_of(d, i, rho, vx, vy, p);
    const double c = sqrt(d.gamma * p / rho);
    const double R = sqrt(d.area[i] / kPi);
    double wx = 0.0, wy = 0.0;
    if (d.motion) {
      wx = vx;
      wy = vy;
      const double dx = d.sx[i] - d.px[i], dy = d.sy[i] - d.py[i];
      const double dd = sqrt(dx * dx + dy * dy);
      if (dd > d.eta * R) {
        wx += d.chi * c * dx / dd;
        wy += d.chi * c * dy / dd;
      }
    }
    const double ux = vx - wx, uy = vy - wy;
    const double s = c + sqrt(ux * ux + uy * uy);
    t = R / s;
    if (!(t > 0.0)) t = INFINITY;  // NaN or non-positive: reported by the host check
  }
  for (int o = 32; o > 0; o >>= 1) t = fmin(t, __shfl_xor(t, o));
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smin[0];
    for (int w = 1; w < kTile / 64; ++w) m = fmin(m, smin[w]);
    unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    atomicMin(d.cfl_min, bits);
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

size_t run_ws_bytes(int64_t n) {
  return rich::kHeader + align_up((size_t)n * rich::kRecDoubles * sizeof(double), 256);
}

bool valid_mesh(const rich_mesh* m) {
  return m && m->n_cells > 0 && m->n_cells <= (int64_t)rich::kCellMask && m->n_edges >= 0 &&
         m->n_edges < (int64_t)INT32_MAX / 2 && m->n_csr >= 0 && m->n_csr < (int64_t)INT32_MAX &&
         m->px && m->py && m->sx && m->sy && m->area && m->off && m->eoff &&
         (m->n_edges == 0 || (m->e_i && m->e_j && m->e_len && m->e_fx && m->e_fy)) &&
         (m->n_csr == 0 || m->idx) && m->box[2] > m->box[0] && m->box[3] > m->box[1] &&
         (m->bc == RICH_BOUNDARY_WALLS || m->bc == RICH_BOUNDARY_PERIODIC);
}

bool valid_state(const rich_state* s, int64_t n, bool need_points) {
  return s && s->n_cells == n && s->M && s->Px && s->Py && s->E &&
         (!need_points || (s->x && s->y));
}

bool valid_params(const rich_params* p) {
  return p && p->gamma > 1.0 && std::isfinite(p->gamma) && p->riemann >= 0 && p->riemann <= 1 &&
         p->motion >= 0 && p->motion <= 1 && p->limiter >= 0 && p->limiter <= 4;
}

RunDesc make_desc(const rich_mesh* m, const rich_state* src, const rich_state* base,
                  rich_state* out, double h, const rich_params* p, char* ws) {
  RunDesc d;
  std::memset(&d, 0, sizeof(d));
  d.px = m->px; d.py = m->py; d.sx = m->sx; d.sy = m->sy; d.area = m->area;
  d.e_i = m->e_i; d.e_j = m->e_j; d.e_len = m->e_len; d.e_fx = m->e_fx; d.e_fy = m->e_fy;
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
  d.flag = reinterpret_cast<int32_t*>(ws);
  d.cfl_min = reinterpret_cast<unsigned long long*>(ws + 8);
  d.rec = reinterpret_cast<double*>(ws + rich::kHeader);
  d.x0 = m->box[0]; d.y0 = m->box[1]; d.x1 = m->box[2]; d.y1 = m->box[3];
  d.Lx = m->box[2] - m->box[0];
  d.Ly = m->box[3] - m->box[1];
  d.h = h;
  d.gamma = p->gamma; d.theta = p->theta; d.delta_v = p->delta_v; d.delta_p = p->delta_p;
  d.chi = p->chi; d.eta = p->eta;
  d.n = (int32_t)m->n_cells;
  d.n_edges = (int32_t)m->n_edges;
  d.n_csr = (int32_t)m->n_csr;
  d.bc = (int32_t)m->bc;
  d.riemann = p->riemann; d.motion = p->motion; d.limiter = p->limiter;
  return d;
}

int launch_stage(const RunDesc& d, int riemann, hipStream_t st) {
  const int n_tiles = (d.n + rich::kTile - 1) / rich::kTile;
  hipLaunchKernelGGL(rich::k_clear, dim3(1), dim3(64), 0, st, d.flag, d.cfl_min);
  hipLaunchKernelGGL(rich::k_cell<false>, dim3(n_tiles), dim3(rich::kTile), 0, st, d,
                     (const RunDesc*)nullptr, (const int32_t*)nullptr, 1, n_tiles);
  if (riemann == 1)
    hipLaunchKernelGGL((rich::k_flux<1, false>), dim3(n_tiles), dim3(rich::kTile), 0, st, d,
                       (const RunDesc*)nullptr, (const int32_t*)nullptr, 1, n_tiles);
  else
    hipLaunchKernelGGL((rich::k_flux<0, false>), dim3(n_tiles), dim3(rich::kTile), 0, st, d,
                       (const RunDesc*)nullptr, (const int32_t*)nullptr, 1, n_tiles);
  return hip_status(hipGetLastError());
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

int rich_stage_flags(void* ws, void* stream, int32_t* flags) {
  if (!ws || !flags) return RICH_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess) return RICH_E_DEVICE;
  if (hipMemcpy(flags, ws, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}

int rich_cfl_dt(const rich_mesh* m, const rich_state* s, const rich_params* p, double* dt,
                void* ws, size_t ws_bytes, void* stream) {
  if (!valid_mesh(m) || !valid_params(p) || !dt || !ws) return RICH_E_INVAL;
  if (!valid_state(s, m->n_cells, false)) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(m->n_cells)) return RICH_E_NOMEM;
  hipStream_t st = static_cast<hipStream_t>(stream);
  RunDesc d = make_desc(m, s, nullptr, nullptr, 0.0, p, static_cast<char*>(ws));
  const int nb = (d.n + rich::kTile - 1) / rich::kTile;
  hipLaunchKernelGGL(rich::k_clear, dim3(1), dim3(64), 0, st, d.flag, d.cfl_min);
  hipLaunchKernelGGL(rich::k_cfl, dim3(nb), dim3(rich::kTile), 0, st, d);
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
