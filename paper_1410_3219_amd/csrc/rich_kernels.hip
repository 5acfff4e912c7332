// Kernels and C-ABI of one stage of RICH's moving-mesh Godunov scheme on
// gfx950 (MI355X).  See rich.h for the interface and rich_device.hpp for the
// per-cell and per-edge arithmetic.
//
// One stage is two kernels over tiles of kTile consecutive cells (cells come
// in Hilbert order, so a tile is a compact patch of the mesh):
//   k_cell  two lanes per cell: primitives, point velocity, gradient and
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
// cells are each other's halo, then share an L2.  Batched launches run one
// block per tile of all runs and find each tile's run in a table.
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
#include <unordered_map>
#include <vector>

#include "rich.h"
#include "rich_device.hpp"

static_assert(sizeof(rich_cell) == 48, "rich_cell is three 16-byte chunks");
static_assert(sizeof(rich_edge) == 32, "rich_edge is two 16-byte chunks");

namespace rich {

#ifndef RICH_LPC
#define RICH_LPC 2
#endif
#ifndef RICH_CELL_MAXE
#define RICH_CELL_MAXE 6  // CSR entries per cell loaded level by level (the rest in a loop)
#endif
#ifndef RICH_CELL_PRE
#define RICH_CELL_PRE 1  // further CSR entries per lane whose entry and edge load with the first
#endif
#ifndef RICH_CELL_WAVES
#define RICH_CELL_WAVES 1  // minimum waves per SIMD the register budget must allow
#endif
#ifndef RICH_FLUX_WAVES
// minimum waves per SIMD of the HLLC flux pass: four (a 128-register budget,
// met without spills) hide its gathers better than three (2048^2 wave:
// 477 -> 438 us); the exact solver's pass would spill at four
#define RICH_FLUX_WAVES 4
#endif
#ifndef RICH_FLUX_TILE
#define RICH_FLUX_TILE 256
#endif
constexpr int kTile = RICH_FLUX_TILE;          // k_flux: default cells per tile = threads per block
constexpr int kCellThreads = 256;   // k_cell: threads per block
constexpr int kLpc = RICH_LPC;      // k_cell: lanes per cell
constexpr int kNumXcd = 8;
constexpr size_t kHeader = 256;  // per-run workspace header

// block -> tile, so that XCD x (blocks x, x+8, ...) gets one contiguous range
// of tiles.  A bijection on [0, nb) for any nb; a grid smaller than nb passes
// the virtual block index of each grid-stride round.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb / kNumXcd, rem = nb % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return x * q + min(x, rem) + k;
}
// The same ranges, each walked from its end: XCD x's k-th block takes the
// k-th tile from the end of the range (a bijection as well).  The flux pass
// walks this way, so that it starts on the records the cell pass wrote last,
// which the caches still hold (2048^2 wave: 512 -> 503 us).
__device__ __forceinline__ int xcd_tile_rev(int b, int nb) {
  const int q = nb / kNumXcd, rem = nb % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  const int cnt = q + (x < rem ? 1 : 0);
  return x * q + min(x, rem) + (cnt - 1 - k);
}


// Batched launches take a table with one entry per tile of the launch:
// {descriptor index of the tile's run, index of the run's first tile}, so a
// block finds its run with one load.

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
// A1-A4: LPC lanes per cell.  Lane l of a cell's group walks the CSR entries
// l, l+LPC, ... (neighbour gathers, gradient terms of eq. slope, neighbour
// bounds, pressure-ratio test), the partial results are combined with a fixed
// xor-shuffle tree (so every lane of the group holds the same bits), then the
// limiter pass is split the same way and each lane writes 16/LPC doubles of
// the cell's 128-byte record.  More lanes per cell shorten each lane's chain
// of dependent gathers and put more loads in flight.
// ---------------------------------------------------------------------------
// The value of lane (lane ^ O).  Within a quad of lanes (O = 1, 2) this is
// a DPP quad permutation on the vector ALU (no LDS round trip); further
// apart it is a shuffle.  Moves bits exactly.
template <int O>
__device__ __forceinline__ int lane_xor(int v) {
  if constexpr (O == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (O == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else {
    return __shfl_xor(v, O);
  }
}
template <int O>
__device__ __forceinline__ double lane_xor(double v) {
  const int lo = lane_xor<O>(__double2loint(v));
  const int hi = lane_xor<O>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Reductions over the LPC lanes of a cell (a fixed xor tree: every lane of
// the group ends with the same bits).
template <int LPC, int O = 1>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (O < LPC) return group_sum<LPC, 2 * O>(v + lane_xor<O>(v));
  return v;
}
template <int LPC, int O = 1>
__device__ __forceinline__ double group_max(double v) {
  if constexpr (O < LPC) return group_max<LPC, 2 * O>(dmax(v, lane_xor<O>(v)));
  return v;
}
template <int LPC, int O = 1>
__device__ __forceinline__ double group_min(double v) {
  if constexpr (O < LPC) return group_min<LPC, 2 * O>(dmin(v, lane_xor<O>(v)));
  return v;
}
template <int LPC, int O = 1>
__device__ __forceinline__ int group_or(int v) {
  if constexpr (O < LPC) return group_or<LPC, 2 * O>(v | lane_xor<O>(v));
  return v;
}

// The value a DPP control gives each lane (lanes outside row_mask keep
// their own); moves bits exactly.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_of(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xF, false),
                          __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xF, false));
}
// Minimum over the wave (64 lanes, whose groups of LPC lanes hold equal
// values) of values that are never NaN, held by lane 63, with DPP moves
// only: quads (quad permutations), eights (half-row mirror), rows (row
// mirror), then each row's last lane broadcast into the next row and lane 31
// into the upper half.
template <int LPC>
__device__ __forceinline__ double wave_min_cells(double t) {
  if constexpr (LPC < 2) t = dmin(t, dpp_of<0xB1>(t));  // quad_perm [1,0,3,2]
  if constexpr (LPC < 4) t = dmin(t, dpp_of<0x4E>(t));  // quad_perm [2,3,0,1]
  t = dmin(t, dpp_of<0x141>(t));                         // row_half_mirror
  t = dmin(t, dpp_of<0x140>(t));                         // row_mirror
  t = dmin(t, dpp_of<0x142, 0xA>(t));                    // row_bcast:15 into rows 1, 3
  t = dmin(t, dpp_of<0x143, 0xC>(t));                    // row_bcast:31 into rows 2, 3
  return t;
}
// Minimum over the block of the cell pass: the waves' minima through LDS,
// one barrier, valid in thread 0.  (One minimum per wave instead, with no
// barrier, was no faster, and the final reduction then reads four times as
// many minima.)
template <int LPC>
__device__ __forceinline__ double block_min_cells(double t) {
  __shared__ double sm[kCellThreads / 64];
  t = wave_min_cells<LPC>(t);
  if ((threadIdx.x & 63) == 63) sm[threadIdx.x >> 6] = t;
  __syncthreads();
  double m = sm[0];
#pragma unroll
  for (int w = 1; w < kCellThreads / 64; ++w) m = dmin(m, sm[w]);
  return m;
}

// DBG: also write each cell's branch record to dbg[i]: bit 0 the shock
// flag, bit 1 the cell-rounding correction applied, bits 2..5 alpha < 1 for
// rho, vx, vy, p.  The production instantiations have DBG = false.
template <int LPC, bool BATCH, bool DBG = false>
__global__ __launch_bounds__(kCellThreads, RICH_CELL_WAVES) void k_cell(RunDesc one,
                                                       const RunDesc* __restrict__ descs,
                                                       const int2* __restrict__ tile_run,
                                                       int n_tiles,
                                                       uint8_t* __restrict__ dbg) {
  constexpr int CPB = kCellThreads / LPC;  // cells per block
  constexpr int MAXE = RICH_CELL_MAXE / LPC;  // entries per lane loaded level by level
  constexpr int PRE = RICH_CELL_PRE;
  constexpr int ME = MAXE + PRE;  // entries whose CSR entry and edge are loaded early
  const int lane = (int)threadIdx.x % LPC;
  const int cl = (int)threadIdx.x / LPC;
  for (int b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    const int tt = xcd_tile(b, n_tiles);
    const int2 tr = BATCH ? tile_run[tt] : make_int2(0, 0);
    const RunDesc& d = BATCH ? descs[tr.x] : one;
    const int i0 = (tt - tr.y) * CPB + cl;
    const bool active = i0 < d.n;
    const int i = active ? i0 : 0;
    bool bad = false;

    double rix, riy, A, six, siy;
    load_cell(d, i, rix, riy, A, six, siy);
    // The CSR range and the first entries go out with the cell's own loads
    // (an inactive lane or a range outside the CSR gets no entries, and a
    // bad range flags the run; an entry past the cell's end reads entry k0,
    // in range, and is marked invalid).
    int k0 = d.off[i], k1 = d.off[i + 1];
    if (!active || k0 < 0 || k1 < k0 || k1 > d.n_csr) {
      if (active) bad = true;
      k1 = k0;
    }
    bool val[ME];
    int ent[ME];
    {
      const int kc = max(0, min(k0, d.n_csr - 1));
#pragma unroll
      for (int m = 0; m < ME; ++m) {
        const int k = k0 + lane + m * LPC;
        val[m] = k < k1;
        ent[m] = d.idx[val[m] ? k : kc];
      }
    }
    if (active && !(A > 0.0 && A < INFINITY)) bad = true;  // a mesh cell without a volume
    double rho, vx, vy, p;
    prim_of(d, i, A, rho, vx, vy, p);
    // A2 (section 6) and, fused into the cell pass, the cell's Courant ratio
    // (A0), reduced to the block's minimum at the end of the tile (each
    // cell's lanes agree)
    const Kin kin = kinematics(d, A, rho, vx, vy, p, rix, riy, six, siy);
    const double c = kin.c, R = kin.R, wx = kin.wx, wy = kin.wy;
    const bool rounded = kin.rounded;
    const double phi[4] = {rho, vx, vy, p};
    // neighbour values and point across one CSR entry (mirror for a wall)
    auto nb_values = [&](const NbE& v, double* pj, double& rjx, double& rjy) {
      if (v.wall) {
        pj[0] = rho;
        mirror_vec(v.wall, vx, vy, pj[1], pj[2]);
        pj[3] = p;
        mirror_point(d, v.wall, rix, riy, rjx, rjy);
      } else {
        double Aj;
        load_point_area(d, v.j, rjx, rjy, Aj);
        prim_of(d, v.j, Aj, pj[0], pj[1], pj[2], pj[3]);
        rjx += v.shx;
        rjy += v.shy;
      }
    };

    // A3: eq. (slope), r_ij = r_i - r_j
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double pmax[4] = {rho, vx, vy, p}, pmin[4] = {rho, vx, vy, p};
    int pflag = 0;
    double fdx[ME], fdy[ME];
    // Per entry the weights L c_ij / |r_ij| and L r_ij / (2 |r_ij|) are
    // formed once; each field then adds (phi_j - phi_i) times the first minus
    // (phi_i + phi_j) times the second with two fused multiply-adds per
    // component.
    auto accumulate = [&](const NbE& v, const double* pj, double vrx, double vry) {
      const double rx = rix - vrx, ry = riy - vry;
      const double Lr = v.L * rsqrt(rx * rx + ry * ry);
      const double cx = v.fx - 0.5 * (rix + vrx), cy = v.fy - 0.5 * (riy + vry);
      const double ux = Lr * cx, uy = Lr * cy;
      const double hLr = 0.5 * Lr;
      const double nx = hLr * rx, ny = hLr * ry;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double dphi = pj[q] - phi[q];
        const double sum = phi[q] + pj[q];
        g[2 * q] = fma(-sum, nx, fma(dphi, ux, g[2 * q]));
        g[2 * q + 1] = fma(-sum, ny, fma(dphi, uy, g[2 * q + 1]));
        pmax[q] = dmax(pmax[q], pj[q]);
        pmin[q] = dmin(pmin[q], pj[q]);
      }
      if (pressure_jump(d.delta_p, p, pj[3])) pflag = 1;
    };
    // The first MAXE/LPC entries of each lane go level by level: all CSR
    // entries, then all edges, then all neighbours, each level's loads issued
    // together with in-range indices and no branch between them (an entry
    // past the cell's end reads entry k0 and is ignored), so that a lane waits
    // for three memory round trips instead of three per entry.
    {
      int ee[ME];
#pragma unroll
      for (int m = 0; m < ME; ++m) {
        int e = ent[m] >> 1;
        if (val[m] && (e < 0 || e >= d.n_edges)) {
          bad = true;
          val[m] = false;
        }
        ee[m] = val[m] ? e : 0;
      }
      uint32_t ej[ME];
      int ei[ME];
      double eL[ME], efx[ME], efy[ME];
#pragma unroll
      for (int m = 0; m < ME; ++m) {
        const EdgeRec er = load_edge(d, ee[m]);
        ej[m] = er.j;
        ei[m] = er.i;
        eL[m] = er.L;
        efx[m] = er.fx;
        efy[m] = er.fy;
      }
      NbE v[ME];
#pragma unroll
      for (int m = 0; m < ME; ++m) {
        const int side = ent[m] & 1;
        const int code = (int)(ej[m] >> 28);
        v[m].L = eL[m];
        v[m].fx = efx[m];
        v[m].fy = efy[m];
        shift_of(d, code, v[m].shx, v[m].shy);
        v[m].wall = (side == 0 && code >= 9) ? code : 0;
        int j = side == 0 ? (int)(ej[m] & kCellMask) : ei[m];
        if (side) {
          v[m].shx = -v[m].shx;
          v[m].shy = -v[m].shy;
          v[m].fx += v[m].shx;
          v[m].fy += v[m].shy;
        }
        if (v[m].wall) j = i;
        if (val[m] && (j < 0 || j >= d.n)) {
          bad = true;
          j = i;
        }
        v[m].j = val[m] ? j : i;
      }
      double nA[MAXE], nM[MAXE], nPx[MAXE], nPy[MAXE], nE[MAXE], nx_[MAXE], ny_[MAXE];
#pragma unroll
      for (int m = 0; m < MAXE; ++m) {
        const int j = v[m].j;
        load_point_area(d, j, nx_[m], ny_[m], nA[m]);
        nM[m] = d.sM[j];
        nPx[m] = d.sPx[j];
        nPy[m] = d.sPy[j];
        nE[m] = d.sE[j];
      }
#pragma unroll
      for (int m = 0; m < MAXE; ++m) {
        fdx[m] = 0.0;
        fdy[m] = 0.0;
        if (val[m]) {
          double pj[4], vrx, vry;
          if (v[m].wall) {
            pj[0] = rho;
            mirror_vec(v[m].wall, vx, vy, pj[1], pj[2]);
            pj[3] = p;
            mirror_point(d, v[m].wall, rix, riy, vrx, vry);
          } else {
            prim_from(d, nA[m], nM[m], nPx[m], nPy[m], nE[m], pj[0], pj[1], pj[2], pj[3]);
            vrx = nx_[m] + v[m].shx;
            vry = ny_[m] + v[m].shy;
          }
          accumulate(v[m], pj, vrx, vry);
          fdx[m] = v[m].fx - six;
          fdy[m] = v[m].fy - siy;
        }
      }
      // entries loaded early past the level-by-level ones: their neighbours
      // cost one more round trip, not three
#pragma unroll
      for (int m = MAXE; m < ME; ++m) {
        fdx[m] = 0.0;
        fdy[m] = 0.0;
        if (val[m]) {
          double pj[4], vrx, vry;
          nb_values(v[m], pj, vrx, vry);
          accumulate(v[m], pj, vrx, vry);
          fdx[m] = v[m].fx - six;
          fdy[m] = v[m].fy - siy;
        }
      }
    }
    for (int k = k0 + lane + ME * LPC; k < k1; k += LPC) {
      const NbE v = nb_edge(d, i, d.idx[k], bad);
      double pj[4], vrx, vry;
      nb_values(v, pj, vrx, vry);
      accumulate(v, pj, vrx, vry);
    }
    double G[8];
    const double rA = rcp(A);
#pragma unroll
    for (int q = 0; q < 8; ++q) G[q] = group_sum<LPC>(g[q]) * rA;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      pmax[q] = group_max<LPC>(pmax[q]);
      pmin[q] = group_min<LPC>(pmin[q]);
    }
    bool shock = group_or<LPC>(pflag) != 0;
    if (-(G[2] + G[5]) * R > d.delta_v * c) shock = true;  // -div v > delta_v c / R, R > 0

    // A4: limiter
    double alpha[4] = {1.0, 1.0, 1.0, 1.0};
    int local = -1;
    if (d.limiter == 0) local = shock ? 1 : 0;
    if (d.limiter == 1) local = 0;
    if (d.limiter == 2) local = 1;
    if (d.limiter == 4) alpha[0] = alpha[1] = alpha[2] = alpha[3] = 0.0;
    if (local == 0) {
      // global limiter: min_j psi_ij is attained at the largest positive and
      // the most negative change (division is monotone in the denominator)
      double dmax[4] = {0, 0, 0, 0}, dmin[4] = {0, 0, 0, 0};
      auto bound = [&](double dx, double dy) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double dphi = G[2 * q] * dx + G[2 * q + 1] * dy;
          dmax[q] = rich::dmax(dmax[q], dphi);
          dmin[q] = rich::dmin(dmin[q], dphi);
        }
      };
#pragma unroll
      for (int m = 0; m < ME; ++m)
        if (k0 + lane + m * LPC < k1) bound(fdx[m], fdy[m]);
      for (int k = k0 + lane + ME * LPC; k < k1; k += LPC) {
        const NbE v = nb_edge(d, i, d.idx[k], bad);
        bound(v.fx - six, v.fy - siy);
      }
      // alpha = min(1, (phi_max - phi)/dmax, (phi_min - phi)/dmin) over the
      // bounds that apply (dmax > 0, dmin < 0): both ratios are >= 0, the
      // smaller one is picked by cross-multiplication and only it is divided
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        dmax[q] = group_max<LPC>(dmax[q]);
        dmin[q] = group_min<LPC>(dmin[q]);
        const bool ua = dmax[q] > 0.0, ub = dmin[q] < 0.0;
        const double na = pmax[q] - phi[q], da = dmax[q];
        const double nb = phi[q] - pmin[q], db = -dmin[q];
        const bool pick_a = ua && (!ub || na * db < nb * da);
        const double r = ddiv(pick_a ? na : nb, pick_a ? da : db);
        if (ua || ub) alpha[q] = rich::dmin(alpha[q], r);
      }
    } else if (local == 1) {
      for (int k = k0 + lane; k < k1; k += LPC) {
        const NbE v = nb_edge(d, i, d.idx[k], bad);
        double pj[4], vrx, vry;
        nb_values(v, pj, vrx, vry);
        const double dx = v.fx - six, dy = v.fy - siy;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double dphi = G[2 * q] * dx + G[2 * q + 1] * dy;
          const double psi =
              (dphi != 0.0) ? dmax(ddiv(d.theta * (pj[q] - phi[q]), dphi), 0.0) : 1.0;
          alpha[q] = dmin(alpha[q], psi);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) alpha[q] = group_min<LPC>(alpha[q]);
    }
    const int bad_any = group_or<LPC>(bad ? 1 : 0);
    if (active) {
      double rec[kRecDoubles];
#pragma unroll
      for (int q = 0; q < 8; ++q) rec[R_G + q] = G[q] * alpha[q / 2];
      // the change of the stored primitives: with extrapolated fluxes
      // (section 2.3) they are advanced half a step with the time derivatives
      // the limited gradients give in the primitive Euler equations,
      // following the cell's point (v - w); otherwise none
      double adv[4] = {0.0, 0.0, 0.0, 0.0};
      if (d.integrator == 1) {
        const double* g = rec + R_G;
        const double ux = vx - wx, uy = vy - wy;
        const double div = g[2] + g[5];
        const double rho_t = -(ux * g[0] + uy * g[1]) - rho * div;
        const double vx_t = -(ux * g[2] + uy * g[3]) - g[6] / rho;
        const double vy_t = -(ux * g[4] + uy * g[5]) - g[7] / rho;
        const double p_t = -(ux * g[6] + uy * g[7]) - d.gamma * p * div;
        const double hh = 0.5 * (d.h_dev != nullptr ? d.h_factor * (*d.h_dev) : d.h);
        adv[0] = hh * rho_t;
        adv[1] = hh * vx_t;
        adv[2] = hh * vy_t;
        adv[3] = hh * p_t;
      }
      {
        // the reconstruction moved from the centroid to the point
        const double ox = rix - six, oy = riy - siy;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          rec[q] = (phi[q] + adv[q]) + rec[R_G + 2 * q] * ox + rec[R_G + 2 * q + 1] * oy;
      }
      rec[R_WX] = wx;
      rec[R_WY] = wy;
      rec[R_PX] = rix;
      rec[R_PY] = riy;
      constexpr int PER = kRecDoubles / LPC;  // doubles written by each lane
      double2* dst = reinterpret_cast<double2*>(d.rec + (size_t)i * kRecDoubles + lane * PER);
#pragma unroll
      for (int k = 0; k < PER / 2; ++k) {
        // select this lane's slice with compile-time indices only
        double a0 = rec[2 * k], a1 = rec[2 * k + 1];
#pragma unroll
        for (int l = 1; l < LPC; ++l)
          if (lane == l) {
            a0 = rec[l * PER + 2 * k];
            a1 = rec[l * PER + 2 * k + 1];
          }
        dst[k] = make_double2(a0, a1);
      }
      if (bad_any && lane == 0) atomicOr(d.flag, RICH_FLAG_DOMAIN);
      if constexpr (DBG) {
        if (lane == 0) {
          int bits = (shock ? 1 : 0) | (rounded ? 2 : 0);
#pragma unroll
          for (int q = 0; q < 4; ++q) bits |= (alpha[q] < 1.0 ? 4 << q : 0);
          dbg[i] = (uint8_t)bits;
        }
      }
    }
    if (d.cfl_blocks != nullptr) {
      const double ti = active ? courant_ratio(kin, vx, vy) : INFINITY;
      const double bm = block_min_cells<LPC>(ti);
      if (threadIdx.x == 0) d.cfl_blocks[tt] = bm;
    }
  }
}

// ---------------------------------------------------------------------------
// A5-A8: one block per tile of kTile cells.
//   phase 0  classify the tile's CSR entries: an edge the tile owns (first
//            cell inside the tile, within the LDS capacity) is found at its
//            position in the owned range; any other edge goes on a list
//   phase 1  all lanes compute the owned edges and the listed edges, once
//            each, into LDS
//   phase 2  one lane per cell sums its entries in CSR order
// Fluxes of edges whose first cell lies in another tile are computed by both
// tiles, with the same code on the same inputs, hence the same bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wrap_once(double v, double lo, double hi) {
  const double L = hi - lo;
  if (v < lo) v += L;
  if (v >= hi) v -= L;
  return v;
}

// A5-A7 for edge e from the records of its two cells in the workspace.
template <int RIEMANN>
__device__ __forceinline__ bool flux_of_edge(const RunDesc& d, int e, double* LF,
                                             uint8_t* br = nullptr) {
  double ri[kRecDoubles], rj[kRecDoubles];
  if (e < 0 || e >= d.n_edges) {
    LF[0] = LF[1] = LF[2] = LF[3] = 0.0;
    return false;
  }
  const EdgeRec er = load_edge(d, e);
  const int i = er.i;
  const uint32_t ej = er.j;
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
  return edge_flux_at<RIEMANN>(d, i, ej, er.fx, er.fy, er.L, ri, rj, LF, br);
}

// Debug record of the Riemann solver's branch on every edge (one thread per
// edge), from the cell records of the stage; arithmetic identical to k_flux.
template <int RIEMANN>
__global__ __launch_bounds__(256) void k_edge_bits(RunDesc d, uint8_t* bits) {
  const int e = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (e >= d.n_edges) return;
  double LF[4];
  uint8_t b = 0;
  if (!flux_of_edge<RIEMANN>(d, e, LF, &b)) b |= 8;
  bits[e] = b;
}

template <int RIEMANN, bool BATCH, int TILE = kTile>
__global__ __launch_bounds__(TILE, RIEMANN == 0 ? RICH_FLUX_WAVES : 1) void k_flux(RunDesc one, const RunDesc* __restrict__ descs,
                                                const int2* __restrict__ tile_run,
                                                int n_tiles) {
  // LDS capacities in proportion to the tile: fluxes of the owned edges
  // (about 3 per cell), of other edges the tile's cells need (its border),
  // and the classification of the tile's CSR entries (about 6 per cell)
  constexpr int kEdgeCap = TILE * 25 / 8, kForCap = TILE * 3 / 4, kMapCap = TILE * 9;
  __shared__ double sF[4][kEdgeCap + kForCap];
  __shared__ int s_forE[kForCap];
  __shared__ short s_map[kMapCap];  // (flux slot << 1) | side, or -1
  __shared__ int s_off[TILE + 1];  // the tile's CSR offsets
  __shared__ int s_nfor;
  const int tid = (int)threadIdx.x;
  for (int b = blockIdx.x; b < n_tiles; b += gridDim.x) {
    const int t = xcd_tile_rev(b, n_tiles);
    const int2 tr = BATCH ? tile_run[t] : make_int2(0, 0);
    const RunDesc& d = BATCH ? descs[tr.x] : one;
    const int c0 = (t - tr.y) * TILE;
    const int c1 = min(c0 + TILE, d.n);
    const int e0 = d.eoff[c0];
    const int ne = max(0, min(d.eoff[c1] - e0, kEdgeCap));
    const int kb = d.off[c0];
    const int S = max(0, min(d.off[c1], d.n_csr) - kb);
    const int Sm = min(S, kMapCap);
    bool ok = true;
    if (tid == 0) s_nfor = 0;
    for (int c = tid; c <= c1 - c0; c += TILE) s_off[c] = d.off[c0 + c];
    __syncthreads();
    // all of a lane's CSR entries are loaded first (independent loads in
    // flight together), then classified
    constexpr int MPT = kMapCap / TILE;
    int ent[MPT];
#pragma unroll
    for (int r = 0; r < MPT; ++r) {
      const int s = tid + r * TILE;
      ent[r] = s < Sm ? d.idx[kb + s] : -1;
    }
#pragma unroll
    for (int r = 0; r < MPT; ++r) {
      const int s = tid + r * TILE;
      if (s >= Sm) break;
      const int entry = ent[r];
      const int e = entry >> 1;
      int m = -1;
      if (e >= e0 && e < e0 + ne) {
        m = e - e0;
      } else if (e >= 0 && e < d.n_edges) {
        const int f = atomicAdd(&s_nfor, 1);
        if (f < kForCap) {
          s_forE[f] = e;
          m = kEdgeCap + f;
        }
      }
      s_map[s] = (short)(m < 0 ? -1 : (m << 1) | (entry & 1));
    }
    __syncthreads();
    const int nfor = min(s_nfor, kForCap);
    for (int w = tid; w < ne + nfor; w += TILE) {
      const int e = w < ne ? e0 + w : s_forE[w - ne];
      const int pos = w < ne ? w : kEdgeCap + (w - ne);
      double LF[4];
      if (!flux_of_edge<RIEMANN>(d, e, LF)) ok = false;
#pragma unroll
      for (int q = 0; q < 4; ++q) sF[q][pos] = LF[q];
    }
    __syncthreads();
    const int i = c0 + tid;
    if (i < c1) {
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int k0 = s_off[tid], k1 = s_off[tid + 1];
      if (k0 < kb || k1 < k0 || k1 > kb + S) {
        ok = false;
        k1 = k0;
      }
      for (int k = k0; k < k1; ++k) {
        const int s = k - kb;
        const int ms = s < Sm ? (int)s_map[s] : -1;
        double LF[4];
        int side;
        if (ms >= 0) {
          const int m = ms >> 1;
          side = ms & 1;
#pragma unroll
          for (int q = 0; q < 4; ++q) LF[q] = sF[q][m];
        } else {
          const int entry = d.idx[k];
          side = entry & 1;
          if (!flux_of_edge<RIEMANN>(d, entry >> 1, LF)) ok = false;
        }
        if (side) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] -= LF[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] += LF[q];
        }
      }
      const double h = d.h_dev != nullptr ? d.h_factor * (*d.h_dev) : d.h;
      // (loading these before the flux sum keeps them live across the
      // foreign-edge fallback and costs occupancy)
      const double bM = d.bM[i], bPx = d.bPx[i], bPy = d.bPy[i], bE = d.bE[i];
      const double bx = d.bx[i], by = d.by[i];
      const double2 wi = *reinterpret_cast<const double2*>(d.rec + (size_t)i * kRecDoubles + R_WX);
      const double M = bM - h * acc[0];
      double Px = bPx - h * acc[1];
      double Py = bPy - h * acc[2];
      double E = bE - h * acc[3];
      double gx = d.gx, gy = d.gy;
      if (d.ax != nullptr) {  // the cell's own acceleration
        gx += d.ax[i];
        gy += d.ay[i];
      }
      if (gx != 0.0 || gy != 0.0) {
        // external acceleration: h (0, M g, P.g) of the stage's source totals
        const double sm = d.sM[i], spx = d.sPx[i], spy = d.sPy[i];
        Px += h * (sm * gx);
        Py += h * (sm * gy);
        E += h * (spx * gx + spy * gy);
      }
      double x = bx + h * wi.x;
      double y = by + h * wi.y;
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
// from the records that k_cell wrote.
__global__ __launch_bounds__(kCflThreads) void k_adot(RunDesc d, double* adot) {
  const int i = blockIdx.x * kCflThreads + threadIdx.x;
  if (i >= d.n) return;
  double rix, riy;
  load_point(d, i, rix, riy);
  const double* ri = d.rec + (size_t)i * kRecDoubles;
  const double wix = ri[R_WX], wiy = ri[R_WY];
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
      const double* rj = d.rec + (size_t)v.j * kRecDoubles;
      wjx = rj[R_WX];
      wjy = rj[R_WY];
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
    const Kin kin = kinematics(d, A, rho, vx, vy, p, pxi, pyi, sxi, syi);
    const double ti = courant_ratio(kin, vx, vy);
    t = fmin(t, ti);
  }
  const double m = block_min(t, smin);
  if (threadIdx.x == 0) block_out[blockIdx.x] = m;
}

constexpr int kCflFinalThreads = 1024;
constexpr int kCflBatchThreads = 256;
// The minimum of nb block minima, as a bit pattern in *out; with dt_out also
// dt = cfl * minimum in *dt_out, and the domain flag when that is not a
// positive number.  NT threads; min is order-free, so the result does not
// depend on NT.
template <int NT>
__device__ __forceinline__ void cfl_finish(const double* block_in, int nb,
                                           unsigned long long* out, double cfl, double* dt_out,
                                           int32_t* flag) {
  __shared__ double smin[NT / 64];
  // four independent minima per thread, so the loads of a thread overlap
  double t0 = INFINITY, t1 = INFINITY, t2 = INFINITY, t3 = INFINITY;
  int b = threadIdx.x;
  for (; b + 3 * NT < nb; b += 4 * NT) {
    t0 = fmin(t0, block_in[b]);
    t1 = fmin(t1, block_in[b + NT]);
    t2 = fmin(t2, block_in[b + 2 * NT]);
    t3 = fmin(t3, block_in[b + 3 * NT]);
  }
  for (; b < nb; b += NT) t0 = fmin(t0, block_in[b]);
  double t = fmin(fmin(t0, t1), fmin(t2, t3));
  for (int o = 32; o > 0; o >>= 1) t = fmin(t, __shfl_xor(t, o));
  if ((threadIdx.x & 63) == 0) smin[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = smin[0];
    for (int w = 1; w < NT / 64; ++w) m = fmin(m, smin[w]);
    *out = (unsigned long long)__double_as_longlong(m);
    if (dt_out != nullptr) {
      const double dt = cfl * m;
      *dt_out = dt;
      if (!(dt > 0.0) || !isfinite(dt)) atomicOr(flag, RICH_FLAG_DOMAIN);
    }
  }
}

__global__ __launch_bounds__(kCflFinalThreads) void k_cfl_final(const double* block_in, int nb,
                                                                unsigned long long* out,
                                                                double cfl, double* dt_out,
                                                                int32_t* flag) {
  cfl_finish<kCflFinalThreads>(block_in, nb, out, cfl, dt_out, flag);
}

// Batched Courant stage: block k finishes run k of the cell plan (entries
// tile_start[k] .. tile_start[k + 1] - 1 of the batch's block minima, which
// every descriptor's cfl_blocks points to, are its cell tiles) and writes
// the run's step where its descriptor's h_dev points.
__global__ __launch_bounds__(kCflBatchThreads) void k_cfl_final_batch(
    const RunDesc* __restrict__ descs, const int32_t* __restrict__ tile_start, int n_runs) {
  const int k = blockIdx.x;
  if (k >= n_runs) return;
  const RunDesc& d = descs[tile_start[n_runs + 1 + k]];
  if (d.cfl_blocks == nullptr || d.h_dev == nullptr) {
    // descriptors of a stage without device steps: nothing to finish
    if (threadIdx.x == 0) atomicOr(d.flag, RICH_FLAG_DOMAIN);
    return;
  }
  const int t0 = tile_start[k];
  cfl_finish<kCflBatchThreads>(d.cfl_blocks + t0, tile_start[k + 1] - t0, d.cfl_min, d.cfl,
                               const_cast<double*>(d.h_dev), d.flag);
}

}  // namespace rich

// ===========================================================================
// Host side
// ===========================================================================
using rich::RunDesc;

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? RICH_OK : RICH_E_DEVICE; }

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr int64_t kCellsPerBlock = rich::kCellThreads / rich::kLpc;
constexpr size_t kDtOffset = 16;  // header: flag @0, Courant minimum @8, dt @16

constexpr size_t run_ws_size(int64_t n) {
  return rich::kHeader + ((size_t)n * rich::kRecDoubles * sizeof(double) + 255) / 256 * 256 +
         ((size_t)((n + kCellsPerBlock - 1) / kCellsPerBlock) * sizeof(double) + 255) / 256 * 256;
}
size_t run_ws_bytes(int64_t n) { return run_ws_size(n); }

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
  d.flag = reinterpret_cast<int32_t*>(ws);
  d.cfl_min = reinterpret_cast<unsigned long long*>(ws + 8);
  d.rec = reinterpret_cast<double*>(ws + rich::kHeader);
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

int launch_stage(const RunDesc& d, int riemann, hipStream_t st, uint8_t* dbg_cell = nullptr,
                 uint8_t* dbg_edge = nullptr) {
  constexpr int T = rich::kTile;
  const int n_tiles = (d.n + T - 1) / T;
  constexpr int CPB = rich::kCellThreads / rich::kLpc;
  const int n_ctiles = (d.n + CPB - 1) / CPB;
  hipLaunchKernelGGL(rich::k_clear, dim3(1), dim3(64), 0, st, d.flag, d.cfl_min);
  int pc = prof_begin("k_cell", st);
  if (dbg_cell != nullptr)
    hipLaunchKernelGGL((rich::k_cell<rich::kLpc, false, true>), dim3(n_ctiles),
                       dim3(rich::kCellThreads), 0, st, d, (const RunDesc*)nullptr,
                       (const int2*)nullptr, n_ctiles, dbg_cell);
  else
    hipLaunchKernelGGL((rich::k_cell<rich::kLpc, false>), dim3(n_ctiles),
                       dim3(rich::kCellThreads), 0, st, d, (const RunDesc*)nullptr,
                       (const int2*)nullptr, n_ctiles, (uint8_t*)nullptr);
  prof_end(pc, st);
  if (dbg_edge != nullptr && d.n_edges > 0) {
    const int eb = (int)((d.n_edges + 255) / 256);
    if (riemann == 1)
      hipLaunchKernelGGL(rich::k_edge_bits<1>, dim3(eb), dim3(256), 0, st, d, dbg_edge);
    else
      hipLaunchKernelGGL(rich::k_edge_bits<0>, dim3(eb), dim3(256), 0, st, d, dbg_edge);
  }
  if (d.cfl_blocks != nullptr)   // dt from the cell kernel's Courant minima
    hipLaunchKernelGGL(rich::k_cfl_final, dim3(1), dim3(rich::kCflFinalThreads), 0, st,
                       (const double*)d.cfl_blocks, n_ctiles, d.cfl_min, d.cfl,
                       const_cast<double*>(d.h_dev), d.flag);
  int pf = prof_begin("k_flux", st);
  if (riemann == 1)
    hipLaunchKernelGGL((rich::k_flux<1, false>), dim3(n_tiles), dim3(T), 0, st, d,
                       (const RunDesc*)nullptr, (const int2*)nullptr, n_tiles);
  else
    hipLaunchKernelGGL((rich::k_flux<0, false>), dim3(n_tiles), dim3(T), 0, st, d,
                       (const RunDesc*)nullptr, (const int2*)nullptr, n_tiles);
  prof_end(pf, st);
  return hip_status(hipGetLastError());
}

}  // namespace

// ---------------------------------------------------------------------------
// batch workspace:  [descriptors][plans][flags][Courant minima][steps]
//                   [records...][Courant block minima][tile -> run tables]
// Everything before the records depends on the number of runs only.
// ---------------------------------------------------------------------------
struct BatchLayout {
  size_t desc, plan, flags, cfl, dt, rec, cflb, tab, total;
  std::vector<size_t> rec_off;
};

BatchLayout batch_layout(int32_t n, const int64_t* n_cells) {
  constexpr int CPB = rich::kCellThreads / rich::kLpc;
  BatchLayout L;
  size_t o = 0;
  L.desc = o;
  o += align_up((size_t)n * sizeof(RunDesc), 256);
  L.plan = o;
  o += align_up((size_t)3 * (2 * (size_t)n + 1) * sizeof(int32_t), 256);
  L.flags = o;
  o += align_up((size_t)n * sizeof(int32_t), 256);
  L.cfl = o;
  o += align_up((size_t)n * sizeof(unsigned long long), 256);
  L.dt = o;
  o += align_up((size_t)n * sizeof(double), 256);
  L.rec = o;
  L.rec_off.resize(n);
  size_t tiles = 0, flux_tiles = 0;   // flux tiles: at most those of the smallest tile, 128
  for (int32_t r = 0; r < n; ++r) {
    L.rec_off[r] = o;
    o += align_up((size_t)n_cells[r] * rich::kRecDoubles * sizeof(double), 256);
    tiles += (size_t)((n_cells[r] + CPB - 1) / CPB);
    flux_tiles += (size_t)((n_cells[r] + 127) / 128);
  }
  L.cflb = o;
  o += align_up(tiles * sizeof(double), 256);
  // tile -> run tables: cell tiles, then the flux tiles of the two solver
  // groups (which partition the runs)
  L.tab = o;
  o += align_up((tiles + flux_tiles) * sizeof(int2), 256);
  L.total = o;
  return L;
}

// Pinned host staging for the descriptor uploads: a ring of buffers, each
// reused only after the copy that last read it has completed.
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

// Copy host blocks into device memory through the pinned ring, on stream
// st.  The whole sequence (pick a buffer, fill it, enqueue the copies,
// record the buffer's event) holds one lock, so host threads that launch
// batches concurrently never share a buffer in flight.
int upload_staged(std::initializer_list<std::pair<void*, std::pair<const void*, size_t>>> blocks,
                  hipStream_t st) {
  std::lock_guard<std::mutex> g(staging_lock());
  size_t total = 0;
  for (const auto& b : blocks) total += b.second.second;
  hipEvent_t ev = nullptr;
  char* host = static_cast<char*>(staging().get(total, &ev));
  if (!host) return RICH_E_NOMEM;
  size_t o = 0;
  for (const auto& b : blocks) {
    if (b.second.second == 0) continue;
    std::memcpy(host + o, b.second.first, b.second.second);
    if (hipMemcpyAsync(b.first, host + o, b.second.second, hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return RICH_E_DEVICE;
    o += b.second.second;
  }
  if (hipEventRecord(ev, st) != hipSuccess) return RICH_E_DEVICE;
  return RICH_OK;
}

// The last plan prepared on each batch workspace: a launch runs only the plan
// whose descriptors the workspace holds (a later prepare on the same
// workspace overwrites them, and kernels launched with another plan's sizes
// would read them out of step).
std::mutex& plan_lock() {
  static std::mutex m;
  return m;
}
std::unordered_map<const void*, int64_t>& plan_registry() {
  static std::unordered_map<const void*, int64_t> r;
  return r;
}
int64_t register_plan(const void* ws) {
  static int64_t serial = 0;
  std::lock_guard<std::mutex> g(plan_lock());
  const int64_t s = ++serial;
  plan_registry()[ws] = s;
  return s;
}
bool plan_is_current(const void* ws, int64_t s) {
  std::lock_guard<std::mutex> g(plan_lock());
  auto it = plan_registry().find(ws);
  return it != plan_registry().end() && it->second == s;
}

// The batched flux kernel of solver k (0 HLLC, 1 exact) with tiles of `tile` cells.
void launch_flux_batch(int k, int tile, int grid, hipStream_t st, const RunDesc& dummy,
                       const RunDesc* dd, const int2* tab, int n_tiles) {
  switch (k * 4 + (tile == 128 ? 0 : tile == 256 ? 1 : 2)) {
    case 0: hipLaunchKernelGGL((rich::k_flux<0, true, 128>), dim3(grid), dim3(128), 0, st, dummy, dd, tab, n_tiles); break;
    case 1: hipLaunchKernelGGL((rich::k_flux<0, true, 256>), dim3(grid), dim3(256), 0, st, dummy, dd, tab, n_tiles); break;
    case 2: hipLaunchKernelGGL((rich::k_flux<0, true, 512>), dim3(grid), dim3(512), 0, st, dummy, dd, tab, n_tiles); break;
    case 4: hipLaunchKernelGGL((rich::k_flux<1, true, 128>), dim3(grid), dim3(128), 0, st, dummy, dd, tab, n_tiles); break;
    case 5: hipLaunchKernelGGL((rich::k_flux<1, true, 256>), dim3(grid), dim3(256), 0, st, dummy, dd, tab, n_tiles); break;
    default: hipLaunchKernelGGL((rich::k_flux<1, true, 512>), dim3(grid), dim3(512), 0, st, dummy, dd, tab, n_tiles); break;
  }
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

// ---------------------------------------------------------------------------
// Scratch of rich_stage_noalloc: one file-scope device array per GPU, sized
// for the largest run that entry point takes.  In host code `scratch` is a
// host-side stand-in for the symbol, never a device address: the address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress, with
// that device current) and kept; only that address reaches kernels.
// ---------------------------------------------------------------------------
constexpr int64_t kNoAllocMaxCells = RICH_NOALLOC_MAX_CELLS;
constexpr size_t kNoAllocBytes = run_ws_size(kNoAllocMaxCells);
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex& scratch_lock() {
  static std::mutex m;
  return m;
}
// The current device's address of `scratch` (looked up on the first call on
// that device), or null on a HIP error.
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  static void* ptr[kMaxDevices] = {};
  std::lock_guard<std::mutex> g(scratch_lock());
  if (ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return nullptr;
    ptr[dev] = p;
  }
  return ptr[dev];
}
}  // namespace

namespace rich {
__global__ void k_copy_flag(const int32_t* flag, int32_t* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = *flag;
}
}  // namespace rich

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

int rich_stage_noalloc(const rich_mesh* m, const rich_state* src, const rich_state* base,
                       rich_state* out, double h, const rich_params* p, int32_t* flag_out,
                       void* stream) {
  if (!valid_mesh(m) || !valid_params(p)) return RICH_E_INVAL;
  const int64_t n = m->n_cells;
  if (!valid_state(src, n, false) || !valid_state(base, n, true) || !valid_state(out, n, true))
    return RICH_E_INVAL;
  if (!std::isfinite(h) || h < 0.0) return RICH_E_INVAL;
  if (out->M == src->M || out->M == base->M || out->x == base->x) return RICH_E_INVAL;
  if (n > kNoAllocMaxCells || run_ws_bytes(n) > kNoAllocBytes) return RICH_E_NOMEM;
  char* ws = static_cast<char*>(scratch_address());
  if (ws == nullptr) return RICH_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  RunDesc d = make_desc(m, src, base, out, h, p, ws);
  const int rc = launch_stage(d, p->riemann, st);  // clears the flag word with a kernel
  if (rc) return rc;
  if (flag_out) hipLaunchKernelGGL(rich::k_copy_flag, dim3(1), dim3(64), 0, st, d.flag, flag_out);
  return hip_status(hipGetLastError());
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
  // extrapolated fluxes need the step inside the cell pass, before its minimum exists
  if (courant && p->integrator == 1) return RICH_E_INVAL;
  if (out->M == src->M || out->M == base->M || out->x == base->x) return RICH_E_INVAL;
  if (ws_bytes < run_ws_bytes(n) || (reinterpret_cast<uintptr_t>(ws) & 255)) return RICH_E_NOMEM;
  if (dt_ws && (reinterpret_cast<uintptr_t>(dt_ws) & 255)) return RICH_E_INVAL;
  char* w = static_cast<char*>(ws);
  RunDesc d = make_desc(m, src, base, out, 0.0, p, w);
  d.h_factor = h_factor;
  if (courant) {
    d.cfl_blocks = reinterpret_cast<double*>(
        w + rich::kHeader + align_up((size_t)n * rich::kRecDoubles * sizeof(double), 256));
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
  constexpr int CPB = rich::kCellThreads / rich::kLpc;
  const int n_ctiles = (d.n + CPB - 1) / CPB;
  // the cell pass writes the point velocities into the records
  hipLaunchKernelGGL(rich::k_clear, dim3(1), dim3(64), 0, st, d.flag, d.cfl_min);
  hipLaunchKernelGGL((rich::k_cell<rich::kLpc, false>), dim3(n_ctiles),
                     dim3(rich::kCellThreads),
                     0, st, d, (const RunDesc*)nullptr, (const int2*)nullptr, n_ctiles,
                     (uint8_t*)nullptr);
  hipLaunchKernelGGL(rich::k_adot, dim3((d.n + rich::kCflThreads - 1) / rich::kCflThreads),
                     dim3(rich::kCflThreads), 0, st, d, adot);
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
  // per-block minima go to the (otherwise idle) record area of the workspace
  hipLaunchKernelGGL(rich::k_cfl, dim3(nb), dim3(rich::kCflThreads), 0, st, d, d.rec);
  hipLaunchKernelGGL(rich::k_cfl_final, dim3(1), dim3(rich::kCflFinalThreads), 0, st,
                     (const double*)d.rec, nb, d.cfl_min, 0.0, (double*)nullptr,
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
  return rich_stage_batch_prepare_tile(n, meshes, src, base, out, h, params, rich::kTile, ws,
                                       ws_bytes, stream, plan);
}

namespace {

// The batched stage's validation and upload; ax, ay (either both null or both
// set) hold each run's per-cell acceleration, null entries meaning none.
// courant: 0 host steps h[r]; 1 each run's step computed in this stage
// (Courant condition on src) and h = h[r] * step; 2 h = h[r] * the step of
// run r that an earlier Courant stage left in the batch workspace dt_ws.
int batch_prepare(int32_t n, const rich_mesh* const* meshes, const rich_state* const* src,
                  const rich_state* const* base, rich_state* const* out, const double* h,
                  const rich_params* const* params, const double* const* ax,
                  const double* const* ay, int32_t tile, void* ws, size_t ws_bytes,
                  void* stream, rich_batch_plan* plan, int courant = 0,
                  const void* dt_ws = nullptr) {
  if (n <= 0 || !meshes || !src || !base || !out || !h || !params || !ws || !plan)
    return RICH_E_INVAL;
  if (courant < 0 || courant > 2 || (courant == 2) != (dt_ws != nullptr)) return RICH_E_INVAL;
  if (dt_ws && (reinterpret_cast<uintptr_t>(dt_ws) & 255)) return RICH_E_INVAL;
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
    // extrapolated fluxes read the step in the cell pass, before this
    // stage's Courant minimum exists
    if (courant == 1 && params[r]->integrator == 1) return RICH_E_INVAL;
    nc[r] = cnt;
  }
  if (reinterpret_cast<uintptr_t>(ws) & 255) return RICH_E_NOMEM;
  BatchLayout L = batch_layout(n, nc.data());
  if (ws_bytes < L.total) return RICH_E_NOMEM;
  char* w = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);

  // descriptors and the three launch plans (cells; fluxes HLLC; fluxes exact)
  constexpr int CPB = rich::kCellThreads / rich::kLpc;
  std::vector<RunDesc> descs(n);
  std::vector<int32_t> plans(3 * (2 * (size_t)n + 1), 0);
  int32_t* pc = plans.data();
  int32_t* pf0 = pc + (2 * n + 1);
  int32_t* pf1 = pf0 + (2 * n + 1);
  std::vector<int32_t> g0, g1;
  for (int32_t r = 0; r < n; ++r) (params[r]->riemann == 1 ? g1 : g0).push_back(r);
  int64_t tc = 0;
  for (int32_t r = 0; r < n; ++r) {
    RunDesc d = make_desc(meshes[r], src[r], base[r], out[r], h[r], params[r], w);
    d.flag = reinterpret_cast<int32_t*>(w + L.flags) + r;
    d.cfl_min = reinterpret_cast<unsigned long long*>(w + L.cfl) + r;
    d.rec = reinterpret_cast<double*>(w + L.rec_off[r]);
    if (courant == 1) {
      d.cfl_blocks = reinterpret_cast<double*>(w + L.cflb);   // indexed by batch cell tile
      d.h_dev = reinterpret_cast<double*>(w + L.dt) + r;
    } else if (courant == 2) {
      d.h_dev = reinterpret_cast<const double*>(static_cast<const char*>(dt_ws) + L.dt) + r;
    }
    if (courant) {
      d.h_factor = h[r];
      d.h = 0.0;
    }
    if (ax) {
      d.ax = ax[r];
      d.ay = ay[r];
    }
    descs[r] = d;
    pc[r] = (int32_t)tc;
    pc[n + 1 + r] = r;
    tc += (nc[r] + CPB - 1) / CPB;
  }
  pc[n] = (int32_t)tc;
  int64_t tf[2] = {0, 0};
  int32_t* pf[2] = {pf0, pf1};
  std::vector<int32_t>* grp[2] = {&g0, &g1};
  for (int k = 0; k < 2; ++k) {
    const int ng = (int)grp[k]->size();
    for (int q = 0; q < ng; ++q) {
      const int32_t r = (*grp[k])[q];
      pf[k][q] = (int32_t)tf[k];
      pf[k][ng + 1 + q] = r;
      tf[k] += (nc[r] + tile - 1) / tile;
    }
    pf[k][ng] = (int32_t)tf[k];
  }
  if (tc > INT32_MAX / 2 || tf[0] > INT32_MAX / 2 || tf[1] > INT32_MAX / 2) return RICH_E_INVAL;

  // tile -> {descriptor index, first tile of its run}: cell tiles, then the
  // flux tiles of the HLLC group, then those of the exact-solver group
  std::vector<int2> tab((size_t)(tc + tf[0] + tf[1]));
  for (int32_t r = 0; r < n; ++r)
    for (int32_t t = pc[r]; t < pc[r + 1]; ++t) tab[(size_t)t] = make_int2(r, pc[r]);
  for (int k = 0, base = (int)tc; k < 2; base += (int)tf[k], ++k) {
    const int ng = (int)grp[k]->size();
    for (int q = 0; q < ng; ++q)
      for (int32_t t = pf[k][q]; t < pf[k][q + 1]; ++t)
        tab[(size_t)base + t] = make_int2(pf[k][ng + 1 + q], pf[k][q]);
  }
  const size_t db = (size_t)n * sizeof(RunDesc), pb = plans.size() * sizeof(int32_t);
  const int up = upload_staged({{w + L.desc, {descs.data(), db}},
                                {w + L.plan, {plans.data(), pb}},
                                {w + L.tab, {tab.data(), tab.size() * sizeof(int2)}}},
                               st);
  if (up) return up;
  plan->table_offset = (int64_t)L.tab;
  plan->serial = register_plan(ws);

  // One block per tile: the hardware dispatcher then balances tiles of
  // uneven cost (shocks, walls) across the CUs as blocks finish, which a
  // persistent grid of resident blocks with a fixed share each does not
  // (2.20 -> 2.11 ms per step for 256 shock tubes of 4.0M cells in all).
  // The kernels still loop over tiles, so any grid is correct.
  plan->flux_tile = tile;
  plan->courant = courant == 1 ? 1 : 0;
  plan->n_runs = n;
  plan->n_cell_tiles = (int32_t)tc;
  plan->n_flux_tiles[0] = (int32_t)tf[0];
  plan->n_flux_tiles[1] = (int32_t)tf[1];
  plan->n_group[0] = (int32_t)g0.size();
  plan->n_group[1] = (int32_t)g1.size();
  plan->grid_cell = (int32_t)tc;
  plan->grid_flux[0] = (int32_t)tf[0];
  plan->grid_flux[1] = (int32_t)tf[1];
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

int rich_stage_batch_prepare_courant(int32_t n, const rich_mesh* const* meshes,
                                     const rich_state* const* src,
                                     const rich_state* const* base, rich_state* const* out,
                                     const double* factor, const rich_params* const* params,
                                     int32_t tile, const void* dt_ws, void* ws, size_t ws_bytes,
                                     void* stream, rich_batch_plan* plan) {
  return batch_prepare(n, meshes, src, base, out, factor, params, nullptr, nullptr, tile, ws,
                       ws_bytes, stream, plan, dt_ws ? 2 : 1, dt_ws);
}

int rich_batch_dt(int32_t n, void* ws, void* stream, double* dt) {
  if (n <= 0 || !ws || !dt) return RICH_E_INVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return RICH_E_INVAL;
  std::vector<int64_t> one(n, 1);
  const BatchLayout L = batch_layout(n, one.data());
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RICH_E_DEVICE;
  if (hipMemcpy(dt, static_cast<char*>(ws) + L.dt, (size_t)n * sizeof(double),
                hipMemcpyDeviceToHost) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}

int rich_stage_batch_launch(const rich_batch_plan* plan, void* ws, void* stream) {
  if (!plan || !ws || plan->n_runs <= 0 || plan->n_cell_tiles <= 0 || plan->grid_cell <= 0)
    return RICH_E_INVAL;
  if (reinterpret_cast<uintptr_t>(ws) & 255) return RICH_E_NOMEM;
  if (!plan_is_current(ws, plan->serial)) return RICH_E_INVAL;
  const int32_t n = plan->n_runs;
  std::vector<int64_t> one(n, 1);
  const BatchLayout L = batch_layout(n, one.data());   // descriptor and plan offsets
  char* w = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const RunDesc* dd = reinterpret_cast<const RunDesc*>(w + L.desc);
  const int32_t* dplan = reinterpret_cast<const int32_t*>(w + L.plan);
  const int32_t* dpc = dplan;   // cell plan: run tile prefix, descriptor indices
  RunDesc dummy;
  std::memset(&dummy, 0, sizeof(dummy));
  hipLaunchKernelGGL(rich::k_clear_batch, dim3((n + 255) / 256), dim3(256), 0, st, dd, n);
  int pcl = prof_begin("k_cell", st);
  const int2* tab = reinterpret_cast<const int2*>(w + plan->table_offset);
  hipLaunchKernelGGL((rich::k_cell<rich::kLpc, true>), dim3(plan->grid_cell),
                     dim3(rich::kCellThreads), 0, st, dummy, dd, tab, plan->n_cell_tiles,
                     (uint8_t*)nullptr);
  prof_end(pcl, st);
  if (plan->courant)   // each run's step from its cell kernel's Courant minima
    hipLaunchKernelGGL(rich::k_cfl_final_batch, dim3(n), dim3(rich::kCflBatchThreads), 0, st,
                       dd, dpc, n);
  int pfl = prof_begin("k_flux", st);
  const int2* ftab = tab + plan->n_cell_tiles;   // flux tiles of group 0, then of group 1
  for (int k = 0; k < 2; ++k) {
    if (plan->n_group[k] > 0 && plan->grid_flux[k] > 0)
      launch_flux_batch(k, plan->flux_tile, plan->grid_flux[k], st, dummy, dd, ftab,
                        plan->n_flux_tiles[k]);
    ftab += plan->n_flux_tiles[k];
  }
  prof_end(pfl, st);
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
  const int rc = batch_prepare(n, meshes, src, base, out, h, params, ax, ay, rich::kTile, ws,
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
                          rich::kTile, ws, ws_bytes, stream, &plan);
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

// Two host blocks copied to device memory through the pinned staging ring of
// the batched stage (enqueued on st; the caller's blocks may be reused at
// once): the batched re-tessellation's descriptors travel this way, so that
// it need not wait on the stream.
namespace rich_host {
int upload2(void* d0, const void* h0, size_t n0, void* d1, const void* h1, size_t n1,
            hipStream_t st) {
  return upload_staged({{d0, {h0, n0}}, {d1, {h1, n1}}}, st);
}
}  // namespace rich_host
