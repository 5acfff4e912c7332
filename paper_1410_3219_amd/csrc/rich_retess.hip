// Device re-tessellation of moved mesh points (section 2.1: the mesh is the
// Voronoi tessellation of its points, rebuilt after every move).
//
// Cell i of the new mesh is the set of points nearer to the new point r_i
// than to each candidate point, within the box for walls (its sides are the
// bisectors with the point's mirror images).  The candidates are the
// neighbours and the neighbours' neighbours of the cell in a previous mesh of
// the same points, each at its nearest periodic image (a periodic box of at
// least 16 cells, whose neighbours enclose each point).  The cell so found
// always contains the true Voronoi cell; it equals it when every true
// neighbour was a candidate.  The kernels certify that (every kept edge seen
// alike by both cells; the areas summing to the box area) instead of
// assuming it, and report failure so that the caller rebuilds on the host.
//
// No polygon is edited: each candidate's bisector is cut down to the part
// that every other candidate allows (two bounds kept as fractions), and the
// candidates with a non-empty part are the cell's edges; their parts' ends
// are the vertices.  The candidates (in LDS: 10 slots per cell, 16 for the
// few cells that need more, and the 4 mirrors of a walled box in registers)
// are the wall mirrors and the previous neighbours; a neighbour's neighbour
// enters only
// when its bisector crosses the cell those give (one further than twice the
// largest vertex distance cannot, and is skipped at once).  The loops over
// candidates have straight-line bodies, so the lanes of a wave stay together.
//
// Most cells keep their neighbours from one step to the next; for those a
// cheaper proof suffices (k_rt_vertex: each vertex of the previous ring's
// consecutive neighbours checked against the other candidates), and the
// clip handles only the cells it leaves.
//
// Pipeline (one launch each, all on the caller's stream):
//   k_rt_begin    clear the result header and the queue counters
//   k_rt_pack     the new points packed in pairs
//   k_rt_vertex   one thread per cell: the cell from its previous ring, when
//                 every vertex passes (else queued for the clip)
//   k_rt_clip     one thread per queued cell: the cell's edges, area, centroid
//                 (twice: 10 candidate slots over the queue, then 16 for the
//                 cells left over)
//   k_rt_classify keep / own each slot by the input stage's rules, check
//                 each kept edge against the neighbour's slot, count
//   k_rt_scan_*   prefix sums of the counts into off[] and eoff[]
//   k_rt_emit     edge records and the CSR entries of both sides of each edge
//   k_rt_end      fold the flags into the sticky word, count the clipped cells
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "rich.h"

namespace retess {

constexpr uint32_t kMask = 0x0FFFFFFFu;
constexpr int kShift = 28;
constexpr int kMaxFan = 20;    // edges of a finished cell (RICH_RETESS_FAN beyond)
static_assert(kMaxFan <= 64, "a kept slot's rank fits the six upper bits of its flag byte");
// Candidate slots of a cell in LDS (neighbours and entrants): the clip runs
// with kSlotsFast of them, which lets a compute unit hold 3 waves per SIMD
// (LDS bound: 2.5 with 12); the few cells that need more are marked and
// clipped again by a second launch with kSlotsWide.
constexpr int kSlotsFast = 10;
constexpr int kSlotsWide = 16;
constexpr int32_t kDegRetry = -1;   // deg[i] of a cell left to the wide launch
constexpr int32_t kDegClip = -2;    // deg[i] of a cell the vertex check left to the clip
// The cells the vertex check leaves are queued for the clip in kSeg
// segments (block b of a run appends to segment b % kSeg), each with its own
// counter on its own 128-byte line, so that the blocks' appends do not all
// meet on one address; the clip then runs dense waves over the queue.
constexpr int kSeg = 64;
constexpr int kSegStride = 32;      // int32 counters 128 bytes apart
constexpr int kRetry = 1 << 30;     // (private bit) more candidates than slots
                               // (a walled box adds its 4 mirrors, held in registers)
constexpr int kRingMax = 64;   // CSR entries read per cell of the previous mesh
constexpr int kThreads = 64;
constexpr int kScanThreads = 1024;
static_assert(kScanThreads % kThreads == 0, "a scan block covers whole cell blocks");
constexpr double kPi = 3.14159265358979323846;
// neighbour codes of the reflecting walls x = x0, x = x1, y = y0, y = y1 in
// the top bits of rich_edge.j (the neighbour is the cell's own mirror image)
constexpr int kWallX0 = 9, kWallX1 = 10, kWallY0 = 11, kWallY1 = 12;

struct Hdr {  // first 64 bytes of the workspace
  int32_t flags, sticky;
  int64_t n_edges, n_csr, n_dropped;
  double area_sum;
  int64_t n_wall;   // kept wall edges (each one CSR entry)
  int64_t n_clip;   // cells the vertex check left to the clip
  int64_t pad;
};
static_assert(sizeof(Hdr) == 64, "result header");

// One classify block's sums: area of its cells, dropped edge slots, kept
// wall edges.  Written per block and reduced in a fixed order by the scan,
// rather than added into the header with atomics (every block's atomics on
// one header line serialised the kernel).
struct CPart {
  double area;
  long long drop, walls, pad;
};

struct Args {
  // previous mesh (candidates)
  const int32_t* p_off;
  const int32_t* p_idx;
  const rich_edge* p_edges;
  int64_t p_n_csr, p_n_edges;
  // new points and output
  const double *x, *y;
  double2* xy;         // [n] the new points packed in pairs (filled by k_rt_pack)
  rich_cell* cells;
  rich_edge* edges;
  int32_t *off, *idx, *eoff;
  int64_t cap_edges, cap_csr;
  // workspace
  Hdr* hdr;
  int32_t* deg;        // [n]
  int32_t* s_nb;       // [n][kMaxFan] generating point: cell | code << 28
  double* s_geo;       // [n][kMaxFan][3] edge length, midpoint x, midpoint y
  uint8_t* s_flag;     // [n][kMaxFan] bit 0 kept, bit 1 owned, bits 2-6 rank among kept
  uint8_t* s_back;     // [n][kMaxFan] owned edge: its slot in the neighbour's row
  int64_t* bsum;       // [2][n_scan_blocks] block totals of kept / owned
  CPart* cpart;        // [cell blocks] classify block sums, reduced by the scan
  int32_t* qcnt;       // [kSeg * kSegStride] queue segment counters (every kSegStride-th)
  int32_t* queue;      // [kSeg][qcap] cells left to the clip
  int32_t qcap;        // capacity of a segment: kThreads * ceil(cell blocks / kSeg)
  // geometry
  double x0, y0, x1, y1, Lx, Ly;
  int32_t n, bc, n_scan_blocks;
};

// Many runs in one launch: run r's descriptor is descs[r]; its blocks of
// kThreads cells are cstart[r] .. cstart[r+1]-1 and its scan blocks of
// kScanThreads cells sstart[r] .. sstart[r+1]-1; hdr_out[r] receives its
// result header at the end.
struct Batch {
  const Args* descs;
  const int32_t* cstart;
  const int32_t* sstart;
  Hdr* hdr_out;
  int32_t* flags_out;   // each run's flags, for rich_retess_batch_flags_async
  int32_t n_runs;
};

// Run of block b in a start table of n_runs + 1 entries.
__device__ __forceinline__ int run_of_block(const int32_t* __restrict__ start, int n_runs, int b) {
  int lo = 0, hi = n_runs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The descriptor of this block's run and the block's index within the run.
template <bool B>
__device__ __forceinline__ const Args& block_run(const Args& one, const int32_t* start,
                                                 const Batch& bt, int& blk) {
  if (!B) {
    blk = blockIdx.x;
    return one;
  }
  const int r = run_of_block(start, bt.n_runs, blockIdx.x);
  blk = blockIdx.x - start[r];
  return bt.descs[r];
}

__device__ __forceinline__ int32_t pack(int cell, int code) {
  return (int32_t)((uint32_t)cell | ((uint32_t)code << kShift));
}
// periodic image shift (sx, sy) in box lengths <-> code 1..8 (0 is no shift)
__device__ __forceinline__ int shift_code(int sx, int sy) {
  const int k = (sx + 1) * 3 + (sy + 1);
  return k < 4 ? k + 1 : k;
}
__device__ __forceinline__ void code_shift(int code, int& sx, int& sy) {
  const int k = code <= 4 ? code - 1 : code;
  sx = k / 3 - 1;
  sy = k % 3 - 1;
}
__device__ __forceinline__ int back_code(int code) { return code == 0 ? 0 : 9 - code; }

// The point p with p.a = |a|^2/2 and p.b = |b|^2/2 (the Voronoi vertex of the
// origin and the points a and b); false unless b is counter-clockwise of a.
__device__ __forceinline__ bool bisector_meet(double ax, double ay, double bx, double by,
                                              double& px, double& py) {
  const double det = ax * by - ay * bx;
  const double ha = 0.5 * (ax * ax + ay * ay), hb = 0.5 * (bx * bx + by * by);
  px = (ha * by - hb * ay) / det;
  py = (ax * hb - ha * bx) / det;
  return det > 0.0;
}

// Neighbour cell of CSR entry k of the previous mesh (-1 if out of range).
__device__ __forceinline__ int prev_neighbour(const Args& a, int k) {
  const int ent = a.p_idx[k];
  const int e = ent >> 1;
  if (ent < 0 || e >= a.p_n_edges) return -1;
  if (ent & 1) return a.p_edges[e].i;
  return (int)((uint32_t)a.p_edges[e].j & kMask);
}

template <bool B>
__global__ void k_rt_begin(Args one, Batch bt) {
  const Args& a = B ? bt.descs[blockIdx.x] : one;
  Hdr* h = a.hdr;
  for (int t = threadIdx.x; t < kSeg; t += blockDim.x) a.qcnt[t * kSegStride] = 0;
  if (threadIdx.x == 0) {
    h->flags = 0;
    h->n_edges = 0;
    h->n_csr = 0;
    h->n_dropped = 0;
    h->area_sum = 0.0;
    h->n_wall = 0;
    h->n_clip = 0;
  }
}

// The new points packed in pairs, so that a candidate's point is one 16-byte
// load (the kernels gather them by cell index many times over).
template <bool B>
__global__ __launch_bounds__(kThreads) void k_rt_pack(Args one, Batch bt) {
  int blk;
  const Args& a = block_run<B>(one, bt.cstart, bt, blk);
  const int i = blk * kThreads + threadIdx.x;
  if (i < a.n) a.xy[i] = make_double2(a.x[i], a.y[i]);
}

template <bool B>
__global__ void k_rt_end(Args one, Batch bt) {
  const Args& a = B ? bt.descs[blockIdx.x] : one;
  Hdr* h = a.hdr;
  // the cells the vertex check queued for the clip (one wave sums the
  // segment counters)
  int c = 0;
  for (int t = threadIdx.x; t < kSeg; t += blockDim.x) c += a.qcnt[t * kSegStride];
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (threadIdx.x == 0) {
    h->n_clip = c;
    h->sticky |= h->flags;
    if (B) {
      bt.hdr_out[blockIdx.x] = *h;
      bt.flags_out[blockIdx.x] = h->flags;
    }
  }
}

// ---------------------------------------------------------------------------
// the cell of one point
// ---------------------------------------------------------------------------
// A lane's candidate slots in LDS: slot u of the lane holds the displacement d
// from r_i to a generating point and its id (cell | code << 28); slot u of
// lane t lives at [u * kThreads + t], so a wave's accesses to one slot are
// consecutive.
// Slots below BASE are not in LDS (a walled box's mirrors, held in
// registers); slot u >= BASE lives at LDS slot u - BASE.
template <int BASE>
struct Slots {
  double* dx;
  double* dy;
  int32_t* id;
  __device__ double& x(int u) const { return dx[(u - BASE) * kThreads]; }
  __device__ double& y(int u) const { return dy[(u - BASE) * kThreads]; }
  __device__ int32_t& n(int u) const { return id[(u - BASE) * kThreads]; }
};


// The part of the bisector of displacement (dux, duy) (the line
// p.d = |d|^2/2, parametrised p(t) = d/2 + t (-duy, dux), t increasing
// counter-clockwise about r_i) that satisfies p.d_v <= |d_v|^2/2 for every
// slot v of mask vm except `self`: [t_lo, t_hi].  The bounds are kept as
// fractions and compared by cross-multiplication, so the loop divides
// nothing.  Returns false when that part is empty, or when a slot of the
// same id comes before `self` (a duplicate); *bounded is false when one end
// is open (the slots do not enclose the point).
template <bool WALLS>
__device__ __forceinline__ bool bisector_part(const Slots<WALLS ? 4 : 0>& S, double wy0,
                                              double wx1, double wy2, double wx3, uint32_t vm,
                                              int nv, int self, double dux, double duy,
                                              int32_t idu, double& tlo, double& thi,
                                              bool& bounded) {
  const double mux = 0.5 * dux, muy = 0.5 * duy;
  const double eux = -duy, euy = dux;
  // No bound yet is hn / hd = +inf and ln / ld = -inf: the first finite
  // bound of each side then wins its comparison (b and a are finite), so
  // no flag tracks whether a side is bounded.
  double ln = -INFINITY, ld = 1.0, hn = INFINITY, hd = 1.0;
  bool empty = false;
  // straight-line bodies (selects, no branches); the mirrors' constraints
  auto cut = [&](double dvx, double dvy, bool act) {
    const double a0 = eux * dvx + euy * dvy;
    const double b0 = 0.5 * (dvx * dvx + dvy * dvy) - (mux * dvx + muy * dvy);
    const double a = act ? a0 : 0.0;
    const double b = act ? b0 : 1.0;
    // a > 0: t <= b / a;  a < 0: t >= (-b) / (-a);  a = 0, b < 0: no t
    const bool up = a > 0.0 && b * hd < hn * a;
    hn = up ? b : hn;
    hd = up ? a : hd;
    const bool dn = a < 0.0 && -b * ld > ln * -a;
    ln = dn ? -b : ln;
    ld = dn ? -a : ld;
    empty = empty || (a == 0.0 && b < 0.0);
  };
  constexpr int BASE = WALLS ? 4 : 0;
  if constexpr (WALLS) {  // the mirrors (0, wy0), (wx1, 0), (0, wy2), (wx3, 0) first
    cut(0.0, wy0, (vm & 1u) && self != 0);
    cut(wx1, 0.0, ((vm >> 1) & 1u) && self != 1);
    cut(0.0, wy2, ((vm >> 2) & 1u) && self != 2);
    cut(wx3, 0.0, ((vm >> 3) & 1u) && self != 3);
  }
  // then the lane's LDS slots
#pragma unroll 4
  for (int v = BASE; v < nv; ++v) {
    const double dvx = S.x(v), dvy = S.y(v);
    const bool use = ((vm >> v) & 1u) && v != self;
    const bool same = use && S.n(v) == idu;
    empty = empty || (same && v < self);
    const bool act = use && !same;
    const double a0 = eux * dvx + euy * dvy;
    const double b0 = 0.5 * (dvx * dvx + dvy * dvy) - (mux * dvx + muy * dvy);
    const double a = act ? a0 : 0.0;
    const double b = act ? b0 : 1.0;
    // a > 0: t <= b / a;  a < 0: t >= (-b) / (-a);  a = 0, b < 0: no t
    const bool up = a > 0.0 && b * hd < hn * a;
    hn = up ? b : hn;
    hd = up ? a : hd;
    const bool dn = a < 0.0 && -b * ld > ln * -a;
    ln = dn ? -b : ln;
    ld = dn ? -a : ld;
    empty = empty || (a == 0.0 && b < 0.0);
  }
  bounded = ln != -INFINITY && hn != INFINITY;
  if (empty || !bounded || !(ln * hd < hn * ld)) return false;
  tlo = ln / ld;
  thi = hn / hd;
  return true;
}

// The cells and points of CSR entries k0 .. k0+CH-1 of the previous mesh
// (those below k1), loaded level by level: entries, then their edges, then
// the points, each level's loads in flight together.  c[m] = -1 for an entry
// past k1, out of range, or naming cell `self` (its point load reads cell 0;
// no edge is read for an entry out of range).
template <int CH>
__device__ __forceinline__ void ring_chunk(const Args& a, int k0, int k1, int self, int* c,
                                           double* cx, double* cy) {
#pragma unroll
  for (int m = 0; m < CH; ++m) c[m] = k0 + m < k1 ? a.p_idx[k0 + m] : -1;
#pragma unroll
  for (int m = 0; m < CH; ++m) {
    const int ent = c[m];
    const int e = ent >> 1;
    int cell = -1;
    if (ent >= 0 && e < a.p_n_edges) {  // no load for an entry out of range
      const rich_edge& pe = a.p_edges[e];
      cell = (ent & 1) ? pe.i : (int)((uint32_t)pe.j & kMask);
    }
    c[m] = (cell < 0 || cell >= a.n || cell == self) ? -1 : cell;
  }
#pragma unroll
  for (int m = 0; m < CH; ++m) {
    const int cell = c[m] < 0 ? 0 : c[m];
    const double2 p = a.xy[cell];
    cx[m] = p.x;
    cy[m] = p.y;
  }
}

// Counter-clockwise order of directions: the upper half-plane (from angle 0
// inclusive) before the lower one, then by the sign of the cross product.
__device__ __forceinline__ bool ccw_before(double ax, double ay, double bx, double by) {
  const int ha = (ay < 0.0 || (ay == 0.0 && ax < 0.0)) ? 1 : 0;
  const int hb = (by < 0.0 || (by == 0.0 && bx < 0.0)) ? 1 : 0;
  if (ha != hb) return ha < hb;
  return ax * by - ay * bx > 0.0;
}

// One thread per cell that the vertex check left (deg = kDegClip; the
// other lanes return at once).  With walls, slots 0-3 hold the point's mirrors
// (they bound it); then come the cell's neighbours in the previous mesh; the
// first pass finds the polygon those allow.  The neighbours' neighbours then enter only when their
// bisector crosses that polygon, into slots that bound nothing; the second
// pass gives the cell, its area, centroid and edges in counter-clockwise
// order.  Every slot v is tried against every slot u (a fixed loop with no
// polygon to edit), so lanes of a wave stay together.  The candidate slots
// are the block's LDS, which sets how many waves a compute unit holds: a cell
// has SL of them, and a walled box's four mirrors (slots 0-3) are held in
// registers, so both kinds of run give SL slots to neighbours and entrants.
// The first launch (SL = kSlotsFast) leaves a cell that needs more slots
// marked (deg = kDegRetry) instead of failing the mesh; the second (WIDE,
// SL = kSlotsWide) clips only those cells, with the same arithmetic, and
// fails the mesh if even that is not enough.  Each launch serves one kind of
// run (a batch of both kinds takes two launches of each), so a run's results
// never depend on the other runs.
template <bool B, bool WALLS, int SL, bool WIDE>
__global__ __launch_bounds__(kThreads) void k_rt_clip(Args one, Batch bt) {
  constexpr int BASE = WALLS ? 4 : 0;   // mirror slots, held in registers
  constexpr int NS = SL + BASE;         // candidates per cell
  static_assert(NS <= 32, "slot masks are 32-bit");
  constexpr int kFull = WIDE ? RICH_RETESS_FAN : kRetry;   // out of slots
  __shared__ double s_dx[SL * kThreads], s_dy[SL * kThreads];
  __shared__ int32_t s_id[SL * kThreads];
  int blk;
  const Args& a = block_run<B>(one, bt.cstart, bt, blk);
  if ((a.bc == (int)RICH_BOUNDARY_PERIODIC) == WALLS) return;  // the other launch's run
  int i;
  if (WIDE) {
    i = blk * kThreads + threadIdx.x;
    if (i >= a.n || a.deg[i] != kDegRetry) return;   // done by an earlier launch
  } else {
    // entry e of queue segment blk % kSeg (e < qcap for every block of the run)
    const int seg = blk % kSeg;
    const int e = (blk / kSeg) * kThreads + (int)threadIdx.x;
    if (e >= a.qcnt[seg * kSegStride]) return;
    i = a.queue[(size_t)seg * a.qcap + e];
    if (i < 0 || i >= a.n || a.deg[i] != kDegClip) return;
  }
  const Slots<BASE> S{s_dx + threadIdx.x, s_dy + threadIdx.x, s_id + threadIdx.x};
  // a walled box: the point's mirrors across the walls y0, x1, y1, x0 (slots
  // 0-3) are the displacements (0, wy0), (wx1, 0), (0, wy2), (wx3, 0)
  double wy0 = 0.0, wx1 = 0.0, wy2 = 0.0, wx3 = 0.0;
  const double xi = a.x[i], yi = a.y[i];
  int bad = 0;
  constexpr bool periodic = !WALLS;
  // live slots are 0 .. nv-1; vm marks those that hold a candidate
  int nv = 0;
  uint32_t vm = 0u;
  if (periodic) {
    // no bounds: the neighbours enclose the point (a cell they leave open
    // is reported, and rebuilt on the host)
    if (!(xi >= a.x0 && xi < a.x1 && yi >= a.y0 && yi < a.y1)) bad |= RICH_RETESS_POINT;
  } else {
    if (!(xi > a.x0 && xi < a.x1 && yi > a.y0 && yi < a.y1)) bad |= RICH_RETESS_POINT;
    // the point's mirrors across the walls y0, x1, y1, x0
    wy0 = 2.0 * (a.y0 - yi);
    wx1 = 2.0 * (a.x1 - xi);
    wy2 = 2.0 * (a.y1 - yi);
    wx3 = 2.0 * (a.x0 - xi);
    nv = 4;
    vm = 0xFu;
  }
  // candidate u: displacement and id (with walls, u < 4 is a mirror)
  auto cand = [&](int u, double& dx, double& dy) -> int32_t {
    if (WALLS && u < 4) {
      dx = u == 1 ? wx1 : (u == 3 ? wx3 : 0.0);
      dy = u == 0 ? wy0 : (u == 2 ? wy2 : 0.0);
      return pack(i, u == 0 ? kWallY0 : u == 1 ? kWallX1 : u == 2 ? kWallY1 : kWallX0);
    }
    dx = S.x(u);
    dy = S.y(u);
    return S.n(u);
  };

  // displacement of cell c from r_i (nearest periodic image) and its id
  auto displacement = [&](int c, double xc, double yc, double& dx, double& dy) -> int32_t {
    dx = xc - xi;
    dy = yc - yi;
    int code = 0;
    if (periodic) {
      int sx = 0, sy = 0;
      if (dx > 0.5 * a.Lx) { dx -= a.Lx; sx = -1; } else if (dx < -0.5 * a.Lx) { dx += a.Lx; sx = 1; }
      if (dy > 0.5 * a.Ly) { dy -= a.Ly; sy = -1; } else if (dy < -0.5 * a.Ly) { dy += a.Ly; sy = 1; }
      if (sx != 0 || sy != 0) code = shift_code(sx, sy);
    }
    return pack(c, code);
  };

  int k0 = 0, k1 = 0;
  if (!bad) {
    k0 = a.p_off[i];
    k1 = a.p_off[i + 1];
    if (k0 < 0 || k1 < k0 || k1 > a.p_n_csr) {
      bad |= RICH_RETESS_CLIP;
      k1 = k0;
    } else if (k1 - k0 > NS - nv) {
      bad |= kFull;
      k1 = k0;
    }
  }
  constexpr int CH = 8;  // candidates loaded together
  for (int k = k0; k < k1; k += CH) {
    int c[CH];
    double cx[CH], cy[CH];
    ring_chunk<CH>(a, k, k1, i, c, cx, cy);
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      if (c[m] < 0) continue;
      double dx, dy;
      S.n(nv) = displacement(c[m], cx[m], cy[m], dx, dy);
      S.x(nv) = dx;
      S.y(nv) = dy;
      vm |= 1u << nv;
      ++nv;
    }
  }

  // first pass: the polygon of the bounds and the first ring, and the
  // largest distance of its vertices
  uint32_t em = 0;
  double r2 = 0.0;
  if (!bad) {
    for (int u = 0; u < nv; ++u) {
      if (!((vm >> u) & 1u)) continue;
      double tlo, thi;
      bool bounded;
      double dux, duy;
      const int32_t idu = cand(u, dux, duy);
      if (bisector_part<WALLS>(S, wy0, wx1, wy2, wx3, vm, nv, u, dux, duy, idu, tlo, thi, bounded)) {
        em |= 1u << u;
        const double px = 0.5 * dux - thi * duy, py = 0.5 * duy + thi * dux;
        r2 = fmax(r2, px * px + py * py);
      } else if (!bounded) {
        bad |= RICH_RETESS_CLIP;
      }
    }
  }

  // second ring: a candidate enters when its bisector crosses the polygon
  // (a candidate further than twice the largest vertex distance cannot).
  // The cheap tests (distance, already a slot) run as the candidates are
  // loaded; the survivors wait in a short queue and meet the polygon test
  // in their order when the queue is full or the ring is done, so that the
  // wave runs the costly test a few times per cell instead of once per
  // candidate position (whichever lane of the wave needed it).  Candidates
  // meet the test in the same order, against the same slots, as one by one.
  constexpr int QN = 4;   // 2, 6 and 8 measured slower
  double qx[QN], qy[QN];
  int32_t qid[QN];
  int qn = 0;
  auto flush = [&]() {
#pragma unroll
    for (int p = 0; p < QN; ++p) {
      if (p >= qn || bad) continue;
      double tlo, thi;
      bool bounded;
      if (!bisector_part<WALLS>(S, wy0, wx1, wy2, wx3, vm, nv, -1, qx[p], qy[p], qid[p], tlo,
                                thi, bounded))
        continue;
      // a new slot, else one whose bisector bounds nothing (it stays
      // redundant as candidates are added)
      int u = nv;
      if (nv < NS) {
        ++nv;
      } else {
        // (a mirror is never reused)
        const uint32_t usable = ~em & ((1u << NS) - 1u) & ~((1u << BASE) - 1u);
        if (usable == 0u) {
          bad |= kFull;
          continue;
        }
        u = __ffs(usable) - 1;
      }
      S.x(u) = qx[p];
      S.y(u) = qy[p];
      S.n(u) = qid[p];
      vm |= 1u << u;
      em |= 1u << u;   // holds a cutting candidate now: not reusable
    }
    qn = 0;
  };
  for (int k = k0; k < k1 && !bad; ++k) {
    const int j = prev_neighbour(a, k);
    if (j < 0 || j >= a.n || j == i) continue;
    const int l0 = a.p_off[j], l1 = a.p_off[j + 1];
    if (l0 < 0 || l1 < l0 || l1 > a.p_n_csr || l1 - l0 > kRingMax) {
      bad |= RICH_RETESS_CLIP;
      break;
    }
    for (int l = l0; l < l1 && !bad; l += CH) {
      int cc[CH];
      double ccx[CH], ccy[CH];
      ring_chunk<CH>(a, l, l1, i, cc, ccx, ccy);
      for (int m = 0; m < CH; ++m) {
        if (cc[m] < 0) continue;
        double dx, dy;
        const int32_t id = displacement(cc[m], ccx[m], ccy[m], dx, dy);
        if (4.0 * r2 <= dx * dx + dy * dy) continue;
        // (over every slot, the loads issued together; vm marks the live ones)
        bool known = false;
#pragma unroll
        for (int v = BASE; v < NS; ++v) known = known || (v < nv && ((vm >> v) & 1u) && S.n(v) == id);
#pragma unroll
        for (int p = 0; p < QN; ++p) known = known || (p < qn && qid[p] == id);
        if (known) continue;
#pragma unroll
        for (int p = 0; p < QN; ++p) {
          if (p == qn) {
            qx[p] = dx;
            qy[p] = dy;
            qid[p] = id;
          }
        }
        if (++qn == QN) flush();
      }
    }
  }
  if (!bad) flush();

  rich_cell cr;
  cr.px = xi;
  cr.py = yi;
  cr.pad = 0.0;
  if (bad) {
    // out of slots alone: left to the wide launch; anything else fails the mesh
    const int pub = bad & ~kRetry;
    if (pub) atomicOr(&a.hdr->flags, pub);
    a.deg[i] = pub ? 0 : kDegRetry;
    cr.area = 0.0;
    cr.sx = xi;
    cr.sy = yi;
    a.cells[i] = cr;
    return;
  }
  // second pass: each candidate's part of its bisector.  A live one (an
  // edge) is written at once, at its counter-clockwise rank among all the
  // candidates (same direction: by slot), and its triangle with the point
  // is added to the shoelace sums in slot order; the positions left by
  // candidates that bound nothing are closed up afterwards, which leaves
  // the live ones in counter-clockwise order.
  uint32_t fm = 0, holes = 0;
  double A2 = 0.0, cx = 0.0, cy = 0.0;
  const size_t s0 = (size_t)i * kMaxFan;
  for (int u = 0; u < nv; ++u) {
    if (!((vm >> u) & 1u)) continue;
    double dux, duy;
    const int32_t idu = cand(u, dux, duy);
    int rank = 0;
    for (int v = 0; v < nv; ++v) {
      if (!((vm >> v) & 1u) || v == u) continue;
      double vx, vy;
      cand(v, vx, vy);
      rank += (ccw_before(vx, vy, dux, duy) || (v < u && !ccw_before(dux, duy, vx, vy))) ? 1 : 0;
    }
    double tlo, thi;
    bool bounded;
    if (!bisector_part<WALLS>(S, wy0, wx1, wy2, wx3, vm, nv, u, dux, duy, idu, tlo, thi, bounded)) {
      if (!bounded) bad |= RICH_RETESS_CLIP;
      holes |= 1u << rank;
      continue;
    }
    fm |= 1u << u;
    const double ux = 0.5 * dux - tlo * duy, uy = 0.5 * duy + tlo * dux;
    const double wx = 0.5 * dux - thi * duy, wy = 0.5 * duy + thi * dux;
    const double c = ux * wy - uy * wx;
    A2 += c;
    cx += (ux + wx) * c;
    cy += (uy + wy) * c;
    const double ex = wx - ux, ey = wy - uy;
    a.s_nb[s0 + rank] = idu;   // rank < number of candidates <= NS < kMaxFan
    double* g = a.s_geo + 3 * (s0 + rank);
    g[0] = sqrt(ex * ex + ey * ey);
    g[1] = xi + 0.5 * (ux + wx);
    g[2] = yi + 0.5 * (uy + wy);
  }
  const int deg = __popc(fm);
  if (deg < 3 || deg > kMaxFan) bad |= deg > kMaxFan ? RICH_RETESS_FAN : RICH_RETESS_CLIP;
  if (!bad && holes != 0u) {
    __threadfence_block();  // this lane's row writes above are read back below
    const int total = __popc(vm);
    for (int p = 0, q = 0; p < total; ++p) {
      if ((holes >> p) & 1u) continue;
      if (q != p) {
        a.s_nb[s0 + q] = a.s_nb[s0 + p];
        const double* g = a.s_geo + 3 * (s0 + p);
        double* h = a.s_geo + 3 * (s0 + q);
        const double g0 = g[0], g1 = g[1], g2 = g[2];
        h[0] = g0;
        h[1] = g1;
        h[2] = g2;
      }
      ++q;
    }
  }
  if (bad) {
    atomicOr(&a.hdr->flags, bad);
    a.deg[i] = 0;
    cr.area = 0.0;
    cr.sx = xi;
    cr.sy = yi;
    a.cells[i] = cr;
    return;
  }
  a.deg[i] = deg;
  cr.area = 0.5 * A2;
  cr.sx = xi + cx / (3.0 * A2);
  cr.sy = yi + cy / (3.0 * A2);
  a.cells[i] = cr;
}

// ---------------------------------------------------------------------------
// the cell of one point when it keeps its previous neighbours
// ---------------------------------------------------------------------------
// Under the small moves of a time step most cells keep their neighbours, and
// the previous mesh lists them counter-clockwise.  Then the cell's vertices
// are the points equidistant from r_i and two consecutive neighbours, and
// the cell is proved by checking each vertex against every other candidate
// (one dot product), instead of cutting every bisector by every other one.
// The proof holds in exact arithmetic when every consecutive pair turns
// counter-clockwise by less than half a turn (and more than kVertexSin), the
// ring winds once, and every vertex lies inside every other candidate's half
// plane by a margin far above the rounding of the test (kVertexMargin of the
// candidate's half squared distance plus the largest squared vertex distance;
// with one margin for all vertices, the vertex of largest projection on a
// candidate decides for all of them): the polygon is then the intersection of the
// candidates' half planes, and its edges (all of positive length, well above
// the input stage's cut for dropping one) are the ring's neighbours.  The
// candidates are the clip's: the mirrors of a walled box, the ring, and the
// neighbours' neighbours that could reach a vertex.  A cell that fails any
// of these tests (a new neighbour, a lost one, a near-degenerate vertex, a
// ring longer than kRingFast or next to a wall) is queued for the clip
// launches (deg = kDegClip), which decide every case.
constexpr int kRingFast = 8;            // ring entries held in registers
constexpr double kVertexMargin = 1e-9;  // relative margin of every vertex test
constexpr double kVertexSin = 0.05;     // least sine of a consecutive pair's angle

// (launch bounds for 4 waves per SIMD: a few registers spill, which costs
// less than the latency 3 waves leave exposed)
template <bool B, bool WALLS>
__global__ __launch_bounds__(kThreads, 4) void k_rt_vertex(Args one, Batch bt) {
  constexpr int N = kRingFast;
  int blk;
  const Args& a = block_run<B>(one, bt.cstart, bt, blk);
  const int i = blk * kThreads + threadIdx.x;
  if (i >= a.n) return;
  if ((a.bc == (int)RICH_BOUNDARY_PERIODIC) == WALLS) return;  // the other launch's run
  const double xi = a.x[i], yi = a.y[i];
  bool ok = WALLS ? (xi > a.x0 && xi < a.x1 && yi > a.y0 && yi < a.y1)
                  : (xi >= a.x0 && xi < a.x1 && yi >= a.y0 && yi < a.y1);
  int k0 = a.p_off[i], k1 = a.p_off[i + 1];
  const int n = k1 - k0;
  ok = ok && k0 >= 0 && n >= 3 && n <= N && k1 <= a.p_n_csr;
  if (!ok) k1 = k0;   // (nothing of the ring is loaded)

  // displacement of cell c from r_i (nearest periodic image) and its id.
  // The image is sought only when some lane of the wave needs it (a wave
  // holds nearby cells, so all but the waves at the box's edges skip it);
  // otherwise the plain difference is that image and its code is 0.
  auto displacement = [&](int c, double xc, double yc, double& dx, double& dy) -> int32_t {
    dx = xc - xi;
    dy = yc - yi;
    int code = 0;
    if (!WALLS && __any(fabs(dx) > 0.5 * a.Lx || fabs(dy) > 0.5 * a.Ly)) {
      int sx = 0, sy = 0;
      if (dx > 0.5 * a.Lx) { dx -= a.Lx; sx = -1; } else if (dx < -0.5 * a.Lx) { dx += a.Lx; sx = 1; }
      if (dy > 0.5 * a.Ly) { dy -= a.Ly; sy = -1; } else if (dy < -0.5 * a.Ly) { dy += a.Ly; sy = 1; }
      if (sx != 0 || sy != 0) code = shift_code(sx, sy);
    }
    return pack(c, code);
  };

  // the ring: displacements, half squared lengths, ids (a wall entry or an
  // entry out of range fails the cell)
  int c[N];
  double dx[N], dy[N], h[N];
  int32_t id[N];
  {
    double cx[N], cy[N];
    ring_chunk<N>(a, k0, k1, i, c, cx, cy);
#pragma unroll
    for (int m = 0; m < N; ++m) {
      ok = ok && (m >= n || c[m] >= 0);
      id[m] = displacement(c[m] < 0 ? 0 : c[m], cx[m], cy[m], dx[m], dy[m]);
      h[m] = 0.5 * (dx[m] * dx[m] + dy[m] * dy[m]);
    }
  }

  // vertex k: equidistant from r_i, ring entries k and k+1 (cyclically)
  double vx[N], vy[N];
  double r2 = 0.0;
  int wraps = 0, start = 0;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const bool last = k + 1 >= n;
    const double ax = dx[k], ay = dy[k], ha = h[k];
    const double bx = last ? dx[0] : dx[k + 1 < N ? k + 1 : 0];
    const double by = last ? dy[0] : dy[k + 1 < N ? k + 1 : 0];
    const double hb = last ? h[0] : h[k + 1 < N ? k + 1 : 0];
    const double det = ax * by - ay * bx;
    // det = |a| |b| sin(angle); a turn of less than half a turn, by a margin
    const bool turn = det > 0.0 && det * det > (4.0 * kVertexSin * kVertexSin) * ha * hb;
    const double inv = 1.0 / (turn ? det : 1.0);
    vx[k] = (ha * by - hb * ay) * inv;
    vy[k] = (ax * hb - ha * bx) * inv;
    const double q = vx[k] * vx[k] + vy[k] * vy[k];
    if (k < n) {
      ok = ok && turn;
      r2 = fmax(r2, q);
      // the ring winds once: exactly one step passes angle 0
      if (ccw_before(bx, by, ax, ay)) {
        ++wraps;
        start = last ? 0 : k + 1;
      }
    }
  }
  ok = ok && wraps == 1;

  // every vertex inside every other candidate's half plane, by the margin
  const double mr = kVertexMargin * r2;
  auto inside = [&](int k, double ux, double uy, double hu) -> bool {
    return hu - (vx[k] * ux + vy[k] * uy) > kVertexMargin * hu + mr;
  };
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int v = 0; v < N; ++v) {
      // not the vertex's own two entries (k and k+1, cyclically)
      const bool own = v == k || (v == k + 1 && k + 1 < n) || (v == 0 && k + 1 == n);
      if (k < n && v < n && !own) ok = ok && inside(k, dx[v], dy[v], h[v]);
    }
  }
  if (WALLS) {
    // the point's mirrors across the walls y0, x1, y1, x0
    const double wy0 = 2.0 * (a.y0 - yi), wx1 = 2.0 * (a.x1 - xi);
    const double wy2 = 2.0 * (a.y1 - yi), wx3 = 2.0 * (a.x0 - xi);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      if (k < n) {
        ok = ok && inside(k, 0.0, wy0, 0.5 * wy0 * wy0) && inside(k, wx1, 0.0, 0.5 * wx1 * wx1) &&
             inside(k, 0.0, wy2, 0.5 * wy2 * wy2) && inside(k, wx3, 0.0, 0.5 * wx3 * wx3);
      }
    }
  }

  // the neighbours' neighbours: one nearer than twice the largest vertex
  // distance (with the margin) that is not in the ring must leave every
  // vertex inside its half plane
  const double reach = 4.0 * r2 * (1.0 + kVertexMargin);
  for (int m = 0; m < n && ok; ++m) {
    int j = c[0];
#pragma unroll
    for (int t = 1; t < N; ++t) j = t == m ? c[t] : j;
    const int l0 = a.p_off[j], l1 = a.p_off[j + 1];
    if (l0 < 0 || l1 < l0 || l1 > a.p_n_csr || l1 - l0 > kRingMax) {
      ok = false;
      break;
    }
    constexpr int CH = 8;
    for (int l = l0; l < l1 && ok; l += CH) {
      int cc[CH];
      double ccx[CH], ccy[CH];
      ring_chunk<CH>(a, l, l1, i, cc, ccx, ccy);
#pragma unroll
      for (int t = 0; t < CH; ++t) {
        if (cc[t] < 0) continue;
        double ux, uy;
        const int32_t idu = displacement(cc[t], ccx[t], ccy[t], ux, uy);
        const double d2 = ux * ux + uy * uy;
        if (!(d2 < reach)) continue;
        bool known = false;
#pragma unroll
        for (int v = 0; v < N; ++v) known = known || (v < n && id[v] == idu);
        if (known) continue;
        // the largest projection of a vertex on the candidate
        double p = vx[0] * ux + vy[0] * uy;
#pragma unroll
        for (int k = 1; k < N; ++k)
          if (k < n) p = fmax(p, vx[k] * ux + vy[k] * uy);
        const double hu = 0.5 * d2;
        ok = ok && hu - p > kVertexMargin * hu + mr;
      }
    }
  }

  // a failing cell is appended to the block's queue segment (one atomic
  // per wave; a block is one wave)
  static_assert(kThreads == 64, "a block is one wave");
  const unsigned long long fails = __ballot(!ok);
  if (fails != 0ull) {
    const int lane = (int)threadIdx.x;
    const int leader = __ffsll((long long)__ballot(true)) - 1;
    const int seg = blk % kSeg;
    int base = 0;
    if (lane == leader) base = atomicAdd(&a.qcnt[seg * kSegStride], __popcll(fails));
    base = __shfl(base, leader);
    if (!ok) {
      a.queue[(size_t)seg * a.qcap + base + __popcll(fails & ((1ull << lane) - 1ull))] = i;
      a.deg[i] = kDegClip;
      return;
    }
  }
  // edge k runs from vertex k-1 to vertex k; its slot is its counter-
  // clockwise rank, counted from the entry of least angle
  double pvx = vx[0], pvy = vy[0];
#pragma unroll
  for (int t = 1; t < N; ++t) {
    pvx = t == n - 1 ? vx[t] : pvx;
    pvy = t == n - 1 ? vy[t] : pvy;
  }
  double A2 = 0.0, sx = 0.0, sy = 0.0;
  const size_t s0 = (size_t)i * kMaxFan;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k < n) {
      const double ux = pvx, uy = pvy, wx = vx[k], wy = vy[k];
      const double cr = ux * wy - uy * wx;
      A2 += cr;
      sx += (ux + wx) * cr;
      sy += (uy + wy) * cr;
      const double ex = wx - ux, ey = wy - uy;
      const int rank = k >= start ? k - start : k - start + n;
      a.s_nb[s0 + rank] = id[k];
      double* g = a.s_geo + 3 * (s0 + rank);
      g[0] = sqrt(ex * ex + ey * ey);
      g[1] = xi + 0.5 * (ux + wx);
      g[2] = yi + 0.5 * (uy + wy);
      pvx = wx;
      pvy = wy;
    }
  }
  a.deg[i] = n;
  rich_cell cr;
  cr.px = xi;
  cr.py = yi;
  cr.pad = 0.0;
  cr.area = 0.5 * A2;
  cr.sx = xi + sx / (3.0 * A2);
  cr.sy = yi + sy / (3.0 * A2);
  a.cells[i] = cr;
}

// ---------------------------------------------------------------------------
// keep / own, certification, counts.  This kernel and the two emit kernels
// give each cell a group of kGroup lanes, one per slot (a cell's slots are
// contiguous, so a group's loads and stores are too, and the lanes of a
// wave do like work); a block still covers kThreads cells.
// ---------------------------------------------------------------------------
constexpr int kGroup = 8;
constexpr int kGroupThreads = kThreads * kGroup;
static_assert(64 % kGroup == 0, "groups do not straddle waves");

// The group's bits of a wave-wide ballot.
__device__ __forceinline__ uint32_t group_bits(bool v) {
  const unsigned long long m = __ballot(v);
  const int first = (int)(threadIdx.x & 63) & ~(kGroup - 1);
  return (uint32_t)(m >> first) & ((1u << kGroup) - 1u);
}

template <bool B>
__global__ __launch_bounds__(kGroupThreads) void k_rt_classify(Args one, Batch bt) {
  int blk;
  const Args& a = block_run<B>(one, bt.cstart, bt, blk);
  constexpr int NW = kGroupThreads / 64;
  __shared__ double s_area[NW];
  __shared__ long long s_drop[NW], s_wall[NW];
  const int l = (int)threadIdx.x % kGroup;
  const int i = blk * kThreads + (int)threadIdx.x / kGroup;
  double area = 0.0;
  long long drop = 0, walls = 0;
  int n_keep = 0, n_own = 0, bad = 0;
  if (i < a.n) {
    const int d = a.deg[i];
    const double Ai = a.cells[i].area;
    if (l == 0) {
      area = Ai;
      if (d == 0 || !(Ai > 0.0)) bad |= RICH_RETESS_CLIP;
    }
    const double Ri = sqrt(Ai / kPi);
    const size_t s0 = (size_t)i * kMaxFan;
    int kept_before = 0;   // kept slots of the group's earlier rounds
    for (int q = l; q < d; q += kGroup) {
      const int32_t id = a.s_nb[s0 + q];
      const int j = (int)((uint32_t)id & kMask);
      const int code = (int)((uint32_t)id >> kShift);
      const double Rj = sqrt(a.cells[j].area / kPi);
      const double* g = a.s_geo + 3 * (s0 + q);
      const double L = g[0];
      const bool keep = L >= 1e-12 * 0.5 * (Ri + Rj);
      bool own;
      if (code >= kWallX0) own = true;
      else if (j != i) own = i < j;
      else own = code >= 5;
      // a kept slot's rank among the cell's kept slots (its CSR position)
      const uint32_t km = group_bits(keep);
      const int rank = kept_before + __popc(km & ((1u << l) - 1u));
      kept_before += __popc(km);
      a.s_flag[s0 + q] = (uint8_t)((keep ? 1 : 0) | (keep && own ? 2 : 0) | (rank << 2));
      if (!keep) {
        ++drop;
        continue;
      }
      ++n_keep;
      if (own) ++n_own;
      if (code >= kWallX0) {
        ++walls;
        continue;
      }
      // the owner finds the same edge in the neighbour's slots; that every
      // other kept slot is such a match follows from the counts (checked
      // once they are summed: kept = 2 owned - walls)
      if (!own) continue;
      const int32_t want = pack(i, back_code(code));
      const int dj = a.deg[j];
      const size_t t0 = (size_t)j * kMaxFan;
      // the first match among the neighbour's slots: its first eight in two
      // 16-byte loads (a row holds kMaxFan slots, so they are in bounds;
      // those past its degree are ignored), the rest one at a time
      static_assert(kMaxFan >= 8 && (kMaxFan * 4) % 16 == 0, "rows of 16-byte chunks");
      const int4* rowv = reinterpret_cast<const int4*>(a.s_nb + t0);
      const int4 v0 = rowv[0], v1 = rowv[1];
      const int32_t ids[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
      int found = -1;
#pragma unroll
      for (int t = 7; t >= 0; --t)
        if (t < dj && ids[t] == want) found = t;
      for (int t = 8; found < 0 && t < dj; ++t)
        if (a.s_nb[t0 + t] == want) found = t;
      if (found < 0) { bad |= RICH_RETESS_ASYM; continue; }
      a.s_back[s0 + q] = (uint8_t)found;
      const double* gj = a.s_geo + 3 * (t0 + found);
      const double Lj = gj[0];
      double fxj = gj[1], fyj = gj[2];
      if (code != 0) {  // the neighbour sees the edge one image away
        int sx, sy;
        code_shift(code, sx, sy);
        fxj += sx * a.Lx;
        fyj += sy * a.Ly;
      }
      const double tol = 1e-9 * (Ri + Rj);
      if (!(Lj >= 1e-12 * 0.5 * (Ri + Rj)) || fabs(L - Lj) > tol ||
          fabs(g[1] - fxj) > tol || fabs(g[2] - fyj) > tol)
        bad |= RICH_RETESS_ASYM;
    }
  }
  // the cell's counts and flags over its group
  for (int o = kGroup / 2; o > 0; o >>= 1) {
    n_keep += __shfl_xor(n_keep, o);
    n_own += __shfl_xor(n_own, o);
    bad |= __shfl_xor(bad, o);
  }
  if (i < a.n && l == 0) {
    if (bad) atomicOr(&a.hdr->flags, bad);
    a.off[i + 1] = n_keep;  // counts; the scan makes them offsets
    a.eoff[i + 1] = n_own;
  }
  // block sums of the areas and of the dropped edges
  for (int o = 32; o > 0; o >>= 1) {
    area += __shfl_xor(area, o);
    drop += __shfl_xor(drop, o);
    walls += __shfl_xor(walls, o);
  }
  if ((threadIdx.x & 63) == 0) {
    s_area[threadIdx.x >> 6] = area;
    s_drop[threadIdx.x >> 6] = drop;
    s_wall[threadIdx.x >> 6] = walls;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    CPart c;
    c.area = 0.0;
    c.drop = 0;
    c.walls = 0;
    c.pad = 0;
    for (int w = 0; w < NW; ++w) {
      c.area += s_area[w];
      c.drop += s_drop[w];
      c.walls += s_wall[w];
    }
    a.cpart[blk] = c;
  }
}

// ---------------------------------------------------------------------------
// prefix sums of the kept / owned counts (in place in off[1..n], eoff[1..n])
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_scan2(int& v0, int& v1, int* s0, int* s1, int& tot0,
                                            int& tot1) {
  // inclusive scan over the block of two values per thread
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int u0 = __shfl_up(v0, o), u1 = __shfl_up(v1, o);
    if (lane >= o) { v0 += u0; v1 += u1; }
  }
  if (lane == 63) { s0[wv] = v0; s1[wv] = v1; }
  __syncthreads();
  if (wv == 0) {
    constexpr int NW = kScanThreads / 64;
    int w0 = lane < NW ? s0[lane] : 0, w1 = lane < NW ? s1[lane] : 0;
    for (int o = 1; o < NW; o <<= 1) {
      const int u0 = __shfl_up(w0, o), u1 = __shfl_up(w1, o);
      if (lane >= o) { w0 += u0; w1 += u1; }
    }
    if (lane < NW) { s0[lane] = w0; s1[lane] = w1; }
  }
  __syncthreads();
  if (wv > 0) { v0 += s0[wv - 1]; v1 += s1[wv - 1]; }
  tot0 = s0[kScanThreads / 64 - 1];
  tot1 = s1[kScanThreads / 64 - 1];
  __syncthreads();
}

template <bool B>
__global__ __launch_bounds__(kScanThreads) void k_rt_scan_local(Args one, Batch bt) {
  int blk;
  const Args& a = block_run<B>(one, bt.sstart, bt, blk);
  __shared__ int s0[kScanThreads / 64], s1[kScanThreads / 64];
  const int i = blk * kScanThreads + threadIdx.x;
  int v0 = i < a.n ? a.off[i + 1] : 0;
  int v1 = i < a.n ? a.eoff[i + 1] : 0;
  int t0, t1;
  block_scan2(v0, v1, s0, s1, t0, t1);
  if (i < a.n) {
    a.off[i + 1] = v0;
    a.eoff[i + 1] = v1;
  }
  if (threadIdx.x == 0) {
    a.bsum[blk] = t0;
    a.bsum[a.n_scan_blocks + blk] = t1;
  }
  // the sums of the classify blocks of this block's cells, in order, into
  // the first of them (the scan of the block totals reads only those)
  constexpr int CPB = kScanThreads / kThreads;
  const int nc = (a.n + kThreads - 1) / kThreads;
  if (threadIdx.x == 0) {
    CPart c = a.cpart[blk * CPB];
    for (int t = 1; t < CPB && blk * CPB + t < nc; ++t) {
      const CPart p = a.cpart[blk * CPB + t];
      c.area += p.area;
      c.drop += p.drop;
      c.walls += p.walls;
    }
    a.cpart[blk * CPB] = c;
  }
}

// one block: exclusive scan of the block totals, totals and the checks that
// need every cell (areas, capacities)
template <bool B>
__global__ __launch_bounds__(kScanThreads) void k_rt_scan_blocks(Args one, Batch bt) {
  const Args& a = B ? bt.descs[blockIdx.x] : one;
  __shared__ long long s0[kScanThreads], s1[kScanThreads];
  constexpr int NW = kScanThreads / 64;
  __shared__ double s_area[NW];
  __shared__ long long s_drop[NW], s_wall[NW];
  // the classify blocks' sums (those of each scan block gathered by
  // k_rt_scan_local): each thread every kScanThreads-th scan block, a fixed
  // xor tree over each wave, then thread 0 over the waves in order (a fixed
  // order throughout, so the area sum is reproducible)
  const int nb_scan = a.n_scan_blocks;
  {
    constexpr int CPB = kScanThreads / kThreads;   // classify blocks per scan block
    double ar = 0.0;
    long long dr = 0, wl = 0;
    for (int c = threadIdx.x; c < nb_scan; c += kScanThreads) {
      const CPart p = a.cpart[c * CPB];
      ar += p.area;
      dr += p.drop;
      wl += p.walls;
    }
    for (int o = 32; o > 0; o >>= 1) {
      ar += __shfl_xor(ar, o);
      dr += __shfl_xor(dr, o);
      wl += __shfl_xor(wl, o);
    }
    if ((threadIdx.x & 63) == 0) {
      s_area[threadIdx.x >> 6] = ar;
      s_drop[threadIdx.x >> 6] = dr;
      s_wall[threadIdx.x >> 6] = wl;
    }
  }
  const int nb = a.n_scan_blocks;
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
  long long c0 = 0, c1 = 0;
  for (int b = b0; b < b1; ++b) {
    c0 += a.bsum[b];
    c1 += a.bsum[nb + b];
  }
  s0[threadIdx.x] = c0;
  s1[threadIdx.x] = c1;
  __syncthreads();
  if (threadIdx.x == 0) {
    double ar = 0.0;
    long long dr = 0, wl = 0;
    for (int w = 0; w < NW; ++w) {
      ar += s_area[w];
      dr += s_drop[w];
      wl += s_wall[w];
    }
    a.hdr->area_sum = ar;
    a.hdr->n_dropped = dr;
    a.hdr->n_wall = wl;
  }
  // serial over the 1024 chunk sums by one thread: 1024 additions
  if (threadIdx.x == 0) {
    long long r0 = 0, r1 = 0;
    for (int t = 0; t < kScanThreads; ++t) {
      const long long u0 = s0[t], u1 = s1[t];
      s0[t] = r0;
      s1[t] = r1;
      r0 += u0;
      r1 += u1;
    }
    Hdr* h = a.hdr;
    h->n_csr = r0;
    h->n_edges = r1;
    int f = 0;
    if (r0 > a.cap_csr || r1 > a.cap_edges) f |= RICH_RETESS_CAP;
    if (r0 != 2 * r1 - h->n_wall) f |= RICH_RETESS_ASYM;   // an unmatched kept slot
    const double box = a.Lx * a.Ly;
    if (!(fabs(h->area_sum - box) <= 1e-10 * box)) f |= RICH_RETESS_AREA;
    if (f) h->flags |= f;
  }
  __syncthreads();
  long long r0 = s0[threadIdx.x], r1 = s1[threadIdx.x];
  for (int b = b0; b < b1; ++b) {
    const long long u0 = a.bsum[b], u1 = a.bsum[nb + b];
    a.bsum[b] = r0;
    a.bsum[nb + b] = r1;
    r0 += u0;
    r1 += u1;
  }
}

template <bool B>
__global__ __launch_bounds__(kScanThreads) void k_rt_scan_add(Args one, Batch bt) {
  int blk;
  const Args& a = block_run<B>(one, bt.sstart, bt, blk);
  const int i = blk * kScanThreads + threadIdx.x;
  if (i == 0) {
    a.off[0] = 0;
    a.eoff[0] = 0;
  }
  if (i < a.n) {
    a.off[i + 1] += (int32_t)a.bsum[blk];
    a.eoff[i + 1] += (int32_t)a.bsum[a.n_scan_blocks + blk];
  }
}

// ---------------------------------------------------------------------------
// edge records and CSR entries
// ---------------------------------------------------------------------------
// Each cell writes, for every edge it owns (its owned slots in slot order
// from eoff[i]): the edge record, its own CSR entry 2 e at the slot's rank
// among its kept slots, and, unless the edge is a wall, the neighbour's entry
// 2 e + 1 at the rank among the neighbour's kept slots of the slot that sees
// the edge (classify stored each kept slot's rank in its flag byte).  A certified mesh has every kept slot the owned or the other side
// of exactly one owned edge (classify matched each owned edge to one slot of
// the neighbour, and kept = 2 owned - walls), so each CSR entry is written
// once, and each cell's entries run counter-clockwise (slot order).  A
// failed re-tessellation leaves a mesh without edges.
template <bool B>
__global__ __launch_bounds__(kGroupThreads) void k_rt_emit(Args one, Batch bt) {
  int blk;
  const Args& a = block_run<B>(one, bt.cstart, bt, blk);
  const int l = (int)threadIdx.x % kGroup;
  const int i = blk * kThreads + (int)threadIdx.x / kGroup;
  if (i >= a.n) return;  // whole groups
  if (a.hdr->flags != 0) {
    if (l == 0) {
      a.off[i + 1] = 0;
      a.eoff[i + 1] = 0;
      if (i == 0) {
        a.off[0] = 0;
        a.eoff[0] = 0;
      }
    }
    return;
  }
  const int d = a.deg[i];
  const size_t s0 = (size_t)i * kMaxFan;
  const int k = a.off[i];
  int e = a.eoff[i];
  for (int base = 0; base < d; base += kGroup) {
    const int q = base + l;
    const uint8_t f = q < d ? a.s_flag[s0 + q] : (uint8_t)0;
    const uint32_t mo = group_bits((f & 3) == 3);
    const uint32_t below = (1u << l) - 1u;
    if ((f & 3) == 3) {
      const int ee = e + __popc(mo & below);
      const int32_t id = a.s_nb[s0 + q];
      const double* g = a.s_geo + 3 * (s0 + q);
      rich_edge r;
      r.fx = g[1];
      r.fy = g[2];
      r.len = g[0];
      r.i = i;
      r.j = id;
      a.edges[ee] = r;
      a.idx[k + (f >> 2)] = 2 * ee;
      if ((int)((uint32_t)id >> kShift) < kWallX0) {
        const int j = (int)((uint32_t)id & kMask);
        const int t = a.s_back[s0 + q];
        a.idx[a.off[j] + (a.s_flag[(size_t)j * kMaxFan + t] >> 2)] = 2 * ee + 1;
      }
    }
    e += __popc(mo);
  }
}

}  // namespace retess

// ===========================================================================
// Host side
// ===========================================================================
// (rich_kernels.hip) two host blocks to device memory through a pinned
// staging ring, enqueued on the stream
namespace rich_host {
int upload2(void* d0, const void* h0, size_t n0, void* d1, const void* h1, size_t n1,
            hipStream_t st);
}
namespace {

size_t rt_align(size_t v) { return (v + 255) / 256 * 256; }

struct RtLayout {
  size_t deg, s_nb, s_geo, s_flag, s_back, bsum, cpart, qcnt, queue, xy, total;
  int nb, qcap;
};

RtLayout rt_layout(int64_t n) {
  RtLayout L;
  const size_t slots = (size_t)n * retess::kMaxFan;
  L.nb = (int)((n + retess::kScanThreads - 1) / retess::kScanThreads);
  size_t o = 256;  // result header
  L.deg = o;    o += rt_align(4 * (size_t)n);
  L.s_nb = o;   o += rt_align(4 * slots);
  L.s_geo = o;  o += rt_align(24 * slots);
  L.s_flag = o; o += rt_align(slots);
  L.s_back = o; o += rt_align(slots);
  L.bsum = o;   o += rt_align(16 * (size_t)L.nb);
  L.cpart = o;
  const int64_t blocks = (n + retess::kThreads - 1) / retess::kThreads;
  o += rt_align(sizeof(retess::CPart) * (size_t)blocks);
  L.qcnt = o;   o += rt_align(4 * (size_t)retess::kSeg * retess::kSegStride);
  L.qcap = (int)(retess::kThreads * ((blocks + retess::kSeg - 1) / retess::kSeg));
  L.queue = o;  o += rt_align(4 * (size_t)retess::kSeg * (size_t)L.qcap);
  L.xy = o;     o += rt_align(16 * (size_t)n);
  L.total = o;
  return L;
}

void rt_capacity(int64_t n, int64_t* ce, int64_t* cc) {
  const int64_t r = (int64_t)std::ceil(std::sqrt((double)n));
  *ce = 3 * n + 8 * r + 64;
  *cc = 2 * *ce;
}

// Checks one run's arguments and fills its descriptor; RICH_OK or the status.
int make_args(const rich_mesh* prev, const double* x, const double* y,
              const rich_mesh_bufs* out, void* ws, size_t ws_bytes, retess::Args& a,
              RtLayout& L) {
  if (!prev || !x || !y || !out || !ws) return RICH_E_INVAL;
  const int64_t n = prev->n_cells;
  if (n <= 0 || n > (int64_t)retess::kMask || out->n_cells != n) return RICH_E_INVAL;
  if (!prev->off || !prev->eoff || (prev->n_csr > 0 && !prev->idx) ||
      (prev->n_edges > 0 && !prev->edges) || prev->n_csr < 0 || prev->n_edges < 0 ||
      prev->n_csr >= (int64_t)INT32_MAX || prev->n_edges >= (int64_t)INT32_MAX)
    return RICH_E_INVAL;
  if (!out->cells || !out->edges || !out->off || !out->idx || !out->eoff ||
      (reinterpret_cast<uintptr_t>(out->cells) & 15) ||
      (reinterpret_cast<uintptr_t>(out->edges) & 15) || out->cap_edges <= 0 ||
      out->cap_csr <= 0 || out->cap_csr >= (int64_t)INT32_MAX)
    return RICH_E_INVAL;
  if (!(prev->box[2] > prev->box[0]) || !(prev->box[3] > prev->box[1]) ||
      !std::isfinite(prev->box[0]) || !std::isfinite(prev->box[1]) ||
      !std::isfinite(prev->box[2]) || !std::isfinite(prev->box[3]))
    return RICH_E_INVAL;
  if (prev->bc != RICH_BOUNDARY_WALLS && prev->bc != RICH_BOUNDARY_PERIODIC) return RICH_E_INVAL;
  if (prev->bc == RICH_BOUNDARY_PERIODIC && n < 16) return RICH_E_INVAL;
  L = rt_layout(n);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws) & 255)) return RICH_E_NOMEM;

  char* w = static_cast<char*>(ws);
  std::memset(&a, 0, sizeof(a));
  a.p_off = prev->off;
  a.p_idx = prev->idx;
  a.p_edges = prev->edges;
  a.p_n_csr = prev->n_csr;
  a.p_n_edges = prev->n_edges;
  a.x = x;
  a.y = y;
  a.cells = out->cells;
  a.edges = out->edges;
  a.off = out->off;
  a.idx = out->idx;
  a.eoff = out->eoff;
  a.cap_edges = out->cap_edges;
  a.cap_csr = out->cap_csr;
  a.hdr = reinterpret_cast<retess::Hdr*>(w);
  a.deg = reinterpret_cast<int32_t*>(w + L.deg);
  a.s_nb = reinterpret_cast<int32_t*>(w + L.s_nb);
  a.s_geo = reinterpret_cast<double*>(w + L.s_geo);
  a.s_flag = reinterpret_cast<uint8_t*>(w + L.s_flag);
  a.s_back = reinterpret_cast<uint8_t*>(w + L.s_back);
  a.bsum = reinterpret_cast<int64_t*>(w + L.bsum);
  a.cpart = reinterpret_cast<retess::CPart*>(w + L.cpart);
  a.qcnt = reinterpret_cast<int32_t*>(w + L.qcnt);
  a.queue = reinterpret_cast<int32_t*>(w + L.queue);
  a.qcap = L.qcap;
  a.xy = reinterpret_cast<double2*>(w + L.xy);
  a.x0 = prev->box[0];
  a.y0 = prev->box[1];
  a.x1 = prev->box[2];
  a.y1 = prev->box[3];
  a.Lx = a.x1 - a.x0;
  a.Ly = a.y1 - a.y0;
  a.n = (int32_t)n;
  a.bc = (int32_t)prev->bc;
  a.n_scan_blocks = L.nb;
  return RICH_OK;
}

// The eleven launches of one re-tessellation of one kind of box (B: of n_runs runs at once, with
// gc cell blocks and gs scan blocks in all).
template <bool B>
void launch_all(const retess::Args& a, const retess::Batch& bt, int gc, int gs, int n_runs,
                bool walls, bool periodic, hipStream_t st) {
  using namespace retess;
  hipLaunchKernelGGL(k_rt_begin<B>, dim3(n_runs), dim3(64), 0, st, a, bt);
  hipLaunchKernelGGL(k_rt_pack<B>, dim3(gc), dim3(kThreads), 0, st, a, bt);
  if (walls) {
    hipLaunchKernelGGL((k_rt_vertex<B, true>), dim3(gc), dim3(kThreads), 0, st, a, bt);
    hipLaunchKernelGGL((k_rt_clip<B, true, kSlotsFast, false>), dim3(gc), dim3(kThreads), 0, st,
                       a, bt);
    hipLaunchKernelGGL((k_rt_clip<B, true, kSlotsWide, true>), dim3(gc), dim3(kThreads), 0, st,
                       a, bt);
  }
  if (periodic) {
    hipLaunchKernelGGL((k_rt_vertex<B, false>), dim3(gc), dim3(kThreads), 0, st, a, bt);
    hipLaunchKernelGGL((k_rt_clip<B, false, kSlotsFast, false>), dim3(gc), dim3(kThreads), 0, st,
                       a, bt);
    hipLaunchKernelGGL((k_rt_clip<B, false, kSlotsWide, true>), dim3(gc), dim3(kThreads), 0, st,
                       a, bt);
  }
  hipLaunchKernelGGL(k_rt_classify<B>, dim3(gc), dim3(kGroupThreads), 0, st, a, bt);
  hipLaunchKernelGGL(k_rt_scan_local<B>, dim3(gs), dim3(kScanThreads), 0, st, a, bt);
  hipLaunchKernelGGL(k_rt_scan_blocks<B>, dim3(n_runs), dim3(kScanThreads), 0, st, a, bt);
  hipLaunchKernelGGL(k_rt_scan_add<B>, dim3(gs), dim3(kScanThreads), 0, st, a, bt);
  hipLaunchKernelGGL(k_rt_emit<B>, dim3(gc), dim3(kGroupThreads), 0, st, a, bt);
  hipLaunchKernelGGL(k_rt_end<B>, dim3(n_runs), dim3(64), 0, st, a, bt);
}

// Batch workspace: descriptors, the two start tables, result headers, flags.
size_t batch_hdr_offset(int32_t n) {
  return rt_align(sizeof(retess::Args) * (size_t)n) + rt_align(8 * ((size_t)n + 1));
}
size_t batch_flags_offset(int32_t n) {
  return batch_hdr_offset(n) + rt_align(sizeof(retess::Hdr) * (size_t)n);
}
size_t batch_bytes(int32_t n) { return batch_flags_offset(n) + rt_align(4 * (size_t)n); }

}  // namespace

extern "C" {

int rich_retess_capacity(int64_t n_cells, int64_t* cap_edges, int64_t* cap_csr) {
  if (n_cells <= 0 || n_cells > (int64_t)retess::kMask || !cap_edges || !cap_csr)
    return RICH_E_INVAL;
  rt_capacity(n_cells, cap_edges, cap_csr);
  if (*cap_csr >= (int64_t)INT32_MAX) return RICH_E_INVAL;
  return RICH_OK;
}

int rich_retess_workspace_size(int64_t n_cells, size_t* bytes) {
  if (n_cells <= 0 || n_cells > (int64_t)retess::kMask || !bytes) return RICH_E_INVAL;
  *bytes = rt_layout(n_cells).total;
  return RICH_OK;
}

int rich_retess(const rich_mesh* prev, const double* x, const double* y,
                const rich_mesh_bufs* out, void* ws, size_t ws_bytes, void* stream) {
  retess::Args a;
  RtLayout L;
  const int rc = make_args(prev, x, y, out, ws, ws_bytes, a, L);
  if (rc) return rc;
  const int64_t n = prev->n_cells;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int gc = (int)((n + retess::kThreads - 1) / retess::kThreads);
  const bool periodic = a.bc == (int)RICH_BOUNDARY_PERIODIC;
  launch_all<false>(a, retess::Batch{}, gc, L.nb, 1, !periodic, periodic, st);
  return hipGetLastError() == hipSuccess ? RICH_OK : RICH_E_DEVICE;
}

int rich_retess_view(const rich_mesh_bufs* out, const double box[4], uint32_t bc,
                     rich_mesh* m) {
  if (!out || !box || !m || out->n_cells <= 0) return RICH_E_INVAL;
  m->n_cells = out->n_cells;
  m->n_edges = out->cap_edges;
  m->n_csr = out->cap_csr;
  m->cells = out->cells;
  m->edges = out->edges;
  m->off = out->off;
  m->idx = out->idx;
  m->eoff = out->eoff;
  for (int k = 0; k < 4; ++k) m->box[k] = box[k];
  m->bc = bc;
  return RICH_OK;
}

int rich_retess_batch_workspace_size(int32_t n, size_t* bytes) {
  if (n <= 0 || !bytes) return RICH_E_INVAL;
  *bytes = batch_bytes(n);
  return RICH_OK;
}

int rich_retess_batch(int32_t n, const rich_mesh* const* prev, const double* const* x,
                      const double* const* y, const rich_mesh_bufs* const* out,
                      void* const* ws, const size_t* ws_bytes, void* bws, size_t bws_bytes,
                      void* stream) {
  if (n <= 0 || !prev || !x || !y || !out || !ws || !ws_bytes || !bws) return RICH_E_INVAL;
  if (bws_bytes < batch_bytes(n) || (reinterpret_cast<uintptr_t>(bws) & 255)) return RICH_E_NOMEM;
  std::vector<retess::Args> args((size_t)n);
  std::vector<int32_t> starts(2 * ((size_t)n + 1));
  int64_t gc = 0, gs = 0;
  for (int32_t r = 0; r < n; ++r) {
    RtLayout L;
    const int rc = make_args(prev[r], x[r], y[r], out[r], ws[r], ws_bytes[r], args[r], L);
    if (rc) return rc;
    for (int32_t q = 0; q < r; ++q)
      if (ws[q] == ws[r]) return RICH_E_INVAL;   // runs need workspaces of their own
    starts[r] = (int32_t)gc;
    starts[n + 1 + r] = (int32_t)gs;
    gc += (prev[r]->n_cells + retess::kThreads - 1) / retess::kThreads;
    gs += L.nb;
    if (gc >= INT32_MAX / 2 || gs >= INT32_MAX / 2) return RICH_E_INVAL;
  }
  starts[n] = (int32_t)gc;
  starts[2 * (size_t)n + 1] = (int32_t)gs;
  char* b = static_cast<char*>(bws);
  const size_t o_start = rt_align(sizeof(retess::Args) * (size_t)n);
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the host arrays die with this call: they go through the pinned staging
  // ring, whose copies are enqueued on the stream (no wait)
  const int up = rich_host::upload2(b, args.data(), sizeof(retess::Args) * (size_t)n,
                                    b + o_start, starts.data(), starts.size() * sizeof(int32_t),
                                    st);
  if (up != RICH_OK) return up;
  retess::Batch bt;
  bt.descs = reinterpret_cast<const retess::Args*>(b);
  bt.cstart = reinterpret_cast<const int32_t*>(b + o_start);
  bt.sstart = bt.cstart + n + 1;
  bt.hdr_out = reinterpret_cast<retess::Hdr*>(b + batch_hdr_offset(n));
  bt.flags_out = reinterpret_cast<int32_t*>(b + batch_flags_offset(n));
  bt.n_runs = n;
  bool walls = false, periodic = false;
  for (const retess::Args& r : args) {
    walls = walls || r.bc != (int)RICH_BOUNDARY_PERIODIC;
    periodic = periodic || r.bc == (int)RICH_BOUNDARY_PERIODIC;
  }
  launch_all<true>(args[0], bt, (int)gc, (int)gs, n, walls, periodic, st);
  return hipGetLastError() == hipSuccess ? RICH_OK : RICH_E_DEVICE;
}

int rich_retess_batch_result(int32_t n, void* bws, void* stream, rich_retess_info* info,
                             int32_t* status) {
  if (n <= 0 || !bws || !info || !status) return RICH_E_INVAL;
  const size_t o_hdr = batch_hdr_offset(n);
  std::vector<retess::Hdr> h((size_t)n);
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess ||
      hipMemcpy(h.data(), static_cast<char*>(bws) + o_hdr, sizeof(retess::Hdr) * (size_t)n,
                hipMemcpyDeviceToHost) != hipSuccess)
    return RICH_E_DEVICE;
  for (int32_t r = 0; r < n; ++r) {
    info[r].flags = h[r].flags;
    info[r].sticky = h[r].sticky;
    info[r].n_edges = h[r].n_edges;
    info[r].n_csr = h[r].n_csr;
    info[r].n_dropped = h[r].n_dropped;
    info[r].area_sum = h[r].area_sum;
    info[r].n_clipped = h[r].n_clip;
    status[r] = h[r].flags ? RICH_E_MESH : RICH_OK;
  }
  return RICH_OK;
}

int rich_retess_batch_flags_async(int32_t n, void* bws, void* stream, int32_t* host_flags) {
  if (n <= 0 || !bws || !host_flags) return RICH_E_INVAL;
  if (hipMemcpyAsync(host_flags, static_cast<char*>(bws) + batch_flags_offset(n),
                     sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                     static_cast<hipStream_t>(stream)) != hipSuccess)
    return RICH_E_DEVICE;
  return RICH_OK;
}

int rich_retess_result(void* ws, void* stream, rich_retess_info* info) {
  if (!ws || !info) return RICH_E_INVAL;
  if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return RICH_E_DEVICE;
  retess::Hdr h;
  if (hipMemcpy(&h, ws, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return RICH_E_DEVICE;
  info->flags = h.flags;
  info->sticky = h.sticky;
  info->n_edges = h.n_edges;
  info->n_csr = h.n_csr;
  info->n_dropped = h.n_dropped;
  info->area_sum = h.area_sum;
  info->n_clipped = h.n_clip;
  return h.flags ? RICH_E_MESH : RICH_OK;
}

}  // extern "C"
