// Index arithmetic of the sweeps that does not touch memory, kept apart so
// that host code (and host-side checks) can evaluate exactly what the kernels
// compute.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define RFV_HD __host__ __device__ __forceinline__
#else
#define RFV_HD inline
#endif

namespace rfv {

enum FaceMode : int { FACE_TRANSMISSIVE = 0, FACE_PERIODIC = 1, FACE_HALO = 2 };

// Interior index to load for position j (may lie in [-2, n+1]) along an axis:
// transmissive faces clamp, periodic faces wrap, halo faces read the padding.
RFV_HD int face_index(int j, int n, int mode_lo, int mode_hi) {
  if (j < 0) return mode_lo == FACE_TRANSMISSIVE ? 0 : (mode_lo == FACE_PERIODIC ? j + n : j);
  if (j >= n) return mode_hi == FACE_TRANSMISSIVE ? n - 1 : (mode_hi == FACE_PERIODIC ? j - n : j);
  return j;
}

// Position of thread tid of an x-sweep chunk in the flattened (row, x) space of
// a grid with row length lx = nx + 4 (padded x positions), ny rows per plane
// and nz planes.  The chunk's first position F0 (= tile * chunk - 2, so -2 for
// the first chunk) is decoded once per wave with one division; each lane then
// walks forward from it, wrapping rows and planes, which costs a few
// compares instead of three per-lane divisions.  Lanes past either end of the
// space are marked invalid and clamped onto its first or last position so
// that their loads stay in bounds.
struct XPos {
  int il;        // padded x index (0 .. lx-1) of the lane's position
  int j0, k0;    // row and plane of the chunk's first in-range position (uniform)
  int dj, dk;    // lane row/plane minus (j0, k0); dj may be negative after a plane wrap
  bool valid;
};

RFV_HD XPos x_position(int tid, int F0, int lx, int ny, int nz) {
  XPos r;
  const int total = lx * ny * nz;
  const int F0c = F0 < 0 ? 0 : F0;
  const int row0 = F0c / lx;
  const int il0 = F0c - row0 * lx;
  r.j0 = row0 % ny;
  r.k0 = row0 / ny;
  const int f = F0 + tid;
  r.valid = f >= 0 && f < total;
  const int fc = f < 0 ? 0 : (f >= total ? total - 1 : f);
  int il = il0 + (fc - F0c);
  int j = r.j0, k = r.k0;
  while (il >= lx) {
    il -= lx;
    if (++j == ny) {
      j = 0;
      ++k;
    }
  }
  r.il = il;
  r.dj = j - r.j0;
  r.dk = k - r.k0;
  return r;
}

// Wave strips of the fused x-y pass: a row of nx cells takes nsx strips of
// `cells` cells, each held by one wave with two ghost lanes on either side;
// the last strip holds the tail of t = nx - (nsx - 1) cells cells.  When k
// = min(64 / (t + 4), RFV_STRIP_KMAX, nz) >= 3, the tails of k consecutive
// rows (at consecutive z) share one wave, sub-strip h taking lanes h (t + 4)
// .. h (t + 4) + t + 3.  A group of k rows then takes per = k (nsx - 1) + 1
// waves: its rows' full strips, row-major, then the shared tails.  A wave
// of shared tails runs the instructions of any other wave but takes longer,
// its loads spanning k planes: measured about 1.5 to 1.9 times a full wave
// for k = 2 and 3, and several times for k = 4 to 8.  So two tails keep a
// wave each (on rows of 384 cells sharing gained 1.7 % on the FP32 x-y
// pass of a single grid, 3.9 % in FP64, and lost 1.1 % on FP32 sub-blocks
// linked along x), and at most three share one (rows of 370 cells: 5.8 %
// faster in FP32 and 2.6 % in FP64 with three, 3.7 and 1.8 % with four, 3.3
// and 1.5 % with up to twelve; rows of 256 cells in FP64: 8.3 %).
#ifndef RFV_STRIP_KMAX
#define RFV_STRIP_KMAX 3
#endif
struct StripPlan {
  int nsx;    // strips per row
  int tail;   // cells of the last strip
  int k;      // rows whose tails share a wave (1: no sharing)
  int per;    // waves per group of k rows
};
RFV_HD StripPlan strip_plan(int nx, int nz, int cells) {
  StripPlan s;
  s.nsx = (nx + cells - 1) / cells;
  s.tail = nx - (s.nsx - 1) * cells;
  s.k = 64 / (s.tail + 4);
  if (s.k > RFV_STRIP_KMAX) s.k = RFV_STRIP_KMAX;
  if (s.k > nz) s.k = nz;
  if (s.k < 3) s.k = 1;
  s.per = s.k * (s.nsx - 1) + 1;
  return s;
}

// The strip that wave fw (in launch order) holds, and the part of it that
// lane `lane` takes: row kw + h (at z; kw is uniform over the wave), x from
// xoff + lane_in - 2.  The lanes past the last sub-strip's ghost lanes join
// that sub-strip at lane_in > ncx + 3; like the lanes past ncx + 1 of any
// strip they hold no cell.
struct StripLane {
  int xoff;     // x of the strip's first cell
  int ncx;      // cells of the strip
  int kw;       // row of sub-strip 0
  int h;        // sub-strip of the lane
  int lane_in;  // lane within its sub-strip (0 .. ncx + 3 hold x - 2 .. x + 1)
};
RFV_HD StripLane strip_lane(const StripPlan& sp, int fw, int lane, int cells) {
  StripLane r;
  const int grp = fw / sp.per;
  const int w = fw - grp * sp.per;
  const int nfull = sp.nsx - 1;
  const bool tailw = w >= sp.k * nfull;
  const int q = tailw ? 0 : w / (nfull > 0 ? nfull : 1);
  r.xoff = tailw ? nfull * cells : (w - q * nfull) * cells;
  r.ncx = tailw ? sp.tail : cells;
  r.kw = grp * sp.k + q;
  int h = tailw ? lane / (sp.tail + 4) : 0;
  if (h > sp.k - 1) h = sp.k - 1;
  r.h = h;
  r.lane_in = lane - h * (sp.tail + 4);
  return r;
}

// Dispatch order of a launch over tiles of the given costs, for a part whose
// workgroups go round-robin to nxcd XCDs (workgroup w to XCD w mod nxcd), each
// of which starts its workgroups in index order as CUs free up.  With tiles
// of uneven cost (grids of different extents, short last segments), handing
// each XCD an equal number of tiles leaves some XCDs working after the others
// finish.  So the tile list is cut into nxcd contiguous runs of about equal
// cost (each tile goes to the run that holds the midpoint of its share), one
// per XCD, and each run is taken costliest tile first, ties in list order (a
// grid's tiles stay neighbours and share halo cells in that XCD's L2).  Entry
// s of `order` is the tile that slot s takes, -1 for none: slot s belongs to
// XCD s mod nxcd, and there are nxcd times the longest run of slots.  Where
// all tiles cost the same the order is left empty: equal runs in list order
// are what a launch without one does (xcd_order).  Host only.
inline void dispatch_order(const std::vector<int32_t>& cost, int nxcd, std::vector<int32_t>& order) {
  order.clear();
  if (cost.empty() ||
      std::all_of(cost.begin(), cost.end(), [&](int32_t c) { return c == cost[0]; }))
    return;
  int64_t total = 0;
  for (int32_t c : cost) total += c;
  std::vector<std::vector<int32_t>> run((size_t)nxcd);
  int64_t acc = 0;
  for (size_t t = 0; t < cost.size(); ++t) {
    const int64_t x = std::min<int64_t>(nxcd - 1, (2 * acc + cost[t]) * nxcd / (2 * total));
    run[(size_t)x].push_back((int32_t)t);
    acc += cost[t];
  }
  size_t longest = 0;
  for (auto& r : run) {
    std::stable_sort(r.begin(), r.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    longest = std::max(longest, r.size());
  }
  order.assign((size_t)nxcd * longest, -1);
  for (size_t x = 0; x < run.size(); ++x)
    for (size_t i = 0; i < run[x].size(); ++i) order[i * nxcd + x] = run[x][i];
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Renumber them so
// that each XCD takes one contiguous run of tiles: neighbouring tiles share
// halo cells and then share that XCD's L2.
RFV_HD int64_t xcd_order(int64_t b, int64_t nblocks) {
  const int64_t x = b & 7, k = b >> 3, q = nblocks >> 3, r = nblocks & 7;
  return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

}  // namespace rfv
