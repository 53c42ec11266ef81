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
