// Host check of the sweeps' index arithmetic (fv_index.hpp) against its plain
// definition: divisions of the flattened position, the wave strips' lane
// map; and of the launches' dispatch orders against the properties that
// define them.  Prints "ok" or
// the first mismatch and exits non-zero.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <initializer_list>
#include <vector>

#include "fv_index.hpp"

using namespace rfv;

static int check_x(int nx, int ny, int nz, int nt) {
  const int lx = nx + 4, total = lx * ny * nz, c = nt - 4;
  const int tiles = (total + c - 1) / c;
  for (int lt = 0; lt < tiles; ++lt) {
    for (int tid = 0; tid < nt; ++tid) {
      const int f = lt * c - 2 + tid;
      const bool valid = f >= 0 && f < total;
      const int fc = f < 0 ? 0 : (f >= total ? total - 1 : f);
      const int row = fc / lx, il = fc % lx, j = row % ny, k = row / ny;
      const XPos p = x_position(tid, lt * c - 2, lx, ny, nz);
      const int f0 = lt * c - 2 < 0 ? 0 : lt * c - 2;
      const bool ok = p.valid == valid && p.il == il && p.j0 + p.dj == j && p.k0 + p.dk == k &&
                      p.j0 == (f0 / lx) % ny && p.k0 == (f0 / lx) / ny;
      if (!ok) {
        std::printf("x_position mismatch n=(%d,%d,%d) nt=%d tile=%d tid=%d: got il=%d j=%d k=%d "
                    "valid=%d, want il=%d j=%d k=%d valid=%d\n", nx, ny, nz, nt, lt, tid, p.il,
                    p.j0 + p.dj, p.k0 + p.dk, (int)p.valid, il, j, k, (int)valid);
        return 1;
      }
    }
  }
  return 0;
}

static int check_face() {
  for (int n = 1; n <= 9; ++n)
    for (int j = -2; j < n + 2; ++j) {
      const int t = face_index(j, n, FACE_TRANSMISSIVE, FACE_TRANSMISSIVE);
      const int p = face_index(j, n, FACE_PERIODIC, FACE_PERIODIC);
      const int h = face_index(j, n, FACE_HALO, FACE_HALO);
      const int want_t = j < 0 ? 0 : (j >= n ? n - 1 : j);
      const int want_p = ((j % n) + n) % n;
      if (t != want_t || h != j || (n >= 2 && p != want_p)) {
        std::printf("face_index mismatch n=%d j=%d\n", n, j);
        return 1;
      }
    }
  return 0;
}

// dispatch_order: every tile exactly once; XCD x takes slots x, x + nxcd, ...
// with its empty slots last; its tiles are one contiguous run of the list,
// the runs in list order, each costliest first with ties in list order, and
// each run's cost within one tile's cost of an equal share.
static int check_order(const std::vector<int32_t>& cost, int nxcd) {
  std::vector<int32_t> order;
  dispatch_order(cost, nxcd, order);
  const int64_t T = (int64_t)cost.size();
  bool uniform = true;
  int32_t cmax = 0;
  int64_t total = 0;
  for (int32_t c : cost) {
    uniform = uniform && c == cost[0];
    cmax = c > cmax ? c : cmax;
    total += c;
  }
  if (uniform) {
    if (!order.empty()) { std::printf("dispatch_order: uniform costs gave an order\n"); return 1; }
    return 0;
  }
  if (order.size() % nxcd) { std::printf("dispatch_order: %zu slots\n", order.size()); return 1; }
  std::vector<int> seen((size_t)T, 0);
  const size_t per = order.size() / nxcd;
  int64_t next = 0;  // first tile of the next run
  size_t longest = 0;
  for (int x = 0; x < nxcd; ++x) {
    std::vector<int32_t> r;
    bool ended = false;
    for (size_t i = 0; i < per; ++i) {
      const int32_t t = order[i * nxcd + x];
      if (t < 0) { ended = true; continue; }
      if (ended || t >= T || seen[t]++) { std::printf("dispatch_order: bad slot %zu\n", i * nxcd + x); return 1; }
      r.push_back(t);
    }
    longest = r.size() > longest ? r.size() : longest;
    int64_t lo = T, hi = -1, rc = 0;
    for (size_t i = 0; i < r.size(); ++i) {
      lo = r[i] < lo ? r[i] : lo;
      hi = r[i] > hi ? r[i] : hi;
      rc += cost[r[i]];
      if (i && (cost[r[i]] > cost[r[i - 1]] || (cost[r[i]] == cost[r[i - 1]] && r[i] < r[i - 1]))) {
        std::printf("dispatch_order: run %d not costliest first\n", x);
        return 1;
      }
    }
    if (!r.empty() && (lo != next || hi - lo + 1 != (int64_t)r.size())) {
      std::printf("dispatch_order: run %d not contiguous from %lld\n", x, (long long)next);
      return 1;
    }
    next += (int64_t)r.size();
    if (std::llabs(rc * nxcd - total) > (int64_t)cmax * nxcd) {
      std::printf("dispatch_order: run %d costs %lld of %lld\n", x, (long long)rc, (long long)total);
      return 1;
    }
  }
  if (next != T || longest != per) { std::printf("dispatch_order: runs cover %lld of %lld\n", (long long)next, (long long)T); return 1; }
  return 0;
}

static int check_orders() {
  uint64_t s = 2104;
  auto rnd = [&](int m) {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return (int)((s >> 33) % (uint64_t)m);
  };
  for (int trial = 0; trial < 400; ++trial) {
    const int T = 1 + rnd(trial < 200 ? 40 : 4000);
    const int kind = rnd(3);
    std::vector<int32_t> cost((size_t)T);
    for (int t = 0; t < T; ++t)
      cost[t] = kind == 0 ? 6 + rnd(129)                    // any length
                : kind == 1 ? (t % 5 == 4 ? 6 + rnd(64) : 134)  // full segments, short last ones
                            : 70;                           // uniform
    if (check_order(cost, 8) || check_order(cost, 3)) return 1;
  }
  return 0;
}

// Wave strips: over the waves that cover a grid's rows (groups of the strip
// plan, rounded up to whole workgroups of `wpt` waves), every cell (x, z) of
// the nx x nz rows is held by exactly one lane, and the four lanes around
// it hold x - 2 .. x + 2 of the same row (so the lane shifts read the
// stencil); no wave spans more than 12 rows past its first.
static int check_strips(int nx, int nz, int cells, int wpt) {
  const StripPlan sp = strip_plan(nx, nz, cells);
  const int64_t items = (int64_t)(nz + sp.k - 1) / sp.k * sp.per;
  const int64_t waves = (items + wpt - 1) / wpt * wpt;
  std::vector<int> seen((size_t)nx * nz, 0);
  for (int fw = 0; fw < waves; ++fw) {
    StripLane l[64];
    for (int ln = 0; ln < 64; ++ln) l[ln] = strip_lane(sp, fw, ln, cells);
    if (l[0].kw >= nz) continue;
    for (int ln = 0; ln < 64; ++ln) {
      const int kk = l[ln].kw + l[ln].h, xl = l[ln].lane_in - 2;
      if (l[ln].kw != l[0].kw || l[ln].h > 11) {
        std::printf("strips nx=%d nz=%d: wave %d lane %d row %d\n", nx, nz, fw, ln, kk);
        return 1;
      }
      if (kk >= nz || xl < 0 || xl >= l[ln].ncx) continue;
      const int x = l[ln].xoff + xl;
      if (x >= nx || ++seen[(size_t)kk * nx + x] != 1) {
        std::printf("strips nx=%d nz=%d: cell (%d, %d) again at wave %d\n", nx, nz, x, kk, fw);
        return 1;
      }
      for (int d = -2; d <= 2; ++d) {
        const int m = ln + d;
        if (m < 0 || m > 63 || l[m].kw + l[m].h != kk || l[m].xoff + l[m].lane_in - 2 != x + d) {
          std::printf("strips nx=%d nz=%d: lane %d of wave %d, neighbour %d\n", nx, nz, ln, fw, d);
          return 1;
        }
      }
    }
  }
  for (size_t i = 0; i < seen.size(); ++i)
    if (seen[i] != 1) {
      std::printf("strips nx=%d nz=%d: cell %zu not held\n", nx, nz, i);
      return 1;
    }
  return 0;
}

int main() {
  if (check_face()) return 1;
  if (check_orders()) return 1;
  for (int nx : {1, 2, 5, 24, 28, 29, 59, 60, 61, 64, 80, 120, 121, 150, 256, 384, 385, 512, 1000})
    for (int nz : {1, 2, 3, 5, 12, 13, 25})
      for (int wpt : {1, 4})
        if (check_strips(nx, nz, 60, wpt)) return 1;
  const int nxs[] = {1, 2, 3, 5, 17, 32, 61, 124, 125, 252, 253, 256, 300, 512};
  const int nys[] = {1, 3, 7, 16};
  const int nzs[] = {1, 2, 5};
  for (int nt : {128, 256})
    for (int nx : nxs)
      for (int ny : nys)
        for (int nz : nzs)
          if (check_x(nx, ny, nz, nt)) return 1;
  std::printf("ok\n");
  return 0;
}
