// C ABI of libripple_fv: argument validation, contexts, cached per-batch plans
// (device workspaces, tile lists, halo task lists, captured graphs), the step
// loop, diagnostics and the layout / tiling autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "fv_internal.hpp"
#include "ripple_fv.h"

using namespace rfv;

// The scratch array of ripple_fv_run_batch_noalloc (see scratch_address).
static __device__ __align__(256) unsigned char scratch[RIPPLE_FV_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int64_t MAX_BYTES = int64_t(1) << 46;
constexpr int MAX_PLANS = 16;
constexpr int GRAPH_MAX_STEPS = 64;  // steps captured in one graph
constexpr int MAX_GRAPHS = 4;        // cached graphs per plan

// Workspace of ripple_fv_run_batch_noalloc: a file-scope device array, one
// copy per device, held until the process ends.  In host code its name is a
// host-side stand-in, not a device address; the device address comes from
// hipGetSymbolAddress, taken once per device (scratch_address) with that
// device current, and only that address is handed to kernels and copies.
constexpr int NOALLOC_MAX_GRIDS = RIPPLE_FV_NOALLOC_MAX_GRIDS;
constexpr size_t SCRATCH_BYTES = RIPPLE_FV_NOALLOC_SCRATCH_BYTES;

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
unsigned char* scratch_ptr[MAX_DEVICES] = {};

// Device address of `device`'s scratch array (the device must be current).
hipError_t scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[device] = static_cast<unsigned char*>(p);
  }
  *out = scratch_ptr[device];
  return hipSuccess;
}

// Launch description of a batch over storage owned elsewhere: by a cached
// Plan (heap vectors and one device allocation) or, in the allocation-free
// entry point, by stack arrays and the device scratch array.  The enqueue
// functions read only this.
struct PlanCore {
  int n = 0;
  int dtype = 0, lay = 0;
  Tiling tl{};
  const ripple_fv_grid* grids = nullptr;  // host descriptors [n]
  bool fused = false;                   // x and y sweeps as one pass
  int seg_xy = 0;                       // rows per tile of the fused pass
  int seg_z = 0;                        // cells per tile of the z sweep
  int xmode = XM_ROWS;                  // form of the fused pass
  bool planar = false;                  // every grid one cell thick in z: no z sweep
  bool planar_fused = false;            // ... and the x-y pass (wave strips) is the step
  // the step returns the state to its first buffer (else the passes alternate
  // the two buffers from step to step)
  bool in_place() const { return fused || (planar && !planar_fused); }
  // host: tile prefix sums [n + 1] of the x, y, z, wave-speed and fused x-y
  // launches; halo copy tasks per axis (at most 2 n each); descriptors with
  // the current buffer pointers [n]
  const int64_t* tiles[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  const HaloTask* halo[3] = {nullptr, nullptr, nullptr};
  int nhalo[3] = {0, 0, 0};
  int64_t halo_area[3] = {0, 0, 0};
  const DevGrid* h_grids = nullptr;
  // dispatch orders of the batched y, z and fused x-y launches (slots of
  // each; 0: none, each XCD then takes one contiguous run of the tiles)
  const int32_t* order[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int64_t nslots[5] = {0, 0, 0, 0, 0};
  // device copies and per-grid slots
  DevGrid* d_grids = nullptr;
  int64_t* d_tiles[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  int32_t* d_order[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  HaloTask* d_halo[3] = {nullptr, nullptr, nullptr};
  double* d_lam = nullptr;
  double* d_t = nullptr;
  double* d_dt = nullptr;
  unsigned long long* d_s = nullptr;

  Work work(unsigned int* flag) const {
    Work w;
    w.grids = d_grids;
    w.ngrids = n;
    w.pad_ = 0;
    w.lam = d_lam;
    w.t = d_t;
    w.dt = d_dt;
    w.s_acc = d_s;
    w.flag = flag;
    return w;
  }
};

// Byte offsets of the device workspace of a batch of n grids with nhalo[]
// halo tasks per axis and nslots[] dispatch slots per launch kind (null: no
// dispatch orders): descriptors, tile prefix sums, halo tasks, dispatch
// orders, then the per-grid dt / lambda / time / wave-speed slots (each part
// 256-byte aligned).
struct WsLayout {
  size_t grids, tiles[5], halo[3], order[5], lam, t, dt, s, total;
};

WsLayout ws_layout(int n, const int nhalo[3], const int64_t* nslots) {
  auto align = [](size_t v) { return (v + 255) & ~size_t(255); };
  WsLayout L;
  size_t off = 0;
  L.grids = off; off = align(off + sizeof(DevGrid) * n);
  for (int k = 0; k < 5; ++k) { L.tiles[k] = off; off = align(off + sizeof(int64_t) * (n + 1)); }
  for (int k = 0; k < 3; ++k) { L.halo[k] = off; off = align(off + sizeof(HaloTask) * (nhalo[k] + 1)); }
  for (int k = 0; k < 5; ++k) {
    L.order[k] = off;
    off = align(off + sizeof(int32_t) * (nslots ? nslots[k] : 0));
  }
  L.lam = off; off = align(off + sizeof(double) * 3 * n);
  L.t = off; off = align(off + sizeof(double) * n);
  L.dt = off; off = align(off + sizeof(double) * n);
  L.s = off; off = align(off + sizeof(unsigned long long) * 3 * n);
  L.total = off;
  return L;
}

void ws_bind(PlanCore& P, char* base, const WsLayout& L) {
  P.d_grids = reinterpret_cast<DevGrid*>(base + L.grids);
  for (int k = 0; k < 5; ++k) P.d_tiles[k] = reinterpret_cast<int64_t*>(base + L.tiles[k]);
  for (int k = 0; k < 5; ++k)
    P.d_order[k] = P.nslots[k] ? reinterpret_cast<int32_t*>(base + L.order[k]) : nullptr;
  for (int k = 0; k < 3; ++k) P.d_halo[k] = reinterpret_cast<HaloTask*>(base + L.halo[k]);
  P.d_lam = reinterpret_cast<double*>(base + L.lam);
  P.d_t = reinterpret_cast<double*>(base + L.t);
  P.d_dt = reinterpret_cast<double*>(base + L.dt);
  P.d_s = reinterpret_cast<unsigned long long*>(base + L.s);
}

// A cached plan: owns the host arrays, the device workspace and the graphs.
struct Plan : PlanCore {
  std::vector<ripple_fv_grid> grid_store;
  std::vector<int64_t> tile_store[5];
  std::vector<HaloTask> halo_store[3];
  std::vector<int32_t> order_store[5];
  std::vector<DevGrid> h_grid_store;
  void* dmem = nullptr;                 // device workspace (one allocation)
  // descriptor staging for buffer-pointer updates
  DevGrid* h_pinned = nullptr;
  hipEvent_t upload_done = nullptr;
  bool upload_pending = false;
  bool uploaded = false;
  // captured step loops by step count, and the cfl / launch mode they were
  // captured with
  std::map<int, hipGraphExec_t> graphs;
  double graph_cfl = -1.0;
  bool graph_per_grid = false;

  // (waits for the device first: a launched graph may still be running)
  void drop_graphs() {
    if (graphs.empty()) return;
    hipDeviceSynchronize();
    for (auto& kv : graphs) hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~Plan() {
    drop_graphs();
    if (upload_done) {
      hipEventSynchronize(upload_done);
      hipEventDestroy(upload_done);
    }
    if (h_pinned) hipHostFree(h_pinned);
    if (dmem) hipFree(dmem);
  }
};

}  // namespace

struct ripple_fv_ctx {
  int device = 0;
  int cu_count = 256;
  std::string err;
  unsigned int* flag = nullptr;     // device
  double* partials = nullptr;       // device, DIAG_MAX_BLOCKS * 20
  hipStream_t cap_stream = nullptr; // private stream used only for graph capture
  std::map<std::string, std::unique_ptr<Plan>> plans;
  std::deque<std::string> plan_order;
  std::vector<hipEvent_t> events;   // profiling event pool
  double prof_ms[RIPPLE_FV_NKERNELS] = {0};
  int64_t prof_n[RIPPLE_FV_NKERNELS] = {0};
  std::map<std::string, std::vector<ripple_fv_grid>> tune_cache;
  unsigned char* scratch = nullptr; // device address of this device's scratch array
};

namespace {

ripple_fv_status fail(ripple_fv_ctx* ctx, ripple_fv_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return st;
}

#define HIP_OR_FAIL(ctx, call)                                                            \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((ctx), RIPPLE_FV_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

bool valid_block(int v, std::initializer_list<int> allowed) {
  return std::find(allowed.begin(), allowed.end(), v) != allowed.end();
}

// Validate a descriptor and compute its pitches and size (ripple_fv_grid_init).
ripple_fv_status grid_check(const ripple_fv_grid* g, int64_t pitch[3], int64_t* bytes,
                            int32_t* x_origin, std::string* why) {
  for (int d = 0; d < 3; ++d) {
    if (g->n[d] < 1) { *why = "extent < 1"; return RIPPLE_FV_E_INVALID; }
    if (!(g->dx[d] > 0.0) || !std::isfinite(g->dx[d])) { *why = "dx <= 0"; return RIPPLE_FV_E_INVALID; }
    if (g->bc[d] != RIPPLE_FV_TRANSMISSIVE && g->bc[d] != RIPPLE_FV_PERIODIC) {
      *why = "unknown boundary condition";
      return RIPPLE_FV_E_INVALID;
    }
  }
  if (g->dtype != RIPPLE_FV_F32 && g->dtype != RIPPLE_FV_F64) { *why = "unknown dtype"; return RIPPLE_FV_E_INVALID; }
  if (g->layout == RIPPLE_FV_AOSOA) {
    if (!valid_block(g->aosoa_w, {16, 32, 64})) { *why = "aosoa_w must be 16, 32 or 64"; return RIPPLE_FV_E_INVALID; }
  } else if (g->layout == RIPPLE_FV_AOS || g->layout == RIPPLE_FV_SOA) {
    if (g->aosoa_w != 0) { *why = "aosoa_w must be 0 unless layout is AOSOA"; return RIPPLE_FV_E_INVALID; }
  } else {
    *why = "unknown layout";
    return RIPPLE_FV_E_INVALID;
  }
  if (!valid_block(g->x_block, {0, 128, 256}) || !valid_block(g->yz_block, {0, 64, 128, 256}) ||
      g->yz_segment < 0 || (g->yz_segment > 0 && g->yz_segment < 4) || g->yz_segment > 4096 ||
      g->persist < 0 || g->persist > 64 || !valid_block(g->yz_cols, {0, 1, 2, 4}) ||
      !valid_block(g->split_xy, {0, 1, 2, 3}) || g->reserved != 0) {
    *why = "bad tiling knobs";
    return RIPPLE_FV_E_INVALID;
  }
  // AoS: even row pitch, so pairs of x cells start on 8-byte (FP32) / 16-byte
  // (FP64) boundaries.  SoA / AoSoA: interior rows start on 128-byte lines
  // (AoSoA: on a block), so y and z sweeps touch no partial lines.
  const int64_t elem = g->dtype == RIPPLE_FV_F32 ? 4 : 8;
  int64_t align = 2, ox = HALO;
  if (g->layout != RIPPLE_FV_AOS) {
    align = 128 / elem;
    if (g->layout == RIPPLE_FV_AOSOA && g->aosoa_w > align) align = g->aosoa_w;
    ox = align;
  }
  const int64_t px = (g->n[0] + 4 + align - 1) / align * align;
  const int64_t py = g->n[1] + 4, pz = g->n[2] + 4;
  const int64_t cells = (px * py * pz + ox + 63) / 64 * 64;
  // 32-bit tile-local index spaces in the kernels
  if ((int64_t)(g->n[0] + 4) * g->n[1] * g->n[2] >= (int64_t(1) << 31) || cells >= (int64_t(1) << 40)) {
    *why = "grid too large";
    return RIPPLE_FV_E_INVALID;
  }
  const int64_t b = cells * 5 * elem;
  if (b > MAX_BYTES) { *why = "grid too large"; return RIPPLE_FV_E_INVALID; }
  // Per-lane byte offsets from a tile's wave-uniform base are 32-bit buffer
  // offsets.  The tiles that span the most memory are the rows form of the
  // fused x-y pass (up to XY_THREADS / n0 rows at consecutive z), the waves
  // of the strips form that share the tails of up to RFV_STRIP_KMAX rows at
  // consecutive z, and the separate y sweep (lanes across x, then z: up to 2
  // * 256 / n0 + 1 planes); every other tile stays within a few rows.  Bound
  // the largest span generously by max(2 * XY_THREADS / n0, RFV_STRIP_KMAX)
  // + 2 planes (at most n2): that many plane pitches plus a row pitch and the
  // alignment slack, times the cells' element stride (5 in AoS and AoSoA).
  {
    const int64_t planes = std::min<int64_t>(
        g->n[2], std::max<int64_t>(2 * XY_THREADS / g->n[0], RFV_STRIP_KMAX) + 2);
    const int64_t span_cells = (planes - 1) * px * py + px + ox + 64;
    const int64_t stride = g->layout == RIPPLE_FV_SOA ? 1 : 5;
    if (span_cells * stride * elem >= (int64_t(1) << 31)) {
      *why = "grid too large for 32-bit lane offsets (a thin x extent with large y-z planes)";
      return RIPPLE_FV_E_INVALID;
    }
  }
  pitch[0] = px;
  pitch[1] = py;
  pitch[2] = pz;
  *bytes = b;
  *x_origin = (int32_t)ox;
  return RIPPLE_FV_OK;
}

Tiling tiling_of(const ripple_fv_grid& g) {
  Tiling t;
  t.x_block = g.x_block ? g.x_block : 256;
  t.yz_block = g.yz_block ? g.yz_block : 256;
  t.yz_segment = g.yz_segment ? g.yz_segment : 128;
  t.persist = g.persist;
  // two x cells per y/z thread pays off where it widens the accesses (FP32
  // SoA/AoSoA); FP64 always runs one (two FP64 cells per thread do not fit
  // the register file without spilling); four (16-byte accesses) only where
  // a component's cells are adjacent, so AoS takes two for four
  if (g.dtype == RIPPLE_FV_F64)
    t.yz_cols = 1;
  else
    t.yz_cols = g.yz_cols ? g.yz_cols : (g.layout != RIPPLE_FV_AOS ? 2 : 1);
  if (t.yz_cols == 4 && g.layout == RIPPLE_FV_AOS) t.yz_cols = 2;
  t.split_xy = g.split_xy;
  return t;
}

// A descriptor must have been through ripple_fv_grid_init (pitch, bytes filled).
ripple_fv_status grid_ok(ripple_fv_ctx* ctx, const ripple_fv_grid* g) {
  if (!g) return fail(ctx, RIPPLE_FV_E_INVALID, "NULL grid");
  int64_t pitch[3], bytes;
  int32_t ox;
  std::string why;
  ripple_fv_status st = grid_check(g, pitch, &bytes, &ox, &why);
  if (st != RIPPLE_FV_OK) return fail(ctx, st, why);
  if (pitch[0] != g->pitch[0] || pitch[1] != g->pitch[1] || pitch[2] != g->pitch[2] ||
      bytes != g->bytes || ox != g->x_origin)
    return fail(ctx, RIPPLE_FV_E_INVALID, "grid not initialised (call ripple_fv_grid_init)");
  return RIPPLE_FV_OK;
}

// Device pointer check: non-NULL, 256-byte aligned (state buffers), and inside a
// device allocation with at least `bytes` bytes from it.
ripple_fv_status ptr_ok(ripple_fv_ctx* ctx, const void* p, int64_t bytes, int64_t align,
                        const char* what) {
  if (!p) return fail(ctx, RIPPLE_FV_E_INVALID, std::string("NULL ") + what);
  if (reinterpret_cast<uintptr_t>(p) % align != 0)
    return fail(ctx, RIPPLE_FV_E_INVALID, std::string(what) + " misaligned");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess || !base) {
    (void)hipGetLastError();
    return fail(ctx, RIPPLE_FV_E_INVALID, std::string(what) + " is not device memory");
  }
  const char* b = static_cast<const char*>(base);
  const char* q = static_cast<const char*>(p);
  if (q < b || q + bytes > b + size)
    return fail(ctx, RIPPLE_FV_E_INVALID, std::string(what) + " is smaller than required");
  return RIPPLE_FV_OK;
}

// Cell slots per buffer (the SoA component stride).
int64_t cell_slots(const ripple_fv_grid& g) {
  return g.bytes / (5 * (g.dtype == RIPPLE_FV_F32 ? 4 : 8));
}

Desc desc_of(const ripple_fv_grid& g, const void* buf) {
  Desc d;
  d.buf = const_cast<void*>(buf);
  for (int i = 0; i < 3; ++i) d.n[i] = g.n[i];
  d.lay = lay_of(g);
  d.dtype = g.dtype;
  d.ox = g.x_origin;
  d.px = g.pitch[0];
  d.pxy = g.pitch[0] * g.pitch[1];
  d.ptot = cell_slots(g);
  return d;
}

int group_of(const ripple_fv_grid& g, int index) { return g.group < 0 ? index : g.group; }

// Plan key: the descriptors' bytes (buffer pointers are not part of it).
std::string plan_key(int n, const ripple_fv_grid* grids) {
  return std::string(reinterpret_cast<const char*>(grids), sizeof(ripple_fv_grid) * (size_t)n);
}

ripple_fv_status validate_batch(ripple_fv_ctx* ctx, int n, const ripple_fv_grid* grids) {
  if (n < 1 || !grids) return fail(ctx, RIPPLE_FV_E_INVALID, "empty batch");
  for (int g = 0; g < n; ++g) {
    ripple_fv_status st = grid_ok(ctx, &grids[g]);
    if (st) return st;
  }
  const ripple_fv_grid& g0 = grids[0];
  for (int g = 1; g < n; ++g) {
    const ripple_fv_grid& G = grids[g];
    if (G.dtype != g0.dtype || G.layout != g0.layout || G.aosoa_w != g0.aosoa_w)
      return fail(ctx, RIPPLE_FV_E_UNSUPPORTED, "grids of a batch must share layout and dtype");
    if (G.x_block != g0.x_block || G.yz_block != g0.yz_block || G.yz_segment != g0.yz_segment ||
        G.persist != g0.persist || G.yz_cols != g0.yz_cols || G.split_xy != g0.split_xy)
      return fail(ctx, RIPPLE_FV_E_UNSUPPORTED, "grids of a batch must share tiling knobs");
  }
  for (int g = 0; g < n; ++g) {
    const ripple_fv_grid& G = grids[g];
    const int grp = group_of(G, g);
    if (grp < 0 || grp >= n) return fail(ctx, RIPPLE_FV_E_INVALID, "group index out of range");
    if (group_of(grids[grp], grp) != grp)
      return fail(ctx, RIPPLE_FV_E_INVALID, "group leader must belong to its own group");
    for (int d = 0; d < 3; ++d)
      if (grids[grp].dx[d] != G.dx[d])
        return fail(ctx, RIPPLE_FV_E_INVALID, "grids of a group must share dx");
    for (int f = 0; f < 6; ++f) {
      const int h = G.nbr[f];
      if (h < 0) {
        if (h != -1) return fail(ctx, RIPPLE_FV_E_INVALID, "bad neighbour index");
        continue;
      }
      if (h >= n) return fail(ctx, RIPPLE_FV_E_INVALID, "neighbour index out of range");
      const int axis = f / 2;
      const ripple_fv_grid& H = grids[h];
      for (int d = 0; d < 3; ++d)
        if (d != axis && H.n[d] != G.n[d])
          return fail(ctx, RIPPLE_FV_E_INVALID, "linked sub-blocks must match across the face");
      if (H.nbr[f ^ 1] != g)
        return fail(ctx, RIPPLE_FV_E_INVALID, "sub-block links must be reciprocal");
      if (H.n[axis] < 2) return fail(ctx, RIPPLE_FV_E_INVALID, "neighbour too thin");
    }
  }
  return RIPPLE_FV_OK;
}

// The launch shape of a validated batch, computed on the host into caller
// storage (no allocation): tiles[k] hold n + 1 prefix sums each, halo[k] up
// to 2 n tasks each, h_grids n descriptors (buffer pointers left null).
void plan_shape(PlanCore& P, int n, const ripple_fv_grid* grids, int64_t* const tiles[5],
                HaloTask* const halo[3], DevGrid* h_grids, int cu_count) {
  P.n = n;
  P.dtype = grids[0].dtype;
  P.lay = lay_of(grids[0]);
  P.tl = tiling_of(grids[0]);
  P.grids = grids;
  // Grids one cell thick in z skip the z sweep.  Their x and y sweeps run
  // as one pass in the wave-strip form (whatever split_xy other than 1 asks
  // for: the rows form does not reduce wave speeds), which is then the whole
  // step and reduces the next step's wave speeds; with split_xy = 1 or rows
  // under XY_MIN_NX cells they run separately and the y sweep reduces them.
  P.planar = true;
  for (int g = 0; g < n; ++g) P.planar = P.planar && grids[g].n[2] == 1;
  P.fused = P.tl.split_xy != 1 && !P.planar;
  P.planar_fused = P.tl.split_xy != 1 && P.planar;
  for (int g = 0; g < n; ++g) {
    P.fused = P.fused && xy_eligible(grids[g]);
    P.planar_fused = P.planar_fused && xy_eligible(grids[g]);
  }
  // The fused pass marches tiles of seg_xy rows along y.  Where that leaves
  // fewer than XY_MIN_TILES tiles (thin or two-dimensional grids) the
  // segments shrink, down to 16 rows (or the configured segment if that is
  // shorter), so that the launch fills the device.
  P.seg_xy = P.tl.yz_segment;
  P.xmode = XM_ROWS;
  if (P.fused) P.xmode = xy_mode(P.dtype, grids, n, P.tl.split_xy);
  if (P.planar_fused) P.xmode = XM_WAVES;
  if (P.fused || P.planar_fused) {
    int64_t count = 0;
    for (int g = 0; g < n; ++g) count += tiles_xy(grids[g], P.seg_xy, P.xmode);
    if (count < XY_MIN_TILES)
      P.seg_xy = (int)std::max<int64_t>(std::min(16, P.seg_xy),
                                        (int64_t)P.seg_xy * count / XY_MIN_TILES);
  }
  // The z sweep marches tiles of seg_z cells.  Unless the grids set a
  // segment, it takes the longest segment (the fewest per column) that
  // leaves at least Z_MIN_TILES_PER_CU tiles per compute unit (down to
  // Z_MIN_SEGMENT cells), provided those tiles then take about one round (at
  // most Z_ROUND_TILES_PER_CU per compute unit; three workgroups of the z
  // sweep fit a CU in FP32 and FP64); otherwise the library's 128-cell
  // segment.  A tile then re-reads its 4 halo cells over more cells, and the
  // launch has no long, partly filled last round.  Measured on the z sweep:
  // 512^3 FP32 1.115 ms with 128-cell segments (2048 tiles), 1.137 with 256
  // (1024), 1.059 with whole columns (512 tiles); 512^3 FP64 2.23-2.24 ms
  // with 128, 2.157 with whole columns (1024 tiles); 256^3 FP32 0.171 ms
  // with 128 (256 tiles), 0.136 with 64 (512); 256^3 FP64 0.278 ms with 128
  // (512 tiles), 0.290 with 64 and with 256; the 64-grid batch 0.937 ms with
  // 128 (2328 tiles), 0.971 with whole columns (1575 tiles: two rounds and a
  // few).
  P.seg_z = P.tl.yz_segment;
  if (grids[0].yz_segment == 0) {
    int nzmax = 1;
    for (int g = 0; g < n; ++g) nzmax = std::max(nzmax, grids[g].n[2]);
    for (int parts = 1;; ++parts) {
      const int seg = (nzmax + parts - 1) / parts;
      int64_t count = 0;
      for (int g = 0; g < n; ++g) count += tiles_yz(grids[g], 2, P.tl.yz_block, seg, P.tl.yz_cols);
      if (count >= (int64_t)Z_MIN_TILES_PER_CU * cu_count || seg <= Z_MIN_SEGMENT) {
        const bool one_round = count <= (int64_t)Z_ROUND_TILES_PER_CU * cu_count;
        P.seg_z = one_round ? std::max(seg, std::min(Z_MIN_SEGMENT, nzmax))
                            : std::min(seg, P.tl.yz_segment);
        break;
      }
    }
  }
  for (int k = 0; k < 5; ++k) tiles[k][0] = 0;
  for (int g = 0; g < n; ++g) {
    tiles[4][g + 1] = tiles[4][g] + (P.fused || P.planar_fused ? tiles_xy(grids[g], P.seg_xy, P.xmode) : 0);
    tiles[0][g + 1] = tiles[0][g] + tiles_x(grids[g], P.tl.x_block);
    tiles[1][g + 1] = tiles[1][g] + tiles_yz(grids[g], 1, P.tl.yz_block, P.tl.yz_segment, P.tl.yz_cols);
    tiles[2][g + 1] = tiles[2][g] + tiles_yz(grids[g], 2, P.tl.yz_block, P.seg_z, P.tl.yz_cols);
    tiles[3][g + 1] = tiles[3][g] + tiles_ws(grids[g]);
  }
  for (int k = 0; k < 5; ++k) P.tiles[k] = tiles[k];
  for (int axis = 0; axis < 3; ++axis) {
    int count = 0;
    P.halo_area[axis] = 0;
    for (int g = 0; g < n; ++g) {
      const ripple_fv_grid& G = grids[g];
      for (int side = 0; side < 2; ++side) {
        const int h = G.nbr[2 * axis + side];
        if (h < 0) continue;
        HaloTask t;
        t.dst = g;
        t.src = h;
        t.side = side;
        t.pad_ = 0;
        halo[axis][count++] = t;
        const int64_t area = (int64_t)G.n[axis == 0 ? 1 : 0] * G.n[axis == 2 ? 1 : 2];
        P.halo_area[axis] = std::max(P.halo_area[axis], area);
      }
    }
    P.nhalo[axis] = count;
    P.halo[axis] = halo[axis];
  }
  for (int g = 0; g < n; ++g) {
    const ripple_fv_grid& G = grids[g];
    DevGrid& D = h_grids[g];
    std::memset(&D, 0, sizeof(D));
    for (int d = 0; d < 3; ++d) {
      D.n[d] = G.n[d];
      D.dx[d] = G.dx[d];
      for (int side = 0; side < 2; ++side) {
        const int f = 2 * d + side;
        // a one-cell axis is its own periodic image: transmissive and periodic
        // faces then read the same cell
        D.mode[f] = G.nbr[f] >= 0 ? FACE_HALO
                    : (G.bc[d] == RIPPLE_FV_PERIODIC && G.n[d] >= 2 ? FACE_PERIODIC
                                                                     : FACE_TRANSMISSIVE);
      }
    }
    D.px = G.pitch[0];
    D.pxy = G.pitch[0] * G.pitch[1];
    D.ptot = cell_slots(G);
    D.ox = G.x_origin;
    D.group = group_of(G, g);
    D.nbr_x[0] = G.nbr[0];
    D.nbr_x[1] = G.nbr[1];
  }
  P.h_grids = h_grids;
}

// Dispatch order of the batched launch of kind k (1: y sweep, 2: z sweep, 4:
// fused x-y pass) from the cells each tile marches (dispatch_order in
// fv_index.hpp); a tile costs those cells plus the 4 halo cells and about 2
// of pipeline fill.
void tile_order(const PlanCore& P, int k, std::vector<int32_t>& order) {
  std::vector<int32_t> cost((size_t)P.tiles[k][P.n]);
  for (int g = 0; g < P.n; ++g) {
    const ripple_fv_grid& G = P.grids[g];
    for (int64_t t = P.tiles[k][g]; t < P.tiles[k][g + 1]; ++t) {
      const int64_t lt = t - P.tiles[k][g];
      const int len = k == 4 ? tile_len_xy(G, P.seg_xy, lt)
                             : tile_len_yz(G, k, P.tl.yz_block, k == 2 ? P.seg_z : P.tl.yz_segment,
                                           P.tl.yz_cols, lt);
      cost[(size_t)t] = len + 2 * HALO + 2;
    }
  }
  dispatch_order(cost, NXCD, order);
}

ripple_fv_status build_plan(ripple_fv_ctx* ctx, int n, const ripple_fv_grid* grids, Plan** out) {
  const std::string key = plan_key(n, grids);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    *out = it->second.get();
    return RIPPLE_FV_OK;
  }
  std::unique_ptr<Plan> P(new Plan());
  P->grid_store.assign(grids, grids + n);
  int64_t* tiles[5];
  HaloTask* halo[3];
  for (int k = 0; k < 5; ++k) {
    P->tile_store[k].assign(n + 1, 0);
    tiles[k] = P->tile_store[k].data();
  }
  for (int k = 0; k < 3; ++k) {
    P->halo_store[k].resize(2 * (size_t)n);
    halo[k] = P->halo_store[k].data();
  }
  P->h_grid_store.resize(n);
  plan_shape(*P, n, P->grid_store.data(), tiles, halo, P->h_grid_store.data(), ctx->cu_count);
  for (int k : {1, 2, 4}) {
    if (P->tiles[k][n] == 0) continue;
    tile_order(*P, k, P->order_store[k]);
    if (P->order_store[k].empty()) continue;
    P->order[k] = P->order_store[k].data();
    P->nslots[k] = (int64_t)P->order_store[k].size();
  }
  // device workspace
  const WsLayout L = ws_layout(n, P->nhalo, P->nslots);
  if (hipMalloc(&P->dmem, L.total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RIPPLE_FV_E_NOMEM, "plan workspace allocation failed");
  }
  ws_bind(*P, static_cast<char*>(P->dmem), L);
  for (int k = 0; k < 5; ++k)
    HIP_OR_FAIL(ctx, hipMemcpy(P->d_tiles[k], P->tiles[k], sizeof(int64_t) * (n + 1),
                               hipMemcpyHostToDevice));
  for (int k = 0; k < 3; ++k)
    if (P->nhalo[k])
      HIP_OR_FAIL(ctx, hipMemcpy(P->d_halo[k], P->halo[k], sizeof(HaloTask) * P->nhalo[k],
                                 hipMemcpyHostToDevice));
  for (int k = 0; k < 5; ++k)
    if (P->nslots[k])
      HIP_OR_FAIL(ctx, hipMemcpy(P->d_order[k], P->order[k], sizeof(int32_t) * P->nslots[k],
                                 hipMemcpyHostToDevice));
  HIP_OR_FAIL(ctx, hipMemset(P->d_lam, 0, sizeof(double) * 3 * n));
  HIP_OR_FAIL(ctx, hipMemset(P->d_t, 0, sizeof(double) * n));
  HIP_OR_FAIL(ctx, hipMemset(P->d_dt, 0, sizeof(double) * n));
  HIP_OR_FAIL(ctx, hipMemset(P->d_s, 0, sizeof(unsigned long long) * 3 * n));
  HIP_OR_FAIL(ctx, hipHostMalloc(reinterpret_cast<void**>(&P->h_pinned), sizeof(DevGrid) * n,
                                 hipHostMallocDefault));
  HIP_OR_FAIL(ctx, hipEventCreateWithFlags(&P->upload_done, hipEventDisableTiming));
  if ((int)ctx->plans.size() >= MAX_PLANS) {
    HIP_OR_FAIL(ctx, hipDeviceSynchronize());
    ctx->plans.erase(ctx->plan_order.front());
    ctx->plan_order.pop_front();
  }
  *out = P.get();
  ctx->plan_order.push_back(key);
  ctx->plans[key] = std::move(P);
  return RIPPLE_FV_OK;
}

// Put the current buffer pointers into the plan's device descriptors
// (stream-ordered; skipped when unchanged since the last upload).
ripple_fv_status upload_buffers(ripple_fv_ctx* ctx, Plan* P, void* const* a, void* const* b,
                                hipStream_t s) {
  bool changed = !P->uploaded;
  for (int g = 0; g < P->n; ++g) {
    void* na = a[g];
    void* nb = b ? b[g] : nullptr;
    DevGrid& D = P->h_grid_store[g];
    if (D.buf[0] != na || D.buf[1] != nb) changed = true;
    D.buf[0] = na;
    D.buf[1] = nb;
  }
  if (!changed) return RIPPLE_FV_OK;
  if (P->upload_pending) HIP_OR_FAIL(ctx, hipEventSynchronize(P->upload_done));
  std::memcpy(P->h_pinned, P->h_grid_store.data(), sizeof(DevGrid) * P->n);
  HIP_OR_FAIL(ctx, hipMemcpyAsync(P->d_grids, P->h_pinned, sizeof(DevGrid) * P->n,
                                  hipMemcpyHostToDevice, s));
  HIP_OR_FAIL(ctx, hipEventRecord(P->upload_done, s));
  P->upload_pending = true;
  P->uploaded = true;
  return RIPPLE_FV_OK;
}

int blocks_for(const ripple_fv_ctx* ctx, const Tiling& tl, int64_t tiles) {
  int64_t b = tiles;
  if (tl.persist > 0) b = std::min<int64_t>(tiles, (int64_t)tl.persist * ctx->cu_count);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 0x7fffffff));
}

// Workgroups of a launch through a dispatch order of `slots` entries (a
// multiple of NXCD): one per slot, or with persistent launches as many as
// fit, rounded down to a multiple of NXCD so that each workgroup's slots lie
// on its own XCD.
int blocks_for_slots(const ripple_fv_ctx* ctx, const Tiling& tl, int64_t slots) {
  int64_t b = slots;
  if (tl.persist > 0) b = std::min<int64_t>(slots, (int64_t)tl.persist * ctx->cu_count);
  b = std::min<int64_t>(b, 0x7fffffff) / NXCD * NXCD;
  return (int)std::max<int64_t>(NXCD, b);
}

// Set a batched launch of kind k over all tiles, through the plan's dispatch
// order where it has one; returns the workgroup count.
int batched_range(const ripple_fv_ctx* ctx, const PlanCore* P, int k, TileRange& r) {
  r.first = 0;
  r.count = P->tiles[k][P->n];
  r.order = P->d_order[k];
  r.slots = r.order ? P->nslots[k] : 0;
  return r.order ? blocks_for_slots(ctx, P->tl, r.slots) : blocks_for(ctx, P->tl, r.count);
}

// Launches of one kernel kind, optionally bracketed by profiling events.
struct Launcher {
  ripple_fv_ctx* ctx;
  hipStream_t s;
  bool profile;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> marks;
  size_t next_event = 0;
  ripple_fv_status begin(int kind, hipEvent_t* e1) {
    if (!profile) return RIPPLE_FV_OK;
    if (next_event + 2 > ctx->events.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        HIP_OR_FAIL(ctx, hipEventCreate(&e));
        ctx->events.push_back(e);
      }
    }
    hipEvent_t a = ctx->events[next_event], b = ctx->events[next_event + 1];
    next_event += 2;
    HIP_OR_FAIL(ctx, hipEventRecord(a, s));
    marks.push_back({kind, {a, b}});
    *e1 = b;
    return RIPPLE_FV_OK;
  }
  ripple_fv_status end(hipEvent_t e1) {
    if (!profile) return RIPPLE_FV_OK;
    HIP_OR_FAIL(ctx, hipEventRecord(e1, s));
    return RIPPLE_FV_OK;
  }
  ripple_fv_status collect() {
    if (!profile || marks.empty()) return RIPPLE_FV_OK;
    HIP_OR_FAIL(ctx, hipEventSynchronize(marks.back().second.second));
    for (auto& m : marks) {
      float ms = 0.f;
      HIP_OR_FAIL(ctx, hipEventElapsedTime(&ms, m.second.first, m.second.second));
      ctx->prof_ms[m.first] += ms;
      ctx->prof_n[m.first] += 1;
    }
    marks.clear();
    next_event = 0;
    return RIPPLE_FV_OK;
  }
};

#define LAUNCH_OR_FAIL(ctx, call) HIP_OR_FAIL(ctx, call)

// Enqueue one sweep along `axis` for every grid (persistent launch over the
// batch's tile list, or one launch per grid).
ripple_fv_status enqueue_sweep(ripple_fv_ctx* ctx, const PlanCore* P, Launcher& L, int axis, int in, int out,
                               int fuse_s, bool per_grid) {
  SweepParams sp{};
  sp.w = P->work(ctx->flag);
  sp.in = in;
  sp.out = out;
  sp.seg = axis == 2 ? P->seg_z : P->tl.yz_segment;
  sp.fuse_s = fuse_s;
  sp.tiles.tile_start = P->d_tiles[axis];
  hipEvent_t e1 = nullptr;
  ripple_fv_status st = L.begin(RIPPLE_FV_K_SWEEP_X + axis, &e1);
  if (st) return st;
  const int64_t* pre = P->tiles[axis];
  if (per_grid) {
    for (int g = 0; g < P->n; ++g) {
      sp.tiles.first = pre[g];
      sp.tiles.count = pre[g + 1] - pre[g];
      LAUNCH_OR_FAIL(ctx, launch_sweep(P->dtype, P->lay, axis, P->tl, sp,
                                       blocks_for(ctx, P->tl, sp.tiles.count), L.s));
    }
  } else {
    const int blocks = batched_range(ctx, P, axis, sp.tiles);
    LAUNCH_OR_FAIL(ctx, launch_sweep(P->dtype, P->lay, axis, P->tl, sp, blocks, L.s));
  }
  return L.end(e1);
}

// Enqueue the fused x-then-y sweep (plans whose grids all allow it).
ripple_fv_status enqueue_sweep_xy(ripple_fv_ctx* ctx, const PlanCore* P, Launcher& L, int in, int out,
                                  int fuse_s, bool per_grid) {
  SweepParams sp{};
  sp.w = P->work(ctx->flag);
  sp.in = in;
  sp.out = out;
  sp.seg = P->seg_xy;
  sp.fuse_s = fuse_s;
  sp.xmode = P->xmode;
  sp.link_x = 0;
  for (int g = 0; g < P->n; ++g)
    if (P->h_grids[g].mode[0] == FACE_HALO || P->h_grids[g].mode[1] == FACE_HALO) sp.link_x = 1;
  sp.tiles.tile_start = P->d_tiles[4];
  hipEvent_t e1 = nullptr;
  ripple_fv_status st = L.begin(RIPPLE_FV_K_SWEEP_XY, &e1);
  if (st) return st;
  const int64_t* pre = P->tiles[4];
  if (per_grid) {
    for (int g = 0; g < P->n; ++g) {
      sp.tiles.first = pre[g];
      sp.tiles.count = pre[g + 1] - pre[g];
      LAUNCH_OR_FAIL(ctx, launch_sweep_xy(P->dtype, P->lay, P->tl, sp,
                                          blocks_for(ctx, P->tl, sp.tiles.count), L.s));
    }
  } else {
    const int blocks = batched_range(ctx, P, 4, sp.tiles);
    LAUNCH_OR_FAIL(ctx, launch_sweep_xy(P->dtype, P->lay, P->tl, sp, blocks, L.s));
  }
  return L.end(e1);
}

ripple_fv_status enqueue_halo(ripple_fv_ctx* ctx, const PlanCore* P, Launcher& L, int axis, int buf,
                              int ext = 0) {
  if (P->nhalo[axis] == 0) return RIPPLE_FV_OK;
  hipEvent_t e1 = nullptr;
  ripple_fv_status st = L.begin(RIPPLE_FV_K_HALO, &e1);
  if (st) return st;
  LAUNCH_OR_FAIL(ctx, launch_halo(P->dtype, P->lay, P->work(ctx->flag), buf, axis, ext,
                                  P->d_halo[axis], P->nhalo[axis],
                                  P->halo_area[axis], L.s));
  return L.end(e1);
}

ripple_fv_status enqueue_wavespeed(ripple_fv_ctx* ctx, const PlanCore* P, Launcher& L, int buf,
                                   unsigned long long* s_out, bool per_grid) {
  hipEvent_t e1 = nullptr;
  ripple_fv_status st = L.begin(RIPPLE_FV_K_WAVESPEED, &e1);
  if (st) return st;
  TileRange tr{};
  tr.tile_start = P->d_tiles[3];
  const int64_t* pre = P->tiles[3];
  Tiling tl = P->tl;
  if (per_grid) {
    for (int g = 0; g < P->n; ++g) {
      tr.first = pre[g];
      tr.count = pre[g + 1] - pre[g];
      LAUNCH_OR_FAIL(ctx, launch_wavespeed(P->dtype, P->lay, P->work(ctx->flag), buf, tr, s_out,
                                           blocks_for(ctx, tl, tr.count), L.s));
    }
  } else {
    tr.first = 0;
    tr.count = pre[P->n];
    LAUNCH_OR_FAIL(ctx, launch_wavespeed(P->dtype, P->lay, P->work(ctx->flag), buf, tr, s_out,
                                         blocks_for(ctx, tl, tr.count), L.s));
  }
  return L.end(e1);
}

ripple_fv_status enqueue_dt(ripple_fv_ctx* ctx, const PlanCore* P, Launcher& L, double cfl, double fixed_dt,
                            int reset_s, double* dt_out) {
  hipEvent_t e1 = nullptr;
  ripple_fv_status st = L.begin(RIPPLE_FV_K_DT, &e1);
  if (st) return st;
  LAUNCH_OR_FAIL(ctx, launch_dt(P->work(ctx->flag), cfl, fixed_dt, reset_s, dt_out, L.s));
  return L.end(e1);
}

// One step starting from buffer `cur`: dt, then x (cur -> oth), y (oth -> cur),
// z (cur -> oth) with the new state's wave speeds folded into the slots; or,
// in a fused plan, x-y (cur -> oth) and z (oth -> cur).
ripple_fv_status enqueue_step(ripple_fv_ctx* ctx, const PlanCore* P, Launcher& L, int cur, double cfl,
                              double fixed_dt, double* dt_out, bool per_grid) {
  const int oth = 1 - cur;
  ripple_fv_status st = enqueue_dt(ctx, P, L, cfl, fixed_dt, 1, dt_out);
  if (P->fused) {
    // the fused pass x-sweeps the y padding rows itself: they take the raw
    // neighbour rows first; its lanes past a linked x face read the x
    // neighbour's cells directly (its y padding rows holding the corners), so
    // no x copy precedes it
    if (!st) st = enqueue_halo(ctx, P, L, 1, cur);
    if (!st) st = enqueue_sweep_xy(ctx, P, L, cur, oth, 0, per_grid);
    if (!st) st = enqueue_halo(ctx, P, L, 2, oth);
    if (!st) st = enqueue_sweep(ctx, P, L, 2, oth, cur, 1, per_grid);
    return st;
  }
  if (P->planar_fused) {
    // a sweep along a one-cell axis changes nothing (see below): the x-y
    // pass is the whole step and reduces the next step's wave speeds
    if (!st) st = enqueue_halo(ctx, P, L, 1, cur);
    if (!st) st = enqueue_sweep_xy(ctx, P, L, cur, oth, 1, per_grid);
    return st;
  }
  if (!st) st = enqueue_halo(ctx, P, L, 0, cur);
  if (!st) st = enqueue_sweep(ctx, P, L, 0, cur, oth, 0, per_grid);
  if (!st) st = enqueue_halo(ctx, P, L, 1, oth);
  if (P->planar) {
    // a sweep along a one-cell axis reads the same state on both faces of
    // every cell and leaves it unchanged bit for bit: skip it, and let the y
    // sweep reduce the wave speeds for the next step instead
    if (!st) st = enqueue_sweep(ctx, P, L, 1, oth, cur, 1, per_grid);
    return st;
  }
  if (!st) st = enqueue_sweep(ctx, P, L, 1, oth, cur, 0, per_grid);
  if (!st) st = enqueue_halo(ctx, P, L, 2, cur);
  if (!st) st = enqueue_sweep(ctx, P, L, 2, cur, oth, 1, per_grid);
  return st;
}

// After an odd number of separate-sweep steps the state is in the work
// buffers: copy it back.
ripple_fv_status enqueue_copy_back(ripple_fv_ctx* ctx, const PlanCore* P, hipStream_t s) {
  for (int g = 0; g < P->n; ++g)
    HIP_OR_FAIL(ctx, hipMemcpyAsync(P->h_grids[g].buf[0], P->h_grids[g].buf[1], P->grids[g].bytes,
                                    hipMemcpyDeviceToDevice, s));
  return RIPPLE_FV_OK;
}

ripple_fv_status capture_graph(ripple_fv_ctx* ctx, Plan* P, int nsteps, double cfl, bool per_grid,
                               hipGraphExec_t* out) {
  hipStream_t cs = ctx->cap_stream;
  HIP_OR_FAIL(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  Launcher L{ctx, cs, false, {}, 0};
  ripple_fv_status st = RIPPLE_FV_OK;
  for (int k = 0; k < nsteps && !st; ++k)
    st = enqueue_step(ctx, P, L, P->in_place() ? 0 : (k & 1), cfl, 0.0, nullptr, per_grid);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (st) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(ctx, RIPPLE_FV_E_DEVICE, std::string("capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(ctx, RIPPLE_FV_E_DEVICE, std::string("instantiate: ") + hipGetErrorString(e));
  return RIPPLE_FV_OK;
}

ripple_fv_status set_device(ripple_fv_ctx* ctx) {
  if (!ctx) return RIPPLE_FV_E_INVALID;
  ctx->err.clear();
  HIP_OR_FAIL(ctx, hipSetDevice(ctx->device));
  return RIPPLE_FV_OK;
}

// Shared body of ripple_fv_run_batch / ripple_fv_step.
ripple_fv_status run(ripple_fv_ctx* ctx, int n, const ripple_fv_grid* grids, void* const* u_a,
                     void* const* u_b, int nsteps, double cfl, double fixed_dt, double* dt_out,
                     int flags, hipStream_t s) {
  if (nsteps < 0) return fail(ctx, RIPPLE_FV_E_INVALID, "nsteps < 0");
  if (fixed_dt > 0.0) {
    if (!std::isfinite(fixed_dt)) return fail(ctx, RIPPLE_FV_E_INVALID, "dt not finite");
  } else if (!(cfl > 0.0 && cfl <= 1.0)) {
    return fail(ctx, RIPPLE_FV_E_INVALID, "cfl must be in (0, 1]");
  }
  if (std::isnan(fixed_dt)) return fail(ctx, RIPPLE_FV_E_INVALID, "dt is NaN");
  if (flags & ~(RIPPLE_FV_RUN_GRAPH | RIPPLE_FV_RUN_PER_GRID | RIPPLE_FV_RUN_PROFILE))
    return fail(ctx, RIPPLE_FV_E_INVALID, "unknown flags");
  if ((flags & RIPPLE_FV_RUN_GRAPH) && (flags & RIPPLE_FV_RUN_PROFILE))
    return fail(ctx, RIPPLE_FV_E_INVALID, "GRAPH and PROFILE are exclusive");
  ripple_fv_status st = validate_batch(ctx, n, grids);
  if (st) return st;
  if (!u_a || !u_b) return fail(ctx, RIPPLE_FV_E_INVALID, "NULL buffer list");
  for (int g = 0; g < n; ++g) {
    if ((st = ptr_ok(ctx, u_a[g], grids[g].bytes, 256, "u"))) return st;
    if ((st = ptr_ok(ctx, u_b[g], grids[g].bytes, 256, "work"))) return st;
    if (u_a[g] == u_b[g]) return fail(ctx, RIPPLE_FV_E_INVALID, "u and work alias");
  }
  Plan* P = nullptr;
  if ((st = build_plan(ctx, n, grids, &P))) return st;
  if ((st = upload_buffers(ctx, P, u_a, u_b, s))) return st;
  if (nsteps == 0) return RIPPLE_FV_OK;
  const bool per_grid = flags & RIPPLE_FV_RUN_PER_GRID;
  Launcher L{ctx, s, (flags & RIPPLE_FV_RUN_PROFILE) != 0, {}, 0};
  LAUNCH_OR_FAIL(ctx, launch_fill_f64(P->d_t, n, 0.0, s));
  if (!(fixed_dt > 0.0)) {
    LAUNCH_OR_FAIL(ctx, launch_fill_u64(P->d_s, 3 * (int64_t)n, 0ull, s));
    if ((st = enqueue_wavespeed(ctx, P, L, 0, nullptr, per_grid))) return st;
  }
  if ((flags & RIPPLE_FV_RUN_GRAPH) && !(fixed_dt > 0.0) && !dt_out) {
    if (P->graph_cfl != cfl || P->graph_per_grid != per_grid) {
      P->drop_graphs();
      P->graph_cfl = cfl;
      P->graph_per_grid = per_grid;
    }
    // whole step loops of up to GRAPH_MAX_STEPS steps per graph launch (an
    // even count on the separate-sweep path, whose steps alternate buffers),
    // then one graph for the remainder; graphs are cached by step count
    int chunk = std::min(nsteps, GRAPH_MAX_STEPS);
    if (!P->in_place() && chunk > 1) chunk &= ~1;
    auto graph_for = [&](int k, hipGraphExec_t* out) -> ripple_fv_status {
      auto it = P->graphs.find(k);
      if (it != P->graphs.end()) {
        *out = it->second;
        return RIPPLE_FV_OK;
      }
      ripple_fv_status s2 = capture_graph(ctx, P, k, cfl, per_grid, out);
      if (!s2) P->graphs[k] = *out;
      return s2;
    };
    const int rem = nsteps % chunk;
    if ((int)P->graphs.size() + 2 > MAX_GRAPHS && (!P->graphs.count(chunk) || (rem && !P->graphs.count(rem))))
      P->drop_graphs();
    hipGraphExec_t gc = nullptr, gr = nullptr;
    if ((st = graph_for(chunk, &gc))) return st;
    if (rem && (st = graph_for(rem, &gr))) return st;
    for (int k = 0; k + chunk <= nsteps; k += chunk) HIP_OR_FAIL(ctx, hipGraphLaunch(gc, s));
    if (rem) HIP_OR_FAIL(ctx, hipGraphLaunch(gr, s));
    // (the copy back stays outside the graphs: its pointers change with the buffers)
    if (!P->in_place() && (nsteps & 1)) return enqueue_copy_back(ctx, P, s);
    return RIPPLE_FV_OK;
  }
  for (int k = 0; k < nsteps; ++k) {
    if ((st = enqueue_step(ctx, P, L, P->in_place() ? 0 : (k & 1), cfl, fixed_dt, dt_out, per_grid)))
      return st;
  }
  if (!P->in_place() && (nsteps & 1) && (st = enqueue_copy_back(ctx, P, s))) return st;
  return L.collect();
}

}  // namespace

namespace rfv {

ripple_fv_status ctx_begin(ripple_fv_ctx* ctx) { return set_device(ctx); }

ripple_fv_status ctx_fail(ripple_fv_ctx* ctx, ripple_fv_status st, const char* msg) {
  return fail(ctx, st, msg);
}

ripple_fv_status ctx_ptr_ok(ripple_fv_ctx* ctx, const void* p, int64_t bytes, int64_t align,
                            const char* what) {
  return ptr_ok(ctx, p, bytes, align, what);
}

}  // namespace rfv

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

ripple_fv_status ripple_fv_grid_init(ripple_fv_grid* g) {
  if (!g) return RIPPLE_FV_E_INVALID;
  int64_t pitch[3], bytes;
  int32_t ox;
  std::string why;
  ripple_fv_status st = grid_check(g, pitch, &bytes, &ox, &why);
  if (st) return st;
  for (int d = 0; d < 3; ++d) g->pitch[d] = pitch[d];
  g->bytes = bytes;
  g->x_origin = ox;
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_create(ripple_fv_ctx** out, int32_t device) {
  if (!out) return RIPPLE_FV_E_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return RIPPLE_FV_E_DEVICE;
  }
  if (device < 0 || device >= count) return RIPPLE_FV_E_INVALID;
  std::unique_ptr<ripple_fv_ctx> ctx(new ripple_fv_ctx());
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) return RIPPLE_FV_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return RIPPLE_FV_E_DEVICE;
  ctx->cu_count = prop.multiProcessorCount;
  if (hipMalloc(&ctx->flag, 256) != hipSuccess) return RIPPLE_FV_E_NOMEM;
  if (hipMemset(ctx->flag, 0, 256) != hipSuccess) return RIPPLE_FV_E_DEVICE;
  if (hipMalloc(&ctx->partials, sizeof(double) * DIAG_MAX_BLOCKS * 20) != hipSuccess)
    return RIPPLE_FV_E_NOMEM;
  if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return RIPPLE_FV_E_DEVICE;
  if (scratch_address(device, &ctx->scratch) != hipSuccess) {
    (void)hipGetLastError();
    return RIPPLE_FV_E_DEVICE;
  }
  *out = ctx.release();
  return RIPPLE_FV_OK;
}

void ripple_fv_destroy(ripple_fv_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  ctx->plans.clear();
  for (hipEvent_t e : ctx->events) hipEventDestroy(e);
  if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
  if (ctx->partials) hipFree(ctx->partials);
  if (ctx->flag) hipFree(ctx->flag);
  delete ctx;
}

ripple_fv_status ripple_fv_import(ripple_fv_ctx* ctx, const ripple_fv_grid* g, const double* src,
                                  int32_t variables, void* u, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  if (variables != RIPPLE_FV_PRIMITIVE && variables != RIPPLE_FV_CONSERVED)
    return fail(ctx, RIPPLE_FV_E_INVALID, "unknown variables kind");
  const int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
  if ((st = ptr_ok(ctx, src, ncell * 5 * 8, 8, "src"))) return st;
  if ((st = ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  HIP_OR_FAIL(ctx, launch_import(desc_of(*g, u), src, variables == RIPPLE_FV_PRIMITIVE,
                                 (hipStream_t)stream));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_export(ripple_fv_ctx* ctx, const ripple_fv_grid* g, const void* u,
                                  double* dst, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  const int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
  if ((st = ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  if ((st = ptr_ok(ctx, dst, ncell * 5 * 8, 8, "dst"))) return st;
  HIP_OR_FAIL(ctx, launch_export(desc_of(*g, u), dst, (hipStream_t)stream));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_convert(ripple_fv_ctx* ctx, const ripple_fv_grid* gs, const void* src,
                                   const ripple_fv_grid* gd, void* dst, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, gs)) || (st = grid_ok(ctx, gd))) return st;
  for (int d = 0; d < 3; ++d)
    if (gs->n[d] != gd->n[d]) return fail(ctx, RIPPLE_FV_E_INVALID, "extents differ");
  if ((st = ptr_ok(ctx, src, gs->bytes, 256, "src"))) return st;
  if ((st = ptr_ok(ctx, dst, gd->bytes, 256, "dst"))) return st;
  if (src == dst) return fail(ctx, RIPPLE_FV_E_INVALID, "src and dst alias");
  HIP_OR_FAIL(ctx, launch_convert(desc_of(*gs, src), desc_of(*gd, dst), (hipStream_t)stream));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_max_wavespeed(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                         const void* u, double* s_dev, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  if ((st = ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  if ((st = ptr_ok(ctx, s_dev, 24, 8, "s_dev"))) return st;
  ripple_fv_grid one = *g;
  one.group = -1;
  for (int f = 0; f < 6; ++f) one.nbr[f] = -1;
  Plan* P = nullptr;
  if ((st = build_plan(ctx, 1, &one, &P))) return st;
  void* a[1] = {const_cast<void*>(u)};
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_buffers(ctx, P, a, nullptr, s))) return st;
  unsigned long long* out = reinterpret_cast<unsigned long long*>(s_dev);
  HIP_OR_FAIL(ctx, launch_fill_u64(out, 3, 0ull, s));
  Launcher L{ctx, s, false, {}, 0};
  return enqueue_wavespeed(ctx, P, L, 0, out, false);
}

ripple_fv_status ripple_fv_sweep(ripple_fv_ctx* ctx, const ripple_fv_grid* g, int32_t axis,
                                 const void* u_in, void* u_out, double dt, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  if (axis < 0 || axis > RIPPLE_FV_AXIS_XY)
    return fail(ctx, RIPPLE_FV_E_INVALID, "axis must be 0, 1, 2 or RIPPLE_FV_AXIS_XY");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, RIPPLE_FV_E_INVALID, "dt must be > 0");
  if ((st = ptr_ok(ctx, u_in, g->bytes, 256, "u_in"))) return st;
  if ((st = ptr_ok(ctx, u_out, g->bytes, 256, "u_out"))) return st;
  if (u_in == u_out) return fail(ctx, RIPPLE_FV_E_INVALID, "u_in and u_out alias");
  // Linked faces read u_in's padding: keep them as halo faces (a self link
  // marks them; the sweep itself copies nothing).
  ripple_fv_grid one = *g;
  one.group = -1;
  for (int f = 0; f < 6; ++f) one.nbr[f] = one.nbr[f] >= 0 ? 0 : -1;
  Plan* P = nullptr;
  if ((st = build_plan(ctx, 1, &one, &P))) return st;
  void* a[1] = {const_cast<void*>(u_in)};
  void* b[1] = {u_out};
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_buffers(ctx, P, a, b, s))) return st;
  Launcher L{ctx, s, false, {}, 0};
  if ((st = enqueue_dt(ctx, P, L, 1.0, dt, 0, nullptr))) return st;
  if (axis == RIPPLE_FV_AXIS_XY) {
    // a linked grid would need the corner padding that run_batch fills
    const bool linked = g->nbr[0] >= 0 || g->nbr[1] >= 0 || g->nbr[2] >= 0 || g->nbr[3] >= 0;
    if (!P->fused || linked)
      return fail(ctx, RIPPLE_FV_E_UNSUPPORTED,
                  "fused x-y sweep needs n[0] >= 16, n[2] >= 2, unlinked x and y faces and "
                  "split_xy != 1");
    return enqueue_sweep_xy(ctx, P, L, 0, 1, 0, false);
  }
  return enqueue_sweep(ctx, P, L, axis, 0, 1, 0, false);
}

ripple_fv_status ripple_fv_step(ripple_fv_ctx* ctx, const ripple_fv_grid* g, void* u,
                                void* work, double cfl, double dt, double* dt_dev,
                                void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  for (int f = 0; f < 6; ++f)
    if (g->nbr[f] >= 0)
      return fail(ctx, RIPPLE_FV_E_INVALID, "ripple_fv_step takes a whole grid; use run_batch for sub-blocks");
  if (dt_dev && (st = ptr_ok(ctx, dt_dev, 8, 8, "dt_dev"))) return st;
  ripple_fv_grid one = *g;
  one.group = -1;
  void* a[1] = {u};
  void* b[1] = {work};
  return run(ctx, 1, &one, a, b, 1, cfl, dt, dt_dev, 0, (hipStream_t)stream);
}

ripple_fv_status ripple_fv_run_batch(ripple_fv_ctx* ctx, int32_t n, const ripple_fv_grid* grids,
                                     void* const* u, void* const* work, int32_t nsteps,
                                     double cfl, int32_t flags, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  return run(ctx, n, grids, u, work, nsteps, cfl, 0.0, nullptr, flags, (hipStream_t)stream);
}

ripple_fv_status ripple_fv_run_batch_noalloc(ripple_fv_ctx* ctx, int32_t n,
                                             const ripple_fv_grid* grids, void* const* u,
                                             void* const* work, int32_t nsteps, double cfl,
                                             void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if (n > NOALLOC_MAX_GRIDS)
    return fail(ctx, RIPPLE_FV_E_INVALID,
                "ripple_fv_run_batch_noalloc: more than RIPPLE_FV_NOALLOC_MAX_GRIDS (64) grids");
  if (nsteps < 0) return fail(ctx, RIPPLE_FV_E_INVALID, "nsteps < 0");
  if (!(cfl > 0.0 && cfl <= 1.0)) return fail(ctx, RIPPLE_FV_E_INVALID, "cfl must be in (0, 1]");
  if ((st = validate_batch(ctx, n, grids))) return st;
  if (!u || !work) return fail(ctx, RIPPLE_FV_E_INVALID, "NULL buffer list");
  for (int g = 0; g < n; ++g) {
    if ((st = ptr_ok(ctx, u[g], grids[g].bytes, 256, "u"))) return st;
    if ((st = ptr_ok(ctx, work[g], grids[g].bytes, 256, "work"))) return st;
    if (u[g] == work[g]) return fail(ctx, RIPPLE_FV_E_INVALID, "u and work alias");
  }
  if (!ctx->scratch) return fail(ctx, RIPPLE_FV_E_DEVICE, "no scratch address for this device");
  // launch shape and workspace image on the host stack
  PlanCore P;
  int64_t tiles[5][NOALLOC_MAX_GRIDS + 1];
  HaloTask halo[3][2 * NOALLOC_MAX_GRIDS];
  DevGrid hg[NOALLOC_MAX_GRIDS];
  int64_t* tp[5] = {tiles[0], tiles[1], tiles[2], tiles[3], tiles[4]};
  HaloTask* hp[3] = {halo[0], halo[1], halo[2]};
  plan_shape(P, n, grids, tp, hp, hg, ctx->cu_count);
  for (int g = 0; g < n; ++g) {
    hg[g].buf[0] = u[g];
    hg[g].buf[1] = work[g];
  }
  const WsLayout L = ws_layout(n, P.nhalo, nullptr);
  if (L.total > SCRATCH_BYTES) return fail(ctx, RIPPLE_FV_E_INVALID, "workspace exceeds the scratch array");
  alignas(16) unsigned char img[SCRATCH_BYTES];
  std::memset(img, 0, L.total);  // dt, lambda, time and wave-speed slots start at zero
  std::memcpy(img + L.grids, hg, sizeof(DevGrid) * n);
  for (int k = 0; k < 5; ++k) std::memcpy(img + L.tiles[k], tiles[k], sizeof(int64_t) * (n + 1));
  for (int k = 0; k < 3; ++k) std::memcpy(img + L.halo[k], halo[k], sizeof(HaloTask) * P.nhalo[k]);
  ws_bind(P, reinterpret_cast<char*>(ctx->scratch), L);
  hipStream_t s = (hipStream_t)stream;
  HIP_OR_FAIL(ctx, launch_upload(ctx->scratch, img, L.total, s));
  if (nsteps == 0) return RIPPLE_FV_OK;
  Launcher Lc{ctx, s, false, {}, 0};
  if ((st = enqueue_wavespeed(ctx, &P, Lc, 0, nullptr, false))) return st;
  for (int k = 0; k < nsteps; ++k)
    if ((st = enqueue_step(ctx, &P, Lc, P.in_place() ? 0 : (k & 1), cfl, 0.0, nullptr, false)))
      return st;
  if (!P.in_place() && (nsteps & 1)) return enqueue_copy_back(ctx, &P, s);
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_batch_time(ripple_fv_ctx* ctx, int32_t n, const ripple_fv_grid* grids,
                                      double* t_host, double* dt_host) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if (n < 1 || !grids || !t_host) return fail(ctx, RIPPLE_FV_E_INVALID, "bad arguments");
  auto it = ctx->plans.find(plan_key(n, grids));
  if (it == ctx->plans.end()) return fail(ctx, RIPPLE_FV_E_INVALID, "no run for these grids");
  Plan* P = it->second.get();
  HIP_OR_FAIL(ctx, hipDeviceSynchronize());
  HIP_OR_FAIL(ctx, hipMemcpy(t_host, P->d_t, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (dt_host) HIP_OR_FAIL(ctx, hipMemcpy(dt_host, P->d_dt, sizeof(double) * n, hipMemcpyDeviceToHost));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_partition(const ripple_fv_grid* whole, const int32_t parts[3],
                                     int32_t first_index, ripple_fv_grid* sub) {
  if (!whole || !parts || !sub || first_index < 0) return RIPPLE_FV_E_INVALID;
  int64_t pitch[3], bytes;
  int32_t ox;
  std::string why;
  if (grid_check(whole, pitch, &bytes, &ox, &why)) return RIPPLE_FV_E_INVALID;
  for (int d = 0; d < 3; ++d)
    if (parts[d] < 1 || (parts[d] > 1 && whole->n[d] / parts[d] < 2)) return RIPPLE_FV_E_INVALID;
  for (int d = 0; d < 3; ++d)
    if (whole->nbr[d * 2] >= 0 || whole->nbr[d * 2 + 1] >= 0) return RIPPLE_FV_E_INVALID;
  const int px = parts[0], py = parts[1], pz = parts[2];
  auto idx = [&](int a, int b, int c) { return first_index + a + px * (b + py * c); };
  int p3[3] = {px, py, pz};
  for (int c = 0; c < pz; ++c)
    for (int b = 0; b < py; ++b)
      for (int a = 0; a < px; ++a) {
        ripple_fv_grid& S = sub[a + px * (b + py * c)];
        S = *whole;
        const int coord[3] = {a, b, c};
        for (int d = 0; d < 3; ++d) {
          const int nn = whole->n[d], k = coord[d], np = p3[d];
          S.n[d] = nn / np + (k < nn % np ? 1 : 0);
          for (int side = 0; side < 2; ++side) {
            int nb[3] = {a, b, c};
            nb[d] += side == 0 ? -1 : 1;
            const bool inside = nb[d] >= 0 && nb[d] < np;
            if (!inside && whole->bc[d] == RIPPLE_FV_PERIODIC) nb[d] = (nb[d] + np) % np;
            // (a one-cell axis is not linked to itself: its faces read the cell)
            S.nbr[2 * d + side] =
                (inside || (whole->bc[d] == RIPPLE_FV_PERIODIC && nn >= 2)) ? idx(nb[0], nb[1], nb[2])
                                                                           : -1;
          }
        }
        S.group = first_index;
        if (ripple_fv_grid_init(&S)) return RIPPLE_FV_E_INVALID;
      }
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_halo_exchange(ripple_fv_ctx* ctx, int32_t n,
                                         const ripple_fv_grid* grids, void* const* u,
                                         int32_t axis, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if (axis < 0 || axis > 2) return fail(ctx, RIPPLE_FV_E_INVALID, "axis must be 0, 1 or 2");
  if ((st = validate_batch(ctx, n, grids))) return st;
  if (!u) return fail(ctx, RIPPLE_FV_E_INVALID, "NULL buffer list");
  for (int g = 0; g < n; ++g)
    if ((st = ptr_ok(ctx, u[g], grids[g].bytes, 256, "u"))) return st;
  Plan* P = nullptr;
  if ((st = build_plan(ctx, n, grids, &P))) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = upload_buffers(ctx, P, u, u, s))) return st;
  Launcher L{ctx, s, false, {}, 0};
  return enqueue_halo(ctx, P, L, axis, 0);
}

ripple_fv_status ripple_fv_conserved_sums(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                          const void* u, double* sums_dev, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  if ((st = ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  if ((st = ptr_ok(ctx, sums_dev, 40, 8, "sums_dev"))) return st;
  const int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
  const int nb = (int)std::min<int64_t>(DIAG_MAX_BLOCKS, (ncell + DIAG_BLOCK - 1) / DIAG_BLOCK);
  HIP_OR_FAIL(ctx, launch_sums(desc_of(*g, u), ctx->partials, nb, sums_dev, (hipStream_t)stream));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_error_norms(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                       const void* u, const double* ref_dev, double* l1_dev,
                                       double* linf_dev, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if ((st = grid_ok(ctx, g))) return st;
  const int64_t ncell = (int64_t)g->n[0] * g->n[1] * g->n[2];
  if ((st = ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  if ((st = ptr_ok(ctx, ref_dev, ncell * 40, 8, "ref_dev"))) return st;
  if ((st = ptr_ok(ctx, l1_dev, 40, 8, "l1_dev"))) return st;
  if ((st = ptr_ok(ctx, linf_dev, 40, 8, "linf_dev"))) return st;
  const int nb = (int)std::min<int64_t>(DIAG_MAX_BLOCKS, (ncell + DIAG_BLOCK - 1) / DIAG_BLOCK);
  HIP_OR_FAIL(ctx, launch_norms(desc_of(*g, u), ref_dev, ctx->partials, nb, l1_dev, linf_dev,
                                (hipStream_t)stream));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_stream_copy(ripple_fv_ctx* ctx, void* dst, const void* src,
                                       int64_t bytes, int32_t flags, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if (bytes < 0 || bytes % 16 != 0) return fail(ctx, RIPPLE_FV_E_INVALID, "bytes must be a multiple of 16");
  if (flags & ~1) return fail(ctx, RIPPLE_FV_E_INVALID, "unknown flags");
  if (bytes == 0) return RIPPLE_FV_OK;
  if ((st = ptr_ok(ctx, src, bytes, 16, "src"))) return st;
  if ((st = ptr_ok(ctx, dst, bytes, 16, "dst"))) return st;
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + bytes && b < a + bytes) return fail(ctx, RIPPLE_FV_E_INVALID, "src and dst overlap");
  HIP_OR_FAIL(ctx, launch_stream_copy(dst, src, bytes, flags & 1, (hipStream_t)stream));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_check(ripple_fv_ctx* ctx) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  HIP_OR_FAIL(ctx, hipDeviceSynchronize());
  unsigned int flag = 0;
  HIP_OR_FAIL(ctx, hipMemcpy(&flag, ctx->flag, sizeof(flag), hipMemcpyDeviceToHost));
  if (flag) {
    const unsigned int zero = 0;
    HIP_OR_FAIL(ctx, hipMemcpy(ctx->flag, &zero, sizeof(zero), hipMemcpyHostToDevice));
    return fail(ctx, RIPPLE_FV_E_NONPHYSICAL, "non-physical state (rho <= 0, p <= 0 or non-finite)");
  }
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_fv_profile(ripple_fv_ctx* ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return RIPPLE_FV_E_INVALID;
  for (int k = 0; k < RIPPLE_FV_NKERNELS; ++k) {
    ms[k] = ctx->prof_ms[k];
    launches[k] = ctx->prof_n[k];
    ctx->prof_ms[k] = 0.0;
    ctx->prof_n[k] = 0;
  }
  return RIPPLE_FV_OK;
}

const char* ripple_fv_status_string(ripple_fv_status s) {
  switch (s) {
    case RIPPLE_FV_OK: return "ok";
    case RIPPLE_FV_E_INVALID: return "invalid argument";
    case RIPPLE_FV_E_UNSUPPORTED: return "unsupported";
    case RIPPLE_FV_E_DEVICE: return "HIP error";
    case RIPPLE_FV_E_NONPHYSICAL: return "non-physical state";
    case RIPPLE_FV_E_NOMEM: return "out of memory";
    default: return "unknown status";
  }
}

const char* ripple_fv_last_error(ripple_fv_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"

// ---------------------------------------------------------------------------
// Autotuner
// ---------------------------------------------------------------------------

namespace {

struct TuneBufs {
  std::vector<void*> a, b;
  std::vector<int64_t> bytes;
  ~TuneBufs() {
    for (void* p : a) if (p) hipFree(p);
    for (void* p : b) if (p) hipFree(p);
  }
};

// Timing of one candidate: median and spread (largest minus smallest) of
// TUNE_REPEATS replays of a captured graph of TUNE_STEPS steps, in ms per
// replay.  Graph replay is the launch mode of a batch's long runs, and the
// median of several replays keeps one noisy timing from deciding the pick.
constexpr int TUNE_STEPS = 4;
constexpr int TUNE_REPEATS = 5;
// Timings within this fraction of the fastest count as equal (run-to-run
// differences of the same configuration on one device reach about 1 %).
constexpr double TUNE_TIE = 0.02;

struct TuneTime {
  double median = 0.0;
  double spread = 0.0;
};

// Time the batch described by `cand` on a synthetic smooth state (one eager
// warm-up step, one untimed graph run that captures the graph, then the
// timed replays).  Every candidate runs in the same buffers (B, sized for
// the largest layout of each grid), so no candidate gains or loses from
// where its memory happens to lie.
TuneTime time_candidate(ripple_fv_ctx* ctx, std::vector<ripple_fv_grid>& cand, double* W,
                        TuneBufs& B, hipStream_t s, ripple_fv_status* st) {
  *st = RIPPLE_FV_OK;
  TuneTime out;
  const int n = (int)cand.size();
  for (auto& g : cand) {
    if (ripple_fv_grid_init(&g)) { *st = fail(ctx, RIPPLE_FV_E_INVALID, "tuner candidate"); return out; }
  }
  for (int g = 0; g < n; ++g) {
    if (cand[g].bytes > B.bytes[g]) { *st = fail(ctx, RIPPLE_FV_E_INVALID, "tuner buffer too small"); return out; }
    hipError_t e = launch_tune_state(W, cand[g].n, s);
    if (e == hipSuccess) e = launch_import(desc_of(cand[g], B.a[g]), W, 1, s);
    if (e != hipSuccess) { *st = fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e)); return out; }
  }
  auto drop_plan = [&]() {
    // the candidate's plan refers to the tuner's buffers, freed when it returns
    const std::string key = plan_key(n, cand.data());
    ctx->plans.erase(key);
    for (auto it = ctx->plan_order.begin(); it != ctx->plan_order.end(); ++it)
      if (*it == key) { ctx->plan_order.erase(it); break; }
  };
  *st = run(ctx, n, cand.data(), B.a.data(), B.b.data(), 1, 0.9, 0.0, nullptr, 0, s);
  if (!*st)
    *st = run(ctx, n, cand.data(), B.a.data(), B.b.data(), TUNE_STEPS, 0.9, 0.0, nullptr,
              RIPPLE_FV_RUN_GRAPH, s);
  std::vector<double> ms;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!*st && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    *st = fail(ctx, RIPPLE_FV_E_DEVICE, "tuner events");
  for (int r = 0; r < TUNE_REPEATS && !*st; ++r) {
    hipEventRecord(e0, s);
    *st = run(ctx, n, cand.data(), B.a.data(), B.b.data(), TUNE_STEPS, 0.9, 0.0, nullptr,
              RIPPLE_FV_RUN_GRAPH, s);
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float t = 0.f;
    hipEventElapsedTime(&t, e0, e1);
    ms.push_back(t);
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipDeviceSynchronize();
  drop_plan();
  if (*st) return out;
  std::sort(ms.begin(), ms.end());
  out.median = ms[ms.size() / 2];
  out.spread = ms.back() - ms.front();
  return out;
}

}  // namespace

extern "C" ripple_fv_status ripple_fv_batch_tune(ripple_fv_ctx* ctx, int32_t n,
                                                 const ripple_fv_grid* in,
                                                 ripple_fv_grid* chosen, void* stream) {
  ripple_fv_status st = set_device(ctx);
  if (st) return st;
  if (n < 1 || !in || !chosen) return fail(ctx, RIPPLE_FV_E_INVALID, "bad arguments");
  std::vector<ripple_fv_grid> base(in, in + n);
  for (auto& g : base) {
    g.layout = RIPPLE_FV_SOA;
    g.aosoa_w = 0;
    g.x_block = g.yz_block = g.yz_segment = g.persist = g.yz_cols = g.split_xy = 0;
    if (ripple_fv_grid_init(&g)) return fail(ctx, RIPPLE_FV_E_INVALID, "bad grid descriptor");
  }
  if ((st = validate_batch(ctx, n, base.data()))) return st;
  const std::string key = plan_key(n, base.data());
  auto hit = ctx->tune_cache.find(key);
  if (hit != ctx->tune_cache.end()) {
    std::copy(hit->second.begin(), hit->second.end(), chosen);
    return RIPPLE_FV_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  int64_t max_cell = 0;
  for (auto& g : base) max_cell = std::max<int64_t>(max_cell, (int64_t)g.n[0] * g.n[1] * g.n[2]);
  double* W = nullptr;
  if (hipMalloc(&W, sizeof(double) * 5 * max_cell) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RIPPLE_FV_E_NOMEM, "tuner state allocation failed");
  }
  // one pair of buffers per grid, large enough for every layout tried
  TuneBufs B;
  B.a.assign(n, nullptr);
  B.b.assign(n, nullptr);
  B.bytes.assign(n, 0);
  for (int g = 0; g < n && !st; ++g) {
    for (int L : {RIPPLE_FV_SOA, RIPPLE_FV_AOS, RIPPLE_FV_AOSOA})
      for (int w : {16, 32, 64}) {
        ripple_fv_grid v = base[g];
        v.layout = L;
        v.aosoa_w = L == RIPPLE_FV_AOSOA ? w : 0;
        if (ripple_fv_grid_init(&v) == RIPPLE_FV_OK) B.bytes[g] = std::max(B.bytes[g], v.bytes);
      }
    if (hipMalloc(&B.a[g], B.bytes[g]) != hipSuccess || hipMalloc(&B.b[g], B.bytes[g]) != hipSuccess) {
      (void)hipGetLastError();
      st = fail(ctx, RIPPLE_FV_E_NOMEM, "tuner buffer allocation failed");
    }
  }
  if (st) {
    hipFree(W);
    return st;
  }
  // Coordinate search in stages (layout; x-sweep workgroup; y/z chunk width
  // and segment; x cells per y/z thread; fused or separate x-y; persistent
  // launches), starting from the default (SoA, library defaults).  Each stage
  // times the incumbent again beside its candidates, all built from the
  // incumbent, and takes the first configuration in the order [incumbent,
  // candidates in the listed order] whose median is within a tolerance of
  // the stage's fastest median: the larger of the timings' largest spread
  // and TUNE_TIE of the fastest median.  So the incumbent stays unless a
  // candidate beats it by more than the tolerance, and configurations whose
  // timings differ by less than the noise resolve the same way on every run.
  std::vector<ripple_fv_grid> best = base;
  auto stage = [&](const std::vector<std::vector<ripple_fv_grid>>& cands) -> ripple_fv_status {
    ripple_fv_status s2;
    std::vector<std::vector<ripple_fv_grid>> order;
    order.push_back(best);
    order.insert(order.end(), cands.begin(), cands.end());
    std::vector<TuneTime> t(order.size());
    double fastest = 1e300, spread = 0.0;
    for (size_t i = 0; i < order.size(); ++i) {
      t[i] = time_candidate(ctx, order[i], W, B, s, &s2);
      if (s2) return s2;
      fastest = std::min(fastest, t[i].median);
      spread = std::max(spread, t[i].spread);
    }
    const double tol = std::max(spread, TUNE_TIE * fastest);
    for (size_t i = 0; i < order.size(); ++i)
      if (t[i].median <= fastest + tol) {
        best = order[i];
        break;
      }
    return RIPPLE_FV_OK;
  };
  auto with = [&](auto edit) {
    std::vector<ripple_fv_grid> c = best;
    for (auto& g : c) edit(g);
    return c;
  };
  std::vector<std::vector<ripple_fv_grid>> cands;
  // 1. layout
  const int layouts[4][2] = {{RIPPLE_FV_AOS, 0}, {RIPPLE_FV_AOSOA, 16}, {RIPPLE_FV_AOSOA, 32},
                             {RIPPLE_FV_AOSOA, 64}};
  for (auto& L : layouts)
    cands.push_back(with([&](ripple_fv_grid& g) { g.layout = L[0]; g.aosoa_w = L[1]; }));
  st = stage(cands);
  // 2. x sweep workgroup
  if (!st) {
    cands.clear();
    cands.push_back(with([&](ripple_fv_grid& g) { g.x_block = 128; }));
    st = stage(cands);
  }
  // 3. y/z sweep chunk width and segment length (longer segments and wider
  // chunks first: fewer tiles and fewer re-read halo cells)
  if (!st) {
    cands.clear();
    for (int sg : {128, 64, 32, 16})
      for (int yb : {256, 128, 64})
        if (!(yb == 256 && sg == 128))
          cands.push_back(with([&](ripple_fv_grid& g) { g.yz_block = yb; g.yz_segment = sg; }));
    st = stage(cands);
  }
  // 4. x cells per y/z thread (FP32; FP64 runs one cell per thread), fused or
  // separate x and y sweeps
  if (!st && base[0].dtype != RIPPLE_FV_F64) {
    cands.clear();
    for (int cols : {1, 4}) cands.push_back(with([&](ripple_fv_grid& g) { g.yz_cols = cols; }));
    st = stage(cands);
  }
  if (!st) {
    cands.clear();
    for (int split : {1, 2, 3}) cands.push_back(with([&](ripple_fv_grid& g) { g.split_xy = split; }));
    st = stage(cands);
  }
  // 5. persistent launches
  if (!st) {
    cands.clear();
    for (int pc : {2, 4, 8}) cands.push_back(with([&](ripple_fv_grid& g) { g.persist = pc; }));
    st = stage(cands);
  }
  hipFree(W);
  if (st) return st;
  for (auto& g : best) ripple_fv_grid_init(&g);
  ctx->tune_cache[key] = best;
  std::copy(best.begin(), best.end(), chosen);
  return RIPPLE_FV_OK;
}
