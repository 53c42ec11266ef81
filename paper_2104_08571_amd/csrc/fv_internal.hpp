// Internal declarations shared by the kernel and C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_index.hpp"
#include "ripple_fv.h"

namespace rfv {

constexpr int NV = RIPPLE_FV_NVAR;
constexpr int HALO = RIPPLE_FV_HALO;

// Storage layouts as compiled kernel variants.
enum Lay : int { LAY_AOS = 0, LAY_SOA = 1, LAY_AOSOA16 = 2, LAY_AOSOA32 = 3, LAY_AOSOA64 = 4,
                 LAY_COUNT = 5 };

// Device copy of one grid of a batch.  Read by every kernel through a
// wave-uniform index, so the compiler keeps it in scalar registers.
struct DevGrid {
  void* buf[2];        // state buffers A (initial) and B
  int32_t n[3];        // interior extents
  int32_t mode[6];     // FaceMode per face (-x, +x, -y, +y, -z, +z)
  int64_t px, pxy;     // padded pitch of a row and of a plane, in cells
  int64_t ptot;        // cell slots per buffer (SoA component stride)
  double dx[3];
  int32_t group;       // index of the grid whose wave-speed slot and dt this grid uses
  int32_t ox;          // padded x index of interior x = 0
  int32_t nbr_x[2];    // batch index of the sub-block linked at -x / +x (-1: none)
};

// Per-batch device workspace handed to the kernels.
struct Work {
  const DevGrid* grids;
  int32_t ngrids;
  int32_t pad_;
  double* lam;                     // [ngrids * 3] dt / dx_d
  double* t;                       // [ngrids] time reached
  double* dt;                      // [ngrids] last dt
  unsigned long long* s_acc;       // [ngrids * 3] wave-speed maxima (double bits), by group
  unsigned int* flag;              // sticky non-physical flag
};

// Tiles of one sweep: tile_start[g] is the first tile of grid g, tile_start[ngrids]
// the total.  A launch processes tiles [first, first + count).  With an order
// table the launch has `slots` dispatch slots (a multiple of NXCD, as is its
// workgroup count) and slot s takes tile first + order[s] (none where
// order[s] < 0); without one, each XCD takes one contiguous run of the list.
struct TileRange {
  const int64_t* tile_start;
  int64_t first;
  int64_t count;
  const int32_t* order;
  int64_t slots;
};

// XCDs of the part.  Workgroups are dispatched round-robin over them, in
// workgroup-index order.
constexpr int NXCD = 8;

struct SweepParams {
  Work w;
  TileRange tiles;
  int32_t in, out;     // buffer index read / written
  int32_t seg;         // cells per thread along the sweep axis (y, z sweeps)
  int32_t fuse_s;      // accumulate wave speeds of the output (z sweep)
  int32_t xmode;       // fused pass: XM_ROWS or XM_WAVES
  int32_t link_x;      // fused pass: some grid has an x face linked to a sub-block
};

struct HaloTask {
  int32_t dst, src;    // grid indices
  int32_t side;        // 0: dst face -axis <- src high interior; 1: dst face +axis <- src low interior
  int32_t pad_;
};

// Tiling knobs resolved from a descriptor (defaults applied).
struct Tiling {
  int x_block;     // threads per workgroup of the x sweep (128 or 256)
  int yz_block;    // lanes per workgroup of the y/z sweeps (64, 128, 256)
  int yz_segment;  // cells per thread along y/z
  int persist;     // workgroups per CU for persistent launches, 0 = one per tile
  int yz_cols;     // adjacent x cells per thread in the y/z sweeps (1 or 2)
  int split_xy;    // 1: separate x and y sweeps; 2, 3: fused, rows / wave-strip form
};

int lay_of(const ripple_fv_grid& g);

// Tile counts of one grid (must match the kernels' decoding).
int64_t tiles_x(const ripple_fv_grid& g, int x_block);
int64_t tiles_yz(const ripple_fv_grid& g, int axis, int yz_block, int yz_segment, int yz_cols);
int64_t tiles_ws(const ripple_fv_grid& g);
// Fused x-then-y sweep, in one of two forms of the x exchange:
//  XM_ROWS   workgroups of XY_THREADS lanes owning whole x rows (one lane per
//            cell, plus four ghost lanes per row when an x face is linked),
//            neighbours exchanged through LDS (three barriers per row);
//  XM_WAVES  every wave owns a strip of XY_WAVE_CELLS cells of one row plus
//            two ghost lanes on each side and exchanges neighbours by lane
//            shifts: no LDS and no barriers, any row length.
constexpr int XM_ROWS = 0, XM_WAVES = 1;
constexpr int XY_MIN_NX = 16;
constexpr int XY_THREADS = 512;
constexpr int XY_WAVE_CELLS = 60;
constexpr int XY_WAVE_THREADS = 256;   // workgroup of the wave-strip form
constexpr int64_t XY_MIN_TILES = 2048;
constexpr int Z_MIN_TILES_PER_CU = 2;   // z sweep: segments as long as this allows
constexpr int Z_ROUND_TILES_PER_CU = 4; // ... while the tiles take about one round
constexpr int Z_MIN_SEGMENT = 16;
bool xy_eligible(const ripple_fv_grid& g);
// Form of the fused pass for a batch of grids of precision dtype and the
// split_xy knob (0: cheaper form by the cost model, 2: rows where every row
// fits a workgroup, 3: wave strips).
int xy_mode(int dtype, const ripple_fv_grid* grids, int n, int split_xy);
int64_t tiles_xy(const ripple_fv_grid& g, int yz_segment, int xmode);
int tile_len_yz(const ripple_fv_grid& g, int axis, int yz_block, int yz_segment, int yz_cols,
                int64_t lt);
int tile_len_xy(const ripple_fv_grid& g, int seg, int64_t lt);
constexpr int WS_BLOCK = 256;
constexpr int WS_CELLS_PER_THREAD = 4;

// Kernel launchers (return hipError_t of the launch).
hipError_t launch_sweep(int dtype, int lay, int axis, const Tiling& tl, const SweepParams& p,
                        int grid_blocks, hipStream_t s);
hipError_t launch_sweep_xy(int dtype, int lay, const Tiling& tl, const SweepParams& p,
                           int grid_blocks, hipStream_t s);
hipError_t launch_wavespeed(int dtype, int lay, const Work& w, int in, TileRange tr,
                            unsigned long long* s_out, int grid_blocks, hipStream_t s);
hipError_t launch_dt(const Work& w, double cfl, double fixed_dt, int reset_s, double* dt_out,
                     hipStream_t s);
// ext: padding layers to cover on each side of the first axis across the face
hipError_t launch_halo(int dtype, int lay, const Work& w, int buf, int axis, int ext,
                       const HaloTask* tasks, int ntasks, int64_t max_area, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
// Copy `bytes` (a multiple of 8, dst 8-byte aligned) from host memory to
// device memory through kernel arguments, in chunks of UploadChunk::w.
struct UploadChunk {
  uint32_t off;        // byte offset of the chunk in the destination
  uint32_t nwords;     // 8-byte words that follow
  uint64_t w[240];
};
hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s);
// Plain 16-byte-access device copy of `bytes` (a multiple of 16); nt: the
// stores carry the non-temporal hint.
hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, int nt, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);

// Generic (runtime layout) transfer and diagnostics kernels.
struct Desc {
  void* buf;
  int32_t n[3];
  int32_t lay;
  int32_t dtype;
  int32_t ox;          // padded x index of interior x = 0
  int64_t px, pxy, ptot;
};
hipError_t launch_import(const Desc& d, const double* src, int primitive, hipStream_t s);
hipError_t launch_export(const Desc& d, double* dst, hipStream_t s);
hipError_t launch_convert(const Desc& src, const Desc& dst, hipStream_t s);
hipError_t launch_tune_state(double* W, const int n[3], hipStream_t s);
hipError_t launch_sums(const Desc& d, double* partials, int nblocks, double* out, hipStream_t s);
hipError_t launch_norms(const Desc& d, const double* ref, double* partials, int nblocks,
                        double* l1, double* linf, hipStream_t s);
// Context services for entry points outside the step's translation unit:
// select the context's device and clear its error text; record an error;
// check that a device pointer is aligned and covers `bytes`.
ripple_fv_status ctx_begin(ripple_fv_ctx* ctx);
ripple_fv_status ctx_fail(ripple_fv_ctx* ctx, ripple_fv_status st, const char* msg);
ripple_fv_status ctx_ptr_ok(ripple_fv_ctx* ctx, const void* p, int64_t bytes, int64_t align,
                            const char* what);

constexpr int DIAG_BLOCK = 256;
constexpr int DIAG_MAX_BLOCKS = 1024;

}  // namespace rfv
