// HIP kernels for gfx950: the split finite-volume Euler step and its helpers.
//
// Hot kernels (templated on precision and layout):
//  - k_sweep_x   : update along x.  A workgroup stages a chunk of consecutive
//                  cells of the flattened (row, x) index space -- every
//                  interior row followed by its padding columns -- in LDS, so
//                  global loads and stores are contiguous runs of memory and
//                  the x stencil is read from LDS.
//  - k_sweep_yz  : update along y or z.  Lanes cover consecutive cells of the
//                  plane across the sweep (coalesced), and each thread marches
//                  along the sweep axis with a five-cell register window, so
//                  every cell is read once per sweep (plus 4 cells per segment).
//                  The z sweep can also reduce the new state's wave speeds
//                  for the next step's time step.
//  - k_wavespeed : per-cell |u_d| + c and the max over each grid.
//  - k_dt        : time step per grid from the maxima (kept on the device so a
//                  captured step loop needs no host round trip).
//  - k_halo      : copies two interior layers of a sub-block into its
//                  neighbour's padding.
// Physical boundaries are applied while loading (transmissive = clamp to the
// edge cell, periodic = wrap), so no pass over the padding is needed; faces
// linked to a neighbouring sub-block read the padding that k_halo filled.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fv_internal.hpp"
#include "fv_index.hpp"
#include "fv_layout.hpp"
#include "fv_math.hpp"

namespace rfv {

// ---------------------------------------------------------------------------
// Tile bookkeeping
// ---------------------------------------------------------------------------

// Grid owning global tile t: the last g with tile_start[g] <= t.
__device__ __forceinline__ int find_grid(const int64_t* start, int n, int64_t t) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return uniform(lo);
}

// Dispatch slots of a launch over a tile range, the first slot of this
// workgroup, and the tile (relative to r.first) that slot b takes, -1 for
// none.  With an order table workgroup w takes slots w, w + gridDim.x, ...,
// all on the XCD that w is dispatched to (gridDim.x is a multiple of NXCD);
// without one each XCD takes one contiguous run of the tile list, since
// neighbouring tiles share halo cells and then share that XCD's L2.
__device__ __forceinline__ int64_t slot_count(const TileRange& r) {
  return r.order ? r.slots : r.count;
}
__device__ __forceinline__ int64_t first_slot(const TileRange& r) {
  return r.order ? (int64_t)blockIdx.x : xcd_order(blockIdx.x, gridDim.x);
}
__device__ __forceinline__ int64_t slot_tile(const TileRange& r, int64_t b) {
  return r.order ? (int64_t)r.order[b] : b;
}


// Maximum of two non-negative values by their bit patterns (they order like
// unsigned integers); a NaN pattern exceeds every finite one, so it wins.
__device__ __forceinline__ float bits_max(float a, float b) {
  return __builtin_bit_cast(float, max(__builtin_bit_cast(uint32_t, a), __builtin_bit_cast(uint32_t, b)));
}
__device__ __forceinline__ double bits_max(double a, double b) {
  const uint64_t x = __builtin_bit_cast(uint64_t, a), y = __builtin_bit_cast(uint64_t, b);
  return __builtin_bit_cast(double, x > y ? x : y);
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = bits_max(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce per-thread wave-speed maxima over the workgroup and fold them into
// the group's slot.  The global maximum only grows, so a tile whose maximum
// does not exceed the value already seen skips the atomic.
template <typename T>
__device__ __forceinline__ void fold_wavespeeds(T s[3], bool bad, unsigned long long* slot,
                                                unsigned int* flag, T* lds /* 3 * 16 */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwave = blockDim.x >> 6;
  if (bad) *flag = 1u;
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = wave_max(s[d]);
  if (lane == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) lds[wave * 3 + d] = s[d];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    T m = lds[threadIdx.x];
    for (int wv = 1; wv < nwave; ++wv) m = bits_max(m, lds[wv * 3 + threadIdx.x]);
    const unsigned long long bits = __double_as_longlong((double)m);
    if (bits > __atomic_load_n(&slot[threadIdx.x], __ATOMIC_RELAXED))
      atomicMax(&slot[threadIdx.x], bits);
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// x sweep
// ---------------------------------------------------------------------------


// Chunk of NT consecutive positions of the flattened (row, x) space, rows
// being the interior (j, k) pairs and positions within a row running over
// x = -2 .. n0+1 (the padded columns).  Thread t holds position
// P0 - 2 + t; threads 2 .. NT-3 write the interior cells among them, so each
// chunk produces up to NT - 4 cells and overlaps its neighbours by 4.
template <typename T, int LAY, int NT>
__global__ void __launch_bounds__(NT) k_sweep_x(SweepParams p, const DevGrid* __restrict__ grids,
                                                const int64_t* __restrict__ tile_start,
                                                const double* __restrict__ lamv) {
  constexpr int C = NT - 4;
  __shared__ T sA[5][NT];
  __shared__ T sB[5][NT];
  const int tid = threadIdx.x;
  for (int64_t b = first_slot(p.tiles); b < slot_count(p.tiles); b += gridDim.x) {
    const int64_t tb = slot_tile(p.tiles, b);
    if (tb < 0) continue;
    const int64_t gt = uniform(p.tiles.first + tb);
    const int g = find_grid(tile_start, p.w.ngrids, gt);
    const DevGrid& G = grids[g];
    const int lt = (int)(gt - tile_start[g]);
    const int nx = G.n[0], ny = G.n[1];
    const XPos xp = x_position(tid, lt * C - 2, nx + 4, ny, G.n[2]);
    const int i = face_index(xp.il - 2, nx, G.mode[0], G.mode[1]);
    // uniform base: the chunk's first row, aligned down to 64 cells
    const int64_t qrow0 = (int64_t)(xp.k0 + 2) * G.pxy + (int64_t)(xp.j0 + 2) * G.px;
    const int64_t q0 = uniform(qrow0 & ~int64_t(63));
    const uint32_t rowoff = (uint32_t)(qrow0 - q0) + (uint32_t)xp.dk * (uint32_t)G.pxy +
                            (uint32_t)xp.dj * (uint32_t)G.px;
    const bool valid = xp.valid;
    const int il = xp.il;
    const uint32_t lane_ld = Layout<LAY>::rel(rowoff + (uint32_t)(i + G.ox)) * (uint32_t)sizeof(T);
    const uint32_t lane_st = Layout<LAY>::rel(rowoff + (uint32_t)(il - 2 + G.ox)) * (uint32_t)sizeof(T);
    const T lam = (T)lamv[g * 3 + 0];
    const T hl = T(0.5) * lam;

    T u[5];
    load_cell_rel<T, LAY>(G.buf[p.in], q0, G.ptot, lane_ld, u);
#pragma unroll
    for (int c = 0; c < 5; ++c) sA[c][tid] = u[c];
    __syncthreads();

    T bl[5], br[5];
    if (tid >= 1 && tid <= NT - 2) {
      T dm[5], dp[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        dm[c] = u[c] - sA[c][tid - 1];
        dp[c] = sA[c][tid + 1] - u[c];
      }
      hancock<T, 0>(u, dm, dp, hl, bl, br);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 5; ++c) sA[c][tid] = br[c];
    __syncthreads();

    T fx[5];
    if (tid >= 2 && tid <= NT - 2) {
      T left[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) left[c] = sA[c][tid - 1];
      hllc<T, 0>(left, bl, fx);   // face between positions tid-1 and tid
#pragma unroll
      for (int c = 0; c < 5; ++c) sB[c][tid] = fx[c];
    }
    __syncthreads();
    if (tid >= 2 && tid <= NT - 3 && valid && il >= 2 && il < nx + 2) {
      T o[5], fp[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) fp[c] = sB[c][tid + 1];
      update(u, lam, fp, fx, o);
      store_cell_rel<T, LAY>(G.buf[p.out], q0, G.ptot, lane_st, o);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// y / z sweeps
// ---------------------------------------------------------------------------

// Tile = (chunk of blockDim.x column groups of the plane across the sweep, x
// fastest) x (segment of p.seg cells along D).  A column group is COLS
// adjacent cells along x that one thread advances together: in SoA and AoSoA
// their values move as one 8- or 16-byte access per component, which the
// memory pipeline sustains far better than 4-byte accesses.  Segment index
// runs fastest so that the segments of one column, which overlap by four
// cells, are processed by neighbouring workgroups.
//
// Each thread marches along D.  The cells it holds live in a ring of
// YZ_RING register slots: U_j (the cell being written), U_{j+1}, U_{j+2} (the
// stencil of the reconstruction at j+1) and YZ_RING - 3 cells loaded ahead,
// so every load is issued YZ_RING - 3 iterations before its first use.  The
// loop is unrolled by the ring length, which makes every slot index a
// compile-time constant.
//
// Addressing: all lanes of a tile sit at the same index j along D, so the row
// address of component c at j is wave-uniform (scalar registers) and each
// lane adds a fixed 32-bit offset for the whole tile.
#ifndef RFV_YZ_RING
#define RFV_YZ_RING 5
#endif
// Tile order of the y/z sweeps: 0 = segments of one column chunk fastest;
// 1 = column chunks fastest (the tiles in flight cover a band of segments).
#ifndef RFV_YZ_ORDER
#define RFV_YZ_ORDER 0
#endif
// Cache policy of the z sweep's loads and stores in SoA and AoSoA:
// non-temporal (2, the buffer instructions' nt bit).  Each cell is read and
// written once and no other tile reads it in the same launch (but for the 4
// halo cells of a segment).  Measured against the default policy: 512^3
// FP32 z sweep 1.047 -> 1.014 ms, FP64 2.234 -> 2.216 ms; 256^3 FP64 0.275
// -> 0.265 ms; the 64-grid batch 0.941 -> 0.856 ms.  AoS (whose lanes' 40-
// or 20-byte cells share lines) and the y sweep keep the default: the 256^3
// FP64 AoS z sweep took 0.404 ms against 0.329.
#ifndef RFV_Z_LOAD_POLICY
#define RFV_Z_LOAD_POLICY 2
#endif
#ifndef RFV_Z_STORE_POLICY
#define RFV_Z_STORE_POLICY 2
#endif
template <typename T, int LAY, int D, bool FUSE, int COLS>
__global__ void __launch_bounds__(256) k_sweep_yz(SweepParams p, const DevGrid* __restrict__ grids,
                                                  const int64_t* __restrict__ tile_start,
                                                  const double* __restrict__ lamv) {
  constexpr int K = RFV_YZ_RING;  // ring slots
  static_assert(K >= 4, "ring must hold the stencil and one cell ahead");
  constexpr bool NTZ = D == 2 && LAY != LAY_AOS;
  constexpr int LDP = NTZ ? RFV_Z_LOAD_POLICY : LD_POL;
  constexpr int STP = NTZ ? RFV_Z_STORE_POLICY : ST_POL;
  __shared__ T red[3 * 16];
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  for (int64_t b = first_slot(p.tiles); b < slot_count(p.tiles); b += gridDim.x) {
    const int64_t tb = slot_tile(p.tiles, b);
    if (tb < 0) continue;
    const int64_t gt = uniform(p.tiles.first + tb);
    const int g = find_grid(tile_start, p.w.ngrids, gt);
    const DevGrid& G = grids[g];
    const int64_t lt = gt - tile_start[g];
    const uint32_t na = G.n[0];
    const uint32_t nb = G.n[D == 1 ? 2 : 1];
    const int nd = G.n[D];
    const int nseg = (nd + p.seg - 1) / p.seg;
    const uint32_t npr = (na + COLS - 1) / COLS;  // column groups per row
    const uint32_t ngroups = npr * nb;
#if RFV_YZ_ORDER
    const int64_t nchunk = (ngroups + nt - 1) / nt;
    const int s = (int)(lt / nchunk);
    const int64_t chunk = lt - (int64_t)s * nchunk;
#else
    const int64_t chunk = lt / nseg;
    const int s = (int)(lt - chunk * nseg);
#endif
    const uint32_t f0 = (uint32_t)(chunk * nt);
    const uint32_t fl = f0 + tid;
    const bool active = fl < ngroups;
    const uint32_t fc = active ? fl : ngroups - 1;
    const uint32_t ib = fc / npr, ia = (fc - ib * npr) * COLS;
    const uint32_t ib0 = f0 / npr, ia0 = (f0 - ib0 * npr) * COLS;
    bool act[COLS];
#pragma unroll
    for (int k = 0; k < COLS; ++k) act[k] = active && ia + k < na;
    const int64_t across = D == 1 ? G.pxy : G.px;
    const int64_t stride = D == 1 ? G.px : G.pxy;
    const int64_t qlane = (int64_t)(ia + G.ox) + (int64_t)(ib + 2) * across;
    const int64_t qfirst = (int64_t)(ia0 + G.ox) + (int64_t)(ib0 + 2) * across;
    const int64_t q0 = uniform(qfirst & ~int64_t(63));
    const uint32_t lane = Layout<LAY>::rel((uint32_t)(qlane - q0)) * (uint32_t)sizeof(T);
    const int mlo = G.mode[2 * D], mhi = G.mode[2 * D + 1];
    const void* src = G.buf[p.in];
    void* dst = G.buf[p.out];
    const T lam = (T)lamv[g * 3 + D];
    const T hl = T(0.5) * lam;
    const int j0 = s * p.seg;
    const int len = min(p.seg, nd - j0);
    const int jlast = j0 + len + 1;  // last cell the segment reads
    const int64_t ptot = G.ptot;

    auto row = [&](int j) -> int64_t {
      return q0 + (int64_t)(face_index(min(j, jlast), nd, mlo, mhi) + 2) * stride;
    };

    // slot of cell j' is (j' - j0 + 2) mod K
    T ring[K][COLS][5];
    T dprev[COLS][5], dnext[5], bl[5], br[COLS][5], brp[COLS][5], fprev[COLS][5];
#pragma unroll
    for (int k = 0; k < K; ++k) load_group<T, LAY, COLS, LDP>(src, row(j0 - 2 + k), ptot, lane, ring[k]);
#pragma unroll
    for (int m = 0; m < COLS; ++m) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        dprev[m][c] = ring[1][m][c] - ring[0][m][c];
        dnext[c] = ring[2][m][c] - ring[1][m][c];
      }
      hancock<T, D>(ring[1][m], dprev[m], dnext, hl, bl, brp[m]);   // cell j0 - 1
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        dprev[m][c] = dnext[c];
        dnext[c] = ring[3][m][c] - ring[2][m][c];
      }
      hancock<T, D>(ring[2][m], dprev[m], dnext, hl, bl, br[m]);    // cell j0
      hllc<T, D>(brp[m], bl, fprev[m]);                             // face j0 - 1/2
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        brp[m][c] = br[m][c];
        dprev[m][c] = dnext[c];
      }
    }
    load_group<T, LAY, COLS, LDP>(src, row(j0 + K - 2), ptot, lane, ring[0]);

    T smax[3] = {T(0), T(0), T(0)};
    bool bad = false;
    // At iteration o (cell j = j0 + o): ring[(o+2)%K] = U_j, ring[(o+3)%K] = U_{j+1},
    // ring[(o+4)%K] = U_{j+2}; dprev = U_{j+1} - U_j, brp = Ub^R_j, fprev = F_{j-1/2}.
    // The slot of U_{j-1}, dead now, receives U_{j+K-1}.
    for (int o0 = 0; o0 < len; o0 += K) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int o = o0 + k;
        if (o >= len) break;
        const int j = j0 + o;
        load_group<T, LAY, COLS, LDP>(src, row(j + K - 1), ptot, lane, ring[(k + 1) % K]);
        T out[COLS][5];
#pragma unroll
        for (int m = 0; m < COLS; ++m) {
          const T* uj = ring[(k + 2) % K][m];
          const T* uj1 = ring[(k + 3) % K][m];
          const T* uj2 = ring[(k + 4) % K][m];
#pragma unroll
          for (int c = 0; c < 5; ++c) dnext[c] = uj2[c] - uj1[c];
          hancock<T, D>(uj1, dprev[m], dnext, hl, bl, br[m]);       // cell j + 1
          T fcur[5];
          hllc<T, D>(brp[m], bl, fcur);                             // face j + 1/2
          update(uj, lam, fcur, fprev[m], out[m]);
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            fprev[m][c] = fcur[c];
            brp[m][c] = br[m][c];
            dprev[m][c] = dnext[c];
          }
        }
        if (act[0])
          store_group<T, LAY, COLS, STP>(dst, q0 + (int64_t)(j + 2) * stride, ptot, lane, out, act);
        if (FUSE) {
#pragma unroll
          for (int m = 0; m < COLS; ++m) {
            T sc[3];
            bool b_ = false;
            wavespeeds(out[m], sc, b_);
            if (act[m]) {
#pragma unroll
              for (int d = 0; d < 3; ++d) smax[d] = bits_max(smax[d], sc[d]);
              bad |= b_;
            }
          }
        }
      }
    }
    if (FUSE) fold_wavespeeds<T>(smax, bad, p.w.s_acc + 3 * G.group, p.w.flag, red);
  }
}

// ---------------------------------------------------------------------------
// Fused x-then-y sweep
// ---------------------------------------------------------------------------

// The y sweep of cell (i, j, k) reads the x-swept states of column (i, k) at
// rows j-2 .. j+2 only, and the x sweep of a row needs nothing but that row.
// So lanes that hold a stretch of an x row (with its neighbours) can march
// along y, x-sweep each row they load and feed the result straight into the
// y sweep's register window: the state is read and written once for both
// sweeps.  Each cell undergoes exactly the arithmetic
// of k_sweep_x followed by k_sweep_yz along y, so the result is bitwise that
// of the two separate kernels.
//
// Two forms of the x exchange (XM):
//
// XM_ROWS.  Tile = (R whole x rows at consecutive z) x (segment of p.seg
// rows along y).  A row takes P lanes: one per cell (P = n0), or, when an x
// face is linked to a sub-block, one per padded position x = -2 .. n0+1
// (P = n0 + 4) so that the four ghost lanes load the cells beyond the faces
// (a linked face's from the neighbouring sub-block).  Otherwise the lanes
// holding cells 0, 1, n0-2, n0-1 also write the
// ghost slots the boundary condition defines (wrap or clamp).  Per loaded
// row: publish the cells to LDS; reconstruct and publish each cell's right
// evolved state; compute each cell's left face flux and publish it; update.
// The ghost reconstruction and the right-most face come from the periodic
// partner cell, or are computed by the edge lane otherwise.
//
// XM_WAVES.  Every wave owns a strip of up to XY_WAVE_CELLS cells of one row
// and a y segment; its 64 lanes hold the positions x = x0-2 .. x0+61, and
// the four outside the strip (ghost lanes) load the cells their positions
// name: the neighbouring strips' cells inside the row, at its ends what the
// face names (clamped or wrapped, or the linked sub-block's cells).
// Neighbours are read by whole-wave
// lane shifts, so waves are independent (no LDS, no barriers) and a row may
// have any length; every lane runs the whole x sweep and the strip's cells
// take exactly the arithmetic of an unbroken row.  The workgroup's waves take
// consecutive (z, strip) pairs in row-major order.
//
// Rows outside the grid along y are the mapped interior rows (periodic,
// transmissive) or the padding rows of a linked face, which hold the
// neighbour's state before this pass (the y halo copy fills them); at their
// x ends a linked x face's lanes read the x neighbour's own y padding rows,
// which hold the diagonal neighbour's cells.  The pass x-sweeps them like
// any other row.
//
// Rings: raw rows are loaded PF iterations before they are x-swept (PF = 3
// in the rows form, 1 in the wave strips); x-swept rows j, j+1, j+2 are
// held while cell j is updated (period 3).
//
// Iterations per trip of the marching loop, a multiple of the ring period 3.
// Loads issued in an earlier trip are waited for at a trip's first use (the
// wait counter is merged conservatively at the loop head), so longer trips
// keep a little more in flight.  Measured at 512^3 in the rows form, FP32:
// 3 -> 1.444 ms, 6 -> 1.394, 9 -> 1.387, 12 -> 1.397; FP64: 3.874 / 3.852 /
// 3.888 / 3.902, and at 15 the FP64 loop outgrows the instruction cache
// (5.27 ms).
#ifndef RFV_XY_UNROLL_F32
#define RFV_XY_UNROLL_F32 9
#endif
#ifndef RFV_XY_UNROLL_F64
#define RFV_XY_UNROLL_F64 6
#endif
// FP32 wave strips loading two rows ahead: 6 rows per trip (a multiple of 2
// and 3; 12 measured the same)
#ifndef RFV_XY_UNROLL_WAVES2_F32
#define RFV_XY_UNROLL_WAVES2_F32 6
#endif
template <typename T, int PF> constexpr int xy_unroll() {
  return sizeof(T) == 8 ? RFV_XY_UNROLL_F64 : (PF == 2 ? RFV_XY_UNROLL_WAVES2_F32 : RFV_XY_UNROLL_F32);
}
// Waves per SIMD the wave-strip form is compiled for (caps its registers;
// the variant that also reduces wave speeds is left uncapped: it needs 163
// registers in FP64, three waves per SIMD).
#ifndef RFV_XY_WAVE_OCC_F32
#define RFV_XY_WAVE_OCC_F32 1
#endif
#ifndef RFV_XY_WAVE_OCC_F64
#define RFV_XY_WAVE_OCC_F64 3
#endif
template <typename T> constexpr int xy_wave_occupancy() {
  return sizeof(T) == 4 ? RFV_XY_WAVE_OCC_F32 : RFV_XY_WAVE_OCC_F64;
}
// Rows loaded ahead of their x sweep (1, 2 or 3).  The wave strips that
// also reduce wave speeds (one-pass planar step) load one row ahead: that
// frees 10 registers per lane in FP32 and 20 in FP64 (163 with the
// reduction: three waves per SIMD instead of two), and measured faster: the
// one-pass planar step at 6400 x 4000 took 0.317 ms against 0.364 with
// three rows ahead in FP32, 0.539 against 0.569 in FP64.  The 3D strips load
// two rows ahead, except strips reading linked x neighbours (one).  Against
// one row ahead: FP64 (164 registers, still three waves per SIMD) 512^3 x-y
// 2.67 -> 2.61 ms, 256^3 0.362 -> 0.341 ms; FP32 512^3 strips 1.481 -> 1.455
// ms, the 64-grid batch in strips 1.119 -> 1.103 ms, but the 2 x 2 x 2
// linked sub-blocks of 768^3 5.54 -> 5.58 ms; and the FP64 AoS variant with
// linked x faces would need more than the 168 registers of three waves.
#ifndef RFV_XY_PF_ROWS
#define RFV_XY_PF_ROWS 3
#endif
#ifndef RFV_XY_PF_WAVES_F32
#define RFV_XY_PF_WAVES_F32 2
#endif
#ifndef RFV_XY_PF_WAVES_LINKED
#define RFV_XY_PF_WAVES_LINKED 1
#endif
#ifndef RFV_XY_PF_WAVES_F64
#define RFV_XY_PF_WAVES_F64 2
#endif
template <typename T, int XM, bool FUSE, bool LINKX> constexpr int xy_prefetch() {
  return XM != XM_WAVES   ? RFV_XY_PF_ROWS
         : FUSE           ? 1
         : LINKX          ? RFV_XY_PF_WAVES_LINKED
         : sizeof(T) == 8 ? RFV_XY_PF_WAVES_F64
                          : RFV_XY_PF_WAVES_F32;
}

// Cache policy of the fused pass's stores: non-temporal (2) for the FP32
// rows form (512^3: 1.306 -> 1.283 ms), the default elsewhere (FP64 strips
// 2.609 -> 2.660 ms with non-temporal stores).
#ifndef RFV_XY_ROWS_STORE_POLICY_F32
#define RFV_XY_ROWS_STORE_POLICY_F32 2
#endif
template <typename T, int XM> constexpr int xy_store_policy() {
  return XM == XM_ROWS && sizeof(T) == 4 ? RFV_XY_ROWS_STORE_POLICY_F32 : ST_POL;
}

// XM: form of the x exchange (XM_ROWS, XM_WAVES); the forms differ only in
// which lanes hold which cells and how neighbours are read.  FUSE (wave
// strips only): also reduce |u_d| + c of the new states into the group's
// wave-speed slots, for grids one cell thick in z, where this pass is the
// whole step.
template <typename T, int LAY, int XM, bool FUSE, bool LINKX>
__global__ void __launch_bounds__(XM == XM_WAVES ? XY_WAVE_THREADS : XY_THREADS)
    __attribute__((amdgpu_waves_per_eu(XM == XM_WAVES && !FUSE ? xy_wave_occupancy<T>() : 1)))
    k_sweep_xy(SweepParams p, const DevGrid* __restrict__ grids,
               const int64_t* __restrict__ tile_start, const double* __restrict__ lamv) {
  constexpr bool WAVES = XM == XM_WAVES;
  static_assert(WAVES || !FUSE, "the rows form does not reduce wave speeds");
  constexpr int NT = WAVES ? XY_WAVE_THREADS : XY_THREADS;
  // LDS slots per component: R rows of n0 + 4 slots, R <= NT / XY_MIN_NX
  constexpr int LN = WAVES ? 1 : NT + 4 * (NT / XY_MIN_NX);
  __shared__ T sU[5][LN];
  __shared__ T sR[5][LN];
  __shared__ T sF[5][LN];
  const int tid = threadIdx.x;
  for (int64_t b = first_slot(p.tiles); b < slot_count(p.tiles); b += gridDim.x) {
    const int64_t tb = slot_tile(p.tiles, b);
    if (tb < 0) continue;
    const int64_t gt = uniform(p.tiles.first + tb);
    const int g = find_grid(tile_start, p.w.ngrids, gt);
    const DevGrid& G = grids[g];
    const int lt = (int)(gt - tile_start[g]);
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const bool linked_x = G.mode[0] == FACE_HALO || G.mode[1] == FACE_HALO;
    const int nseg = (ny + p.seg - 1) / p.seg;
    const int s = lt % nseg;
    const int rest = lt / nseg;
    // XM_WAVES: wave wv takes entry rest * R + wv of the waves of the strip
    // plan (groups of k rows at consecutive z: their full strips row-major,
    // then their shared tails); XM_ROWS: the tile's R rows lie at
    // consecutive z from rest * R.
    const bool ghost_lanes = WAVES || linked_x;
    const int R = WAVES ? NT / 64 : NT / (ghost_lanes ? nx + 4 : nx);  // rows per tile
    const int wv = WAVES ? uniform(tid >> 6) : 0;
    const int fw = rest * R + wv;
    int xoff = 0, ncx = nx, kw = 0, h = 0, lane_in = 0;
    if constexpr (WAVES) {
      const StripLane sl = strip_lane(strip_plan(nx, nz, XY_WAVE_CELLS), fw, (int)__lane_id(),
                                      XY_WAVE_CELLS);
      xoff = sl.xoff;
      ncx = sl.ncx;
      kw = sl.kw;
      h = sl.h;
      lane_in = sl.lane_in;
    }
    const int P = WAVES ? 64 : (ghost_lanes ? nx + 4 : nx);  // lanes per row
    const int rs = WAVES ? wv : tid / P;           // row slot of this lane
    // the lane's x relative to xoff (-2 .. ncx+1 with ghost lanes)
    const int xl_ = WAVES ? lane_in - 2 : tid - rs * P - (ghost_lanes ? 2 : 0);
    const int x = xoff + xl_;                      // ... and in the row
    const int kk = WAVES ? kw + h : rest * R + rs;
    if (WAVES && kw >= nz) continue;               // (uniform over the wave)
    const bool row_on = (WAVES || rs < R) && kk < nz;  // the lane belongs to a row
    const bool on = row_on && xl_ >= 0 && xl_ < ncx;  // ... and holds a cell
    // both x faces periodic: the ghost reconstruction and the last face are
    // those of the partner cells (any other case computes them)
    const bool periodic_x =
        !ghost_lanes && G.mode[0] == FACE_PERIODIC && G.mode[1] == FACE_PERIODIC;
    const int LP = nx + 4;                         // LDS row pitch
    const int lb = (row_on ? rs : 0) * LP + 2;     // LDS slot of cell 0 of the lane's row
    const int xl = row_on ? xl_ : 0;               // LDS slot the lane writes: lb + xl
    const int xr = on ? xl_ : 0;                   // slot whose neighbours it reads
    // addresses: column (x, kk) at row j is q0 + (j + 2) Px + lane offset; a
    // ghost lane reads the cell its face names (clamped, wrapped or padding)
    const int kb = WAVES ? kw : rest * R;          // first z of the wave's or tile's rows
    const int kc = row_on ? kk : kb;
    const int xq = WAVES ? min(x, nx + 1) : x;
    const int xc = row_on ? face_index(xq, nx, G.mode[0], G.mode[1]) : 0;
    const int64_t qlane = (int64_t)(kc + 2) * G.pxy + (xc + G.ox);
    const int64_t q0 = uniform(((int64_t)(kb + 2) * G.pxy + G.ox) & ~int64_t(63));
    const uint32_t lane = Layout<LAY>::rel((uint32_t)(qlane - q0)) * (uint32_t)sizeof(T);
    const uint32_t lane_st =
        Layout<LAY>::rel((uint32_t)(qlane - q0 + (x - xc))) * (uint32_t)sizeof(T);
    const int mlo = G.mode[2], mhi = G.mode[3];
    const void* src = G.buf[p.in];
    void* dst = G.buf[p.out];
    const T lamx = (T)lamv[g * 3 + 0];
    const T hlx = T(0.5) * lamx;
    const T lamy = (T)lamv[g * 3 + 1];
    const T hly = T(0.5) * lamy;
    const int j0 = s * p.seg;
    const int len = min(p.seg, ny - j0);
    const int jlast = j0 + len + 1;
    const int64_t ptot = G.ptot;

    auto row = [&](int j) -> int64_t {
      return q0 + (int64_t)(face_index(min(j, jlast), ny, mlo, mhi) + 2) * G.px;
    };

    // Lanes past an x face linked to a sub-block read that neighbour's cells
    // (the state this pass starts from) instead of this grid's padding, so no
    // x halo copy precedes the pass.  Outside the y interior they read the
    // neighbour's y padding rows, which the y halo copy before the pass
    // filled from the diagonal neighbour (the corner cells).  The lanes load
    // this grid's padding first (in bounds, unused) and the neighbour's cells
    // over it.
    struct Nbr {
      const void* src;
      int64_t base, px, ptot;
      uint32_t lane;
      int mlo, mhi;
      bool mine, any;
    };
    auto nbr_source = [&](int side) {
      Nbr r{};
      if (!LINKX || G.mode[side] != FACE_HALO) return r;
      const DevGrid& N = grids[uniform(G.nbr_x[side])];
      r.mine = row_on && (side == 0 ? x < 0 : xq >= nx);
      const int xn = r.mine ? (side == 0 ? N.n[0] + x : xq - nx) : 0;
      r.src = N.buf[p.in];
      r.px = N.px;
      r.ptot = N.ptot;
      r.mlo = N.mode[2];
      r.mhi = N.mode[3];
      r.base = uniform(((int64_t)(kb + 2) * N.pxy + N.ox) & ~int64_t(63));
      r.lane = Layout<LAY>::rel((uint32_t)((int64_t)(kc + 2) * N.pxy + xn + N.ox - r.base)) *
               (uint32_t)sizeof(T);
      r.any = __any(r.mine);
      return r;
    };
    const Nbr nlo = nbr_source(0), nhi = nbr_source(1);
    auto load_row = [&](int j, T out[5]) __attribute__((always_inline)) {
      load_cell_rel<T, LAY>(src, row(j), ptot, lane, out);
      if constexpr (!LINKX) return;
      if (nlo.any && nlo.mine)
        load_cell_rel<T, LAY>(nlo.src, nlo.base + (int64_t)(face_index(min(j, jlast), ny, nlo.mlo,
                                                                       nlo.mhi) + 2) * nlo.px,
                              nlo.ptot, nlo.lane, out);
      if (nhi.any && nhi.mine)
        load_cell_rel<T, LAY>(nhi.src, nhi.base + (int64_t)(face_index(min(j, jlast), ny, nhi.mlo,
                                                                       nhi.mhi) + 2) * nhi.px,
                              nhi.ptot, nhi.lane, out);
    };

    // x sweep of one row held by the lanes: u (this lane's cell) -> o
    auto xsweep = [&](const T u[5], T o[5]) __attribute__((always_inline)) {
      if constexpr (WAVES) {
        // the same operations as below, with neighbours read by lane shifts
        T bl[5], br[5];
        {
          T dm[5], dp[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            dm[c] = u[c] - from_below(u[c]);
            dp[c] = from_above(u[c]) - u[c];
          }
          hancock<T, 0>(u, dm, dp, hlx, bl, br);
        }
        T fl[5];
        {
          T left[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) left[c] = from_below(br[c]);
          hllc<T, 0>(left, bl, fl);                      // face x - 1/2
        }
        T fp[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) fp[c] = from_above(fl[c]);
        update(u, lamx, fp, fl, o);
        return;
      }
      if (row_on && (on || ghost_lanes)) {
#pragma unroll
        for (int c = 0; c < 5; ++c) sU[c][lb + xl] = u[c];
        if (on && !ghost_lanes) {
          if (periodic_x) {
            if (xl_ >= ncx - 2) {
#pragma unroll
              for (int c = 0; c < 5; ++c) sU[c][lb + xl_ - ncx] = u[c];
            }
            if (xl_ < 2) {
#pragma unroll
              for (int c = 0; c < 5; ++c) sU[c][lb + ncx + xl_] = u[c];
            }
          } else {
            if (xl_ == 0) {
#pragma unroll
              for (int c = 0; c < 5; ++c) sU[c][lb - 1] = sU[c][lb - 2] = u[c];
            }
            if (xl_ == ncx - 1) {
#pragma unroll
              for (int c = 0; c < 5; ++c) sU[c][lb + ncx] = sU[c][lb + ncx + 1] = u[c];
            }
          }
        }
      }
      __syncthreads();
      T bl[5], br[5];
      {
        T dm[5], dp[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          dm[c] = u[c] - sU[c][lb + xr - 1];
          dp[c] = sU[c][lb + xr + 1] - u[c];
        }
        hancock<T, 0>(u, dm, dp, hlx, bl, br);
      }
      if (on) {
#pragma unroll
        for (int c = 0; c < 5; ++c) sR[c][lb + xl_] = br[c];
        if (periodic_x && xl_ == ncx - 1) {
#pragma unroll
          for (int c = 0; c < 5; ++c) sR[c][lb - 1] = br[c];
        }
        if (!periodic_x && xl_ == 0) {
          // ghost cell -1: stencil u_{-2}, u_{-1}, u_0
          T ug[5], dm[5], dp[5], gl[5], gr[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            ug[c] = sU[c][lb - 1];
            dm[c] = ug[c] - sU[c][lb - 2];
            dp[c] = u[c] - ug[c];
          }
          hancock<T, 0>(ug, dm, dp, hlx, gl, gr);
#pragma unroll
          for (int c = 0; c < 5; ++c) sR[c][lb - 1] = gr[c];
        }
      }
      __syncthreads();
      T fl[5];
      {
        T left[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) left[c] = sR[c][lb + xr - 1];
        hllc<T, 0>(left, bl, fl);                        // face x - 1/2
      }
      if (on) {
#pragma unroll
        for (int c = 0; c < 5; ++c) sF[c][lb + xl_] = fl[c];
        if (periodic_x) {
          if (xl_ == 0) {
#pragma unroll
            for (int c = 0; c < 5; ++c) sF[c][lb + ncx] = fl[c];
          }
        } else if (xl_ == ncx - 1) {
          // ghost cell n0: stencil u_{n0-1}, u_{n0}, u_{n0+1}; face n0 - 1/2
          T ug[5], dm[5], dp[5], gl[5], gr[5], fg[5];
#pragma unroll
          for (int c = 0; c < 5; ++c) {
            ug[c] = sU[c][lb + ncx];
            dm[c] = ug[c] - u[c];
            dp[c] = sU[c][lb + ncx + 1] - ug[c];
          }
          hancock<T, 0>(ug, dm, dp, hlx, gl, gr);
          hllc<T, 0>(br, gl, fg);
#pragma unroll
          for (int c = 0; c < 5; ++c) sF[c][lb + ncx] = fg[c];
        }
      }
      __syncthreads();
      T fp[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) fp[c] = sF[c][lb + xr + 1];
      update(u, lamx, fp, fl, o);
    };

    // raw ring slot of row r: (r - (j0 - 2)) mod PF (rows are loaded PF rows
    // before they are x-swept); x-swept ring slot: (r - (j0 - 2)) mod 3
    constexpr int PF = xy_prefetch<T, XM, FUSE, LINKX>();
    T raw[PF][5];
    T xs[3][5];
    T dprev[5], dnext[5], bl[5], br[5], brp[5], fprev[5];
    T smax[3] = {T(0), T(0), T(0)};
    bool bad = false;
#pragma unroll
    for (int k = 0; k < PF; ++k) load_row(j0 - 2 + k, raw[k]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      xsweep(raw[i % PF], xs[i % 3]);                               // rows j0-2 .. j0+1
      load_row(j0 - 2 + i + PF, raw[i % PF]);
      if (i == 2) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          dprev[c] = xs[1][c] - xs[0][c];
          dnext[c] = xs[2][c] - xs[1][c];
        }
        hancock<T, 1>(xs[1], dprev, dnext, hly, bl, brp);          // cell j0 - 1
#pragma unroll
        for (int c = 0; c < 5; ++c) dprev[c] = dnext[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) dnext[c] = xs[0][c] - xs[2][c];
    hancock<T, 1>(xs[2], dprev, dnext, hly, bl, br);                // cell j0
    hllc<T, 1>(brp, bl, fprev);                                     // face j0 - 1/2
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      brp[c] = br[c];
      dprev[c] = dnext[c];
    }

    // Iteration o (cell j = j0 + o), k = o mod U: xs[(k+2)%3] = U_j,
    // xs[k%3] = U_{j+1}; row j+2 is x-swept from raw[(k+4)%PF] into
    // xs[(k+1)%3] (the slot of U_{j-1}), and row j+2+PF is loaded into the
    // raw slot just consumed.  dprev = U_{j+1} - U_j, brp = Ub^R_j,
    // fprev = F_{j-1/2}.
    constexpr int U = xy_unroll<T, PF>();
    static_assert(U % 3 == 0 && U % PF == 0, "the loop must advance the rings by whole periods");
    for (int o0 = 0; o0 < len; o0 += U) {
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const int o = o0 + k;
        if (o >= len) break;
        const int j = j0 + o;
        xsweep(raw[(k + 4) % PF], xs[(k + 1) % 3]);                // row j + 2
        load_row(j + 2 + PF, raw[(k + 4) % PF]);
        const T* uj = xs[(k + 2) % 3];
        const T* uj1 = xs[k % 3];
        const T* uj2 = xs[(k + 1) % 3];
#pragma unroll
        for (int c = 0; c < 5; ++c) dnext[c] = uj2[c] - uj1[c];
        hancock<T, 1>(uj1, dprev, dnext, hly, bl, br);             // cell j + 1
        T fcur[5], out[5];
        hllc<T, 1>(brp, bl, fcur);                                 // face j + 1/2
        update(uj, lamy, fcur, fprev, out);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          fprev[c] = fcur[c];
          brp[c] = br[c];
          dprev[c] = dnext[c];
        }
        if (on) store_cell_rel<T, LAY, xy_store_policy<T, XM>()>(dst, q0 + (int64_t)(j + 2) * G.px, ptot, lane_st, out);
        if constexpr (FUSE) {
          T sc[3];
          bool b_ = false;
          wavespeeds(out, sc, b_);
          if (on) {
#pragma unroll
            for (int d = 0; d < 3; ++d) smax[d] = bits_max(smax[d], sc[d]);
            bad |= b_;
          }
        }
      }
    }
    if constexpr (FUSE) {
      // per wave: no barrier, the waves of a workgroup are independent
      if (bad) *p.w.flag = 1u;
      unsigned long long* slot = p.w.s_acc + 3 * G.group;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const unsigned long long bits = __double_as_longlong((double)wave_max(smax[d]));
        if (__lane_id() == 0 && bits > __atomic_load_n(&slot[d], __ATOMIC_RELAXED))
          atomicMax(&slot[d], bits);
      }
    }
    if constexpr (!WAVES) __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Wave speeds, time step, halo copies, fills
// ---------------------------------------------------------------------------

template <typename T, int LAY>
__global__ void __launch_bounds__(WS_BLOCK) k_wavespeed(Work w, int in, TileRange tr,
                                                        unsigned long long* s_out,
                                                        const DevGrid* __restrict__ grids,
                                                        const int64_t* __restrict__ tile_start) {
  __shared__ T red[3 * 16];
  for (int64_t b = first_slot(tr); b < slot_count(tr); b += gridDim.x) {
    const int64_t tb = slot_tile(tr, b);
    if (tb < 0) continue;
    const int64_t gt = uniform(tr.first + tb);
    const int g = find_grid(tile_start, w.ngrids, gt);
    const DevGrid& G = grids[g];
    const int64_t lt = gt - tile_start[g];
    const uint32_t nx = G.n[0], ny = G.n[1];
    const uint32_t ncell = nx * ny * (uint32_t)G.n[2];
    T smax[3] = {T(0), T(0), T(0)};
    bool bad = false;
#pragma unroll
    for (int m = 0; m < WS_CELLS_PER_THREAD; ++m) {
      const int64_t f = lt * (WS_BLOCK * WS_CELLS_PER_THREAD) + m * WS_BLOCK + threadIdx.x;
      if (f < ncell) {
        const uint32_t fu = (uint32_t)f;
        const uint32_t row = fu / nx;
        const uint32_t i = fu - row * nx, jj = row % ny, kk = row / ny;
        const int64_t q = (int64_t)(kk + 2) * G.pxy + (int64_t)(jj + 2) * G.px + (i + G.ox);
        T u[5], s[3];
        bool b_;
        load_cell<T, LAY>(G.buf[in], q, G.ptot, u);
        wavespeeds(u, s, b_);
#pragma unroll
        for (int d = 0; d < 3; ++d) smax[d] = bits_max(smax[d], s[d]);
        bad |= b_;
      }
    }
    unsigned long long* slot = s_out ? s_out : w.s_acc + 3 * G.group;
    fold_wavespeeds<T>(smax, bad, slot, w.flag, red);
  }
}

// dt = cfl * min_d dx_d / S_d per grid from its group's maxima (or a fixed
// dt), lam = dt / dx_d, time accumulated.  One workgroup; when reset_s is
// set the maxima are cleared afterwards so the next z sweep can accumulate
// the following step's values.
__global__ void __launch_bounds__(256) k_dt(Work w, double cfl, double fixed_dt, int reset_s,
                                            double* dt_out) {
  for (int g = threadIdx.x; g < w.ngrids; g += blockDim.x) {
    const DevGrid& G = w.grids[g];
    double dt;
    if (fixed_dt > 0.0) {
      dt = fixed_dt;
    } else {
      const unsigned long long* s = w.s_acc + 3 * G.group;
      double r = G.dx[0] / __longlong_as_double(s[0]);
      for (int d = 1; d < 3; ++d) {
        const double q = G.dx[d] / __longlong_as_double(s[d]);
        if (q < r) r = q;
      }
      dt = cfl * r;
      if (!(dt > 0.0) || !(dt < __builtin_huge_val())) {
        *w.flag = 1u;
        dt = 0.0;
      }
    }
    for (int d = 0; d < 3; ++d) w.lam[g * 3 + d] = dt / G.dx[d];
    w.t[g] += dt;
    w.dt[g] = dt;
    if (dt_out && g == 0) *dt_out = dt;
  }
  if (reset_s) {
    __syncthreads();
    for (int g = threadIdx.x; g < w.ngrids; g += blockDim.x)
      for (int d = 0; d < 3; ++d) w.s_acc[g * 3 + d] = 0ull;
  }
}

// Task = one linked face.  Two layers of the plane across `axis` (interior
// extents, which match between the two sub-blocks) are copied from the
// source's interior edge into the destination's padding.
template <typename T, int LAY>
// `ext` extends the first axis across the face by that many padding layers on
// each side (the x copy that precedes a fused x-y pass also fills the corner
// cells of the y padding rows, which the y copy filled just before).
__global__ void __launch_bounds__(256) k_halo(Work w, int buf, int axis, int ext,
                                              const HaloTask* tasks) {
  const HaloTask tk = tasks[blockIdx.y];
  const DevGrid& Gd = w.grids[tk.dst];
  const DevGrid& Gs = w.grids[tk.src];
  const int a0 = axis == 0 ? 1 : 0, a1 = axis == 2 ? 1 : 2;  // axes across
  const uint32_t na = (a0 == 0 ? Gd.n[0] : Gd.n[1]) + 2 * ext;
  const uint32_t nb = a1 == 1 ? Gd.n[1] : Gd.n[2];
  const uint32_t area = na * nb;
  const int64_t d_a0 = a0 == 1 ? Gd.px : 1, d_a1 = a1 == 1 ? Gd.px : Gd.pxy;
  const int64_t s_a0 = a0 == 1 ? Gs.px : 1, s_a1 = a1 == 1 ? Gs.px : Gs.pxy;
  const int64_t d_ax = axis == 0 ? 1 : (axis == 1 ? Gd.px : Gd.pxy);
  const int64_t s_ax = axis == 0 ? 1 : (axis == 1 ? Gs.px : Gs.pxy);
  const int nd = axis == 0 ? Gd.n[0] : (axis == 1 ? Gd.n[1] : Gd.n[2]);
  const int ns = axis == 0 ? Gs.n[0] : (axis == 1 ? Gs.n[1] : Gs.n[2]);
  // padded index origin along the copy axis and along the first axis across
  const int d_o = axis == 0 ? Gd.ox : 2, s_o = axis == 0 ? Gs.ox : 2;
  const int d_o0 = a0 == 0 ? Gd.ox : 2, s_o0 = a0 == 0 ? Gs.ox : 2;
  for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < 2 * area;
       e += gridDim.x * blockDim.x) {
    // x faces: the two layers are adjacent cells of one row, so neighbouring
    // lanes take the two layers of a row (one 64-byte sector per component
    // and row, fetched once); y and z faces: lanes run along x rows
    const uint32_t layer = axis == 0 ? (e & 1u) : e / area;
    const uint32_t r = axis == 0 ? (e >> 1) : e - layer * area;
    const int ia = (int)(r % na) - ext;
    const uint32_t ib = r / na;
    // index along the axis: destination padding, source interior edge
    const int dpos = (tk.side == 0 ? (int)layer - 2 : nd + (int)layer) + d_o;
    const int spos = (tk.side == 0 ? ns - 2 + (int)layer : (int)layer) + s_o;
    const int64_t across_d = (int64_t)(ia + d_o0) * d_a0 + (int64_t)(ib + 2) * d_a1;
    const int64_t across_s = (int64_t)(ia + s_o0) * s_a0 + (int64_t)(ib + 2) * s_a1;
    T u[5];
    load_cell<T, LAY>(Gs.buf[buf], across_s + spos * s_ax, Gs.ptot, u);
    store_cell<T, LAY>(Gd.buf[buf], across_d + dpos * d_ax, Gd.ptot, u);
  }
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Host byte image -> device memory, carried in the kernel's arguments: the
// copy needs no staging buffer and no allocation, and a captured launch keeps
// its own copy of the bytes.
__global__ void __launch_bounds__(256) k_upload(unsigned char* dst, UploadChunk c) {
  uint64_t* d = reinterpret_cast<uint64_t*>(dst + c.off);
  for (uint32_t i = threadIdx.x; i < c.nwords; i += blockDim.x) d[i] = c.w[i];
}

// ---------------------------------------------------------------------------
// Transfer and diagnostic kernels (runtime layout; not on the hot path)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t desc_q(const Desc& d, int64_t f) {
  const int64_t nx = d.n[0], ny = d.n[1];
  const int64_t i = f % nx, row = f / nx, j = row % ny, k = row / ny;
  return (k + 2) * d.pxy + (j + 2) * d.px + (i + d.ox);
}

__device__ __forceinline__ double load_rt(const Desc& d, int64_t q, int c) {
  const int64_t o = offset_rt(d.lay, q, c, d.ptot);
  return d.dtype == RIPPLE_FV_F32 ? (double)static_cast<const float*>(d.buf)[o]
                                  : static_cast<const double*>(d.buf)[o];
}

__device__ __forceinline__ void store_rt(const Desc& d, int64_t q, int c, double v) {
  const int64_t o = offset_rt(d.lay, q, c, d.ptot);
  if (d.dtype == RIPPLE_FV_F32) static_cast<float*>(d.buf)[o] = (float)v;
  else static_cast<double*>(d.buf)[o] = v;
}

// Primitive input: E = p / (gamma - 1) + rho |u|^2 / 2, computed in FP64.
__global__ void k_import(Desc d, const double* src, int primitive) {
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < ncell;
       f += (int64_t)gridDim.x * blockDim.x) {
    double v[5];
    for (int c = 0; c < 5; ++c) v[c] = src[c * ncell + f];
    if (primitive) {
      const double rho = v[0], uu = v[1], vv = v[2], ww = v[3], pp = v[4];
      v[1] = rho * uu;
      v[2] = rho * vv;
      v[3] = rho * ww;
      v[4] = pp / (1.4 - 1.0) + 0.5 * rho * (uu * uu + vv * vv + ww * ww);
    }
    const int64_t q = desc_q(d, f);
    for (int c = 0; c < 5; ++c) store_rt(d, q, c, v[c]);
  }
}

__global__ void k_export(Desc d, double* dst) {
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < ncell;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = desc_q(d, f);
    for (int c = 0; c < 5; ++c) dst[c * ncell + f] = load_rt(d, q, c);
  }
}

__global__ void k_convert(Desc s, Desc d) {
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < ncell;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t qs = desc_q(s, f), qd = desc_q(d, f);
    for (int c = 0; c < 5; ++c) store_rt(d, qd, c, load_rt(s, qs, c));
  }
}

// Fixed-order tree reduction of NVAL doubles per thread over a block:
// kind 0 = sum, 1 = max, chosen per value index.
template <int NVAL>
__device__ __forceinline__ void block_reduce(double v[NVAL], const int kind[NVAL], double* lds) {
  const int tid = threadIdx.x;
  for (int k = 0; k < NVAL; ++k) lds[k * DIAG_BLOCK + tid] = v[k];
  __syncthreads();
  for (int w = DIAG_BLOCK / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int k = 0; k < NVAL; ++k) {
        const double a = lds[k * DIAG_BLOCK + tid], b = lds[k * DIAG_BLOCK + tid + w];
        lds[k * DIAG_BLOCK + tid] = kind[k] ? __builtin_fmax(a, b) : a + b;
      }
    __syncthreads();
  }
  for (int k = 0; k < NVAL; ++k) v[k] = lds[k * DIAG_BLOCK];
  __syncthreads();
}

__global__ void __launch_bounds__(DIAG_BLOCK) k_sums(Desc d, double* partials) {
  __shared__ double lds[5 * DIAG_BLOCK];
  const int kind[5] = {0, 0, 0, 0, 0};
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t f = blockIdx.x * (int64_t)DIAG_BLOCK + threadIdx.x; f < ncell;
       f += (int64_t)gridDim.x * DIAG_BLOCK) {
    const int64_t q = desc_q(d, f);
    for (int c = 0; c < 5; ++c) acc[c] += load_rt(d, q, c);
  }
  block_reduce<5>(acc, kind, lds);
  if (threadIdx.x == 0)
    for (int c = 0; c < 5; ++c) partials[blockIdx.x * 5 + c] = acc[c];
}

__global__ void __launch_bounds__(DIAG_BLOCK) k_norms(Desc d, const double* ref, double* partials) {
  __shared__ double lds[20 * DIAG_BLOCK];
  const int kind[20] = {0, 0, 1, 1, 0, 0, 1, 1, 0, 0, 1, 1, 0, 0, 1, 1, 0, 0, 1, 1};
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  double acc[20];
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  for (int64_t f = blockIdx.x * (int64_t)DIAG_BLOCK + threadIdx.x; f < ncell;
       f += (int64_t)gridDim.x * DIAG_BLOCK) {
    const int64_t q = desc_q(d, f);
    for (int c = 0; c < 5; ++c) {
      const double a = load_rt(d, q, c), b = ref[c * ncell + f];
      const double e = __builtin_fabs(a - b), m = __builtin_fabs(b);
      acc[4 * c + 0] += e;
      acc[4 * c + 1] += m;
      acc[4 * c + 2] = __builtin_fmax(acc[4 * c + 2], e);
      acc[4 * c + 3] = __builtin_fmax(acc[4 * c + 3], m);
    }
  }
  block_reduce<20>(acc, kind, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < 20; ++k) partials[blockIdx.x * 20 + k] = acc[k];
}

template <int NVAL>
__global__ void __launch_bounds__(DIAG_BLOCK) k_finish(const double* partials, int nblocks,
                                                       double* out, int with_max) {
  __shared__ double lds[NVAL * DIAG_BLOCK];
  int kind[NVAL];
  for (int k = 0; k < NVAL; ++k) kind[k] = with_max ? ((k & 3) >= 2) : 0;
  double acc[NVAL];
  for (int k = 0; k < NVAL; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += DIAG_BLOCK)
    for (int k = 0; k < NVAL; ++k) {
      const double v = partials[b * NVAL + k];
      acc[k] = kind[k] ? __builtin_fmax(acc[k], v) : acc[k] + v;
    }
  block_reduce<NVAL>(acc, kind, lds);
  if (threadIdx.x == 0)
    for (int k = 0; k < NVAL; ++k) out[k] = acc[k];
}

// Relative norms per variable from the four totals sum|u - ref|, sum|ref|,
// max|u - ref|, max|ref| (k_norms layout): l1 = sum|u - ref| / sum|ref| and
// linf = max|u - ref| / max|ref|; a vanishing reference gives 0 where the
// error vanishes too, else +inf.
__device__ __forceinline__ double rel_norm(double err, double ref) {
  return ref > 0.0 ? err / ref : (err == 0.0 ? 0.0 : __builtin_huge_val());
}

__global__ void __launch_bounds__(DIAG_BLOCK) k_finish_norms(const double* partials, int nblocks,
                                                             double* l1, double* linf) {
  __shared__ double lds[20 * DIAG_BLOCK];
  int kind[20];
  for (int k = 0; k < 20; ++k) kind[k] = (k & 3) >= 2;
  double acc[20];
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += DIAG_BLOCK)
    for (int k = 0; k < 20; ++k) {
      const double v = partials[b * 20 + k];
      acc[k] = kind[k] ? __builtin_fmax(acc[k], v) : acc[k] + v;
    }
  block_reduce<20>(acc, kind, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      l1[c] = rel_norm(acc[4 * c + 0], acc[4 * c + 1]);
      linf[c] = rel_norm(acc[4 * c + 2], acc[4 * c + 3]);
    }
  }
}

// Smooth periodic primitive state used by the autotuner to time candidates
// (rho = 1 + 0.2 sin, small velocities, p = 1), planar FP64 [5][n2][n1][n0].
__global__ void k_tune_state(double* W, int nx, int ny, int nz) {
  const int64_t ncell = (int64_t)nx * ny * nz;
  const double two_pi = 6.283185307179586;
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < ncell;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = f % nx, row = f / nx, j = row % ny, k = row / ny;
    const double x = (i + 0.5) / nx, y = (j + 0.5) / ny, z = (k + 0.5) / nz;
    W[f] = 1.0 + 0.2 * sin(two_pi * (x + y + z));
    W[ncell + f] = 0.1 * sin(two_pi * y);
    W[2 * ncell + f] = 0.1 * sin(two_pi * z);
    W[3 * ncell + f] = 0.1 * sin(two_pi * x);
    W[4 * ncell + f] = 1.0;
  }
}

// ---------------------------------------------------------------------------
// Host-side tile counts and launchers
// ---------------------------------------------------------------------------

int lay_of(const ripple_fv_grid& g) {
  if (g.layout == RIPPLE_FV_AOS) return LAY_AOS;
  if (g.layout == RIPPLE_FV_SOA) return LAY_SOA;
  return g.aosoa_w == 16 ? LAY_AOSOA16 : (g.aosoa_w == 32 ? LAY_AOSOA32 : LAY_AOSOA64);
}

int64_t tiles_x(const ripple_fv_grid& g, int x_block) {
  const int64_t total = (int64_t)(g.n[0] + 4) * g.n[1] * g.n[2];
  const int64_t c = x_block - 4;
  return (total + c - 1) / c;
}

int64_t tiles_yz(const ripple_fv_grid& g, int axis, int yz_block, int yz_segment, int yz_cols) {
  const int64_t ngroups = (int64_t)((g.n[0] + yz_cols - 1) / yz_cols) * g.n[axis == 1 ? 2 : 1];
  const int64_t nchunk = (ngroups + yz_block - 1) / yz_block;
  const int64_t nseg = (g.n[axis] + yz_segment - 1) / yz_segment;
  return nchunk * nseg;
}

// Tiles of the fused sweep (must match the kernel's decoding).
bool xy_eligible(const ripple_fv_grid& g) { return g.n[0] >= XY_MIN_NX; }

// Lanes per row of the rows form (0: the row does not fit a workgroup).
static int xy_row_lanes(const ripple_fv_grid& g) {
  const int P = (g.nbr[0] >= 0 || g.nbr[1] >= 0) ? g.n[0] + 4 : g.n[0];
  return P <= XY_THREADS ? P : 0;
}

// Cost of a wave-strip lane-row relative to a lane-row of the rows form.
// FP64, measured at 512^3: 2.89 against 3.37 ms with 576 strip lanes per 512
// cells.  FP32: the rows form won on a 512^3 grid (1.35 against 1.54 ms,
// both forms using every lane of their workgroups but 11 % of the strip
// lanes holding no cell) and on a 256^3 grid (0.200 against 0.236 ms, two
// rows per workgroup), the strips on 2 x 2 x 2 sub-blocks of 384^3 with
// linked x faces (5.26 against 6.01 ms, rows of 388 lanes in 512-lane
// workgroups); any value between 0.89 and 1.14 picks the faster form in all
// three.
static double xy_wave_cost(int dtype) { return dtype == RIPPLE_FV_F64 ? 0.76 : 1.0; }

int xy_mode(int dtype, const ripple_fv_grid* grids, int n, int split_xy) {
  if (split_xy == 3) return XM_WAVES;
  // lanes occupied, summed over the batch's rows, of either form (whole
  // tiles of R rows; whole groups of k rows sharing their tails)
  double rows = 0.0, waves = 0.0;
  for (int i = 0; i < n; ++i) {
    const ripple_fv_grid& g = grids[i];
    const int P = xy_row_lanes(g);
    if (P == 0) return XM_WAVES;
    const int R = XY_THREADS / P;
    rows += (double)XY_THREADS * ((g.n[2] + R - 1) / R) * g.n[1];
    const StripPlan sp = strip_plan(g.n[0], g.n[2], XY_WAVE_CELLS);
    waves += xy_wave_cost(dtype) * 64.0 * sp.per * ((g.n[2] + sp.k - 1) / sp.k) * g.n[1];
  }
  return split_xy == 0 && waves < rows ? XM_WAVES : XM_ROWS;
}

int64_t tiles_xy(const ripple_fv_grid& g, int yz_segment, int xmode) {
  const int64_t nseg = (g.n[1] + yz_segment - 1) / yz_segment;
  if (xmode == XM_WAVES) {
    const StripPlan sp = strip_plan(g.n[0], g.n[2], XY_WAVE_CELLS);
    const int64_t items = (int64_t)(g.n[2] + sp.k - 1) / sp.k * sp.per;
    const int64_t waves = XY_WAVE_THREADS / 64;
    return (items + waves - 1) / waves * nseg;
  }
  const int64_t rows = XY_THREADS / xy_row_lanes(g);
  return (g.n[2] + rows - 1) / rows * nseg;
}

// Cells along the sweep axis that tile lt of a grid marches (its segment's
// length), in the tile numbering the kernels decode.
int tile_len_yz(const ripple_fv_grid& g, int axis, int yz_block, int yz_segment, int yz_cols,
                int64_t lt) {
  const int nd = g.n[axis];
#if RFV_YZ_ORDER
  const int64_t ngroups = (int64_t)((g.n[0] + yz_cols - 1) / yz_cols) * g.n[axis == 1 ? 2 : 1];
  const int64_t nchunk = (ngroups + yz_block - 1) / yz_block;
  const int s = (int)(lt / nchunk);
#else
  (void)yz_block;
  (void)yz_cols;
  const int64_t nseg = (nd + yz_segment - 1) / yz_segment;
  const int s = (int)(lt % nseg);
#endif
  return std::min(yz_segment, nd - s * yz_segment);
}

int tile_len_xy(const ripple_fv_grid& g, int seg, int64_t lt) {
  const int64_t nseg = (g.n[1] + seg - 1) / seg;
  const int s = (int)(lt % nseg);
  return std::min(seg, g.n[1] - s * seg);
}

int64_t tiles_ws(const ripple_fv_grid& g) {
  const int64_t ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const int64_t per = WS_BLOCK * WS_CELLS_PER_THREAD;
  return (ncell + per - 1) / per;
}

template <typename T, int LAY, int COLS>
static hipError_t sweep_yz_cols(int axis, const Tiling& tl, const SweepParams& p, int blocks,
                                hipStream_t s) {
  const DevGrid* G = p.w.grids;
  const int64_t* TS = p.tiles.tile_start;
  const double* L = p.w.lam;
  if (axis == 1 && p.fuse_s)   // last sweep of a step on grids one cell thick in z
    hipLaunchKernelGGL((k_sweep_yz<T, LAY, 1, true, COLS>), dim3(blocks), dim3(tl.yz_block), 0, s, p, G, TS, L);
  else if (axis == 1)
    hipLaunchKernelGGL((k_sweep_yz<T, LAY, 1, false, COLS>), dim3(blocks), dim3(tl.yz_block), 0, s, p, G, TS, L);
  else if (p.fuse_s)
    hipLaunchKernelGGL((k_sweep_yz<T, LAY, 2, true, COLS>), dim3(blocks), dim3(tl.yz_block), 0, s, p, G, TS, L);
  else
    hipLaunchKernelGGL((k_sweep_yz<T, LAY, 2, false, COLS>), dim3(blocks), dim3(tl.yz_block), 0, s, p, G, TS, L);
  return hipGetLastError();
}

template <typename T, int LAY>
static hipError_t sweep_typed(int axis, const Tiling& tl, const SweepParams& p, int blocks,
                              hipStream_t s) {
  const DevGrid* G = p.w.grids;
  const int64_t* TS = p.tiles.tile_start;
  const double* L = p.w.lam;
  if (axis == 0) {
    if (tl.x_block == 128)
      hipLaunchKernelGGL((k_sweep_x<T, LAY, 128>), dim3(blocks), dim3(128), 0, s, p, G, TS, L);
    else
      hipLaunchKernelGGL((k_sweep_x<T, LAY, 256>), dim3(blocks), dim3(256), 0, s, p, G, TS, L);
  } else {
    // FP64 runs one cell per thread only (see sweep_xy_typed)
    if constexpr (sizeof(T) == 4) {
      if (tl.yz_cols == 2) return sweep_yz_cols<T, LAY, 2>(axis, tl, p, blocks, s);
      if constexpr (LAY != LAY_AOS)
        if (tl.yz_cols == 4) return sweep_yz_cols<T, LAY, 4>(axis, tl, p, blocks, s);
    }
    return sweep_yz_cols<T, LAY, 1>(axis, tl, p, blocks, s);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t sweep_lay(int lay, int axis, const Tiling& tl, const SweepParams& p, int blocks,
                            hipStream_t s) {
  switch (lay) {
    case LAY_AOS: return sweep_typed<T, LAY_AOS>(axis, tl, p, blocks, s);
    case LAY_SOA: return sweep_typed<T, LAY_SOA>(axis, tl, p, blocks, s);
    case LAY_AOSOA16: return sweep_typed<T, LAY_AOSOA16>(axis, tl, p, blocks, s);
    case LAY_AOSOA32: return sweep_typed<T, LAY_AOSOA32>(axis, tl, p, blocks, s);
    default: return sweep_typed<T, LAY_AOSOA64>(axis, tl, p, blocks, s);
  }
}

hipError_t launch_sweep(int dtype, int lay, int axis, const Tiling& tl, const SweepParams& p,
                        int grid_blocks, hipStream_t s) {
  if (p.tiles.count <= 0) return hipSuccess;
  return dtype == RIPPLE_FV_F32 ? sweep_lay<float>(lay, axis, tl, p, grid_blocks, s)
                                : sweep_lay<double>(lay, axis, tl, p, grid_blocks, s);
}

template <typename T, int LAY, bool LINKX>
static hipError_t sweep_xy_linked(const SweepParams& p, int blocks, hipStream_t s) {
  if (p.xmode == XM_WAVES && p.fuse_s)
    hipLaunchKernelGGL((k_sweep_xy<T, LAY, XM_WAVES, true, LINKX>), dim3(blocks),
                       dim3(XY_WAVE_THREADS), 0, s, p, p.w.grids, p.tiles.tile_start, p.w.lam);
  else if (p.xmode == XM_WAVES)
    hipLaunchKernelGGL((k_sweep_xy<T, LAY, XM_WAVES, false, LINKX>), dim3(blocks),
                       dim3(XY_WAVE_THREADS), 0, s, p, p.w.grids, p.tiles.tile_start, p.w.lam);
  else
    hipLaunchKernelGGL((k_sweep_xy<T, LAY, XM_ROWS, false, LINKX>), dim3(blocks), dim3(XY_THREADS),
                       0, s, p, p.w.grids, p.tiles.tile_start, p.w.lam);
  return hipGetLastError();
}

// Batches with an x face linked to a sub-block run the variant whose lanes
// past such a face read the neighbour's cells; the others carry no code for it.
template <typename T, int LAY>
static hipError_t sweep_xy_typed(const Tiling&, const SweepParams& p, int blocks, hipStream_t s) {
  return p.link_x ? sweep_xy_linked<T, LAY, true>(p, blocks, s)
                  : sweep_xy_linked<T, LAY, false>(p, blocks, s);
}

template <typename T>
static hipError_t sweep_xy_lay(int lay, const Tiling& tl, const SweepParams& p, int blocks,
                               hipStream_t s) {
  switch (lay) {
    case LAY_AOS: return sweep_xy_typed<T, LAY_AOS>(tl, p, blocks, s);
    case LAY_SOA: return sweep_xy_typed<T, LAY_SOA>(tl, p, blocks, s);
    case LAY_AOSOA16: return sweep_xy_typed<T, LAY_AOSOA16>(tl, p, blocks, s);
    case LAY_AOSOA32: return sweep_xy_typed<T, LAY_AOSOA32>(tl, p, blocks, s);
    default: return sweep_xy_typed<T, LAY_AOSOA64>(tl, p, blocks, s);
  }
}

hipError_t launch_sweep_xy(int dtype, int lay, const Tiling& tl, const SweepParams& p,
                           int grid_blocks, hipStream_t s) {
  if (p.tiles.count <= 0) return hipSuccess;
  return dtype == RIPPLE_FV_F32 ? sweep_xy_lay<float>(lay, tl, p, grid_blocks, s)
                                : sweep_xy_lay<double>(lay, tl, p, grid_blocks, s);
}

template <typename T>
static hipError_t ws_lay(int lay, const Work& w, int in, TileRange tr, unsigned long long* so,
                         int blocks, hipStream_t s) {
  switch (lay) {
    case LAY_AOS: hipLaunchKernelGGL((k_wavespeed<T, LAY_AOS>), dim3(blocks), dim3(WS_BLOCK), 0, s, w, in, tr, so, w.grids, tr.tile_start); break;
    case LAY_SOA: hipLaunchKernelGGL((k_wavespeed<T, LAY_SOA>), dim3(blocks), dim3(WS_BLOCK), 0, s, w, in, tr, so, w.grids, tr.tile_start); break;
    case LAY_AOSOA16: hipLaunchKernelGGL((k_wavespeed<T, LAY_AOSOA16>), dim3(blocks), dim3(WS_BLOCK), 0, s, w, in, tr, so, w.grids, tr.tile_start); break;
    case LAY_AOSOA32: hipLaunchKernelGGL((k_wavespeed<T, LAY_AOSOA32>), dim3(blocks), dim3(WS_BLOCK), 0, s, w, in, tr, so, w.grids, tr.tile_start); break;
    default: hipLaunchKernelGGL((k_wavespeed<T, LAY_AOSOA64>), dim3(blocks), dim3(WS_BLOCK), 0, s, w, in, tr, so, w.grids, tr.tile_start); break;
  }
  return hipGetLastError();
}

hipError_t launch_wavespeed(int dtype, int lay, const Work& w, int in, TileRange tr,
                            unsigned long long* s_out, int grid_blocks, hipStream_t s) {
  if (tr.count <= 0) return hipSuccess;
  return dtype == RIPPLE_FV_F32 ? ws_lay<float>(lay, w, in, tr, s_out, grid_blocks, s)
                                : ws_lay<double>(lay, w, in, tr, s_out, grid_blocks, s);
}

hipError_t launch_dt(const Work& w, double cfl, double fixed_dt, int reset_s, double* dt_out,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_dt, dim3(1), dim3(256), 0, s, w, cfl, fixed_dt, reset_s, dt_out);
  return hipGetLastError();
}

template <typename T>
static hipError_t halo_lay(int lay, const Work& w, int buf, int axis, int ext,
                           const HaloTask* tasks, dim3 grid, hipStream_t s) {
  switch (lay) {
    case LAY_AOS: hipLaunchKernelGGL((k_halo<T, LAY_AOS>), grid, dim3(256), 0, s, w, buf, axis, ext, tasks); break;
    case LAY_SOA: hipLaunchKernelGGL((k_halo<T, LAY_SOA>), grid, dim3(256), 0, s, w, buf, axis, ext, tasks); break;
    case LAY_AOSOA16: hipLaunchKernelGGL((k_halo<T, LAY_AOSOA16>), grid, dim3(256), 0, s, w, buf, axis, ext, tasks); break;
    case LAY_AOSOA32: hipLaunchKernelGGL((k_halo<T, LAY_AOSOA32>), grid, dim3(256), 0, s, w, buf, axis, ext, tasks); break;
    default: hipLaunchKernelGGL((k_halo<T, LAY_AOSOA64>), grid, dim3(256), 0, s, w, buf, axis, ext, tasks); break;
  }
  return hipGetLastError();
}

hipError_t launch_halo(int dtype, int lay, const Work& w, int buf, int axis, int ext,
                       const HaloTask* tasks, int ntasks, int64_t max_area, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  int64_t bx = (2 * max_area + 255) / 256;
  if (bx > 4096) bx = 4096;
  const dim3 grid((unsigned)bx, (unsigned)ntasks);
  return dtype == RIPPLE_FV_F32 ? halo_lay<float>(lay, w, buf, axis, ext, tasks, grid, s)
                                : halo_lay<double>(lay, w, buf, axis, ext, tasks, grid, s);
}

hipError_t launch_upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  UploadChunk c;
  const unsigned char* p = static_cast<const unsigned char*>(src);
  for (size_t off = 0; off < bytes; off += sizeof(c.w)) {
    const size_t len = bytes - off < sizeof(c.w) ? bytes - off : sizeof(c.w);
    c.off = (uint32_t)off;
    c.nwords = (uint32_t)((len + 7) / 8);
    c.w[c.nwords - 1] = 0;
    __builtin_memcpy(c.w, p + off, len);
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, static_cast<unsigned char*>(dst), c);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Plain device copy, the reference stream for HBM bandwidth: every byte read
// once and written once in 16-byte accesses, four per thread, consecutive
// lanes on consecutive addresses.  NT: the stores carry the non-temporal hint.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ void __launch_bounds__(256) k_stream_copy(const u32x4* __restrict__ src,
                                                     u32x4* __restrict__ dst, int64_t n16) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  u32x4 v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k * 256;
    if (i < n16) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t i = base + k * 256;
    if (i < n16) {
      if constexpr (NT) __builtin_nontemporal_store(v[k], &dst[i]);
      else dst[i] = v[k];
    }
  }
}

hipError_t launch_stream_copy(void* dst, const void* src, int64_t bytes, int nt, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  const int64_t blocks = (n16 + 1023) / 1024;
  if (nt)
    hipLaunchKernelGGL(k_stream_copy<true>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n16);
  else
    hipLaunchKernelGGL(k_stream_copy<false>, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n16);
  return hipGetLastError();
}

static unsigned fill_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

static unsigned cell_blocks(const Desc& d) {
  const int64_t ncell = (int64_t)d.n[0] * d.n[1] * d.n[2];
  int64_t b = (ncell + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

hipError_t launch_import(const Desc& d, const double* src, int primitive, hipStream_t s) {
  hipLaunchKernelGGL(k_import, dim3(cell_blocks(d)), dim3(256), 0, s, d, src, primitive);
  return hipGetLastError();
}

hipError_t launch_export(const Desc& d, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_export, dim3(cell_blocks(d)), dim3(256), 0, s, d, dst);
  return hipGetLastError();
}

hipError_t launch_convert(const Desc& src, const Desc& dst, hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(cell_blocks(dst)), dim3(256), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_tune_state(double* W, const int n[3], hipStream_t s) {
  const int64_t ncell = (int64_t)n[0] * n[1] * n[2];
  int64_t b = (ncell + 255) / 256;
  b = b > 65536 ? 65536 : b;
  hipLaunchKernelGGL(k_tune_state, dim3((unsigned)b), dim3(256), 0, s, W, n[0], n[1], n[2]);
  return hipGetLastError();
}

hipError_t launch_sums(const Desc& d, double* partials, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sums, dim3(nblocks), dim3(DIAG_BLOCK), 0, s, d, partials);
  hipLaunchKernelGGL((k_finish<5>), dim3(1), dim3(DIAG_BLOCK), 0, s, partials, nblocks, out, 0);
  return hipGetLastError();
}

hipError_t launch_norms(const Desc& d, const double* ref, double* partials, int nblocks,
                        double* l1, double* linf, hipStream_t s) {
  hipLaunchKernelGGL(k_norms, dim3(nblocks), dim3(DIAG_BLOCK), 0, s, d, ref, partials);
  hipLaunchKernelGGL(k_finish_norms, dim3(1), dim3(DIAG_BLOCK), 0, s, partials, nblocks, l1, linf);
  return hipGetLastError();
}

}  // namespace rfv
