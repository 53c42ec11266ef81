// Two-dimensional flux difference with the FORCE flux (Ripple paper, section
// "Flux Difference in Two Dimensions"; FORCE: Toro 1996 and Toro, "Riemann
// Solvers and Numerical Methods for Fluid Dynamics", section 7.4.2) and the
// C-ABI entry points declared in ripple_force2d.h.
//
// For every cell
//   D = (F_{i+1/2} - F_{i-1/2}) + (G_{j+1/2} - G_{j-1/2}),
//   FORCE face flux = (F_LF + F(U_RI)) / 2,
//   F_LF = (F(UL) + F(UR)) / 2 + (UL - UR) / (2 lam),
//   U_RI = (UL + UR) / 2 + lam (F(UL) - F(UR)) / 2,
// with lam = dt/dx along the face's axis.  State (rho, m_x, m_y, E).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "fv_internal.hpp"
#include "fv_layout.hpp"
#include "fv_math.hpp"
#include "ripple_force2d.h"

namespace rfv {
namespace {

constexpr int NV2 = RIPPLE_FORCE2D_NVAR;
constexpr int F2_OUT = 62;           // output columns per wave (lanes 1 .. 62)
constexpr int F2_MAX_BLOCK = 1024;

// Element offsets of the four-component layouts.  rel(r): offset of cell
// q0 + r relative to cell q0 for any q0 that is a multiple of the block
// width (AoSoA) -- every row start is one.
template <int LAY> struct Layout4;
template <> struct Layout4<LAY_AOS> {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t) {
    return q * NV2 + c;
  }
  static __device__ __forceinline__ uint32_t rel(uint32_t r) { return r * NV2; }
};
template <> struct Layout4<LAY_SOA> {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t ctot) {
    return c * ctot + q;
  }
  static __device__ __forceinline__ uint32_t rel(uint32_t r) { return r; }
};
template <int LOGW> struct Layout4Blocked {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t) {
    return (((q >> LOGW) * NV2 + c) << LOGW) + (q & ((int64_t(1) << LOGW) - 1));
  }
  static __device__ __forceinline__ uint32_t rel(uint32_t r) {
    return ((r >> LOGW) * (uint32_t)NV2 << LOGW) + (r & ((1u << LOGW) - 1u));
  }
};
template <> struct Layout4<LAY_AOSOA16> : Layout4Blocked<4> {};
template <> struct Layout4<LAY_AOSOA32> : Layout4Blocked<5> {};
template <> struct Layout4<LAY_AOSOA64> : Layout4Blocked<6> {};

__device__ __host__ __forceinline__ int64_t off4_rt(int lay, int64_t q, int c, int64_t ctot) {
  switch (lay) {
    case LAY_AOS: return Layout4<LAY_AOS>::off(q, c, ctot);
    case LAY_SOA: return Layout4<LAY_SOA>::off(q, c, ctot);
    case LAY_AOSOA16: return Layout4<LAY_AOSOA16>::off(q, c, ctot);
    case LAY_AOSOA32: return Layout4<LAY_AOSOA32>::off(q, c, ctot);
    default: return Layout4<LAY_AOSOA64>::off(q, c, ctot);
  }
}

// One row's four components for the lanes of a wave: row start q0 (uniform,
// a multiple of the block width), per-lane byte offset `lane`.  AoS cells
// are 16 (FP32) or 32 (FP64) contiguous bytes and move as 128-bit accesses.
template <typename T, int LAY>
__device__ __forceinline__ void load_row(const void* buf, int64_t q0, int64_t ctot, uint32_t lane,
                                         T u[NV2]) {
  if constexpr (LAY == LAY_AOS) {
    const void* base = static_cast<const T*>(buf) + q0 * NV2;
    if constexpr (sizeof(T) == 4) {
      gload_n<T, 4>(base, lane, u);
    } else {
      gload_n<T, 2>(base, lane, u);
      gload_n<T, 2>(base, lane + 16u, u + 2);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NV2; ++c)
      u[c] = gload<T>(static_cast<const T*>(buf) + Layout4<LAY>::off(q0, c, ctot), lane);
  }
}

template <typename T, int LAY>
__device__ __forceinline__ void store_row(void* buf, int64_t q0, int64_t ctot, uint32_t lane,
                                          const T u[NV2]) {
  if constexpr (LAY == LAY_AOS) {
    void* base = static_cast<T*>(buf) + q0 * NV2;
    if constexpr (sizeof(T) == 4) {
      gstore_n<T, 4>(base, lane, u);
    } else {
      gstore_n<T, 2>(base, lane, u);
      gstore_n<T, 2>(base, lane + 16u, u + 2);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NV2; ++c)
      gstore<T>(static_cast<T*>(buf) + Layout4<LAY>::off(q0, c, ctot), lane, u[c]);
  }
}

// Four consecutive FP32 values as one 16-byte LDS read.
__device__ __forceinline__ void ldv4(const float* p, float u[4]) {
  using V = float __attribute__((ext_vector_type(4)));
  const V v = *reinterpret_cast<const V*>(p);
  u[0] = v[0];
  u[1] = v[1];
  u[2] = v[2];
  u[3] = v[3];
}

// Physical fluxes of one state along x (F) and y (G), sharing 1/rho and p:
//   F = (m_x, m_x u + p, m_y u, u (E + p)),  G = (m_y, m_x v, m_y v + p, v (E + p)),
//   p = (gamma - 1) E - ((gamma - 1)/2) |m|^2 / rho.
template <typename T>
__device__ __forceinline__ void phys_fluxes(const T u[NV2], T F[NV2], T G[NV2]) {
  const T r = Arith<T>::recip(u[0]);
  const T vx = u[1] * r, vy = u[2] * r;
  const T m2 = fma_(u[2], u[2], u[1] * u[1]);
  const T p = fma_(T(-0.5) * gamma_m1<T>() * m2, r, gamma_m1<T>() * u[3]);
  const T e = u[3] + p;
  F[0] = u[1];
  F[1] = fma_(u[1], vx, p);
  F[2] = u[2] * vx;
  F[3] = vx * e;
  G[0] = u[2];
  G[1] = u[1] * vy;
  G[2] = fma_(u[2], vy, p);
  G[3] = vy * e;
}

// FORCE flux along D between UL and UR whose physical fluxes along D are FL,
// FR.  hinv = 1 / (2 lam), hl = lam / 2.
template <typename T, int D>
__device__ __forceinline__ void force_face(const T UL[NV2], const T UR[NV2], const T FL[NV2],
                                           const T FR[NV2], T hinv, T hl, T out[NV2]) {
  T lf[NV2], ri[NV2];
#pragma unroll
  for (int c = 0; c < NV2; ++c) {
    lf[c] = fma_(hinv, UL[c] - UR[c], T(0.5) * (FL[c] + FR[c]));
    ri[c] = fma_(hl, FL[c] - FR[c], T(0.5) * (UL[c] + UR[c]));
  }
  const T r = Arith<T>::recip(ri[0]);
  const T un = ri[1 + D] * r;
  const T m2 = fma_(ri[2], ri[2], ri[1] * ri[1]);
  const T p = fma_(T(-0.5) * gamma_m1<T>() * m2, r, gamma_m1<T>() * ri[3]);
  T f[NV2];
  f[0] = ri[1 + D];
  f[1] = ri[1] * un;
  f[2] = ri[2] * un;
  f[1 + D] = fma_(ri[1 + D], un, p);
  f[3] = un * (ri[3] + p);
#pragma unroll
  for (int c = 0; c < NV2; ++c) out[c] = T(0.5) * (lf[c] + f[c]);
}

struct F2Params {
  const void* u;
  void* d;
  int32_t nx, ny;
  int32_t mode[4];     // FaceMode of -x, +x, -y, +y
  int64_t px;          // padded row pitch in cells
  int64_t ctot;        // cell slots (SoA component stride)
  int32_t ox;          // padded x index of interior x = 0
  int32_t seg;         // rows per wave
  int32_t nstrip;      // strips of F2_OUT columns
  int32_t pad_;
  int64_t ntiles;      // nstrip * segments
  double hinv_x, hl_x, hinv_y, hl_y;
};

// One wave per tile = (strip of 64 lanes over columns strip * 62 - 1 ..
// strip * 62 + 62) x (segment of `seg` rows).  Lane l holds column
// strip * 62 - 1 + l; lanes 1 .. 62 produce outputs, lanes 0 and 63 supply
// the x neighbours.  Each lane computes the x face on its upper side (the
// neighbour's state and flux arrive by a lane shift) and receives the lower
// face from the lane below; along y the wave marches up the segment,
// carrying the lower y face and the physical fluxes of the current row, and
// loads one row ahead.  Every face flux is evaluated once per wave.  Waves
// are independent: no LDS, no barrier.
template <typename T, int LAY>
__global__ void __launch_bounds__(F2_MAX_BLOCK) k_force2d(F2Params p) {
  using L = Layout4<LAY>;
  const int lane = threadIdx.x & 63;
  const int64_t t = uniform(xcd_order(blockIdx.x, gridDim.x) * (int64_t)(blockDim.x >> 6) +
                            (int64_t)(threadIdx.x >> 6));
  if (t >= p.ntiles) return;
  const int strip = (int)(t % p.nstrip);
  const int sg = (int)(t / p.nstrip);
  const int nx = p.nx, ny = p.ny;
  const int col = strip * F2_OUT - 1 + lane;
  // lanes past the upper ghost column load it too (in bounds, discarded)
  const int mc = face_index(min(col, nx), nx, p.mode[0], p.mode[1]);
  const bool out = lane >= 1 && lane <= F2_OUT && col < nx;
  const uint32_t ld = L::rel((uint32_t)(mc + p.ox)) * (uint32_t)sizeof(T);
  const uint32_t st = L::rel((uint32_t)(min(col, nx) + p.ox)) * (uint32_t)sizeof(T);
  const int mylo = p.mode[2], myhi = p.mode[3];
  const int64_t px = p.px, ctot = p.ctot;
  const T hinv_x = (T)p.hinv_x, hl_x = (T)p.hl_x;
  const T hinv_y = (T)p.hinv_y, hl_y = (T)p.hl_y;
  const int j0 = sg * p.seg;
  const int j1 = min(j0 + p.seg, ny);
  auto row_q = [&](int j) -> int64_t {
    return (int64_t)(face_index(j, ny, mylo, myhi) + 1) * px;
  };

  // Rows j and j + 1 sit in two of three row buffers while the third
  // receives row j + 2, loaded one row ahead.  The march is unrolled by three
  // so that the buffers rotate by name: a loaded row is never copied, and its
  // first use waits only for itself, not for the loads and stores issued
  // after it.  (Loading two rows ahead measured no faster.)
  T r0[NV2], r1[NV2], r2[NV2];
  T Fc[NV2], Gc[NV2], gprev[NV2];
  {
    T um[NV2], Fm[NV2], Gm[NV2];
    load_row<T, LAY>(p.u, row_q(j0 - 1), ctot, ld, um);
    load_row<T, LAY>(p.u, row_q(j0), ctot, ld, r0);
    load_row<T, LAY>(p.u, row_q(j0 + 1), ctot, ld, r1);   // j0 + 1 <= j1 always
    phys_fluxes(um, Fm, Gm);
    phys_fluxes(r0, Fc, Gc);
    force_face<T, 1>(um, r0, Gm, Gc, hinv_y, hl_y, gprev);
  }
  // Output row j from uc = row j and un = row j + 1 (Fc, Gc: fluxes of uc;
  // gprev: y face j - 1/2); loads row j + 2 into nxt when the segment needs it.
  auto row = [&](const T(&uc)[NV2], const T(&un)[NV2], T(&nxt)[NV2], int j) {
    if (j + 2 <= j1) load_row<T, LAY>(p.u, row_q(j + 2), ctot, ld, nxt);
    // x faces of row j: upper face here, lower face from the lane below
    T ur[NV2], fr[NV2], fx[NV2];
#pragma unroll
    for (int c = 0; c < NV2; ++c) {
      ur[c] = from_above(uc[c]);
      fr[c] = from_above(Fc[c]);
    }
    force_face<T, 0>(uc, ur, Fc, fr, hinv_x, hl_x, fx);
    // y face j + 1/2
    T Fn[NV2], Gn[NV2], gy[NV2];
    phys_fluxes(un, Fn, Gn);
    force_face<T, 1>(uc, un, Gc, Gn, hinv_y, hl_y, gy);
    T dd[NV2];
#pragma unroll
    for (int c = 0; c < NV2; ++c) dd[c] = (fx[c] - from_below(fx[c])) + (gy[c] - gprev[c]);
    if (out) store_row<T, LAY>(p.d, (int64_t)(j + 1) * px, ctot, st, dd);
#pragma unroll
    for (int c = 0; c < NV2; ++c) {
      Fc[c] = Fn[c];
      Gc[c] = Gn[c];
      gprev[c] = gy[c];
    }
  };
  int j = j0;
  for (; j + 3 <= j1; j += 3) {
    row(r0, r1, r2, j);
    row(r1, r2, r0, j + 1);
    row(r2, r0, r1, j + 2);
  }
  if (j < j1) row(r0, r1, r2, j);
  if (j + 1 < j1) row(r1, r2, r0, j + 1);
}

// The same tiles with the rows staged through LDS (the paper's strided
// shared-memory variant, table "tab:flux", and its contiguous counterpart):
// each wave copies every row it needs into a ring of three row slots in its
// own LDS region with direct global-to-LDS loads (the data bypasses the
// vector registers; lane l of a 4-byte load fills bytes 4 l .. 4 l + 3 of
// the slot part, of a 16-byte load 16 l .. 16 l + 15), then reads its own
// cell and its upper x neighbour's from there instead of loading the row
// into registers and shifting it across lanes.  Row j + 2 is copied while
// row j is computed.  Computed fluxes still move by lane shifts.  Waves are
// independent: no barrier.
//
// Slot layout (bytes): FP32 planar, component c at 256 c (4 bytes per lane);
// FP64 planar, the low and high words of component c at 512 c and 512 c +
// 256; AoS FP32, the 16-byte cells at 0; AoS FP64, the two halves of the
// 32-byte cells at 0 and 1024.
template <typename T> constexpr int f2_slot_bytes() { return sizeof(T) == 4 ? 1024 : 2048; }
constexpr int F2_STAGE_MAX_BLOCK = 512;   // 3 slots x 8 waves: at most 48 KB of LDS

using f2_lds_ptr = __attribute__((address_space(3))) void*;

template <int BYTES>
__device__ __forceinline__ void f2_copy_to_lds(const void* src, unsigned char* dst) {
  static_assert(BYTES == 4 || BYTES == 16, "4- or 16-byte loads");
  if constexpr (BYTES == 4) __builtin_amdgcn_global_load_lds(src, (f2_lds_ptr)dst, 4, 0, 0);
  else __builtin_amdgcn_global_load_lds(src, (f2_lds_ptr)dst, 16, 0, 0);
}

template <typename T, int LAY>
__global__ void __launch_bounds__(F2_STAGE_MAX_BLOCK) k_force2d_lds(F2Params p) {
  using L = Layout4<LAY>;
  extern __shared__ __attribute__((aligned(16))) unsigned char f2_lds[];
  constexpr int SB = f2_slot_bytes<T>();
  const int lane = threadIdx.x & 63;
  const int64_t t = uniform(xcd_order(blockIdx.x, gridDim.x) * (int64_t)(blockDim.x >> 6) +
                            (int64_t)(threadIdx.x >> 6));
  if (t >= p.ntiles) return;
  unsigned char* region = f2_lds + (threadIdx.x >> 6) * 3 * SB;
  const int strip = (int)(t % p.nstrip);
  const int sg = (int)(t / p.nstrip);
  const int nx = p.nx, ny = p.ny;
  const int col = strip * F2_OUT - 1 + lane;
  const int mc = face_index(min(col, nx), nx, p.mode[0], p.mode[1]);
  const bool out = lane >= 1 && lane <= F2_OUT && col < nx;
  const uint32_t ld = L::rel((uint32_t)(mc + p.ox)) * (uint32_t)sizeof(T);
  const uint32_t st = L::rel((uint32_t)(min(col, nx) + p.ox)) * (uint32_t)sizeof(T);
  const int mylo = p.mode[2], myhi = p.mode[3];
  const int64_t px = p.px, ctot = p.ctot;
  const T hinv_x = (T)p.hinv_x, hl_x = (T)p.hl_x;
  const T hinv_y = (T)p.hinv_y, hl_y = (T)p.hl_y;
  const int j0 = sg * p.seg;
  const int j1 = min(j0 + p.seg, ny);
  auto row_q = [&](int j) -> int64_t {
    return (int64_t)(face_index(j, ny, mylo, myhi) + 1) * px;
  };
  // slot of row j: rows j0 - 1, j0, j0 + 1, j0 + 2, ... take slots 0, 1, 2, 0, ...
  auto slot = [&](int j) -> unsigned char* { return region + ((j - j0 + 1) % 3) * SB; };
  auto copy_row = [&](int j) {
    unsigned char* dst = slot(j);
    const int64_t q0 = row_q(j);
    if constexpr (LAY == LAY_AOS) {
      const unsigned char* src =
          static_cast<const unsigned char*>(p.u) + q0 * NV2 * (int64_t)sizeof(T) + ld;
      f2_copy_to_lds<16>(src, dst);
      if constexpr (sizeof(T) == 8) f2_copy_to_lds<16>(src + 16, dst + 1024);
    } else {
#pragma unroll
      for (int c = 0; c < NV2; ++c) {
        const unsigned char* src =
            reinterpret_cast<const unsigned char*>(static_cast<const T*>(p.u) + L::off(q0, c, ctot)) + ld;
        if constexpr (sizeof(T) == 4) {
          f2_copy_to_lds<4>(src, dst + 256 * c);
        } else {
          f2_copy_to_lds<4>(src, dst + 512 * c);
          f2_copy_to_lds<4>(src + 4, dst + 512 * c + 256);
        }
      }
    }
  };
  // the state of lane k's cell in the row held by slot s
  auto read_cell = [&](const unsigned char* s, int k, T u[NV2]) {
    if constexpr (LAY == LAY_AOS) {
      if constexpr (sizeof(T) == 4) {
        ldv4(reinterpret_cast<const float*>(s + 16 * k), u);
      } else {
        const double* a = reinterpret_cast<const double*>(s + 16 * k);
        const double* b = reinterpret_cast<const double*>(s + 1024 + 16 * k);
        u[0] = a[0];
        u[1] = a[1];
        u[2] = b[0];
        u[3] = b[1];
      }
    } else {
#pragma unroll
      for (int c = 0; c < NV2; ++c) {
        if constexpr (sizeof(T) == 4) {
          u[c] = reinterpret_cast<const float*>(s + 256 * c)[k];
        } else {
          const uint32_t lo = reinterpret_cast<const uint32_t*>(s + 512 * c)[k];
          const uint32_t hi = reinterpret_cast<const uint32_t*>(s + 512 * c + 256)[k];
          u[c] = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
        }
      }
    }
  };
  const int east = min(lane + 1, 63);

  T uc[NV2], Fc[NV2], Gc[NV2], gprev[NV2];
  {
    copy_row(j0 - 1);
    copy_row(j0);
    copy_row(j0 + 1);                           // j0 + 1 <= j1 always
    __builtin_amdgcn_s_waitcnt(0);
    T um[NV2], Fm[NV2], Gm[NV2];
    read_cell(slot(j0 - 1), lane, um);
    read_cell(slot(j0), lane, uc);
    phys_fluxes(um, Fm, Gm);
    phys_fluxes(uc, Fc, Gc);
    force_face<T, 1>(um, uc, Gm, Gc, hinv_y, hl_y, gprev);
  }
  for (int j = j0; j < j1; ++j) {
    // rows j and j + 1 are in their slots; copy row j + 2 into the slot of
    // row j - 1 (no longer read) while row j is computed
    __builtin_amdgcn_s_waitcnt(0);
    if (j + 2 <= j1) copy_row(j + 2);
    T un[NV2], ur[NV2], fr[NV2], fx[NV2];
    read_cell(slot(j + 1), lane, un);
    read_cell(slot(j), east, ur);
#pragma unroll
    for (int c = 0; c < NV2; ++c) fr[c] = from_above(Fc[c]);
    force_face<T, 0>(uc, ur, Fc, fr, hinv_x, hl_x, fx);
    T Fn[NV2], Gn[NV2], gy[NV2];
    phys_fluxes(un, Fn, Gn);
    force_face<T, 1>(uc, un, Gc, Gn, hinv_y, hl_y, gy);
    T dd[NV2];
#pragma unroll
    for (int c = 0; c < NV2; ++c) dd[c] = (fx[c] - from_below(fx[c])) + (gy[c] - gprev[c]);
    if (out) store_row<T, LAY>(p.d, (int64_t)(j + 1) * px, ctot, st, dd);
#pragma unroll
    for (int c = 0; c < NV2; ++c) {
      uc[c] = un[c];
      Fc[c] = Fn[c];
      Gc[c] = Gn[c];
      gprev[c] = gy[c];
    }
  }
}

// Transfers between FP64 planar arrays and the padded storage (not timed).
struct D2 {
  void* buf;
  int32_t nx, ny, lay, dtype, ox;
  int32_t pad_;
  int64_t px, ctot;
};

__global__ void k_import2d(D2 d, const double* src, int primitive, int with_pad) {
  const int64_t sx = d.nx + 2 * with_pad, sy = d.ny + 2 * with_pad;
  const int64_t ncell = sx * sy;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncell;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t jj = k / sx, ii = k - jj * sx;
    const int64_t i = ii - with_pad, j = jj - with_pad;
    double w[NV2];
#pragma unroll
    for (int c = 0; c < NV2; ++c) w[c] = src[c * ncell + k];
    if (primitive) {
      const double rho = w[0], u = w[1], v = w[2], pr = w[3];
      w[1] = rho * u;
      w[2] = rho * v;
      w[3] = pr / (1.4 - 1.0) + 0.5 * rho * (u * u + v * v);
    }
    const int64_t q = (j + 1) * d.px + i + d.ox;
#pragma unroll
    for (int c = 0; c < NV2; ++c) {
      const int64_t o = off4_rt(d.lay, q, c, d.ctot);
      if (d.dtype == RIPPLE_FV_F32) static_cast<float*>(d.buf)[o] = (float)w[c];
      else static_cast<double*>(d.buf)[o] = w[c];
    }
  }
}

__global__ void k_export2d(D2 d, double* dst) {
  const int64_t ncell = (int64_t)d.nx * d.ny;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ncell;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = k / d.nx, i = k - j * d.nx;
    const int64_t q = (j + 1) * d.px + i + d.ox;
#pragma unroll
    for (int c = 0; c < NV2; ++c) {
      const int64_t o = off4_rt(d.lay, q, c, d.ctot);
      dst[c * ncell + k] = d.dtype == RIPPLE_FV_F32 ? (double)static_cast<const float*>(d.buf)[o]
                                                    : static_cast<const double*>(d.buf)[o];
    }
  }
}

int lay_of2(const ripple_force2d_grid& g) {
  if (g.layout == RIPPLE_FV_AOS) return LAY_AOS;
  if (g.layout == RIPPLE_FV_SOA) return LAY_SOA;
  return g.aosoa_w == 16 ? LAY_AOSOA16 : (g.aosoa_w == 32 ? LAY_AOSOA32 : LAY_AOSOA64);
}

int64_t slots2(const ripple_force2d_grid& g) {
  return g.bytes / (NV2 * (g.dtype == RIPPLE_FV_F32 ? 4 : 8));
}

D2 d2_of(const ripple_force2d_grid& g, const void* buf) {
  D2 d{};
  d.buf = const_cast<void*>(buf);
  d.nx = g.n[0];
  d.ny = g.n[1];
  d.lay = lay_of2(g);
  d.dtype = g.dtype;
  d.ox = g.x_origin;
  d.px = g.pitch[0];
  d.ctot = slots2(g);
  return d;
}

int transfer_blocks(int64_t ncell) {
  return (int)std::min<int64_t>(std::max<int64_t>((ncell + 255) / 256, 1), 65536);
}

// Rows per wave: 8 unless set.  Short segments keep the waves that run at
// the same time on a compact band of rows, so the rows above and below a
// segment and the sectors that neighbouring strips share are served from L2;
// measured at 32768^2: 4 to 8 rows equal, 16 about 8 % and 128 about 35 %
// slower, despite the two extra rows a segment reads.
int f2_segment(const ripple_force2d_grid& g) { return g.segment > 0 ? g.segment : 8; }

template <typename T, int LAY>
hipError_t launch_force2d_typed(const F2Params& p, int block, int stage, hipStream_t s) {
  if (stage) block = std::min(block, F2_STAGE_MAX_BLOCK);
  const int wpb = block / 64;
  const int64_t blocks = (p.ntiles + wpb - 1) / wpb;
  if (stage)
    hipLaunchKernelGGL((k_force2d_lds<T, LAY>), dim3((unsigned)blocks), dim3(block),
                       wpb * 3 * f2_slot_bytes<T>(), s, p);
  else
    hipLaunchKernelGGL((k_force2d<T, LAY>), dim3((unsigned)blocks), dim3(block), 0, s, p);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_force2d_dtype(int lay, const F2Params& p, int block, int stage, hipStream_t s) {
  switch (lay) {
    case LAY_AOS: return launch_force2d_typed<T, LAY_AOS>(p, block, stage, s);
    case LAY_SOA: return launch_force2d_typed<T, LAY_SOA>(p, block, stage, s);
    case LAY_AOSOA16: return launch_force2d_typed<T, LAY_AOSOA16>(p, block, stage, s);
    case LAY_AOSOA32: return launch_force2d_typed<T, LAY_AOSOA32>(p, block, stage, s);
    default: return launch_force2d_typed<T, LAY_AOSOA64>(p, block, stage, s);
  }
}

constexpr int64_t F2_MAX_EXTENT = int64_t(1) << 20;
constexpr int64_t F2_MAX_BYTES = int64_t(1) << 46;

// Why a descriptor's inputs are invalid, or nullptr.
const char* grid2_invalid(const ripple_force2d_grid& g) {
  for (int d = 0; d < 2; ++d) {
    if (g.n[d] < 1 || g.n[d] > F2_MAX_EXTENT) return "extent out of range [1, 2^20]";
    if (g.bc[d] != RIPPLE_FV_TRANSMISSIVE && g.bc[d] != RIPPLE_FV_PERIODIC &&
        g.bc[d] != RIPPLE_FORCE2D_PADDED)
      return "unknown boundary kind";
  }
  if (g.dtype != RIPPLE_FV_F32 && g.dtype != RIPPLE_FV_F64) return "unknown dtype";
  if (g.layout == RIPPLE_FV_AOSOA) {
    if (g.aosoa_w != 16 && g.aosoa_w != 32 && g.aosoa_w != 64) return "aosoa_w must be 16, 32 or 64";
  } else if (g.layout == RIPPLE_FV_AOS || g.layout == RIPPLE_FV_SOA) {
    if (g.aosoa_w != 0) return "aosoa_w must be 0 unless the layout is AOSOA";
  } else {
    return "unknown layout";
  }
  if (g.block != 0 && g.block != 64 && g.block != 128 && g.block != 256 && g.block != 512 &&
      g.block != 1024)
    return "block must be 0, 64, 128, 256, 512 or 1024";
  if (g.segment < 0) return "segment < 0";
  if (g.stage != 0 && g.stage != 1) return "stage must be 0 or 1";
  return nullptr;
}

ripple_fv_status grid2_check(const ripple_force2d_grid& g, int64_t* pitch, int64_t* bytes,
                             int32_t* x_origin, std::string* why) {
  if (const char* bad = grid2_invalid(g)) {
    *why = bad;
    return RIPPLE_FV_E_INVALID;
  }
  const int64_t s = g.dtype == RIPPLE_FV_F32 ? 4 : 8;
  int64_t ox, px;
  if (g.layout == RIPPLE_FV_AOS) {
    ox = 1;
    px = (int64_t)g.n[0] + 2;
  } else {
    int64_t a = 128 / s;
    if (g.layout == RIPPLE_FV_AOSOA) a = std::max<int64_t>(a, g.aosoa_w);
    ox = a;
    px = ((int64_t)g.n[0] + 2 + a - 1) / a * a;
  }
  const int64_t py = (int64_t)g.n[1] + 2;
  const int64_t slots = (px * py + ox + 63) / 64 * 64;
  const int64_t b = slots * NV2 * s;
  if (b > F2_MAX_BYTES) {
    *why = "buffer above 2^46 bytes";
    return RIPPLE_FV_E_INVALID;
  }
  pitch[0] = px;
  pitch[1] = py;
  *bytes = b;
  *x_origin = (int32_t)ox;
  return RIPPLE_FV_OK;
}

ripple_fv_status grid2_ok(ripple_fv_ctx* ctx, const ripple_force2d_grid* g) {
  if (!g) return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "NULL grid");
  int64_t pitch[2], bytes;
  int32_t ox;
  std::string why;
  const ripple_fv_status st = grid2_check(*g, pitch, &bytes, &ox, &why);
  if (st) return ctx_fail(ctx, st, why.c_str());
  if (pitch[0] != g->pitch[0] || pitch[1] != g->pitch[1] || bytes != g->bytes || ox != g->x_origin)
    return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "descriptor not initialised by ripple_force2d_grid_init");
  return RIPPLE_FV_OK;
}

int face_mode2(int bc) {
  return bc == RIPPLE_FV_PERIODIC ? FACE_PERIODIC
                                  : (bc == RIPPLE_FORCE2D_PADDED ? FACE_HALO : FACE_TRANSMISSIVE);
}

}  // namespace
}  // namespace rfv

using namespace rfv;

extern "C" {

ripple_fv_status ripple_force2d_grid_init(ripple_force2d_grid* g) {
  if (!g) return RIPPLE_FV_E_INVALID;
  int64_t pitch[2], bytes;
  int32_t ox;
  std::string why;
  const ripple_fv_status st = grid2_check(*g, pitch, &bytes, &ox, &why);
  if (st) return st;
  g->pitch[0] = pitch[0];
  g->pitch[1] = pitch[1];
  g->bytes = bytes;
  g->x_origin = ox;
  g->pad_ = 0;
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_force2d_import(ripple_fv_ctx* ctx, const ripple_force2d_grid* g,
                                       const double* src, int32_t variables, void* u,
                                       void* stream) {
  ripple_fv_status st = ctx_begin(ctx);
  if (st) return st;
  if ((st = grid2_ok(ctx, g))) return st;
  const int with_pad = (variables & RIPPLE_FORCE2D_WITH_PADDING) ? 1 : 0;
  const int kind = variables & ~RIPPLE_FORCE2D_WITH_PADDING;
  if (kind != RIPPLE_FV_PRIMITIVE && kind != RIPPLE_FV_CONSERVED)
    return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "unknown variables kind");
  const int64_t ncell = ((int64_t)g->n[0] + 2 * with_pad) * ((int64_t)g->n[1] + 2 * with_pad);
  if ((st = ctx_ptr_ok(ctx, src, ncell * NV2 * 8, 8, "src"))) return st;
  if ((st = ctx_ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  hipLaunchKernelGGL(k_import2d, dim3(transfer_blocks(ncell)), dim3(256), 0, (hipStream_t)stream,
                     d2_of(*g, u), src, kind == RIPPLE_FV_PRIMITIVE ? 1 : 0, with_pad);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx_fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_force2d_export(ripple_fv_ctx* ctx, const ripple_force2d_grid* g,
                                       const void* u, double* dst, void* stream) {
  ripple_fv_status st = ctx_begin(ctx);
  if (st) return st;
  if ((st = grid2_ok(ctx, g))) return st;
  const int64_t ncell = (int64_t)g->n[0] * g->n[1];
  if ((st = ctx_ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  if ((st = ctx_ptr_ok(ctx, dst, ncell * NV2 * 8, 8, "dst"))) return st;
  hipLaunchKernelGGL(k_export2d, dim3(transfer_blocks(ncell)), dim3(256), 0, (hipStream_t)stream,
                     d2_of(*g, u), dst);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return ctx_fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e));
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_force2d_flux_difference(ripple_fv_ctx* ctx, const ripple_force2d_grid* g,
                                                const void* u, double lam_x, double lam_y,
                                                void* d, void* stream) {
  ripple_fv_status st = ctx_begin(ctx);
  if (st) return st;
  if ((st = grid2_ok(ctx, g))) return st;
  if (!(std::isfinite(lam_x) && lam_x > 0.0 && std::isfinite(lam_y) && lam_y > 0.0))
    return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "lam_x and lam_y must be finite and > 0");
  if ((st = ctx_ptr_ok(ctx, u, g->bytes, 256, "u"))) return st;
  if ((st = ctx_ptr_ok(ctx, d, g->bytes, 256, "d"))) return st;
  const char* a = static_cast<const char*>(u);
  const char* b = static_cast<const char*>(d);
  if (a < b + g->bytes && b < a + g->bytes) return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "u and d overlap");
  F2Params p{};
  p.u = u;
  p.d = d;
  p.nx = g->n[0];
  p.ny = g->n[1];
  p.mode[0] = p.mode[1] = face_mode2(g->bc[0]);
  p.mode[2] = p.mode[3] = face_mode2(g->bc[1]);
  p.px = g->pitch[0];
  p.ctot = slots2(*g);
  p.ox = g->x_origin;
  p.seg = f2_segment(*g);
  p.nstrip = (g->n[0] + F2_OUT - 1) / F2_OUT;
  p.ntiles = (int64_t)p.nstrip * ((g->n[1] + p.seg - 1) / p.seg);
  p.hinv_x = 0.5 / lam_x;
  p.hl_x = 0.5 * lam_x;
  p.hinv_y = 0.5 / lam_y;
  p.hl_y = 0.5 * lam_y;
  const int block = g->block ? g->block : 256;
  const int lay = lay_of2(*g);
  const hipError_t e = g->dtype == RIPPLE_FV_F32
                           ? launch_force2d_dtype<float>(lay, p, block, g->stage, (hipStream_t)stream)
                           : launch_force2d_dtype<double>(lay, p, block, g->stage, (hipStream_t)stream);
  if (e != hipSuccess) return ctx_fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e));
  return RIPPLE_FV_OK;
}

}  // extern "C"
