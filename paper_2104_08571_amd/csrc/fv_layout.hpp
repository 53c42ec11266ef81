// Address maps of the three cell layouts (the paper's polymorphic data layout,
// section "Polymorphic Data Layout", plus a blocked AoSoA variant).
//
// q is the padded linear cell index ((k + 2) Py + j + 2) Px + i + ox of cell
// (i, j, k); ptot is the number of cell slots per buffer.
//   AoS      q * 5 + c                        (contiguous cell)
//   SoA      c * ptot + q                     (strided components)
//   AoSoA<W> ((q / W) * 5 + c) * W + q % W    (W consecutive cells per component block)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_internal.hpp"

namespace rfv {

template <int LAY> struct Layout;

// off(q, c): element offset of component c of cell q.
// rel(r):    offset of cell q0 + r relative to cell q0, for any q0 that is a
//            multiple of 64 (so rel does not depend on c or q0):
//            off(q0 + r, c) = off(q0, c) + rel(r).
template <> struct Layout<LAY_AOS> {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t) {
    return q * 5 + c;
  }
  static __device__ __forceinline__ uint32_t rel(uint32_t r) { return r * 5u; }
};

template <> struct Layout<LAY_SOA> {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t ptot) {
    return c * ptot + q;
  }
  static __device__ __forceinline__ uint32_t rel(uint32_t r) { return r; }
};

template <int LOGW> struct LayoutBlocked {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t) {
    return (((q >> LOGW) * 5 + c) << LOGW) + (q & ((int64_t(1) << LOGW) - 1));
  }
  static __device__ __forceinline__ uint32_t rel(uint32_t r) {
    return ((r >> LOGW) * 5u << LOGW) + (r & ((1u << LOGW) - 1u));
  }
};
template <> struct Layout<LAY_AOSOA16> : LayoutBlocked<4> {};
template <> struct Layout<LAY_AOSOA32> : LayoutBlocked<5> {};
template <> struct Layout<LAY_AOSOA64> : LayoutBlocked<6> {};

// Hot-path memory access.  An access is split into a wave-uniform base --
// the address of component c of an aligned cell q0, held in scalar registers
// as a raw buffer resource -- and a 32-bit per-lane byte offset rel(r) * s.
// Buffer instructions add the two in the address unit, so addressing costs no
// vector ALU work.  Lane offsets stay far below the 2 GiB record limit (the
// host bounds grid shapes accordingly).
constexpr int BUFFER_DWORD3 = 0x00020000;  // raw buffer, gfx9-family format word
constexpr int BUFFER_RECORDS = 0x7fffffff;
// Cache-policy bits of the hot-path loads and stores (0: the default policy).
#ifndef RFV_LOAD_POLICY
#define RFV_LOAD_POLICY 0
#endif
#ifndef RFV_STORE_POLICY
#define RFV_STORE_POLICY 0
#endif
constexpr int LD_POL = RFV_LOAD_POLICY;
constexpr int ST_POL = RFV_STORE_POLICY;

// Values that are the same in every lane, stated as such so the compiler keeps
// them in scalar registers (without this it may treat a tile's grid index as
// divergent and fall back to vector loads and per-lane resource loops).
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ void* uniform(const void* p) {
  return reinterpret_cast<void*>(uniform((int64_t)reinterpret_cast<uintptr_t>(p)));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, BUFFER_RECORDS, BUFFER_DWORD3);
}

template <typename T, int POL = LD_POL>
__device__ __forceinline__ T gload(const void* base, uint32_t lane_bytes) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc(base), (int)lane_bytes, 0, POL));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc(base), (int)lane_bytes, 0, POL));
  }
}

template <typename T, int POL = ST_POL>
__device__ __forceinline__ void gstore(void* base, uint32_t lane_bytes, T v) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rsrc(base), (int)lane_bytes, 0, POL);
  } else {
    using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(rsrc(base), 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rsrc(base), (int)lane_bytes, 0, POL);
  }
}

// N consecutive elements of T at base + lane_bytes, as one buffer access of
// 4, 8 or 16 bytes.
template <typename T, int N, int POL = LD_POL>
__device__ __forceinline__ void gload_n(const void* base, uint32_t lane_bytes, T out[N]) {
  constexpr int B = (int)sizeof(T) * N;
  static_assert(B == 4 || B == 8 || B == 16, "unsupported access width");
  if constexpr (B == 4) {
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(rsrc(base), (int)lane_bytes, 0, POL);
    __builtin_memcpy(out, &v, B);
  } else if constexpr (B == 8) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc(base), (int)lane_bytes, 0, POL);
    __builtin_memcpy(out, &v, B);
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rsrc(base), (int)lane_bytes, 0, POL);
    __builtin_memcpy(out, &v, B);
  }
}

template <typename T, int N, int POL = ST_POL>
__device__ __forceinline__ void gstore_n(void* base, uint32_t lane_bytes, const T in[N]) {
  constexpr int B = (int)sizeof(T) * N;
  static_assert(B == 4 || B == 8 || B == 16, "unsupported access width");
  if constexpr (B == 4) {
    uint32_t v;
    __builtin_memcpy(&v, in, B);
    __builtin_amdgcn_raw_buffer_store_b32(v, rsrc(base), (int)lane_bytes, 0, POL);
  } else if constexpr (B == 8) {
    decltype(__builtin_amdgcn_raw_buffer_load_b64(rsrc(base), 0, 0, 0)) v;
    __builtin_memcpy(&v, in, B);
    __builtin_amdgcn_raw_buffer_store_b64(v, rsrc(base), (int)lane_bytes, 0, POL);
  } else {
    decltype(__builtin_amdgcn_raw_buffer_load_b128(rsrc(base), 0, 0, 0)) v;
    __builtin_memcpy(&v, in, B);
    __builtin_amdgcn_raw_buffer_store_b128(v, rsrc(base), (int)lane_bytes, 0, POL);
  }
}

// Uniform base address of component c of aligned cell q0.
template <typename T, int LAY>
__device__ __forceinline__ const void* comp_base(const void* buf, int64_t q0, int c, int64_t ptot) {
  return static_cast<const T*>(buf) + Layout<LAY>::off(q0, c, ptot);
}

template <typename T, int LAY, int POL = LD_POL>
__device__ __forceinline__ void load_cell_rel(const void* buf, int64_t q0, int64_t ptot,
                                              uint32_t lane_bytes, T u[5]) {
  if constexpr (LAY == LAY_AOS && sizeof(T) == 8) {
    // a 40-byte FP64 cell (8-byte aligned) as 16 + 16 + 8 bytes: three
    // accesses per lane instead of five
    const void* b = comp_base<T, LAY>(buf, q0, 0, ptot);
    gload_n<T, 2, POL>(b, lane_bytes, u);
    gload_n<T, 2, POL>(b, lane_bytes + 16u, u + 2);
    u[4] = gload<T, POL>(b, lane_bytes + 32u);
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) u[c] = gload<T, POL>(comp_base<T, LAY>(buf, q0, c, ptot), lane_bytes);
  }
}

template <typename T, int LAY, int POL = ST_POL>
__device__ __forceinline__ void store_cell_rel(void* buf, int64_t q0, int64_t ptot,
                                               uint32_t lane_bytes, const T u[5]) {
  if constexpr (LAY == LAY_AOS && sizeof(T) == 8) {
    void* b = const_cast<void*>(comp_base<T, LAY>(buf, q0, 0, ptot));
    gstore_n<T, 2, POL>(b, lane_bytes, u);
    gstore_n<T, 2, POL>(b, lane_bytes + 16u, u + 2);
    gstore<T, POL>(b, lane_bytes + 32u, u[4]);
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c)
      gstore<T, POL>(const_cast<void*>(comp_base<T, LAY>(buf, q0, c, ptot)), lane_bytes, u[c]);
  }
}

// COLS consecutive cells along x starting at cell q0 + r, r a multiple of COLS:
// u[k][c] is component c of cell k.  In SoA and AoSoA the COLS values of one
// component are adjacent in memory and move as one wider access; in AoS each
// cell is read on its own.
template <typename T, int LAY, int COLS, int POL = LD_POL>
__device__ __forceinline__ void load_group(const void* buf, int64_t q0, int64_t ptot,
                                           uint32_t lane_bytes, T u[COLS][5]) {
  if constexpr (COLS == 1) {
    load_cell_rel<T, LAY, POL>(buf, q0, ptot, lane_bytes, u[0]);
  } else if constexpr (LAY == LAY_AOS) {
#pragma unroll
    for (int k = 0; k < COLS; ++k)
      load_cell_rel<T, LAY, POL>(buf, q0, ptot, lane_bytes + (uint32_t)(5 * k * sizeof(T)), u[k]);
  } else {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      T v[COLS];
      gload_n<T, COLS, POL>(comp_base<T, LAY>(buf, q0, c, ptot), lane_bytes, v);
#pragma unroll
      for (int k = 0; k < COLS; ++k) u[k][c] = v[k];
    }
  }
}

// Store of a group: act[k] says whether cell k lies inside the row.  A
// whole group moves as one wider access per component (SoA, AoSoA); the
// group that straddles the end of a row stores its cells one by one.
template <typename T, int LAY, int COLS, int POL = ST_POL>
__device__ __forceinline__ void store_group(void* buf, int64_t q0, int64_t ptot,
                                            uint32_t lane_bytes, const T u[COLS][5],
                                            const bool act[COLS]) {
  if constexpr (COLS == 1) {
    store_cell_rel<T, LAY, POL>(buf, q0, ptot, lane_bytes, u[0]);
  } else if constexpr (LAY == LAY_AOS) {
#pragma unroll
    for (int k = 0; k < COLS; ++k)
      if (act[k])
        store_cell_rel<T, LAY, POL>(buf, q0, ptot, lane_bytes + (uint32_t)(5 * k * sizeof(T)), u[k]);
  } else {
    if (act[COLS - 1]) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        T v[COLS];
#pragma unroll
        for (int k = 0; k < COLS; ++k) v[k] = u[k][c];
        gstore_n<T, COLS, POL>(const_cast<void*>(comp_base<T, LAY>(buf, q0, c, ptot)), lane_bytes, v);
      }
    } else {
#pragma unroll
      for (int k = 0; k < COLS - 1; ++k)
        if (act[k])
          store_cell_rel<T, LAY, POL>(buf, q0, ptot, lane_bytes + (uint32_t)(k * sizeof(T)), u[k]);
    }
  }
}

// Full 64-bit element offsets (kernels off the hot path).
template <typename T, int LAY>
__device__ __forceinline__ void load_cell(const void* buf, int64_t q, int64_t ptot, T u[5]) {
  const __attribute__((address_space(1))) T* p = (const __attribute__((address_space(1))) T*)buf;
#pragma unroll
  for (int c = 0; c < 5; ++c) u[c] = p[Layout<LAY>::off(q, c, ptot)];
}

template <typename T, int LAY>
__device__ __forceinline__ void store_cell(void* buf, int64_t q, int64_t ptot, const T u[5]) {
  __attribute__((address_space(1))) T* p = (__attribute__((address_space(1))) T*)buf;
#pragma unroll
  for (int c = 0; c < 5; ++c) p[Layout<LAY>::off(q, c, ptot)] = u[c];
}

// Runtime-dispatched offset, for the non-hot transfer and diagnostic kernels.
__device__ __forceinline__ int64_t offset_rt(int lay, int64_t q, int c, int64_t ptot) {
  switch (lay) {
    case LAY_AOS: return Layout<LAY_AOS>::off(q, c, ptot);
    case LAY_SOA: return Layout<LAY_SOA>::off(q, c, ptot);
    case LAY_AOSOA16: return Layout<LAY_AOSOA16>::off(q, c, ptot);
    case LAY_AOSOA32: return Layout<LAY_AOSOA32>::off(q, c, ptot);
    default: return Layout<LAY_AOSOA64>::off(q, c, ptot);
  }
}

}  // namespace rfv
