// Address maps of the three cell layouts (the paper's polymorphic data layout,
// section "Polymorphic Data Layout", plus a blocked AoSoA variant).
//
// q is the padded linear cell index (k Py + j) Px + i; ptot = Px Py Pz.
//   AoS      q * 5 + c                        (contiguous cell)
//   SoA      c * ptot + q                     (strided components)
//   AoSoA<W> ((q / W) * 5 + c) * W + q % W    (W consecutive cells per component block)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fv_internal.hpp"

namespace rfv {

template <int LAY> struct Layout;

template <> struct Layout<LAY_AOS> {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t) {
    return q * 5 + c;
  }
};

template <> struct Layout<LAY_SOA> {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t ptot) {
    return c * ptot + q;
  }
};

template <int LOGW> struct LayoutBlocked {
  static __device__ __host__ __forceinline__ int64_t off(int64_t q, int c, int64_t) {
    return (((q >> LOGW) * 5 + c) << LOGW) + (q & ((int64_t(1) << LOGW) - 1));
  }
};
template <> struct Layout<LAY_AOSOA16> : LayoutBlocked<4> {};
template <> struct Layout<LAY_AOSOA32> : LayoutBlocked<5> {};
template <> struct Layout<LAY_AOSOA64> : LayoutBlocked<6> {};

template <typename T, int LAY>
__device__ __forceinline__ void load_cell(const void* buf, int64_t q, int64_t ptot, T u[5]) {
  const T* p = static_cast<const T*>(buf);
#pragma unroll
  for (int c = 0; c < 5; ++c) u[c] = p[Layout<LAY>::off(q, c, ptot)];
}

template <typename T, int LAY>
__device__ __forceinline__ void store_cell(void* buf, int64_t q, int64_t ptot, const T u[5]) {
  T* p = static_cast<T*>(buf);
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
