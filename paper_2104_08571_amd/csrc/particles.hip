// Particle update in three dimensions (Ripple paper, section "Particle Update
// in Three Dimensions"): x <- x + v dt per particle, and the C-ABI entry
// points declared in ripple_particles.h.
//
// A pure stream: each particle's six components are read once and its three
// position components written once (9 elements per particle), so the kernel
// is bound by HBM bandwidth and the layout decides how the accesses coalesce.
//   SoA / AoSoA: a lane takes a group of 16 bytes per component (4 FP32 or
//     2 FP64 particles), six 128-bit loads and three 128-bit stores.
//   AoS: a lane takes one particle, its 6 contiguous elements as three
//     64-bit (FP32) or 128-bit (FP64) accesses.
// Staged (the paper's shared-memory variants): each wave first copies the
// bytes of its 64 lanes' particles into its own LDS region with direct
// global-to-LDS loads (global_load_lds_dwordx4: the data bypasses the vector
// registers, lane l of a load filling bytes 16 l .. 16 l + 15 of the
// region), waits for them, and computes from LDS; the positions go back to
// HBM as above.  For AoS the copy is fully coalesced 16-byte chunks of the
// wave's contiguous 64 particles; for SoA / AoSoA it is the same 16-byte
// groups the register path loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "fv_internal.hpp"
#include "fv_layout.hpp"
#include "ripple_particles.h"

namespace rfv {
namespace {

constexpr int NC = RIPPLE_PARTICLES_NCOMP;

// Element offset of component c of particle k.
__device__ __host__ __forceinline__ int64_t poff(int lay, int64_t k, int c, int64_t slots) {
  switch (lay) {
    case LAY_AOS: return k * NC + c;
    case LAY_SOA: return c * slots + k;
    case LAY_AOSOA16: return ((k >> 4) * NC + c) * 16 + (k & 15);
    case LAY_AOSOA32: return ((k >> 5) * NC + c) * 32 + (k & 31);
    default: return ((k >> 6) * NC + c) * 64 + (k & 63);
  }
}

template <int LAY> struct PLog;
template <> struct PLog<LAY_AOSOA16> { static constexpr int W = 16; };
template <> struct PLog<LAY_AOSOA32> { static constexpr int W = 32; };
template <> struct PLog<LAY_AOSOA64> { static constexpr int W = 64; };

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// N consecutive elements as one vector access (p aligned to its size).
template <typename T, int N>
__device__ __forceinline__ void ldv(const T* p, T out[N]) {
  using V = T __attribute__((ext_vector_type(N)));
  const V v = *reinterpret_cast<const V*>(p);
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = v[i];
}
template <typename T, int N>
__device__ __forceinline__ void stv(T* p, const T in[N]) {
  using V = T __attribute__((ext_vector_type(N)));
  V v;
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = in[i];
  *reinterpret_cast<V*>(p) = v;
}

struct PParams {
  void* buf;
  int64_t n;
  int64_t slots;
  double dt;
};

// SoA and AoSoA: groups of G = 16 / sizeof(T) consecutive particles, which
// share a block of every component (G divides the block width).  A group
// that runs past n falls back to one particle at a time.
template <typename T, int LAY>
__global__ void __launch_bounds__(1024) k_particles_planar(PParams p) {
  constexpr int G = 16 / (int)sizeof(T);
  const T dt = (T)p.dt;
  T* __restrict__ b = static_cast<T*>(p.buf);
  const int64_t ngroups = (p.n + G - 1) / G;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ngroups; g += stride) {
    const int64_t k0 = g * G;
    int64_t base[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (LAY == LAY_SOA) base[c] = c * p.slots + k0;
      else base[c] = ((k0 / PLog<LAY>::W) * NC + c) * PLog<LAY>::W + (k0 % PLog<LAY>::W);
    }
    if (k0 + G <= p.n) {
      T x[3][G], v[3][G];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ldv<T, G>(b + base[d], x[d]);
        ldv<T, G>(b + base[3 + d], v[d]);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int i = 0; i < G; ++i) x[d][i] = fma_t(v[d][i], dt, x[d][i]);
        stv<T, G>(b + base[d], x[d]);
      }
    } else {
      for (int64_t i = 0; k0 + i < p.n; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) b[base[d] + i] = fma_t(b[base[3 + d] + i], dt, b[base[d] + i]);
    }
  }
}

// AoS: one particle per lane, its six elements contiguous (8-byte aligned in
// FP32, 16-byte aligned in FP64).
template <typename T>
__global__ void __launch_bounds__(1024) k_particles_aos(PParams p) {
  const T dt = (T)p.dt;
  T* __restrict__ b = static_cast<T*>(p.buf);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < p.n; k += stride) {
    T* q = b + k * NC;
    T e[NC];
    ldv<T, 2>(q, e);
    ldv<T, 2>(q + 2, e + 2);
    ldv<T, 2>(q + 4, e + 4);
    T x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = fma_t(e[3 + d], dt, e[d]);
    stv<T, 2>(q, x);
    q[2] = x[2];
  }
}

// LDS region of one wave in the staged kernels: the planar form holds 16
// bytes per lane and component, the AoS form the wave's 64 contiguous
// particles (rounded up to whole 1 KB loads).
template <typename T> constexpr int stage_bytes_planar() { return NC * 64 * 16; }
template <typename T> constexpr int stage_bytes_aos() { return (64 * NC * (int)sizeof(T) + 1023) / 1024 * 1024; }
constexpr int STAGE_MAX_BLOCK = 512;   // staged kernels: at most 48 KB of LDS per workgroup

using lds_ptr = __attribute__((address_space(3))) void*;

// Direct copy of 16 bytes per active lane from src (per lane) to the wave's
// LDS region dst (uniform) + 16 lane.
__device__ __forceinline__ void copy16_to_lds(const void* src, unsigned char* dst) {
  __builtin_amdgcn_global_load_lds(src, (lds_ptr)dst, 16, 0, 0);
}

template <typename T, int LAY>
__global__ void __launch_bounds__(STAGE_MAX_BLOCK) k_particles_planar_lds(PParams p) {
  constexpr int G = 16 / (int)sizeof(T);
  extern __shared__ __attribute__((aligned(16))) unsigned char p_lds[];
  const int lane = threadIdx.x & 63;
  unsigned char* region = p_lds + (threadIdx.x >> 6) * stage_bytes_planar<T>();
  const T dt = (T)p.dt;
  T* __restrict__ b = static_cast<T*>(p.buf);
  const int64_t ngroups = (p.n + G - 1) / G;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = uniform((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
       w * 64 < ngroups; w += nwaves) {
    const int64_t k0 = (w * 64 + lane) * G;
    int64_t base[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (LAY == LAY_SOA) base[c] = c * p.slots + k0;
      else base[c] = ((k0 / PLog<LAY>::W) * NC + c) * PLog<LAY>::W + (k0 % PLog<LAY>::W);
    }
    if ((w * 64 + 64) * G <= p.n) {          // (uniform) every lane holds G particles
#pragma unroll
      for (int c = 0; c < NC; ++c) copy16_to_lds(b + base[c], region + c * 1024);
      __builtin_amdgcn_s_waitcnt(0);
      T x[3][G], v[3][G];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ldv<T, G>(reinterpret_cast<const T*>(region + d * 1024 + lane * 16), x[d]);
        ldv<T, G>(reinterpret_cast<const T*>(region + (3 + d) * 1024 + lane * 16), v[d]);
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int i = 0; i < G; ++i) x[d][i] = fma_t(v[d][i], dt, x[d][i]);
        stv<T, G>(b + base[d], x[d]);
      }
    } else {
      for (int64_t i = 0; i < G && k0 + i < p.n; ++i)
#pragma unroll
        for (int d = 0; d < 3; ++d) b[base[d] + i] = fma_t(b[base[3 + d] + i], dt, b[base[d] + i]);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(STAGE_MAX_BLOCK) k_particles_aos_lds(PParams p) {
  constexpr int REC = NC * (int)sizeof(T);    // bytes per particle
  constexpr int NCH = 64 * REC / 16;          // 16-byte chunks of a wave's particles
  extern __shared__ __attribute__((aligned(16))) unsigned char p_lds[];
  const int lane = threadIdx.x & 63;
  unsigned char* region = p_lds + (threadIdx.x >> 6) * stage_bytes_aos<T>();
  const T dt = (T)p.dt;
  T* __restrict__ b = static_cast<T*>(p.buf);
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t w = uniform((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
       w * 64 < p.n; w += nwaves) {
    const int64_t k = w * 64 + lane;
    T* q = b + k * NC;
    T e[NC];
    if (w * 64 + 64 <= p.n) {                   // (uniform) the wave's 64 particles exist
      const unsigned char* src = reinterpret_cast<const unsigned char*>(b + w * 64 * NC);
#pragma unroll
      for (int i = 0; i < (NCH + 63) / 64; ++i)
        if (i * 64 + lane < NCH) copy16_to_lds(src + (i * 64 + lane) * 16, region + i * 1024);
      __builtin_amdgcn_s_waitcnt(0);
      const T* r = reinterpret_cast<const T*>(region + lane * REC);
      ldv<T, 2>(r, e);
      ldv<T, 2>(r + 2, e + 2);
      ldv<T, 2>(r + 4, e + 4);
    } else {
      if (k >= p.n) continue;
      ldv<T, 2>(q, e);
      ldv<T, 2>(q + 2, e + 2);
      ldv<T, 2>(q + 4, e + 4);
    }
    T x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = fma_t(e[3 + d], dt, e[d]);
    stv<T, 2>(q, x);
    q[2] = x[2];
  }
}

struct PDesc {
  void* buf;
  int64_t n, slots;
  int32_t lay, dtype;
};

__global__ void k_pimport(PDesc d, const double* src) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < d.n;
       k += (int64_t)gridDim.x * blockDim.x)
    for (int c = 0; c < NC; ++c) {
      const int64_t o = poff(d.lay, k, c, d.slots);
      const double v = src[c * d.n + k];
      if (d.dtype == RIPPLE_FV_F32) static_cast<float*>(d.buf)[o] = (float)v;
      else static_cast<double*>(d.buf)[o] = v;
    }
}

__global__ void k_pexport(PDesc d, double* dst) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < d.n;
       k += (int64_t)gridDim.x * blockDim.x)
    for (int c = 0; c < NC; ++c) {
      const int64_t o = poff(d.lay, k, c, d.slots);
      dst[c * d.n + k] = d.dtype == RIPPLE_FV_F32 ? (double)static_cast<const float*>(d.buf)[o]
                                                  : static_cast<const double*>(d.buf)[o];
    }
}

int play_of(const ripple_particles& p) {
  if (p.layout == RIPPLE_FV_AOS) return LAY_AOS;
  if (p.layout == RIPPLE_FV_SOA) return LAY_SOA;
  return p.aosoa_w == 16 ? LAY_AOSOA16 : (p.aosoa_w == 32 ? LAY_AOSOA32 : LAY_AOSOA64);
}

constexpr int64_t P_MAX_N = int64_t(1) << 34;

ripple_fv_status pcheck(const ripple_particles& p, int64_t* slots, int64_t* bytes, const char** why) {
  *why = nullptr;
  if (p.n < 1 || p.n > P_MAX_N) *why = "n out of range [1, 2^34]";
  else if (p.dtype != RIPPLE_FV_F32 && p.dtype != RIPPLE_FV_F64) *why = "unknown dtype";
  else if (p.layout == RIPPLE_FV_AOSOA && p.aosoa_w != 16 && p.aosoa_w != 32 && p.aosoa_w != 64)
    *why = "aosoa_w must be 16, 32 or 64";
  else if ((p.layout == RIPPLE_FV_AOS || p.layout == RIPPLE_FV_SOA) && p.aosoa_w != 0)
    *why = "aosoa_w must be 0 unless the layout is AOSOA";
  else if (p.layout != RIPPLE_FV_AOS && p.layout != RIPPLE_FV_SOA && p.layout != RIPPLE_FV_AOSOA)
    *why = "unknown layout";
  else if (p.block != 0 && p.block != 64 && p.block != 128 && p.block != 256 && p.block != 512 &&
           p.block != 1024)
    *why = "block must be 0, 64, 128, 256, 512 or 1024";
  else if (p.stage != 0 && p.stage != 1)
    *why = "stage must be 0 or 1";
  if (*why) return RIPPLE_FV_E_INVALID;
  *slots = (p.n + 63) / 64 * 64;
  *bytes = *slots * NC * (p.dtype == RIPPLE_FV_F32 ? 4 : 8);
  return RIPPLE_FV_OK;
}

ripple_fv_status p_ok(ripple_fv_ctx* ctx, const ripple_particles* p) {
  if (!p) return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "NULL descriptor");
  int64_t slots, bytes;
  const char* why;
  if (pcheck(*p, &slots, &bytes, &why)) return ctx_fail(ctx, RIPPLE_FV_E_INVALID, why);
  if (slots != p->slots || bytes != p->bytes)
    return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "descriptor not initialised by ripple_particles_init");
  return RIPPLE_FV_OK;
}

PDesc pdesc(const ripple_particles& p, const void* buf) {
  return PDesc{const_cast<void*>(buf), p.n, p.slots, play_of(p), p.dtype};
}

int stream_blocks(int64_t items, int block) {
  return (int)std::min<int64_t>(std::max<int64_t>((items + block - 1) / block, 1), 1 << 20);
}

template <typename T>
hipError_t launch_update(int lay, const PParams& pp, int block, int stage, hipStream_t s) {
  const int64_t items = lay == LAY_AOS ? pp.n : (pp.n + 16 / (int)sizeof(T) - 1) / (16 / (int)sizeof(T));
  if (stage) {
    block = std::min(block, STAGE_MAX_BLOCK);
    const dim3 grid(stream_blocks(items, block)), threads(block);
    const int waves = block / 64;
    switch (lay) {
      case LAY_AOS:
        hipLaunchKernelGGL((k_particles_aos_lds<T>), grid, threads, waves * stage_bytes_aos<T>(), s, pp);
        break;
      case LAY_SOA:
        hipLaunchKernelGGL((k_particles_planar_lds<T, LAY_SOA>), grid, threads,
                           waves * stage_bytes_planar<T>(), s, pp);
        break;
      case LAY_AOSOA16:
        hipLaunchKernelGGL((k_particles_planar_lds<T, LAY_AOSOA16>), grid, threads,
                           waves * stage_bytes_planar<T>(), s, pp);
        break;
      case LAY_AOSOA32:
        hipLaunchKernelGGL((k_particles_planar_lds<T, LAY_AOSOA32>), grid, threads,
                           waves * stage_bytes_planar<T>(), s, pp);
        break;
      default:
        hipLaunchKernelGGL((k_particles_planar_lds<T, LAY_AOSOA64>), grid, threads,
                           waves * stage_bytes_planar<T>(), s, pp);
        break;
    }
    return hipGetLastError();
  }
  const dim3 grid(stream_blocks(items, block)), threads(block);
  switch (lay) {
    case LAY_AOS: hipLaunchKernelGGL((k_particles_aos<T>), grid, threads, 0, s, pp); break;
    case LAY_SOA: hipLaunchKernelGGL((k_particles_planar<T, LAY_SOA>), grid, threads, 0, s, pp); break;
    case LAY_AOSOA16: hipLaunchKernelGGL((k_particles_planar<T, LAY_AOSOA16>), grid, threads, 0, s, pp); break;
    case LAY_AOSOA32: hipLaunchKernelGGL((k_particles_planar<T, LAY_AOSOA32>), grid, threads, 0, s, pp); break;
    default: hipLaunchKernelGGL((k_particles_planar<T, LAY_AOSOA64>), grid, threads, 0, s, pp); break;
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace rfv

using namespace rfv;

extern "C" {

ripple_fv_status ripple_particles_init(ripple_particles* p) {
  if (!p) return RIPPLE_FV_E_INVALID;
  int64_t slots, bytes;
  const char* why;
  const ripple_fv_status st = pcheck(*p, &slots, &bytes, &why);
  if (st) return st;
  p->slots = slots;
  p->bytes = bytes;
  p->pad_ = 0;
  return RIPPLE_FV_OK;
}

ripple_fv_status ripple_particles_import(ripple_fv_ctx* ctx, const ripple_particles* p,
                                         const double* src, void* buf, void* stream) {
  ripple_fv_status st = ctx_begin(ctx);
  if (st || (st = p_ok(ctx, p))) return st;
  if ((st = ctx_ptr_ok(ctx, src, p->n * NC * 8, 8, "src"))) return st;
  if ((st = ctx_ptr_ok(ctx, buf, p->bytes, 256, "buf"))) return st;
  hipLaunchKernelGGL(k_pimport, dim3(stream_blocks(p->n, 256)), dim3(256), 0, (hipStream_t)stream,
                     pdesc(*p, buf), src);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RIPPLE_FV_OK : ctx_fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e));
}

ripple_fv_status ripple_particles_export(ripple_fv_ctx* ctx, const ripple_particles* p,
                                         const void* buf, double* dst, void* stream) {
  ripple_fv_status st = ctx_begin(ctx);
  if (st || (st = p_ok(ctx, p))) return st;
  if ((st = ctx_ptr_ok(ctx, buf, p->bytes, 256, "buf"))) return st;
  if ((st = ctx_ptr_ok(ctx, dst, p->n * NC * 8, 8, "dst"))) return st;
  hipLaunchKernelGGL(k_pexport, dim3(stream_blocks(p->n, 256)), dim3(256), 0, (hipStream_t)stream,
                     pdesc(*p, buf), dst);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RIPPLE_FV_OK : ctx_fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e));
}

ripple_fv_status ripple_particles_update(ripple_fv_ctx* ctx, const ripple_particles* p, void* buf,
                                         double dt, void* stream) {
  ripple_fv_status st = ctx_begin(ctx);
  if (st || (st = p_ok(ctx, p))) return st;
  if (!std::isfinite(dt)) return ctx_fail(ctx, RIPPLE_FV_E_INVALID, "dt must be finite");
  if ((st = ctx_ptr_ok(ctx, buf, p->bytes, 256, "buf"))) return st;
  const PParams pp{buf, p->n, p->slots, dt};
  const int block = p->block ? p->block : 256;
  const int lay = play_of(*p);
  const hipError_t e = p->dtype == RIPPLE_FV_F32
                          ? launch_update<float>(lay, pp, block, p->stage, (hipStream_t)stream)
                          : launch_update<double>(lay, pp, block, p->stage, (hipStream_t)stream);
  return e == hipSuccess ? RIPPLE_FV_OK : ctx_fail(ctx, RIPPLE_FV_E_DEVICE, hipGetErrorString(e));
}

}  // extern "C"
