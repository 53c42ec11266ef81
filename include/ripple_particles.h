/*
 * ripple_particles.h -- particle update in three dimensions for AMD Instinct
 * MI355X (gfx950), C ABI.
 *
 * The Ripple paper's layout benchmark (section "Particle Update in Three
 * Dimensions", table "tab:particle_update"): every particle's position is
 * advanced by its velocity over one time step, x <- x + v dt, for
 * three-dimensional positions and velocities stored contiguously (AoS),
 * strided (SoA) or blocked (AoSoA), in FP32 or FP64 (the paper's section
 * "Polymorphic Data Layout").
 *
 * Shares the status codes, layouts, precisions and the context of
 * ripple_fv.h; the conventions listed there (device pointers, caller-owned
 * buffers, streams, nothing enqueued on error) hold here too.
 */
#ifndef RIPPLE_PARTICLES_H
#define RIPPLE_PARTICLES_H

#include <stdint.h>

#include "ripple_fv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RIPPLE_PARTICLES_NCOMP 6

/* Particle set descriptor.  Fill the inputs, then call ripple_particles_init.
 *
 *  n        number of particles, 1 .. 2^34
 *  layout, dtype, aosoa_w   storage as in ripple_fv.h
 *  block    threads per workgroup (64, 128, 256, 512, 1024; 0 = 256);
 *           never changes results
 *  stage    0: each lane loads its particles into registers; 1: each wave
 *           first copies its particles into LDS with direct global-to-LDS
 *           loads (the paper's shared-memory variants, "ss" and "cs" of
 *           table "tab:particle_update") and computes from there; never
 *           changes results
 *  slots, bytes   OUT
 *
 * Storage.  Component c of particle k -- c = 0, 1, 2 the position x, y, z,
 * c = 3, 4, 5 the velocity -- sits at element
 *     AOS    6 k + c
 *     SOA    c * C + k
 *     AOSOA  ((k / W) * 6 + c) * W + k % W      (W = aosoa_w)
 * with C = slots = n rounded up to a multiple of 64, and bytes = 6 C
 * elements.  Slots beyond n are never read or written. */
typedef struct ripple_particles {
  int64_t n;
  int32_t layout;
  int32_t dtype;
  int32_t aosoa_w;
  int32_t block;
  int32_t stage;
  int32_t pad_;
  int64_t slots;
  int64_t bytes;
} ripple_particles;

/* Validate a descriptor and fill slots and bytes.  E_INVALID on n out of
 * range, unknown enums, bad aosoa_w, block or stage. */
ripple_fv_status ripple_particles_init(ripple_particles* p);

/* Load particles from src, an FP64 planar device array [6][n] (x, y, z,
 * v_x, v_y, v_z), rounded to the descriptor's precision. */
ripple_fv_status ripple_particles_import(ripple_fv_ctx* ctx, const ripple_particles* p,
                                         const double* src, void* buf, void* stream);

/* Copy the particles of buf out as FP64 planar [6][n] (dst, device). */
ripple_fv_status ripple_particles_export(ripple_fv_ctx* ctx, const ripple_particles* p,
                                         const void* buf, double* dst, void* stream);

/* One update in place: position += velocity * dt for every particle, with dt
 * rounded to the working precision and the product and sum formed by one
 * fused multiply-add (one rounding).  Velocities are not modified.  dt must
 * be finite. */
ripple_fv_status ripple_particles_update(ripple_fv_ctx* ctx, const ripple_particles* p, void* buf,
                                         double dt, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RIPPLE_PARTICLES_H */
