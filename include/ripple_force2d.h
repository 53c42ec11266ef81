/*
 * ripple_force2d.h -- two-dimensional flux difference with the FORCE flux on
 * padded grids, for AMD Instinct MI355X (gfx950), C ABI.
 *
 * The Ripple paper's stencil benchmark (section "Flux Difference in Two
 * Dimensions", table "tab:flux"): for every cell of a 2D grid of Euler
 * states, the sum over the two axes of the difference between the numerical
 * fluxes at the cell's upper and lower faces,
 *
 *     D_ij = (F_{i+1/2,j} - F_{i-1/2,j}) + (G_{i,j+1/2} - G_{i,j-1/2}),
 *
 * each face flux from the FORCE scheme (Toro 1996; Toro, "Riemann Solvers
 * and Numerical Methods for Fluid Dynamics", section 7.4.2): the mean of the
 * Lax-Friedrichs flux and the physical flux of the Richtmyer state, with
 * lam_d = dt / dx_d along axis d.  The state per cell is the conserved
 * variables of the 2D Euler equations (rho, m_x, m_y, E), ideal gas,
 * gamma = 1.4.  The first and last cell along each axis read one padding
 * cell beyond the grid (the paper's padded tensors, section "Tensors").
 *
 * Shares the status codes, layouts, precisions, boundary kinds and the
 * context of ripple_fv.h; the conventions listed there (device pointers,
 * caller-owned buffers, streams, nothing enqueued on error) hold here too.
 */
#ifndef RIPPLE_FORCE2D_H
#define RIPPLE_FORCE2D_H

#include <stdint.h>

#include "ripple_fv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RIPPLE_FORCE2D_NVAR 4

/* Boundary kind beside RIPPLE_FV_TRANSMISSIVE and RIPPLE_FV_PERIODIC: the
 * padding cells along this axis already hold the neighbours' values (filled
 * by the caller, e.g. from an adjacent sub-block) and are read as they are. */
#define RIPPLE_FORCE2D_PADDED 2

/* ripple_force2d_import `variables` flag: src covers the padding ring too. */
#define RIPPLE_FORCE2D_WITH_PADDING 2

/* Grid descriptor.  Fill the inputs, then call ripple_force2d_grid_init.
 *
 *  n        interior extents (x, y), each >= 1
 *  bc       per axis: RIPPLE_FV_TRANSMISSIVE (the padding cell repeats the
 *           edge cell), RIPPLE_FV_PERIODIC (it repeats the cell at the other
 *           end) or RIPPLE_FORCE2D_PADDED (it is read from storage)
 *  layout, dtype, aosoa_w   storage as in ripple_fv.h (aosoa_w in
 *           {16, 32, 64} for AOSOA, else 0)
 *  block    threads per workgroup (64, 128, 256, 512, 1024; 0 = 256); never
 *           changes results
 *  segment  rows each wave advances along y (>= 1; 0 = 8); never changes
 *           results
 *  stage    0: each wave loads its rows into registers and exchanges x
 *           neighbours by lane shifts; 1: each wave stages its rows through
 *           LDS with direct global-to-LDS loads and reads its x neighbour's
 *           state there (the paper's shared-memory variant, "ss" of table
 *           "tab:flux"; at most 512 threads per workgroup, larger blocks run
 *           as 512); never changes results
 *  x_origin, pitch, bytes   OUT, see below
 *
 * Storage of one buffer.  Cell (i, j), each index in [-1, n] (interior plus
 * one padding cell per face), has the padded index
 *     q = (j + 1) * Px + i + x_origin
 * and component c (rho, m_x, m_y, E) of it sits at element
 *     AOS    4 q + c
 *     SOA    c * C + q
 *     AOSOA  ((q / W) * 4 + c) * W + q % W      (W = aosoa_w)
 * with C = bytes / (4 * element size) cell slots.  Py = n[1] + 2.  AOS:
 * x_origin = 1, Px = n[0] + 2.  SOA: x_origin = A, Px = n[0] + 2 rounded up
 * to a multiple of A, A = 128 bytes / element size; AOSOA: the same with
 * A = max(128 bytes / element size, aosoa_w).  C = Px Py + x_origin rounded
 * up to a multiple of 64.  In SOA and AOSOA every interior row starts on a
 * 128-byte boundary of the (256-byte aligned) buffer. */
typedef struct ripple_force2d_grid {
  int32_t n[2];
  int32_t bc[2];
  int32_t layout;
  int32_t dtype;
  int32_t aosoa_w;
  int32_t block;
  int32_t segment;
  int32_t stage;
  int32_t x_origin;
  int32_t pad_;
  int64_t pitch[2];
  int64_t bytes;
} ripple_force2d_grid;

/* Validate a descriptor and fill x_origin, pitch[] and bytes.  E_INVALID on
 * extents < 1 or above 2^20, unknown enums, bad aosoa_w, tiling knobs or
 * stage, or a buffer above 2^46 bytes. */
ripple_fv_status ripple_force2d_grid_init(ripple_force2d_grid* g);

/* Load a state.  src: FP64 planar device array [4][n1][n0] (interior), or
 * [4][n1 + 2][n0 + 2] (interior and padding ring, row j + 1 and column i + 1
 * holding cell (i, j)) when `variables` has RIPPLE_FORCE2D_WITH_PADDING set.
 * Base kind RIPPLE_FV_PRIMITIVE: (rho, u, v, p), converted with
 * E = p / (gamma - 1) + rho (u^2 + v^2) / 2 in FP64; RIPPLE_FV_CONSERVED:
 * (rho, m_x, m_y, E).  Values are rounded to the grid's precision.  Cells
 * src does not cover are left untouched. */
ripple_fv_status ripple_force2d_import(ripple_fv_ctx* ctx, const ripple_force2d_grid* g,
                                       const double* src, int32_t variables, void* u,
                                       void* stream);

/* Copy the interior of u (a state or a flux difference) out as FP64 planar
 * [4][n1][n0] (dst, device). */
ripple_fv_status ripple_force2d_export(ripple_fv_ctx* ctx, const ripple_force2d_grid* g,
                                       const void* u, double* dst, void* stream);

/* The flux difference of state u into d (same descriptor: layout, precision
 * and storage), computed in the grid's precision: d's interior cells receive
 * D_ij, its padding is left untouched; u is not modified.  lam_x, lam_y: dt/dx
 * and dt/dy of the FORCE flux, finite and > 0.  u and d must not overlap.
 * Padding cells along a RIPPLE_FORCE2D_PADDED axis must hold valid states.
 * Arithmetic follows IEEE rules: a non-physical state yields non-finite or
 * meaningless outputs but no error. */
ripple_fv_status ripple_force2d_flux_difference(ripple_fv_ctx* ctx, const ripple_force2d_grid* g,
                                                const void* u, double lam_x, double lam_y,
                                                void* d, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RIPPLE_FORCE2D_H */
