/*
 * ripple_fv.h -- padded-tile finite-volume Euler step for AMD Instinct MI355X
 * (gfx950), C ABI.
 *
 * The library advances the three-dimensional compressible Euler equations
 * (ideal gas, gamma = 1.4, conserved variables rho, rho u, rho v, rho w, E)
 * by dimensionally split time steps on padded Cartesian grids.  One step
 * follows the Ripple paper's Euler graph (section "Scaling Performance",
 * listing "Simplified Euler solver graph creation"): per-cell wave speeds, a
 * max reduction, the time step from that maximum, boundary padding, then an
 * out-of-place update along x, then y, then z, with the two state buffers
 * swapped between updates.  Each per-axis update is the MUSCL-Hancock scheme
 * on conserved variables with the minmod slope and the HLLC Riemann solver
 * with Davis wave speeds (Toro, "Riemann Solvers and Numerical Methods for
 * Fluid Dynamics", sections 14.4 and 10.4); the paper leaves that update to
 * the user.
 *
 * Storage follows the paper's padded tensors (section "Tensors": every block
 * carries padding for stencil access) with a halo of two cells on every face,
 * and its polymorphic data layout (section "Polymorphic Data Layout": the
 * same cell type stored contiguously or strided), extended by a blocked
 * layout.  With padded cell indices (i, j, k) -- interior cell (0, 0, 0) at
 * (2, 2, 2) -- pitches Px (even), Py, Pz and q = (k Py + j) Px + i:
 *
 *   RIPPLE_FV_AOS    element (q, c) at  q * 5 + c            (contiguous)
 *   RIPPLE_FV_SOA    element (q, c) at  c * Px Py Pz + q     (strided)
 *   RIPPLE_FV_AOSOA  element (q, c) at  ((q / W) * 5 + c) * W + q % W,
 *                    W = aosoa_w in {16, 32, 64}, Px a multiple of W
 *
 * Component order is (rho, m_x, m_y, m_z, E).  Elements are float (F32) or
 * double (F64); the arithmetic of the update runs in that precision.
 *
 * Conventions shared by every entry point:
 *  - Pointers named u, u_in, u_out, u_a, u_b, src, dst, ref, *_dev are device
 *    pointers on the context's device, at least 256-byte aligned for state
 *    buffers.  All large buffers belong to the caller; the library never
 *    frees them.  A state buffer must hold at least grid.bytes bytes.
 *  - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *    stream).  Work is enqueued asynchronously on it; the call returns once
 *    enqueued.
 *  - Return codes report host-side validation and HIP launch errors only.
 *    On any error nothing has been enqueued.  A state the device finds
 *    non-physical (rho <= 0, p <= 0 or non-finite) sets a sticky flag that
 *    ripple_fv_check reports.
 *  - A context is not thread-safe: use one context per host thread.
 */
#ifndef RIPPLE_FV_H
#define RIPPLE_FV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ripple_fv_status;

enum ripple_fv_status_code {
  RIPPLE_FV_OK = 0,
  RIPPLE_FV_E_INVALID = 1,      /* bad argument: pointer, extent, enum, size */
  RIPPLE_FV_E_UNSUPPORTED = 2,  /* valid but not supported (e.g. mixed layouts in a batch) */
  RIPPLE_FV_E_DEVICE = 3,       /* a HIP call failed; see ripple_fv_last_error */
  RIPPLE_FV_E_NONPHYSICAL = 4,  /* the device met rho <= 0, p <= 0 or a non-finite value */
  RIPPLE_FV_E_NOMEM = 5         /* a workspace allocation failed */
};

enum ripple_fv_layout { RIPPLE_FV_AOS = 0, RIPPLE_FV_SOA = 1, RIPPLE_FV_AOSOA = 2 };
enum ripple_fv_dtype { RIPPLE_FV_F32 = 0, RIPPLE_FV_F64 = 1 };
enum ripple_fv_bc { RIPPLE_FV_TRANSMISSIVE = 0, RIPPLE_FV_PERIODIC = 1 };
enum ripple_fv_variables { RIPPLE_FV_PRIMITIVE = 0, RIPPLE_FV_CONSERVED = 1 };

/* ripple_fv_run_batch flags (bitwise or). */
enum ripple_fv_run_flags {
  RIPPLE_FV_RUN_EAGER = 0,     /* one persistent launch per kernel per step */
  RIPPLE_FV_RUN_GRAPH = 1,     /* replay a captured hipGraph of the step loop */
  RIPPLE_FV_RUN_PER_GRID = 2,  /* one launch per grid per kernel (baseline) */
  RIPPLE_FV_RUN_PROFILE = 4    /* eager, with hipEvents around every launch */
};

/* Kernel kinds reported by ripple_fv_profile. */
enum ripple_fv_kernel_kind {
  RIPPLE_FV_K_WAVESPEED = 0, RIPPLE_FV_K_DT = 1, RIPPLE_FV_K_SWEEP_X = 2,
  RIPPLE_FV_K_SWEEP_Y = 3, RIPPLE_FV_K_SWEEP_Z = 4, RIPPLE_FV_K_HALO = 5,
  RIPPLE_FV_K_SWEEP_XY = 6, RIPPLE_FV_NKERNELS = 7
};

/* ripple_fv_sweep axis values: 0, 1, 2 = x, y, z; RIPPLE_FV_AXIS_XY = the x
 * sweep followed by the y sweep in one fused pass. */
#define RIPPLE_FV_AXIS_XY 3

#define RIPPLE_FV_HALO 2
#define RIPPLE_FV_NVAR 5

/* Grid descriptor.  Fill the inputs, then call ripple_fv_grid_init.
 *
 *  n        interior extents (x, y, z), each >= 1.  An axis one cell thick
 *           makes the grid planar along it: a sweep along that axis reads
 *           the same state on both faces of every cell and changes nothing,
 *           and its periodic and transmissive faces coincide (a two-
 *           dimensional problem is a grid with n[2] = 1 and a dx[2] large
 *           enough that dx[2] / S_z never sets the time step)
 *  bc       boundary condition per axis, applied on both faces that are
 *           physical boundaries (transmissive = constant extrapolation of the
 *           edge cell into the padding; periodic = wrap)
 *  dx       cell widths (> 0); a unit cube has dx[d] = 1 / n[d]
 *  layout, dtype, aosoa_w   storage (aosoa_w in {16, 32, 64} for AOSOA, else 0)
 *  group    grids with the same group share one time step (the sub-blocks of
 *           a partitioned domain); -1 = the grid's own.  A group is named by
 *           the batch index of its first member, which must name itself.
 *  nbr      sub-block links per face (-x, +x, -y, +y, -z, +z): batch index of
 *           the neighbouring sub-block whose interior fills this face's
 *           padding, or -1 when the face is a physical boundary
 *  x_block, yz_block, yz_segment, persist, yz_cols, split_xy   kernel
 *           tiling chosen by ripple_fv_batch_tune (0 = defaults); they never
 *           change results.
 *           x_block: threads per workgroup of the x sweep (128, 256);
 *           yz_block: threads per workgroup of the y/z sweeps (64, 128, 256);
 *           yz_segment: cells each y/z thread advances (>= 4; 0 = 128 for
 *           the y sweep and the fused x-y pass, which shortens it on thin
 *           batches; the z sweep then takes the longest segment that still
 *           gives two tiles per compute unit if there are then at most
 *           four per compute unit, about one round, else 128);
 *           persist: workgroups per CU of persistent launches (0 = one per tile);
 *           yz_cols: adjacent x cells per thread of the separate y and z
 *           sweeps (1, 2, 4; 0 = 2 for FP32 SoA/AoSoA, else 1); FP32 AoS
 *           runs 2 for 4; FP64 always runs 1 (2 and 4 are accepted and mean
 *           1); the fused x-y sweep always runs one cell per thread;
 *           split_xy: how the x and y sweeps run.  0 = as one fused pass
 *           wherever every grid of the batch allows it (n[0] >= 16), in the
 *           form that occupies fewer vector lanes per cell by a measured
 *           cost model: whole rows per workgroup of 512 lanes with
 *           neighbours exchanged through LDS, or strips of 60 cells per wave
 *           with neighbours exchanged by lane shifts (any row length);
 *           1 = always as two separate sweeps; 2 = fused, whole rows where
 *           every row fits a workgroup (n[0] <= 512, 508 with a linked x
 *           face), else strips; 3 = fused, strips.  When every grid is one
 *           cell thick in z, any value but 1 runs the strips form, which
 *           then also reduces the wave speeds
 *  reserved must be 0
 *  x_origin OUT: padded x index of interior cell x = 0 (see below)
 *  pitch, bytes   OUT: padded extents (Px, Py, Pz) and bytes of one buffer
 *
 * Storage of one buffer.  Cell (i, j, k), with each index in [-2, n + 2)
 * (interior plus two padding layers per face), has the padded index
 *     q = ((k + 2) * Py + (j + 2)) * Px + i + x_origin
 * and component c (rho, rho u, rho v, rho w, E) of it sits at element
 *     AOS    5 q + c
 *     SOA    c * C + q
 *     AOSOA  ((q / W) * 5 + c) * W + q % W      (W = aosoa_w)
 * where C = bytes / (5 * element size) is the number of cell slots.  In SOA
 * every interior row starts on a 128-byte boundary of the buffer (the buffer
 * itself being 256-byte aligned), in AOSOA on a block boundary, so sweeps
 * along y and z touch no partial cache lines at row ends. */
typedef struct ripple_fv_grid {
  int32_t n[3];
  int32_t bc[3];
  double dx[3];
  int32_t layout;
  int32_t dtype;
  int32_t aosoa_w;
  int32_t group;
  int32_t nbr[6];
  int32_t x_block;
  int32_t yz_block;
  int32_t yz_segment;
  int32_t persist;
  int32_t yz_cols;
  int32_t split_xy;
  int32_t reserved;
  int32_t x_origin;
  int64_t pitch[3];
  int64_t bytes;
} ripple_fv_grid;

typedef struct ripple_fv_ctx ripple_fv_ctx;

/* Validate a descriptor and fill x_origin, pitch[] and bytes (section
 * "Tensors": padding is part of the tensor's storage).  Py = n[1] + 4,
 * Pz = n[2] + 4.  AOS: x_origin = 2, Px = n[0] + 4 rounded up to even.
 * SOA: x_origin = A, Px = n[0] + 4 rounded up to a multiple of A, where A =
 * 128 bytes / element size (32 for F32, 16 for F64).  AOSOA: the same with
 * A = max(128 bytes / element size, aosoa_w).  The cell-slot count
 * C = Px Py Pz + x_origin rounded up to a multiple of 64.
 * E_INVALID on extents < 1, dx <= 0, unknown enums, bad aosoa_w, bad tiling
 * knobs, or a buffer size above 2^46 bytes. */
ripple_fv_status ripple_fv_grid_init(ripple_fv_grid* g);

/* Create a context on HIP device `device`.  The context owns only small
 * preallocated workspaces (flags, reduction partials, per-batch plans and
 * captured graphs).  E_INVALID for a bad device or NULL ctx, E_DEVICE or
 * E_NOMEM on failure. */
ripple_fv_status ripple_fv_create(ripple_fv_ctx** ctx, int32_t device);
void ripple_fv_destroy(ripple_fv_ctx* ctx);

/* Load an initial state.  src: FP64 planar device array [5][n2][n1][n0],
 * holding primitive (rho, u, v, w, p) or conserved variables per
 * `variables`.  Primitive input is converted with E = p / (gamma - 1) +
 * rho |u|^2 / 2 in FP64, then rounded to the grid's precision.  Writes the
 * interior of u; padding is left untouched. */
ripple_fv_status ripple_fv_import(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                  const double* src, int32_t variables, void* u,
                                  void* stream);

/* Copy the interior of u out as FP64 conserved variables, planar
 * [5][n2][n1][n0] (dst, device). */
ripple_fv_status ripple_fv_export(ripple_fv_ctx* ctx, const ripple_fv_grid* g, const void* u,
                                  double* dst, void* stream);

/* Convert the interior of src (grid gs) into dst (grid gd): layout and/or
 * precision change (the paper's polymorphic layout, section "Polymorphic Data
 * Layout").  gs and gd must have equal n.  FP64 -> FP32 rounds to nearest. */
ripple_fv_status ripple_fv_convert(ripple_fv_ctx* ctx, const ripple_fv_grid* gs, const void* src,
                                   const ripple_fv_grid* gd, void* dst, void* stream);

/* Maximum signal speeds S_d = max over interior cells of |u_d| + c,
 * c = sqrt(gamma p / rho), d = x, y, z (the paper's set_wavespeeds node
 * followed by its max reduction, section "Graphs", paragraph "Reduction").
 * s_dev: 3 doubles (device).  The maximum is exact, so the result does not
 * depend on the reduction order. */
ripple_fv_status ripple_fv_max_wavespeed(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                         const void* u, double* s_dev, void* stream);

/* One sweep along `axis` (0, 1, 2) with time step dt > 0: u_out = the
 * MUSCL-Hancock/HLLC update of u_in along that axis (the paper's
 * update_state_x / update_state_y nodes with concurrent padded access:
 * read u_in and its padding, write u_out).  Physical faces take the
 * boundary condition; faces with a neighbour read u_in's padding, which
 * ripple_fv_halo_exchange fills.  u_in is not modified. */
ripple_fv_status ripple_fv_sweep(ripple_fv_ctx* ctx, const ripple_fv_grid* g, int32_t axis,
                                 const void* u_in, void* u_out, double dt, void* stream);

/* One full step of a whole grid, in place: wave speeds -> dt = cfl * min_d
 * dx_d / S_d (or the fixed dt when dt > 0) -> sweeps x, y, z (section
 * "Graphs": the paper's split Euler example, extended with z).  u holds the
 * state before and after; work is a second buffer of g->bytes that the step
 * clobbers (where the x and y sweeps run as one fused pass the step is
 * u -> work -> u; otherwise the three sweeps ping-pong and the result is
 * copied back; one cell thick in z: u -> work by the one x-y pass and a
 * copy back, or u -> work -> u by separate x and y sweeps).  cfl in (0, 1].
 * dt_dev: optional device double receiving the dt used.
 *
 * In place rather than in -> out: the paper's graph swaps an input and an
 * output tensor after every update (swap_in_out), so a three-update step
 * leaves its result in the other buffer.  Here the x and y updates run as
 * one pass over the state, so a step is two passes, u -> work -> u, and the
 * result is back in u with no copy; an in -> out contract would cost one more
 * read and write of the whole state per step.  Callers that ping-pong
 * buffers keep passing the same pair. */
ripple_fv_status ripple_fv_step(ripple_fv_ctx* ctx, const ripple_fv_grid* g, void* u,
                                void* work, double cfl, double dt, double* dt_dev,
                                void* stream);

/* Advance n independent grids (or sub-blocks of partitioned domains) by
 * nsteps steps, in place: the result is in u[i] for every step count (the
 * work buffers' roles alternate inside, never the caller's; see
 * ripple_fv_step for why the state returns to its own buffer).  Every grid uses its group's dt from the CFL
 * condition.  u[i]: the state of grid i, before and after; work[i]: a second
 * buffer of grids[i].bytes, clobbered.  A step runs the x and y sweeps as one
 * fused pass (u -> work) and the z sweep (work -> u) where every grid allows
 * the fusion (see split_xy); otherwise x (u -> work), y (work -> u), z
 * (u -> work) with the roles swapped every step and one copy back to u after
 * an odd number of steps.  Before each separate sweep along d, faces with a
 * neighbour get their padding copied from the neighbour's interior (the
 * paper's concurrent padded access, section "Tensor Data Dependencies").
 * All grids must share layout, dtype and tiling knobs (else E_UNSUPPORTED).
 * flags: ripple_fv_run_flags.  The first call for a given set of grid
 * descriptors builds and caches a plan (workspaces, tile lists, graphs);
 * later calls with the same descriptors allocate nothing.  When every grid
 * is one cell thick in z the z sweep, which would change nothing, is
 * skipped: a step is one x-y pass (u -> work, roles swapped every step, one
 * copy back after an odd number of steps) that also reduces the next step's
 * wave speeds, or with split_xy = 1 (or n[0] < 16) x (u -> work) and y
 * (work -> u), the y sweep reducing the wave speeds. */
ripple_fv_status ripple_fv_run_batch(ripple_fv_ctx* ctx, int32_t n, const ripple_fv_grid* grids,
                                     void* const* u, void* const* work, int32_t nsteps,
                                     double cfl, int32_t flags, void* stream);

/* ripple_fv_run_batch for callers that cannot allocate: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * advances n grids by nsteps steps exactly as ripple_fv_run_batch with
 * RIPPLE_FV_RUN_EAGER does (same kernels, same results bit for bit, the state
 * in place in u[i], work[i] clobbered), but calls no hipMalloc, hipFree or
 * other allocating routine: the batch's descriptors, tile lists, halo copy
 * tasks and per-grid dt / wave-speed slots live in a file-scope device array
 * of RIPPLE_FV_NOALLOC_SCRATCH_BYTES bytes (32 KiB), which each device the
 * library runs on holds until the process ends.  Each call first writes the
 * whole workspace it uses (zeroed slots included) by small copy kernels that
 * carry the bytes in their arguments, then enqueues the steps on `stream`.
 * Limit: n <= RIPPLE_FV_NOALLOC_MAX_GRIDS (64); more grids give E_INVALID
 * with nothing enqueued.  Every call on one device shares that device's
 * array and leaves its contents behind: calls that overlap on one device
 * (on different streams, or from different contexts) race; calls in the
 * order of one stream do not.  The time reached is not reported
 * (ripple_fv_batch_time covers ripple_fv_run_batch only); the non-physical
 * flag is the context's, read by ripple_fv_check. */
#define RIPPLE_FV_NOALLOC_MAX_GRIDS 64
#define RIPPLE_FV_NOALLOC_SCRATCH_BYTES 32768
ripple_fv_status ripple_fv_run_batch_noalloc(ripple_fv_ctx* ctx, int32_t n,
                                             const ripple_fv_grid* grids, void* const* u,
                                             void* const* work, int32_t nsteps, double cfl,
                                             void* stream);

/* Time reached (t_host[i], since the start of the last ripple_fv_run_batch
 * call on this grid set) and the last dt per grid (dt_host, may be NULL).
 * Synchronises the device. */
ripple_fv_status ripple_fv_batch_time(ripple_fv_ctx* ctx, int32_t n, const ripple_fv_grid* grids,
                                      double* t_host, double* dt_host);

/* Choose layout and tiling for a batch by timing candidates on the device
 * (the paper motivates this: trying every layout by hand is cumbersome,
 * section "Introduction").  `in`: the batch's descriptors (layout fields
 * ignored); `chosen`: OUT, n descriptors with layout, aosoa_w, tiling knobs,
 * pitch and bytes filled.  Allocates temporary buffers; synchronises the
 * device; results are cached in the context per (dtype, extents) set. */
ripple_fv_status ripple_fv_batch_tune(ripple_fv_ctx* ctx, int32_t n, const ripple_fv_grid* in,
                                      ripple_fv_grid* chosen, void* stream);

/* Split a grid into parts[0] x parts[1] x parts[2] sub-blocks on one device
 * (the paper's sub-partitions, section "Tensors").  sub: OUT, the product
 * of parts descriptors, x fastest, each with its own extents (extents split
 * as evenly as possible), dx, nbr links (batch indices offset by
 * first_index) and group = first_index.  The whole grid's periodic axes are
 * linked around, except one-cell axes.  A split axis keeps at least 2 cells
 * per sub-block. */
ripple_fv_status ripple_fv_partition(const ripple_fv_grid* whole, const int32_t parts[3],
                                     int32_t first_index, ripple_fv_grid* sub);

/* Copy the two interior layers next to each linked face along `axis` from
 * the neighbour into the face's padding, for every grid of the batch
 * (the paper's padding-copy nodes, section "Tensor Data Dependencies",
 * "Concurrent access with padding").  u[i]: the buffer of grid i. */
ripple_fv_status ripple_fv_halo_exchange(ripple_fv_ctx* ctx, int32_t n,
                                         const ripple_fv_grid* grids, void* const* u,
                                         int32_t axis, void* stream);

/* Sums over interior cells of each conserved variable, accumulated in FP64
 * in a fixed order (deterministic): sums_dev, 5 doubles (device). */
ripple_fv_status ripple_fv_conserved_sums(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                          const void* u, double* sums_dev, void* stream);

/* Relative error norms of u against ref per conserved variable, over the
 * interior cells, accumulated in FP64 in a fixed order (deterministic):
 *   l1_dev[c]   = sum |u_c - ref_c| / sum |ref_c|
 *   linf_dev[c] = max |u_c - ref_c| / max |ref_c|
 * for c = rho, m_x, m_y, m_z, E (each 5 doubles, device).  A variable whose
 * reference vanishes everywhere gives 0 where u matches it exactly, else
 * +inf.  ref_dev: FP64 conserved variables of the same grid, planar
 * [5][n2][n1][n0] (device).  These are the diagnostic norms the FP32 path's
 * error against an FP64 reference is stated in; the maxima are exact, so
 * linf is one correctly rounded division. */
ripple_fv_status ripple_fv_error_norms(ripple_fv_ctx* ctx, const ripple_fv_grid* g,
                                       const void* u, const double* ref_dev, double* l1_dev,
                                       double* linf_dev, void* stream);

/* Plain device copy of `bytes` (a multiple of 16) from src to dst, each
 * byte read once and written once in 16-byte accesses: the reference
 * stream against which the sweeps' HBM bandwidth is measured, and the
 * known-size program that calibrates hardware byte counters.  flags:
 * RIPPLE_FV_COPY_NONTEMPORAL marks the stores non-temporal.  src and dst
 * must not overlap (E_INVALID). */
#define RIPPLE_FV_COPY_NONTEMPORAL 1
ripple_fv_status ripple_fv_stream_copy(ripple_fv_ctx* ctx, void* dst, const void* src,
                                       int64_t bytes, int32_t flags, void* stream);

/* Wait for the device, then report and clear the sticky non-physical flag:
 * E_NONPHYSICAL if any kernel since the last check met rho <= 0, p <= 0 or
 * a non-finite value (wave-speed kernel and the last sweep of every step),
 * else OK. */
ripple_fv_status ripple_fv_check(ripple_fv_ctx* ctx);

/* Kernel times recorded by RIPPLE_FV_RUN_PROFILE runs since the last call:
 * ms[k] total milliseconds and launches[k] launch counts per
 * ripple_fv_kernel_kind (arrays of RIPPLE_FV_NKERNELS).  Clears them. */
ripple_fv_status ripple_fv_profile(ripple_fv_ctx* ctx, double* ms, int64_t* launches);

/* Static description of a status code. */
const char* ripple_fv_status_string(ripple_fv_status s);

/* Text of the last error on this context ("" if none). */
const char* ripple_fv_last_error(ripple_fv_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RIPPLE_FV_H */
