/*
 * FP64 CPU oracle for one dimensionally split finite-volume time step of the
 * three-dimensional compressible Euler equations on a Cartesian grid.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source, header, table or helper with
 * the HIP library.
 *
 * What it computes, and where each part comes from:
 *
 *  - Step structure (Ripple paper, section "Scaling Performance", listing
 *    "Simplified Euler solver graph creation"): per-cell wave speeds, a max
 *    reduction, the time step from that maximum, boundary padding, then one
 *    split update per axis in a fixed order, out of place, double buffered.
 *  - Padding (paper, section "Tensors"): two ghost layers per face filled by
 *    constant extrapolation (transmissive) or by periodic wrap.
 *  - The per-axis update (the paper leaves it open): the textbook
 *    MUSCL-Hancock scheme on conserved variables (Toro, "Riemann Solvers and
 *    Numerical Methods for Fluid Dynamics", section 14.4) with the minmod
 *    slope, and the HLLC Riemann solver (Toro section 10.4) with Davis wave
 *    speed estimates (Toro eq. 10.48).
 *
 * State layout: planar FP64, component-major, U[c*ncell + (k*ny + j)*nx + i],
 * components (rho, m_x, m_y, m_z, E).  Ideal gas, gamma = 1.4.
 *
 * Built with -O2 -fno-fast-math -ffp-contract=off.  Every output cell is
 * written by one thread from read-only input, so results do not depend on
 * the OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 5
static const double GAMMA = 1.4;

/* Status codes returned by the step and run functions. */
enum {
  ORACLE_OK = 0,
  ORACLE_NONPHYSICAL = 1,   /* rho <= 0, p <= 0 or a non-finite value */
  ORACLE_BAD_ARGS = 2,
  ORACLE_NOMEM = 3
};

/* Stage at which a non-physical state was met (reported in info[1]). */
enum {
  STAGE_DT = 0,        /* state at the start of the step */
  STAGE_INPUT = 1,     /* cell state read by the sweep */
  STAGE_EXTRAP = 2,    /* U^L, U^R */
  STAGE_EVOLVED = 3,   /* evolved boundary states after the half step */
  STAGE_OUTPUT = 4     /* updated cell */
};

int oracle_abi_version(void) { return 1; }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------ */
/* Equation of state and physical flux (Toro ch. 3, eq. 3.2 in x).     */
/* ------------------------------------------------------------------ */

/* p = (gamma - 1) (E - |m|^2 / (2 rho)) */
static double pressure_of(const double U[NV]) {
  double rho = U[0];
  double kinetic = 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / rho;
  return (GAMMA - 1.0) * (U[4] - kinetic);
}

/* A state is physical when all components are finite, rho > 0 and p > 0. */
static int is_physical(const double U[NV]) {
  for (int c = 0; c < NV; ++c)
    if (!isfinite(U[c])) return 0;
  if (!(U[0] > 0.0)) return 0;
  double p = pressure_of(U);
  return isfinite(p) && p > 0.0;
}

double oracle_pressure(const double U[NV]) { return pressure_of(U); }

/* Flux along axis d: (m_d, m_x u_d + p dx_d, m_y u_d + p dy_d,
 * m_z u_d + p dz_d, u_d (E + p)), with u_d = m_d / rho. */
void oracle_flux(const double U[NV], int d, double F[NV]) {
  double rho = U[0];
  double un = U[1 + d] / rho;
  double p = pressure_of(U);
  F[0] = U[1 + d];
  for (int a = 0; a < 3; ++a) F[1 + a] = U[1 + a] * un;
  F[1 + d] += p;
  F[4] = un * (U[4] + p);
}

/* Primitive (rho, u, v, w, p) to conserved (rho, rho u, rho v, rho w, E),
 * E = p / (gamma - 1) + rho |u|^2 / 2.  Planar arrays of ncell cells. */
void oracle_prim_to_cons(int64_t ncell, const double* W, double* U) {
  for (int64_t q = 0; q < ncell; ++q) {
    double rho = W[q];
    double u = W[ncell + q], v = W[2 * ncell + q], w = W[3 * ncell + q];
    double p = W[4 * ncell + q];
    U[q] = rho;
    U[ncell + q] = rho * u;
    U[2 * ncell + q] = rho * v;
    U[3 * ncell + q] = rho * w;
    U[4 * ncell + q] = p / (GAMMA - 1.0) + 0.5 * rho * (u * u + v * v + w * w);
  }
}

/* Conserved to primitive, planar. */
void oracle_cons_to_prim(int64_t ncell, const double* U, double* W) {
  for (int64_t q = 0; q < ncell; ++q) {
    double s[NV];
    for (int c = 0; c < NV; ++c) s[c] = U[c * ncell + q];
    W[q] = s[0];
    W[ncell + q] = s[1] / s[0];
    W[2 * ncell + q] = s[2] / s[0];
    W[3 * ncell + q] = s[3] / s[0];
    W[4 * ncell + q] = pressure_of(s);
  }
}

/* ------------------------------------------------------------------ */
/* Slope limiter.                                                      */
/* ------------------------------------------------------------------ */

/* minmod(a, b): the smaller-magnitude argument when both have the same
 * strict sign, otherwise zero.  Sign tests, not a*b, so tiny slopes do not
 * underflow to a spurious zero. */
double oracle_minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a < b ? a : b;
  if (a < 0.0 && b < 0.0) return a > b ? a : b;
  return 0.0;
}

/* ------------------------------------------------------------------ */
/* HLLC approximate Riemann solver (Toro section 10.4).                */
/* ------------------------------------------------------------------ */

/* Star state U*_K (Toro eq. 10.39) for side K with wave speed S and contact
 * speed Ss, along axis d. */
static void hllc_star(const double U[NV], int d, double S, double Ss,
                      double Us[NV]) {
  double rho = U[0];
  double un = U[1 + d] / rho;
  double p = pressure_of(U);
  double factor = rho * (S - un) / (S - Ss);
  Us[0] = factor;
  for (int a = 0; a < 3; ++a) Us[1 + a] = factor * (U[1 + a] / rho);
  Us[1 + d] = factor * Ss;
  Us[4] = factor * (U[4] / rho + (Ss - un) * (Ss + p / (rho * (S - un))));
}

/* HLLC flux at a face along axis d with left state UL and right state UR.
 * Wave speeds: Davis, S_L = min(u_L - c_L, u_R - c_R),
 * S_R = max(u_L + c_L, u_R + c_R).  Contact speed: Toro eq. 10.37.
 * Flux selection (Toro eq. 10.26), ties resolved in the order
 * 0 <= S_L, 0 <= S*, 0 < S_R. */
void oracle_hllc(const double UL[NV], const double UR[NV], int d,
                 double F[NV]) {
  double rhoL = UL[0], rhoR = UR[0];
  double uL = UL[1 + d] / rhoL, uR = UR[1 + d] / rhoR;
  double pL = pressure_of(UL), pR = pressure_of(UR);
  double cL = sqrt(GAMMA * pL / rhoL), cR = sqrt(GAMMA * pR / rhoR);
  double SL = fmin(uL - cL, uR - cR);
  double SR = fmax(uL + cL, uR + cR);
  double Ss = (pR - pL + rhoL * uL * (SL - uL) - rhoR * uR * (SR - uR)) /
              (rhoL * (SL - uL) - rhoR * (SR - uR));
  double FL[NV], FR[NV], Us[NV];
  if (0.0 <= SL) {
    oracle_flux(UL, d, F);
  } else if (0.0 <= Ss) {
    oracle_flux(UL, d, FL);
    hllc_star(UL, d, SL, Ss, Us);
    for (int c = 0; c < NV; ++c) F[c] = FL[c] + SL * (Us[c] - UL[c]);
  } else if (0.0 < SR) {
    oracle_flux(UR, d, FR);
    hllc_star(UR, d, SR, Ss, Us);
    for (int c = 0; c < NV; ++c) F[c] = FR[c] + SR * (Us[c] - UR[c]);
  } else {
    oracle_flux(UR, d, F);
  }
}

/* ------------------------------------------------------------------ */
/* One MUSCL-Hancock update of a single pencil (Toro section 14.4).     */
/* ------------------------------------------------------------------ */

/* Number of doubles of scratch oracle_sweep_pencil needs for n cells. */
int64_t oracle_pencil_scratch(int n) { return (int64_t)(3 * (n + 4)) * NV; }

/* W: n+4 states, state-major (W[s*5 + c]), state s is cell s-2, so the two
 * ghost cells on each side are already filled.  lam = dt / dx along the
 * pencil's axis d.  out: n updated states, state-major.
 *
 * For cells i = -1 .. n (states s = 1 .. n+2):
 *   slope     D_i   = minmod(U_i - U_{i-1}, U_{i+1} - U_i)   per component
 *   extrap.   U^L_i = U_i - D_i / 2,   U^R_i = U_i + D_i / 2
 *   half step h_i   = (lam / 2) (F(U^L_i) - F(U^R_i))
 *             Ub^L_i = U^L_i + h_i,   Ub^R_i = U^R_i + h_i
 * For faces i+1/2, i = -1 .. n-1:
 *   F_{i+1/2} = HLLC(Ub^R_i, Ub^L_{i+1})
 * For cells i = 0 .. n-1:
 *   out_i = U_i - lam (F_{i+1/2} - F_{i-1/2})
 *
 * Returns 0, or the STAGE_* code of the first non-physical state met with
 * *bad_cell set to its cell index (-2 .. n+1). */
int oracle_sweep_pencil(int n, int d, double lam, const double* W,
                        double* out, double* scratch, int* bad_cell) {
  double* BL = scratch;                 /* Ub^L, n+4 slots */
  double* BR = scratch + (n + 4) * NV;  /* Ub^R, n+4 slots */
  double* FF = scratch + 2 * (n + 4) * NV; /* face flux; slot s = face s-2+1/2 */

  for (int s = 0; s < n + 4; ++s) {
    if (!is_physical(&W[s * NV])) { *bad_cell = s - 2; return STAGE_INPUT; }
  }
  for (int s = 1; s <= n + 2; ++s) {
    const double* Um = &W[(s - 1) * NV];
    const double* U0 = &W[s * NV];
    const double* Up = &W[(s + 1) * NV];
    double UL[NV], UR[NV], FLx[NV], FRx[NV];
    for (int c = 0; c < NV; ++c) {
      double slope = oracle_minmod(U0[c] - Um[c], Up[c] - U0[c]);
      UL[c] = U0[c] - 0.5 * slope;
      UR[c] = U0[c] + 0.5 * slope;
    }
    if (!is_physical(UL) || !is_physical(UR)) {
      *bad_cell = s - 2;
      return STAGE_EXTRAP;
    }
    oracle_flux(UL, d, FLx);
    oracle_flux(UR, d, FRx);
    for (int c = 0; c < NV; ++c) {
      double h = 0.5 * lam * (FLx[c] - FRx[c]);
      BL[s * NV + c] = UL[c] + h;
      BR[s * NV + c] = UR[c] + h;
    }
    if (!is_physical(&BL[s * NV]) || !is_physical(&BR[s * NV])) {
      *bad_cell = s - 2;
      return STAGE_EVOLVED;
    }
  }
  for (int s = 1; s <= n + 1; ++s)
    oracle_hllc(&BR[s * NV], &BL[(s + 1) * NV], d, &FF[s * NV]);
  for (int i = 0; i < n; ++i) {
    const double* U0 = &W[(i + 2) * NV];
    const double* Fm = &FF[(i + 1) * NV]; /* face i-1/2 */
    const double* Fp = &FF[(i + 2) * NV]; /* face i+1/2 */
    for (int c = 0; c < NV; ++c) out[i * NV + c] = U0[c] - lam * (Fp[c] - Fm[c]);
    if (!is_physical(&out[i * NV])) { *bad_cell = i; return STAGE_OUTPUT; }
  }
  return 0;
}

/* ------------------------------------------------------------------ */
/* Ghost cells (paper section "Tensors": padding by constant           */
/* extrapolation; periodic wrap).                                      */
/* ------------------------------------------------------------------ */

/* Source cell index for pencil position i in [-2, n+1] under boundary
 * condition bc (0 transmissive, 1 periodic). */
static int64_t ghost_source(int64_t i, int64_t n, int bc) {
  if (i >= 0 && i < n) return i;
  if (bc == 1) return ((i % n) + n) % n;
  return i < 0 ? 0 : n - 1;
}

/* ------------------------------------------------------------------ */
/* Max wave speed and time step (paper listing "Simplified Euler       */
/* solver graph creation": set_wavespeeds, max reduce, set_dt).        */
/* ------------------------------------------------------------------ */

/* S[d] = max over cells of |u_d| + c, c = sqrt(gamma p / rho).
 * Returns 0, or ORACLE_NONPHYSICAL with *bad set to a linear cell index
 * (the smallest one) when a cell is non-physical. */
int oracle_max_wavespeed(const int n[3], const double* U, double S[3],
                         int64_t* bad) {
  int64_t ncell = (int64_t)n[0] * n[1] * n[2];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int64_t first_bad = -1;
#pragma omp parallel for reduction(max : s0, s1, s2) schedule(static)
  for (int64_t q = 0; q < ncell; ++q) {
    double st[NV];
    for (int c = 0; c < NV; ++c) st[c] = U[c * ncell + q];
    if (!is_physical(st)) {
#pragma omp critical(oracle_bad)
      if (first_bad < 0 || q < first_bad) first_bad = q;
      continue;
    }
    double rho = st[0];
    double c = sqrt(GAMMA * pressure_of(st) / rho);
    double a0 = fabs(st[1] / rho) + c;
    double a1 = fabs(st[2] / rho) + c;
    double a2 = fabs(st[3] / rho) + c;
    if (a0 > s0) s0 = a0;
    if (a1 > s1) s1 = a1;
    if (a2 > s2) s2 = a2;
  }
  S[0] = s0;
  S[1] = s1;
  S[2] = s2;
  if (first_bad >= 0) {
    if (bad) *bad = first_bad;
    return ORACLE_NONPHYSICAL;
  }
  return ORACLE_OK;
}

/* dt = cfl * min_d (dx_d / S_d). */
double oracle_dt(const double S[3], const double dx[3], double cfl) {
  double r = dx[0] / S[0];
  for (int d = 1; d < 3; ++d) {
    double q = dx[d] / S[d];
    if (q < r) r = q;
  }
  return cfl * r;
}

/* ------------------------------------------------------------------ */
/* One sweep of the whole grid along axis d: A -> B.                   */
/* ------------------------------------------------------------------ */

/* info (6 int64): [stage, axis, i, j, k, unused] of the first failure. */
static int sweep_grid(const int n[3], const int bc[3], int d, double lam,
                      const double* A, double* B, int64_t info[6]) {
  const int64_t nx = n[0], ny = n[1], nz = n[2];
  const int64_t ncell = nx * ny * nz;
  const int64_t stride[3] = {1, nx, nx * ny};
  const int64_t len = n[d];
  /* transverse axes, in increasing order */
  const int ta = d == 0 ? 1 : 0;
  const int tb = d == 2 ? 1 : 2;
  const int64_t na = n[ta], nb = n[tb];
  const int64_t npencil = na * nb;
  int failed = 0;
  int64_t fail_q = -1, fail_stage = 0, fail_pos = 0;
  int alloc_failed = 0;

#pragma omp parallel
  {
    double* W = (double*)malloc(sizeof(double) * (size_t)(len + 4) * NV);
    double* O = (double*)malloc(sizeof(double) * (size_t)len * NV);
    double* scr = (double*)malloc(sizeof(double) * (size_t)oracle_pencil_scratch((int)len));
    if (!W || !O || !scr) {
#pragma omp atomic write
      alloc_failed = 1;
    }
#pragma omp for schedule(static)
    for (int64_t pidx = 0; pidx < npencil; ++pidx) {
      if (!W || !O || !scr) continue;
      int64_t a = pidx % na, b = pidx / na;
      int64_t base = a * stride[ta] + b * stride[tb];
      for (int64_t s = 0; s < len + 4; ++s) {
        int64_t src = ghost_source(s - 2, len, bc[d]);
        int64_t q = base + src * stride[d];
        for (int c = 0; c < NV; ++c) W[s * NV + c] = A[c * ncell + q];
      }
      int bad = 0;
      int st = oracle_sweep_pencil((int)len, d, lam, W, O, scr, &bad);
      if (st != 0) {
        int64_t cell = bad < 0 ? 0 : (bad >= len ? len - 1 : bad);
        int64_t q = base + cell * stride[d];
#pragma omp critical(oracle_fail)
        {
          if (!failed || q < fail_q) {
            failed = 1;
            fail_q = q;
            fail_stage = st;
            fail_pos = bad;
          }
        }
        continue;
      }
      for (int64_t i = 0; i < len; ++i) {
        int64_t q = base + i * stride[d];
        for (int c = 0; c < NV; ++c) B[c * ncell + q] = O[i * NV + c];
      }
    }
    free(W);
    free(O);
    free(scr);
  }
  if (alloc_failed) return ORACLE_NOMEM;
  if (failed) {
    info[0] = fail_stage;
    info[1] = d;
    info[2] = fail_q % nx;
    info[3] = (fail_q / nx) % ny;
    info[4] = fail_q / (nx * ny);
    info[5] = fail_pos;
    return ORACLE_NONPHYSICAL;
  }
  return ORACLE_OK;
}

/* One sweep along axis d with a given dt, in place (U <- sweep(U)).
 * Exposed for per-sweep comparisons. */
int oracle_sweep(const int n[3], const double dx[3], const int bc[3], int d,
                 double dt, double* U, int64_t info[6]) {
  if (d < 0 || d > 2) return ORACLE_BAD_ARGS;
  int64_t ncell = (int64_t)n[0] * n[1] * n[2];
  double* B = (double*)malloc(sizeof(double) * (size_t)ncell * NV);
  if (!B) return ORACLE_NOMEM;
  int st = sweep_grid(n, bc, d, dt / dx[d], U, B, info);
  if (st == ORACLE_OK) memcpy(U, B, sizeof(double) * (size_t)ncell * NV);
  free(B);
  return st;
}

/* ------------------------------------------------------------------ */
/* Time stepping.                                                      */
/* ------------------------------------------------------------------ */

/* Advance U (planar, in place) by up to nsteps steps.
 *   order: sweep axes in order (normally {0, 1, 2}: x, then y, then z).
 *   cfl:   Courant number for dt; dt_fixed > 0 overrides the CFL time step.
 *   t_end: if > 0, the last step is shortened so that t reaches t_end, and
 *          stepping stops there.
 * Outputs: *t_out (time reached), dts[s] (dt of step s, if dts != NULL),
 * *steps_done, info[6] describes a failure (info[0] = stage, info[1] = axis,
 * info[2..4] = i, j, k).  Returns an ORACLE_* status. */
int oracle_run(const int n[3], const double dx[3], const int bc[3],
               const int order[3], double cfl, double dt_fixed, int nsteps,
               double t_end, double* U, double* t_out, double* dts,
               int* steps_done, int64_t info[6]) {
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 1 || !(dx[d] > 0.0) || (bc[d] != 0 && bc[d] != 1) ||
        order[d] < 0 || order[d] > 2)
      return ORACLE_BAD_ARGS;
  }
  if (order[0] == order[1] || order[0] == order[2] || order[1] == order[2])
    return ORACLE_BAD_ARGS;
  int64_t ncell = (int64_t)n[0] * n[1] * n[2];
  double* B = (double*)malloc(sizeof(double) * (size_t)ncell * NV);
  if (!B) return ORACLE_NOMEM;
  double t = 0.0;
  int s = 0, st = ORACLE_OK;
  for (int e = 0; e < 6; ++e) info[e] = -1;
  double* cur = U;
  double* nxt = B;
  for (s = 0; s < nsteps; ++s) {
    if (t_end > 0.0 && !(t < t_end)) break;
    double dt = dt_fixed;
    if (!(dt_fixed > 0.0)) {
      double S[3];
      int64_t bad = -1;
      st = oracle_max_wavespeed(n, cur, S, &bad);
      if (st != ORACLE_OK) {
        info[0] = STAGE_DT;
        info[1] = -1;
        info[2] = bad % n[0];
        info[3] = (bad / n[0]) % n[1];
        info[4] = bad / ((int64_t)n[0] * n[1]);
        break;
      }
      dt = oracle_dt(S, dx, cfl);
    }
    if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
    for (int o = 0; o < 3 && st == ORACLE_OK; ++o) {
      int d = order[o];
      st = sweep_grid(n, bc, d, dt / dx[d], cur, nxt, info);
      double* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    if (st != ORACLE_OK) break;
    if (dts) dts[s] = dt;
    t += dt;
  }
  /* three sweeps per step swap the buffers an odd number of times */
  if (cur != U) memcpy(U, cur, sizeof(double) * (size_t)ncell * NV);
  free(B);
  if (t_out) *t_out = t;
  if (steps_done) *steps_done = s;
  return st;
}
