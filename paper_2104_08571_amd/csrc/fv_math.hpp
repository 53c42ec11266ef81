// Per-cell and per-face arithmetic of the split MUSCL-Hancock / HLLC update,
// written for the gfx950 vector ALU.
//
// The update along axis D (Toro, "Riemann Solvers and Numerical Methods for
// Fluid Dynamics": MUSCL-Hancock section 14.4, HLLC section 10.4, Davis wave
// speeds eq. 10.48) for cell i is
//   slope      s_i   = minmod(U_i - U_{i-1}, U_{i+1} - U_i)      (conserved)
//   extrapol.  U^L_i = U_i - s_i/2,  U^R_i = U_i + s_i/2
//   half step  h_i   = (dt/dx)/2 (F(U^L_i) - F(U^R_i)),  Ub^{L,R}_i = U^{L,R}_i + h_i
//   face flux  F_{i+1/2} = HLLC(Ub^R_i, Ub^L_{i+1})
//   update     U'_i  = U_i - (dt/dx) (F_{i+1/2} - F_{i-1/2})
// Components are (rho, m_x, m_y, m_z, E); D selects the normal momentum.
//
// Precision notes.  FP32 uses the hardware reciprocal and square root
// (v_rcp_f32, v_sqrt_f32, 1 ulp) and v_med3_f32 for minmod; FP64 uses the
// hardware estimates refined by a third-order step (about an ulp) in the sweeps and
// IEEE division and square root for the wave speeds.  Each density is inverted once per state and
// velocities and kinetic energy are formed by multiplication.  The build
// disables implicit contraction; fused multiply-adds appear only where written
// (fma_ below), so every inlined copy of these functions -- in every layout,
// tiling, batched, fused or partitioned variant, prologue or loop body --
// performs the same operations on a cell and produces the same bits.
// Expressions follow the textbook formulas except where a rearrangement saves
// ALU work; each such place says so.
#pragma once

#include <hip/hip_runtime.h>

namespace rfv {

template <typename T> struct Arith;

template <> struct Arith<float> {
  static __device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float quot(float a, float b) {
    return a * __builtin_amdgcn_rcpf(b);
  }
  static __device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }
  // 1/a and 1/b: two hardware reciprocals
  static __device__ __forceinline__ void recip2(float a, float b, float& ra, float& rb) {
    ra = __builtin_amdgcn_rcpf(a);
    rb = __builtin_amdgcn_rcpf(b);
  }
  static __device__ __forceinline__ float min(float a, float b) { return __builtin_fminf(a, b); }
  static __device__ __forceinline__ float max(float a, float b) { return __builtin_fmaxf(a, b); }
  // minmod(a, b) is the median of (a, b, 0).
  static __device__ __forceinline__ float minmod(float a, float b) {
    return __builtin_amdgcn_fmed3f(a, b, 0.0f);
  }
};

// FP64 reciprocal and square root for the sweeps: the hardware estimates
// (v_rcp_f64, v_rsq_f64, relative error e of about 2^-24 or less) refined by
// one third-order step each, which leaves an error of order e^3 plus the
// final roundings (about an ulp) in 3 and 5 instructions, where IEEE
// division and square root expand to longer sequences.  With e = 1 - x r
// for the reciprocal estimate r, 1/x = r / (1 - e) = r (1 + e + e^2 + ...);
// with e = 1 - x y^2 for the inverse square root estimate y and s = x y,
// sqrt(x) = s / sqrt(1 - e) = s (1 + e/2 + 3 e^2/8 + ...).  Positive finite
// arguments only (the sweeps' densities, sound speeds and wave-speed
// differences); the time step uses IEEE operations.
template <> struct Arith<double> {
  static __device__ __forceinline__ double recip(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(__builtin_fma(e, e, e), r, r);
  }
  static __device__ __forceinline__ double quot(double a, double b) { return a * recip(b); }
  // 1/a and 1/b from one refined reciprocal of a b (a few ulp; positive a, b
  // whose product stays finite and normal: the sweeps' densities)
  static __device__ __forceinline__ void recip2(double a, double b, double& ra, double& rb) {
    const double r = recip(a * b);
    ra = b * r;
    rb = a * r;
  }
  static __device__ __forceinline__ double root(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double s = x * y;
    const double e = __builtin_fma(-s, y, 1.0);
    return __builtin_fma(s, e * __builtin_fma(e, 0.375, 0.5), s);
  }
  static __device__ __forceinline__ double min(double a, double b) { return __builtin_fmin(a, b); }
  static __device__ __forceinline__ double max(double a, double b) { return __builtin_fmax(a, b); }
  static __device__ __forceinline__ double minmod(double a, double b) {
    return __builtin_fmax(__builtin_fmin(a, b), __builtin_fmin(__builtin_fmax(a, b), 0.0));
  }
};

__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ T gamma_() { return T(1.4); }
template <typename T> __device__ __forceinline__ T gamma_m1() { return T(1.4) - T(1); }

// p = (gamma - 1) (E - |m|^2 / (2 rho)), given rinv = 1 / rho, evaluated as
// (gamma - 1) E - ((gamma - 1) / 2) |m|^2 rinv.
template <typename T>
__device__ __forceinline__ T pressure(const T u[5], T rinv) {
  const T m2 = fma_(u[3], u[3], fma_(u[2], u[2], u[1] * u[1]));
  return fma_(T(-0.5) * gamma_m1<T>() * m2, rinv, gamma_m1<T>() * u[4]);
}

// Physical flux along D given the normal velocity un and pressure p.
template <typename T, int D>
__device__ __forceinline__ void flux(const T u[5], T un, T p, T f[5]) {
  f[0] = u[1 + D];
  f[1] = u[1] * un;
  f[2] = u[2] * un;
  f[3] = u[3] * un;
  f[1 + D] = fma_(u[1 + D], un, p);
  f[4] = un * (u[4] + p);
}

// Slope, extrapolation and Hancock half step for one cell: from the cell
// state u0 and its backward / forward differences dm = U_i - U_{i-1},
// dp = U_{i+1} - U_i, produce the evolved boundary states bl = Ub^L_i and
// br = Ub^R_i.  hl = (dt/dx) / 2.
//
// The flux difference F(U^L) - F(U^R) is formed component by component
// rather than from the two flux vectors, with the same value up to rounding:
// the mass component is -s_n (U^L - U^R = -s), and each product difference
// a b - a' b' is one fused multiply-add on the negated second product.
template <typename T, int D>
__device__ __forceinline__ void hancock(const T u0[5], const T dm[5], const T dp[5], T hl,
                                        T bl[5], T br[5]) {
  T s[5], ul[5], ur[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    s[c] = Arith<T>::minmod(dm[c], dp[c]);
    ul[c] = fma_(T(-0.5), s[c], u0[c]);  // s/2 is exact: one rounding, as u0 - s/2
    ur[c] = fma_(T(0.5), s[c], u0[c]);
  }
  T rl, rr;
  Arith<T>::recip2(ul[0], ur[0], rl, rr);
  const T unl = ul[1 + D] * rl, unr = ur[1 + D] * rr;
  const T pl = pressure(ul, rl), pr = pressure(ur, rr);
  T d[5];
  d[0] = -s[1 + D];
#pragma unroll
  for (int c = 1; c < 4; ++c)
    if (c != 1 + D) d[c] = fma_(ul[c], unl, -(ur[c] * unr));
  d[1 + D] = fma_(ul[1 + D], unl, pl) - fma_(ur[1 + D], unr, pr);
  d[4] = fma_(unl, ul[4] + pl, -(unr * (ur[4] + pr)));
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    bl[c] = fma_(hl, d[c], ul[c]);
    br[c] = fma_(hl, d[c], ur[c]);
  }
}

// HLLC flux along D between left state ul and right state ur.  Davis wave
// speeds; contact speed S* (Toro eq. 10.37); star state (eq. 10.39); flux
// selection (eq. 10.26) with ties resolved as 0 <= S_L, 0 <= S*, 0 < S_R.
// Only the side the contact speed selects is evaluated.  Rearranged for the
// ALU, with the same value up to rounding:
//   rho u = m (the normal momentum) in S*'s numerator;
//   the side k's flux is F_k + S_c (U*_k - U_k) with S_c = min(S_L, 0)
//   (left) or max(S_R, 0) (right), whose correction vanishes exactly when
//   the flux is F_L or F_R;
//   with q = 1 / (S_k - S*) the star state is g U_k plus normal-momentum and
//   energy terms, g = (S_k - u_k) q, so U*_k - U_k is formed from
//   g - 1 = (S* - u_k) q directly (no cancellation where g is close to 1):
//     mass and tangential momenta    (g - 1) U_k
//     normal momentum                rho_k g S* - m_k
//     energy                         (g - 1) E_k + (S* - u_k) (rho_k g S* + p_k q)
//   (p_k / (rho_k (S_k - u_k)) times rho_k g is p_k q);
//   the tangential momentum and energy fluxes u_k m + S_c (g - 1) m and
//   u_k (E_k + p_k) + S_c (g - 1) E_k + ... share the factor
//   w = u_k + S_c (g - 1): m w and E_k w + u_k p_k + ....
template <typename T, int D>
__device__ __forceinline__ void hllc(const T ul[5], const T ur[5], T f[5]) {
  using A = Arith<T>;
  T rl, rr;
  A::recip2(ul[0], ur[0], rl, rr);
  const T mL = ul[1 + D], mR = ur[1 + D];
  const T uL = mL * rl;
  const T uR = mR * rr;
  const T pL = pressure(ul, rl);
  const T pR = pressure(ur, rr);
  const T cL = A::root(gamma_<T>() * pL * rl);
  const T cR = A::root(gamma_<T>() * pR * rr);
  const T SL = A::min(uL - cL, uR - cR);
  const T SR = A::max(uL + cL, uR + cR);
  const T aL = SL - uL, aR = SR - uR;
  const T num = fma_(-mR, aR, fma_(mL, aL, pR - pL));
  const T den = fma_(ul[0], aL, -(ur[0] * aR));
  const T Ss = A::quot(num, den);

  const bool left = (T(0) <= SL) || (T(0) <= Ss);
  T uk[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) uk[c] = left ? ul[c] : ur[c];
  const T unk = left ? uL : uR;
  const T pk = left ? pL : pR;
  const T Sk = left ? SL : SR;
  const T Sc = left ? A::min(SL, T(0)) : A::max(SR, T(0));

  const T q = A::recip(Sk - Ss);
  const T d = Ss - unk;                      // S* - u_k
  const T gm = d * q;                        // g - 1
  const T rs = fma_(uk[0], gm, uk[0]);       // rho*_k = rho_k g
  const T sg = Sc * gm;
  const T w = unk + sg;
  f[0] = fma_(sg, uk[0], uk[1 + D]);
#pragma unroll
  for (int c = 1; c < 4; ++c)
    if (c != 1 + D) f[c] = uk[c] * w;
  f[1 + D] = fma_(Sc, fma_(rs, Ss, -uk[1 + D]), fma_(uk[1 + D], unk, pk));
  f[4] = fma_(Sc * d, fma_(rs, Ss, pk * q), fma_(unk, pk, uk[4] * w));
}

// Conservative update U' = U - lam (F_{i+1/2} - F_{i-1/2}).
template <typename T>
__device__ __forceinline__ void update(const T u[5], T lam, const T fp[5], const T fm[5], T out[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) out[c] = fma_(-lam, fp[c] - fm[c], u[c]);
}

// Whole-wave lane shifts (DPP wave_shr:1 / wave_shl:1): lane l receives the
// value of lane l - 1 (from_below) or l + 1 (from_above).  The end lanes,
// which have no source lane, receive zero (bound_ctrl): such a move needs no
// copy of the old destination value first, and in FP32 the compiler can fold
// it into the instruction that consumes it.  A 64-bit value moves as its two
// 32-bit halves.  The end lanes only ever feed discarded results.
__device__ __forceinline__ float from_below(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_above(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, 0x130, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double shift64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  const uint32_t a = (uint32_t)__builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  const uint32_t b = (uint32_t)__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((uint64_t)b << 32) | a);
}
__device__ __forceinline__ double from_below(double v) { return shift64<0x138>(v); }
__device__ __forceinline__ double from_above(double v) { return shift64<0x130>(v); }

// |u_d| + c for d = x, y, z; `bad` when rho <= 0, p <= 0 or a value is not finite.
template <typename T>
__device__ __forceinline__ void wavespeeds(const T u[5], T s[3], bool& bad) {
  // FP64: IEEE division and square root, so the time step matches a
  // reference computed with them to the last bits
  const T r = sizeof(T) == 8 ? T(1) / u[0] : Arith<T>::recip(u[0]);
  const T p = pressure(u, r);
  const T c = sizeof(T) == 8 ? T(__builtin_sqrt(double(gamma_<T>() * p * r)))
                             : Arith<T>::root(gamma_<T>() * p * r);
  const T inf = T(__builtin_huge_val());
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = __builtin_fabs(u[1 + d] * r) + c;
  bad = !(u[0] > T(0)) || !(p > T(0)) || !(s[0] < inf) || !(s[1] < inf) || !(s[2] < inf);
}

}  // namespace rfv
