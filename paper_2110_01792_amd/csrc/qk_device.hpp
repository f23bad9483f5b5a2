// Device building blocks of the per-cell update (gfx950).
//
// Method: Wibking & Krumholz (2021), arXiv:2110.01792, Section 2.2.
// R is the reconstruction/flux arithmetic type (double on the FP64 path,
// float on the mixed path); anything marked "double" stays FP64 on both.
#pragma once
#include <limits>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qk {

enum : uint32_t { ERR_NEG = 1u, ERR_NEWTON = 2u };

// Geometry of one ghosted box as seen by the kernels (element strides).
struct DevBox {
  int n0, n1, n2, ng;
  int64_t py, pz, vs;
  double inv_dx0, inv_dx1, inv_dx2;
  double dx0, dx1, dx2, dxmin;
};

__device__ __forceinline__ int64_t cell(const DevBox& b, int i, int j, int k) {
  return (int64_t)(k + b.ng) * b.pz + (int64_t)(j + b.ng) * b.py + (i + b.ng);
}

// The cell whose value a ghost at index i holds after the ghost fill, on an
// axis of n >= 4 cells whose faces are periodic or outflow, for i within 4
// cells of the axis (the reach of the stages' halos).  code bit 0: the low
// face is outflow (else periodic); bit 1: the high face.
__device__ __forceinline__ int ghost_image(int i, int n, int code) {
  return i < 0 ? ((code & 1) ? 0 : i + n) : (i >= n ? ((code & 2) ? n - 1 : i - n) : i);
}

template <class R> __device__ __forceinline__ R rmin(R a, R b) { return fmin(a, b); }
template <class R> __device__ __forceinline__ R rmax(R a, R b) { return fmax(a, b); }
// min(max(x, lo), hi) for lo <= hi; in FP32 one median-of-three instruction
// (the same value for finite operands).
template <class R>
__device__ __forceinline__ R rclamp(R x, R lo, R hi) {
  if constexpr (sizeof(R) == 4)
    return __builtin_amdgcn_fmed3f(x, lo, hi);
  else
    return rmin(rmax(x, lo), hi);
}

// ---------------------------------------------------------------------------
// Reciprocal, quotient and square root by Newton's iteration from the
// hardware estimates (v_rcp, v_rsq), for operands the update keeps in the
// normal range (densities, pressures, sound speeds, wave-speed gaps,
// radiation energies): no range scaling and no special-value handling, on
// which the IEEE expansions spend about half their instructions.
//   rcp_nz(b): steps r <- r + r (1 - b r) (two in FP64 from a 2^-24
//     estimate, one in FP32 from a 1-ulp estimate); b finite, nonzero, |b|
//     and 1/|b| normal.  b = 0 gives NaN (IEEE: inf).
//   div_nz(a, b): q = a r, then one residual correction q + r (a - b q).
//   sqrt_pos(x): Goldschmidt's coupled iteration for s ~ sqrt(x) and
//     h ~ 1/(2 sqrt(x)) from g = rsq(x), then residual corrections
//     s + h (x - s s); x > 0 normal.  x = 0 gives NaN (sqrt_nn handles it).
// Each result is the correctly rounded one or within one unit in the last
// place of it.
// ---------------------------------------------------------------------------
template <class R>
__device__ __forceinline__ R rcp_nz(R b) {
  if constexpr (sizeof(R) == 8) {
    R r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, R(1)), r, r);
    return fma(fma(-b, r, R(1)), r, r);
  } else {
    const R r = __builtin_amdgcn_rcpf(b);
    return fma(fma(-b, r, R(1)), r, r);
  }
}
template <class R>
__device__ __forceinline__ R div_nz(R a, R b) {
  const R r = rcp_nz(b), q = a * r;
  return fma(fma(-b, q, a), r, q);
}
template <class R>
__device__ __forceinline__ R sqrt_pos(R x) {
  if constexpr (sizeof(R) == 8) {
    const R g = __builtin_amdgcn_rsq(x);
    R s = x * g, h = R(0.5) * g;
    const R e = fma(-h, s, R(0.5));
    s = fma(s, e, s);
    h = fma(h, e, h);
    s = fma(fma(-s, s, x), h, s);
    return fma(fma(-s, s, x), h, s);
  } else {
    const R g = __builtin_amdgcn_rsqf(x);
    const R s = x * g, h = R(0.5) * g;
    return fma(fma(-s, s, x), h, s);
  }
}
// sqrt_pos extended to x = 0 (returns 0).
template <class R>
__device__ __forceinline__ R sqrt_nn(R x) {
  const R s = sqrt_pos(x);
  return x > R(0) ? s : R(0);
}

// ---------------------------------------------------------------------------
// PPM of one cell from the five cell averages centred on it (Section 2.2.1):
// symmetric fourth-order interface values, clamp to the neighbour range,
// CW84 extremum test with a monotonized-central linear fallback, CW84
// overshoot correction.  Written branch-free (selects) for SIMD execution.
// ---------------------------------------------------------------------------
// Half the monotonized-central slope, sign(dc) min(2|dr|, 2|dl|, |dc|/2) / 2
// (0 at an extremum of the averages), taken as min(|dr|, |dl|, |dc|/4) with
// the sign of dc: scaling by powers of two is exact, so the interface values
// q0 -+ h carry the same bits as q0 -+ slope/2.  Where dr dl > 0 neither h
// nor dc is zero, so copysign agrees with the sign test on dc.
template <class R>
__device__ __forceinline__ R mc_half_slope(R dl, R dr, R dc) {
  const R h = copysign(rmin(rmin(fabs(dr), fabs(dl)), R(0.25) * fabs(dc)), dc);
  return (dr * dl > R(0)) ? h : R(0);
}

// Fourth-order interface value between a and b from the averages a-1 = am,
// a, b, b+1 = bp.  A cell's right value and its right neighbour's left value
// are the same expression on the same operands, so a sweep may carry it.
// FMA selects the fused multiply-add forms (one rounding where the separate
// forms take two); the FP32 radiation reconstruction keeps the separate forms.
template <class R, bool FMA = true>
__device__ __forceinline__ R ppm_iface(R am, R a, R b, R bp) {
  if constexpr (FMA) return fma(R(7.0 / 12.0), a + b, R(-1.0 / 12.0) * (am + bp));
  return R(7.0 / 12.0) * (a + b) - R(1.0 / 12.0) * (am + bp);
}

// PPM limiting of one cell from its unlimited interface values fl, fr.
template <class R, bool FMA = true>
__device__ __forceinline__ void ppm_limit(R qm1, R q0, R qp1, R fl, R fr, R& aL, R& aR) {
  const R lo = rmin(qm1, rmin(q0, qp1));
  const R hi = rmax(qm1, rmax(q0, qp1));
  fl = rclamp(fl, lo, hi);
  fr = rclamp(fr, lo, hi);
  const R dl = q0 - qm1, dr = qp1 - q0, dc = qp1 - qm1;
  const R h = mc_half_slope(dl, dr, dc);
  const bool ext = (fr - q0) * (q0 - fl) <= R(0);
  const R del = fr - fl;
  const R a6 = FMA ? R(6) * fma(R(-0.5), fl + fr, q0) : R(6) * (q0 - R(0.5) * (fl + fr));
  const R da = del * a6, d2 = del * del;
  const bool ovl = da > d2;
  const bool ovr = !ovl && (da < -d2);
  const R q3 = R(3) * q0;
  const R fl2 = ovl ? (FMA ? fma(R(-2), fr, q3) : q3 - R(2) * fr) : fl;
  const R fr2 = ovr ? (FMA ? fma(R(-2), fl, q3) : q3 - R(2) * fl) : fr;
  aL = ext ? q0 - h : fl2;
  aR = ext ? q0 + h : fr2;
}

template <class R, bool FMA = true>
__device__ __forceinline__ void ppm(R qm2, R qm1, R q0, R qp1, R qp2, R& aL, R& aR) {
  ppm_limit<R, FMA>(qm1, q0, qp1, ppm_iface<R, FMA>(qm2, qm1, q0, qp1), ppm_iface<R, FMA>(qm1, q0, qp1, qp2), aL,
                    aR);
}

// PLM with the monotonized-central limiter (Section 2.2.1 alternative).
template <class R>
__device__ __forceinline__ void plm(R qm1, R q0, R qp1, R& aL, R& aR) {
  const R dl = q0 - qm1, dr = qp1 - q0, dc = qp1 - qm1;
  const R h = mc_half_slope(dl, dr, dc);
  aL = q0 - h;
  aR = q0 + h;
}

// Reconstruction selected at run time (uniform across the launch).
template <class R, bool FMA = true>
__device__ __forceinline__ void recon5(R qm2, R qm1, R q0, R qp1, R qp2, int recon, R& aL, R& aR) {
  if (recon == 1)
    plm<R>(qm1, q0, qp1, aL, aR);
  else
    ppm<R, FMA>(qm2, qm1, q0, qp1, qp2, aL, aR);
}

// Radiation reconstruction: fused forms in FP64 only (the FP32 radiation
// flux is a small difference of E_r terms; its measured error against the
// FP64 oracle grows with the fused forms).
template <class R>
constexpr bool kRadFma = sizeof(R) == 8;

// ---------------------------------------------------------------------------
// HLLC flux with PVRS wave speeds (Section 2.2.1; Toro ch. 10).  States are
// primitive (rho, u_normal, u_t1, u_t2, P).  Output flux in the same rotated
// order.  The two tangential speeds enter as one symmetric pair.
// ---------------------------------------------------------------------------
// Gas constants used per face, formed once per launch.
template <class R>
struct GasK {
  R g, inv_gm1, gq;  // gamma, 1/(gamma-1), (gamma+1)/(2 gamma)
};
template <class R>
__device__ __forceinline__ GasK<R> gas_k(double gamma) {
  GasK<R> k;
  k.g = R(gamma);
  k.inv_gm1 = R(1.0 / (gamma - 1.0));
  k.gq = R((gamma + 1.0) / (2.0 * gamma));
  return k;
}

template <class R>
__device__ __forceinline__ void hllc(const R* WL, const R* WR, const GasK<R>& k, R* F) {
  const R rL = WL[0], uL = WL[1], vL = WL[2], wL = WL[3], pL = WL[4];
  const R rR = WR[0], uR = WR[1], vR = WR[2], wR = WR[3], pR = WR[4];
  const R g = k.g;
  const R irL = rcp_nz(rL), irR = rcp_nz(rR);
  const R cL = sqrt_pos(g * pL * irL);
  const R cR = sqrt_pos(g * pR * irR);
  const R rbar = R(0.5) * (rL + rR);
  const R cbar = R(0.5) * (cL + cR);
  const R ps = rmax(R(0), fma(R(-0.5) * (uR - uL) * rbar, cbar, R(0.5) * (pL + pR)));
  // S_L = u_L - c_L q_L with q_L = 1 if p* <= p_L, else sqrt(1 + gq (p*/p_L - 1));
  // there c_L^2 q_L^2 = gamma (p_L + gq (p* - p_L)) / rho_L, so one square root
  // with the side's reciprocal density gives c_L q_L (likewise on the right).
  // Where the gas is at rest p* = p on both sides: whole waves skip the roots.
  R aL = cL, aR = cR;
  const bool shL = ps > pL, shR = ps > pR;
  if (__ballot(shL || shR)) {
    if (shL) aL = sqrt_pos(g * fma(k.gq, ps - pL, pL) * irL);
    if (shR) aR = sqrt_pos(g * fma(k.gq, ps - pR, pR) * irR);
  }
  const R SL = uL - aL;
  const R SR = uR + aR;
  const R Ss = div_nz(fma(-rR * uR, SR - uR, fma(rL * uL, SL - uL, pR - pL)), fma(rL, SL - uL, -rR * (SR - uR)));
  // Side and branch exactly as the four-way selection on (S_L, S*, S_R):
  // 0 <= S_L: left flux; else 0 <= S*: left star; else 0 < S_R: right star;
  // else right flux.  Only the chosen side's energy and fluxes are formed.
  const bool left = (R(0) <= SL) || (R(0) <= Ss);
  const bool star = !(R(0) <= SL) && ((R(0) <= Ss) || (R(0) < SR));
  const R r = left ? rL : rR, u = left ? uL : uR, v = left ? vL : vR, w = left ? wL : wR;
  const R p = left ? pL : pR, S = left ? SL : SR;
  const R E = fma(p, k.inv_gm1, R(0.5) * r * fma(u, u, v * v + w * w));
  const R f0 = r * u, f1 = fma(f0, u, p), f2 = f0 * v, f3 = f0 * w, f4 = u * (E + p);
  // U*_4 = ph (E + (S* - u)(r S* + p / (S - u))) with ph = (S - u) / (S - S*);
  // ph / (S - u) = 1 / (S - S*), so one reciprocal serves both quotients
  // (div_nz forms the same reciprocal; S - S* is nonzero wherever a star state
  // is chosen).  ph is a corrected quotient, so it is exactly 1 where S* = u,
  // as at a stationary contact.
  const R is = rcp_nz(S - Ss);
  const R ph = div_nz(S - u, S - Ss);
  const R Us0 = ph * r, Us1 = ph * (r * Ss), Us2 = ph * (r * v), Us3 = ph * (r * w);
  const R Us4 = fma(ph, fma(Ss - u, r * Ss, E), (Ss - u) * (p * is));
  F[0] = star ? fma(S, Us0 - r, f0) : f0;
  F[1] = star ? fma(S, Us1 - f0, f1) : f1;
  F[2] = star ? fma(S, Us2 - r * v, f2) : f2;
  F[3] = star ? fma(S, Us3 - r * w, f3) : f3;
  F[4] = star ? fma(S, Us4 - E, f4) : f4;
}

// Signal speed |v| + c_s of one cell from its conserved state, in double
// (Section 2.2.1, the CFL condition); sets bad where rho or P is not
// positive.  One reciprocal of rho serves |v| = |m| / rho, the kinetic energy
// and c_s^2 = gamma P / rho.  Every dt reduction uses this function.
__device__ __forceinline__ double signal_speed(const double* q, double gamma, double gm1, bool& bad) {
  const double rho = q[0];
  const double inv = rcp_nz(rho);
  const double m2 = (q[1] * q[1] + q[2] * q[2]) + q[3] * q[3];
  const double P = gm1 * (q[4] - 0.5 * m2 * inv);
  bad = bad || !(rho > 0.0) || !(P > 0.0);
  return sqrt_nn(m2) * inv + sqrt_pos(gamma * P * inv);
}

// Conserved -> primitive.  The internal energy E - |m|^2/(2 rho) is always
// formed in double (cancellation-prone); the rest in R.
template <class R>
__device__ __forceinline__ void cons_to_prim(double rho, double mx, double my, double mz, double E, double gm1,
                                             R* W, bool& bad) {
  const double inv = rcp_nz(rho);
  const double ek = 0.5 * ((mx * mx + my * my) + mz * mz) * inv;
  const double P = gm1 * (E - ek);
  const R ri = R(inv);
  W[0] = R(rho);
  W[1] = R(mx) * ri;
  W[2] = R(my) * ri;
  W[3] = R(mz) * ri;
  W[4] = R(P);
  bad = bad || !(rho > 0.0) || !(P > 0.0);
}

// Flattening coefficient of one cell along one axis before the neighbour
// minimum (Miller & Colella 2002 generalising CW84; CW84 constants).
// p* are pressures at offsets -2..+2, u* the axis velocity at -1, +1.
// The ratio and ramp (two divisions) are formed only where the shock test
// holds: away from shocks whole waves skip them.
template <class R>
__device__ __forceinline__ R chi_tilde(R pm2, R pm1, R pp1, R pp2, R um1, R up1) {
  const R dp1 = pp1 - pm1, dp2 = pp2 - pm2, du = up1 - um1;
  const bool shock = (fabs(dp1) > R(0.33) * rmin(pp1, pm1)) && (du < R(0));
  R t = R(1);
  if (shock) {
    const R z = fabs(dp1) / rmax(fabs(dp2), R(1e-300));
    t = rmin(R(1), rmax(R(0), R(1) - (z - R(0.75)) / (R(0.85) - R(0.75))));
  }
  return t;
}

// float cannot hold 1e-300; the floor only guards a 0/0 when both pressure
// differences vanish, which the shock test already excludes.
template <>
__device__ __forceinline__ float chi_tilde<float>(float pm2, float pm1, float pp1, float pp2, float um1, float up1) {
  const float dp1 = pp1 - pm1, dp2 = pp2 - pm2, du = up1 - um1;
  const bool shock = (fabsf(dp1) > 0.33f * fminf(pp1, pm1)) && (du < 0.0f);
  float t = 1.0f;
  if (shock) {
    const float z = fabsf(dp1) / fmaxf(fabsf(dp2), 1e-30f);
    t = fminf(1.0f, fmaxf(0.0f, 1.0f - (z - 0.75f) / (0.85f - 0.75f)));
  }
  return t;
}

// ---------------------------------------------------------------------------
// Radiation: M1 closure and HLL flux (Section 2.2.2, eq. M1_closure).
// A face state is (E, f) with f = F/(c E); F = c E f.
// ---------------------------------------------------------------------------
// Eddington tensor P/E = a I + b n n, a = (1 - chi)/2, b = (3 chi - 1)/2
// (Section 2.2.2), chi the Eddington factor of f = min(|f|, 1).  b vanishes
// like f^2; the kernels form k = b / f^2 from f2 = f^2:
//   0 Levermore, chi = (3 + 4 f^2) / (5 + 2 s) with s = sqrt(4 - 3 f^2):
//     b = (4 + 12 f^2 - 2 s) / (2 (5 + 2 s)), and 4 - 2 s = 12 f^2 / (4 + 2 s)
//     turns this into b = 3 f^2 / (2 + s), so k = 3 / (2 + s);
//   1 Eddington, chi = 1/3: k = 0;
//   2 Minerbo in the polynomial form chi = 1/3 + (2/15)(3 f^2 - f^3 + 3 f^4)
//     (Cernohorsky & Bludman 1994): k = (3 - f + 3 f^2) / 5.
// Then b = f2 k and a = (1 - b) / 3.  The two states of one face share one
// Levermore quotient, 3 / (2 + s_L) = 3 (2 + s_R) / ((2 + s_L)(2 + s_R))
// with each 2 + s in [3, 4]: one quotient per face where chi and b / |f|^2
// took two per state, and b has no cancellation near f = 0.  The closure
// enters the flux only through k.
template <class R>
__device__ __forceinline__ void closure_k2(R f2L, R f2R, int closure, R& kL, R& kR) {
  if (closure == 1) {
    kL = kR = R(0);
  } else if (closure == 2) {
    kL = ((R(3) - sqrt(f2L)) + R(3) * f2L) * R(0.2);
    kR = ((R(3) - sqrt(f2R)) + R(3) * f2R) * R(0.2);
  } else if constexpr (kRadFma<R>) {  // 4 - 3 f2 in [1, 4], (2 + s_L)(2 + s_R) in [9, 16]
    const R dl = R(2) + sqrt_pos(fma(R(-3), f2L, R(4))), dr = R(2) + sqrt_pos(fma(R(-3), f2R, R(4)));
    const R q = div_nz(R(3), dl * dr);
    kL = q * dr;
    kR = q * dl;
  } else {
    const R dl = R(2) + sqrt_pos(R(4) - R(3) * f2L), dr = R(2) + sqrt_pos(R(4) - R(3) * f2R);
    const R q = div_nz(R(3), dl * dr);
    kL = q * dr;
    kR = q * dl;
  }
}

// |f| > 1 decided on ff = f.f: sqrt is monotone and correctly rounded, and
// sqrt(ff) rounds to a value above 1 exactly when ff exceeds the next number
// above 1, so this is the same test without the square root.
template <class R>
__device__ __forceinline__ bool f_above_one(R ff) {
  return ff > R(1) + std::numeric_limits<R>::epsilon();
}

// Row `d` of the Eddington tensor P/E; Tdd = P_dd/E (the HLL speed is
// chat sqrt(Tdd)).  Cartesian components of f are fx, fy, fz, ff = f.f,
// f2 = min(ff, 1) and k from closure_k2.  b n_d n_i = b f_d f_i / ff =
// k (f2 / ff) f_d f_i, so neither |f| nor a quotient by ff is needed unless a
// fallback state still has |f| > 1 (then f2 / ff = 1 / ff; such waves take
// the branch).
template <class R>
__device__ __forceinline__ void eddington_row(R fx, R fy, R fz, R ff, R f2, R k, int d, R& Tx, R& Ty, R& Tz,
                                              R& Tdd) {
  const R a = (R(1) - f2 * k) * R(1.0 / 3.0);
  R g = k;
  const bool over = ff > R(1);
  if (__ballot(over)) g = over ? k / ff : k;
  const R fd = d == 0 ? fx : (d == 1 ? fy : fz);
  const R gd = g * fd;
  if constexpr (kRadFma<R>) {  // fma(x, y, 0) = x y: the off-diagonal entries are unchanged
    Tx = fma(gd, fx, d == 0 ? a : R(0));
    Ty = fma(gd, fy, d == 1 ? a : R(0));
    Tz = fma(gd, fz, d == 2 ? a : R(0));
  } else {
    Tx = gd * fx + (d == 0 ? a : R(0));
    Ty = gd * fy + (d == 1 ? a : R(0));
    Tz = gd * fz + (d == 2 ? a : R(0));
  }
  Tdd = d == 0 ? Tx : (d == 1 ? Ty : Tz);
}

}  // namespace qk
