// Radiation transport and matter-radiation coupling kernels (gfx950, wave64).
//
// One radiation RK substep (Section 2.2.2) is two launches of rad_stage_kernel:
//   STAGE 1: Ur1 = Ur + dt L(Ur)
//   STAGE 2: Ur <- 0.5 Ur + 0.5 (Ur1 + dt L(Ur1)), then, fused, the per-cell
//            coupling of Section 2.2.3 (Newton exchange, flux source, momentum,
//            work) on the cell just written.
// L is PPM of (E_r, f = F/(c E_r)) along x, y, z, the M1 (or Eddington)
// closure and an HLL flux per face (first-order fallback where a reconstructed
// |f| exceeds 1; optical-depth factor on the dissipation), unsplit divergence.
// Same z-march as the hydro stage: own column in registers, current plane
// with a 3-cell halo in LDS, every face reconstructed and solved once.
#pragma once
#include "hydro_kernels.hpp"

namespace qk {

struct RadParamsDev {
  double c, chat, a_r, kappa_P, kappa_R, gamma, alpha_cv, newton_tol;
  double c_over_chat, chat_over_c, inv_c_chat;  // c / chat, chat / c, 1 / (chat c): formed once on the host
  int newton_max_iter, closure, tau_correction, eos, recon;
  const void* src;  // NULL or per-cell radiation source rate j (state precision)
};

template <class S, class R>
struct RadStageArgs {
  const S* Uin;   // radiation stage input (4 vars)
  const S* Ugh;   // ghost source of the stage input (all-fixed boxes) or NULL
  const S* Un;    // stage 2: radiation U^n at own cell
  S* Uout;        // stage 1: Ur1; stage 2: Ur (in place)
  S* Ug;          // gas state: density read at faces; stage 2 updates m, E
  DevBox b;
  RadParamsDev p;
  const double* dt_ptr;    // hydro dt on the device (or NULL: dt_val)
  const int32_t* nsub_ptr; // substep count on the device (or NULL: nsub_val)
  double dt_val;
  int nsub_val;
  int sub;                 // index of this substep; the launch does nothing if sub >= N
  int zc, gx, gy;
  uint32_t* err;
  uint32_t* iter_max;
  double* reg;             // rad_region_flux_kernel: flux register over the faces
  int rlo[3], rhi[3];      //   bounding [rlo, rhi) (the stage kernel ignores these)
  double rw;               //   register weight: each face adds rw * dt_sub/2 * F
  // Causality rule of the optical-depth correction (used when tau_correction
  // is on): one byte per interior cell, index i + n0 (j + n1 k).
  uint8_t* vfl;            // set to 1 by this stage at cells that violate |F| <= c E_r
  uint8_t* vfl_clear;      // flags of the other stage, cleared by this stage's fix-up
  int per;                 // bit d set: axis d is periodic (a face there joins both ends)
  int img;                 // -1, or: every face periodic or outflow, every extent >= 4, and
                           // the stage input's ghost cells not kept: a cell outside the box
                           // is read at the cell the fill would copy (ghost_image with this
                           // face code; the stage kernel then runs as its IMG instance)
  const uint32_t* nthick;  // number of thick cells of the step (NULL: not counted).  When it is
                           // 0 no face has tau > 1, the factor is 1 everywhere, and the stage
                           // skips the density halo and the optical depths altogether
};

// A cell of a thick-cell list: box index (0 for a single box) and cell.
struct CellRef {
  int box, i, j, k;
};

__device__ __forceinline__ int64_t interior_index(const DevBox& b, int i, int j, int k) {
  return (int64_t)i + (int64_t)b.n0 * ((int64_t)j + (int64_t)b.n1 * k);
}

// Optical depth of a face (Section 2.2.2; the formula is a reading: tau = dx
// kappa_R (rho_L + rho_R)/2) exceeds 1, so the correction scales its flux.
// The stage kernel, the fix-up and the thick-cell list all decide with this
// one expression.
template <class R>
__device__ __forceinline__ R face_tau(R dxd, R kappa, R rhol, R rhor) {
  return dxd * kappa * (R(0.5) * (rhol + rhor));
}

// HLL flux of (E, F) along axis d between face states (E, f), f.f = ffL, ffR
// (Section 2.2.2).  The wave speed chat max(sqrt(T_dd^L), sqrt(T_dd^R)) is
// formed as chat sqrt(max(T_dd^L, T_dd^R)) (sqrt is monotone and correctly
// rounded: the same value).
template <class R>
__device__ __forceinline__ void rad_flux(R EL, R fLx, R fLy, R fLz, R ffL, R ER, R fRx, R fRy, R fRz, R ffR, int d,
                                         int closure, R c, R chat, R ratio, R cc, R eps, R* out) {
  R TLx, TLy, TLz, dL, TRx, TRy, TRz, dR, kL, kR;
  const R f2L = rmin(ffL, R(1)), f2R = rmin(ffR, R(1));
  closure_k2<R>(f2L, f2R, closure, kL, kR);
  eddington_row<R>(fLx, fLy, fLz, ffL, f2L, kL, d, TLx, TLy, TLz, dL);
  eddington_row<R>(fRx, fRy, fRz, ffR, f2R, kR, d, TRx, TRy, TRz, dR);
  const R S = chat * sqrt_nn(rmax(dL, dR));  // T_dd = 0 for a beam across the axis
  const R cEL = c * EL, cER = c * ER;
  const R FLx = cEL * fLx, FLy = cEL * fLy, FLz = cEL * fLz;
  const R FRx = cER * fRx, FRy = cER * fRy, FRz = cER * fRz;
  const R FLd = d == 0 ? FLx : (d == 1 ? FLy : FLz);
  const R FRd = d == 0 ? FRx : (d == 1 ? FRy : FRz);
  const R h = R(0.5) * eps * S;
  if constexpr (kRadFma<R>) {  // the left/right sums stay unfused (symmetric)
    out[0] = fma(-h, ER - EL, R(0.5) * (ratio * FLd + ratio * FRd));
    out[1] = fma(-h, FRx - FLx, R(0.5) * (cc * (EL * TLx) + cc * (ER * TRx)));
    out[2] = fma(-h, FRy - FLy, R(0.5) * (cc * (EL * TLy) + cc * (ER * TRy)));
    out[3] = fma(-h, FRz - FLz, R(0.5) * (cc * (EL * TLz) + cc * (ER * TRz)));
  } else {
    out[0] = R(0.5) * (ratio * FLd + ratio * FRd) - h * (ER - EL);
    out[1] = R(0.5) * (cc * (EL * TLx) + cc * (ER * TRx)) - h * (FRx - FLx);
    out[2] = R(0.5) * (cc * (EL * TLy) + cc * (ER * TRy)) - h * (FRy - FLy);
    out[3] = R(0.5) * (cc * (EL * TLz) + cc * (ER * TRz)) - h * (FRz - FLz);
  }
}

// Face between cell "l" (reconstructed right state aL*) and cell "r": choose
// the reconstructed states or, if either |f| exceeds 1, both cell averages,
// then the optical-depth factor (on every optically thick face, fallback
// faces included), then the flux.  cells(cl, cr) fetches the
// two cell averages; the fallback is rare, so whole waves skip the fetch.
template <class R, class Cells>
__device__ __forceinline__ void rad_face(const R* sl, const R* sr, const Cells& cells, R rhol, R rhor, R dxd,
                                         int d, const RadParamsDev& p, R c, R chat, R ratio, R cc, R* out,
                                         bool tau_off = false) {
  R ffl = (sl[1] * sl[1] + sl[2] * sl[2]) + sl[3] * sl[3];  // f.f of each side
  R ffr = (sr[1] * sr[1] + sr[2] * sr[2]) + sr[3] * sr[3];
  const bool fb = f_above_one(ffl) || f_above_one(ffr);
  R L[4], Rr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    L[v] = sl[v];
    Rr[v] = sr[v];
  }
  if (fb) {
    cells(L, Rr);
    ffl = (L[1] * L[1] + L[2] * L[2]) + L[3] * L[3];
    ffr = (Rr[1] * Rr[1] + Rr[2] * Rr[2]) + Rr[3] * Rr[3];
  }
  R eps = R(1);
  if (p.tau_correction) {
    // min(1, 1/tau) is 1 unless tau > 1: waves with no optically thick face
    // skip the division (a wave-uniform branch).  tau_off: the face touches a
    // cell where the causality rule switched the correction off.
    const R tau = face_tau<R>(dxd, R(p.kappa_R), rhol, rhor);
    const bool thick = !tau_off && tau > R(1);
    if (__ballot(thick)) eps = thick ? rcp_nz(tau) : R(1);
  }
  rad_flux<R>(L[0], L[1], L[2], L[3], ffl, Rr[0], Rr[1], Rr[2], Rr[3], ffr, d, p.closure, c, chat, ratio, cc, eps, out);
}

// Matter-radiation coupling of one cell (Section 2.2.3), FP64 throughout.
// gas = (rho, mx, my, mz, E), rad = (E_r, Fx, Fy, Fz); S is the optional
// radiation source added over dt; returns iterations used, sets *fail when the
// iteration cap is reached.  Quotients by the same denominator (rho, the
// Jacobian entry dF_G/dE_g, the flux factor) are taken once as a reciprocal.
__device__ __forceinline__ int exchange(const RadParamsDev& p, double dt, double S, double* gas, double* rad,
                                        bool& fail) {
  const double rho = gas[0];
  const double c = p.c, ch = p.chat;
  const double coc = p.c_over_chat;
  const double inv_rho = rcp_nz(rho);
  const double Ek0 = 0.5 * ((gas[1] * gas[1] + gas[2] * gas[2]) + gas[3] * gas[3]) * inv_rho;
  const double Eg0 = gas[4] - Ek0;
  const double Er0 = rad[0];
  const double Etot = Eg0 + coc * (Er0 + S);
  const double inv_Etot = rcp_nz(Etot);
  const double k1 = dt * rho * p.kappa_P * ch;         // dR/d(a_r T^4 - E_r)
  const double dFG_dEr = -c * dt * rho * p.kappa_P;
  const double dFR_dEr = 1.0 + ch * dt * rho * p.kappa_P;
  const double gm1 = p.gamma - 1.0;
  const double Tfac = gm1 * inv_rho;                   // T = E_g (gamma-1)/rho
  double Eg = Eg0, Er = Er0;
  int it = 0;
  bool conv = false;
  for (; it < p.newton_max_iter; ++it) {
    double T4, dRdEg;
    if (p.eos == 1) {
      T4 = 4.0 * Eg / p.alpha_cv;
      dRdEg = k1 * (4.0 * p.a_r / p.alpha_cv);  // C_v = alpha T^3 cancels T^3
    } else {
      const double T = Eg * Tfac;
      const double T2 = T * T;
      T4 = T2 * T2;
      dRdEg = k1 * (4.0 * p.a_r * T2 * T) * Tfac;  // 4 a_r T^3 / C_v, C_v = rho/(gamma-1)
    }
    const double R = k1 * (p.a_r * T4 - Er);
    const double FG = (Eg - Eg0) + coc * R;
    const double FR = (Er - Er0) - (R + S);
    if (fabs(FG * inv_Etot) < p.newton_tol && fabs(coc * FR * inv_Etot) < p.newton_tol) {
      conv = true;
      break;
    }
    const double dFG_dEg = 1.0 + coc * dRdEg;
    const double dFR_dEg = -dRdEg;
    const double inv_g = rcp_nz(dFG_dEg);
    const double eta = -dFR_dEg * inv_g;
    const double dEr = div_nz(-(FR + eta * FG), dFR_dEr + eta * dFG_dEr);
    const double dEg = -(FG + dEr * dFG_dEr) * inv_g;
    Eg += dEg;
    Er += dEr;
  }
  fail = fail || !conv;
  const double inv_fac = rcp_nz(1.0 + rho * p.kappa_R * ch * dt);
  const double inv_cc = p.inv_c_chat;
  double m[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double F0 = rad[1 + d];
    const double F1 = F0 * inv_fac;
    m[d] = gas[1 + d] - (F1 - F0) * inv_cc;
    rad[1 + d] = F1;
  }
  const double Ek1 = 0.5 * ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]) * inv_rho;
  const double dEk = Ek1 - Ek0;
  gas[1] = m[0];
  gas[2] = m[1];
  gas[3] = m[2];
  gas[4] = Eg + (Ek0 + dEk);
  rad[0] = Er - p.chat_over_c * dEk;
  return it;
}

template <int NT>
__device__ __forceinline__ void block_umax_to(uint32_t x, uint32_t* dst) {
  __shared__ uint32_t red[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = red[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) m = max(m, red[k]);
    atomicMax(dst, m);
  }
}

// LDS of one radiation tile (SPLIT as for the hydro stage).
template <class R, int TX, int TY, bool SPLIT>
struct RadSmem {
  static constexpr int NXR = (TX + 2) * TY, NYR = TX * (TY + 2);
  static constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1);
  static constexpr int XS = SPLIT ? NXR : (NXR > NYR ? NXR : NYR);
  static constexpr int XFS = SPLIT ? NXF : (NXF > NYF ? NXF : NYF);
  static constexpr int YS = SPLIT ? NYR : XS, YFS = SPLIT ? NYF : XFS;
  R Qp[4][TY + 6][TX + 6];
  R rhoP[TY + 2][TX + 2];
  R xL[4][XS], xR[4][XS];
  R xF[4][XFS];
  R yL[4][SPLIT ? NYR : 1], yR[4][SPLIT ? NYR : 1];
  R yF[4][SPLIT ? NYF : 1];
};

// One tile of columns of one box for substep `a.sub` (the caller has checked
// that the substep is active).  Returns the largest exchange iteration count.
// NT threads (NT >= TX*TY); thread t owns column (t % TX, t / TX).
template <class S, class R, int TX, int TY, int NT, bool SPLIT, int STAGE, bool IMG = false>
__device__ __forceinline__ uint32_t rad_tile(const RadStageArgs<S, R>& a, int tbx, int tby, int tbz, int N,
                                             RadSmem<R, TX, TY, SPLIT>& sm, bool& bad_out, bool& nfail_out) {
  using SM = RadSmem<R, TX, TY, SPLIT>;
  constexpr int NXR = SM::NXR, NYR = SM::NYR, NXF = SM::NXF, NYF = SM::NYF;
  constexpr int XS = SM::XS, YS = SM::YS, XFS = SM::XFS, YFS = SM::YFS;
  constexpr int NHX = 6 * TY, NHY = 6 * TX, NCX = 2 * TY, NCY = 2 * TX;
  constexpr int NH = NHX + NHY + NCX + NCY, HPT = (NH + NT - 1) / NT;
  static_assert(NT >= TX * TY, "one thread per column");
  R* const xL = &sm.xL[0][0];
  R* const xR = &sm.xR[0][0];
  R* const xF = &sm.xF[0][0];
  R* const yL = SPLIT ? &sm.yL[0][0] : xL;
  R* const yR = SPLIT ? &sm.yR[0][0] : xR;
  R* const yF = SPLIT ? &sm.yF[0][0] : xF;
  auto& Qp = sm.Qp;
  auto& rhoP = sm.rhoP;

  const DevBox& b = a.b;
  RadParamsDev p = a.p;
  if (p.tau_correction && a.nthick && *a.nthick == 0u) p.tau_correction = 0;  // no thick face: eps = 1
  const int t = threadIdx.x, tx = t % TX, ty = t / TX;
  const int x0 = tbx * TX, y0 = tby * TY;
  const int tw = min(TX, b.n0 - x0), th = min(TY, b.n1 - y0);
  const int z0 = tbz * a.zc;
  const int z1 = min(z0 + a.zc, b.n2);
  const bool act = tx < tw && ty < th;
  const int i = x0 + tx, j = y0 + ty;
  const int64_t vs = b.vs, pz = b.pz;
  const double dt = (a.dt_ptr ? *a.dt_ptr : a.dt_val) / N;  // substep dt
  const R c = R(p.c), chat = R(p.chat), ratio = R(p.chat / p.c), cc = R(p.c * p.chat);
  const bool tauc = p.tau_correction != 0;
  const S* __restrict__ Uin = a.Uin;
  const S* __restrict__ Ug = a.Ug;
  bool bad = false, nfail = false;
  uint32_t itmax = 0;

  // halo ring of every plane: 3 cells of (E, F) beyond each x and y edge of
  // the tile, 1 cell of gas density (optical-depth factor only)
  HaloCell<S> hc[HPT];
#pragma unroll
  for (int m = 0; m < HPT; ++m) {
    const int it = t + m * NT;
    int xx = 0, yy = 0, kind = 0;
    if (it < NHX) {
      const int c6 = it % 6;
      yy = it / 6;
      xx = c6 < 3 ? c6 - 3 : tw + c6 - 3;
      kind = yy < th ? 1 : 0;
    } else if (it < NHX + NHY) {
      const int r = it - NHX, c6 = r / TX;
      xx = r % TX;
      yy = c6 < 3 ? c6 - 3 : th + c6 - 3;
      kind = xx < tw ? 1 : 0;
    } else if (it < NHX + NHY + NCX) {
      const int r = it - NHX - NHY;
      yy = r >> 1;
      xx = (r & 1) ? tw : -1;
      kind = (tauc && yy < th) ? 2 : 0;
    } else if (it < NH) {
      const int r = it - NHX - NHY - NCX;
      xx = r % TX;
      yy = (r / TX) ? th : -1;
      kind = (tauc && xx < tw) ? 2 : 0;
    }
    hc[m].kind = kind;
    hc[m].src = src_at(Uin, a.Ugh, b, x0 + xx, y0 + yy, z0);
    // IMG: the radiation ring at its ghost images; the density ring (kind 2)
    // where it lies (the gas ghosts are filled)
    hc[m].off = (IMG && kind == 1)
                    ? cell(b, ghost_image(x0 + xx, b.n0, a.img & 3), ghost_image(y0 + yy, b.n1, (a.img >> 2) & 3), 0)
                    : cell(b, x0 + xx, y0 + yy, 0);
    hc[m].lds = kind == 2 ? (yy + 1) * (TX + 2) + (xx + 1) : (yy + 3) * (TX + 6) + (xx + 3);
  }

  R w[4][5];  // own column (E, fx, fy, fz): [var][slot], slot s = plane m-2+s
  R aRz[4], Fz[4];
  R rz_km1 = R(0), rz_k = R(0), rz_k1 = R(0);  // density of own column at k-1, k, k+1 (tau correction)
  double cq[4];                 // own column, plane k+3 (prefetched)
  double hq[HPT][4];            // halo ring of plane k (prefetched)
  double uo[4], un0[4], gas[5];
  double srate = 0.0;  // radiation source rate of own cell (stage 2)

  // (E, F) -> (E, f = F / (c E))
  auto to_q = [&](const double* u, R* Q, bool& flag) {
    const double E = u[0];
    const R Er = R(E);
    const R inv = rcp_nz(c * Er);  // E_r > 0
    Q[0] = Er;
    Q[1] = R(u[1]) * inv;
    Q[2] = R(u[2]) * inv;
    Q[3] = R(u[3]) * inv;
    flag = flag || !(E > 0.0);
  };
  auto load4 = [&](const S* U, int64_t o, double* q) {
#pragma unroll
    for (int v = 0; v < 4; ++v) q[v] = double(U[o + v * vs]);
  };
  auto zimg = [&](int kk) { return IMG ? ghost_image(kk, b.n2, (a.img >> 4) & 3) : kk; };
  auto load_w = [&](int kk, int slot) {
    double q[4];
    load4(src_at(Uin, a.Ugh, b, i, j, kk), cell(b, i, j, zimg(kk)), q);
    R Q[4];
    to_q(q, Q, bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) w[v][slot] = Q[v];
  };
  auto shift_w = [&]() {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int s = 0; s < 4; ++s) w[v][s] = w[v][s + 1];
    }
  };
  // PPM keeps the unlimited upper interface value (fzr) for the next plane,
  // whose lower interface it is (CARRY: the window has moved by one plane).
  R fzr[4];
  auto recon_z = [&](R* L, R* Rr, auto carry) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (p.recon == 1) {
        plm<R>(w[v][1], w[v][2], w[v][3], L[v], Rr[v]);
      } else {
        const R fl =
            decltype(carry)::value ? fzr[v] : ppm_iface<R, kRadFma<R>>(w[v][0], w[v][1], w[v][2], w[v][3]);
        fzr[v] = ppm_iface<R, kRadFma<R>>(w[v][1], w[v][2], w[v][3], w[v][4]);
        ppm_limit<R, kRadFma<R>>(w[v][1], w[v][2], w[v][3], fl, fzr[v], L[v], Rr[v]);
      }
    }
  };
  auto rho_at = [&](int kk) { return R(Ug[cell(b, i, j, kk)]); };

  // z prologue: flux through the bottom face of the chunk
  if (act) {
    R cprev[4];
#pragma unroll
    for (int s = 0; s < 5; ++s) load_w(z0 - 3 + s, s);
    R l[4], rprev[4];
    recon_z(l, rprev, std::false_type{});
#pragma unroll
    for (int v = 0; v < 4; ++v) cprev[v] = w[v][2];  // cell z0-1
    shift_w();
    load_w(z0 + 2, 4);
    R rcur[4], ccur[4];
    recon_z(l, rcur, std::true_type{});
#pragma unroll
    for (int v = 0; v < 4; ++v) ccur[v] = w[v][2];  // cell z0
    R rl = R(0), rr = R(0);
    if (tauc) {
      rl = rho_at(z0 - 1);
      rr = rho_at(z0);
    }
    rad_face<R>(
        rprev, l,
        [&](R* cl, R* cr) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            cl[v] = cprev[v];
            cr[v] = ccur[v];
          }
        },
        rl, rr, R(b.dx2), 2, p, c, chat, ratio, cc, Fz);
#pragma unroll
    for (int v = 0; v < 4; ++v) aRz[v] = rcur[v];
    rz_k = rl;
    rz_k1 = rr;
    load4(src_at(Uin, a.Ugh, b, i, j, z0 + 3), cell(b, i, j, zimg(z0 + 3)), cq);
  }
#pragma unroll
  for (int m = 0; m < HPT; ++m) load_halo<4>(hc[m], hc[m].src, Ug, (int64_t)z0 * pz, vs, hq[m]);
  bad = false;

  for (int k = z0; k < z1; ++k) {
    R rhn = R(0);
    if (act) {
      shift_w();
      R Q[4];
      to_q(cq, Q, bad);  // planes k-1..k+3, plane k in slot 1
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        w[v][4] = Q[v];
        Qp[v][ty + 3][tx + 3] = w[v][1];
      }
      if (tauc) {
        rz_km1 = rz_k;
        rz_k = rz_k1;
        rhoP[ty + 1][tx + 1] = rz_k;
      }
    }
#pragma unroll
    for (int m = 0; m < HPT; ++m) {
      if (hc[m].kind == 1) {
        R Q[4];
        bool dummy = false;
        to_q(hq[m], Q, dummy);
#pragma unroll
        for (int v = 0; v < 4; ++v) (&Qp[v][0][0])[hc[m].lds] = Q[v];
      } else if (hc[m].kind == 2) {
        (&rhoP[0][0])[hc[m].lds] = R(hq[m][0]);
      }
    }
    // loads for the rest of this plane and the next one, in flight during the sweeps
    if (act) {
      const int64_t o = cell(b, i, j, k);
      if (tauc) rhn = R(Ug[o + pz]);
      load4(Uin, o, uo);
      if (STAGE == 2) {
        load4(a.Un, o, un0);
#pragma unroll
        for (int v = 0; v < 5; ++v) gas[v] = double(Ug[o + v * vs]);
        srate = p.src ? double(((const S*)p.src)[o]) : 0.0;
      }
      if (k + 1 < z1) load4(src_at(Uin, a.Ugh, b, i, j, k + 4), cell(b, i, j, zimg(k + 4)), cq);
    }
    if (k + 1 < z1) {
#pragma unroll
      for (int m = 0; m < HPT; ++m) load_halo<4>(hc[m], hc[m].src, Ug, (int64_t)(k + 1) * pz, vs, hq[m]);
    }
    __syncthreads();
    // Does an x or y face of the own cell have tau > 1?  (Read here: the
    // density plane is rewritten for the next plane before its first barrier.)
    bool thick_xy = false;
    if (tauc && act) {
      const R kap = R(p.kappa_R), dx0 = R(b.dx0), dx1 = R(b.dx1);
      thick_xy = face_tau<R>(dx0, kap, rhoP[ty + 1][tx], rz_k) > R(1) ||
                 face_tau<R>(dx0, kap, rz_k, rhoP[ty + 1][tx + 2]) > R(1) ||
                 face_tau<R>(dx1, kap, rhoP[ty][tx + 1], rz_k) > R(1) ||
                 face_tau<R>(dx1, kap, rz_k, rhoP[ty + 2][tx + 1]) > R(1);
    }

    auto x_recon = [&]() {
      for (int it = t; it < NXR; it += NT) {
        const int xx = it % (TX + 2) - 1, yy = it / (TX + 2);
        if (xx <= tw && yy < th) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const R* row = &Qp[v][yy + 3][xx + 1];
            recon5<R, kRadFma<R>>(row[0], row[1], row[2], row[3], row[4], p.recon, xL[v * XS + it], xR[v * XS + it]);
          }
        }
      }
    };
    auto x_faces = [&]() {
      for (int it = t; it < NXF; it += NT) {
        const int fx = it % (TX + 1), yy = it / (TX + 1);
        if (fx <= tw && yy < th) {
          const int il = yy * (TX + 2) + fx, ir = il + 1;
          R sl[4], sr[4], F[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            sl[v] = xR[v * XS + il];
            sr[v] = xL[v * XS + ir];
          }
          const R rl = tauc ? rhoP[yy + 1][fx] : R(0), rr = tauc ? rhoP[yy + 1][fx + 1] : R(0);
          rad_face<R>(
              sl, sr,
              [&](R* cl, R* cr) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  cl[v] = Qp[v][yy + 3][fx + 2];
                  cr[v] = Qp[v][yy + 3][fx + 3];
                }
              },
              rl, rr, R(b.dx0), 0, p, c, chat, ratio, cc, F);
#pragma unroll
          for (int v = 0; v < 4; ++v) xF[v * XFS + it] = F[v];
        }
      }
    };
    auto y_recon = [&]() {
      for (int it = t; it < NYR; it += NT) {
        const int xx = it % TX, yy = it / TX - 1;
        if (xx < tw && yy <= th) {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            recon5<R, kRadFma<R>>(Qp[v][yy + 1][xx + 3], Qp[v][yy + 2][xx + 3], Qp[v][yy + 3][xx + 3], Qp[v][yy + 4][xx + 3],
                      Qp[v][yy + 5][xx + 3], p.recon, yL[v * YS + it], yR[v * YS + it]);
        }
      }
    };
    auto y_faces = [&]() {
      for (int it = t; it < NYF; it += NT) {
        const int xx = it % TX, fy = it / TX;
        if (xx < tw && fy <= th) {
          const int il = fy * TX + xx, ir = il + TX;
          R sl[4], sr[4], F[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            sl[v] = yR[v * YS + il];
            sr[v] = yL[v * YS + ir];
          }
          const R rl = tauc ? rhoP[fy][xx + 1] : R(0), rr = tauc ? rhoP[fy + 1][xx + 1] : R(0);
          rad_face<R>(
              sl, sr,
              [&](R* cl, R* cr) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                  cl[v] = Qp[v][fy + 2][xx + 3];
                  cr[v] = Qp[v][fy + 3][xx + 3];
                }
              },
              rl, rr, R(b.dx1), 1, p, c, chat, ratio, cc, F);
#pragma unroll
          for (int v = 0; v < 4; ++v) yF[v * YFS + it] = F[v];
        }
      }
    };

    R dfx[4], dfy[4];
    if constexpr (SPLIT) {
      x_recon();
      y_recon();
      __syncthreads();
      x_faces();
      y_faces();
      __syncthreads();
      if (act) {
        const int fxi = ty * (TX + 1) + tx, fyi = ty * TX + tx;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          dfx[v] = xF[v * XFS + fxi + 1] - xF[v * XFS + fxi];
          dfy[v] = yF[v * YFS + fyi + TX] - yF[v * YFS + fyi];
        }
      }
    } else {
      x_recon();
      __syncthreads();
      x_faces();
      __syncthreads();
      if (act) {
        const int fxi = ty * (TX + 1) + tx;
#pragma unroll
        for (int v = 0; v < 4; ++v) dfx[v] = xF[v * XFS + fxi + 1] - xF[v * XFS + fxi];
      }
      y_recon();
      __syncthreads();
      y_faces();
      __syncthreads();
      if (act) {
        const int fyi = ty * TX + tx;
#pragma unroll
        for (int v = 0; v < 4; ++v) dfy[v] = yF[v * YFS + fyi + TX] - yF[v * YFS + fyi];
      }
    }

    if (act) {
      if (tauc) rz_k1 = rhn;
      // ---- z sweep: cell k+1 centred in the window
      R aLn[4], aRn[4], Fk[4];
      recon_z(aLn, aRn, std::true_type{});
      rad_face<R>(
          aRz, aLn,
          [&](R* cl, R* cr) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              cl[v] = w[v][1];
              cr[v] = w[v][2];
            }
          },
          rz_k, rz_k1, R(b.dx2), 2, p, c, chat, ratio, cc, Fk);
      const int64_t o = cell(b, i, j, k);
      double un[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double tX = double(dfx[v]) * b.inv_dx0;
        const double tY = double(dfy[v]) * b.inv_dx1;
        const double tZ = double(Fk[v] - Fz[v]) * b.inv_dx2;
        const double L = -((tX + tY) + tZ);
        un[v] = (STAGE == 1) ? uo[v] + dt * L : 0.5 * un0[v] + 0.5 * (uo[v] + dt * L);
        Fz[v] = Fk[v];
        aRz[v] = aRn[v];
      }
      // Causality rule (Section 2.2.2): a cell with an optically thick face
      // (a "thick cell") whose corrected update gives |F| > c E_r is flagged;
      // the fix-up pass redoes the thick cells next to flagged ones with the
      // correction off at the flagged cells' faces.  Stage 2 leaves thick
      // cells (update and coupling) entirely to that pass, and stage 1 leaves
      // it their positivity check.
      bool thick = false;
      if (tauc) {
        const R kap = R(p.kappa_R), dx2 = R(b.dx2);
        thick = thick_xy || face_tau<R>(dx2, kap, rz_km1, rz_k) > R(1) || face_tau<R>(dx2, kap, rz_k, rz_k1) > R(1);
        if (thick && sqrt((un[1] * un[1] + un[2] * un[2]) + un[3] * un[3]) > p.c * un[0])
          a.vfl[interior_index(b, i, j, k)] = 1;
      }
      if (STAGE == 1 || !thick) {
        if (STAGE == 2) {
          const int it = exchange(p, dt, dt * srate, gas, un, nfail);
          itmax = max(itmax, (uint32_t)it);
#pragma unroll
          for (int v = 1; v < 5; ++v) a.Ug[o + v * vs] = S(gas[v]);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) a.Uout[o + v * vs] = S(un[v]);
        if (!thick) bad = bad || !(un[0] > 0.0);
      }
    }
  }
  bad_out = bad_out || bad;
  nfail_out = nfail_out || nfail;
  return itmax;
}

template <class S, class R, int STAGE, bool IMG = false>
__global__ __launch_bounds__(SNT, sizeof(S) == 4 ? (STAGE == 1 ? 4 : 3) : 2) void rad_stage_kernel(RadStageArgs<S, R> a) {
  const int N = a.nsub_ptr ? *a.nsub_ptr : a.nsub_val;
  if (a.sub >= N) return;  // block-uniform: the whole grid skips unused substeps
  __shared__ RadSmem<R, STX, STY, true> sm;
  const TileId tl = tile_of_block(a.gx, a.gy);
  bool bad = false, nfail = false;
  const uint32_t itmax = rad_tile<S, R, STX, STY, SNT, true, STAGE, IMG>(a, tl.bx, tl.by, tl.bz, N, sm, bad, nfail);
  if (bad) atomicOr(a.err, ERR_NEG);
  if (nfail) atomicOr(a.err, ERR_NEWTON);
  if (STAGE == 2) block_umax_to<SNT>(itmax, a.iter_max);
}


// Flux of the radiation stage input through the face between cells
// (i, j, k) - e_d and (i, j, k), computed with the stage kernel's own device
// functions on the same operands (the same bits as the stage kernel's face).
// tau_off: the optical-depth correction is off at this face.
template <class S, class R>
__device__ __forceinline__ void rad_flux_at(const RadStageArgs<S, R>& a, int d, int i, int j, int k, bool tau_off,
                                            R* F) {
  const DevBox& b = a.b;
  const RadParamsDev& p = a.p;
  const R c = R(p.c), chat = R(p.chat), ratio = R(p.chat / p.c), cc = R(p.c * p.chat);
  const int ei = d == 0, ej = d == 1, ek = d == 2;
  R Q[6][4];  // (E, f = F / (c E)) of cells f-3 .. f+2 along d
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int ii = i + ei * (s - 3), jj = j + ej * (s - 3), kk = k + ek * (s - 3);
    const S* src = src_at(a.Uin, a.Ugh, b, ii, jj, kk);
    const int64_t o = a.img >= 0 ? cell(b, ghost_image(ii, b.n0, a.img & 3), ghost_image(jj, b.n1, (a.img >> 2) & 3),
                                        ghost_image(kk, b.n2, (a.img >> 4) & 3))
                                 : cell(b, ii, jj, kk);
    const R Er = R(double(src[o]));
    const R inv = rcp_nz(c * Er);  // E_r > 0
    Q[s][0] = Er;
#pragma unroll
    for (int v = 1; v < 4; ++v) Q[s][v] = R(double(src[o + v * b.vs])) * inv;
  }
  R sl[4], sr[4], tmp[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    recon5<R, kRadFma<R>>(Q[0][v], Q[1][v], Q[2][v], Q[3][v], Q[4][v], p.recon, tmp[v], sl[v]);  // cell f-1, right
    recon5<R, kRadFma<R>>(Q[1][v], Q[2][v], Q[3][v], Q[4][v], Q[5][v], p.recon, sr[v], tmp[v]);  // cell f, left
  }
  R rl = R(0), rr = R(0);
  if (p.tau_correction) {
    rl = R(a.Ug[cell(b, i - ei, j - ej, k - ek)]);
    rr = R(a.Ug[cell(b, i, j, k)]);
  }
  rad_face<R>(
      sl, sr,
      [&](R* cl, R* cr) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          cl[v] = Q[2][v];
          cr[v] = Q[3][v];
        }
      },
      rl, rr, R(d == 0 ? b.dx0 : (d == 1 ? b.dx1 : b.dx2)), d, p, c, chat, ratio, cc, F, tau_off);
}

// Causality flag of cell (i, j, k) set by the stage: across a periodic axis a
// cell outside the box is its image; any other cell outside never violates.
template <class S, class R>
__device__ __forceinline__ bool vflag_at(const RadStageArgs<S, R>& a, int i, int j, int k) {
  const DevBox& b = a.b;
  if ((unsigned)i >= (unsigned)b.n0) {
    if (!(a.per & 1)) return false;
    i = ((i % b.n0) + b.n0) % b.n0;
  }
  if ((unsigned)j >= (unsigned)b.n1) {
    if (!(a.per & 2)) return false;
    j = ((j % b.n1) + b.n1) % b.n1;
  }
  if ((unsigned)k >= (unsigned)b.n2) {
    if (!(a.per & 4)) return false;
    k = ((k % b.n2) + b.n2) % b.n2;
  }
  return a.vfl[interior_index(b, i, j, k)] != 0;
}

// Is any face of cell (i, j, k) optically thick (tau > 1)?  The density of
// the gas state, ghosts included, decides; it does not change during a
// radiation step, so neither does the answer.
template <class S, class R>
__device__ __forceinline__ bool cell_is_thick(const DevBox& b, const S* Ug, R kap, int i, int j, int k) {
  const R rc = R(Ug[cell(b, i, j, k)]);
  bool th = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ei = d == 0, ej = d == 1, ek = d == 2;
    const R dxd = R(d == 0 ? b.dx0 : (d == 1 ? b.dx1 : b.dx2));
    const R rlo = R(Ug[cell(b, i - ei, j - ej, k - ek)]), rhi = R(Ug[cell(b, i + ei, j + ej, k + ek)]);
    th = th || face_tau<R>(dxd, kap, rlo, rc) > R(1) || face_tau<R>(dxd, kap, rc, rhi) > R(1);
  }
  return th;
}

// Fix-up of one thick cell after a radiation stage (the causality rule of
// Section 2.2.2).  A face is uncorrected when either of its cells was flagged
// by the stage; the cell's update is formed again from the stage input with
// those faces (a face is one flux for both of its cells, so the update stays
// conservative).  STAGE 1: only where a thick face of the cell switched; the
// positivity check of the final value either way.  STAGE 2: always (the
// stage kernel left the cell), followed by the coupling of Section 2.2.3.
// Returns the exchange iterations used.
template <class S, class R, int STAGE>
__device__ __forceinline__ uint32_t rad_fix_cell(const RadStageArgs<S, R>& a, int i, int j, int k, int N, bool& bad,
                                                 bool& nfail) {
  const DevBox& b = a.b;
  const RadParamsDev& p = a.p;
  const int64_t vs = b.vs, o = cell(b, i, j, k);
  const R kap = R(p.kappa_R), rc = R(a.Ug[o]);
  const bool vc = vflag_at(a, i, j, k);
  bool sw[3][2];
  bool any = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ei = d == 0, ej = d == 1, ek = d == 2;
    const R dxd = R(d == 0 ? b.dx0 : (d == 1 ? b.dx1 : b.dx2));
    const R rlo = R(a.Ug[cell(b, i - ei, j - ej, k - ek)]), rhi = R(a.Ug[cell(b, i + ei, j + ej, k + ek)]);
    sw[d][0] = vc || vflag_at(a, i - ei, j - ej, k - ek);
    sw[d][1] = vc || vflag_at(a, i + ei, j + ej, k + ek);
    any = any || (sw[d][0] && face_tau<R>(dxd, kap, rlo, rc) > R(1)) ||
          (sw[d][1] && face_tau<R>(dxd, kap, rc, rhi) > R(1));
  }
  if (STAGE == 1 && !any) {
    bad = bad || !(double(a.Uout[o]) > 0.0);
    return 0;
  }
  R Flo[3][4], Fhi[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rad_flux_at<S, R>(a, d, i, j, k, sw[d][0], Flo[d]);
    rad_flux_at<S, R>(a, d, i + (d == 0), j + (d == 1), k + (d == 2), sw[d][1], Fhi[d]);
  }
  const double dt = (a.dt_ptr ? *a.dt_ptr : a.dt_val) / N;
  double un[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double uo = double(a.Uin[o + v * vs]);
    const double tX = double(Fhi[0][v] - Flo[0][v]) * b.inv_dx0;
    const double tY = double(Fhi[1][v] - Flo[1][v]) * b.inv_dx1;
    const double tZ = double(Fhi[2][v] - Flo[2][v]) * b.inv_dx2;
    const double L = -((tX + tY) + tZ);
    un[v] = (STAGE == 1) ? uo + dt * L : 0.5 * double(a.Un[o + v * vs]) + 0.5 * (uo + dt * L);
  }
  uint32_t it = 0;
  if (STAGE == 2) {
    double gas[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) gas[v] = double(a.Ug[o + v * vs]);
    const double srate = p.src ? double(((const S*)p.src)[o]) : 0.0;
    it = (uint32_t)exchange(p, dt, dt * srate, gas, un, nfail);
#pragma unroll
    for (int v = 1; v < 5; ++v) a.Ug[o + v * vs] = S(gas[v]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) a.Uout[o + v * vs] = S(un[v]);
  bad = bad || !(un[0] > 0.0);
  return it;
}

// Append every thick cell of one box to `list` (wave-aggregated atomics).
template <class S, class R>
__device__ __forceinline__ void thick_list_box(const DevBox& b, const S* Ug, double kappa, int box, int64_t t0,
                                               int64_t stride, CellRef* list, uint32_t* count) {
  const int64_t n = (int64_t)b.n0 * b.n1 * b.n2;
  const int lane = threadIdx.x & 63;
  for (int64_t base = t0 - lane; base < n; base += stride) {  // whole waves iterate together
    const int64_t t = base + lane;
    bool th = false;
    int i = 0, j = 0, k = 0;
    if (t < n) {  // n < 2^31 (checked on the host): 32-bit index arithmetic
      const uint32_t u = (uint32_t)t, q = u / (uint32_t)b.n0, kq = q / (uint32_t)b.n1;
      i = (int)(u - q * (uint32_t)b.n0);
      j = (int)(q - kq * (uint32_t)b.n1);
      k = (int)kq;
      th = cell_is_thick<S, R>(b, Ug, R(kappa), i, j, k);
    }
    const unsigned long long m = __ballot(th);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      uint32_t q = 0;
      if (lane == leader) q = atomicAdd(count, (uint32_t)__popcll(m));
      q = (uint32_t)__shfl((int)q, leader, 64);
      if (th) list[q + __popcll(m & ((1ull << lane) - 1ull))] = CellRef{box, i, j, k};
    }
  }
}

template <class S, class R>
__global__ __launch_bounds__(256) void thick_list_kernel(const S* Ug, DevBox b, double kappa, CellRef* list,
                                                         uint32_t* count) {
  thick_list_box<S, R>(b, Ug, kappa, 0, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256, list,
                       count);
}

__global__ void zero_u32_kernel(uint32_t* x) { *x = 0u; }

// Fix-up pass of one radiation stage over the thick cells of a box; also
// clears the other stage's flags at those cells.  Guarded by the device
// substep count like the stage.
template <class S, class R, int STAGE>
__global__ __launch_bounds__(256) void rad_fix_kernel(RadStageArgs<S, R> a, const CellRef* __restrict__ list,
                                                      const uint32_t* count) {
  const int N = a.nsub_ptr ? *a.nsub_ptr : a.nsub_val;
  if (a.sub >= N) return;
  const uint32_t n = *count;
  bool bad = false, nfail = false;
  uint32_t itmax = 0;
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < n; t += gridDim.x * 256u) {
    const CellRef c = list[t];
    itmax = max(itmax, rad_fix_cell<S, R, STAGE>(a, c.i, c.j, c.k, N, bad, nfail));
    a.vfl_clear[interior_index(a.b, c.i, c.j, c.k)] = 0;
  }
  if (bad) atomicOr(a.err, ERR_NEG);
  if (nfail) atomicOr(a.err, ERR_NEWTON);
  if (STAGE == 2) block_umax_to<256>(itmax, a.iter_max);
}

// Flux register of one radiation stage: the fluxes at the faces bounding
// region [rlo, rhi), recomputed from the stage input (and the gas density
// for the optical-depth factor) with the stage kernel's own device functions
// on the same operands, so every face carries the bits the stage used (with
// the causality rule's choice, from the stage's flags); each adds
// rw * dt_sub/2 * F to its slot.  One thread per face; guarded by the device
// substep count like the stage.  Launched after the stage, which leaves its
// input and the density as they were.
template <class S, class R>
__global__ __launch_bounds__(256) void rad_region_flux_kernel(RadStageArgs<S, R> a) {
  const int N = a.nsub_ptr ? *a.nsub_ptr : a.nsub_val;
  if (a.sub >= N) return;
  const int lo[3] = {a.rlo[0], a.rlo[1], a.rlo[2]}, hi[3] = {a.rhi[0], a.rhi[1], a.rhi[2]};
  const int64_t total = region_face_count(lo, hi);
  const double dt = (a.dt_ptr ? *a.dt_ptr : a.dt_val) / N;
  const double w = 0.5 * dt * a.rw;
  const bool rule = a.p.tau_correction != 0 && a.vfl;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const RegionFace rf = region_face(lo, hi, t);
    const int d = rf.d;
    // cell f along d (the face lies between cells f-1 and f)
    const int ei = d == 0, ej = d == 1, ek = d == 2;
    const int i = d == 0 ? (rf.side ? hi[0] : lo[0]) : lo[0] + rf.b;
    const int j = d == 1 ? (rf.side ? hi[1] : lo[1]) : (d == 0 ? lo[1] + rf.b : lo[1] + rf.a);
    const int k = d == 2 ? (rf.side ? hi[2] : lo[2]) : lo[2] + rf.a;
    const bool off = rule && (vflag_at(a, i - ei, j - ej, k - ek) || vflag_at(a, i, j, k));
    R F[4];
    rad_flux_at<S, R>(a, d, i, j, k, off, F);
#pragma unroll
    for (int v = 0; v < 4; ++v) a.reg[reg_slot(lo, hi, d, v, rf.side, rf.a, rf.b, 4)] += w * double(F[v]);
  }
}

// Ghost fill guarded by the device substep count (skipped for unused substeps).
template <class S>
__global__ __launch_bounds__(256) void ghost_kernel_guarded(S* __restrict__ U, DevBox b, GhostBC bc, int nvar,
                                                            const int32_t* nsub_ptr, int nsub_val, int sub) {
  const int N = nsub_ptr ? *nsub_ptr : nsub_val;
  if (sub >= N) return;
  ghost_body<S>(U, b, bc, nvar);
}

}  // namespace qk
