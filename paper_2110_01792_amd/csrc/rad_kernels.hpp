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
  int newton_max_iter, closure, tau_correction, eos, recon;
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
};

// HLL flux of (E, F) along axis d between face states (E, f) (Section 2.2.2).
template <class R>
__device__ __forceinline__ void rad_flux(R EL, R fLx, R fLy, R fLz, R ER, R fRx, R fRy, R fRz, int d, int closure,
                                         R c, R chat, R ratio, R cc, R eps, R* out) {
  R TLx, TLy, TLz, sL, TRx, TRy, TRz, sR;
  eddington_row<R>(fLx, fLy, fLz, d, closure, TLx, TLy, TLz, sL);
  eddington_row<R>(fRx, fRy, fRz, d, closure, TRx, TRy, TRz, sR);
  const R S = chat * rmax(sL, sR);
  const R cEL = c * EL, cER = c * ER;
  const R FLx = cEL * fLx, FLy = cEL * fLy, FLz = cEL * fLz;
  const R FRx = cER * fRx, FRy = cER * fRy, FRz = cER * fRz;
  const R FLd = d == 0 ? FLx : (d == 1 ? FLy : FLz);
  const R FRd = d == 0 ? FRx : (d == 1 ? FRy : FRz);
  const R h = R(0.5) * eps * S;
  out[0] = R(0.5) * (ratio * FLd + ratio * FRd) - h * (ER - EL);
  out[1] = R(0.5) * (cc * (EL * TLx) + cc * (ER * TRx)) - h * (FRx - FLx);
  out[2] = R(0.5) * (cc * (EL * TLy) + cc * (ER * TRy)) - h * (FRy - FLy);
  out[3] = R(0.5) * (cc * (EL * TLz) + cc * (ER * TRz)) - h * (FRz - FLz);
}

// Face between cell "l" (reconstructed right state aL*) and cell "r": choose
// the reconstructed states or, if either |f| exceeds 1, both cell averages,
// then the optical-depth factor, then the flux.
template <class R>
__device__ __forceinline__ void rad_face(const R* sl, const R* sr, const R* cl, const R* cr, R rhol, R rhor, R dxd,
                                         int d, const RadParamsDev& p, R c, R chat, R ratio, R cc, R* out) {
  const R nl = sqrt((sl[1] * sl[1] + sl[2] * sl[2]) + sl[3] * sl[3]);
  const R nr = sqrt((sr[1] * sr[1] + sr[2] * sr[2]) + sr[3] * sr[3]);
  const bool fb = (nl > R(1)) || (nr > R(1));
  R L[4], Rr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    L[v] = fb ? cl[v] : sl[v];
    Rr[v] = fb ? cr[v] : sr[v];
  }
  R eps = R(1);
  if (p.tau_correction) {
    const R tau = dxd * R(p.kappa_R) * (R(0.5) * (rhol + rhor));
    eps = fb ? R(1) : rmin(R(1), R(1) / tau);
  }
  rad_flux<R>(L[0], L[1], L[2], L[3], Rr[0], Rr[1], Rr[2], Rr[3], d, p.closure, c, chat, ratio, cc, eps, out);
}

// Matter-radiation coupling of one cell (Section 2.2.3), FP64 throughout.
// gas = (rho, mx, my, mz, E), rad = (E_r, Fx, Fy, Fz); returns iterations used,
// sets *fail when the iteration cap is reached.
__device__ __forceinline__ int exchange(const RadParamsDev& p, double dt, double* gas, double* rad, bool& fail) {
  const double rho = gas[0];
  const double c = p.c, ch = p.chat;
  const double coc = c / ch;
  const double Ek0 = 0.5 * ((gas[1] * gas[1] + gas[2] * gas[2]) + gas[3] * gas[3]) / rho;
  const double Eg0 = gas[4] - Ek0;
  const double Er0 = rad[0];
  const double Etot = Eg0 + coc * Er0;
  const double inv_Etot = 1.0 / Etot;
  const double k1 = dt * rho * p.kappa_P * ch;         // dR/d(a_r T^4 - E_r)
  const double dFG_dEr = -c * dt * rho * p.kappa_P;
  const double dFR_dEr = 1.0 + ch * dt * rho * p.kappa_P;
  const double gm1 = p.gamma - 1.0;
  const double Tfac = gm1 / rho;                       // T = E_g (gamma-1)/rho
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
    const double FR = (Er - Er0) - R;
    if (fabs(FG * inv_Etot) < p.newton_tol && fabs(coc * FR * inv_Etot) < p.newton_tol) {
      conv = true;
      break;
    }
    const double dFG_dEg = 1.0 + coc * dRdEg;
    const double dFR_dEg = -dRdEg;
    const double eta = -dFR_dEg / dFG_dEg;
    const double dEr = -(FR + eta * FG) / (dFR_dEr + eta * dFG_dEr);
    const double dEg = -(FG + dEr * dFG_dEr) / dFG_dEg;
    Eg += dEg;
    Er += dEr;
  }
  fail = fail || !conv;
  const double fac = 1.0 + rho * p.kappa_R * ch * dt;
  double m[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double F0 = rad[1 + d];
    const double F1 = F0 / fac;
    m[d] = gas[1 + d] - (F1 - F0) / (ch * c);
    rad[1 + d] = F1;
  }
  const double Ek1 = 0.5 * ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]) / rho;
  const double dEk = Ek1 - Ek0;
  gas[1] = m[0];
  gas[2] = m[1];
  gas[3] = m[2];
  gas[4] = Eg + (Ek0 + dEk);
  rad[0] = Er - (ch / c) * dEk;
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

template <class R, int TX, int TY>
struct RadSmem {
  static constexpr int NREC = ((TX + 2) * TY > TX * (TY + 2)) ? (TX + 2) * TY : TX * (TY + 2);
  static constexpr int NFL = ((TX + 1) * TY > TX * (TY + 1)) ? (TX + 1) * TY : TX * (TY + 1);
  R Qp[4][TY + 6][TX + 6];
  R rhoP[TY + 2][TX + 2];
  R recL[4][NREC];
  R recR[4][NREC];
  R fl[4][NFL];
};

// One tile of columns of one box for substep `a.sub` (the caller has checked
// that the substep is active).  Returns the largest exchange iteration count.
template <class S, class R, int TX, int TY, int STAGE>
__device__ __forceinline__ uint32_t rad_tile(const RadStageArgs<S, R>& a, int tbx, int tby, int tbz, int N,
                                             RadSmem<R, TX, TY>& sm, bool& bad_out, bool& nfail_out) {
  constexpr int NT = TX * TY;
  auto& Qp = sm.Qp;
  auto& rhoP = sm.rhoP;
  auto& recL = sm.recL;
  auto& recR = sm.recR;
  auto& fl = sm.fl;
  const DevBox& b = a.b;
  const RadParamsDev& p = a.p;
  const int t = threadIdx.x, tx = t % TX, ty = t / TX;
  const int x0 = tbx * TX, y0 = tby * TY;
  const int tw = min(TX, b.n0 - x0), th = min(TY, b.n1 - y0);
  const int z0 = tbz * a.zc;
  const int z1 = min(z0 + a.zc, b.n2);
  const bool act = tx < tw && ty < th;
  const int i = x0 + tx, j = y0 + ty;
  const int64_t vs = b.vs;
  const double dt = (a.dt_ptr ? *a.dt_ptr : a.dt_val) / N;  // substep dt
  const R c = R(p.c), chat = R(p.chat), ratio = R(p.chat / p.c), cc = R(p.c * p.chat);
  const R inv_c = R(1.0 / p.c);
  const bool tauc = p.tau_correction != 0;
  const S* __restrict__ Uin = a.Uin;
  bool bad = false, nfail = false;
  uint32_t itmax = 0;

  R w[4][5];  // own column (E, fx, fy, fz): [var][slot], slot s = plane m-2+s
  R aRz[4], Fz[4];
  R rz_k = R(0), rz_k1 = R(0);  // density of own column at k and k+1 (tau correction)

  auto load_q = [&](int ii, int jj, int kk, R* Q, bool& flag) {
    const int64_t o = cell(b, ii, jj, kk);
    const S* __restrict__ U = src_at(Uin, a.Ugh, b, ii, jj, kk);
    const double E = double(U[o]);
    const R Er = R(E);
    const R inv = R(1) / (c * Er);
    Q[0] = Er;
    Q[1] = R(U[o + vs]) * inv;
    Q[2] = R(U[o + 2 * vs]) * inv;
    Q[3] = R(U[o + 3 * vs]) * inv;
    flag = flag || !(E > 0.0);
  };
  auto load_w = [&](int kk, int slot) {
    R Q[4];
    load_q(i, j, kk, Q, bad);
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
  auto recon_z = [&](R* L, R* Rr) {
#pragma unroll
    for (int v = 0; v < 4; ++v) recon5<R>(w[v][0], w[v][1], w[v][2], w[v][3], w[v][4], p.recon, L[v], Rr[v]);
  };
  auto rho_at = [&](int kk) { return R(a.Ug[cell(b, i, j, kk)]); };

  // z prologue: flux through the bottom face of the chunk
  R cprev[4];
  if (act) {
#pragma unroll
    for (int s = 0; s < 5; ++s) load_w(z0 - 3 + s, s);
    R l[4], rprev[4];
    recon_z(l, rprev);
#pragma unroll
    for (int v = 0; v < 4; ++v) cprev[v] = w[v][2];  // cell z0-1
    shift_w();
    load_w(z0 + 2, 4);
    R rcur[4], ccur[4];
    recon_z(l, rcur);
#pragma unroll
    for (int v = 0; v < 4; ++v) ccur[v] = w[v][2];  // cell z0
    R rl = R(0), rr = R(0);
    if (tauc) {
      rl = rho_at(z0 - 1);
      rr = rho_at(z0);
    }
    rad_face<R>(rprev, l, cprev, ccur, rl, rr, R(b.dx2), 2, p, c, chat, ratio, cc, Fz);
#pragma unroll
    for (int v = 0; v < 4; ++v) aRz[v] = rcur[v];
    rz_k1 = rr;
  }
  bad = false;

  for (int k = z0; k < z1; ++k) {
    if (act) {
      shift_w();
      load_w(k + 3, 4);  // planes k-1..k+3, plane k in slot 1
#pragma unroll
      for (int v = 0; v < 4; ++v) Qp[v][ty + 3][tx + 3] = w[v][1];
      if (tauc) {
        rz_k = rz_k1;
        rz_k1 = rho_at(k + 1);
        rhoP[ty + 1][tx + 1] = rz_k;
      }
    }
    {
      const int nxh = 6 * th, nyh = 6 * tw, nh = nxh + nyh;
      const int nrx = tauc ? 2 * th : 0, nry = tauc ? 2 * tw : 0;
      for (int it = t; it < nh + nrx + nry; it += NT) {
        if (it < nh) {
          int xx, yy;
          if (it < nxh) {
            const int cc6 = it % 6;
            yy = it / 6;
            xx = cc6 < 3 ? cc6 - 3 : tw + cc6 - 3;
          } else {
            const int r = it - nxh, cc6 = r / tw;
            xx = r % tw;
            yy = cc6 < 3 ? cc6 - 3 : th + cc6 - 3;
          }
          R Q[4];
          bool dummy = false;
          load_q(x0 + xx, y0 + yy, k, Q, dummy);
#pragma unroll
          for (int v = 0; v < 4; ++v) Qp[v][yy + 3][xx + 3] = Q[v];
        } else if (it < nh + nrx) {
          const int r = it - nh;
          const int yy = r >> 1, xx = (r & 1) ? tw : -1;
          rhoP[yy + 1][xx + 1] = R(a.Ug[cell(b, x0 + xx, y0 + yy, k)]);
        } else {
          const int r = it - nh - nrx;
          const int xx = r % tw, yy = (r / tw) ? th : -1;
          rhoP[yy + 1][xx + 1] = R(a.Ug[cell(b, x0 + xx, y0 + yy, k)]);
        }
      }
    }
    __syncthreads();

    // ---- x sweep
    for (int it = t; it < (tw + 2) * th; it += NT) {
      const int xx = it % (tw + 2) - 1, yy = it / (tw + 2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const R* row = &Qp[v][yy + 3][xx + 1];
        recon5<R>(row[0], row[1], row[2], row[3], row[4], p.recon, recL[v][it], recR[v][it]);
      }
    }
    __syncthreads();
    for (int it = t; it < (tw + 1) * th; it += NT) {
      const int fx = it % (tw + 1), yy = it / (tw + 1);
      const int il = yy * (tw + 2) + fx, ir = il + 1;
      R sl[4], sr[4], cl[4], cr[4], F[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sl[v] = recR[v][il];
        sr[v] = recL[v][ir];
        cl[v] = Qp[v][yy + 3][fx + 2];
        cr[v] = Qp[v][yy + 3][fx + 3];
      }
      const R rl = tauc ? rhoP[yy + 1][fx] : R(0), rr = tauc ? rhoP[yy + 1][fx + 1] : R(0);
      rad_face<R>(sl, sr, cl, cr, rl, rr, R(b.dx0), 0, p, c, chat, ratio, cc, F);
#pragma unroll
      for (int v = 0; v < 4; ++v) fl[v][it] = F[v];
    }
    __syncthreads();
    R dfx[4];
    if (act) {
      const int f = ty * (tw + 1) + tx;
#pragma unroll
      for (int v = 0; v < 4; ++v) dfx[v] = fl[v][f + 1] - fl[v][f];
    }

    // ---- y sweep
    for (int it = t; it < tw * (th + 2); it += NT) {
      const int xx = it % tw, yy = it / tw - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        recon5<R>(Qp[v][yy + 1][xx + 3], Qp[v][yy + 2][xx + 3], Qp[v][yy + 3][xx + 3], Qp[v][yy + 4][xx + 3],
                  Qp[v][yy + 5][xx + 3], p.recon, recL[v][it], recR[v][it]);
    }
    __syncthreads();
    for (int it = t; it < tw * (th + 1); it += NT) {
      const int xx = it % tw, fy = it / tw;
      const int il = fy * tw + xx, ir = il + tw;
      R sl[4], sr[4], cl[4], cr[4], F[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sl[v] = recR[v][il];
        sr[v] = recL[v][ir];
        cl[v] = Qp[v][fy + 2][xx + 3];
        cr[v] = Qp[v][fy + 3][xx + 3];
      }
      const R rl = tauc ? rhoP[fy][xx + 1] : R(0), rr = tauc ? rhoP[fy + 1][xx + 1] : R(0);
      rad_face<R>(sl, sr, cl, cr, rl, rr, R(b.dx1), 1, p, c, chat, ratio, cc, F);
#pragma unroll
      for (int v = 0; v < 4; ++v) fl[v][it] = F[v];
    }
    __syncthreads();

    if (act) {
      R dfy[4];
      {
        const int f = ty * tw + tx;
#pragma unroll
        for (int v = 0; v < 4; ++v) dfy[v] = fl[v][f + tw] - fl[v][f];
      }
      // ---- z sweep: cell k+1 centred in the window
      R aLn[4], aRn[4], Fk[4], ck[4], ck1[4];
      recon_z(aLn, aRn);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ck[v] = w[v][1];
        ck1[v] = w[v][2];
      }
      rad_face<R>(aRz, aLn, ck, ck1, rz_k, rz_k1, R(b.dx2), 2, p, c, chat, ratio, cc, Fk);
      const int64_t o = cell(b, i, j, k);
      double un[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double tX = double(dfx[v]) * b.inv_dx0;
        const double tY = double(dfy[v]) * b.inv_dx1;
        const double tZ = double(Fk[v] - Fz[v]) * b.inv_dx2;
        const double L = -((tX + tY) + tZ);
        const double uin = double(Uin[o + v * vs]);
        un[v] = (STAGE == 1) ? uin + dt * L : 0.5 * double(a.Un[o + v * vs]) + 0.5 * (uin + dt * L);
        Fz[v] = Fk[v];
        aRz[v] = aRn[v];
      }
      if (STAGE == 2) {
        double gas[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) gas[v] = double(a.Ug[o + v * vs]);
        const int it = exchange(p, dt, gas, un, nfail);
        itmax = max(itmax, (uint32_t)it);
#pragma unroll
        for (int v = 1; v < 5; ++v) a.Ug[o + v * vs] = S(gas[v]);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) a.Uout[o + v * vs] = S(un[v]);
      bad = bad || !(un[0] > 0.0);
    }
  }
  bad_out = bad_out || bad;
  nfail_out = nfail_out || nfail;
  (void)inv_c;
  return itmax;
}

template <class S, class R, int TX, int TY, int STAGE>
__global__ __launch_bounds__(TX* TY, 2) void rad_stage_kernel(RadStageArgs<S, R> a) {
  const int N = a.nsub_ptr ? *a.nsub_ptr : a.nsub_val;
  if (a.sub >= N) return;  // block-uniform: the whole grid skips unused substeps
  __shared__ RadSmem<R, TX, TY> sm;
  const TileId tl = tile_of_block(a.gx, a.gy);
  bool bad = false, nfail = false;
  const uint32_t itmax = rad_tile<S, R, TX, TY, STAGE>(a, tl.bx, tl.by, tl.bz, N, sm, bad, nfail);
  if (bad) atomicOr(a.err, ERR_NEG);
  if (nfail) atomicOr(a.err, ERR_NEWTON);
  if (STAGE == 2) block_umax_to<TX * TY>(itmax, a.iter_max);
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
