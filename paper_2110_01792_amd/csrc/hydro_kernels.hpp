// Hydrodynamics kernels of the per-cell update (gfx950, wave64).
//
// One SSP-RK2 stage (Section 2.2.1) is two launches:
//   flatten_kernel : multidimensional shock-flattening coefficient chi of
//                    every cell of the box grown by one cell (it needs the
//                    pressure at +-3 along each axis);
//   stage_kernel   : primitive variables, PPM along x, y, z, HLLC at every
//                    face (each face once), unsplit divergence and the RK
//                    combination, fused.
// Both march in z.  A block owns a TX x TY tile of columns.  Each thread keeps
// the primitive variables of its own column over the five planes the z sweep
// needs in registers; the current plane, with a 3-cell halo in x and y, is
// staged in LDS for the x and y sweeps.  Face states and fluxes of a plane
// pass through LDS so that every interface is reconstructed and solved once.
#pragma once
#include "qk_device.hpp"
#include <type_traits>

namespace qk {

template <class S, class R>
struct StageArgs {
  const S* Uin;          // stage input (stencil reads)
  const S* Ugh;          // if non-NULL: ghost cells of the stage input are read here
                         // (boxes whose ghosts are all fixed data: the stage buffer
                         // then needs no ghost copy)
  const S* Un;           // stage 2: U^n at the thread's own cell
  S* Uout;               // stage 1: U^1;  stage 2: U^n (in place)
  const R* chi;          // flattening coefficients of Uin (one variable)
  DevBox b;
  double gamma;
  const double* dt_ptr;  // device dt, or NULL to use dt_val
  double dt_val;
  int zc;                // planes per block
  int gx, gy;            // tiles along x and y
  int recon;             // 0 PPM, 1 PLM
  unsigned long long* smax;  // stage 2: max(|v| + c_s) of the new state (ordered bits), or NULL
  uint32_t* err;
  double* reg;           // region_flux_kernel: flux register over the faces bounding
  int rlo[3], rhi[3];    //   region [rlo, rhi) (the stage kernel ignores these)
  double rw;             //   register weight: each face adds rw * dt/2 * F
  int img;               // IMG kernels: face code of the ghost images (ghost_image; two
                         // bits per axis, x lowest)
};

// Flux-register slot of variable v (of nv) on face `side` (0 low, 1 high) of
// a region for axis-d faces; (a, b) are the face's in-plane cell indices minus
// the region's low corner, (a along the slower axis).  Layout: x faces
// [v][side][k][j], then y faces [v][side][k][i], then z faces [v][side][j][i].
__device__ __forceinline__ int64_t reg_slot(const int* lo, const int* hi, int d, int v, int side, int a, int b,
                                            int nv) {
  const int64_t m0 = hi[0] - lo[0], m1 = hi[1] - lo[1], m2 = hi[2] - lo[2];
  const int64_t nx = 2 * m1 * m2, ny = 2 * m0 * m2;
  if (d == 0) return ((int64_t)(v * 2 + side) * m2 + a) * m1 + b;
  if (d == 1) return nv * nx + ((int64_t)(v * 2 + side) * m2 + a) * m0 + b;
  return nv * (nx + ny) + ((int64_t)(v * 2 + side) * m1 + a) * m0 + b;
}

// 1-D launch: consecutive hardware blocks are dealt round-robin to the 8
// XCDs, each with its own L2.  Re-number them so that every XCD receives one
// contiguous range of tiles (x fastest, then y, then z chunk): neighbouring
// tiles, which share halo planes, then run under the same L2.  XCD x holds
// blocks x, x+8, ...: nb/8 of them, one more for the first nb%8 XCDs.
struct TileId {
  int bx, by, bz;
};
__device__ __forceinline__ TileId tile_of_block(int gx, int gy) {
  const int hw = (int)blockIdx.x, nb = (int)gridDim.x;
  const int x = hw % 8, q = nb / 8, r = nb % 8;
  const int lg = x * q + min(x, r) + hw / 8;
  TileId t;
  t.bx = lg % gx;
  t.by = (lg / gx) % gy;
  t.bz = lg / (gx * gy);
  return t;
}

// Stage input for cell (i, j, k): the ghost source for cells outside the
// interior when one is given.
template <class S>
__device__ __forceinline__ const S* src_at(const S* U, const S* Ugh, const DevBox& b, int i, int j, int k) {
  const bool out = (unsigned)i >= (unsigned)b.n0 || (unsigned)j >= (unsigned)b.n1 || (unsigned)k >= (unsigned)b.n2;
  return (Ugh && out) ? Ugh : U;
}

template <class S>
__device__ __forceinline__ void load_cons(const S* __restrict__ U, int64_t vs, int64_t o, double* q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) q[v] = double(U[o + v * vs]);
}

// Block-wide maximum of a non-negative double, folded into *dst with an
// unsigned 64-bit atomic max on its bit pattern (monotone for x >= 0).
template <int NT>
__device__ __forceinline__ void block_max_to(double x, unsigned long long* dst) {
  __shared__ double red[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k) m = fmax(m, red[k]);
    atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------------------------------------
// Flattening coefficient over cells [-1, n] in every axis.
// ---------------------------------------------------------------------------
template <class S, class R>
struct FlatArgs {
  const S* U;
  const S* Ugh;  // ghost source (see StageArgs) or NULL
  R* chi;
  DevBox b;
  double gm1;
  int zc;
  int img;       // IMG kernels: face code of the ghost images (see StageArgs)
};

template <class R, int TX, int TY>
struct FlatSmem {
  R Pp[TY + 6][TX + 6], uxp[TY + 6][TX + 6], uyp[TY + 6][TX + 6];
  R ctx[TY][TX + 2];
  R cty[TY + 2][TX];
};

// One cell of a plane's halo ring that a thread loads for every plane of its
// tile: its state array, its offset in plane 0 (add k * pz), its flat index in
// the LDS plane and its kind (0 none, 1 primitive state, 2 flattening value).
template <class S>
struct HaloCell {
  const S* src;
  int64_t off;
  int lds, kind;
};

// Prefetch of one halo cell at plane offset pl: NV state variables (kind 1)
// or one value of the auxiliary per-cell array (kind 2) into q (as double).
template <int NV, class S, class T>
__device__ __forceinline__ void load_halo(const HaloCell<S>& h, const S* src, const T* aux, int64_t pl, int64_t vs,
                                          double* q) {
  if (h.kind == 1) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = double(src[h.off + pl + v * vs]);
  } else if (h.kind == 2) {
    q[0] = double(aux[h.off + pl]);
  }
}

// One tile of columns (tile indices over the grown range [-1, n]).  The
// tile's own cells come from each thread's z window; the 3-cell halo ring of
// each plane is prefetched one plane ahead into registers.  NT threads
// (NT >= TX*TY); thread t owns column (t % TX, t / TX).  IMG: every face of
// the box is periodic or outflow (each extent >= 4) and its ghost cells are
// not filled; a cell outside is read at the cell the fill would copy
// (ghost_image with the face code a.img).
template <class S, class R, int TX, int TY, int NT, bool IMG = false>
__device__ __forceinline__ void flatten_tile(const FlatArgs<S, R>& a, int tbx, int tby, int tbz,
                                             FlatSmem<R, TX, TY>& sm) {
  static_assert(NT >= TX * TY, "one thread per column");
  constexpr int NHX = 6 * TY, NHY = 6 * TX, NH = NHX + NHY, HPT = (NH + NT - 1) / NT;
  const DevBox& b = a.b;
  const int t = threadIdx.x, tx = t % TX, ty = t / TX;
  const int xs = -1 + tbx * TX, ys = -1 + tby * TY;
  const int tw = min(TX, b.n0 + 1 - xs), th = min(TY, b.n1 + 1 - ys);
  const int zs = -1 + tbz * a.zc;
  const int ze = min(zs + a.zc, b.n2 + 1);
  const bool act = tx < tw && ty < th;
  const int i = xs + tx, j = ys + ty;
  const int64_t vs = b.vs, pz = b.pz;
  const double gm1 = a.gm1;
  bool bad = false;

  HaloCell<S> hc[HPT];
#pragma unroll
  for (int m = 0; m < HPT; ++m) {
    const int it = t + m * NT;
    int xx = 0, yy = 0, kind = 0;
    if (it < NHX) {
      const int c = it % 6;
      yy = it / 6;
      xx = c < 3 ? c - 3 : tw + c - 3;
      kind = yy < th ? 1 : 0;
    } else if (it < NH) {
      const int r = it - NHX, c = r / TX;
      xx = r % TX;
      yy = c < 3 ? c - 3 : th + c - 3;
      kind = xx < tw ? 1 : 0;
    }
    hc[m].kind = kind;
    hc[m].src = src_at(a.U, a.Ugh, b, xs + xx, ys + yy, 0);
    hc[m].off = IMG ? cell(b, ghost_image(xs + xx, b.n0, a.img & 3), ghost_image(ys + yy, b.n1, (a.img >> 2) & 3), 0)
                    : cell(b, xs + xx, ys + yy, 0);
    hc[m].lds = (yy + 3) * (TX + 6) + (xx + 3);
  }
  // own column and plane index as read (ghost images under IMG)
  const int ir = IMG ? ghost_image(i, b.n0, a.img & 3) : i, jr = IMG ? ghost_image(j, b.n1, (a.img >> 2) & 3) : j;
  auto zimg = [&](int kk) { return IMG ? ghost_image(kk, b.n2, (a.img >> 4) & 3) : kk; };
  // planes -1 and n of the grown range lie outside the interior in z
  auto hsrc = [&](const HaloCell<S>& h, int kk) {
    return (a.Ugh && (unsigned)kk >= (unsigned)b.n2) ? a.Ugh : h.src;
  };

  R P[7], uz[7];    // own column, planes k-3 .. k+3
  R uxq[4], uyq[4];  // own column, planes k .. k+3
  R cz[3];           // chi_tilde_z at k-1, k, k+1
  double cq[5];      // conserved state of plane k+3 (prefetched)
  double hq[HPT][5];  // halo ring of plane k (prefetched)
  auto prim = [&](const double* q, R& p, R& ux, R& uy, R& w) {
    R W[5];
    cons_to_prim<R>(q[0], q[1], q[2], q[3], q[4], gm1, W, bad);
    ux = W[1];
    uy = W[2];
    w = W[3];
    p = W[4];
  };
  if (act) {
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int kk = zs - 3 + s;
      double q[5];
      load_cons(src_at(a.U, a.Ugh, b, i, j, kk), vs, cell(b, ir, jr, zimg(kk)), q);
      R ux, uy;
      prim(q, P[s + 1], ux, uy, uz[s + 1]);
      if (s >= 3) {
        uxq[s - 2] = ux;
        uyq[s - 2] = uy;
      }
    }
    cz[1] = chi_tilde<R>(P[1], P[2], P[4], P[5], uz[2], uz[4]);
    cz[2] = chi_tilde<R>(P[2], P[3], P[5], P[6], uz[3], uz[5]);
    load_cons(src_at(a.U, a.Ugh, b, i, j, zs + 3), vs, cell(b, ir, jr, zimg(zs + 3)), cq);
  }
#pragma unroll
  for (int m = 0; m < HPT; ++m)
    load_halo<5>(hc[m], hsrc(hc[m], zs), (const R*)nullptr, (int64_t)zimg(zs) * pz, vs, hq[m]);

  for (int k = zs; k < ze; ++k) {
    if (act) {
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        P[s] = P[s + 1];
        uz[s] = uz[s + 1];
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        uxq[s] = uxq[s + 1];
        uyq[s] = uyq[s + 1];
      }
      prim(cq, P[6], uxq[3], uyq[3], uz[6]);
      cz[0] = cz[1];
      cz[1] = cz[2];
      cz[2] = chi_tilde<R>(P[2], P[3], P[5], P[6], uz[3], uz[5]);  // at k+1
      sm.Pp[ty + 3][tx + 3] = P[3];
      sm.uxp[ty + 3][tx + 3] = uxq[0];
      sm.uyp[ty + 3][tx + 3] = uyq[0];
    }
#pragma unroll
    for (int m = 0; m < HPT; ++m) {
      if (hc[m].kind == 1) {
        bool dummy = false;
        R W[5];
        cons_to_prim<R>(hq[m][0], hq[m][1], hq[m][2], hq[m][3], hq[m][4], gm1, W, dummy);
        (&sm.Pp[0][0])[hc[m].lds] = W[4];
        (&sm.uxp[0][0])[hc[m].lds] = W[1];
        (&sm.uyp[0][0])[hc[m].lds] = W[2];
      }
    }
    if (k + 1 < ze) {
      if (act) load_cons(src_at(a.U, a.Ugh, b, i, j, k + 4), vs, cell(b, ir, jr, zimg(k + 4)), cq);
#pragma unroll
      for (int m = 0; m < HPT; ++m)
        load_halo<5>(hc[m], hsrc(hc[m], k + 1), (const R*)nullptr, (int64_t)zimg(k + 1) * pz, vs, hq[m]);
    }
    __syncthreads();
    for (int it = t; it < (TX + 2) * TY; it += NT) {
      const int xx = it % (TX + 2) - 1, yy = it / (TX + 2);
      if (xx <= tw && yy < th) {
        const int X = xx + 3, Y = yy + 3;
        sm.ctx[yy][xx + 1] = chi_tilde<R>(sm.Pp[Y][X - 2], sm.Pp[Y][X - 1], sm.Pp[Y][X + 1], sm.Pp[Y][X + 2],
                                          sm.uxp[Y][X - 1], sm.uxp[Y][X + 1]);
      }
    }
    for (int it = t; it < TX * (TY + 2); it += NT) {
      const int xx = it % TX, yy = it / TX - 1;
      if (xx < tw && yy <= th) {
        const int X = xx + 3, Y = yy + 3;
        sm.cty[yy + 1][xx] = chi_tilde<R>(sm.Pp[Y - 2][X], sm.Pp[Y - 1][X], sm.Pp[Y + 1][X], sm.Pp[Y + 2][X],
                                          sm.uyp[Y - 1][X], sm.uyp[Y + 1][X]);
      }
    }
    __syncthreads();
    if (act) {
      const int X = tx + 3, Y = ty + 3;
      const int sx = (sm.Pp[Y][X + 1] - sm.Pp[Y][X - 1] > R(0)) ? 1 : -1;
      const int sy = (sm.Pp[Y + 1][X] - sm.Pp[Y - 1][X] > R(0)) ? 1 : -1;
      const int sz = (P[4] - P[2] > R(0)) ? 1 : -1;
      const R chx = rmin(sm.ctx[ty][tx + 1], sm.ctx[ty][tx + 1 + sx]);
      const R chy = rmin(sm.cty[ty + 1][tx], sm.cty[ty + 1 + sy][tx]);
      const R chz = rmin(cz[1], cz[1 + sz]);
      a.chi[cell(b, i, j, k)] = rmin(chx, rmin(chy, chz));
    }
    __syncthreads();
  }
}

// Single-box flattening: 32 x 30 tiles on 1024 threads.  Each phase is one
// item per thread (34 x 30 x-coefficients, 32 x 32 y-coefficients, a 372-cell
// halo ring), and the halo ring per cell is half that of a 16 x 14 tile.
constexpr int FTX = 32, FTY = 30, FNT = 1024;

// FP32: held to 64 VGPRs (8 waves per SIMD: two 1024-thread blocks per CU,
// the whole grid resident at 256^3) to hide the z-march's load latency.
template <class S, class R, bool IMG = false>
__global__ __launch_bounds__(FNT, sizeof(S) == 4 ? 8 : 4) void flatten_kernel(FlatArgs<S, R> a, int gx, int gy) {
  __shared__ FlatSmem<R, FTX, FTY> sm;
  const TileId tl = tile_of_block(gx, gy);
  flatten_tile<S, R, FTX, FTY, FNT, IMG>(a, tl.bx, tl.by, tl.bz, sm);
}

// ---------------------------------------------------------------------------
// One SSP-RK2 stage, fused.  STAGE 1: Uout = Uin + dt L(Uin).
// STAGE 2: Uout = 0.5 Un + 0.5 (Uin + dt L(Uin)), Uout == Un allowed (each
// cell reads Un only at itself).
// ---------------------------------------------------------------------------
// Reconstruction of the five primitives of one cell, each blended toward the
// cell average with the flattening coefficient ch: a = ch a + (1 - ch) q.
// Where ch = 1 (away from shocks, most of the grid) the blend returns a
// itself, so it is skipped, and whole waves with ch = 1 branch past it.
// qat(v, q) fetches the five averages of variable v along the axis.
template <class R, class Q>
__device__ __forceinline__ void recon_flat5(const Q& qat, R ch, int recon, R* l, R* r) {
  R c[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    R q[5];
    qat(v, q);
    recon5<R>(q[0], q[1], q[2], q[3], q[4], recon, l[v], r[v]);
    c[v] = q[2];
  }
  if (ch != R(1)) {
    const R om = R(1) - ch;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      l[v] = ch * l[v] + om * c[v];
      r[v] = ch * r[v] + om * c[v];
    }
  }
}

// LDS of one stage tile.  SPLIT: x and y face states and fluxes have buffers
// of their own, so both sweeps reconstruct in one phase and solve their faces
// in the next (three barriers per plane).  Otherwise the y sweep reuses the
// x sweep's buffers after it (five barriers, less LDS).
template <class R, int TX, int TY, bool SPLIT>
struct HydroSmem {
  static constexpr int NXR = (TX + 2) * TY, NYR = TX * (TY + 2);
  static constexpr int NXF = (TX + 1) * TY, NYF = TX * (TY + 1);
  static constexpr int XS = SPLIT ? NXR : (NXR > NYR ? NXR : NYR);  // x (shared) state buffer length
  static constexpr int XFS = SPLIT ? NXF : (NXF > NYF ? NXF : NYF);
  static constexpr int YS = SPLIT ? NYR : XS, YFS = SPLIT ? NYF : XFS;
  R Wp[5][TY + 6][TX + 6];
  R chiP[TY + 2][TX + 2];
  R xL[5][XS], xR[5][XS];
  R xF[5][XFS];
  R yL[5][SPLIT ? NYR : 1], yR[5][SPLIT ? NYR : 1];
  R yF[5][SPLIT ? NYF : 1];
};

// One tile of columns of one box: returns the thread's max(|v| + c_s) of the
// new state (stage 2 with a.smax set), sets `bad` on a non-positive state.
// NT threads (NT >= TX*TY); thread t owns column (t % TX, t / TX).
template <class S, class R, int TX, int TY, int NT, bool SPLIT, int STAGE, bool IMG = false>
__device__ __forceinline__ double stage_tile(const StageArgs<S, R>& a, int tbx, int tby, int tbz,
                                             HydroSmem<R, TX, TY, SPLIT>& sm, bool& bad_out) {
  using SM = HydroSmem<R, TX, TY, SPLIT>;
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

  const DevBox& b = a.b;
  const int t = threadIdx.x, tx = t % TX, ty = t / TX;
  const int x0 = tbx * TX, y0 = tby * TY;
  const int tw = min(TX, b.n0 - x0), th = min(TY, b.n1 - y0);
  const int z0 = tbz * a.zc;
  const int z1 = min(z0 + a.zc, b.n2);
  const bool act = tx < tw && ty < th;
  const int i = x0 + tx, j = y0 + ty;
  const int64_t vs = b.vs, pz = b.pz;
  const double dt = a.dt_ptr ? *a.dt_ptr : a.dt_val;
  const double gm1 = a.gamma - 1.0;
  const GasK<R> g = gas_k<R>(a.gamma);
  const S* __restrict__ Uin = a.Uin;
  const R* __restrict__ chi = a.chi;
  bool bad = false;

  // halo ring of every plane: 3 cells of state beyond each x and y edge of
  // the tile, 1 cell of flattening coefficients
  HaloCell<S> hc[HPT];
#pragma unroll
  for (int m = 0; m < HPT; ++m) {
    const int it = t + m * NT;
    int xx = 0, yy = 0, kind = 0, lds = 0;
    if (it < NHX) {
      const int c = it % 6;
      yy = it / 6;
      xx = c < 3 ? c - 3 : tw + c - 3;
      kind = yy < th ? 1 : 0;
    } else if (it < NHX + NHY) {
      const int r = it - NHX, c = r / TX;
      xx = r % TX;
      yy = c < 3 ? c - 3 : th + c - 3;
      kind = xx < tw ? 1 : 0;
    } else if (it < NHX + NHY + NCX) {
      const int r = it - NHX - NHY;
      yy = r >> 1;
      xx = (r & 1) ? tw : -1;
      kind = yy < th ? 2 : 0;
    } else if (it < NH) {
      const int r = it - NHX - NHY - NCX;
      xx = r % TX;
      yy = (r / TX) ? th : -1;
      kind = xx < tw ? 2 : 0;
    }
    lds = kind == 2 ? (yy + 1) * (TX + 2) + (xx + 1) : (yy + 3) * (TX + 6) + (xx + 3);
    hc[m].kind = kind;
    hc[m].src = src_at(Uin, a.Ugh, b, x0 + xx, y0 + yy, z0);
    // IMG: the state ring at its ghost images; the flattening ring (kind 2)
    // where it lies, since the flattening pass covers the grown range
    hc[m].off = (IMG && kind == 1)
                    ? cell(b, ghost_image(x0 + xx, b.n0, a.img & 3), ghost_image(y0 + yy, b.n1, (a.img >> 2) & 3), 0)
                    : cell(b, x0 + xx, y0 + yy, 0);
    hc[m].lds = lds;
  }
  auto zimg = [&](int kk) { return IMG ? ghost_image(kk, b.n2, (a.img >> 4) & 3) : kk; };

  R w[5][5];  // own column primitives: [var][plane slot], slot s = plane m-2+s
  R aRz[5], Fz[5];
  double cq[5];       // conserved state of own column, plane k+3 (prefetched)
  double hq[HPT][5];  // halo ring of plane k (prefetched)
  double uo[5], un[5];
  R chk = R(0);       // chi of own cell, plane k

  auto prim_w = [&](const double* q, int slot) {
    R W[5];
    cons_to_prim<R>(q[0], q[1], q[2], q[3], q[4], gm1, W, bad);
#pragma unroll
    for (int v = 0; v < 5; ++v) w[v][slot] = W[v];
  };
  auto load_w = [&](int kk, int slot) {
    double q[5];
    load_cons(src_at(Uin, a.Ugh, b, i, j, kk), vs, cell(b, i, j, zimg(kk)), q);
    prim_w(q, slot);
  };
  auto shift_w = [&]() {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
#pragma unroll
      for (int s = 0; s < 4; ++s) w[v][s] = w[v][s + 1];
    }
  };
  // z reconstruction of the cell centred in the window; z-rotated output
  // (rho, w, u, v, P) so that it feeds the z Riemann problem directly.  PPM
  // keeps the unlimited upper interface value (fzr) for the next plane, whose
  // lower interface it is (CARRY: the window has moved by one plane since).
  R fzr[5];
  auto recon_z = [&](R ch, R* L, R* Rr, auto carry) {
    R l[5], r[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      if (a.recon == 1) {
        plm<R>(w[v][1], w[v][2], w[v][3], l[v], r[v]);
      } else {
        const R fl = decltype(carry)::value ? fzr[v] : ppm_iface<R>(w[v][0], w[v][1], w[v][2], w[v][3]);
        fzr[v] = ppm_iface<R>(w[v][1], w[v][2], w[v][3], w[v][4]);
        ppm_limit<R>(w[v][1], w[v][2], w[v][3], fl, fzr[v], l[v], r[v]);
      }
    }
    if (ch != R(1)) {
      const R om = R(1) - ch;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        l[v] = ch * l[v] + om * w[v][2];
        r[v] = ch * r[v] + om * w[v][2];
      }
    }
    L[0] = l[0]; L[1] = l[3]; L[2] = l[1]; L[3] = l[2]; L[4] = l[4];
    Rr[0] = r[0]; Rr[1] = r[3]; Rr[2] = r[1]; Rr[3] = r[2]; Rr[4] = r[4];
  };

  if (act) {
#pragma unroll
    for (int s = 0; s < 5; ++s) load_w(z0 - 3 + s, s);  // centred on z0-1
    R l[5], rprev[5];
    recon_z(chi[cell(b, i, j, z0 - 1)], l, rprev, std::false_type{});
    shift_w();
    load_w(z0 + 2, 4);  // centred on z0
    R rcur[5];
    chk = chi[cell(b, i, j, z0)];
    recon_z(chk, l, rcur, std::true_type{});
    hllc<R>(rprev, l, g, Fz);
#pragma unroll
    for (int v = 0; v < 5; ++v) aRz[v] = rcur[v];
    load_cons(src_at(Uin, a.Ugh, b, i, j, z0 + 3), vs, cell(b, i, j, zimg(z0 + 3)), cq);
  }
#pragma unroll
  for (int m = 0; m < HPT; ++m) load_halo<5>(hc[m], hc[m].src, chi, (int64_t)z0 * pz, vs, hq[m]);
  bad = false;
  double smax = 0.0;

  for (int k = z0; k < z1; ++k) {
    R chn = R(0);
    if (act) {
      shift_w();
      prim_w(cq, 4);  // window: planes k-1 .. k+3; plane k in slot 1
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.Wp[v][ty + 3][tx + 3] = w[v][1];
      sm.chiP[ty + 1][tx + 1] = chk;
    }
#pragma unroll
    for (int m = 0; m < HPT; ++m) {
      if (hc[m].kind == 1) {
        R W[5];
        bool dummy = false;
        cons_to_prim<R>(hq[m][0], hq[m][1], hq[m][2], hq[m][3], hq[m][4], gm1, W, dummy);
#pragma unroll
        for (int v = 0; v < 5; ++v) (&sm.Wp[v][0][0])[hc[m].lds] = W[v];
      } else if (hc[m].kind == 2) {
        (&sm.chiP[0][0])[hc[m].lds] = R(hq[m][0]);
      }
    }
    // loads for the rest of this plane and the next one, in flight during the sweeps
    if (act) {
      const int64_t o = cell(b, i, j, k);
      chn = chi[o + pz];
      load_cons(Uin, vs, o, uo);
      if (STAGE == 2) load_cons(a.Un, vs, o, un);
      if (k + 1 < z1) load_cons(src_at(Uin, a.Ugh, b, i, j, k + 4), vs, cell(b, i, j, zimg(k + 4)), cq);
    }
    if (k + 1 < z1) {
#pragma unroll
      for (int m = 0; m < HPT; ++m) load_halo<5>(hc[m], hc[m].src, chi, (int64_t)(k + 1) * pz, vs, hq[m]);
    }
    __syncthreads();

    auto x_recon = [&]() {
      for (int it = t; it < NXR; it += NT) {
        const int xx = it % (TX + 2) - 1, yy = it / (TX + 2);
        if (xx <= tw && yy < th) {
          const R ch = sm.chiP[yy + 1][xx + 1];
          R l[5], r[5];
          recon_flat5<R>(
              [&](int v, R* q) {
                const R* row = &sm.Wp[v][yy + 3][xx + 1];
#pragma unroll
                for (int s = 0; s < 5; ++s) q[s] = row[s];
              },
              ch, a.recon, l, r);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            xL[v * XS + it] = l[v];
            xR[v * XS + it] = r[v];
          }
        }
      }
    };
    auto x_faces = [&]() {
      for (int it = t; it < NXF; it += NT) {
        const int fx = it % (TX + 1), yy = it / (TX + 1);
        if (fx <= tw && yy < th) {
          const int il = yy * (TX + 2) + fx, ir = il + 1;
          R WL[5], WR[5], F[5];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            WL[v] = xR[v * XS + il];
            WR[v] = xL[v * XS + ir];
          }
          hllc<R>(WL, WR, g, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) xF[v * XFS + it] = F[v];
          // a face on a tile edge belongs to the tile on its high side, except the box's last face
        }
      }
    };
    auto y_recon = [&]() {
      for (int it = t; it < NYR; it += NT) {
        const int xx = it % TX, yy = it / TX - 1;
        if (xx < tw && yy <= th) {
          const R ch = sm.chiP[yy + 1][xx + 1];
          R l[5], r[5];
          recon_flat5<R>(
              [&](int v, R* q) {
#pragma unroll
                for (int s = 0; s < 5; ++s) q[s] = sm.Wp[v][yy + 1 + s][xx + 3];
              },
              ch, a.recon, l, r);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            yL[v * YS + it] = l[v];
            yR[v * YS + it] = r[v];
          }
        }
      }
    };
    auto y_faces = [&]() {
      for (int it = t; it < NYF; it += NT) {
        const int xx = it % TX, fy = it / TX;
        if (xx < tw && fy <= th) {
          const int il = fy * TX + xx, ir = il + TX;
          R WL[5] = {yR[il], yR[2 * YS + il], yR[YS + il], yR[3 * YS + il], yR[4 * YS + il]};
          R WR[5] = {yL[ir], yL[2 * YS + ir], yL[YS + ir], yL[3 * YS + ir], yL[4 * YS + ir]};
          R F[5];
          hllc<R>(WL, WR, g, F);
          yF[it] = F[0];
          yF[YFS + it] = F[2];
          yF[2 * YFS + it] = F[1];
          yF[3 * YFS + it] = F[3];
          yF[4 * YFS + it] = F[4];
        }
      }
    };

    R dfx[5], dfy[5];
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
        for (int v = 0; v < 5; ++v) {
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
        for (int v = 0; v < 5; ++v) dfx[v] = xF[v * XFS + fxi + 1] - xF[v * XFS + fxi];
      }
      y_recon();
      __syncthreads();
      y_faces();
      __syncthreads();
      if (act) {
        const int fyi = ty * TX + tx;
#pragma unroll
        for (int v = 0; v < 5; ++v) dfy[v] = yF[v * YFS + fyi + TX] - yF[v * YFS + fyi];
      }
    }

    if (act) {
      // ---- z sweep: cell k+1 is centred in the window
      R aLn[5], aRn[5], Fk[5];
      recon_z(chn, aLn, aRn, std::true_type{});
      hllc<R>(aRz, aLn, g, Fk);
      // un-rotate (rho, w, u, v, E) fluxes to (rho, x, y, z, E)
      R Fn[5] = {Fk[0], Fk[2], Fk[3], Fk[1], Fk[4]};
      R Fo[5] = {Fz[0], Fz[2], Fz[3], Fz[1], Fz[4]};
      const int64_t o = cell(b, i, j, k);
      double unew[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double tX = double(dfx[v]) * b.inv_dx0;
        const double tY = double(dfy[v]) * b.inv_dx1;
        const double tZ = double(Fn[v] - Fo[v]) * b.inv_dx2;
        const double L = -((tX + tY) + tZ);
        if (STAGE == 1) {
          unew[v] = uo[v] + dt * L;
        } else {
          unew[v] = 0.5 * un[v] + 0.5 * (uo[v] + dt * L);
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        a.Uout[o + v * vs] = S(unew[v]);
        Fz[v] = Fk[v];
        aRz[v] = aRn[v];
      }
      chk = chn;
      if (STAGE == 2 && a.smax) {
        double q[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) q[v] = double(S(unew[v]));
        smax = fmax(smax, signal_speed(q, a.gamma, gm1, bad));
      }
    }
  }
  bad_out = bad_out || bad;
  return smax;
}

// Faces bounding region [lo, hi) as one index range: x faces (low side, then
// high side), then y faces, then z faces; within an axis-d side, (a, b) are
// the in-plane cell indices relative to the region (a along the slower of
// the two other axes), as in reg_slot.
struct RegionFace {
  int d, side, a, b;
};

__host__ __device__ __forceinline__ int64_t region_face_count(const int* lo, const int* hi) {
  const int64_t m0 = hi[0] - lo[0], m1 = hi[1] - lo[1], m2 = hi[2] - lo[2];
  return 2 * (m1 * m2 + m0 * m2 + m0 * m1);
}

__device__ __forceinline__ RegionFace region_face(const int* lo, const int* hi, int64_t c) {
  const int64_t m0 = hi[0] - lo[0], m1 = hi[1] - lo[1], m2 = hi[2] - lo[2];
  const int64_t nface[3] = {m1 * m2, m0 * m2, m0 * m1};
  RegionFace f;
  f.d = 0;
  while (c >= 2 * nface[f.d]) {
    c -= 2 * nface[f.d];
    ++f.d;
  }
  f.side = (int)(c / nface[f.d]);
  const int64_t e = c % nface[f.d];
  const int64_t mb = f.d == 0 ? m1 : m0;
  f.a = (int)(e / mb);
  f.b = (int)(e % mb);
  return f;
}

// Flux register of one hydro stage: the fluxes at the faces bounding region
// [rlo, rhi), recomputed from the stage input and its flattening
// coefficients with the stage kernel's own device functions on the same
// operands (conversion, reconstruction with flattening, HLLC, the same
// rotations), so every face carries the bits the stage used; each adds
// rw * dt/2 * F to its slot.  One thread per face.  Launched after the stage,
// which leaves its input and chi as they were.
template <class S, class R>
__global__ __launch_bounds__(256) void region_flux_kernel(StageArgs<S, R> a) {
  const DevBox& b = a.b;
  const int lo[3] = {a.rlo[0], a.rlo[1], a.rlo[2]}, hi[3] = {a.rhi[0], a.rhi[1], a.rhi[2]};
  const int64_t total = region_face_count(lo, hi);
  const double dt = a.dt_ptr ? *a.dt_ptr : a.dt_val;
  const double w = 0.5 * dt * a.rw;
  const double gm1 = a.gamma - 1.0;
  const GasK<R> g = gas_k<R>(a.gamma);
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    const RegionFace rf = region_face(lo, hi, c);
    const int d = rf.d;
    // cell f along d (the face lies between cells f-1 and f); unit step e along d
    const int ei = d == 0, ej = d == 1, ek = d == 2;
    const int i = d == 0 ? (rf.side ? hi[0] : lo[0]) : lo[0] + rf.b;
    const int j = d == 1 ? (rf.side ? hi[1] : lo[1]) : (d == 0 ? lo[1] + rf.b : lo[1] + rf.a);
    const int k = d == 2 ? (rf.side ? hi[2] : lo[2]) : lo[2] + rf.a;
    R W[6][5];  // primitives of cells f-3 .. f+2 along d
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      const int ii = i + ei * (s - 3), jj = j + ej * (s - 3), kk = k + ek * (s - 3);
      double q[5];
      load_cons(src_at(a.Uin, a.Ugh, b, ii, jj, kk), b.vs, cell(b, ii, jj, kk), q);
      bool dummy = false;
      cons_to_prim<R>(q[0], q[1], q[2], q[3], q[4], gm1, W[s], dummy);
    }
    const R chl = a.chi[cell(b, i - ei, j - ej, k - ek)], chr = a.chi[cell(b, i, j, k)];
    R ll[5], rl[5], lr[5], rr[5];
    recon_flat5<R>(
        [&](int v, R* q) {
#pragma unroll
          for (int s = 0; s < 5; ++s) q[s] = W[s][v];
        },
        chl, a.recon, ll, rl);  // cell f-1
    recon_flat5<R>(
        [&](int v, R* q) {
#pragma unroll
          for (int s = 0; s < 5; ++s) q[s] = W[s + 1][v];
        },
        chr, a.recon, lr, rr);  // cell f
    // normal velocity first, as the sweeps order them: x (u, v, w), y (v, u, w), z (w, u, v)
    const R WL[5] = {rl[0], d == 0 ? rl[1] : (d == 1 ? rl[2] : rl[3]), d == 0 ? rl[2] : rl[1],
                     d == 2 ? rl[2] : rl[3], rl[4]};
    const R WR[5] = {lr[0], d == 0 ? lr[1] : (d == 1 ? lr[2] : lr[3]), d == 0 ? lr[2] : lr[1],
                     d == 2 ? lr[2] : lr[3], lr[4]};
    R F[5];
    hllc<R>(WL, WR, g, F);
    const double Fd[5] = {double(F[0]), double(d == 0 ? F[1] : F[2]), double(d == 0 ? F[2] : (d == 1 ? F[1] : F[3])),
                          double(d == 2 ? F[1] : F[3]), double(F[4])};
#pragma unroll
    for (int v = 0; v < 5; ++v) a.reg[reg_slot(lo, hi, d, v, rf.side, rf.a, rf.b, 5)] += w * Fd[v];
  }
}

// Single-box stage: 16 x 14 tiles on 256 threads, so that each sweep phase
// (18 x 14 and 16 x 16 reconstructions, 17 x 14 and 16 x 15 faces) is one
// item per thread.
constexpr int STX = 16, STY = 14, SNT = 256;

template <class S, class R, int STAGE, bool IMG = false>
__global__ __launch_bounds__(SNT) void stage_kernel(StageArgs<S, R> a) {
  __shared__ HydroSmem<R, STX, STY, true> sm;
  const TileId tl = tile_of_block(a.gx, a.gy);
  bool bad = false;
  const double smax = stage_tile<S, R, STX, STY, SNT, true, STAGE, IMG>(a, tl.bx, tl.by, tl.bz, sm, bad);
  if (bad) atomicOr(a.err, ERR_NEG);
  if (STAGE == 2 && a.smax) block_max_to<SNT>(smax, a.smax);
}


// ---------------------------------------------------------------------------
// CFL reduction: max over interior cells of |v| + c_s, folded with an atomic
// max on the ordered bit pattern.
// ---------------------------------------------------------------------------
template <class S, int NT>
__global__ __launch_bounds__(NT) void max_signal_kernel(const S* __restrict__ U, DevBox b, double gamma,
                                                        unsigned long long* smax, uint32_t* err) {
  const int64_t ncell = (int64_t)b.n0 * b.n1 * b.n2;
  const double gm1 = gamma - 1.0;
  double m = 0.0;
  bool bad = false;
  const bool small = ncell < ((int64_t)1 << 31);  // 32-bit index arithmetic (64-bit division is long)
  for (int64_t c = (int64_t)blockIdx.x * NT + threadIdx.x; c < ncell; c += (int64_t)gridDim.x * NT) {
    int i, j, k;
    if (small) {
      const uint32_t u = (uint32_t)c, q = u / (uint32_t)b.n0, kq = q / (uint32_t)b.n1;
      i = (int)(u - q * (uint32_t)b.n0);
      j = (int)(q - kq * (uint32_t)b.n1);
      k = (int)kq;
    } else {
      i = (int)(c % b.n0);
      j = (int)((c / b.n0) % b.n1);
      k = (int)(c / ((int64_t)b.n0 * b.n1));
    }
    double q[5];
    load_cons(U, b.vs, cell(b, i, j, k), q);
    m = fmax(m, signal_speed(q, gamma, gm1, bad));
  }
  if (bad) atomicOr(err, ERR_NEG);
  block_max_to<NT>(m, smax);
}

// dt = cfl * dxmin / smax; with a radiation substep limit dt_r the substep
// count N = ceil(dt/dt_r), capped at nsub_max with dt shrunk to N dt_r.
// Clears the accumulator for its next use.
__global__ void finalize_dt_kernel(unsigned long long* smax_bits, double cfl, double dxmin, double dt_r,
                                   int nsub_max, double* dt_out, int32_t* nsub_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double smax = __longlong_as_double((long long)*smax_bits);
  double dt = cfl * dxmin / smax;
  int n = 0;
  if (dt_r > 0.0) {
    const double r = ceil(dt / dt_r);
    n = (r < 1.0) ? 1 : (r > (double)nsub_max ? nsub_max + 1 : (int)r);
    if (n > nsub_max) {
      n = nsub_max;
      dt = n * dt_r;
    }
  }
  if (dt_out) *dt_out = dt;
  if (nsub_out) *nsub_out = n;
  *smax_bits = 0ull;
}

// ---------------------------------------------------------------------------
// Ghost fill with the result of an x, then y (over the full x extent), then z
// (over the full x-y extent) sequential fill: periodic wrap, zero-gradient
// outflow, fixed faces untouched.  A fixed face with a free radiation flux
// (kind 3) is fixed for every variable except F_x, F_y, F_z of a 4-variable
// (radiation) state, which it fills as outflow.  Sources are never written by
// the same launch (their first out-of-range axis in z, y, x order is a fixed
// face), so one launch fills all ghosts without ordering.
// ---------------------------------------------------------------------------
struct GhostBC {
  int lo[3], hi[3];
  int any_ff;  // some face is of kind 3
};

__device__ __forceinline__ int map_index(int i, int n, int lo, int hi) {
  if (i < 0) return lo == 0 ? ((i % n) + n) % n : (lo == 1 ? 0 : i);
  if (i >= n) return hi == 0 ? i % n : (hi == 1 ? n - 1 : i);
  return i;
}

// The ghost shell of a box as one index range [0, ghost_count): the two z
// slabs (all x and y), then the two y slabs (interior z), then the two x
// slabs (interior y and z); ghost_cell decodes an index into (i, j, k).
__host__ __device__ __forceinline__ int64_t ghost_count(const DevBox& b) {
  const int64_t NX = b.n0 + 2 * b.ng, NY = b.n1 + 2 * b.ng;
  return 2 * b.ng * (NY * NX + (int64_t)b.n2 * NX + (int64_t)b.n2 * b.n1);
}

// The same in 32-bit arithmetic, for boxes with fewer than 2^31 ghost cells
// (64-bit division is a long instruction sequence on the GPU).
__device__ __forceinline__ void ghost_cell32(const DevBox& b, uint32_t c, int& i, int& j, int& k) {
  const int ng = b.ng;
  const uint32_t NX = b.n0 + 2 * ng, NY = b.n1 + 2 * ng, G = 2 * ng;
  const uint32_t nz_slab = G * NY * NX, ny_slab = G * (uint32_t)b.n2 * NX;
  if (c < nz_slab) {
    const uint32_t q = c / NX, kk = q / NY;
    i = (int)(c - q * NX) - ng;
    j = (int)(q - kk * NY) - ng;
    k = (int)kk < ng ? (int)kk - ng : b.n2 + ((int)kk - ng);
  } else if (c < nz_slab + ny_slab) {
    const uint32_t r = c - nz_slab, q = r / NX, kq = q / G;
    i = (int)(r - q * NX) - ng;
    const int jj = (int)(q - kq * G);
    k = (int)kq;
    j = jj < ng ? jj - ng : b.n1 + (jj - ng);
  } else {
    const uint32_t r = c - nz_slab - ny_slab, q = r / G, kq = q / (uint32_t)b.n1;
    const int ii = (int)(r - q * G);
    j = (int)(q - kq * (uint32_t)b.n1);
    k = (int)kq;
    i = ii < ng ? ii - ng : b.n0 + (ii - ng);
  }
}

__device__ __forceinline__ void ghost_cell(const DevBox& b, int64_t c, int& i, int& j, int& k) {
  const int ng = b.ng;
  const int NX = b.n0 + 2 * ng, NY = b.n1 + 2 * ng;
  const int64_t nz_slab = (int64_t)2 * ng * NY * NX;
  const int64_t ny_slab = (int64_t)2 * ng * b.n2 * NX;
  if (c < nz_slab) {
    i = (int)(c % NX) - ng;
    j = (int)((c / NX) % NY) - ng;
    const int kk = (int)(c / ((int64_t)NX * NY));
    k = kk < ng ? kk - ng : b.n2 + (kk - ng);
  } else if (c < nz_slab + ny_slab) {
    const int64_t r = c - nz_slab;
    i = (int)(r % NX) - ng;
    const int jj = (int)((r / NX) % (2 * ng));
    k = (int)(r / ((int64_t)NX * 2 * ng));
    j = jj < ng ? jj - ng : b.n1 + (jj - ng);
  } else {
    const int64_t r = c - nz_slab - ny_slab;
    const int ii = (int)(r % (2 * ng));
    j = (int)((r / (2 * ng)) % b.n1);
    k = (int)(r / ((int64_t)2 * ng * b.n1));
    i = ii < ng ? ii - ng : b.n0 + (ii - ng);
  }
}

// Source cell of ghost (i, j, k), or false if the fill leaves it as it is.
// The x, y, z sequential fill writes a ghost cell in the fill of the last axis
// (in x, y, z order) along which it lies outside; a fixed face there leaves
// it as it is.  Its value comes from the cell mapped along that axis, which in
// turn was filled by the previous axes: map z, then y, then x, stopping at the
// first fixed face met.  free_flux: kind 3 acts as outflow (else as fixed).
__device__ __forceinline__ bool ghost_src(const DevBox& b, const GhostBC& bc, bool free_flux, int i, int j, int k,
                                          int64_t& src) {
  auto kind = [&](int kd) { return kd == 3 ? (free_flux ? 1 : 2) : kd; };
  int si = i, sj = j, sk = k;
  bool stop = false;
  if (k < 0 || k >= b.n2) {
    const int lo = kind(bc.lo[2]), hi = kind(bc.hi[2]);
    if ((k < 0 ? lo : hi) == 2) stop = true; else sk = map_index(k, b.n2, lo, hi);
  }
  if (!stop && (j < 0 || j >= b.n1)) {
    const int lo = kind(bc.lo[1]), hi = kind(bc.hi[1]);
    if ((j < 0 ? lo : hi) == 2) stop = true; else sj = map_index(j, b.n1, lo, hi);
  }
  if (!stop && (i < 0 || i >= b.n0)) {
    const int lo = kind(bc.lo[0]), hi = kind(bc.hi[0]);
    if ((i < 0 ? lo : hi) != 2) si = map_index(i, b.n0, lo, hi);
  }
  if (si == i && sj == j && sk == k) return false;
  src = cell(b, si, sj, sk);
  return true;
}

template <class S>
__device__ __forceinline__ void ghost_body(S* __restrict__ U, const DevBox& b, const GhostBC& bc, int nvar) {
  const int64_t total = ghost_count(b);
  const bool ff = bc.any_ff && nvar == 4;  // radiation flux filled on its own
  const bool small = total < ((int64_t)1 << 31);
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    int i, j, k;
    if (small)
      ghost_cell32(b, (uint32_t)c, i, j, k);
    else
      ghost_cell(b, c, i, j, k);
    const int64_t dst = cell(b, i, j, k);
    int64_t src;
    if (ghost_src(b, bc, false, i, j, k, src))
      for (int v = 0; v < (ff ? 1 : nvar); ++v) U[dst + v * b.vs] = U[src + v * b.vs];
    if (ff && ghost_src(b, bc, true, i, j, k, src))
      for (int v = 1; v < 4; ++v) U[dst + v * b.vs] = U[src + v * b.vs];
  }
}

template <class S>
__global__ __launch_bounds__(256) void ghost_kernel(S* __restrict__ U, DevBox b, GhostBC bc, int nvar) {
  ghost_body<S>(U, b, bc, nvar);
}

// Copy every ghost cell of src into dst (same layout): the stage buffer of a
// box with fixed ghosts starts from the caller's ghost data.
template <class S>
__global__ __launch_bounds__(256) void ghost_copy_kernel(S* __restrict__ dst, const S* __restrict__ src, DevBox b,
                                                         int nvar) {
  const int64_t total = ghost_count(b);
  const bool small = total < ((int64_t)1 << 31);
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    int i, j, k;
    if (small)
      ghost_cell32(b, (uint32_t)c, i, j, k);
    else
      ghost_cell(b, c, i, j, k);
    const int64_t o = cell(b, i, j, k);
    for (int v = 0; v < nvar; ++v) dst[o + v * b.vs] = src[o + v * b.vs];
  }
}

}  // namespace qk
