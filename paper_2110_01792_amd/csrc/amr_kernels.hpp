// AMR coarse-fine operations, refinement ratio 2 (Section 2.2): conservative
// average-down, conservative (MC-limited) linear interpolation onto fine cells
// with linear interpolation in time between two coarse states, and the
// level-synchronisation update of the coarse cells next to a fine region from
// the two levels' flux registers.  One thread per output cell, FP64
// arithmetic, state in S.  Memory-bound gathers over small regions.
#pragma once
#include "hydro_kernels.hpp"

namespace qk {

__device__ __forceinline__ int floor_div2(int i) { return (i >= 0) ? i / 2 : -((1 - i) / 2); }

// Coarse cell off + (I, J, K) <- mean of its 8 children, for the coarse cells
// under the fine interior.
template <class S>
__global__ __launch_bounds__(256) void average_down_kernel(const S* __restrict__ Uf, DevBox fb, S* __restrict__ Uc,
                                                           DevBox cb, int o0, int o1, int o2, int nvar) {
  const int m0 = fb.n0 / 2, m1 = fb.n1 / 2, m2 = fb.n2 / 2;
  const int64_t total = (int64_t)m0 * m1 * m2 * nvar;
  const bool small = total < ((int64_t)1 << 31);  // 32-bit index arithmetic (64-bit division is long)
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    int I, J, K, v;
    if (small) {
      const uint32_t u = (uint32_t)c, q0 = u / (uint32_t)m0, q1 = q0 / (uint32_t)m1, q2 = q1 / (uint32_t)m2;
      I = (int)(u - q0 * (uint32_t)m0);
      J = (int)(q0 - q1 * (uint32_t)m1);
      K = (int)(q1 - q2 * (uint32_t)m2);
      v = (int)q2;
    } else {
      I = (int)(c % m0), J = (int)((c / m0) % m1), K = (int)((c / ((int64_t)m0 * m1)) % m2);
      v = (int)(c / ((int64_t)m0 * m1 * m2));
    }
    const S* f = Uf + (int64_t)v * fb.vs;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += double(f[cell(fb, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), 2 * K + (q >> 2))]);
    Uc[(int64_t)v * cb.vs + cell(cb, o0 + I, o1 + J, o2 + K)] = S(s / 8.0);
  }
}

// Fine cells (ghost layers only, or the whole ghosted box) from the coarse
// state (1 - alpha) U0 + alpha U1: parent value plus a quarter of the
// MC-limited slope per axis toward the child's side (keeps the parent's mean).
template <class S>
__global__ __launch_bounds__(256) void prolong_kernel(const S* __restrict__ U0, const S* __restrict__ U1, double alpha,
                                                      DevBox cb, S* __restrict__ Uf, DevBox fb, int o0, int o1, int o2,
                                                      int nvar, int interior) {
  // index range per variable: the whole ghosted box, or its ghost shell only
  const int ng = fb.ng;
  const int NX = fb.n0 + 2 * ng, NY = fb.n1 + 2 * ng, NZ = fb.n2 + 2 * ng;
  const int64_t per_v = interior ? (int64_t)NX * NY * NZ : ghost_count(fb);
  const int64_t total = per_v * nvar;
  const bool small = total < ((int64_t)1 << 31);  // 32-bit index arithmetic (64-bit division is long)
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    int v, i, j, k;
    if (small) {
      const uint32_t u = (uint32_t)c, pv = (uint32_t)per_v, qv = u / pv, r = u - qv * pv;
      v = (int)qv;
      if (interior) {
        const uint32_t q0 = r / (uint32_t)NX, q1 = q0 / (uint32_t)NY;
        i = (int)(r - q0 * (uint32_t)NX) - ng;
        j = (int)(q0 - q1 * (uint32_t)NY) - ng;
        k = (int)q1 - ng;
      } else {
        ghost_cell32(fb, r, i, j, k);
      }
    } else {
      v = (int)(c / per_v);
      const int64_t r = c - (int64_t)v * per_v;
      if (interior) {
        i = (int)(r % NX) - ng;
        j = (int)((r / NX) % NY) - ng;
        k = (int)(r / ((int64_t)NX * NY)) - ng;
      } else {
        ghost_cell(fb, r, i, j, k);
      }
    }
    const int P[3] = {o0 + floor_div2(i), o1 + floor_div2(j), o2 + floor_div2(k)};
    const int f[3] = {i, j, k};
    const S* a0 = U0 + (int64_t)v * cb.vs;
    const S* a1 = U1 + (int64_t)v * cb.vs;
    auto qc = [&](int x, int y, int z) {
      const int64_t o = cell(cb, x, y, z);
      return (1.0 - alpha) * double(a0[o]) + alpha * double(a1[o]);
    };
    const double q = qc(P[0], P[1], P[2]);
    double u = q;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double qm = qc(P[0] - (d == 0), P[1] - (d == 1), P[2] - (d == 2));
      const double qp = qc(P[0] + (d == 0), P[1] + (d == 1), P[2] + (d == 2));
      const double dl = q - qm, dr = qp - q, dc = qp - qm;
      double s = 0.0;
      if (dl * dr > 0.0) {
        s = fmin(fmin(2.0 * fabs(dl), 2.0 * fabs(dr)), 0.5 * fabs(dc));
        if (dc < 0.0) s = -s;
      }
      u += ((f[d] & 1) ? 0.25 : -0.25) * s;
    }
    Uf[(int64_t)v * fb.vs + cell(fb, i, j, k)] = S(u);
  }
}

// Coarse cells just outside region [lo, hi) (the fine box's footprint): each
// gains +-(coarse register - area mean of the 4 fine register faces) / dx
// (+ through the region's low face, which is the outside cell's right face;
// - through the high face).  One thread per (axis, side, face, variable).
template <class S>
__global__ __launch_bounds__(256) void reflux_kernel(S* __restrict__ Uc, DevBox cb, const double* __restrict__ rc,
                                                     const double* __restrict__ rf, int l0, int l1, int l2, int h0,
                                                     int h1, int h2, int nvar) {
  const int lo[3] = {l0, l1, l2}, hi[3] = {h0, h1, h2};
  const int m0 = h0 - l0, m1 = h1 - l1, m2 = h2 - l2;
  const int flo[3] = {0, 0, 0}, fhi[3] = {2 * m0, 2 * m1, 2 * m2};
  const int64_t nface[3] = {(int64_t)m1 * m2, (int64_t)m0 * m2, (int64_t)m0 * m1};
  const int64_t per_v = 2 * (nface[0] + nface[1] + nface[2]);
  const int64_t total = per_v * nvar;
  const double dxs[3] = {cb.dx0, cb.dx1, cb.dx2};
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < total; c += (int64_t)gridDim.x * 256) {
    const int v = (int)(c / per_v);
    int64_t r = c % per_v;
    int d = 0;
    while (r >= 2 * nface[d]) {
      r -= 2 * nface[d];
      ++d;
    }
    const int side = (int)(r / nface[d]);
    const int64_t e = r % nface[d];
    // in-plane coarse indices (a slower, b faster) of this face
    const int mb = d == 0 ? m1 : m0;
    const int A = (int)(e / mb), B = (int)(e % mb);
    const double cval = rc[reg_slot(lo, hi, d, v, side, A, B, nvar)];
    double fs = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) fs += rf[reg_slot(flo, fhi, d, v, side, 2 * A + (q >> 1), 2 * B + (q & 1), nvar)];
    const double corr = (side ? -1.0 : 1.0) * (cval - fs / 4.0) / dxs[d];
    int x[3];
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    x[d] = side ? hi[d] : lo[d] - 1;
    x[d1] = lo[d1] + B;
    x[d2] = lo[d2] + A;
    const int64_t o = (int64_t)v * cb.vs + cell(cb, x[0], x[1], x[2]);
    Uc[o] = S(double(Uc[o]) + corr);
  }
}

}  // namespace qk
