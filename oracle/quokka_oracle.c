/*
 * Plain FP64 CPU oracle of the QUOKKA per-cell update (Wibking & Krumholz 2021,
 * arXiv:2110.01792).  TEST INFRASTRUCTURE ONLY: the reference that the GPU
 * library is checked against.  It shares no code with the GPU path.
 *
 * Every stage is written as whole-array passes in the order the paper gives:
 * conserved -> primitive, shock flattening, PPM (or PLM) per direction, Riemann flux
 * per face, unsplit divergence, SSP-RK2 combination.  No blocking, fusion or
 * reordering.  Compile with -O2 -ffp-contract=off -fno-fast-math.
 *
 * One exact shortcut is taken: an axis with a single interior cell and
 * non-fixed boundaries has ghost cells that are copies of that cell, so its
 * two face fluxes are computed from identical inputs and cancel exactly, and
 * its flattening coefficient is exactly 1.  Such an axis is skipped ("inactive"),
 * which lets one-dimensional tests run in a 3D box at 1D cost.
 *
 * Parity pins are in tests/test_oracle_*.py; see the header of each function for
 * the passage it follows.
 */
#include "quokka_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* geometry                                                                  */
/* ------------------------------------------------------------------------ */
typedef struct {
  int n[3], ng, N[3];
  size_t vs;          /* elements per variable */
  ptrdiff_t st[3];    /* element stride per axis */
  int act[3];         /* axis active (see file header) */
  int lo[3], hi[3];   /* cell range where primitives are formed */
} geo;

static geo make_geo(const ob_box* b) {
  geo g;
  g.ng = b->ng;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = b->n[d];
    g.N[d] = b->n[d] + 2 * b->ng;
    g.act[d] = !(b->n[d] == 1 && b->bc[d][0] < OB_FIXED && b->bc[d][1] < OB_FIXED);
    g.lo[d] = g.act[d] ? -b->ng : 0;
    g.hi[d] = g.act[d] ? b->n[d] + b->ng : b->n[d];
  }
  g.st[0] = 1;
  g.st[1] = g.N[0];
  g.st[2] = (ptrdiff_t)g.N[0] * g.N[1];
  g.vs = (size_t)g.N[0] * g.N[1] * g.N[2];
  return g;
}

static inline size_t IX(const geo* g, int i, int j, int k) {
  return ((size_t)(k + g->ng) * g->N[1] + (size_t)(j + g->ng)) * g->N[0] + (size_t)(i + g->ng);
}

int oracle_set_threads(int n) {
#ifdef _OPENMP
  /* n <= 0 restores the process default (OMP_NUM_THREADS, else all cores) */
  static int dflt = 0;
  if (dflt == 0) dflt = omp_get_max_threads();
  omp_set_num_threads(n > 0 ? n : dflt);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* boundary conditions: periodic wrap, zero-gradient outflow, fixed          */
/* Filled axis by axis (x, then y over the full x extent, then z over the    */
/* full x-y extent), which also fills edges and corners.  A fixed face with  */
/* a free radiation flux acts as outflow for F_x, F_y, F_z of a radiation     */
/* state (4 variables) and as fixed everywhere else.                          */
/* ------------------------------------------------------------------------ */
static int src_index(int i, int n, int bclo, int bchi) {
  if (i < 0) {
    if (bclo == OB_PERIODIC) return ((i % n) + n) % n;
    if (bclo == OB_OUTFLOW) return 0;
    return i;
  }
  if (i >= n) {
    if (bchi == OB_PERIODIC) return i % n;
    if (bchi == OB_OUTFLOW) return n - 1;
    return i;
  }
  return i;
}

static int kind_for(int kind, int v, int nvar) {
  if (kind != OB_FIXED_FREE_FLUX) return kind;
  return (nvar == 4 && v >= 1) ? OB_OUTFLOW : OB_FIXED;
}

void oracle_fill_ghosts(const ob_box* b, double* U, int nvar) {
  geo g = make_geo(b);
  const int ng = g.ng;
  for (int v = 0; v < nvar; ++v) {
    double* q = U + (size_t)v * g.vs;
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = kind_for(b->bc[d][0], v, nvar);
      hi[d] = kind_for(b->bc[d][1], v, nvar);
    }
    /* x */
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = -ng; i < g.n[0] + ng; ++i) {
          if (i >= 0 && i < g.n[0]) continue;
          int s = src_index(i, g.n[0], lo[0], hi[0]);
          if (s != i) q[IX(&g, i, j, k)] = q[IX(&g, s, j, k)];
        }
    /* y, over full x extent */
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = -ng; j < g.n[1] + ng; ++j) {
        if (j >= 0 && j < g.n[1]) continue;
        int s = src_index(j, g.n[1], lo[1], hi[1]);
        if (s == j) continue;
        for (int i = -ng; i < g.n[0] + ng; ++i) q[IX(&g, i, j, k)] = q[IX(&g, i, s, k)];
      }
    /* z, over full x-y extent */
    for (int k = -ng; k < g.n[2] + ng; ++k) {
      if (k >= 0 && k < g.n[2]) continue;
      int s = src_index(k, g.n[2], lo[2], hi[2]);
      if (s == k) continue;
      for (int j = -ng; j < g.n[1] + ng; ++j)
        for (int i = -ng; i < g.n[0] + ng; ++i) q[IX(&g, i, j, k)] = q[IX(&g, i, j, s)];
    }
  }
}

/* ------------------------------------------------------------------------ */
/* PPM reconstruction of one cell (Section 2.2.1, reconstruction paragraphs). */
/* q[0..4] = cell averages at offsets -2..+2 along the axis.                 */
/*  1. fourth-order interface values, terms grouped symmetrically about the  */
/*     interface (sums of the two symmetric pairs first);                    */
/*  2. clamp each interface value to [min, max] of the cell and its two      */
/*     neighbours;                                                           */
/*  3. CW84 extremum test; on an extremum fall back to a linear profile with */
/*     the monotonized-central slope;                                        */
/*  4. otherwise CW84 overshoot correction on the affected side.             */
/* ------------------------------------------------------------------------ */
static void ppm(double qm2, double qm1, double q0, double qp1, double qp2, double* aL, double* aR) {
  double fl = (7.0 / 12.0) * (qm1 + q0) - (1.0 / 12.0) * (qm2 + qp1);
  double fr = (7.0 / 12.0) * (q0 + qp1) - (1.0 / 12.0) * (qm1 + qp2);
  double lo = fmin(qm1, fmin(q0, qp1));
  double hi = fmax(qm1, fmax(q0, qp1));
  fl = fmin(fmax(fl, lo), hi);
  fr = fmin(fmax(fr, lo), hi);
  if ((fr - q0) * (q0 - fl) <= 0.0) {
    double dl = q0 - qm1, dr = qp1 - q0, dc = qp1 - qm1;
    double s = 0.0;
    if (dr * dl > 0.0) {
      s = fmin(fmin(2.0 * fabs(dr), 2.0 * fabs(dl)), 0.5 * fabs(dc));
      if (dc < 0.0) s = -s;
    }
    fl = q0 - 0.5 * s;
    fr = q0 + 0.5 * s;
  } else {
    double del = fr - fl;
    double a6 = 6.0 * (q0 - 0.5 * (fl + fr));
    if (del * a6 > del * del)
      fl = 3.0 * q0 - 2.0 * fr;
    else if (del * a6 < -(del * del))
      fr = 3.0 * q0 - 2.0 * fl;
  }
  *aL = fl;
  *aR = fr;
}

void oracle_ppm_cell(const double q[5], double out[2]) { ppm(q[0], q[1], q[2], q[3], q[4], &out[0], &out[1]); }

/* PLM with the monotonized-central slope limiter (Section 2.2.1, the
 * compile-time alternative to PPM; van Leer 1977): slope 0 at an extremum of
 * the cell averages, else sign(dc) min(2|dr|, 2|dl|, |dc|/2); interface values
 * q -+ slope/2. */
static void plm(double qm1, double q0, double qp1, double* aL, double* aR) {
  const double dl = q0 - qm1, dr = qp1 - q0, dc = qp1 - qm1;
  double s = 0.0;
  if (dr * dl > 0.0) {
    s = fmin(fmin(2.0 * fabs(dr), 2.0 * fabs(dl)), 0.5 * fabs(dc));
    if (dc < 0.0) s = -s;
  }
  *aL = q0 - 0.5 * s;
  *aR = q0 + 0.5 * s;
}

void oracle_plm_cell(const double q[3], double out[2]) { plm(q[0], q[1], q[2], &out[0], &out[1]); }

static void reconstruct(int recon, const double* q, size_t o, ptrdiff_t s, double* l, double* r) {
  if (recon == 1)
    plm(q[o - s], q[o], q[o + s], l, r);
  else
    ppm(q[o - 2 * s], q[o - s], q[o], q[o + s], q[o + 2 * s], l, r);
}

/* ------------------------------------------------------------------------ */
/* HLLC flux with PVRS wave-speed estimates (Section 2.2.1, Riemann solver   */
/* paragraph; Toro 2013 ch. 10).  States are primitive and rotated so that   */
/* index 1 is the face-normal velocity.  The star state is grouped so that a */
/* stationary contact is preserved exactly, and the two tangential speeds    */
/* enter the kinetic energy as one symmetric pair, so relabelling x and y    */
/* changes no bit of any flux.                                               */
/* ------------------------------------------------------------------------ */
void oracle_hllc(const double WL[5], const double WR[5], double g, double F[5]) {
  const double rL = WL[0], uL = WL[1], vL = WL[2], wL = WL[3], pL = WL[4];
  const double rR = WR[0], uR = WR[1], vR = WR[2], wR = WR[3], pR = WR[4];
  const double cL = sqrt(g * pL / rL);
  const double cR = sqrt(g * pR / rR);
  const double EL = pL / (g - 1.0) + 0.5 * rL * (uL * uL + (vL * vL + wL * wL));
  const double ER = pR / (g - 1.0) + 0.5 * rR * (uR * uR + (vR * vR + wR * wR));
  const double rbar = 0.5 * (rL + rR);
  const double cbar = 0.5 * (cL + cR);
  const double pstar = fmax(0.0, 0.5 * (pL + pR) - 0.5 * (uR - uL) * rbar * cbar);
  const double qL = (pstar <= pL) ? 1.0 : sqrt(1.0 + ((g + 1.0) / (2.0 * g)) * (pstar / pL - 1.0));
  const double qR = (pstar <= pR) ? 1.0 : sqrt(1.0 + ((g + 1.0) / (2.0 * g)) * (pstar / pR - 1.0));
  const double SL = uL - cL * qL;
  const double SR = uR + cR * qR;
  const double Ss = ((pR - pL) + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                    (rL * (SL - uL) - rR * (SR - uR));

  const double FL[5] = {rL * uL, rL * uL * uL + pL, rL * uL * vL, rL * uL * wL, uL * (EL + pL)};
  const double FR[5] = {rR * uR, rR * uR * uR + pR, rR * uR * vR, rR * uR * wR, uR * (ER + pR)};

  if (0.0 <= SL) {
    for (int n = 0; n < 5; ++n) F[n] = FL[n];
  } else if (0.0 <= Ss) {
    const double UL[5] = {rL, rL * uL, rL * vL, rL * wL, EL};
    const double ph = (SL - uL) / (SL - Ss);
    const double Us[5] = {ph * rL, ph * (rL * Ss), ph * (rL * vL), ph * (rL * wL),
                          ph * (EL + (Ss - uL) * (rL * Ss + pL / (SL - uL)))};
    for (int n = 0; n < 5; ++n) F[n] = FL[n] + SL * (Us[n] - UL[n]);
  } else if (0.0 < SR) {
    const double UR[5] = {rR, rR * uR, rR * vR, rR * wR, ER};
    const double ph = (SR - uR) / (SR - Ss);
    const double Us[5] = {ph * rR, ph * (rR * Ss), ph * (rR * vR), ph * (rR * wR),
                          ph * (ER + (Ss - uR) * (rR * Ss + pR / (SR - uR)))};
    for (int n = 0; n < 5; ++n) F[n] = FR[n] + SR * (Us[n] - UR[n]);
  } else {
    for (int n = 0; n < 5; ++n) F[n] = FR[n];
  }
}

/* ------------------------------------------------------------------------ */
/* Hydrodynamic right-hand side L(U) (Section 2.2.1).                        */
/* ------------------------------------------------------------------------ */
static void to_prim(const double* U, size_t vs, size_t o, double g, double W[5]) {
  const double rho = U[o], mx = U[vs + o], my = U[2 * vs + o], mz = U[3 * vs + o], E = U[4 * vs + o];
  const double ek = 0.5 * ((mx * mx + my * my) + mz * mz) / rho;
  W[0] = rho;
  W[1] = mx / rho;
  W[2] = my / rho;
  W[3] = mz / rho;
  W[4] = (g - 1.0) * (E - ek);
}

/* Flattening coefficient of one cell along one axis before the neighbour
 * minimum (Miller & Colella 2002 generalisation of CW84, constants of CW84). */
static double chi_tilde(const double* P, const double* u, size_t o, ptrdiff_t s) {
  const double dp1 = P[o + s] - P[o - s];
  const double dp2 = P[o + 2 * s] - P[o - 2 * s];
  const double du = u[o + s] - u[o - s];
  const int shock = (fabs(dp1) > 0.33 * fmin(P[o + s], P[o - s])) && (du < 0.0);
  if (!shock) return 1.0;
  const double z = fabs(dp1) / fmax(fabs(dp2), 1e-300);
  return fmin(1.0, fmax(0.0, 1.0 - (z - 0.75) / (0.85 - 0.75)));
}

#define LOOP3(K0, K1, J0, J1, I0, I1)                               \
  _Pragma("omp parallel for collapse(2) schedule(static)")          \
  for (int k = (K0); k < (K1); ++k)                                 \
    for (int j = (J0); j < (J1); ++j)                               \
      for (int i = (I0); i < (I1); ++i)

/* Shock flattening (Section 2.2.1; CW84 with the multidimensional extension
 * of Miller & Colella 2002): per-axis coefficient chi_tilde over the cells
 * whose +-2 neighbours exist, the minimum with the neighbour toward the
 * higher pressure, then the minimum over axes, for cells [-1, n] of every
 * active axis.  W holds the primitive variables (P in W[4]). */
static void flatten_coeffs(const geo* g, const double* W, double* cht, double* chi) {
  const size_t vs = g->vs;
  const double* P = W + 4 * vs;
  for (int d = 0; d < 3; ++d) {
    double* c = cht + d * vs;
    if (!g->act[d]) continue;
    int lo[3] = {g->lo[0], g->lo[1], g->lo[2]}, hi[3] = {g->hi[0], g->hi[1], g->hi[2]};
    lo[d] += 2;
    hi[d] -= 2;
    const double* u = W + (1 + d) * vs;
    LOOP3(lo[2], hi[2], lo[1], hi[1], lo[0], hi[0]) {
      const size_t o = IX(g, i, j, k);
      c[o] = chi_tilde(P, u, o, g->st[d]);
    }
  }
  {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = g->act[d] ? -1 : 0;
      hi[d] = g->act[d] ? g->n[d] + 1 : g->n[d];
    }
    LOOP3(lo[2], hi[2], lo[1], hi[1], lo[0], hi[0]) {
      const size_t o = IX(g, i, j, k);
      double x = 1.0;
      for (int d = 0; d < 3; ++d) {
        if (!g->act[d]) continue;
        const ptrdiff_t s = g->st[d];
        const double dp1 = P[o + s] - P[o - s];
        const ptrdiff_t sh = (dp1 > 0.0) ? s : -s;
        const double* c = cht + d * vs;
        x = fmin(x, fmin(c[o], c[o + sh]));
      }
      chi[o] = x;
    }
  }
}

/* The flattening coefficient chi of Section 2.2.1 for every cell of the box
 * grown by one cell along each active axis (0 elsewhere), from the
 * conserved state U (ghosts filled). */
void oracle_flatten_chi(const ob_box* b, const double* U, double gam, double* chi) {
  geo g = make_geo(b);
  const size_t vs = g.vs;
  double* W = (double*)calloc(5 * vs, sizeof(double));
  double* cht = (double*)calloc(3 * vs, sizeof(double));
  memset(chi, 0, vs * sizeof(double));
  LOOP3(g.lo[2], g.hi[2], g.lo[1], g.hi[1], g.lo[0], g.hi[0]) {
    const size_t o = IX(&g, i, j, k);
    double w[5];
    to_prim(U, vs, o, gam, w);
    for (int v = 0; v < 5; ++v) W[v * vs + o] = w[v];
  }
  flatten_coeffs(&g, W, cht, chi);
  free(W);
  free(cht);
}

static void record_region(const geo* g, const double* Fd, int nvar, const ob_region* r, double* reg, double w);

static void hydro_rhs(const ob_box* b, const double* U, double gam, int recon, double* L, ob_stats* st,
                      const ob_region* r, double* reg, double w);

void oracle_hydro_rhs(const ob_box* b, const double* U, double gam, int recon, double* L, ob_stats* st) {
  hydro_rhs(b, U, gam, recon, L, st, NULL, NULL, 0.0);
}

static void hydro_rhs(const ob_box* b, const double* U, double gam, int recon, double* L, ob_stats* st,
                      const ob_region* r, double* reg, double w) {
  geo g = make_geo(b);
  const size_t vs = g.vs;
  double* W = (double*)malloc(5 * vs * sizeof(double));
  double* cht = (double*)malloc(3 * vs * sizeof(double));
  double* chi = (double*)malloc(vs * sizeof(double));
  double* aL = (double*)malloc(5 * vs * sizeof(double));
  double* aR = (double*)malloc(5 * vs * sizeof(double));
  double* Fd = (double*)malloc(3 * 5 * vs * sizeof(double));
  int64_t neg = 0;

  /* 1. conserved -> primitive */
  LOOP3(g.lo[2], g.hi[2], g.lo[1], g.hi[1], g.lo[0], g.hi[0]) {
    const size_t o = IX(&g, i, j, k);
    double w[5];
    to_prim(U, vs, o, gam, w);
    for (int v = 0; v < 5; ++v) W[v * vs + o] = w[v];
  }
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const size_t o = IX(&g, i, j, k);
        if (!(W[o] > 0.0) || !(W[4 * vs + o] > 0.0)) ++neg;
      }

  /* 2. shock flattening */
  flatten_coeffs(&g, W, cht, chi);

  /* 3-4. per axis: PPM of (rho, vx, vy, vz, P) with flattening, then HLLC at
   *      every face.  Face c-1/2 is stored at cell c. */
  for (int d = 0; d < 3; ++d) {
    double* F = Fd + (size_t)d * 5 * vs;
    if (!g.act[d]) continue;
    const ptrdiff_t s = g.st[d];
    int lo[3] = {0, 0, 0}, hi[3] = {g.n[0], g.n[1], g.n[2]};
    lo[d] = -1;
    hi[d] = g.n[d] + 1;
    LOOP3(lo[2], hi[2], lo[1], hi[1], lo[0], hi[0]) {
      const size_t o = IX(&g, i, j, k);
      const double x = chi[o];
      for (int v = 0; v < 5; ++v) {
        const double* q = W + v * vs;
        double l, r;
        reconstruct(recon, q, o, s, &l, &r);
        aL[v * vs + o] = x * l + (1.0 - x) * q[o];
        aR[v * vs + o] = x * r + (1.0 - x) * q[o];
      }
    }
    int lo2[3] = {0, 0, 0}, hi2[3] = {g.n[0], g.n[1], g.n[2]};
    hi2[d] = g.n[d] + 1;
    /* rotation: normal velocity first, then the two tangential ones */
    const int t1 = (d == 0) ? 2 : 1;
    const int t2 = (d == 2) ? 2 : 3;
    const int nv = 1 + d;
    LOOP3(lo2[2], hi2[2], lo2[1], hi2[1], lo2[0], hi2[0]) {
      const size_t o = IX(&g, i, j, k);
      const size_t ol = o - s;
      const double WLr[5] = {aR[ol], aR[nv * vs + ol], aR[t1 * vs + ol], aR[t2 * vs + ol], aR[4 * vs + ol]};
      const double WRr[5] = {aL[o], aL[nv * vs + o], aL[t1 * vs + o], aL[t2 * vs + o], aL[4 * vs + o]};
      double f[5];
      oracle_hllc(WLr, WRr, gam, f);
      F[0 * vs + o] = f[0];
      F[nv * vs + o] = f[1];
      F[t1 * vs + o] = f[2];
      F[t2 * vs + o] = f[3];
      F[4 * vs + o] = f[4];
    }
  }

  /* 5. unsplit divergence, x and y first so that the two are symmetric */
  LOOP3(0, g.n[2], 0, g.n[1], 0, g.n[0]) {
    const size_t o = IX(&g, i, j, k);
    for (int v = 0; v < 5; ++v) {
      double t[3];
      for (int d = 0; d < 3; ++d) {
        if (!g.act[d]) {
          t[d] = 0.0;
          continue;
        }
        const double* F = Fd + (size_t)d * 5 * vs + v * vs;
        t[d] = (F[o + g.st[d]] - F[o]) / b->dx[d];
      }
      L[v * vs + o] = -((t[0] + t[1]) + t[2]);
    }
  }
  if (reg) record_region(&g, Fd, 5, r, reg, w);
  if (st) st->neg_cells += neg;
  free(W);
  free(cht);
  free(chi);
  free(aL);
  free(aR);
  free(Fd);
}

/* Add w * F at every face on the boundary of region r (face c-1/2 of axis d
 * is stored at cell c in Fd, nvar variables per axis). */
static void record_region(const geo* g, const double* Fd, int nvar, const ob_region* r, double* reg, double w) {
  const int m0 = r->hi[0] - r->lo[0], m1 = r->hi[1] - r->lo[1], m2 = r->hi[2] - r->lo[2];
  const size_t nx = (size_t)2 * m1 * m2, ny = (size_t)2 * m0 * m2;
  /* axes skipped as inactive (one cell, non-fixed) carry no fluxes here */
  if (!g->act[0] || !g->act[1] || !g->act[2]) return;
  double* rx = reg;
  double* ry = reg + nvar * nx;
  double* rz = reg + nvar * (nx + ny);
  for (int v = 0; v < nvar; ++v)
    for (int side = 0; side < 2; ++side) {
      const int fx = side ? r->hi[0] : r->lo[0], fy = side ? r->hi[1] : r->lo[1], fz = side ? r->hi[2] : r->lo[2];
      for (int k = r->lo[2]; k < r->hi[2]; ++k)
        for (int j = r->lo[1]; j < r->hi[1]; ++j)
          rx[((size_t)(v * 2 + side) * m2 + (k - r->lo[2])) * m1 + (j - r->lo[1])] +=
              w * Fd[(size_t)(0 * nvar + v) * g->vs + IX(g, fx, j, k)];
      for (int k = r->lo[2]; k < r->hi[2]; ++k)
        for (int i = r->lo[0]; i < r->hi[0]; ++i)
          ry[((size_t)(v * 2 + side) * m2 + (k - r->lo[2])) * m0 + (i - r->lo[0])] +=
              w * Fd[(size_t)(1 * nvar + v) * g->vs + IX(g, i, fy, k)];
      for (int j = r->lo[1]; j < r->hi[1]; ++j)
        for (int i = r->lo[0]; i < r->hi[0]; ++i)
          rz[((size_t)(v * 2 + side) * m1 + (j - r->lo[1])) * m0 + (i - r->lo[0])] +=
              w * Fd[(size_t)(2 * nvar + v) * g->vs + IX(g, i, j, fz)];
    }
}

/* ------------------------------------------------------------------------ */
/* Time step (Section 2.2.1, eqs. for |lambda| and Delta t): the CFL number  */
/* multiplies min(dx) / max over interior cells of (|v| + c_s).              */
/* ------------------------------------------------------------------------ */
double oracle_hydro_max_signal(const ob_box* b, const double* U, double gam) {
  geo g = make_geo(b);
  double smax = 0.0;
#pragma omp parallel for collapse(2) reduction(max : smax)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        double w[5];
        to_prim(U, g.vs, IX(&g, i, j, k), gam, w);
        const double vv = sqrt((w[1] * w[1] + w[2] * w[2]) + w[3] * w[3]);
        const double cs = sqrt(gam * w[4] / w[0]);
        const double s = vv + cs;
        if (s > smax) smax = s;
      }
  return smax;
}

static double dx_min(const ob_box* b) {
  double m = b->dx[0];
  for (int d = 1; d < 3; ++d)
    if (b->dx[d] < m) m = b->dx[d];
  return m;
}

/* One SSP-RK2 step (Shu & Osher 1988): U1 = U + dt L(U);
 * U <- 0.5 U + 0.5 (U1 + dt L(U1)); ghosts refilled after each stage. */
static void rk2_interior(const geo* g, int nvar, double* Un, const double* U1, const double* L1, double dt) {
  LOOP3(0, g->n[2], 0, g->n[1], 0, g->n[0]) {
    const size_t o = IX(g, i, j, k);
    for (int v = 0; v < nvar; ++v) {
      const size_t p = v * g->vs + o;
      Un[p] = 0.5 * Un[p] + 0.5 * (U1[p] + dt * L1[p]);
    }
  }
}

static void euler_interior(const geo* g, int nvar, const double* Un, double* U1, const double* L, double dt) {
  LOOP3(0, g->n[2], 0, g->n[1], 0, g->n[0]) {
    const size_t o = IX(g, i, j, k);
    for (int v = 0; v < nvar; ++v) {
      const size_t p = v * g->vs + o;
      U1[p] = Un[p] + dt * L[p];
    }
  }
}

static void hydro_rk2_reg(const ob_box* b, double* U, double gam, double dt, int recon, ob_stats* st,
                          const ob_region* r, double* reg, double w) {
  geo g = make_geo(b);
  const size_t nb = 5 * g.vs * sizeof(double);
  double* U1 = (double*)malloc(nb);
  double* Lb = (double*)calloc(5 * g.vs, sizeof(double));
  memcpy(U1, U, nb); /* fixed ghosts of the stage state equal those of U */
  /* U^{n+1} = U^n + dt/2 (L(U^n) + L(U^1)): each stage's fluxes enter with dt/2 */
  hydro_rhs(b, U, gam, recon, Lb, st, r, reg, 0.5 * dt * w);
  euler_interior(&g, 5, U, U1, Lb, dt);
  oracle_fill_ghosts(b, U1, 5);
  hydro_rhs(b, U1, gam, recon, Lb, st, r, reg, 0.5 * dt * w);
  rk2_interior(&g, 5, U, U1, Lb, dt);
  oracle_fill_ghosts(b, U, 5);
  free(U1);
  free(Lb);
}

static void hydro_rk2(const ob_box* b, double* U, double gam, double dt, int recon, ob_stats* st) {
  geo g = make_geo(b);
  const size_t nb = 5 * g.vs * sizeof(double);
  double* U1 = (double*)malloc(nb);
  double* Lb = (double*)calloc(5 * g.vs, sizeof(double));
  memcpy(U1, U, nb); /* fixed ghosts of the stage state equal those of U */
  oracle_hydro_rhs(b, U, gam, recon, Lb, st);
  euler_interior(&g, 5, U, U1, Lb, dt);
  oracle_fill_ghosts(b, U1, 5);
  oracle_hydro_rhs(b, U1, gam, recon, Lb, st);
  rk2_interior(&g, 5, U, U1, Lb, dt);
  oracle_fill_ghosts(b, U, 5);
  free(U1);
  free(Lb);
}

void oracle_hydro_step(const ob_box* b, double* U, double gam, double cfl, double dt_in, int recon, ob_stats* st) {
  oracle_fill_ghosts(b, U, 5);
  double dt = dt_in;
  if (!(dt > 0.0)) dt = cfl * dx_min(b) / oracle_hydro_max_signal(b, U, gam);
  hydro_rk2(b, U, gam, dt, recon, st);
  if (st) {
    st->dt = dt;
    st->nsub = 0;
  }
}

void oracle_hydro_step_reg(const ob_box* b, double* U, double gam, double cfl, double dt_in, int recon,
                           const ob_region* r, double* reg, double weight, ob_stats* st) {
  oracle_fill_ghosts(b, U, 5);
  double dt = dt_in;
  if (!(dt > 0.0)) dt = cfl * dx_min(b) / oracle_hydro_max_signal(b, U, gam);
  hydro_rk2_reg(b, U, gam, dt, recon, st, r, reg, weight);
  if (st) {
    st->dt = dt;
    st->nsub = 0;
  }
}

/* ------------------------------------------------------------------------ */
/* AMR coarse-fine operations, refinement ratio 2 (Section 2.2: conservative */
/* linear interpolation onto fine cells, conservative average-down, flux-     */
/* register synchronisation of the coarse cells next to the fine region).     */
/* ------------------------------------------------------------------------ */
static inline int fdiv2(int i) { return (i >= 0) ? i / 2 : -((1 - i) / 2); } /* floor(i / 2) */

void oracle_average_down(const ob_box* fine, const double* Uf, const ob_box* coarse, double* Uc,
                         const int32_t off[3], int nvar) {
  geo gf = make_geo(fine), gc = make_geo(coarse);
  for (int v = 0; v < nvar; ++v)
    for (int K = 0; K < fine->n[2] / 2; ++K)
      for (int J = 0; J < fine->n[1] / 2; ++J)
        for (int I = 0; I < fine->n[0] / 2; ++I) {
          const double* f = Uf + (size_t)v * gf.vs;
          double s = 0.0;
          for (int c = 0; c < 8; ++c) s += f[IX(&gf, 2 * I + (c & 1), 2 * J + ((c >> 1) & 1), 2 * K + (c >> 2))];
          Uc[(size_t)v * gc.vs + IX(&gc, off[0] + I, off[1] + J, off[2] + K)] = s / 8.0;
        }
}

void oracle_prolong(const ob_box* coarse, const double* Uc0, const double* Uc1, double alpha, const ob_box* fine,
                    double* Uf, const int32_t off[3], int nvar, int interior) {
  geo gf = make_geo(fine), gc = make_geo(coarse);
  const int ng = fine->ng;
  for (int v = 0; v < nvar; ++v) {
    const double* c0 = Uc0 + (size_t)v * gc.vs;
    const double* c1 = Uc1 + (size_t)v * gc.vs;
    for (int k = -ng; k < fine->n[2] + ng; ++k)
      for (int j = -ng; j < fine->n[1] + ng; ++j)
        for (int i = -ng; i < fine->n[0] + ng; ++i) {
          const int in = i >= 0 && i < fine->n[0] && j >= 0 && j < fine->n[1] && k >= 0 && k < fine->n[2];
          if (in && !interior) continue;
          const int P[3] = {off[0] + fdiv2(i), off[1] + fdiv2(j), off[2] + fdiv2(k)};
          const int f[3] = {i, j, k};
          /* coarse value at time (1 - alpha) t0 + alpha t1 */
          #define QC(a, b, c) ((1.0 - alpha) * c0[IX(&gc, a, b, c)] + alpha * c1[IX(&gc, a, b, c)])
          const double q = QC(P[0], P[1], P[2]);
          double u = q;
          for (int d = 0; d < 3; ++d) {
            int m[3] = {P[0], P[1], P[2]}, p[3] = {P[0], P[1], P[2]};
            m[d] -= 1;
            p[d] += 1;
            const double qm = QC(m[0], m[1], m[2]), qp = QC(p[0], p[1], p[2]);
            const double dl = q - qm, dr = qp - q, dc = qp - qm;
            double s = 0.0;
            if (dl * dr > 0.0) {
              s = fmin(fmin(2.0 * fabs(dl), 2.0 * fabs(dr)), 0.5 * fabs(dc));
              if (dc < 0.0) s = -s;
            }
            /* child centre at -1/4 (even fine index) or +1/4 (odd) of the coarse cell */
            u += ((f[d] & 1) ? 0.25 : -0.25) * s;
          }
          #undef QC
          Uf[(size_t)v * gf.vs + IX(&gf, i, j, k)] = u;
        }
  }
}

void oracle_reflux(const ob_box* coarse, double* Uc, const ob_region* r, const double* reg_c, const ob_box* fine,
                   const double* reg_f, int nvar) {
  geo gc = make_geo(coarse);
  const int m0 = r->hi[0] - r->lo[0], m1 = r->hi[1] - r->lo[1], m2 = r->hi[2] - r->lo[2];
  const int f0 = fine->n[0], f1 = fine->n[1], f2 = fine->n[2];
  const size_t cx = (size_t)2 * m1 * m2, cy = (size_t)2 * m0 * m2;
  const size_t fx = (size_t)2 * f1 * f2, fy = (size_t)2 * f0 * f2;
  for (int v = 0; v < nvar; ++v)
    for (int side = 0; side < 2; ++side) {
      /* low face: the outside cell has it as its right face, and gains
         (coarse - fine) / dx; high face: left face, gains (fine - coarse) / dx */
      const double sg = side ? -1.0 : 1.0;
      for (int K = 0; K < m2; ++K)
        for (int J = 0; J < m1; ++J) {
          const double c = reg_c[((size_t)(v * 2 + side) * m2 + K) * m1 + J];
          double fs = 0.0;
          for (int q = 0; q < 4; ++q)
            fs += reg_f[((size_t)(v * 2 + side) * f2 + 2 * K + (q >> 1)) * f1 + 2 * J + (q & 1)];
          const int I = side ? r->hi[0] : r->lo[0] - 1;
          Uc[(size_t)v * gc.vs + IX(&gc, I, r->lo[1] + J, r->lo[2] + K)] += sg * (c - fs / 4.0) / coarse->dx[0];
        }
      for (int K = 0; K < m2; ++K)
        for (int I = 0; I < m0; ++I) {
          const double c = reg_c[nvar * cx + ((size_t)(v * 2 + side) * m2 + K) * m0 + I];
          double fs = 0.0;
          for (int q = 0; q < 4; ++q)
            fs += reg_f[nvar * fx + ((size_t)(v * 2 + side) * f2 + 2 * K + (q >> 1)) * f0 + 2 * I + (q & 1)];
          const int J = side ? r->hi[1] : r->lo[1] - 1;
          Uc[(size_t)v * gc.vs + IX(&gc, r->lo[0] + I, J, r->lo[2] + K)] += sg * (c - fs / 4.0) / coarse->dx[1];
        }
      for (int J = 0; J < m1; ++J)
        for (int I = 0; I < m0; ++I) {
          const double c = reg_c[nvar * (cx + cy) + ((size_t)(v * 2 + side) * m1 + J) * m0 + I];
          double fs = 0.0;
          for (int q = 0; q < 4; ++q)
            fs += reg_f[nvar * (fx + fy) + ((size_t)(v * 2 + side) * f1 + 2 * J + (q >> 1)) * f0 + 2 * I + (q & 1)];
          const int K = side ? r->hi[2] : r->lo[2] - 1;
          Uc[(size_t)v * gc.vs + IX(&gc, r->lo[0] + I, r->lo[1] + J, K)] += sg * (c - fs / 4.0) / coarse->dx[2];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Radiation closure (Section 2.2.2, eq. M1_closure and the Levermore        */
/* Eddington factor).  fhat = |F|/(cE) is capped at 1 for the closure only. */
/* With F = 0 the direction-dependent term is dropped.                       */
/* ------------------------------------------------------------------------ */
double oracle_closure_chi(double f, int closure) {
  if (closure == 1) return 1.0 / 3.0;
  if (closure == 2) /* Minerbo (1978), polynomial form of Cernohorsky & Bludman (1994) */
    return 1.0 / 3.0 + (2.0 / 15.0) * (3.0 * f * f - f * f * f + 3.0 * f * f * f * f);
  return (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
}

void oracle_closure_pressure(double E, const double F[3], double c, int closure, double P[9]) {
  const double Fn = sqrt((F[0] * F[0] + F[1] * F[1]) + F[2] * F[2]);
  const double fh = fmin(Fn / (c * E), 1.0);
  const double chi = oracle_closure_chi(fh, closure);
  const double a = 0.5 * (1.0 - chi);
  const double bb = 0.5 * (3.0 * chi - 1.0);
  double n[3] = {0.0, 0.0, 0.0};
  if (Fn > 0.0)
    for (int i = 0; i < 3; ++i) n[i] = F[i] / Fn;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double iso = (i == j) ? a : 0.0;
      P[3 * i + j] = (Fn > 0.0) ? E * (iso + bb * n[i] * n[j]) : E * iso;
    }
}

/* HLL flux of (E_r, F) along axis dir under the reduced speed of light
 * (eqs. rad_energy, rad_flux): physical flux ((chat/c) F_d, c chat P_d*);
 * both wave speeds are +-chat * sqrt(P_dd / E), the larger of the two face
 * states, with the Eddington tensor frozen (Balsara 1999).  eps scales the
 * upwind dissipation (optical-depth correction). */
void oracle_hll_rad(double EL, const double FL[3], double ER, const double FR[3], int dir, const ob_rad* p,
                    double eps, double flux[4]) {
  double PL[9], PR[9];
  oracle_closure_pressure(EL, FL, p->c, p->closure, PL);
  oracle_closure_pressure(ER, FR, p->c, p->closure, PR);
  const double sL = sqrt(PL[4 * dir] / EL);
  const double sR = sqrt(PR[4 * dir] / ER);
  const double S = p->chat * fmax(sL, sR);
  const double cc = p->c * p->chat;
  const double ratio = p->chat / p->c;
  const double phL[4] = {ratio * FL[dir], cc * PL[3 * dir + 0], cc * PL[3 * dir + 1], cc * PL[3 * dir + 2]};
  const double phR[4] = {ratio * FR[dir], cc * PR[3 * dir + 0], cc * PR[3 * dir + 1], cc * PR[3 * dir + 2]};
  const double UL[4] = {EL, FL[0], FL[1], FL[2]};
  const double UR[4] = {ER, FR[0], FR[1], FR[2]};
  for (int n = 0; n < 4; ++n) flux[n] = 0.5 * (phL[n] + phR[n]) - 0.5 * eps * S * (UR[n] - UL[n]);
}

/* Radiation face fluxes of one stage input (Section 2.2.2): PPM (no
 * flattening) of E_r and the reduced flux f = F/(c E_r); per-face first-order
 * fallback when either reconstructed |f| exceeds 1; closure; HLL.  Fc[d]
 * carries the optical-depth factor eps = min(1, 1/tau), tau = dx kappa_R
 * (rho_L + rho_R)/2 (the paper names the correction, not its formula: a
 * reading); Fu[d] is the same flux with eps = 1.  The two are equal (the same
 * bits) at faces with tau <= 1 or with the correction off.  Fu may be NULL. */
static void rad_faces(const ob_box* b, const double* Ur, const double* Ug, const ob_rad* p, double* Fc, double* Fu,
                      ob_stats* st) {
  geo g = make_geo(b);
  const size_t vs = g.vs;
  double* Q = (double*)malloc(4 * vs * sizeof(double));
  double* aL = (double*)malloc(4 * vs * sizeof(double));
  double* aR = (double*)malloc(4 * vs * sizeof(double));
  const double c = p->c;
  int64_t neg = 0;

  LOOP3(g.lo[2], g.hi[2], g.lo[1], g.hi[1], g.lo[0], g.hi[0]) {
    const size_t o = IX(&g, i, j, k);
    const double E = Ur[o];
    Q[o] = E;
    for (int d = 0; d < 3; ++d) Q[(1 + d) * vs + o] = Ur[(1 + d) * vs + o] / (c * E);
  }
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i)
        if (!(Ur[IX(&g, i, j, k)] > 0.0)) ++neg;

  for (int d = 0; d < 3; ++d) {
    if (!g.act[d]) continue;
    double* F = Fc + (size_t)d * 4 * vs;
    double* G = Fu ? Fu + (size_t)d * 4 * vs : NULL;
    const ptrdiff_t s = g.st[d];
    int lo[3] = {0, 0, 0}, hi[3] = {g.n[0], g.n[1], g.n[2]};
    lo[d] = -1;
    hi[d] = g.n[d] + 1;
    LOOP3(lo[2], hi[2], lo[1], hi[1], lo[0], hi[0]) {
      const size_t o = IX(&g, i, j, k);
      for (int v = 0; v < 4; ++v) {
        const double* q = Q + v * vs;
        reconstruct(p->recon, q, o, s, &aL[v * vs + o], &aR[v * vs + o]);
      }
    }
    int lo2[3] = {0, 0, 0}, hi2[3] = {g.n[0], g.n[1], g.n[2]};
    hi2[d] = g.n[d] + 1;
    LOOP3(lo2[2], hi2[2], lo2[1], hi2[1], lo2[0], hi2[0]) {
      const size_t o = IX(&g, i, j, k);
      const size_t ol = o - s;
      double EL = aR[ol], ER = aL[o];
      const double fL[3] = {aR[vs + ol], aR[2 * vs + ol], aR[3 * vs + ol]};
      const double fR[3] = {aL[vs + o], aL[2 * vs + o], aL[3 * vs + o]};
      const double nL = sqrt((fL[0] * fL[0] + fL[1] * fL[1]) + fL[2] * fL[2]);
      const double nR = sqrt((fR[0] * fR[0] + fR[1] * fR[1]) + fR[2] * fR[2]);
      double FLv[3], FRv[3];
      if ((nL > 1.0) || (nR > 1.0)) {
        EL = Ur[ol];
        ER = Ur[o];
        for (int m = 0; m < 3; ++m) {
          FLv[m] = Ur[(1 + m) * vs + ol];
          FRv[m] = Ur[(1 + m) * vs + o];
        }
      } else {
        for (int m = 0; m < 3; ++m) {
          FLv[m] = c * EL * fL[m];
          FRv[m] = c * ER * fR[m];
        }
      }
      double eps = 1.0;
      if (p->tau_correction) {
        const double tau = b->dx[d] * p->kappa_R * (0.5 * (Ug[ol] + Ug[o]));
        eps = fmin(1.0, 1.0 / tau);
      }
      double f[4];
      oracle_hll_rad(EL, FLv, ER, FRv, d, p, eps, f);
      for (int v = 0; v < 4; ++v) F[v * vs + o] = f[v];
      if (G) {
        oracle_hll_rad(EL, FLv, ER, FRv, d, p, 1.0, f);
        for (int v = 0; v < 4; ++v) G[v * vs + o] = f[v];
      }
    }
  }
  if (st) st->neg_cells += neg;
  free(Q);
  free(aL);
  free(aR);
}

/* Unsplit divergence L = -((dF_x/dx + dF_y/dy) + dF_z/dz) of 4 variables. */
static void rad_divergence(const ob_box* b, const double* Fd, double* L) {
  geo g = make_geo(b);
  const size_t vs = g.vs;
  LOOP3(0, g.n[2], 0, g.n[1], 0, g.n[0]) {
    const size_t o = IX(&g, i, j, k);
    for (int v = 0; v < 4; ++v) {
      double t[3];
      for (int d = 0; d < 3; ++d) {
        if (!g.act[d]) {
          t[d] = 0.0;
          continue;
        }
        const double* F = Fd + (size_t)d * 4 * vs + v * vs;
        t[d] = (F[o + g.st[d]] - F[o]) / b->dx[d];
      }
      L[v * vs + o] = -((t[0] + t[1]) + t[2]);
    }
  }
}

/* Right-hand side of the radiation transport with the optical-depth factor as
 * given (no state is formed, so the causality rule of the stage does not enter). */
void oracle_rad_rhs(const ob_box* b, const double* Ur, const double* Ug, const ob_rad* p, double* L, ob_stats* st) {
  geo g = make_geo(b);
  double* Fd = (double*)calloc(3 * 4 * g.vs, sizeof(double));
  rad_faces(b, Ur, Ug, p, Fd, NULL, st);
  rad_divergence(b, Fd, L);
  free(Fd);
}

/* One radiation RK stage (Section 2.2.2): Uout = Uin + dt L(Uin) (Ubase NULL,
 * first stage) or Uout = Ubase/2 + (Uin + dt L(Uin))/2 (second stage), over
 * interior cells.
 * Causality rule: the optical-depth correction is disabled for the cells
 * where it produces a causality-violating state.  Reading: the stage is
 * formed with the corrected fluxes; every interior cell whose resulting state
 * has |F| > c E_r is a violating cell; at every face of a violating cell the
 * uncorrected flux replaces the corrected one (a face is one flux for both of
 * its cells, so the update stays conservative) and the stage is formed again
 * from the stage input.  One pass; ghost cells are never updated, so they
 * never violate.  The faces used are recorded in the region register. */
static void rad_stage(const ob_box* b, const double* Uin, const double* Ubase, const double* Ug, const ob_rad* p,
                      double dt, double* Uout, const ob_region* r, double* reg, double w, ob_stats* st) {
  geo g = make_geo(b);
  const size_t vs = g.vs;
  double* Fc = (double*)calloc(3 * 4 * vs, sizeof(double));
  /* tau_correction 1: the correction with the causality rule; 2: the correction
     everywhere (no rule; for comparison) */
  double* Fu = (p->tau_correction == 1) ? (double*)calloc(3 * 4 * vs, sizeof(double)) : NULL;
  double* L = (double*)calloc(4 * vs, sizeof(double));
  rad_faces(b, Uin, Ug, p, Fc, Fu, st);
  rad_divergence(b, Fc, L);
  if (Ubase) {
    memcpy(Uout, Ubase, 4 * vs * sizeof(double));
    rk2_interior(&g, 4, Uout, Uin, L, dt);
  } else {
    euler_interior(&g, 4, Uin, Uout, L, dt);
  }
  if (Fu) {
    double* viol = (double*)calloc(vs, sizeof(double));
    int64_t nviol = 0;
    for (int k = 0; k < g.n[2]; ++k)
      for (int j = 0; j < g.n[1]; ++j)
        for (int i = 0; i < g.n[0]; ++i) {
          const size_t o = IX(&g, i, j, k);
          const double Fx = Uout[vs + o], Fy = Uout[2 * vs + o], Fz = Uout[3 * vs + o];
          if (sqrt((Fx * Fx + Fy * Fy) + Fz * Fz) > p->c * Uout[o]) {
            viol[o] = 1.0;
            ++nviol;
          }
        }
    if (nviol > 0) {
      /* a ghost cell across a periodic boundary is its image's cell, so a face
         there is switched with the face it repeats; other ghosts never violate */
      ob_box bp = *b;
      for (int d = 0; d < 3; ++d)
        for (int t = 0; t < 2; ++t)
          if (bp.bc[d][t] != OB_PERIODIC) bp.bc[d][t] = OB_FIXED;
      oracle_fill_ghosts(&bp, viol, 1);
      /* face between cells o - st[d] and o along d: uncorrected if either violates */
      for (int d = 0; d < 3; ++d) {
        if (!g.act[d]) continue;
        const ptrdiff_t s = g.st[d];
        int hi2[3] = {g.n[0], g.n[1], g.n[2]};
        hi2[d] = g.n[d] + 1;
        for (int k = 0; k < hi2[2]; ++k)
          for (int j = 0; j < hi2[1]; ++j)
            for (int i = 0; i < hi2[0]; ++i) {
              const size_t o = IX(&g, i, j, k);
              if (viol[o] != 0.0 || viol[o - s] != 0.0)
                for (int v = 0; v < 4; ++v) {
                  const size_t q = (size_t)d * 4 * vs + v * vs + o;
                  Fc[q] = Fu[q];
                }
            }
      }
      rad_divergence(b, Fc, L);
      if (Ubase) {
        memcpy(Uout, Ubase, 4 * vs * sizeof(double));
        rk2_interior(&g, 4, Uout, Uin, L, dt);
      } else {
        euler_interior(&g, 4, Uin, Uout, L, dt);
      }
      if (st) st->causal_cells += nviol;
    }
    free(viol);
  }
  if (reg) record_region(&g, Fc, 4, r, reg, w);
  free(Fc);
  free(Fu);
  free(L);
}

void oracle_rad_stage(const ob_box* b, const double* Uin, const double* Ubase, const double* Ug, const ob_rad* p,
                      double dt, double* Uout, ob_stats* st) {
  rad_stage(b, Uin, Ubase, Ug, p, dt, Uout, NULL, NULL, 0.0, st);
}

void oracle_rad_transport_substep(const ob_box* b, double* Ur, const double* Ug, const ob_rad* p, double dt,
                                  ob_stats* st) {
  oracle_rad_transport_substep_reg(b, Ur, Ug, p, dt, NULL, NULL, 0.0, st);
}

void oracle_rad_transport_substep_reg(const ob_box* b, double* Ur, const double* Ug, const ob_rad* p, double dt,
                                      const ob_region* r, double* reg, double weight, ob_stats* st) {
  geo g = make_geo(b);
  const size_t nb = 4 * g.vs * sizeof(double);
  double* U1 = (double*)malloc(nb);
  double* U2 = (double*)malloc(nb);
  memcpy(U1, Ur, nb); /* fixed ghosts of the stage state equal those of Ur */
  rad_stage(b, Ur, NULL, Ug, p, dt, U1, r, reg, 0.5 * dt * weight, st);
  oracle_fill_ghosts(b, U1, 4);
  rad_stage(b, U1, Ur, Ug, p, dt, U2, r, reg, 0.5 * dt * weight, st);
  memcpy(Ur, U2, nb);
  oracle_fill_ghosts(b, Ur, 4);
  free(U1);
  free(U2);
}

/* ------------------------------------------------------------------------ */
/* Matter-radiation coupling of one cell (Section 2.2.3).                    */
/*  (a) backward-Euler energy exchange solved by Newton-Raphson on (E_g,E_r) */
/*      with R = dt rho kappa_P chat (a_r T^4 - E_r), the Jacobian and the   */
/*      eta elimination of the paper, residuals checked before each update;  */
/*  (b) backward-Euler flux source F <- F / (1 + rho kappa_F chat dt), and   */
/*      the equal and opposite change of gas momentum, dm = -dF/(chat c);    */
/*  (c) work term from the change of gas kinetic energy.                     */
/* gas = (rho, mx, my, mz, E), rad = (E_r, Fx, Fy, Fz).  Returns 0 on        */
/* convergence, 1 if the iteration cap was reached.                          */
/* ------------------------------------------------------------------------ */
int oracle_exchange_cell(const ob_rad* p, double dt, double Ssrc, double* gas, double* rad, int* iters) {
  const double rho = gas[0];
  const double c = p->c, ch = p->chat;
  const double Ek0 = 0.5 * ((gas[1] * gas[1] + gas[2] * gas[2]) + gas[3] * gas[3]) / rho;
  const double Eg0 = gas[4] - Ek0;
  const double Er0 = rad[0];
  const double Etot = Eg0 + (c / ch) * (Er0 + Ssrc);
  double Eg = Eg0, Er = Er0;
  int it, ok = 0;
  for (it = 0; it < p->newton_max_iter; ++it) {
    double T4, dTdE_T3; /* a_r T^4 and 4 a_r T^3 / C_v */
    if (p->eos == 1) {
      T4 = 4.0 * Eg / p->alpha_cv;
      const double T = sqrt(sqrt(T4));
      const double Cv = p->alpha_cv * T * T * T;
      dTdE_T3 = 4.0 * p->a_r * T * T * T / Cv;
    } else {
      const double T = Eg * (p->gamma - 1.0) / rho;
      const double Cv = rho / (p->gamma - 1.0);
      T4 = (T * T) * (T * T);
      dTdE_T3 = 4.0 * p->a_r * T * T * T / Cv;
    }
    const double R = dt * rho * p->kappa_P * ch * (p->a_r * T4 - Er);
    const double FG = (Eg - Eg0) + (c / ch) * R;
    const double FR = (Er - Er0) - (R + Ssrc);
    if (fabs(FG / Etot) < p->newton_tol && fabs((c / ch) * FR / Etot) < p->newton_tol) {
      ok = 1;
      break;
    }
    const double dRdEg = dt * rho * p->kappa_P * ch * dTdE_T3;
    const double dFG_dEg = 1.0 + (c / ch) * dRdEg;
    const double dFG_dEr = -c * dt * rho * p->kappa_P;
    const double dFR_dEg = -dRdEg;
    const double dFR_dEr = 1.0 + ch * dt * rho * p->kappa_P;
    const double eta = -dFR_dEg / dFG_dEg;
    const double dEr = -(FR + eta * FG) / (dFR_dEr + eta * dFG_dEr);
    const double dEg = -(FG + dEr * dFG_dEr) / dFG_dEg;
    Eg += dEg;
    Er += dEr;
  }
  if (iters) *iters = it;

  /* (b) flux and momentum */
  const double fac = 1.0 + rho * p->kappa_R * ch * dt;
  double m[3];
  for (int d = 0; d < 3; ++d) {
    const double F0 = rad[1 + d];
    const double F1 = F0 / fac;
    m[d] = gas[1 + d] - (F1 - F0) / (ch * c);
    rad[1 + d] = F1;
  }
  /* (c) work */
  const double Ek1 = 0.5 * ((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]) / rho;
  const double dEk = Ek1 - Ek0;
  gas[1] = m[0];
  gas[2] = m[1];
  gas[3] = m[2];
  gas[4] = Eg + (Ek0 + dEk);
  rad[0] = Er - (ch / c) * dEk;
  return ok ? 0 : 1;
}

void oracle_exchange_all(const ob_box* b, double* Ug, double* Ur, const ob_rad* p, double dt, ob_stats* st) {
  geo g = make_geo(b);
  int64_t fails = 0, itmax = 0;
#pragma omp parallel for collapse(2) reduction(+ : fails) reduction(max : itmax)
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const size_t o = IX(&g, i, j, k);
        double gas[5], rad[4];
        for (int v = 0; v < 5; ++v) gas[v] = Ug[v * g.vs + o];
        for (int v = 0; v < 4; ++v) rad[v] = Ur[v * g.vs + o];
        int it = 0;
        const double S = p->src ? dt * p->src[o] : 0.0;
        fails += oracle_exchange_cell(p, dt, S, gas, rad, &it);
        if (it > itmax) itmax = it;
        for (int v = 0; v < 5; ++v) Ug[v * g.vs + o] = gas[v];
        for (int v = 0; v < 4; ++v) Ur[v * g.vs + o] = rad[v];
      }
  if (st) {
    st->newton_fail += fails;
    if (itmax > st->newton_iter_max) st->newton_iter_max = itmax;
  }
}

/* Repeated exchange on one cell with no transport (the energy-exchange test
 * of Section 3.2).  Writes a_r-free T^4 every `every` steps into T4_out (if
 * given) and returns the final T^4. */
double oracle_exchange_series(const ob_rad* p, double dt, double S, int64_t nsteps, double* gas, double* rad,
                              double* T4_out, int64_t every) {
  double T4 = 0.0;
  for (int64_t s = 0; s < nsteps; ++s) {
    int it;
    oracle_exchange_cell(p, dt, S, gas, rad, &it);
    const double Eg = gas[4] - 0.5 * ((gas[1] * gas[1] + gas[2] * gas[2]) + gas[3] * gas[3]) / gas[0];
    if (p->eos == 1) {
      T4 = 4.0 * Eg / p->alpha_cv;
    } else {
      const double T = Eg * (p->gamma - 1.0) / gas[0];
      T4 = (T * T) * (T * T);
    }
    if (T4_out && every > 0 && ((s + 1) % every) == 0) T4_out[(s + 1) / every - 1] = T4;
  }
  return T4;
}

/* ------------------------------------------------------------------------ */
/* Radiation-hydrodynamics step (Section 2.2, operator split; Section 2.2.4  */
/* substep cap).  Hydro dt from the gas CFL condition; radiation substep     */
/* limit CFL*min(dx)/chat; N = ceil(dt_h/dt_r) capped at N_sub,max, shrinking */
/* dt_h to N dt_r when capped; then hydro RK2 and N x (radiation RK2 +       */
/* coupling) with dt_h / N.                                                  */
/* ------------------------------------------------------------------------ */
static int nsub_for(double* dt_h, double dt_r, int nsub_max) {
  double r = ceil(*dt_h / dt_r);
  int N = (r < 1.0) ? 1 : (r > (double)nsub_max ? nsub_max + 1 : (int)r);
  if (N > nsub_max) {
    N = nsub_max;
    *dt_h = N * dt_r;
  }
  return N;
}

void oracle_rhd_step(const ob_box* b, double* Ug, double* Ur, const ob_rad* p, double dt_in, ob_stats* st) {
  oracle_fill_ghosts(b, Ug, 5);
  oracle_fill_ghosts(b, Ur, 4);
  double dt_h = dt_in;
  if (!(dt_h > 0.0)) dt_h = p->cfl * dx_min(b) / oracle_hydro_max_signal(b, Ug, p->gamma);
  const double dt_r = p->cfl * dx_min(b) / p->chat;
  const int N = nsub_for(&dt_h, dt_r, p->nsub_max);
  const double dts = dt_h / N;
  hydro_rk2(b, Ug, p->gamma, dt_h, p->recon, st);
  for (int s = 0; s < N; ++s) {
    oracle_rad_transport_substep(b, Ur, Ug, p, dts, st);
    oracle_exchange_all(b, Ug, Ur, p, dts, st);
    oracle_fill_ghosts(b, Ug, 5);
    oracle_fill_ghosts(b, Ur, 4);
  }
  if (st) {
    st->dt = dt_h;
    st->nsub = N;
  }
}

/* One level step over independent boxes whose ghost cells are held at their
 * given values: one level-wide hydro dt (minimum over boxes), one substep
 * count from chat, every box advanced with them.  Ur[i] == NULL marks a
 * hydro-only box. */
void oracle_batch_step(int32_t nbox, const ob_box* boxes, double* const* Ug, double* const* Ur, double gamma_h,
                       double cfl, int recon_h, const ob_rad* p_in, ob_stats* st) {
  ob_rad q = *p_in;  /* a level step takes no per-cell source */
  q.src = NULL;
  const ob_rad* p = &q;
  double dt_h = INFINITY, dxm = INFINITY;
  int any_rad = 0;
  for (int i = 0; i < nbox; ++i) {
    const double gam = Ur[i] ? p->gamma : gamma_h;
    const double dt = cfl * dx_min(&boxes[i]) / oracle_hydro_max_signal(&boxes[i], Ug[i], gam);
    if (dt < dt_h) dt_h = dt;
    if (Ur[i]) {
      any_rad = 1;
      if (dx_min(&boxes[i]) < dxm) dxm = dx_min(&boxes[i]);
    }
  }
  int N = 0;
  if (any_rad) N = nsub_for(&dt_h, cfl * dxm / p->chat, p->nsub_max);
  for (int i = 0; i < nbox; ++i) {
    const double gam = Ur[i] ? p->gamma : gamma_h;
    hydro_rk2(&boxes[i], Ug[i], gam, dt_h, Ur[i] ? p->recon : recon_h, st);
    if (!Ur[i]) continue;
    for (int s = 0; s < N; ++s) {
      oracle_rad_transport_substep(&boxes[i], Ur[i], Ug[i], p, dt_h / N, st);
      oracle_exchange_all(&boxes[i], Ug[i], Ur[i], p, dt_h / N, st);
    }
  }
  if (st) {
    st->dt = dt_h;
    st->nsub = N;
  }
}
