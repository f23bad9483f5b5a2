/*
 * Plain FP64 CPU oracle for the per-cell radiation-hydrodynamics update of
 * Wibking & Krumholz (2021), "QUOKKA: a code for two-moment AMR radiation
 * hydrodynamics on GPUs" (arXiv:2110.01792).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, constant or helper with the GPU library.
 *
 * Pins: the tests check every function against closed forms, invariants, the
 * paper's printed results or exact solutions.  The optical-depth factor of
 * the radiation HLL flux is named but not written down by the paper; its
 * form here, min(1, 1/tau) on the dissipation of every radiation variable, is
 * a reading.  That reading is pinned by the closed-form decay of grid-scale
 * modes (where only the scaled dissipation acts), and the causality rule
 * that switches the factor off by its defining properties.
 *
 * Array layout used by every entry point: one contiguous float64 array per
 * state, shape (nvar, nz+2ng, ny+2ng, nx+2ng), x fastest.  Gas state has
 * nvar = 5 (rho, rho*vx, rho*vy, rho*vz, E); radiation state has nvar = 4
 * (E_r, F_x, F_y, F_z).
 */
#ifndef QUOKKA_ORACLE_H
#define QUOKKA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary kinds.  OB_FIXED_FREE_FLUX: Dirichlet ghosts (held as given, like
 * OB_FIXED) except the radiation flux F_x, F_y, F_z of a radiation state
 * (4 variables), whose ghosts are zero-gradient copies (like OB_OUTFLOW). */
enum { OB_PERIODIC = 0, OB_OUTFLOW = 1, OB_FIXED = 2, OB_FIXED_FREE_FLUX = 3 };

typedef struct {
  int32_t n[3];      /* interior cells per axis */
  int32_t ng;        /* ghost layers (>= 4) */
  double dx[3];      /* cell widths */
  int32_t bc[3][2];  /* per axis, lo/hi boundary kind */
} ob_box;

typedef struct {
  double c, chat, a_r, kappa_P, kappa_R, gamma, alpha_cv, cfl, newton_tol;
  int32_t newton_max_iter, nsub_max, closure, tau_correction, eos, recon;
  const double* src;  /* NULL, or the radiation energy source rate j per cell (one variable
                         in the box layout); the coupling adds S = dt j (Section 2.2.3) */
} ob_rad;   /* closure: 0 Levermore, 1 Eddington, 2 Minerbo.  eos: 0 ideal (P = rho T),
               1 E_g = alpha T^4 / 4.  recon: 0 PPM, 1 PLM (hydro and radiation).
               tau_correction: 0 off; 1 the optical-depth factor with the
               causality rule of Section 2.2.2; 2 the factor everywhere
               (no rule; for comparison). */

/* Result counters returned by the step drivers. */
typedef struct {
  int64_t neg_cells;      /* cells with rho<=0, P<=0 or E_r<=0 met */
  int64_t newton_fail;    /* cells whose exchange solve hit the iteration cap */
  int64_t newton_iter_max;/* largest iteration count of any cell */
  int32_t nsub;           /* radiation substeps taken */
  double dt;              /* hydro step actually taken */
  int64_t causal_cells;   /* radiation stage updates redone without the optical-depth
                             correction at their faces (|F| > c E_r; Section 2.2.2) */
} ob_stats;

void   oracle_fill_ghosts(const ob_box* b, double* U, int nvar);
double oracle_hydro_max_signal(const ob_box* b, const double* U, double gamma);
void   oracle_hydro_rhs(const ob_box* b, const double* U, double gamma, int recon, double* L, ob_stats* st);
void   oracle_hydro_step(const ob_box* b, double* U, double gamma, double cfl, double dt_in, int recon,
                         ob_stats* st);
/* Flattening coefficient chi (Section 2.2.1) of every cell of the box grown by
 * one cell along each active axis; 0 elsewhere; chi has the layout of one variable. */
void   oracle_flatten_chi(const ob_box* b, const double* U, double gamma, double* chi);
void   oracle_rad_rhs(const ob_box* b, const double* Ur, const double* Ug, const ob_rad* p, double* L, ob_stats* st);
void   oracle_rad_transport_substep(const ob_box* b, double* Ur, const double* Ug, const ob_rad* p, double dt, ob_stats* st);
/* One radiation RK stage over interior cells: Uout = Uin + dt L(Uin) if Ubase
 * is NULL, else Uout = Ubase/2 + (Uin + dt L(Uin))/2; Uout's ghosts are left
 * as they are.  With tau_correction == 1 the causality rule of Section 2.2.2
 * applies (see rad_stage). */
void   oracle_rad_stage(const ob_box* b, const double* Uin, const double* Ubase, const double* Ug, const ob_rad* p,
                        double dt, double* Uout, ob_stats* st);
int    oracle_exchange_cell(const ob_rad* p, double dt, double S, double* rho_m_E /*5*/, double* Er_F /*4*/,
                            int* iters);
void   oracle_exchange_all(const ob_box* b, double* Ug, double* Ur, const ob_rad* p, double dt, ob_stats* st);
double oracle_exchange_series(const ob_rad* p, double dt, double S, int64_t nsteps, double* gas /*5*/,
                              double* rad /*4*/, double* T4_out, int64_t every);
void   oracle_rhd_step(const ob_box* b, double* Ug, double* Ur, const ob_rad* p, double dt_in, ob_stats* st);
void   oracle_batch_step(int32_t nbox, const ob_box* boxes, double* const* Ug, double* const* Ur,
                         double gamma_h, double cfl, int recon_h, const ob_rad* p, ob_stats* st);
/* AMR level synchronisation (Section 2.2, refinement ratio 2).  A region is a
 * range [lo, hi) of a box's interior cells.  A flux register over a region
 * holds, per face on the region's boundary, the time-integrated flux
 * sum over RK stages of weight * dt/2 * F (FP64), laid out as
 *   x faces [v][side][k - lo2][j - lo1], then y faces [v][side][k - lo2][i - lo0],
 *   then z faces [v][side][j - lo1][i - lo0]   (side 0: face lo, 1: face hi),
 * nvar variables (5 gas, 4 radiation): 2 nvar (m1 m2 + m0 m2 + m0 m1) doubles
 * for m = hi - lo. */
typedef struct {
  int32_t lo[3], hi[3];
} ob_region;
void   oracle_hydro_step_reg(const ob_box* b, double* U, double gamma, double cfl, double dt_in, int recon,
                             const ob_region* r, double* reg, double weight, ob_stats* st);
/* One radiation RK2 transport substep adding weight * dt/2 * F of both stages
 * at the faces bounding r to reg (4 variables: E_r, F_x, F_y, F_z). */
void   oracle_rad_transport_substep_reg(const ob_box* b, double* Ur, const double* Ug, const ob_rad* p, double dt,
                                        const ob_region* r, double* reg, double weight, ob_stats* st);
/* Coarse cells off + (I/2) over the fine interior get the mean of their 8 children. */
void   oracle_average_down(const ob_box* fine, const double* Uf, const ob_box* coarse, double* Uc,
                           const int32_t off[3], int nvar);
/* Fine cells (ghosts only, or interior and ghosts) from the coarse state
 * (1 - alpha) Uc0 + alpha Uc1 by MC-limited linear interpolation that keeps
 * each coarse cell's mean; fine cell 0 lies in coarse cell off. */
void   oracle_prolong(const ob_box* coarse, const double* Uc0, const double* Uc1, double alpha, const ob_box* fine,
                      double* Uf, const int32_t off[3], int nvar, int interior);
/* Coarse cells just outside region r (the fine box's footprint) get the
 * difference between the coarse register (over r) and the area mean of the
 * fine register (over the whole fine box) on each boundary face. */
void   oracle_reflux(const ob_box* coarse, double* Uc, const ob_region* r, const double* reg_c, const ob_box* fine,
                     const double* reg_f, int nvar);
double oracle_closure_chi(double fhat, int closure);
void   oracle_closure_pressure(double E, const double F[3], double c, int closure, double P[9]);
void   oracle_ppm_cell(const double q[5], double out_aL_aR[2]);
void   oracle_plm_cell(const double q[3], double out_aL_aR[2]);
void   oracle_hllc(const double WL[5], const double WR[5], double gamma, double flux[5]);
void   oracle_hll_rad(double EL, const double FL[3], double ER, const double FR[3], int dir,
                      const ob_rad* p, double eps, double flux[4]);
int    oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
