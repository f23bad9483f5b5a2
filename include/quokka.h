/*
 * quokka.h -- C ABI of the MI355X (gfx950) library for the explicit per-cell
 * radiation-hydrodynamics update of Wibking & Krumholz (2021), "QUOKKA: a code
 * for two-moment AMR radiation hydrodynamics on GPUs" (arXiv:2110.01792).
 *
 * Library: libquokka_mi355x.so (HIP).  Every state pointer is a DEVICE pointer
 * owned by the caller; the library never frees caller memory.  Calls are
 * asynchronous on the given HIP stream (NULL = default stream) unless stated.
 *
 * State layout (every entry point): structure of arrays, variable-major, x
 * fastest, ghost cells included:
 *     U[v * var_stride + (k + ng) * pitch_z + (j + ng) * pitch_y + (i + ng)]
 * for interior cells 0 <= i < n[0], 0 <= j < n[1], 0 <= k < n[2].
 * Gas state: 5 variables (rho, rho vx, rho vy, rho vz, E)       (Section 3.1.1)
 * Radiation:  4 variables (E_r, F_x, F_y, F_z)                    (Section 2.1)
 * Element type: double for QK_F64, float for QK_MIXED.
 *
 * Errors: argument errors are detected on the host and returned at once with
 * no work queued (QK_EINVAL).  Conditions found on the device (non-positive
 * density, pressure or radiation energy; an exchange solve that reaches its
 * iteration cap) set sticky bits in the context's device error word; they are
 * reported by the next call that synchronises (quokka_sync_status, or any call
 * given a non-NULL dt_host).  The library never exits or aborts.
 *
 * Threading: a context serves one stream at a time; calls on one context that
 * overlap in time race on its scratch memory.
 */
#ifndef QUOKKA_H
#define QUOKKA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qk_ctx qk_ctx;

typedef enum {
  QK_OK = 0,
  QK_EINVAL = 1,     /* bad argument (detected on the host, nothing queued) */
  QK_ENOMEM = 2,     /* device allocation failed */
  QK_EHIP = 3,       /* a HIP runtime call failed */
  QK_ENEGATIVE = 4,  /* rho <= 0, P <= 0 or E_r <= 0 met on the device */
  QK_ENEWTON = 5     /* an exchange solve hit newton_max_iter (Section 2.2.3) */
} qk_status;

/* QK_MIXED: float state arrays, float reconstruction and flux arithmetic;
 * double for E - rho v^2/2, the exchange solve and the stage accumulation. */
typedef enum { QK_F64 = 0, QK_MIXED = 1 } qk_precision;

/* Boundary kind per box face.  PERIODIC must pair (lo and hi of one axis).
 * FIXED: the ghost cells are caller data and are never written.
 * FIXED_FREE_FLUX: Dirichlet ends that hold the gas state and the radiation
 * energy but not the radiation flux (Section 3.3.1's radiation pressure tube:
 * its steady state fixes rho, v and T): every variable is FIXED except
 * F_x, F_y, F_z of a 4-variable (radiation) state, which are filled as
 * OUTFLOW.  Not accepted by quokka_batch_step. */
typedef enum { QK_BC_PERIODIC = 0, QK_BC_OUTFLOW = 1, QK_BC_FIXED = 2, QK_BC_FIXED_FREE_FLUX = 3 } qk_bc;

typedef struct {
  int32_t n[3];        /* interior cells per axis, each >= 1                    */
  int32_t ng;          /* ghost layers, >= 4 (PPM needs +-2, flattening +-3, and
                          the face next to the boundary the flattening of the
                          first ghost cell)                                       */
  int64_t pitch_y;     /* element stride between rows;   0 = n[0] + 2 ng          */
  int64_t pitch_z;     /* element stride between planes; 0 = pitch_y (n[1]+2ng) */
  int64_t var_stride;  /* element stride between variables; 0 = pitch_z (n[2]+2ng) */
  /* Size limits (QK_EINVAL beyond them): 5 * var_stride <= 2^40 elements, and
     the one-tile-per-block stage grid, (n[0]/16)(n[1]/14)(n[2]/8) blocks of 256
     work-items rounded up, within 2^32 - 1 work-items (the flattening grid,
     32 x 30 tiles of 1024, likewise); 4096^3 is beyond it, 2048^3 within.   */
  double dx[3];        /* cell widths                                           */
  int32_t bc[3][2];    /* qk_bc per axis, lo then hi                            */
} qk_box;

/* Hydrodynamics (Section 2.2.1): PPM in primitive variables with
 * multidimensional shock flattening, HLLC with PVRS wave speeds, SSP-RK2. */
typedef struct {
  double gamma;            /* ideal-gas adiabatic index */
  double cfl;              /* CFL number C0/D: dt = cfl * min(dx) / max(|v| + c_s) */
  int32_t reconstruction;  /* 0 PPM (default), 1 PLM with the MC limiter (Section 2.2.1) */
} qk_hydro_params;

/* Radiation (Sections 2.1, 2.2.2, 2.2.3) under the reduced speed of light. */
typedef struct {
  double c, chat;         /* speed of light and its reduced value              */
  double a_r;             /* radiation constant                                */
  double kappa_P, kappa_R;/* Planck and Rosseland mean opacities (constant)     */
  double gamma;           /* gas adiabatic index                               */
  double alpha_cv;        /* eos 1: E_g = alpha_cv T^4 / 4 (C_v = alpha T^3)   */
  double cfl;             /* radiation substep dt_r = cfl * min(dx) / chat     */
  double newton_tol;      /* relative tolerance of the exchange solve          */
  int32_t newton_max_iter;/* iteration cap (400 in the paper)                  */
  int32_t nsub_max;       /* substep cap per hydro step (10 in the paper)      */
  int32_t closure;        /* 0 Levermore (M1), 1 Eddington (P = E/3 I),
                             2 Minerbo (polynomial form)                       */
  int32_t tau_correction; /* 0 off; 1: optical-depth correction (Section 2.2.2):
                             the HLL dissipation of every face is scaled by
                             min(1, 1/tau), tau = dx kappa_R (rho_L + rho_R)/2,
                             and switched off again at the faces of each cell
                             where the corrected stage gives |F| > c E_r (the
                             stage is then formed again there; both cells of
                             such a face take the uncorrected flux).  Needs
                             n[0] n[1] n[2] < 2^31 per box.                    */
  int32_t eos;            /* 0: P = rho T, E_g = rho T/(gamma-1); 1: alpha T^4 */
  int32_t reconstruction; /* 0 PPM, 1 PLM, for E_r and f (Section 2.2.2) and, in
                             quokka_rhd_step, for the hydro step as well       */
  const void* source;     /* NULL, or a DEVICE array of the radiation energy
                             source rate j per cell (one variable in the box's
                             layout and precision: pitch_y, pitch_z; ghosts
                             unused; caller-owned).  Each coupling update adds
                             S = dt_sub * j, the optional source term of
                             Section 2.2.3, to the radiation residual and to
                             the convergence scale E_tot.  Must be NULL for
                             quokka_batch_step (QK_EINVAL otherwise).         */
} qk_rad_params;

/* Create a context on HIP device `device` (its scratch, device error word and
 * batch-graph cache).  Returns QK_EINVAL for a bad device index. */
qk_status quokka_ctx_create(int device, qk_ctx** out);
void quokka_ctx_destroy(qk_ctx* ctx);
/* Text of the last error on this context (static storage of the context). */
const char* quokka_last_error(const qk_ctx* ctx);

/* Fill the ghost cells of `nvar` variables: periodic wrap, zero-gradient
 * outflow (copy of the nearest interior cell), fixed left untouched; edges
 * and corners as by an x, then y, then z sequential fill. */
qk_status quokka_fill_ghosts(qk_ctx* ctx, const qk_box* box, void* U, int32_t nvar, qk_precision prec,
                             void* stream);

/* Time step of one (R)HD step from the gas state (Section 2.2.1 eq. signal and
 * the dt that follows): dt = cfl * min(dx) / max over interior (|v| + c_s).
 * With rp != NULL also the radiation substep count (Section 2.2.4):
 * N = ceil(dt / dt_r), dt_r = rp->cfl * min(dx) / chat; if N > nsub_max then
 * N = nsub_max and dt = N dt_r.  Results go to dt_dev / nsub_dev (device,
 * either may be NULL) and, if dt_host != NULL, to the host (synchronises and
 * reports sticky device errors). */
qk_status quokka_compute_dt(qk_ctx* ctx, const qk_box* box, const void* U_gas, qk_precision prec,
                            const qk_hydro_params* hp, const qk_rad_params* rp, double* dt_dev,
                            int32_t* nsub_dev, double* dt_host, void* stream);

/* One SSP-RK2 hydro step in place (Section 2.2.1).  The input ghosts must be
 * valid (quokka_fill_ghosts); the output ghosts are refilled.  dt: read from
 * dt_dev if non-NULL, else dt_in if > 0, else computed from U as in
 * quokka_compute_dt.  If dt_next_dev != NULL the CFL dt of the new state is
 * written there (fused into the second stage; no extra pass). */
qk_status quokka_hydro_step(qk_ctx* ctx, const qk_box* box, void* U_gas, qk_precision prec,
                            const qk_hydro_params* hp, const double* dt_dev, double dt_in, double* dt_next_dev,
                            void* stream);

/* Radiation subsystem over one hydro step (Sections 2.2.2, 2.2.3): N times
 * { RK2 transport of (E_r, F) with dt/N; per-cell implicit exchange, flux
 * source, momentum and work terms }, updating U_rad and (momentum, energy of)
 * U_gas.  dt and N are read from dt_dev / nsub_dev (as written by
 * quokka_compute_dt) if non-NULL, else N = ceil(dt_in / dt_r), which must not
 * exceed nsub_max (QK_EINVAL otherwise).  Gas ghosts must be valid (density is
 * read at faces); all ghosts are refilled at the end. */
qk_status quokka_rad_step(qk_ctx* ctx, const qk_box* box, void* U_gas, void* U_rad, qk_precision prec,
                          const qk_rad_params* rp, const double* dt_dev, const int32_t* nsub_dev, double dt_in,
                          void* stream);

/* One radiation-hydrodynamics step (Section 2.2 operator split): compute_dt
 * with the substep cap, hydro step, radiation step.  dt_host as in
 * quokka_compute_dt (receives the hydro dt taken). */
qk_status quokka_rhd_step(qk_ctx* ctx, const qk_box* box, void* U_gas, void* U_rad, qk_precision prec,
                          const qk_rad_params* rp, double* dt_host, void* stream);

/* One level step over nbox independent boxes whose ghosts are FIXED data
 * (every bc entry must be QK_BC_FIXED): one level-wide hydro dt (minimum CFL
 * step over boxes; hydro-only boxes use hp->gamma, radiation boxes rp->gamma),
 * shrunk as in quokka_compute_dt when any box carries radiation; every box
 * advanced with it; U_rad[i] == NULL marks a hydro-only box.  Each RK stage of
 * every box runs in one persistent launch over a (box, tile) work list; the
 * whole step is captured once per box list into a HIP graph and replayed.
 * boxes, U_gas and U_rad are host arrays of length nbox.  Replays share the
 * context's scratch: a call on another stream than the previous call's waits
 * on the device for the previous replay, and a call with a different box list
 * (or state pointers) first waits on the host for it, then re-plans. */
qk_status quokka_batch_step(qk_ctx* ctx, const qk_box* boxes, int32_t nbox, void* const* U_gas,
                            void* const* U_rad, qk_precision prec, const qk_hydro_params* hp,
                            const qk_rad_params* rp, double* dt_host, void* stream);

/* Tile family (8: 8 x 8 columns; 16: 16 x 16; 14: 16 x 14 with separate x
 * and y sweep buffers) and z-chunk length chosen for the last batch step, and
 * the autotuner's score of that choice (ms; 0 when the choice came from the
 * cache).  The autotuner times the side-effect-free first stages of each
 * candidate on the caller's boxes the first time a box-shape signature is
 * seen, and scores it as hydro first stage + nsub_max x radiation first stage
 * (the weights of a level step), each the fastest of three runs; results
 * persist in the JSON file named by the environment variable QK_TUNE_CACHE,
 * if set. */
qk_status quokka_batch_config(qk_ctx* ctx, int32_t* tile, int32_t* zc, double* tune_ms);

/* quokka_hydro_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same step, the same kernels and the same bits, but the
 * stage buffer and the flattening array live in a static device array of the
 * library (128 MiB per GPU, held from the library's first context on that GPU
 * until the process ends) instead of context scratch, and no measurement
 * events are recorded.  Calls no hipMalloc, hipFree or allocating library
 * routine.  Limit: 5 var_stride + var_stride elements (rounded up to 256
 * bytes for the first part) must fit in 128 MiB: one 128^3 FP64 box with 4
 * ghost layers (or 160^3 in FP32); larger boxes return QK_EINVAL.  Nothing in
 * the array needs to start at zero (each call writes every element it
 * reads).  Every call on one GPU, from any context, shares that GPU's array:
 * calls that overlap in time on one GPU race. */
qk_status quokka_hydro_step_noalloc(qk_ctx* ctx, const qk_box* box, void* U_gas, qk_precision prec,
                                    const qk_hydro_params* hp, const double* dt_dev, double dt_in,
                                    double* dt_next_dev, void* stream);

/* ------------------------------------------------------------------------
 * AMR level synchronisation, refinement ratio 2 (Section 2.2: conservative
 * linear interpolation onto fine cells, conservative average-down, and the
 * flux-register update of the coarse cells next to a fine region).
 * A region is a range [lo, hi) of a box's interior cells (non-empty).
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t lo[3], hi[3];
} qk_region;

/* A flux register over a region is a caller-owned FP64 DEVICE array of
 * 10 (m1 m2 + m0 m2 + m0 m1) doubles (gas), m = hi - lo: x faces [v][side][k][j],
 * then y faces [v][side][k][i], then z faces [v][side][j][i], indices relative
 * to lo, side 0 the region's low face and 1 its high face, v the 5 gas
 * variables.  quokka_hydro_step_reg is quokka_hydro_step (no fused next dt)
 * that also ADDS weight * dt/2 * F of both RK stages (the step's
 * time-integrated flux) at every face on the region's boundary; the caller
 * zeroes the register.  Regions must lie in the box interior (QK_EINVAL). */
qk_status quokka_hydro_step_reg(qk_ctx* ctx, const qk_box* box, void* U_gas, qk_precision prec,
                                const qk_hydro_params* hp, const double* dt_dev, double dt_in,
                                const qk_region* region, double* reg, double weight, void* stream);

/* quokka_rad_step with a flux register over `region` for the radiation
 * variables (E_r, F_x, F_y, F_z; the register layout above with 4 variables:
 * 8 (m1 m2 + m0 m2 + m0 m1) doubles): every substep's two stages ADD
 * weight * dt_sub/2 * F at the region's boundary faces. */
qk_status quokka_rad_step_reg(qk_ctx* ctx, const qk_box* box, void* U_gas, void* U_rad, qk_precision prec,
                              const qk_rad_params* rp, const double* dt_dev, const int32_t* nsub_dev, double dt_in,
                              const qk_region* region, double* reg, double weight, void* stream);

/* Coarse cells off + (I, J, K), 0 <= I < n_fine/2 (per axis), get the mean of
 * their 8 fine children (nvar variables, 1..16; same precision on both levels).
 * Fine extents must be even and the footprint inside the coarse interior. */
qk_status quokka_average_down(qk_ctx* ctx, const qk_box* fine, const void* U_fine, const qk_box* coarse,
                              void* U_coarse, const int32_t off[3], int32_t nvar, qk_precision prec, void* stream);

/* Fine cells from the coarse level at time (1 - alpha) t0 + alpha t1 (states
 * U_c0 and U_c1 of nvar variables, 1..16; alpha in [0, 1]): the parent's value plus a quarter of the
 * MC-limited slope per axis toward the child's side, which keeps every
 * parent's mean.  Fine cell 0 lies in coarse cell off.  interior == 0 fills the
 * fine ghost layers only (fill-patch of a fine box with FIXED ghosts); != 0
 * fills the whole ghosted fine box (a new fine grid).  The parents and their
 * slope neighbours must lie in the coarse ghosted array, whose ghosts the
 * caller has filled. */
qk_status quokka_prolong(qk_ctx* ctx, const qk_box* coarse, const void* U_c0, const void* U_c1, double alpha,
                         const qk_box* fine, void* U_fine, const int32_t off[3], int32_t nvar, int32_t interior,
                         qk_precision prec, void* stream);

/* Level synchronisation: `region` is the fine box's footprint on the coarse
 * level (fine extents = 2 (hi - lo)); reg_coarse is the coarse step's register
 * over it, reg_fine the sum of the fine steps' registers over the whole fine
 * box, both with nvar variables (5 gas, 4 radiation).  Each coarse cell just outside a boundary face gains
 * (R_coarse - mean of the 4 fine faces) / dx through the region's low face and
 * minus that through its high face. */
qk_status quokka_reflux(qk_ctx* ctx, const qk_box* coarse, void* U_coarse, const qk_region* region,
                        const double* reg_coarse, const qk_box* fine, const double* reg_fine, int32_t nvar,
                        qk_precision prec, void* stream);

/* Wait for the stream, then return and clear the first sticky device error
 * (QK_ENEGATIVE, QK_ENEWTON) or QK_OK. */
qk_status quokka_sync_status(qk_ctx* ctx, void* stream);

/* Number of exchange-solve iterations of the slowest cell since the last call
 * (synchronises; resets the counter). */
int32_t quokka_newton_iter_max(qk_ctx* ctx, void* stream);

/* Measurement: while enabled, every launch of a kernel class is bracketed by
 * HIP events recorded on the stream it is launched on.  quokka_kernel_time
 * synchronises and returns the summed event time (ms) and launch count of a
 * class since timing was (re)enabled. */
typedef enum {
  QK_K_HYDRO_STAGE = 0, /* fused hydro RK stage (both stages) */
  QK_K_FLATTEN = 1,     /* shock-flattening pass              */
  QK_K_RAD_STAGE = 2,   /* radiation RK stage 1               */
  QK_K_RAD_COUPLE = 3,  /* radiation RK stage 2 + coupling    */
  QK_K_GHOST = 4,       /* ghost fill                         */
  QK_K_BATCH = 5,       /* persistent batched stage kernels   */
  QK_K_NCLASS = 6
} qk_kernel_class;
qk_status quokka_timing(qk_ctx* ctx, int32_t enable);
qk_status quokka_kernel_time(qk_ctx* ctx, int32_t kclass, double* ms_total, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
