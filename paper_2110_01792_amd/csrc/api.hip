// C ABI of the MI355X per-cell update library (declarations and contracts in
// include/quokka.h).  Host-side validation, scratch management and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "quokka.h"
#include "hydro_kernels.hpp"
#include "rad_kernels.hpp"
#include "batch.hpp"
#include "amr_kernels.hpp"

using namespace qk;

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
namespace {
// Device scalar block (one allocation): accumulators and step scalars.
struct Scalars {
  unsigned long long smax_a;  // CFL accumulator for compute_dt
  unsigned long long smax_b;  // CFL accumulator for dt_next of a hydro step
  double dt;                  // step dt written by compute_dt
  double dt_aux;
  int32_t nsub;
  uint32_t err;               // sticky ERR_* bits
  uint32_t newton_iter_max;
  uint32_t nthick;            // length of the thick-cell list of the radiation step
  uint32_t pad[8];
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};
}  // namespace

// Event pairs around kernel launches of one class (measurement only).
struct KernelTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int cls, hipStream_t s) {
    if (!on) return;
    Rec r{cls, get(), get()};
    if (!r.a || !r.b) return;
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
  }
  void end(int cls, hipStream_t s) {
    if (!on || recs.empty() || recs.back().cls != cls) return;
    (void)hipEventRecord(recs.back().b, s);
  }
  void reset() {
    recs.clear();
    used = 0;
  }
  ~KernelTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Batched level step: graph, scratch and work lists for one box list, plus
// the autotuned (tile, z-chunk) per box-shape signature.
struct BatchCache {
  uint64_t key = 0;
  bool valid = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cs = nullptr;
  hipEvent_t done = nullptr;  // recorded after every graph launch, on the caller's stream of that call
  void* pool = nullptr;
  size_t pool_bytes = 0;
  void* meta = nullptr;
  size_t meta_bytes = 0;
  int tile = 16, zc = 32;
  double tune_ms = 0.0;
  std::vector<std::pair<uint64_t, std::pair<int, int>>> tuned;
  bool tune_file_read = false;
};

void batch_cache_clear(BatchCache& c) {
  if (c.exec) (void)hipGraphExecDestroy(c.exec);
  if (c.graph) (void)hipGraphDestroy(c.graph);
  if (c.pool) (void)hipFree(c.pool);
  if (c.meta) (void)hipFree(c.meta);
  if (c.cs) (void)hipStreamDestroy(c.cs);
  if (c.done) (void)hipEventDestroy(c.done);
  c = BatchCache();
}

// ---------------------------------------------------------------------------
// Scratch of the no-allocation hydro step (quokka_hydro_step_noalloc): its
// stage buffer and flattening array, sized for one 128^3 box (the paper's AMR
// box size) with 4 ghost layers in FP64: 136^3 cells x (5 + 1) x 8 B =
// 115 MiB.  Each GPU the library runs on holds its own copy at its own
// address until the process ends; host code uses that address (looked up
// once per device), never the symbol itself.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device must be current).
void* scratch_address(int device, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    g_scratch_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_ptr[device] = g_scratch_err[device] == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
  }
  *err = g_scratch_err[device];
  return g_scratch_ptr[device];
}
}  // namespace

struct qk_ctx {
  int device = 0;
  std::string last_error;
  void* noalloc_scratch = nullptr;   // this device's `scratch` (NULL: lookup failed)
  hipError_t noalloc_err = hipSuccess;
  Scalars* sc = nullptr;
  Buf stage_g, stage_r, chi;
  Buf vflags;  // causality flags of the two radiation stages (kept zero between uses)
  Buf tlist;   // thick-cell list of the radiation step
  BatchCache batch;
  KernelTimer timer;
};

namespace {

qk_status fail(qk_ctx* ctx, qk_status st, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return st;
}

qk_status hip_check(qk_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return QK_OK;
  return fail(ctx, QK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

qk_status ensure(qk_ctx* ctx, Buf& b, size_t bytes, bool zeroed = false) {
  if (b.bytes >= bytes) return QK_OK;
  if (b.p) {
    (void)hipDeviceSynchronize();  // queued work may still use the old buffer
    (void)hipFree(b.p);
  }
  b.p = nullptr;
  b.bytes = 0;
  if (hipMalloc(&b.p, bytes) != hipSuccess) return fail(ctx, QK_ENOMEM, "scratch allocation failed");
  if (zeroed && hipMemset(b.p, 0, bytes) != hipSuccess) return fail(ctx, QK_EHIP, "scratch clear failed");
  b.bytes = bytes;
  return QK_OK;
}

// Full geometry of a validated box.
struct HostBox {
  DevBox d;
  int64_t elems;  // var_stride
  int bc[3][2];
  bool any_fixed;
};

qk_status check_box(qk_ctx* ctx, const qk_box* b, HostBox& hb) {
  if (!b) return fail(ctx, QK_EINVAL, "box is NULL");
  for (int d = 0; d < 3; ++d) {
    if (b->n[d] < 1) return fail(ctx, QK_EINVAL, "box extent < 1");
    if (!(b->dx[d] > 0.0) || !std::isfinite(b->dx[d])) return fail(ctx, QK_EINVAL, "cell width must be > 0");
    for (int s = 0; s < 2; ++s)
      if (b->bc[d][s] < 0 || b->bc[d][s] > 3) return fail(ctx, QK_EINVAL, "unknown boundary kind");
    if ((b->bc[d][0] == QK_BC_PERIODIC) != (b->bc[d][1] == QK_BC_PERIODIC))
      return fail(ctx, QK_EINVAL, "periodic boundaries must pair");
  }
  if (b->ng < 4) return fail(ctx, QK_EINVAL, "ng must be >= 4");
  const int64_t NX = b->n[0] + 2 * (int64_t)b->ng, NY = b->n[1] + 2 * (int64_t)b->ng,
                NZ = b->n[2] + 2 * (int64_t)b->ng;
  const int64_t py = b->pitch_y ? b->pitch_y : NX;
  const int64_t pz = b->pitch_z ? b->pitch_z : py * NY;
  const int64_t vs = b->var_stride ? b->var_stride : pz * NZ;
  if (py < NX || pz < py * NY || vs < pz * NZ) return fail(ctx, QK_EINVAL, "pitches too small for the extents");
  if (vs * 5 > ((int64_t)1 << 40)) return fail(ctx, QK_EINVAL, "box too large");
  // A dispatch covers at most 2^32 - 1 work-items.  The stage and flattening
  // launches give each block one tile and one z-chunk, and the launch plan
  // never cuts chunks shorter than 8 planes, so this bounds both grids.
  {
    auto blocks = [](int64_t m0, int64_t m1, int64_t m2, int tx, int ty) {
      return ((m0 + tx - 1) / tx) * ((m1 + ty - 1) / ty) * std::max<int64_t>(1, (m2 + 7) / 8);
    };
    const int64_t lim = 0xffffffffLL;
    if (blocks(b->n[0], b->n[1], b->n[2], STX, STY) * SNT > lim ||
        blocks(b->n[0] + 2, b->n[1] + 2, b->n[2] + 2, FTX, FTY) * FNT > lim)
      return fail(ctx, QK_EINVAL, "box too large for one launch grid");
  }
  DevBox& d = hb.d;
  d.n0 = b->n[0];
  d.n1 = b->n[1];
  d.n2 = b->n[2];
  d.ng = b->ng;
  d.py = py;
  d.pz = pz;
  d.vs = vs;
  d.dx0 = b->dx[0];
  d.dx1 = b->dx[1];
  d.dx2 = b->dx[2];
  d.inv_dx0 = 1.0 / b->dx[0];
  d.inv_dx1 = 1.0 / b->dx[1];
  d.inv_dx2 = 1.0 / b->dx[2];
  d.dxmin = std::min(b->dx[0], std::min(b->dx[1], b->dx[2]));
  hb.elems = vs;
  hb.any_fixed = false;
  for (int a = 0; a < 3; ++a)
    for (int s = 0; s < 2; ++s) {
      hb.bc[a][s] = b->bc[a][s];
      if (b->bc[a][s] == QK_BC_FIXED || b->bc[a][s] == QK_BC_FIXED_FREE_FLUX) hb.any_fixed = true;
    }
  return QK_OK;
}

qk_status check_prec(qk_ctx* ctx, qk_precision p) {
  if (p != QK_F64 && p != QK_MIXED) return fail(ctx, QK_EINVAL, "unknown precision");
  return QK_OK;
}

qk_status check_hydro(qk_ctx* ctx, const qk_hydro_params* hp) {
  if (!hp) return fail(ctx, QK_EINVAL, "hydro params NULL");
  if (!(hp->gamma > 1.0) || !(hp->cfl > 0.0)) return fail(ctx, QK_EINVAL, "need gamma > 1 and cfl > 0");
  if (hp->reconstruction < 0 || hp->reconstruction > 1) return fail(ctx, QK_EINVAL, "unknown reconstruction");
  return QK_OK;
}

qk_status check_rad(qk_ctx* ctx, const qk_rad_params* rp) {
  if (!rp) return fail(ctx, QK_EINVAL, "rad params NULL");
  if (!(rp->c > 0) || !(rp->chat > 0) || !(rp->a_r > 0) || !(rp->gamma > 1.0) || !(rp->cfl > 0) ||
      !(rp->newton_tol > 0) || rp->newton_max_iter < 1 || rp->nsub_max < 1 || rp->closure < 0 ||
      rp->closure > 2 || rp->eos < 0 || rp->eos > 1 || !(rp->kappa_P >= 0) || !(rp->kappa_R >= 0) ||
      (rp->eos == 1 && !(rp->alpha_cv > 0)) || rp->reconstruction < 0 || rp->reconstruction > 1 ||
      rp->tau_correction < 0 || rp->tau_correction > 1)
    return fail(ctx, QK_EINVAL, "invalid radiation parameters");
  return QK_OK;
}

GhostBC ghost_bc(const HostBox& hb) {
  GhostBC g;
  g.any_ff = 0;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = hb.bc[a][0];
    g.hi[a] = hb.bc[a][1];
    if (g.lo[a] == QK_BC_FIXED_FREE_FLUX || g.hi[a] == QK_BC_FIXED_FREE_FLUX) g.any_ff = 1;
  }
  return g;
}

int grid_for(int64_t n, int per_block, int cap) {
  int64_t g = (n + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

// Face code of the ghost images the stage kernels can read instead of ghost
// cells (ghost_image: two bits per axis, x lowest, a set bit an outflow face),
// or -1 when a face holds fixed data or an extent is below 4 cells.
int image_code(const HostBox& hb) {
  const int n[3] = {hb.d.n0, hb.d.n1, hb.d.n2};
  int code = 0;
  for (int q = 0; q < 3; ++q) {
    if (n[q] < 4) return -1;
    for (int t = 0; t < 2; ++t) {
      if (hb.bc[q][t] == QK_BC_OUTFLOW)
        code |= 1 << (2 * q + t);
      else if (hb.bc[q][t] != QK_BC_PERIODIC)
        return -1;
    }
  }
  return code;
}

template <class S>
void launch_ghosts(const HostBox& hb, S* U, int nvar, hipStream_t s) {
  const DevBox& d = hb.d;
  const int64_t NX = d.n0 + 2 * d.ng, NY = d.n1 + 2 * d.ng;
  const int64_t total = 2 * d.ng * NY * NX + 2 * d.ng * d.n2 * NX + 2 * d.ng * (int64_t)d.n2 * d.n1;
  bool all_fixed = true;
  for (int a = 0; a < 3; ++a)
    for (int t = 0; t < 2; ++t) all_fixed = all_fixed && hb.bc[a][t] == QK_BC_FIXED;
  if (all_fixed) return;
  hipLaunchKernelGGL(ghost_kernel<S>, dim3(grid_for(total, 256, 4096)), dim3(256), 0, s, U, d, ghost_bc(hb), nvar);
}

template <class S>
void launch_ghost_copy(const HostBox& hb, S* dst, const S* src, int nvar, hipStream_t s) {
  const DevBox& d = hb.d;
  const int64_t total = ghost_count(d);
  hipLaunchKernelGGL(ghost_copy_kernel<S>, dim3(grid_for(total, 256, 8192)), dim3(256), 0, s, dst, src, d, nvar);
}

// Flux register of a stage launch: faces bounding region [lo, hi) add
// w * dt/2 * F into reg (see reg_slot for the layout).
struct RegRec {
  double* reg;
  int lo[3], hi[3];
  double w;
};

struct Launch {
  int gx, gy, gz, zc;
};

constexpr int kStageChunkPlanes = 16;  // z-chunk length the stage kernels aim at (see plan)

// Blocks of `kernel` resident on the whole device at once (occupancy x CUs).
template <class K>
int resident_grid(K kernel, int threads) {
  int dev = 0, ncu = 0, per = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
  return std::max(1, ncu) * per;
}

// Column tiles of tx x ty and the z chunk per block.  Blocks run in
// "generations" of `resident` at a time; the chunk count c minimises
// generations x (planes per chunk + the chunk's z prologue, ~2.5 planes),
// with at least 8 planes per chunk, so that the last generation is not a
// nearly empty one.  zc_target > 0 asks for chunks of at most about that many
// planes: the stage kernels run best with ~16 (measured at 256^3: hydro stage
// 1.44 -> 1.37 ms, radiation stages 1.29/1.69 -> 1.25/1.63 ms against the
// model's 52-plane chunks, whose long blocks finish unevenly at the end of a
// launch); the flattening pass is best with the model's choice.
Launch plan(int n0, int n1, int n2, int tx, int ty, int resident, int zc_target = 0) {
  Launch L;
  L.gx = (n0 + tx - 1) / tx;
  L.gy = (n1 + ty - 1) / ty;
  const int64_t nxy = (int64_t)L.gx * L.gy;
  const int cmin = zc_target > 0 ? std::max(1, (n2 + zc_target / 2) / zc_target) : 1;
  const int cmax = std::max(cmin, n2 / 8);
  double best = 1e300;
  int bc = cmin;
  for (int c = cmin; c <= cmax; ++c) {
    const int zc = (n2 + c - 1) / c, gz = (n2 + zc - 1) / zc;
    const int64_t gens = (nxy * gz + resident - 1) / std::max(1, resident);
    const double cost = (double)gens * (zc + 2.5);
    if (cost < best - 1e-9) {
      best = cost;
      bc = c;
    }
  }
  L.zc = (n2 + bc - 1) / bc;
  L.gz = (n2 + L.zc - 1) / L.zc;
  return L;
}

// img: -1, or the face code under which the kernels read ghost images (see
// image_code) instead of ghost cells.
template <class S, class R>
void launch_flatten(const HostBox& hb, const S* U, R* chi, double gamma, hipStream_t s, int img = -1) {
  const DevBox& d = hb.d;
  static const int res = resident_grid(flatten_kernel<S, R>, FNT);
  static const int res_i = resident_grid(flatten_kernel<S, R, true>, FNT);
  Launch L = plan(d.n0 + 2, d.n1 + 2, d.n2 + 2, FTX, FTY, img >= 0 ? res_i : res);
  FlatArgs<S, R> a;
  a.U = U;
  a.Ugh = nullptr;
  a.chi = chi;
  a.b = d;
  a.gm1 = gamma - 1.0;
  a.zc = L.zc;
  a.img = img;
  if (img >= 0)
    hipLaunchKernelGGL((flatten_kernel<S, R, true>), dim3(L.gx * L.gy * L.gz), dim3(FNT), 0, s, a, L.gx, L.gy);
  else
    hipLaunchKernelGGL((flatten_kernel<S, R>), dim3(L.gx * L.gy * L.gz), dim3(FNT), 0, s, a, L.gx, L.gy);
}

template <class S, class R, int STAGE>
void launch_stage(const HostBox& hb, const S* Uin, const S* Un, S* Uout, const R* chi, double gamma,
                  const double* dt_ptr, double dt_val, unsigned long long* smax, uint32_t* err, int recon,
                  hipStream_t s, const RegRec* rec = nullptr, int img = -1) {
  const DevBox& d = hb.d;
  static const int res = resident_grid(stage_kernel<S, R, STAGE>, SNT);
  static const int res_i = resident_grid(stage_kernel<S, R, STAGE, true>, SNT);
  Launch L = plan(d.n0, d.n1, d.n2, STX, STY, img >= 0 ? res_i : res, kStageChunkPlanes);
  StageArgs<S, R> a;
  a.Uin = Uin;
  a.Ugh = nullptr;
  a.Un = Un;
  a.Uout = Uout;
  a.chi = chi;
  a.b = d;
  a.gamma = gamma;
  a.dt_ptr = dt_ptr;
  a.dt_val = dt_val;
  a.zc = L.zc;
  a.gx = L.gx;
  a.gy = L.gy;
  a.smax = smax;
  a.err = err;
  a.recon = recon;
  a.reg = rec ? rec->reg : nullptr;
  for (int q = 0; q < 3; ++q) {
    a.rlo[q] = rec ? rec->lo[q] : 0;
    a.rhi[q] = rec ? rec->hi[q] : 0;
  }
  a.rw = rec ? rec->w : 0.0;
  a.img = img;
  if (img >= 0)
    hipLaunchKernelGGL((stage_kernel<S, R, STAGE, true>), dim3(L.gx * L.gy * L.gz), dim3(SNT), 0, s, a);
  else
    hipLaunchKernelGGL((stage_kernel<S, R, STAGE>), dim3(L.gx * L.gy * L.gz), dim3(SNT), 0, s, a);
  if (rec) {
    const int64_t nf = region_face_count(rec->lo, rec->hi);
    hipLaunchKernelGGL((region_flux_kernel<S, R>), dim3(grid_for(nf, 256, 4096)), dim3(256), 0, s, a);
  }
}

template <class S>
void launch_max_signal(const HostBox& hb, const S* U, double gamma, unsigned long long* acc, uint32_t* err,
                       hipStream_t s) {
  const int64_t n = (int64_t)hb.d.n0 * hb.d.n1 * hb.d.n2;
  hipLaunchKernelGGL((max_signal_kernel<S, 256>), dim3(grid_for(n, 256 * 8, 2048)), dim3(256), 0, s, U, hb.d,
                     gamma, acc, err);
}

// dt of the hydro step: device pointer to use (possibly computed here)
template <class S>
const double* resolve_dt(qk_ctx* ctx, const HostBox& hb, const S* U, double gamma, double cfl, const double* dt_dev,
                         double dt_in, double* dt_val, hipStream_t s) {
  *dt_val = dt_in;
  if (dt_dev) return dt_dev;
  if (dt_in > 0.0) return nullptr;
  launch_max_signal<S>(hb, U, gamma, &ctx->sc->smax_a, &ctx->sc->err, s);
  hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(64), 0, s, &ctx->sc->smax_a, cfl, hb.d.dxmin, 0.0, 0,
                     &ctx->sc->dt, (int32_t*)nullptr);
  return &ctx->sc->dt;
}

// One hydro step with the given stage buffer U1 (5 variables, U's layout)
// and flattening array chi (one variable).  Allocates nothing; timed == false
// records no measurement events.
template <class S, class R>
qk_status hydro_step_core(qk_ctx* ctx, const HostBox& hb, S* U, S* U1, R* chi, const qk_hydro_params* hp,
                          const double* dt_dev, double dt_in, double* dt_next, hipStream_t s, const RegRec* rec,
                          bool timed) {
  double dtv;
  const double* dtp = resolve_dt<S>(ctx, hb, U, hp->gamma, hp->cfl, dt_dev, dt_in, &dtv, s);
  KernelTimer& T = ctx->timer;
  auto tb = [&](int c) {
    if (timed) T.begin(c, s);
  };
  auto te = [&](int c) {
    if (timed) T.end(c, s);
  };
  if (hb.any_fixed) launch_ghost_copy<S>(hb, U1, U, 5, s);
  tb(QK_K_FLATTEN);
  launch_flatten<S, R>(hb, U, chi, hp->gamma, s);
  te(QK_K_FLATTEN);
  tb(QK_K_HYDRO_STAGE);
  launch_stage<S, R, 1>(hb, U, U, U1, chi, hp->gamma, dtp, dtv, nullptr, &ctx->sc->err, hp->reconstruction, s, rec);
  te(QK_K_HYDRO_STAGE);
  // A box whose faces are all periodic or outflow (and no flux register)
  // leaves the ghosts of the stage buffer unfilled: the second stage and its
  // flattening pass read a cell outside the box at the cell the fill copies.
  const int img = rec ? -1 : image_code(hb);
  if (img < 0) {
    tb(QK_K_GHOST);
    launch_ghosts<S>(hb, U1, 5, s);
    te(QK_K_GHOST);
  }
  tb(QK_K_FLATTEN);
  launch_flatten<S, R>(hb, U1, chi, hp->gamma, s, img);
  te(QK_K_FLATTEN);
  tb(QK_K_HYDRO_STAGE);
  launch_stage<S, R, 2>(hb, U1, U, U, chi, hp->gamma, dtp, dtv, dt_next ? &ctx->sc->smax_b : nullptr,
                        &ctx->sc->err, hp->reconstruction, s, rec, img);
  te(QK_K_HYDRO_STAGE);
  tb(QK_K_GHOST);
  launch_ghosts<S>(hb, U, 5, s);
  te(QK_K_GHOST);
  if (dt_next)
    hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(64), 0, s, &ctx->sc->smax_b, hp->cfl, hb.d.dxmin, 0.0, 0,
                       dt_next, (int32_t*)nullptr);
  return hip_check(ctx, hipGetLastError(), "hydro step launch");
}

template <class S, class R>
qk_status hydro_step_t(qk_ctx* ctx, const HostBox& hb, S* U, const qk_hydro_params* hp, const double* dt_dev,
                       double dt_in, double* dt_next, hipStream_t s, const RegRec* rec = nullptr) {
  qk_status st;
  const size_t ne = (size_t)hb.elems;
  if ((st = ensure(ctx, ctx->stage_g, 5 * ne * sizeof(S))) != QK_OK) return st;
  if ((st = ensure(ctx, ctx->chi, ne * sizeof(R))) != QK_OK) return st;
  return hydro_step_core<S, R>(ctx, hb, U, (S*)ctx->stage_g.p, (R*)ctx->chi.p, hp, dt_dev, dt_in, dt_next, s, rec,
                               true);
}

qk_status read_status(qk_ctx* ctx, hipStream_t s) {
  qk_status st = hip_check(ctx, hipStreamSynchronize(s), "stream synchronize");
  if (st != QK_OK) return st;
  uint32_t err = 0;
  if ((st = hip_check(ctx, hipMemcpy(&err, &ctx->sc->err, 4, hipMemcpyDeviceToHost), "read error word")) != QK_OK)
    return st;
  if (err) {
    (void)hipMemset(&ctx->sc->err, 0, 4);
    if (err & ERR_NEG) return fail(ctx, QK_ENEGATIVE, "non-positive density, pressure or radiation energy");
    return fail(ctx, QK_ENEWTON, "exchange solve reached its iteration cap");
  }
  return QK_OK;
}

}  // namespace

#include "api_rad.inc"
#include "api_batch.inc"
#include "api_amr.inc"

// ---------------------------------------------------------------------------
// exported entry points
// ---------------------------------------------------------------------------
extern "C" {

qk_status quokka_ctx_create(int device, qk_ctx** out) {
  if (!out) return QK_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return QK_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return QK_EHIP;
  qk_ctx* c = new qk_ctx();
  c->device = device;
  if (hipMalloc((void**)&c->sc, sizeof(Scalars)) != hipSuccess) {
    delete c;
    return QK_ENOMEM;
  }
  (void)hipMemset(c->sc, 0, sizeof(Scalars));
  c->noalloc_scratch = scratch_address(device, &c->noalloc_err);
  (void)hipDeviceSynchronize();
  *out = c;
  return QK_OK;
}

void quokka_ctx_destroy(qk_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  batch_cache_clear(ctx->batch);
  for (Buf* b : {&ctx->stage_g, &ctx->stage_r, &ctx->chi, &ctx->vflags, &ctx->tlist})
    if (b->p) (void)hipFree(b->p);
  if (ctx->sc) (void)hipFree(ctx->sc);
  delete ctx;
}

const char* quokka_last_error(const qk_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

qk_status quokka_fill_ghosts(qk_ctx* ctx, const qk_box* box, void* U, int32_t nvar, qk_precision prec,
                             void* stream) {
  if (!ctx) return QK_EINVAL;
  HostBox hb;
  qk_status st;
  if ((st = check_box(ctx, box, hb)) != QK_OK || (st = check_prec(ctx, prec)) != QK_OK) return st;
  if (!U || nvar < 1 || nvar > 16) return fail(ctx, QK_EINVAL, "bad state pointer or variable count");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  if (prec == QK_F64)
    launch_ghosts<double>(hb, (double*)U, nvar, s);
  else
    launch_ghosts<float>(hb, (float*)U, nvar, s);
  return hip_check(ctx, hipGetLastError(), "ghost fill launch");
}

qk_status quokka_compute_dt(qk_ctx* ctx, const qk_box* box, const void* U_gas, qk_precision prec,
                            const qk_hydro_params* hp, const qk_rad_params* rp, double* dt_dev, int32_t* nsub_dev,
                            double* dt_host, void* stream) {
  if (!ctx) return QK_EINVAL;
  HostBox hb;
  qk_status st;
  if ((st = check_box(ctx, box, hb)) != QK_OK || (st = check_prec(ctx, prec)) != QK_OK) return st;
  if (!U_gas) return fail(ctx, QK_EINVAL, "state pointer is NULL");
  if (!hp && !rp) return fail(ctx, QK_EINVAL, "need hydro or radiation parameters");
  if (hp && (st = check_hydro(ctx, hp)) != QK_OK) return st;
  if (rp && (st = check_rad(ctx, rp)) != QK_OK) return st;
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const double gamma = rp ? rp->gamma : hp->gamma;
  const double cfl = hp ? hp->cfl : rp->cfl;
  if (prec == QK_F64)
    launch_max_signal<double>(hb, (const double*)U_gas, gamma, &ctx->sc->smax_a, &ctx->sc->err, s);
  else
    launch_max_signal<float>(hb, (const float*)U_gas, gamma, &ctx->sc->smax_a, &ctx->sc->err, s);
  const double dt_r = rp ? rp->cfl * hb.d.dxmin / rp->chat : 0.0;
  hipLaunchKernelGGL(finalize_dt_kernel, dim3(1), dim3(64), 0, s, &ctx->sc->smax_a, cfl, hb.d.dxmin, dt_r,
                     rp ? rp->nsub_max : 0, dt_dev ? dt_dev : &ctx->sc->dt, nsub_dev ? nsub_dev : &ctx->sc->nsub);
  if ((st = hip_check(ctx, hipGetLastError(), "compute_dt launch")) != QK_OK) return st;
  if (dt_host) {
    if ((st = read_status(ctx, s)) != QK_OK) return st;
    return hip_check(ctx, hipMemcpy(dt_host, dt_dev ? dt_dev : &ctx->sc->dt, 8, hipMemcpyDeviceToHost), "read dt");
  }
  return QK_OK;
}

qk_status quokka_hydro_step(qk_ctx* ctx, const qk_box* box, void* U_gas, qk_precision prec,
                            const qk_hydro_params* hp, const double* dt_dev, double dt_in, double* dt_next_dev,
                            void* stream) {
  if (!ctx) return QK_EINVAL;
  HostBox hb;
  qk_status st;
  if ((st = check_box(ctx, box, hb)) != QK_OK || (st = check_prec(ctx, prec)) != QK_OK ||
      (st = check_hydro(ctx, hp)) != QK_OK)
    return st;
  if (!U_gas) return fail(ctx, QK_EINVAL, "state pointer is NULL");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  if (prec == QK_F64) return hydro_step_t<double, double>(ctx, hb, (double*)U_gas, hp, dt_dev, dt_in, dt_next_dev, s);
  return hydro_step_t<float, float>(ctx, hb, (float*)U_gas, hp, dt_dev, dt_in, dt_next_dev, s);
}

qk_status quokka_hydro_step_noalloc(qk_ctx* ctx, const qk_box* box, void* U_gas, qk_precision prec,
                                    const qk_hydro_params* hp, const double* dt_dev, double dt_in,
                                    double* dt_next_dev, void* stream) {
  if (!ctx) return QK_EINVAL;
  HostBox hb;
  qk_status st;
  if ((st = check_box(ctx, box, hb)) != QK_OK || (st = check_prec(ctx, prec)) != QK_OK ||
      (st = check_hydro(ctx, hp)) != QK_OK)
    return st;
  if (!U_gas) return fail(ctx, QK_EINVAL, "state pointer is NULL");
  if (!ctx->noalloc_scratch)
    return fail(ctx, QK_EHIP, std::string("no-allocation scratch unavailable: ") + hipGetErrorString(ctx->noalloc_err));
  const size_t es = prec == QK_F64 ? 8 : 4, ne = (size_t)hb.elems;
  const size_t off_chi = (5 * ne * es + 255) & ~(size_t)255, need = off_chi + ne * es;
  if (need > kNoAllocScratchBytes)
    return fail(ctx, QK_EINVAL, "box needs " + std::to_string(need) + " bytes of scratch; the no-allocation step has " +
                                    std::to_string(kNoAllocScratchBytes) + " (one 128^3 FP64 box with 4 ghost layers)");
  (void)hipSetDevice(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ctx->noalloc_scratch;
  if (prec == QK_F64)
    return hydro_step_core<double, double>(ctx, hb, (double*)U_gas, (double*)base, (double*)(base + off_chi), hp,
                                           dt_dev, dt_in, dt_next_dev, s, nullptr, false);
  return hydro_step_core<float, float>(ctx, hb, (float*)U_gas, (float*)base, (float*)(base + off_chi), hp, dt_dev,
                                       dt_in, dt_next_dev, s, nullptr, false);
}

qk_status quokka_sync_status(qk_ctx* ctx, void* stream) {
  if (!ctx) return QK_EINVAL;
  (void)hipSetDevice(ctx->device);
  return read_status(ctx, (hipStream_t)stream);
}

qk_status quokka_timing(qk_ctx* ctx, int32_t enable) {
  if (!ctx) return QK_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  ctx->timer.reset();
  ctx->timer.on = enable != 0;
  return QK_OK;
}

qk_status quokka_kernel_time(qk_ctx* ctx, int32_t kclass, double* ms_total, int64_t* launches) {
  if (!ctx || !ms_total || !launches || kclass < 0 || kclass >= QK_K_NCLASS) return QK_EINVAL;
  (void)hipSetDevice(ctx->device);
  qk_status st = hip_check(ctx, hipDeviceSynchronize(), "synchronize");
  if (st != QK_OK) return st;
  double tot = 0.0;
  int64_t n = 0;
  for (const auto& r : ctx->timer.recs) {
    if (r.cls != kclass) continue;
    float ms = 0.f;
    if ((st = hip_check(ctx, hipEventElapsedTime(&ms, r.a, r.b), "event time")) != QK_OK) return st;
    tot += ms;
    ++n;
  }
  *ms_total = tot;
  *launches = n;
  return QK_OK;
}

int32_t quokka_newton_iter_max(qk_ctx* ctx, void* stream) {
  if (!ctx) return -1;
  (void)hipSetDevice(ctx->device);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return -1;
  uint32_t v = 0;
  if (hipMemcpy(&v, &ctx->sc->newton_iter_max, 4, hipMemcpyDeviceToHost) != hipSuccess) return -1;
  (void)hipMemset(&ctx->sc->newton_iter_max, 0, 4);
  return (int32_t)v;
}

}  // extern "C"
