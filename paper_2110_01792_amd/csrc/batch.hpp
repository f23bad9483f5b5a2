// Batched level step: many independent boxes (fixed ghost cells) advanced by
// persistent kernels over a (box, tile) work list.
//
// Each launch runs a grid sized to the chip (blocks resident per CU x CUs);
// a block repeatedly takes the next work item from a device counter
// (atomicAdd, one per item, every block exits once the counter passes the
// list) and runs the same per-tile device function the single-box kernels
// use, so a batched box and the same box run alone give identical bits.
// Work lists are sorted largest tile first.  Tile families: 8 x 8 columns on
// 64 threads and 16 x 16 on 256 (x and y sweeps share LDS buffers), and the
// single-box shape 16 x 14 on 256 threads with separate x/y buffers (every
// sweep phase one item per thread, three barriers per plane).  The flattening
// pass runs on the single-box flattening tile (32 x 30 on 1024 threads) in
// every family.  Ghost cells of a stage buffer are read from the box's own
// fixed ghosts (ghost-source pointer), so no copies.
#pragma once
#include "rad_kernels.hpp"

namespace qk {

template <class S, class R>
struct BatchBox {
  DevBox b;
  S* U;      // gas state (caller memory)
  S* U1;     // gas stage buffer (library scratch)
  R* chi;    // flattening coefficients (library scratch)
  S* Ur;     // radiation state (caller memory) or NULL
  S* Ur1;    // radiation stage buffer (library scratch) or NULL
  double gamma;
  int zc_stage, zc_flat;
  int recon;  // hydro reconstruction of this box (0 PPM, 1 PLM)
  uint8_t* vf[2];  // causality flags of radiation stages 1 and 2 (library scratch) or NULL
};

struct WorkItem {
  int box, bx, by, bz;
};

// Take the next item index; block-uniform.
__device__ __forceinline__ int next_item(int* counter, int* slot) {
  if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
  __syncthreads();
  const int it = *slot;
  __syncthreads();
  return it;
}

__global__ void zero_counters_kernel(int* c, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

template <class S, class R, int TX, int TY, int NT>
__global__ __launch_bounds__(NT, sizeof(S) == 4 ? NT / 128 : NT / 256) void batch_flatten_kernel(const BatchBox<S, R>* __restrict__ boxes,
                                                               const WorkItem* __restrict__ items, int nitems,
                                                               int* counter, int stage) {
  __shared__ FlatSmem<R, TX, TY> sm;
  __shared__ int slot;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= nitems) break;
    const WorkItem w = items[it];
    const BatchBox<S, R>& bb = boxes[w.box];
    FlatArgs<S, R> a;
    a.U = stage == 1 ? bb.U : bb.U1;
    a.Ugh = stage == 1 ? nullptr : bb.U;
    a.chi = bb.chi;
    a.b = bb.b;
    a.gm1 = bb.gamma - 1.0;
    a.zc = bb.zc_flat;
    a.img = -1;
    flatten_tile<S, R, TX, TY, NT>(a, w.bx, w.by, w.bz, sm);
  }
}

template <class S, class R, int TX, int TY, int NT, bool SPLIT, int STAGE>
__global__ __launch_bounds__(NT) void batch_stage_kernel(const BatchBox<S, R>* __restrict__ boxes,
                                                             const WorkItem* __restrict__ items, int nitems,
                                                             int* counter, const double* dt_ptr, uint32_t* err) {
  __shared__ HydroSmem<R, TX, TY, SPLIT> sm;
  __shared__ int slot;
  bool bad = false;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= nitems) break;
    const WorkItem w = items[it];
    const BatchBox<S, R>& bb = boxes[w.box];
    StageArgs<S, R> a;
    a.Uin = STAGE == 1 ? bb.U : bb.U1;
    a.Ugh = STAGE == 1 ? nullptr : bb.U;
    a.Un = bb.U;
    a.Uout = STAGE == 1 ? bb.U1 : bb.U;
    a.chi = bb.chi;
    a.b = bb.b;
    a.gamma = bb.gamma;
    a.dt_ptr = dt_ptr;
    a.dt_val = 0.0;
    a.zc = bb.zc_stage;
    a.gx = a.gy = 1;
    a.smax = nullptr;
    a.err = err;
    a.recon = bb.recon;
    a.reg = nullptr;
    a.img = -1;
    stage_tile<S, R, TX, TY, NT, SPLIT, STAGE>(a, w.bx, w.by, w.bz, sm, bad);
    __syncthreads();
  }
  if (bad) atomicOr(err, ERR_NEG);
}

// Arguments of one radiation stage of batched box bb (ghosts are fixed data:
// the stage buffer reads its ghost cells from the box's own state).
template <class S, class R, int STAGE>
__device__ __forceinline__ RadStageArgs<S, R> batch_rad_args(const BatchBox<S, R>& bb, const RadParamsDev& p,
                                                             const double* dt_ptr, const int32_t* nsub_ptr, int N,
                                                             int sub, uint32_t* err, uint32_t* iter_max,
                                                             const uint32_t* nthick) {
  RadStageArgs<S, R> a;
  a.Uin = STAGE == 1 ? bb.Ur : bb.Ur1;
  a.Ugh = STAGE == 1 ? nullptr : bb.Ur;
  a.Un = bb.Ur;
  a.Uout = STAGE == 1 ? bb.Ur1 : bb.Ur;
  a.Ug = bb.U;
  a.b = bb.b;
  a.p = p;
  a.dt_ptr = dt_ptr;
  a.nsub_ptr = nsub_ptr;
  a.dt_val = 0.0;
  a.nsub_val = N;
  a.sub = sub;
  a.zc = bb.zc_stage;
  a.gx = a.gy = 1;
  a.err = err;
  a.iter_max = iter_max;
  a.reg = nullptr;
  a.vfl = bb.vf[STAGE - 1];
  a.vfl_clear = bb.vf[2 - STAGE];
  a.per = 0;
  a.img = -1;
  a.nthick = nthick;
  return a;
}

template <class S, class R, int TX, int TY, int NT, bool SPLIT, int STAGE>
__global__ __launch_bounds__(NT, sizeof(S) == 4 ? (STAGE == 1 ? 4 : 3) : 2) void batch_rad_kernel(const BatchBox<S, R>* __restrict__ boxes,
                                                              const WorkItem* __restrict__ items, int nitems,
                                                              int* counter, RadParamsDev p, const double* dt_ptr,
                                                              const int32_t* nsub_ptr, int sub, uint32_t* err,
                                                              uint32_t* iter_max, const uint32_t* nthick) {
  const int N = *nsub_ptr;
  if (sub >= N) return;
  __shared__ RadSmem<R, TX, TY, SPLIT> sm;
  __shared__ int slot;
  bool bad = false, nfail = false;
  uint32_t itmax = 0;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= nitems) break;
    const WorkItem w = items[it];
    const RadStageArgs<S, R> a =
        batch_rad_args<S, R, STAGE>(boxes[w.box], p, dt_ptr, nsub_ptr, N, sub, err, iter_max, nthick);
    itmax = max(itmax, rad_tile<S, R, TX, TY, NT, SPLIT, STAGE>(a, w.bx, w.by, w.bz, N, sm, bad, nfail));
    __syncthreads();
  }
  if (bad) atomicOr(err, ERR_NEG);
  if (nfail) atomicOr(err, ERR_NEWTON);
  if (STAGE == 2) block_umax_to<NT>(itmax, iter_max);
}

// Thick cells (a face with tau > 1) of every radiation box: block row y
// serves box y.
template <class S, class R>
__global__ __launch_bounds__(256) void batch_thick_list_kernel(const BatchBox<S, R>* __restrict__ boxes,
                                                               double kappa, CellRef* list, uint32_t* count) {
  const BatchBox<S, R>& bb = boxes[blockIdx.y];
  if (!bb.Ur) return;
  thick_list_box<S, R>(bb.b, bb.U, kappa, (int)blockIdx.y, (int64_t)blockIdx.x * 256 + threadIdx.x,
                       (int64_t)gridDim.x * 256, list, count);
}

// Fix-up pass of one radiation stage over the thick cells of every box.
template <class S, class R, int STAGE>
__global__ __launch_bounds__(256) void batch_rad_fix_kernel(const BatchBox<S, R>* __restrict__ boxes, RadParamsDev p,
                                                            const double* dt_ptr, const int32_t* nsub_ptr, int sub,
                                                            const CellRef* __restrict__ list, const uint32_t* count,
                                                            uint32_t* err, uint32_t* iter_max) {
  const int N = *nsub_ptr;
  if (sub >= N) return;
  const uint32_t n = *count;
  bool bad = false, nfail = false;
  uint32_t itmax = 0;
  for (uint32_t t = blockIdx.x * 256u + threadIdx.x; t < n; t += gridDim.x * 256u) {
    const CellRef c = list[t];
    const RadStageArgs<S, R> a =
        batch_rad_args<S, R, STAGE>(boxes[c.box], p, dt_ptr, nsub_ptr, N, sub, err, iter_max, count);
    itmax = max(itmax, rad_fix_cell<S, R, STAGE>(a, c.i, c.j, c.k, N, bad, nfail));
    a.vfl_clear[interior_index(a.b, c.i, c.j, c.k)] = 0;
  }
  if (bad) atomicOr(err, ERR_NEG);
  if (nfail) atomicOr(err, ERR_NEWTON);
  if (STAGE == 2) block_umax_to<256>(itmax, iter_max);
}

// Level CFL: max over every interior cell of every box of |v| + c_s (each box
// with its own gamma), over the stage work list.
template <class S, class R, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void batch_max_signal_kernel(const BatchBox<S, R>* __restrict__ boxes,
                                                                  const WorkItem* __restrict__ items, int nitems,
                                                                  int* counter, unsigned long long* smax,
                                                                  uint32_t* err) {
  __shared__ int slot;
  double m = 0.0;
  bool bad = false;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= nitems) break;
    const WorkItem w = items[it];
    const BatchBox<S, R>& bb = boxes[w.box];
    const DevBox& b = bb.b;
    const int i = w.bx * TX + tx, j = w.by * TY + ty;
    if (i >= b.n0 || j >= b.n1) continue;
    const int z0 = w.bz * bb.zc_stage, z1 = min(z0 + bb.zc_stage, b.n2);
    const double g = bb.gamma, gm1 = g - 1.0;
    for (int k = z0; k < z1; ++k) {
      double q[5];
      load_cons(bb.U, b.vs, cell(b, i, j, k), q);
      m = fmax(m, signal_speed(q, g, gm1, bad));
    }
  }
  if (bad) atomicOr(err, ERR_NEG);
  block_max_to<TX * TY>(m, smax);
}

}  // namespace qk
