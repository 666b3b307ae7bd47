// Batched launches: one grid advances many independent problems (uneven
// mesh sizes, same dimension, degree, physics and precision).  Block b of a
// batched grid belongs to the problem pid with first[pid] <= b <
// first[pid + 1]; it runs the same kernel body as the single-problem launch
// with that problem's arguments and its local block index b - first[pid].
// The argument arrays and block prefixes live in device memory, written once
// when the batch is bound, so a whole step can be captured as a HIP graph.
#pragma once
#include "kernels.hpp"
#include "kernels_sys.hpp"

namespace cem {

struct BatchMap {
  const int* first;    // [nprob + 1] prefix sums of the problems' block counts
  int nprob;
};

// problem of block b (uniform per block: a scalar binary search).  The
// element passes, the gathers and the tiles of non-periodic lines take their
// blocks in XCD-aware order (consecutive blocks on one XCD share its L2 for
// the halos and tables they have in common: element pass 1 of the 512-problem
// Euler batch measured 4% faster); the update and the streaming line kernels
// keep launch order, which measured faster for them.
__device__ __forceinline__ int batch_find(const BatchMap& m, int b, int* local) {
  typedef const int __attribute__((address_space(4))) ci;
  const ci* f = (const ci*)m.first;
  int lo = 0, hi = m.nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (f[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  *local = b - f[lo];
  return lo;
}

template <class TI, class TO>
__global__ void __launch_bounds__(256) kb_line(const LineArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  k_line_body<TI, TO>(args[pid], lb);
}

template <int P, int RE, class TI, class TO>
__global__ void __launch_bounds__(256) kb_line_x(const LineFastArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  k_line_x_body<P, RE, TI, TO>(args[pid], lb);
}

// the problem's 2D grid (gx tiles across lines, runs along the line) is
// flattened: local block lb -> (lb % gx, lb / gx)
template <int P, int RE, class TI, class TO>
__global__ void __launch_bounds__(256) kb_line_y(const LineFastArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  const int gx = args[pid].gx;
  k_line_y_body<P, RE, TI, TO>(args[pid], lb % gx, lb / gx);
}

// matrix-core line tiles: local block lb -> (lb % gx, lb / gx) as above
template <int P, bool AX0, class TI, class TO>
__global__ void __launch_bounds__(256) kb_line_mfma(const LineFastArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  const int gx = args[pid].gx;
  k_line_mfma_body<P, AX0, TI, TO>(args[pid], lb % gx, lb / gx);
}

// line operators of non-periodic lines (one output per thread)
__global__ void __launch_bounds__(256) kb_line_bnd(const BndLineArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  k_line_bnd_body(args[pid], lb);
}

// the LDS-tiled runs of long non-periodic lines: local block lb -> (tile
// lb % gx along the line, component lb / gx), gx tiles of 256 R outputs.
// Each problem has its own end-block weights, read by the blocks of all its
// components: consecutive blocks on one XCD, so that they share its L2
// (in launch order, consecutive blocks go to different XCDs)
template <int P, int RE>
__global__ void __launch_bounds__(256) kb_line_bnd_runs(const BndLineArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  const BndLineArgs& a = args[pid];
  const int gx = (int)((a.N + 256 * P * RE - 1) / (256 * P * RE));
  k_line_bnd_runs_body<P, RE>(a, lb % gx, lb / gx);
}

// element pass 1 with one thread per element (1D)
template <int D, int P, int PH, bool WS, class RT>
__global__ void __launch_bounds__(128) kb_elem1(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem1_body<D, P, PH, WS, RT>(args[pid], lb);
}

// the stage dt of every problem: one block per problem
__global__ void __launch_bounds__(1024) kb_stage_dt(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  k_stage_dt_body(args[pid]);
}

template <int P, int PH, bool WS, class RT>
__global__ void CEM_TILE_BOUNDS kb_elem1_tile(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem1_tile_body<P, PH, WS, RT>(args[pid], lb);
}

template <int P, int PH, bool WS, class RT>
__global__ void __launch_bounds__(256) kb_elem1_tile2(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem1_tile2_body<P, PH, WS, RT>(args[pid], lb);
}

template <int D, int P, int PH, class RT>
__global__ void CEM_SYS1_BOUNDS kb_elem1_sys(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem1_sys_body<D, P, PH, RT, 1>(args[pid], lb);
}

template <int D, int P, int PH, class RT>
__global__ void CEM_SYS1_BOUNDS kb_resid_sys(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem1_sys_body<D, P, PH, RT, 2>(args[pid], lb);
}

template <int D, int P, int M, int RE, class RT>
__global__ void __launch_bounds__(256) kb_gather_line_x(const StageArgs* __restrict__ sargs,
                                                        const LineFastArgs* __restrict__ largs, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_gather_line_x_body<D, P, M, RE, RT>(sargs[pid], largs[pid], lb);
}

template <int D, int P, int M, class RT>
__global__ void __launch_bounds__(256) kb_gather_r(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_gather_r_body<D, P, M, RT>(args[pid], lb);
}

template <int D, int P, int PH, class RT>
__global__ void __launch_bounds__(128) kb_elem2(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem2_body<D, P, PH, RT>(args[pid], lb);
}

template <int D, int P, int PH, class RT>
__global__ void CEM_SYS2_BOUNDS kb_elem2_sys(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, xcd_block(blockIdx.x, gridDim.x), &lb);
  k_elem2_sys_body<D, P, PH, RT>(args[pid], lb);
}

template <int D, int P, int PH>
__global__ void __launch_bounds__(256) kb_update(const StageArgs* __restrict__ args, BatchMap m) {
  int lb;
  const int pid = batch_find(m, blockIdx.x, &lb);
  k_update_body<D, P, PH>(args[pid], lb);
}

}  // namespace cem
