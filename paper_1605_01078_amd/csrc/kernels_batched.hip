// Batched mode: many independent FP64 GEMMs C_p := alpha*A_p*B_p + beta*C_p in one persistent
// launch, each with its own Strassen level (0, 1, 2) and tile shape (128 x 128 or 64 x 64).
//
// A work item is (problem, tile position): the workgroup that takes it runs every product of
// the problem's table on that tile and adds each to its C destinations (the ABC variant,
// owner computes, so the result is bitwise that of a single call with the same level and tile
// shape).  Items are listed in decreasing cost and handed out through one atomic counter, so
// the longest ones start first and the tail is short.  The counter is cleared by a small kernel
// of its own (not a memset), which keeps the pair of launches capturable in a graph.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "plan.h"
#include "tile_fp64.h"

namespace smx {

__constant__ TableDev g_tables_batched[kNumTables];

hipError_t upload_tables_batched(const TableDev* tabs) {
  return hipMemcpyToSymbol(HIP_SYMBOL(g_tables_batched), tabs, sizeof(TableDev) * kNumTables, 0,
                           hipMemcpyHostToDevice);
}

namespace {

__global__ void clear_counter_kernel(unsigned* counter) {
  if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class Tile>
__device__ __forceinline__ void run_item(const GemmArgs& g, int tile, double* lds) {
  const TableDev& tab = g_tables_batched[g.tab];
  const int ti = tile % g.tiles_m, tj = tile / g.tiles_m;
  const int64_t row0 = (int64_t)ti * (Tile::WM * 2), col0 = (int64_t)tj * (Tile::WN * 2);
  for (int r = 0; r < tab.nprod; ++r) {
    const ProdDesc& pd = tab.prod[r];
    typename Tile::Acc acc;
    Tile::product(g, pd, row0, col0, lds, acc);
    Tile::update_c(g, pd, row0, col0, acc);
  }
}

template <bool VEC>
__global__ __launch_bounds__(256, 2) void batched_kernel(const BatchProblem* probs,
                                                         const BatchItem* items, int n_items,
                                                         unsigned* counter) {
  using T128 = Fp64Tile<128, 128, 16, 4, VEC>;
  using T64 = Fp64Tile<64, 64, 16, 4, VEC>;
  static_assert(T128::LDS_DOUBLES >= T64::LDS_DOUBLES, "LDS");
  __shared__ double lds[T128::LDS_DOUBLES];
  __shared__ int s_item;
  for (;;) {
    if (threadIdx.x == 0)
      s_item = (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int it = s_item;
    __syncthreads();   // s_item is rewritten by the next round
    if (it >= n_items) break;   // every workgroup ends once the list is exhausted
    const BatchItem w = items[it];
    const BatchProblem& p = probs[w.problem];
    if (p.cfg == 0) run_item<T128>(p.g, w.tile, lds);
    else run_item<T64>(p.g, w.tile, lds);
  }
}

}  // namespace

hipError_t launch_batched(const BatchProblem* probs, const BatchItem* items, int n_items,
                          unsigned* counter, bool vec, int grid, hipStream_t s) {
  hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  if (vec) hipLaunchKernelGGL(batched_kernel<true>, dim3(grid), dim3(256), 0, s, probs, items, n_items, counter);
  else hipLaunchKernelGGL(batched_kernel<false>, dim3(grid), dim3(256), 0, s, probs, items, n_items, counter);
  return hipGetLastError();
}

const void* batched_kernel_fn(bool vec) {
  return vec ? reinterpret_cast<const void*>(&batched_kernel<true>)
             : reinterpret_cast<const void*>(&batched_kernel<false>);
}
const void* clear_counter_fn() { return reinterpret_cast<const void*>(&clear_counter_kernel); }

}  // namespace smx
