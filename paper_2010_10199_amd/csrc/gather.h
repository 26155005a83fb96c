// K3 gather (forward), binned: one workgroup per (term, right-hand side, run of the term's
// cell-sorted nodes).  The term's grid (halo layout) is staged in LDS; each thread gathers
// the window sum of its nodes.  Because consecutive threads hold nodes of the same cell,
// the 64 lanes of a wavefront read the same grid points and the LDS reads are broadcasts
// rather than bank conflicts.  Each term's result goes into its own output slot,
// slot[s][v], indexed by virtual node; k_reduce_f sums the slots in a fixed order.
#pragma once

#include "gt_internal.h"

namespace gt {

template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(kGatherBS) void k_gather_sorted(const T *__restrict__ xT, int64_t Mx,
                                                             const GatherItem *__restrict__ items,
                                                             const int32_t *__restrict__ perm,
                                                             const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                             const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                             int64_t vstride, int slot_base,
                                                             cx_t<T> *__restrict__ slots, int64_t Vtot) {
  using C = cx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *G = reinterpret_cast<C *>(smem_raw);
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each XCD takes a
  // contiguous range of items (items are grouped by term), so a term's scattered slot writes
  // meet in one L2 and leave it as whole lines.
  const GatherItem it = items[xcd_contiguous(blockIdx.x, gridDim.x)];
  const DevTerm tm = terms[op.term_begin + it.tl];
  const C *src = grids + (int64_t)it.r * grid_total + tm.grid_off;
  const int tid = threadIdx.x;
  for (int i = tid; i < op.gsize; i += kGatherBS) G[i] = src[i];
  int32_t node[kGatherNodes];
#pragma unroll
  for (int k = 0; k < kGatherNodes; ++k) {
    const int i = tid + k * kGatherBS;
    node[k] = i < it.count ? perm[it.q0 + i] : -1;
  }
  __syncthreads();
  C *out = slots + (int64_t)(slot_base + op.term_begin + it.tl) * Vtot + (int64_t)it.r * vstride;
#pragma unroll
  for (int k = 0; k < kGatherNodes; ++k) {
    if (node[k] >= 0) out[node[k]] = gather_term<T, ORDER, MH>(G, xT, Mx, node[k], tm, op);
  }
}

}  // namespace gt
