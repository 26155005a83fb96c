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

// K3 gather, one wavefront per run of at most 64 nodes of one grid cell (nodes of a cell
// are contiguous in the binning's order).  All lanes of the wavefront then touch the same
// 2m x ... x 2m block of the grid, so its address is uniform: the grid values are read
// with scalar loads into scalar registers and enter the lanes' FMAs as scalar operands,
// with no LDS staging and no per-lane grid reads.  Each lane evaluates its node's window
// (offsets within the cell) and accumulates the sum in registers; results go to the term's
// output slot as in k_gather_sorted.  Used when the cells hold enough nodes to keep most
// lanes busy (see the plan).
template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(256) void k_gather_cell(const T *__restrict__ xT, int64_t Mx,
                                                     const CellItem *__restrict__ items, int nitems,
                                                     const int32_t *__restrict__ perm,
                                                     const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                     const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                     int64_t vstride, int slot_base, cx_t<T> *__restrict__ slots,
                                                     int64_t Vtot) {
  using C = cx_t<T>;
  constexpr int W = 2 * MH;
  const int l = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // consecutive items (one term) share an XCD, as in k_gather_sorted
  const int ii = xcd_contiguous(blockIdx.x, gridDim.x) * 4 + wv;
  if (ii >= nitems) return;   // whole wavefront; no workgroup barrier follows
  const CellItem it = items[ii];
  const int r = it.r + (int)blockIdx.y;
  const DevTerm tm = terms[op.term_begin + it.tl];
  const C *__restrict__ G = grids + (int64_t)r * grid_total + tm.grid_off;
  const int n = op.n, P = op.P;
  const bool act = l < it.count;
  const int32_t node = perm[it.q0 + (act ? l : 0)];
  int f0, f1 = 0, f2 = 0;
  T p0[W], p1[W], p2[W];
  window_values<T, MH>(frac_offset<T>(xT[(int64_t)tm.c0 * Mx + node], n, f0) * (T)2 - (T)1, op.poly, p0);
  if (ORDER >= 2)
    window_values<T, MH>(frac_offset<T>(xT[(int64_t)tm.c1 * Mx + node], n, f1) * (T)2 - (T)1, op.poly, p1);
  if (ORDER >= 3)
    window_values<T, MH>(frac_offset<T>(xT[(int64_t)tm.c2 * Mx + node], n, f2) * (T)2 - (T)1, op.poly, p2);
  // the cell, the same for every node of the item (lane 0 always holds a node)
  const int c0 = __builtin_amdgcn_readfirstlane(f0), c1 = __builtin_amdgcn_readfirstlane(f1),
            c2 = __builtin_amdgcn_readfirstlane(f2);
  T re = 0, im = 0;
  if (ORDER == 1) {
    const C *g = G + c0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const C v = g[j];
      re = fma(p0[j], v.x, re);
      im = fma(p0[j], v.y, im);
    }
  } else if (ORDER == 2) {
    int row = wrap_start(c0, MH, n);
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const C *g = G + (int64_t)row * P + c1;
      T br = 0, bi = 0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const C v = g[j];
        br = fma(p1[j], v.x, br);
        bi = fma(p1[j], v.y, bi);
      }
      re = fma(p0[a], br, re);
      im = fma(p0[a], bi, im);
      row = row + 1 == n ? 0 : row + 1;
    }
  } else {
    int r0 = wrap_start(c0, MH, n);
    const int r1s = wrap_start(c1, MH, n);
#pragma unroll 1
    for (int a = 0; a < W; ++a) {
      int r1 = r1s;
      T br = 0, bi = 0;
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const C *g = G + ((int64_t)r0 * n + r1) * P + c2;
        T cr = 0, ci = 0;
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const C v = g[j];
          cr = fma(p2[j], v.x, cr);
          ci = fma(p2[j], v.y, ci);
        }
        br = fma(p1[b], cr, br);
        bi = fma(p1[b], ci, bi);
        r1 = r1 + 1 == n ? 0 : r1 + 1;
      }
      re = fma(p0[a], br, re);
      im = fma(p0[a], bi, im);
      r0 = r0 + 1 == n ? 0 : r0 + 1;
    }
  }
  if (act) slots[(int64_t)(slot_base + op.term_begin + it.tl) * Vtot + (int64_t)r * vstride + node] = cmake<T>(re, im);
}

}  // namespace gt
