// Shared launches for plans of orders 1 and 2 with window forms: each launch runs the same
// step of both orders (and of the empty set) side by side, so a transform takes three
// launches per direction instead of five (forward) and eight (adjoint):
//   forward:  k_fwd_pack2 (K1 + K2 of both orders), k_fwd_gather2 (K3), k_reduce_f (sum over u)
//   adjoint:  k_adj_spread2 (K4 of both orders, empty-set partial sums),
//             k_adj_fold2 (folds of both orders, empty-set coefficient),
//             k_adj_dft2 (K2 + K5 of both orders)
// Every part runs the body its own kernel runs, on the same work items and in the same
// summation order, so the results equal those of the separate launches bit for bit.  A
// workgroup belongs to exactly one part (the part test is uniform over the workgroup), so the
// bodies' workgroup barriers are reached by all of its threads.
#pragma once

#include "gt_internal.h"

namespace gt {

// Blocks [b0, b0 + nx * ny) of a launch run one part, as block (x, y) of a grid nx x ny
// (x fastest).
struct Part {
  int b0, nx, ny;
};

__device__ __forceinline__ bool in_part(int b, const Part &p, Blk &bk) {
  const int l = b - p.b0;
  if (l < 0 || l >= p.nx * p.ny) return false;
  bk.y = l / p.nx;
  bk.x = l - bk.y * p.nx;
  return true;
}

// The same for a part that starts at a multiple of 8 blocks, its blocks renumbered so that
// each XCD (block b runs on XCD b mod 8) takes one contiguous range of the part's blocks
// (as the separate gathers renumber theirs): every part is spread over all XCDs.
__device__ __forceinline__ bool in_part_xcd(int b, const Part &p, Blk &bk) {
  int l = b - p.b0;
  if (l < 0 || l >= p.nx * p.ny) return false;
  l = xcd_contiguous(l, p.nx * p.ny);
  bk.y = l / p.nx;
  bk.x = l - bk.y * p.nx;
  return true;
}

template <typename T>
struct FwdPackArgs {
  const cx_t<T> *fhat;
  const T *colscale;
  int64_t ncoef;
  const DevTerm *terms;
  cx_t<T> *grids;
  int64_t grid_total;
  OrderParams<T> op1, op2;
  int slices1, slices2;   // plain packs: workgroups per term
  int nslab;              // polynomial pack of order 2: slabs of kPolyRows cell rows per term
  cx_t<T> *kpoly;
  Part p1, p2;
};

// PMH > 0: order 2 packs straight into the per-cell window polynomials (FP32, m = PMH).
template <typename T, int PMH>
__global__ __launch_bounds__(kPackBS) void k_fwd_pack2(FwdPackArgs<T> a) {
  Blk bk;
  if (in_part((int)blockIdx.x, a.p1, bk)) {
    pack_fwd_body<T, 1>(bk, a.fhat, a.colscale, a.ncoef, a.terms, a.op1, a.grids, a.grid_total, a.slices1);
  } else if (in_part((int)blockIdx.x, a.p2, bk)) {
    if constexpr (PMH > 0)
      pack_poly2_body<PMH>(bk, a.fhat, a.colscale, a.ncoef, a.terms, a.op2, a.nslab, a.kpoly);
    else
      pack_fwd_body<T, 2>(bk, a.fhat, a.colscale, a.ncoef, a.terms, a.op2, a.grids, a.grid_total, a.slices2);
  }
}

template <typename T>
struct FwdGatherArgs {
  const T *x;
  int64_t Mtot;
  const DevTerm *terms;
  const cx_t<T> *grids;
  int64_t grid_total;
  OrderParams<T> op1, op2;
  const int32_t *perm1, *perm2;
  const GatherItem *gi1, *gi2;       // sorted form: one item per workgroup
  const CellItem *ci1, *ci2;         // cell and polynomial forms: four items per workgroup
  int nci1, nci2;
  const T *xs2;                      // polynomial form: sorted coordinates and coefficients
  const cx_t<T> *kpoly;
  int64_t vstride;
  int sbase1, sbase2;
  cx_t<T> *slots;
  int64_t Vtot;
  Part p1, p2;
};

// Each part starts at a multiple of 8 blocks and is renumbered XCD-contiguous on its own (as
// the separate gathers are), so consecutive items share an XCD's L2 and every part runs on all
// XCDs (renumbering the whole launch at once gave one XCD the order-1 part alone: 52 against
// 34 µs for the two separate gathers).  K1, K2: the orders' gather forms
// (GT_GATHER_SORTED, _CELL, _POLY); each instance holds only the two bodies it runs, so it
// needs no more registers than the larger of them.
template <typename T, int MH, int K1, int K2>
__global__ __launch_bounds__(256) void k_fwd_gather2(FwdGatherArgs<T> a) {
  static_assert(K1 != GT_GATHER_POLY && (K2 != GT_GATHER_POLY || std::is_same<T, float>::value), "no such form");
  const int b = (int)blockIdx.x;
  Blk bk;
  if (in_part_xcd(b, a.p1, bk)) {
    if constexpr (K1 == GT_GATHER_SORTED)
      gather_sorted_body<T, 1, MH>(bk, a.x, a.Mtot, a.gi1, a.perm1, a.terms, a.op1, a.grids, a.grid_total, a.vstride,
                                   a.sbase1, a.slots, a.Vtot);
    else
      gather_cell_body<T, 1, MH>(bk, a.x, a.Mtot, a.ci1, a.nci1, a.perm1, a.terms, a.op1, a.grids, a.grid_total,
                                 a.vstride, a.sbase1, a.slots, a.Vtot);
  } else if (in_part_xcd(b, a.p2, bk)) {
    if constexpr (K2 == GT_GATHER_POLY)
      gather_poly2_body<T>(bk, a.xs2, a.ci2, a.nci2, a.perm2, a.op2, a.kpoly, a.vstride, a.sbase2, a.slots, a.Vtot);
    else if constexpr (K2 == GT_GATHER_SORTED)
      gather_sorted_body<T, 2, MH>(bk, a.x, a.Mtot, a.gi2, a.perm2, a.terms, a.op2, a.grids, a.grid_total, a.vstride,
                                   a.sbase2, a.slots, a.Vtot);
    else
      gather_cell_body<T, 2, MH>(bk, a.x, a.Mtot, a.ci2, a.nci2, a.perm2, a.terms, a.op2, a.grids, a.grid_total,
                                 a.vstride, a.sbase2, a.slots, a.Vtot);
  }
}

template <typename T>
struct AdjSpreadArgs {
  const T *x;
  int64_t Mtot;
  const DevTerm *terms;
  const cx_t<T> *y;
  const SpreadItem *si1;   // order 1: binned spread into partial grids
  OrderParams<T> op1;
  SpreadArgs sa1;
  cx_t<T> *gpart1;
  int64_t gstride1;
  const T *xs2;            // order 2: tile spread into patches
  const int32_t *perm2;
  OrderParams<T> op2;
  Tile2Args ta;
  cx_t<T> *patch;
  const WorkItem *gitems;  // empty set: partial sums of the samples
  double *ysum;
  Part p1, p2, pe;
};

// Workgroups of four wavefronts: the tile spread's own size; the binned order-1 spread runs
// its cells over four wavefronts instead of kSpreadWaves.  The order-1 workgroups come first
// in the launch, so they start first and run beside the tile spread's (placed after them,
// the tile spread's first round would fill the compute units and the order-1 work would
// only start as it drains).
template <typename T, int MH>
__global__ __launch_bounds__(64 * kTileWaves) void k_adj_spread2(AdjSpreadArgs<T> a) {
  Blk bk;
  if (in_part((int)blockIdx.x, a.p2, bk))
    spread_tile2_body<T, MH>(bk, a.xs2, a.perm2, a.op2, a.ta, a.y, a.patch);
  else if (in_part((int)blockIdx.x, a.p1, bk))
    spread_binned_body<T, 1, MH, kTileWaves>(bk, a.x, a.Mtot, a.si1, a.terms, a.op1, a.sa1, a.y, a.gpart1, a.gstride1);
  else if (in_part((int)blockIdx.x, a.pe, bk))
    empty_part_body<T>(bk, a.gitems, a.y, a.ysum);
}

template <typename T>
struct AdjFoldArgs {
  const DevTerm *terms;
  const cx_t<T> *gpart1;   // order 1: partial grids -> folded grids
  int64_t gstride1;
  const int32_t *sitem_begin1;
  OrderParams<T> op1;
  cx_t<T> *gsum1;
  const cx_t<T> *patch;    // order 2: patches -> column sums, one unit per wavefront
  const int32_t *tileseg;
  OrderParams<T> op2;
  Tile2Args ta;
  int B, ts, nunits2;
  cx_t<T> *hcol2;
  const int32_t *gitem_begin;   // empty set: its coefficient from the partial sums
  const double *ysum;
  int64_t ncoef;
  cx_t<T> *fhat;
  Part p1, p2, pe;
};

// Order 2: four of k_fold_tilesum's units (its one-wavefront workgroups) per workgroup, each
// wavefront with its own LDS tile sums and no workgroup barrier.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_fold2(AdjFoldArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Blk bk;
  if (in_part((int)blockIdx.x, a.p2, bk)) {
    const int wv = threadIdx.x >> 6, u = bk.x * 4 + wv;
    if (u >= a.nunits2) return;   // whole wavefront
    cx_t<T> *tsum = reinterpret_cast<cx_t<T> *>(smem_raw) + (size_t)wv * a.ta.ntile * 64;
    fold_tilesum_body<T>(Blk{u, bk.y}, tsum, a.patch, a.tileseg, a.op2, a.ta, a.B, a.ts, a.hcol2);
  } else if (in_part((int)blockIdx.x, a.p1, bk)) {
    fold_partials_body<T>(bk, a.gpart1, a.gstride1, a.sitem_begin1, a.terms, a.op1, 1, a.gsum1);
  } else if (in_part((int)blockIdx.x, a.pe, bk)) {
    empty_adj_body<T>(bk, a.gitem_begin, a.ysum, a.ncoef, a.fhat);
  }
}

template <typename T>
struct AdjDftArgs {
  const DevTerm *terms;
  const T *colscale;
  int64_t ncoef;
  cx_t<T> *fhat;
  const cx_t<T> *gsum1;   // order 1: folded grids
  OrderParams<T> op1;
  const cx_t<T> *hcol2;   // order 2: column sums of the patches
  OrderParams<T> op2;
  int ntile2, ts2, nsplit2;
  Part p1, p2;
};

// Workgroups of 2 kPackBS threads (the order-2 DFT's size; the order-1 body strides over
// its work by the workgroup size).
template <typename T>
__global__ __launch_bounds__(2 * kPackBS) void k_adj_dft2(AdjDftArgs<T> a) {
  Blk bk;
  if (in_part((int)blockIdx.x, a.p2, bk))
    dft_adj_body<T, 2>(bk, a.hcol2, a.terms, a.op2, a.colscale, a.ncoef, a.fhat, a.ntile2, a.ts2, a.nsplit2);
  else if (in_part((int)blockIdx.x, a.p1, bk))
    dft_adj_body<T, 1>(bk, a.gsum1, a.terms, a.op1, a.colscale, a.ncoef, a.fhat, 0, 0, 1);
}

}  // namespace gt
