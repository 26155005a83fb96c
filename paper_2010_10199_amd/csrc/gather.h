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
__device__ __forceinline__ void gather_sorted_body(const Blk bk, const T *__restrict__ xT, int64_t Mx,
                                                   const GatherItem *__restrict__ items,
                                                   const int32_t *__restrict__ perm,
                                                   const DevTerm *__restrict__ terms, const OrderParams<T> &op,
                                                   const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                   int64_t vstride, int slot_base, cx_t<T> *__restrict__ slots,
                                                   int64_t Vtot) {
  using C = cx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *G = reinterpret_cast<C *>(smem_raw);
  const GatherItem it = items[bk.x];
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

// Workgroups are dealt to the 8 XCDs round-robin; they are renumbered so that each XCD takes
// a contiguous range of items (items are grouped by term), so a term's scattered slot writes
// meet in one L2 and leave it as whole lines.
template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(kGatherBS) void k_gather_sorted(const T *__restrict__ xT, int64_t Mx,
                                                             const GatherItem *__restrict__ items,
                                                             const int32_t *__restrict__ perm,
                                                             const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                             const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                             int64_t vstride, int slot_base,
                                                             cx_t<T> *__restrict__ slots, int64_t Vtot) {
  gather_sorted_body<T, ORDER, MH>(Blk{xcd_contiguous(blockIdx.x, gridDim.x), 0}, xT, Mx, items, perm, terms, op,
                                   grids, grid_total, vstride, slot_base, slots, Vtot);
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
__device__ __forceinline__ void gather_cell_body(const Blk bk, const T *__restrict__ xT, int64_t Mx,
                                                 const CellItem *__restrict__ items, int nitems,
                                                 const int32_t *__restrict__ perm,
                                                 const DevTerm *__restrict__ terms, const OrderParams<T> &op,
                                                 const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                 int64_t vstride, int slot_base, cx_t<T> *__restrict__ slots,
                                                 int64_t Vtot) {
  using C = cx_t<T>;
  constexpr int W = 2 * MH;
  const int l = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ii = bk.x * 4 + wv;
  if (ii >= nitems) return;   // whole wavefront; no workgroup barrier follows
  const CellItem it = items[ii];
  const int r = it.r + bk.y;
  const DevTerm tm = terms[op.term_begin + it.tl];
  const C *__restrict__ G = grids + (int64_t)r * grid_total + tm.grid_off;
  const int n = op.n, P = op.P;
  const bool act = l < it.count;
  const int32_t node = perm[it.q0 + (act ? l : 0)];
  // the item's cell (the binning's cell of each of its nodes); offsets z relative to it
  const int c0 = it.cell[0], c1 = it.cell[1], c2 = it.cell[2];
  const T nf = (T)n;
  T p0[W], p1[W], p2[W];
  window_values<T, MH>(fma(nf, xT[(int64_t)tm.c0 * Mx + node], (T)(n / 2 - c0)) * (T)2 - (T)1, op.poly, p0);
  if (ORDER >= 2)
    window_values<T, MH>(fma(nf, xT[(int64_t)tm.c1 * Mx + node], (T)(n / 2 - c1)) * (T)2 - (T)1, op.poly, p1);
  if (ORDER >= 3)
    window_values<T, MH>(fma(nf, xT[(int64_t)tm.c2 * Mx + node], (T)(n / 2 - c2)) * (T)2 - (T)1, op.poly, p2);
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

// consecutive items (one term) share an XCD, as in k_gather_sorted
template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(256) void k_gather_cell(const T *__restrict__ xT, int64_t Mx,
                                                     const CellItem *__restrict__ items, int nitems,
                                                     const int32_t *__restrict__ perm,
                                                     const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                     const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                     int64_t vstride, int slot_base, cx_t<T> *__restrict__ slots,
                                                     int64_t Vtot) {
  gather_cell_body<T, ORDER, MH>(Blk{xcd_contiguous(blockIdx.x, gridDim.x), (int)blockIdx.y}, xT, Mx, items, nitems,
                                 perm, terms, op, grids, grid_total, vstride, slot_base, slots, Vtot);
}

// ------------------------------------------------------------------ order-2 gather in the
// polynomial basis of the window (FP32).
// Window point j of a node in cell f is the polynomial psi_j(z) = sum_q c[j][q] z^q of the
// node's offset z = 2 (n x + n/2 - f) - 1, the same polynomials for every cell.  The gather
// sum of a node in cell (f0, f1) is therefore a bivariate polynomial in (z0, z1) whose
// coefficients depend on the cell only:
//   f = sum_{a,j} psi_a(z0) psi_j(z1) G[f0-m+1+a][f1+j] = sum_{q',q} z0^q' z1^q K[q'][q],
//   K[q'][q] = sum_{a,j} c[a][q'] c[j][q] G[f0-m+1+a][f1+j]   (rows mod n, halo columns).
// k_pack_poly2 computes K for every cell of every term (the pack's DFT, then two separable
// passes, the window coefficients as scalar operands); k_gather_poly2 then evaluates the
// polynomial per node: (D+1) Horner sums in z1 and one in z0, 2 (D+1) D FMAs instead of the
// (2m)^2 complex window terms and the 4m window evaluations of the direct sum.

// The two separable passes for the cell rows F0 .. F0 + kPolyRows - 1 of one term and
// right-hand side, from the grid rows they need, Gs[hr] = row (F0 - m + 1 + hr) mod n
// (HR = kPolyRows + 2m - 1 rows of P halo columns, in LDS):
//   H[hr][f1][q] = sum_j c[j][q] Gs[hr][f1 + j]               (LDS, row stride NQ + 1)
//   K[f0][f1][q'][q] = sum_a c[a][q'] H[f0 - F0 + a][f1][q]    (kpoly: (r, term, f0, f1) blocks
//                                                               of NQ^2 complex, q fastest)
// The window coefficients c (2m x NQ, all points) are uniform scalar operands.  Ends with the
// second pass (callers place a barrier between their writes of Gs and this call).
template <int MH>
__device__ __forceinline__ void poly2_passes(const cx_t<float> *Gs, cx_t<float> *H, int n, int P,
                                             const float *__restrict__ c, int F0, int nt, int tl, int r,
                                             cx_t<float> *__restrict__ kpoly) {
  using C = cx_t<float>;
  constexpr int W = 2 * MH, NQ = Deg<float>::value + 1, HR = kPolyRows + W - 1, HS = NQ + 1;
  for (int task = threadIdx.x; task < HR * n; task += blockDim.x) {
    const int hr = task / n, f1 = task - hr * n;
    const C *g = Gs + hr * P + f1;
    C gv[W];
#pragma unroll
    for (int j = 0; j < W; ++j) gv[j] = g[j];
    C *hp = H + (hr * n + f1) * HS;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        sr = fmaf(c[j * NQ + q], gv[j].x, sr);
        si = fmaf(c[j * NQ + q], gv[j].y, si);
      }
      hp[q] = cmake<float>(sr, si);
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < kPolyRows * n * NQ; task += blockDim.x) {
    const int q = task % NQ, rest = task / NQ, f1 = rest % n, fr = rest / n, f0 = F0 + fr;
    if (f0 >= n) continue;
    C hv[W];
#pragma unroll
    for (int a = 0; a < W; ++a) hv[a] = H[((fr + a) * n + f1) * HS + q];
    C *dst = kpoly + ((((int64_t)r * nt + tl) * n + f0) * n + f1) * (NQ * NQ) + q;
#pragma unroll
    for (int qq = 0; qq < NQ; ++qq) {
      float sr = 0.f, si = 0.f;
#pragma unroll
      for (int a = 0; a < W; ++a) {
        sr = fmaf(c[a * NQ + qq], hv[a].x, sr);
        si = fmaf(c[a * NQ + qq], hv[a].y, si);
      }
      dst[qq * NQ] = cmake<float>(sr, si);
    }
  }
}

// Forward pack of the order-2 terms straight into the polynomial coefficients: workgroup =
// (term, right-hand side, kPolyRows cell rows).  The first two stages compute what k_pack_fwd
// computes (deconvolved coefficients A, then the DFT along the last axis, B), with the DFT
// factors tabulated in LDS; the last stage evaluates only the HR grid rows that the cell rows
// need, into LDS, and poly2_passes turns them into the cells' coefficients.  The grid itself
// is not stored.
template <int MH>
__device__ __forceinline__ void pack_poly2_body(const Blk bk, const cx_t<float> *__restrict__ fhat,
                                                const float *__restrict__ colscale, int64_t ncoef,
                                                const DevTerm *__restrict__ terms, const OrderParams<float> &op,
                                                int nslab, cx_t<float> *__restrict__ kpoly) {
  using C = cx_t<float>;
  constexpr int W = 2 * MH, NQ = Deg<float>::value + 1, HR = kPolyRows + W - 1, HS = NQ + 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int K = op.nfreq, n = op.n, P = op.P, h = op.N / 2, mm1 = MH - 1;
  const int nt = op.term_end - op.term_begin;
  const int tl = bk.x / nslab, F0 = (bk.x - tl * nslab) * kPolyRows, r = bk.y;
  const DevTerm tm = terms[op.term_begin + tl];
  const C *__restrict__ src = fhat + (int64_t)r * ncoef + tm.coef_off;
  const float *__restrict__ cs = colscale ? colscale + tm.coef_off : nullptr;
  const float *__restrict__ Dc = op.deconv;
  C *H = reinterpret_cast<C *>(smem_raw);   // HR x n x HS
  C *Gs = H + HR * n * HS;                  // HR x P
  C *A = Gs + HR * P;                       // K x K
  C *B = A + K * K;                         // K x n
  C *Wt = B + K * n;                        // K x n: e^{2 pi i k_a l / n}, k_a = -h..-1, 1..h-1
  const int tid = threadIdx.x, BS = blockDim.x;
  for (int i = tid; i < K * n; i += BS) {
    const int a = i / n, l = i - a * n, k = a < h ? a - h : a - h + 1;
    int e = (k * l) % n;
    e = e < 0 ? e + n : e;
    Wt[i] = cmake<float>(op.roots[2 * e], op.roots[2 * e + 1]);
  }
  for (int i = tid; i < K * K; i += BS) {
    const int a1 = i / K, a2 = i - a1 * K;
    const C v = src[i];
    const float sc = Dc[a1] * Dc[a2] * (cs ? cs[i] : 1.f);
    A[i] = cmake<float>(v.x * sc, v.y * sc);
  }
  __syncthreads();
  for (int i = tid; i < K * n; i += BS) {
    const int a1 = i / n, l2 = i - a1 * n;
    float re = 0.f, im = 0.f;
    for (int a2 = 0; a2 < K; ++a2) {
      const C v = A[a1 * K + a2], w = Wt[a2 * n + l2];
      re = fmaf(v.x, w.x, fmaf(-v.y, w.y, re));
      im = fmaf(v.x, w.y, fmaf(v.y, w.x, im));
    }
    B[i] = cmake<float>(re, im);
  }
  __syncthreads();
  for (int i = tid; i < HR * P; i += BS) {
    const int hr = i / P, p = i - hr * P;
    int l1 = (F0 - mm1 + hr) % n;
    l1 = l1 < 0 ? l1 + n : l1;
    int l2 = (p - mm1) % n;   // halo column -> grid column
    l2 = l2 < 0 ? l2 + n : l2;
    float re = 0.f, im = 0.f;
    for (int a1 = 0; a1 < K; ++a1) {
      const C v = B[a1 * n + l2], w = Wt[a1 * n + l1];
      re = fmaf(v.x, w.x, fmaf(-v.y, w.y, re));
      im = fmaf(v.x, w.y, fmaf(v.y, w.x, im));
    }
    Gs[i] = cmake<float>(re, im);
  }
  __syncthreads();
  poly2_passes<MH>(Gs, H, n, P, op.poly, F0, nt, tl, r, kpoly);
}

template <int MH>
__global__ __launch_bounds__(kPackBS) void k_pack_poly2(const cx_t<float> *__restrict__ fhat,
                                                        const float *__restrict__ colscale, int64_t ncoef,
                                                        const DevTerm *__restrict__ terms, OrderParams<float> op,
                                                        int nslab, cx_t<float> *__restrict__ kpoly) {
  pack_poly2_body<MH>(Blk{(int)blockIdx.x, (int)blockIdx.y}, fhat, colscale, ncoef, terms, op, nslab, kpoly);
}

typedef float v16f_t __attribute__((ext_vector_type(16)));

// Four consecutive 64-byte rows at a wavefront-uniform, 64-byte aligned address into scalar
// registers, as one round trip: the four scalar loads are issued back to back and waited for
// inside the same statement (the compiler otherwise waits after each row).  The outputs are
// early-clobber, so no row overlaps the address registers while the loads are in flight.
// The statement takes two values as (unused) inputs and so follows their computation: a
// second group takes the partial sums of the first, so each group is consumed as soon as it
// arrives and two groups are never live at once.
// The address is the same in every lane; it is moved into scalar registers explicitly, since
// the compiler may otherwise hand the "s" operand a vector register pair when it cannot tell
// that the value is uniform.
__device__ __forceinline__ void sload_rows4(const void *pv, v16f_t (&r)[4], float dep0, float dep1) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(pv);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(a & 0xffffffffull));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(a >> 32));
  const void *p = reinterpret_cast<const void *>(((unsigned long long)hi << 32) | lo);
  asm volatile(
      "s_load_dwordx16 %0, %4, 0x0\n\t"
      "s_load_dwordx16 %1, %4, 0x40\n\t"
      "s_load_dwordx16 %2, %4, 0x80\n\t"
      "s_load_dwordx16 %3, %4, 0xc0\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&s"(r[0]), "=&s"(r[1]), "=&s"(r[2]), "=&s"(r[3])
      : "s"(p), "v"(dep0), "v"(dep1)
      : "memory");
}

// One wavefront per run of at most 64 nodes of one cell (the cell gather's work items): the
// cell's (D+1)^2 coefficients are read with scalar loads and enter the lanes' Horner sums
// as scalar operands; the node coordinates come from the binning's sorted copy (xs, two
// per position).  Results go to the term's output slot as in k_gather_sorted.
template <typename T>
__device__ __forceinline__ void gather_poly2_body(const Blk bk, const float *__restrict__ xs,
                                                  const CellItem *__restrict__ items, int nitems,
                                                  const int32_t *__restrict__ perm, const OrderParams<float> &op,
                                                  const cx_t<float> *__restrict__ kpoly, int64_t vstride,
                                                  int slot_base, cx_t<float> *__restrict__ slots, int64_t Vtot) {
  static_assert(std::is_same<T, float>::value, "FP32 only");
  using C = cx_t<float>;
  constexpr int NQ = Deg<float>::value + 1;
  const int l = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ii = bk.x * 4 + wv;
  if (ii >= nitems) return;   // whole wavefront; no workgroup barrier follows
  const CellItem it = items[ii];
  const int r = it.r + bk.y;
  const int n = op.n, nt = op.term_end - op.term_begin;
  const bool act = l < it.count;
  const int c0 = it.cell[0], c1 = it.cell[1];
  const C *__restrict__ K = kpoly + ((((int64_t)r * nt + it.tl) * n + c0) * n + c1) * (NQ * NQ);
  const int pos = it.q0 + (act ? l : 0);
  // The node index and coordinates are read with relaxed workgroup-scope loads (plain global
  // loads): unlike reads through the read-only arguments, they keep their place ahead of the
  // coefficient loads, so both are in flight together.
  const int32_t node = __hip_atomic_load(perm + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const unsigned long long xb = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(xs) + pos,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const cx_t<float> xv = cmake<float>(__uint_as_float((unsigned)xb), __uint_as_float((unsigned)(xb >> 32)));
  const float nf = (float)n;
  const float z0 = fmaf(nf, xv.x, (float)(n / 2 - c0)) * 2.f - 1.f;
  const float z1 = fmaf(nf, xv.y, (float)(n / 2 - c1)) * 2.f - 1.f;
  static_assert(NQ == 8, "four 64-byte coefficient rows per load group");
  float fr = 0.f, fi = 0.f;
  // rows NQ-1 .. 4 of K, then rows 3 .. 0: two round trips for the cell's coefficients
#pragma unroll
  for (int grp = 1; grp >= 0; --grp) {
    v16f_t rows[4];
    sload_rows4(K + grp * 4 * NQ, rows, fr, fi);
#pragma unroll
    for (int qq = 3; qq >= 0; --qq) {
      const v16f_t &kr = rows[qq];
      float tr = kr[2 * NQ - 2], ti = kr[2 * NQ - 1];
#pragma unroll
      for (int q = NQ - 2; q >= 0; --q) {
        tr = fmaf(tr, z1, kr[2 * q]);
        ti = fmaf(ti, z1, kr[2 * q + 1]);
      }
      fr = fmaf(fr, z0, tr);
      fi = fmaf(fi, z0, ti);
    }
  }
  if (act) slots[(int64_t)(slot_base + op.term_begin + it.tl) * Vtot + (int64_t)r * vstride + node] = cmake<float>(fr, fi);
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_poly2(const float *__restrict__ xs,
                                                      const CellItem *__restrict__ items, int nitems,
                                                      const int32_t *__restrict__ perm,
                                                      OrderParams<float> op,
                                                      const cx_t<float> *__restrict__ kpoly, int64_t vstride,
                                                      int slot_base, cx_t<float> *__restrict__ slots, int64_t Vtot) {
  gather_poly2_body<T>(Blk{xcd_contiguous(blockIdx.x, gridDim.x), (int)blockIdx.y}, xs, items, nitems, perm, op, kpoly,
                       vstride, slot_base, slots, Vtot);
}

}  // namespace gt
