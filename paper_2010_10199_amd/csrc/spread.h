// K4 spread (adjoint), binned.  Orders 1 and 3: k_spread_binned, one workgroup of
// kSpreadWaves wavefronts per (term, right-hand side, range of cells), the cells dealt
// round-robin to the wavefronts.  Order 2: k_spread_tile2 below.
//
// The nodes of a term are sorted by the grid cell of their first window point (binning.hip).
// For one cell all nodes share the same window position, so the cell's contribution to the
// grid is a sum of outer products of window vectors:
//   order 1:  g[j]          += sum_v y_v psi_v[j]
//   order 3:  g[j1][j2][j3] += sum_v (y_v psi0_v[j1]) psi1_v[j2] psi2_v[j3]
// i.e. a dense contraction over the cell's nodes, done with 16x16x4 MFMA (4 nodes per step,
// window points padded to 16).  The patch is then added once per cell into the workgroup's
// LDS grid (FP64, LDS atomics): one LDS update per cell and window point instead of one per
// node and window point.
//
// In an MFMA step lane l works on window point l%16 of node l/16 (both operands use the
// same point index), so each lane keeps the polynomial coefficients of its window point in
// registers, and inside a cell the window argument is one FMA: z = 2 n x + (n - 2 fl - 1).
#pragma once

#include "gt_internal.h"

namespace gt {

typedef float v4f_t __attribute__((ext_vector_type(4)));
typedef double v4d_t __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator element r of
// lane l is D[row(l, r)][l%16] (FP32: rows 4(l/16)+r; FP64: rows 4r+l/16, measured).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc = v4f_t;
  static __device__ __forceinline__ acc run(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
  using acc = v4d_t;
  static __device__ __forceinline__ acc run(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
};

struct SpreadArgs {
  const int32_t *perm;     // order's sorted node indices (term-major, Mtot per term)
  const int64_t *cstart;   // first sorted position per (term, dataset, cell) key
  int32_t B;               // datasets (1 for shared nodes)
  int64_t ncell;           // binning keys per (term, dataset)
  int64_t vstride;         // virtual node of (r, node) = r * vstride + node  (M, or 0 when ragged)
  int32_t copies;          // order 1: 1 (one LDS grid, atomic adds) or kSpreadWaves (grid copies)
};

// Coefficients of one window point's polynomial, held in registers; zero past the window.
template <typename T>
struct WinPoint {
  T c[Deg<T>::value + 1];
  __device__ __forceinline__ void load(const T *__restrict__ poly, int j, int W) {
    constexpr int D = Deg<T>::value;
    const int jj = j < W ? j : W - 1;
#pragma unroll
    for (int q = 0; q <= D; ++q) c[q] = j < W ? poly[jj * (D + 1) + q] : (T)0;
  }
  __device__ __forceinline__ T operator()(T z) const {
    constexpr int D = Deg<T>::value;
    T acc = c[D];
#pragma unroll
    for (int q = D - 1; q >= 0; --q) acc = fma(acc, z, c[q]);
    return acc;
  }
};

// WV wavefronts per workgroup (kSpreadWaves on its own; fewer inside a shared launch), the
// item's cells dealt round-robin to them.
// Order 1 with sa.copies = kSpreadWaves: cell c0 + j adds its patch with plain adds into grid
// copy j mod kSpreadWaves, and the copies are summed in order at the end.  A copy is only
// ever written by one wavefront (WV divides kSpreadWaves), in increasing cell order, so the
// result depends neither on the timing of the wavefronts (the atomic adds into one shared
// grid meet in any order where neighbouring cells' windows overlap) nor on WV.  The plan
// takes this whenever the copies fit in LDS.
template <typename T, int ORDER, int MH, int WV>
__device__ __forceinline__ void spread_binned_body(const Blk bk, const T *__restrict__ xT, int64_t Mx,
                                                   const SpreadItem *__restrict__ items,
                                                   const DevTerm *__restrict__ terms, const OrderParams<T> &op,
                                                   const SpreadArgs &sa, const cx_t<T> *__restrict__ y,
                                                   cx_t<T> *__restrict__ gpart, int64_t gstride) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  constexpr int W = 2 * MH;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *G = reinterpret_cast<double2 *>(smem_raw);
  const SpreadItem it = items[bk.x];
  const int tl = bk.y;
  const DevTerm tm = terms[op.term_begin + tl];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, i16 = l & 15, kk = l >> 4;
  const int n = op.n, P = op.P, gsize = op.gsize;
  static_assert(kSpreadWaves % WV == 0, "a grid copy belongs to one wavefront");
  const int copies = ORDER == 1 ? sa.copies : 1;
  for (int i = threadIdx.x; i < copies * gsize; i += 64 * WV) G[i] = make_double2(0.0, 0.0);
  WinPoint<T> wp;
  wp.load(op.poly, i16, W);
  __syncthreads();
  const int64_t key0 = ((int64_t)tl * sa.B + it.b) * sa.ncell;
  const int64_t vbase = (int64_t)it.r * sa.vstride;
  const T *x0p = xT + (int64_t)tm.c0 * Mx;
  const T *x1p = xT + (int64_t)(ORDER >= 2 ? tm.c1 : tm.c0) * Mx;
  const T *x2p = xT + (int64_t)(ORDER >= 3 ? tm.c2 : tm.c0) * Mx;
  const T two_n = (T)(2 * n);
  for (int c = it.c0 + wv; c < it.c1; c += WV) {   // cells round-robin over the waves
    const int64_t p0 = sa.cstart[key0 + c], p1 = sa.cstart[key0 + c + 1];
    if (p1 <= p0) continue;
    // cell -> first window index per axis; z = 2 n x + (n - 2 fl - 1)
    int fl0, fl1 = 0, fl2 = 0;
    if (ORDER == 1) {
      fl0 = c;
    } else if (ORDER == 2) {
      fl0 = c / n;
      fl1 = c - fl0 * n;
    } else {
      fl0 = c / (n * n);
      const int rem = c - fl0 * n * n;
      fl1 = rem / n;
      fl2 = rem - fl1 * n;
    }
    const T zc0 = (T)(n - 2 * fl0 - 1), zc1 = (T)(n - 2 * fl1 - 1), zc2 = (T)(n - 2 * fl2 - 1);
    static_assert(ORDER != 2, "order 2 uses k_spread_tile2");
    if (ORDER == 1) {
      acc_t dre = {0, 0, 0, 0};
      // batches of 64 nodes: lane l loads node l of the batch once; the MFMA steps take the
      // window arguments and samples of their 4 nodes from those lanes
      for (int64_t b0 = p0; b0 < p1; b0 += 64) {
        const int64_t q = b0 + l;
        const bool valid = q < p1;
        const int32_t node = sa.perm[valid ? q : p0];
        cx_t<T> yl = y[vbase + node];
        const T za = fma(two_n, x0p[node], zc0);
        if (!valid) yl = cmake<T>(0, 0);
        const int steps = (int)((p1 - b0 + 3) >> 2) < 16 ? (int)((p1 - b0 + 3) >> 2) : 16;
        for (int st = 0; st < steps; ++st) {
          const int src = 4 * st + kk;
          const T z0 = __shfl(za, src, 64);
          const T yr = __shfl(yl.x, src, 64), yi = __shfl(yl.y, src, 64);
          const T w0 = wp(z0);
          const T a = i16 == 0 ? yr : (i16 == 1 ? yi : (T)0);
          dre = MF::run(a, w0, dre);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = MF::row(l, r);
        if (i16 < W && row < 2) {
          double2 *Gc = G + (copies > 1 ? ((c - it.c0) % copies) * gsize : 0);   // this cell's copy
          double *dst = row == 0 ? &Gc[fl0 + i16].x : &Gc[fl0 + i16].y;
          if (copies > 1)
            *dst += (double)dre[r];   // distinct addresses per lane; the wavefront's LDS order
          else
            atomicAdd(dst, (double)dre[r]);
        }
      }
    } else {
      // order 3: accumulator tiles over j2 (16 columns = j3), processed in passes of TP tiles
      constexpr int TP = sizeof(T) == 4 ? (W < 8 ? W : 8) : (W < 4 ? W : 4);
      const int rs0 = wrap_start(fl0, MH, n), rs1 = wrap_start(fl1, MH, n);
      for (int t0 = 0; t0 < W; t0 += TP) {
        acc_t dre[TP], dim[TP];
#pragma unroll
        for (int u = 0; u < TP; ++u) {
          dre[u] = acc_t{0, 0, 0, 0};
          dim[u] = acc_t{0, 0, 0, 0};
        }
        for (int64_t b0 = p0; b0 < p1; b0 += 64) {
          const int64_t q = b0 + l;
          const bool valid = q < p1;
          const int32_t node = sa.perm[valid ? q : p0];
          cx_t<T> yl = y[vbase + node];
          const T za = fma(two_n, x0p[node], zc0);
          const T zb = fma(two_n, x1p[node], zc1);
          const T zd = fma(two_n, x2p[node], zc2);
          if (!valid) yl = cmake<T>(0, 0);
          const int steps = (int)((p1 - b0 + 3) >> 2) < 16 ? (int)((p1 - b0 + 3) >> 2) : 16;
          for (int st = 0; st < steps; ++st) {
            const int src = 4 * st + kk;
            const T a = wp(__shfl(za, src, 64));
            const T ar = a * __shfl(yl.x, src, 64), ai = a * __shfl(yl.y, src, 64);
            const T p1own = wp(__shfl(zb, src, 64));
            const T p2own = wp(__shfl(zd, src, 64));
#pragma unroll
            for (int u = 0; u < TP; ++u) {
              const int t = t0 + u;
              const T p1t = __shfl(p1own, (l & 48) | (t < 16 ? t : 15), 64);
              const T b = (t < W) ? p1t * p2own : (T)0;
              dre[u] = MF::run(ar, b, dre[u]);
              dim[u] = MF::run(ai, b, dim[u]);
            }
          }
        }
#pragma unroll
        for (int u = 0; u < TP; ++u) {
          const int t = t0 + u;
          if (t >= W) continue;
          const int g1 = (rs1 + t) % n;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = MF::row(l, r);
            if (row < W && i16 < W) {
              const int g0 = (rs0 + row) % n;
              double2 *dst = &G[((int64_t)g0 * n + g1) * P + fl2 + i16];
              atomicAdd(&dst->x, (double)dre[u][r]);
              atomicAdd(&dst->y, (double)dim[u][r]);
            }
          }
        }
      }
    }
  }
  __syncthreads();
  cx_t<T> *out = gpart + (int64_t)bk.x * gstride + tm.gpart_off;
  for (int i = threadIdx.x; i < gsize; i += 64 * WV) {
    double re = G[i].x, im = G[i].y;
    for (int w = 1; w < copies; ++w) {
      re += G[w * gsize + i].x;
      im += G[w * gsize + i].y;
    }
    out[i] = cmake<T>((T)re, (T)im);
  }
}

template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(64 * kSpreadWaves) void k_spread_binned(const T *__restrict__ xT, int64_t Mx,
                                                                     const SpreadItem *__restrict__ items,
                                                                     const DevTerm *__restrict__ terms,
                                                                     OrderParams<T> op, SpreadArgs sa,
                                                                     const cx_t<T> *__restrict__ y,
                                                                     cx_t<T> *__restrict__ gpart, int64_t gstride) {
  spread_binned_body<T, ORDER, MH, kSpreadWaves>(Blk{(int)blockIdx.x, (int)blockIdx.y}, xT, Mx, items, terms, op, sa,
                                                 y, gpart, gstride);
}

// Order-3 spread, MFMA tiles without window padding.  For one cell the contribution
//   g[j1][j2][j3] += sum_v (y_v psi0_v[j1]) psi1_v[j2] psi2_v[j3]
// is the product of a (real/imaginary part, j1) x node matrix with a node x (j2, j3) matrix:
// rows 2W (one 16-row tile at W = 8), columns W^2 in 16-column tiles (column 16 ct + i holds
// j2 = (16 ct + i) / W, j3 = (16 ct + i) % W).  At the FP32 path's W = 8 a step of four nodes
// takes 4 MFMAs instead of the 16 of a tile per j2 padded to 16 x 16; at W = 16 the count is
// unchanged.  Lane (node b, i) evaluates the window of its own point i mod W on all three axes
// (one Horner sum each, the point's coefficients held in registers) and takes the other
// points it needs from the lanes holding them (shuffles within the node's 16 lanes).  Column
// tiles are taken CP at a time (accumulator registers), each pass walking the cell's nodes.
// Per cell the accumulators are added into the workgroup's FP64 LDS grid (atomics, as in
// k_spread_binned), which is written out as the workgroup's partial grid.
template <typename T, int MH>
__global__ __launch_bounds__(64 * kSpreadWaves) void k_spread_cell3(const T *__restrict__ xT, int64_t Mx,
                                                                    const SpreadItem *__restrict__ items,
                                                                    const DevTerm *__restrict__ terms,
                                                                    OrderParams<T> op, SpreadArgs sa,
                                                                    const cx_t<T> *__restrict__ y,
                                                                    cx_t<T> *__restrict__ gpart, int64_t gstride) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  constexpr int W = 2 * MH;
  constexpr int RT = (2 * W + 15) / 16, CT = (W * W + 15) / 16;
  constexpr int CP = sizeof(T) == 4 ? (CT < 4 ? CT : 4) : (CT < 4 ? CT : 4);   // column tiles per pass
  static_assert(RT * CP <= 8, "accumulator registers");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *G = reinterpret_cast<double2 *>(smem_raw);
  const SpreadItem it = items[blockIdx.x];
  const int tl = blockIdx.y;
  const DevTerm tm = terms[op.term_begin + tl];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, i16 = l & 15, kk = l >> 4, base = l & 48;
  const int n = op.n, P = op.P, gsize = op.gsize;
  for (int i = threadIdx.x; i < gsize; i += 64 * kSpreadWaves) G[i] = make_double2(0.0, 0.0);
  WinPoint<T> wp;   // the lane's own window point i mod W, all three axes
  wp.load(op.poly, i16 % W, W);
  __syncthreads();
  const int64_t key0 = ((int64_t)tl * sa.B + it.b) * sa.ncell;
  const int64_t vbase = (int64_t)it.r * sa.vstride;
  const T *x0p = xT + (int64_t)tm.c0 * Mx, *x1p = xT + (int64_t)tm.c1 * Mx, *x2p = xT + (int64_t)tm.c2 * Mx;
  const T two_n = (T)(2 * n);
  for (int c = it.c0 + wv; c < it.c1; c += kSpreadWaves) {   // cells round-robin over the waves
    const int64_t p0 = sa.cstart[key0 + c], p1 = sa.cstart[key0 + c + 1];
    if (p1 <= p0) continue;
    const int fl0 = c / (n * n), rem = c - fl0 * n * n, fl1 = rem / n, fl2 = rem - fl1 * n;
    const T zc0 = (T)(n - 2 * fl0 - 1), zc1 = (T)(n - 2 * fl1 - 1), zc2 = (T)(n - 2 * fl2 - 1);
    const int rs0 = wrap_start(fl0, MH, n), rs1 = wrap_start(fl1, MH, n);
    for (int ct0 = 0; ct0 < CT; ct0 += CP) {
      acc_t acc[RT][CP];
#pragma unroll
      for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int u = 0; u < CP; ++u) acc[a][u] = acc_t{0, 0, 0, 0};
      for (int64_t b0 = p0; b0 < p1; b0 += 64) {
        const int64_t q = b0 + l;
        const bool valid = q < p1;
        const int32_t node = sa.perm[valid ? q : p0];
        cx_t<T> yl = y[vbase + node];
        const T za = fma(two_n, x0p[node], zc0);
        const T zb = fma(two_n, x1p[node], zc1);
        const T zd = fma(two_n, x2p[node], zc2);
        if (!valid) yl = cmake<T>(0, 0);
        const int steps = (int)((p1 - b0 + 3) >> 2) < 16 ? (int)((p1 - b0 + 3) >> 2) : 16;
        for (int st = 0; st < steps; ++st) {
          const int src = 4 * st + kk;
          const T w0 = wp(__shfl(za, src, 64));
          const T w1 = wp(__shfl(zb, src, 64));
          const T w2 = wp(__shfl(zd, src, 64));
          const T yr = __shfl(yl.x, src, 64), yi = __shfl(yl.y, src, 64);
          T av[RT];
#pragma unroll
          for (int a = 0; a < RT; ++a) {
            const int row = 16 * a + i16;
            const int part = row / W, j1 = row % W;
            const T p0v = ((16 * a) % W == 0) ? w0 : __shfl(w0, base | j1, 64);
            av[a] = row < 2 * W ? p0v * (part ? yi : yr) : (T)0;
          }
#pragma unroll
          for (int u = 0; u < CP; ++u) {
            const int ct = ct0 + u;
            if (ct >= CT) break;
            const int col = 16 * ct + i16;
            const int j2 = col / W, j3 = col % W;
            const T p2v = ((16 * ct) % W == 0) ? w2 : __shfl(w2, base | j3, 64);
            const T p1v = __shfl(w1, base | (j2 < W ? j2 : 0), 64);
            const T bv = col < W * W ? p1v * p2v : (T)0;
#pragma unroll
            for (int a = 0; a < RT; ++a) acc[a][u] = MF::run(av[a], bv, acc[a][u]);
          }
        }
      }
      // accumulator element e of lane l: row MF::row(l, e) of row tile a, column 16 ct + i16
#pragma unroll
      for (int u = 0; u < CP; ++u) {
        const int ct = ct0 + u;
        if (ct >= CT) break;
        const int col = 16 * ct + i16;
        if (col >= W * W) continue;
        const int j2 = col / W, j3 = col % W;
        const int g1 = (rs1 + j2) % n;
#pragma unroll
        for (int a = 0; a < RT; ++a)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int row = 16 * a + MF::row(l, e);
            if (row >= 2 * W) continue;
            const int part = row / W, j1 = row % W;
            const int g0 = (rs0 + j1) % n;
            double2 *dst = &G[((int64_t)g0 * n + g1) * P + fl2 + j3];
            atomicAdd(part ? &dst->y : &dst->x, (double)acc[a][u][e]);
          }
      }
    }
  }
  __syncthreads();
  cx_t<T> *out = gpart + (int64_t)blockIdx.x * gstride + tm.gpart_off;
  for (int i = threadIdx.x; i < gsize; i += 64 * kSpreadWaves) out[i] = cmake<T>((T)G[i].x, (T)G[i].y);
}

// Orders the LDS accesses of one wavefront: staging writes by some lanes before reads by
// other lanes of the same wavefront (and those reads before the next overwrite).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Order-2 spread on tiles of TS x TS grid cells, TS = 17 - 2m (the binning numbers cells
// tile-major, so a tile's nodes are contiguous in sorted order).  Every node of a tile has
// its 2m x 2m window inside one 16 x 16 patch of the grid, at offset (s0, s1) = its cell
// minus the tile's first cell, so the tile's contribution is the patch
//   Pt[i][j] = sum_v A_v[i] B_v[j],   A_v[s0 + a] = y_v psi(axis 0)[a],  B_v[s1 + b] = psi(axis 1)[b],
// a dense contraction over the tile's nodes, done with 16x16x4 MFMA (4 nodes per step).
//
// Each wavefront owns a run of sorted positions of one (term, dataset) from the plan's work
// list and walks it in batches of 32: lanes 0..31 evaluate the window along axis 0 of one
// node each, lanes 32..63 along axis 1, and both halves stage their shifted, zero-padded
// real 16-vectors in LDS with the same instructions; the batch's samples go to LDS beside
// them.  8 MFMA steps read the rows back as operands and form A = y psi(axis 0) as they
// read it (the same single product as staging it, so the patch does not change), samples of
// nodes outside the batch or the tile being zero.  The nodes of a batch usually share one
// tile; when a tile ends inside the batch, the batch is run once per tile with the other
// tiles' samples zeroed, each run taking only the MFMA steps that hold nodes of its tile (as
// does a short last batch).  At each tile change the wavefront stores its finished patch, with plain
// stores, in its next patch slot (slots are numbered per wavefront in tile order); the
// fold kernel adds the patches into the grids in a fixed order.  Nothing is shared between
// wavefronts, so there are no atomics and no workgroup barriers.
//
// Inputs stream with a four-deep register pipeline: sorted node indices and the sorted
// coordinates (plan array xs) three batches ahead, the samples (gathered through the node
// index) one batch ahead.
template <typename T>
struct TileStage {
  int32_t p;    // node index
  cx_t<T> x;    // the node's coordinates along the term's two axes
  cx_t<T> y;    // sample
};

struct Tile2Args {
  const int32_t *waves;    // per wavefront: first position, end position, first patch slot, dataset
  int32_t nwaves;
  int32_t ntile;           // tiles per axis
  int64_t nseg;            // patch slots per right-hand side
  int64_t vstride;         // sample of (r, node) = y[r * vstride + node]  (M, or 0 when ragged)
  int32_t ragged;          // datasets own their samples: r = dataset, one set of slots
};

// floor(f / TS) for 0 <= f < 2^15 + 3 (every grid index: n <= 8 x 4096 + 2) as
// floor(f K / 2^S), K = ceil(2^S / TS), with the full-rate 24-bit multiply: S is the largest
// shift with f K < 2^32 and f (K TS - 2^S) < 2^S over that range (then the product's excess
// over f / TS stays below 1 / TS, so the floor is exact).
constexpr unsigned kCellMax = (1u << 15) + 3;
constexpr int div_shift(int ts) {
  for (int S = 23; S >= 8; --S) {
    const unsigned long long K = ((1ull << S) + ts - 1) / ts, e = K * ts - (1ull << S);
    if (K * kCellMax < (1ull << 32) && e * kCellMax < (1ull << S) && K < (1ull << 24)) return S;
  }
  return -1;
}
template <int TS>
__device__ __forceinline__ int div_tile(int f) {
  if constexpr (TS == 1) {
    return f;
  } else {
    constexpr int S = div_shift(TS);
    static_assert(S > 0, "no exact 24-bit division for this tile side");
    constexpr unsigned K = (unsigned)(((1ull << S) + TS - 1) / TS);
    return (int)(__umul24((unsigned)f, K) >> S);
  }
}

// Window values as window_values computes them, with the leading coefficient of each part in
// a vector register (lead[2j]: even part of point j, lead[2j + 1]: odd part), so the first
// step of each Horner chain reads one scalar operand instead of two (no register move).
template <typename T, int MH>
__device__ __forceinline__ void window_values_lead(T z, const T *cf, const T *lead, T (&psi)[2 * MH]) {
  constexpr int D = Deg<T>::value;
  constexpr int DE = D - (D & 1), DO = D - 1 + (D & 1);
  static_assert(DE >= 2 && DO >= 3, "two steps per part at least");
  const T z2 = z * z;
#pragma unroll
  for (int j = 0; j < MH; ++j) {
    const T *c = cf + j * (D + 1);
    T e = fma(lead[2 * j], z2, c[DE - 2]);
#pragma unroll
    for (int q = DE - 4; q >= 0; q -= 2) e = fma(e, z2, c[q]);
    T o = fma(lead[2 * j + 1], z2, c[DO - 2]);
#pragma unroll
    for (int q = DO - 4; q >= 1; q -= 2) o = fma(o, z2, c[q]);
    o *= z;
    psi[j] = e + o;
    psi[2 * MH - 1 - j] = e - o;
  }
}

// Window values as window_values computes them, the coefficients read as vector operands
// (from a table in LDS: every lane reads the same entries).
template <typename T, int MH>
__device__ __forceinline__ void window_values_plain(T z, const T *c0, T (&psi)[2 * MH]) {
  constexpr int D = Deg<T>::value;
  constexpr int DE = D - (D & 1), DO = D - 1 + (D & 1);
  const T z2 = z * z;
#pragma unroll
  for (int j = 0; j < MH; ++j) {
    const T *c = c0 + j * (D + 1);
    T e = c[DE];
#pragma unroll
    for (int q = DE - 2; q >= 0; q -= 2) e = fma(e, z2, c[q]);
    T o = c[DO];
#pragma unroll
    for (int q = DO - 2; q >= 1; q -= 2) o = fma(o, z2, c[q]);
    o *= z;
    psi[j] = e + o;
    psi[2 * MH - 1 - j] = e - o;
  }
}

template <typename T, int MH>
__device__ __forceinline__ void spread_tile2_body(const Blk bk, const T *__restrict__ xs,
                                                  const int32_t *__restrict__ perm, const OrderParams<T> &op,
                                                  const Tile2Args &ta, const cx_t<T> *__restrict__ y,
                                                  cx_t<T> *__restrict__ patch) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  using C = cx_t<T>;
  constexpr int W = 2 * MH, TS = tile_side(MH), UB = kTileBatch, SR = kTileRow;
  static_assert(TS >= 1 && TS + W - 1 == 16, "tile patch must be 16 x 16");
  static_assert(UB == 32, "one node per lane pair of a wavefront");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int l = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform per wavefront
  const int h = l >> 5, j = l & 31, i16 = l & 15, kk = l >> 4;
  T *SAw = reinterpret_cast<T *>(smem_raw + (size_t)wv * tile_lds_wave(sizeof(T)));   // UB x SR, axis 0
  T *SBw = SAw + UB * SR;                                                               // UB x SR, axis 1
  C *Yw = reinterpret_cast<C *>(SBw + UB * SR);                                         // UB samples
  T *const myrow = (h ? SBw : SAw) + j * SR;
  const int w = bk.x * kTileWaves + wv;
  if (w >= ta.nwaves) return;   // whole wavefront; the kernel has no workgroup barrier
  const int32_t qbeg = ta.waves[4 * w], qend = ta.waves[4 * w + 1];
  int64_t slot = ta.waves[4 * w + 2];
  const int r = ta.ragged ? ta.waves[4 * w + 3] : bk.y;
  if (!ta.ragged) slot += (int64_t)bk.y * ta.nseg;
  const int nbat = (qend - qbeg + UB - 1) / UB;
  const int64_t vbase = (int64_t)r * ta.vstride;
  const int n = op.n, ntile = ta.ntile;
  // window polynomial coefficients of points 0..m-1 (the others mirror them): FP32 (8 per
  // point) in scalar registers, with the leading coefficient of each part in a vector
  // register; FP64 (15 per point, more than the scalar registers hold: the compiler keeps
  // them in vector-register lanes and reads them back one by one for every batch) in the
  // wavefront's LDS, read as vector operands where used, up to m = 7 (at m = 8 that form
  // takes over 300 registers, so it keeps the scalar form)
  constexpr int NC = MH * (Deg<T>::value + 1);
  constexpr bool kLead = std::is_same<T, float>::value;
  constexpr bool kTable = !kLead && MH <= 7;
  T *const tbl = reinterpret_cast<T *>(Yw + UB);   // (kTable) NC coefficients
  T cf[kTable ? 1 : NC];
  T lead[2 * MH];
  if constexpr (kTable) {
    for (int i = l; i < NC; i += 64) tbl[i] = op.poly[i];
    wave_lds_sync();
  } else {
#pragma unroll
    for (int i = 0; i < NC; ++i) cf[i] = wave_uniform(op.poly[i]);
  }
  if constexpr (kLead) {
#pragma unroll
    for (int i = 0; i < MH; ++i) {
      constexpr int D = Deg<T>::value;
      lead[2 * i] = cf[i * (D + 1) + D - (D & 1)];
      lead[2 * i + 1] = cf[i * (D + 1) + D - 1 + (D & 1)];
      asm volatile("" : "+v"(lead[2 * i]));   // held in vector registers from here on
      asm volatile("" : "+v"(lead[2 * i + 1]));
    }
  }

  // Loads are issued unconditionally (positions past the wavefront's range are clamped to
  // its last node), so the wait counts stay exact across the unrolled pipeline.
  const C *__restrict__ xs2 = reinterpret_cast<const C *>(xs);
  auto issue_px = [&](TileStage<T> &s, int k) {
    int32_t q = qbeg + k * UB + j;
    q = q < qend ? q : qend - 1;
    s.p = perm[q];
    s.x = xs2[q];
  };
  auto issue_y = [&](TileStage<T> &s) { s.y = y[vbase + s.p]; };

  acc_t are = {0, 0, 0, 0}, aim = {0, 0, 0, 0};
  int cur_tile = -1;
  bool dirty = false;
  auto store_patch = [&]() {   // patch row MF::row(l, r), column i16
    C *dst = patch + slot * 256 + i16;
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[MF::row(l, q) * 16] = cmake<T>((T)are[q], (T)aim[q]);
    ++slot;
    are = acc_t{0, 0, 0, 0};
    aim = acc_t{0, 0, 0, 0};
  };
  auto process = [&](const TileStage<T> &st, int k) {
    const bool valid = qbeg + k * UB + j < qend;
    // this lane's axis: cell and offset; the other axis: cell only
    int fh, fo;
    const T z = frac_offset<T>(h ? st.x.y : st.x.x, n, fh) * (T)2 - (T)1;
    (void)frac_offset<T>(h ? st.x.x : st.x.y, n, fo);
    T psi[W];
    if constexpr (kLead)
      window_values_lead<T, MH>(z, cf, lead, psi);
    else if constexpr (kTable)
      window_values_plain<T, MH>(z, tbl, psi);
    else
      window_values<T, MH>(z, cf, psi);
    const int ty = div_tile<TS>(h ? fo : fh), tx = div_tile<TS>(h ? fh : fo);
    const int tile = valid ? (int)__umul24((unsigned)ty, (unsigned)ntile) + tx : 0x7fffffff;
    const int s = fh - __mul24(h ? tx : ty, TS);
    // the row: zeros where a window at some offset s in [0, TS) may not reach ([0, 16 - W)
    // and [W, 16)), then the window values at [s, s + W), over them (a wavefront's LDS
    // writes take effect in order)
#pragma unroll
    for (int q = 0; q < 16 - W; ++q) {
      myrow[q] = (T)0;
      myrow[W + q] = (T)0;
    }
#pragma unroll
    for (int a = 0; a < W; ++a) myrow[s + a] = psi[a];
    unsigned long long pending = __ballot(valid);
    while (pending) {
      const int t = __builtin_amdgcn_readlane(tile, __ffsll((long long)pending) - 1);
      const bool in = tile == t;
      if (t != cur_tile) {
        if (dirty) store_patch();
        cur_tile = t;
      }
      Yw[j] = in ? st.y : cmake<T>((T)0, (T)0);   // (both halves write the same value)
      // the tile's nodes lie in steps q0 .. q1 (node j in step j / 4; lane j holds node j);
      // the other steps carry zero samples only and are skipped, which leaves the patch as it is
      constexpr bool kSkip = std::is_same<T, float>::value || MH == 8;
      const unsigned long long inm = __ballot(in);
      const unsigned lo = (unsigned)inm;
      const int q0 = (__ffs((int)lo) - 1) >> 2, q1 = (31 - __clz((int)lo)) >> 2;
      wave_lds_sync();
      // (FP64 below m = 8 runs every step: the second path costs it a wavefront per SIMD)
      if (!kSkip || (q0 == 0 && q1 == UB / 4 - 1)) {   // every step holds a node of the tile
        T av[UB / 4], bv[UB / 4];
        C yv[UB / 4];
#pragma unroll
        for (int q = 0; q < UB / 4; ++q) {
          av[q] = SAw[(4 * q + kk) * SR + i16];
          bv[q] = SBw[(4 * q + kk) * SR + i16];
          yv[q] = Yw[4 * q + kk];
        }
#pragma unroll
        for (int q = 0; q < UB / 4; ++q) {
          are = MF::run(av[q] * yv[q].x, bv[q], are);
          aim = MF::run(av[q] * yv[q].y, bv[q], aim);
        }
      } else {
#pragma unroll 1
        for (int q = q0; q <= q1; ++q) {
          const T av = SAw[(4 * q + kk) * SR + i16], bv = SBw[(4 * q + kk) * SR + i16];
          const C yv = Yw[4 * q + kk];
          are = MF::run(av * yv.x, bv, are);
          aim = MF::run(av * yv.y, bv, aim);
        }
      }
      wave_lds_sync();
      dirty = true;
      pending &= ~inm;
    }
  };

  if (nbat > 0) {
    TileStage<T> S[4];
    issue_px(S[0], 0);
    issue_px(S[1], 1);
    issue_px(S[2], 2);
    issue_y(S[0]);
    for (int k0 = 0; k0 < nbat; k0 += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + u;
        issue_px(S[(u + 3) & 3], k + 3);
        issue_y(S[(u + 1) & 3]);
        if (k < nbat) process(S[u], k);
      }
    }
  }
  if (dirty) store_patch();
}

template <typename T, int MH>
__global__ __launch_bounds__(64 * kTileWaves) void k_spread_tile2(const T *__restrict__ xs,
                                                                  const int32_t *__restrict__ perm, OrderParams<T> op,
                                                                  Tile2Args ta, const cx_t<T> *__restrict__ y,
                                                                  cx_t<T> *__restrict__ patch) {
  spread_tile2_body<T, MH>(Blk{(int)blockIdx.x, (int)blockIdx.y}, xs, perm, op, ta, y, patch);
}

// Fold of the order-2 tile patches into the folded grids, in two separable passes with a
// fixed summation order (so the result is deterministic): the columns here, the rows at the
// start of the order-2 adjoint DFT (k_dft_adj).
// k_fold_cols: one thread per (right-hand side, term, tile row ty, patch row pr, grid column
//   l1) adds, over the halo columns p = l1 + m - 1 (mod n), the tile columns tx whose patch
//   covers p and each tile's patches in slot order, the patch entries (pr, p - tx ts):
//   hcol[(r * terms + tl) * ntile + ty][pr][l1].
//   The (p, tx, slot) sequence is flattened: the tiles' slot ranges are read first, all at
//   once, and the patch entries are then loaded eight at a time and added in sequence order,
//   so a thread has its loads in flight together instead of one per loop step.
//   Needs P <= 2n (at most two halo positions per column); NX >= 15 / ts + 1 bounds the
//   tiles covering one halo column.
template <typename T, int NX>
__global__ __launch_bounds__(256) void k_fold_cols(const cx_t<T> *__restrict__ patch,
                                                   const int32_t *__restrict__ tileseg, OrderParams<T> op,
                                                   Tile2Args ta, int B, int ts, cx_t<T> *__restrict__ hcol) {
  constexpr int NC = 2 * NX, U = 8;   // (p, tx) combinations; loads per step
  const int n = op.n, P = op.P, mm1 = op.m - 1, ntile = ta.ntile, ntiles = ntile * ntile;
  const int nt = op.term_end - op.term_begin;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // ((tl * ntile + ty) * 16 + pr) * n + l1
  if (idx >= (int64_t)nt * ntile * 16 * n) return;
  const int r = blockIdx.y;
  const int l1 = (int)(idx % n);
  const int pr = (int)((idx / n) & 15);
  const int64_t tty = idx / (16 * n);   // tl * ntile + ty
  const int tl = (int)(tty / ntile), ty = (int)(tty - (int64_t)tl * ntile);
  const int b = ta.ragged ? r : 0;
  const int64_t pbase = ta.ragged ? 0 : (int64_t)r * ta.nseg;
  const int32_t *tsg = tileseg + ((int64_t)tl * B + b) * ntiles + ty * ntile;
  // combination c = (pi, k): halo column p = p0 + pi n (if p < P), tile tx = tx0(p) + k (if
  // tx <= tx1(p)); its slots [cs, cs + cc) and patch column co = p - tx ts
  const int p0 = (l1 + mm1) % n;
  int txa[2], txb[2];
#pragma unroll
  for (int pi = 0; pi < 2; ++pi) {   // first tile ceil((p - 15) / ts) clamped at 0, last floor(p / ts)
    const int p = p0 + pi * n;
    txa[pi] = max(0, p - 16 + ts) / ts;
    txb[pi] = p < P ? min(p / ts, ntile - 1) : -1;
  }
  int s0[NC], s1[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {   // every bound load issued before the first use
    const int tx = txa[c / NX] + c % NX;
    const int txc = tx <= txb[c / NX] ? tx : 0;   // valid rows of tsg hold ntile + 1 bounds
    s0[c] = tsg[txc];
    s1[c] = tsg[txc + 1];
  }
  int cs[NC], cc[NC], co[NC], pre[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int tx = txa[c / NX] + c % NX;
    cs[c] = s0[c];
    cc[c] = tx <= txb[c / NX] ? s1[c] - s0[c] : 0;
    co[c] = p0 + (c / NX) * n - tx * ts;
  }
  int total = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    pre[c] = total;
    total += cc[c];
  }
  const cx_t<T> *src = patch + pbase * 256 + pr * 16;
  T re = 0, im = 0;
  for (int j0 = 0; j0 < total; j0 += U) {
    cx_t<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u < total ? j0 + u : total - 1;   // past the end: reload the last entry
      int sg = 0, col = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c)   // the last combination starting at or before j (never empty)
        if (j >= pre[c]) {
          sg = cs[c] + (j - pre[c]);
          col = co[c];
        }
      v[u] = src[(int64_t)sg * 256 + col];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j0 + u < total) {
        re += v[u].x;
        im += v[u].y;
      }
  }
  hcol[((int64_t)r * nt * ntile + tty) * 16 * n + pr * n + l1] = cmake<T>(re, im);
}

// k_fold_tilesum: the same column sums with coalesced patch reads, one wavefront per (right-
//   hand side, term, tile row ty, group of four patch rows).  The patches of one tile row are
//   the consecutive slots of its tiles, so lane (pr, k) reads entry (pr, k) of every slot of
//   the row in turn (a load instruction covers four whole patch rows), sixteen slots in
//   flight; the tile of a slot comes from a ballot over the row's tile bounds.  Each lane
//   sums its entry over the slots of each tile, in slot order, into LDS (tile sums, zero for
//   tiles without patches); the wavefront then forms every output column of its rows as the
//   sum over the halo columns p = l1 + m - 1 (mod n), ascending, and over the tiles tx
//   covering p, ascending, of the tile sums at (pr, p - tx ts).
//   Needs P <= 2n and ntile <= 32 (LDS: ntile x 64 entries).
template <typename T>
__device__ __forceinline__ void fold_tilesum_body(const Blk bk, cx_t<T> *tsum, const cx_t<T> *__restrict__ patch,
                                                  const int32_t *__restrict__ tileseg, const OrderParams<T> &op,
                                                  const Tile2Args &ta, int B, int ts, cx_t<T> *__restrict__ hcol) {
  // tsum: this wavefront's LDS, [tx][row of the group][column], 64 per tile
  using C = cx_t<T>;
  constexpr int U = 16;
  const int n = op.n, P = op.P, mm1 = op.m - 1, ntile = ta.ntile, ntiles = ntile * ntile;
  const int nt = op.term_end - op.term_begin;
  const int lane = threadIdx.x & 63;
  const int g = bk.x & 3;                // patch rows 4g .. 4g + 3
  const int tty = bk.x >> 2;             // tl * ntile + ty
  const int tl = tty / ntile, ty = tty - tl * ntile;
  const int r = bk.y;
  const int b = ta.ragged ? r : 0;
  const int64_t pbase = ta.ragged ? 0 : (int64_t)r * ta.nseg;
  const int32_t *tsg = tileseg + ((int64_t)tl * B + b) * ntiles + ty * ntile;
  const int bound = lane < ntile ? tsg[lane] : 0x7fffffff;   // first slot of tile `lane`
  const int sbeg = tsg[0], send = tsg[ntile];
  for (int tx = 0; tx < ntile; ++tx) tsum[tx * 64 + lane] = cmake<T>((T)0, (T)0);
  const C *src = patch + (pbase + sbeg) * 256 + 64 * g + lane;
  T sr = 0, si = 0;
  int ct = -1;   // tile being summed
  for (int j0 = sbeg; j0 < send; j0 += U) {
    C v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u < send ? j0 + u : send - 1;   // past the end: reload the last slot
      v[u] = src[(int64_t)(j - sbeg) * 256];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u;
      if (j < send) {
        // tile of slot j: the last tile whose first slot is <= j (bounds are nondecreasing)
        const int tx = __popcll(__ballot(bound <= j)) - 1;
        if (tx != ct) {
          if (ct >= 0) tsum[ct * 64 + lane] = cmake<T>(sr, si);
          sr = 0;
          si = 0;
          ct = tx;
        }
        sr += v[u].x;
        si += v[u].y;
      }
    }
  }
  if (ct >= 0) tsum[ct * 64 + lane] = cmake<T>(sr, si);
  wave_lds_sync();   // the tile sums are this wavefront's own
  for (int o = lane; o < 4 * n; o += 64) {
    const int rl = o / n, l1 = o - rl * n;
    const int p0 = (l1 + mm1) % n;
    T re = 0, im = 0;
    for (int p = p0; p < P; p += n) {
      const int tx0 = max(0, p - 16 + ts) / ts, tx1 = min(p / ts, ntile - 1);
      for (int tx = tx0; tx <= tx1; ++tx) {
        const C t = tsum[tx * 64 + rl * 16 + (p - tx * ts)];
        re += t.x;
        im += t.y;
      }
    }
    hcol[((int64_t)r * nt * ntile + tty) * 16 * n + (4 * g + rl) * n + l1] = cmake<T>(re, im);
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_fold_tilesum(const cx_t<T> *__restrict__ patch,
                                                     const int32_t *__restrict__ tileseg, OrderParams<T> op,
                                                     Tile2Args ta, int B, int ts, cx_t<T> *__restrict__ hcol) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fold_tilesum_body<T>(Blk{(int)blockIdx.x, (int)blockIdx.y}, reinterpret_cast<cx_t<T> *>(smem_raw), patch, tileseg,
                       op, ta, B, ts, hcol);
}

// k_fold_cols_seq: the same sums, one (p, tx, slot) step at a time, for grids narrower than
//   the halo (n < 2m - 1, where a column has more than two halo positions).
template <typename T>
__global__ __launch_bounds__(256) void k_fold_cols_seq(const cx_t<T> *__restrict__ patch,
                                                       const int32_t *__restrict__ tileseg, OrderParams<T> op,
                                                       Tile2Args ta, int B, int ts, cx_t<T> *__restrict__ hcol) {
  const int n = op.n, P = op.P, mm1 = op.m - 1, ntile = ta.ntile, ntiles = ntile * ntile;
  const int nt = op.term_end - op.term_begin;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // ((tl * ntile + ty) * 16 + pr) * n + l1
  if (idx >= (int64_t)nt * ntile * 16 * n) return;
  const int r = blockIdx.y;
  const int l1 = (int)(idx % n);
  const int pr = (int)((idx / n) & 15);
  const int64_t tty = idx / (16 * n);   // tl * ntile + ty
  const int tl = (int)(tty / ntile), ty = (int)(tty - (int64_t)tl * ntile);
  const int b = ta.ragged ? r : 0;
  const int64_t pbase = ta.ragged ? 0 : (int64_t)r * ta.nseg;
  const int32_t *tsg = tileseg + ((int64_t)tl * B + b) * ntiles + ty * ntile;
  T re = 0, im = 0;
  for (int p = (l1 + mm1) % n; p < P; p += n) {
    const int tx0 = p >= 15 ? (p - 15 + ts - 1) / ts : 0;
    const int tx1 = p / ts < ntile - 1 ? p / ts : ntile - 1;
    for (int tx = tx0; tx <= tx1; ++tx) {
      const cx_t<T> *src = patch + pbase * 256 + pr * 16 + (p - tx * ts);
      for (int sg = tsg[tx]; sg < tsg[tx + 1]; ++sg) {
        const cx_t<T> v = src[(int64_t)sg * 256];
        re += v.x;
        im += v.y;
      }
    }
  }
  hcol[((int64_t)r * nt * ntile + tty) * 16 * n + pr * n + l1] = cmake<T>(re, im);
}

}  // namespace gt
