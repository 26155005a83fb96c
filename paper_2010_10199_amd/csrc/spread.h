// K4 spread (adjoint): binned; one workgroup of kSpreadWaves wavefronts per (term,
// right-hand side, range of cells), the cells dealt round-robin to the wavefronts.
//
// The nodes of a term are sorted by the grid cell of their first window point (binning.hip).
// For one cell all nodes share the same window position, so the cell's contribution to the
// grid is a sum of outer products of window vectors:
//   order 1:  g[j]          += sum_v y_v psi_v[j]
//   order 2:  g[j1][j2]     += sum_v (y_v psi0_v[j1]) psi1_v[j2]
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
  int64_t ncell;           // n^order
  int64_t vstride;         // virtual node of (r, node) = r * vstride + node  (M, or 0 when ragged)
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

template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(64 * kSpreadWaves) void k_spread_binned(const T *__restrict__ xT, int64_t Mx,
                                                                     const SpreadItem *__restrict__ items,
                                                                     const DevTerm *__restrict__ terms,
                                                                     OrderParams<T> op, SpreadArgs sa,
                                                                     const cx_t<T> *__restrict__ y,
                                                                     cx_t<T> *__restrict__ gpart, int64_t gstride) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  constexpr int W = 2 * MH;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *G = reinterpret_cast<double2 *>(smem_raw);
  const SpreadItem it = items[blockIdx.x];
  const int tl = blockIdx.y;
  const DevTerm tm = terms[op.term_begin + tl];
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, i16 = l & 15, kk = l >> 4;
  const int n = op.n, P = op.P, gsize = op.gsize;
  for (int i = threadIdx.x; i < gsize; i += 64 * kSpreadWaves) G[i] = make_double2(0.0, 0.0);
  WinPoint<T> wp;
  wp.load(op.poly, i16, W);
  __syncthreads();
  const int64_t key0 = ((int64_t)tl * sa.B + it.b) * sa.ncell;
  const int64_t vbase = (int64_t)it.r * sa.vstride;
  const T *x0p = xT + (int64_t)tm.c0 * Mx;
  const T *x1p = xT + (int64_t)(ORDER >= 2 ? tm.c1 : tm.c0) * Mx;
  const T *x2p = xT + (int64_t)(ORDER >= 3 ? tm.c2 : tm.c0) * Mx;
  const T two_n = (T)(2 * n);
  for (int c = it.c0 + wv; c < it.c1; c += kSpreadWaves) {   // cells round-robin over the waves
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
    if (ORDER == 1 || ORDER == 2) {
      acc_t dre = {0, 0, 0, 0}, dim = {0, 0, 0, 0};
      // batches of 64 nodes: lane l loads node l of the batch once; the MFMA steps take the
      // window arguments and samples of their 4 nodes from those lanes
      for (int64_t b0 = p0; b0 < p1; b0 += 64) {
        const int64_t q = b0 + l;
        const bool valid = q < p1;
        const int32_t node = sa.perm[valid ? q : p0];
        cx_t<T> yl = y[vbase + node];
        const T za = fma(two_n, x0p[node], zc0);
        const T zb = ORDER == 2 ? fma(two_n, x1p[node], zc1) : (T)0;
        if (!valid) yl = cmake<T>(0, 0);
        const int steps = (int)((p1 - b0 + 3) >> 2) < 16 ? (int)((p1 - b0 + 3) >> 2) : 16;
        for (int st = 0; st < steps; ++st) {
          const int src = 4 * st + kk;
          const T z0 = __shfl(za, src, 64);
          const T yr = __shfl(yl.x, src, 64), yi = __shfl(yl.y, src, 64);
          const T w0 = wp(z0);
          if (ORDER == 1) {
            const T a = i16 == 0 ? yr : (i16 == 1 ? yi : (T)0);
            dre = MF::run(a, w0, dre);
          } else {
            const T w1 = wp(__shfl(zb, src, 64));
            dre = MF::run(w0 * yr, w1, dre);
            dim = MF::run(w0 * yi, w1, dim);
          }
        }
      }
      const int rs = wrap_start(fl0, MH, n);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = MF::row(l, r);
        if (ORDER == 1) {
          if (i16 < W && row < 2) {
            double *dst = row == 0 ? &G[fl0 + i16].x : &G[fl0 + i16].y;
            atomicAdd(dst, (double)dre[r]);
          }
        } else if (row < W && i16 < W) {
          const int gr = (rs + row) % n;
          double2 *dst = &G[gr * P + fl1 + i16];
          atomicAdd(&dst->x, (double)dre[r]);
          atomicAdd(&dst->y, (double)dim[r]);
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
  cx_t<T> *out = gpart + (int64_t)blockIdx.x * gstride + tm.gpart_off;
  for (int i = threadIdx.x; i < gsize; i += 64 * kSpreadWaves) out[i] = cmake<T>((T)G[i].x, (T)G[i].y);
}

}  // namespace gt
