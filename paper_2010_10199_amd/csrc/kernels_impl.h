// Kernels of the grouped Fourier transform (templated on the real type T).
// Included once per precision by kernels_f32.hip and kernels_f64.hip.
//
// One term u of order t = |u| is a t-dimensional nonequispaced FFT (eq. somafm):
//   forward:  K1 pack     ghat_l = fhat_l * prod_j (-1)^{l_j} / Phi_hat(l_j), zero rows dropped
//             K2 DFT      g[l] = sum_k ghat_k e^{+2 pi i <k, l>/n}, pruned to the N-1 non-zero
//                         input frequencies per axis, written into the halo layout
//             K3 gather   f_v += sum_{window} g[l] prod_j Phi(n x_j - l_j), summed over all terms
//   adjoint:  K4 spread   grid[l] += y_v prod_j Phi(n x_j - l_j) in LDS, per node chunk
//             K2 DFT      e^{-2 pi i <k, l>/n}, only the N-1 non-zero output frequencies per axis
//             K5 unpack   times the same deconvolution factors, written in group order
// The empty set contributes fhat_0 to every node (forward) and sum_v y_v (adjoint).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gt_internal.h"

namespace gt {

template <typename T>
__device__ __forceinline__ cx_t<T> cmake(T a, T b) {
  cx_t<T> c;
  c.x = a;
  c.y = b;
  return c;
}

// ------------------------------------------------------------------ reductions (wave64)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Block-wide sum of two doubles; result valid in thread 0.  `sh` holds >= 2*(BS/64) doubles.
__device__ __forceinline__ void block_sum2(double &a, double &b, double *sh) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[2 * w] = a;
    sh[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0;
    b = 0;
    for (int i = 0; i < nw; ++i) {
      a += sh[2 * i];
      b += sh[2 * i + 1];
    }
  }
}

// A value that is the same in every lane of the wavefront, held in a scalar register.  Loads
// from kernel-argument pointers are scalar loads already when the compiler can see that
// nothing stores to that memory before them; in a launch that runs several kernel bodies it
// may not, and the loaded tables would take vector registers instead.
__device__ __forceinline__ float wave_uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Bijection on [0, nb) giving the blocks of each XCD (block b runs on XCD b mod 8) one
// contiguous range of logical indices.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7, x = b & 7, j = b >> 3;
  return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

// ------------------------------------------------------------------ window
// Grid index of the first window point and the 2m window values of one coordinate.
// s = n x + n/2 in [0, n) places grid index 0 at x = -1/2; window point j sits at
// grid index fl - m + 1 + j, i.e. at halo index fl + j, with tau = (m - 1 + fr) - j.
template <typename T>
__device__ __forceinline__ T frac_offset(T x, int n, int &fl) {
  const T nf = (T)n;
  int f = (int)floor(fma(nf, x, (T)(n / 2)));
  f = f < 0 ? 0 : (f > n - 1 ? n - 1 : f);
  fl = f;
  return fma(nf, x, (T)(n / 2 - f));   // exact product, one rounding: fractional offset
}

// All 2m window values.  The window is even, so point 2m-1-j is point j at -z (the host
// mirrors the coefficients exactly); one even part E(z^2) and one odd part z O(z^2) give
// both values of a pair: psi_j = E + zO, psi_{2m-1-j} = E - zO.
template <typename T, int MH>
__device__ __forceinline__ void window_values(T z, const T *__restrict__ poly, T (&psi)[2 * MH]) {
  constexpr int D = Deg<T>::value;
  constexpr int DE = D - (D & 1);          // highest even power
  constexpr int DO = D - 1 + (D & 1);      // highest odd power
  const T z2 = z * z;
#pragma unroll
  for (int j = 0; j < MH; ++j) {
    const T *c = poly + j * (D + 1);   // the same table in every lane
    T e = wave_uniform(c[DE]);
#pragma unroll
    for (int q = DE - 2; q >= 0; q -= 2) e = fma(e, z2, wave_uniform(c[q]));
    T o = wave_uniform(c[DO]);
#pragma unroll
    for (int q = DO - 2; q >= 1; q -= 2) o = fma(o, z2, wave_uniform(c[q]));
    o *= z;
    psi[j] = e + o;
    psi[2 * MH - 1 - j] = e - o;
  }
}

// Value and d/dz of window point j's polynomial.
template <typename T>
__device__ __forceinline__ void window_point_d(T z, const T *__restrict__ c, T &val, T &der) {
  constexpr int D = Deg<T>::value;
  T p = c[D], dp = (T)0;
#pragma unroll
  for (int q = D - 1; q >= 0; --q) {
    dp = fma(dp, z, p);
    p = fma(p, z, c[q]);
  }
  val = p;
  der = dp;
}

template <typename T>
__device__ __forceinline__ T window_point(T z, const T *__restrict__ c) {
  constexpr int D = Deg<T>::value;
  T acc = c[D];
#pragma unroll
  for (int q = D - 1; q >= 0; --q) acc = fma(acc, z, c[q]);
  return acc;
}

__device__ __forceinline__ int wrap_start(int fl, int mh, int n) {
  int r = (fl - mh + 1) % n;
  return r < 0 ? r + n : r;
}

// ------------------------------------------------------------------ node preparation
// (scale: 1, or 1/2 for the cosine basis, whose nodes x map to t = x / 2 on the torus)
template <typename T>
__global__ void k_prepare_nodes(const T *__restrict__ x, int64_t Mtot, int d, T scale, T *__restrict__ xT,
                                int32_t *__restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mtot * d) return;
  const int64_t node = i / d;
  const int c = (int)(i - node * d);
  T v = x[i];
  if (!isfinite(v)) {
    atomicOr(flag, 1);
    v = (T)0;
  }
  v *= scale;   // exact for 1 and 1/2
  if (!(v >= (T)-0.5 && v < (T)0.5)) {   // reduce modulo 1 only when outside [-1/2, 1/2)
    v = v - floor(v + (T)0.5);
    if (v >= (T)0.5 || v < (T)-0.5) v = (T)-0.5;
  }
  xT[(int64_t)c * Mtot + node] = v;
}

static __global__ void k_zero_i32(int32_t *p) { *p = 0; }

// ------------------------------------------------------------------ K1 + K2 forward

// One workgroup per (term, right-hand side).  Pruned separable inverse DFT from the
// (N-1)^t non-zero frequencies onto the n^t grid, written in the halo layout.
// The last stage's outputs are split over `slices` workgroups per term (each recomputes the
// earlier, smaller stages), so a launch has slices x terms workgroups.
template <typename T, int ORDER>
__device__ __forceinline__ void pack_fwd_body(const Blk bk, const cx_t<T> *__restrict__ fhat,
                                              const T *__restrict__ colscale, int64_t ncoef,
                                              const DevTerm *__restrict__ terms, const OrderParams<T> &op,
                                              cx_t<T> *__restrict__ grids, int64_t grid_total, int slices) {
  using C = cx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *S = reinterpret_cast<C *>(smem_raw);
  const int tid = threadIdx.x, BS = blockDim.x;
  const int slice = bk.x % slices;
  const DevTerm tm = terms[op.term_begin + bk.x / slices];
  const int r = bk.y;
  const C *src = fhat + (int64_t)r * ncoef + tm.coef_off;
  const T *cs = colscale ? colscale + tm.coef_off : nullptr;
  C *dst = grids + (int64_t)r * grid_total + tm.grid_off;
  const int K = op.nfreq, n = op.n, P = op.P, h = op.N / 2, mm1 = op.m - 1;
  // LDS: the DFT stage arrays, then the table of DFT factors
  const size_t stage = sizeof(C) * (ORDER == 1 ? (size_t)K
                                   : ORDER == 2 ? (size_t)K * K + (size_t)K * n
                                                : (size_t)K * K * K + (size_t)K * K * n + (size_t)K * n * n);
  // DFT factors e^{2 pi i k_a l / n} (k_a = -h..-1, 1..h-1, a = 0..K-1) tabulated after the
  // stage arrays (first read after the first barrier); order 1 (bandwidths up to several
  // hundred) keeps only the n roots of unity there and steps the exponent (k_a l) mod n
  C *Wt = reinterpret_cast<C *>(smem_raw + stage);
  if (ORDER == 1) {
    for (int i = tid; i < n; i += BS) Wt[i] = cmake<T>(op.roots[2 * i], op.roots[2 * i + 1]);
  } else {
    for (int i = tid; i < K * n; i += BS) {
      const int a = i / n, l = i - a * n, k = a < h ? a - h : a - h + 1;
      int e = (k * l) % n;
      e = e < 0 ? e + n : e;
      Wt[i] = cmake<T>(op.roots[2 * e], op.roots[2 * e + 1]);
    }
  }
  const T *__restrict__ Dc = op.deconv;
  auto unpad = [&](int p) {
    int l = (p - mm1) % n;
    return l < 0 ? l + n : l;
  };

  if (ORDER == 1) {
    for (int a = tid; a < K; a += BS) {
      C v = src[a];
      T sc = Dc[a] * (cs ? cs[a] : (T)1);
      S[a] = cmake<T>(v.x * sc, v.y * sc);
    }
    __syncthreads();
    const int p0 = (int)((int64_t)P * slice / slices), p1 = (int)((int64_t)P * (slice + 1) / slices);
    for (int p = p0 + tid; p < p1; p += BS) {
      const int l = unpad(p);
      T re = 0, im = 0;
      int e = (int)(((int64_t)(n - h) * l) % n);   // k = -h
      for (int a = 0; a < K; ++a) {
        const C v = S[a], w = Wt[e];
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
        e += (a == h - 1) ? 2 * l : l;   // k_a -> k_{a+1}, skipping k = 0
        while (e >= n) e -= n;
      }
      dst[p] = cmake<T>(re, im);
    }
  } else if (ORDER == 2) {
    C *A = S;              // K x K
    C *B = S + K * K;      // K x n
    for (int i = tid; i < K * K; i += BS) {
      const int a1 = i / K, a2 = i - a1 * K;
      C v = src[i];
      T sc = Dc[a1] * Dc[a2] * (cs ? cs[i] : (T)1);
      A[i] = cmake<T>(v.x * sc, v.y * sc);
    }
    __syncthreads();
    for (int i = tid; i < K * n; i += BS) {
      const int a1 = i / n, l2 = i - a1 * n;
      T re = 0, im = 0;
      for (int a2 = 0; a2 < K; ++a2) {
        const C v = A[a1 * K + a2], w = Wt[a2 * n + l2];
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
      }
      B[i] = cmake<T>(re, im);
    }
    __syncthreads();
    const int i0 = (int)((int64_t)n * P * slice / slices), i1 = (int)((int64_t)n * P * (slice + 1) / slices);
    for (int i = i0 + tid; i < i1; i += BS) {
      const int l1 = i / P, p2 = i - l1 * P, l2 = unpad(p2);
      T re = 0, im = 0;
      for (int a1 = 0; a1 < K; ++a1) {
        const C v = B[a1 * n + l2], w = Wt[a1 * n + l1];
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
      }
      dst[i] = cmake<T>(re, im);
    }
  } else {
    C *A = S;                          // K^3
    C *B = A + K * K * K;              // K x K x n
    C *Cc = B + K * K * n;             // K x n x n
    for (int i = tid; i < K * K * K; i += BS) {
      const int a1 = i / (K * K), rem = i - a1 * K * K, a2 = rem / K, a3 = rem - a2 * K;
      C v = src[i];
      T sc = Dc[a1] * Dc[a2] * Dc[a3] * (cs ? cs[i] : (T)1);
      A[i] = cmake<T>(v.x * sc, v.y * sc);
    }
    __syncthreads();
    for (int i = tid; i < K * K * n; i += BS) {
      const int a12 = i / n, l3 = i - a12 * n;
      T re = 0, im = 0;
      for (int a3 = 0; a3 < K; ++a3) {
        const C v = A[a12 * K + a3], w = Wt[a3 * n + l3];
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
      }
      B[i] = cmake<T>(re, im);
    }
    __syncthreads();
    for (int i = tid; i < K * n * n; i += BS) {
      const int a1 = i / (n * n), rem = i - a1 * n * n, l2 = rem / n, l3 = rem - l2 * n;
      T re = 0, im = 0;
      for (int a2 = 0; a2 < K; ++a2) {
        const C v = B[(a1 * K + a2) * n + l3], w = Wt[a2 * n + l2];
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
      }
      Cc[i] = cmake<T>(re, im);
    }
    __syncthreads();
    const int i0 = (int)((int64_t)n * n * P * slice / slices), i1 = (int)((int64_t)n * n * P * (slice + 1) / slices);
    for (int i = i0 + tid; i < i1; i += BS) {
      const int l1 = i / (n * P), rem = i - l1 * n * P, l2 = rem / P, p3 = rem - l2 * P, l3 = unpad(p3);
      T re = 0, im = 0;
      for (int a1 = 0; a1 < K; ++a1) {
        const C v = Cc[(a1 * n + l2) * n + l3], w = Wt[a1 * n + l1];
        re = fma(v.x, w.x, fma(-v.y, w.y, re));
        im = fma(v.x, w.y, fma(v.y, w.x, im));
      }
      dst[i] = cmake<T>(re, im);
    }
  }
}

template <typename T, int ORDER>
__global__ __launch_bounds__(kPackBS) void k_pack_fwd(const cx_t<T> *__restrict__ fhat, const T *__restrict__ colscale,
                                                      int64_t ncoef, const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                      cx_t<T> *__restrict__ grids, int64_t grid_total, int slices) {
  pack_fwd_body<T, ORDER>(Blk{(int)blockIdx.x, (int)blockIdx.y}, fhat, colscale, ncoef, terms, op, grids, grid_total,
                          slices);
}

// ------------------------------------------------------------------ K3 gather
// Workgroup = (256 virtual nodes of one right-hand side) x (a block of terms of one order).
// Each term's grid is staged in LDS; each thread accumulates its node's sum over the block.
template <typename T, int ORDER, int MH>
__device__ __forceinline__ cx_t<T> gather_term(const cx_t<T> *__restrict__ G, const T *__restrict__ xT, int64_t Mx,
                                               int64_t xi, const DevTerm &tm, const OrderParams<T> &op) {
  constexpr int W = 2 * MH;
  const int n = op.n, P = op.P;
  T re = 0, im = 0;
  if (ORDER == 1) {
    int f0;
    const T z0 = frac_offset<T>(xT[(int64_t)tm.c0 * Mx + xi], n, f0) * (T)2 - (T)1;
    T p0[W];
    window_values<T, MH>(z0, op.poly, p0);
    const cx_t<T> *g = G + f0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
      const cx_t<T> v = g[j];
      re = fma(p0[j], v.x, re);
      im = fma(p0[j], v.y, im);
    }
  } else if (ORDER == 2) {
    int f0, f1;
    const T z0 = frac_offset<T>(xT[(int64_t)tm.c0 * Mx + xi], n, f0) * (T)2 - (T)1;
    const T z1 = frac_offset<T>(xT[(int64_t)tm.c1 * Mx + xi], n, f1) * (T)2 - (T)1;
    T p0[W], p1[W];
    window_values<T, MH>(z0, op.poly, p0);
    window_values<T, MH>(z1, op.poly, p1);
    int r = wrap_start(f0, MH, n);
#pragma unroll
    for (int j1 = 0; j1 < W; ++j1) {
      const cx_t<T> *row = G + r * P + f1;
      T br = 0, bi = 0;
#pragma unroll
      for (int j2 = 0; j2 < W; ++j2) {
        const cx_t<T> v = row[j2];
        br = fma(p1[j2], v.x, br);
        bi = fma(p1[j2], v.y, bi);
      }
      re = fma(p0[j1], br, re);
      im = fma(p0[j1], bi, im);
      r = (r + 1 == n) ? 0 : r + 1;
    }
  } else {
    int f0, f1, f2;
    const T z0 = frac_offset<T>(xT[(int64_t)tm.c0 * Mx + xi], n, f0) * (T)2 - (T)1;
    const T z1 = frac_offset<T>(xT[(int64_t)tm.c1 * Mx + xi], n, f1) * (T)2 - (T)1;
    const T z2 = frac_offset<T>(xT[(int64_t)tm.c2 * Mx + xi], n, f2) * (T)2 - (T)1;
    T p1[W], p2[W];
    window_values<T, MH>(z1, op.poly, p1);
    window_values<T, MH>(z2, op.poly, p2);
    int r0 = wrap_start(f0, MH, n);
    const int r1s = wrap_start(f1, MH, n);
    constexpr int D = Deg<T>::value;
#pragma unroll 1
    for (int j1 = 0; j1 < W; ++j1) {
      const T w0 = window_point<T>(z0, op.poly + j1 * (D + 1));
      const cx_t<T> *plane = G + (int64_t)r0 * n * P + f2;
      int r1 = r1s;
      T br = 0, bi = 0;
#pragma unroll
      for (int j2 = 0; j2 < W; ++j2) {
        const cx_t<T> *row = plane + r1 * P;
        T cr = 0, ci = 0;
#pragma unroll
        for (int j3 = 0; j3 < W; ++j3) {
          const cx_t<T> v = row[j3];
          cr = fma(p2[j3], v.x, cr);
          ci = fma(p2[j3], v.y, ci);
        }
        br = fma(p1[j2], cr, br);
        bi = fma(p1[j2], ci, bi);
        r1 = (r1 + 1 == n) ? 0 : r1 + 1;
      }
      re = fma(w0, br, re);
      im = fma(w0, bi, im);
      r0 = (r0 + 1 == n) ? 0 : r0 + 1;
    }
  }
  return cmake<T>(re, im);
}

// f_v = (accumulate ? f_v : fhat_empty(r)) + sum over the term slots.  Workgroup = 64 nodes
// x 4 parts; part p sums slots p, p+4, ...; the parts are combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void k_reduce_f(const cx_t<T> *__restrict__ fhat, int64_t ncoef,
                                                  const WorkItem *__restrict__ items,
                                                  const cx_t<T> *__restrict__ slots, int nslots, int64_t Vtot,
                                                  int accumulate, cx_t<T> *__restrict__ f) {
  __shared__ cx_t<T> part[4][64];
  const WorkItem it = items[blockIdx.x >> 2];
  const int node = ((blockIdx.x & 3) << 6) + (threadIdx.x & 63), p = threadIdx.x >> 6;
  const bool active = node < it.count;
  const int64_t v = it.v0 + node;
  T re = 0, im = 0;
  if (active) {
    // slots p, p + 4, ... in order; sixteen loads in flight per step (past the end: reload
    // the step's first slot, not added)
    constexpr int U = 16;
    for (int b0 = p; b0 < nslots; b0 += 4 * U) {
      cx_t<T> q[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = b0 + 4 * u < nslots ? b0 + 4 * u : b0;
        q[u] = slots[(int64_t)b * Vtot + v];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (b0 + 4 * u < nslots) {
          re += q[u].x;
          im += q[u].y;
        }
    }
  }
  part[p][threadIdx.x & 63] = cmake<T>(re, im);
  __syncthreads();
  if (p == 0 && active) {
    cx_t<T> acc = accumulate ? f[v] : fhat[(int64_t)it.r * ncoef];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc.x += part[q][threadIdx.x].x;
      acc.y += part[q][threadIdx.x].y;
    }
    f[v] = acc;
  }
}

}  // namespace gt
#include "gather.h"   // K3 gather (binned, one slot per term)
#include "spread.h"   // K4 spread (binned, MFMA)
#include "direct.h"   // direct sums of small groups (MFMA), forward and adjoint
namespace gt {

// Empty-set coefficient fhat_empty(r) = sum_v y_v, in two launches: k_empty_part sums one
// gather item per workgroup (FP64) into ysum; k_empty_adj, one workgroup per right-hand side,
// adds that side's partials in item order and writes the coefficient.  (One launch whose last
// workgroup adds the partials needs a device-scope fence per workgroup, an L2 write-back that
// slowed the adjoint kernels running beside it.)
template <typename T>
__device__ __forceinline__ void empty_part_body(const Blk bk, const WorkItem *__restrict__ items,
                                                const cx_t<T> *__restrict__ y, double *__restrict__ ysum) {
  __shared__ double sh[2 * (kGatherBS / 64)];
  const WorkItem it = items[bk.x];
  double a = 0, b = 0;
  if ((int)threadIdx.x < it.count) {
    const cx_t<T> v = y[it.v0 + threadIdx.x];
    a = v.x;
    b = v.y;
  }
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) {
    ysum[2 * bk.x] = a;
    ysum[2 * bk.x + 1] = b;
  }
}

template <typename T>
__global__ __launch_bounds__(kGatherBS) void k_empty_part(const WorkItem *__restrict__ items,
                                                          const cx_t<T> *__restrict__ y, double *__restrict__ ysum) {
  empty_part_body<T>(Blk{(int)blockIdx.x, 0}, items, y, ysum);
}

template <typename T>
__device__ __forceinline__ void empty_adj_body(const Blk bk, const int32_t *__restrict__ item_begin,
                                               const double *__restrict__ ysum, int64_t ncoef,
                                               cx_t<T> *__restrict__ fhat) {
  __shared__ double sh[2 * (kGatherBS / 64)];
  const int r = bk.x;
  double a = 0, b = 0;
  for (int i = item_begin[r] + threadIdx.x; i < item_begin[r + 1]; i += kGatherBS) {
    a += ysum[2 * i];
    b += ysum[2 * i + 1];
  }
  block_sum2(a, b, sh);
  if (threadIdx.x == 0) fhat[(int64_t)r * ncoef] = cmake<T>((T)a, (T)b);
}

template <typename T>
__global__ __launch_bounds__(kGatherBS) void k_empty_adj(const int32_t *__restrict__ item_begin,
                                                         const double *__restrict__ ysum, int64_t ncoef,
                                                         cx_t<T> *__restrict__ fhat) {
  empty_adj_body<T>(Blk{(int)blockIdx.x, 0}, item_begin, ysum, ncoef, fhat);
}

// ------------------------------------------------------------------ fold of the spread partials
// One output per unpadded grid point l of (right-hand side, term): sum over the spread items
// of that right-hand side and over the halo copies p of l (p = l + m - 1 mod n, + n, ...),
// in FP64.  Workgroup = 64 points x 4 parts (part q takes items q, q+4, ...), combined in a
// fixed order.  gsum layout: [r][term_local][outer][n] with outer = n^(order-1).
template <typename T>
__device__ __forceinline__ void fold_partials_body(const Blk bk, const cx_t<T> *__restrict__ gpart, int64_t gstride,
                                                   const int32_t *__restrict__ item_begin,
                                                   const DevTerm *__restrict__ terms, const OrderParams<T> &op,
                                                   int order, cx_t<T> *__restrict__ gsum) {
  __shared__ double part[4][64][2];
  const int n = op.n, P = op.P, mm1 = op.m - 1;
  const int nt = op.term_end - op.term_begin;
  const int64_t outer = order == 1 ? 1 : (order == 2 ? n : (int64_t)n * n);
  const int64_t per_term = outer * n;
  const int64_t idx = (int64_t)bk.x * 64 + (threadIdx.x & 63);
  const int q = threadIdx.x >> 6;
  const bool active = idx < per_term * nt;
  const int r = bk.y;
  const int tl = active ? (int)(idx / per_term) : 0;
  const int64_t rem = idx - (int64_t)tl * per_term;
  const int64_t o = rem / n;
  const int l = (int)(rem - o * n);
  double re = 0, im = 0;
  if (active) {
    const DevTerm tm = terms[op.term_begin + tl];
    const int s0 = item_begin[r] + q, s1 = item_begin[r + 1];
    const int p0 = (l + mm1) % n;
    if (P <= 2 * n) {
      // at most two halo copies p0, p0 + n: items q, q + 4, ... eight at a time, both copies'
      // loads in flight together (past the end: reload the step's first item, not added)
      constexpr int U = 8;
      const bool two = p0 + n < P;
      for (int sa = s0; sa < s1; sa += 4 * U) {
        cx_t<T> v0[U], v1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int s = sa + 4 * u < s1 ? sa + 4 * u : sa;
          const cx_t<T> *src = gpart + (int64_t)s * gstride + tm.gpart_off + o * P;
          v0[u] = src[p0];
          v1[u] = src[two ? p0 + n : p0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (sa + 4 * u < s1) {
            re += (double)v0[u].x;
            im += (double)v0[u].y;
            if (two) {
              re += (double)v1[u].x;
              im += (double)v1[u].y;
            }
          }
      }
    } else {
      for (int s = s0; s < s1; s += 4) {
        const cx_t<T> *src = gpart + (int64_t)s * gstride + tm.gpart_off + o * P;
        for (int p = p0; p < P; p += n) {
          const cx_t<T> v = src[p];
          re += (double)v.x;
          im += (double)v.y;
        }
      }
    }
  }
  part[q][threadIdx.x & 63][0] = re;
  part[q][threadIdx.x & 63][1] = im;
  __syncthreads();
  if (q == 0 && active) {
    re = part[0][threadIdx.x][0] + part[1][threadIdx.x][0] + part[2][threadIdx.x][0] + part[3][threadIdx.x][0];
    im = part[0][threadIdx.x][1] + part[1][threadIdx.x][1] + part[2][threadIdx.x][1] + part[3][threadIdx.x][1];
    gsum[((int64_t)r * nt + tl) * per_term + rem] = cmake<T>((T)re, (T)im);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fold_partials(const cx_t<T> *__restrict__ gpart, int64_t gstride,
                                                       const int32_t *__restrict__ item_begin,
                                                       const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                       int order, cx_t<T> *__restrict__ gsum) {
  fold_partials_body<T>(Blk{(int)blockIdx.x, (int)blockIdx.y}, gpart, gstride, item_begin, terms, op, order, gsum);
}

// ------------------------------------------------------------------ K2 + K5 adjoint
// One workgroup per (term, right-hand side): the folded grid, pruned forward DFT to the
// (N-1)^t non-zero frequencies, deconvolve, write in group order.
template <typename T, int ORDER>
__device__ __forceinline__ void dft_adj_body(const Blk bk, const cx_t<T> *__restrict__ gsum,
                                             const DevTerm *__restrict__ terms, const OrderParams<T> &op,
                                             const T *__restrict__ colscale, int64_t ncoef,
                                             cx_t<T> *__restrict__ fhat, int ntile, int ts, int nsplit) {
  using C = cx_t<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *S = reinterpret_cast<C *>(smem_raw);
  const int tid = threadIdx.x, BS = blockDim.x;
  // order 2: nsplit workgroups per term, workgroup sp computing the coefficient columns
  // a2 in [sp K / nsplit, (sp + 1) K / nsplit) (both DFT stages split along a2)
  const int tl = bk.x / nsplit, sp = bk.x - tl * nsplit;
  const DevTerm tm = terms[op.term_begin + tl];
  const int r = bk.y;
  const int nt = op.term_end - op.term_begin;
  const int K = op.nfreq, n = op.n, h = op.N / 2;
  // LDS: the DFT stage arrays, then the table of DFT factors (then, order 2, the column sums)
  const size_t stage = sizeof(C) * (ORDER == 1 ? (size_t)n
                                   : ORDER == 2 ? (size_t)n * n + (size_t)n * K
                                                : (size_t)n * n * n + (size_t)n * n * K);
  // DFT factors e^{2 pi i k_a l / n} (k_a = -h..-1, 1..h-1, a = 0..K-1) tabulated after the
  // stage arrays (first read after the first barrier); the sums below use their conjugates
  C *Wt = reinterpret_cast<C *>(smem_raw + stage);
  if (ORDER == 1) {   // order 1: the n roots of unity only, exponent stepped (as in k_pack_fwd)
    for (int i = tid; i < n; i += BS) Wt[i] = cmake<T>(op.roots[2 * i], op.roots[2 * i + 1]);
  } else {
    for (int i = tid; i < K * n; i += BS) {   // Wt[l * K + a]: threads that differ in a read neighbours
      const int l = i / K, a = i - l * K, k = a < h ? a - h : a - h + 1;
      int e = (k * l) % n;
      e = e < 0 ? e + n : e;
      Wt[i] = cmake<T>(op.roots[2 * e], op.roots[2 * e + 1]);
    }
  }
  const T *__restrict__ Dc = op.deconv;
  C *dst = fhat + (int64_t)r * ncoef + tm.coef_off;
  const T *cs = colscale ? colscale + tm.coef_off : nullptr;
  const int outer = ORDER == 1 ? 1 : (ORDER == 2 ? n : n * n);
  C *G = S;
  if (ORDER == 2 && ntile != 0) {
    // order 2 from the tile spread: gsum holds the column-folded patches
    // hcol[ty][pr][l1] of this term; grid row l0 collects the patch rows that land on it
    // (start row of tile row ty plus pr, modulo n), tile rows in order
    // (staged in LDS after the DFT stages and the table of DFT factors)
    // (read from global memory when it does not fit: ntile < 0 asks for that)
    const bool staged = ntile > 0;
    ntile = staged ? ntile : -ntile;
    const int mm1 = op.m - 1;
    const C *hc = gsum + ((int64_t)r * nt + tl) * ntile * 16 * n;
    C *HCl = reinterpret_cast<C *>(smem_raw + stage + (size_t)K * n * sizeof(C));
    if (staged) {
      const int nh = ntile * 16 * n;
      for (int i0 = tid; i0 < nh; i0 += 4 * BS) {   // four loads in flight per thread
        C v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = hc[i0 + u * BS < nh ? i0 + u * BS : i0];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (i0 + u * BS < nh) HCl[i0 + u * BS] = v[u];
      }
      __syncthreads();
    }
    const C *HC = staged ? HCl : hc;
    int rs0 = (-mm1) % n;
    rs0 = rs0 < 0 ? rs0 + n : rs0;   // start row of tile row 0
    for (int i = tid; i < n * n; i += BS) {
      const int l0 = i / n, l1 = i - l0 * n;
      T re = 0, im = 0;
      int rs = rs0;
      for (int ty = 0; ty < ntile; ++ty) {
        int pr = l0 - rs;
        pr = pr < 0 ? pr + n : pr;
        for (; pr < 16; pr += n) {
          const C v = HC[(ty * 16 + pr) * n + l1];
          re += v.x;
          im += v.y;
        }
        rs += ts;
        while (rs >= n) rs -= n;
      }
      G[i] = cmake<T>(re, im);
    }
  } else {
    const C *src = gsum + ((int64_t)r * nt + tl) * outer * n;
    for (int i = tid; i < outer * n; i += BS) G[i] = src[i];
  }
  __syncthreads();
  // conj twiddles: e^{-2 pi i k l / n}
  if (ORDER == 1) {
    // each sum split over 8 adjacent lanes (lanes i with the same i >> 3, l in eighths of
    // [0, n)), the parts added by lane shuffles in a fixed order
    for (int i = tid; i < 8 * K; i += BS) {
      const int a = i >> 3, part = i & 7;
      T re = 0, im = 0;
      // walk l with exponent (k_a * l) mod n
      const int k = a - h + (a >= h ? 1 : 0);
      const int km = k < 0 ? k + n : k;
      const int la = (part * n) >> 3, lb = ((part + 1) * n) >> 3;
      int e = (int)(((int64_t)km * la) % n);
      for (int l = la; l < lb; ++l) {
        const C v = G[l];
        const T c = Wt[e].x, s = Wt[e].y;
        re = fma(v.x, c, fma(v.y, s, re));
        im = fma(v.y, c, fma(-v.x, s, im));
        e += km;
        if (e >= n) e -= n;
      }
      re += __shfl_xor(re, 1);
      im += __shfl_xor(im, 1);
      re += __shfl_xor(re, 2);
      im += __shfl_xor(im, 2);
      re += __shfl_xor(re, 4);
      im += __shfl_xor(im, 4);
      if (part == 0) {
        const T sc = Dc[a] * (cs ? cs[a] : (T)1);
        dst[a] = cmake<T>(re * sc, im * sc);
      }
    }
  } else if (ORDER == 2) {
    // Each sum is split over adjacent lanes (two for the first stage, four for the second,
    // lanes i with the same i >> 1 or i >> 2, always in the same loop iteration) and the
    // parts are added by lane shuffles in a fixed order.
    const int a2lo = sp * K / nsplit, KW = (sp + 1) * K / nsplit - a2lo;   // this workgroup's columns
    C *H = S + n * n;   // n x KW
    for (int i = tid; i < 2 * n * KW; i += BS) {
      const int o = i >> 1, half = i & 1;
      const int l1 = o / KW, a2 = a2lo + (o - l1 * KW);
      const C *w = Wt + a2;
      T re = 0, im = 0;
      for (int l2 = (half * n) >> 1; l2 < ((half + 1) * n) >> 1; ++l2) {
        const C v = G[l1 * n + l2];
        const T c = w[l2 * K].x, s = w[l2 * K].y;
        re = fma(v.x, c, fma(v.y, s, re));
        im = fma(v.y, c, fma(-v.x, s, im));
      }
      re += __shfl_xor(re, 1);
      im += __shfl_xor(im, 1);
      if (half == 0) H[o] = cmake<T>(re, im);
    }
    __syncthreads();
    for (int i = tid; i < 4 * K * KW; i += BS) {
      const int oo = i >> 2, part = i & 3;
      const int a1 = oo / KW, a2w = oo - a1 * KW, a2 = a2lo + a2w, o = a1 * K + a2;
      const C *w = Wt + a1;
      T re = 0, im = 0;
      for (int l1 = (part * n) >> 2; l1 < ((part + 1) * n) >> 2; ++l1) {
        const C v = H[l1 * KW + a2w];
        const T c = w[l1 * K].x, s = w[l1 * K].y;
        re = fma(v.x, c, fma(v.y, s, re));
        im = fma(v.y, c, fma(-v.x, s, im));
      }
      re += __shfl_xor(re, 1);
      im += __shfl_xor(im, 1);
      re += __shfl_xor(re, 2);
      im += __shfl_xor(im, 2);
      if (part == 0) {
        const T sc = Dc[a1] * Dc[a2] * (cs ? cs[o] : (T)1);
        dst[o] = cmake<T>(re * sc, im * sc);
      }
    }
  } else {
    C *H1 = S + n * n * n;   // n x n x K
    C *H2 = S;               // n x K x K (overwrites G after H1 is complete)
    for (int i = tid; i < n * n * K; i += BS) {
      const int l12 = i / K, a3 = i - l12 * K;
      const C *w = Wt + a3;
      T re = 0, im = 0;
      for (int l3 = 0; l3 < n; ++l3) {
        const C v = G[l12 * n + l3];
        const T c = w[l3 * K].x, s = w[l3 * K].y;
        re = fma(v.x, c, fma(v.y, s, re));
        im = fma(v.y, c, fma(-v.x, s, im));
      }
      H1[i] = cmake<T>(re, im);
    }
    __syncthreads();
    for (int i = tid; i < n * K * K; i += BS) {
      const int l1 = i / (K * K), rem = i - l1 * K * K, a2 = rem / K, a3 = rem - a2 * K;
      const C *w = Wt + a2;
      T re = 0, im = 0;
      for (int l2 = 0; l2 < n; ++l2) {
        const C v = H1[(l1 * n + l2) * K + a3];
        const T c = w[l2 * K].x, s = w[l2 * K].y;
        re = fma(v.x, c, fma(v.y, s, re));
        im = fma(v.y, c, fma(-v.x, s, im));
      }
      H2[i] = cmake<T>(re, im);
    }
    __syncthreads();
    for (int i = tid; i < K * K * K; i += BS) {
      const int a1 = i / (K * K), rem = i - a1 * K * K, a2 = rem / K, a3 = rem - a2 * K;
      const C *w = Wt + a1;
      T re = 0, im = 0;
      for (int l1 = 0; l1 < n; ++l1) {
        const C v = H2[(l1 * K + a2) * K + a3];
        const T c = w[l1 * K].x, s = w[l1 * K].y;
        re = fma(v.x, c, fma(v.y, s, re));
        im = fma(v.y, c, fma(-v.x, s, im));
      }
      const T sc = Dc[a1] * Dc[a2] * Dc[a3] * (cs ? cs[i] : (T)1);
      dst[i] = cmake<T>(re * sc, im * sc);
    }
  }
}

template <typename T, int ORDER>
__global__ __launch_bounds__(ORDER == 2 ? 2 * kPackBS : kPackBS) void k_dft_adj(const cx_t<T> *__restrict__ gsum,
                                                     const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                     const T *__restrict__ colscale, int64_t ncoef,
                                                     cx_t<T> *__restrict__ fhat, int ntile, int ts, int nsplit) {
  dft_adj_body<T, ORDER>(Blk{(int)blockIdx.x, (int)blockIdx.y}, gsum, terms, op, colscale, ncoef, fhat, ntile, ts,
                         nsplit);
}

// ------------------------------------------------------------------ K9 node gradient
// Workgroup = 256 virtual nodes x all terms of one order.  Derivative of the gathered sum
// with respect to each coordinate of the term (window derivative d/dx = 2 n d/dz); the
// contribution Re(conj(D) g_v) is accumulated per node and coordinate in LDS.
template <typename T, int ORDER, int MH>
__global__ __launch_bounds__(kGatherBS) void k_node_grad(const T *__restrict__ xT, int64_t Mx, int d,
                                                         const WorkItem *__restrict__ items,
                                                         const DevTerm *__restrict__ terms, OrderParams<T> op,
                                                         const cx_t<T> *__restrict__ grids, int64_t grid_total,
                                                         const cx_t<T> *__restrict__ gup, T *__restrict__ gxp) {
  using C = cx_t<T>;
  constexpr int W = 2 * MH;
  constexpr int D = Deg<T>::value;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *G = reinterpret_cast<C *>(smem_raw);
  T *acc = reinterpret_cast<T *>(smem_raw + (size_t)op.gsize * sizeof(C));   // d x 256
  const WorkItem it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const bool active = tid < it.count;
  const int64_t xi = it.x0 + tid;
  for (int c = 0; c < d; ++c) acc[c * kGatherBS + tid] = (T)0;
  C gv = cmake<T>(0, 0);
  if (active) gv = gup[it.v0 + tid];
  const C *gbase = grids + (int64_t)it.r * grid_total;
  const int n = op.n, P = op.P;
  const T dscale = (T)(2 * n);
  for (int term = op.term_begin; term < op.term_end; ++term) {
    const DevTerm tm = terms[term];
    const C *src = gbase + tm.grid_off;
    __syncthreads();
    for (int i = tid; i < op.gsize; i += kGatherBS) G[i] = src[i];
    __syncthreads();
    if (!active) continue;
    if (ORDER == 1) {
      int f0;
      const T z0 = frac_offset<T>(xT[(int64_t)tm.c0 * Mx + xi], n, f0) * (T)2 - (T)1;
      T dr = 0, di = 0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        T w, dw;
        window_point_d<T>(z0, op.poly + j * (D + 1), w, dw);
        const C v = G[f0 + j];
        dr = fma(dw, v.x, dr);
        di = fma(dw, v.y, di);
      }
      acc[tm.c0 * kGatherBS + tid] += dscale * (dr * gv.x + di * gv.y);
    } else if (ORDER == 2) {
      int f0, f1;
      const T z0 = frac_offset<T>(xT[(int64_t)tm.c0 * Mx + xi], n, f0) * (T)2 - (T)1;
      const T z1 = frac_offset<T>(xT[(int64_t)tm.c1 * Mx + xi], n, f1) * (T)2 - (T)1;
      T p0[W], d0[W], p1[W], d1[W];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        window_point_d<T>(z0, op.poly + j * (D + 1), p0[j], d0[j]);
        window_point_d<T>(z1, op.poly + j * (D + 1), p1[j], d1[j]);
      }
      int r = wrap_start(f0, MH, n);
      T a0r = 0, a0i = 0, a1r = 0, a1i = 0;
#pragma unroll
      for (int j1 = 0; j1 < W; ++j1) {
        const C *row = G + r * P + f1;
        T br = 0, bi = 0, cr = 0, ci = 0;
#pragma unroll
        for (int j2 = 0; j2 < W; ++j2) {
          const C v = row[j2];
          br = fma(p1[j2], v.x, br);
          bi = fma(p1[j2], v.y, bi);
          cr = fma(d1[j2], v.x, cr);
          ci = fma(d1[j2], v.y, ci);
        }
        a0r = fma(d0[j1], br, a0r);
        a0i = fma(d0[j1], bi, a0i);
        a1r = fma(p0[j1], cr, a1r);
        a1i = fma(p0[j1], ci, a1i);
        r = (r + 1 == n) ? 0 : r + 1;
      }
      acc[tm.c0 * kGatherBS + tid] += dscale * (a0r * gv.x + a0i * gv.y);
      acc[tm.c1 * kGatherBS + tid] += dscale * (a1r * gv.x + a1i * gv.y);
    } else {
      int f0, f1, f2;
      const T z0 = frac_offset<T>(xT[(int64_t)tm.c0 * Mx + xi], n, f0) * (T)2 - (T)1;
      const T z1 = frac_offset<T>(xT[(int64_t)tm.c1 * Mx + xi], n, f1) * (T)2 - (T)1;
      const T z2 = frac_offset<T>(xT[(int64_t)tm.c2 * Mx + xi], n, f2) * (T)2 - (T)1;
      T p1[W], d1[W], p2[W], d2[W];
#pragma unroll
      for (int j = 0; j < W; ++j) {
        window_point_d<T>(z1, op.poly + j * (D + 1), p1[j], d1[j]);
        window_point_d<T>(z2, op.poly + j * (D + 1), p2[j], d2[j]);
      }
      int r0 = wrap_start(f0, MH, n);
      const int r1s = wrap_start(f1, MH, n);
      T a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0;
#pragma unroll 1
      for (int j1 = 0; j1 < W; ++j1) {
        T w0, dw0;
        window_point_d<T>(z0, op.poly + j1 * (D + 1), w0, dw0);
        const C *plane = G + (int64_t)r0 * n * P + f2;
        int r1 = r1s;
        T br = 0, bi = 0, b1r = 0, b1i = 0, b2r = 0, b2i = 0;
#pragma unroll
        for (int j2 = 0; j2 < W; ++j2) {
          const C *row = plane + r1 * P;
          T cr = 0, ci = 0, er = 0, ei = 0;
#pragma unroll
          for (int j3 = 0; j3 < W; ++j3) {
            const C v = row[j3];
            cr = fma(p2[j3], v.x, cr);
            ci = fma(p2[j3], v.y, ci);
            er = fma(d2[j3], v.x, er);
            ei = fma(d2[j3], v.y, ei);
          }
          br = fma(p1[j2], cr, br);
          bi = fma(p1[j2], ci, bi);
          b1r = fma(d1[j2], cr, b1r);
          b1i = fma(d1[j2], ci, b1i);
          b2r = fma(p1[j2], er, b2r);
          b2i = fma(p1[j2], ei, b2i);
          r1 = (r1 + 1 == n) ? 0 : r1 + 1;
        }
        a0r = fma(dw0, br, a0r);
        a0i = fma(dw0, bi, a0i);
        a1r = fma(w0, b1r, a1r);
        a1i = fma(w0, b1i, a1i);
        a2r = fma(w0, b2r, a2r);
        a2i = fma(w0, b2i, a2i);
        r0 = (r0 + 1 == n) ? 0 : r0 + 1;
      }
      acc[tm.c0 * kGatherBS + tid] += dscale * (a0r * gv.x + a0i * gv.y);
      acc[tm.c1 * kGatherBS + tid] += dscale * (a1r * gv.x + a1i * gv.y);
      acc[tm.c2 * kGatherBS + tid] += dscale * (a2r * gv.x + a2i * gv.y);
    }
  }
  __syncthreads();
  if (active)
    for (int c = 0; c < d; ++c) gxp[(it.v0 + tid) * d + c] = acc[c * kGatherBS + tid];
}

// gx[i][c] = sum over orders and over right-hand sides sharing node i of the partials.
// (scale: d t / d x of the node map, 1/2 for the cosine basis, else 1)
template <typename T>
__global__ void k_reduce_gx(const T *__restrict__ gxp, int norders, int64_t Vtot, int64_t Mtot, int R, bool ragged,
                            int d, T scale, T *__restrict__ gx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mtot * d) return;
  const int64_t node = i / d;
  const int c = (int)(i - node * d);
  T s = 0;
  for (int o = 0; o < norders; ++o) {
    const T *base = gxp + (int64_t)o * Vtot * d;
    if (ragged) {
      s += base[node * d + c];
    } else {
      for (int r = 0; r < R; ++r) s += base[((int64_t)r * Mtot + node) * d + c];
    }
  }
  gx[i] = scale * s;
}

// ------------------------------------------------------------------ cosine basis
// Half-period cosine groups (Sec. 5): phi_k(x) = sqrt(2)^{|u|} prod_{j in u} cos(pi k_j x_j),
// k_j = 1..N-1.  With t = x / 2, cos(pi k x) = (e^{2 pi i k t} + e^{-2 pi i k t}) / 2, so the
// cosine group of bandwidth N is the exponential group of bandwidth 2N (frequencies -N..N-1)
// at the nodes t with coefficients ghat_l = 2^{-|u|/2} fhat_{|l|} (zero where some |l_j| = N),
// and the adjoint folds the exponential adjoint: fhat_k = 2^{-|u|/2} sum over the 2^{|u|} sign
// patterns s of hhat_{s k} (the basis is real, so no conjugation enters).
// Internal index per axis a = 0..2N-2 holds l = a - N (a < N) or a - N + 1; external e = 0..N-2
// holds k = e + 1.  Both layouts row-major, last axis fastest.
// One workgroup per (term, right-hand side): ghat over the term's internal group.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_cos_expand(const cx_t<T> *__restrict__ fhat, const T *__restrict__ colscale,
                                                       int64_t ncoef, const CosTerm *__restrict__ ct,
                                                       int64_t ncoef_int, cx_t<T> *__restrict__ ghat) {
  const int r = blockIdx.y;
  if (blockIdx.x == 0) {   // the empty set (phi_0 = 1)
    if (threadIdx.x == 0) {
      const cx_t<T> v = fhat[(int64_t)r * ncoef];
      const T c = colscale ? colscale[0] : (T)1;
      ghat[(int64_t)r * ncoef_int] = cmake<T>(c * v.x, c * v.y);
    }
    return;
  }
  const CosTerm tm = ct[blockIdx.x - 1];
  const int t = tm.t, N = tm.N, Ki = 2 * N - 1, Ke = N - 1;
  int64_t size = 1;
  for (int j = 0; j < t; ++j) size *= Ki;
  const T norm = t == 1 ? (T)0.70710678118654752440 : (t == 2 ? (T)0.5 : (T)0.35355339059327376220);
  for (int64_t i = threadIdx.x; i < size; i += kVecBS) {
    int64_t rest = i, e = 0, pw = 1;
    bool zero = false;
    for (int j = t - 1; j >= 0; --j) {   // last axis fastest
      const int a = (int)(rest % Ki);
      rest /= Ki;
      const int l = a < N ? a - N : a - N + 1;
      const int k = l < 0 ? -l : l;
      zero |= k == N;
      e += (int64_t)(k - 1) * pw;
      pw *= Ke;
    }
    cx_t<T> out = cmake<T>((T)0, (T)0);
    if (!zero) {
      const cx_t<T> v = fhat[(int64_t)r * ncoef + tm.ext_off + e];
      const T c = norm * (colscale ? colscale[tm.ext_off + e] : (T)1);
      out = cmake<T>(c * v.x, c * v.y);
    }
    ghat[(int64_t)r * ncoef_int + tm.int_off + i] = out;
  }
}

// One workgroup per (term, right-hand side): fhat over the term's external group.
template <typename T>
__global__ __launch_bounds__(kVecBS) void k_cos_fold(const cx_t<T> *__restrict__ hhat, int64_t ncoef_int,
                                                     const CosTerm *__restrict__ ct, const T *__restrict__ colscale,
                                                     int64_t ncoef, cx_t<T> *__restrict__ fhat) {
  const int r = blockIdx.y;
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      const cx_t<T> v = hhat[(int64_t)r * ncoef_int];
      const T c = colscale ? colscale[0] : (T)1;
      fhat[(int64_t)r * ncoef] = cmake<T>(c * v.x, c * v.y);
    }
    return;
  }
  const CosTerm tm = ct[blockIdx.x - 1];
  const int t = tm.t, N = tm.N, Ki = 2 * N - 1, Ke = N - 1;
  int64_t size = 1;
  for (int j = 0; j < t; ++j) size *= Ke;
  const T norm = t == 1 ? (T)0.70710678118654752440 : (t == 2 ? (T)0.5 : (T)0.35355339059327376220);
  for (int64_t e = threadIdx.x; e < size; e += kVecBS) {
    int kk[3] = {0, 0, 0};
    int64_t rest = e;
    for (int j = t - 1; j >= 0; --j) {
      kk[j] = (int)(rest % Ke) + 1;
      rest /= Ke;
    }
    T sr = 0, si = 0;
    for (int sgn = 0; sgn < (1 << t); ++sgn) {   // sign patterns, a fixed order
      int64_t idx = 0;
      for (int j = 0; j < t; ++j) {
        const int l = (sgn >> j) & 1 ? -kk[j] : kk[j];
        idx = idx * Ki + (l < 0 ? l + N : l + N - 1);
      }
      const cx_t<T> v = hhat[(int64_t)r * ncoef_int + tm.int_off + idx];
      sr += v.x;
      si += v.y;
    }
    const T c = norm * (colscale ? colscale[tm.ext_off + e] : (T)1);
    fhat[(int64_t)r * ncoef + tm.ext_off + e] = cmake<T>(c * sr, c * si);
  }
}

// ------------------------------------------------------------------ launchers
}  // namespace gt
#include "fused.h"   // shared launches of orders 1 and 2
namespace gt {

template <typename T>
static OrderParams<T> order_params(const gt_plan *pl, int t) {
  const OrderHost &o = pl->ord[t];
  OrderParams<T> op;
  op.N = o.N;
  op.n = o.n;
  op.P = o.P;
  op.m = o.m;
  op.gsize = o.gsize;
  op.nfreq = o.N - 1;
  op.term_begin = o.term_begin;
  op.term_end = o.term_end;
  op.deconv = (const T *)o.d_deconv;
  op.roots = (const T *)o.d_roots;
  op.poly = (const T *)o.d_poly;
  return op;
}

template <typename K>
static int set_lds(K kernel, size_t bytes) {
  if (bytes > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(max dynamic LDS)");
  }
  return GT_OK;
}

static int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return GT_OK;
}

#define GT_DISPATCH_M(m, MACRO) \
  switch (m) {                  \
    case 2: MACRO(2); break;    \
    case 3: MACRO(3); break;    \
    case 4: MACRO(4); break;    \
    case 5: MACRO(5); break;    \
    case 6: MACRO(6); break;    \
    case 7: MACRO(7); break;    \
    case 8: MACRO(8); break;    \
    default: return fail(GT_EUNSUPPORTED, "window half-width outside 2..8"); \
  }

template <typename T>
static size_t pack_lds(const gt_plan *pl, int t) {
  const OrderHost &o = pl->ord[t];
  const size_t K = o.N - 1, n = o.n;
  const size_t c = sizeof(cx_t<T>);
  return c * (t == 1 ? K : t == 2 ? K * K + K * n : K * K * K + K * K * n + K * n * n) + c * (t == 1 ? n : K * n);
}

template <typename T>
static size_t adj_lds(const gt_plan *pl, int t) {
  const OrderHost &o = pl->ord[t];
  const size_t K = o.N - 1, n = o.n;
  const size_t c = sizeof(cx_t<T>);
  return c * (t == 1 ? n : t == 2 ? n * n + n * K : n * n * n + n * n * K) + c * (t == 1 ? n : K * n);
}

template <typename T>
static int launch_pack(gt_plan *pl, const void *fhat, const T *colscale, hipStream_t s, int only = 0) {
  using C = cx_t<T>;
  for (int t = 1; t <= pl->ds; ++t) {
    if (only && t != only) continue;
    const OrderHost &o = pl->ord[t];
    const int nt = o.term_end - o.term_begin;
    if (nt == 0) continue;
    OrderParams<T> op = order_params<T>(pl, t);
    const size_t lds = pack_lds<T>(pl, t);
    const int slices = t == 1 ? 4 : 8;
    dim3 grid(nt * slices, pl->R);
    prof_begin(s, t == 1 ? "pack_fwd_1d" : t == 2 ? "pack_fwd_2d" : "pack_fwd_3d");
    if (t == 1) {
      if (int rc = set_lds(k_pack_fwd<T, 1>, lds)) return rc;
      hipLaunchKernelGGL((k_pack_fwd<T, 1>), grid, dim3(kPackBS), lds, s, (const C *)fhat, colscale, pl->ncoef_int,
                         pl->d_terms, op, (C *)pl->d_grid, pl->grid_total, slices);
    } else if (t == 2) {
      if (int rc = set_lds(k_pack_fwd<T, 2>, lds)) return rc;
      hipLaunchKernelGGL((k_pack_fwd<T, 2>), grid, dim3(kPackBS), lds, s, (const C *)fhat, colscale, pl->ncoef_int,
                         pl->d_terms, op, (C *)pl->d_grid, pl->grid_total, slices);
    } else {
      if (int rc = set_lds(k_pack_fwd<T, 3>, lds)) return rc;
      hipLaunchKernelGGL((k_pack_fwd<T, 3>), grid, dim3(kPackBS), lds, s, (const C *)fhat, colscale, pl->ncoef_int,
                         pl->d_terms, op, (C *)pl->d_grid, pl->grid_total, slices);
    }
    prof_end(s);
    if (int rc = check_launch("k_pack_fwd")) return rc;
  }
  return GT_OK;
}

// Orders are independent until the final sums, so the order-1 kernels (and the empty
// set's) run on the plan's side stream, forked from and joined back into the caller's
// stream with events (inside a graph capture this makes parallel branches).  Not while
// per-launch profiling is on, nor when the plan's tuning turned it off.
static bool fork_side(gt_plan *pl, hipStream_t s) {
  if (!pl->side || !pl->use_side || prof_enabled() || pl->ds < 2) return false;
  if (hipEventRecord(pl->ev_fork, s) != hipSuccess) return false;
  return hipStreamWaitEvent(pl->side, pl->ev_fork, 0) == hipSuccess;
}
static int join_side(gt_plan *pl, hipStream_t s) {
  GT_HIP(hipEventRecord(pl->ev_join, pl->side));
  GT_HIP(hipStreamWaitEvent(s, pl->ev_join, 0));
  return GT_OK;
}

static DirectArgs direct_args(const gt_plan *pl, int t) {
  DirectArgs da;
  da.K = pl->ord[t].N - 1;
  da.G = 1;
  for (int a = 0; a < t; ++a) da.G *= da.K;
  da.half = pl->ord[t].N / 2;
  da.R = pl->R;
  da.M = pl->M;
  da.ncoef = pl->ncoef_int;
  return da;
}

// Direct forward of order t: f += sum over the order's terms (after the window orders'
// reduction, on the same stream).
template <typename T>
static int launch_direct_fwd(gt_plan *pl, int t, const void *fhat, const T *colscale, void *f, hipStream_t s) {
  using C = cx_t<T>;
  const OrderHost &o = pl->ord[t];
  const DirectArgs da = direct_args(pl, t);
  const int rtw = direct_fwd_rtw(pl, t), ct = pl->R <= 8 ? 1 : 2;
  const size_t rows = 64 * (size_t)rtw + kDirPad, KR = (size_t)(da.G / da.K), KR2 = KR + (KR & 1);
  const size_t breals = (((size_t)da.G + 1) * (16 * ct + 1) + 3) & ~(size_t)3;
  const size_t lds = breals * sizeof(T) +
                     (2 * ((size_t)da.K + 1) + (t >= 2 ? KR2 : 0) + (t == 3 ? 2 * (size_t)da.K : 0)) * rows * sizeof(C) +
                     (size_t)t * 64 * rtw * sizeof(T);
  const int nb = 64 * rtw;
  dim3 grid((unsigned)((pl->M + nb - 1) / nb));
  prof_begin(s, t == 1 ? "direct_fwd_1d" : t == 2 ? "direct_fwd_2d" : "direct_fwd_3d");
#define GT_LAUNCH_DF(ORD, CT, RTW)                                                                               \
  {                                                                                                              \
    if (int rc = set_lds(k_direct_fwd<T, ORD, CT, RTW>, lds)) return rc;                                         \
    hipLaunchKernelGGL((k_direct_fwd<T, ORD, CT, RTW>), grid, dim3(256), lds, s, (const T *)pl->d_x, pl->d_terms, \
                       o.term_begin, o.term_end, da, (const C *)fhat, colscale, (C *)f);                          \
  }
#define GT_LAUNCH_DF_O(ORD)                     \
  {                                             \
    if (ct == 1 && rtw == 1) GT_LAUNCH_DF(ORD, 1, 1) \
    else if (ct == 1 && rtw == 2) GT_LAUNCH_DF(ORD, 1, 2) \
    else if (ct == 1) GT_LAUNCH_DF(ORD, 1, 4)        \
    else if (rtw == 1) GT_LAUNCH_DF(ORD, 2, 1)       \
    else if (rtw == 2) GT_LAUNCH_DF(ORD, 2, 2)       \
    else GT_LAUNCH_DF(ORD, 2, 4)                     \
  }
  if (t == 1) GT_LAUNCH_DF_O(1)
  else if (t == 2) GT_LAUNCH_DF_O(2)
  else GT_LAUNCH_DF_O(3)
#undef GT_LAUNCH_DF_O
#undef GT_LAUNCH_DF
  prof_end(s);
  return check_launch("k_direct_fwd");
}

// Direct adjoint of order t: slice partials, then their sums into the order's coefficients.
template <typename T>
static int launch_direct_adj(gt_plan *pl, int t, const void *y, const T *colscale, void *fhat, hipStream_t s) {
  using C = cx_t<T>;
  const OrderHost &o = pl->ord[t];
  const DirectArgs da = direct_args(pl, t);
  const int nt = o.term_end - o.term_begin, S = o.dir_nslice, rtw = direct_adj_rtw(pl, t);
  if (!o.d_dpart || S < 1 || rtw < 1) return fail(GT_EINVAL, "direct adjoint not set up");
  const size_t lds = (3 * (size_t)da.K + 1 + (t >= 2 ? (size_t)(da.G / da.K) : 0) + (t == 3 ? 2 * (size_t)da.K : 0)) *
                     kDirRowA * sizeof(C);
  prof_begin(s, t == 1 ? "direct_adj_1d" : t == 2 ? "direct_adj_2d" : "direct_adj_3d");
#define GT_LAUNCH_DA(ORD, RTW)                                                                                   \
  {                                                                                                              \
    if (int rc = set_lds(k_direct_adj<T, ORD, RTW>, lds)) return rc;                                             \
    hipLaunchKernelGGL((k_direct_adj<T, ORD, RTW>), dim3((unsigned)S, (unsigned)nt), dim3(256), lds, s,          \
                       (const T *)pl->d_x, pl->d_terms, o.term_begin, da, S, (const C *)y, (T *)o.d_dpart);      \
  }
#define GT_LAUNCH_DA_O(ORD)                              \
  {                                                      \
    if (rtw == 1) GT_LAUNCH_DA(ORD, 1)                   \
    else if (rtw == 2) GT_LAUNCH_DA(ORD, 2)              \
    else if (rtw == 4) GT_LAUNCH_DA(ORD, 4)              \
    else GT_LAUNCH_DA(ORD, 8)                            \
  }
  if (t == 1) GT_LAUNCH_DA_O(1)
  else if (t == 2) GT_LAUNCH_DA_O(2)
  else GT_LAUNCH_DA_O(3)
#undef GT_LAUNCH_DA_O
#undef GT_LAUNCH_DA
  if (int rc = check_launch("k_direct_adj")) return rc;
  hipLaunchKernelGGL((k_direct_adj_sum<T>), dim3((unsigned)((da.G * da.R + 255) / 256), (unsigned)nt), dim3(256), 0, s,
                     (const T *)o.d_dpart, pl->d_terms, o.term_begin, da, S, 64 * rtw, colscale, (C *)fhat);
  prof_end(s);
  return check_launch("k_direct_adj_sum");
}

static Tile2Args tile2_args(const gt_plan *pl) {
  const OrderHost &o = pl->ord[2];
  Tile2Args ta;
  ta.waves = o.d_waves2;
  ta.nwaves = o.nwaves2;
  ta.ntile = o.ntile;
  ta.nseg = o.nseg2;
  ta.vstride = pl->ragged ? 0 : pl->M;
  ta.ragged = pl->ragged ? 1 : 0;
  return ta;
}

// ---- shared launches of orders 1 and 2 (fused.h)

// Forward: packs of both orders, gathers of both orders, then the sum over u.
template <typename T>
static int fused_forward(gt_plan *pl, const void *fhat, const T *colscale, void *f, hipStream_t s) {
  using C = cx_t<T>;
  const OrderHost &o1 = pl->ord[1], &o2 = pl->ord[2];
  const int nt1 = o1.term_end - o1.term_begin, nt2 = o2.term_end - o2.term_begin, R = pl->R;
  const bool poly = std::is_same<T, float>::value && o2.path == GT_GATHER_POLY;
  // 1. K1 + K2 of both orders (order 2 straight into the window polynomials when it gathers
  //    in that basis)
  FwdPackArgs<T> pa;
  pa.fhat = (const C *)fhat;
  pa.colscale = colscale;
  pa.ncoef = pl->ncoef_int;
  pa.terms = pl->d_terms;
  pa.grids = (C *)pl->d_grid;
  pa.grid_total = pl->grid_total;
  pa.op1 = order_params<T>(pl, 1);
  pa.op2 = order_params<T>(pl, 2);
  pa.slices1 = 4;
  pa.slices2 = 8;
  pa.nslab = (o2.n + kPolyRows - 1) / kPolyRows;
  pa.kpoly = (C *)o2.d_kpoly;
  pa.p1 = Part{0, nt1 * pa.slices1, R};
  pa.p2 = Part{pa.p1.nx * R, nt2 * (poly ? pa.nslab : pa.slices2), R};
  const unsigned nbp = (unsigned)(pa.p2.b0 + pa.p2.nx * pa.p2.ny);
  const size_t plds = std::max(pack_lds<T>(pl, 1), poly ? poly_pack_lds(o2) : pack_lds<T>(pl, 2));
  prof_begin(s, "pack_fwd_12");
  if (poly) {
    if constexpr (std::is_same<T, float>::value) {
#define GT_LAUNCH_FPACK(MH)                                                                  \
  {                                                                                          \
    if (int rc = set_lds(k_fwd_pack2<T, MH>, plds)) return rc;                               \
    hipLaunchKernelGGL((k_fwd_pack2<T, MH>), dim3(nbp), dim3(kPackBS), plds, s, pa);         \
  }
      GT_DISPATCH_M(o2.m, GT_LAUNCH_FPACK)
#undef GT_LAUNCH_FPACK
    }
  } else {
    if (int rc = set_lds(k_fwd_pack2<T, 0>, plds)) return rc;
    hipLaunchKernelGGL((k_fwd_pack2<T, 0>), dim3(nbp), dim3(kPackBS), plds, s, pa);
  }
  prof_end(s);
  if (int rc = check_launch("k_fwd_pack2")) return rc;
  // 2. K3 of both orders, each term into its slot (term u -> slot u - 1)
  FwdGatherArgs<T> ga;
  ga.x = (const T *)pl->d_x;
  ga.Mtot = pl->Mtot;
  ga.terms = pl->d_terms;
  ga.grids = (const C *)pl->d_grid;
  ga.grid_total = pl->grid_total;
  ga.op1 = pa.op1;
  ga.op2 = pa.op2;
  ga.perm1 = o1.d_perm;
  ga.perm2 = o2.d_perm;
  ga.xs2 = (const T *)o2.d_xs;
  ga.kpoly = (const C *)o2.d_kpoly;
  ga.vstride = pl->ragged ? 0 : pl->M;
  ga.sbase1 = ga.sbase2 = -1;
  ga.slots = (C *)pl->d_fpart;
  ga.Vtot = pl->Vtot;
  size_t glds = 0;
  int b0 = 0;
  auto gpart = [&](const OrderHost &o, int nt, const GatherItem *&gi, const CellItem *&ci, int &nci) {
    Part p;
    gi = nullptr;
    ci = nullptr;
    nci = 0;
    if (o.path == GT_GATHER_SORTED) {
      const int i0 = o.gitem_begin[0], i1 = o.gitem_begin[nt];
      gi = o.d_gitems + i0;
      p = Part{b0, i1 - i0, 1};
      glds = std::max(glds, (size_t)o.gsize * sizeof(C));
    } else {
      const int c0 = o.citem_begin[0], c1 = o.citem_begin[nt];
      ci = o.d_citems + c0;
      nci = c1 - c0;
      p = Part{b0, (nci + 3) / 4, pl->ragged ? 1 : R};
    }
    b0 += (p.nx * p.ny + 7) / 8 * 8;   // the next part starts at a multiple of 8 blocks
    return p;
  };
  ga.p1 = gpart(o1, nt1, ga.gi1, ga.ci1, ga.nci1);
  ga.p2 = gpart(o2, nt2, ga.gi2, ga.ci2, ga.nci2);
  prof_begin(s, "gather_12");
#define GT_LAUNCH_FG(MH, K1, K2)                                                                 \
  {                                                                                              \
    if (int rc = set_lds(k_fwd_gather2<T, MH, K1, K2>, glds)) return rc;                         \
    hipLaunchKernelGGL((k_fwd_gather2<T, MH, K1, K2>), dim3((unsigned)b0), dim3(256), glds, s, ga); \
  }
#define GT_LAUNCH_FGATHER(MH)                                                                          \
  {                                                                                                    \
    const bool s1 = o1.path == GT_GATHER_SORTED;                                                       \
    if (o2.path == GT_GATHER_POLY) {                                                                   \
      if constexpr (std::is_same<T, float>::value) {                                                   \
        if (s1) GT_LAUNCH_FG(MH, GT_GATHER_SORTED, GT_GATHER_POLY)                                     \
        else GT_LAUNCH_FG(MH, GT_GATHER_CELL, GT_GATHER_POLY)                                          \
      }                                                                                                \
    } else if (o2.path == GT_GATHER_SORTED) {                                                          \
      if (s1) GT_LAUNCH_FG(MH, GT_GATHER_SORTED, GT_GATHER_SORTED)                                     \
      else GT_LAUNCH_FG(MH, GT_GATHER_CELL, GT_GATHER_SORTED)                                          \
    } else {                                                                                           \
      if (s1) GT_LAUNCH_FG(MH, GT_GATHER_SORTED, GT_GATHER_CELL)                                       \
      else GT_LAUNCH_FG(MH, GT_GATHER_CELL, GT_GATHER_CELL)                                            \
    }                                                                                                  \
  }
  GT_DISPATCH_M(o1.m, GT_LAUNCH_FGATHER)
#undef GT_LAUNCH_FGATHER
#undef GT_LAUNCH_FG
  prof_end(s);
  if (int rc = check_launch("k_fwd_gather2")) return rc;
  // 3. the sum over u per node, with the empty set's coefficient
  const int ngi = (int)pl->gitems.size();
  prof_begin(s, "reduce_f");
  hipLaunchKernelGGL((k_reduce_f<T>), dim3(4 * ngi), dim3(256), 0, s, (const C *)fhat, pl->ncoef_int, pl->d_gitems,
                     (const C *)pl->d_fpart, nt1 + nt2, pl->Vtot, 0, (C *)f);
  prof_end(s);
  return check_launch("k_reduce_f");
}

// Adjoint: spreads of both orders with the empty set's partial sums, folds of both orders
// with the empty set's coefficient, then the DFTs of both orders.
template <typename T>
static int fused_adjoint(gt_plan *pl, const void *y, const T *colscale, void *fhat, hipStream_t s) {
  using C = cx_t<T>;
  const OrderHost &o1 = pl->ord[1], &o2 = pl->ord[2];
  const int nt1 = o1.term_end - o1.term_begin, nt2 = o2.term_end - o2.term_begin, R = pl->R;
  const int ngi = (int)pl->gitems.size();
  const OrderParams<T> op1 = order_params<T>(pl, 1), op2 = order_params<T>(pl, 2);
  const Tile2Args ta = tile2_args(pl);
  // 1. K4: order 2 on tiles, order 1 binned, the empty set's partial sums
  AdjSpreadArgs<T> sa;
  sa.x = (const T *)pl->d_x;
  sa.Mtot = pl->Mtot;
  sa.terms = pl->d_terms;
  sa.y = (const C *)y;
  sa.si1 = o1.d_sitems;
  sa.op1 = op1;
  sa.sa1.perm = o1.d_perm;
  sa.sa1.cstart = o1.d_cstart;
  sa.sa1.B = pl->ragged ? R : 1;
  sa.sa1.ncell = o1.nkey;
  sa.sa1.vstride = pl->ragged ? 0 : pl->M;
  sa.sa1.copies = spread1_copies(pl);
  sa.gpart1 = (C *)o1.d_gpart;
  sa.gstride1 = o1.gpart_stride;
  sa.xs2 = (const T *)o2.d_xs;
  sa.perm2 = (const int32_t *)o2.d_perm;
  sa.op2 = op2;
  sa.ta = ta;
  sa.patch = (C *)o2.d_patch;
  sa.gitems = pl->d_gitems;
  sa.ysum = pl->d_ysum;
  sa.p1 = Part{0, (int)o1.sitems.size(), nt1};
  sa.pe = Part{sa.p1.nx * sa.p1.ny, ngi, 1};
  sa.p2 = Part{sa.pe.b0 + sa.pe.nx, (o2.nwaves2 + kTileWaves - 1) / kTileWaves, pl->ragged ? 1 : R};
  const unsigned nbs = (unsigned)(sa.p2.b0 + sa.p2.nx * sa.p2.ny);
  // padded so that at most tile_wg_cu workgroups share a compute unit
  const size_t slds = std::max({kTileWaves * tile_lds_wave(sizeof(T)),
                                pl->lds_limit / o2.tile_wg_cu,
                                (size_t)sa.sa1.copies * o1.gsize * sizeof(double2)});
  prof_begin(s, "spread_12");
#define GT_LAUNCH_FSPREAD(MH)                                                                \
  {                                                                                          \
    if (int rc = set_lds(k_adj_spread2<T, MH>, slds)) return rc;                             \
    hipLaunchKernelGGL((k_adj_spread2<T, MH>), dim3(nbs), dim3(64 * kTileWaves), slds, s, sa); \
  }
  GT_DISPATCH_M(o1.m, GT_LAUNCH_FSPREAD)
#undef GT_LAUNCH_FSPREAD
  prof_end(s);
  if (int rc = check_launch("k_adj_spread2")) return rc;
  // 2. folds: order-2 patches into column sums (tile-sum form), order-1 partial grids, and
  //    the empty set's coefficient
  AdjFoldArgs<T> fa;
  fa.terms = pl->d_terms;
  fa.gpart1 = (const C *)o1.d_gpart;
  fa.gstride1 = o1.gpart_stride;
  fa.sitem_begin1 = o1.d_sitem_begin;
  fa.op1 = op1;
  fa.gsum1 = (C *)o1.d_gsum;
  fa.patch = (const C *)o2.d_patch;
  fa.tileseg = o2.d_tileseg;
  fa.op2 = op2;
  fa.ta = ta;
  fa.B = pl->ragged ? R : 1;
  fa.ts = o2.ts;
  fa.nunits2 = nt2 * o2.ntile * 4;
  fa.hcol2 = (C *)o2.d_tsum;
  fa.gitem_begin = pl->d_gitem_begin;
  fa.ysum = (const double *)pl->d_ysum;
  fa.ncoef = pl->ncoef_int;
  fa.fhat = (C *)fhat;
  fa.p2 = Part{0, nt2 * o2.ntile, R};
  const int64_t pts1 = (int64_t)o1.n * nt1;
  fa.p1 = Part{fa.p2.nx * fa.p2.ny, (int)((pts1 + 63) / 64), R};
  fa.pe = Part{fa.p1.b0 + fa.p1.nx * fa.p1.ny, R, 1};
  const unsigned nbf = (unsigned)(fa.pe.b0 + fa.pe.nx);
  const size_t flds = (size_t)4 * o2.ntile * 64 * sizeof(C);
  prof_begin(s, "fold_12");
  if (int rc = set_lds(k_adj_fold2<T>, flds)) return rc;
  hipLaunchKernelGGL((k_adj_fold2<T>), dim3(nbf), dim3(256), flds, s, fa);
  prof_end(s);
  if (int rc = check_launch("k_adj_fold2")) return rc;
  // 3. K2 + K5 of both orders
  AdjDftArgs<T> da;
  da.terms = pl->d_terms;
  da.colscale = colscale;
  da.ncoef = pl->ncoef_int;
  da.fhat = (C *)fhat;
  da.gsum1 = (const C *)o1.d_gsum;
  da.op1 = op1;
  da.hcol2 = (const C *)o2.d_tsum;
  da.op2 = op2;
  const size_t lds_h = (size_t)o2.ntile * 16 * o2.n * sizeof(C);
  const bool stage_h = adj_lds<T>(pl, 2) + lds_h <= pl->lds_limit;
  da.ntile2 = stage_h ? o2.ntile : -o2.ntile;
  da.ts2 = o2.ts;
  da.nsplit2 = std::max(1, std::min(4, (o2.N - 1) / 8));
  da.p2 = Part{0, nt2 * da.nsplit2, R};
  da.p1 = Part{da.p2.nx * da.p2.ny, nt1, R};
  const unsigned nbd = (unsigned)(da.p1.b0 + da.p1.nx * da.p1.ny);
  const size_t dlds = std::max(adj_lds<T>(pl, 1), adj_lds<T>(pl, 2) + (stage_h ? lds_h : 0));
  prof_begin(s, "dft_adj_12");
  if (int rc = set_lds(k_adj_dft2<T>, dlds)) return rc;
  hipLaunchKernelGGL((k_adj_dft2<T>), dim3(nbd), dim3(2 * kPackBS), dlds, s, da);
  prof_end(s);
  return check_launch("k_adj_dft2");
}

template <typename T>
static int forward_core(gt_plan *pl, const void *fhat, const T *colscale, void *f, hipStream_t s) {
  using C = cx_t<T>;
  const int ngi = (int)pl->gitems.size();
  if (ngi == 0) return launch_pack<T>(pl, fhat, colscale, s);
  if (pl->use_fused && fused_available(pl)) return fused_forward<T>(pl, fhat, colscale, f, s);
  // The window orders' terms, numbered 1..nt_all in term order without the direct orders'
  // (position = term - dshift[t]), in blocks of nslots; each block: gathers into slots, then
  // one reduction.  The direct orders add their sums afterwards.
  int dshift[kMaxOrder + 1] = {0, 0, 0, 0};
  int nt_all = 0;
  for (int t = 1, nd = 0; t <= pl->ds; ++t) {
    const OrderHost &o = pl->ord[t];
    dshift[t] = nd;
    if (o.path == GT_GATHER_DIRECT)
      nd += o.term_end - o.term_begin;
    else
      nt_all += o.term_end - o.term_begin;
  }
  const int S = std::max(1, pl->nslots);
  for (int g0 = 1, blk = 0; blk == 0 || g0 <= nt_all; g0 += S, ++blk) {
    const int g1 = std::min(nt_all + 1, g0 + S);
    const bool fk = fork_side(pl, s);
    for (int t = 1; t <= pl->ds; ++t) {
      const hipStream_t st = (fk && t == 1) ? pl->side : s;
      const OrderHost &o = pl->ord[t];
      if (o.path == GT_GATHER_DIRECT) continue;
      bool packed = false;
      if constexpr (std::is_same<T, float>::value) {
        if (blk == 0 && t == 2 && o.path == GT_GATHER_POLY) {   // order 2: pack straight into per-cell polynomials
          const OrderParams<float> opf = order_params<float>(pl, 2);
          const int nt2 = o.term_end - o.term_begin, nslab = (o.n + kPolyRows - 1) / kPolyRows;
          const size_t plds = poly_pack_lds(o);
          dim3 pgrid((unsigned)(nt2 * nslab), (unsigned)pl->R);
          prof_begin(st, "pack_fwd_2d");
#define GT_LAUNCH_PPACK(MH)                                                                                      \
  {                                                                                                              \
    if (int rc = set_lds(k_pack_poly2<MH>, plds)) return rc;                                                     \
    hipLaunchKernelGGL((k_pack_poly2<MH>), pgrid, dim3(kPackBS), plds, st, (const C *)fhat, colscale, pl->ncoef_int, \
                       pl->d_terms, opf, nslab, (C *)o.d_kpoly);                                                 \
  }
          GT_DISPATCH_M(o.m, GT_LAUNCH_PPACK)
#undef GT_LAUNCH_PPACK
          prof_end(st);
          if (int rc = check_launch("k_pack_poly2")) return rc;
          packed = true;
        }
      }
      if (blk == 0 && !packed)
        if (int rc = launch_pack<T>(pl, fhat, colscale, st, t)) return rc;
      const int tb = std::max(g0 + dshift[t], o.term_begin), te = std::min(g1 + dshift[t], o.term_end);
      if (tb >= te) continue;
      const int sbase = -(g0 + dshift[t]);   // slot of term u: u + sbase
      OrderParams<T> op = order_params<T>(pl, t);
      if (o.path != GT_GATHER_SORTED) {   // cell gather: one wavefront per run of a cell's nodes
        const int c0 = o.citem_begin[tb - o.term_begin], c1 = o.citem_begin[te - o.term_begin];
        if (c1 <= c0) continue;
        const int64_t vstride = pl->ragged ? 0 : pl->M;
        dim3 grid((unsigned)((c1 - c0 + 3) / 4), pl->ragged ? 1u : (unsigned)pl->R);
        prof_begin(st, t == 1 ? "gather_1d" : t == 2 ? "gather_2d" : "gather_3d");
        if constexpr (std::is_same<T, float>::value) {
          if (t == 2 && o.path == GT_GATHER_POLY) {
            hipLaunchKernelGGL((k_gather_poly2<T>), grid, dim3(256), 0, st, (const T *)o.d_xs, o.d_citems + c0,
                               c1 - c0, o.d_perm, op, (const C *)o.d_kpoly, vstride, sbase,
                               (C *)pl->d_fpart, pl->Vtot);
            prof_end(st);
            if (int rc = check_launch("k_gather_poly2")) return rc;
            continue;
          }
        }
#define GT_LAUNCH_CELL(MH)                                                                                          \
  {                                                                                                                 \
    if (t == 1)                                                                                                     \
      hipLaunchKernelGGL((k_gather_cell<T, 1, MH>), grid, dim3(256), 0, st, (const T *)pl->d_x, pl->Mtot,           \
                         o.d_citems + c0, c1 - c0, o.d_perm, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, \
                         vstride, sbase, (C *)pl->d_fpart, pl->Vtot);                                                 \
    else if (t == 2)                                                                                                \
      hipLaunchKernelGGL((k_gather_cell<T, 2, MH>), grid, dim3(256), 0, st, (const T *)pl->d_x, pl->Mtot,           \
                         o.d_citems + c0, c1 - c0, o.d_perm, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, \
                         vstride, sbase, (C *)pl->d_fpart, pl->Vtot);                                                 \
    else                                                                                                            \
      hipLaunchKernelGGL((k_gather_cell<T, 3, MH>), grid, dim3(256), 0, st, (const T *)pl->d_x, pl->Mtot,           \
                         o.d_citems + c0, c1 - c0, o.d_perm, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, \
                         vstride, sbase, (C *)pl->d_fpart, pl->Vtot);                                                 \
  }
        GT_DISPATCH_M(o.m, GT_LAUNCH_CELL)
#undef GT_LAUNCH_CELL
        prof_end(st);
        if (int rc = check_launch("k_gather_cell")) return rc;
        continue;
      }
      const int i0 = o.gitem_begin[tb - o.term_begin], i1 = o.gitem_begin[te - o.term_begin];
      if (i1 <= i0) continue;
      const size_t lds = (size_t)o.gsize * sizeof(C);
      const GatherItem *items = o.d_gitems + i0;
      const int64_t vstride = pl->ragged ? 0 : pl->M;
      dim3 grid(i1 - i0);
      prof_begin(st, t == 1 ? "gather_1d" : t == 2 ? "gather_2d" : "gather_3d");
#define GT_LAUNCH_GATHER(MH)                                                                                      \
  {                                                                                                               \
    if (t == 1) {                                                                                                 \
      if (int rc = set_lds(k_gather_sorted<T, 1, MH>, lds)) return rc;                                            \
      hipLaunchKernelGGL((k_gather_sorted<T, 1, MH>), grid, dim3(kGatherBS), lds, st, (const T *)pl->d_x, pl->Mtot, \
                         items, o.d_perm, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, vstride, sbase,  \
                         (C *)pl->d_fpart, pl->Vtot);                                                            \
    } else if (t == 2) {                                                                                          \
      if (int rc = set_lds(k_gather_sorted<T, 2, MH>, lds)) return rc;                                            \
      hipLaunchKernelGGL((k_gather_sorted<T, 2, MH>), grid, dim3(kGatherBS), lds, st, (const T *)pl->d_x, pl->Mtot, \
                         items, o.d_perm, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, vstride, sbase,  \
                         (C *)pl->d_fpart, pl->Vtot);                                                            \
    } else {                                                                                                      \
      if (int rc = set_lds(k_gather_sorted<T, 3, MH>, lds)) return rc;                                            \
      hipLaunchKernelGGL((k_gather_sorted<T, 3, MH>), grid, dim3(kGatherBS), lds, st, (const T *)pl->d_x, pl->Mtot, \
                         items, o.d_perm, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, vstride, sbase,  \
                         (C *)pl->d_fpart, pl->Vtot);                                                            \
    }                                                                                                             \
  }
      GT_DISPATCH_M(o.m, GT_LAUNCH_GATHER)
#undef GT_LAUNCH_GATHER
      prof_end(st);
      if (int rc = check_launch("k_gather_sorted")) return rc;
    }
    if (fk)
      if (int rc = join_side(pl, s)) return rc;
    prof_begin(s, "reduce_f");
    hipLaunchKernelGGL((k_reduce_f<T>), dim3(4 * ngi), dim3(256), 0, s, (const C *)fhat, pl->ncoef_int, pl->d_gitems,
                       (const C *)pl->d_fpart, g1 - g0, pl->Vtot, blk > 0 ? 1 : 0, (C *)f);
    prof_end(s);
    if (int rc = check_launch("k_reduce_f")) return rc;
    if (nt_all <= 0) break;
  }
  for (int t = 1; t <= pl->ds; ++t)
    if (pl->ord[t].path == GT_GATHER_DIRECT)
      if (int rc = launch_direct_fwd<T>(pl, t, fhat, colscale, f, s)) return rc;
  return GT_OK;
}


template <typename T>
static int adjoint_core(gt_plan *pl, const void *y, const T *colscale, void *fhat, hipStream_t s) {
  using C = cx_t<T>;
  const int ngi = (int)pl->gitems.size();
  if (pl->use_fused && fused_available(pl)) return fused_adjoint<T>(pl, y, colscale, fhat, s);
  const bool fk = fork_side(pl, s);
  for (int t = 1; t <= pl->ds; ++t) {
    const hipStream_t st = (fk && t == 1) ? pl->side : s;
    const OrderHost &o = pl->ord[t];
    const int nt = o.term_end - o.term_begin;
    const int nsi = (int)o.sitems.size();
    if (nt > 0 && o.adj_form == GT_ADJ_DIRECT) {
      if (int rc = launch_direct_adj<T>(pl, t, y, colscale, fhat, st)) return rc;
      continue;
    }
    if (nt == 0 || (t == 2 ? o.nwaves2 == 0 : nsi == 0)) continue;
    OrderParams<T> op = order_params<T>(pl, t);
    SpreadArgs sa;
    sa.perm = o.d_perm;
    sa.cstart = o.d_cstart;
    sa.B = pl->ragged ? pl->R : 1;
    sa.ncell = o.nkey;
    sa.vstride = pl->ragged ? 0 : pl->M;
    sa.copies = t == 1 ? spread1_copies(pl) : 1;
    const size_t lds = (size_t)sa.copies * o.gsize * sizeof(double2);
    dim3 grid(nsi, nt);
    prof_begin(st, t == 1 ? "spread_1d" : t == 2 ? "spread_2d" : "spread_3d");
#define GT_LAUNCH_SPREAD(MH)                                                                                      \
  {                                                                                                               \
    if (t == 1) {                                                                                                 \
      if (int rc = set_lds(k_spread_binned<T, 1, MH>, lds)) return rc;                                            \
      hipLaunchKernelGGL((k_spread_binned<T, 1, MH>), grid, dim3(64 * kSpreadWaves), lds, st, (const T *)pl->d_x, pl->Mtot,       \
                         o.d_sitems, pl->d_terms, op, sa, (const C *)y, (C *)o.d_gpart, o.gpart_stride);         \
    } else {                                                                                                      \
      if (int rc = set_lds(k_spread_cell3<T, MH>, lds)) return rc;                                                \
      hipLaunchKernelGGL((k_spread_cell3<T, MH>), grid, dim3(64 * kSpreadWaves), lds, st, (const T *)pl->d_x, pl->Mtot,           \
                         o.d_sitems, pl->d_terms, op, sa, (const C *)y, (C *)o.d_gpart, o.gpart_stride);         \
    }                                                                                                             \
  }
    const Tile2Args ta = tile2_args(pl);
#define GT_LAUNCH_TILE2(MH)                                                                                       \
  {                                                                                                               \
    /* padded so that at most tile_wg_cu workgroups share a compute unit */                                   \
    const size_t lds2 = std::max<size_t>(kTileWaves * tile_lds_wave(sizeof(T)),    \
                                         pl->lds_limit / o.tile_wg_cu);                                           \
    if (int rc = set_lds(k_spread_tile2<T, MH>, lds2)) return rc;                                                 \
    hipLaunchKernelGGL((k_spread_tile2<T, MH>), dim3((unsigned)((o.nwaves2 + kTileWaves - 1) / kTileWaves),     \
                       (unsigned)(pl->ragged ? 1 : pl->R)), dim3(64 * kTileWaves), lds2, st, (const T *)o.d_xs,      \
                       (const int32_t *)o.d_perm, op, ta, (const C *)y, (C *)o.d_patch);                           \
  }
    if (t == 2) {
      GT_DISPATCH_M(o.m, GT_LAUNCH_TILE2)
    } else {
      GT_DISPATCH_M(o.m, GT_LAUNCH_SPREAD)
    }
#undef GT_LAUNCH_TILE2
#undef GT_LAUNCH_SPREAD
    prof_end(st);
    if (int rc = check_launch("k_spread")) return rc;
  }
  for (int t = 1; t <= pl->ds; ++t) {
    const hipStream_t st = (fk && t == 1) ? pl->side : s;
    const OrderHost &o = pl->ord[t];
    const int nt = o.term_end - o.term_begin;
    if (nt == 0 || o.adj_form == GT_ADJ_DIRECT) continue;
    OrderParams<T> op = order_params<T>(pl, t);
    // order 2: the adjoint DFT stages the column-folded patches in LDS when they fit
    const size_t lds_h = t == 2 ? (size_t)o.ntile * 16 * o.n * sizeof(C) : 0;
    const bool stage_h = t == 2 && adj_lds<T>(pl, t) + lds_h <= pl->lds_limit;
    const size_t lds = adj_lds<T>(pl, t) + (stage_h ? lds_h : 0);
    if (t == 2) {
      prof_begin(st, "fold_2d");
      const int64_t ncol = (int64_t)nt * o.ntile * 16 * o.n;
      if (o.P <= 2 * o.n && o.ntile <= 32) {
        // coalesced form: one wavefront per (term, tile row, four patch rows), tile sums in LDS
        hipLaunchKernelGGL((k_fold_tilesum<T>), dim3((unsigned)(nt * o.ntile * 4), pl->R), dim3(64),
                           (size_t)o.ntile * 64 * sizeof(C), st, (const C *)o.d_patch, o.d_tileseg, op,
                           tile2_args(pl), pl->ragged ? pl->R : 1, o.ts, (C *)o.d_tsum);
      } else {
        // flattened form when a column has at most two halo positions (P <= 2n), else one step
        // at a time.  Tiles covering one halo column: at most 15 / ts + 1 <= 16.  (Rows of more
        // than 32 tiles only occur for ts = 1 within the grid sizes the plan accepts.)
        auto fold = o.P > 2 * o.n ? k_fold_cols_seq<T> : k_fold_cols<T, 16>;
        hipLaunchKernelGGL(fold, dim3((unsigned)((ncol + 255) / 256), pl->R), dim3(256), 0, st,
                           (const C *)o.d_patch, o.d_tileseg, op, tile2_args(pl), pl->ragged ? pl->R : 1, o.ts,
                           (C *)o.d_tsum);
      }
      prof_end(st);
      if (int rc = check_launch("k_fold_cols")) return rc;
    } else {
      const int64_t outer = t == 1 ? 1 : (int64_t)o.n * o.n;
      const int64_t pts = outer * o.n * nt;
      prof_begin(st, t == 1 ? "fold_1d" : "fold_3d");
      hipLaunchKernelGGL((k_fold_partials<T>), dim3((unsigned)((pts + 63) / 64), pl->R), dim3(256), 0, st,
                         (const C *)o.d_gpart, o.gpart_stride, o.d_sitem_begin, pl->d_terms, op, t, (C *)o.d_gsum);
      prof_end(st);
      if (int rc = check_launch("k_fold_partials")) return rc;
    }
    dim3 grid(nt, pl->R);
    prof_begin(st, t == 1 ? "dft_adj_1d" : t == 2 ? "dft_adj_2d" : "dft_adj_3d");
    if (t == 1) {
      if (int rc = set_lds(k_dft_adj<T, 1>, lds)) return rc;
      hipLaunchKernelGGL((k_dft_adj<T, 1>), grid, dim3(kPackBS), lds, st, (const C *)o.d_gsum, pl->d_terms, op,
                         colscale, pl->ncoef_int, (C *)fhat, 0, 0, 1);
    } else if (t == 2) {
      if (int rc = set_lds(k_dft_adj<T, 2>, lds)) return rc;
      // up to four workgroups per term (column ranges of at least 8 frequencies)
      const int nsplit = std::max(1, std::min(4, (o.N - 1) / 8));
      hipLaunchKernelGGL((k_dft_adj<T, 2>), dim3(nt * nsplit, pl->R), dim3(2 * kPackBS), lds, st,
                         (const C *)o.d_tsum, pl->d_terms, op, colscale, pl->ncoef_int, (C *)fhat,
                         stage_h ? o.ntile : -o.ntile, o.ts, nsplit);
    } else {
      if (int rc = set_lds(k_dft_adj<T, 3>, lds)) return rc;
      hipLaunchKernelGGL((k_dft_adj<T, 3>), grid, dim3(kPackBS), lds, st, (const C *)o.d_gsum, pl->d_terms, op,
                         colscale, pl->ncoef_int, (C *)fhat, 0, 0, 1);
    }
    prof_end(st);
    if (int rc = check_launch("k_dft_adj")) return rc;
  }
  if (ngi > 0) {
    const hipStream_t st = fk ? pl->side : s;
    prof_begin(st, "empty_adj");
    hipLaunchKernelGGL((k_empty_part<T>), dim3(ngi), dim3(kGatherBS), 0, st, pl->d_gitems, (const C *)y,
                       pl->d_ysum);
    hipLaunchKernelGGL((k_empty_adj<T>), dim3(pl->R), dim3(kGatherBS), 0, st, pl->d_gitem_begin,
                       (const double *)pl->d_ysum, pl->ncoef_int, (C *)fhat);
    prof_end(st);
    if (int rc = check_launch("k_empty_adj")) return rc;
  }
  if (fk)
    if (int rc = join_side(pl, s)) return rc;
  return GT_OK;
}

template <typename T>
static int cos_expand(gt_plan *pl, const void *fhat, const T *colscale, hipStream_t s) {
  using C = cx_t<T>;
  hipLaunchKernelGGL((k_cos_expand<T>), dim3((unsigned)pl->nterms, (unsigned)pl->R), dim3(kVecBS), 0, s,
                     (const C *)fhat, colscale, pl->ncoef, pl->d_cterms, pl->ncoef_int, (C *)pl->d_gcos);
  return check_launch("k_cos_expand");
}

// Forward and adjoint in the plan's basis.  The exponential basis runs the transform kernels
// directly; the cosine basis expands the coefficients (with the column scaling) into the
// plan's exponential coefficient buffer first, or folds the exponential adjoint out of it.
template <typename T>
int launch_forward(gt_plan *pl, const void *fhat, const T *colscale, void *f, hipStream_t s) {
  if (pl->basis != GT_BASIS_COS) return forward_core<T>(pl, fhat, colscale, f, s);
  if (int rc = cos_expand<T>(pl, fhat, colscale, s)) return rc;
  return forward_core<T>(pl, pl->d_gcos, nullptr, f, s);
}

template <typename T>
int launch_adjoint(gt_plan *pl, const void *y, const T *colscale, void *fhat, hipStream_t s) {
  using C = cx_t<T>;
  if (pl->basis != GT_BASIS_COS) return adjoint_core<T>(pl, y, colscale, fhat, s);
  if (int rc = adjoint_core<T>(pl, y, nullptr, pl->d_gcos, s)) return rc;
  hipLaunchKernelGGL((k_cos_fold<T>), dim3((unsigned)pl->nterms, (unsigned)pl->R), dim3(kVecBS), 0, s,
                     (const C *)pl->d_gcos, pl->ncoef_int, pl->d_cterms, colscale, pl->ncoef, (C *)fhat);
  return check_launch("k_cos_fold");
}

template <typename T>
int launch_node_grad(gt_plan *pl, const void *fhat, const void *g, void *gx, hipStream_t s) {
  using C = cx_t<T>;
  if (pl->ds == 0) {
    // no term depends on the nodes
    const int64_t total = pl->Mtot * pl->d;
    hipLaunchKernelGGL((k_reduce_gx<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const T *)nullptr, 0,
                       pl->Vtot, pl->Mtot, pl->R, pl->ragged, pl->d, (T)pl->node_scale, (T *)gx);
    return check_launch("k_reduce_gx");
  }
  if (pl->basis == GT_BASIS_COS) {
    if (int rc = cos_expand<T>(pl, fhat, nullptr, s)) return rc;
    fhat = pl->d_gcos;
  }
  if (int rc = launch_pack<T>(pl, fhat, nullptr, s)) return rc;
  if (!pl->d_gxp) {
    const size_t bytes = (size_t)pl->ds * pl->Vtot * pl->d * sizeof(T);
    if (int rc = dev_alloc(&pl->d_gxp, bytes, s)) return rc;
  }
  void *gxp = pl->d_gxp;
  const int ngi = (int)pl->gitems.size();
  int rc = GT_OK;
  for (int t = 1; t <= pl->ds && rc == GT_OK; ++t) {
    const OrderHost &o = pl->ord[t];
    OrderParams<T> op = order_params<T>(pl, t);
    const size_t lds = (size_t)o.gsize * sizeof(C) + (size_t)pl->d * kGatherBS * sizeof(T);
    if (lds > pl->lds_limit) {
      rc = fail(GT_EUNSUPPORTED, "node gradient needs more LDS than available (d too large for this grid)");
      break;
    }
    T *out = (T *)gxp + (size_t)(t - 1) * pl->Vtot * pl->d;
    prof_begin(s, t == 1 ? "node_grad_1d" : t == 2 ? "node_grad_2d" : "node_grad_3d");
#define GT_LAUNCH_NG(MH)                                                                                              \
  {                                                                                                                   \
    if (t == 1) {                                                                                                     \
      if ((rc = set_lds(k_node_grad<T, 1, MH>, lds))) break;                                                         \
      hipLaunchKernelGGL((k_node_grad<T, 1, MH>), dim3(ngi), dim3(kGatherBS), lds, s, (const T *)pl->d_x, pl->Mtot,    \
                         pl->d, pl->d_gitems, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, (const C *)g, out); \
    } else if (t == 2) {                                                                                              \
      if ((rc = set_lds(k_node_grad<T, 2, MH>, lds))) break;                                                         \
      hipLaunchKernelGGL((k_node_grad<T, 2, MH>), dim3(ngi), dim3(kGatherBS), lds, s, (const T *)pl->d_x, pl->Mtot,    \
                         pl->d, pl->d_gitems, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, (const C *)g, out); \
    } else {                                                                                                          \
      if ((rc = set_lds(k_node_grad<T, 3, MH>, lds))) break;                                                         \
      hipLaunchKernelGGL((k_node_grad<T, 3, MH>), dim3(ngi), dim3(kGatherBS), lds, s, (const T *)pl->d_x, pl->Mtot,    \
                         pl->d, pl->d_gitems, pl->d_terms, op, (const C *)pl->d_grid, pl->grid_total, (const C *)g, out); \
    }                                                                                                                 \
  }
    switch (o.m) {
      case 2: GT_LAUNCH_NG(2); break;
      case 3: GT_LAUNCH_NG(3); break;
      case 4: GT_LAUNCH_NG(4); break;
      case 5: GT_LAUNCH_NG(5); break;
      case 6: GT_LAUNCH_NG(6); break;
      case 7: GT_LAUNCH_NG(7); break;
      case 8: GT_LAUNCH_NG(8); break;
      default: rc = fail(GT_EUNSUPPORTED, "window half-width outside 2..8");
    }
#undef GT_LAUNCH_NG
    prof_end(s);
    if (rc == GT_OK) rc = check_launch("k_node_grad");
  }
  if (rc == GT_OK) {
    const int64_t total = pl->Mtot * pl->d;
    hipLaunchKernelGGL((k_reduce_gx<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const T *)gxp,
                       pl->ds, pl->Vtot, pl->Mtot, pl->R, pl->ragged, pl->d, (T)pl->node_scale, (T *)gx);
    rc = check_launch("k_reduce_gx");
  }
  return rc;
}

template <typename T>
int launch_prepare_nodes(gt_plan *pl, const void *x, hipStream_t s) {
  const int64_t total = pl->Mtot * pl->d;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, pl->d_flag);
  if (total > 0)
    hipLaunchKernelGGL((k_prepare_nodes<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const T *)x,
                       pl->Mtot, pl->d, (T)pl->node_scale, (T *)pl->d_x, pl->d_flag);
  return check_launch("k_prepare_nodes");
}

}  // namespace gt
