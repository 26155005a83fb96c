// Direct sums of the terms of one order, without window or FFT grid: the product of
// Definition def:skatoons written out,
//   forward  f_r(x_v) += sum_{k in I_u} fhat_{r,k} e^{2 pi i k . x_{v,u}}
//   adjoint  fhat_{r,k} = sum_v y_{r,v} e^{-2 pi i k . x_{v,u}}
// as dense contractions on 16x16x4 MFMA.  For a small group (|I_u| = (N - 1)^{|u|} against
// the window's (2m)^{|u|} points per node, e.g. N = 6 in three dimensions: 125 against 512 at
// m = 4, 4096 at m = 8) with several right-hand sides these take fewer operations than the
// window path, and they are exact up to rounding.  Shared nodes only (one node set, R <= 16
// right-hand sides as the columns of the contraction).
//
// Phases: per node and axis of the term, e^{2 pi i x} from sincospi(2x), and the band
// k = -N/2..-1, 1..N/2-1 by repeated multiplication, kept in LDS as [axis][k][node]; the phase
// of a frequency of the group is the product over its axes (frequencies row-major over the
// axes, last axis fastest, as the coefficient vector orders them).
//
// MFMA operands (lane l supplies A[l%16][l/16] and B[l/16][l%16]; see Mfma in spread.h),
// real form of the complex products:
//   forward:  rows = 16 nodes, K = (frequency kf, part p of the phase), columns = (r, part c of f);
//             f_re += ph_re F_re - ph_im F_im,  f_im += ph_re F_im + ph_im F_re,
//             so B[(kf,p)][(r,c)] = F_re if p == c, F_im if (p,c) = (0,1), -F_im if (1,0).
//             K slot q of step s holds kf = 2s + q/2, p = q%2.
//   adjoint:  rows = (kf, part c of fhat), K = (node v, part p of y), columns = r;
//             fhat_re += ph_re y_re + ph_im y_im,  fhat_im += ph_re y_im - ph_im y_re,
//             so A[(kf,c)][(v,p)] = ph_re if p == c, ph_im if (c,p) = (0,1), -ph_im if (1,0).
//             K slot q of step s holds v = 2s + q/2, p = q%2.
#pragma once

#include "spread.h"

namespace gt {

struct DirectArgs {
  int32_t K;       // frequencies per axis, N - 1
  int32_t G;       // frequencies of a group, K^order
  int32_t half;    // N / 2
  int32_t R;       // right-hand sides (<= 16)
  int64_t M;       // nodes
  int64_t ncoef;   // coefficient stride of one right-hand side
};

__device__ __forceinline__ void sincos_2pi(float x, float *s, float *c) { sincospif(2.0f * x, s, c); }
__device__ __forceinline__ void sincos_2pi(double x, double *s, double *c) { sincospi(2.0 * x, s, c); }

// Phases of one axis over the band, written to dst[idx * stride] in the group's index order
// (idx = k + N/2 for k < 0, k + N/2 - 1 for k > 0).
template <typename T>
__device__ __forceinline__ void band_phases(T x, int half, cx_t<T> *dst, int stride) {
  T s, c;
  sincos_2pi(x, &s, &c);
  T er = 1, ei = 0;
  for (int j = 1; j <= half; ++j) {
    const T nr = er * c - ei * s, ni = fma(er, s, ei * c);
    er = nr;
    ei = ni;
    dst[(half - j) * stride] = cmake<T>(er, -ei);
    if (j < half) dst[(half - 1 + j) * stride] = cmake<T>(er, ei);
  }
}

template <typename T>
__device__ __forceinline__ cx_t<T> cmul_(cx_t<T> a, cx_t<T> b) {
  return cmake<T>(a.x * b.x - a.y * b.y, fma(a.x, b.y, a.y * b.x));
}

// Forward, all terms [tb, te) of one order: each workgroup takes 4 x RTW x 16 consecutive
// nodes (RTW row tiles of 16 nodes per wavefront) and adds sum_u F_u fhat_u for its nodes into
// f (R x M), accumulating over the terms in registers.  Columns: CT blocks of 8 right-hand
// sides.  LDS: G x 8 CT coefficients and ORDER x K x nodes phases, complex.
template <typename T, int ORDER, int CT, int RTW>
__global__ __launch_bounds__(256) void k_direct_fwd(const T *__restrict__ xT, const DevTerm *__restrict__ terms,
                                                    int tb, int te, DirectArgs da,
                                                    const cx_t<T> *__restrict__ fhat,
                                                    const T *__restrict__ colscale, cx_t<T> *__restrict__ f) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  using C = cx_t<T>;
  constexpr int RP = 8 * CT;             // right-hand sides per column block, padded
  constexpr int NW = 16 * RTW;           // nodes per wavefront (RTW row tiles of 16)
  constexpr int NB = 4 * NW;             // nodes per workgroup
  extern __shared__ __align__(16) unsigned char smem_direct[];
  C *sF = reinterpret_cast<C *>(smem_direct);     // G x RP
  C *sE = sF + (size_t)da.G * RP;                   // ORDER x K x NB
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, i16 = lane & 15;
  const int64_t v0 = (int64_t)blockIdx.x * NB;
  const int K = da.K, G = da.G;
  acc_t acc[RTW][CT];
#pragma unroll
  for (int j = 0; j < RTW; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[j][c] = acc_t{0, 0, 0, 0};
  const bool cim = (i16 & 1) != 0;       // column part: imaginary part of f
  const bool pim = (q & 1) != 0;         // K part: imaginary part of the phase
  for (int u = tb; u < te; ++u) {
    const DevTerm dt = terms[u];
    __syncthreads();                     // the previous term's LDS reads are done
    for (int i = threadIdx.x; i < G * RP; i += 256) {
      const int r = i / G, kf = i - r * G;
      C val = cmake<T>(0, 0);
      if (r < da.R) {
        val = fhat[(int64_t)r * da.ncoef + dt.coef_off + kf];
        if (colscale) {
          const T cs = colscale[dt.coef_off + kf];
          val.x *= cs;
          val.y *= cs;
        }
      }
      sF[kf * RP + r] = val;
    }
    for (int i = threadIdx.x; i < ORDER * NB; i += 256) {
      const int a = i / NB, n = i - a * NB;
      const int ax = a == 0 ? dt.c0 : (a == 1 ? dt.c1 : dt.c2);
      const int64_t v = v0 + n;
      const T x = v < da.M ? xT[(int64_t)ax * da.M + v] : (T)0;
      band_phases<T>(x, da.half, sE + (size_t)a * K * NB + n, NB);
    }
    __syncthreads();
    int id[ORDER];
    {
      int k = q >> 1;
#pragma unroll
      for (int a = ORDER - 1; a >= 0; --a) {
        id[a] = k % K;
        k /= K;
      }
    }
    int kf = q >> 1;
    const int nsteps = (2 * G + 3) >> 2;
    for (int s = 0; s < nsteps; ++s) {
      T av[RTW], bv[CT];
#pragma unroll
      for (int j = 0; j < RTW; ++j) av[j] = 0;
#pragma unroll
      for (int c = 0; c < CT; ++c) bv[c] = 0;
      if (kf < G) {
#pragma unroll
        for (int j = 0; j < RTW; ++j) {
          const int nd = wave * NW + j * 16 + i16;
          C e = sE[(size_t)id[0] * NB + nd];
          if (ORDER > 1) e = cmul_<T>(e, sE[((size_t)K + id[ORDER > 1 ? 1 : 0]) * NB + nd]);
          if (ORDER > 2) e = cmul_<T>(e, sE[((size_t)2 * K + id[ORDER > 2 ? 2 : 0]) * NB + nd]);
          av[j] = pim ? e.y : e.x;
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          const C F = sF[kf * RP + ((i16 + 16 * c) >> 1)];
          bv[c] = pim == cim ? F.x : (cim ? F.y : -F.y);
        }
      }
#pragma unroll
      for (int j = 0; j < RTW; ++j)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[j][c] = MF::run(av[j], bv[c], acc[j][c]);
      kf += 2;
      id[ORDER - 1] += 2;
#pragma unroll
      for (int a = ORDER - 1; a > 0; --a)
        while (id[a] >= K) {
          id[a] -= K;
          ++id[a - 1];
        }
    }
  }
  // D[row][col] with col = i16 + 16c: right-hand side col / 2, real part in even columns
#pragma unroll
  for (int j = 0; j < RTW; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const T mine = acc[j][c][e];
        const T other = __shfl_xor(mine, 1);
        const int64_t v = v0 + wave * NW + j * 16 + MF::row(lane, e);
        const int r = (i16 + 16 * c) >> 1;
        if (!cim && v < da.M && r < da.R) {
          C o = f[(int64_t)r * da.M + v];
          o.x += mine;
          o.y += other;
          f[(int64_t)r * da.M + v] = o;
        }
      }
}

// Adjoint, one term per blockIdx.y (term tb + blockIdx.y), the nodes split into nslice equal
// ranges (blockIdx.x): per 64-node chunk the samples (64 x 16 right-hand sides) and the
// phases are staged in LDS, then each wavefront accumulates its RTW row tiles
// (rows 16 (wave + 4 j) + 0..15) over the chunk's nodes, two nodes per MFMA step.  The
// partial sums go to part[((term * nslice + slice) * 64 RTW + row) * 16 + r].
template <typename T, int ORDER, int RTW>
__global__ __launch_bounds__(256) void k_direct_adj(const T *__restrict__ xT, const DevTerm *__restrict__ terms, int tb,
                                                    DirectArgs da, int nslice, const cx_t<T> *__restrict__ y,
                                                    T *__restrict__ part) {
  using MF = Mfma<T>;
  using acc_t = typename MF::acc;
  using C = cx_t<T>;
  constexpr int ROWS = 64 * RTW;
  __shared__ C sY[64 * 16];
  extern __shared__ __align__(16) unsigned char smem_direct[];
  C *sE = reinterpret_cast<C *>(smem_direct);      // ORDER x K x 64
  const DevTerm dt = terms[tb + blockIdx.y];
  const int slice = blockIdx.x;
  const int64_t n0 = da.M * slice / nslice, n1 = da.M * (slice + 1) / nslice;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, i16 = lane & 15;
  const int K = da.K, G = da.G;
  const bool cim = (i16 & 1) != 0;       // row part: imaginary part of fhat
  const bool pim = (q & 1) != 0;         // K part: imaginary part of y
  // the phase-table offsets of this lane's rows
  int eoff[RTW][ORDER];
  bool valid[RTW];
#pragma unroll
  for (int j = 0; j < RTW; ++j) {
    const int kf = (16 * (wave + 4 * j) + i16) >> 1;
    valid[j] = kf < G;
    int k = valid[j] ? kf : 0;
#pragma unroll
    for (int a = ORDER - 1; a >= 0; --a) {
      eoff[j][a] = (a * K + k % K) * 64;
      k /= K;
    }
  }
  acc_t acc[RTW];
#pragma unroll
  for (int j = 0; j < RTW; ++j) acc[j] = acc_t{0, 0, 0, 0};
  for (int64_t nb = n0; nb < n1; nb += 64) {
    __syncthreads();
    for (int i = threadIdx.x; i < 16 * 64; i += 256) {
      const int r = i >> 6, n = i & 63;
      const int64_t v = nb + n;
      sY[n * 16 + r] = (r < da.R && v < n1) ? y[(int64_t)r * da.M + v] : cmake<T>(0, 0);
    }
    for (int i = threadIdx.x; i < ORDER * 64; i += 256) {
      const int a = i >> 6, n = i & 63;
      const int ax = a == 0 ? dt.c0 : (a == 1 ? dt.c1 : dt.c2);
      const int64_t v = nb + n;
      const T x = v < n1 ? xT[(int64_t)ax * da.M + v] : (T)0;
      band_phases<T>(x, da.half, sE + (size_t)a * K * 64 + n, 64);
    }
    __syncthreads();
#pragma unroll 2
    for (int s = 0; s < 32; ++s) {
      const int n = 2 * s + (q >> 1);
      const C yv = sY[n * 16 + i16];
      const T bv = pim ? yv.y : yv.x;
#pragma unroll
      for (int j = 0; j < RTW; ++j) {
        T av = 0;
        if (valid[j]) {
          C e = sE[eoff[j][0] + n];
          if (ORDER > 1) e = cmul_<T>(e, sE[eoff[j][ORDER > 1 ? 1 : 0] + n]);
          if (ORDER > 2) e = cmul_<T>(e, sE[eoff[j][ORDER > 2 ? 2 : 0] + n]);
          av = pim == cim ? e.x : (cim ? -e.y : e.y);
        }
        acc[j] = MF::run(av, bv, acc[j]);
      }
    }
  }
  T *out = part + ((int64_t)blockIdx.y * nslice + slice) * ROWS * 16;
#pragma unroll
  for (int j = 0; j < RTW; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(16 * (wave + 4 * j) + MF::row(lane, e)) * 16 + i16] = acc[j][e];
}

// Sums the adjoint partials over the node slices in slice order and writes the group's
// coefficients (times the column scale, if any): fhat[r][coef_off + kf].
template <typename T>
__global__ __launch_bounds__(256) void k_direct_adj_sum(const T *__restrict__ part, const DevTerm *__restrict__ terms,
                                                        int tb, DirectArgs da, int nslice, int rows,
                                                        const T *__restrict__ colscale, cx_t<T> *__restrict__ fhat) {
  const int tl = blockIdx.y;
  const DevTerm dt = terms[tb + tl];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= da.G * da.R) return;
  const int r = i / da.G, kf = i - r * da.G;
  const T *p = part + (int64_t)tl * nslice * rows * 16;
  T re = 0, im = 0;
  for (int sl = 0; sl < nslice; ++sl) {
    re += p[((int64_t)sl * rows + 2 * kf) * 16 + r];
    im += p[((int64_t)sl * rows + 2 * kf + 1) * 16 + r];
  }
  const T cs = colscale ? colscale[dt.coef_off + kf] : (T)1;
  fhat[(int64_t)r * da.ncoef + dt.coef_off + kf] = cmake<T>(re * cs, im * cs);
}

}  // namespace gt
